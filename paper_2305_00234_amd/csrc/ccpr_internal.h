// Internal declarations shared by the gfx950 kernels and the host runtime.
//
// Private field scaling (the C-ABI is SI): with alpha the source scale of a
// run,
//   E' = alpha E,  H' = alpha eta0 H,  J'_p = alpha (dt/eps0) J_p,
//   s' = alpha (dt/eps0) J_src,
// so that the curl coefficient is the Courant number S and every material
// constant is dimensionless:
//   eps'(rho)   = eps_inf(rho)
//   sigma'(rho) = sigma(rho) dt / (2 eps0)
//   k_p         = (1 + a_p dt/2)/(1 - a_p dt/2), held as k_p - 1 = a_p dt/(1 - a_p dt/2)
//                 (FP32 keeps the pole's decay rate to full relative precision)
//   beta'_p     = c_p dt / (1 - a_p dt/2)
// E update (trapezoid rule on sigma E and on the pole-pair currents, bilinear
// rule on dJ/dt = a J + eps0 c dE/dt):
//   A = eps' + sigma' + sum_p kap_p Re beta'_p
//   E^{n+1} = E^n + (S curl H' - s' - 2 sigma' E^n - sum_p kap_p Re{(1+k_p) J'_p})/A
//   J'_p^{n+1} = k_p J'_p^n + beta'_p (E^{n+1} - E^n)
// Gradient factor per design edge (dt * d/drho of Ampere's residual at fixed
// fields, in scaled units; T_SI = (eps0/alpha) T'):
//   T' = deps (E^{n+1}-E^n) + dsig'_eff (E^{n+1}+E^n) + sum_p dkap_p Re{J'^{n+1}+J'^n}
#pragma once

#include <stdint.h>

#define CCPR_PMAX 8     // pole pairs per axis (both materials together)
#define CCPR_ROWS 4     // y rows per thread in the fused step kernel

struct AxisMat {
    float eps1, deps;   // eps'(rho) = eps1 + rho*deps
    float sig1, dsig;   // sigma'(rho) = sig1 + rho*dsig + rho*(1-rho)*gam
    float gam;
    int np;             // pole pairs on this axis; the first np1 belong to slot 1
    int np1;
    int jofs;           // first flat pair index of this axis in the J arrays
    float kr[CCPR_PMAX], ki[CCPR_PMAX];  // k_p - 1 (real, imag)
    float br[CCPR_PMAX], bi[CCPR_PMAX];  // beta'_p
};

// Everything one fused leapfrog step needs.  Passed by value.
struct StepArgs {
    int nx, ny, nz;
    long long plane;            // nx*ny
    float S;                    // Courant number
    const float* Ei[3];         // E^n
    float* Eo[3];               // E^{n+1}
    const float* Hi[3];         // H^{n-1/2}
    float* Ho[3];               // H^{n+1/2}

    // design box
    int dlo[3], ddim[3];
    long long nd;
    const float* rho;
    float* J;                   // [(2*q + {0:re,1:im}) * nd + v]
    AxisMat mat[3];

    // CPML: per axis, (b, a, 1/kappa, 0) at integer (E) and half-integer (H)
    // positions; psi slabs per derivative axis (see slab_index)
    int npml;
    const float4* pmlE[3];
    const float4* pmlH[3];
    float* psiE[3];
    const float* psiHi[3];
    float* psiHo[3];

    int n;                      // step index: this launch advances n -> n+1

    // current source on the E edges of a small box: src[(n*sncell + c)*3 + axis]
    int src_on, slo[3], sdim[3], sncell, snsteps;
    const float* src;
    double* ssh;                // FP64 shadow of E on the source edges [sncell][3]

    // TF/SF plane wave (axis-aligned): incident E' at integer positions
    // [lo_d, hi_d] (row n = E^n) and H' at half-integer positions
    // [lo_d-1, hi_d] (row n = H^{n+1/2}) along the propagation axis d.
    int pw_on, pw_d, pw_p, pw_t, pwlo[3], pwhi[3], pw_spanE, pw_spanH;
    float sg_Ep_d, sg_Ed_p, sg_Ht_d, sg_Hd_t;
    const float* incE;
    const float* incH;

    // gap monitor: gap[((n+1)*gncell + c)*3 + axis] = E^{n+1}
    int gap_on, glo[3], gdim[3], gncell;
    float* gap;

    float* Tout;                // forward record [3][nd] for this step, or null
    const float* Tin;           // adjoint: forward factor paired with this step
    double* grad;               // adjoint: per-voxel accumulator

    // launch geometry
    int tz;                     // planes per block
    int nys;                    // y strips
    int nblk;                   // total blocks
};

struct SlabDims {
    int nx, ny, nz, npml;
};

// Index in the psi slab of derivative axis a for component slot ci (0: the
// component (a+1)%3, 1: (a+2)%3), on side 0 (low) / 1 (high).
__host__ __device__ inline long long slab_index(int a, int ci, int side, int i, int j, int k,
                                                int nx, int ny, int nz, int npml)
{
    if (a == 0) {
        int ii = side ? i - (nx - npml) : i;
        return ((((long long)(ci * 2 + side) * nz + k) * ny + j) * npml + ii);
    } else if (a == 1) {
        int jj = side ? j - (ny - npml) : j;
        return ((((long long)(ci * 2 + side) * nz + k) * npml + jj) * nx + i);
    } else {
        int kk = side ? k - (nz - npml) : k;
        return ((((long long)(ci * 2 + side) * npml + kk) * ny + j) * nx + i);
    }
}

__host__ __device__ inline long long slab_size(int a, int nx, int ny, int nz, int npml)
{
    long long cross = a == 0 ? (long long)ny * nz : a == 1 ? (long long)nx * nz : (long long)nx * ny;
    return 4LL * npml * cross;  // 2 components x 2 sides
}

// Launchers (ccpr_kernels.hip)
int ccpr_launch_step(const StepArgs& a, int maxpairs, void* stream);
int ccpr_launch_fill(float* p, long long n, float v, void* stream);
int ccpr_launch_fill_d(double* p, long long n, double v, void* stream);
int ccpr_launch_copy(float* dst, const float* src, long long n, void* stream);
int ccpr_launch_scale(float* dst, const float* src, long long n, float s, void* stream);
int ccpr_launch_grad_out(double* dst, const double* acc, long long n, double s, void* stream);
int ccpr_launch_copy_d(double* dst, const double* src, long long n, void* stream);
int ccpr_launch_incident_line(const double* wave, int nw, int M, int L, double coef, int lo_d,
                              int hi_d, int sgn, int ref, double* lineE, double* lineH,
                              float* incE, float* incH, void* stream);
int ccpr_launch_objective(const float* gap, int M, int ne, int kind, double omega_dt, int nb,
                          int nend, double* scal, double* work, float* adj, void* stream);
int ccpr_launch_check_rho(const float* rho, long long n, double* flag, void* stream);
