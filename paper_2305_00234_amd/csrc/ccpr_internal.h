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
//                 (keeps the pole's decay rate to full relative precision)
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
#define CCPR_YPAD 4     // padded y extent is a multiple of this (largest strip height)

// Field arrays (E, H, both buffers) are component-major (all x components,
// then all y, then all z; component stride npad floats) and ghost-padded so the
// step kernel never predicates a load: x is padded to nxp = nx rounded up to
// 64, y to nyp = (ny rounded up to CCPR_YPAD) + 2 with one zero row below, z to
// nzp = nz + 2 with one zero plane below and above.  Cell (i,j,k) of component
// c lives at c*npad + ((k+1)*nyp + (j+1))*nxp + i; ghost cells are zero and
// never written.  Kernels address a component with 32-bit byte offsets from
// its own base, so npad*4 must stay below 2^32.

// One TF/SF face correction: field word at byte offset 'off' of E (or H)
// (component included, so 64-bit), incident table column m, coefficient coef
// (sign, side and Courant number folded in);
// uidx = component * nx*ny*nz + (k*ny + j)*nx + i.
struct TfEntry {
    unsigned long long off;
    int m;
    float coef;
    unsigned uidx;
};

// Material constants of one axis.  The E increment and the pole-current
// recurrences are evaluated in FP64 arithmetic from FP64 constants (a metal's
// conductivity and its Drude pole nearly cancel in A and in the numerator, and
// the recurrences' intermediate roundings would otherwise dominate); fields
// and currents are stored in FP32, the gradient factor is formed in FP32.
struct AxisMat {
    double eps1, deps;  // eps'(rho) = eps1 + rho*deps
    double sig1, dsig;  // sigma'(rho) = sig1 + rho*dsig + rho*(1-rho)*gam
    double gam;
    double krd[CCPR_PMAX], kid[CCPR_PMAX];  // k_p - 1 (real, imag)
    double brd[CCPR_PMAX], bid[CCPR_PMAX];  // beta'_p
    float epsf, depsf, dsigf, gamf;         // FP32 copies for the gradient factor
    int np;             // pole pairs on this axis; the first np1 belong to slot 1
    int np1;
    int jofs;           // first flat pair index of this axis in the J arrays
};

// Per-edge design (one density per E edge): the kernels run over the box of
// N + 1 cells per axis that holds every design edge of an N-cell design, and
// component c has design edges on the sub-box of extents N_l + 1 - delta(c,l)
// (its far face along its own axis has none: those edges are vacuum).
// Densities and gradients are held per component, x edges then y then z, each
// x fastest in its own sub-box.
struct EdgeMap {
    int on;                     // 1: per-edge design; 0: one density per voxel
    int ebox[3][3];             // [component][axis] extents of the component's edges
    long long eoff[3];          // first density / gradient index of each component
};

// Step data the kernel needs only inside rare branches (design voxels, CPML
// layers, sources, TF/SF faces, the gap monitor, the gradient history).  It
// lives in device memory (one block per state), so the hot loop keeps its
// scalar registers for the field bases.
struct StepCold {
    // design box (per-edge designs: the box of N + 1 cells per axis)
    int dlo[3], ddim[3];
    long long nd;
    const float* rho;           // per voxel [nd], or per edge (see EdgeMap)
    float* J;                   // [(2*q + {0:re,1:im}) * nd + v]
    AxisMat mat[3];
    EdgeMap em;

    // CPML: per axis, (b, a, 1/kappa, 0) at integer (E) and half-integer (H)
    // positions; psi memories per derivative axis, two components each
    // (second component at +slab_size/2):
    //   x: [k][j][xs], xs in [0,2 npml) (low layer then high layer)
    //   y: [k][ys][i (nxp)], ys in [0,2 npml)
    //   z: [zs][j][i (nxp)], zs in [0,2 npml)
    const float4* pmlE[3];
    const float4* pmlH[3];
    float* psiE[3];
    float* psiH[2][3];          // [buffer][axis]; H-side psi is double-buffered
                                // (read psi_in, write psi_in ^ 1)

    // current source on the E edges of a small box: src[(n*sncell + c)*3 + axis]
    int src_on, slo[3], sdim[3], sncell, snsteps;
    const float* src;
    double* ssh;                // FP64 shadow of E on the source edges [sncell][3]

    // TF/SF plane wave (axis-aligned): incident E' at integer positions
    // [lo_d, hi_d] (row n = E^n) and H' at half-integer positions
    // [lo_d-1, hi_d] (row n = H^{n+1/2}) along the propagation axis d, rows
    // 0..tf_rows-1.  The face corrections are a list of field words (TfEntry):
    // the first tf_nE add coef*incH[n][m] to E^{n+1} after step n, the next
    // tf_nH add coef*incE[n][m] to H^{n-1/2} before step n reads it.
    int pw_on, pw_spanE, pw_spanH, tf_rows, tf_nE, tf_nH;
    const float* incE;
    const float* incH;
    const struct TfEntry* tf;

    // gap monitor: gap[((n+1)*gncell + c)*3 + axis] = E^{n+1}
    int gap_on, glo[3], gdim[3], gncell;
    float* gap;

    float* T;                   // time-exact mode: gradient history [slot][3][nd];
                                // DFT mode: [12][nd], the forward transform of T
                                // (re, im of x, y, z) then the adjoint projection
    double* grad;               // adjoint: accumulator per voxel, or per edge (EdgeMap)
};

// Row classes (one word per (j,k), per state) and lane classes (one word per
// x position): which rare work a row / a lane can need.
#define CCPR_ROW_YPML 1u        // row inside a y CPML layer
#define CCPR_ROW_ZPML 2u        // plane inside a z CPML layer
#define CCPR_ROW_DES 4u         // row crosses the design box
#define CCPR_ROW_SRC 8u         // row crosses the source box
#define CCPR_LANE_PML 1u        // x inside a CPML layer
#define CCPR_LANE_DES 2u        // x inside the design box
#define CCPR_LANE_SRC 4u        // x inside the source box

// Kernel argument of one leapfrog step (the fused grid kernel and the
// auxiliary kernel of the design / source / gap cells share it).
struct StepArgs {
    const float* Ei;            // E^n (component-major, padded)
    float* Eo;                  // E^{n+1}
    const float* Hi;            // H^{n-1/2}
    float* Ho;                  // H^{n+1/2}
    const unsigned* rowf;       // row classes [k*ny + j]
    const unsigned* lanef;      // lane classes [nxp]
    float* drive;               // S curl H' of design voxels [3][nd], then source cells [sncell][3]
    const int4* extra;          // non-design cells finished by the post kernel: (i, j, k, kind)
    long long nextra;
    unsigned cstride;           // bytes between field components (npad*4)
    int stream_st;              // 1: write the streamed state with nontemporal stores
    int nx, ny, nz, nxp, nyp;
    int rows;                   // y rows per thread (2 or 4)
    int npml;
    float S;                    // Courant number
    int n;                      // step index: this launch advances n -> n+1
    int psi_in;                 // which H-side psi buffer holds psi^{n-1/2}
    int tslot;                  // gradient-history slot of this step (-1: none)
    int mode;                   // CCPR_MODE_* bits
    float phc, phs;             // DFT modes: cos, sin of omega dt n (forward step n)
                                // or of omega dt m (adjoint field m)
    const StepCold* cold;
    const unsigned* halt;       // nonzero: the divergence watchdog tripped; every
                                // step kernel returns at once
    const int2* zr;             // plane range [k0, k1) of each logical z-chunk
    const int2* tiles;          // this launch's tiles: (y-strip, logical z-chunk)
    int nys;                    // y strips
    int nblk;                   // blocks of this launch (tiles in the list)
};

#define CCPR_EXTRA_SOURCE 1     // source cell outside the design box
#define CCPR_EXTRA_GAP 2        // gap-monitor cell outside the design and source boxes

#define CCPR_MODE_RECORD 1      // forward: write T of this step to slot tslot
#define CCPR_MODE_CORREL 2      // adjoint: grad += E^{n+1} . T[tslot]
#define CCPR_MODE_GAP 4         // forward: record the gap monitor
#define CCPR_MODE_DFT_T 8       // forward, DFT mode: T_hat += T exp(-j phase)
#define CCPR_MODE_DFT_P 16      // adjoint, DFT mode: P += E^{n+1} exp(-j phase)

// ---- batched steps of several solves (the serving engine): one grid, one
// aux and one post launch advance up to CCPR_BATCH_MAX solves of the same
// padded x width by one leapfrog step each.  A solve's recorded step:
#define CCPR_BATCH_MAX 8
struct BatchStep {
    StepArgs a;                 // its StepArgs (tiles = all its tiles, nblk = their count)
    int maxpairs;               // pole pairs of its widest axis
    long long nd;               // design-box cells (aux kernel)
    int fused;                  // 1: post of this step + pre of the next (fused post kernel)
    long long nxs, nmisc, ntfh; // x-layer cells, misc cells, next step's TF/SF H words
};
// Kernel argument of the batched launches: block b of a launch belongs to
// solve s with start[s] <= b < start[s + 1].
struct BatchArgs {
    StepArgs a[CCPR_BATCH_MAX];
    int n;
    int gstart[CCPR_BATCH_MAX + 1], astart[CCPR_BATCH_MAX + 1], pstart[CCPR_BATCH_MAX + 1];
    int fused[CCPR_BATCH_MAX], rpb[CCPR_BATCH_MAX];
    long long nbx[CCPR_BATCH_MAX], nmisc[CCPR_BATCH_MAX], ntfh[CCPR_BATCH_MAX], nxs[CCPR_BATCH_MAX];
};

// floats of the psi memory of derivative axis a (both components)
__host__ __device__ inline long long slab_size(int a, int nx, int ny, int nz, int nxp, int npml)
{
    const long long t = 2LL * npml;
    return 2 * (a == 0 ? (long long)nz * ny * t : a == 1 ? (long long)nz * t * nxp : t * ny * nxp);
}

// Launchers (ccpr_kernels.hip)
// fused grid step over the tiles of a.tiles (pml: the CPML variant); events
// given are recorded by the dispatch itself (on the stream when no tiles)
int ccpr_launch_grid(const StepArgs& a, bool pml, void* stream, void* start_event = nullptr,
                     void* stop_event = nullptr);
// interior tiles that own design cells, with the design update fused in
// (per-voxel design, time-exact gradient; rows 2, nxp <= 512, maxpairs <= 8)
int ccpr_launch_grid_des(const StepArgs& a, int maxpairs, void* stream);
// aux kernel over the nd cells of the design box (edge: per-edge design)
int ccpr_launch_aux(const StepArgs& a, int maxpairs, long long nd, bool edge, void* stream);
// before a step: x-CPML and TF/SF corrections of H^{n-1/2} (nxs x-layer cells,
// ntf TF/SF H words)
int ccpr_launch_pre(const StepArgs& a, long long nxs, long long ntf, void* stream);
// after the aux kernel: x-CPML of E^{n+1} (nxs x-layer cells) and the
// nmisc = nextra + tf_nE source / gap cells and TF/SF E words
int ccpr_launch_post(const StepArgs& a, long long nxs, long long nmisc, void* stream);
// after the aux kernel when the next step follows at once: the post work of
// step n and the pre work of step n+1 (ntfh TF/SF H words) in one launch
// (2 npml <= 256); stop_event, if given, is recorded by the dispatch itself
int ccpr_launch_post_fused(const StepArgs& a, long long nmisc, long long ntfh, void* stream,
                           void* stop_event = nullptr);
// the recorded steps st[0..k) (1 <= k <= CCPR_BATCH_MAX, same nxp, 2 rows per
// thread, 2 npml <= 256) as one batched grid, aux and post launch each
int ccpr_launch_batch(const BatchStep* st, int k, void* stream);
int ccpr_launch_fill(float* p, long long n, float v, void* stream);
int ccpr_launch_fill_d(double* p, long long n, double v, void* stream);
int ccpr_launch_copy(float* dst, const float* src, long long n, void* stream);
int ccpr_launch_scale(float* dst, const float* src, long long n, float s, void* stream);
int ccpr_launch_extract(float* dst, const float* src, int comp, int nx, int ny, int nz, int nxp, int nyp,
                        float f, void* stream);
// dst = acc * (*scale)
// DFT-mode gradient: grad[v] = sum_k Re{A_k W T_hat_k} with A_k from the
// adjoint projection P_k and the inverse window normal matrix (i00, i01, i11),
// W = (wc, ws)
int ccpr_launch_dft_grad(double* grad, const float* acc, long long nd, const int ddim[3], const EdgeMap& em,
                         double i00, double i01, double i11, double wc, double ws, void* stream);
// spectrum of the recorded gap field at nf angular frequencies (device
// arrays omega[nf], out[nf])
int ccpr_launch_gap_spectrum(const float* gap, int M, int ne, double dt, const double* omega, int nf, double scale,
                             double* out, void* stream);
int ccpr_launch_grad_out(double* dst, const double* acc, long long n, const double* scale, void* stream);
// SI objective and scales of a forward run into scal[4..6] (kind 1: DFT, 0: time)
int ccpr_launch_finish(double* scal, int kind, double a, double dt, double dx, double eps0, void* stream);
int ccpr_launch_copy_d(double* dst, const double* src, long long n, void* stream);
int ccpr_launch_incident_line(const double* wave, int nw, int M, int L, double coef, int lo_d,
                              int hi_d, int sgn, int ref, double* lineE, double* lineH,
                              float* incE, float* incH, void* stream);
int ccpr_launch_objective(const float* gap, int M, int ne, int kind, double omega_dt, int nb,
                          int nend, double* scal, double* work, float* adj, void* stream);
int ccpr_launch_check_rho(const float* rho, long long n, double* flag, void* stream);
// divergence watchdog after step n of a run: trips when an E edge of the
// monitor box [lo, lo + dim) of the field state a.Eo is not finite or above
// limit (scaled units): halt[0] = 1 (the step kernels of every later step
// return at once) and scal[7] = n + 1 (steps done when it tripped), once
int ccpr_launch_watch(const StepArgs& a, const int lo[3], const int dim[3], float limit, int n, unsigned* halt,
                      double* scal, void* stream);
