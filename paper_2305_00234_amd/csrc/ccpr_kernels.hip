// gfx950 kernels of the CCPR-FDTD path.
//
// ccpr_step_kernel performs one full leapfrog step -- H^{n-1/2} -> H^{n+1/2}
// (Faraday, supplement Eq. Maxwells2 c) and E^n -> E^{n+1} with the CCPR
// pole-pair currents (Eqs. Maxwells2 a, b; interpolation Eqs. eps_mixed,
// sigma_mixed, Poles_mixed) -- plus CPML, sources, TF/SF corrections, the gap
// monitor, the forward gradient record and the adjoint gradient correlation
// (Eq. Gradient_FDTD), in ONE pass over memory: every field word is read once
// and written once per step (48 bytes per vacuum cell).
//
// Work decomposition (memory-bound stencil, no MFMA):
//  - a workgroup spans the whole x extent (blockDim = nx rounded up to 64),
//    so x-neighbours come from wave shuffles plus one LDS word per wave seam;
//  - each thread owns CCPR_ROWS consecutive y rows (register blocking) and the
//    workgroup marches over a chunk of tz z-planes, keeping the previous
//    plane's new H and the next plane's old E in registers;
//  - H^{n+1/2} is recomputed on one halo row (y = j0-1) and one halo plane
//    (z = k0-1) so the E update never waits on another workgroup.  E, H and
//    the H-side CPML memories are therefore double-buffered (read old, write
//    new); pole currents and E-side CPML memories are touched only by their
//    owner and are updated in place;
//  - workgroups are numbered so that each XCD gets a contiguous run of
//    y-strips: neighbouring strips share their halo rows in the same L2.
#include <hip/hip_runtime.h>

#include "ccpr_internal.h"

namespace {

constexpr int R = CCPR_ROWS;

__device__ __forceinline__ bool in_box(int i, int j, int k, const int* lo, const int* dim)
{
    return (unsigned)(i - lo[0]) < (unsigned)dim[0] && (unsigned)(j - lo[1]) < (unsigned)dim[1] &&
           (unsigned)(k - lo[2]) < (unsigned)dim[2];
}

__device__ __forceinline__ int box_index(int i, int j, int k, const int* lo, const int* dim)
{
    return ((k - lo[2]) * dim[1] + (j - lo[1])) * dim[0] + (i - lo[0]);
}

// Stretched derivative on the H side: psi^{n+1/2} = b psi^{n-1/2} + a d,
// returns d/kappa + psi.  Only the owner of the H point stores psi.
template <int AX>
__device__ __forceinline__ float pml_h(const StepArgs& a, int ci, int pos, int i, int j, int k,
                                       float d, bool own)
{
    const int N = AX == 0 ? a.nx : AX == 1 ? a.ny : a.nz;
    const int side = pos < a.npml ? 0 : 1;
    (void)N;
    const float4 cf = a.pmlH[AX][pos];
    const long long s = slab_index(AX, ci, side, i, j, k, a.nx, a.ny, a.nz, a.npml);
    const float psi = fmaf(cf.x, a.psiHi[AX][s], cf.y * d);
    if (own) a.psiHo[AX][s] = psi;
    return fmaf(d, cf.z, psi);
}

template <int AX>
__device__ __forceinline__ float pml_e(const StepArgs& a, int ci, int pos, int i, int j, int k,
                                       float d)
{
    const int side = pos < a.npml ? 0 : 1;
    const float4 cf = a.pmlE[AX][pos];
    const long long s = slab_index(AX, ci, side, i, j, k, a.nx, a.ny, a.nz, a.npml);
    const float psi = fmaf(cf.x, a.psiE[AX][s], cf.y * d);
    a.psiE[AX][s] = psi;
    return fmaf(d, cf.z, psi);
}

__device__ __forceinline__ bool in_slab(int pos, int N, int npml)
{
    return npml > 0 && (pos < npml || pos >= N - npml);
}

// TF/SF correction to (curl E)_c at an H point (see host code for the face
// bookkeeping): H just outside a face sees the total E on the face.
__device__ __forceinline__ float tfsf_h(const StepArgs& a, int c, int cd, int cp, int ct)
{
    const int d = a.pw_d, p = a.pw_p, t = a.pw_t;
    const float* inc = a.incE + (long long)a.n * a.pw_spanE;
    const int lod = a.pwlo[d], hid = a.pwhi[d];
    if (c == t) {
        if (ct >= a.pwlo[t] && ct <= a.pwhi[t] && cp >= a.pwlo[p] && cp < a.pwhi[p]) {
            if (cd == lod - 1) return -a.sg_Ht_d * inc[0];
            if (cd == hid) return a.sg_Ht_d * inc[hid - lod];
        }
    } else if (c == d) {
        if (cd >= lod && cd <= hid && cp >= a.pwlo[p] && cp < a.pwhi[p]) {
            if (ct == a.pwlo[t] - 1) return -a.sg_Hd_t * inc[cd - lod];
            if (ct == a.pwhi[t]) return a.sg_Hd_t * inc[cd - lod];
        }
    }
    return 0.f;
}

// TF/SF correction to (curl H)_c at an E point on a face of the total-field
// box: the E point is total, its outside H neighbour is scattered.
__device__ __forceinline__ float tfsf_e(const StepArgs& a, int c, int cd, int cp, int ct)
{
    const int d = a.pw_d, p = a.pw_p, t = a.pw_t;
    const float* inc = a.incH + (long long)a.n * a.pw_spanH;
    const int lod = a.pwlo[d], hid = a.pwhi[d];
    if (c == p) {
        if (ct >= a.pwlo[t] && ct <= a.pwhi[t] && cp >= a.pwlo[p] && cp < a.pwhi[p]) {
            if (cd == lod) return -a.sg_Ep_d * inc[0];
            if (cd == hid) return a.sg_Ep_d * inc[hid - lod + 1];
        }
    } else if (c == d) {
        if (ct >= a.pwlo[t] && ct <= a.pwhi[t] && cd >= lod && cd < hid) {
            if (cp == a.pwlo[p]) return -a.sg_Ed_p * inc[cd - lod + 1];
            if (cp == a.pwhi[p]) return a.sg_Ed_p * inc[cd - lod + 1];
        }
    }
    return 0.f;
}

// Dispersive E update of component C at design voxel v (see ccpr_internal.h).
// sh (may be null): FP64 shadow of E on a source edge; E^{n+1} is then
// accumulated in FP64 and rounded once.
template <int C, int PMAX>
__device__ __forceinline__ float e_disp(const StepArgs& a, float E, float drive, float rho,
                                        long long v, float* T, double* sh)
{
    const AxisMat& m = a.mat[C];
    const float om = 1.f - rho;
    const float eps = fmaf(rho, m.deps, m.eps1);
    const float sig = fmaf(rho, m.dsig, m.sig1) + rho * om * m.gam;
    float A = eps + sig;
    float acc = 0.f, rold = 0.f;
    float jr[PMAX > 0 ? PMAX : 1], ji[PMAX > 0 ? PMAX : 1];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        if (p < m.np) {
            const long long q = m.jofs + p;
            jr[p] = a.J[(2 * q) * a.nd + v];
            ji[p] = a.J[(2 * q + 1) * a.nd + v];
            const float kap = p < m.np1 ? om : rho;
            A = fmaf(kap, m.br[p], A);
            // Re{(1 + k_p) J} with 1 + k_p = 2 + (k_p - 1)
            acc = fmaf(kap, fmaf(2.f + m.kr[p], jr[p], -m.ki[p] * ji[p]), acc);
            rold += p < m.np1 ? -jr[p] : jr[p];
        }
    }
    const float inc = (drive - 2.f * sig * E - acc) / A;
    float En;
    if (sh) { *sh += (double)inc; En = (float)*sh; }
    else En = E + inc;
    const float dE = En - E;
    float rnew = 0.f;
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        if (p < m.np) {
            const long long q = m.jofs + p;
            // J^{n+1} = J + (k_p - 1) J + beta'_p dE
            const float nr = jr[p] + fmaf(m.kr[p], jr[p], fmaf(-m.ki[p], ji[p], m.br[p] * dE));
            const float ni = ji[p] + fmaf(m.kr[p], ji[p], fmaf(m.ki[p], jr[p], m.bi[p] * dE));
            a.J[(2 * q) * a.nd + v] = nr;
            a.J[(2 * q + 1) * a.nd + v] = ni;
            rnew += p < m.np1 ? -nr : nr;
        }
    }
    *T = fmaf(m.deps, dE, fmaf(m.dsig + (1.f - 2.f * rho) * m.gam, En + E, rnew + rold));
    return En;
}

template <int PMAX>
__global__ __launch_bounds__(1024) void ccpr_step_kernel(const StepArgs a)
{
    __shared__ float xe[2][R + 1][16];
    __shared__ float xh[2][R][16];

    // XCD-aware tile order: hardware hands workgroups to the 8 XCDs round
    // robin; give each XCD a contiguous range of logical tiles.
    const int b = blockIdx.x;
    const int per = a.nblk >> 3, rem = a.nblk & 7;
    const int xcd = b & 7, q = b >> 3;
    const int L = xcd * per + (xcd < rem ? xcd : rem) + q;
    const int ys = L % a.nys, zc = L / a.nys;
    const int j0 = ys * R;
    const int k0 = zc * a.tz;
    const int k1 = min(k0 + a.tz, a.nz);

    const int i = threadIdx.x;
    const int lane = i & 63, w = i >> 6, nw = blockDim.x >> 6;
    const bool xin = i < a.nx;
    const float S = a.S;
    const bool xpml = in_slab(i, a.nx, a.npml);

    // registers: E^n on the current plane (rows j0-1 .. j0+R), next plane,
    // H^{n+1/2} of the previous plane (x, y comps, rows j0 .. j0+R-1)
    float ex[R + 2], ey[R + 2], ez[R + 2];
    float nex[R + 2], ney[R + 2], nez[R + 2];
    float hxm[R + 1], hym[R + 1];
    float hx[R + 1], hy[R + 1], hz[R + 1];

    auto row_ok = [&](int j, int k) { return xin && j >= 0 && j < a.ny && k >= 0 && k < a.nz; };
    auto load_plane = [&](int k, float* px, float* py, float* pz) {
#pragma unroll
        for (int r = 0; r < R + 2; ++r) {
            const int j = j0 - 1 + r;
            const bool ok = row_ok(j, k);
            const long long o = (long long)k * a.plane + (long long)j * a.nx + i;
            px[r] = ok ? a.Ei[0][o] : 0.f;
            py[r] = (ok && r <= R) ? a.Ei[1][o] : 0.f;
            pz[r] = ok ? a.Ei[2][o] : 0.f;
        }
    };

    load_plane(k0 - 1, ex, ey, ez);
#pragma unroll
    for (int r = 0; r <= R; ++r) { hxm[r] = 0.f; hym[r] = 0.f; }

    for (int kk = k0 - 1; kk < k1; ++kk) {
        load_plane(kk + 1, nex, ney, nez);

        // ---- x+1 neighbours of E^n on this plane (Ey rows 0..R, Ez rows 0..R)
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r <= R; ++r) { xe[0][r][w] = ey[r]; xe[1][r][w] = ez[r]; }
        }
        __syncthreads();
        float eyr[R + 1], ezr[R + 1];
#pragma unroll
        for (int r = 0; r <= R; ++r) {
            eyr[r] = __shfl_down(ey[r], 1);
            ezr[r] = __shfl_down(ez[r], 1);
            if (lane == 63) {
                eyr[r] = (w + 1 < nw) ? xe[0][r][w + 1] : 0.f;
                ezr[r] = (w + 1 < nw) ? xe[1][r][w + 1] : 0.f;
            }
        }

        // ---- H^{n+1/2} on rows j0-1 .. j0+R-1 of plane kk
        const bool kok = kk >= 0;
        const bool zpml = in_slab(kk, a.nz, a.npml);
#pragma unroll
        for (int r = 0; r <= R; ++r) {
            const int j = j0 - 1 + r;
            const bool ok = kok && row_ok(j, kk);
            const bool own = ok && r >= 1 && kk >= k0;
            const long long o = (long long)kk * a.plane + (long long)j * a.nx + i;
            float hxo = 0.f, hyo = 0.f, hzo = 0.f;
            if (ok) { hxo = a.Hi[0][o]; hyo = a.Hi[1][o]; hzo = a.Hi[2][o]; }
            // Hx: d1 = y (Ez), d2 = z (Ey);  Hy: d1 = z (Ex), d2 = x (Ez);
            // Hz: d1 = x (Ey), d2 = y (Ex)   -- forward differences
            float dxA = ez[r + 1] - ez[r], dxB = ney[r] - ey[r];
            float dyA = nex[r] - ex[r], dyB = ezr[r] - ez[r];
            float dzA = eyr[r] - ey[r], dzB = ex[r + 1] - ex[r];
            if (ok && a.npml > 0) {
                const bool ypml = in_slab(j, a.ny, a.npml);
                if (ypml) {
                    dxA = pml_h<1>(a, 1, j, i, j, kk, dxA, own);
                    dzB = pml_h<1>(a, 0, j, i, j, kk, dzB, own);
                }
                if (zpml) {
                    dxB = pml_h<2>(a, 0, kk, i, j, kk, dxB, own);
                    dyA = pml_h<2>(a, 1, kk, i, j, kk, dyA, own);
                }
                if (xpml) {
                    dyB = pml_h<0>(a, 0, i, i, j, kk, dyB, own);
                    dzA = pml_h<0>(a, 1, i, i, j, kk, dzA, own);
                }
            }
            float cx = dxA - dxB, cy = dyA - dyB, cz = dzA - dzB;
            if (a.pw_on && ok) {
                const int cd = a.pw_d == 0 ? i : a.pw_d == 1 ? j : kk;
                const int cp = a.pw_p == 0 ? i : a.pw_p == 1 ? j : kk;
                const int ct = a.pw_t == 0 ? i : a.pw_t == 1 ? j : kk;
                cx += tfsf_h(a, 0, cd, cp, ct);
                cy += tfsf_h(a, 1, cd, cp, ct);
                cz += tfsf_h(a, 2, cd, cp, ct);
            }
            hx[r] = ok ? fmaf(-S, cx, hxo) : 0.f;
            hy[r] = ok ? fmaf(-S, cy, hyo) : 0.f;
            hz[r] = ok ? fmaf(-S, cz, hzo) : 0.f;
            if (own) { a.Ho[0][o] = hx[r]; a.Ho[1][o] = hy[r]; a.Ho[2][o] = hz[r]; }
        }

        // ---- x-1 neighbours of H^{n+1/2} (Hy, Hz rows 1..R)
        if (lane == 63) {
#pragma unroll
            for (int r = 1; r <= R; ++r) { xh[0][r - 1][w] = hy[r]; xh[1][r - 1][w] = hz[r]; }
        }
        __syncthreads();
        float hyl[R + 1], hzl[R + 1];
#pragma unroll
        for (int r = 1; r <= R; ++r) {
            hyl[r] = __shfl_up(hy[r], 1);
            hzl[r] = __shfl_up(hz[r], 1);
            if (lane == 0) {
                hyl[r] = w > 0 ? xh[0][r - 1][w - 1] : 0.f;
                hzl[r] = w > 0 ? xh[1][r - 1][w - 1] : 0.f;
            }
        }

        // ---- E^{n+1} on rows j0 .. j0+R-1 of plane kk
        if (kk >= k0) {
            const bool zp = in_slab(kk, a.nz, a.npml);
#pragma unroll
            for (int r = 1; r <= R; ++r) {
                const int j = j0 - 1 + r;
                if (!row_ok(j, kk)) continue;
                const long long o = (long long)kk * a.plane + (long long)j * a.nx + i;
                // (curl H)_x: d1 = y (Hz), d2 = z (Hy); (curl H)_y: d1 = z (Hx),
                // d2 = x (Hz); (curl H)_z: d1 = x (Hy), d2 = y (Hx)  -- backward
                float gxA = hz[r] - hz[r - 1], gxB = hy[r] - hym[r];
                float gyA = hx[r] - hxm[r], gyB = hz[r] - hzl[r];
                float gzA = hy[r] - hyl[r], gzB = hx[r] - hx[r - 1];
                if (a.npml > 0) {
                    if (in_slab(j, a.ny, a.npml)) {
                        gxA = pml_e<1>(a, 1, j, i, j, kk, gxA);
                        gzB = pml_e<1>(a, 0, j, i, j, kk, gzB);
                    }
                    if (zp) {
                        gxB = pml_e<2>(a, 0, kk, i, j, kk, gxB);
                        gyA = pml_e<2>(a, 1, kk, i, j, kk, gyA);
                    }
                    if (xpml) {
                        gyB = pml_e<0>(a, 0, i, i, j, kk, gyB);
                        gzA = pml_e<0>(a, 1, i, i, j, kk, gzA);
                    }
                }
                float cx = gxA - gxB, cy = gyA - gyB, cz = gzA - gzB;
                if (a.pw_on) {
                    const int cd = a.pw_d == 0 ? i : a.pw_d == 1 ? j : kk;
                    const int cp = a.pw_p == 0 ? i : a.pw_p == 1 ? j : kk;
                    const int ct = a.pw_t == 0 ? i : a.pw_t == 1 ? j : kk;
                    cx += tfsf_e(a, 0, cd, cp, ct);
                    cy += tfsf_e(a, 1, cd, cp, ct);
                    cz += tfsf_e(a, 2, cd, cp, ct);
                }
                float dx_ = S * cx, dy_ = S * cy, dz_ = S * cz;
                double* sh = nullptr;  // FP64 shadow of E on source edges
                if (a.src_on && in_box(i, j, kk, a.slo, a.sdim)) {
                    const int ci = box_index(i, j, kk, a.slo, a.sdim);
                    if (a.n < a.snsteps) {
                        const float* s = a.src + ((long long)a.n * a.sncell + ci) * 3;
                        dx_ -= s[0];
                        dy_ -= s[1];
                        dz_ -= s[2];
                    }
                    if (a.ssh) sh = a.ssh + (long long)ci * 3;
                }
                const float e0x = ex[r], e0y = ey[r], e0z = ez[r];
                float nxv, nyv, nzv;
                if (PMAX >= 0 && a.nd > 0 && in_box(i, j, kk, a.dlo, a.ddim)) {
                    const long long v = box_index(i, j, kk, a.dlo, a.ddim);
                    const float rho = a.rho[v];
                    float Tx, Ty, Tz;
                    nxv = e_disp<0, PMAX>(a, e0x, dx_, rho, v, &Tx, sh);
                    nyv = e_disp<1, PMAX>(a, e0y, dy_, rho, v, &Ty, sh ? sh + 1 : nullptr);
                    nzv = e_disp<2, PMAX>(a, e0z, dz_, rho, v, &Tz, sh ? sh + 2 : nullptr);
                    if (j == 0 || kk == 0) nxv = 0.f;  // never inside a valid design box
                    if (a.Tout) {
                        a.Tout[v] = Tx;
                        a.Tout[a.nd + v] = Ty;
                        a.Tout[2 * a.nd + v] = Tz;
                    }
                    if (a.Tin) {
                        const double g = (double)nxv * a.Tin[v] + (double)nyv * a.Tin[a.nd + v] +
                                         (double)nzv * a.Tin[2 * a.nd + v];
                        a.grad[v] += g;
                    }
                } else if (sh) {
                    sh[0] += (double)dx_;
                    sh[1] += (double)dy_;
                    sh[2] += (double)dz_;
                    nxv = (float)sh[0];
                    nyv = (float)sh[1];
                    nzv = (float)sh[2];
                } else {
                    nxv = e0x + dx_;
                    nyv = e0y + dy_;
                    nzv = e0z + dz_;
                }
                // tangential E on the walls stays zero
                if (j == 0 || kk == 0) nxv = 0.f;
                if (i == 0 || kk == 0) nyv = 0.f;
                if (i == 0 || j == 0) nzv = 0.f;
                a.Eo[0][o] = nxv;
                a.Eo[1][o] = nyv;
                a.Eo[2][o] = nzv;
                if (a.gap_on && in_box(i, j, kk, a.glo, a.gdim)) {
                    float* g = a.gap + ((long long)(a.n + 1) * a.gncell + box_index(i, j, kk, a.glo, a.gdim)) * 3;
                    g[0] = nxv;
                    g[1] = nyv;
                    g[2] = nzv;
                }
            }
        }

        // ---- rotate registers
#pragma unroll
        for (int r = 0; r <= R; ++r) { hxm[r] = hx[r]; hym[r] = hy[r]; }
#pragma unroll
        for (int r = 0; r < R + 2; ++r) { ex[r] = nex[r]; ey[r] = ney[r]; ez[r] = nez[r]; }
    }
}

__global__ void fill_kernel(float* p, long long n, float v)
{
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x)
        p[t] = v;
}

__global__ void fill_d_kernel(double* p, long long n, double v)
{
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x)
        p[t] = v;
}

__global__ void copy_kernel(float* __restrict__ d, const float* __restrict__ s, long long n)
{
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x)
        d[t] = s[t];
}

__global__ void scale_kernel(float* __restrict__ d, const float* __restrict__ s, long long n, float f)
{
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x)
        d[t] = s[t] * f;
}

__global__ void grad_out_kernel(double* __restrict__ d, const double* __restrict__ acc, long long n,
                                double f)
{
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x)
        d[t] = acc[t] * f;
}

__global__ void copy_d_kernel(double* __restrict__ d, const double* __restrict__ s, long long n)
{
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x)
        d[t] = s[t];
}

// Exact 1-D auxiliary FDTD line for the TF/SF plane wave (same dx, dt and
// Courant number as the 3-D grid, so an axis-aligned plane wave matches the
// 3-D Yee update exactly).  One workgroup; FP64; hard source E[0] = wave[n].
// Writes incE row n = E^n at 3-D positions [lo_d, hi_d] and incH row n =
// H^{n+1/2} at 3-D positions [lo_d-1, hi_d] + 1/2.
__global__ void incident_line_kernel(const double* wave, int nw, int M, int L, double coef,
                                     int lo_d, int hi_d, int sgn, int ref, double* E, double* H,
                                     float* incE, float* incH)
{
    const int spanE = hi_d - lo_d + 1, spanH = hi_d - lo_d + 2;
    for (int u = threadIdx.x; u <= L; u += blockDim.x) { E[u] = 0.0; H[u] = 0.0; }
    __syncthreads();
    if (threadIdx.x == 0) E[0] = nw > 0 ? wave[0] : 0.0;
    __syncthreads();
    for (int n = 0; n <= M; ++n) {
        for (int q = threadIdx.x; q < spanE; q += blockDim.x) {
            const int u = sgn * (lo_d + q - ref);
            incE[(long long)n * spanE + q] = (float)E[u];
        }
        if (n == M) break;
        for (int u = threadIdx.x; u < L; u += blockDim.x) H[u] += coef * (E[u + 1] - E[u]);
        __syncthreads();
        for (int q = threadIdx.x; q < spanH; q += blockDim.x) {
            const int q3 = lo_d - 1 + q;
            const int u = sgn > 0 ? q3 - ref : ref - q3 - 1;
            incH[(long long)n * spanH + q] = (float)H[u];
        }
        for (int u = 1 + threadIdx.x; u < L; u += blockDim.x) E[u] += coef * (H[u] - H[u - 1]);
        __syncthreads();
        if (threadIdx.x == 0) E[0] = (n + 1 < nw) ? wave[n + 1] : 0.0;
        __syncthreads();
    }
}

// Objective from the gap history (one workgroup, FP64):
//  DFT:  D_e = sum_{n=0..M} E_e^n e^{-j w n dt};  F' = sum |D_e|^2;
//        scale = max |D_e|; adjoint drive r_{p,e} = Re{conj(D_e) e^{-j w (M-p) dt}}.
//  TIME: F' = sum_{n in window} sum_e (E_e^n)^2; scale = max |E| over the window;
//        adjoint drive r_{p,e} = E_e^{M-p} (M-p in the window).
// adj[p*ne + e] = r / scale; scal[0] = F', scal[1] = scale.
__global__ void objective_kernel(const float* gap, int M, int ne, int kind, double wdt, int nb,
                                 int nend, double* scal, double* work, float* adj)
{
    __shared__ double sF[1024], sM[1024];
    double f = 0.0, mx = 0.0;
    const int lo = nb < 0 ? 0 : nb, hi = nend > M + 1 ? M + 1 : nend;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        if (kind == 1) {
            double re = 0.0, im = 0.0;
            for (int n = 0; n <= M; ++n) {
                double s, c;
                sincos(wdt * n, &s, &c);
                const double v = gap[(long long)n * ne + e];
                re += v * c;
                im -= v * s;
            }
            work[2 * e] = re;
            work[2 * e + 1] = im;
            f += re * re + im * im;
            mx = fmax(mx, sqrt(re * re + im * im));
        } else {
            for (int n = lo; n < hi; ++n) {
                const double v = gap[(long long)n * ne + e];
                f += v * v;
                mx = fmax(mx, fabs(v));
            }
        }
    }
    sF[threadIdx.x] = f;
    sM[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sF[threadIdx.x] += sF[threadIdx.x + s];
            sM[threadIdx.x] = fmax(sM[threadIdx.x], sM[threadIdx.x + s]);
        }
        __syncthreads();
    }
    const double F = sF[0];
    const double sc = sM[0] > 0.0 ? sM[0] : 1.0;
    if (threadIdx.x == 0) { scal[0] = F; scal[1] = sc; }
    const long long tot = (long long)M * ne;
    for (long long t = threadIdx.x; t < tot; t += blockDim.x) {
        const int p = (int)(t / ne), e = (int)(t % ne);
        const int m = M - p;
        double r = 0.0;
        if (kind == 1) {
            double s, c;
            sincos(wdt * m, &s, &c);
            // Re{(re - j im)(c - j s)} = re c - im s
            r = work[2 * e] * c - work[2 * e + 1] * s;
        } else if (m >= lo && m < hi) {
            r = gap[(long long)m * ne + e];
        }
        adj[t] = (float)(r / sc);
    }
}

// Density check for device input: flag[0] = 1 if any value is non-finite or
// outside [0,1].
__global__ void check_rho_kernel(const float* rho, long long n, double* flag)
{
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x) {
        const float r = rho[t];
        if (!(r >= 0.f && r <= 1.f)) flag[0] = 1.0;
    }
}

int grid_for(long long n) { long long g = (n + 255) / 256; return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096); }

}  // namespace

int ccpr_launch_step(const StepArgs& a, int maxpairs, void* stream)
{
    const int threads = ((a.nx + 63) / 64) * 64;
    dim3 grid(a.nblk), block(threads);
    hipStream_t s = (hipStream_t)stream;
    if (maxpairs <= 0) hipLaunchKernelGGL(ccpr_step_kernel<0>, grid, block, 0, s, a);
    else if (maxpairs <= 1) hipLaunchKernelGGL(ccpr_step_kernel<1>, grid, block, 0, s, a);
    else if (maxpairs <= 2) hipLaunchKernelGGL(ccpr_step_kernel<2>, grid, block, 0, s, a);
    else if (maxpairs <= 3) hipLaunchKernelGGL(ccpr_step_kernel<3>, grid, block, 0, s, a);
    else if (maxpairs <= 4) hipLaunchKernelGGL(ccpr_step_kernel<4>, grid, block, 0, s, a);
    else if (maxpairs <= 6) hipLaunchKernelGGL(ccpr_step_kernel<6>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(ccpr_step_kernel<8>, grid, block, 0, s, a);
    return (int)hipGetLastError();
}

int ccpr_launch_fill(float* p, long long n, float v, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, p, n, v);
    return (int)hipGetLastError();
}

int ccpr_launch_fill_d(double* p, long long n, double v, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(fill_d_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, p, n, v);
    return (int)hipGetLastError();
}

int ccpr_launch_copy(float* d, const float* s, long long n, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, d, s, n);
    return (int)hipGetLastError();
}

int ccpr_launch_scale(float* d, const float* s, long long n, float f, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, d, s, n, f);
    return (int)hipGetLastError();
}

int ccpr_launch_copy_d(double* d, const double* s, long long n, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(copy_d_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, d, s, n);
    return (int)hipGetLastError();
}

int ccpr_launch_grad_out(double* d, const double* acc, long long n, double f, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(grad_out_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, d, acc,
                       n, f);
    return (int)hipGetLastError();
}

int ccpr_launch_incident_line(const double* wave, int nw, int M, int L, double coef, int lo_d,
                              int hi_d, int sgn, int ref, double* lineE, double* lineH,
                              float* incE, float* incH, void* stream)
{
    hipLaunchKernelGGL(incident_line_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, wave, nw,
                       M, L, coef, lo_d, hi_d, sgn, ref, lineE, lineH, incE, incH);
    return (int)hipGetLastError();
}

int ccpr_launch_objective(const float* gap, int M, int ne, int kind, double omega_dt, int nb,
                          int nend, double* scal, double* work, float* adj, void* stream)
{
    hipLaunchKernelGGL(objective_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, gap, M, ne,
                       kind, omega_dt, nb, nend, scal, work, adj);
    return (int)hipGetLastError();
}

int ccpr_launch_check_rho(const float* rho, long long n, double* flag, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(check_rho_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, rho, n,
                       flag);
    return (int)hipGetLastError();
}
