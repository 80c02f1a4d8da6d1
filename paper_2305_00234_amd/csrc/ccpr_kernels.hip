// gfx950 kernels of the CCPR-FDTD path.
//
// One leapfrog step -- H^{n-1/2} -> H^{n+1/2} (Faraday, supplement
// Eq. Maxwells2 c) and E^n -> E^{n+1} with the CCPR pole-pair currents
// (Eqs. Maxwells2 a, b; interpolation Eqs. eps_mixed, sigma_mixed,
// Poles_mixed) -- is a short sequence of launches:
//  - ccpr_pre_kernel: the x-CPML and TF/SF corrections of H^{n-1/2} (only
//    when the previous step's post launch did not already apply them);
//  - ccpr_step_kernel streams the whole grid once (every E and H word read
//    once and written once: 48 bytes per cell) with the vacuum update and the
//    y/z CPML memories, as two concurrent launches (tiles that touch a y or z
//    CPML layer, interior tiles).  For design and source cells it also stores
//    the E drive S curl H';
//  - ccpr_aux_kernel, one thread per cell of the design box (a per-edge
//    design's box of N + 1 cells, each edge with its own density), redoes
//    those cells' E update from E^n and the drive: CCPR pole-pair currents,
//    source current, the forward gradient record and the adjoint gradient
//    correlation (Eq. Gradient_FDTD, or the running transforms of the
//    DFT-mode estimator), and the gap monitor;
//  - ccpr_post_kernel: the x-CPML correction of E^{n+1}, the source and gap
//    cells outside the design and the TF/SF E faces; ccpr_post_fused_kernel
//    does the same and also the next step's pre work when that step follows
//    at once;
//  - watch_kernel (every few steps when the divergence watchdog is on):
//    checks the gap box and sets a halt word that every step kernel reads
//    first.
// Keeping the dispersive work and the x layers out of the grid kernel keeps
// its loop at the register and instruction budget of a plain Yee update.
// Options: ccpr_step_des_kernel runs the interior tiles that own design cells
// with the aux kernel's update fused into their z-march (slower on the
// workloads measured, off by default); the ccpr_batch_*_kernel launches run
// the same bodies for up to CCPR_BATCH_MAX solves of one padded x width
// (serving engine).
//
// Grid kernel decomposition (memory-bound stencil, no MFMA):
//  - a workgroup spans the whole x extent (blockDim = nx rounded up to 64),
//    so x-neighbours come from DPP wave shifts plus one LDS word per wave seam;
//  - each thread owns R consecutive y rows (register blocking) and the
//    workgroup marches over a chunk of z-planes, keeping the previous plane's
//    new H and the next plane's old E in registers;
//  - H^{n+1/2} is recomputed on one halo row (y = j0-1) and one halo plane
//    (z = k0-1) so the E update never waits on another workgroup.  E, H and
//    the H-side CPML memories are therefore double-buffered (read old, write
//    new); pole currents and E-side CPML memories are touched only by their
//    owner and are updated in place;
//  - workgroups are numbered so that each XCD gets a contiguous run of
//    tiles: neighbouring y-strips share their halo rows in the same L2.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "ccpr_internal.h"

namespace {

__device__ __forceinline__ bool in_box(int i, int j, int k, const int* lo, const int* dim)
{
    return (unsigned)(i - lo[0]) < (unsigned)dim[0] && (unsigned)(j - lo[1]) < (unsigned)dim[1] &&
           (unsigned)(k - lo[2]) < (unsigned)dim[2];
}

__device__ __forceinline__ int box_index(int i, int j, int k, const int* lo, const int* dim)
{
    return ((k - lo[2]) * dim[1] + (j - lo[1])) * dim[0] + (i - lo[0]);
}

// Dispersive E update of component C at design voxel v (see ccpr_internal.h),
// on currents already in registers: jr/ji hold J^n on entry and J^{n+1} on
// exit.  sh (may be null): FP64 shadow of E on a source edge; E^{n+1} is then
// accumulated in FP64 and rounded once, and the new shadow value returned in
// *shn for the caller to store (no store here: the material constants of the
// later components then stay scalar loads).
template <int C, int PMAX>
__device__ __forceinline__ float e_disp(const StepCold& c, float E, float drive, float rho, float* jr,
                                        float* ji, float* T, const double* sh, double* shn)
{
    const AxisMat& m = c.mat[C];
    const double r = rho, om = 1.0 - r;
    const double sig = fma(r, m.dsig, m.sig1) + r * om * m.gam;
    double A = fma(r, m.deps, m.eps1) + sig;
    double num = fma(-2.0 * sig, (double)E, (double)drive);
    float rold = 0.f;
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        if (p < m.np) {
            const double kap = p < m.np1 ? om : r;
            A = fma(kap, m.brd[p], A);
            // num -= kap Re{(1 + k_p) J} with 1 + k_p = 2 + (k_p - 1)
            num = fma(-kap, fma(2.0 + m.krd[p], (double)jr[p], -m.kid[p] * (double)ji[p]), num);
            rold += p < m.np1 ? -jr[p] : jr[p];
        }
    }
    // 1/A: FP32 reciprocal refined by one Newton step (FP64 accurate)
    double ra = (double)(1.0f / (float)A);
    ra = ra * fma(-A, ra, 2.0);
    const double inc = num * ra;
    float En;
    if (sh) { *shn = *sh + inc; En = (float)*shn; }
    else En = (float)((double)E + inc);
    const float dE = En - E;
    float rnew = 0.f;
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        if (p < m.np) {
            // J^{n+1} = J + (k_p - 1) J + beta'_p dE
            // (FP64 arithmetic, one rounding to the FP32 store)
            const double jrd = jr[p], jid = ji[p], dEd = dE;
            jr[p] = (float)(jrd + fma(m.krd[p], jrd, fma(-m.kid[p], jid, m.brd[p] * dEd)));
            ji[p] = (float)(jid + fma(m.krd[p], jid, fma(m.kid[p], jrd, m.bid[p] * dEd)));
            rnew += p < m.np1 ? -jr[p] : jr[p];
        }
    }
    const float rf = rho;
    *T = fmaf(m.depsf, dE, fmaf(m.dsigf + (1.f - 2.f * rf) * m.gamf, En + E, rnew + rold));
    return En;
}

// Store of a value that is not read again within the step.  When the state
// is larger than the last-level cache (StepArgs::stream_st, set by the host)
// it is written with a nontemporal store: the state then streams through HBM
// once per step, and keeping these writes out of the caches leaves them to the
// reads (measured: 670 -> 643 us per step on the 320^3 gold workload).  Small
// states that fit in the cache keep ordinary stores.  The choice is a
// template parameter: a run-time flag lets the compiler merge the two stores
// into one ordinary store before the flag is known.
template <bool NT>
__device__ __forceinline__ void st_stream(float* p, float v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Pole currents of component C at voxel v: load / store (pairs p < np;
// on = false: the edge has no currents, all zero).
template <int C, int PMAX>
__device__ __forceinline__ void j_load(const StepCold& c, long long v, float* jr, float* ji, bool on = true)
{
    const AxisMat& m = c.mat[C];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        jr[p] = 0.f;
        ji[p] = 0.f;
        if (on && p < m.np) {
            const long long q = m.jofs + p;
            jr[p] = c.J[(2 * q) * c.nd + v];
            ji[p] = c.J[(2 * q + 1) * c.nd + v];
        }
    }
}
template <int C, int PMAX, bool NT>
__device__ __forceinline__ void j_store(const StepCold& c, long long v, const float* jr, const float* ji)
{
    const AxisMat& m = c.mat[C];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        if (p < m.np) {
            const long long q = m.jofs + p;
            st_stream<NT>(&c.J[(2 * q) * c.nd + v], jr[p]);
            st_stream<NT>(&c.J[(2 * q + 1) * c.nd + v], ji[p]);
        }
    }
}

// x-neighbour exchange on the 64 lanes of a wave (DPP wave shifts, one VALU
// op each): lane i receives lane i+1 (shl) / lane i-1 (shr); the lane at the
// wave seam receives 'edge' instead.
__device__ __forceinline__ float from_right(float v, float edge)
{
    return __builtin_amdgcn_update_dpp(edge, v, 0x130, 0xf, 0xf, false);  // wave_shl:1
}
__device__ __forceinline__ float from_left(float v, float edge)
{
    return __builtin_amdgcn_update_dpp(edge, v, 0x138, 0xf, 0xf, false);  // wave_shr:1
}


// 32-bit byte offsets from a uniform base: lets the compiler use the
// SGPR-base + VGPR-offset addressing form (no 64-bit address math per access).
__device__ __forceinline__ float ldf(const float* base, unsigned boff)
{
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + boff);
}
__device__ __forceinline__ void stf(float* base, unsigned boff, float v)
{
    *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + boff) = v;
}
// st_stream at a byte offset from a field base.
template <bool NT>
__device__ __forceinline__ void stf_nt(float* base, unsigned boff, float v)
{
    st_stream<NT>(reinterpret_cast<float*>(reinterpret_cast<char*>(base) + boff), v);
}

// Component c of a field buffer (components npad floats = cs bytes apart).
// The base is formed in 64-bit arithmetic (uniform, scalar registers), so the
// per-lane byte offsets of ldf / stf stay 32-bit within one component: a
// component may hold up to 2^30 floats.
__device__ __forceinline__ const float* fcomp(const float* base, unsigned cs, int c)
{
    return reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (size_t)cs * (size_t)c);
}
__device__ __forceinline__ float* fcomp(float* base, unsigned cs, int c)
{
    return reinterpret_cast<float*>(reinterpret_cast<char*>(base) + (size_t)cs * (size_t)c);
}
// Field word at a 64-bit byte offset (TF/SF face list).
__device__ __forceinline__ float* fword(const float* base, unsigned long long boff)
{
    return reinterpret_cast<float*>(const_cast<char*>(reinterpret_cast<const char*>(base)) + boff);
}

// CPML memory update on one derivative d with the (prefetched) old memory p:
// p' = b p + a d (stored by the owner only); returns d/kappa + p'.
__device__ __forceinline__ float cpml(float d, float4 cf, float p, float* pout, unsigned idx, bool store)
{
    const float q = fmaf(cf.x, p, cf.y * d);
    if (store) pout[idx] = q;
    return fmaf(d, cf.z, q);
}

template <int PMAX, bool NT, bool DFT, bool EDGE, bool REG>
__device__ __forceinline__ void design_cell(const StepArgs& a, const long long v, const int i, const int j,
                                            const int kk, const unsigned o, const float* e_in,
                                            const float* d_in);

// Fused leapfrog step over the whole grid: vacuum update of H and E with the
// y and z CPML.  For design and source cells the E drive S (curl H) is also
// stored; ccpr_aux_kernel then finishes those cells and the TF/SF E faces.
// DP >= 0 (interior tiles that own design cells, per-voxel designs, the
// time-exact gradient): the design cells' CCPR update runs here instead, on
// E^n and the drive still in registers (design_cell with at most DP pole
// pairs per axis), and no drive is stored for them.
// The x CPML and the TF/SF H faces are applied to H^{n-1/2} beforehand by
// ccpr_pre_kernel, the x CPML of E^{n+1} afterwards by ccpr_post_kernel: the
// x layers then cost no extra work inside the x-spanning workgroup.
// R = 2 rows per thread for any nx (blockDim up to 1024); R = 4 keeps more
// rows in registers and is limited to blockDim <= 512.  PML = false is the
// variant for tiles that touch no y or z CPML layer (no CPML code at all);
// PML = true fetches the tile's CPML memories together with the fields at the
// top of every plane.  The two variants run concurrently on their own tile
// lists.  NT: nontemporal stores of the new fields (large states).
// Tile L of a.tiles (the body of ccpr_step_kernel and of the batched grid
// kernel); xe, xh: the workgroup's LDS words at the wave seams.
template <int R, bool PML, bool NT, int DP = -1>
__device__ __forceinline__ void grid_tile(const StepArgs& a, const int L, float (*xe)[R + 1][16],
                                          float (*xh)[R][16])
{
    const StepCold& c = *a.cold;
    // Logical z-chunk zl covers planes zr[zl] = [k0, k1): the host sizes
    // chunks to equal work (CPML planes cost more) and spreads them over the
    // XCDs.
    const int2 tile = a.tiles[L];  // (y-strip, logical z-chunk)
    const int ys = tile.x;
    const int2 kr = a.zr[tile.y];
    const int j0 = ys * R;
    const int k0 = kr.x, k1 = kr.y;

    const int i = threadIdx.x;
    const int lane = i & 63;
    const int w = __builtin_amdgcn_readfirstlane(i >> 6);
    const int nw = blockDim.x >> 6;
    const bool xin = i < a.nx;
    const float S = a.S;
    const unsigned nxp = a.nxp, nyp = a.nyp, cs = a.cstride;
    const int npml = a.npml;
    const int ny = a.ny, nz = a.nz;
    const unsigned lf = a.lanef[i];
    const bool anypml = PML && npml > 0;
    const unsigned np2 = 2u * (unsigned)npml;
    const unsigned szy = (unsigned)nz * np2 * nxp;
    const unsigned szz = np2 * ny * nxp;
    // CPML memory and coefficient pointers, read once before the first store
    // (scalar loads of global pointers; reloaded inside the loop they would
    // be vector loads and flat accesses)
    const float* const pyHi = c.psiH[a.psi_in][1];
    const float* const pzHi = c.psiH[a.psi_in][2];
    float* const pyHo = c.psiH[a.psi_in ^ 1][1];
    float* const pzHo = c.psiH[a.psi_in ^ 1][2];
    float* const pyE = c.psiE[1];
    float* const pzE = c.psiE[2];
    const float4* const cfHy = c.pmlH[1];
    const float4* const cfHz = c.pmlH[2];
    const float4* const cfEy = c.pmlE[1];
    const float4* const cfEz = c.pmlE[2];

    auto poff = [&](int k, int r) -> unsigned {
        return (((unsigned)(k + 1) * nyp + (unsigned)(j0 + r)) * nxp + (unsigned)i) * 4u;
    };
    auto yidx = [&](int k, int j) -> unsigned {
        const int ysl = j < npml ? j : j - (ny - npml) + npml;
        return ((unsigned)k * np2 + ysl) * nxp + i;
    };
    auto zidx = [&](int k, int j) -> unsigned {
        const int zsl = k < npml ? k : k - (nz - npml) + npml;
        return ((unsigned)zsl * ny + j) * nxp + i;
    };

    float ex[R + 2], ey[R + 2], ez[R + 2];     // E^n, plane kk
    float nex[R + 2], ney[R + 2], nez[R + 2];  // E^n, plane kk+1
    float hxm[R + 1], hym[R + 1];              // H^{n+1/2}, plane kk-1
    float hx[R + 1], hy[R + 1], hz[R + 1];     // H^{n+1/2}, plane kk

#pragma unroll
    for (int r = 0; r < R + 2; ++r) {
        const unsigned o = poff(k0 - 1, r);
        ex[r] = ldf(a.Ei, o);
        ey[r] = ldf(fcomp(a.Ei, cs, 1), o);
        ez[r] = ldf(fcomp(a.Ei, cs, 2), o);
    }
#pragma unroll
    for (int r = 0; r <= R; ++r) { hxm[r] = 0.f; hym[r] = 0.f; }

    for (int kk = k0 - 1; kk < k1; ++kk) {
        // ---- loads: E^n of plane kk+1, H^{n-1/2} of plane kk (ghost rows and
        // planes are zero).  Two words of the z halo are never used and not
        // read: Ez of plane k1 (the last H update takes only the z-differences
        // of Ex and Ey) and Hz of the halo plane k0-1 (the first E update
        // takes only Hx and Hy from below).
        float hxo[R + 1], hyo[R + 1], hzo[R + 1];
        const bool zlast = kk + 1 >= k1, zhalo = kk < k0;  // uniform
#pragma unroll
        for (int r = 0; r < R + 2; ++r) {
            const unsigned o = poff(kk + 1, r);
            nex[r] = ldf(a.Ei, o);
            ney[r] = ldf(fcomp(a.Ei, cs, 1), o);
            nez[r] = zlast ? 0.f : ldf(fcomp(a.Ei, cs, 2), o);
        }
#pragma unroll
        for (int r = 0; r <= R; ++r) {
            const unsigned o = poff(kk, r);
            hxo[r] = ldf(a.Hi, o);
            hyo[r] = ldf(fcomp(a.Hi, cs, 1), o);
            hzo[r] = zhalo ? 0.f : ldf(fcomp(a.Hi, cs, 2), o);
        }

        // ---- row classes of this plane.  Row r is H row j0-1+r; E rows are r = 1..R.
        bool rowv[R + 1];
        unsigned rf[R + 1];
#pragma unroll
        for (int r = 0; r <= R; ++r) {
            const int j = j0 - 1 + r;
            rowv[r] = j >= 0 && j < ny && kk >= 0;
            rf[r] = rowv[r] ? a.rowf[(unsigned)kk * ny + j] : 0u;
        }
        // ---- CPML memories of this plane (PML variant), fetched with the fields
        float pyh[R + 1][2], pzh[R + 1][2], pye[R + 1][2], pze[R + 1][2];
        if (anypml) {
            const bool ecur = kk >= k0;
#pragma unroll
            for (int r = 0; r <= R; ++r) {
                const int j = j0 - 1 + r;
                pyh[r][0] = pyh[r][1] = pzh[r][0] = pzh[r][1] = 0.f;
                pye[r][0] = pye[r][1] = pze[r][0] = pze[r][1] = 0.f;
                if (rf[r] & CCPR_ROW_YPML) {
                    const unsigned y = yidx(kk, j);
                    pyh[r][0] = pyHi[szy + y];
                    pyh[r][1] = pyHi[y];
                    if (r >= 1 && ecur) {
                        pye[r][0] = pyE[szy + y];
                        pye[r][1] = pyE[y];
                    }
                }
                if (rf[r] & CCPR_ROW_ZPML) {
                    const unsigned z = zidx(kk, j);
                    pzh[r][0] = pzHi[z];
                    pzh[r][1] = pzHi[szz + z];
                    if (r >= 1 && ecur) {
                        pze[r][0] = pzE[z];
                        pze[r][1] = pzE[szz + z];
                    }
                }
            }
        }

        // ---- E^n at x+1 (Ey, Ez on rows 0..R)
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r <= R; ++r) { xe[0][r][w] = ey[r]; xe[1][r][w] = ez[r]; }
        }
        __syncthreads();
        float eyr[R + 1], ezr[R + 1];
        const bool has_right = w + 1 < nw;
#pragma unroll
        for (int r = 0; r <= R; ++r) {
            eyr[r] = from_right(ey[r], has_right ? xe[0][r][w + 1] : 0.f);
            ezr[r] = from_right(ez[r], has_right ? xe[1][r][w + 1] : 0.f);
        }

        // ---- H^{n+1/2} on rows j0-1 .. j0+R-1 of plane kk
#pragma unroll
        for (int r = 0; r <= R; ++r) {
            const int j = j0 - 1 + r;
            const bool own = rowv[r] && r >= 1 && kk >= k0;    // uniform
            // Hx: y-derivative of Ez minus z-derivative of Ey; Hy: z of Ex minus
            // x of Ez; Hz: x of Ey minus y of Ex -- forward differences
            float dxA = ez[r + 1] - ez[r], dxB = ney[r] - ey[r];
            float dyA = nex[r] - ex[r], dyB = ezr[r] - ez[r];
            float dzA = eyr[r] - ey[r], dzB = ex[r + 1] - ex[r];
            if (anypml) {
                if (rf[r] & CCPR_ROW_YPML) {
                    const float4 cf = cfHy[j];
                    const unsigned y = yidx(kk, j);
                    dxA = cpml(dxA, cf, pyh[r][0], pyHo, szy + y, own && xin);
                    dzB = cpml(dzB, cf, pyh[r][1], pyHo, y, own && xin);
                }
                if (rf[r] & CCPR_ROW_ZPML) {
                    const float4 cf = cfHz[kk];
                    const unsigned z = zidx(kk, j);
                    dxB = cpml(dxB, cf, pzh[r][0], pzHo, z, own && xin);
                    dyA = cpml(dyA, cf, pzh[r][1], pzHo, szz + z, own && xin);
                }
            }
            hx[r] = fmaf(-S, dxA - dxB, hxo[r]);
            hy[r] = fmaf(-S, dyA - dyB, hyo[r]);
            hz[r] = fmaf(-S, dzA - dzB, hzo[r]);
            if (own && xin) {
                const unsigned o = poff(kk, r);
                stf_nt<NT>(a.Ho, o, hx[r]);
                stf_nt<NT>(fcomp(a.Ho, cs, 1), o, hy[r]);
                stf_nt<NT>(fcomp(a.Ho, cs, 2), o, hz[r]);
            }
        }

        // ---- H^{n+1/2} at x-1 (Hy, Hz on rows 1..R)
        if (lane == 63) {
#pragma unroll
            for (int r = 1; r <= R; ++r) { xh[0][r - 1][w] = hy[r]; xh[1][r - 1][w] = hz[r]; }
        }
        __syncthreads();
        float hyl[R + 1], hzl[R + 1];
#pragma unroll
        for (int r = 1; r <= R; ++r) {
            hyl[r] = from_left(hy[r], w > 0 ? xh[0][r - 1][w - 1] : 0.f);
            hzl[r] = from_left(hz[r], w > 0 ? xh[1][r - 1][w - 1] : 0.f);
        }

        // ---- E^{n+1} on rows j0 .. j0+R-1 of plane kk
        if (kk >= k0) {
#pragma unroll
            for (int r = 1; r <= R; ++r) {
                const int j = j0 - 1 + r;
                if (j >= ny) continue;  // uniform
                // (curl H)_x: y-derivative of Hz minus z-derivative of Hy;
                // (curl H)_y: z of Hx minus x of Hz; (curl H)_z: x of Hy minus
                // y of Hx -- backward differences
                float gxA = hz[r] - hz[r - 1], gxB = hy[r] - hym[r];
                float gyA = hx[r] - hxm[r], gyB = hz[r] - hzl[r];
                float gzA = hy[r] - hyl[r], gzB = hx[r] - hx[r - 1];
                if (anypml) {
                    if (rf[r] & CCPR_ROW_YPML) {
                        const float4 cf = cfEy[j];
                        const unsigned y = yidx(kk, j);
                        gxA = cpml(gxA, cf, pye[r][0], pyE, szy + y, xin);
                        gzB = cpml(gzB, cf, pye[r][1], pyE, y, xin);
                    }
                    if (rf[r] & CCPR_ROW_ZPML) {
                        const float4 cf = cfEz[kk];
                        const unsigned z = zidx(kk, j);
                        gxB = cpml(gxB, cf, pze[r][0], pzE, z, xin);
                        gyA = cpml(gyA, cf, pze[r][1], pzE, szz + z, xin);
                    }
                }
                const float dx_ = S * (gxA - gxB), dy_ = S * (gyA - gyB), dz_ = S * (gzA - gzB);
                float nxv = ex[r] + dx_, nyv = ey[r] + dy_, nzv = ez[r] + dz_;
                // tangential E on the walls stays zero
                if (j == 0 || kk == 0) nxv = 0.f;
                if (kk == 0) nyv = 0.f;
                if (j == 0) nzv = 0.f;
                if (i == 0) { nyv = 0.f; nzv = 0.f; }
                // design-box cells get their E^{n+1} from the aux kernel (which
                // reads E^n and the drive): no store here
                const bool des = (rf[r] & CCPR_ROW_DES) && (lf & CCPR_LANE_DES);
                if (xin && !des) {
                    const unsigned o = poff(kk, r);
                    stf_nt<NT>(a.Eo, o, nxv);
                    stf_nt<NT>(fcomp(a.Eo, cs, 1), o, nyv);
                    stf_nt<NT>(fcomp(a.Eo, cs, 2), o, nzv);
                }
                // design / source cells: hand the drive to the aux kernel
                // (or, DP >= 0, finish the design cell here)
                if (des) {
                    const long long v = box_index(i, j, kk, c.dlo, c.ddim);
                    if constexpr (DP >= 0) {
                        const float ein[3] = {ex[r], ey[r], ez[r]};
                        const float din[3] = {dx_, dy_, dz_};
                        design_cell<DP, NT, false, false, true>(a, v, i, j, kk, poff(kk, r), ein, din);
                    } else {
                        a.drive[v] = dx_;
                        a.drive[c.nd + v] = dy_;
                        a.drive[2 * c.nd + v] = dz_;
                    }
                } else if ((rf[r] & CCPR_ROW_SRC) && (lf & CCPR_LANE_SRC)) {
                    float* d = a.drive + 3 * c.nd + (long long)box_index(i, j, kk, c.slo, c.sdim) * 3;
                    d[0] = dx_;
                    d[1] = dy_;
                    d[2] = dz_;
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

template <int R, bool PML, bool NT>
__global__ __launch_bounds__(R == 2 ? 1024 : 512) void ccpr_step_kernel(const StepArgs a)
{
    __shared__ float xe[2][R + 1][16];
    __shared__ float xh[2][R][16];
    if (*a.halt) return;  // the divergence watchdog stopped the run
    // XCD-aware tile order: hardware hands workgroups to the 8 XCDs round
    // robin; give each XCD a contiguous range of the tile list (neighbouring
    // y-strips share halo rows in that XCD's L2).
    const int b = blockIdx.x;
    const int per = a.nblk >> 3, rem = a.nblk & 7;
    const int xcd = b & 7, q = b >> 3;
    grid_tile<R, PML, NT>(a, xcd * per + (xcd < rem ? xcd : rem) + q, xe, xh);
}

// Interior tiles that own design cells, with the design update fused in
// (R = 2; blockDim = nxp <= 512, which leaves the compiler up to 256 VGPRs).
template <bool NT, int DP>
__global__ __launch_bounds__(512) void ccpr_step_des_kernel(const StepArgs a)
{
    __shared__ float xe[2][3][16];
    __shared__ float xh[2][2][16];
    if (*a.halt) return;  // the divergence watchdog stopped the run
    const int b = blockIdx.x;
    const int per = a.nblk >> 3, rem = a.nblk & 7;
    const int xcd = b & 7, q = b >> 3;
    grid_tile<2, false, NT, DP>(a, xcd * per + (xcd < rem ? xcd : rem) + q, xe, xh);
}

// Finish the design voxels the fused step left to it, one thread per voxel:
// CCPR pole-pair update of the three E edges from E^n and the stored drive
// (minus a source current if the voxel is also a source cell), the gradient
// record (forward) or correlation (adjoint), and the gap monitor.  E^{n+1} of
// these cells is written over the fused kernel's vacuum value.
// Design voxels, one thread per voxel in box order (x fastest).  NT:
// nontemporal stores of the currents, fields and history (large states).
// E update of an edge of the kernel box that is not a design edge (the far
// face of a per-edge design along the edge's own axis): vacuum, E += drive.
__device__ __forceinline__ float e_vac(float E, float drive, const double* sh, double* shn)
{
    if (sh) {
        *shn = *sh + (double)drive;
        return (float)*shn;
    }
    return E + drive;
}

// Density / gradient index of component C at box cell (xi, yi, zi) of a
// per-edge design, or -1 where C has no design edge.
template <int C>
__device__ __forceinline__ long long edge_index(const EdgeMap& m, int xi, int yi, int zi)
{
    const int* b = m.ebox[C];
    if (xi >= b[0] || yi >= b[1] || zi >= b[2]) return -1;
    return m.eoff[C] + ((long long)zi * b[1] + yi) * b[0] + xi;
}

// Design-box cell v = (i, j, kk) (box index, x fastest; o: byte offset of
// its field words): the CCPR update of its three E edges, the pole currents,
// the gradient record / correlation or DFT accumulation, the source shadow
// and the gap monitor.  REG = false: E^n and the drive S (curl H) come from
// memory (ccpr_aux_kernel, after the grid pass stored the drive); REG = true:
// from the caller's registers e_in, d_in (the grid pass with the design
// update fused in).  The arithmetic is the same either way.
template <int PMAX, bool NT, bool DFT, bool EDGE, bool REG>
__device__ __forceinline__ void design_cell(const StepArgs& a, const long long v, const int i, const int j,
                                            const int kk, const unsigned o, const float* e_in,
                                            const float* d_in)
{
    const StepCold& c = *a.cold;
    const unsigned cs = a.cstride;
    const int n = a.n;
    // every load first (the current stores alias the later loads otherwise)
    constexpr int PN = PMAX > 0 ? PMAX : 1;
    // design edges of this cell: per voxel all three share the voxel's
    // density and gradient; per edge each has its own index (-1: not a
    // design edge)
    long long gx = v, gy = v, gz = v;
    if constexpr (EDGE) {
        const int xi = i - c.dlo[0], yi = j - c.dlo[1], zi = kk - c.dlo[2];
        gx = edge_index<0>(c.em, xi, yi, zi);
        gy = edge_index<1>(c.em, xi, yi, zi);
        gz = edge_index<2>(c.em, xi, yi, zi);
    }
    const bool onx = !EDGE || gx >= 0, ony = !EDGE || gy >= 0, onz = !EDGE || gz >= 0;
    float jrx[PN], jix[PN], jry[PN], jiy[PN], jrz[PN], jiz[PN];
    j_load<0, PMAX>(c, v, jrx, jix, onx);
    j_load<1, PMAX>(c, v, jry, jiy, ony);
    j_load<2, PMAX>(c, v, jrz, jiz, onz);
    float e0x, e0y, e0z, dx_, dy_, dz_;
    if constexpr (REG) {
        e0x = e_in[0]; e0y = e_in[1]; e0z = e_in[2];
        dx_ = d_in[0]; dy_ = d_in[1]; dz_ = d_in[2];
    } else {
        e0x = ldf(a.Ei, o); e0y = ldf(fcomp(a.Ei, cs, 1), o); e0z = ldf(fcomp(a.Ei, cs, 2), o);
        dx_ = a.drive[v]; dy_ = a.drive[c.nd + v]; dz_ = a.drive[2 * c.nd + v];
    }
    float rhox, rhoy, rhoz;
    if constexpr (EDGE) {
        rhox = onx ? c.rho[gx] : 0.f;
        rhoy = ony ? c.rho[gy] : 0.f;
        rhoz = onz ? c.rho[gz] : 0.f;
    } else {
        rhox = rhoy = rhoz = c.rho[v];
    }
    float Tox = 0.f, Toy = 0.f, Toz = 0.f;
    double g0 = 0.0, g0y = 0.0, g0z = 0.0;
    float* Tslot = c.T + (long long)a.tslot * 3 * c.nd;
    if (a.mode & CCPR_MODE_CORREL) {
        Tox = Tslot[v];
        Toy = Tslot[c.nd + v];
        Toz = Tslot[2 * c.nd + v];
        if constexpr (EDGE) {
            if (onx) g0 = c.grad[gx];
            if (ony) g0y = c.grad[gy];
            if (onz) g0z = c.grad[gz];
        } else {
            g0 = c.grad[v];
        }
    }
    // DFT mode (DFT: the launch carries CCPR_MODE_DFT_T or _P): running
    // transforms (re, im per component) of T (forward) or of the adjoint E
    // (adjoint window)
    float* const dacc = c.T + ((a.mode & CCPR_MODE_DFT_P) ? 6 * c.nd : 0);
    float dq[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if constexpr (DFT) {
#pragma unroll
        for (int q = 0; q < 6; ++q) dq[q] = dacc[q * c.nd + v];
    }
    double* sh = nullptr;
    if (c.src_on && in_box(i, j, kk, c.slo, c.sdim)) {
        const int ci = box_index(i, j, kk, c.slo, c.sdim);
        if (n < c.snsteps) {
            const float* s = c.src + ((long long)n * c.sncell + ci) * 3;
            dx_ -= s[0];
            dy_ -= s[1];
            dz_ -= s[2];
        }
        if (c.ssh) sh = c.ssh + (long long)ci * 3;
    }
    float Tx = 0.f, Ty = 0.f, Tz = 0.f;
    double shn[3];
    float nxv, nyv, nzv;
    if (!EDGE || onx) nxv = e_disp<0, PMAX>(c, e0x, dx_, rhox, jrx, jix, &Tx, sh, &shn[0]);
    else nxv = e_vac(e0x, dx_, sh, &shn[0]);
    if (!EDGE || ony) nyv = e_disp<1, PMAX>(c, e0y, dy_, rhoy, jry, jiy, &Ty, sh ? sh + 1 : nullptr, &shn[1]);
    else nyv = e_vac(e0y, dy_, sh ? sh + 1 : nullptr, &shn[1]);
    if (!EDGE || onz) nzv = e_disp<2, PMAX>(c, e0z, dz_, rhoz, jrz, jiz, &Tz, sh ? sh + 2 : nullptr, &shn[2]);
    else nzv = e_vac(e0z, dz_, sh ? sh + 2 : nullptr, &shn[2]);
    if (sh) {
        sh[0] = shn[0];
        sh[1] = shn[1];
        sh[2] = shn[2];
    }
    if (!EDGE || onx) j_store<0, PMAX, NT>(c, v, jrx, jix);
    if (!EDGE || ony) j_store<1, PMAX, NT>(c, v, jry, jiy);
    if (!EDGE || onz) j_store<2, PMAX, NT>(c, v, jrz, jiz);
    stf_nt<NT>(a.Eo, o, nxv);
    stf_nt<NT>(fcomp(a.Eo, cs, 1), o, nyv);
    stf_nt<NT>(fcomp(a.Eo, cs, 2), o, nzv);
    if (a.mode & CCPR_MODE_RECORD) {
        st_stream<NT>(&Tslot[v], Tx);
        st_stream<NT>(&Tslot[c.nd + v], Ty);
        st_stream<NT>(&Tslot[2 * c.nd + v], Tz);
    }
    if (a.mode & CCPR_MODE_CORREL) {
        if constexpr (EDGE) {
            if (onx) c.grad[gx] = g0 + (double)nxv * Tox;
            if (ony) c.grad[gy] = g0y + (double)nyv * Toy;
            if (onz) c.grad[gz] = g0z + (double)nzv * Toz;
        } else {
            c.grad[v] = g0 + ((double)nxv * Tox + (double)nyv * Toy + (double)nzv * Toz);
        }
    }
    if constexpr (DFT) {
        // x exp(-j phase) = x (cos - j sin)
        const bool fwd = (a.mode & CCPR_MODE_DFT_T) != 0;
        const float x0 = fwd ? Tx : nxv, x1 = fwd ? Ty : nyv, x2 = fwd ? Tz : nzv;
        dacc[v] = fmaf(x0, a.phc, dq[0]);
        dacc[c.nd + v] = fmaf(-x0, a.phs, dq[1]);
        dacc[2 * c.nd + v] = fmaf(x1, a.phc, dq[2]);
        dacc[3 * c.nd + v] = fmaf(-x1, a.phs, dq[3]);
        dacc[4 * c.nd + v] = fmaf(x2, a.phc, dq[4]);
        dacc[5 * c.nd + v] = fmaf(-x2, a.phs, dq[5]);
    }
    if ((a.mode & CCPR_MODE_GAP) && in_box(i, j, kk, c.glo, c.gdim)) {
        float* g = c.gap + ((long long)(n + 1) * c.gncell + box_index(i, j, kk, c.glo, c.gdim)) * 3;
        g[0] = nxv;
        g[1] = nyv;
        g[2] = nzv;
    }
}

// Design-box cell t (x fastest): the body of ccpr_aux_kernel and of the
// batched aux kernel.
template <int PMAX, bool NT, bool DFT, bool EDGE>
__device__ __forceinline__ void aux_cell(const StepArgs& a, const unsigned t)
{
    const StepCold& c = *a.cold;
    if (t >= (unsigned)c.nd) return;
    const unsigned dx = c.ddim[0], dy = c.ddim[1];
    const unsigned row = t / dx;  // 32-bit: the design box holds < 2^31 voxels
    const int i = c.dlo[0] + (int)(t - row * dx);
    const int j = c.dlo[1] + (int)(row % dy);
    const int kk = c.dlo[2] + (int)(row / dy);
    const unsigned o = (((unsigned)(kk + 1) * a.nyp + (unsigned)(j + 1)) * a.nxp + (unsigned)i) * 4u;
    design_cell<PMAX, NT, DFT, EDGE, false>(a, (long long)t, i, j, kk, o, nullptr, nullptr);
}

template <int PMAX, bool NT, bool DFT, bool EDGE>
__global__ __launch_bounds__(256) void ccpr_aux_kernel(const StepArgs a)
{
    if (*a.halt) return;  // the divergence watchdog stopped the run
    aux_cell<PMAX, NT, DFT, EDGE>(a, blockIdx.x * blockDim.x + threadIdx.x);
}

// Cells outside the design box: source and gap cells (e in [0, nextra)),
// then the TF/SF E face words.  Runs in the post kernel's launch.
__device__ __forceinline__ void aux_misc(const StepArgs& a, long long e)
{
    const StepCold& c = *a.cold;
    const unsigned cs = a.cstride;
    const int n = a.n;
    if (e >= a.nextra) {
        // TF/SF E faces: E^{n+1} += coef*incH[n][m]
        const long long f = e - a.nextra;
        if (f < c.tf_nE) {
            const TfEntry q = c.tf[f];
            if (n < c.tf_rows) {
                float* w = fword(a.Eo, q.off);
                *w = *w + q.coef * c.incH[(long long)n * c.pw_spanH + q.m];
            }
        }
        return;
    }
    const int4 cell = a.extra[e];  // (i, j, k, CCPR_EXTRA_*)
    const int i = cell.x, j = cell.y, kk = cell.z;
    const unsigned o = (((unsigned)(kk + 1) * a.nyp + (unsigned)(j + 1)) * a.nxp + (unsigned)i) * 4u;
    float nxv, nyv, nzv;
    if (cell.w == CCPR_EXTRA_SOURCE) {
        const int ci = box_index(i, j, kk, c.slo, c.sdim);
        const float* d = a.drive + 3 * c.nd + (long long)ci * 3;
        float dx_ = d[0], dy_ = d[1], dz_ = d[2];
        if (n < c.snsteps) {
            const float* s = c.src + ((long long)n * c.sncell + ci) * 3;
            dx_ -= s[0];
            dy_ -= s[1];
            dz_ -= s[2];
        }
        double* sh = c.ssh + (long long)ci * 3;
        sh[0] += (double)dx_;
        sh[1] += (double)dy_;
        sh[2] += (double)dz_;
        nxv = (float)sh[0];
        nyv = (float)sh[1];
        nzv = (float)sh[2];
        // tangential E on the walls stays zero
        if (j == 0 || kk == 0) nxv = 0.f;
        if (i == 0 || kk == 0) nyv = 0.f;
        if (i == 0 || j == 0) nzv = 0.f;
        stf(a.Eo, o, nxv);
        stf(fcomp(a.Eo, cs, 1), o, nyv);
        stf(fcomp(a.Eo, cs, 2), o, nzv);
    } else {
        nxv = ldf(a.Eo, o);
        nyv = ldf(fcomp(a.Eo, cs, 1), o);
        nzv = ldf(fcomp(a.Eo, cs, 2), o);
    }
    if ((a.mode & CCPR_MODE_GAP) && in_box(i, j, kk, c.glo, c.gdim)) {
        float* g = c.gap + ((long long)(n + 1) * c.gncell + box_index(i, j, kk, c.glo, c.gdim)) * 3;
        g[0] = nxv;
        g[1] = nyv;
        g[2] = nzv;
    }
}

// Before step n: corrections to H^{n-1/2} (a.Hi) that turn the grid
// kernel's vacuum Faraday update into the full one.
//  - x CPML (threads [0, 2 npml ny nz)): with d the forward x-difference of
//    E^n, psi' = b psi + a d and d -> d/kappa + psi', so
//    Hy += S((1/kappa - 1) d(Ez) + psi'),  Hz -= S((1/kappa - 1) d(Ey) + psi');
//  - TF/SF H faces (the next tf_nH threads): H += coef*incE[n][m].
__global__ __launch_bounds__(256) void ccpr_pre_kernel(const StepArgs a, long long nxs)
{
    if (*a.halt) return;
    const StepCold& c = *a.cold;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    float* H = const_cast<float*>(a.Hi);
    const unsigned cs = a.cstride;
    if (t < nxs) {
        const int np2 = 2 * a.npml;
        const int xs = (int)(t % np2);
        const long long u = t / np2;
        const int j = (int)(u % a.ny), k = (int)(u / a.ny);
        const int i = xs < a.npml ? xs : a.nx - np2 + xs;
        const unsigned o = (((unsigned)(k + 1) * a.nyp + (unsigned)(j + 1)) * a.nxp + (unsigned)i) * 4u;
        const bool right = i + 1 < a.nx;
        const float dEz = (right ? ldf(fcomp(a.Ei, cs, 2), o + 4) : 0.f) - ldf(fcomp(a.Ei, cs, 2), o);
        const float dEy = (right ? ldf(fcomp(a.Ei, cs, 1), o + 4) : 0.f) - ldf(fcomp(a.Ei, cs, 1), o);
        const float4 cf = c.pmlH[0][i];
        const unsigned x = (unsigned)u * np2 + xs;
        const unsigned sz = (unsigned)a.nz * a.ny * np2;
        const float* pin = c.psiH[a.psi_in][0];
        float* pout = c.psiH[a.psi_in ^ 1][0];
        const float p0 = fmaf(cf.x, pin[x], cf.y * dEz);
        const float p1 = fmaf(cf.x, pin[sz + x], cf.y * dEy);
        pout[x] = p0;
        pout[sz + x] = p1;
        stf(fcomp(H, cs, 1), o, ldf(fcomp(H, cs, 1), o) + a.S * fmaf(cf.z - 1.f, dEz, p0));
        stf(fcomp(H, cs, 2), o, ldf(fcomp(H, cs, 2), o) - a.S * fmaf(cf.z - 1.f, dEy, p1));
        return;
    }
    const long long f = t - nxs;
    if (c.pw_on && f < c.tf_nH && a.n < c.tf_rows) {
        const TfEntry q = c.tf[c.tf_nE + f];
        float* w = fword(H, q.off);
        *w = *w + q.coef * c.incE[(long long)a.n * c.pw_spanE + q.m];
    }
}

// After step n (grid and aux kernels): the x CPML of E^{n+1} (a.Eo) from
// H^{n+1/2} (a.Ho) (threads [0, nxs)), and the cells of aux_misc (the next
// nmisc threads).  With d the backward x-difference of H:
//   Ey -= S((1/kappa - 1) d(Hz) + psi'),  Ez += S((1/kappa - 1) d(Hy) + psi').
// Tangential E on the walls stays zero.
__device__ __forceinline__ void post_cell(const StepArgs& a, const long long t, long long nxs, long long nmisc)
{
    const StepCold& c = *a.cold;
    if (t >= nxs) {
        if (t - nxs < nmisc) aux_misc(a, t - nxs);
        return;
    }
    const unsigned cs = a.cstride;
    const int np2 = 2 * a.npml;
    const int xs = (int)(t % np2);
    const long long u = t / np2;
    const int j = (int)(u % a.ny), k = (int)(u / a.ny);
    const int i = xs < a.npml ? xs : a.nx - np2 + xs;
    if (i == 0) return;
    const unsigned o = (((unsigned)(k + 1) * a.nyp + (unsigned)(j + 1)) * a.nxp + (unsigned)i) * 4u;
    const float dHz = ldf(fcomp(a.Ho, cs, 2), o) - ldf(fcomp(a.Ho, cs, 2), o - 4);
    const float dHy = ldf(fcomp(a.Ho, cs, 1), o) - ldf(fcomp(a.Ho, cs, 1), o - 4);
    const float4 cf = c.pmlE[0][i];
    const unsigned x = (unsigned)u * np2 + xs;
    const unsigned sz = (unsigned)a.nz * a.ny * np2;
    float* ps = c.psiE[0];
    const float p0 = fmaf(cf.x, ps[x], cf.y * dHz);
    const float p1 = fmaf(cf.x, ps[sz + x], cf.y * dHy);
    ps[x] = p0;
    ps[sz + x] = p1;
    if (k != 0) stf(fcomp(a.Eo, cs, 1), o, ldf(fcomp(a.Eo, cs, 1), o) - a.S * fmaf(cf.z - 1.f, dHz, p0));
    if (j != 0) stf(fcomp(a.Eo, cs, 2), o, ldf(fcomp(a.Eo, cs, 2), o) + a.S * fmaf(cf.z - 1.f, dHy, p1));
}

__global__ __launch_bounds__(256) void ccpr_post_kernel(const StepArgs a, long long nxs, long long nmisc)
{
    if (*a.halt) return;
    post_cell(a, (long long)blockIdx.x * blockDim.x + threadIdx.x, nxs, nmisc);
}

// After step n when step n+1 follows at once: the work of ccpr_post_kernel
// for step n and of ccpr_pre_kernel for step n+1 in one launch.  Blocks
// [0, nbx) hold whole x-layer rows (rpb rows of 2 npml cells each): first the
// x CPML of E^{n+1} exactly as ccpr_post_kernel, then, after a barrier, the x
// CPML pre-correction of H^{n+1/2} for step n+1 exactly as ccpr_pre_kernel,
// from the E^{n+1} values just finished (the neighbour at x+1 from LDS within
// the layer; the first cell past the low layer from memory, which no thread
// of this launch writes; zero past the high wall).  H^{n+1/2} of a row is
// read before the barrier and changed only after it, by its own cell.  The
// other blocks run the aux_misc cells of step n and the TF/SF H words of step
// n+1 (cells disjoint from the x layers and from each other).  NT: the x-layer
// words are written with nontemporal stores (large states; measured 553 ->
// 549 us per step at 320^3).
// Block blk (256 threads) of ccpr_post_fused_kernel and of the batched post
// kernel; se: the block's LDS exchange.
template <bool NT>
__device__ __forceinline__ void post_fused_block(const StepArgs& a, int rpb, long long nbx, long long nmisc,
                                                 long long ntfh, long long blk, float (*se)[256])
{
    const StepCold& c = *a.cold;
    const int tid = threadIdx.x;
    if (blk >= nbx) {
        const long long t = (blk - nbx) * blockDim.x + tid;
        if (t < nmisc) {
            aux_misc(a, t);
            return;
        }
        const long long f = t - nmisc;
        if (f < ntfh && a.n + 1 < c.tf_rows) {
            const TfEntry q = c.tf[c.tf_nE + f];
            float* w = fword(a.Ho, q.off);
            *w = *w + q.coef * c.incE[(long long)(a.n + 1) * c.pw_spanE + q.m];
        }
        return;
    }
    const unsigned cs = a.cstride;
    const int np2 = 2 * a.npml;
    const int rl = tid / np2, xs = tid - rl * np2;
    const long long u = blk * rpb + rl;  // row k*ny + j
    const bool valid = rl < rpb && u < (long long)a.ny * a.nz;
    const int j = (int)(u % a.ny), k = (int)(u / a.ny);
    const int i = xs < a.npml ? xs : a.nx - np2 + xs;
    const unsigned o = (((unsigned)(k + 1) * a.nyp + (unsigned)(j + 1)) * a.nxp + (unsigned)i) * 4u;
    const unsigned x = (unsigned)u * np2 + xs;
    const unsigned sz = (unsigned)a.nz * a.ny * np2;
    float hy = 0.f, hz = 0.f, ey = 0.f, ez = 0.f;
    // loads of the H pre-correction that nothing in this launch writes, issued
    // with the first phase's: the other H-side psi buffer, its coefficients
    // and, for the last cell of the low layer, E^{n+1} just inside the layer
    float4 cfh = make_float4(0.f, 0.f, 0.f, 0.f);
    float ph0 = 0.f, ph1 = 0.f, eyr = 0.f, ezr = 0.f;  // E^{n+1} at x+1 (zero past the high wall)
    if (valid) {
        cfh = c.pmlH[0][i];
        const float* pin = c.psiH[a.psi_in ^ 1][0];
        ph0 = pin[x];
        ph1 = pin[sz + x];
        if (xs == a.npml - 1) {
            eyr = ldf(fcomp(a.Eo, cs, 1), o + 4);
            ezr = ldf(fcomp(a.Eo, cs, 2), o + 4);
        }
        hy = ldf(fcomp(a.Ho, cs, 1), o);
        hz = ldf(fcomp(a.Ho, cs, 2), o);
        ey = ldf(fcomp(a.Eo, cs, 1), o);
        ez = ldf(fcomp(a.Eo, cs, 2), o);
        if (i > 0) {
            const float dHz = hz - ldf(fcomp(a.Ho, cs, 2), o - 4);
            const float dHy = hy - ldf(fcomp(a.Ho, cs, 1), o - 4);
            const float4 cf = c.pmlE[0][i];
            float* ps = c.psiE[0];
            const float p0 = fmaf(cf.x, ps[x], cf.y * dHz);
            const float p1 = fmaf(cf.x, ps[sz + x], cf.y * dHy);
            st_stream<NT>(&ps[x], p0);
            st_stream<NT>(&ps[sz + x], p1);
            if (k != 0) {
                ey = ey - a.S * fmaf(cf.z - 1.f, dHz, p0);
                stf_nt<NT>(fcomp(a.Eo, cs, 1), o, ey);
            }
            if (j != 0) {
                ez = ez + a.S * fmaf(cf.z - 1.f, dHy, p1);
                stf_nt<NT>(fcomp(a.Eo, cs, 2), o, ez);
            }
        }
        se[0][tid] = ey;
        se[1][tid] = ez;
    }
    __syncthreads();
    if (!valid) return;
    if (xs != a.npml - 1 && xs != np2 - 1) {
        eyr = se[0][tid + 1];
        ezr = se[1][tid + 1];
    }
    const float dEz = ezr - ez, dEy = eyr - ey;
    float* pout = c.psiH[a.psi_in][0];
    const float p0 = fmaf(cfh.x, ph0, cfh.y * dEz);
    const float p1 = fmaf(cfh.x, ph1, cfh.y * dEy);
    st_stream<NT>(&pout[x], p0);
    st_stream<NT>(&pout[sz + x], p1);
    stf_nt<NT>(fcomp(a.Ho, cs, 1), o, hy + a.S * fmaf(cfh.z - 1.f, dEz, p0));
    stf_nt<NT>(fcomp(a.Ho, cs, 2), o, hz - a.S * fmaf(cfh.z - 1.f, dEy, p1));
}

template <bool NT>
__global__ __launch_bounds__(256) void ccpr_post_fused_kernel(const StepArgs a, int rpb, long long nbx,
                                                              long long nmisc, long long ntfh)
{
    __shared__ float se[2][256];
    if (*a.halt) return;
    post_fused_block<NT>(a, rpb, nbx, nmisc, ntfh, blockIdx.x, se);
}

// ---- batched steps (serving engine): the same bodies as ccpr_step_kernel
// (CPML variant on every tile), ccpr_aux_kernel (time-exact, one density per
// voxel) and ccpr_post_fused_kernel / ccpr_post_kernel, each block taking
// its solve's StepArgs from the kernel argument.  No XCD tile remap: a
// solve's tiles are few.
__device__ __forceinline__ int batch_solve(const int* start, int n, int b)
{
    int s = 0;
    while (s + 1 < n && b >= start[s + 1]) ++s;
    return s;
}

template <bool NT>
__global__ __launch_bounds__(1024) void ccpr_batch_grid_kernel(const BatchArgs B)
{
    __shared__ float xe[2][3][16];
    __shared__ float xh[2][2][16];
    const int s = batch_solve(B.gstart, B.n, blockIdx.x);
    const StepArgs& a = B.a[s];
    if (*a.halt) return;
    grid_tile<2, true, NT>(a, (int)blockIdx.x - B.gstart[s], xe, xh);
}

template <int PMAX, bool NT>
__global__ __launch_bounds__(256) void ccpr_batch_aux_kernel(const BatchArgs B)
{
    const int s = batch_solve(B.astart, B.n, blockIdx.x);
    const StepArgs& a = B.a[s];
    if (*a.halt) return;
    aux_cell<PMAX, NT, false, false>(a, ((unsigned)blockIdx.x - (unsigned)B.astart[s]) * 256u + threadIdx.x);
}

template <bool NT>
__global__ __launch_bounds__(256) void ccpr_batch_post_kernel(const BatchArgs B)
{
    __shared__ float se[2][256];
    const int s = batch_solve(B.pstart, B.n, blockIdx.x);
    const StepArgs& a = B.a[s];
    if (*a.halt) return;
    const long long blk = (long long)blockIdx.x - B.pstart[s];
    if (B.fused[s]) post_fused_block<NT>(a, B.rpb[s], B.nbx[s], B.nmisc[s], B.ntfh[s], blk, se);
    else post_cell(a, blk * 256 + threadIdx.x, B.nxs[s], B.nmisc[s]);
}

// DFT-mode gradient of each design voxel (see ccpr_set_gradient_mode): the
// adjoint amplitude A_k = a - j b solves the window's least-squares normal
// equations [a; b] = inv [Re P_k; -Im P_k] (inverse i00 i01; i01 i11), and
// grad = sum_k Re{A_k W T_hat_k}, all in FP64.
// per voxel: grad[v] = sum over the three edges; per edge (em.on): each
// design edge's own term at its index
__global__ void dft_grad_kernel(double* grad, const float* acc, long long nd, int dx, int dy, const EdgeMap em,
                                double i00, double i01, double i11, double wc, double ws)
{
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nd;
         v += (long long)gridDim.x * blockDim.x) {
        double gk[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double tr = acc[(2 * k) * nd + v], ti = acc[(2 * k + 1) * nd + v];
            const double rc = acc[(6 + 2 * k) * nd + v], rs = -(double)acc[(7 + 2 * k) * nd + v];
            const double ar = i00 * rc + i01 * rs, ab = i01 * rc + i11 * rs;  // A = ar - j ab
            // A W = (ar wc + ab ws) + j (ar ws - ab wc)
            const double awr = ar * wc + ab * ws, awi = ar * ws - ab * wc;
            gk[k] = awr * tr - awi * ti;
        }
        if (em.on) {
            const int xi = (int)(v % dx), yi = (int)((v / dx) % dy), zi = (int)(v / ((long long)dx * dy));
            const long long e0 = edge_index<0>(em, xi, yi, zi), e1 = edge_index<1>(em, xi, yi, zi),
                            e2 = edge_index<2>(em, xi, yi, zi);
            if (e0 >= 0) grad[e0] = gk[0];
            if (e1 >= 0) grad[e1] = gk[1];
            if (e2 >= 0) grad[e2] = gk[2];
        } else {
            grad[v] = gk[0] + gk[1] + gk[2];
        }
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

// one component of the interior of a ghost-padded field, scaled:
// out[(k*ny+j)*nx+i]
__global__ void extract_kernel(float* __restrict__ d, const float* __restrict__ s, int comp, int nx,
                               int ny, int nz, int nxp, int nyp, float f)
{
    const long long n = (long long)nx * ny * nz;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(t % nx);
        const long long u = t / nx;
        const int j = (int)(u % ny), k = (int)(u / ny);
        d[t] = s[(long long)comp * nxp * nyp * (nz + 2) + ((long long)(k + 1) * nyp + (j + 1)) * nxp + i] * f;
    }
}

__global__ void grad_out_kernel(double* __restrict__ d, const double* __restrict__ acc, long long n,
                                const double* __restrict__ scale)
{
    const double f = *scale;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x)
        d[t] = acc[t] * f;
}

// SI results of a forward run from the objective kernel's scaled sums
// (scal[0] = F', scal[1] = adjoint source scale) and the run's field scale a:
//   DFT objective:  F = (dt/a)^2 F',  gradient scale 2 dt^2 s / a^2,
//                   adjoint field scale eps0 a / (2 dt^2 s);
//   time objective: F = (eps0/2) dx^3 dt F' / a^2,  gradient scale
//                   eps0 dt dx^3 s / a^2, adjoint field scale a / (dt dx^3 s).
// Written to scal[4] (F), scal[5] (gradient scale), scal[6] (adjoint scale).
__global__ void finish_kernel(double* scal, int kind, double a, double dt, double dx, double eps0)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double s = scal[1], dx3 = dx * dx * dx;
    if (kind == 1) {
        scal[4] = (dt / a) * (dt / a) * scal[0];
        scal[5] = 2.0 * dt * dt * s / (a * a);
        scal[6] = eps0 * a / (2.0 * dt * dt * s);
    } else {
        scal[4] = 0.5 * eps0 * dx3 * dt * scal[0] / (a * a);
        scal[5] = eps0 * dt * dx3 * s / (a * a);
        scal[6] = a / (dt * dx3 * s);
    }
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
// Spectrum of the recorded gap field: block f takes angular frequency
// omega[f]; out[f] = mean over the ne edges of |scale * sum_{n=0..M} E_e^n
// exp(-j omega[f] dt n)|^2 (FP64 sums, fixed order).
__global__ __launch_bounds__(256) void gap_spectrum_kernel(const float* gap, int M, int ne, double dt,
                                                           const double* omega, double scale, double* out)
{
    __shared__ double part[256];
    const double wdt = omega[blockIdx.x] * dt;
    double acc = 0.0;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int n = 0; n <= M; ++n) {
            double sn, cn;
            sincos(wdt * n, &sn, &cn);
            const double v = gap[(long long)n * ne + e];
            re += v * cn;
            im -= v * sn;
        }
        acc += (re * re + im * im) * scale * scale;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) part[threadIdx.x] += part[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = part[0] / (double)ne;
}

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

// Divergence watchdog (one workgroup): every E edge of the monitor box
// [lo, lo + dim) in the field state E just written must be finite and at most
// limit in magnitude (scaled units: the source's peak is 1).  On the first
// violation halt[0] = 1 -- the step kernels of every later launch read it and
// return at once -- and scal[7] = step (the steps done when it tripped).
__global__ __launch_bounds__(256) void watch_kernel(const float* E, unsigned cstride, int nxp, int nyp, int3 lo,
                                                    int3 dim, float limit, int step, unsigned* halt, double* scal)
{
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const int n = dim.x * dim.y * dim.z;
    int b = 0;
    for (int t = threadIdx.x; t < 3 * n; t += blockDim.x) {
        const int c = t / n, q = t - c * n;
        const int i = lo.x + q % dim.x, j = lo.y + (q / dim.x) % dim.y, k = lo.z + q / (dim.x * dim.y);
        const float v = ldf(fcomp(E, cstride, c), (((unsigned)(k + 1) * nyp + (unsigned)(j + 1)) * nxp + (unsigned)i) * 4u);
        if (!(fabsf(v) <= limit)) b = 1;  // not finite, or too large
    }
    if (b) atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0 && bad && halt[0] == 0u) {
        halt[0] = 1u;
        scal[7] = (double)step;
    }
}

int grid_for(long long n) { long long g = (n + 255) / 256; return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096); }

}  // namespace

template <int R, bool NT>
void launch_grid_rows(const StepArgs& a, bool pml, dim3 grid, dim3 block, hipStream_t s, hipEvent_t ev0,
                      hipEvent_t ev1)
{
    // with events, they are recorded by the dispatch itself (no separate
    // marker between this kernel and its neighbours on the stream)
    if (pml) {
        if (ev0 || ev1) hipExtLaunchKernelGGL((ccpr_step_kernel<R, true, NT>), grid, block, 0, s, ev0, ev1, 0, a);
        else hipLaunchKernelGGL((ccpr_step_kernel<R, true, NT>), grid, block, 0, s, a);
    } else {
        if (ev0 || ev1) hipExtLaunchKernelGGL((ccpr_step_kernel<R, false, NT>), grid, block, 0, s, ev0, ev1, 0, a);
        else hipLaunchKernelGGL((ccpr_step_kernel<R, false, NT>), grid, block, 0, s, a);
    }
}

int ccpr_launch_grid(const StepArgs& a, bool pml, void* stream, void* start_event, void* stop_event)
{
    hipEvent_t ev0 = (hipEvent_t)start_event, ev1 = (hipEvent_t)stop_event;
    hipStream_t s = (hipStream_t)stream;
    if (a.nblk <= 0) {
        if (ev0) (void)hipEventRecord(ev0, s);
        if (ev1) (void)hipEventRecord(ev1, s);
        return (int)hipGetLastError();
    }
    dim3 grid(a.nblk), block(a.nxp);
    if (a.rows == 2) {
        if (a.stream_st) launch_grid_rows<2, true>(a, pml, grid, block, s, ev0, ev1);
        else launch_grid_rows<2, false>(a, pml, grid, block, s, ev0, ev1);
    } else {
        if (a.stream_st) launch_grid_rows<4, true>(a, pml, grid, block, s, ev0, ev1);
        else launch_grid_rows<4, false>(a, pml, grid, block, s, ev0, ev1);
    }
    return (int)hipGetLastError();
}

template <bool NT>
void launch_des_nt(const StepArgs& a, int maxpairs, dim3 grid, dim3 block, hipStream_t s)
{
    if (maxpairs <= 1) hipLaunchKernelGGL((ccpr_step_des_kernel<NT, 1>), grid, block, 0, s, a);
    else if (maxpairs <= 2) hipLaunchKernelGGL((ccpr_step_des_kernel<NT, 2>), grid, block, 0, s, a);
    else if (maxpairs <= 3) hipLaunchKernelGGL((ccpr_step_des_kernel<NT, 3>), grid, block, 0, s, a);
    else if (maxpairs <= 4) hipLaunchKernelGGL((ccpr_step_des_kernel<NT, 4>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((ccpr_step_des_kernel<NT, 8>), grid, block, 0, s, a);
}

int ccpr_launch_grid_des(const StepArgs& a, int maxpairs, void* stream)
{
    if (a.nblk <= 0) return 0;
    if (a.rows != 2 || a.nxp > 512 || maxpairs > 8) return (int)hipErrorInvalidValue;
    dim3 grid(a.nblk), block(a.nxp);
    hipStream_t s = (hipStream_t)stream;
    if (a.stream_st) launch_des_nt<true>(a, maxpairs, grid, block, s);
    else launch_des_nt<false>(a, maxpairs, grid, block, s);
    return (int)hipGetLastError();
}

template <bool NT, bool DFT, bool EDGE>
void launch_aux_nt(const StepArgs& a, int maxpairs, dim3 ag, dim3 ab, hipStream_t s)
{
    if (maxpairs <= 0) hipLaunchKernelGGL((ccpr_aux_kernel<0, NT, DFT, EDGE>), ag, ab, 0, s, a);
    else if (maxpairs <= 1) hipLaunchKernelGGL((ccpr_aux_kernel<1, NT, DFT, EDGE>), ag, ab, 0, s, a);
    else if (maxpairs <= 2) hipLaunchKernelGGL((ccpr_aux_kernel<2, NT, DFT, EDGE>), ag, ab, 0, s, a);
    else if (maxpairs <= 3) hipLaunchKernelGGL((ccpr_aux_kernel<3, NT, DFT, EDGE>), ag, ab, 0, s, a);
    else if (maxpairs <= 4) hipLaunchKernelGGL((ccpr_aux_kernel<4, NT, DFT, EDGE>), ag, ab, 0, s, a);
    else if (maxpairs <= 6) hipLaunchKernelGGL((ccpr_aux_kernel<6, NT, DFT, EDGE>), ag, ab, 0, s, a);
    else hipLaunchKernelGGL((ccpr_aux_kernel<8, NT, DFT, EDGE>), ag, ab, 0, s, a);
}

template <bool EDGE>
void launch_aux_mode(const StepArgs& a, int maxpairs, dim3 ag, dim3 ab, hipStream_t s)
{
    const bool dft = (a.mode & (CCPR_MODE_DFT_T | CCPR_MODE_DFT_P)) != 0;
    if (a.stream_st) {
        if (dft) launch_aux_nt<true, true, EDGE>(a, maxpairs, ag, ab, s);
        else launch_aux_nt<true, false, EDGE>(a, maxpairs, ag, ab, s);
    } else {
        if (dft) launch_aux_nt<false, true, EDGE>(a, maxpairs, ag, ab, s);
        else launch_aux_nt<false, false, EDGE>(a, maxpairs, ag, ab, s);
    }
}

int ccpr_launch_aux(const StepArgs& a, int maxpairs, long long nd, bool edge, void* stream)
{
    if (nd <= 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    dim3 ag((unsigned)((nd + 255) / 256)), ab(256);
    if (edge) launch_aux_mode<true>(a, maxpairs, ag, ab, s);
    else launch_aux_mode<false>(a, maxpairs, ag, ab, s);
    return (int)hipGetLastError();
}

int ccpr_launch_batch(const BatchStep* st, int k, void* stream)
{
    if (k < 1 || k > CCPR_BATCH_MAX) return (int)hipErrorInvalidValue;
    BatchArgs B;
    std::memset(&B, 0, sizeof B);
    B.n = k;
    int maxp = 0;
    long long g = 0, x = 0, q = 0;
    for (int s = 0; s < k; ++s) {
        const BatchStep& t = st[s];
        if (t.a.nxp != st[0].a.nxp || t.a.rows != 2 || 2 * t.a.npml > 256) return (int)hipErrorInvalidValue;
        B.a[s] = t.a;
        maxp = std::max(maxp, t.maxpairs);
        const int np2 = 2 * t.a.npml;
        B.rpb[s] = np2 > 0 ? 256 / np2 : 1;
        B.nbx[s] = np2 > 0 ? ((long long)t.a.ny * t.a.nz + B.rpb[s] - 1) / B.rpb[s] : 0;
        B.nmisc[s] = t.nmisc;
        B.ntfh[s] = t.ntfh;
        B.nxs[s] = t.nxs;
        B.fused[s] = t.fused;
        B.gstart[s] = (int)g;
        B.astart[s] = (int)x;
        B.pstart[s] = (int)q;
        g += t.a.nblk;
        x += (t.nd + 255) / 256;
        q += t.fused ? B.nbx[s] + (t.nmisc + t.ntfh + 255) / 256 : (t.nxs + t.nmisc + 255) / 256;
    }
    if (g > 0x7fffffff || x > 0x7fffffff || q > 0x7fffffff) return (int)hipErrorInvalidValue;
    B.gstart[k] = (int)g;
    B.astart[k] = (int)x;
    B.pstart[k] = (int)q;
    hipStream_t hs = (hipStream_t)stream;
    const bool nt = st[0].a.stream_st != 0;
    if (g > 0) {
        if (nt) hipLaunchKernelGGL(ccpr_batch_grid_kernel<true>, dim3((unsigned)g), dim3(st[0].a.nxp), 0, hs, B);
        else hipLaunchKernelGGL(ccpr_batch_grid_kernel<false>, dim3((unsigned)g), dim3(st[0].a.nxp), 0, hs, B);
    }
    if (x > 0) {
#define CCPR_BAUX(P)                                                                                     \
    do {                                                                                                 \
        if (nt) hipLaunchKernelGGL((ccpr_batch_aux_kernel<P, true>), dim3((unsigned)x), dim3(256), 0, hs, B); \
        else hipLaunchKernelGGL((ccpr_batch_aux_kernel<P, false>), dim3((unsigned)x), dim3(256), 0, hs, B); \
    } while (0)
        if (maxp <= 0) CCPR_BAUX(0);
        else if (maxp <= 1) CCPR_BAUX(1);
        else if (maxp <= 2) CCPR_BAUX(2);
        else if (maxp <= 3) CCPR_BAUX(3);
        else if (maxp <= 4) CCPR_BAUX(4);
        else if (maxp <= 6) CCPR_BAUX(6);
        else CCPR_BAUX(8);
#undef CCPR_BAUX
    }
    if (q > 0) {
        if (nt) hipLaunchKernelGGL(ccpr_batch_post_kernel<true>, dim3((unsigned)q), dim3(256), 0, hs, B);
        else hipLaunchKernelGGL(ccpr_batch_post_kernel<false>, dim3((unsigned)q), dim3(256), 0, hs, B);
    }
    return (int)hipGetLastError();
}

int ccpr_launch_pre(const StepArgs& a, long long nxs, long long ntf, void* stream)
{
    const long long n = nxs + ntf;
    if (n <= 0) return 0;
    hipLaunchKernelGGL(ccpr_pre_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, a,
                       nxs);
    return (int)hipGetLastError();
}

int ccpr_launch_post(const StepArgs& a, long long nxs, long long nmisc, void* stream)
{
    const long long n = nxs + nmisc;
    if (n <= 0) return 0;
    hipLaunchKernelGGL(ccpr_post_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       a, nxs, nmisc);
    return (int)hipGetLastError();
}

int ccpr_launch_post_fused(const StepArgs& a, long long nmisc, long long ntfh, void* stream, void* stop_event)
{
    const int np2 = 2 * a.npml;
    if (np2 > 256) return (int)hipErrorInvalidValue;
    const int rpb = np2 > 0 ? 256 / np2 : 1;
    const long long nrows = np2 > 0 ? (long long)a.ny * a.nz : 0;
    const long long nbx = (nrows + rpb - 1) / rpb;
    const long long nb = nbx + (nmisc + ntfh + 255) / 256;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev = (hipEvent_t)stop_event;
    if (nb <= 0) {
        if (ev) (void)hipEventRecord(ev, s);
        return (int)hipGetLastError();
    }
    if (a.stream_st) {
        if (ev) hipExtLaunchKernelGGL(ccpr_post_fused_kernel<true>, dim3((unsigned)nb), dim3(256), 0, s, nullptr, ev,
                                      0, a, rpb, nbx, nmisc, ntfh);
        else hipLaunchKernelGGL(ccpr_post_fused_kernel<true>, dim3((unsigned)nb), dim3(256), 0, s, a, rpb, nbx,
                                nmisc, ntfh);
    } else {
        if (ev) hipExtLaunchKernelGGL(ccpr_post_fused_kernel<false>, dim3((unsigned)nb), dim3(256), 0, s, nullptr, ev,
                                      0, a, rpb, nbx, nmisc, ntfh);
        else hipLaunchKernelGGL(ccpr_post_fused_kernel<false>, dim3((unsigned)nb), dim3(256), 0, s, a, rpb, nbx,
                                nmisc, ntfh);
    }
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

int ccpr_launch_extract(float* d, const float* src, int comp, int nx, int ny, int nz, int nxp, int nyp,
                        float f, void* stream)
{
    const long long n = (long long)nx * ny * nz;
    hipLaunchKernelGGL(extract_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, d, src, comp,
                       nx, ny, nz, nxp, nyp, f);
    return (int)hipGetLastError();
}

int ccpr_launch_dft_grad(double* grad, const float* acc, long long nd, const int ddim[3], const EdgeMap& em,
                         double i00, double i01, double i11, double wc, double ws, void* stream)
{
    if (nd <= 0) return 0;
    hipLaunchKernelGGL(dft_grad_kernel, dim3(grid_for(nd)), dim3(256), 0, (hipStream_t)stream, grad, acc, nd,
                       ddim[0], ddim[1], em, i00, i01, i11, wc, ws);
    return (int)hipGetLastError();
}

int ccpr_launch_grad_out(double* d, const double* acc, long long n, const double* scale, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(grad_out_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, d, acc,
                       n, scale);
    return (int)hipGetLastError();
}

int ccpr_launch_finish(double* scal, int kind, double a, double dt, double dx, double eps0, void* stream)
{
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, scal, kind, a, dt, dx, eps0);
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

int ccpr_launch_gap_spectrum(const float* gap, int M, int ne, double dt, const double* omega, int nf, double scale,
                             double* out, void* stream)
{
    if (nf <= 0 || ne <= 0) return 0;
    hipLaunchKernelGGL(gap_spectrum_kernel, dim3((unsigned)nf), dim3(256), 0, (hipStream_t)stream, gap, M, ne, dt,
                       omega, scale, out);
    return (int)hipGetLastError();
}

int ccpr_launch_watch(const StepArgs& a, const int lo[3], const int dim[3], float limit, int n, unsigned* halt,
                      double* scal, void* stream)
{
    hipLaunchKernelGGL(watch_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, (const float*)a.Eo, a.cstride,
                       a.nxp, a.nyp, make_int3(lo[0], lo[1], lo[2]), make_int3(dim[0], dim[1], dim[2]), limit,
                       n + 1, halt, scal);
    return (int)hipGetLastError();
}

int ccpr_launch_check_rho(const float* rho, long long n, double* flag, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(check_rho_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, rho, n,
                       flag);
    return (int)hipGetLastError();
}
