// gfx950 kernels of the design filtering and projection (Sec. "Filtering and
// projection"): the cone filter of Eq. FilterFunction, the smoothed Heaviside
// of Eq. Projection, their chain rule (Eq. GradientsFiltered) and the measure
// of non-discreteness (Eq. MeasureOfNon-discretness), on the per-voxel density
// grid of the design box ([nz][ny][nx], x fastest; distances in voxels).
//
// The filter is a 3-D stencil over the sphere |d| < R (R <= 17 voxels).  A
// workgroup owns a 16 x 16 tile of one output plane; for every z offset it
// stages the input plane's tile plus an R-wide halo in LDS as (value, inside)
// pairs, with the cone weights of that offset's disk, and each lane sums the
// disk straight from LDS, so every input word is read from HBM once per
// (output plane, offset) workgroup and the taps cost LDS reads only.  Loop
// bounds are uniform per workgroup.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/ccprfdtd.h"

namespace {

constexpr int kFT = 16;                   // output tile edge (x and y)
constexpr int kMaxRi = 16;                // largest integer offset (radius <= 17)
constexpr int kTW = kFT + 2 * kMaxRi;     // staged tile edge

// Eq. FilterFunction and Eq. Projection: rho -> rho_t (filtered), rho_b
// (projected) and W (cone-weight sum of the design voxels in the sphere).
__global__ __launch_bounds__(256) void filter_project_kernel(const float* __restrict__ rho, float* rho_t,
                                                             float* rho_b, float* wsum, int nx, int ny, int nz,
                                                             float R, int Ri, float beta, float eta, float tbe,
                                                             float inv_den)
{
    __shared__ float2 tile[kTW * kTW];  // (density, 1) inside the box, (0, 0) outside
    __shared__ float wts[(2 * kMaxRi + 1) * (2 * kMaxRi + 1)];  // cone weights of one z offset
    const int tx = threadIdx.x % kFT, ty = threadIdx.x / kFT;
    const int i = blockIdx.x * kFT + tx, j = blockIdx.y * kFT + ty, k = blockIdx.z;
    const int W = kFT + 2 * Ri, D = 2 * Ri + 1;
    const int gx0 = blockIdx.x * kFT - Ri, gy0 = blockIdx.y * kFT - Ri;
    float num = 0.f, den = 0.f;
    for (int dz = -Ri; dz <= Ri; ++dz) {
        const int kk = k + dz;
        const float rz2 = R * R - (float)(dz * dz);
        if (kk < 0 || kk >= nz || rz2 <= 0.f) continue;  // uniform
        __syncthreads();
        for (int t = threadIdx.x; t < W * W; t += blockDim.x) {
            const int ly = t / W, lx = t - ly * W;
            const int gx = gx0 + lx, gy = gy0 + ly;
            const bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
            tile[t] = in ? make_float2(rho[((long long)kk * ny + gy) * nx + gx], 1.f) : make_float2(0.f, 0.f);
        }
        for (int t = threadIdx.x; t < D * D; t += blockDim.x) {
            const int qy = t / D - Ri, qx = t % D - Ri;
            wts[t] = R - sqrtf((float)(qx * qx + qy * qy + dz * dz));  // used inside the sphere only
        }
        __syncthreads();
        for (int dy = -Ri; dy <= Ri; ++dy) {
            const float ry2 = rz2 - (float)(dy * dy);
            if (ry2 <= 0.f) continue;  // uniform
            const int dxm = (int)ceilf(sqrtf(ry2)) - 1;  // dx^2 < ry2
            const float2* row = tile + (ty + Ri + dy) * W + (tx + Ri);
            const float* wrow = wts + (dy + Ri) * D + Ri;
            for (int dx = -dxm; dx <= dxm; ++dx) {
                const float w = wrow[dx];
                const float2 v = row[dx];
                num = fmaf(w, v.x, num);
                den = fmaf(w, v.y, den);
            }
        }
    }
    if (i < nx && j < ny) {
        const long long n = ((long long)k * ny + j) * nx + i;
        const float rt = num / den;
        rho_t[n] = rt;
        wsum[n] = den;
        rho_b[n] = (tbe + tanhf(beta * (rt - eta))) * inv_den;
    }
}

// Eq. GradientsFiltered: dF/drho[n] = sum_m w(m,n) v[m] over the design
// voxels m of the sphere around n, v = dF/drho_b * d rho_b/d rho_t / W,
// all in FP64 (the staged tile holds v, zero outside the box).
__global__ __launch_bounds__(256) void filter_project_grad_kernel(const double* __restrict__ g_b,
                                                                  const float* __restrict__ rho_t,
                                                                  const float* __restrict__ wsum, double* g,
                                                                  int nx, int ny, int nz, float R, int Ri,
                                                                  double beta, double eta, double inv_den)
{
    __shared__ double tile[kTW * kTW];
    __shared__ float wts[(2 * kMaxRi + 1) * (2 * kMaxRi + 1)];  // cone weights of one z offset
    const int tx = threadIdx.x % kFT, ty = threadIdx.x / kFT;
    const int i = blockIdx.x * kFT + tx, j = blockIdx.y * kFT + ty, k = blockIdx.z;
    const int W = kFT + 2 * Ri, D = 2 * Ri + 1;
    const int gx0 = blockIdx.x * kFT - Ri, gy0 = blockIdx.y * kFT - Ri;
    double acc = 0.0;
    for (int dz = -Ri; dz <= Ri; ++dz) {
        const int kk = k + dz;
        const float rz2 = R * R - (float)(dz * dz);
        if (kk < 0 || kk >= nz || rz2 <= 0.f) continue;  // uniform
        __syncthreads();
        for (int t = threadIdx.x; t < W * W; t += blockDim.x) {
            const int ly = t / W, lx = t - ly * W;
            const int gx = gx0 + lx, gy = gy0 + ly;
            double v = 0.0;
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
                const long long m = ((long long)kk * ny + gy) * nx + gx;
                const double th = tanh(beta * ((double)rho_t[m] - eta));
                v = g_b[m] * (beta * (1.0 - th * th) * inv_den) / (double)wsum[m];
            }
            tile[t] = v;
        }
        for (int t = threadIdx.x; t < D * D; t += blockDim.x) {
            const int qy = t / D - Ri, qx = t % D - Ri;
            wts[t] = R - sqrtf((float)(qx * qx + qy * qy + dz * dz));
        }
        __syncthreads();
        for (int dy = -Ri; dy <= Ri; ++dy) {
            const float ry2 = rz2 - (float)(dy * dy);
            if (ry2 <= 0.f) continue;  // uniform
            const int dxm = (int)ceilf(sqrtf(ry2)) - 1;
            const double* row = tile + (ty + Ri + dy) * W + (tx + Ri);
            const float* wrow = wts + (dy + Ri) * D + Ri;
            for (int dx = -dxm; dx <= dxm; ++dx) acc = fma((double)wrow[dx], row[dx], acc);
        }
    }
    if (i < nx && j < ny) g[((long long)k * ny + j) * nx + i] = acc;
}

// Eq. MeasureOfNon-discretness: one workgroup, fixed summation order (wave
// shuffles, then LDS), so the result does not depend on the launch.
__global__ __launch_bounds__(1024) void nondiscreteness_kernel(const float* __restrict__ rb, long long n, double* out)
{
    __shared__ double part[16];
    double s = 0.0;
    for (long long t = threadIdx.x; t < n; t += blockDim.x) {
        const double r = rb[t];
        s += 4.0 * r * (1.0 - r);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += part[w];
        out[0] = tot / (double)n * 100.0;
    }
}

// ---- per-edge design variables (one density per E edge at the staggered
// edge centres: x edges at (i+1/2, j, k), y edges at (i, j+1/2, k), z edges at
// (i, j, k+1/2) of an N-cell design, component c holding N_l + 1 - delta(c,l)
// edges along axis l; flat arrays hold the x, y, z edges in turn, each x
// fastest).  Eq. FilterFunction's sphere around an edge then takes in the
// edges of all three components; between component b and the output's
// component a the index offset o maps to the distance |o + h_b - h_a|, h_c the
// half-cell vector along axis c.  One launch per output component; a
// workgroup owns a 16 x 16 tile of one of its planes and, for every input
// component and z offset, stages the input plane's tile plus an H-wide halo
// (H = ceil(R) bounds every offset: |o| < R + 1/2) in LDS.

constexpr int kMaxH = 17;
constexpr int kTWE = kFT + 2 * kMaxH;

struct EdgeGeom {
    int shp[3][3];       // [component] (x, y, z) extents of its edges
    long long off[3];    // first flat index of each component
};

// sum over the taps of input component b around the output tile; 'stage'
// fills the tile (one LDS word per position, zero outside b's edges) and
// 'tap' consumes one staged word with its weight.  Offsets and weights are
// uniform across the workgroup: each z offset's cone weights (zero outside
// the sphere) are tabulated once in LDS (wts, (2H+1)^2 words) while the
// tile is staged, so a tap costs two LDS reads and the accumulation.
template <typename Stage, typename Tap>
__device__ __forceinline__ void edge_taps(int a, int b, const EdgeGeom& g, int k, float R, float R2, int H,
                                          float* wts, Stage stage, Tap tap)
{
    const int tx = threadIdx.x % kFT, ty = threadIdx.x / kFT;
    const float sx = 0.5f * ((b == 0) - (a == 0)), sy = 0.5f * ((b == 1) - (a == 1)),
                sz = 0.5f * ((b == 2) - (a == 2));
    const int W = kFT + 2 * H, D = 2 * H + 1;
    for (int dz = -H; dz <= H; ++dz) {
        const int kk = k + dz;
        const float fz = (float)dz + sz;
        const float rz2 = R2 - fz * fz;
        if (kk < 0 || kk >= g.shp[b][2] || rz2 <= 0.f) continue;  // uniform
        __syncthreads();
        stage(kk, W);
        for (int t = threadIdx.x; t < D * D; t += blockDim.x) {
            const int qy = t / D, qx = t - qy * D;
            const float fx = (float)(qx - H) + sx, fy = (float)(qy - H) + sy;
            const float d2 = fx * fx + fy * fy + fz * fz;
            wts[t] = d2 < R2 ? R - sqrtf(d2) : 0.f;
        }
        __syncthreads();
        for (int dy = -H; dy <= H; ++dy) {
            const float fy = (float)dy + sy;
            const float ry2 = rz2 - fy * fy;
            if (ry2 <= 0.f) continue;  // uniform
            const float rr = sqrtf(ry2);
            const int dxl = max(-H, (int)floorf(-sx - rr)), dxh = min(H, (int)ceilf(-sx + rr));
            const int rowb = (ty + H + dy) * W + (tx + H);
            const float* wrow = wts + (dy + H) * D + H;
            for (int dx = dxl; dx <= dxh; ++dx) tap(rowb + dx, wrow[dx]);  // zero weight outside the sphere
        }
    }
}

__global__ __launch_bounds__(256) void edge_filter_project_kernel(const float* __restrict__ rho, float* rho_t,
                                                                  float* rho_b, float* wsum, const EdgeGeom g,
                                                                  int a, float R, float R2, int H, float beta,
                                                                  float eta, float tbe, float inv_den)
{
    __shared__ float2 tile[kTWE * kTWE];  // (density, 1) on an edge of b, (0, 0) elsewhere
    __shared__ float wts[(2 * kMaxH + 1) * (2 * kMaxH + 1)];
    const int tx = threadIdx.x % kFT, ty = threadIdx.x / kFT;
    const int i = blockIdx.x * kFT + tx, j = blockIdx.y * kFT + ty, k = blockIdx.z;
    const int gx0 = blockIdx.x * kFT - H, gy0 = blockIdx.y * kFT - H;
    float num = 0.f, den = 0.f;
    for (int b = 0; b < 3; ++b) {
        const int bx = g.shp[b][0], by = g.shp[b][1];
        const float* src = rho + g.off[b];
        auto stage = [&](int kk, int W) {
            for (int t = threadIdx.x; t < W * W; t += blockDim.x) {
                const int ly = t / W, lx = t - ly * W;
                const int gx = gx0 + lx, gy = gy0 + ly;
                const bool in = gx >= 0 && gx < bx && gy >= 0 && gy < by;
                tile[t] = in ? make_float2(src[((long long)kk * by + gy) * bx + gx], 1.f) : make_float2(0.f, 0.f);
            }
        };
        auto tap = [&](int idx, float w) {
            const float2 v = tile[idx];
            num = fmaf(w, v.x, num);
            den = fmaf(w, v.y, den);
        };
        edge_taps(a, b, g, k, R, R2, H, wts, stage, tap);
    }
    if (i < g.shp[a][0] && j < g.shp[a][1]) {
        const long long n = g.off[a] + ((long long)k * g.shp[a][1] + j) * g.shp[a][0] + i;
        const float rt = num / den;
        rho_t[n] = rt;
        wsum[n] = den;
        rho_b[n] = (tbe + tanhf(beta * (rt - eta))) * inv_den;
    }
}

__global__ __launch_bounds__(256) void edge_filter_project_grad_kernel(const double* __restrict__ g_b,
                                                                       const float* __restrict__ rho_t,
                                                                       const float* __restrict__ wsum, double* gout,
                                                                       const EdgeGeom g, int a, float R, float R2,
                                                                       int H, double beta, double eta,
                                                                       double inv_den)
{
    __shared__ double tile[kTWE * kTWE];  // v = dF/drho_b * drho_b/drho_t / W on an edge of b, 0 elsewhere
    __shared__ float wts[(2 * kMaxH + 1) * (2 * kMaxH + 1)];
    const int tx = threadIdx.x % kFT, ty = threadIdx.x / kFT;
    const int i = blockIdx.x * kFT + tx, j = blockIdx.y * kFT + ty, k = blockIdx.z;
    const int gx0 = blockIdx.x * kFT - H, gy0 = blockIdx.y * kFT - H;
    double acc = 0.0;
    for (int b = 0; b < 3; ++b) {
        const int bx = g.shp[b][0], by = g.shp[b][1];
        const long long ob = g.off[b];
        auto stage = [&](int kk, int W) {
            for (int t = threadIdx.x; t < W * W; t += blockDim.x) {
                const int ly = t / W, lx = t - ly * W;
                const int gx = gx0 + lx, gy = gy0 + ly;
                double v = 0.0;
                if (gx >= 0 && gx < bx && gy >= 0 && gy < by) {
                    const long long m = ob + ((long long)kk * by + gy) * bx + gx;
                    const double th = tanh(beta * ((double)rho_t[m] - eta));
                    v = g_b[m] * (beta * (1.0 - th * th) * inv_den) / (double)wsum[m];
                }
                tile[t] = v;
            }
        };
        auto tap = [&](int idx, float w) { acc = fma((double)w, tile[idx], acc); };
        edge_taps(a, b, g, k, R, R2, H, wts, stage, tap);
    }
    if (i < g.shp[a][0] && j < g.shp[a][1]) gout[g.off[a] + ((long long)k * g.shp[a][1] + j) * g.shp[a][0] + i] = acc;
}

EdgeGeom edge_geom(const int* d)
{
    EdgeGeom g{};
    long long o = 0;
    for (int c = 0; c < 3; ++c) {
        long long n = 1;
        for (int l = 0; l < 3; ++l) {
            g.shp[c][l] = d[l] + (l == c ? 0 : 1);
            n *= g.shp[c][l];
        }
        g.off[c] = o;
        o += n;
    }
    return g;
}

bool edge_dims_ok(const int* d)
{
    return d && d[0] >= 1 && d[1] >= 1 && d[2] >= 1 && d[2] + 1 <= 65535;
}

bool dims_ok(const int* d)
{
    return d && d[0] >= 1 && d[1] >= 1 && d[2] >= 1 && d[2] <= 65535;
}

int radius_to_offsets(double R)
{
    // largest integer offset with |d| < R
    return (int)std::ceil(R) - 1;
}

}  // namespace

extern "C" {

ccpr_status ccpr_filter_project(const float* rho, float* rho_filtered, float* rho_projected, float* weight_sum,
                                const int dims[3], double radius, double beta, double eta, void* hip_stream)
{
    if (!rho || !rho_filtered || !rho_projected || !weight_sum || !dims_ok(dims)) return CCPR_EINVAL;
    if (!(radius >= 1.0 && radius <= 17.0) || !(beta > 0) || !(eta >= 0 && eta <= 1)) return CCPR_EINVAL;
    const int Ri = radius_to_offsets(radius);
    const double den = std::tanh(beta * eta) + std::tanh(beta * (1.0 - eta));
    dim3 grid((unsigned)((dims[0] + kFT - 1) / kFT), (unsigned)((dims[1] + kFT - 1) / kFT), (unsigned)dims[2]);
    hipLaunchKernelGGL(filter_project_kernel, grid, dim3(kFT * kFT), 0, (hipStream_t)hip_stream, rho, rho_filtered,
                       rho_projected, weight_sum, dims[0], dims[1], dims[2], (float)radius, Ri, (float)beta,
                       (float)eta, (float)std::tanh(beta * eta), (float)(1.0 / den));
    return hipGetLastError() == hipSuccess ? CCPR_OK : CCPR_EDEVICE;
}

ccpr_status ccpr_filter_project_grad(const double* dF_dprojected, const float* rho_filtered, const float* weight_sum,
                                     double* dF_drho, const int dims[3], double radius, double beta, double eta,
                                     void* hip_stream)
{
    if (!dF_dprojected || !rho_filtered || !weight_sum || !dF_drho || !dims_ok(dims)) return CCPR_EINVAL;
    if (!(radius >= 1.0 && radius <= 17.0) || !(beta > 0) || !(eta >= 0 && eta <= 1)) return CCPR_EINVAL;
    const int Ri = radius_to_offsets(radius);
    const double den = std::tanh(beta * eta) + std::tanh(beta * (1.0 - eta));
    dim3 grid((unsigned)((dims[0] + kFT - 1) / kFT), (unsigned)((dims[1] + kFT - 1) / kFT), (unsigned)dims[2]);
    hipLaunchKernelGGL(filter_project_grad_kernel, grid, dim3(kFT * kFT), 0, (hipStream_t)hip_stream, dF_dprojected,
                       rho_filtered, weight_sum, dF_drho, dims[0], dims[1], dims[2], (float)radius, Ri, beta, eta,
                       1.0 / den);
    return hipGetLastError() == hipSuccess ? CCPR_OK : CCPR_EDEVICE;
}

ccpr_status ccpr_filter_project_edges(const float* rho, float* rho_filtered, float* rho_projected,
                                      float* weight_sum, const int dims[3], double radius, double beta, double eta,
                                      void* hip_stream)
{
    if (!rho || !rho_filtered || !rho_projected || !weight_sum || !edge_dims_ok(dims)) return CCPR_EINVAL;
    if (!(radius >= 1.0 && radius <= 17.0) || !(beta > 0) || !(eta >= 0 && eta <= 1)) return CCPR_EINVAL;
    const EdgeGeom g = edge_geom(dims);
    const int H = (int)std::ceil(radius);
    const double den = std::tanh(beta * eta) + std::tanh(beta * (1.0 - eta));
    for (int a = 0; a < 3; ++a) {
        dim3 grid((unsigned)((g.shp[a][0] + kFT - 1) / kFT), (unsigned)((g.shp[a][1] + kFT - 1) / kFT),
                  (unsigned)g.shp[a][2]);
        hipLaunchKernelGGL(edge_filter_project_kernel, grid, dim3(kFT * kFT), 0, (hipStream_t)hip_stream, rho,
                           rho_filtered, rho_projected, weight_sum, g, a, (float)radius, (float)(radius * radius), H,
                           (float)beta, (float)eta, (float)std::tanh(beta * eta), (float)(1.0 / den));
    }
    return hipGetLastError() == hipSuccess ? CCPR_OK : CCPR_EDEVICE;
}

ccpr_status ccpr_filter_project_grad_edges(const double* dF_dprojected, const float* rho_filtered,
                                           const float* weight_sum, double* dF_drho, const int dims[3], double radius,
                                           double beta, double eta, void* hip_stream)
{
    if (!dF_dprojected || !rho_filtered || !weight_sum || !dF_drho || !edge_dims_ok(dims)) return CCPR_EINVAL;
    if (!(radius >= 1.0 && radius <= 17.0) || !(beta > 0) || !(eta >= 0 && eta <= 1)) return CCPR_EINVAL;
    const EdgeGeom g = edge_geom(dims);
    const int H = (int)std::ceil(radius);
    const double den = std::tanh(beta * eta) + std::tanh(beta * (1.0 - eta));
    for (int a = 0; a < 3; ++a) {
        dim3 grid((unsigned)((g.shp[a][0] + kFT - 1) / kFT), (unsigned)((g.shp[a][1] + kFT - 1) / kFT),
                  (unsigned)g.shp[a][2]);
        hipLaunchKernelGGL(edge_filter_project_grad_kernel, grid, dim3(kFT * kFT), 0, (hipStream_t)hip_stream,
                           dF_dprojected, rho_filtered, weight_sum, dF_drho, g, a, (float)radius,
                           (float)(radius * radius), H, beta, eta, 1.0 / den);
    }
    return hipGetLastError() == hipSuccess ? CCPR_OK : CCPR_EDEVICE;
}

ccpr_status ccpr_nondiscreteness(const float* rho_projected, long long n, double* out, void* hip_stream)
{
    if (!rho_projected || !out || n < 1) return CCPR_EINVAL;
    hipLaunchKernelGGL(nondiscreteness_kernel, dim3(1), dim3(1024), 0, (hipStream_t)hip_stream, rho_projected, n,
                       out);
    return hipGetLastError() == hipSuccess ? CCPR_OK : CCPR_EDEVICE;
}

}  // extern "C"
