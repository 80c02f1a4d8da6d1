// Host runtime of the CCPR-FDTD library: the C-ABI of include/ccprfdtd.h.
//
// Responsibilities: argument validation, FP64 precompute of the scaled
// material / CPML constants, carving the caller's workspace, ordering the
// kernel launches of the forward run, the adjoint run with segment
// checkpoint/recompute, and the gradient read-out.  Every arithmetic step of
// the path itself runs in the gfx950 kernels of ccpr_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ccprfdtd.h"
#include "ccpr_internal.h"
#include "ccpr_pipeline.h"

namespace {

constexpr double kEps0 = 8.8541878128e-12;
constexpr double kMu0 = 1.25663706212e-6;
constexpr double kC0 = 299792458.0;

typedef std::complex<double> cd;

struct MatHost {
    double eps = 1.0, sig = 0.0;
    std::vector<cd> a, c;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    // fixed part
    size_t Eb[2][2], Hb[2][2];   // [state][parity] -> 3*ncell floats
    size_t Jb[2];                // [state]
    size_t psiE[2];              // [state] all three slabs
    size_t psiH[2][2];           // [state][parity]
    size_t ssh[2];               // [state] FP64 shadow of E on source edges
    size_t cold[2];              // [state] StepCold block
    size_t rowf[2], lanef[2];    // [state] row / lane class words
    size_t extra[2];             // [state] aux-kernel cell list
    size_t zr;                   // z-chunk plane ranges of the step kernel
    size_t tiles;                // tile lists of the step kernel (interior, then CPML)
    size_t drive;                // S curl H' of design and source cells (scratch of one step)
    size_t rho, pmlE, pmlH, scal, gradacc, work;
    size_t halt;                 // divergence watchdog word (see ccpr_launch_watch)
    size_t fixed_end;
    // variable part
    size_t src_fwd, src_adj, wave, lineE, lineH, incE, incH, tf, gap, T, ckpt, stage;
    size_t total;
    int K = 0, S = 1;            // segment length / count
    int R = 1;                   // resident segments: the last R segments keep the
                                 // forward run's history; the others are recomputed
    size_t ckpt_bytes = 0;
    int inc_steps = 0, line_L = 0;
};

}  // namespace

struct ccpr_solver {
    ccpr_grid g{};
    double dt = 0;
    long long ncell = 0;        // nx*ny*nz
    int nxp = 0, nyp = 0, nzp = 0;
    long long npad = 0;         // nxp*nyp*nzp: floats per padded field component
    int rows = 2;               // y rows per thread of the step kernel
    std::string err;
    MatHost mat[2][3];
    // design: the box [dlo, dlo + ddim) of nd cells the kernels run over.
    // Per-edge designs (edge) have ncl cells and one density per E edge; their
    // box holds ncl + 1 cells per axis, and nrho is the number of edges.
    bool has_design = false;
    int dlo[3]{}, ddim[3]{};
    long long nd = 0;
    bool edge = false;
    int ncl[3]{};
    long long nrho = 0;
    double gamma = 0;
    std::vector<float> rho_host;
    bool rho_on_host = false, rho_uploaded = false;
    // source
    int src_kind = 0;  // 0 none, 1 dipole, 2 plane wave
    int dip_cell[3]{}, dip_axis = 0;
    int pw_d = 2, pw_sgn = 1, pw_p = 0, pw_lo[3]{}, pw_hi[3]{};
    std::vector<double> wave;
    double alpha = 1.0;  // forward source scale
    // objective
    bool has_obj = false;
    int obj_kind = 1, glo[3]{}, gdim[3]{}, gncell = 0, nb = 0, ne = -1;
    double omega = 0;
    int ckpt_every = 0;
    int resident_max = 0;       // at most this many resident segments (0: as many as fit)
    bool grad_dft = false;      // DFT-mode gradient estimator (CCPR_GRAD_DFT)
    // workspace
    char* ws = nullptr;
    uint64_t ws_bytes = 0;
    int static_dev = -1;        // device whose static workspace is bound (-1: none)
    hipStream_t stream = nullptr;
    int maxpairs = 0, npairs_total = 0;
    int tz = 5;                 // nominal planes per z-chunk of the step kernel
    // run state
    int parity[2] = {0, 0};
    // pre_done[st]: the last step's post launch also applied the next step's
    // pre-corrections (H^{n+1/2} is no longer the plain state until that step
    // runs); fuse_ok[st]: that fusion is safe for this configuration
    bool pre_done[2] = {false, false};
    bool fuse_ok[2] = {false, false};
    int step_count = 0;
    int src_table_steps = -1;   // steps covered by the uploaded forward source table
    Layout lay{};
    bool have_forward = false, have_adjoint = false;
    // an adjoint run that recomputed segments wrote their history over the
    // first resident segment's: a second adjoint needs a new forward run
    bool hist_stale = false;
    long long fwd_serial = 0;   // successful forward runs so far
    // divergence watchdog: check the gap box every watch_every steps of the
    // forward and adjoint runs (0: off) against watch_limit (scaled units)
    int watch_every = 128;
    double watch_limit = 1e15;
    bool watch_run = false;     // inside a forward / adjoint loop
    int M = 0;
    double F = 0, adj_alpha = 1.0, grad_scale = 0;
    int current_state = 0;  // 0 forward, 1 adjoint (for get_field)
    AxisMat mats[3]{};
    StepCold cold_host[2]{};
    std::vector<unsigned> rowf_host[2], lanef_host[2];
    std::vector<int4> extra_host[2];
    std::vector<TfEntry> tf_host;
    std::vector<int2> zr_host;  // plane range of each logical z-chunk
    // tiles (y-strip, logical z-chunk): interior tiles, then the interior
    // tiles that own design cells when the grid pass finishes the design
    // cells itself (des_on), then the CPML tiles
    std::vector<int2> tiles_host;
    int ntiles_int = 0, ntiles_des = 0, ntiles_pml = 0;
    bool des_fuse = false;      // run the design update inside the grid pass where it can
    bool des_on = false;        // the current plan does it (ntiles_des > 0)
    hipStream_t stream2 = nullptr;  // second stream: CPML tiles run beside the interior ones
    bool own_stream2 = false;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr, pdone_ev = nullptr;
    // post_ev is recorded by a step's post dispatch itself (no marker packet);
    // post_armed: nothing has been launched since, so the next step of state
    // post_armed_st may fork on it
    hipEvent_t post_ev = nullptr;
    bool post_armed = false;
    int post_armed_st = -1;
    // split passes alternate the two streams' roles: lead2 = the step sequence
    // currently continues on stream2 (join_lead() returns it to 'stream')
    bool lead2 = false;
    int tf_nE = 0, tf_nH = 0;
    long long fixed_key[4] = {-1, -1, -1, -1};
    // diagnostics
    double stat_ms = 0;
    long long stat_launches = 0;
    double stat_grid_ms = 0;
    long long stat_grid_launches = 0;
    bool timing = false;
    int timing_every = 1;           // time every k-th grid pass of the timed loops
    long long pass_no = 0;          // grid passes launched inside timed loops
    std::vector<hipEvent_t> tev;    // events around grid passes (start, end on each stream) of the current loop
    size_t tev_used = 0;
    bool timed_loop = false;        // inside a forward / adjoint loop with timing on
    // resumable solve (serving engine): phase 0 forward, 1 objective,
    // 2 adjoint (sub 0: recompute the segment, 1: adjoint steps), 3 all enqueued
    int pipe_phase = 3, pipe_n = 0, pipe_seg = 0, pipe_sub = 0, pipe_k = 0;
    // batched serving (ccpr_pipe_set_batched): launch_step records the grid /
    // aux / post work of a step instead of launching it; ccpr_pipe_flush
    // launches the recorded steps of several solves together
    bool batched = false;
    bool rec_pending = false, rec_watch = false;
    BatchStep rec{};
};

namespace {

std::string g_create_err;

ccpr_status fail(ccpr_solver* s, ccpr_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) s->err = buf;
    else g_create_err = buf;
    return st;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (hipError_t)(x);                                                   \
        if (e_ != hipSuccess) return fail(s, CCPR_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

long long psi_total(const ccpr_solver* s)
{
    if (s->g.npml <= 0) return 0;
    long long t = 0;
    for (int a = 0; a < 3; ++a) t += slab_size(a, s->g.nx, s->g.ny, s->g.nz, s->nxp, s->g.npml);
    return t;
}

int pairs_on_axis(const ccpr_solver* s, int ax)
{
    return (int)(s->mat[0][ax].a.size() + s->mat[1][ax].a.size());
}

void recount_pairs(ccpr_solver* s)
{
    s->maxpairs = 0;
    s->npairs_total = 0;
    for (int ax = 0; ax < 3; ++ax) {
        s->maxpairs = std::max(s->maxpairs, pairs_on_axis(s, ax));
        s->npairs_total += pairs_on_axis(s, ax);
    }
}

int plane_span(const ccpr_solver* s) { return s->pw_hi[s->pw_d] - s->pw_lo[s->pw_d] + 1; }

// Number of TF/SF face words (E and H) of the plane-wave box.
long long tf_count(const ccpr_solver* s)
{
    const int d = s->pw_d, p = s->pw_p, t = 3 - d - p;
    const long long Ld = s->pw_hi[d] - s->pw_lo[d], Lp = s->pw_hi[p] - s->pw_lo[p],
                    Lt = s->pw_hi[t] - s->pw_lo[t];
    return 2 * (Lt + 1) * Lp + 2 * (Lt + 1) * Ld + 2 * (Lt + 1) * Lp + 2 * (Ld + 1) * Lp;
}

// DFT-mode fit window: the adjoint fields m in [M-L+1, M] with L the whole
// periods of 2 pi/(omega dt) steps that fit in half the run, rounded to whole
// steps (half the run when that is less than a period; 2 <= L <= M).
int dft_window(int M, double omega, double dt)
{
    const double per = 2.0 * 3.14159265358979323846 / (omega * dt);
    const int q = (int)std::floor(0.5 * M / per);
    int L = q >= 1 ? (int)std::lround(q * per) : M / 2;
    L = std::max(L, std::min(M, 2));
    return std::min(L, M);
}

// density values and gradient values: one per voxel, or one per design edge
long long n_rho(const ccpr_solver* s) { return s->edge ? s->nrho : s->nd; }

// edge map of a per-edge design (EdgeMap::on = 0 for per-voxel designs)
EdgeMap edge_map(const ccpr_solver* s)
{
    EdgeMap m{};
    if (!s->edge) return m;
    m.on = 1;
    long long o = 0;
    for (int c = 0; c < 3; ++c) {
        long long n = 1;
        for (int l = 0; l < 3; ++l) {
            m.ebox[c][l] = s->ncl[l] + (l == c ? 0 : 1);
            n *= m.ebox[c][l];
        }
        m.eoff[c] = o;
        o += n;
    }
    return m;
}

size_t stage_bytes(const ccpr_solver* s)
{
    return std::max((size_t)s->ncell * 4, (size_t)std::max(n_rho(s), 1LL) * 8);
}

// Workspace layout for a solve of M steps (M = 0: stepping only) in segments
// of K_req steps (0: one segment) with R_req resident segments.
Layout make_layout(const ccpr_solver* s, int M, int K_req, int R_req = 1)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    const size_t nc = (size_t)s->npad;
    const size_t nd = (size_t)std::max<long long>(s->nd, 1);
    const size_t psi = (size_t)psi_total(s);
    for (int st = 0; st < 2; ++st) {
        for (int p = 0; p < 2; ++p) L.Eb[st][p] = take(3 * nc * 4);
        for (int p = 0; p < 2; ++p) L.Hb[st][p] = take(3 * nc * 4);
        L.Jb[st] = take(2 * (size_t)std::max(s->npairs_total, 1) * nd * 4);
        L.psiE[st] = take(std::max<size_t>(psi, 1) * 4);
        for (int p = 0; p < 2; ++p) L.psiH[st][p] = take(std::max<size_t>(psi, 1) * 4);
        L.ssh[st] = take((size_t)std::max(s->gncell, 1) * 3 * 8);
    }
    L.cold[0] = take(sizeof(StepCold));
    L.cold[1] = take(sizeof(StepCold));
    const size_t nsrc = (size_t)std::max(s->gncell, 1);  // dipole: 1 cell; adjoint: the gap box
    for (int st = 0; st < 2; ++st) {
        L.rowf[st] = take((size_t)s->g.ny * s->g.nz * 4);
        L.lanef[st] = take((size_t)s->nxp * 4);
        L.extra[st] = take((2 * nsrc + 1) * sizeof(int4));
    }
    L.drive = take((3 * nd + 3 * nsrc) * 4);
    L.zr = take((size_t)(s->g.nz + 1) * sizeof(int2));
    L.tiles = take((size_t)((s->g.ny + 1) / 2 + 1) * (s->g.nz + 1) * sizeof(int2));
    L.rho = take((size_t)std::max(n_rho(s), 1LL) * 4);
    L.pmlE = take((size_t)(s->g.nx + s->g.ny + s->g.nz) * 16);
    L.pmlH = take((size_t)(s->g.nx + s->g.ny + s->g.nz) * 16);
    L.scal = take(16 * 8);
    L.gradacc = take((size_t)std::max(n_rho(s), 1LL) * 8);
    L.work = take((size_t)std::max(s->gncell * 3, 1) * 16);
    L.halt = take(16);
    L.fixed_end = o;
    // forward source tables cover the solve (or the waveform when stepping)
    const int nw = (int)s->wave.size();
    const int steps = M > 0 ? M : std::max(nw, 1);
    L.inc_steps = steps;
    L.src_fwd = take((size_t)steps * 3 * 4);
    if (s->src_kind == 2) {
        const int span = plane_span(s);
        L.line_L = span + 16 + steps / 2 + 16;
        L.wave = take((size_t)std::max(nw, 1) * 8);
        L.lineE = take((size_t)(L.line_L + 1) * 8);
        L.lineH = take((size_t)(L.line_L + 1) * 8);
        L.incE = take((size_t)(steps + 1) * span * 4);
        L.incH = take((size_t)(steps + 1) * (span + 1) * 4);
        L.tf = take((size_t)tf_count(s) * sizeof(TfEntry));
    }
    if (M > 0) {
        L.src_adj = take((size_t)M * std::max(s->gncell, 1) * 3 * 4);
        L.gap = take((size_t)(M + 1) * std::max(s->gncell, 1) * 3 * 4);
        // DFT mode: one segment, no history; the T region holds the running
        // transforms [12][nd] instead
        int K = s->grad_dft ? M : K_req > 0 ? std::min(K_req, M) : M;
        L.K = K;
        L.S = (M + K - 1) / K;
        // the history holds the last R segments (R K steps); checkpoints start
        // the segments 1 .. S-R-1 that are recomputed (segment 0 starts from zero)
        L.R = std::max(1, std::min(R_req, L.S));
        L.T = take(s->grad_dft ? 12 * nd * 4 : (size_t)L.R * K * 3 * nd * 4);
        L.ckpt_bytes = (6 * nc + 2 * (size_t)std::max(s->npairs_total, 1) * nd + 2 * psi) * 4 + 8 * 3 * 8;
        L.ckpt = take((size_t)std::max(L.S - L.R - 1, 0) * align256(L.ckpt_bytes));
    }
    L.stage = take(stage_bytes(s));
    L.total = o;
    return L;
}

template <typename T>
T* wsp(ccpr_solver* s, size_t off) { return reinterpret_cast<T*>(s->ws + off); }

ccpr_status need_bound(ccpr_solver* s)
{
    if (!s->ws) return fail(s, CCPR_ESTATE, "no workspace bound");
    return CCPR_OK;
}

// Scaled material constants of one axis (FP64 -> FP32 kernel constants).
void axis_mat(const ccpr_solver* s, int ax, int jofs, AxisMat& m)
{
    const MatHost& m1 = s->mat[0][ax];
    const MatHost& m2 = s->mat[1][ax];
    const double dt = s->dt, h = dt / (2 * kEps0);
    m.eps1 = m1.eps;
    m.deps = m2.eps - m1.eps;
    m.sig1 = m1.sig * h;
    m.dsig = (m2.sig - m1.sig) * h;
    m.gam = s->gamma * h;
    m.epsf = (float)m.eps1;
    m.depsf = (float)m.deps;
    m.dsigf = (float)m.dsig;
    m.gamf = (float)m.gam;
    m.np1 = (int)m1.a.size();
    m.np = (int)(m1.a.size() + m2.a.size());
    m.jofs = jofs;
    int q = 0;
    for (int slot = 0; slot < 2; ++slot) {
        const MatHost& mm = slot == 0 ? m1 : m2;
        for (size_t p = 0; p < mm.a.size(); ++p, ++q) {
            const cd a = mm.a[p], c = mm.c[p];
            const cd den = 1.0 - a * dt / 2.0;
            const cd km1 = a * dt / den;  // k_p - 1, free of cancellation
            const cd b = c * dt / den;
            m.krd[q] = km1.real();
            m.kid[q] = km1.imag();
            m.brd[q] = b.real();
            m.bid[q] = b.imag();
        }
    }
    for (; q < CCPR_PMAX; ++q) m.krd[q] = m.kid[q] = m.brd[q] = m.bid[q] = 0.0;
}

// CPML coefficient (b, a, 1/kappa) at position pos (cell units) along an axis
// of N cells.
void pml_point(const ccpr_solver* s, int N, double pos, float* out)
{
    const int np = s->g.npml;
    double xi = 0;
    if (np > 0) {
        double d = std::max(std::max(np - pos, pos - (N - np)), 0.0);
        xi = std::min(d, (double)np) / np;
    }
    const double eta0 = std::sqrt(kMu0 / kEps0);
    const double m = s->g.pml_order;
    const double smax = s->g.pml_sigma_scale * 0.8 * (m + 1) / (eta0 * s->g.dx);
    const double sig = smax * std::pow(xi, m);
    const double kap = 1 + (s->g.pml_kappa_max - 1) * std::pow(xi, m);
    const double al = s->g.pml_alpha_max * (1 - xi);
    const double b = std::exp(-(sig / kap + al) * s->dt / kEps0);
    const double a = sig > 0 ? sig * (b - 1) / (sig * kap + kap * kap * al) : 0.0;
    out[0] = (float)b;
    out[1] = (float)a;
    out[2] = (float)(1.0 / kap);
    out[3] = 0.f;
}

ccpr_status upload_static(ccpr_solver* s)
{
    const int n3[3] = {s->g.nx, s->g.ny, s->g.nz};
    std::vector<float> e, h;
    for (int ax = 0; ax < 3; ++ax)
        for (int q = 0; q < n3[ax]; ++q) {
            float v[4];
            pml_point(s, n3[ax], q, v);
            e.insert(e.end(), v, v + 4);
            pml_point(s, n3[ax], q + 0.5, v);
            h.insert(h.end(), v, v + 4);
        }
    HIPCHK(hipMemcpyAsync(s->ws + s->lay.pmlE, e.data(), e.size() * 4, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->ws + s->lay.pmlH, h.data(), h.size() * 4, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return CCPR_OK;
}

ccpr_status upload_rho(ccpr_solver* s)
{
    if (!s->ws || !s->has_design || !s->rho_on_host || s->rho_uploaded) return CCPR_OK;
    HIPCHK(hipMemcpyAsync(s->ws + s->lay.rho, s->rho_host.data(), s->rho_host.size() * 4,
                          hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->rho_uploaded = true;
    return CCPR_OK;
}

// Make the solver's stream wait for a step sequence that ended on stream2
// (every launch outside the step loop goes to the solver's stream).
ccpr_status join_lead(ccpr_solver* s)
{
    s->post_armed = false;
    if (!s->lead2) return CCPR_OK;
    HIPCHK(hipEventRecord(s->join_ev, s->stream2));
    HIPCHK(hipStreamWaitEvent(s->stream, s->join_ev, 0));
    s->lead2 = false;
    return CCPR_OK;
}

ccpr_status zero_state(ccpr_solver* s, int st)
{
    {
        ccpr_status j = join_lead(s);
        if (j) return j;
    }
    const Layout& L = s->lay;
    const long long psi = psi_total(s);
    HIPCHK(ccpr_launch_fill(wsp<float>(s, L.Eb[st][0]), 3 * s->npad, 0.f, s->stream));
    HIPCHK(ccpr_launch_fill(wsp<float>(s, L.Eb[st][1]), 3 * s->npad, 0.f, s->stream));
    HIPCHK(ccpr_launch_fill(wsp<float>(s, L.Hb[st][0]), 3 * s->npad, 0.f, s->stream));
    HIPCHK(ccpr_launch_fill(wsp<float>(s, L.Hb[st][1]), 3 * s->npad, 0.f, s->stream));
    HIPCHK(ccpr_launch_fill(wsp<float>(s, L.Jb[st]), 2LL * s->npairs_total * std::max(s->nd, 1LL), 0.f,
                            s->stream));
    HIPCHK(ccpr_launch_fill(wsp<float>(s, L.psiE[st]), psi, 0.f, s->stream));
    HIPCHK(ccpr_launch_fill(wsp<float>(s, L.psiH[st][0]), psi, 0.f, s->stream));
    HIPCHK(ccpr_launch_fill(wsp<float>(s, L.psiH[st][1]), psi, 0.f, s->stream));
    HIPCHK(ccpr_launch_fill_d(wsp<double>(s, L.ssh[st]), (long long)std::max(s->gncell, 1) * 3, 0.0, s->stream));
    s->parity[st] = 0;
    s->pre_done[st] = false;
    return CCPR_OK;
}

// Forward source tables (scaled by alpha) for 'steps' steps.
ccpr_status prepare_source(ccpr_solver* s, int steps)
{
    const Layout& L = s->lay;
    const int nw = (int)s->wave.size();
    double mx = 0;
    for (double v : s->wave) mx = std::max(mx, std::fabs(v));
    if (!(mx > 0)) mx = 1.0;
    if (s->src_kind == 1) {
        s->alpha = kEps0 / (s->dt * mx);
        std::vector<float> t((size_t)steps * 3, 0.f);
        for (int n = 0; n < steps && n < nw; ++n) t[(size_t)n * 3 + s->dip_axis] = (float)(s->wave[n] / mx);
        HIPCHK(hipMemcpyAsync(s->ws + L.src_fwd, t.data(), t.size() * 4, hipMemcpyHostToDevice, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    } else if (s->src_kind == 2) {
        s->alpha = 1.0 / mx;
        std::vector<double> w(nw);
        for (int n = 0; n < nw; ++n) w[n] = s->wave[n] / mx;
        HIPCHK(hipMemcpyAsync(s->ws + L.wave, w.data(), w.size() * 8, hipMemcpyHostToDevice, s->stream));
        const int d = s->pw_d, p = s->pw_p, t = 3 - d - p;
        auto levi = [](int a, int b, int c) {
            return ((a == 0 && b == 1 && c == 2) || (a == 1 && b == 2 && c == 0) || (a == 2 && b == 0 && c == 1)) ? 1 : -1;
        };
        const double coef = levi(p, d, t) * s->pw_sgn * s->g.courant;
        const int ref = s->pw_sgn > 0 ? s->pw_lo[d] - 2 : s->pw_hi[d] + 2;
        HIPCHK(ccpr_launch_incident_line(wsp<double>(s, L.wave), nw, steps, L.line_L, coef, s->pw_lo[d],
                                         s->pw_hi[d], s->pw_sgn, ref, wsp<double>(s, L.lineE),
                                         wsp<double>(s, L.lineH), wsp<float>(s, L.incE),
                                         wsp<float>(s, L.incH), s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    s->src_table_steps = steps;
    return CCPR_OK;
}

int sigma_ca(int c, int a) { return a == (c + 1) % 3 ? 1 : -1; }

// TF/SF face words of the plane-wave box (total field inside [lo, hi]).  In
// the coordinates (d, p, t) = (propagation, polarisation, third axis):
//  E_p on the d-faces and E_d on the p-faces are total-field points whose
//  outside H neighbour is scattered-field: the incident H is added to their
//  curl;  H_t on the d-planes and H_d on the t-planes just outside are
//  scattered-field points whose inside E neighbour is total-field: the
//  incident E is removed from their curl.  sigma_ca gives the sign with which
//  a derivative along axis a enters (curl)_c.  The scaled update is
//  E += S(curl H + corr),  H -= S(curl E + corr),  so coef = +-S*sigma for E
//  words and -+S*sigma for H words.  E words come first in 'out'.
ccpr_status build_tf(ccpr_solver* s, const StepCold& C)
{
    auto& out = s->tf_host;
    out.clear();
    const int d = s->pw_d, p = s->pw_p, t = 3 - d - p;
    const int* lo = s->pw_lo;
    const int* hi = s->pw_hi;
    const double S = s->g.courant;
    const int nx = s->g.nx, ny = s->g.ny;
    auto push = [&](int comp, int cd, int cp, int ct, int m, double coef) {
        int x[3];
        x[d] = cd;
        x[p] = cp;
        x[t] = ct;
        TfEntry e;
        const long long cell = ((long long)(x[2] + 1) * s->nyp + (x[1] + 1)) * s->nxp + x[0];
        e.off = (unsigned long long)((comp * s->npad + cell) * 4);
        e.m = m;
        e.coef = (float)coef;
        e.uidx = (unsigned)(comp * s->ncell + ((long long)x[2] * ny + x[1]) * nx + x[0]);
        out.push_back(e);
    };
    auto inside = [](const int* x, const int* blo, const int* bdim) {
        return x[0] >= blo[0] && x[0] < blo[0] + bdim[0] && x[1] >= blo[1] && x[1] < blo[1] + bdim[1] &&
               x[2] >= blo[2] && x[2] < blo[2] + bdim[2];
    };
    bool clash = false;
    auto e_word = [&](int comp, int cd, int cp, int ct, int m, double coef) {
        int x[3];
        x[d] = cd;
        x[p] = cp;
        x[t] = ct;
        if (C.nd > 0 && inside(x, C.dlo, C.ddim)) clash = true;
        if (C.gap_on && inside(x, C.glo, C.gdim)) clash = true;
        push(comp, cd, cp, ct, m, coef);
    };
    const double sEp = sigma_ca(p, d), sEd = sigma_ca(d, p), sHt = sigma_ca(t, d), sHd = sigma_ca(d, t);
    // E_p on the d-faces
    for (int ct = lo[t]; ct <= hi[t]; ++ct)
        for (int cp = lo[p]; cp < hi[p]; ++cp) {
            e_word(p, lo[d], cp, ct, 0, -S * sEp);
            e_word(p, hi[d], cp, ct, hi[d] - lo[d] + 1, S * sEp);
        }
    // E_d on the p-faces
    for (int ct = lo[t]; ct <= hi[t]; ++ct)
        for (int cd = lo[d]; cd < hi[d]; ++cd) {
            e_word(d, cd, lo[p], ct, cd - lo[d] + 1, -S * sEd);
            e_word(d, cd, hi[p], ct, cd - lo[d] + 1, S * sEd);
        }
    s->tf_nE = (int)out.size();
    // H_t on the d-planes just outside
    for (int ct = lo[t]; ct <= hi[t]; ++ct)
        for (int cp = lo[p]; cp < hi[p]; ++cp) {
            push(t, lo[d] - 1, cp, ct, 0, S * sHt);
            push(t, hi[d], cp, ct, hi[d] - lo[d], -S * sHt);
        }
    // H_d on the t-planes just outside
    for (int cd = lo[d]; cd <= hi[d]; ++cd)
        for (int cp = lo[p]; cp < hi[p]; ++cp) {
            push(d, cd, cp, lo[t] - 1, cd - lo[d], S * sHd);
            push(d, cd, cp, hi[t], cd - lo[d], -S * sHd);
        }
    s->tf_nH = (int)out.size() - s->tf_nE;
    if ((long long)out.size() > tf_count(s))
        return fail(s, CCPR_EINVAL, "internal: TF/SF word count %zu above %lld", out.size(), tf_count(s));
    if (clash)
        return fail(s, CCPR_ENOTSUP, "the TF/SF boundary must lie in the background: it crosses the design or gap box");
    return CCPR_OK;
}

// Cold step data of state st (0 forward, 1 adjoint): everything the kernel
// reads only in its rare branches.  Written to the workspace once per pass.
void fill_cold(ccpr_solver* s, int st, StepCold& C)
{
    const Layout& L = s->lay;
    C = StepCold{};
    if (s->has_design) {
        for (int a = 0; a < 3; ++a) { C.dlo[a] = s->dlo[a]; C.ddim[a] = s->ddim[a]; }
        C.nd = s->nd;
        C.rho = wsp<float>(s, L.rho);
        C.J = wsp<float>(s, L.Jb[st]);
        for (int ax = 0; ax < 3; ++ax) C.mat[ax] = s->mats[ax];
        C.em = edge_map(s);
    }
    if (s->g.npml > 0) {
        const int n3[3] = {s->g.nx, s->g.ny, s->g.nz};
        size_t offc = 0, offs = 0;
        for (int a = 0; a < 3; ++a) {
            C.pmlE[a] = wsp<float4>(s, L.pmlE) + offc;
            C.pmlH[a] = wsp<float4>(s, L.pmlH) + offc;
            C.psiE[a] = wsp<float>(s, L.psiE[st]) + offs;
            C.psiH[0][a] = wsp<float>(s, L.psiH[st][0]) + offs;
            C.psiH[1][a] = wsp<float>(s, L.psiH[st][1]) + offs;
            offc += n3[a];
            offs += slab_size(a, s->g.nx, s->g.ny, s->g.nz, s->nxp, s->g.npml);
        }
    }
    if (st == 0 && s->src_kind == 1) {
        C.src_on = 1;
        for (int a = 0; a < 3; ++a) { C.slo[a] = s->dip_cell[a]; C.sdim[a] = 1; }
        C.sncell = 1;
        C.snsteps = s->src_table_steps;
        C.src = wsp<float>(s, L.src_fwd);
        C.ssh = wsp<double>(s, L.ssh[0]);
    } else if (st == 0 && s->src_kind == 2) {
        C.pw_on = 1;
        C.pw_spanE = plane_span(s);
        C.pw_spanH = plane_span(s) + 1;
        C.tf_rows = L.inc_steps + 1;
        C.tf_nE = s->tf_nE;
        C.tf_nH = s->tf_nH;
        C.incE = wsp<float>(s, L.incE);
        C.incH = wsp<float>(s, L.incH);
        C.tf = wsp<TfEntry>(s, L.tf);
    } else if (st == 1) {
        C.src_on = 1;
        for (int a = 0; a < 3; ++a) { C.slo[a] = s->glo[a]; C.sdim[a] = s->gdim[a]; }
        C.sncell = s->gncell;
        C.snsteps = s->M;
        C.src = wsp<float>(s, L.src_adj);
        C.ssh = wsp<double>(s, L.ssh[1]);
    }
    if (st == 0 && s->has_obj && L.gap) {
        C.gap_on = 1;
        for (int a = 0; a < 3; ++a) { C.glo[a] = s->glo[a]; C.gdim[a] = s->gdim[a]; }
        C.gncell = s->gncell;
        C.gap = wsp<float>(s, L.gap);
    }
    if (L.T) C.T = wsp<float>(s, L.T);
    C.grad = wsp<double>(s, L.gradacc);
}

// Row classes [k*ny + j] and lane classes [i] of state st (see CCPR_ROW_*,
// CCPR_LANE_*): which rare branches a row / a lane can need.
void fill_classes(const ccpr_solver* s, const StepCold& C, std::vector<unsigned>& rowf,
                  std::vector<unsigned>& lanef)
{
    const int nx = s->g.nx, ny = s->g.ny, nz = s->g.nz, np = s->g.npml;
    auto in = [](int v, int lo, int hi_excl) { return v >= lo && v < hi_excl; };
    rowf.assign((size_t)ny * nz, 0u);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            unsigned f = 0;
            if (np > 0 && (j < np || j >= ny - np)) f |= CCPR_ROW_YPML;
            if (np > 0 && (k < np || k >= nz - np)) f |= CCPR_ROW_ZPML;
            if (C.nd > 0 && in(j, C.dlo[1], C.dlo[1] + C.ddim[1]) && in(k, C.dlo[2], C.dlo[2] + C.ddim[2]))
                f |= CCPR_ROW_DES;
            if (C.src_on && in(j, C.slo[1], C.slo[1] + C.sdim[1]) && in(k, C.slo[2], C.slo[2] + C.sdim[2]))
                f |= CCPR_ROW_SRC;
            rowf[(size_t)k * ny + j] = f;
        }
    lanef.assign((size_t)s->nxp, 0u);
    for (int i = 0; i < nx; ++i) {
        unsigned f = 0;
        if (np > 0 && (i < np || i >= nx - np)) f |= CCPR_LANE_PML;
        if (C.nd > 0 && in(i, C.dlo[0], C.dlo[0] + C.ddim[0])) f |= CCPR_LANE_DES;
        if (C.src_on && in(i, C.slo[0], C.slo[0] + C.sdim[0])) f |= CCPR_LANE_SRC;
        lanef[i] = f;
    }
}

// Cells outside the design box that the post kernel finishes: source cells
// (E update from the stored drive minus the source current) and gap-monitor
// cells outside both boxes (monitor only).
void fill_extra(const StepCold& C, std::vector<int4>& ex)
{
    ex.clear();
    auto in_box = [](int i, int j, int k, const int* lo, const int* dim) {
        return i >= lo[0] && i < lo[0] + dim[0] && j >= lo[1] && j < lo[1] + dim[1] && k >= lo[2] &&
               k < lo[2] + dim[2];
    };
    const bool des = C.nd > 0;
    if (C.src_on)
        for (int k = C.slo[2]; k < C.slo[2] + C.sdim[2]; ++k)
            for (int j = C.slo[1]; j < C.slo[1] + C.sdim[1]; ++j)
                for (int i = C.slo[0]; i < C.slo[0] + C.sdim[0]; ++i)
                    if (!(des && in_box(i, j, k, C.dlo, C.ddim))) ex.push_back(make_int4(i, j, k, CCPR_EXTRA_SOURCE));
    if (C.gap_on)
        for (int k = C.glo[2]; k < C.glo[2] + C.gdim[2]; ++k)
            for (int j = C.glo[1]; j < C.glo[1] + C.gdim[1]; ++j)
                for (int i = C.glo[0]; i < C.glo[0] + C.gdim[0]; ++i)
                    if (!(des && in_box(i, j, k, C.dlo, C.ddim)) && !(C.src_on && in_box(i, j, k, C.slo, C.sdim)))
                        ex.push_back(make_int4(i, j, k, CCPR_EXTRA_GAP));
}

// z-chunks of the step kernel: about nz/tz chunks of equal estimated cost
// (a plane in a z CPML layer also streams its psi memories: weight 1.6), so
// that the XCDs, which each take an equal share of the chunks, finish
// together.  Logical chunk q of XCD-contiguous order gets physical chunk
// (q % 8) * (n/8) + q / 8 when n is a multiple of 8, which spreads the
// expensive chunks over the XCDs.
#ifndef CCPR_ZPML_PLANE_COST
#define CCPR_ZPML_PLANE_COST 1.6
#endif
void plan_chunks(ccpr_solver* s)
{
    const int nz = s->g.nz, np = s->g.npml;
    int n = std::max(1, std::min(nz, (nz + s->tz - 1) / s->tz));
    if (n >= 8 && nz >= 8 * ((n + 7) / 8)) n = (n + 7) / 8 * 8;
    std::vector<double> cum(nz + 1, 0.0);
    for (int k = 0; k < nz; ++k)
        cum[k + 1] = cum[k] + ((np > 0 && (k < np || k >= nz - np)) ? CCPR_ZPML_PLANE_COST : 1.0);
    std::vector<int> b(n + 1);
    b[0] = 0;
    b[n] = nz;
    int k = 0;
    for (int m = 1; m < n; ++m) {
        const double target = cum[nz] * m / n;
        while (k < nz && cum[k + 1] <= target) ++k;
        if (k + 1 <= nz && target - cum[k] > cum[k + 1] - target) ++k;
        b[m] = std::max(b[m - 1] + 1, std::min(k, nz - (n - m)));
    }
    std::vector<int2> phys(n);
    for (int m = 0; m < n; ++m) phys[m] = make_int2(b[m], b[m + 1]);
    s->zr_host.resize(n);
#ifndef CCPR_CHUNK_SPREAD
#define CCPR_CHUNK_SPREAD 1
#endif
    for (int q = 0; q < n; ++q) s->zr_host[q] = phys[CCPR_CHUNK_SPREAD && n % 8 == 0 ? (q % 8) * (n / 8) + q / 8 : q];
    // tiles (y-strip of 'rows' rows, logical z-chunk) in logical order, split
    // by whether any of their H or E rows (halo row and plane included) lies
    // in a y or z CPML layer; interior tiles whose own rows and planes hold
    // design cells are marked
    const int ny = s->g.ny, R = s->rows, nys = (ny + R - 1) / R;
    std::vector<int2> in, pm;
    std::vector<char> owns_design;
    bool design_in_pml = false;
    for (int q = 0; q < n; ++q)
        for (int ys = 0; ys < nys; ++ys) {
            bool pml = false;
            if (np > 0) {
                const int j0 = ys * R - 1, j1 = std::min(ys * R + R, ny);  // rows j0..j1-1
                const int k0 = s->zr_host[q].x - 1, k1 = s->zr_host[q].y;  // planes k0..k1-1
                pml = j0 < np || j1 > ny - np || k0 < np || k1 > nz - np;
            }
            bool des = false;
            if (s->has_design) {
                const int ja = ys * R, jb = std::min(ys * R + R, ny);      // own rows ja..jb-1
                const int ka = s->zr_host[q].x, kb = s->zr_host[q].y;      // own planes ka..kb-1
                des = ja < s->dlo[1] + s->ddim[1] && jb > s->dlo[1] && ka < s->dlo[2] + s->ddim[2] &&
                      kb > s->dlo[2];
            }
            if (pml) {
                pm.push_back(make_int2(ys, q));
                design_in_pml = design_in_pml || des;
            } else {
                in.push_back(make_int2(ys, q));
                owns_design.push_back(des ? 1 : 0);
            }
        }
    // When enabled (ccpr_set_design_fusion), the design update runs inside
    // the grid pass (design tiles as a launch of their own after the CPML
    // tiles) for per-voxel designs with the time-exact gradient when the pass
    // is split in two launches, nx <= 512 and no CPML tile owns a design
    // cell; otherwise in the aux pass.
    const long long nds = std::count(owns_design.begin(), owns_design.end(), (char)1);
    s->des_on = s->des_fuse && nds > 0 && !s->edge && !s->grad_dft && R == 2 && s->nxp <= 512 &&
                s->maxpairs <= 8 && !design_in_pml && (long long)in.size() >= 1024 && pm.size() >= 128 &&
                s->static_dev < 0 && !s->batched;
    s->tiles_host.clear();
    std::vector<int2> ds;
    for (size_t t = 0; t < in.size(); ++t) (s->des_on && owns_design[t] ? ds : s->tiles_host).push_back(in[t]);
    s->ntiles_int = (int)s->tiles_host.size();
    s->ntiles_des = (int)ds.size();
    s->ntiles_pml = (int)pm.size();
    s->tiles_host.insert(s->tiles_host.end(), ds.begin(), ds.end());
    s->tiles_host.insert(s->tiles_host.end(), pm.begin(), pm.end());
}

ccpr_status upload_cold(ccpr_solver* s, int st)
{
    plan_chunks(s);
    HIPCHK(hipMemcpyAsync(s->ws + s->lay.zr, s->zr_host.data(), s->zr_host.size() * sizeof(int2),
                          hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->ws + s->lay.tiles, s->tiles_host.data(), s->tiles_host.size() * sizeof(int2),
                          hipMemcpyHostToDevice, s->stream));
    // (no second stream on the static workspace: creating one is a resource
    // allocation its callers cannot make)
    if (s->ntiles_pml > 0 && s->ntiles_int + s->ntiles_des > 0 && !s->stream2 && s->static_dev < 0 &&
        !s->batched) {
        HIPCHK(hipStreamCreateWithFlags(&s->stream2, hipStreamNonBlocking));
        s->own_stream2 = true;
    }
    if (s->stream2 && !s->fork_ev) {
        HIPCHK(hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&s->join_ev, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&s->pdone_ev, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&s->post_ev, hipEventDisableTiming));
    }
    // source and gap cells outside the design are finished in the same post
    // launch as the x-CPML pass of E, so they must lie outside the x layers
    if (s->g.npml > 0) {
        auto off_x_layers = [&](const int* lo, const int* dim) {
            return lo[0] >= s->g.npml && lo[0] + dim[0] <= s->g.nx - s->g.npml;
        };
        const int one[3] = {1, 1, 1};
        if (s->src_kind == 1 && !off_x_layers(s->dip_cell, one))
            return fail(s, CCPR_ENOTSUP, "the dipole cell must lie outside the x CPML layers");
        if (s->has_obj && !off_x_layers(s->glo, s->gdim))
            return fail(s, CCPR_ENOTSUP, "the gap box must lie outside the x CPML layers");
    }
    if (st == 0 && s->src_kind == 2) {
        fill_cold(s, st, s->cold_host[st]);
        ccpr_status e = build_tf(s, s->cold_host[st]);
        if (e) return e;
        HIPCHK(hipMemcpyAsync(s->ws + s->lay.tf, s->tf_host.data(), s->tf_host.size() * sizeof(TfEntry),
                              hipMemcpyHostToDevice, s->stream));
    }
    fill_cold(s, st, s->cold_host[st]);
    fill_classes(s, s->cold_host[st], s->rowf_host[st], s->lanef_host[st]);
    fill_extra(s->cold_host[st], s->extra_host[st]);
    // the fused post launch reads E^{n+1} of the first cell past the low x
    // layer while its other blocks finish the source cells: no source cell
    // may sit there
    s->fuse_ok[st] = 2 * s->g.npml <= 256;
    for (const int4& e : s->extra_host[st])
        if (e.w == CCPR_EXTRA_SOURCE && s->g.npml > 0 && e.x == s->g.npml) s->fuse_ok[st] = false;
    if (!s->extra_host[st].empty())
        HIPCHK(hipMemcpyAsync(s->ws + s->lay.extra[st], s->extra_host[st].data(),
                              s->extra_host[st].size() * sizeof(int4), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->ws + s->lay.cold[st], &s->cold_host[st], sizeof(StepCold),
                          hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->ws + s->lay.rowf[st], s->rowf_host[st].data(), s->rowf_host[st].size() * 4,
                          hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->ws + s->lay.lanef[st], s->lanef_host[st].data(), s->lanef_host[st].size() * 4,
                          hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return CCPR_OK;
}

StepArgs hot_args(ccpr_solver* s, int st)
{
    const Layout& L = s->lay;
    StepArgs A{};
    const int par = s->parity[st];
    A.Ei = wsp<float>(s, L.Eb[st][par]);
    A.Eo = wsp<float>(s, L.Eb[st][par ^ 1]);
    A.Hi = wsp<float>(s, L.Hb[st][par]);
    A.Ho = wsp<float>(s, L.Hb[st][par ^ 1]);
    A.rowf = wsp<unsigned>(s, L.rowf[st]);
    A.lanef = wsp<unsigned>(s, L.lanef[st]);
    A.drive = wsp<float>(s, L.drive);
    A.extra = wsp<int4>(s, L.extra[st]);
    A.nextra = (long long)s->extra_host[st].size();
    A.cstride = (unsigned)(s->npad * 4);
    // nontemporal stores once the double-buffered fields exceed the 256 MB
    // last-level cache (smaller states are reused from it between steps)
    A.stream_st = 48.0 * (double)s->npad > 256.0 * (1 << 20) ? 1 : 0;
    A.nx = s->g.nx; A.ny = s->g.ny; A.nz = s->g.nz;
    A.nxp = s->nxp; A.nyp = s->nyp; A.rows = s->rows;
    A.npml = s->g.npml;
    A.S = (float)s->g.courant;
    A.psi_in = par;
    A.tslot = -1;
    A.mode = 0;
    A.phc = A.phs = 0.f;
    A.cold = wsp<StepCold>(s, L.cold[st]);
    A.halt = wsp<unsigned>(s, L.halt);
    A.zr = wsp<int2>(s, L.zr);
    A.tiles = wsp<int2>(s, L.tiles);
    A.nys = (s->g.ny + s->rows - 1) / s->rows;
    A.nblk = s->ntiles_int;
    return A;
}

// One leapfrog step of state st.  fuse: the next step of this state follows
// at once (no checkpoint or field read in between), so the post launch also
// applies its pre-corrections.
ccpr_status launch_step(ccpr_solver* s, StepArgs& A, int st, bool fuse)
{
    const StepCold& C = s->cold_host[st];
    const long long nxs = s->g.npml > 0 ? 2LL * s->g.npml * s->g.ny * s->g.nz : 0;
    const long long ndes = s->has_design ? s->nd : 0;
    const long long nmisc = A.nextra + (C.pw_on ? C.tf_nE : 0);
    // Ls leads this step (its previous work is the last step's post); with a
    // split pass the other stream Fs runs the interior tiles, aux and post
    // and leads the next step, so the only wait that is not already
    // satisfied (Fs on the fork event) overlaps the CPML-tile launch.
    hipStream_t Ls = s->lead2 ? s->stream2 : s->stream;
    hipStream_t Fs = s->lead2 ? s->stream : s->stream2;
    // the last step's post dispatch records post_ev and nothing follows it on
    // the lead stream (no pre launch either: that post applied it)
    const bool armed = s->post_armed && s->post_armed_st == st && s->pre_done[st];
    s->post_armed = false;
    int e = s->pre_done[st] ? 0 : ccpr_launch_pre(A, nxs, C.pw_on ? C.tf_nH : 0, Ls);
    s->pre_done[st] = false;
    if (s->batched) {
        // record the grid (every tile, CPML variant), aux and post work of
        // this step for the next ccpr_pipe_flush
        if (e != 0) return fail(s, CCPR_EDEVICE, "pre kernel launch: %s", hipGetErrorString((hipError_t)e));
        if (s->rec_pending) return fail(s, CCPR_ESTATE, "internal: a recorded step was not flushed");
        fuse = fuse && s->fuse_ok[st];
        s->rec.a = A;
        s->rec.a.nblk = s->ntiles_int + s->ntiles_des + s->ntiles_pml;
        s->rec.maxpairs = s->maxpairs;
        s->rec.nd = ndes;
        s->rec.fused = fuse ? 1 : 0;
        s->rec.nxs = nxs;
        s->rec.nmisc = nmisc;
        s->rec.ntfh = C.pw_on ? C.tf_nH : 0;
        s->rec_watch = s->watch_run && s->watch_every > 0 && s->has_obj && (A.n + 1) % s->watch_every == 0;
        s->rec_pending = true;
        s->pre_done[st] = fuse;
        s->parity[st] ^= 1;
        return CCPR_OK;
    }
    const bool tm = s->timing && s->timed_loop && (s->pass_no++ % s->timing_every) == 0;
    if (tm) {
        while (s->tev.size() < s->tev_used + 3) {
            hipEvent_t ev;
            HIPCHK(hipEventCreate(&ev));
            s->tev.push_back(ev);
        }
        HIPCHK(hipEventRecord(s->tev[s->tev_used], Ls));
    }
    // grid kernel: CPML tiles and interior tiles as two concurrent launches
    // (both read step-n state only and write disjoint cells); with the design
    // update in the grid pass, the design tiles follow the CPML tiles
    const int nint = s->ntiles_int, ndt = s->ntiles_des, npt = s->ntiles_pml;
    StepArgs Ap = A;
    Ap.tiles = A.tiles + nint + ndt;
    Ap.nblk = npt;
    // the split pays for its fork only with enough tiles on both sides
    const bool split = s->stream2 && nint + ndt >= 1024 && npt >= 128;
    const bool fdes = split && ndt > 0;  // design cells finished in the grid pass
    // interior tiles (with the design tiles unless those run fused)
    StepArgs Ai = A;
    Ai.nblk = fdes ? nint : nint + ndt;
    bool two = false;
    hipStream_t As = Ls;  // stream of aux and post
    if (e == 0) {
        if (nint + ndt == 0 || (!split && npt > 0)) {
            Ap.tiles = A.tiles;  // one launch over all tiles
            Ap.nblk = nint + ndt + npt;
            e = ccpr_launch_grid(Ap, true, Ls);
        } else if (npt == 0) {
            e = ccpr_launch_grid(Ai, false, Ls);
        } else {
            // the slower CPML tiles go first; the interior tiles fill the
            // device around them; aux waits for the CPML launch too (normally
            // long finished by then)
            // the fork is the last post dispatch's own event where it can be,
            // and the CPML dispatch records "CPML done" itself: an event
            // record between two kernels costs a marker packet (≈ 1 µs per
            // step, measured); on a timed pass the timing events double as
            // the fork and "CPML done" events
            const bool att = !tm && !fdes;
            hipEvent_t fork = tm ? s->tev[s->tev_used] : (armed ? s->post_ev : s->fork_ev);
            hipEvent_t pdone = tm ? s->tev[s->tev_used + 1] : s->pdone_ev;
            if (!tm && !armed) HIPCHK(hipEventRecord(fork, Ls));
            StepArgs Ad = A;
            Ad.tiles = A.tiles + nint;
            Ad.nblk = ndt;
            e = ccpr_launch_grid(Ap, true, Ls, nullptr, att ? pdone : nullptr);
            if (e == 0 && fdes) e = ccpr_launch_grid_des(Ad, s->maxpairs, Ls);
            if (!att) HIPCHK(hipEventRecord(pdone, Ls));
            HIPCHK(hipStreamWaitEvent(Fs, fork, 0));
            if (e == 0) e = ccpr_launch_grid(Ai, false, Fs);
            if (tm) HIPCHK(hipEventRecord(s->tev[s->tev_used + 2], Fs));
            HIPCHK(hipStreamWaitEvent(Fs, pdone, 0));
            As = Fs;
            s->lead2 = !s->lead2;
            two = true;
        }
    }
    // timed pass: start before the first launch, end with the later of the
    // two launches
    if (tm) {
        if (!two) {
            HIPCHK(hipEventRecord(s->tev[s->tev_used + 1], Ls));
            HIPCHK(hipEventRecord(s->tev[s->tev_used + 2], Ls));
        }
        s->tev_used += 3;
    }
    // aux and post touch disjoint cells but share the device better in
    // sequence than side by side (measured)
    if (e == 0 && !fdes) e = ccpr_launch_aux(A, s->maxpairs, ndes, s->edge, As);
    fuse = fuse && s->fuse_ok[st];
    const bool watch = s->watch_run && s->watch_every > 0 && s->has_obj && (A.n + 1) % s->watch_every == 0;
    // the next step of this state follows at once: its fork is this dispatch
    const bool arm = fuse && !watch && s->post_ev;
    if (e == 0)
        e = fuse ? ccpr_launch_post_fused(A, nmisc, C.pw_on ? C.tf_nH : 0, As, arm ? s->post_ev : nullptr)
                 : ccpr_launch_post(A, nxs, nmisc, As);
    if (e == 0 && arm) {
        s->post_armed = true;
        s->post_armed_st = st;
    }
    if (e == 0 && watch)
        e = ccpr_launch_watch(A, s->glo, s->gdim, (float)s->watch_limit, A.n, wsp<unsigned>(s, s->lay.halt),
                              wsp<double>(s, s->lay.scal), As);
    if (e != 0) return fail(s, CCPR_EDEVICE, "step kernel launch: %s", hipGetErrorString((hipError_t)e));
    s->pre_done[st] = fuse;
    s->parity[st] ^= 1;
    return CCPR_OK;
}

// Marks a forward / adjoint loop: launch_step runs the divergence watchdog
// only inside one.
struct WatchScope {
    ccpr_solver* s;
    explicit WatchScope(ccpr_solver* x) : s(x) { s->watch_run = true; }
    ~WatchScope() { s->watch_run = false; }
};

// Re-arm the divergence watchdog (halt word and the step it records).
ccpr_status clear_halt(ccpr_solver* s)
{
    HIPCHK(ccpr_launch_fill(wsp<float>(s, s->lay.halt), 2, 0.f, s->stream));
    HIPCHK(ccpr_launch_fill_d(wsp<double>(s, s->lay.scal) + 7, 1, 0.0, s->stream));
    return CCPR_OK;
}

// Forward step n of a full run starts a segment whose state is saved as a
// checkpoint (slot seg-1): segments 1 .. S-R-1, the ones the adjoint recomputes.
bool saves_checkpoint(const Layout& L, int n)
{
    if (L.K <= 0 || n % L.K != 0) return false;
    const int seg = n / L.K;
    return seg >= 1 && seg < L.S - L.R;
}

// History slot of forward step n during the forward run: resident segments
// (the last R) keep their records, in order; -1 for the recomputed ones.
int forward_slot(const Layout& L, int n)
{
    const int seg = n / L.K, first = L.S - L.R;
    return seg >= first ? n - first * L.K : -1;
}

// First history slot of segment seg during the adjoint run: a resident
// segment's own place, or slot 0 where a recomputed segment is written.
int segment_base(const Layout& L, int seg)
{
    const int first = L.S - L.R;
    return seg >= first ? (seg - first) * L.K : 0;
}

// Whether forward step m of a full run follows its predecessor at once: not
// past the end and not after a checkpoint save (which must see the plain state).
bool fuse_forward(const ccpr_solver* s, int m)
{
    if (m >= s->M) return false;
    return !saves_checkpoint(s->lay, m);
}

// One forward step n of the forward state; tslot >= 0 records the gradient
// factor of this step into that history slot.
ccpr_status forward_step(ccpr_solver* s, int n, int tslot, bool gap, bool fuse)
{
    StepArgs A = hot_args(s, 0);
    A.n = n;
    A.mode = gap && s->has_obj ? CCPR_MODE_GAP : 0;
    if (s->grad_dft) {
        // DFT mode: T_hat += T^{n+1/2} exp(-j omega dt n) instead of the history
        const double ph = s->omega * s->dt * n;
        A.mode |= CCPR_MODE_DFT_T;
        A.phc = (float)std::cos(ph);
        A.phs = (float)std::sin(ph);
    } else {
        A.tslot = tslot;
        if (tslot >= 0) A.mode |= CCPR_MODE_RECORD;
    }
    return launch_step(s, A, 0, fuse);
}

// Adjoint step p = M-1-n (it pairs with forward step n, whose record is in
// history slot n - n0): time-exact correlation with that slot, or, in DFT
// mode, the projection of the new adjoint field Et^{p+1} when it lies in the
// fit window.
ccpr_status adjoint_step(ccpr_solver* s, int n, int n0, bool fuse)
{
    StepArgs A = hot_args(s, 1);
    const int p = s->M - 1 - n;
    A.n = p;
    if (s->grad_dft) {
        const int m = p + 1;
        if (m >= s->M - dft_window(s->M, s->omega, s->dt) + 1) {
            const double ph = s->omega * s->dt * m;
            A.mode = CCPR_MODE_DFT_P;
            A.phc = (float)std::cos(ph);
            A.phs = (float)std::sin(ph);
        }
    } else {
        A.tslot = n - n0;
        A.mode = CCPR_MODE_CORREL;
    }
    return launch_step(s, A, 1, fuse);
}

// DFT mode, after the adjoint run: the window's least-squares normal matrix
// (host FP64) and the per-voxel gradient into the accumulator.
ccpr_status dft_finish(ccpr_solver* s)
{
    {
        ccpr_status j = join_lead(s);
        if (j) return j;
    }
    const int M = s->M, Lw = dft_window(M, s->omega, s->dt);
    const double th = s->omega * s->dt;
    double scc = 0, sss = 0, scs = 0;
    for (int m = M - Lw + 1; m <= M; ++m) {
        const double c = std::cos(th * m), sn = std::sin(th * m);
        scc += c * c;
        sss += sn * sn;
        scs += c * sn;
    }
    const double det = scc * sss - scs * scs;
    if (!(det > 0)) return fail(s, CCPR_EINVAL, "DFT-mode fit window is degenerate (omega dt a multiple of pi?)");
    const EdgeMap em = edge_map(s);
    HIPCHK(ccpr_launch_dft_grad(wsp<double>(s, s->lay.gradacc), wsp<float>(s, s->lay.T), s->nd, s->ddim, em, sss / det,
                                -scs / det, scc / det, std::cos(th * M), std::sin(th * M), s->stream));
    return CCPR_OK;
}

// add the recorded grid-kernel event triples to the statistics (the stream is
// synchronised by the caller)
ccpr_status harvest_grid_events(ccpr_solver* s)
{
    for (size_t q = 0; q + 2 < s->tev_used; q += 3) {
        float m1 = 0, m2 = 0;
        HIPCHK(hipEventElapsedTime(&m1, s->tev[q], s->tev[q + 1]));
        HIPCHK(hipEventElapsedTime(&m2, s->tev[q], s->tev[q + 2]));
        s->stat_grid_ms += std::max(m1, m2);
        s->stat_grid_launches += 1;
    }
    s->tev_used = 0;
    return CCPR_OK;
}

// copy the forward state (current parity) to / from checkpoint slot c
ccpr_status checkpoint(ccpr_solver* s, int slot, bool save)
{
    {
        ccpr_status j = join_lead(s);
        if (j) return j;
    }
    // a checkpoint holds the plain state between two steps
    if (save && s->pre_done[0]) return fail(s, CCPR_EDEVICE, "internal: checkpoint of a pre-corrected state");
    if (!save) s->pre_done[0] = false;
    const Layout& L = s->lay;
    float* ck = wsp<float>(s, L.ckpt + (size_t)slot * align256(L.ckpt_bytes));
    const int par = save ? s->parity[0] : 0;
    const long long nc3 = 3 * s->npad, nj = 2LL * s->npairs_total * std::max(s->nd, 1LL);
    const long long psi = psi_total(s);
    struct { float* dev; long long n; } parts[5] = {
        {wsp<float>(s, L.Eb[0][par]), nc3},
        {wsp<float>(s, L.Hb[0][par]), nc3},
        {wsp<float>(s, L.Jb[0]), nj},
        {wsp<float>(s, L.psiE[0]), psi},
        {wsp<float>(s, L.psiH[0][par]), psi},
    };
    long long off = 0;
    for (auto& p : parts) {
        if (save) HIPCHK(ccpr_launch_copy(ck + off, p.dev, p.n, s->stream));
        else HIPCHK(ccpr_launch_copy(p.dev, ck + off, p.n, s->stream));
        off += p.n;
    }
    // FP64 shadow of the dipole edge (the forward source box is one cell)
    double* cks = reinterpret_cast<double*>(ck + ((off + 1) & ~1LL));
    if (save) HIPCHK(ccpr_launch_copy_d(cks, wsp<double>(s, L.ssh[0]), 3, s->stream));
    else HIPCHK(ccpr_launch_copy_d(wsp<double>(s, L.ssh[0]), cks, 3, s->stream));
    if (!save) s->parity[0] = 0;
    return CCPR_OK;
}

ccpr_status check_ready(ccpr_solver* s, bool need_obj)
{
    ccpr_status st = need_bound(s);
    if (st) return st;
    if (s->src_kind == 0) return fail(s, CCPR_ESTATE, "no source set");
    if (need_obj && !s->has_obj) return fail(s, CCPR_ESTATE, "no objective set");
    if (need_obj && !s->has_design) return fail(s, CCPR_ESTATE, "no design set");
    if (need_obj && s->grad_dft && (s->obj_kind != CCPR_OBJ_DFT_E2 || !(s->omega > 0)))
        return fail(s, CCPR_EINVAL, "the DFT gradient mode needs the DFT objective (omega > 0)");
    return CCPR_OK;
}

void build_mats(ccpr_solver* s)
{
    int jofs = 0;
    for (int ax = 0; ax < 3; ++ax) {
        axis_mat(s, ax, jofs, s->mats[ax]);
        jofs += pairs_on_axis(s, ax);
    }
}

// Re-carve the fixed part of the workspace when the configuration that sizes
// it (design voxels, pole pairs, gap cells) changed; re-upload what lives
// there and zero both states.
ccpr_status refresh_fixed(ccpr_solver* s, bool force)
{
    if (!s->ws) return CCPR_OK;
    Layout L = make_layout(s, 0, 0);
    if (L.fixed_end > s->ws_bytes)
        return fail(s, CCPR_ENOMEM, "workspace of %llu bytes, need at least %llu", (unsigned long long)s->ws_bytes,
                    (unsigned long long)L.fixed_end);
    const long long key[4] = {s->nd, s->npairs_total, s->gncell, (long long)L.fixed_end};
    const bool changed = force || std::memcmp(key, s->fixed_key, sizeof key) != 0;
    s->lay = L;
    if (!changed) return CCPR_OK;
    std::memcpy(s->fixed_key, key, sizeof key);
    ccpr_status st = upload_static(s);
    if (st) return st;
    s->rho_uploaded = false;
    if (!s->rho_on_host && s->has_design) s->has_design = false;  // device densities must be set again
    HIPCHK(ccpr_launch_fill_d(wsp<double>(s, s->lay.scal), 16, 0.0, s->stream));
    st = clear_halt(s);
    if (st) return st;
    st = zero_state(s, 0);
    if (st) return st;
    st = zero_state(s, 1);
    if (st) return st;
    s->src_table_steps = -1;
    s->step_count = 0;
    s->have_forward = s->have_adjoint = false;
    return upload_rho(s);
}

ccpr_status adopt_layout(ccpr_solver* s, int M)
{
    ccpr_status st0 = refresh_fixed(s, false);
    if (st0) return st0;
    build_mats(s);
    int K = s->ckpt_every;
    const int rmax = s->resident_max;
    Layout L = make_layout(s, M, K);
    // most resident segments (fewest recomputed steps) that fit, for segment
    // length Kt
    auto best_r = [&](int Kt) {
        Layout b = make_layout(s, M, Kt, 1);
        const int lim = rmax > 0 ? std::min(rmax, b.S) : b.S;
        for (int r = lim; r > 1; --r) {
            Layout t = make_layout(s, M, Kt, r);
            if (t.total <= s->ws_bytes) return t;
        }
        return b;
    };
    auto recomputed = [&](const Layout& t) { return (t.S - t.R) * t.K; };  // the last segment is resident
    if (M > 0 && !s->grad_dft) {
        if (K > 0) {
            L = best_r(K);
        } else if (L.total > s->ws_bytes) {
            // the whole history does not fit: choose the segment length that
            // recomputes the fewest steps (then the fewest segments)
            bool found = false;
            for (int S = 2; S <= std::min(M, 128); ++S) {
                const int Kt = (M + S - 1) / S;
                Layout t = best_r(Kt);
                if (t.total > s->ws_bytes) continue;
                if (!found || recomputed(t) < recomputed(L)) L = t;
                found = true;
            }
            if (!found) {
                // fall back to the smallest segment count that fits with one resident segment
                for (int S = 129; S <= M; ++S) {
                    L = make_layout(s, M, (M + S - 1) / S);
                    if (L.total <= s->ws_bytes) break;
                }
            }
        }
    }
    if (L.total > s->ws_bytes)
        return fail(s, CCPR_ENOMEM, "workspace of %llu bytes, need %llu", (unsigned long long)s->ws_bytes,
                    (unsigned long long)L.total);
    s->lay = L;
    return CCPR_OK;
}

// Objective of the finished forward run (gap record -> F', adjoint source
// table) and its SI values on the device (scal[4..6]).
ccpr_status launch_objective(ccpr_solver* s)
{
    {
        ccpr_status j = join_lead(s);
        if (j) return j;
    }
    const Layout& L = s->lay;
    const int M = s->M;
    const int ne = s->gncell * 3;
    const int nend = s->ne < 0 ? M + 1 : s->ne;
    const int kind = s->obj_kind == CCPR_OBJ_DFT_E2 ? 1 : 0;
    HIPCHK(ccpr_launch_objective(wsp<float>(s, L.gap), M, ne, kind, s->omega * s->dt, s->nb, nend,
                                 wsp<double>(s, L.scal), wsp<double>(s, L.work), wsp<float>(s, L.src_adj),
                                 s->stream));
    HIPCHK(ccpr_launch_finish(wsp<double>(s, L.scal), kind, s->alpha, s->dt, s->g.dx, kEps0, s->stream));
    return CCPR_OK;
}

// Host copy of scal[0..7] after a forward run: validity checks and the SI values.
ccpr_status check_results(ccpr_solver* s, const double* scal)
{
    if (!s->rho_on_host && scal[2] != 0.0)
        return fail(s, CCPR_EINVAL, "device densities must be finite and within [0,1]");
    s->F = scal[4];
    s->grad_scale = scal[5];
    s->adj_alpha = scal[6];
    if (scal[7] > 0) {
        s->step_count = (int)scal[7];
        return fail(s, CCPR_EDIVERGED,
                    "the fields diverged: the watchdog found a gap-box field above %g (or not finite) after %d steps",
                    s->watch_limit, (int)scal[7]);
    }
    if (!std::isfinite(s->F) || !std::isfinite(scal[1]))
        return fail(s, CCPR_EDIVERGED, "objective is not finite: the fields diverged");
    return CCPR_OK;
}

// Shared by ccpr_set_design (edge = false: one density per voxel of dims)
// and ccpr_set_design_edges (edge = true: dims cells, one density per E edge,
// kernel box of dims + 1 cells).
ccpr_status set_design_common(ccpr_solver* s, const int lo[3], const int dims[3], double gamma, const float* rho,
                              int mem, bool edge)
{
    if (!s) return CCPR_EINVAL;
    if (!lo || !dims || !rho || (mem != CCPR_MEM_HOST && mem != CCPR_MEM_DEVICE))
        return fail(s, CCPR_EINVAL, "bad design arguments");
    const int n3[3] = {s->g.nx, s->g.ny, s->g.nz};
    const int m = std::max(s->g.npml, 1);
    int box[3];
    for (int a = 0; a < 3; ++a) {
        if (dims[a] < 1) return fail(s, CCPR_EINVAL, "design dimensions must be positive");
        box[a] = dims[a] + (edge ? 1 : 0);
        if (lo[a] < m || lo[a] + box[a] > n3[a] - s->g.npml)
            return fail(s, CCPR_EINVAL, edge ? "design box (with the far-face edges) must lie inside the grid, "
                                               "off the walls and outside the CPML"
                                             : "design box must lie inside the grid, off the walls and outside the CPML");
    }
    if (!std::isfinite(gamma) || gamma < 0) return fail(s, CCPR_EINVAL, "gamma must be finite and >= 0");
    const long long nd = (long long)box[0] * box[1] * box[2];
    if (nd > 0x7fffffffLL) return fail(s, CCPR_ENOTSUP, "design box above 2^31 voxels");
    long long nr = nd;
    if (edge) {
        nr = 0;
        for (int c = 0; c < 3; ++c)
            nr += (long long)(dims[0] + (c != 0)) * (dims[1] + (c != 1)) * (dims[2] + (c != 2));
    }
    if (mem == CCPR_MEM_HOST) {
        for (long long v = 0; v < nr; ++v)
            if (!(rho[v] >= 0.f && rho[v] <= 1.f))
                return fail(s, CCPR_EINVAL, "density %lld is %g: must be finite and in [0,1]", v, (double)rho[v]);
    } else if (!s->ws) {
        return fail(s, CCPR_ESTATE, "device densities need a bound workspace");
    }
    for (int a = 0; a < 3; ++a) { s->dlo[a] = lo[a]; s->ddim[a] = box[a]; s->ncl[a] = dims[a]; }
    s->nd = nd;
    s->edge = edge;
    s->nrho = nr;
    s->gamma = gamma;
    s->have_forward = s->have_adjoint = false;
    if (mem == CCPR_MEM_HOST) {
        s->rho_host.assign(rho, rho + nr);
        s->rho_on_host = true;
        s->rho_uploaded = false;
        s->has_design = true;
        ccpr_status st = refresh_fixed(s, false);
        if (st) return st;
        return upload_rho(s);
    } else {
        s->rho_on_host = false;
        s->rho_host.clear();
        s->has_design = true;
        ccpr_status st = refresh_fixed(s, false);
        if (st) return st;
        s->has_design = true;
        HIPCHK(hipMemcpyAsync(s->ws + s->lay.rho, rho, nr * 4, hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(ccpr_launch_fill_d(wsp<double>(s, s->lay.scal) + 2, 1, 0.0, s->stream));
        HIPCHK(ccpr_launch_check_rho(wsp<float>(s, s->lay.rho), nr, wsp<double>(s, s->lay.scal) + 2, s->stream));
    }
    return CCPR_OK;
}

// ---- static workspace (ccpr_bind_static_workspace)
// The library's own device memory for callers that cannot allocate: a
// file-scope array that each device holds from the first bind on it until
// the process ends.  In host code its name is only a stand-in; the device
// address comes from hipGetSymbolAddress, once per device with that device
// current, and is the only handle host code uses.  One solver at a time is
// bound to a device's array (a new bind unbinds the previous solver).
constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxStaticDevices];
ccpr_solver* g_static_owner[kMaxStaticDevices];

// Forget the static workspace of s's device if s holds it (lock held).
void release_static_locked(ccpr_solver* s)
{
    if (s->static_dev >= 0 && g_static_owner[s->static_dev] == s) g_static_owner[s->static_dev] = nullptr;
    s->static_dev = -1;
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[CCPR_STATIC_WORKSPACE_BYTES];

// ======================================================================= ABI
extern "C" {

ccpr_status ccpr_create(const ccpr_grid* g, ccpr_solver** out)
{
    if (!out) return fail(nullptr, CCPR_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) return fail(nullptr, CCPR_EINVAL, "grid is NULL");
    if (g->nx < 2 || g->ny < 2 || g->nz < 2) return fail(nullptr, CCPR_EINVAL, "grid must be at least 2 cells per axis");
    if (!(g->dx > 0) || !std::isfinite(g->dx)) return fail(nullptr, CCPR_EINVAL, "dx must be positive");
    if (!(g->courant > 0) || !std::isfinite(g->courant)) return fail(nullptr, CCPR_EINVAL, "courant must be positive");
    if (g->courant > 1.0 / std::sqrt(3.0) + 1e-12)
        return fail(nullptr, CCPR_ECFL, "courant %g exceeds the 3-D Yee limit 1/sqrt(3)", g->courant);
    if (g->npml < 0 || 2 * g->npml + 2 > std::min(g->nx, std::min(g->ny, g->nz)))
        return fail(nullptr, CCPR_EINVAL, "CPML thickness %d too large for the grid", g->npml);
    if (g->npml > 0 && (!(g->pml_order >= 0) || !(g->pml_kappa_max >= 1) || !(g->pml_alpha_max >= 0) ||
                        !(g->pml_sigma_scale >= 0)))
        return fail(nullptr, CCPR_EINVAL, "bad CPML grading parameters");
    if (g->nx > CCPR_MAX_NX) return fail(nullptr, CCPR_ENOTSUP, "nx %d exceeds %d", g->nx, CCPR_MAX_NX);
    ccpr_solver* s = new ccpr_solver();
    s->g = *g;
    s->dt = g->courant * g->dx / kC0;
    s->ncell = (long long)g->nx * g->ny * g->nz;
    s->nxp = (g->nx + 63) / 64 * 64;
    s->nyp = (g->ny + CCPR_YPAD - 1) / CCPR_YPAD * CCPR_YPAD + 2;
    s->nzp = g->nz + 2;
    s->npad = (long long)s->nxp * s->nyp * s->nzp;
    if (s->npad * 4 >= 0xffffffffLL) {
        delete s;
        return fail(nullptr, CCPR_ENOTSUP, "grid too large: a padded field component exceeds 2^30 floats");
    }
    *out = s;
    return CCPR_OK;
}

void ccpr_destroy(ccpr_solver* s)
{
    if (!s) return;
    if (s->ws) (void)hipStreamSynchronize(s->stream);
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        release_static_locked(s);
    }
    for (hipEvent_t ev : s->tev) (void)hipEventDestroy(ev);
    if (s->stream2) (void)hipStreamSynchronize(s->stream2);
    if (s->fork_ev) (void)hipEventDestroy(s->fork_ev);
    if (s->join_ev) (void)hipEventDestroy(s->join_ev);
    if (s->pdone_ev) (void)hipEventDestroy(s->pdone_ev);
    if (s->post_ev) (void)hipEventDestroy(s->post_ev);
    if (s->stream2 && s->own_stream2) (void)hipStreamDestroy(s->stream2);
    delete s;
}

const char* ccpr_last_error(const ccpr_solver* s) { return s ? s->err.c_str() : g_create_err.c_str(); }

ccpr_status ccpr_set_material(ccpr_solver* s, int slot, int axis, double eps_inf, double sigma, int npairs,
                              const double* a, const double* c)
{
    if (!s) return CCPR_EINVAL;
    if (slot < 1 || slot > 2 || axis < 0 || axis > 2 || npairs < 0 || (npairs > 0 && (!a || !c)))
        return fail(s, CCPR_EINVAL, "bad material arguments");
    if (!std::isfinite(eps_inf) || !std::isfinite(sigma) || eps_inf <= 0 || sigma < 0)
        return fail(s, CCPR_EINVAL, "eps_inf must be positive and sigma non-negative");
    MatHost m;
    m.eps = eps_inf;
    m.sig = sigma;
    for (int p = 0; p < npairs; ++p) {
        for (int q = 0; q < 2; ++q)
            if (!std::isfinite(a[2 * p + q]) || !std::isfinite(c[2 * p + q]))
                return fail(s, CCPR_EINVAL, "non-finite pole or residue");
        // a pole in the right half plane grows without any field driving it
        if (a[2 * p] > 0) return fail(s, CCPR_EINVAL, "pole pair %d has Re a > 0 (a growing, non-passive pole)", p);
        m.a.push_back(cd(a[2 * p], a[2 * p + 1]));
        m.c.push_back(cd(c[2 * p], c[2 * p + 1]));
    }
    const int other = (int)s->mat[2 - slot][axis].a.size();
    if (npairs + other > CCPR_MAX_PAIRS_PER_AXIS)
        return fail(s, CCPR_ENOTSUP, "%d pole pairs on axis %d exceed %d", npairs + other, axis,
                    CCPR_MAX_PAIRS_PER_AXIS);
    s->mat[slot - 1][axis] = m;
    recount_pairs(s);
    s->have_forward = s->have_adjoint = false;
    return refresh_fixed(s, false);
}

ccpr_status ccpr_set_design(ccpr_solver* s, const int lo[3], const int dims[3], double gamma, const float* rho,
                            int mem)
{
    return set_design_common(s, lo, dims, gamma, rho, mem, false);
}

ccpr_status ccpr_set_design_edges(ccpr_solver* s, const int lo[3], const int dims[3], double gamma,
                                  const float* rho, int mem)
{
    return set_design_common(s, lo, dims, gamma, rho, mem, true);
}

ccpr_status ccpr_set_source_dipole(ccpr_solver* s, const int cell[3], int axis, const double* wave, int nsteps)
{
    if (!s) return CCPR_EINVAL;
    if (!cell || axis < 0 || axis > 2 || nsteps < 1 || !wave) return fail(s, CCPR_EINVAL, "bad dipole arguments");
    const int n3[3] = {s->g.nx, s->g.ny, s->g.nz};
    for (int a = 0; a < 3; ++a)
        if (cell[a] < 0 || cell[a] >= n3[a]) return fail(s, CCPR_EINVAL, "dipole cell outside the grid");
    for (int n = 0; n < nsteps; ++n)
        if (!std::isfinite(wave[n])) return fail(s, CCPR_EINVAL, "non-finite waveform sample");
    s->src_kind = 1;
    for (int a = 0; a < 3; ++a) s->dip_cell[a] = cell[a];
    s->dip_axis = axis;
    s->wave.assign(wave, wave + nsteps);
    s->src_table_steps = -1;
    s->have_forward = s->have_adjoint = false;
    return CCPR_OK;
}

ccpr_status ccpr_set_source_planewave(ccpr_solver* s, int prop_axis, int sign, int pol_axis, const int lo[3],
                                      const int hi[3], const double* wave, int nsteps)
{
    if (!s) return CCPR_EINVAL;
    if (prop_axis < 0 || prop_axis > 2 || pol_axis < 0 || pol_axis > 2 || prop_axis == pol_axis ||
        (sign != 1 && sign != -1) || !lo || !hi || !wave || nsteps < 1)
        return fail(s, CCPR_EINVAL, "bad plane-wave arguments");
    const int n3[3] = {s->g.nx, s->g.ny, s->g.nz};
    for (int a = 0; a < 3; ++a)
        if (lo[a] < s->g.npml + 1 || hi[a] <= lo[a] || hi[a] > n3[a] - s->g.npml - 2)
            return fail(s, CCPR_EINVAL, "TF/SF box must lie strictly inside the grid and outside the CPML");
    for (int n = 0; n < nsteps; ++n)
        if (!std::isfinite(wave[n])) return fail(s, CCPR_EINVAL, "non-finite waveform sample");
    s->src_kind = 2;
    s->pw_d = prop_axis;
    s->pw_sgn = sign;
    s->pw_p = pol_axis;
    for (int a = 0; a < 3; ++a) { s->pw_lo[a] = lo[a]; s->pw_hi[a] = hi[a]; }
    s->wave.assign(wave, wave + nsteps);
    s->src_table_steps = -1;
    s->have_forward = s->have_adjoint = false;
    return CCPR_OK;
}

ccpr_status ccpr_set_objective(ccpr_solver* s, int kind, const int lo[3], const int dims[3], double omega,
                               int n_begin, int n_end)
{
    if (!s) return CCPR_EINVAL;
    if ((kind != CCPR_OBJ_TIME_E2 && kind != CCPR_OBJ_DFT_E2) || !lo || !dims || !std::isfinite(omega))
        return fail(s, CCPR_EINVAL, "bad objective arguments");
    const int n3[3] = {s->g.nx, s->g.ny, s->g.nz};
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1 || lo[a] < 1 || lo[a] + dims[a] > n3[a])
            return fail(s, CCPR_EINVAL, "gap box outside the grid");
    if ((long long)dims[0] * dims[1] * dims[2] > 65536) return fail(s, CCPR_ENOTSUP, "gap box above 65536 cells");
    s->obj_kind = kind;
    for (int a = 0; a < 3; ++a) { s->glo[a] = lo[a]; s->gdim[a] = dims[a]; }
    s->gncell = dims[0] * dims[1] * dims[2];
    s->omega = omega;
    s->nb = n_begin;
    s->ne = n_end;
    s->has_obj = true;
    s->have_forward = s->have_adjoint = false;
    return refresh_fixed(s, false);
}

ccpr_status ccpr_set_checkpointing(ccpr_solver* s, int every)
{
    if (!s) return CCPR_EINVAL;
    if (every < 0) return fail(s, CCPR_EINVAL, "checkpoint_every must be >= 0");
    s->ckpt_every = every;
    return CCPR_OK;
}

ccpr_status ccpr_set_gradient_mode(ccpr_solver* s, int mode)
{
    if (!s) return CCPR_EINVAL;
    if (mode != CCPR_GRAD_TIME_EXACT && mode != CCPR_GRAD_DFT) return fail(s, CCPR_EINVAL, "unknown gradient mode");
    s->grad_dft = mode == CCPR_GRAD_DFT;
    s->have_forward = s->have_adjoint = false;
    return CCPR_OK;
}

ccpr_status ccpr_workspace_size(const ccpr_solver* s, int nsteps, uint64_t* bytes)
{
    if (!s || !bytes || nsteps < 0) return CCPR_EINVAL;
    *bytes = make_layout(s, nsteps, s->ckpt_every).total;
    return CCPR_OK;
}

ccpr_status ccpr_workspace_size_max(const ccpr_solver* s, int nsteps, uint64_t* bytes)
{
    if (!s || !bytes || nsteps < 0) return CCPR_EINVAL;
    const Layout L = make_layout(s, nsteps, s->ckpt_every);
    const int r = s->resident_max > 0 ? std::min(s->resident_max, L.S) : L.S;
    *bytes = make_layout(s, nsteps, s->ckpt_every, r).total;
    return CCPR_OK;
}

ccpr_status ccpr_set_resident_segments(ccpr_solver* s, int max_resident)
{
    if (!s) return CCPR_EINVAL;
    if (max_resident < 0) return fail(s, CCPR_EINVAL, "resident segments must be >= 0");
    s->resident_max = max_resident;
    return CCPR_OK;
}

ccpr_status ccpr_bind_workspace(ccpr_solver* s, void* dev_ptr, uint64_t bytes, void* hip_stream)
{
    if (!s) return CCPR_EINVAL;
    if (!dev_ptr || ((uintptr_t)dev_ptr & 255)) return fail(s, CCPR_EINVAL, "workspace must be 256-byte aligned");
    Layout L = make_layout(s, 0, 0);
    if (L.fixed_end > bytes) return fail(s, CCPR_ENOMEM, "workspace of %llu bytes, need at least %llu",
                                         (unsigned long long)bytes, (unsigned long long)L.total);
    if (s->ws) (void)hipStreamSynchronize(s->stream);
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        release_static_locked(s);
    }
    s->ws = (char*)dev_ptr;
    s->ws_bytes = bytes;
    s->stream = (hipStream_t)hip_stream;
    s->lay = L;
    return refresh_fixed(s, true);
}

ccpr_status ccpr_bind_static_workspace(ccpr_solver* s, void* hip_stream)
{
    if (!s) return CCPR_EINVAL;
    Layout L = make_layout(s, 0, 0);
    if (L.fixed_end > CCPR_STATIC_WORKSPACE_BYTES)
        return fail(s, CCPR_ENOMEM, "the fixed part of this solve's workspace is %llu bytes: above the %llu-byte "
                                    "static workspace", (unsigned long long)L.fixed_end,
                    (unsigned long long)CCPR_STATIC_WORKSPACE_BYTES);
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxStaticDevices) return fail(s, CCPR_ENOTSUP, "device %d: no static workspace", dev);
    if (s->ws) (void)hipStreamSynchronize(s->stream);
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (!g_static_ptr[dev]) {
            // once per device, with that device current
            hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(s, CCPR_EDEVICE, "hipGetSymbolAddress(static workspace): %s", hipGetErrorString(e));
            g_static_ptr[dev] = ptr;
        }
        ptr = g_static_ptr[dev];
        ccpr_solver* prev = g_static_owner[dev];
        if (prev && prev != s) {
            // the previous solver loses the array: its calls now report that
            // no workspace is bound
            if (prev->ws) (void)hipStreamSynchronize(prev->stream);
            prev->ws = nullptr;
            prev->ws_bytes = 0;
            prev->have_forward = prev->have_adjoint = false;
            prev->static_dev = -1;
            std::memset(prev->fixed_key, 0xff, sizeof prev->fixed_key);
        }
        release_static_locked(s);
        g_static_owner[dev] = s;
        s->static_dev = dev;
    }
    s->ws = (char*)ptr;
    s->ws_bytes = CCPR_STATIC_WORKSPACE_BYTES;
    s->stream = (hipStream_t)hip_stream;
    s->lay = L;
    return refresh_fixed(s, true);
}

ccpr_status ccpr_reset(ccpr_solver* s)
{
    if (!s) return CCPR_EINVAL;
    ccpr_status st = need_bound(s);
    if (st) return st;
    s->step_count = 0;
    s->current_state = 0;
    st = clear_halt(s);
    if (st) return st;
    return zero_state(s, 0);
}

ccpr_status ccpr_step(ccpr_solver* s, int n)
{
    if (!s) return CCPR_EINVAL;
    if (n < 0) return fail(s, CCPR_EINVAL, "negative step count");
    ccpr_status st = check_ready(s, false);
    if (st) return st;
    if (s->src_table_steps < 0 || s->src_table_steps != s->lay.inc_steps || s->have_forward) {
        st = adopt_layout(s, 0);
        if (st) return st;
        st = upload_rho(s);
        if (st) return st;
        st = prepare_source(s, s->lay.inc_steps);
        if (st) return st;
        s->have_forward = s->have_adjoint = false;
    }
    if (s->src_kind == 2 && s->step_count + n > s->lay.inc_steps)
        return fail(s, CCPR_ENOTSUP, "plane-wave stepping is limited to the waveform length (%d steps)",
                    s->lay.inc_steps);
    build_mats(s);
    st = upload_cold(s, 0);
    if (st) return st;
    st = clear_halt(s);
    if (st) return st;
    s->current_state = 0;
    for (int q = 0; q < n; ++q) {
        st = forward_step(s, s->step_count, -1, false, q + 1 < n);
        if (st) return st;
        s->step_count++;
    }
    return join_lead(s);
}

int ccpr_step_count(const ccpr_solver* s) { return s ? s->step_count : -1; }

ccpr_status ccpr_get_field(ccpr_solver* s, int comp, float* out, int mem)
{
    if (!s) return CCPR_EINVAL;
    if (comp < 0 || comp > 5 || !out || (mem != CCPR_MEM_HOST && mem != CCPR_MEM_DEVICE))
        return fail(s, CCPR_EINVAL, "bad get_field arguments");
    ccpr_status st = need_bound(s);
    if (st) return st;
    const int state = s->current_state;
    const double a = state == 0 ? s->alpha : s->adj_alpha;
    const double eta0 = std::sqrt(kMu0 / kEps0);
    const float f = (float)(comp < 3 ? 1.0 / a : 1.0 / (a * eta0));
    const int par = s->parity[state];
    const float* src = comp < 3 ? wsp<float>(s, s->lay.Eb[state][par]) : wsp<float>(s, s->lay.Hb[state][par]);
    const int cc = comp % 3;
    if (mem == CCPR_MEM_DEVICE) {
        HIPCHK(ccpr_launch_extract(out, src, cc, s->g.nx, s->g.ny, s->g.nz, s->nxp, s->nyp, f, s->stream));
    } else {
        float* stage = wsp<float>(s, s->lay.stage);
        HIPCHK(ccpr_launch_extract(stage, src, cc, s->g.nx, s->g.ny, s->g.nz, s->nxp, s->nyp, f, s->stream));
        HIPCHK(hipMemcpyAsync(out, stage, s->ncell * 4, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    return CCPR_OK;
}

ccpr_status ccpr_forward(ccpr_solver* s, int nsteps, double* objective_out)
{
    if (!s) return CCPR_EINVAL;
    if (nsteps < 1) return fail(s, CCPR_EINVAL, "nsteps must be >= 1");
    ccpr_status st = check_ready(s, true);
    if (st) return st;
    st = adopt_layout(s, nsteps);
    if (st) return st;
    st = upload_rho(s);
    if (st) return st;
    st = prepare_source(s, nsteps);
    if (st) return st;
    const Layout& L = s->lay;
    const int M = nsteps, K = L.K, S = L.S;
    s->M = M;
    st = zero_state(s, 0);
    if (st) return st;
    st = upload_cold(s, 0);
    if (st) return st;
    HIPCHK(ccpr_launch_fill(wsp<float>(s, L.gap), (long long)s->gncell * 3, 0.f, s->stream));
    if (s->grad_dft) HIPCHK(ccpr_launch_fill(wsp<float>(s, L.T), 12 * std::max(s->nd, 1LL), 0.f, s->stream));
    st = clear_halt(s);
    if (st) return st;
    s->have_forward = s->have_adjoint = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (s->timing) {
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, s->stream));
    }
    s->timed_loop = s->timing;
    {
        WatchScope watch(s);
        for (int n = 0; n < M; ++n) {
            if (saves_checkpoint(L, n)) {
                st = checkpoint(s, n / K - 1, true);
                if (st) return st;
            }
            st = forward_step(s, n, forward_slot(L, n), true, fuse_forward(s, n + 1));
            if (st) return st;
        }
    }
    st = join_lead(s);
    if (st) return st;
    if (s->timing) {
        HIPCHK(hipEventRecord(e1, s->stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        s->stat_ms += ms;
        s->stat_launches += M;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        st = harvest_grid_events(s);
        if (st) return st;
    }
    s->timed_loop = false;
    s->step_count = M;
    s->current_state = 0;
    const int ne = s->gncell * 3;
    const int nend = s->ne < 0 ? M + 1 : s->ne;
    st = launch_objective(s);
    if (st) return st;
    double scal[8];
    HIPCHK(hipMemcpyAsync(scal, wsp<double>(s, L.scal), sizeof scal, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    st = check_results(s, scal);
    if (st) return st;
    s->have_forward = true;
    s->have_adjoint = false;
    s->hist_stale = false;
    ++s->fwd_serial;
    if (objective_out) *objective_out = s->F;
    return CCPR_OK;
}

ccpr_status ccpr_adjoint(ccpr_solver* s)
{
    if (!s) return CCPR_EINVAL;
    if (!s->have_forward) return fail(s, CCPR_ESTATE, "adjoint needs a completed forward run");
    if (s->hist_stale)
        return fail(s, CCPR_ESTATE, "the last adjoint run recomputed segments over the forward history: "
                                    "run ccpr_forward again before another adjoint");
    const Layout& L = s->lay;
    const int M = s->M, K = L.K, S = L.S;
    const long long ndm = std::max(s->nd, 1LL);
    ccpr_status st = zero_state(s, 1);
    if (st) return st;
    st = upload_cold(s, 1);
    if (st) return st;
    HIPCHK(ccpr_launch_fill_d(wsp<double>(s, L.gradacc), std::max(n_rho(s), 1LL), 0.0, s->stream));
    if (s->grad_dft) HIPCHK(ccpr_launch_fill(wsp<float>(s, L.T) + 6 * ndm, 6 * ndm, 0.f, s->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms_total = 0;
    s->timed_loop = s->timing;
    WatchScope watch(s);
    s->have_adjoint = false;
    // recomputed segments write their history over the first resident one's
    s->hist_stale = S > L.R && !s->grad_dft;
    for (int seg = S - 1; seg >= 0; --seg) {
        const int n0 = seg * K, n1 = std::min(M, n0 + K);
        if (seg < S - L.R) {
            // recompute the forward segment from its checkpoint, writing the history
            if (seg == 0) st = zero_state(s, 0);
            else st = checkpoint(s, seg - 1, false);
            if (st) return st;
            for (int n = n0; n < n1; ++n) {
                st = forward_step(s, n, n - n0, false, n + 1 < n1);
                if (st) return st;
            }
            st = join_lead(s);
            if (st) return st;
        }
        const int h0 = n0 - segment_base(L, seg);  // history slot of step n is n - h0
        if (s->timing) {
            HIPCHK(hipEventCreate(&e0));
            HIPCHK(hipEventCreate(&e1));
            HIPCHK(hipEventRecord(e0, s->stream));
        }
        for (int n = n1 - 1; n >= n0; --n) {
            st = adjoint_step(s, n, h0, n > 0);
            if (st) return st;
        }
        st = join_lead(s);
        if (st) return st;
        if (s->timing) {
            HIPCHK(hipEventRecord(e1, s->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            ms_total += ms;
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            st = harvest_grid_events(s);
            if (st) return st;
        }
    }
    s->timed_loop = false;
    if (s->timing) {
        s->stat_ms += ms_total;
        s->stat_launches += M;
    }
    if (s->grad_dft) {
        st = dft_finish(s);
        if (st) return st;
    }
    s->current_state = 1;
    if (s->watch_every > 0) {
        double tripped = 0;
        HIPCHK(hipMemcpyAsync(&tripped, wsp<double>(s, L.scal) + 7, sizeof tripped, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        if (tripped > 0)
            return fail(s, CCPR_EDIVERGED,
                        "the adjoint fields diverged: the watchdog found a gap-box field above %g (or not finite) "
                        "after %d adjoint steps", s->watch_limit, (int)tripped);
    }
    s->have_adjoint = true;
    return CCPR_OK;
}

ccpr_status ccpr_gradient(ccpr_solver* s, double* grad, int mem)
{
    if (!s) return CCPR_EINVAL;
    if (!grad || (mem != CCPR_MEM_HOST && mem != CCPR_MEM_DEVICE)) return fail(s, CCPR_EINVAL, "bad gradient arguments");
    if (!s->have_adjoint) return fail(s, CCPR_ESTATE, "gradient needs a completed adjoint run");
    const double* f = wsp<double>(s, s->lay.scal) + 5;  // gradient scale, on the device
    if (mem == CCPR_MEM_DEVICE) {
        HIPCHK(ccpr_launch_grad_out(grad, wsp<double>(s, s->lay.gradacc), n_rho(s), f, s->stream));
    } else {
        double* stage = wsp<double>(s, s->lay.stage);
        HIPCHK(ccpr_launch_grad_out(stage, wsp<double>(s, s->lay.gradacc), n_rho(s), f, s->stream));
        HIPCHK(hipMemcpyAsync(grad, stage, n_rho(s) * 8, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    return CCPR_OK;
}

ccpr_status ccpr_gap_spectrum(ccpr_solver* s, const double* omega, int nf, double* mean_E2)
{
    if (!s) return CCPR_EINVAL;
    if (!omega || !mean_E2 || nf < 1) return fail(s, CCPR_EINVAL, "bad gap-spectrum arguments");
    if (!s->have_forward) return fail(s, CCPR_ESTATE, "the gap spectrum needs a completed forward run");
    const Layout& L = s->lay;
    const size_t sb = stage_bytes(s);
    if ((size_t)nf * 16 > sb) return fail(s, CCPR_EINVAL, "too many frequencies (at most %zu)", sb / 16);
    for (int f = 0; f < nf; ++f)
        if (!std::isfinite(omega[f])) return fail(s, CCPR_EINVAL, "non-finite frequency");
    ccpr_status st = join_lead(s);
    if (st) return st;
    double* dev = wsp<double>(s, L.stage);
    HIPCHK(hipMemcpyAsync(dev, omega, nf * sizeof(double), hipMemcpyHostToDevice, s->stream));
    // recorded E' = alpha E: the SI transform is dt / alpha times the sum
    HIPCHK(ccpr_launch_gap_spectrum(wsp<float>(s, L.gap), s->M, s->gncell * 3, s->dt, dev, nf, s->dt / s->alpha,
                                    dev + nf, s->stream));
    HIPCHK(hipMemcpyAsync(mean_E2, dev + nf, nf * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return CCPR_OK;
}

// ---- diagnostics (declared in ccprfdtd.h)
ccpr_status ccpr_set_timing(ccpr_solver* s, int enable)
{
    if (!s) return CCPR_EINVAL;
    if (enable < 0) return fail(s, CCPR_EINVAL, "timing period must be >= 0");
    s->timing = enable != 0;
    s->timing_every = enable > 1 ? enable : 1;
    s->pass_no = 0;
    s->stat_ms = 0;
    s->stat_launches = 0;
    s->stat_grid_ms = 0;
    s->stat_grid_launches = 0;
    return CCPR_OK;
}

ccpr_status ccpr_get_timing(const ccpr_solver* s, double* step_ms_total, long long* step_launches)
{
    if (!s || !step_ms_total || !step_launches) return CCPR_EINVAL;
    *step_ms_total = s->stat_ms;
    *step_launches = s->stat_launches;
    return CCPR_OK;
}

ccpr_status ccpr_get_grid_timing(const ccpr_solver* s, double* grid_ms_total, long long* grid_launches)
{
    if (!s || !grid_ms_total || !grid_launches) return CCPR_EINVAL;
    *grid_ms_total = s->stat_grid_ms;
    *grid_launches = s->stat_grid_launches;
    return CCPR_OK;
}

ccpr_status ccpr_get_info(const ccpr_solver* s, int* segments, int* segment_steps, int* tile_planes)
{
    if (!s) return CCPR_EINVAL;
    if (segments) *segments = s->lay.S;
    if (segment_steps) *segment_steps = s->lay.K;
    if (tile_planes) *tile_planes = s->tz;
    return CCPR_OK;
}

ccpr_status ccpr_get_resident_segments(const ccpr_solver* s, int* resident)
{
    if (!s || !resident) return CCPR_EINVAL;
    *resident = s->lay.R;
    return CCPR_OK;
}

ccpr_status ccpr_set_tile_planes(ccpr_solver* s, int planes)
{
    if (!s) return CCPR_EINVAL;
    if (planes < 1 || planes > 4096) return fail(s, CCPR_EINVAL, "tile planes must be in [1,4096]");
    s->tz = planes;
    return CCPR_OK;
}

ccpr_status ccpr_set_watchdog(ccpr_solver* s, int every, double limit)
{
    if (!s) return CCPR_EINVAL;
    if (every < 0 || !(limit > 0) || !std::isfinite(limit) || limit > 3e38)
        return fail(s, CCPR_EINVAL, "watchdog: every must be >= 0 and 0 < limit <= 3e38");
    s->watch_every = every;
    s->watch_limit = limit;
    return CCPR_OK;
}

long long ccpr_forward_serial(const ccpr_solver* s)
{
    if (!s || !s->have_forward || s->hist_stale) return -1;
    return s->fwd_serial;
}

ccpr_status ccpr_set_design_fusion(ccpr_solver* s, int on)
{
    if (!s) return CCPR_EINVAL;
    if (on != 0 && on != 1) return fail(s, CCPR_EINVAL, "design fusion must be 0 or 1");
    s->des_fuse = on != 0;
    return CCPR_OK;
}

ccpr_status ccpr_get_design_fusion(const ccpr_solver* s, int* fused)
{
    if (!s || !fused) return CCPR_EINVAL;
    *fused = s->des_on && s->ntiles_des > 0 ? 1 : 0;
    return CCPR_OK;
}

ccpr_status ccpr_set_tile_rows(ccpr_solver* s, int rows)
{
    if (!s) return CCPR_EINVAL;
    if (rows != 2 && rows != 4) return fail(s, CCPR_EINVAL, "tile rows must be 2 or 4");
    if (rows == 4 && s->nxp > 512) return fail(s, CCPR_ENOTSUP, "4 tile rows need nx <= 512");
    s->rows = rows;
    return CCPR_OK;
}

}  // extern "C"

// ================================================== resumable solve (engine)

ccpr_status ccpr_pipe_begin(ccpr_solver* s, int nsteps)
{
    if (!s) return CCPR_EINVAL;
    if (nsteps < 1) return fail(s, CCPR_EINVAL, "nsteps must be >= 1");
    ccpr_status st = check_ready(s, true);
    if (st) return st;
    if (!s->rho_on_host) return fail(s, CCPR_ENOTSUP, "served solves take host densities");
    st = adopt_layout(s, nsteps);
    if (st) return st;
    st = upload_rho(s);
    if (st) return st;
    st = prepare_source(s, nsteps);
    if (st) return st;
    s->M = nsteps;
    st = zero_state(s, 0);
    if (st) return st;
    st = upload_cold(s, 0);
    if (st) return st;
    st = upload_cold(s, 1);
    if (st) return st;
    HIPCHK(ccpr_launch_fill(wsp<float>(s, s->lay.gap), (long long)s->gncell * 3, 0.f, s->stream));
    if (s->grad_dft)
        HIPCHK(ccpr_launch_fill(wsp<float>(s, s->lay.T), 12 * std::max(s->nd, 1LL), 0.f, s->stream));
    st = clear_halt(s);
    if (st) return st;
    s->have_forward = s->have_adjoint = false;
    s->pipe_phase = 0;
    s->pipe_n = 0;
    return CCPR_OK;
}

int ccpr_pipe_advance(ccpr_solver* s, int max_steps)
{
    const Layout& L = s->lay;
    const int M = s->M, K = L.K, S = L.S;
    int done = 0;
    ccpr_status st = CCPR_OK;
    WatchScope watch(s);
    while (done < max_steps && s->pipe_phase != 3) {
        if (s->pipe_phase == 0) {  // forward step n
            const int n = s->pipe_n;
            if (n == M) {
                s->pipe_phase = 1;
                continue;
            }
            if (saves_checkpoint(L, n)) {
                st = checkpoint(s, n / K - 1, true);
                if (st) return st;
            }
            st = forward_step(s, n, forward_slot(L, n), true, fuse_forward(s, n + 1));
            if (st) return st;
            ++s->pipe_n;
            ++done;
        } else if (s->pipe_phase == 1) {  // objective, adjoint set-up
            st = launch_objective(s);
            if (st) return st;
            st = zero_state(s, 1);
            if (st) return st;
            HIPCHK(ccpr_launch_fill_d(wsp<double>(s, L.gradacc), std::max(n_rho(s), 1LL), 0.0, s->stream));
            if (s->grad_dft) {
                const long long ndm = std::max(s->nd, 1LL);
                HIPCHK(ccpr_launch_fill(wsp<float>(s, L.T) + 6 * ndm, 6 * ndm, 0.f, s->stream));
            }
            s->pipe_phase = 2;
            s->pipe_seg = S - 1;
            s->pipe_sub = 1;  // the last segments' history is already written
            s->pipe_k = 0;
        } else {  // adjoint over segment pipe_seg
            const int seg = s->pipe_seg;
            const int n0 = seg * K, n1 = std::min(M, n0 + K);
            if (s->pipe_sub == 0) {  // recompute the forward segment, writing the history
                if (s->pipe_k == 0) {
                    st = seg == 0 ? zero_state(s, 0) : checkpoint(s, seg - 1, false);
                    if (st) return st;
                }
                const int n = n0 + s->pipe_k;
                st = forward_step(s, n, n - n0, false, n + 1 < n1);
                if (st) return st;
                ++done;
                if (++s->pipe_k == n1 - n0) {
                    s->pipe_sub = 1;
                    s->pipe_k = 0;
                }
            } else {  // adjoint step p pairs with forward step n
                const int n = n1 - 1 - s->pipe_k;
                st = adjoint_step(s, n, n0 - segment_base(L, seg), n > 0);
                if (st) return st;
                ++done;
                if (n == n0) {
                    if (--s->pipe_seg < 0) {
                        if (s->grad_dft) {
                            st = dft_finish(s);
                            if (st) return st;
                        }
                        s->pipe_phase = 3;
                        s->step_count = M;
                        s->current_state = 1;
                    } else {
                        s->pipe_sub = s->pipe_seg >= S - L.R ? 1 : 0;  // resident: no recompute
                        s->pipe_k = 0;
                    }
                } else {
                    ++s->pipe_k;
                }
            }
        }
    }
    st = join_lead(s);
    if (st) return st;
    return done;
}

ccpr_status ccpr_pipe_results(ccpr_solver* s, double* scal_host, double* grad_host)
{
    const Layout& L = s->lay;
    double* stage = wsp<double>(s, L.stage);
    HIPCHK(ccpr_launch_grad_out(stage, wsp<double>(s, L.gradacc), n_rho(s), wsp<double>(s, L.scal) + 5, s->stream));
    HIPCHK(hipMemcpyAsync(grad_host, stage, n_rho(s) * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(scal_host, wsp<double>(s, L.scal), 8 * sizeof(double), hipMemcpyDeviceToHost,
                          s->stream));
    return CCPR_OK;
}

ccpr_status ccpr_pipe_check(ccpr_solver* s, const double* scal_host, double* F)
{
    ccpr_status st = check_results(s, scal_host);
    if (st) return st;
    s->have_forward = s->have_adjoint = true;
    s->hist_stale = s->lay.S > s->lay.R && !s->grad_dft;
    ++s->fwd_serial;
    if (F) *F = s->F;
    return CCPR_OK;
}

long long ccpr_pipe_design_voxels(const ccpr_solver* s) { return s->has_design ? n_rho(s) : 0; }

static_assert(CCPR_PIPE_BATCH_MAX == CCPR_BATCH_MAX, "batch sizes of the engine and the kernels differ");

int ccpr_pipe_batch_class(const ccpr_solver* s)
{
    // batched launches cover one density per voxel, the time-exact gradient,
    // 2 rows per thread and x layers that fit the fused post kernel's blocks
    if (s->edge || s->grad_dft || s->rows != 2 || 2 * s->g.npml > 256) return -1;
    return s->nxp;
}

ccpr_status ccpr_pipe_set_batched(ccpr_solver* s, int on)
{
    {
        ccpr_status j = join_lead(s);
        if (j) return j;
    }
    if (on && ccpr_pipe_batch_class(s) < 0) return fail(s, CCPR_ENOTSUP, "this solve cannot be batched");
    s->batched = on != 0;
    s->rec_pending = false;
    return CCPR_OK;
}

ccpr_status ccpr_pipe_flush(ccpr_solver* const* ss, int k, void* stream)
{
    BatchStep st[CCPR_BATCH_MAX];
    ccpr_solver* who[CCPR_BATCH_MAX];
    int m = 0;
    for (int q = 0; q < k; ++q) {
        ccpr_solver* s = ss[q];
        if (!s->rec_pending) continue;
        if (m == CCPR_BATCH_MAX || (m > 0 && s->rec.a.nxp != st[0].a.nxp)) return CCPR_EINVAL;
        st[m] = s->rec;
        who[m++] = s;
    }
    if (m == 0) return CCPR_OK;
    const int e = ccpr_launch_batch(st, m, stream);
    ccpr_status res = e == 0 ? CCPR_OK : CCPR_EDEVICE;
    for (int q = 0; q < m; ++q) {
        ccpr_solver* s = who[q];
        s->rec_pending = false;
        if (e != 0) {
            fail(s, CCPR_EDEVICE, "batched step launch: %s", hipGetErrorString((hipError_t)e));
            continue;
        }
        if (s->rec_watch) {
            const int w = ccpr_launch_watch(s->rec.a, s->glo, s->gdim, (float)s->watch_limit, s->rec.a.n,
                                            wsp<unsigned>(s, s->lay.halt), wsp<double>(s, s->lay.scal), stream);
            if (w != 0) res = fail(s, CCPR_EDEVICE, "watchdog launch: %s", hipGetErrorString((hipError_t)w));
        }
    }
    return res;
}

ccpr_status ccpr_pipe_set_stream2(ccpr_solver* s, void* stream2)
{
    {
        ccpr_status j = join_lead(s);
        if (j) return j;
    }
    if (s->stream2 && s->own_stream2) {
        HIPCHK(hipStreamSynchronize(s->stream2));
        HIPCHK(hipStreamDestroy(s->stream2));
    }
    s->stream2 = (hipStream_t)stream2;
    s->own_stream2 = false;
    return CCPR_OK;
}

void ccpr_pipe_unbind(ccpr_solver* s)
{
    s->ws = nullptr;
    s->ws_bytes = 0;
    s->stream = nullptr;
    if (!s->own_stream2) s->stream2 = nullptr;  // the engine's stream goes back to its pool
    s->have_forward = s->have_adjoint = false;
    s->rho_uploaded = false;
    s->lead2 = false;  // (the engine unbinds after the solve's work completed)
    s->post_armed = false;
    s->pre_done[0] = s->pre_done[1] = false;
    s->batched = false;
    s->rec_pending = false;
    std::memset(s->fixed_key, 0xff, sizeof s->fixed_key);
}
