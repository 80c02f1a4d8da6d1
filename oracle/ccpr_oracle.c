/*
 * ccpr_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see the
 * header).  Every routine follows the paper's equations as directly as it can,
 * loop by loop, with no blocking, fusion or reordering: one pass updates H,
 * one pass updates E, exactly as the leapfrog is written.
 *
 * Citations refer to the paper "Free-form inverse design of arbitrary
 * dispersive materials in nanophotonics" (main text and its supplement).
 *
 * Discretisation of the CCPR auxiliary differential equation.  The paper
 * delegates it to its material reference; this oracle uses the reading that
 * keeps the scheme second order and unconditionally stable for passive poles:
 *   - Ampere's law (supplement Eq. Maxwells2 a) is taken at t=(n+1/2)dt with
 *     the trapezoid rule on sigma*E and on the pole-pair currents;
 *   - each pole-pair current J_p = dQ_p/dt obeys dJ_p/dt = a_p J_p + eps0 c_p
 *     dE/dt (time derivative of Eq. Maxwells2 b), discretised by the bilinear
 *     (trapezoid) rule:
 *         J_p^{n+1} = k_p J_p^n + beta_p (E^{n+1} - E^n),
 *         k_p = (1 + a_p dt/2)/(1 - a_p dt/2), beta_p = eps0 c_p/(1 - a_p dt/2);
 *   - the pair's real current 2 Re{dQ/dt} averaged over the step is
 *     Re{J^{n+1} + J^n}.
 * The single-edge impulse response of this update reproduces the CCPR
 * permittivity exactly at the bilinear-warped frequency (2/dt) tan(w dt/2);
 * tests pin that.
 */
#include "ccpr_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EPS0 8.8541878128e-12
#define MU0 1.25663706212e-6
#define C0 299792458.0

typedef double complex cplx;

typedef struct {
    double eps_inf, sigma;
    int np;
    cplx a[OR_MAX_PAIRS], c[OR_MAX_PAIRS];
} or_mat;

/* Per-edge update coefficients at a given density (Eqs. eps_mixed,
 * sigma_mixed, Poles_mixed). */
typedef struct {
    double A, B;             /* E^{n+1} = (B E^n + curl - src - sum)/A          */
    double deps, dsig;       /* d eps_inf/d rho, d sigma/d rho                  */
    int np;                  /* pole pairs over both materials                  */
    double kap[2 * OR_MAX_PAIRS];  /* kappa^(i)(rho) of each pair              */
    double dkap[2 * OR_MAX_PAIRS]; /* d kappa^(i)/d rho = -1 or +1             */
    cplx k[2 * OR_MAX_PAIRS], beta[2 * OR_MAX_PAIRS];
} edge_coef;

struct or_sim {
    int n[3];
    double dx, S, dt;
    int npml;
    double pml_m, pml_kmax, pml_amax, pml_sscale;
    double *bE[3], *aE[3], *kE[3]; /* CPML at integer positions per axis      */
    double *bH[3], *aH[3], *kH[3]; /* CPML at half-integer positions per axis */
    double* F[6];                  /* Ex Ey Ez Hx Hy Hz                        */
    double* psiE[3][3];            /* [component][derivative axis]             */
    double* psiH[3][3];
    or_mat mat[2][3];
    /* design: one density per design edge (Sec. "FDTD implementation and
     * design export").  The edges of component c form the box
     * [dlo, dlo + edim[c]); edge e of c is eoff[c] + its index in that box
     * (x fastest).  A per-voxel design gives each component the voxel box
     * and copies the voxel's density to its three edges; a per-edge design
     * of N cells gives component c the extents N_l + 1 - delta(c,l). */
    int dlo[3], ddim[3], nd;     /* cell box; nd = its cell count          */
    int per_edge;
    int edim[3][3];
    size_t eoff[4];              /* eoff[3]: number of design edges        */
    double gamma;
    double* rho;                 /* [eoff[3]]                              */
    cplx* J;                     /* [eoff[3]][2*OR_MAX_PAIRS]              */
    /* dipole */
    int dip_on, dip_cell[3], dip_axis, dip_nw;
    double* dip_wave;
    /* plane wave */
    int pw_on, pw_d, pw_sgn, pw_p, pw_t, pw_lo[3], pw_hi[3], pw_nw, pw_L, pw_ref2;
    double pw_levi;
    double *pw_wave, *pw_E, *pw_H;
    /* box source */
    int bs_on, bs_lo[3], bs_dim[3], bs_ncell, bs_nsteps;
    double* bs_table;
    int step;
    /* copy of the six fields at the end of the last forward run of
     * or_gradient / or_gradient_dft / or_objective (NULL until kept) */
    double* fwd_end[6];
    /* diagnostic (or_set_fp32_storage): round the stored state to FP32 */
    int fp32_store;
};

static size_t idx3(const or_sim* s, int i, int j, int k)
{
    return ((size_t)k * s->n[1] + j) * s->n[0] + i;
}

static size_t ncells(const or_sim* s) { return (size_t)s->n[0] * s->n[1] * s->n[2]; }

/* Field value with the implicit zero planes beyond the grid (PEC walls). */
static double fget(const or_sim* s, const double* a, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= s->n[0] || j >= s->n[1] || k >= s->n[2]) return 0.0;
    return a[idx3(s, i, j, k)];
}

/* ---------------------------------------------------------------- CPML --- */
/* Convolutional PML (Methods "Technical details": CPML layers surround the
 * domain).  Grading parameters are not given in the paper; this follows the
 * standard CFS-CPML recursive convolution with polynomial grading. */
static void pml_point(const or_sim* s, int N, double pos, double* b, double* a, double* kap)
{
    double xi = 0.0;
    if (s->npml > 0) {
        double dl = (double)s->npml - pos, dh = pos - (double)(N - s->npml);
        double d = dl > dh ? dl : dh;
        if (d < 0.0) d = 0.0;
        if (d > s->npml) d = s->npml;
        xi = d / s->npml;
    }
    double eta0 = sqrt(MU0 / EPS0);
    double smax = s->pml_sscale * 0.8 * (s->pml_m + 1.0) / (eta0 * s->dx);
    double sig = smax * pow(xi, s->pml_m);
    double k = 1.0 + (s->pml_kmax - 1.0) * pow(xi, s->pml_m);
    double al = s->pml_amax * (1.0 - xi);
    *b = exp(-(sig / k + al) * s->dt / EPS0);
    *a = sig > 0.0 ? sig * (*b - 1.0) / (sig * k + k * k * al) : 0.0;
    *kap = k;
}

or_sim* or_create(int nx, int ny, int nz, double dx, double courant, int npml,
                  double pml_m, double pml_kappa_max, double pml_alpha_max,
                  double pml_sigma_scale)
{
    if (nx < 1 || ny < 1 || nz < 1 || !(dx > 0) || !(courant > 0) || npml < 0) return NULL;
    if (2 * npml > nx || 2 * npml > ny || 2 * npml > nz) return NULL;
    or_sim* s = (or_sim*)calloc(1, sizeof(or_sim));
    s->n[0] = nx; s->n[1] = ny; s->n[2] = nz;
    s->dx = dx; s->S = courant; s->dt = courant * dx / C0;
    s->npml = npml; s->pml_m = pml_m; s->pml_kmax = pml_kappa_max;
    s->pml_amax = pml_alpha_max; s->pml_sscale = pml_sigma_scale;
    for (int a = 0; a < 3; ++a) {
        int N = s->n[a];
        s->bE[a] = malloc(N * sizeof(double)); s->aE[a] = malloc(N * sizeof(double));
        s->kE[a] = malloc(N * sizeof(double)); s->bH[a] = malloc(N * sizeof(double));
        s->aH[a] = malloc(N * sizeof(double)); s->kH[a] = malloc(N * sizeof(double));
        for (int q = 0; q < N; ++q) {
            pml_point(s, N, (double)q, &s->bE[a][q], &s->aE[a][q], &s->kE[a][q]);
            pml_point(s, N, q + 0.5, &s->bH[a][q], &s->aH[a][q], &s->kH[a][q]);
        }
    }
    size_t nc = ncells(s);
    for (int c = 0; c < 6; ++c) s->F[c] = calloc(nc, sizeof(double));
    if (npml > 0)
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d)
                if (c != d) {
                    s->psiE[c][d] = calloc(nc, sizeof(double));
                    s->psiH[c][d] = calloc(nc, sizeof(double));
                }
    for (int sl = 0; sl < 2; ++sl)
        for (int a = 0; a < 3; ++a) s->mat[sl][a].eps_inf = 1.0; /* vacuum */
    return s;
}

void or_destroy(or_sim* s)
{
    if (!s) return;
    for (int a = 0; a < 3; ++a) {
        free(s->bE[a]); free(s->aE[a]); free(s->kE[a]);
        free(s->bH[a]); free(s->aH[a]); free(s->kH[a]);
    }
    for (int c = 0; c < 6; ++c) free(s->F[c]);
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) { free(s->psiE[c][d]); free(s->psiH[c][d]); }
    free(s->rho); free(s->J); free(s->dip_wave);
    free(s->pw_wave); free(s->pw_E); free(s->pw_H); free(s->bs_table);
    for (int c = 0; c < 6; ++c) free(s->fwd_end[c]);
    free(s);
}

double or_dt(const or_sim* s) { return s->dt; }

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int or_set_material(or_sim* s, int slot, int axis, double eps_inf, double sigma,
                    int np, const double* a, const double* c)
{
    if (slot < 1 || slot > 2 || axis < 0 || axis > 2 || np < 0 || np > OR_MAX_PAIRS) return -1;
    or_mat* m = &s->mat[slot - 1][axis];
    m->eps_inf = eps_inf; m->sigma = sigma; m->np = np;
    for (int p = 0; p < np; ++p) {
        m->a[p] = a[2 * p] + I * a[2 * p + 1];
        m->c[p] = c[2 * p] + I * c[2 * p + 1];
    }
    return 0;
}

static int set_design_boxes(or_sim* s, const int* lo, const int* dims, int per_edge, double gamma)
{
    for (int a = 0; a < 3; ++a) {
        if (lo[a] < 0 || dims[a] < 1) return -1;
        if (lo[a] + dims[a] + (per_edge ? 1 : 0) > s->n[a]) return -1;
    }
    memcpy(s->dlo, lo, sizeof(s->dlo));
    memcpy(s->ddim, dims, sizeof(s->ddim));
    s->nd = dims[0] * dims[1] * dims[2];
    s->per_edge = per_edge;
    s->gamma = gamma;
    s->eoff[0] = 0;
    for (int c = 0; c < 3; ++c) {
        size_t n = 1;
        for (int l = 0; l < 3; ++l) {
            s->edim[c][l] = dims[l] + ((per_edge && l != c) ? 1 : 0);
            n *= (size_t)s->edim[c][l];
        }
        s->eoff[c + 1] = s->eoff[c] + n;
    }
    free(s->rho); free(s->J);
    s->rho = malloc(s->eoff[3] * sizeof(double));
    s->J = calloc(s->eoff[3] * 2 * OR_MAX_PAIRS, sizeof(cplx));
    return (s->rho && s->J) ? 0 : -1;
}

int or_set_design(or_sim* s, const int* lo, const int* dims, double gamma, const double* rho)
{
    if (set_design_boxes(s, lo, dims, 0, gamma)) return -1;
    for (int c = 0; c < 3; ++c) memcpy(s->rho + s->eoff[c], rho, (size_t)s->nd * sizeof(double));
    return 0;
}

int or_set_design_edges(or_sim* s, const int* lo, const int* dims, double gamma, const double* rho)
{
    if (set_design_boxes(s, lo, dims, 1, gamma)) return -1;
    memcpy(s->rho, rho, s->eoff[3] * sizeof(double));
    return 0;
}

long long or_design_outputs(const or_sim* s) { return s->per_edge ? (long long)s->eoff[3] : (long long)s->nd; }

int or_set_dipole(or_sim* s, const int* cell, int axis, const double* wave, int nw)
{
    if (axis < 0 || axis > 2 || nw < 0) return -1;
    for (int a = 0; a < 3; ++a) if (cell[a] < 0 || cell[a] >= s->n[a]) return -1;
    memcpy(s->dip_cell, cell, sizeof(s->dip_cell));
    s->dip_axis = axis; s->dip_nw = nw;
    free(s->dip_wave);
    s->dip_wave = malloc((nw > 0 ? nw : 1) * sizeof(double));
    memcpy(s->dip_wave, wave, nw * sizeof(double));
    s->dip_on = 1;
    return 0;
}

/* Levi-Civita symbol for a permutation of (0,1,2). */
static int levi(int a, int b, int c)
{
    if (a == b || b == c || a == c) return 0;
    return ((a == 0 && b == 1) || (a == 1 && b == 2) || (a == 2 && b == 0)) ? 1 : -1;
}

int or_set_planewave(or_sim* s, int prop_axis, int sign, int pol_axis,
                     const int* lo, const int* hi, const double* wave, int nw)
{
    if (prop_axis < 0 || prop_axis > 2 || pol_axis < 0 || pol_axis > 2 ||
        prop_axis == pol_axis || (sign != 1 && sign != -1) || nw < 1) return -1;
    for (int a = 0; a < 3; ++a)
        if (lo[a] < 1 || hi[a] <= lo[a] || hi[a] >= s->n[a] - 1) return -1;
    s->pw_d = prop_axis; s->pw_sgn = sign; s->pw_p = pol_axis;
    s->pw_t = 3 - prop_axis - pol_axis;
    s->pw_levi = levi(s->pw_p, s->pw_d, s->pw_t);
    memcpy(s->pw_lo, lo, sizeof(s->pw_lo));
    memcpy(s->pw_hi, hi, sizeof(s->pw_hi));
    s->pw_nw = nw;
    free(s->pw_wave);
    s->pw_wave = malloc(nw * sizeof(double));
    memcpy(s->pw_wave, wave, nw * sizeof(double));
    /* 1-D auxiliary line: u = 0 two cells before the box along the direction
     * of travel; long enough that the far-end reflection cannot come back
     * within nw steps (information moves at most one cell per step). */
    int d = prop_axis;
    s->pw_ref2 = sign > 0 ? 2 * (lo[d] - 2) : 2 * (hi[d] + 2);
    s->pw_L = (hi[d] - lo[d]) + 8 + nw / 2 + 8;
    free(s->pw_E); free(s->pw_H);
    s->pw_E = calloc(s->pw_L + 1, sizeof(double));
    s->pw_H = calloc(s->pw_L + 1, sizeof(double));
    s->pw_on = 1;
    s->pw_E[0] = wave[0];
    return 0;
}

int or_set_box_source(or_sim* s, const int* lo, const int* dims, const double* table, int nsteps)
{
    for (int a = 0; a < 3; ++a)
        if (lo[a] < 0 || dims[a] < 1 || lo[a] + dims[a] > s->n[a]) return -1;
    memcpy(s->bs_lo, lo, sizeof(s->bs_lo));
    memcpy(s->bs_dim, dims, sizeof(s->bs_dim));
    s->bs_ncell = dims[0] * dims[1] * dims[2];
    s->bs_nsteps = nsteps;
    free(s->bs_table);
    size_t n = (size_t)nsteps * s->bs_ncell * 3;
    s->bs_table = malloc((n > 0 ? n : 1) * sizeof(double));
    memcpy(s->bs_table, table, n * sizeof(double));
    s->bs_on = 1;
    return 0;
}

void or_clear_sources(or_sim* s) { s->dip_on = 0; s->pw_on = 0; s->bs_on = 0; }

void or_reset(or_sim* s)
{
    size_t nc = ncells(s);
    for (int c = 0; c < 6; ++c) memset(s->F[c], 0, nc * sizeof(double));
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
            if (s->psiE[c][d]) memset(s->psiE[c][d], 0, nc * sizeof(double));
            if (s->psiH[c][d]) memset(s->psiH[c][d], 0, nc * sizeof(double));
        }
    if (s->J) memset(s->J, 0, s->eoff[3] * 2 * OR_MAX_PAIRS * sizeof(cplx));
    if (s->pw_E) {
        memset(s->pw_E, 0, (s->pw_L + 1) * sizeof(double));
        memset(s->pw_H, 0, (s->pw_L + 1) * sizeof(double));
        s->pw_E[0] = s->pw_wave[0];
    }
    s->step = 0;
}

int or_step_count(const or_sim* s) { return s->step; }

int or_get_forward_end_field(const or_sim* s, int comp, double* out)
{
    if (comp < 0 || comp > 5 || !s->fwd_end[comp]) return -1;
    memcpy(out, s->fwd_end[comp], ncells(s) * sizeof(double));
    return 0;
}

void or_get_field(const or_sim* s, int comp, double* out)
{
    memcpy(out, s->F[comp], ncells(s) * sizeof(double));
}

void or_set_field(or_sim* s, int comp, const double* in)
{
    memcpy(s->F[comp], in, ncells(s) * sizeof(double));
}

/* ------------------------------------------------------ material model --- */
/* Interpolated CCPR coefficients of one edge (Eqs. eps_mixed, sigma_mixed,
 * Poles_mixed) and the trapezoid / bilinear update constants. */
static void edge_coef_at(const or_sim* s, int axis, double rho, double gamma, edge_coef* ec)
{
    const or_mat* m1 = &s->mat[0][axis];
    const or_mat* m2 = &s->mat[1][axis];
    double eps = (1.0 - rho) * m1->eps_inf + rho * m2->eps_inf;
    double sig = (1.0 - rho) * m1->sigma + rho * m2->sigma + rho * (1.0 - rho) * gamma;
    double dt = s->dt;
    ec->deps = m2->eps_inf - m1->eps_inf;
    ec->dsig = m2->sigma - m1->sigma + (1.0 - 2.0 * rho) * gamma;
    ec->np = 0;
    double sumb = 0.0;
    for (int i = 0; i < 2; ++i) {
        const or_mat* m = i == 0 ? m1 : m2;
        double kap = i == 0 ? 1.0 - rho : rho;
        for (int p = 0; p < m->np; ++p) {
            int q = ec->np++;
            ec->kap[q] = kap;
            ec->dkap[q] = i == 0 ? -1.0 : 1.0;
            ec->k[q] = (1.0 + m->a[p] * dt / 2.0) / (1.0 - m->a[p] * dt / 2.0);
            ec->beta[q] = EPS0 * m->c[p] / (1.0 - m->a[p] * dt / 2.0);
            sumb += kap * creal(ec->beta[q]);
        }
    }
    ec->A = EPS0 * eps / dt + sig / 2.0 + sumb;
    ec->B = EPS0 * eps / dt - sig / 2.0 + sumb;
}

static void vacuum_coef(const or_sim* s, edge_coef* ec)
{
    ec->A = ec->B = EPS0 / s->dt;
    ec->deps = ec->dsig = 0.0;
    ec->np = 0;
}

/* One edge: E^n -> E^{n+1} and J_p^n -> J_p^{n+1}.  curl = (curl H)_k at
 * (n+1/2)dt [A/m^2], src = J_src at (n+1/2)dt.  If T is not NULL it receives
 * dt * d/drho of Ampere's residual at fixed fields (the forward factor of the
 * gradient): eps0 deps (E^{n+1}-E^n) + dsig dt (E^{n+1}+E^n)/2
 *          + dt sum_p dkap_p Re{J_p^{n+1} + J_p^n}. */
static double edge_update(const edge_coef* ec, double dt, double E, double curl, double src,
                          cplx* J, double* T)
{
    double acc = 0.0;
    for (int p = 0; p < ec->np; ++p) acc += ec->kap[p] * creal((1.0 + ec->k[p]) * J[p]);
    double En = (ec->B * E + curl - src - acc) / ec->A;
    double R = 0.0;
    for (int p = 0; p < ec->np; ++p) {
        cplx Jn = ec->k[p] * J[p] + ec->beta[p] * (En - E);
        R += ec->dkap[p] * creal(Jn + J[p]);
        J[p] = Jn;
    }
    if (T) *T = EPS0 * ec->deps * (En - E) + ec->dsig * dt * (En + E) / 2.0 + dt * R;
    return En;
}

/* ------------------------------------------------- TF/SF plane wave ------ */
/* Doubled coordinates: E_c at (2i,2j,2k)+e_c, H_c at (2i+1,2j+1,2k+1)-e_c. */
static int in_tf(const or_sim* s, const int* P)
{
    for (int a = 0; a < 3; ++a)
        if (P[a] < 2 * s->pw_lo[a] || P[a] > 2 * s->pw_hi[a]) return 0;
    return 1;
}

/* Incident value at doubled coordinate P2 along the propagation axis: E on
 * even u2, H on odd u2 of the 1-D line. */
static double inc_at(const or_sim* s, int P2)
{
    int u2 = s->pw_sgn * (P2 - s->pw_ref2);
    if (u2 < 0) return 0.0;
    double v;
    if ((u2 & 1) == 0) v = u2 / 2 <= s->pw_L ? s->pw_E[u2 / 2] : 0.0;
    else v = (u2 - 1) / 2 <= s->pw_L ? s->pw_H[(u2 - 1) / 2] : 0.0;
    return s->fp32_store ? (double)(float)v : v;
}

/* E_e at cell (i,j,k) as seen by an H point whose TF status is tfH. */
static double e_seen(const or_sim* s, int e, int i, int j, int k, int tfH)
{
    double v = fget(s, s->F[e], i, j, k);
    if (s->pw_on && e == s->pw_p) {
        int P[3] = {2 * i, 2 * j, 2 * k};
        P[e] += 1;
        int tf = in_tf(s, P);
        if (tfH && !tf) v += inc_at(s, P[s->pw_d]);
        if (!tfH && tf) v -= inc_at(s, P[s->pw_d]);
    }
    return v;
}

static double h_seen(const or_sim* s, int h, int i, int j, int k, int tfE)
{
    double v = fget(s, s->F[3 + h], i, j, k);
    if (s->pw_on && h == s->pw_t) {
        int P[3] = {2 * i + 1, 2 * j + 1, 2 * k + 1};
        P[h] -= 1;
        int tf = in_tf(s, P);
        if (tfE && !tf) v += inc_at(s, P[s->pw_d]);
        if (!tfE && tf) v -= inc_at(s, P[s->pw_d]);
    }
    return v;
}

/* 1-D line, same dx and dt as the 3-D grid, so an axis-aligned plane wave is
 * reproduced exactly.  dE_p/dt = (levi/eps0) dH_t/dx_d,
 * dH_t/dt = (levi/mu0) dE_p/dx_d, with dx_d = sgn du. */
static void line_update_H(or_sim* s)
{
    double c = s->pw_levi * s->pw_sgn * s->dt / (MU0 * s->dx);
    for (int u = 0; u < s->pw_L; ++u) s->pw_H[u] += c * (s->pw_E[u + 1] - s->pw_E[u]);
}

static void line_update_E(or_sim* s, int n_next)
{
    double c = s->pw_levi * s->pw_sgn * s->dt / (EPS0 * s->dx);
    for (int u = 1; u < s->pw_L; ++u) s->pw_E[u] += c * (s->pw_H[u] - s->pw_H[u - 1]);
    s->pw_E[0] = n_next < s->pw_nw ? s->pw_wave[n_next] : 0.0;
}

/* --------------------------------------------------------- leapfrog ------ */
static int in_box(const int* lo, const int* dim, int i, int j, int k)
{
    return i >= lo[0] && i < lo[0] + dim[0] && j >= lo[1] && j < lo[1] + dim[1] &&
           k >= lo[2] && k < lo[2] + dim[2];
}

/* Design edge of component c at cell (i,j,k), or -1. */
static long long design_edge(const or_sim* s, int c, int i, int j, int k)
{
    if (s->eoff[3] == 0 || !in_box(s->dlo, s->edim[c], i, j, k)) return -1;
    const int* d = s->edim[c];
    return (long long)s->eoff[c] +
           ((long long)(k - s->dlo[2]) * d[1] + (j - s->dlo[1])) * d[0] + (i - s->dlo[0]);
}

/* H^{n+1/2} = H^{n-1/2} - (dt/mu0) curl E^n (supplement Eq. Maxwells2 c). */
static void update_H(or_sim* s)
{
    const double dx = s->dx, ch = s->dt / MU0;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < s->n[2]; ++k)
        for (int j = 0; j < s->n[1]; ++j)
            for (int i = 0; i < s->n[0]; ++i)
                for (int c = 0; c < 3; ++c) {
                    int d1 = (c + 1) % 3, d2 = (c + 2) % 3;
                    int cell[3] = {i, j, k};
                    int P[3] = {2 * i + 1, 2 * j + 1, 2 * k + 1};
                    P[c] -= 1;
                    int tf = s->pw_on ? in_tf(s, P) : 0;
                    int n1[3] = {i, j, k}, n2[3] = {i, j, k};
                    n1[d1] += 1;
                    n2[d2] += 1;
                    /* (curl E)_c = dE_d2/dx_d1 - dE_d1/dx_d2 (forward differences) */
                    double dA = (e_seen(s, d2, n1[0], n1[1], n1[2], tf) -
                                 e_seen(s, d2, i, j, k, tf)) / dx;
                    double dB = (e_seen(s, d1, n2[0], n2[1], n2[2], tf) -
                                 e_seen(s, d1, i, j, k, tf)) / dx;
                    double curl;
                    if (s->npml > 0) {
                        size_t id = idx3(s, i, j, k);
                        int q1 = cell[d1], q2 = cell[d2];
                        double* p1 = &s->psiH[c][d1][id];
                        double* p2 = &s->psiH[c][d2][id];
                        *p1 = s->bH[d1][q1] * *p1 + s->aH[d1][q1] * dA;
                        *p2 = s->bH[d2][q2] * *p2 + s->aH[d2][q2] * dB;
                        curl = dA / s->kH[d1][q1] + *p1 - dB / s->kH[d2][q2] - *p2;
                    } else {
                        curl = dA - dB;
                    }
                    s->F[3 + c][idx3(s, i, j, k)] -= ch * curl;
                }
}

/* E^{n+1} from Ampere's law with the CCPR currents (supplement Eq. Maxwells2
 * a, b).  If T is not NULL, T[e] receives the gradient factor of design
 * edge e. */
static void update_E(or_sim* s, double* T)
{
    const double dx = s->dx;
    const int n = s->step;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < s->n[2]; ++k)
        for (int j = 0; j < s->n[1]; ++j)
            for (int i = 0; i < s->n[0]; ++i)
                for (int c = 0; c < 3; ++c) {
                    int d1 = (c + 1) % 3, d2 = (c + 2) % 3;
                    int cell[3] = {i, j, k};
                    size_t id = idx3(s, i, j, k);
                    if (cell[d1] == 0 || cell[d2] == 0) { /* tangential on a wall */
                        s->F[c][id] = 0.0;
                        continue;
                    }
                    int P[3] = {2 * i, 2 * j, 2 * k};
                    P[c] += 1;
                    int tf = s->pw_on ? in_tf(s, P) : 0;
                    int m1[3] = {i, j, k}, m2[3] = {i, j, k};
                    m1[d1] -= 1;
                    m2[d2] -= 1;
                    /* (curl H)_c = dH_d2/dx_d1 - dH_d1/dx_d2 (backward differences) */
                    double dA = (h_seen(s, d2, i, j, k, tf) -
                                 h_seen(s, d2, m1[0], m1[1], m1[2], tf)) / dx;
                    double dB = (h_seen(s, d1, i, j, k, tf) -
                                 h_seen(s, d1, m2[0], m2[1], m2[2], tf)) / dx;
                    double curl;
                    if (s->npml > 0) {
                        int q1 = cell[d1], q2 = cell[d2];
                        double* p1 = &s->psiE[c][d1][id];
                        double* p2 = &s->psiE[c][d2][id];
                        *p1 = s->bE[d1][q1] * *p1 + s->aE[d1][q1] * dA;
                        *p2 = s->bE[d2][q2] * *p2 + s->aE[d2][q2] * dB;
                        curl = dA / s->kE[d1][q1] + *p1 - dB / s->kE[d2][q2] - *p2;
                    } else {
                        curl = dA - dB;
                    }
                    double src = 0.0;
                    if (s->dip_on && c == s->dip_axis && i == s->dip_cell[0] &&
                        j == s->dip_cell[1] && k == s->dip_cell[2] && n < s->dip_nw)
                        src += s->dip_wave[n];
                    if (s->bs_on && n < s->bs_nsteps && in_box(s->bs_lo, s->bs_dim, i, j, k)) {
                        int ci = ((k - s->bs_lo[2]) * s->bs_dim[1] + (j - s->bs_lo[1])) * s->bs_dim[0] +
                                 (i - s->bs_lo[0]);
                        src += s->bs_table[((size_t)n * s->bs_ncell + ci) * 3 + c];
                    }
                    edge_coef ec;
                    cplx* J = NULL;
                    double* Tp = NULL;
                    const long long e = design_edge(s, c, i, j, k);
                    if (e >= 0) {
                        edge_coef_at(s, c, s->rho[e], s->gamma, &ec);
                        J = &s->J[(size_t)e * 2 * OR_MAX_PAIRS];
                        if (T) Tp = &T[e];
                    } else {
                        vacuum_coef(s, &ec);
                    }
                    s->F[c][id] = edge_update(&ec, s->dt, s->F[c][id], curl, src, J, Tp);
                }
}

/* Diagnostic FP32 storage: every stored state word rounded to FP32. */
static void round_fp32(double* a, size_t n)
{
    if (!a) return;
    for (size_t q = 0; q < n; ++q) a[q] = (double)(float)a[q];
}

static void store_fp32(or_sim* s, int h)
{
    const size_t nc = ncells(s);
    for (int c = 0; c < 3; ++c) {
        round_fp32(s->F[h ? 3 + c : c], nc);
        for (int d = 0; d < 3; ++d) round_fp32(h ? s->psiH[c][d] : s->psiE[c][d], nc);
    }
    if (!h && s->J) round_fp32((double*)s->J, s->eoff[3] * 2 * OR_MAX_PAIRS * 2);
}

static void step_once(or_sim* s, double* T)
{
    update_H(s);
    if (s->pw_on) line_update_H(s);
    if (s->fp32_store) store_fp32(s, 1);
    update_E(s, T);
    if (s->pw_on) line_update_E(s, s->step + 1);
    if (s->fp32_store) store_fp32(s, 0);
    s->step += 1;
}

void or_set_fp32_storage(or_sim* s, int on) { s->fp32_store = on != 0; }

int or_get_pml_coef(const or_sim* s, int axis, int half, int q, double* b, double* a, double* kappa)
{
    if (!s || axis < 0 || axis > 2 || q < 0 || q >= s->n[axis] || !b || !a || !kappa) return -1;
    *b = half ? s->bH[axis][q] : s->bE[axis][q];
    *a = half ? s->aH[axis][q] : s->aE[axis][q];
    *kappa = half ? s->kH[axis][q] : s->kE[axis][q];
    return 0;
}

void or_run(or_sim* s, int nsteps)
{
    for (int n = 0; n < nsteps; ++n) step_once(s, NULL);
}

/* ------------------------------------------- objective and gradient ----- */
static int gap_ok(const or_sim* s, const int* lo, const int* dims)
{
    for (int a = 0; a < 3; ++a)
        if (lo[a] < 0 || dims[a] < 1 || lo[a] + dims[a] > s->n[a]) return 0;
    return 1;
}

static void record_gap(const or_sim* s, const int* lo, const int* dims, double* out)
{
    int c = 0;
    for (int k = lo[2]; k < lo[2] + dims[2]; ++k)
        for (int j = lo[1]; j < lo[1] + dims[1]; ++j)
            for (int i = lo[0]; i < lo[0] + dims[0]; ++i, ++c)
                for (int a = 0; a < 3; ++a) out[c * 3 + a] = s->F[a][idx3(s, i, j, k)];
}

/* Forward run with gap recording, then the objective and its derivative
 * dF/dE^n at every gap edge.  Gradient factors (one per design edge e): with
 * T_hist the whole history T^{n+1/2} is kept; with T_hat (and T_hist NULL)
 * only its transform at omega, T_hat[e] = sum_{n=0}^{M-1} T_e^{n+1/2}
 * exp(-j omega n dt). */
static int forward_and_objective(or_sim* s, int M, int kind, const int* glo, const int* gdim,
                                 double omega, int nb, int ne, double* T_hist, cplx* T_hat,
                                 double* F_out, double* hist, double* dFdE)
{
    int ncell = gdim[0] * gdim[1] * gdim[2];
    const size_t nE = s->eoff[3];
    double* T_step = (!T_hist && T_hat) ? malloc(nE * sizeof(double)) : NULL;
    if (T_hat) memset(T_hat, 0, nE * sizeof(cplx));
    or_reset(s);
    record_gap(s, glo, gdim, hist);
    for (int n = 0; n < M; ++n) {
        double* T = T_hist ? T_hist + (size_t)n * nE : T_step;
        step_once(s, T);
        record_gap(s, glo, gdim, hist + (size_t)(n + 1) * ncell * 3);
        if (T_hat) {
            cplx ph = cexp(-I * omega * n * s->dt);
            for (size_t q = 0; q < nE; ++q) T_hat[q] += T[q] * ph;
        }
    }
    free(T_step);
    for (int c = 0; c < 6; ++c) {
        if (!s->fwd_end[c]) s->fwd_end[c] = malloc(ncells(s) * sizeof(double));
        memcpy(s->fwd_end[c], s->F[c], ncells(s) * sizeof(double));
    }
    double dt = s->dt, F = 0.0;
    size_t ne_tot = (size_t)(M + 1) * ncell * 3;
    memset(dFdE, 0, ne_tot * sizeof(double));
    if (kind == OR_OBJ_DFT) {
        /* E_hat_e = dt sum_{n=0..M} E_e^n e^{-j w n dt};  F = sum_e |E_hat_e|^2 */
        for (int e = 0; e < ncell * 3; ++e) {
            cplx Eh = 0.0;
            for (int n = 0; n <= M; ++n) Eh += hist[(size_t)n * ncell * 3 + e] * cexp(-I * omega * n * dt);
            Eh *= dt;
            F += creal(Eh * conj(Eh));
            for (int n = 0; n <= M; ++n)
                dFdE[(size_t)n * ncell * 3 + e] = 2.0 * creal(conj(Eh) * dt * cexp(-I * omega * n * dt));
        }
    } else {
        /* Eq. (2) by the rectangle rule, eps_inf of the gap = 1 (air). */
        double w = 0.5 * EPS0 * s->dx * s->dx * s->dx * dt;
        for (int n = nb < 0 ? 0 : nb; n < ne && n <= M; ++n)
            for (int e = 0; e < ncell * 3; ++e) {
                double E = hist[(size_t)n * ncell * 3 + e];
                F += w * E * E;
                dFdE[(size_t)n * ncell * 3 + e] = 2.0 * w * E;
            }
    }
    *F_out = F;
    return 0;
}

int or_objective(or_sim* s, int nsteps, int obj_kind, const int* gap_lo, const int* gap_dims,
                 double omega, int n_begin, int n_end, double* F_out)
{
    if (nsteps < 1 || !gap_ok(s, gap_lo, gap_dims)) return -1;
    int ncell = gap_dims[0] * gap_dims[1] * gap_dims[2];
    size_t ne = (size_t)(nsteps + 1) * ncell * 3;
    double* hist = malloc(ne * sizeof(double));
    double* dFdE = malloc(ne * sizeof(double));
    forward_and_objective(s, nsteps, obj_kind, gap_lo, gap_dims, omega, n_begin, n_end, NULL,
                          NULL, F_out, hist, dFdE);
    free(hist); free(dFdE);
    return 0;
}

/* Adjoint run shared by both gradient estimators.  The adjoint system
 * (supplement Eqs. Tranformations, AdjointSystem) is the forward update run
 * again from zero fields with the time-reversed source S_adj = dF/dE: at
 * adjoint step p the gap edges carry the current (1/dt) dF/dE^{M-p}, injected
 * exactly like J_src, and the forward sources are off.  After adjoint step p
 * visit(s, p, ctx) sees the adjoint fields Et^{p+1}.  The forward sources are
 * restored afterwards; the simulation is left holding the adjoint fields. */
static int adjoint_run(or_sim* s, int M, const int* gap_lo, const int* gap_dims,
                       const double* dFdE, void (*visit)(or_sim*, int, void*), void* ctx)
{
    int ncell = gap_dims[0] * gap_dims[1] * gap_dims[2];
    double* adj = calloc((size_t)M * ncell * 3, sizeof(double));
    if (!adj) return -1;
    for (int p = 0; p < M; ++p)
        for (int e = 0; e < ncell * 3; ++e)
            adj[(size_t)p * ncell * 3 + e] = dFdE[(size_t)(M - p) * ncell * 3 + e] / s->dt;

    int dip_on = s->dip_on, pw_on = s->pw_on, bs_on = s->bs_on;
    int bs_lo[3], bs_dim[3], bs_nsteps = s->bs_nsteps;
    double* bs_table = s->bs_table;
    memcpy(bs_lo, s->bs_lo, sizeof(bs_lo));
    memcpy(bs_dim, s->bs_dim, sizeof(bs_dim));
    s->bs_table = NULL;
    s->dip_on = 0;
    s->pw_on = 0;
    or_set_box_source(s, gap_lo, gap_dims, adj, M);
    or_reset(s);
    for (int p = 0; p < M; ++p) {
        step_once(s, NULL);
        visit(s, p, ctx);
    }
    /* restore the forward sources */
    free(s->bs_table);
    s->bs_table = bs_table;
    memcpy(s->bs_lo, bs_lo, sizeof(bs_lo));
    memcpy(s->bs_dim, bs_dim, sizeof(bs_dim));
    s->bs_nsteps = bs_nsteps;
    s->bs_ncell = bs_dim[0] * bs_dim[1] * bs_dim[2];
    s->bs_on = bs_on;
    s->dip_on = dip_on;
    s->pw_on = pw_on;
    free(adj);
    return 0;
}

/* Field of design edge e (component c of its cell). */
static double design_edge_E(const or_sim* s, size_t e)
{
    int c = 0;
    while (e >= s->eoff[c + 1]) ++c;
    const int* d = s->edim[c];
    const size_t q = e - s->eoff[c];
    const int i = (int)(q % d[0]), j = (int)((q / d[0]) % d[1]), k = (int)(q / ((size_t)d[0] * d[1]));
    return s->F[c][idx3(s, s->dlo[0] + i, s->dlo[1] + j, s->dlo[2] + k)];
}

/* Gradient read-out: per-edge designs return the edge values; per-voxel
 * designs sum the three edges of each voxel (the voxel's density drives all
 * three). */
static void gradient_out(const or_sim* s, const double* ge, double* out)
{
    if (s->per_edge) {
        memcpy(out, ge, s->eoff[3] * sizeof(double));
        return;
    }
    for (int v = 0; v < s->nd; ++v) out[v] = ge[v] + ge[s->eoff[1] + v] + ge[s->eoff[2] + v];
}

typedef struct {
    int M;
    const double* T_hist;
    double* grad;           /* per design edge */
} exact_ctx;

static void exact_visit(or_sim* s, int p, void* vctx)
{
    exact_ctx* c = (exact_ctx*)vctx;
    const size_t nE = s->eoff[3];
    const double* T = c->T_hist + (size_t)(c->M - 1 - p) * nE;
    for (size_t e = 0; e < nE; ++e) c->grad[e] += design_edge_E(s, e) * T[e];
}

/* Time-exact discrete gradient.  Writing Et^m for the adjoint E after m
 * adjoint steps, the gradient (Eq. Gradient_FDTD with the index pairing of
 * the exact discrete adjoint) with respect to the density of design edge e is
 *   dF/drho_e = sum_{n=0}^{M-1} Et_e^{M-n} T_e^{n+1/2},
 * where T is the per-edge factor recorded by edge_update; a voxel's density
 * collects the sum over its three edges. */
int or_gradient(or_sim* s, int nsteps, int obj_kind, const int* gap_lo, const int* gap_dims,
                double omega, int n_begin, int n_end, double* F_out, double* grad_out,
                double* gap_hist_out)
{
    if (nsteps < 1 || s->eoff[3] < 1 || !gap_ok(s, gap_lo, gap_dims)) return -1;
    const int M = nsteps;
    const size_t nE = s->eoff[3];
    int ncell = gap_dims[0] * gap_dims[1] * gap_dims[2];
    size_t ne = (size_t)(M + 1) * ncell * 3;
    double* hist = malloc(ne * sizeof(double));
    double* dFdE = malloc(ne * sizeof(double));
    double* T_hist = malloc((size_t)M * nE * sizeof(double));
    double* ge = calloc(nE, sizeof(double));
    if (!hist || !dFdE || !T_hist || !ge) { free(hist); free(dFdE); free(T_hist); free(ge); return -1; }
    forward_and_objective(s, M, obj_kind, gap_lo, gap_dims, omega, n_begin, n_end, T_hist, NULL,
                          F_out, hist, dFdE);
    if (gap_hist_out) memcpy(gap_hist_out, hist, ne * sizeof(double));
    exact_ctx c = {M, T_hist, ge};
    int rc = adjoint_run(s, M, gap_lo, gap_dims, dFdE, exact_visit, &c);
    if (rc == 0) gradient_out(s, ge, grad_out);
    free(hist); free(dFdE); free(T_hist); free(ge);
    return rc;
}

int or_dft_window(int nsteps, double omega, double dt)
{
    const double per = 2.0 * acos(-1.0) / (omega * dt);   /* steps per period */
    const int q = (int)floor(0.5 * nsteps / per);   /* whole periods in half the run */
    int L = q >= 1 ? (int)lround(q * per) : nsteps / 2;
    if (L < 2) L = nsteps < 2 ? nsteps : 2;
    if (L > nsteps) L = nsteps;
    return L;
}

typedef struct {
    int m0;                 /* first adjoint field index of the window */
    double theta;           /* omega dt */
    cplx* P;                /* per design edge: sum over the window of Et^m exp(-j theta m) */
    double scc, sss, scs;   /* the window's normal matrix */
} dft_ctx;

static void dft_visit(or_sim* s, int p, void* vctx)
{
    dft_ctx* c = (dft_ctx*)vctx;
    const int m = p + 1;
    if (m < c->m0) return;
    const double cs = cos(c->theta * m), sn = sin(c->theta * m);
    c->scc += cs * cs;
    c->sss += sn * sn;
    c->scs += cs * sn;
    const cplx ph = cexp(-I * c->theta * m);
    for (size_t e = 0; e < s->eoff[3]; ++e) c->P[e] += design_edge_E(s, e) * ph;
}

/* Single-frequency (DFT-mode) gradient estimator for OR_OBJ_DFT.  The adjoint
 * source of the DFT objective is a sinusoid of frequency omega; once its
 * transient has died out the adjoint field is Et^m = Re{A exp(j theta m)},
 * theta = omega dt, with one complex amplitude A per design edge.  Put into
 * the time-exact sum above this gives
 *   dF/drho_e ~ Re{ A_e exp(j theta M) T_hat_e },
 *   T_hat_e = sum_{n=0}^{M-1} T_e^{n+1/2} exp(-j theta n),
 * so the forward run keeps only T_hat and the adjoint run only a projection.
 * A is the least-squares fit of a cos(theta m) + b sin(theta m) (A = a - j b)
 * to Et^m over the window of the last L adjoint fields, m in [M-L+1, M], with
 * L = or_dft_window(M, omega, dt): the whole periods that fit in half the
 * run (half the run if that is less than one period).  The estimate tends to
 * the time-exact gradient as the run outlasts the forward pulse and the
 * adjoint transient. */
int or_gradient_dft(or_sim* s, int nsteps, const int* gap_lo, const int* gap_dims, double omega,
                    double* F_out, double* grad_out)
{
    if (nsteps < 2 || s->eoff[3] < 1 || !(omega > 0) || !gap_ok(s, gap_lo, gap_dims)) return -1;
    const int M = nsteps;
    const size_t nE = s->eoff[3];
    int ncell = gap_dims[0] * gap_dims[1] * gap_dims[2];
    size_t ne = (size_t)(M + 1) * ncell * 3;
    double* hist = malloc(ne * sizeof(double));
    double* dFdE = malloc(ne * sizeof(double));
    cplx* T_hat = malloc(nE * sizeof(cplx));
    cplx* P = calloc(nE, sizeof(cplx));
    double* ge = malloc(nE * sizeof(double));
    if (!hist || !dFdE || !T_hat || !P || !ge) {
        free(hist); free(dFdE); free(T_hat); free(P); free(ge);
        return -1;
    }
    forward_and_objective(s, M, OR_OBJ_DFT, gap_lo, gap_dims, omega, 0, -1, NULL, T_hat, F_out,
                          hist, dFdE);
    const int L = or_dft_window(M, omega, s->dt);
    dft_ctx c = {M - L + 1, omega * s->dt, P, 0.0, 0.0, 0.0};
    if (adjoint_run(s, M, gap_lo, gap_dims, dFdE, dft_visit, &c)) {
        free(hist); free(dFdE); free(T_hat); free(P); free(ge);
        return -1;
    }
    /* [scc scs; scs sss] [a; b] = [sum Et cos; sum Et sin] = [Re P; -Im P] */
    const double det = c.scc * c.sss - c.scs * c.scs;
    const cplx W = cexp(I * omega * s->dt * M);
    for (size_t e = 0; e < nE; ++e) {
        const double rc = creal(P[e]), rs = -cimag(P[e]);
        const double a = (c.sss * rc - c.scs * rs) / det;
        const double b = (c.scc * rs - c.scs * rc) / det;
        ge[e] = creal((a - I * b) * W * T_hat[e]);
    }
    gradient_out(s, ge, grad_out);
    free(hist); free(dFdE); free(T_hat); free(P); free(ge);
    return 0;
}

/* ---------------------------------------------------- test helpers ------ */
int or_edge_response(const or_sim* s, int axis, double rho, double gamma, const double* src,
                     int nsteps, double* E_out)
{
    if (axis < 0 || axis > 2 || nsteps < 0) return -1;
    edge_coef ec;
    edge_coef_at(s, axis, rho, gamma, &ec);
    cplx J[2 * OR_MAX_PAIRS] = {0};
    double E = 0.0;
    E_out[0] = 0.0;
    for (int n = 0; n < nsteps; ++n) {
        E = edge_update(&ec, s->dt, E, 0.0, src[n], J, NULL);
        E_out[n + 1] = E;
    }
    return 0;
}

/* Eq. CCPRModel with the interpolation of Eqs. eps_mixed, sigma_mixed,
 * Poles_mixed (e^{jwt} convention). */
void or_eps_ccpr(const or_sim* s, int axis, double rho, double gamma, double w, double* re,
                 double* im)
{
    const or_mat* m1 = &s->mat[0][axis];
    const or_mat* m2 = &s->mat[1][axis];
    cplx jw = I * w;
    cplx eps = (1.0 - rho) * m1->eps_inf + rho * m2->eps_inf;
    eps += ((1.0 - rho) * m1->sigma + rho * m2->sigma + rho * (1.0 - rho) * gamma) / (jw * EPS0);
    for (int i = 0; i < 2; ++i) {
        const or_mat* m = i == 0 ? m1 : m2;
        double kap = i == 0 ? 1.0 - rho : rho;
        for (int p = 0; p < m->np; ++p)
            eps += kap * (m->c[p] / (jw - m->a[p]) + conj(m->c[p]) / (jw - conj(m->a[p])));
    }
    *re = creal(eps);
    *im = cimag(eps);
}
