/*
 * ccpr_oracle.h -- plain FP64 CPU oracle for the CCPR-FDTD forward / adjoint /
 * gradient path of "Free-form inverse design of arbitrary dispersive materials
 * in nanophotonics" (Gedeon, Hassan, Cala Lesina).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, imports or
 * calls this code.  It may be used only by tests/, by the smoke check and by
 * the CPU-baseline leg of the benchmark.  It shares no source, header, table or
 * helper with the GPU path.
 *
 * Units are SI throughout (V/m, A/m, A/m^2, seconds, metres).
 *
 * Grid convention (standard Yee cell, Methods "FDTD implementation"):
 *   Ex[k][j][i] at ((i+1/2)d, j d, k d)    Hx[k][j][i] at (i d, (j+1/2)d, (k+1/2)d)
 *   Ey[k][j][i] at (i d, (j+1/2)d, k d)    Hy[k][j][i] at ((i+1/2)d, j d, (k+1/2)d)
 *   Ez[k][j][i] at (i d, j d, (k+1/2)d)    Hz[k][j][i] at ((i+1/2)d, (j+1/2)d, k d)
 * with i in [0,nx), j in [0,ny), k in [0,nz), x fastest in memory.  Perfect
 * electric walls sit at x=0 and x=nx*d (same for y, z): tangential E on the
 * index-0 planes is held at zero and the planes at index n are implicit zeros.
 *
 * Design voxel (i,j,k) owns the three E edges Ex, Ey, Ez stored at [k][j][i].
 */
#ifndef CCPR_ORACLE_H
#define CCPR_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_PAIRS 8  /* pole pairs per material and axis */

typedef struct or_sim or_sim;

/* Create a simulation on an nx*ny*nz grid with cell size dx [m] and Courant
 * number S = c0*dt/dx.  npml = CPML thickness in cells (0: bare PEC walls).
 * CPML grading: sigma = sigma_max*xi^m, kappa = 1+(kappa_max-1)*xi^m,
 * alpha = alpha_max*(1-xi), sigma_max = sigma_scale*0.8*(m+1)/(eta0*dx).
 * Returns NULL on invalid arguments. */
or_sim* or_create(int nx, int ny, int nz, double dx, double courant, int npml,
                  double pml_m, double pml_kappa_max, double pml_alpha_max,
                  double pml_sigma_scale);
void or_destroy(or_sim* s);
double or_dt(const or_sim* s);

/* CCPR coefficients (Eq. CCPRModel) of material slot (1 = the rho=0 material,
 * 2 = the rho=1 material) for one field axis (0,1,2 = x,y,z).  a and c hold
 * np complex numbers as (re,im) pairs.  Returns 0 or -1. */
int or_set_material(or_sim* s, int slot, int axis, double eps_inf, double sigma,
                    int np, const double* a, const double* c);

/* Design box [lo, lo+dims) with one density per voxel (x fastest) and the
 * conductivity damping gamma of Eq. sigma_mixed.  Outside the box: vacuum. */
int or_set_design(or_sim* s, const int* lo, const int* dims, double gamma,
                  const double* rho);

/* Design of dims = N cells at lo with one density per E edge (Sec. "FDTD
 * implementation and design export"): component c has the edges of the box
 * [lo, lo + N + 1 - e_c) (N_l + 1 - delta(c,l) along axis l), so the box's
 * boundary edges are design variables too.  rho holds the x edges, then the
 * y edges, then the z edges, each x fastest.  The gradient then has one
 * value per edge in the same order (or_design_outputs values). */
int or_set_design_edges(or_sim* s, const int* lo, const int* dims, double gamma,
                        const double* rho);

/* Number of gradient values: voxels (or_set_design) or edges
 * (or_set_design_edges). */
long long or_design_outputs(const or_sim* s);

/* Point current J_src [A/m^2] on the 'axis' edge of 'cell'; wave[n] is the
 * value at t=(n+1/2)dt for n in [0,nw). */
int or_set_dipole(or_sim* s, const int* cell, int axis, const double* wave, int nw);

/* Total-field / scattered-field plane wave travelling along +/- prop_axis,
 * E polarised along pol_axis.  The total-field box spans cell corners
 * [lo, hi] (inclusive, in cell units).  wave[n] is the incident E [V/m] at the
 * launch point at t = n dt, n in [0,nw). */
int or_set_planewave(or_sim* s, int prop_axis, int sign, int pol_axis,
                     const int* lo, const int* hi, const double* wave, int nw);

/* Current source on every E edge owned by the cells of box [lo, lo+dims):
 * table[(n*ncell + c)*3 + axis] at t=(n+1/2)dt (cells x-fastest). */
int or_set_box_source(or_sim* s, const int* lo, const int* dims,
                      const double* table, int nsteps);

void or_clear_sources(or_sim* s);
void or_reset(or_sim* s);          /* zero all fields and the step counter   */
void or_run(or_sim* s, int nsteps); /* advance nsteps full leapfrog steps      */
int  or_step_count(const or_sim* s);
/* comp 0..5 = Ex,Ey,Ez,Hx,Hy,Hz; out holds nz*ny*nx doubles. */
void or_get_field(const or_sim* s, int comp, double* out);
/* comp 0..5 of the state at the end of the forward run inside the last
 * or_gradient / or_gradient_dft / or_objective call (the call itself leaves
 * the adjoint fields, or the forward ones); -1 before any such call. */
int or_get_forward_end_field(const or_sim* s, int comp, double* out);
/* overwrite a field component (tests: eigenmode initial states) */
void or_set_field(or_sim* s, int comp, const double* in);

#define OR_OBJ_TIME 0 /* F = eps0/2 * d^3 dt * sum_{n in window} sum_gap E^2   */
#define OR_OBJ_DFT  1 /* F = sum_gap |dt * sum_{n=0..M} E^n exp(-j w n dt)|^2  */

/* Forward run of nsteps with the sources currently set, the objective over the
 * gap box [gap_lo, gap_lo+gap_dims), then the adjoint run and the time-exact
 * discrete gradient dF/drho per design voxel.  Window [n_begin, n_end) applies
 * to OR_OBJ_TIME.  grad_out has one double per design voxel; gap_hist_out (may
 * be NULL) receives E at the gap edges, [(n*ncell+c)*3+axis], n in [0,M].
 * Leaves the simulation holding the adjoint fields.  Returns 0 or -1. */
int or_gradient(or_sim* s, int nsteps, int obj_kind, const int* gap_lo,
                const int* gap_dims, double omega, int n_begin, int n_end,
                double* F_out, double* grad_out, double* gap_hist_out);

/* DFT-mode gradient estimator for OR_OBJ_DFT (single frequency omega): the
 * forward run keeps T_hat_k(v) = sum_n T_k^{n+1/2}(v) exp(-j omega n dt)
 * instead of the history; the adjoint field's steady state is fitted as
 * Et^m = Re{A exp(j omega dt m)} (least squares over the last L adjoint
 * fields, L = or_dft_window); grad_v = sum_k Re{A_k exp(j omega dt M) T_hat_k}.
 * Approximate: tends to or_gradient's result as the fields decay within the
 * run.  Leaves the simulation holding the adjoint fields.  Returns 0 or -1. */
int or_gradient_dft(or_sim* s, int nsteps, const int* gap_lo, const int* gap_dims,
                    double omega, double* F_out, double* grad_out);

/* Adjoint fields in the DFT-mode fit window: the whole periods of
 * 2 pi / (omega dt) steps that fit in half the run, rounded to whole steps
 * (half the run when that is less than one period; at least 2, at most
 * nsteps). */
int or_dft_window(int nsteps, double omega, double dt);

/* Objective only (forward run, no adjoint). */
int or_objective(or_sim* s, int nsteps, int obj_kind, const int* gap_lo,
                 const int* gap_dims, double omega, int n_begin, int n_end,
                 double* F_out);

/* Single-edge material response with the curl switched off: the 'axis' edge
 * of a voxel of density rho, driven by src[n] at t=(n+1/2)dt, n in [0,nsteps).
 * E_out[n] = E^n for n in [0, nsteps]. */
int or_edge_response(const or_sim* s, int axis, double rho, double gamma,
                     const double* src, int nsteps, double* E_out);

/* Closed-form interpolated relative permittivity (Eq. CCPRModel with
 * Eqs. eps_mixed, sigma_mixed, Poles_mixed) at angular frequency w (e^{jwt}). */
void or_eps_ccpr(const or_sim* s, int axis, double rho, double gamma, double w,
                 double* re, double* im);

int or_num_threads(void);

/* Diagnostic, not part of the reference: with on != 0 every stored state
 * word (fields, CPML memories, pole currents, incident-wave values as read)
 * is rounded to FP32 after each half-step update, the arithmetic staying
 * FP64.  It measures the floor that FP32 storage alone puts under any FP32
 * implementation of the same recurrence. */
void or_set_fp32_storage(or_sim* s, int on);

/* CPML recursive-convolution coefficients along axis (0..2) at integer node q
 * (half = 0) or at q + 1/2 (half = 1), 0 <= q < n[axis]: psi' = b psi + a d,
 * derivative scaled by 1/kappa.  For the pins only.  Returns 0, or -1 for bad
 * arguments. */
int or_get_pml_coef(const or_sim* s, int axis, int half, int q, double* b, double* a, double* kappa);

#ifdef __cplusplus
}
#endif
#endif
