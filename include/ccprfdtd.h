/*
 * ccprfdtd.h -- C-ABI of the MI355X (gfx950) CCPR-FDTD forward / adjoint /
 * gradient library.
 *
 * The library solves the density-based inverse-design problem of Gedeon,
 * Hassan and Cala Lesina, "Free-form inverse design of arbitrary dispersive
 * materials in nanophotonics":
 *   maximise F[E] over rho in [0,1], subject to Maxwell's equations with the
 *   complex-conjugate pole-residue (CCPR) model (Eq. CCPRModel), the density
 *   interpolation of Eqs. eps_mixed, sigma_mixed, Poles_mixed, and a diagonal
 *   permittivity tensor (Sec. "Time-domain adjoint formulation");
 * by a 3-D Yee FDTD forward run, a time-reversed adjoint run that is the same
 * solver with another source (supplement Eqs. Tranformations, AdjointSystem),
 * and the design gradient accumulated from forward/adjoint field correlations
 * (Eq. Gradient_FDTD, in the exact discrete index pairing).
 *
 * Conventions
 *  - Units are SI at this interface (m, s, V/m, A/m, A/m^2, S/m, rad/s).
 *    Field scaling used inside the library is private.
 *  - Grid: cells i in [0,nx), j in [0,ny), k in [0,nz); x fastest in every
 *    array.  Ex[k][j][i] sits at ((i+1/2)dx, j dx, k dx), Ey at
 *    (i dx, (j+1/2)dx, k dx), Ez at (i dx, j dx, (k+1/2)dx), Hx at
 *    (i dx, (j+1/2)dx, (k+1/2)dx), Hy at ((i+1/2)dx, j dx, (k+1/2)dx), Hz at
 *    ((i+1/2)dx, (j+1/2)dx, k dx).  Perfect electric walls bound the domain
 *    (behind the CPML when one is requested).
 *  - Design voxel (i,j,k) carries one density that drives the three E edges
 *    stored at [k][j][i]; the gradient is one value per voxel.
 *  - Ownership: every pointer argument is caller-owned.  Host buffers are
 *    consumed before the call returns.  Device buffers (mem == CCPR_MEM_DEVICE)
 *    are read or written by work enqueued on the bound stream and must stay
 *    valid until that work completes.  The workspace is borrowed, never freed.
 *  - Errors: every call returns a ccpr_status; no exception crosses the ABI.
 *    ccpr_last_error() describes the last failure of that solver.
 *  - Threading: one host thread per solver at a time.  Solvers are
 *    independent; several may share a device and a stream.
 */
#ifndef CCPRFDTD_H
#define CCPRFDTD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CCPR_OK = 0,
    CCPR_EINVAL = -1,    /* bad shape, enum, NaN or out-of-range density      */
    CCPR_ECFL = -2,      /* Courant number above 1/sqrt(3)                     */
    CCPR_ENOMEM = -3,    /* workspace too small                                */
    CCPR_EDEVICE = -4,   /* HIP runtime error                                  */
    CCPR_ESTATE = -5,    /* call out of order (e.g. adjoint before forward)    */
    CCPR_EDIVERGED = -6, /* non-finite or exploding fields                     */
    CCPR_ENOTSUP = -7    /* valid request outside what the library supports    */
} ccpr_status;

enum { CCPR_MEM_HOST = 0, CCPR_MEM_DEVICE = 1 };
enum { CCPR_OBJ_TIME_E2 = 0, CCPR_OBJ_DFT_E2 = 1 };
enum { CCPR_GRAD_TIME_EXACT = 0, CCPR_GRAD_DFT = 1 };
enum { CCPR_EX = 0, CCPR_EY, CCPR_EZ, CCPR_HX, CCPR_HY, CCPR_HZ };

#define CCPR_MAX_PAIRS_PER_AXIS 8 /* pole pairs over both materials, per axis */
#define CCPR_MAX_NX 1024          /* x extent handled by one workgroup row    */
#define CCPR_STATIC_WORKSPACE_BYTES (64ull << 20) /* ccpr_bind_static_workspace */

typedef struct ccpr_solver ccpr_solver;

/* Grid and absorbing boundary.  dt = courant * dx / c0; courant must be in
 * (0, 1/sqrt(3)].  npml cells of CFS-CPML line every wall (0 = bare PEC).
 * Grading (Methods, "Technical details": only the thickness is given; these
 * are the standard polynomial CFS-CPML parameters):
 *   xi = depth/npml, sigma = sigma_scale*0.8*(m+1)/(eta0*dx) * xi^m,
 *   kappa = 1 + (kappa_max-1) xi^m, alpha = alpha_max (1-xi). */
typedef struct {
    int nx, ny, nz;
    double dx;
    double courant;
    int npml;
    double pml_order;       /* m, typically 3                    */
    double pml_kappa_max;   /* typically 1                       */
    double pml_alpha_max;   /* S/m, typically 0.05               */
    double pml_sigma_scale; /* typically 1                       */
} ccpr_grid;

/* Create a solver (host state only; no device work until a workspace is
 * bound).  Validates the grid: CCPR_EINVAL for non-positive sizes or a CPML
 * thicker than half the grid, CCPR_ECFL for courant > 1/sqrt(3), CCPR_ENOTSUP
 * for nx > CCPR_MAX_NX.  *out receives the handle (NULL on error). */
ccpr_status ccpr_create(const ccpr_grid* g, ccpr_solver** out);

/* Destroy a solver.  Does not free the bound workspace (caller-owned).
 * Waits for the solver's outstanding stream work. */
void ccpr_destroy(ccpr_solver* s);

/* Text of the last error of this solver ("" if none).  Valid until the next
 * call on the same solver.  s may be NULL (returns the last creation error). */
const char* ccpr_last_error(const ccpr_solver* s);

/* CCPR coefficients of one material for one field axis (Eq. CCPRModel;
 * diagonal anisotropy by per-axis calls, Sec. "Time-domain adjoint
 * formulation").  slot 1 is the material at rho = 0, slot 2 at rho = 1
 * (Eqs. eps_mixed, sigma_mixed, Poles_mixed).  a, c: npairs complex numbers as
 * (re, im) doubles [1/s].  Unset slots are vacuum (eps_inf 1, no poles).
 * CCPR_EINVAL for axis/slot out of range, npairs < 0, non-finite values or
 * a pole with Re a > 0 (it grows on its own: not a passive material; other
 * non-passive sets, e.g. a negative static susceptibility, make the fields
 * grow and the next ccpr_forward return CCPR_EDIVERGED);
 * CCPR_ENOTSUP if the two slots together exceed CCPR_MAX_PAIRS_PER_AXIS on an
 * axis. */
ccpr_status ccpr_set_material(ccpr_solver* s, int slot, int axis, double eps_inf,
                              double sigma, int npairs, const double* a, const double* c);

/* Design box [lo, lo+dims) with one density per voxel (float, x fastest,
 * dims[0]*dims[1]*dims[2] values) and the conductivity damping gamma [S/m] of
 * Eq. sigma_mixed.  The box must lie inside the grid and outside the CPML.
 * Densities must be finite and within [0,1] (checked for host input; for
 * device input the check runs on the device and is reported by the next
 * ccpr_forward / ccpr_step).  mem = CCPR_MEM_DEVICE requires a bound
 * workspace: the copy is enqueued on the bound stream.  Outside the box the
 * medium is vacuum. */
ccpr_status ccpr_set_design(ccpr_solver* s, const int lo[3], const int dims[3], double gamma,
                            const float* rho, int mem);

/* Design of dims = (Nx, Ny, Nz) cells at lo with one density per E edge
 * (Sec. "FDTD implementation and design export": the density rho_{k,n} sits
 * at each E_k position, N~_k = prod_l (N_l + 1 - delta_kl) of them, so the
 * edges on the box's far faces are design variables too).  Component k's
 * edges are those of cells [lo, lo + N + 1 - e_k) (e_k the unit vector of
 * axis k); rho holds the x edges, then the y edges, then the z edges, each
 * block x fastest in its own extents (N~_x + N~_y + N~_z floats).  Each edge's
 * density sets its own material (Eqs. eps_mixed, sigma_mixed, Poles_mixed);
 * the far-face edges along their own axis (E_k at index lo_k + N_k) are not
 * design edges and stay vacuum.  The cells [lo, lo + N + 1) must lie inside
 * the grid, off the walls and outside the CPML.  Checks, memory kinds and
 * ownership as ccpr_set_design.  ccpr_gradient then returns one value per
 * edge in the same order and layout. */
ccpr_status ccpr_set_design_edges(ccpr_solver* s, const int lo[3], const int dims[3], double gamma,
                                  const float* rho, int mem);

/* Point current source (host data): J_src [A/m^2] on the 'axis' edge of
 * 'cell', wave[n] being its value at t = (n+1/2) dt for n in [0,nsteps); zero
 * afterwards.  Replaces any previous source.  The cell must lie outside the x
 * CPML layers (CCPR_ENOTSUP at the next run otherwise): source cells are
 * finished in the same launch as the x-CPML pass of E. */
ccpr_status ccpr_set_source_dipole(ccpr_solver* s, const int cell[3], int axis,
                                   const double* wave, int nsteps);

/* Axis-aligned plane wave by total-field/scattered-field (host data),
 * travelling along sign * prop_axis with E along pol_axis (Sec. "Topology
 * Optimization Setup": the excitation is a polarised plane wave).  The total
 * field box spans cell corners [lo, hi] (inclusive), strictly inside the grid
 * and outside the CPML.  wave[n] is the incident E [V/m] at the launch point of
 * an exact 1-D auxiliary line at t = n dt, n in [0,nsteps).  Replaces any
 * previous source. */
ccpr_status ccpr_set_source_planewave(ccpr_solver* s, int prop_axis, int sign, int pol_axis,
                                      const int lo[3], const int hi[3], const double* wave,
                                      int nsteps);

/* Objective over the gap box [lo, lo+dims) using all three E edges of each gap
 * cell:
 *   CCPR_OBJ_TIME_E2: F = eps0/2 dx^3 dt sum_{n in [n_begin,n_end)} sum E^2
 *                     (Eq. 2, rectangle rule, air in the gap);
 *   CCPR_OBJ_DFT_E2:  F = sum |dt sum_{n=0..M} E^n exp(-j omega n dt)|^2.
 * n_end < 0 means "through the last step".  The gap box must lie outside the
 * x CPML layers (CCPR_ENOTSUP at the next run otherwise: its cells are the
 * adjoint run's source cells). */
ccpr_status ccpr_set_objective(ccpr_solver* s, int kind, const int lo[3], const int dims[3],
                               double omega, int n_begin, int n_end);

/* Forward-history checkpointing for the time-exact gradient.  The forward run
 * stores one gradient factor (3 floats) per design voxel and step; when the
 * full history does not fit, the run is split into segments of
 * checkpoint_every steps.  The last segments whose history fits the bound
 * workspace keep the forward run's records ("resident" segments); the others
 * start from state checkpoints and are recomputed during the adjoint.
 * 0 = choose the segment length that recomputes the fewest steps within the
 * bound workspace.  Results are bit-identical for every segmentation. */
ccpr_status ccpr_set_checkpointing(ccpr_solver* s, int checkpoint_every);

/* At most max_resident resident segments (0, the default: as many as fit the
 * workspace).  1 recomputes every segment but the last, with the smallest
 * history buffer.  CCPR_EINVAL if negative. */
ccpr_status ccpr_set_resident_segments(ccpr_solver* s, int max_resident);

/* Gradient estimator (default CCPR_GRAD_TIME_EXACT: the exact discrete
 * gradient of ccpr_gradient, from the stored or recomputed forward history).
 * CCPR_GRAD_DFT, for the single-frequency objective CCPR_OBJ_DFT_E2 only
 * (CCPR_EINVAL at ccpr_forward otherwise): on-the-fly DFT correlation.  The
 * adjoint source of that objective is a sinusoid of frequency omega, so once
 * its transient has died out the adjoint field is Et^m = Re{A exp(j th m)},
 * th = omega dt, one complex amplitude A per design edge; in the sum of Eq.
 * Gradient_FDTD this gives
 *   dF/drho_v ~ sum_k Re{ A_k(v) exp(j th M) That_k(v) },
 *   That_k(v) = sum_{n=0}^{M-1} T_k^{n+1/2}(v) exp(-j th n).
 * The forward run keeps That (6 floats per voxel) instead of the history, the
 * adjoint run projects Et^m onto exp(-j th m) over the window of its last L
 * fields (L: the whole periods of 2 pi / th steps that fit in half the run,
 * rounded to whole steps; half the run if shorter than one period), and A is
 * the least-squares fit a - j b of a cos(th m) + b sin(th m) over that window.
 * Needs no checkpoints (checkpoint_every is ignored) and 48 bytes per design
 * voxel; approximate: it tends to the time-exact gradient as the run
 * outlasts the forward pulse and the adjoint transient. */
ccpr_status ccpr_set_gradient_mode(ccpr_solver* s, int mode);

/* Device bytes needed for a forward + adjoint + gradient solve of nsteps
 * (nsteps = 0: field stepping only) with the current configuration and
 * checkpoint_every (0: full history), with one resident segment.  Drives
 * admission in serving. */
ccpr_status ccpr_workspace_size(const ccpr_solver* s, int nsteps, uint64_t* bytes);

/* The most device bytes such a solve can use: every segment resident (at
 * most max_resident of them), so nothing is recomputed.  Between the two
 * sizes the solver keeps as many of the last segments resident as fit. */
ccpr_status ccpr_workspace_size_max(const ccpr_solver* s, int nsteps, uint64_t* bytes);

/* Borrow a device buffer of 'bytes' (256-byte aligned) as workspace and bind a
 * HIP stream (hipStream_t, may be NULL for the null stream).  The library
 * never allocates device memory itself.  Rebinding resets the solver. */
ccpr_status ccpr_bind_workspace(ccpr_solver* s, void* dev_ptr, uint64_t bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): bind the
 * library's own static workspace of the current device instead of a caller
 * buffer -- a file-scope device array of CCPR_STATIC_WORKSPACE_BYTES (64 MiB)
 * that each device holds from its first such bind until the process ends.
 * Same semantics as ccpr_bind_workspace with that buffer; neither this call
 * nor the solves run on it allocate (no hipMalloc / hipFree, no stream or
 * event creation: the grid pass runs as one launch on hip_stream).
 * Limits: a solve whose workspace (ccpr_workspace_size) exceeds the array
 * fails with CCPR_ENOMEM at bind time (fixed part) or at ccpr_forward (with
 * its history), with a message naming both sizes.  One solver per device at
 * a time: binding another solver to the same device's array unbinds the
 * previous one (its later calls report CCPR_ESTATE, no workspace bound),
 * and the array keeps the last solve's contents (every run clears what must
 * start at zero).  Work of two solvers on one device's array must not
 * overlap in time: calls that overlap race. */
ccpr_status ccpr_bind_static_workspace(ccpr_solver* s, void* hip_stream);

/* Forward run of nsteps from zero fields, recording the gap monitor and the
 * gradient history (DFT gradient mode: its transform), then the objective
 * (synchronises the stream to return *objective_out, which may be NULL).
 * CCPR_EDIVERGED when the divergence watchdog (ccpr_set_watchdog) tripped
 * -- every step after it is skipped on the device, and ccpr_step_count then
 * returns the steps done when it tripped -- or when the objective is not
 * finite (a non-passive material); the solve is then not usable for
 * ccpr_adjoint. */
ccpr_status ccpr_forward(ccpr_solver* s, int nsteps, double* objective_out);

/* Adjoint run (same update, zero initial fields, time-reversed source
 * (1/dt) dF/dE at the gap edges, no incident wave) with the gradient
 * correlation; recomputes checkpointed segments as needed.  Stream-ordered
 * (with the watchdog on it synchronises at the end to read it:
 * CCPR_EDIVERGED if it tripped).  CCPR_ESTATE before a successful
 * ccpr_forward, and for a second adjoint of the same forward run when this
 * one recomputed segments (their history overwrote the first resident
 * segment's; ccpr_forward_serial then returns -1). */
ccpr_status ccpr_adjoint(ccpr_solver* s);

/* Serial number of the forward run whose state the next ccpr_adjoint would
 * use (it counts the successful forward runs of this solver), or -1 when no
 * such state exists: no forward run yet, a configuration change since, or an
 * adjoint run that recomputed segments over its history.  Callers that hold
 * on to a forward result (a differentiable objective's backward) compare it
 * with the serial they saw and run the forward again on a mismatch. */
long long ccpr_forward_serial(const ccpr_solver* s);

/* Divergence watchdog (failure detection): after every 'every'-th step of
 * the forward and adjoint runs (including the serving engine's), one small
 * launch checks the E edges of the gap box; if one is not finite or larger
 * than 'limit' in units of the run's source amplitude (the incident wave's
 * peak, or the peak current of the dipole / adjoint source per step: a
 * passive medium stays orders of magnitude below the default 1e15), every
 * later step kernel of the run returns at once and the run reports
 * CCPR_EDIVERGED.  every = 0 turns it off (default: every 128 steps).
 * CCPR_EINVAL for every < 0 or limit outside (0, 3e38]. */
ccpr_status ccpr_set_watchdog(ccpr_solver* s, int every, double limit);

/* Spectrum of the gap field recorded by the last ccpr_forward (the monitor of
 * Eq. Objective_analyitically_enhancement read in the frequency domain, as
 * the paper's averaged gap-enhancement spectra): for each of nf angular
 * frequencies omega[f] [rad/s],
 *   mean_E2[f] = (1/ne) sum_e |dt sum_{n=0..M} E_e^n exp(-j omega[f] n dt)|^2
 * over the ne = 3 x (gap cells) edges, in (V s / m)^2.  Dividing by the same
 * quantity of the incident field gives the averaged enhancement spectrum.
 * Host arrays; synchronises.  CCPR_ESTATE before ccpr_forward; CCPR_EINVAL
 * for more frequencies than the workspace's staging area holds (one per 16
 * bytes of max(4 cells, 8 density values)). */
ccpr_status ccpr_gap_spectrum(ccpr_solver* s, const double* omega, int nf, double* mean_E2);

/* dF/drho per design voxel (FP64: in SI units the objective of a weak source
 * is far below the FP32 range), dims of the design box, x fastest, written to
 * host memory (synchronises) or device memory (stream-ordered); after
 * ccpr_set_design_edges, one value per design edge in the layout of its
 * densities.  Eq. Gradient_FDTD in the exact discrete pairing, per edge e
 *   dF/drho_e = sum_{n=0}^{M-1} Et_e^{M-n} T_e^{n+1/2}
 * and per voxel the sum over its three edges:
 *   dF/drho_v = sum_k sum_{n=0}^{M-1} Et_k^{M-n}(v) T_k^{n+1/2}(v),
 *   T = eps0 deps_k (E^{n+1}-E^n) + dsig_k,eff dt (E^{n+1}+E^n)/2
 *       + dt sum_p dkappa_p Re{J_p^{n+1}+J_p^n},
 * Et^m the adjoint E after m adjoint steps, dsig_eff = sig2-sig1+(1-2 rho) gamma
 * (DFT gradient mode: the estimate of ccpr_set_gradient_mode).
 * CCPR_ESTATE before ccpr_adjoint. */
ccpr_status ccpr_gradient(ccpr_solver* s, double* grad, int mem);

/* Zero the fields and the step counter (forward source active). */
ccpr_status ccpr_reset(ccpr_solver* s);

/* Advance n leapfrog steps with the configured forward source and no
 * recording. */
ccpr_status ccpr_step(ccpr_solver* s, int n);

/* Copy one field component (comp = CCPR_EX..CCPR_HZ, SI units) of the current
 * state -- the forward state after ccpr_step/ccpr_forward, the adjoint state
 * after ccpr_adjoint -- into nz*ny*nx floats (host: synchronises; device:
 * stream-ordered). */
ccpr_status ccpr_get_field(ccpr_solver* s, int comp, float* out, int mem);

/* Number of leapfrog steps taken since the last reset (forward state). */
int ccpr_step_count(const ccpr_solver* s);

/* ---- diagnostics ------------------------------------------------------- */

/* Enable (1) or disable (0) stream-event timing of the leapfrog loops of
 * ccpr_forward and ccpr_adjoint, and clear the counters.  Timing records HIP
 * events on the bound stream around each loop and around every launch of the
 * grid kernel (the one that streams all cells), and synchronises the stream
 * at the end of each loop.  enable = k > 1 times only every k-th grid pass
 * (the loops are still timed whole): fewer events in the stream, the same
 * average pass duration.  CCPR_EINVAL if negative. */
ccpr_status ccpr_set_timing(ccpr_solver* s, int enable);

/* Accumulated event time [ms] of the timed leapfrog loops and the number of
 * leapfrog steps they contain (their ratio is the average step time, all
 * kernels of a step and launch gaps included). */
ccpr_status ccpr_get_timing(const ccpr_solver* s, double* step_ms_total, long long* step_launches);

/* Accumulated event time [ms] of the timed grid passes inside the timed
 * loops and their number (their ratio is the grid pass's average duration).  A pass is
 * one launch of the grid kernel, or two concurrent launches (CPML tiles on
 * the bound stream, interior tiles on a second stream); it is timed from an
 * event on the bound stream before the first launch to the later of the
 * events recorded after each launch on its own stream. */
ccpr_status ccpr_get_grid_timing(const ccpr_solver* s, double* grid_ms_total, long long* grid_launches);

/* Segment count and length of the last ccpr_forward layout, and the number of
 * z-planes one workgroup of the step kernel marches over.  Any pointer may be
 * NULL. */
ccpr_status ccpr_get_info(const ccpr_solver* s, int* segments, int* segment_steps, int* tile_planes);

/* Resident segments of the last ccpr_forward layout (segments - resident of
 * them are recomputed by ccpr_adjoint).  CCPR_EINVAL for NULL arguments. */
ccpr_status ccpr_get_resident_segments(const ccpr_solver* s, int* resident);

/* Launch shape: nominal z-planes per workgroup of the step kernel (default
 * 5; the planes are split into about nz/planes chunks of equal estimated
 * cost, so chunks in the CPML are thinner).  Results do not depend on it. */
ccpr_status ccpr_set_tile_planes(ccpr_solver* s, int planes);

/* Launch shape: y rows per thread of the step kernel, 2 (default) or 4
 * (4 only for nx <= 512: CCPR_ENOTSUP otherwise).  Results do not depend on
 * it. */
ccpr_status ccpr_set_tile_rows(ccpr_solver* s, int rows);

/* Launch shape: on = 1 lets the grid pass finish the design cells itself --
 * the CCPR pole-pair update, pole currents, gradient record or correlation
 * and gap monitor of supplement Eqs. Maxwells2 a, b and Eq. Gradient_FDTD,
 * computed from E^n and curl H still in registers -- in a launch of the
 * tiles that own design cells after the CPML tiles; on = 0 (default) leaves
 * them to the separate design pass, which is faster on the configurations
 * measured (the fused launch runs its design cells plane by plane inside the
 * z-march, at a quarter of the occupancy).  The grid pass does it only for
 * one density per voxel with the time-exact gradient, nx <= 512, at most 8
 * pole pairs per axis, no design cell in a tile that touches the y or z
 * CPML, and grids large enough for the split grid pass; otherwise the
 * separate pass runs whatever the setting.  Results do not depend on it
 * (the arithmetic is the same).  Takes effect at the next forward or
 * adjoint run.  CCPR_EINVAL unless on is 0 or 1. */
ccpr_status ccpr_set_design_fusion(ccpr_solver* s, int on);

/* *fused = 1 if the last planned run finished the design cells in the grid
 * pass (see ccpr_set_design_fusion), else 0.  CCPR_EINVAL for NULL. */
ccpr_status ccpr_get_design_fusion(const ccpr_solver* s, int* fused);

/* ---- serving engine ----------------------------------------------------- */
/* Continuous batching of whole solves (forward run, objective, adjoint run,
 * gradient: the path of ccpr_forward + ccpr_adjoint + ccpr_gradient) for many
 * solvers of different grids and pole counts.  The engine owns one device
 * arena and a worker thread: it admits submitted solves in arrival order
 * while the arena (first fit) and the slot limit allow and binds each to its
 * own slice of the arena.  Solves with one density per voxel and the
 * time-exact gradient are batched: those of one padded x width (nx rounded up
 * to 64) share a HIP stream, and each batched grid, aux and post launch
 * advances up to 8 of them by one leapfrog step (a table in the launch maps
 * workgroups to solves); their other work (checkpoints, objective, results)
 * is enqueued per solve on the same stream in order.  Other solves get HIP
 * streams of their own and are fed with chunks of leapfrog steps so their
 * kernels overlap on the device.  A solve's objective and gradient are the
 * same bit for bit as on its own (the same arithmetic in the same order).
 * When a solve finishes, its results are copied to host memory and its slice
 * (and streams) are released. */

typedef struct ccpr_engine ccpr_engine;

enum { CCPR_JOB_QUEUED = 0, CCPR_JOB_RUNNING = 1, CCPR_JOB_DONE = 2, CCPR_JOB_FAILED = 3 };

/* Design filtering and projection (Sec. Filtering and projection), on the
 * per-voxel density grid of the design box: dims = (nx, ny, nz), arrays of
 * nx*ny*nz values, x fastest, distances in voxels.  All pointers are device
 * memory owned by the caller; the calls are stream-ordered on hip_stream
 * (hipStream_t, may be NULL) and do not synchronise.  They take no solver:
 * CCPR_EINVAL for bad arguments, CCPR_EDEVICE when the launch fails (no
 * message is kept).
 *
 * ccpr_filter_project: Eq. FilterFunction, the cone filter
 *   rho_filtered[n] = sum_m w(n,m) rho[m] / sum_m w(n,m),  w = R - |r_m - r_n|,
 * over the design voxels m with |r_m - r_n| < R (1 <= radius <= 17), writing
 * the weight sum weight_sum[n] = sum_m w(n,m) for the backward pass; then Eq.
 * Projection, the smoothed Heaviside
 *   rho_projected = (tanh(beta eta) + tanh(beta (rho_filtered - eta)))
 *                   / (tanh(beta eta) + tanh(beta (1 - eta))),
 * beta > 0, 0 <= eta <= 1.  FP32. */
ccpr_status ccpr_filter_project(const float* rho, float* rho_filtered, float* rho_projected, float* weight_sum,
                                const int dims[3], double radius, double beta, double eta, void* hip_stream);

/* Eq. GradientsFiltered, the chain rule of ccpr_filter_project:
 *   dF_drho[n] = sum_m dF_dprojected[m] * drho_projected/drho_filtered[m]
 *                * w(m,n) / weight_sum[m],
 * from that call's rho_filtered and weight_sum (same dims, radius, beta,
 * eta).  FP64 in and out. */
ccpr_status ccpr_filter_project_grad(const double* dF_dprojected, const float* rho_filtered, const float* weight_sum,
                                     double* dF_drho, const int dims[3], double radius, double beta, double eta,
                                     void* hip_stream);

/* ccpr_filter_project and ccpr_filter_project_grad for a per-edge design
 * (ccpr_set_design_edges; Sec. "FDTD implementation and design export"):
 * dims = (Nx, Ny, Nz) cells, arrays of N~_x + N~_y + N~_z values in the
 * per-edge layout (x edges, then y, then z, each x fastest in its extents
 * N_l + 1 - delta_kl).  Each density sits at its edge centre, (i+1/2, j, k)
 * for x edges, (i, j+1/2, k) for y, (i, j, k+1/2) for z, and Eq.
 * FilterFunction's sphere takes in the edges of all three components within
 * R of it.  Same arguments, precision and errors as the per-voxel calls. */
ccpr_status ccpr_filter_project_edges(const float* rho, float* rho_filtered, float* rho_projected,
                                      float* weight_sum, const int dims[3], double radius, double beta, double eta,
                                      void* hip_stream);
ccpr_status ccpr_filter_project_grad_edges(const double* dF_dprojected, const float* rho_filtered,
                                           const float* weight_sum, double* dF_drho, const int dims[3], double radius,
                                           double beta, double eta, void* hip_stream);

/* Eq. MeasureOfNon-discretness: *out = sum 4 rho (1 - rho) / n x 100 (per
 * cent) over n projected densities, FP64, written to device memory; the
 * summation order is fixed (bitwise reproducible). */
ccpr_status ccpr_nondiscreteness(const float* rho_projected, long long n, double* out, void* hip_stream);

/* arena: device memory the engine sub-allocates for the solves' workspaces
 * (256-byte aligned, caller-owned, valid until ccpr_engine_destroy returns);
 * max_active: solves on the device at once (1..64); chunk_steps: leapfrog
 * steps enqueued per solve per turn.  The engine creates its HIP streams (two
 * per slot, default priority) here.  CCPR_EINVAL on bad arguments,
 * CCPR_EDEVICE if the streams or the slots' pinned result buffers cannot be
 * created. */
ccpr_status ccpr_engine_create(void* arena, uint64_t arena_bytes, int max_active, int chunk_steps,
                               ccpr_engine** out);

/* Queue a solve of nsteps forward (and as many adjoint) steps.  The solver must
 * have its materials, host densities (CCPR_MEM_HOST), source and objective
 * set; the engine binds it to arena memory while the job runs, so the caller
 * must not use it until the job is DONE or FAILED (afterwards it is unbound).
 * CCPR_ENOMEM if its workspace (ccpr_workspace_size) exceeds the arena,
 * CCPR_ESTATE if the solver already has a job in flight.  *ticket names the
 * job. */
ccpr_status ccpr_engine_submit(ccpr_engine* e, ccpr_solver* s, int nsteps, uint64_t* ticket);

/* Current state of a job (CCPR_JOB_*); CCPR_EINVAL for an unknown ticket. */
ccpr_status ccpr_engine_poll(ccpr_engine* e, uint64_t ticket, int* state);

/* Block until the job is DONE or FAILED; *state (may be NULL) receives it. */
ccpr_status ccpr_engine_wait(ccpr_engine* e, uint64_t ticket, int* state);

/* Results of a DONE job: the objective (SI), the gradient (host, design-box
 * shape, x fastest, FP64) and times[3] = {submitted, admitted to the device,
 * done} in seconds since the engine was created; any pointer may be NULL.
 * CCPR_ESTATE before DONE, CCPR_EDEVICE for a FAILED job
 * (ccpr_engine_last_error says why). */
ccpr_status ccpr_engine_result(ccpr_engine* e, uint64_t ticket, double* objective, double* grad,
                               double* times);

/* Forget a DONE or FAILED job. */
ccpr_status ccpr_engine_release(ccpr_engine* e, uint64_t ticket);

/* Batch the solves admitted from now on (on = 1, the default) or give every
 * solve its own streams (on = 0; for comparisons).  CCPR_EINVAL for NULL. */
ccpr_status ccpr_engine_set_batching(ccpr_engine* e, int on);

const char* ccpr_engine_last_error(const ccpr_engine* e);

/* Finish every queued and running job, stop the worker, free the engine. */
void ccpr_engine_destroy(ccpr_engine* e);

#ifdef __cplusplus
}
#endif
#endif
