// Resumable solve: the forward run, the objective, the adjoint run (with
// segment recompute) and the gradient read-out of one solver, enqueued a few
// leapfrog steps at a time on the solver's bound stream.  Used by the serving
// engine (ccpr_engine.cpp) to interleave many solves; the results are the
// same as ccpr_forward + ccpr_adjoint + ccpr_gradient (same kernels, same
// order).
#pragma once

#include <stdint.h>

#include "../../include/ccprfdtd.h"

// Host set-up for a solve of nsteps (layout, tables, zeroed state).  The
// solver must be bound and its stream idle; synchronises that stream.
ccpr_status ccpr_pipe_begin(ccpr_solver* s, int nsteps);

// Enqueue up to max_steps more leapfrog steps (forward, then the objective,
// then the adjoint); returns how many were enqueued (0 once everything is),
// or a negative ccpr_status on error.
int ccpr_pipe_advance(ccpr_solver* s, int max_steps);

// Enqueue the copies of the SI results: scal[0..7] (scal[4] = F) and the
// gradient (nd doubles) into pinned host buffers.
ccpr_status ccpr_pipe_results(ccpr_solver* s, double* scal_host, double* grad_host);

// Check the copied scal[] of a finished solve; returns the objective in *F.
ccpr_status ccpr_pipe_check(ccpr_solver* s, const double* scal_host, double* F);

long long ccpr_pipe_design_voxels(const ccpr_solver* s);

// Forget the bound workspace (the engine reuses its memory).
void ccpr_pipe_unbind(ccpr_solver* s);

// Second stream for the solver's concurrent grid launches (owned by the
// caller, default priority); must be set before ccpr_pipe_begin.
ccpr_status ccpr_pipe_set_stream2(ccpr_solver* s, void* stream2);

#define CCPR_PIPE_BATCH_MAX 8  // solves per batched launch

// Batched serving.  ccpr_pipe_batch_class: the padded x width of a solve that
// the batched launches can advance (solves of one width are batched
// together), or -1 (per-edge designs, DFT-mode gradients, 4 rows per thread).
int ccpr_pipe_batch_class(const ccpr_solver* s);

// Switch recording on (before ccpr_pipe_begin, with every solve of a batch
// bound to one stream): ccpr_pipe_advance(s, 1) then records its leapfrog
// step (work before it, such as checkpoints, is enqueued at once) instead of
// launching it.  CCPR_ENOTSUP if ccpr_pipe_batch_class is -1.
ccpr_status ccpr_pipe_set_batched(ccpr_solver* s, int on);

// Launch the steps recorded by ss[0..k) (at most CCPR_BATCH_MAX of them, of
// one padded x width) as one batched grid, aux and post launch on stream, then
// their watchdog checks; the solves' results are the same as unbatched.
ccpr_status ccpr_pipe_flush(ccpr_solver* const* ss, int k, void* stream);
