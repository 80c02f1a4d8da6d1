// Serving engine: continuous batching of forward + adjoint + gradient solves.
//
// The caller hands over one device arena (allocated by torch in the binding)
// and submits configured solvers.  A worker thread admits queued solves in
// arrival order while the arena (first fit) and the slot limit allow and
// binds each to its own slice of the arena.  Solves that the batched launches
// can advance (ccpr_pipe_batch_class) are grouped by padded x width: the
// solves of one width share a stream and advance together, one leapfrog step
// each per batched grid / aux / post launch (up to CCPR_PIPE_BATCH_MAX solves
// per launch), so a step of many small solves costs three launches instead of
// three per solve.  Other solves get streams of their own and are fed with
// chunks of leapfrog steps, round robin, so their kernels overlap on the
// device.  A finished solve's
// objective and gradient are copied to its slot's pinned host buffers, its
// slice and streams are released, and the next queued solve is admitted.
// Pinned buffers belong to the slots and are allocated once at creation
// (grown by doubling when a larger design arrives; outgrown buffers are kept
// until the engine is destroyed), so no pinned free -- which would
// synchronise the device -- happens while solves run.  Every solve
// runs the same kernels in the same order as a solve on its own, so its
// results do not depend on what else is running.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ccprfdtd.h"
#include "ccpr_pipeline.h"

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Job {
    uint64_t ticket = 0;
    ccpr_solver* s = nullptr;
    int nsteps = 0;
    uint64_t bytes = 0;
    int state = CCPR_JOB_QUEUED;
    uint64_t off = 0;             // arena slice
    hipStream_t stream = nullptr, stream2 = nullptr;  // from the engine's pool (unbatched solves)
    int cls = -1;                 // batched solves: their class (padded x width)
    std::deque<hipEvent_t> inflight;  // one event per enqueued chunk
    bool enqueued_all = false;
    hipEvent_t done_ev = nullptr;
    int slot = -1;                // result buffers of this slot
    double* scal_host = nullptr;  // pinned [8] (the slot's)
    double* grad_host = nullptr;  // pinned [nd] (the slot's)
    long long nd = 0;
    double F = 0;
    std::vector<double> grad;
    double t_submit = 0, t_admit = 0, t_done = 0;
    std::string err;
};

struct Block {
    uint64_t off, len;
};

// Batched solves of one padded x width: one stream (from the pool) and the
// chunks of batched steps in flight on it.
struct ClassQ {
    hipStream_t stream = nullptr;
    std::vector<Job*> jobs;           // running, in admission order
    std::deque<hipEvent_t> inflight;  // one event per enqueued chunk
};

struct Slot {
    bool busy = false;
    double* scal = nullptr;   // pinned [8]
    double* grad = nullptr;   // pinned [cap]
    long long cap = 0;
};

}  // namespace

struct ccpr_engine {
    char* arena = nullptr;
    uint64_t arena_bytes = 0;
    int max_active = 4;
    int chunk = 32;
    std::vector<Block> free_list;  // sorted by offset
    std::mutex mu;
    std::condition_variable cv;   // worker wake-up and job completion
    bool stop = false;
    std::deque<Job*> queue;
    std::vector<Job*> active;
    std::map<uint64_t, Job*> jobs;
    uint64_t next_ticket = 1;
    std::vector<hipStream_t> streams;  // pool: two per slot, created once
    std::vector<Slot> slots;           // max_active result-buffer slots
    std::map<int, ClassQ> classes;     // batched solves by padded x width
    bool batching = true;              // group batchable solves (ccpr_engine_set_batching)
    std::vector<double*> retired;      // outgrown pinned buffers (freed at destroy)
    double t0 = 0;                     // creation time (job times are relative to it)
    std::thread worker;
    std::string err;
};

namespace {

constexpr uint64_t kAlign = 256;

bool arena_alloc(ccpr_engine* e, uint64_t bytes, uint64_t* off)
{
    bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
    for (size_t q = 0; q < e->free_list.size(); ++q) {
        Block& b = e->free_list[q];
        if (b.len >= bytes) {
            *off = b.off;
            b.off += bytes;
            b.len -= bytes;
            if (b.len == 0) e->free_list.erase(e->free_list.begin() + q);
            return true;
        }
    }
    return false;
}

void arena_free(ccpr_engine* e, uint64_t off, uint64_t bytes)
{
    bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
    auto it = std::lower_bound(e->free_list.begin(), e->free_list.end(), off,
                               [](const Block& b, uint64_t o) { return b.off < o; });
    it = e->free_list.insert(it, Block{off, bytes});
    // merge with the neighbours
    size_t q = it - e->free_list.begin();
    if (q + 1 < e->free_list.size() && e->free_list[q].off + e->free_list[q].len == e->free_list[q + 1].off) {
        e->free_list[q].len += e->free_list[q + 1].len;
        e->free_list.erase(e->free_list.begin() + q + 1);
    }
    if (q > 0 && e->free_list[q - 1].off + e->free_list[q - 1].len == e->free_list[q].off) {
        e->free_list[q - 1].len += e->free_list[q].len;
        e->free_list.erase(e->free_list.begin() + q);
    }
}

// A class with no solves left gives its stream back once its chunks are done.
void retire_class_if_idle(ccpr_engine* e, int cls)
{
    auto it = e->classes.find(cls);
    if (it == e->classes.end() || !it->second.jobs.empty()) return;
    ClassQ& q = it->second;
    (void)hipStreamSynchronize(q.stream);
    for (hipEvent_t ev : q.inflight) (void)hipEventDestroy(ev);
    e->streams.push_back(q.stream);
    e->classes.erase(it);
}

void release_device(ccpr_engine* e, Job* j)
{
    if (j->cls >= 0) {
        ClassQ& q = e->classes[j->cls];
        q.jobs.erase(std::remove(q.jobs.begin(), q.jobs.end(), j), q.jobs.end());
    }
    for (hipEvent_t ev : j->inflight) (void)hipEventDestroy(ev);
    j->inflight.clear();
    if (j->done_ev) (void)hipEventDestroy(j->done_ev);
    j->done_ev = nullptr;
    if (j->stream) e->streams.push_back(j->stream);
    if (j->stream2) e->streams.push_back(j->stream2);
    j->stream = j->stream2 = nullptr;
    if (j->slot >= 0) e->slots[j->slot].busy = false;
    j->slot = -1;
    j->scal_host = j->grad_host = nullptr;
    ccpr_pipe_unbind(j->s);
    arena_free(e, j->off, j->bytes);
    j->cls = -1;  // (the worker retires classes left without solves)
}

void fail_job(ccpr_engine* e, Job* j, const std::string& why)
{
    // the solve's work may still run on either of its streams (a split grid
    // pass leaves its second launch on the other one), or on its class's
    if (j->stream) (void)hipStreamSynchronize(j->stream);
    if (j->stream2) (void)hipStreamSynchronize(j->stream2);
    if (j->cls >= 0) (void)hipStreamSynchronize(e->classes[j->cls].stream);
    j->err = why;
    release_device(e, j);
    j->t_done = now_s();
    j->state = CCPR_JOB_FAILED;
}

// Admit a queued job: arena slice, stream, pinned result buffers, host set-up.
// Called by the worker with the lock held (set-up is short and synchronous on
// the job's new, idle stream).
bool admit(ccpr_engine* e, Job* j)
{
    uint64_t off;
    if (!arena_alloc(e, j->bytes, &off)) return false;
    j->off = off;
    std::string why;
    hipStream_t bind_stream = nullptr;
    const int cls = e->batching ? ccpr_pipe_batch_class(j->s) : -1;
    if (cls > 0 && (e->classes.count(cls) || !e->streams.empty())) {
        ClassQ& q = e->classes[cls];
        if (!q.stream) {
            q.stream = e->streams.back();
            e->streams.pop_back();
        }
        q.jobs.push_back(j);
        j->cls = cls;
        bind_stream = q.stream;
    } else if (e->streams.size() < 2) {
        why = "no free stream";
    } else {
        j->stream = e->streams.back();
        e->streams.pop_back();
        j->stream2 = e->streams.back();
        e->streams.pop_back();
        bind_stream = j->stream;
    }
    j->nd = ccpr_pipe_design_voxels(j->s);
    if (why.empty()) {
        for (size_t q = 0; q < e->slots.size(); ++q)
            if (!e->slots[q].busy) {
                j->slot = (int)q;
                break;
            }
        if (j->slot < 0) {
            why = "no free result slot";
        } else {
            Slot& sl = e->slots[j->slot];
            if (sl.cap < std::max(j->nd, 1LL)) {
                long long cap = std::max(sl.cap, 1LL << 16);
                while (cap < j->nd) cap *= 2;
                double* g = nullptr;
                if (hipHostMalloc((void**)&g, cap * sizeof(double), hipHostMallocDefault) != hipSuccess) {
                    why = "hipHostMalloc failed";
                } else {
                    if (sl.grad) e->retired.push_back(sl.grad);
                    sl.grad = g;
                    sl.cap = cap;
                }
            }
            if (why.empty()) {
                sl.busy = true;
                j->scal_host = sl.scal;
                j->grad_host = sl.grad;
            }
        }
    }
    if (why.empty() && j->cls < 0 && ccpr_pipe_set_stream2(j->s, j->stream2) != CCPR_OK)
        why = std::string("stream: ") + ccpr_last_error(j->s);
    if (why.empty() && ccpr_bind_workspace(j->s, e->arena + off, j->bytes, bind_stream) != CCPR_OK)
        why = std::string("bind: ") + ccpr_last_error(j->s);
    if (why.empty() && ccpr_pipe_set_batched(j->s, j->cls >= 0) != CCPR_OK)
        why = std::string("batching: ") + ccpr_last_error(j->s);
    if (why.empty() && ccpr_pipe_begin(j->s, j->nsteps) != CCPR_OK)
        why = std::string("set-up: ") + ccpr_last_error(j->s);
    j->t_admit = now_s();
    if (!why.empty()) {
        fail_job(e, j, why);
        return true;
    }
    j->state = CCPR_JOB_RUNNING;
    return true;
}

// Feed one running job: retire finished chunks, enqueue up to two chunks in
// flight, and after the last chunk the result copies.  Returns true if it did
// any work.
hipStream_t job_stream(ccpr_engine* e, Job* j) { return j->cls >= 0 ? e->classes[j->cls].stream : j->stream; }

// After the last enqueued work of a solve: its result copies and completion
// event.  Returns false (and fails the job) on error.
bool enqueue_results(ccpr_engine* e, Job* j)
{
    if (ccpr_pipe_results(j->s, j->scal_host, j->grad_host) != CCPR_OK ||
        hipEventCreateWithFlags(&j->done_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(j->done_ev, job_stream(e, j)) != hipSuccess) {
        fail_job(e, j, std::string("results: ") + ccpr_last_error(j->s));
        return false;
    }
    j->enqueued_all = true;
    return true;
}

// A solve whose completion event fired: check and copy its results.
void finish_job(ccpr_engine* e, Job* j)
{
    double F = 0;
    if (ccpr_pipe_check(j->s, j->scal_host, &F) != CCPR_OK) {
        fail_job(e, j, std::string("check: ") + ccpr_last_error(j->s));
        return;
    }
    j->F = F;
    j->grad.assign(j->grad_host, j->grad_host + j->nd);
    release_device(e, j);
    j->t_done = now_s();
    j->state = CCPR_JOB_DONE;
}

// Feed the batched solves of one class: retire finished chunks and solves,
// and keep up to two chunks of batched steps in flight.  Each round of a
// chunk advances every solve of the class by one leapfrog step (after the
// other work that precedes that step) and launches the recorded steps
// together.  Returns true if it did any work.
bool feed_class(ccpr_engine* e, ClassQ& q)
{
    bool worked = false;
    while (!q.inflight.empty() && hipEventQuery(q.inflight.front()) == hipSuccess) {
        (void)hipEventDestroy(q.inflight.front());
        q.inflight.pop_front();
        worked = true;
    }
    std::vector<Job*> done;
    for (Job* j : q.jobs)
        if (j->enqueued_all && hipEventQuery(j->done_ev) == hipSuccess) done.push_back(j);
    for (Job* j : done) {
        finish_job(e, j);
        worked = true;
    }
    if (q.inflight.size() >= 2) return worked;
    bool any = false;
    for (int r = 0; r < e->chunk; ++r) {
        std::vector<ccpr_solver*> rec;
        std::vector<Job*> failed;
        const std::vector<Job*> jobs = q.jobs;  // (failures remove jobs from q.jobs)
        for (Job* j : jobs) {
            if (j->enqueued_all || j->state != CCPR_JOB_RUNNING) continue;
            const int n = ccpr_pipe_advance(j->s, 1);
            if (n < 0) failed.push_back(j);
            else if (n == 0) enqueue_results(e, j);
            else rec.push_back(j->s);
        }
        for (Job* j : failed) fail_job(e, j, std::string("step: ") + ccpr_last_error(j->s));
        if (rec.empty()) break;
        any = true;
        for (size_t b = 0; b < rec.size(); b += CCPR_PIPE_BATCH_MAX) {
            const int k = (int)std::min<size_t>(CCPR_PIPE_BATCH_MAX, rec.size() - b);
            if (ccpr_pipe_flush(rec.data() + b, k, q.stream) != CCPR_OK) {
                for (Job* j : std::vector<Job*>(q.jobs))
                    for (int c = 0; c < k; ++c)
                        if (j->s == rec[b + c]) fail_job(e, j, std::string("batched step: ") + ccpr_last_error(j->s));
            }
        }
    }
    if (any) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
            if (hipEventRecord(ev, q.stream) == hipSuccess) q.inflight.push_back(ev);
            else (void)hipEventDestroy(ev);
        }
        worked = true;
    }
    return worked;
}

bool feed(ccpr_engine* e, Job* j)
{
    bool worked = false;
    while (!j->inflight.empty() && hipEventQuery(j->inflight.front()) == hipSuccess) {
        (void)hipEventDestroy(j->inflight.front());
        j->inflight.pop_front();
        worked = true;
    }
    while (!j->enqueued_all && j->inflight.size() < 2) {
        const int n = ccpr_pipe_advance(j->s, e->chunk);
        if (n < 0) {
            fail_job(e, j, std::string("step: ") + ccpr_last_error(j->s));
            return true;
        }
        if (n == 0) {
            enqueue_results(e, j);
            worked = true;
            break;
        }
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(ev, j->stream) != hipSuccess) {
            fail_job(e, j, "hipEventRecord failed");
            return true;
        }
        j->inflight.push_back(ev);
        worked = true;
    }
    if (j->state == CCPR_JOB_RUNNING && j->enqueued_all && hipEventQuery(j->done_ev) == hipSuccess) {
        finish_job(e, j);
        worked = true;
    }
    return worked;
}

void worker_loop(ccpr_engine* e)
{
    std::unique_lock<std::mutex> lk(e->mu);
    while (true) {
        if (e->stop && e->queue.empty() && e->active.empty()) break;
        // admission in arrival order while slots and arena allow
        while (!e->queue.empty() && (int)e->active.size() < e->max_active) {
            Job* j = e->queue.front();
            if (!admit(e, j)) break;
            e->queue.pop_front();
            if (j->state == CCPR_JOB_RUNNING) e->active.push_back(j);
            else e->cv.notify_all();
        }
        bool worked = false;
        std::vector<int> cls;
        for (auto& kv : e->classes) cls.push_back(kv.first);
        for (int c : cls) worked |= feed_class(e, e->classes[c]);
        for (int c : cls) retire_class_if_idle(e, c);
        for (size_t q = 0; q < e->active.size();) {
            Job* j = e->active[q];
            if (j->cls < 0 && j->state == CCPR_JOB_RUNNING) worked |= feed(e, j);
            if (j->state == CCPR_JOB_DONE || j->state == CCPR_JOB_FAILED) {
                e->active.erase(e->active.begin() + q);
                e->cv.notify_all();
            } else {
                ++q;
            }
        }
        if (!worked) {
            // nothing retired or enqueued: let the device progress
            e->cv.wait_for(lk, std::chrono::microseconds(50));
        }
    }
}

}  // namespace

extern "C" {

ccpr_status ccpr_engine_create(void* arena, uint64_t arena_bytes, int max_active, int chunk_steps,
                               ccpr_engine** out)
{
    if (!out) return CCPR_EINVAL;
    *out = nullptr;
    if (!arena || ((uintptr_t)arena & 255) || arena_bytes < kAlign || max_active < 1 || max_active > 64 ||
        chunk_steps < 1)
        return CCPR_EINVAL;
    ccpr_engine* e = new ccpr_engine();
    e->arena = (char*)arena;
    e->arena_bytes = arena_bytes & ~(kAlign - 1);
    e->max_active = max_active;
    e->chunk = chunk_steps;
    e->free_list.push_back(Block{0, e->arena_bytes});
    bool ok = true;
    for (int q = 0; q < 2 * max_active && ok; ++q) {
        hipStream_t st;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (ok) e->streams.push_back(st);
    }
    e->slots.resize(max_active);
    for (Slot& sl : e->slots) {
        if (!ok) break;
        sl.cap = 1 << 16;
        ok = hipHostMalloc((void**)&sl.scal, 8 * sizeof(double), hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&sl.grad, sl.cap * sizeof(double), hipHostMallocDefault) == hipSuccess;
    }
    if (!ok) {
        for (hipStream_t x : e->streams) (void)hipStreamDestroy(x);
        for (Slot& sl : e->slots) {
            if (sl.scal) (void)hipHostFree(sl.scal);
            if (sl.grad) (void)hipHostFree(sl.grad);
        }
        delete e;
        return CCPR_EDEVICE;
    }
    e->t0 = now_s();
    e->worker = std::thread(worker_loop, e);
    *out = e;
    return CCPR_OK;
}

ccpr_status ccpr_engine_submit(ccpr_engine* e, ccpr_solver* s, int nsteps, uint64_t* ticket)
{
    if (!e || !s || !ticket || nsteps < 1) return CCPR_EINVAL;
    uint64_t bytes = 0;
    ccpr_status st = ccpr_workspace_size(s, nsteps, &bytes);
    if (st) return st;
    std::lock_guard<std::mutex> lk(e->mu);
    if (e->stop) return CCPR_ESTATE;
    if (((bytes + kAlign - 1) & ~(kAlign - 1)) > e->arena_bytes) {
        e->err = "the solve's workspace exceeds the engine's arena";
        return CCPR_ENOMEM;
    }
    for (auto& kv : e->jobs)
        if (kv.second->s == s && (kv.second->state == CCPR_JOB_QUEUED || kv.second->state == CCPR_JOB_RUNNING)) {
            e->err = "this solver already has a job in flight";
            return CCPR_ESTATE;
        }
    Job* j = new Job();
    j->ticket = e->next_ticket++;
    j->s = s;
    j->nsteps = nsteps;
    j->bytes = bytes;
    j->t_submit = now_s();
    e->jobs[j->ticket] = j;
    e->queue.push_back(j);
    *ticket = j->ticket;
    e->cv.notify_all();
    return CCPR_OK;
}

ccpr_status ccpr_engine_poll(ccpr_engine* e, uint64_t ticket, int* state)
{
    if (!e || !state) return CCPR_EINVAL;
    std::lock_guard<std::mutex> lk(e->mu);
    auto it = e->jobs.find(ticket);
    if (it == e->jobs.end()) return CCPR_EINVAL;
    *state = it->second->state;
    return CCPR_OK;
}

ccpr_status ccpr_engine_wait(ccpr_engine* e, uint64_t ticket, int* state)
{
    if (!e) return CCPR_EINVAL;
    std::unique_lock<std::mutex> lk(e->mu);
    auto it = e->jobs.find(ticket);
    if (it == e->jobs.end()) return CCPR_EINVAL;
    Job* j = it->second;
    e->cv.wait(lk, [&] { return j->state == CCPR_JOB_DONE || j->state == CCPR_JOB_FAILED; });
    if (state) *state = j->state;
    return CCPR_OK;
}

ccpr_status ccpr_engine_result(ccpr_engine* e, uint64_t ticket, double* objective, double* grad,
                               double* times)
{
    if (!e) return CCPR_EINVAL;
    std::lock_guard<std::mutex> lk(e->mu);
    auto it = e->jobs.find(ticket);
    if (it == e->jobs.end()) return CCPR_EINVAL;
    Job* j = it->second;
    if (j->state == CCPR_JOB_FAILED) {
        e->err = j->err;
        return CCPR_EDEVICE;
    }
    if (j->state != CCPR_JOB_DONE) return CCPR_ESTATE;
    if (objective) *objective = j->F;
    if (grad) std::memcpy(grad, j->grad.data(), j->grad.size() * sizeof(double));
    if (times) {
        times[0] = j->t_submit - e->t0;
        times[1] = j->t_admit - e->t0;
        times[2] = j->t_done - e->t0;
    }
    return CCPR_OK;
}

ccpr_status ccpr_engine_release(ccpr_engine* e, uint64_t ticket)
{
    if (!e) return CCPR_EINVAL;
    std::lock_guard<std::mutex> lk(e->mu);
    auto it = e->jobs.find(ticket);
    if (it == e->jobs.end()) return CCPR_EINVAL;
    if (it->second->state != CCPR_JOB_DONE && it->second->state != CCPR_JOB_FAILED) return CCPR_ESTATE;
    delete it->second;
    e->jobs.erase(it);
    return CCPR_OK;
}

ccpr_status ccpr_engine_set_batching(ccpr_engine* e, int on)
{
    if (!e) return CCPR_EINVAL;
    std::lock_guard<std::mutex> lk(e->mu);
    e->batching = on != 0;
    return CCPR_OK;
}

const char* ccpr_engine_last_error(const ccpr_engine* e) { return e ? e->err.c_str() : ""; }

void ccpr_engine_destroy(ccpr_engine* e)
{
    if (!e) return;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        e->stop = true;
        e->cv.notify_all();
    }
    e->worker.join();
    for (auto& kv : e->jobs) delete kv.second;
    for (hipStream_t st : e->streams) (void)hipStreamDestroy(st);
    for (Slot& sl : e->slots) {
        if (sl.scal) (void)hipHostFree(sl.scal);
        if (sl.grad) (void)hipHostFree(sl.grad);
    }
    for (double* p : e->retired) (void)hipHostFree(p);
    delete e;
}

}  // extern "C"
