// Executor for many operator applications in flight at once (the serving path).
//
// An executor owns a few slots, each with its own HIP stream.  Starting an
// operation on a slot enqueues all of it at once: the initial state (direct
// launches), then the time loop as replays of a captured graph of K steps,
// then the final extraction.  With a replay limit (el_exec_set_ahead) only that
// many replays are in flight per slot; el_exec_poll / el_exec_pump / el_exec_wait
// enqueue the next ones as earlier ones complete, so a slot's stream never holds
// more than that much queued work ahead of other streams sharing its hardware
// queue.  The trace row of each step comes from a device
// counter that the step's own kernels advance, so the same K-step graph is
// valid for every chunk.  Operations on different slots run concurrently on the
// device; the host only polls completion events, so it is free to build the
// next plans while the GPU works.  Results are identical to el_forward /
// el_adjoint on the same plan: the same kernels run in the same order.
#include <string>

#include "el_impl.h"

namespace {

struct ExecSlot {
    bool busy = false;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t ready = nullptr;   // inputs written: recorded on the caller's stream
    el_plan plan = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    // what is left of the operation to enqueue (replay limit)
    int op = EL_OP_FORWARD;
    const void *in = nullptr;
    void *out = nullptr;
    int full_left = 0;            // K-step replays not yet enqueued
    bool rem_left = false;        // the remainder replay not yet enqueued
    bool tail_done = true;        // the final work and completion events are enqueued
    std::vector<hipEvent_t> ring; // one event after each replay in flight (ahead > 0)
    int head = 0, count = 0;
};

}  // namespace

struct el_exec_ {
    int device = 0;
    int chunk = 64;
    int ahead = 0;                // replays in flight per slot; 0 = all at once
    std::vector<ExecSlot> slots;
};

using namespace el;

namespace {

el_status hipf(hipError_t e, const char *what) {
    return el::set_error(EL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define EX_TRY(expr, what)                          \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return hipf(e_, what); \
    } while (0)

// One time step with the trace row taken from the device counter: the forward velocity pass
// gathers row *ctr (the stresses of the previous step) in extra blocks and the stress pass
// advances the counter; the adjoint velocity pass steps it back and the adjoint stress pass
// adds Theta^T y of that row.
template <typename T>
hipError_t launch_step(el_plan p, const Dev<T> &d, int op, void *traces, int *ctr, hipStream_t s) {
    hipError_t e;
    const Relax<T> &rx = plan_relax<T>(p);
    if (op == EL_OP_FORWARD) {
        e = launch_velocity(d, p->tiles, s, &p->rec, static_cast<double *>(traces), nullptr, ctr);
        if (e == hipSuccess) e = launch_relax(d, p->tiles, rx, false, s);
        if (e == hipSuccess) e = launch_stress(d, p->tiles, s, ctr);
    } else {
        e = launch_adj_velocity(d, p->tiles, s, ctr);
        if (e == hipSuccess) e = launch_relax(d, p->tiles, rx, true, s);
        if (e == hipSuccess) e = launch_adj_stress(d, p->tiles, s, &p->rec, static_cast<const double *>(traces), ctr);
    }
    return e;
}

template <typename T>
el_status capture(el_plan p, const Dev<T> &d, int op, int steps, void *traces, int *ctr, hipStream_t s,
                  hipGraphExec_t *out) {
    hipGraph_t g = nullptr;
    EX_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t e = hipSuccess;
    for (int m = 0; m < steps && e == hipSuccess; ++m) e = launch_step(p, d, op, traces, ctr, s);
    const hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (e2 == hipSuccess && g) (void)hipGraphDestroy(g);
        return hipf(e != hipSuccess ? e : e2, "capture of the step graph");
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    EX_TRY(e, "instantiate the step graph");
    return EL_OK;
}

// Enqueue the slot's remaining replays, at most ex->ahead of them in flight (all when
// ahead = 0), then, once every replay is enqueued, the final work and completion events.
template <typename T>
el_status feed(el_exec ex, ExecSlot &sl, const Dev<T> &d) {
    if (sl.tail_done) return EL_OK;
    el_plan p = sl.plan;
    const hipStream_t s = sl.stream;
    const int M = p->g.nsteps, L = p->nrec;
    const int cap = ex->ahead;
    while (cap > 0 && sl.count > 0 && hipEventQuery(sl.ring[sl.head]) == hipSuccess) {
        sl.head = (sl.head + 1) % cap;
        --sl.count;
    }
    while ((sl.full_left > 0 || sl.rem_left) && (cap == 0 || sl.count < cap)) {
        const bool full = sl.full_left > 0;
        EX_TRY(hipGraphLaunch(sl.graph[full ? 0 : 1], s), "graph launch");
        if (full)
            --sl.full_left;
        else
            sl.rem_left = false;
        if (cap > 0) {
            EX_TRY(hipEventRecord(sl.ring[(sl.head + sl.count) % cap], s), "record replay end");
            ++sl.count;
        }
    }
    if (sl.full_left > 0 || sl.rem_left) return EL_OK;
    if (sl.op == EL_OP_FORWARD)
        EX_TRY(launch_gather(d, p->rec, static_cast<double *>(sl.out) + (size_t)(M - 1) * L, s), "gather");
    if (p->fluid_path && p->fast_tiles > 0) EX_TRY(launch_fluid_fill(d, p->tiles, s), "fluid fill");
    if (sl.op == EL_OP_ADJOINT) EX_TRY(launch_extract(d, static_cast<T *>(sl.out), s), "extract");
    EX_TRY(hipEventRecord(p->done, s), "record plan completion");
    EX_TRY(hipEventRecord(sl.done, s), "record slot completion");
    sl.tail_done = true;
    return EL_OK;
}

el_status feed_slot(el_exec ex, ExecSlot &sl) {
    if (!sl.busy || sl.tail_done) return EL_OK;
    return sl.plan->g.precision == EL_F64 ? feed(ex, sl, sl.plan->dd) : feed(ex, sl, sl.plan->df);
}

template <typename T>
el_status start_op(el_exec ex, ExecSlot &sl, el_plan p, const Dev<T> &d, int op, const void *in, void *out,
                   hipStream_t after) {
    const hipStream_t s = sl.stream;
    const int M = p->g.nsteps, L = p->nrec;
    int *ctr = reinterpret_cast<int *>(p->ws + p->L.counter);
    void *traces = op == EL_OP_FORWARD ? out : const_cast<void *>(in);
    // the caller's stream may still be writing the input (or using the output)
    EX_TRY(hipEventRecord(sl.ready, after), "record the caller's stream");
    EX_TRY(hipStreamWaitEvent(s, sl.ready, 0), "order after the caller's stream");
    EX_TRY(hipStreamWaitEvent(s, p->done, 0), "order after the plan's previous operation");
    EX_TRY(launch_zero_state(d, s), "zero state");
    EX_TRY(launch_relax_zero(p->tiles, plan_relax<T>(p), s), "relaxation state");
    if (op == EL_OP_FORWARD) {
        EX_TRY(launch_inject(d, static_cast<const T *>(in), s), "inject");
        EX_TRY(launch_set_counter(ctr, 0, s), "counter");
    } else {
        EX_TRY(launch_scatter(d, p->rec, static_cast<const double *>(in) + (size_t)(M - 1) * L, s), "scatter");
        EX_TRY(launch_set_counter(ctr, M - 1, s), "counter");
    }
    const int nupd = M - 1;
    const int K = nupd < ex->chunk ? nupd : ex->chunk;
    const int nfull = K > 0 ? nupd / K : 0;
    const int rem = nupd - nfull * K;
    if (K > 0) {
        el_status st = capture(p, d, op, K, traces, ctr, s, &sl.graph[0]);
        if (st != EL_OK) return st;
    }
    if (rem > 0) {
        el_status st = capture(p, d, op, rem, traces, ctr, s, &sl.graph[1]);
        if (st != EL_OK) return st;
    }
    sl.op = op;
    sl.in = in;
    sl.out = out;
    sl.full_left = nfull;
    sl.rem_left = rem > 0;
    sl.tail_done = false;
    sl.head = sl.count = 0;
    return feed<T>(ex, sl, d);
}

void release(ExecSlot &sl) {
    for (auto &g : sl.graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    sl.plan = nullptr;
    sl.busy = false;
    sl.tail_done = true;
    sl.full_left = 0;
    sl.rem_left = false;
    sl.head = sl.count = 0;
}

// Enqueue the rest of a slot's operation and wait for it.
el_status drain(el_exec ex, ExecSlot &sl) {
    while (sl.busy && !sl.tail_done) {
        if (sl.count > 0) EX_TRY(hipEventSynchronize(sl.ring[sl.head]), "wait for a replay");
        el_status st = feed_slot(ex, sl);
        if (st != EL_OK) return st;
    }
    if (sl.busy) EX_TRY(hipEventSynchronize(sl.done), "wait");
    return EL_OK;
}

el_status check_exec(el_exec ex, int slot) {
    if (!ex) return el::set_error(EL_EINVAL, "executor is NULL");
    if (slot < 0 || slot >= (int)ex->slots.size())
        return el::set_error(EL_EINVAL, "slot %d outside 0..%d", slot, (int)ex->slots.size() - 1);
    int dev = -1;
    EX_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != ex->device) return el::set_error(EL_EINVAL, "current device %d is not the executor's device %d", dev, ex->device);
    return EL_OK;
}

}  // namespace

extern "C" {

el_status el_exec_create(el_exec *out, int32_t max_slots, int32_t chunk_steps) {
    if (!out) return el::set_error(EL_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 64) return el::set_error(EL_EINVAL, "max_slots must be in 1..64");
    if (chunk_steps < 1) return el::set_error(EL_EINVAL, "chunk_steps must be >= 1");
    el_exec ex = new el_exec_();
    ex->chunk = chunk_steps;
    hipError_t e = hipGetDevice(&ex->device);
    ex->slots.resize(max_slots);
    for (auto &sl : ex->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ready, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        el_exec_destroy(ex);
        return hipf(e, "executor set-up");
    }
    *out = ex;
    return EL_OK;
}

el_status el_exec_destroy(el_exec ex) {
    if (!ex) return EL_OK;
    for (auto &sl : ex->slots) {
        if (sl.busy) (void)drain(ex, sl);
        release(sl);
        for (auto &e : sl.ring) (void)hipEventDestroy(e);
        sl.ring.clear();
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.ready) (void)hipEventDestroy(sl.ready);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete ex;
    return EL_OK;
}

el_status el_exec_start(el_exec ex, el_plan plan, int32_t op, const void *in, void *out, void *stream,
                        int32_t *slot) {
    if (!ex || !plan || !slot) return el::set_error(EL_EINVAL, "executor, plan or slot is NULL");
    *slot = -1;
    if (op != EL_OP_FORWARD && op != EL_OP_ADJOINT) return el::set_error(EL_EINVAL, "op must be EL_OP_FORWARD or EL_OP_ADJOINT");
    if (!in || !out) {
        if (!(plan->nrec == 0 && ((op == EL_OP_FORWARD && in) || (op == EL_OP_ADJOINT && out))))
            return el::set_error(EL_EINVAL, "in or out is NULL");
    }
    if (plan->device != ex->device) return el::set_error(EL_EINVAL, "plan and executor are on different devices");
    int k = -1;
    for (int q = 0; q < (int)ex->slots.size(); ++q)
        if (!ex->slots[q].busy) {
            k = q;
            break;
        }
    if (k < 0) return el::set_error(EL_EBUSY, "all %d executor slots are busy", (int)ex->slots.size());
    el_status st = check_exec(ex, k);
    if (st != EL_OK) return st;
    ExecSlot &sl = ex->slots[k];
    sl.plan = plan;
    const hipStream_t after = reinterpret_cast<hipStream_t>(stream);
    st = plan->g.precision == EL_F64 ? start_op(ex, sl, plan, plan->dd, op, in, out, after)
                                     : start_op(ex, sl, plan, plan->df, op, in, out, after);
    if (st != EL_OK) {
        (void)hipStreamSynchronize(sl.stream);
        release(sl);
        return st;
    }
    sl.busy = true;
    *slot = k;
    return EL_OK;
}

el_status el_exec_poll(el_exec ex, int32_t slot, int32_t *done) {
    el_status st = check_exec(ex, slot);
    if (st != EL_OK) return st;
    if (!done) return el::set_error(EL_EINVAL, "done is NULL");
    ExecSlot &sl = ex->slots[slot];
    if (!sl.busy) {
        *done = 1;
        return EL_OK;
    }
    st = feed_slot(ex, sl);
    if (st != EL_OK) return st;
    if (!sl.tail_done) {
        *done = 0;
        return EL_OK;
    }
    const hipError_t e = hipEventQuery(sl.done);
    if (e == hipErrorNotReady) {
        *done = 0;
        return EL_OK;
    }
    if (e != hipSuccess) return hipf(e, "poll");
    release(sl);
    *done = 1;
    return EL_OK;
}

el_status el_exec_wait(el_exec ex, int32_t slot) {
    el_status st = check_exec(ex, slot);
    if (st != EL_OK) return st;
    ExecSlot &sl = ex->slots[slot];
    if (!sl.busy) return EL_OK;
    st = drain(ex, sl);
    if (st != EL_OK) return st;
    release(sl);
    return EL_OK;
}

el_status el_exec_pump(el_exec ex) {
    if (!ex) return el::set_error(EL_EINVAL, "executor is NULL");
    for (int q = 0; q < (int)ex->slots.size(); ++q) {
        el_status st = check_exec(ex, q);
        if (st != EL_OK) return st;
        st = feed_slot(ex, ex->slots[q]);
        if (st != EL_OK) return st;
    }
    return EL_OK;
}

el_status el_exec_set_ahead(el_exec ex, int32_t replays) {
    if (!ex) return el::set_error(EL_EINVAL, "executor is NULL");
    if (replays < 0 || replays > 1024) return el::set_error(EL_EINVAL, "replays must be in 0..1024");
    for (auto &sl : ex->slots)
        if (sl.busy) return el::set_error(EL_EBUSY, "a slot is running an operation");
    // no limit until every slot has its events (a failure leaves the executor unlimited)
    ex->ahead = 0;
    for (auto &sl : ex->slots) {
        for (auto &e : sl.ring) (void)hipEventDestroy(e);
        sl.ring.clear();
        sl.head = sl.count = 0;
    }
    for (auto &sl : ex->slots) {
        for (int n = 0; n < replays; ++n) {
            hipEvent_t e = nullptr;
            EX_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming), "replay events");
            sl.ring.push_back(e);
        }
    }
    ex->ahead = replays;
    return EL_OK;
}

el_status el_exec_slots(el_exec ex, int32_t *total, int32_t *busy) {
    if (!ex) return el::set_error(EL_EINVAL, "executor is NULL");
    int b = 0;
    for (auto &sl : ex->slots) b += sl.busy ? 1 : 0;
    if (total) *total = (int32_t)ex->slots.size();
    if (busy) *busy = b;
    return EL_OK;
}

}  // extern "C"
