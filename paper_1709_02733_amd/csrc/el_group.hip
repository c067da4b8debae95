// Grouped time stepping of many operator applications (the serving path's batching).
//
// A group holds up to max_members operations (H p0 or H^T y), each on its own plan: grids,
// media, step counts and receiver sets may all differ, only the precision is the group's.
// el_group_run advances every running member by one time step per tick with ONE launch per
// sub-update for up to kGroupMax members at a time (the blocks of each member's tiles side by
// side in the grid), so small grids share the device instead of each filling a fraction of
// it.  Members join (el_group_add) and leave (last step, el_group_remove) between ticks: the
// launch arguments are rebuilt for each tick from the running members, nothing is captured.
// A member runs the same kernels on the same cells in the same order as el_forward /
// el_adjoint on its plan, so its result is bitwise that of the direct call.
#include <climits>
#include <string>

#include "el_impl.h"

using namespace el;

namespace {

struct Member {
    bool used = false;      // the slot holds an operation (running, or its last work in flight)
    bool running = false;   // takes part in the coming ticks
    bool withdrawn = false;
    el_plan plan = nullptr;
    int op = EL_OP_FORWARD;
    const void *in = nullptr;
    void *out = nullptr;
    int steps = 0;          // updates enqueued
    int total = 0;          // updates of the operation: nsteps - 1
    hipEvent_t done = nullptr;
};

}  // namespace

struct el_group_ {
    int device = 0;
    int precision = EL_F32;
    hipStream_t stream = nullptr;
    hipEvent_t ready = nullptr;            // caller's stream at el_group_add
    std::vector<Member> m;
    std::vector<hipEvent_t> runs;          // end of each el_group_run still tracked (el_group_sync)
};

namespace {

el_status hipf(hipError_t e, const char *what) {
    return el::set_error(EL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define GR_TRY(expr, what)                           \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hipf(e_, what); \
    } while (0)

template <typename T> Dev<T> &plan_dev(el_plan p);
template <> Dev<float> &plan_dev<float>(el_plan p) { return p->df; }
template <> Dev<double> &plan_dev<double>(el_plan p) { return p->dd; }

el_status check_group(el_group g) {
    if (!g) return el::set_error(EL_EINVAL, "group is NULL");
    int dev = -1;
    GR_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != g->device) return el::set_error(EL_EINVAL, "current device %d is not the group's device %d", dev, g->device);
    return EL_OK;
}

el_status check_slot(el_group g, int slot) {
    el_status st = check_group(g);
    if (st != EL_OK) return st;
    if (slot < 0 || slot >= (int)g->m.size()) return el::set_error(EL_EINVAL, "slot %d outside 0..%d", slot, (int)g->m.size() - 1);
    return EL_OK;
}

// The operation's last work (after its final update) and its completion events.
template <typename T>
el_status finish(el_group g, Member &mb) {
    el_plan p = mb.plan;
    const Dev<T> &d = plan_dev<T>(p);
    const hipStream_t s = g->stream;
    if (!mb.withdrawn) {
        if (mb.op == EL_OP_FORWARD && p->nrec > 0)
            GR_TRY(launch_gather(d, p->rec, static_cast<double *>(mb.out) + (size_t)mb.total * p->nrec, s), "gather");
        if (p->fluid_path && p->fast_tiles > 0) GR_TRY(launch_fluid_fill(d, p->tiles, s), "fluid fill");
        if (mb.op == EL_OP_ADJOINT) GR_TRY(launch_extract(d, static_cast<T *>(mb.out), s), "extract");
    }
    GR_TRY(hipEventRecord(p->done, s), "record plan completion");
    GR_TRY(hipEventRecord(mb.done, s), "record member completion");
    mb.running = false;
    return EL_OK;
}

template <typename T>
el_status start(el_group g, Member &mb) {
    el_plan p = mb.plan;
    const Dev<T> &d = plan_dev<T>(p);
    const hipStream_t s = g->stream;
    const int M = p->g.nsteps, L = p->nrec;
    GR_TRY(launch_zero_state(d, s), "zero state");
    GR_TRY(launch_relax_zero(p->tiles, plan_relax<T>(p), s), "relaxation state");
    if (mb.op == EL_OP_FORWARD)
        GR_TRY(launch_inject(d, static_cast<const T *>(mb.in), s), "inject");
    else
        GR_TRY(launch_scatter(d, p->rec, static_cast<const double *>(mb.in) + (size_t)(M - 1) * L, s), "scatter");
    mb.running = true;
    if (mb.total == 0) return finish<T>(g, mb);
    return EL_OK;
}

// Member lists of one tick, in slot order, for the grouped launches of one direction.
struct Batch {
    int n = 0;
    Member *mb[kGroupMax];
};

// One grouped launch of `pass` over the members of b (pass 0 gathers the forward trace row of
// the step each member is about to take; pass 3 adds Theta^T y of the adjoint row).
template <typename T>
el_status grouped(el_group g, const Batch &b, int pass) {
    Grp<T, kGroupMax> gp{};
    int blocks = 0;
    for (int q = 0; q < b.n; ++q) {
        Member &mb = *b.mb[q];
        el_plan p = mb.plan;
        const int L = p->nrec, M = p->g.nsteps;
        gp.d[q] = plan_dev<T>(p);
        gp.tl[q] = p->tiles;
        gp.r[q] = Rec{};
        gp.row[q] = nullptr;
        gp.first[q] = blocks;
        blocks += 8 * p->tiles.per;
        if (pass == 0 && L > 0) {
            // forward update k is m = k+1; its velocity pass gathers row m-1 = k
            gp.r[q] = p->rec;
            gp.row[q] = static_cast<double *>(mb.out) + (size_t)mb.steps * L;
            blocks += gather_blocks(L);
        }
        if (pass == 3 && p->rec.npts > 0) {
            // adjoint update k is m = M-1-k; its stress pass adds Theta^T y of row m-1
            gp.r[q] = p->rec;
            gp.row[q] = const_cast<double *>(static_cast<const double *>(mb.in)) + (size_t)(M - 2 - mb.steps) * L;
        }
        blocks = (blocks + 7) / 8 * 8;
    }
    for (int q = b.n; q <= kGroupMax; ++q) gp.first[q] = blocks;
    gp.n = b.n;
    if (blocks == 0) return EL_OK;
    GR_TRY(launch_group_pass(gp, pass, g->stream), "grouped launch");
    return EL_OK;
}

template <typename T>
el_status tick(el_group g) {
    std::vector<Batch> fwd, adj;
    for (auto &mb : g->m) {
        if (!mb.running) continue;
        std::vector<Batch> &v = mb.op == EL_OP_FORWARD ? fwd : adj;
        if (v.empty() || v.back().n == kGroupMax) v.emplace_back();
        v.back().mb[v.back().n++] = &mb;
    }
    el_status st = EL_OK;
    for (auto &b : fwd)
        if ((st = grouped<T>(g, b, 0)) != EL_OK) return st;
    for (auto &b : adj)
        if ((st = grouped<T>(g, b, 2)) != EL_OK) return st;
    for (auto &mb : g->m)
        if (mb.running) {
            const Relax<T> &rx = plan_relax<T>(mb.plan);
            GR_TRY(launch_relax(plan_dev<T>(mb.plan), mb.plan->tiles, rx, mb.op == EL_OP_ADJOINT, g->stream),
                   "relaxation");
        }
    for (auto &b : fwd)
        if ((st = grouped<T>(g, b, 1)) != EL_OK) return st;
    for (auto &b : adj)
        if ((st = grouped<T>(g, b, 3)) != EL_OK) return st;
    for (auto &mb : g->m)
        if (mb.running && ++mb.steps == mb.total)
            if ((st = finish<T>(g, mb)) != EL_OK) return st;
    return EL_OK;
}

void release(Member &mb) {
    mb.used = mb.running = mb.withdrawn = false;
    mb.plan = nullptr;
    mb.in = nullptr;
    mb.out = nullptr;
}

}  // namespace

extern "C" {

el_status el_group_create(el_group *out, int32_t max_members, int32_t precision) {
    if (!out) return el::set_error(EL_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_members < 1 || max_members > 64) return el::set_error(EL_EINVAL, "max_members must be in 1..64");
    if (precision != EL_F32 && precision != EL_F64) return el::set_error(EL_EINVAL, "precision must be EL_F32 or EL_F64");
    el_group g = new el_group_();
    g->precision = precision;
    hipError_t e = hipGetDevice(&g->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->ready, hipEventDisableTiming);
    g->m.resize(max_members);
    for (auto &mb : g->m)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&mb.done, hipEventDisableTiming);
    if (e != hipSuccess) {
        el_group_destroy(g);
        return hipf(e, "group set-up");
    }
    *out = g;
    return EL_OK;
}

el_status el_group_destroy(el_group g) {
    if (!g) return EL_OK;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    for (auto &mb : g->m)
        if (mb.done) (void)hipEventDestroy(mb.done);
    for (auto &e : g->runs) (void)hipEventDestroy(e);
    if (g->ready) (void)hipEventDestroy(g->ready);
    if (g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
    return EL_OK;
}

el_status el_group_add(el_group g, el_plan plan, int32_t op, const void *in, void *out, void *stream, int32_t *slot) {
    el_status st = check_group(g);
    if (st != EL_OK) return st;
    if (!plan || !slot) return el::set_error(EL_EINVAL, "plan or slot is NULL");
    *slot = -1;
    if (op != EL_OP_FORWARD && op != EL_OP_ADJOINT) return el::set_error(EL_EINVAL, "op must be EL_OP_FORWARD or EL_OP_ADJOINT");
    if (!in || !out) {
        if (!(plan->nrec == 0 && ((op == EL_OP_FORWARD && in) || (op == EL_OP_ADJOINT && out))))
            return el::set_error(EL_EINVAL, "in or out is NULL");
    }
    if (plan->device != g->device) return el::set_error(EL_EINVAL, "plan and group are on different devices");
    if (plan->g.precision != g->precision) return el::set_error(EL_EINVAL, "plan precision differs from the group's");
    int k = -1;
    for (int q = 0; q < (int)g->m.size(); ++q) {
        if (g->m[q].used && g->m[q].plan == plan) return el::set_error(EL_EINVAL, "plan is already a member (slot %d)", q);
        if (k < 0 && !g->m[q].used) k = q;
    }
    if (k < 0) return el::set_error(EL_EBUSY, "all %d group slots are in use", (int)g->m.size());
    // the caller's stream may still be writing the input; the plan's previous operation may run
    GR_TRY(hipEventRecord(g->ready, reinterpret_cast<hipStream_t>(stream)), "record the caller's stream");
    GR_TRY(hipStreamWaitEvent(g->stream, g->ready, 0), "order after the caller's stream");
    GR_TRY(hipStreamWaitEvent(g->stream, plan->done, 0), "order after the plan's previous operation");
    Member &mb = g->m[k];
    mb.used = true;
    mb.withdrawn = false;
    mb.plan = plan;
    mb.op = op;
    mb.in = in;
    mb.out = out;
    mb.steps = 0;
    mb.total = plan->g.nsteps - 1;
    st = g->precision == EL_F64 ? start<double>(g, mb) : start<float>(g, mb);
    if (st != EL_OK) {
        (void)hipStreamSynchronize(g->stream);
        release(mb);
        return st;
    }
    *slot = k;
    return EL_OK;
}

el_status el_group_run(el_group g, int32_t ticks) {
    el_status st = check_group(g);
    if (st != EL_OK) return st;
    if (ticks < 0) return el::set_error(EL_EINVAL, "ticks must be >= 0");
    // release the events of runs that have completed (a caller need not sync to keep the
    // list short)
    while (!g->runs.empty() && hipEventQuery(g->runs.front()) == hipSuccess) {
        (void)hipEventDestroy(g->runs.front());
        g->runs.erase(g->runs.begin());
    }
    for (int t = 0; t < ticks; ++t) {
        bool any = false;
        for (auto &mb : g->m) any = any || mb.running;
        if (!any) break;
        st = g->precision == EL_F64 ? tick<double>(g) : tick<float>(g);
        if (st != EL_OK) return st;
    }
    hipEvent_t e = nullptr;
    GR_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming), "run event");
    g->runs.push_back(e);
    GR_TRY(hipEventRecord(e, g->stream), "record run end");
    return EL_OK;
}

el_status el_group_sync(el_group g, int32_t pending) {
    el_status st = check_group(g);
    if (st != EL_OK) return st;
    if (pending < 0) return el::set_error(EL_EINVAL, "pending must be >= 0");
    if (pending == 0) {
        // everything enqueued so far (runs, joins, withdrawals) has completed
        GR_TRY(hipStreamSynchronize(g->stream), "wait for the group");
        for (auto &e : g->runs) (void)hipEventDestroy(e);
        g->runs.clear();
        return EL_OK;
    }
    while ((int)g->runs.size() > pending) {
        GR_TRY(hipEventSynchronize(g->runs.front()), "wait for a run");
        (void)hipEventDestroy(g->runs.front());
        g->runs.erase(g->runs.begin());
    }
    return EL_OK;
}

el_status el_group_poll(el_group g, int32_t slot, int32_t *steps_done, int32_t *done) {
    el_status st = check_slot(g, slot);
    if (st != EL_OK) return st;
    Member &mb = g->m[slot];
    if (steps_done) *steps_done = mb.used ? mb.steps : 0;
    if (!done) return EL_OK;
    if (!mb.used || mb.running) {
        *done = mb.used ? 0 : 1;
        return EL_OK;
    }
    const hipError_t e = hipEventQuery(mb.done);
    if (e == hipErrorNotReady) {
        *done = 0;
        return EL_OK;
    }
    if (e != hipSuccess) return hipf(e, "poll");
    release(mb);
    *done = 1;
    return EL_OK;
}

el_status el_group_remove(el_group g, int32_t slot) {
    el_status st = check_slot(g, slot);
    if (st != EL_OK) return st;
    Member &mb = g->m[slot];
    if (!mb.used || !mb.running) return EL_OK;
    mb.withdrawn = true;
    GR_TRY(hipEventRecord(mb.plan->done, g->stream), "record plan completion");
    GR_TRY(hipEventRecord(mb.done, g->stream), "record member completion");
    mb.running = false;
    return EL_OK;
}

el_status el_group_members(el_group g, int32_t *total, int32_t *used, int32_t *running) {
    if (!g) return el::set_error(EL_EINVAL, "group is NULL");
    int u = 0, r = 0;
    for (auto &mb : g->m) {
        u += mb.used ? 1 : 0;
        r += mb.running ? 1 : 0;
    }
    if (total) *total = (int32_t)g->m.size();
    if (used) *used = u;
    if (running) *running = r;
    return EL_OK;
}

}  // extern "C"
