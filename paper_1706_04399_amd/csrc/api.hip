// C ABI entry points: argument validation, state layout and launch order.
// See include/dpso.h for the contract of each call.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "dpso.h"
#include "errors.hpp"
#include "kernels.hpp"
#include "tune.hpp"

namespace dpso {

namespace {
thread_local char g_error[512] = "";
}

dpso_status fail(dpso_status code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof g_error, fmt, ap);
    va_end(ap);
    return code;
}

dpso_status ok()
{
    g_error[0] = 0;
    return DPSO_OK;
}

const char *last_error() { return g_error; }

}  // namespace dpso

using dpso::fail;
using dpso::ok;

namespace {

dpso_status hip_fail(hipError_t e, const char *what)
{
    return fail(DPSO_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

dpso_status check_params(const dpso_params *p, int32_t n)
{
    if (!p) return fail(DPSO_E_INVAL, "params is NULL");
    if (n < 1) return fail(DPSO_E_INVAL, "n = %d must be at least 1", n);
    if (n > DPSO_MAX_N) return fail(DPSO_E_RANGE, "n = %d exceeds DPSO_MAX_N = %d", n, DPSO_MAX_N);
    if (p->swarm_size < 1 || p->swarm_size > DPSO_MAX_SWARM)
        return fail(DPSO_E_INVAL, "swarm_size = %d outside 1..%d", p->swarm_size, DPSO_MAX_SWARM);
    if (p->max_generations < 0 || p->max_generations > (1 << 30))
        return fail(DPSO_E_INVAL, "max_generations = %d outside 0..2^30", p->max_generations);
    if (p->w_q16 > 131072 || p->phi1_q16 > 131072 || p->phi2_q16 > 131072)
        return fail(DPSO_E_INVAL, "coefficients must be at most 2.0 (131072 in Q16)");
    if (p->mutation_period < 0) return fail(DPSO_E_INVAL, "mutation_period must be >= 0");
    if (p->ee_trigger < DPSO_EE_OFF || p->ee_trigger > DPSO_EE_ALWAYS)
        return fail(DPSO_E_INVAL, "ee_trigger = %d is not a DPSO_EE_* value", p->ee_trigger);
    if (p->ee_max_moves < 0) return fail(DPSO_E_INVAL, "ee_max_moves must be >= 0");
    if (p->stall_limit < 0) return fail(DPSO_E_INVAL, "stall_limit must be >= 0");
    if (p->det_permille < 0 || p->det_permille > 1000)
        return fail(DPSO_E_INVAL, "det_permille = %d outside 0..1000", p->det_permille);
    if (p->ee_neighbourhood != DPSO_NB_TWO_OPT && p->ee_neighbourhood != DPSO_NB_NODE_SWAP)
        return fail(DPSO_E_INVAL, "ee_neighbourhood = %d is not a DPSO_NB_* value", p->ee_neighbourhood);
    if (p->mutation_swaps < 0 || p->mutation_swaps > 65536)
        return fail(DPSO_E_INVAL, "mutation_swaps = %d outside 0..65536", p->mutation_swaps);
    if (p->velocity_cap < 0 || p->velocity_cap > n)
        return fail(DPSO_E_INVAL, "velocity_cap = %d outside 0..n = %d", p->velocity_cap, n);
    return DPSO_OK;
}

dpso::KParams kernel_params(const dpso_params *p)
{
    dpso::KParams k{};
    k.seed = p->seed;
    k.instance = p->instance;
    k.w_q16 = p->w_q16;
    k.phi1_q16 = p->phi1_q16;
    k.phi2_q16 = p->phi2_q16;
    k.mutation_period = p->mutation_period;
    k.ee_trigger = p->ee_trigger;
    k.ee_max_moves = p->ee_max_moves;
    k.stall_limit = p->stall_limit;
    k.max_generations = p->max_generations;
    int64_t m = (int64_t(p->swarm_size) * p->det_permille + 999) / 1000;
    k.det_count = int32_t(m < p->swarm_size ? m : p->swarm_size);
    k.ee_neighbourhood = p->ee_neighbourhood;
    k.mutation_swaps = p->mutation_swaps;
    k.velocity_cap = p->velocity_cap;
    return k;
}

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

dpso::Inst make_inst(const int32_t *d_dist, void *d_state, const dpso::Layout &L, const dpso_params *params)
{
    dpso::Inst I{};
    I.D = d_dist;
    I.st = dpso::make_view(d_state, L);
    I.kp = kernel_params(params);
    I.cap = L.cap;
    return I;
}

// Reads the header of a state (synchronising the stream).
dpso_status read_header(const void *d_state, dpso::Hdr *h, hipStream_t s)
{
    if (!d_state) return fail(DPSO_E_INVAL, "state is NULL");
    HIP_TRY(hipMemcpyAsync(h, d_state, sizeof *h, hipMemcpyDeviceToHost, s), "read state header");
    HIP_TRY(hipStreamSynchronize(s), "synchronise stream");
    if (h->magic != dpso::kMagic || h->n < 1 || h->n > DPSO_MAX_N || h->S < 1 ||
        h->S > DPSO_MAX_SWARM || h->cap < 1)
        return fail(DPSO_E_STATE, "state buffer is not an initialised swarm");
    if (h->err)
        return fail(DPSO_E_STATE, "state rejected by dpso_run: it does not match n / swarm_size / velocity mode");
    return DPSO_OK;
}

// Canonical difference to - from (positions scanned left to right; a
// position holding the wrong label gets the right one by exchanging the two
// labels). Writes the label pairs to out[2 * len]; returns len.
int host_difference(const uint16_t *from, const uint16_t *to, int n, uint16_t *out,
                    std::vector<uint16_t> &cur, std::vector<uint16_t> &pos)
{
    cur.assign(from, from + n);
    pos.resize(size_t(n));
    for (int i = 0; i < n; ++i) pos[cur[i]] = uint16_t(i);
    int len = 0;
    for (int q = 0; q < n; ++q) {
        const uint16_t a = cur[q], b = to[q];
        if (a == b) continue;
        out[2 * len] = a;
        out[2 * len + 1] = b;
        ++len;
        const uint16_t j = pos[b];
        cur[q] = b;
        cur[j] = a;
        pos[b] = uint16_t(q);
        pos[a] = j;
    }
    return len;
}

// A pair of tours (from, to) whose canonical difference is the given list:
// to holds the second labels at positions 0..len-1 (then the other labels in
// increasing order) and from is to with the exchanges undone in reverse
// order. Returns false if the list is not a canonical difference.
bool host_velocity_tours(const uint16_t *pairs, int len, int n, uint16_t *from, uint16_t *to)
{
    std::vector<uint8_t> used(static_cast<size_t>(n), 0);
    for (int i = 0; i < len; ++i) {
        const uint16_t a = pairs[2 * i], b = pairs[2 * i + 1];
        if (a >= n || b >= n || a == b || used[b]) return false;
        used[b] = 1;
        to[i] = b;
    }
    int q = len;
    for (int label = 0; label < n; ++label)
        if (!used[label]) to[q++] = uint16_t(label);
    std::vector<uint16_t> pos(static_cast<size_t>(n), 0);
    for (int i = 0; i < n; ++i) {
        from[i] = to[i];
        pos[to[i]] = uint16_t(i);
    }
    for (int i = len - 1; i >= 0; --i) {
        const uint16_t a = pairs[2 * i], b = pairs[2 * i + 1];
        const uint16_t ia = pos[a], ib = pos[b];
        from[ia] = b;
        from[ib] = a;
        pos[a] = ib;
        pos[b] = ia;
    }
    std::vector<uint16_t> check(size_t(2 * n)), cur, scratch;
    return host_difference(from, to, n, check.data(), cur, scratch) == len &&
           std::equal(check.begin(), check.begin() + 2 * len, pairs);
}

// Device workspace of a batch: the descriptors of all instances with two
// prefix tables (per particle, per instance), and for every move class and
// every edge-exchange class the descriptors of its members with their
// particle prefix.
// Move classes: threads per particle 64 / 128 / 256 / 512, one launch each; in it
// every member runs at its own positions per thread (the move's mixed batch
// kernel), not at its class's largest.
constexpr int kMoveClasses = 4;

int move_class(int tpb) { return tpb == 64 ? 0 : tpb == 128 ? 1 : tpb == 512 ? 3 : 2; }

int move_class_threads(int mc) { return 64 << mc; }

struct BatchLayout {
    size_t inst, first_items, first_inst, cls_inst[dpso::kExchangeClasses], cls_first[dpso::kExchangeClasses],
        mv_inst[kMoveClasses], mv_first[kMoveClasses], total;
};

BatchLayout batch_layout(int32_t count)
{
    BatchLayout B{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = dpso::align256(o + bytes); return at; };
    B.inst = take(sizeof(dpso::Inst) * size_t(count));
    B.first_items = take(4 * size_t(count + 1));
    B.first_inst = take(4 * size_t(count + 1));
    for (int c = 0; c < dpso::kExchangeClasses; ++c) {
        B.cls_inst[c] = take(sizeof(dpso::Inst) * size_t(count));
        B.cls_first[c] = take(4 * size_t(count + 1));
    }
    for (int c = 0; c < kMoveClasses; ++c) {
        B.mv_inst[c] = take(sizeof(dpso::Inst) * size_t(count));
        B.mv_first[c] = take(4 * size_t(count + 1));
    }
    B.total = o;
    return B;
}

// A class of a batch: its members (descriptors and particle prefix) and
// the launch it needs.
struct ClassPlan {
    dpso::Batch members;
    int total = 0, max_ns = 0, grid = 0;
};

// Launch order of a class's members. DPSO_ORDER_INDEX keeps the batch's
// order. DPSO_ORDER_LPT puts the members with the most work (swarm times n^2
// for the edge exchange, times n for the move) first, so the longest blocks
// start first (longest-processing-time order). DPSO_ORDER_XCD, with 8 or more
// members, also deals them, most work first, to eight XCD groups: each to the
// group with the least work that has room for its particles (a group holds
// at most ceil(total / 8) plus the largest swarm); the grouping is kept only
// if no group's work or particle count exceeds the mean by more than an
// eighth, else the launch is ungrouped in LPT order. Groups are listed one
// after another, most work first within each.
struct ClassOrder {
    std::vector<int> order;  // member positions in launch order
    bool groups = false;
    int xcount[8] = {};      // particles of each XCD group
};

ClassOrder order_class(const std::vector<int64_t> &work, const std::vector<int64_t> &swarm, int mode)
{
    ClassOrder o;
    const size_t m = work.size();
    o.order.resize(m);
    for (size_t k = 0; k < m; ++k) o.order[k] = int(k);
    if (mode == DPSO_ORDER_INDEX || m == 0) return o;
    std::stable_sort(o.order.begin(), o.order.end(), [&](int a, int b) { return work[size_t(a)] > work[size_t(b)]; });
    if (mode != DPSO_ORDER_XCD || m < 8) return o;
    int64_t total = 0, total_work = 0, biggest = 0;
    for (size_t k = 0; k < m; ++k) {
        total += swarm[k];
        total_work += work[k];
        biggest = std::max(biggest, swarm[k]);
    }
    const int64_t cap = (total + 7) / 8 + biggest;
    std::vector<int> group[8];
    int64_t load[8] = {}, parts[8] = {};
    for (int k : o.order) {
        int best = -1;
        for (int x = 0; x < 8; ++x)
            if (parts[x] + swarm[size_t(k)] <= cap && (best < 0 || load[x] < load[best])) best = x;
        if (best < 0) return o;  // no room anywhere: ungrouped
        group[best].push_back(k);
        load[best] += work[size_t(k)];
        parts[best] += swarm[size_t(k)];
    }
    for (int x = 0; x < 8; ++x)
        if (8 * load[x] > 9 * total_work / 8 || 8 * parts[x] > 9 * total / 8) return o;
    o.order.clear();
    for (int x = 0; x < 8; ++x) {
        o.order.insert(o.order.end(), group[x].begin(), group[x].end());
        o.xcount[x] = int(parts[x]);
    }
    o.groups = true;
    return o;
}

struct BatchPlan {
    dpso::Batch items, instances;
    ClassPlan cls[dpso::kExchangeClasses], mv[kMoveClasses];
    int total = 0, max_ns = 0;
    bool mixed[dpso::kExchangeClasses] = {};  // classes holding a merge group's members, launched mixed
    bool any_mutation = false, any_exchange = false;
};

// Validates every item, writes the tables to the workspace (synchronising
// the stream) and returns the launch plan. Each instance's move and exchange
// classes follow the configuration of its n among all the batch's
// particles.
dpso_status plan_batch(const dpso_batch_item *items, int32_t count, void *d_work, size_t work_bytes,
                       hipStream_t s, BatchPlan &plan)
{
    if (!items || !d_work) return fail(DPSO_E_INVAL, "items and d_work must be non-NULL");
    if (count < 1 || count > DPSO_MAX_BATCH)
        return fail(DPSO_E_INVAL, "batch of %d instances outside 1..%d", count, DPSO_MAX_BATCH);
    const BatchLayout BL = batch_layout(count);
    if (work_bytes < BL.total) return fail(DPSO_E_NOMEM, "workspace of %zu bytes, %zu needed", work_bytes, BL.total);
    std::vector<unsigned char> host(BL.total, 0);
    auto inst = reinterpret_cast<dpso::Inst *>(host.data() + BL.inst);
    auto first_items = reinterpret_cast<int32_t *>(host.data() + BL.first_items);
    auto first_inst = reinterpret_cast<int32_t *>(host.data() + BL.first_inst);
    int64_t total = 0;
    for (int32_t i = 0; i < count; ++i) {
        const dpso_batch_item &it = items[i];
        dpso_status st = check_params(&it.params, it.n);
        if (st) {
            char why[512];
            strncpy(why, dpso::last_error(), sizeof why);
            why[sizeof why - 1] = 0;
            return fail(st, "item %d: %s", i, why);
        }
        if (!it.d_dist || !it.d_state) return fail(DPSO_E_INVAL, "item %d: d_dist and d_state must be non-NULL", i);
        const dpso::Layout L = dpso::make_layout(it.n, it.params.swarm_size, it.params.max_generations + 1);
        if (it.state_bytes < L.total)
            return fail(DPSO_E_NOMEM, "item %d: state buffer of %zu bytes, %zu needed", i, it.state_bytes, L.total);
        total += it.params.swarm_size;
    }
    if (total > (int64_t(1) << 30)) return fail(DPSO_E_RANGE, "batch holds %lld particles", (long long)total);
    std::vector<int> cls_members[dpso::kExchangeClasses], mv_members[kMoveClasses];
    int64_t run = 0;
    for (int32_t i = 0; i < count; ++i) {
        const dpso_batch_item &it = items[i];
        const dpso::Layout L = dpso::make_layout(it.n, it.params.swarm_size, it.params.max_generations + 1);
        inst[i] = make_inst(it.d_dist, it.d_state, L, &it.params);
        first_items[i] = int32_t(run);
        first_inst[i] = i;
        run += it.params.swarm_size;
        plan.max_ns = std::max(plan.max_ns, L.ns);
        plan.any_mutation |= it.params.mutation_period > 0;
        const dpso::Tune tune = dpso::tuning_for(it.n, total);
        mv_members[move_class(tune.move_threads)].push_back(i);
        if (it.params.ee_trigger != DPSO_EE_OFF) {
            plan.any_exchange = true;
            cls_members[dpso::exchange_class(it.n, it.d_dist, it.params.ee_neighbourhood, tune.exchange_rows)]
                .push_back(i);
        }
    }
    // a batch small enough merges the 16-bit row classes of each merge group
    // (one, two or four wavefronts per particle) into the group's largest (one
    // launch, each instance with its own class's code)
    for (int group = 1; group <= 3 && total <= dpso::batch_merge(); ++group) {
        int top = -1, classes = 0;
        for (int c = 0; c < dpso::kExchangeClasses; ++c)
            if (dpso::exchange_merge_group(c) == group && !cls_members[c].empty()) {
                top = c;
                ++classes;
            }
        if (classes > 1) {
            for (int c = 0; c < top; ++c)
                if (dpso::exchange_merge_group(c) == group) {
                    cls_members[top].insert(cls_members[top].end(), cls_members[c].begin(), cls_members[c].end());
                    cls_members[c].clear();
                }
            plan.mixed[top] = true;
        }
    }
    first_items[count] = int32_t(total);
    first_inst[count] = count;
    unsigned char *dev = static_cast<unsigned char *>(d_work);
    plan.total = int(total);
    plan.items = dpso::Batch{reinterpret_cast<const dpso::Inst *>(dev + BL.inst),
                             reinterpret_cast<const int32_t *>(dev + BL.first_items), count};
    plan.instances = dpso::Batch{reinterpret_cast<const dpso::Inst *>(dev + BL.inst),
                                 reinterpret_cast<const int32_t *>(dev + BL.first_inst), count};
    const int order = dpso::batch_order();
    // a class's table in launch order (see order_class), its particle prefix
    // and launch size
    auto write_class = [&](ClassPlan &cp, const std::vector<int> &members, bool quadratic, size_t inst_off,
                           size_t first_off) {
        std::vector<int64_t> work(members.size()), swarm(members.size());
        for (size_t k = 0; k < members.size(); ++k) {
            const int64_t n = items[members[k]].n;
            swarm[k] = items[members[k]].params.swarm_size;
            work[k] = swarm[k] * (quadratic ? n * n : n);
        }
        const ClassOrder o = order_class(work, swarm, order);
        auto ci = reinterpret_cast<dpso::Inst *>(host.data() + inst_off);
        auto cf = reinterpret_cast<int32_t *>(host.data() + first_off);
        int acc = 0;
        for (size_t k = 0; k < o.order.size(); ++k) {
            const int i = members[size_t(o.order[k])];
            ci[k] = inst[i];
            cf[k] = acc;
            acc += items[i].params.swarm_size;
            cp.max_ns = std::max(cp.max_ns, (items[i].n + 63) & ~63);
        }
        cf[o.order.size()] = acc;
        cp.total = acc;
        cp.members = dpso::Batch{reinterpret_cast<const dpso::Inst *>(dev + inst_off),
                                 reinterpret_cast<const int32_t *>(dev + first_off), int32_t(members.size())};
        cp.grid = acc;
        if (o.groups) {
            cp.members.groups = 8;
            int base = 0, rows = 0;
            for (int x = 0; x < 8; ++x) {
                cp.members.xbase[x] = base;
                cp.members.xcount[x] = o.xcount[x];
                base += o.xcount[x];
                rows = std::max(rows, o.xcount[x]);
            }
            cp.grid = 8 * rows;
        }
    };
    for (int c = 0; c < dpso::kExchangeClasses; ++c)
        write_class(plan.cls[c], cls_members[c], true, BL.cls_inst[c], BL.cls_first[c]);
    for (int c = 0; c < kMoveClasses; ++c)
        write_class(plan.mv[c], mv_members[c], false, BL.mv_inst[c], BL.mv_first[c]);
    HIP_TRY(hipMemcpyAsync(d_work, host.data(), host.size(), hipMemcpyHostToDevice, s), "copy batch tables");
    HIP_TRY(hipStreamSynchronize(s), "synchronise stream");
    return DPSO_OK;
}

// All launches of `generations` generations of a batch: per generation, one
// move launch per move class, the mutation, the first global best, one
// exchange launch per exchange class (the merged 16-bit row classes as one)
// and the second global best (with the end of the generation), one after
// another on `s`.
hipError_t enqueue_batch(const BatchPlan &P, int32_t generations, hipStream_t s)
{
    hipError_t e = dpso::launch_batch_check(P.items, P.instances, P.total, P.max_ns, s);
    for (int c = 0; c < dpso::kExchangeClasses && e == hipSuccess && P.any_exchange; ++c)
        e = dpso::launch_batch_2opt_prepare(c, P.cls[c].members, P.cls[c].max_ns, s);
    for (int32_t g = 0; g < generations && e == hipSuccess; ++g) {
        for (int c = 0; c < kMoveClasses && e == hipSuccess; ++c)
            if (P.mv[c].members.count > 0)
                e = dpso::launch_batch_move(move_class_threads(c), P.mv[c].members, P.mv[c].grid, P.mv[c].max_ns, s);
        if (e == hipSuccess && P.any_mutation)
            e = dpso::launch_batch_mutation(P.items, P.instances, P.total, P.max_ns, s);
        if (e == hipSuccess) e = dpso::launch_batch_gbest(P.items, P.instances, P.total, P.max_ns, 1, s);
        if (P.any_exchange) {
            for (int c = 0; c < dpso::kExchangeClasses && e == hipSuccess; ++c)
                if (P.cls[c].members.count > 0)
                    e = P.mixed[c]
                            ? dpso::launch_batch_2opt_mixed(c, P.cls[c].members, P.cls[c].grid, P.cls[c].max_ns, s)
                            : dpso::launch_batch_2opt(c, P.cls[c].members, P.cls[c].grid, P.cls[c].max_ns, s);
            if (e == hipSuccess) e = dpso::launch_batch_gbest(P.items, P.instances, P.total, P.max_ns, 3, s);
        } else if (e == hipSuccess) {
            e = dpso::launch_batch_end(P.items, P.instances, P.total, P.max_ns, s);
        }
    }
    return e;
}

// Event pool for dpso_run_profiled, reused across calls.
std::mutex g_event_mutex;
std::vector<hipEvent_t> g_events;

dpso_status events(size_t count, std::vector<hipEvent_t> &out)
{
    std::lock_guard<std::mutex> lock(g_event_mutex);
    while (g_events.size() < count) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e), "create event");
        g_events.push_back(e);
    }
    out.assign(g_events.begin(), g_events.begin() + count);
    return DPSO_OK;
}

// times: events between every phase; exchange_only: events around the
// edge-exchange launches only (their summed time into times->ms_exchange).
dpso_status run_impl(const int32_t *d_dist, int32_t n, const dpso_params *params, void *d_state,
                     size_t state_bytes, int32_t generations, void *stream, dpso_phase_times *times,
                     bool exchange_only = false, const dpso::Tune *force = nullptr)
{
    dpso_status st = check_params(params, n);
    if (st) return st;
    if (!d_dist || !d_state) return fail(DPSO_E_INVAL, "d_dist and d_state must be non-NULL");
    if (generations < 0) return fail(DPSO_E_INVAL, "generations must be >= 0");
    const dpso::Layout L = dpso::make_layout(n, params->swarm_size, params->max_generations + 1);
    if (state_bytes < L.total)
        return fail(DPSO_E_NOMEM, "state buffer of %zu bytes, %zu needed", state_bytes, L.total);
    const dpso::Inst I = make_inst(d_dist, d_state, L, params);
    const dpso::KParams &kp = I.kp;
    const dpso::Tune tune = force ? dpso::resolve_tuning(*force, n, params->swarm_size)
                                  : dpso::tuning_for(n, params->swarm_size);
    const int cls = dpso::exchange_class(n, d_dist, kp.ee_neighbourhood, tune.exchange_rows);
    hipStream_t s = as_stream(stream);
    std::vector<hipEvent_t> ev;
    constexpr int kMarks = 6;  // after move, mutation, gbest, exchange, gbest, end
    const bool all = times && !exchange_only;
    const bool ex = times && exchange_only && kp.ee_trigger != DPSO_EE_OFF;
    if (all && (st = events(size_t(generations) * kMarks + 1, ev))) return st;
    if (ex && (st = events(size_t(generations) * 2, ev))) return st;
    size_t mark = 0;
    auto stamp = [&]() -> hipError_t { return all ? hipEventRecord(ev[mark++], s) : hipSuccess; };
    auto stamp_ex = [&]() -> hipError_t { return ex ? hipEventRecord(ev[mark++], s) : hipSuccess; };
    HIP_TRY(dpso::launch_check(I, s), "launch check");
    if (kp.ee_trigger != DPSO_EE_OFF) HIP_TRY(dpso::launch_2opt_prepare(I, cls, s), "launch exchange set-up");
    HIP_TRY(stamp(), "record event");
    for (int32_t g = 0; g < generations; ++g) {
        HIP_TRY(dpso::launch_move(I, tune.move_threads, s), "launch move");
        HIP_TRY(stamp(), "record event");
        if (kp.mutation_period > 0) HIP_TRY(dpso::launch_mutation(I, s), "launch mutation");
        HIP_TRY(stamp(), "record event");
        HIP_TRY(dpso::launch_gbest(I, 1, s), "launch gbest");
        HIP_TRY(stamp(), "record event");
        HIP_TRY(stamp_ex(), "record event");
        if (kp.ee_trigger != DPSO_EE_OFF) HIP_TRY(dpso::launch_2opt(I, cls, s), "launch 2-opt");
        HIP_TRY(stamp(), "record event");
        HIP_TRY(stamp_ex(), "record event");
        // with the exchange on, the end of the generation runs in the global
        // best's launch (the control phase then times nothing)
        if (kp.ee_trigger != DPSO_EE_OFF) HIP_TRY(dpso::launch_gbest(I, 3, s), "launch gbest");
        HIP_TRY(stamp(), "record event");
        if (kp.ee_trigger == DPSO_EE_OFF) HIP_TRY(dpso::launch_end(I, s), "launch end");
        HIP_TRY(stamp(), "record event");
    }
    if (times && exchange_only) {
        HIP_TRY(hipStreamSynchronize(s), "synchronise stream");
        dpso_phase_times t{};
        for (size_t i = 0; i + 1 < mark; i += 2) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev[i], ev[i + 1]), "event time");
            t.ms_exchange += ms;
        }
        t.generations = generations;
        t.exchange_launches = kp.ee_trigger != DPSO_EE_OFF ? generations : 0;
        *times = t;
    } else if (times) {
        HIP_TRY(hipStreamSynchronize(s), "synchronise stream");
        dpso_phase_times t{};
        float *slot[kMarks] = {&t.ms_move, &t.ms_mutation, &t.ms_gbest,
                               &t.ms_exchange, &t.ms_gbest, &t.ms_control};
        for (int32_t g = 0; g < generations; ++g)
            for (int k = 0; k < kMarks; ++k) {
                float ms = 0.f;
                const size_t i = size_t(g) * kMarks + k;
                HIP_TRY(hipEventElapsedTime(&ms, ev[i], ev[i + 1]), "event time");
                *slot[k] += ms;
            }
        if (generations > 0) HIP_TRY(hipEventElapsedTime(&t.ms_total, ev[0], ev[mark - 1]), "event time");
        t.generations = generations;
        t.exchange_launches = kp.ee_trigger != DPSO_EE_OFF ? generations : 0;
        *times = t;
    }
    return ok();
}

// Scene checks shared by both distance-builder entry points (before any
// device work, so they run without a GPU).
dpso_status check_scene(const dpso_scene *scene, const int32_t *d_dist)
{
    if (!scene || !d_dist) return fail(DPSO_E_INVAL, "scene and d_dist must be non-NULL");
    const int32_t n = scene->n, nb = scene->n_boxes;
    if (n < 1) return fail(DPSO_E_INVAL, "scene has n = %d viewpoints", n);
    if (n > DPSO_MAX_N) return fail(DPSO_E_RANGE, "n = %d exceeds DPSO_MAX_N", n);
    if (nb < 0 || (nb > 0 && !scene->boxes_mm) || !scene->vp_mm)
        return fail(DPSO_E_INVAL, "bad box list (n_boxes = %d)", nb);
    if (int64_t(n) + 8 * int64_t(nb) > DPSO_MAX_GRAPH)
        return fail(DPSO_E_RANGE, "n + 8 * n_boxes = %lld exceeds DPSO_MAX_GRAPH = %d",
                    (long long)(int64_t(n) + 8 * int64_t(nb)), DPSO_MAX_GRAPH);
    if (scene->clearance_mm < 0) return fail(DPSO_E_INVAL, "clearance must be >= 0");
    const int64_t lim = int64_t(1) << 26;
    for (int64_t i = 0; i < 3 * int64_t(n); ++i)
        if (scene->vp_mm[i] <= -lim || scene->vp_mm[i] >= lim)
            return fail(DPSO_E_RANGE, "viewpoint coordinate %d outside (-2^26, 2^26)", scene->vp_mm[i]);
    for (int32_t b = 0; b < nb; ++b)
        for (int a = 0; a < 3; ++a) {
            const int64_t lo = scene->boxes_mm[6 * b + a], hi = scene->boxes_mm[6 * b + 3 + a];
            if (lo > hi) return fail(DPSO_E_INVAL, "box %d has lo > hi on axis %d", b, a);
            if (lo - scene->clearance_mm <= -lim || hi + scene->clearance_mm >= lim)
                return fail(DPSO_E_RANGE, "inflated box %d outside (-2^26, 2^26)", b);
        }
    return DPSO_OK;
}

dpso_status build_dist_on(const dpso_scene *scene, int32_t *d_dist, void *work, hipStream_t s)
{
    int range_error = 0;
    HIP_TRY(dpso::build_dist(scene->vp_mm, scene->n, scene->boxes_mm, scene->n_boxes, scene->clearance_mm,
                             d_dist, work, s, &range_error),
            "build_dist");
    if (range_error) return fail(DPSO_E_RANGE, "a finite path cost reaches DPSO_D_INF");
    return ok();
}

// Workspace of dpso_build_dist_noalloc: one static buffer per device, held
// until the process ends. Its device address is looked up once per device
// (with that device current); host code uses only that address, never the
// array's own name, which on the host is a stand-in and not device memory.
__device__ __align__(256) unsigned char dist_scratch[DPSO_NOALLOC_WORK_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

dpso_status noalloc_scratch(void **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(DPSO_E_DEVICE, "device %d outside 0..%d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(dist_scratch)), "address of the static workspace");
        if (!p) return fail(DPSO_E_DEVICE, "static workspace has no device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DPSO_OK;
}

}  // namespace

// ------------------------------------------------------------ autotuner

namespace {

uint64_t fnv1a(uint64_t h, const void *data, size_t bytes)
{
    const unsigned char *p = static_cast<const unsigned char *>(data);
    for (size_t k = 0; k < bytes; ++k) {
        h ^= p[k];
        h *= 1099511628211ull;
    }
    return h;
}

// Digest of what a run computes: the swarm's tours, personal bests,
// velocities and costs (the first n labels of each row, or the stored
// transpositions of a raw velocity), the global best, the trace and the
// header's progress counters. Scratch regions (mutation marks, the 16-bit
// copy of D) are left out. Synchronises the stream.
dpso_status state_digest(const void *d_state, hipStream_t s, uint64_t *out)
{
    dpso::Hdr h;
    dpso_status st = read_header(d_state, &h, s);
    if (st) return st;
    const dpso::Layout L = dpso::make_layout(h.n, h.S, h.cap);
    const char *b = static_cast<const char *>(d_state);
    const size_t S = size_t(h.S), ns = size_t(L.ns), n = size_t(h.n);
    std::vector<uint16_t> X(S * ns), P(S * ns), V(S * 2 * ns), G(ns);
    std::vector<int32_t> VL(S);
    std::vector<int64_t> F(S), FP(S), trace(size_t(h.t) + 1);
    HIP_TRY(hipMemcpyAsync(X.data(), b + L.X, X.size() * 2, hipMemcpyDeviceToHost, s), "copy X");
    HIP_TRY(hipMemcpyAsync(P.data(), b + L.P, P.size() * 2, hipMemcpyDeviceToHost, s), "copy P");
    HIP_TRY(hipMemcpyAsync(V.data(), b + L.V, V.size() * 2, hipMemcpyDeviceToHost, s), "copy V");
    HIP_TRY(hipMemcpyAsync(VL.data(), b + L.VL, S * 4, hipMemcpyDeviceToHost, s), "copy VL");
    HIP_TRY(hipMemcpyAsync(F.data(), b + L.F, S * 8, hipMemcpyDeviceToHost, s), "copy F");
    HIP_TRY(hipMemcpyAsync(FP.data(), b + L.FP, S * 8, hipMemcpyDeviceToHost, s), "copy FP");
    HIP_TRY(hipMemcpyAsync(G.data(), b + L.G, ns * 2, hipMemcpyDeviceToHost, s), "copy G");
    HIP_TRY(hipMemcpyAsync(trace.data(), b + L.trace, trace.size() * 8, hipMemcpyDeviceToHost, s), "copy trace");
    HIP_TRY(hipStreamSynchronize(s), "synchronise stream");
    uint64_t d = 14695981039346656037ull;
    const int64_t counters[] = {h.t, h.stall, h.done, h.FG, int64_t(h.n_sweeps), int64_t(h.n_moves),
                                int64_t(h.n_reshuffled)};
    d = fnv1a(d, counters, sizeof counters);
    for (size_t p = 0; p < S; ++p) {
        d = fnv1a(d, X.data() + p * ns, n * 2);
        d = fnv1a(d, P.data() + p * ns, n * 2);
        const uint16_t *v = V.data() + p * 2 * ns;
        if (h.velocity_cap > 0) {
            d = fnv1a(d, v, size_t(std::max(VL[p], 0)) * 4);
        } else if (VL[p]) {
            d = fnv1a(d, v, n * 2);
            d = fnv1a(d, v + ns, n * 2);
        }
    }
    d = fnv1a(d, VL.data(), S * 4);
    d = fnv1a(d, F.data(), S * 8);
    d = fnv1a(d, FP.data(), S * 8);
    d = fnv1a(d, G.data(), n * 2);
    d = fnv1a(d, trace.data(), trace.size() * 8);
    *out = d;
    return DPSO_OK;
}

}  // namespace

extern "C" {

const char *dpso_version(void) { return "dpso-mi355x 0.2 (gfx950)"; }

const char *dpso_last_error(void) { return dpso::last_error(); }

dpso_status dpso_validate_params(const dpso_params *params, int32_t n)
{
    dpso_status st = check_params(params, n);
    return st ? st : ok();
}

size_t dpso_state_bytes(int32_t n, int32_t swarm_size, int32_t max_generations)
{
    if (n < 1 || n > DPSO_MAX_N || swarm_size < 1 || swarm_size > DPSO_MAX_SWARM ||
        max_generations < 0 || max_generations > (1 << 30))
        return 0;
    return dpso::make_layout(n, swarm_size, max_generations + 1).total;
}

dpso_status dpso_request_footprint(int32_t n, const dpso_params *params, size_t budget, size_t *bytes)
{
    dpso_status st = check_params(params, n);
    if (st) return st;
    const size_t need = dpso::make_layout(n, params->swarm_size, params->max_generations + 1).total +
                        size_t(n) * size_t(n) * 4;
    if (bytes) *bytes = need;
    if (need > budget)
        return fail(DPSO_E_ADMIT, "request needs %zu bytes of device memory, the budget is %zu", need, budget);
    return ok();
}

size_t dpso_dist_work_bytes(int32_t n, int32_t n_boxes)
{
    if (n < 1 || n > DPSO_MAX_N || n_boxes < 0 || int64_t(n) + 8 * int64_t(n_boxes) > DPSO_MAX_GRAPH)
        return 0;
    return dpso::dist_work_bytes(n, n_boxes);
}

dpso_status dpso_build_dist(const dpso_scene *scene, int32_t *d_dist, void *d_work, size_t work_bytes,
                            void *stream)
{
    if (!d_work) return fail(DPSO_E_INVAL, "d_work must be non-NULL");
    dpso_status st = check_scene(scene, d_dist);
    if (st) return st;
    const size_t need = dpso::dist_work_bytes(scene->n, scene->n_boxes);
    if (work_bytes < need) return fail(DPSO_E_NOMEM, "workspace of %zu bytes, %zu needed", work_bytes, need);
    return build_dist_on(scene, d_dist, d_work, as_stream(stream));
}

dpso_status dpso_build_dist_noalloc(const dpso_scene *scene, int32_t *d_dist, void *stream)
{
    dpso_status st = check_scene(scene, d_dist);
    if (st) return st;
    const size_t need = dpso::dist_work_bytes(scene->n, scene->n_boxes);
    if (need > DPSO_NOALLOC_WORK_BYTES)
        return fail(DPSO_E_NOMEM, "scene needs %zu bytes of workspace, more than the %d of the static buffer",
                    need, DPSO_NOALLOC_WORK_BYTES);
    void *work = nullptr;
    if ((st = noalloc_scratch(&work))) return st;
    return build_dist_on(scene, d_dist, work, as_stream(stream));
}

dpso_status dpso_init_nn(const int32_t *d_dist, int32_t n, const dpso_params *params, void *d_state,
                         size_t state_bytes, void *stream)
{
    dpso_status st = check_params(params, n);
    if (st) return st;
    if (!d_dist || !d_state) return fail(DPSO_E_INVAL, "d_dist and d_state must be non-NULL");
    const dpso::Layout L = dpso::make_layout(n, params->swarm_size, params->max_generations + 1);
    if (state_bytes < L.total)
        return fail(DPSO_E_NOMEM, "state buffer of %zu bytes, %zu needed", state_bytes, L.total);
    const dpso::Inst I = make_inst(d_dist, d_state, L, params);
    HIP_TRY(dpso::launch_init(I, as_stream(stream)), "launch init");
    return ok();
}

dpso_status dpso_run(const int32_t *d_dist, int32_t n, const dpso_params *params, void *d_state,
                     size_t state_bytes, int32_t generations, void *stream)
{
    return run_impl(d_dist, n, params, d_state, state_bytes, generations, stream, nullptr);
}

dpso_status dpso_run_profiled(const int32_t *d_dist, int32_t n, const dpso_params *params, void *d_state,
                              size_t state_bytes, int32_t generations, dpso_phase_times *times,
                              void *stream)
{
    if (!times) return fail(DPSO_E_INVAL, "times is NULL");
    return run_impl(d_dist, n, params, d_state, state_bytes, generations, stream, times);
}

dpso_status dpso_run_timed(const int32_t *d_dist, int32_t n, const dpso_params *params, void *d_state,
                           size_t state_bytes, int32_t generations, dpso_phase_times *times, void *stream)
{
    if (!times) return fail(DPSO_E_INVAL, "times must be non-NULL");
    return run_impl(d_dist, n, params, d_state, state_bytes, generations, stream, times, true);
}

dpso_status dpso_autotune(const int32_t *d_dist, int32_t n, const dpso_params *params, void *d_state,
                          size_t state_bytes, int32_t generations, void *d_scratch, size_t scratch_bytes,
                          dpso_tune_result *results, int32_t max_results, int32_t *n_results,
                          dpso_tuning *chosen, void *stream)
{
    dpso_status st = check_params(params, n);
    if (st) return st;
    if (!d_dist || !d_state || !d_scratch) return fail(DPSO_E_INVAL, "d_dist, d_state and d_scratch must be non-NULL");
    if (generations < 1) return fail(DPSO_E_INVAL, "generations must be >= 1");
    if (max_results < 0 || (max_results > 0 && !results)) return fail(DPSO_E_INVAL, "bad results array");
    const dpso::Layout L = dpso::make_layout(n, params->swarm_size, params->max_generations + 1);
    if (state_bytes < L.total) return fail(DPSO_E_NOMEM, "state buffer of %zu bytes, %zu needed", state_bytes, L.total);
    if (scratch_bytes < L.total) return fail(DPSO_E_NOMEM, "scratch of %zu bytes, %zu needed", scratch_bytes, L.total);
    hipStream_t s = as_stream(stream);
    dpso::Hdr h;
    if ((st = read_header(d_state, &h, s))) return st;
    if (h.n != n || h.S != params->swarm_size) return fail(DPSO_E_STATE, "state does not hold n = %d, swarm %d", n, params->swarm_size);
    if (int64_t(h.t) + generations > params->max_generations)
        return fail(DPSO_E_RANGE, "the state is at generation %d: %d more pass max_generations = %d", h.t,
                    generations, params->max_generations);
    HIP_TRY(hipMemcpyAsync(d_scratch, d_state, L.total, hipMemcpyDeviceToDevice, s), "snapshot state");
    hipEvent_t ev[2];
    std::vector<hipEvent_t> pool;
    if ((st = events(2, pool))) return st;
    ev[0] = pool[0];
    ev[1] = pool[1];
    const dpso::Tune dflt = dpso::default_tuning(n, params->swarm_size);
    std::vector<dpso_tune_result> done;
    // one candidate: two timed runs from the snapshot, the digest of the second
    auto trial = [&](const dpso::Tune &t) -> dpso_status {
        dpso_tune_result r{};
        r.config.move_threads = t.move_threads;
        r.config.exchange_rows = t.exchange_rows;
        r.ms = -1.f;
        for (int rep = 0; rep < 2; ++rep) {
            HIP_TRY(hipMemcpyAsync(d_state, d_scratch, L.total, hipMemcpyDeviceToDevice, s), "restore state");
            HIP_TRY(hipEventRecord(ev[0], s), "record event");
            dpso_status rs = run_impl(d_dist, n, params, d_state, state_bytes, generations, stream, nullptr, false, &t);
            if (rs) return rs;
            HIP_TRY(hipEventRecord(ev[1], s), "record event");
            HIP_TRY(hipEventSynchronize(ev[1]), "synchronise event");
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]), "event time");
            if (r.ms < 0.f || ms < r.ms) r.ms = ms;
        }
        dpso_status ds = state_digest(d_state, s, &r.digest);
        if (ds) return ds;
        done.push_back(r);
        return DPSO_OK;
    };
    auto finish = [&](dpso_status code) -> dpso_status {
        // leave the state as it was, whatever happened
        const hipError_t e1 = hipMemcpyAsync(d_state, d_scratch, L.total, hipMemcpyDeviceToDevice, s);
        const hipError_t e2 = hipStreamSynchronize(s);
        if (code == DPSO_OK && e1 != hipSuccess) return hip_fail(e1, "restore state");
        if (code == DPSO_OK && e2 != hipSuccess) return hip_fail(e2, "synchronise stream");
        return code;
    };
    // phase 1: threads per particle in the move, the exchange at its default
    const int ns = L.ns;
    for (int tpb : {64, 128, 256, 512}) {
        if (!dpso::move_threads_ok(tpb, ns)) continue;
        st = trial(dpso::Tune{tpb, dflt.exchange_rows});
        if (st) return finish(st);
    }
    size_t best = 0;
    for (size_t k = 1; k < done.size(); ++k)
        if (done[k].ms < done[best].ms) best = k;
    // phase 2: the exchange's row form with the fastest move
    const bool exchange = params->ee_trigger != DPSO_EE_OFF && params->ee_neighbourhood == DPSO_NB_TWO_OPT;
    if (exchange) {
        const int tpb = done[best].config.move_threads;
        for (int rows : {DPSO_ROWS_U16, DPSO_ROWS_I32, DPSO_ROWS_BLOCK, DPSO_ROWS_U16_PAIR, DPSO_ROWS_U16_QUAD}) {
            if (rows == dflt.exchange_rows) continue;
            if (rows == DPSO_ROWS_U16 && !dpso::packed_rows(n)) continue;
            if (rows == DPSO_ROWS_U16_PAIR && !(dpso::packed_rows(n) && n > 128)) continue;
            if (rows == DPSO_ROWS_U16_QUAD && !(dpso::packed_rows(n) && n > 256)) continue;
            if (rows == DPSO_ROWS_I32 && n > 1024) continue;
            // an n off 16 bytes takes 16-bit rows for int32 ones: the same kernel
            if (rows == DPSO_ROWS_I32 && (n & 3) != 0 && dpso::packed_rows(n)) continue;
            st = trial(dpso::Tune{tpb, rows});
            if (st) return finish(st);
        }
    }
    for (size_t k = 0; k < done.size(); ++k) {
        if (done[k].digest != done[0].digest)
            return finish(fail(DPSO_E_STATE, "configurations disagree: %d threads / rows %d and %d threads / rows %d",
                               done[0].config.move_threads, done[0].config.exchange_rows,
                               done[k].config.move_threads, done[k].config.exchange_rows));
        if (done[k].ms < done[best].ms) best = k;
    }
    st = finish(DPSO_OK);
    if (st) return st;
    if ((st = dpso_tuning_set(n, params->swarm_size, &done[best].config))) return st;
    for (int32_t k = 0; k < max_results && size_t(k) < done.size(); ++k) results[k] = done[size_t(k)];
    if (n_results) *n_results = int32_t(done.size());
    if (chosen) *chosen = done[best].config;
    return ok();
}

dpso_status dpso_get_info(const void *d_state, dpso_info *info, void *stream)
{
    if (!info) return fail(DPSO_E_INVAL, "info is NULL");
    dpso::Hdr h;
    dpso_status st = read_header(d_state, &h, as_stream(stream));
    if (st) return st;
    info->n = h.n;
    info->swarm_size = h.S;
    info->trace_capacity = h.cap;
    info->generation = h.t;
    info->stall = h.stall;
    info->done = h.done;
    info->best_cost = h.FG;
    info->sweeps = int64_t(h.n_sweeps);
    info->moves = int64_t(h.n_moves);
    info->reshuffled = int64_t(h.n_reshuffled);
    return ok();
}

dpso_status dpso_get_best(const void *d_state, int32_t *h_tour, int64_t *h_cost, int32_t *h_generation,
                          int64_t *h_trace, void *stream)
{
    hipStream_t s = as_stream(stream);
    dpso::Hdr h;
    dpso_status st = read_header(d_state, &h, s);
    if (st) return st;
    const dpso::Layout L = dpso::make_layout(h.n, h.S, h.cap);
    const char *base = static_cast<const char *>(d_state);
    std::vector<uint16_t> g(size_t(h.n));
    HIP_TRY(hipMemcpyAsync(g.data(), base + L.G, size_t(h.n) * 2, hipMemcpyDeviceToHost, s), "copy G");
    if (h_trace)
        HIP_TRY(hipMemcpyAsync(h_trace, base + L.trace, size_t(h.t + 1) * 8, hipMemcpyDeviceToHost, s),
                "copy trace");
    HIP_TRY(hipStreamSynchronize(s), "synchronise stream");
    if (h_tour)
        for (int32_t k = 0; k < h.n; ++k) h_tour[k] = g[k];
    if (h_cost) *h_cost = h.FG;
    if (h_generation) *h_generation = h.t;
    return ok();
}

dpso_status dpso_export_state(const void *d_state, int32_t n, int32_t swarm_size, dpso_host_state *out,
                              void *stream)
{
    if (!out || !out->X || !out->P || !out->V || !out->vlen || !out->F || !out->FP || !out->G)
        return fail(DPSO_E_INVAL, "every array of the host state must be non-NULL");
    hipStream_t s = as_stream(stream);
    dpso::Hdr h;
    dpso_status st = read_header(d_state, &h, s);
    if (st) return st;
    if (h.n != n || h.S != swarm_size)
        return fail(DPSO_E_STATE, "state holds n = %d, swarm %d; asked for n = %d, swarm %d", h.n, h.S, n,
                    swarm_size);
    const dpso::Layout L = dpso::make_layout(h.n, h.S, h.cap);
    const char *b = static_cast<const char *>(d_state);
    const size_t S = size_t(h.S);
    HIP_TRY(hipMemcpy2DAsync(out->X, size_t(n) * 2, b + L.X, size_t(L.ns) * 2, size_t(n) * 2, S,
                             hipMemcpyDeviceToHost, s), "copy X");
    HIP_TRY(hipMemcpy2DAsync(out->P, size_t(n) * 2, b + L.P, size_t(L.ns) * 2, size_t(n) * 2, S,
                             hipMemcpyDeviceToHost, s), "copy P");
    std::vector<uint16_t> vt(S * 2 * size_t(L.ns));
    std::vector<int32_t> has_v(S);
    HIP_TRY(hipMemcpyAsync(vt.data(), b + L.V, vt.size() * 2, hipMemcpyDeviceToHost, s), "copy V");
    HIP_TRY(hipMemcpyAsync(has_v.data(), b + L.VL, S * 4, hipMemcpyDeviceToHost, s), "copy VL");
    HIP_TRY(hipMemcpyAsync(out->F, b + L.F, S * 8, hipMemcpyDeviceToHost, s), "copy F");
    HIP_TRY(hipMemcpyAsync(out->FP, b + L.FP, S * 8, hipMemcpyDeviceToHost, s), "copy FP");
    HIP_TRY(hipMemcpyAsync(out->G, b + L.G, size_t(n) * 2, hipMemcpyDeviceToHost, s), "copy G");
    if (out->trace)
        HIP_TRY(hipMemcpyAsync(out->trace, b + L.trace, size_t(h.t + 1) * 8, hipMemcpyDeviceToHost, s),
                "copy trace");
    HIP_TRY(hipStreamSynchronize(s), "synchronise stream");
    std::vector<uint16_t> cur, pos;
    for (size_t p = 0; p < S; ++p) {
        uint16_t *row = out->V + p * size_t(n) * 2;
        std::fill(row, row + size_t(n) * 2, uint16_t(0));
        const uint16_t *from = vt.data() + p * 2 * L.ns;
        if (h.velocity_cap > 0) {  // a transposition list, held as it is
            out->vlen[p] = has_v[p];
            std::copy(from, from + 2 * size_t(has_v[p]), row);
        } else {
            out->vlen[p] = has_v[p] ? host_difference(from, from + L.ns, n, row, cur, pos) : 0;
        }
    }
    out->generation = h.t;
    out->stall = h.stall;
    out->done = h.done;
    out->best_cost = h.FG;
    return ok();
}

dpso_status dpso_import_state(void *d_state, size_t state_bytes, int32_t n, int32_t swarm_size,
                              const dpso_host_state *in, void *stream)
{
    if (!in || !in->X || !in->P || !in->V || !in->vlen || !in->F || !in->FP || !in->G || !in->trace)
        return fail(DPSO_E_INVAL, "every array of the host state must be non-NULL");
    hipStream_t s = as_stream(stream);
    dpso::Hdr h;
    dpso_status st = read_header(d_state, &h, s);
    if (st) return st;
    if (h.n != n || h.S != swarm_size)
        return fail(DPSO_E_STATE, "state holds n = %d, swarm %d; asked for n = %d, swarm %d", h.n, h.S, n,
                    swarm_size);
    const dpso::Layout L = dpso::make_layout(h.n, h.S, h.cap);
    if (state_bytes < L.total) return fail(DPSO_E_NOMEM, "state buffer too small");
    if (in->generation < 0 || in->generation >= h.cap)
        return fail(DPSO_E_RANGE, "generation %d outside the trace capacity %d", in->generation, h.cap);
    const size_t S = size_t(h.S);
    std::vector<uint8_t> seen(static_cast<size_t>(n), 0);
    auto is_perm = [&](const uint16_t *t) {
        std::fill(seen.begin(), seen.end(), 0);
        for (int32_t k = 0; k < n; ++k) {
            if (t[k] >= n || seen[t[k]]) return false;
            seen[t[k]] = 1;
        }
        return true;
    };
    for (size_t p = 0; p < S; ++p) {
        if (!is_perm(in->X + p * n) || !is_perm(in->P + p * n))
            return fail(DPSO_E_INVAL, "tour of particle %zu is not a permutation", p);
        const int32_t most = h.velocity_cap > 0 ? h.velocity_cap : n - 1;
        if (in->vlen[p] < 0 || in->vlen[p] > most)
            return fail(DPSO_E_INVAL, "velocity length of particle %zu out of range", p);
    }
    std::vector<uint16_t> vt(S * 2 * size_t(L.ns), 0);
    std::vector<int32_t> has_v(S);
    for (size_t p = 0; p < S; ++p) {
        const uint16_t *pairs = in->V + p * size_t(n) * 2;
        uint16_t *from = vt.data() + p * 2 * L.ns;
        if (h.velocity_cap > 0) {  // raw velocity: any list of labels
            for (int32_t k = 0; k < 2 * in->vlen[p]; ++k)
                if (pairs[k] >= n) return fail(DPSO_E_INVAL, "velocity of particle %zu names a label >= n", p);
            std::copy(pairs, pairs + 2 * size_t(in->vlen[p]), from);
            has_v[p] = in->vlen[p];
            continue;
        }
        has_v[p] = in->vlen[p] > 0;
        if (has_v[p] && !host_velocity_tours(pairs, in->vlen[p], n, from, from + L.ns))
            return fail(DPSO_E_INVAL, "velocity of particle %zu is not a canonical difference of two tours", p);
    }
    if (!is_perm(in->G)) return fail(DPSO_E_INVAL, "global best is not a permutation");
    char *b = static_cast<char *>(d_state);
    HIP_TRY(hipMemcpy2DAsync(b + L.X, size_t(L.ns) * 2, in->X, size_t(n) * 2, size_t(n) * 2, S,
                             hipMemcpyHostToDevice, s), "copy X");
    HIP_TRY(hipMemcpy2DAsync(b + L.P, size_t(L.ns) * 2, in->P, size_t(n) * 2, size_t(n) * 2, S,
                             hipMemcpyHostToDevice, s), "copy P");
    HIP_TRY(hipMemcpyAsync(b + L.V, vt.data(), vt.size() * 2, hipMemcpyHostToDevice, s), "copy V");
    HIP_TRY(hipMemcpyAsync(b + L.VL, has_v.data(), S * 4, hipMemcpyHostToDevice, s), "copy VL");
    HIP_TRY(hipMemcpyAsync(b + L.F, in->F, S * 8, hipMemcpyHostToDevice, s), "copy F");
    HIP_TRY(hipMemcpyAsync(b + L.FP, in->FP, S * 8, hipMemcpyHostToDevice, s), "copy FP");
    HIP_TRY(hipMemcpyAsync(b + L.G, in->G, size_t(n) * 2, hipMemcpyHostToDevice, s), "copy G");
    HIP_TRY(hipMemcpyAsync(b + L.trace, in->trace, size_t(in->generation + 1) * 8, hipMemcpyHostToDevice, s),
            "copy trace");
    h.t = in->generation;
    h.stall = in->stall;
    h.done = in->done;
    h.FG = in->best_cost;
    h.improved = 0;
    h.ee_ran = 0;
    HIP_TRY(hipMemcpyAsync(d_state, &h, sizeof h, hipMemcpyHostToDevice, s), "write header");
    HIP_TRY(hipStreamSynchronize(s), "synchronise stream");
    return ok();
}


// ------------------------------------------------------------------ batches

size_t dpso_batch_work_bytes(int32_t count)
{
    if (count < 1 || count > DPSO_MAX_BATCH) return 0;
    return batch_layout(count).total;
}

dpso_status dpso_init_batch(const dpso_batch_item *items, int32_t count, void *d_work, size_t work_bytes,
                            void *stream)
{
    BatchPlan plan;
    dpso_status st = plan_batch(items, count, d_work, work_bytes, as_stream(stream), plan);
    if (st) return st;
    hipStream_t s = as_stream(stream);
    HIP_TRY(dpso::launch_batch_init(plan.items, plan.instances, plan.total, plan.max_ns, s), "launch init");
    HIP_TRY(hipStreamSynchronize(s), "synchronise stream");
    return ok();
}

dpso_status dpso_run_batch(const dpso_batch_item *items, int32_t count, int32_t generations, void *d_work,
                           size_t work_bytes, void *stream)
{
    if (generations < 0) return fail(DPSO_E_INVAL, "generations must be >= 0");
    BatchPlan plan;
    dpso_status st = plan_batch(items, count, d_work, work_bytes, as_stream(stream), plan);
    if (st) return st;
    hipStream_t s = as_stream(stream);
    // launched as they are enqueued: the host stays ahead of the GPU (a few
    // µs a launch against ~0.1-2 ms of kernels a generation), and capturing
    // the run into a graph first would cost its capture and instantiation
    // (thousands of nodes) before any work starts
    hipError_t e = enqueue_batch(plan, generations, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "batched run");
    return ok();
}

}  // extern "C"
