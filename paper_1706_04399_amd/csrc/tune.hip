// The launch-configuration table: one per device, filled by the autotuner
// (dpso_autotune) or by the caller (dpso_tuning_set), read on every run.
#include <mutex>

#include "dpso.h"
#include "errors.hpp"
#include "kernels.hpp"
#include "tune.hpp"

namespace dpso {

namespace {

constexpr int kMaxDevices = 64;

struct Table {
    Tune entry[kTuneNBuckets][kTunePBuckets];  // {0, 0}: empty
    int order;                                 // DPSO_ORDER_*, 0: default
    bool merge_set;                            // false: the default merge limit
    int64_t merge;                             // batches of at most this many particles merge
};

constexpr int kDefaultOrder = DPSO_ORDER_LPT;
constexpr int64_t kDefaultMerge = DPSO_MERGE_DEFAULT_PARTICLES;

std::mutex g_table_mutex;
Table g_tables[kMaxDevices];

int current_device()
{
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= kMaxDevices) d = 0;
    return d;
}

int bucket_max_n(int b) { return b >= 12 ? 4096 : 1 << b; }

}  // namespace

int tune_bucket_n(int n)
{
    int b = 1;
    while (b < 12 && n > (1 << b)) ++b;
    return b;
}

int tune_bucket_p(int64_t particles)
{
    return particles <= 128 ? 0 : particles <= 512 ? 1 : particles <= 1024 ? 2 : particles <= 2048 ? 3
                                                                               : particles <= 8192 ? 4 : 5;
}

// Built-in choices, from the autotuner's measurements on MI355X (facades,
// edge exchange every generation) and from batched and served runs. A lone
// swarm of at most 1024 particles takes int32 rows straight into LDS for
// multiples of 4 up to n = 256, where they take one load chunk either way
// and ran faster than 16-bit rows (n = 200, swarm 1024: 6.4 against 7.1 ms
// for 64 generations). With more particles in flight — large swarms and
// batches, whose move and exchange classes run one after another — every
// n from 8 to 1024 takes 16-bit rows, which keeps one exchange class per
// column count (the batched workload: 320 solves/s against 290 with int32
// rows for the multiples of 4). Among at most 1024 particles, which leave
// most SIMDs idle, the other n above 128 take 16-bit rows with two wavefronts
// per particle, and among at most 512 those above 256 with four (n = 800,
// swarm 512: 2.75 ms for 12 generations with four, 3.30 with two, 3.82 with
// one; served re-planning p99 126 ms against 135 with pairs only and 140 with
// one wavefront). The move
// runs one wavefront per particle for
// a lone swarm of at most 128 (the cheapest barriers) and, among more than
// 8192 particles, for n <= 512 (the GPU is full whatever the width, and
// narrow blocks waste no lanes); 256 threads otherwise.
Tune default_tuning(int n, int64_t particles)
{
    Tune t;
    const int ns = (n + 63) & ~63;
    const bool aligned = (n & 3) == 0;
    if (particles > 8192)
        t.move_threads = n <= 512 ? 64 : 256;
    else if (particles <= 128)
        t.move_threads = move_threads_ok(64, ns) ? 64 : 256;
    else
        t.move_threads = 256;
    const bool i32 = !packed_rows(n) || (particles <= 1024 && aligned && n <= 256);
    const bool quad = particles <= 512 && n > 256, pair = particles <= 1024 && n > 128;
    t.exchange_rows = n > 1024 ? DPSO_ROWS_BLOCK
                      : i32    ? DPSO_ROWS_I32
                      : quad   ? DPSO_ROWS_U16_QUAD
                      : pair   ? DPSO_ROWS_U16_PAIR
                               : DPSO_ROWS_U16;
    return t;
}

// int32 rows of an n that is not a multiple of 4 do not start on 16 bytes and
// would pass through registers, several times slower than 16-bit rows: such
// an n takes 16-bit rows whenever it has them (a bucket's pick is made on an
// aligned n).
Tune resolve_tuning(Tune t, int n, int64_t particles)
{
    const Tune d = default_tuning(n, particles);
    const int ns = (n + 63) & ~63;
    if (!move_threads_ok(t.move_threads, ns)) t.move_threads = d.move_threads;
    if (t.exchange_rows == DPSO_ROWS_I32 && (n & 3) != 0 && packed_rows(n)) t.exchange_rows = DPSO_ROWS_U16;
    // four wavefronts per particle split at least 256 rows, two at least 128;
    // smaller n take fewer
    if (t.exchange_rows == DPSO_ROWS_U16_QUAD && packed_rows(n) && n <= 256) t.exchange_rows = DPSO_ROWS_U16_PAIR;
    if (t.exchange_rows == DPSO_ROWS_U16_PAIR && packed_rows(n) && n <= 128) t.exchange_rows = DPSO_ROWS_U16;
    const bool ok = t.exchange_rows == DPSO_ROWS_BLOCK || (t.exchange_rows == DPSO_ROWS_I32 && n <= 1024) ||
                    (t.exchange_rows == DPSO_ROWS_U16 && packed_rows(n)) ||
                    (t.exchange_rows == DPSO_ROWS_U16_PAIR && packed_rows(n) && n > 128) ||
                    (t.exchange_rows == DPSO_ROWS_U16_QUAD && packed_rows(n) && n > 256);
    if (!ok) t.exchange_rows = d.exchange_rows;
    return t;
}

int batch_order()
{
    std::lock_guard<std::mutex> lock(g_table_mutex);
    const int o = g_tables[current_device()].order;
    return o == DPSO_ORDER_DEFAULT ? kDefaultOrder : o;
}

int64_t batch_merge()
{
    std::lock_guard<std::mutex> lock(g_table_mutex);
    const Table &t = g_tables[current_device()];
    return t.merge_set ? t.merge : kDefaultMerge;
}

Tune tuning_for(int n, int64_t particles)
{
    Tune t{0, 0};
    {
        std::lock_guard<std::mutex> lock(g_table_mutex);
        t = g_tables[current_device()].entry[tune_bucket_n(n)][tune_bucket_p(particles)];
    }
    return resolve_tuning(t, n, particles);
}

}  // namespace dpso

using dpso::fail;
using dpso::ok;

extern "C" {

dpso_status dpso_tuning_get(int32_t n, int32_t particles, dpso_tuning *out)
{
    if (!out) return fail(DPSO_E_INVAL, "out is NULL");
    if (n < 1 || n > DPSO_MAX_N) return fail(DPSO_E_RANGE, "n = %d outside 1..DPSO_MAX_N", n);
    if (particles < 1) return fail(DPSO_E_INVAL, "particles = %d must be at least 1", particles);
    const dpso::Tune t = dpso::tuning_for(n, particles);
    out->move_threads = t.move_threads;
    out->exchange_rows = t.exchange_rows;
    return ok();
}

dpso_status dpso_tuning_set(int32_t n, int32_t particles, const dpso_tuning *t)
{
    if (n < 1 || n > DPSO_MAX_N) return fail(DPSO_E_RANGE, "n = %d outside 1..DPSO_MAX_N", n);
    if (particles < 1) return fail(DPSO_E_INVAL, "particles = %d must be at least 1", particles);
    const int bn = dpso::tune_bucket_n(n), bp = dpso::tune_bucket_p(particles);
    dpso::Tune e{0, 0};
    if (t) {
        if (t->move_threads != 0 && t->move_threads != 64 && t->move_threads != 128 && t->move_threads != 256 &&
            t->move_threads != 512)
            return fail(DPSO_E_INVAL, "move_threads = %d is not 0, 64, 128, 256 or 512", t->move_threads);
        if (t->exchange_rows < DPSO_ROWS_AUTO || t->exchange_rows > DPSO_ROWS_U16_QUAD)
            return fail(DPSO_E_INVAL, "exchange_rows = %d is not a DPSO_ROWS_* value", t->exchange_rows);
        const int top = dpso::bucket_max_n(bn), ns = (top + 63) & ~63;
        if (t->move_threads != 0 && !dpso::move_threads_ok(t->move_threads, ns))
            return fail(DPSO_E_RANGE, "%d threads per particle cannot serve n = %d (at most 16 positions each)",
                        t->move_threads, top);
        if ((t->exchange_rows == DPSO_ROWS_U16 || t->exchange_rows == DPSO_ROWS_I32 ||
             t->exchange_rows == DPSO_ROWS_U16_PAIR || t->exchange_rows == DPSO_ROWS_U16_QUAD) && n > 1024)
            return fail(DPSO_E_RANGE, "the wavefront exchange serves n up to 1024");
        e.move_threads = t->move_threads;
        e.exchange_rows = t->exchange_rows;
    }
    std::lock_guard<std::mutex> lock(dpso::g_table_mutex);
    dpso::g_tables[dpso::current_device()].entry[bn][bp] = e;
    return ok();
}

dpso_status dpso_tuning_reset(void)
{
    std::lock_guard<std::mutex> lock(dpso::g_table_mutex);
    dpso::g_tables[dpso::current_device()] = dpso::Table{};
    return ok();
}

dpso_status dpso_batch_order_set(int32_t order)
{
    if (order < DPSO_ORDER_DEFAULT || order > DPSO_ORDER_XCD)
        return fail(DPSO_E_INVAL, "batch order %d is not a DPSO_ORDER_* value", order);
    std::lock_guard<std::mutex> lock(dpso::g_table_mutex);
    dpso::g_tables[dpso::current_device()].order = order;
    return ok();
}

int32_t dpso_batch_order_get(void) { return dpso::batch_order(); }

dpso_status dpso_batch_merge_set(int64_t max_particles)
{
    std::lock_guard<std::mutex> lock(dpso::g_table_mutex);
    dpso::Table &t = dpso::g_tables[dpso::current_device()];
    t.merge_set = max_particles >= 0;
    t.merge = max_particles;
    return ok();
}

int64_t dpso_batch_merge_get(void) { return dpso::batch_merge(); }

}  // extern "C"
