// Launch configuration of the generation loop and the per-device table the
// autotuner fills. Every configuration computes the same result; the table
// only decides which kernels run.
#pragma once

#include <stdint.h>

namespace dpso {

struct Tune {
    int move_threads;   // 64, 128, 256 or 512 threads per particle in the move
    int exchange_rows;  // DPSO_ROWS_U16, _I32 or _BLOCK (resolved, never AUTO)
};

// Buckets: n in (2^(b-1), 2^b] (b = 1 .. 12, n <= 2 in bucket 1) and the
// particles launched together (<= 128, <= 512, <= 1024, <= 2048, <= 8192,
// more).
constexpr int kTuneNBuckets = 13;
constexpr int kTunePBuckets = 6;
int tune_bucket_n(int n);
int tune_bucket_p(int64_t particles);

// The built-in configuration for n among `particles` particles.
Tune default_tuning(int n, int64_t particles);

// Makes a (possibly partial) configuration valid for n: a zero or unusable
// field takes the default's value.
Tune resolve_tuning(Tune t, int n, int64_t particles);

// The configuration for n among `particles` on the current device: its
// table entry, else the default, resolved for n.
Tune tuning_for(int n, int64_t particles);

// The batch order of the current device (DPSO_ORDER_INDEX, _LPT or _XCD).
int batch_order();

// Batches of at most this many particles run their 16-bit row exchange
// classes in one launch (current device).
int64_t batch_merge();

// The exchange class of an instance under a configuration (see
// twoopt.hip); D's alignment decides between the int32 kernels.
int exchange_class(int n, const int32_t *D, int neighbourhood, int rows);

}  // namespace dpso
