// Host-side launchers of the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "state.hpp"
#include "tune.hpp"

namespace dpso {

// swarm.hip: one instance (descriptor by value)
hipError_t launch_init(const Inst &I, hipStream_t s);
hipError_t launch_check(const Inst &I, hipStream_t s);
// the move at tpb (64, 128, 256 or 512) threads per particle; move_threads_ok
// tells whether tpb serves row stride ns (at most 16 positions per thread)
bool move_threads_ok(int tpb, int ns);
hipError_t launch_move(const Inst &I, int tpb, hipStream_t s);
hipError_t launch_mutation(const Inst &I, hipStream_t s);
hipError_t launch_gbest(const Inst &I, int mode, hipStream_t s);
hipError_t launch_end(const Inst &I, hipStream_t s);

// swarm.hip: many instances. `items` has one block per particle (total
// blocks), `instances` one block per instance; max_ns sizes dynamic LDS.
hipError_t launch_batch_init(const Batch &items, const Batch &instances, int total, int max_ns, hipStream_t s);
hipError_t launch_batch_check(const Batch &items, const Batch &instances, int total, int max_ns, hipStream_t s);
// the move of one move class (instances sharing tpb; `items` its table)
hipError_t launch_batch_move(int tpb, const Batch &items, int total, int max_ns, hipStream_t s);
hipError_t launch_batch_mutation(const Batch &items, const Batch &instances, int total, int max_ns,
                                 hipStream_t s);
hipError_t launch_batch_gbest(const Batch &items, const Batch &instances, int total, int max_ns, int mode,
                              hipStream_t s);
hipError_t launch_batch_end(const Batch &items, const Batch &instances, int total, int max_ns, hipStream_t s);

// twoopt.hip: the edge-exchange kernel depends on the neighbourhood, on n
// (columns held per lane), on the row form of the configuration and on the
// alignment of D (exchange_class, tune.hpp); instances of one class share a
// launch. The last class is the node-swap neighbourhood.
constexpr int kExchangeClasses = 22;
hipError_t launch_2opt(const Inst &I, int cls, hipStream_t s);
hipError_t launch_batch_2opt(int cls, const Batch &items, int total, int max_ns, hipStream_t s);
// Classes that stage 16-bit rows can share a launch with the other classes
// of their merge group (1: one wavefront per particle, 2: two, 3: four; 0: none):
// launch_batch_2opt_mixed runs `items`, instances of class `cls` or of
// smaller classes of its group, in one launch, each with its own class's
// body.
int exchange_merge_group(int cls);
hipError_t launch_batch_2opt_mixed(int cls, const Batch &items, int total, int max_ns, hipStream_t s);
// Per-run set-up of the exchange: classes that stage 16-bit rows refresh the
// state's packed copy of D (after the run's first launch, which clears the
// header's maximum). `members` is a class's instance table; max_n bounds n.
hipError_t launch_2opt_prepare(const Inst &I, int cls, hipStream_t s);
hipError_t launch_batch_2opt_prepare(int cls, const Batch &members, int max_n, hipStream_t s);

// nodeswap.hip: the node-swap neighbourhood (one workgroup per particle).
hipError_t launch_node_swap(const Inst *one, const Batch &items, int grid, int max_ns, hipStream_t s);

// dist.hip
size_t dist_work_bytes(int32_t n, int32_t n_boxes);
// Builds the travelling-cost matrix; *range_error receives 1 if a finite
// path cost reached the blocked-pair sentinel. Synchronises the stream.
hipError_t build_dist(const int32_t *h_vp, int32_t n, const int32_t *h_boxes, int32_t n_boxes,
                      int32_t clearance, int32_t *d_dist, void *d_work, hipStream_t s,
                      int *range_error);

}  // namespace dpso
