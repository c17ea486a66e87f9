// Host-side launchers of the device kernels (one translation unit each).
#pragma once

#include <hip/hip_runtime.h>

#include "state.hpp"

namespace dpso {

// swarm.hip
hipError_t launch_init(const int32_t *D, const View &st, const KParams &kp, int32_t cap, hipStream_t s);
hipError_t launch_check(const View &st, int32_t cap, hipStream_t s);
hipError_t launch_move(const int32_t *D, const View &st, const KParams &kp, hipStream_t s);
hipError_t launch_mutation(const int32_t *D, const View &st, const KParams &kp, hipStream_t s);
hipError_t launch_gbest(const View &st, const KParams &kp, int mode, hipStream_t s);
hipError_t launch_end(const View &st, const KParams &kp, hipStream_t s);

// twoopt.hip
hipError_t launch_2opt(const int32_t *D, const View &st, const KParams &kp, hipStream_t s);

// dist.hip
size_t dist_work_bytes(int32_t n, int32_t n_boxes);
// Builds the travelling-cost matrix; *range_error receives 1 if a finite
// path cost reached the blocked-pair sentinel. Synchronises the stream.
hipError_t build_dist(const int32_t *h_vp, int32_t n, const int32_t *h_boxes, int32_t n_boxes,
                      int32_t clearance, int32_t *d_dist, void *d_work, hipStream_t s,
                      int *range_error);

}  // namespace dpso
