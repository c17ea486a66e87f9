// The matrix contract every swarm call relies on (Sect. 2: one symmetric
// travelling cost per pair of viewpoints and none from a viewpoint to itself;
// Sect. 2.3: a blocked pair costs DPSO_D_INF): D[i][i] = 0, D[i][j] = D[j][i],
// 0 <= D[i][j] <= DPSO_D_INF. One workgroup per 64 x 64 tile reads the tile
// and its mirror tile with coalesced row loads into LDS and compares them
// there; the smallest row-major index of a broken entry is kept with a 64-bit
// atomicMin.
#include <stdint.h>

#include <algorithm>

#include "device.hpp"
#include "dpso.h"
#include "errors.hpp"

namespace dpso {

namespace {

constexpr int kTile = 64;
constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_check_dist(const int32_t *__restrict__ D, int32_t n, int32_t tiles,
                                                         unsigned long long *first)
{
    __shared__ int32_t a[kTile][kTile + 1], b[kTile][kTile + 1];
    const int64_t t = blockIdx.x;
    const int32_t ti = int32_t(t / tiles), tj = int32_t(t % tiles);
    const int64_t r0 = int64_t(ti) * kTile, c0 = int64_t(tj) * kTile;
    const int c = threadIdx.x % kTile, r = threadIdx.x / kTile;  // 4 rows per pass
    for (int rr = r; rr < kTile; rr += kThreads / kTile) {
        const int64_t i = r0 + rr, j = c0 + c, i2 = c0 + rr, j2 = r0 + c;
        a[rr][c] = i < n && j < n ? D[i * n + j] : 0;   // tile (ti, tj)
        b[rr][c] = i2 < n && j2 < n ? D[i2 * n + j2] : 0;  // mirror tile (tj, ti)
    }
    __syncthreads();
    unsigned long long bad = ~0ull;
    for (int rr = r; rr < kTile; rr += kThreads / kTile) {
        const int64_t i = r0 + rr, j = c0 + c;
        if (i >= n || j >= n) continue;
        const int32_t v = a[rr][c];
        const bool broken = v < 0 || v > DPSO_D_INF || (i == j && v != 0) || v != b[c][rr];
        if (broken) bad = min(bad, (unsigned long long)(i * n + j));
    }
    if (bad != ~0ull) atomicMin(first, bad);
}

}  // namespace

}  // namespace dpso

extern "C" dpso_status dpso_check_dist(const int32_t *d_dist, int32_t n, void *d_work, size_t work_bytes,
                                       int64_t *h_bad, void *stream)
{
    using namespace dpso;
    if (!d_dist || !d_work || !h_bad) return fail(DPSO_E_INVAL, "d_dist, d_work and h_bad must be non-NULL");
    if (n < 1 || n > DPSO_MAX_N) return fail(DPSO_E_RANGE, "n = %d outside 1..DPSO_MAX_N", n);
    if (work_bytes < 8) return fail(DPSO_E_NOMEM, "workspace of %zu bytes, 8 needed", work_bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto *first = static_cast<unsigned long long *>(d_work);
    const unsigned long long none = ~0ull;
    unsigned long long got = none;
    const int32_t tiles = (n + kTile - 1) / kTile;
    hipError_t e = hipMemcpyAsync(first, &none, 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        k_check_dist<<<unsigned(int64_t(tiles) * tiles), kThreads, 0, s>>>(d_dist, n, tiles, first);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&got, first, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(DPSO_E_DEVICE, "matrix check: %s", hipGetErrorString(e));
    *h_bad = got == none ? -1 : int64_t(got);
    if (got != none)
        return fail(DPSO_E_RANGE, "entry (%lld, %lld) breaks the matrix contract", (long long)(got / unsigned(n)),
                    (long long)(got % unsigned(n)));
    return ok();
}
