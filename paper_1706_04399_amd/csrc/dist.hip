// Obstacle-aware travelling costs between viewpoints (Sect. 2.2-2.3).
//
// Graph nodes are the n viewpoints followed by the 8 corners of every box
// inflated by the clearance. Two nodes are joined iff the straight segment
// between them misses the open interior of every inflated box; the edge
// costs its Euclidean length in mm rounded half up. All-pairs shortest paths
// (Floyd-Warshall, one launch per pivot) then give the viewpoint block.
// Everything is exact integer arithmetic.
#include <vector>

#include "device.hpp"
#include "kernels.hpp"

namespace dpso {

namespace {

constexpr int64_t kNoEdge = int64_t(1) << 62;
constexpr int32_t kBlocked = 268435455;  // 2^28 - 1

struct Work {
    int64_t *node;  // [V][3]
    int64_t *box;   // [nb][6] inflated lo, hi
    int64_t *W;     // [V][V]
    int32_t *flag;  // [1]
};

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

Work carve(void *base, int V, int nb)
{
    char *b = static_cast<char *>(base);
    Work w;
    w.node = reinterpret_cast<int64_t *>(b);
    b += a256(size_t(V) * 3 * 8);
    w.box = reinterpret_cast<int64_t *>(b);
    b += a256(size_t(nb > 0 ? nb : 1) * 6 * 8);
    w.W = reinterpret_cast<int64_t *>(b);
    b += a256(size_t(V) * V * 8);
    w.flag = reinterpret_cast<int32_t *>(b);
    return w;
}

// Segment u -> v against the open box (lo, hi). Along the segment
// P(s) = u + s (v - u), s in [0, 1], each axis admits an open range of s;
// the segment enters the box iff the three ranges and [0, 1] overlap.
// Ranges are kept as fractions num / den with den > 0.
__device__ bool crosses_box(const int64_t *u, const int64_t *v, const int64_t *bx)
{
    int64_t enter_n = -1, enter_d = 1, leave_n = 2, leave_d = 1;
    for (int a = 0; a < 3; ++a) {
        const int64_t lo = bx[a], hi = bx[3 + a], delta = v[a] - u[a];
        if (delta == 0) {
            if (u[a] <= lo || u[a] >= hi) return false;
            continue;
        }
        const int64_t den = delta > 0 ? delta : -delta;
        const int64_t in_n = delta > 0 ? lo - u[a] : u[a] - hi;
        const int64_t out_n = delta > 0 ? hi - u[a] : u[a] - lo;
        if (in_n * enter_d > enter_n * den) { enter_n = in_n; enter_d = den; }
        if (out_n * leave_d < leave_n * den) { leave_n = out_n; leave_d = den; }
    }
    return enter_n * leave_d < leave_n * enter_d && enter_n < enter_d && leave_n > 0;
}

// sqrt(s) rounded half up, exactly: r = floor(sqrt(s)), plus one when
// (r + 1/2)^2 <= s, i.e. 4 s >= (2 r + 1)^2.
__device__ int64_t rounded_length(int64_t dx, int64_t dy, int64_t dz)
{
    const uint64_t s = uint64_t(dx * dx + dy * dy + dz * dz);
    uint64_t r = uint64_t(sqrt(double(s)));
    while (r * r > s) --r;
    while ((r + 1) * (r + 1) <= s) ++r;
    const uint64_t twice = 2 * r + 1;
    return int64_t(4 * s >= twice * twice ? r + 1 : r);
}

__global__ void k_edges(Work w, int V, int nb)
{
    const int u = blockIdx.y, v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    int64_t cost = 0;
    if (u != v) {
        const int64_t *pu = w.node + 3 * u, *pv = w.node + 3 * v;
        bool blocked = false;
        for (int b = 0; b < nb && !blocked; ++b) blocked = crosses_box(pu, pv, w.box + 6 * b);
        cost = blocked ? kNoEdge : rounded_length(pv[0] - pu[0], pv[1] - pu[1], pv[2] - pu[2]);
    }
    w.W[size_t(u) * V + v] = cost;
}

// Relaxation through pivot k. Row k and column k do not change in this
// step (W[k][k] = 0), so every thread reads settled values.
__global__ void k_relax(int64_t *W, int V, int k)
{
    const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= V) return;
    const int64_t a = W[size_t(i) * V + k], b = W[size_t(k) * V + j];
    if (a >= kNoEdge || b >= kNoEdge) return;
    int64_t &c = W[size_t(i) * V + j];
    if (a + b < c) c = a + b;
}

__global__ void k_extract(const int64_t *W, int V, int n, int32_t *D, int32_t *flag)
{
    const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t c = W[size_t(i) * V + j];
    int32_t out;
    if (c >= kNoEdge) {
        out = kBlocked;
    } else if (c >= kBlocked) {
        out = kBlocked;
        *flag = 1;
    } else {
        out = int32_t(c);
    }
    D[size_t(i) * n + j] = out;
}

__global__ void k_clear_flag(int32_t *flag) { *flag = 0; }

}  // namespace

size_t dist_work_bytes(int32_t n, int32_t n_boxes)
{
    const size_t V = size_t(n) + 8 * size_t(n_boxes);
    return a256(V * 3 * 8) + a256(size_t(n_boxes > 0 ? n_boxes : 1) * 6 * 8) + a256(V * V * 8) + 256;
}

hipError_t build_dist(const int32_t *h_vp, int32_t n, const int32_t *h_boxes, int32_t nb,
                      int32_t clearance, int32_t *d_dist, void *d_work, hipStream_t s,
                      int *range_error)
{
    const int V = n + 8 * nb;
    Work w = carve(d_work, V, nb);
    std::vector<int64_t> node(size_t(V) * 3), box(size_t(nb > 0 ? nb : 1) * 6);
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) node[3 * i + a] = h_vp[3 * i + a];
    for (int b = 0; b < nb; ++b) {
        for (int a = 0; a < 3; ++a) {
            box[6 * b + a] = int64_t(h_boxes[6 * b + a]) - clearance;
            box[6 * b + 3 + a] = int64_t(h_boxes[6 * b + 3 + a]) + clearance;
        }
        for (int c = 0; c < 8; ++c)
            for (int a = 0; a < 3; ++a)
                node[3 * (n + 8 * b + c) + a] = box[6 * b + ((c >> a) & 1 ? 3 : 0) + a];
    }
    hipError_t e = hipMemcpyAsync(w.node, node.data(), node.size() * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w.box, box.data(), box.size() * 8, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    const dim3 blk(256);
    k_clear_flag<<<1, 1, 0, s>>>(w.flag);
    k_edges<<<dim3((V + 255) / 256, V), blk, 0, s>>>(w, V, nb);
    for (int k = n; k < V; ++k) k_relax<<<dim3((V + 255) / 256, V), blk, 0, s>>>(w.W, V, k);
    for (int k = 0; k < n; ++k) k_relax<<<dim3((V + 255) / 256, V), blk, 0, s>>>(w.W, V, k);
    k_extract<<<dim3((n + 255) / 256, n), blk, 0, s>>>(w.W, V, n, d_dist, w.flag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int32_t flag = 0;
    if ((e = hipMemcpyAsync(&flag, w.flag, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    *range_error = flag;
    return hipSuccess;
}

}  // namespace dpso
