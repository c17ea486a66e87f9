// Obstacle-aware travelling costs between viewpoints (Sect. 2.2-2.3).
//
// Graph nodes are the n viewpoints followed by the 8 corners of every box
// inflated by the clearance. Two nodes are joined iff the straight segment
// between them misses the open interior of every inflated box; the edge
// costs its Euclidean length in mm rounded half up. All-pairs shortest paths
// then give the viewpoint block. Everything is exact integer arithmetic.
//
// All-pairs shortest paths: blocked Floyd-Warshall over 64 x 64 tiles of the
// node matrix (padded to a multiple of 64 with isolated nodes). Round kb
// closes the paths whose intermediate nodes lie in node block kb, in two
// launches: the tiles of block row and block column kb, each closed together
// with the diagonal tile (kb, kb) under the pivots of block kb; then every
// remaining tile (i, j) against the closed tiles (i, kb) and (kb, j). Paths found this way are those of the per-pivot algorithm, only
// grouped by blocks of pivots, so the result is the same exact matrix.
//
// Costs are uint32: finite costs are clamped to DPSO_D_INF (= 2^28 - 1; a
// finite path cost that reaches it is a range error anyway), a pair with no
// path holds 2^32 - 1, and sums saturate there (the clamped add of the
// vector unit), so "no path" absorbs every sum. Stored values are clamped
// again at least every fourth pivot; between two clampings a value is the
// cost of a path of at most four clamped pieces, so a sum of two values stays
// below 8 (2^28 - 1) < 2^32 - 1: a finite sum never saturates. Clamping
// commutes with the min-plus steps, so every cost below DPSO_D_INF is exact
// and the classes "no path" and "finite, too large" are kept apart.
#include "device.hpp"
#include "kernels.hpp"

namespace dpso {

namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;  // no path
constexpr uint32_t kCap = 268435455u;    // 2^28 - 1: the blocked-pair sentinel
constexpr int kT = 64;                   // tile edge
constexpr int kPitchT = kT + 4;          // row pitch of a transposed tile in LDS

struct Work {
    int32_t *vp;     // [n][3] viewpoints, mm
    int32_t *boxes;  // [nb][6] lo xyz, hi xyz, mm (not inflated)
    uint32_t *W;     // [Vp][Vp] path costs
    int32_t *flag;   // [1] range error
};

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

int padded(int V) { return (V + kT - 1) / kT * kT; }

Work carve(void *base, int n, int nb, int Vp)
{
    char *b = static_cast<char *>(base);
    Work w;
    w.vp = reinterpret_cast<int32_t *>(b);
    b += a256(size_t(n) * 3 * 4);
    w.boxes = reinterpret_cast<int32_t *>(b);
    b += a256(size_t(nb > 0 ? nb : 1) * 6 * 4);
    w.W = reinterpret_cast<uint32_t *>(b);
    b += a256(size_t(Vp) * Vp * 4);
    w.flag = reinterpret_cast<int32_t *>(b);
    return w;
}

// Coordinates of graph node u: a viewpoint, or corner c of inflated box b
// (bit a of c picks the high side on axis a).
__device__ inline void node_xyz(const Work &w, int n, int clearance, int u, int64_t p[3])
{
    if (u < n) {
        for (int a = 0; a < 3; ++a) p[a] = w.vp[3 * u + a];
        return;
    }
    const int b = (u - n) >> 3, c = (u - n) & 7;
    for (int a = 0; a < 3; ++a)
        p[a] = (c >> a) & 1 ? int64_t(w.boxes[6 * b + 3 + a]) + clearance
                            : int64_t(w.boxes[6 * b + a]) - clearance;
}

// Segment u -> v against the open box (lo, hi). Along the segment
// P(s) = u + s (v - u), s in [0, 1], each axis admits an open range of s;
// the segment enters the box iff the three ranges and [0, 1] overlap.
// Ranges are kept as fractions num / den with den > 0.
__device__ bool crosses_box(const int64_t *u, const int64_t *v, const int64_t *lo_hi)
{
    int64_t enter_n = -1, enter_d = 1, leave_n = 2, leave_d = 1;
    for (int a = 0; a < 3; ++a) {
        const int64_t lo = lo_hi[a], hi = lo_hi[3 + a], delta = v[a] - u[a];
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

// Edge costs of the visibility graph; padding nodes V..Vp-1 are isolated.
// Each pair u < v is tested once and written to both (u, v) and (v, u).
__global__ void k_edges(Work w, int n, int nb, int clearance, int V, int Vp)
{
    const int u = blockIdx.y, v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= Vp || v < u) return;
    uint32_t cost = 0;
    if (u != v) {
        if (v >= V) {
            cost = kNone;
        } else {
            int64_t pu[3], pv[3];
            node_xyz(w, n, clearance, u, pu);
            node_xyz(w, n, clearance, v, pv);
            bool blocked = false;
            for (int b = 0; b < nb && !blocked; ++b) {
                int64_t lh[6];
                for (int a = 0; a < 3; ++a) {
                    lh[a] = int64_t(w.boxes[6 * b + a]) - clearance;
                    lh[3 + a] = int64_t(w.boxes[6 * b + 3 + a]) + clearance;
                }
                blocked = crosses_box(pu, pv, lh);
            }
            if (blocked) {
                cost = kNone;
            } else {
                const int64_t len = rounded_length(pv[0] - pu[0], pv[1] - pu[1], pv[2] - pu[2]);
                cost = len < int64_t(kCap) ? uint32_t(len) : kCap;
            }
        }
    }
    w.W[size_t(u) * Vp + v] = cost;
    w.W[size_t(v) * Vp + u] = cost;
}

__device__ __forceinline__ uint32_t settle(uint32_t v) { return v == kNone ? kNone : min(v, kCap); }

// a + b, saturating at 2^32 - 1 (one clamped add).
__device__ __forceinline__ uint32_t add_sat(uint32_t a, uint32_t b) { return __builtin_elementwise_add_sat(a, b); }

// Thread t of 256 owns rows r0..r0+3 and columns c0..c0+3 of a tile.
__device__ __forceinline__ int own_row(int t) { return (t >> 4) * 4; }
__device__ __forceinline__ int own_col(int t) { return (t & 15) * 4; }

// Tile (bi, bj) of W into LDS, rows of 64 (coalesced 256-byte rows).
__device__ void load_tile(uint32_t (*S)[kT], const uint32_t *W, int Vp, int bi, int bj, int t)
{
    const int c = (t & 15) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = (t >> 4) + 16 * q;
        *reinterpret_cast<uint4 *>(&S[r][c]) =
            *reinterpret_cast<const uint4 *>(W + size_t(bi * kT + r) * Vp + bj * kT + c);
    }
}

// Tile (bi, bj) of W into LDS transposed: S[k][r] = W[r][k].
__device__ void load_tile_t(uint32_t (*S)[kPitchT], const uint32_t *W, int Vp, int bi, int bj)
{
    const int t = threadIdx.x, c = (t & 15) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = (t >> 4) + 16 * q;
        const uint4 v = *reinterpret_cast<const uint4 *>(W + size_t(bi * kT + r) * Vp + bj * kT + c);
        S[c][r] = v.x;
        S[c + 1][r] = v.y;
        S[c + 2][r] = v.z;
        S[c + 3][r] = v.w;
    }
}

// One tile whose operands include itself: for k = 0..63 in order,
// C[i][j] = min(C[i][j], L[i][k] + T[k][j]) where L or T is C (or both).
// At step k row k and column k of C do not change (the diagonal tile's
// D[k][k] is 0), so the reads of step k race only with writes of the values
// they read; one barrier per step orders step k's writes before step k+1's
// reads. Values are clamped after every fourth step (and so when stored at
// the end); the clamping races only with reads of values in the same class.
__device__ void closure_steps(uint32_t (*C)[kT], const uint32_t (*L)[kT], const uint32_t (*T)[kT], int t)
{
    const int r0 = own_row(t), c0 = own_col(t);
    uint32_t c[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int p = 0; p < 4; ++p) c[q][p] = C[r0 + q][c0 + p];
    for (int k4 = 0; k4 < kT; k4 += 4) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = k4 + kk;
            uint32_t l[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) l[q] = L[r0 + q][k];
            const uint4 tv = *reinterpret_cast<const uint4 *>(&T[k][c0]);
            const uint32_t tt[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    c[q][p] = min(c[q][p], add_sat(l[q], tt[p]));
                    if (kk == 3) c[q][p] = settle(c[q][p]);
                }
                *reinterpret_cast<uint4 *>(&C[r0 + q][c0]) = make_uint4(c[q][0], c[q][1], c[q][2], c[q][3]);
            }
            __syncthreads();
        }
    }
}

__device__ void store_tile(uint32_t *W, int Vp, int bi, int bj, const uint32_t (*S)[kT], int t)
{
    const int c = (t & 15) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = (t >> 4) + 16 * q;
        *reinterpret_cast<uint4 *>(W + size_t(bi * kT + r) * Vp + bj * kT + c) =
            *reinterpret_cast<const uint4 *>(&S[r][c]);
    }
}

// The diagonal tile closed over its own nodes (the whole round when the
// matrix is a single tile).
__global__ __launch_bounds__(256) void k_fw_diag(uint32_t *W, int Vp, int kb)
{
    __shared__ __align__(16) uint32_t C[kT][kT];
    load_tile(C, W, Vp, kb, kb, threadIdx.x);
    __syncthreads();
    closure_steps(C, C, C, threadIdx.x);
    store_tile(W, Vp, kb, kb, C, threadIdx.x);
}

// Round kb, first launch: blocks 0..R-2 take the tiles (kb, j) of block row
// kb, blocks R-1..2R-3 the tiles (i, kb) of block column kb (j, i != kb).
// Rows of block kb evolve under the pivots of block kb independently of the
// other rows (and columns likewise), so each block closes its own copy of the
// diagonal tile (threads 0..255) in step with its tile (threads 256..511):
// pivot k reads column k and row k of that copy, which do not change at k.
// Block 0 stores the closed diagonal tile.
__global__ __launch_bounds__(512) void k_fw_cross(uint32_t *W, int Vp, int kb, int R)
{
    __shared__ __align__(16) uint32_t C[kT][kT];
    __shared__ __align__(16) uint32_t Dg[kT][kT];
    const bool row = int(blockIdx.x) < R - 1;
    const int o = row ? int(blockIdx.x) : int(blockIdx.x) - (R - 1);
    const int other = o < kb ? o : o + 1;
    const int bi = row ? kb : other, bj = row ? other : kb;
    const int t = threadIdx.x & 255;
    const bool diag = threadIdx.x < 256;
    if (diag)
        load_tile(Dg, W, Vp, kb, kb, t);
    else
        load_tile(C, W, Vp, bi, bj, t);
    __syncthreads();
    // one call site for every thread, so all waves meet the same barriers
    uint32_t(*own)[kT] = diag ? Dg : C;
    const uint32_t(*left)[kT] = diag || row ? Dg : C;
    const uint32_t(*top)[kT] = diag || !row ? Dg : C;
    closure_steps(own, left, top, t);
    if (!diag)
        store_tile(W, Vp, bi, bj, C, t);
    else if (blockIdx.x == 0)
        store_tile(W, Vp, kb, kb, Dg, t);
}

// Round kb, third launch: every tile (i, j) with i, j != kb against the
// closed tiles (i, kb) and (kb, j). Independent of its own values, so the
// tile stays in registers; operands in LDS (the left one transposed so both
// are read as 16-byte vectors), two pivots per min3.
__global__ __launch_bounds__(256) void k_fw_rest(uint32_t *W, int Vp, int kb)
{
    __shared__ __align__(16) uint32_t At[kT][kPitchT];
    __shared__ __align__(16) uint32_t B[kT][kT];
    const int bi = int(blockIdx.y) < kb ? int(blockIdx.y) : int(blockIdx.y) + 1;
    const int bj = int(blockIdx.x) < kb ? int(blockIdx.x) : int(blockIdx.x) + 1;
    const int t = threadIdx.x, r0 = own_row(t), c0 = own_col(t);
    load_tile_t(At, W, Vp, bi, kb);
    load_tile(B, W, Vp, kb, bj, t);
    uint32_t c[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint4 v = *reinterpret_cast<const uint4 *>(W + size_t(bi * kT + r0 + q) * Vp + bj * kT + c0);
        c[q][0] = v.x; c[q][1] = v.y; c[q][2] = v.z; c[q][3] = v.w;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kT; k += 2) {
        const uint4 a0 = *reinterpret_cast<const uint4 *>(&At[k][r0]);
        const uint4 a1 = *reinterpret_cast<const uint4 *>(&At[k + 1][r0]);
        const uint4 b0 = *reinterpret_cast<const uint4 *>(&B[k][c0]);
        const uint4 b1 = *reinterpret_cast<const uint4 *>(&B[k + 1][c0]);
        const uint32_t x0[4] = {a0.x, a0.y, a0.z, a0.w}, x1[4] = {a1.x, a1.y, a1.z, a1.w};
        const uint32_t y0[4] = {b0.x, b0.y, b0.z, b0.w}, y1[4] = {b1.x, b1.y, b1.z, b1.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int p = 0; p < 4; ++p)
                c[q][p] = min(c[q][p], min(add_sat(x0[q], y0[p]), add_sat(x1[q], y1[p])));
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        *reinterpret_cast<uint4 *>(W + size_t(bi * kT + r0 + q) * Vp + bj * kT + c0) =
            make_uint4(settle(c[q][0]), settle(c[q][1]), settle(c[q][2]), settle(c[q][3]));
}

__global__ void k_extract(const uint32_t *W, int Vp, int n, int32_t *D, int32_t *flag)
{
    const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t c = W[size_t(i) * Vp + j];
    int32_t out;
    if (c == kNone) {
        out = int32_t(kCap);
    } else if (c >= kCap) {
        out = int32_t(kCap);
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
    const size_t Vp = size_t(padded(n + 8 * n_boxes));
    return a256(size_t(n) * 3 * 4) + a256(size_t(n_boxes > 0 ? n_boxes : 1) * 6 * 4) + a256(Vp * Vp * 4) + 256;
}

hipError_t build_dist(const int32_t *h_vp, int32_t n, const int32_t *h_boxes, int32_t nb,
                      int32_t clearance, int32_t *d_dist, void *d_work, hipStream_t s,
                      int *range_error)
{
    const int V = n + 8 * nb, Vp = padded(V), R = Vp / kT;
    Work w = carve(d_work, n, nb, Vp);
    hipError_t e = hipMemcpyAsync(w.vp, h_vp, size_t(n) * 3 * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && nb > 0)
        e = hipMemcpyAsync(w.boxes, h_boxes, size_t(nb) * 6 * 4, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    k_clear_flag<<<1, 1, 0, s>>>(w.flag);
    k_edges<<<dim3((Vp + 255) / 256, Vp), dim3(256), 0, s>>>(w, n, nb, clearance, V, Vp);
    for (int kb = 0; kb < R; ++kb) {
        if (R == 1) {
            k_fw_diag<<<1, 256, 0, s>>>(w.W, Vp, kb);
        } else {
            k_fw_cross<<<2 * (R - 1), 512, 0, s>>>(w.W, Vp, kb, R);
            k_fw_rest<<<dim3(R - 1, R - 1), 256, 0, s>>>(w.W, Vp, kb);
        }
    }
    k_extract<<<dim3((n + 255) / 256, n), dim3(256), 0, s>>>(w.W, Vp, n, d_dist, w.flag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int32_t flag = 0;
    if ((e = hipMemcpyAsync(&flag, w.flag, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    *range_error = flag;
    return hipSuccess;
}

}  // namespace dpso
