// Edge exchange (Sect. 3.2.3): complete 2-opt search per particle.
//
// Exchanging edges (x_i, x_i+1) and (x_j, x_j+1) by reversing x[i+1..j]
// changes the tour cost by
//   delta(i, j) = D[x_i][x_j] + D[x_i+1][x_j+1] - e_i - e_j,
//   e_k = D[x_k][x_k+1]   (indices mod n),
// over every pair of non-adjacent edges: 0 <= i, i+2 <= j <= n-1, except
// (0, n-1). The most improving exchange is taken, ties to the smallest i
// then j: the minimum of the packed key (delta + 2^31) << 32 | i << 16 | j.
//
// One workgroup per particle. Rows of D are staged in LDS in tour order:
// row x_i serves the first term and row x_i+1 the second term of row i of
// the neighbourhood; the next row is loaded while row i is evaluated
// (three row buffers in rotation), so each row of D is read from L2 once
// per sweep.
#include <algorithm>

#include "device.hpp"
#include "dpso.h"
#include "kernels.hpp"

namespace dpso {

namespace {
constexpr int kThreads = 256;
}

__device__ __forceinline__ void twoopt_rows_body(const Inst &I, int p)
{
    const int32_t *__restrict__ D = I.D;
    const View st = I.st;
    const KParams kp = I.kp;
    Hdr *h = st.hdr;
    if (h->err || h->done || !h->ee_ran) return;
    const int n = st.n, ns = st.ns, tid = threadIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint64_t red[kThreads / 64];
    uint16_t *x = reinterpret_cast<uint16_t *>(smem);
    int32_t *e = reinterpret_cast<int32_t *>(x + ns);
    int32_t *rows = e + ns;  // [3][ns]

    uint16_t *xg = st.X + size_t(p) * ns;
    for (int k = tid; k < n; k += kThreads) x[k] = xg[k];
    int64_t F = st.F[p];
    const int64_t fp_old = st.FP[p];  // before the first barrier (thread 0 stores it at the end)
    int moves = 0, sweeps = 0;
    __syncthreads();
    for (;;) {
        ++sweeps;
        uint64_t best = ~0ull;
        if (n >= 4) {
            for (int k = tid; k < n; k += kThreads)
                e[k] = D[size_t(x[k]) * n + x[k + 1 < n ? k + 1 : 0]];
            for (int k = tid; k < n; k += kThreads) {
                rows[k] = D[size_t(x[0]) * n + k];
                rows[ns + k] = D[size_t(x[1]) * n + k];
            }
            __syncthreads();
            for (int i = 0; i + 2 < n; ++i) {
                const int32_t *rA = rows + (i % 3) * ns;
                const int32_t *rB = rows + ((i + 1) % 3) * ns;
                int32_t *rN = rows + ((i + 2) % 3) * ns;
                const int32_t ei = e[i];
                const int jend = i == 0 ? n - 1 : n;
                for (int j = i + 2 + tid; j < jend; j += kThreads) {
                    const int nj = j + 1 < n ? j + 1 : 0;
                    const int32_t d = rA[x[j]] + rB[x[nj]] - ei - e[j];
                    const uint64_t key = (uint64_t(uint32_t(d) + 0x80000000u) << 32) |
                                         (uint64_t(i) << 16) | uint64_t(j);
                    best = key < best ? key : best;
                }
                if (i + 3 < n) {  // row x_i+2 is the second-term row of row i+1
                    const int32_t *src = D + size_t(x[i + 2]) * n;
                    for (int k = tid; k < n; k += kThreads) rN[k] = src[k];
                }
                __syncthreads();
            }
        }
        best = block_min_u64(best, red);
        if (best == ~0ull) break;
        const int32_t d = int32_t(uint32_t(best >> 32) - 0x80000000u);
        if (d >= 0) break;
        const int bi = int((best >> 16) & 0xffffu), bj = int(best & 0xffffu);
        const int len = bj - bi;
        for (int k = tid; k < len / 2; k += kThreads) {
            const uint16_t a = x[bi + 1 + k];
            x[bi + 1 + k] = x[bj - k];
            x[bj - k] = a;
        }
        __syncthreads();
        F += d;
        ++moves;
        if (kp.ee_max_moves > 0 && moves >= kp.ee_max_moves) break;
    }
    for (int k = tid; k < n; k += kThreads) xg[k] = x[k];
    const bool better = F < fp_old;
    if (better)
        for (int k = tid; k < n; k += kThreads) st.P[size_t(p) * ns + k] = x[k];
    if (tid == 0) {
        st.F[p] = F;
        if (better) st.FP[p] = F;
        atomicAdd(reinterpret_cast<unsigned long long *>(&h->n_sweeps), (unsigned long long)sweeps);
        atomicAdd(reinterpret_cast<unsigned long long *>(&h->n_moves), (unsigned long long)moves);
    }
}

// ------------------------------------------------------------------------
// One wavefront per particle, columns in registers.
//
// Lane l owns the columns c = l + 64 m (m < MB, n <= 64 MB). For row i of the
// neighbourhood the wave gathers g_i[c] = D[x_i+1][x_c+1] from the row of
// label x_i+1 staged in LDS: that is the second term of delta(i, c), and,
// moved one column to the right (a wave rotation by one lane through DPP, the
// column at lane 0 coming from lane 63 of the previous register), it is the
// first term D[x_i+1][x_c+1] of delta(i+1, c+1). So every D entry of the
// sweep is gathered once and each delta costs one LDS read and four VALU
// operations. Row i only touches the blocks m >= (i+2)/64 (the triangle
// j >= i+2): rows are processed in phases of 64 with the first block known
// at compile time. Each lane keeps the minimum of its columns per row; the
// best (delta, i) over rows and lanes is reduced at the end and the smallest
// j of row i attaining it is found by recomputing that row.
//
// The pair (0, n-1) is left in the search: its edges share node x_0, and for
// a symmetric D its delta is exactly 0, so it never wins against an
// improving exchange and is never applied.
//
// The global loads of the next two rows are in flight while the current row
// is evaluated; rows alternate between two LDS buffers at a fixed stride so
// the gathers use immediate offsets. A single wave owns its LDS: LDS operations
// of one wave complete in order, and a compiler fence keeps program order.
// Tuning knobs: rows of D in flight per wave (1 or 2), byte offsets of the
// gather labels packed two per register, and the occupancy the register
// allocation aims at (waves per SIMD).
#ifndef DPSO_2OPT_PREFETCH
#define DPSO_2OPT_PREFETCH 1
#endif
#ifndef DPSO_2OPT_PACK
#define DPSO_2OPT_PACK 0
#endif
#ifndef DPSO_2OPT_WAVES
#define DPSO_2OPT_WAVES 4
#endif
// Rows that start on 16 bytes (n a multiple of 4) can go from memory straight
// into LDS (global_load_lds_dwordx4: lane l's 16 bytes land at the buffer
// base + 16 l), with no registers and no LDS store instructions.
#ifndef DPSO_2OPT_DMA
#define DPSO_2OPT_DMA 1
#endif
// Rows staged as 16-bit values (see below) for the n of packed_rows(): all
// n in [8, 1024] except multiples of 4 up to 256, whose int32 rows go
// straight into LDS in one 1 KB load chunk already.
#ifndef DPSO_2OPT_HALF
#define DPSO_2OPT_HALF 1
#endif

// Packed rows. The sweep is bound by staging rows into LDS, 4n bytes each.
// With H = D >> s, s the smallest shift that brings every entry of D under
// 2^16 (0 while distances stay below 65.536 m), a row takes 2n bytes (padded
// to a multiple of 16 bytes, so rows of every n go straight into LDS). Writing
// each entry as D = 2^s h + r (h its entry of H, 0 <= r < 2^s), the sum
//   A(i, j) = H[x_i][x_j] + H[x_i+1][x_j+1] - H[x_i][x_i+1] - H[x_j][x_j+1]
// gives delta(i, j) = 2^s A(i, j) + rho with |rho| <= 2 (2^s - 1). So the
// exchange with the smallest delta, and every exchange tying with it, has
// A <= A_min + T, T = floor(4 (2^s - 1) / 2^s) (0, 2 and 3 for s = 0, 1 and
// s >= 2), and no exchange improves the tour when 2^s A_min >= 2 (2^s - 1).
// Each lane keeps the three smallest keys 1024 A + i of its row minima (a
// minimum and two medians of three per row, branch-free). At the end, with
// A_min the wave's minimum, the rows of the lane keys whose A is <= A_min + T
// are evaluated exactly from D and the smallest (delta, i, j) is taken over
// them; should a lane's third key also be in the window, every row is
// evaluated exactly. The exchange found is the one the int32 sweep finds.
namespace {

constexpr int kPrefetch = DPSO_2OPT_PREFETCH;
constexpr bool kPack = DPSO_2OPT_PACK != 0;
constexpr int kPad = 1 << 30;  // edge cost of padding columns: never the minimum
constexpr int kNone = 0x7fffffff;

__device__ inline int rotate_up(int v)  // lane l receives lane l-1 (lane 0: lane 63)
{
    return __builtin_amdgcn_mov_dpp(v, 0x13C, 0xF, 0xF, false);
}

__device__ inline void compiler_fence() { __asm__ __volatile__("" ::: "memory"); }

constexpr bool kDma = DPSO_2OPT_DMA != 0;
constexpr bool kHalf = DPSO_2OPT_HALF != 0 && kDma;

// s_waitcnt immediates (vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
__device__ inline void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)

__device__ inline void wait_lds() { __builtin_amdgcn_s_waitcnt(0xC07F); }   // lgkmcnt(0)

// LDS-address-space view of the row buffers (taken from the shared array
// itself, so no generic pointer is converted back).
typedef __attribute__((address_space(3))) int32_t lds_int;

// A row of n ints (n a multiple of 4) from memory into an LDS buffer of
// 256 R ints: chunk k of 64 x 16 bytes lands at dst + 256 k. Chunk indices
// are clamped to the row, so lanes past its end repeat the last chunk into
// the buffer's tail.
template <int R>
__device__ inline void dma_row(const int32_t *src, int n, lds_int *dst)
{
    typedef __attribute__((address_space(1))) const void GV;
    typedef __attribute__((address_space(3))) void LV;
    const int lane = threadIdx.x & 63, q = (n >> 2) - 1;
    compiler_fence();
#pragma unroll
    for (int k = 0; k < R; ++k)
        __builtin_amdgcn_global_load_lds((GV *)(src + 4 * min(lane + 64 * k, q)), (LV *)(dst + 256 * k), 16, 0, 0);
    compiler_fence();
}

// A padded row of hs uint16 (hs a multiple of 8) into an LDS buffer: the
// buffer's slot 64 k + lane (16 bytes at byte 1024 k + 16 lane of dst) takes
// chunk src_chunk[k] of the row (chunk c: bytes 16 c .. 16 c + 15, labels
// 8 c .. 8 c + 7), so a chunk can go to any slot.
template <int R>
__device__ inline void dma_half(const uint16_t *src, const int *src_chunk, lds_int *dst)
{
    typedef __attribute__((address_space(1))) const void GV;
    typedef __attribute__((address_space(3))) void LV;
    compiler_fence();
#pragma unroll
    for (int k = 0; k < R; ++k)
        __builtin_amdgcn_global_load_lds((GV *)(reinterpret_cast<const char *>(src) + 16 * src_chunk[k]),
                                         (LV *)(dst + 256 * k), 16, 0, 0);
    compiler_fence();
}

// Chunk placement for the 16-bit rows of one sweep. A row buffer's 16-byte
// slot s covers LDS banks 4 (s mod 8) .. 4 (s mod 8) + 3 (32 banks of 4 bytes,
// a wave's gather served 32 lanes at a time), so the bank of label y is
// 4 g + (y mod 8) / 2 with g the group (slot mod 8) of its chunk y / 8. The
// half-wave of lanes 32 h .. 32 h + 31 of column block m gathers, in every
// row of the sweep where that block is active, the labels x_c+1 of its 32
// columns c, a fixed set for the whole sweep; it takes as many cycles as the
// most distinct dwords any bank holds. Chunks are placed one after another
// into the group that raises the fewest half-waves' maximum load, weighted by
// the rows in which the half-wave gathers; 8 RH slots per group. Returns each
// chunk's slot (slot_of, LDS) and, per lane, the chunk each of its row loads
// fetches (src_chunk); `scratch` holds 328 MB + 256 bytes. Only the
// layout of the staged rows changes, not what is read: results are the same
// for every placement.
template <int MB>
__device__ __forceinline__ void place_chunks(const uint16_t *tour, int n, int nch, unsigned char *scratch,
                                             const unsigned char *&slot_of, int *src_chunk)
{
    constexpr int RH = (MB + 7) / 8, NHW = 2 * MB, CAP = 8 * RH;
    const int lane = threadIdx.x & 63;  // within the wave (two may share a particle)
    unsigned char *hwpos = scratch;                                             // [64 MB]
    uint32_t *load = reinterpret_cast<uint32_t *>(scratch + 64 * MB);           // [NHW][32]
    uint32_t *mx = load + NHW * 32;                                             // [NHW]
    unsigned char *slot = reinterpret_cast<unsigned char *>(mx + NHW);          // [128]
    unsigned char *chunk = slot + 128;                                          // [128]
    for (int k = lane; k < NHW * 32; k += 64) load[k] = 0u;
    if (lane < NHW) mx[lane] = 0u;
    for (int p = lane; p < n; p += 64) {
        const int c = p == 0 ? n - 1 : p - 1;  // the column whose gather reads tour[p]
        hwpos[tour[p]] = (unsigned char)(c >> 5);
    }
    compiler_fence();
    const int g = lane >> 3, r = lane & 7;
    int cnt = 0;  // chunks placed in group g (the same in g's 8 lanes)
    for (int q = 0; q < nch; ++q) {
        const int y = 8 * q + r;
        const int hw = y < n ? int(hwpos[y]) : -1 - lane;
        const int phw = __shfl_xor(hw, 1, 64);
        // y and its dword partner y ^ 1 read in one half-wave count once
        const bool live = y < n && !((r & 1) && phw == hw);
        const int cell = hw * 32 + 4 * g + (r >> 1);
        const uint32_t ld = live ? load[cell] : 0u;
        const uint32_t top = live ? mx[hw] : 1u;
        int cost = live && ld == top ? min(64 * (hw >> 1) + 62, n - 2) : 0;
        cost += __shfl_xor(cost, 1, 64);
        cost += __shfl_xor(cost, 2, 64);
        cost += __shfl_xor(cost, 4, 64);
        int key = cnt < CAP ? cost * 8 + g : 0x7fffffff;
        key = min(key, __shfl_xor(key, 8, 64));
        key = min(key, __shfl_xor(key, 16, 64));
        key = min(key, __shfl_xor(key, 32, 64));
        const int gs = __builtin_amdgcn_readfirstlane(key & 7);
        if (g == gs && live) {
            load[cell] = ld + 1u;
            atomicMax(&mx[hw], ld + 1u);
        }
        const int placed = __builtin_amdgcn_readlane(cnt, 8 * gs);
        if (lane == 0) slot[q] = (unsigned char)(gs + 8 * placed);
        cnt += g == gs;
    }
    compiler_fence();
    for (int s = lane; s < 64 * RH; s += 64) chunk[s] = 0;
    compiler_fence();
    for (int q = lane; q < nch; q += 64) chunk[slot[q]] = (unsigned char)q;
    compiler_fence();
#pragma unroll
    for (int k = 0; k < RH; ++k) src_chunk[k] = chunk[64 * k + lane];
    slot_of = slot;
}

// Row buffers: two per wave, each BS ints. Rows that do not start on 16
// bytes spill up to 3 ints before and after a buffer, so those kernels keep
// guard words around each buffer; aligned kernels keep none (10 KiB of LDS
// per wave at MB = 16: 16 waves per CU).
template <int MB, bool VEC4>
struct WaveCfg {
    static constexpr int RV = (MB + 3) / 4;  // int4 per lane per aligned row
    static constexpr int RH = (MB + 7) / 8;  // 16-byte chunks per lane per uint16 row
    static constexpr int RU = (64 * MB + 3 + 255) / 256;  // ... per row starting off 16 B
    static constexpr int BS = 256 * RV;      // row length capacity (ints) >= 64 MB >= n
    static constexpr int GUARD = VEC4 ? 0 : 4;  // ints before and after each buffer
    static constexpr int STRIDE = BS + GUARD;   // buffer k starts at GUARD + k * STRIDE
    static constexpr int LDS_INTS = GUARD + 2 * STRIDE;
};

// One row of D in flight. Rows are staged as aligned 16-byte chunks: when
// the row starts `shift` ints past a 16-byte boundary (n not a multiple of
// 4), the chunks follow the aligned-down address and each int is written to
// its own index of the LDS buffer, the few ints before 0 and past n landing
// in the buffer's guard words. Chunk indices are clamped to the row's span,
// and such rows are read int by int, only the ints of the row itself, since
// the span can run past the end of the matrix.
template <int MB, bool VEC4>
struct RowPipe {
    static constexpr int R = VEC4 ? WaveCfg<MB, VEC4>::RV : WaveCfg<MB, VEC4>::RU;
    int4 v[R];
    int shift;

    __device__ inline void load(const int32_t *__restrict__ src, int n)
    {
        const int lane = threadIdx.x & 63;
        if constexpr (VEC4) {
            const int4 *s4 = reinterpret_cast<const int4 *>(src);
            const int q = (n >> 2) - 1;
#pragma unroll
            for (int k = 0; k < R; ++k) v[k] = s4[min(lane + 64 * k, q)];
        } else {
            // the ints of the row's 16-byte span, those outside the row read
            // as 0 (the span may run past the end of the matrix)
            shift = int(reinterpret_cast<uintptr_t>(src) & 15) >> 2;
            const int q = ((shift + n + 3) >> 2) - 1;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int e = 4 * min(lane + 64 * k, q) - shift;  // row index of the chunk's first int
                v[k].x = e >= 0 && e < n ? src[e] : 0;
                v[k].y = e + 1 >= 0 && e + 1 < n ? src[e + 1] : 0;
                v[k].z = e + 2 >= 0 && e + 2 < n ? src[e + 2] : 0;
                v[k].w = e + 3 >= 0 && e + 3 < n ? src[e + 3] : 0;
            }
        }
    }

    __device__ inline void store(int32_t *dst, int n) const
    {
        const int lane = threadIdx.x & 63;
        if constexpr (VEC4) {
            int4 *d4 = reinterpret_cast<int4 *>(dst);
            const int q = (n >> 2) - 1;
#pragma unroll
            for (int k = 0; k < R; ++k) d4[min(lane + 64 * k, q)] = v[k];
        } else {
            const int q = ((shift + n + 3) >> 2) - 1;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int e = 4 * min(lane + 64 * k, q) - shift;  // in [-3, n + 3)
                dst[e] = v[k].x;
                dst[e + 1] = v[k].y;
                dst[e + 2] = v[k].z;
                dst[e + 3] = v[k].w;
            }
        }
    }
};

template <int MB, bool VEC4>
struct SweepState {
    // byte offset (4 x_c+1) of each owned column in a row buffer; packed two
    // per register when kPack
    int loff[kPack ? (MB + 1) / 2 : MB];
    int ne[MB];    // -D[x_c][x_c+1], kPad for padding columns
    int g[MB];     // gathers of the previous row
    RowPipe<MB, VEC4> pipe[kPrefetch];  // rows in flight (alternating by row parity)
    int best, best_i;
    // packed rows: the lane's three smallest keys 1024 A + i (k1 <= k2 <= k3),
    // and the chunk each of the lane's row loads fetches
    int k1, k2, k3;
    int src_chunk[(MB + 7) / 8];

    __device__ inline int off(int m) const
    {
        if constexpr (kPack) return (m & 1) ? (loff[m >> 1] >> 16) : (loff[m >> 1] & 0xffff);
        return loff[m];
    }
    __device__ inline void set_off(int m, int v)
    {
        if constexpr (kPack) {
            loff[m >> 1] = (m & 1) ? ((loff[m >> 1] & 0xffff) | (v << 16)) : v;
        } else {
            loff[m] = v;
        }
    }
};

__device__ inline int lds_word(const int32_t *base, int byte_off)
{
    return *reinterpret_cast<const int32_t *>(reinterpret_cast<const char *>(base) + byte_off);
}

// median of three (one v_med3_i32)
__device__ inline int med3(int a, int b, int c) { return max(min(a, b), min(max(a, b), c)); }

// Key of a row minimum of A: A (capped above; larger values are never in
// the window) times 1024 plus the row, so keys order by (A, row).
constexpr int kKeyCap = 1 << 20;
__device__ inline int row_key(int a, int i) { return min(a, kKeyCap) * 1024 + i; }
__device__ inline int key_value(int k) { return k >> 10; }

__device__ inline int lds_half(const int32_t *base, int byte_off)
{
    return *reinterpret_cast<const uint16_t *>(reinterpret_cast<const char *>(base) + byte_off);
}

// Row i with the first active block M0 and buffer BI (0 for even rows);
// HALF: rows of H (16-bit) instead of D.
template <int MB, bool VEC4, bool HALF, int M0, int BI>
__device__ __forceinline__ void sweep_row(SweepState<MB, VEC4> &S, const int32_t *__restrict__ D,
                                          const uint16_t *__restrict__ H, int32_t *bufs, lds_int *lbufs,
                                          const uint16_t *tour, int n, int i, int end)
{
    constexpr int ST = WaveCfg<MB, VEC4>::STRIDE;
    int32_t *cur = bufs + BI * ST;
    const int32_t *prv = bufs + (1 - BI) * ST;
    const int lane = threadIdx.x & 63;
    int ei;
    if constexpr (HALF) {
        // as below, with ne holding -H[x_c][x_c+1] and off the byte offset
        // 2 x_c+1 of a 16-bit row
        constexpr int MP = M0 > 0 ? M0 - 1 : 0;
        const int ne_lo = __builtin_amdgcn_readlane(S.ne[MP], i & 63);
        const int ne_hi = __builtin_amdgcn_readlane(S.ne[M0], i & 63);
        ei = -((M0 > 0 && (i >> 6) < M0) ? ne_lo : ne_hi);
        const int label = tour[i + 2];  // x_i+2 (its offset no longer encodes it)
        wait_vmem();
        wait_lds();
        compiler_fence();
        const int hs = packed_stride(n);
        // the next row, if this wave's rows go on (rows end before `end`)
        if (i + 1 < end) dma_half<WaveCfg<MB, VEC4>::RH>(H + size_t(label) * hs, S.src_chunk, lbufs + (1 - BI) * ST);
    } else if constexpr (kDma && VEC4) {
        // e_i = D[x_i][x_i+1] and the label x_i+2 come from the registers of
        // the lanes owning columns i and i + 1 (in this phase, blocks M0 - 1
        // or M0), not from LDS. The row of x_i+1 went into cur one row ago;
        // once it has landed, prv (read by the previous row) takes the row of
        // x_i+2.
        constexpr int MP = M0 > 0 ? M0 - 1 : 0;
        const int ne_lo = __builtin_amdgcn_readlane(S.ne[MP], i & 63);
        const int ne_hi = __builtin_amdgcn_readlane(S.ne[M0], i & 63);
        ei = -((M0 > 0 && (i >> 6) < M0) ? ne_lo : ne_hi);
        const int of_lo = __builtin_amdgcn_readlane(S.off(MP), (i + 1) & 63);
        const int of_hi = __builtin_amdgcn_readlane(S.off(M0), (i + 1) & 63);
        const int label = ((M0 > 0 && ((i + 1) >> 6) < M0) ? of_lo : of_hi) >> 2;  // x_i+2
        wait_vmem();
        wait_lds();
        compiler_fence();
        if (i + 4 <= n) dma_row<WaveCfg<MB, VEC4>::RV>(D + size_t(label) * n, n, lbufs + (1 - BI) * ST);
    } else {
        constexpr int P = kPrefetch == 2 ? BI : 0;
        S.pipe[P].store(cur, n);  // row of x_i+1, loaded kPrefetch rows ago
        if (i + kPrefetch + 3 <= n) S.pipe[P].load(D + size_t(tour[i + 1 + kPrefetch]) * n, n);
        compiler_fence();
        ei = prv[tour[i + 1]];                 // D[x_i][x_i+1]
    }
    int carry = M0 > 0 ? rotate_up(S.g[M0 > 0 ? M0 - 1 : 0]) : 0;
    int rm = kNone;
#pragma unroll
    for (int m = M0; m < MB; ++m) {
        const int r = rotate_up(S.g[m]);
        const int a = lane == 0 ? carry : r;
        carry = r;
        const int b = HALF ? lds_half(cur, S.off(m)) : lds_word(cur, S.off(m));
        int d = a + b + S.ne[m];
        if (m == M0) {
            if constexpr (HALF) {
                // lanes below i + 2 - 64 M0 (in [0, 64)) hold columns left of the triangle
                const uint64_t left = (uint64_t(1) << (i + 2 - 64 * M0)) - 1;
                d = __builtin_amdgcn_inverse_ballot_w64(left) ? kNone : d;
            } else {
                d = lane + 64 * M0 < i + 2 ? kNone : d;
            }
        }
        rm = min(rm, d);
        S.g[m] = b;
    }
    const int cand = rm - ei;
    if constexpr (HALF) {
        const int key = row_key(cand, i);
        S.k3 = med3(S.k2, S.k3, key);
        S.k2 = med3(S.k1, S.k2, key);
        S.k1 = min(S.k1, key);
    } else if (cand < S.best) {
        S.best = cand;
        S.best_i = i;
    }
}

// Rows [64 M0 - 2, 64 M0 + 62) clipped to the wave's rows [begin, end)
// (begin even; all rows [0, n - 2) for a wave alone), then the next phase.
template <int MB, bool VEC4, bool HALF, int M0>
__device__ __forceinline__ void sweep_phase(SweepState<MB, VEC4> &S, const int32_t *__restrict__ D,
                                            const uint16_t *__restrict__ H, int32_t *bufs, lds_int *lbufs,
                                            const uint16_t *tour, int n, int begin, int end)
{
    const int lo = max(M0 == 0 ? 0 : 64 * M0 - 2, begin);
    const int hi = min(64 * M0 + 62, end);
    for (int i = lo; i < hi; i += 2) {  // lo is even: row parity picks the buffer
        sweep_row<MB, VEC4, HALF, M0, 0>(S, D, H, bufs, lbufs, tour, n, i, end);
        if (i + 1 < hi) sweep_row<MB, VEC4, HALF, M0, 1>(S, D, H, bufs, lbufs, tour, n, i + 1, end);
    }
    if constexpr (M0 + 1 < MB) {
        if (hi < end) sweep_phase<MB, VEC4, HALF, M0 + 1>(S, D, H, bufs, lbufs, tour, n, begin, end);
    }
}

// The first row of wave w of the W (2 or 4) sharing a particle: the rows
// split so that each wave gets about 1/W of the triangle (row i has n - 3 - i
// columns, so wave w starts near (n - 2)(1 - sqrt((W - w) / W)): 75/256 of the
// rows for two waves; 34/256, 75/256 and 128/256 for four), rounded down to
// even; wave W starts at the end.
template <int W>
__device__ inline int wave_first_row(int n, int w)
{
    const int rows = max(n - 2, 0);
    if (w <= 0) return 0;
    if (w >= W) return rows;
    const int f = W == 2 ? 75 : w == 1 ? 34 : w == 2 ? 75 : 128;
    return ((rows * f) >> 8) & ~1;
}

}  // namespace

// W = 2 or 4 (16-bit rows only): W wavefronts share the particle, each
// sweeping its own rows (wave_first_row) with its own row buffers; the
// candidate keys and the exact minimum are combined through LDS, and the tour,
// held once, changes between workgroup barriers.
template <int MB, bool VEC4, bool HALF, int W = 1>
__device__ __forceinline__ void twoopt_wave_body(const Inst &I, int p)
{
    static_assert(W == 1 || ((W == 2 || W == 4) && HALF && VEC4), "wavefronts per particle: 16-bit rows");
    constexpr int ST = WaveCfg<MB, VEC4>::STRIDE, GU = WaveCfg<MB, VEC4>::GUARD;
    const int32_t *__restrict__ D = I.D;
    const View st = I.st;
    const KParams kp = I.kp;
    Hdr *h = st.hdr;
    if (h->err || h->done || !h->ee_ran) return;
    const int n = st.n, ns = st.ns, lane = threadIdx.x & 63, wave = W > 1 ? int(threadIdx.x >> 6) : 0;
    // the wave's rows of the neighbourhood
    const int begin = W > 1 ? wave_first_row<W>(n, wave) : 0;
    const int end = W > 1 ? wave_first_row<W>(n, wave + 1) : n - 2;
    // before the first barrier: thread 0 stores the new personal-best cost at the end
    const int64_t fp_old = W > 1 ? st.FP[p] : 0;
    const uint16_t *__restrict__ H = st.H;
    const int hs = packed_stride(n);  // row stride of H
    // packed rows: the shift, the window T and the bound 2 (2^s - 1) on |rho|
    const int shift = HALF ? pack_shift(h->dmax) : 0;
    const int window = shift == 0 ? 0 : shift == 1 ? 2 : 3;
    const int64_t rho = 2 * ((int64_t(1) << shift) - 1);
    extern __shared__ __align__(16) unsigned char smem[];
    // per wave [guard][buffer 0][guard][buffer 1][guard], buffer k at GU + k * ST;
    // then the tour
    constexpr int WAVE_INTS = GU + 2 * ST;
    int32_t *bufs = reinterpret_cast<int32_t *>(smem) + GU + wave * WAVE_INTS;
    lds_int *lbufs = (lds_int *)smem + GU + wave * WAVE_INTS;  // C-style: an address-space conversion
    uint16_t *tour = reinterpret_cast<uint16_t *>(reinterpret_cast<int32_t *>(smem) + W * WAVE_INTS);
    uint16_t *xg = st.X + size_t(p) * ns;
    for (int k = int(threadIdx.x); k < n; k += 64 * W) tour[k] = xg[k];
    compiler_fence();
    if constexpr (W > 1) __syncthreads();
    int64_t F = st.F[p];
    int moves = 0, sweeps = 0;
    while (true) {
        ++sweeps;
        if (n < 4) break;
        SweepState<MB, VEC4> S;
        S.best = kNone;
        S.best_i = 0;
        S.k1 = S.k2 = S.k3 = kNone;
        const unsigned char *slot_of = nullptr;
        if constexpr (HALF) {
            // the row buffers are free until the first row load below
            wait_lds();
            place_chunks<MB>(tour, n, hs / 8, reinterpret_cast<unsigned char *>(bufs), slot_of, S.src_chunk);
        }
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int c = lane + 64 * m;
            if (c < n) {
                const int a = tour[c], b = tour[c + 1 < n ? c + 1 : 0];
                S.set_off(m, HALF ? 16 * int(slot_of[b >> 3]) + 2 * (b & 7) : 4 * b);
                S.ne[m] = HALF ? -int(H[size_t(a) * hs + b]) : -D[size_t(a) * n + b];
            } else {
                S.set_off(m, 0);
                S.ne[m] = kPad;
            }
        }
        // g <- D[x_b][x_c+1]: the first term of the wave's first row b, one
        // column to the right
        if constexpr (HALF) {
            if (W == 1 || begin < end) {
                wait_lds();  // the placement's reads of the buffers are done
                dma_half<WaveCfg<MB, VEC4>::RH>(H + size_t(tour[begin]) * hs, S.src_chunk, lbufs + ST);
                wait_vmem();
                compiler_fence();
#pragma unroll
                for (int m = 0; m < MB; ++m) S.g[m] = lds_half(bufs + ST, S.off(m));
                dma_half<WaveCfg<MB, VEC4>::RH>(H + size_t(tour[begin + 1]) * hs, S.src_chunk, lbufs);
                sweep_phase<MB, VEC4, HALF, 0>(S, D, H, bufs, lbufs, tour, n, begin, end);
            }
        } else if constexpr (kDma && VEC4) {
            wait_lds();  // earlier reads of both buffers are done
            dma_row<WaveCfg<MB, VEC4>::RV>(D + size_t(tour[0]) * n, n, lbufs + ST);
            wait_vmem();
            compiler_fence();
#pragma unroll
            for (int m = 0; m < MB; ++m) S.g[m] = lds_word(bufs + ST, S.off(m));
            dma_row<WaveCfg<MB, VEC4>::RV>(D + size_t(tour[1]) * n, n, lbufs);
        } else {
            S.pipe[0].load(D + size_t(tour[0]) * n, n);
            S.pipe[0].store(bufs + ST, n);
            compiler_fence();
#pragma unroll
            for (int m = 0; m < MB; ++m) S.g[m] = lds_word(bufs + ST, S.off(m));
#pragma unroll
            for (int k = 0; k < kPrefetch; ++k)
                if (k + 1 < n) S.pipe[k].load(D + size_t(tour[k + 1]) * n, n);
        }
        if constexpr (!HALF) sweep_phase<MB, VEC4, HALF, 0>(S, D, H, bufs, lbufs, tour, n, 0, n - 2);
        int dbest, bi, bj;
        if constexpr (HALF) {
            int kmin = S.k1;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) kmin = min(kmin, __shfl_xor(kmin, off, 64));
            if constexpr (W > 1) {
                __shared__ int red_key[W];
                if (lane == 0) red_key[wave] = kmin;
                __syncthreads();
                kmin = red_key[0];
#pragma unroll
                for (int w = 1; w < W; ++w) kmin = min(kmin, red_key[w]);
            }
            const int amin = key_value(kmin);
            if (int64_t(amin) * (int64_t(1) << shift) >= rho) break;  // no exchange improves
            const int lim = amin + window;
            // exact (delta, i, j) over the rows left in the window
            uint64_t key = ~0ull;
            auto exact_row = [&](int r) {
                const int a0 = tour[r], a1 = tour[r + 1];
                const int er = D[size_t(a0) * n + a1];
#pragma unroll
                for (int m = 0; m < MB; ++m) {
                    const int c = lane + 64 * m;
                    if (c >= r + 2 && c < n && !(r == 0 && c == n - 1)) {
                        const int xc = tour[c], xn = tour[c + 1 < n ? c + 1 : 0];
                        const int d =
                            D[size_t(a0) * n + xc] + D[size_t(a1) * n + xn] - er - D[size_t(xc) * n + xn];
                        const uint64_t k = (uint64_t(uint32_t(d) + 0x80000000u) << 32) | (uint64_t(r) << 16) |
                                           uint64_t(c);
                        key = k < key ? k : key;
                    }
                }
            };
            if (__ballot(key_value(S.k3) <= lim)) {
                for (int r = begin; r < end; ++r) exact_row(r);  // every row of the wave
            } else {
                uint64_t rows = __ballot(key_value(S.k1) <= lim);
                while (rows) {
                    const int k = __ffsll((unsigned long long)rows) - 1;
                    rows &= rows - 1;
                    exact_row(__builtin_amdgcn_readlane(S.k1, k) & 1023);
                }
                rows = __ballot(key_value(S.k2) <= lim);
                while (rows) {
                    const int k = __ffsll((unsigned long long)rows) - 1;
                    rows &= rows - 1;
                    exact_row(__builtin_amdgcn_readlane(S.k2, k) & 1023);
                }
            }
            uint64_t win = wave_min_u64(key);
            if constexpr (W > 1) {
                __shared__ uint64_t red_win[W];
                if (lane == 0) red_win[wave] = win;
                __syncthreads();
                win = red_win[0];
#pragma unroll
                for (int w = 1; w < W; ++w) win = red_win[w] < win ? red_win[w] : win;
            }
            dbest = int(uint32_t(win >> 32) - 0x80000000u);
            if (dbest >= 0) break;
            bi = int((win >> 16) & 0xffffu);
            bj = int(win & 0xffffu);
        } else {
            // best (delta, i) of the wave, smallest i on ties
            const uint64_t key = (uint64_t(uint32_t(S.best) + 0x80000000u) << 32) | uint32_t(S.best_i);
            const uint64_t win = wave_min_u64(key);
            dbest = int(uint32_t(win >> 32) - 0x80000000u);
            if (dbest >= 0) break;
            bi = int(uint32_t(win));
            // smallest j of row bi with delta(bi, j) == dbest
            const int a0 = tour[bi], a1 = tour[bi + 1];
            const int e_bi = D[size_t(a0) * n + a1];
            bj = n;
            for (int m = 0; m < MB && bj == n; ++m) {
                const int c = lane + 64 * m;
                bool hit = false;
                if (c >= bi + 2 && c < n && !(bi == 0 && c == n - 1)) {
                    const int xc = tour[c], xn = tour[c + 1 < n ? c + 1 : 0];
                    const int d = D[size_t(a0) * n + xc] + D[size_t(a1) * n + xn] - e_bi - D[size_t(xc) * n + xn];
                    hit = d == dbest;
                }
                const uint64_t bal = __ballot(hit);
                if (bal) bj = 64 * m + __ffsll((unsigned long long)bal) - 1;
            }
        }
        // reverse tour[bi+1 .. bj]
        const int len = bj - bi;
        for (int k = int(threadIdx.x); k < len / 2; k += 64 * W) {
            const uint16_t t0 = tour[bi + 1 + k];
            tour[bi + 1 + k] = tour[bj - k];
            tour[bj - k] = t0;
        }
        compiler_fence();
        if constexpr (W > 1) __syncthreads();
        F += dbest;
        ++moves;
        if (kp.ee_max_moves > 0 && moves >= kp.ee_max_moves) break;
    }
    for (int k = int(threadIdx.x); k < n; k += 64 * W) xg[k] = tour[k];
    const bool better = F < (W > 1 ? fp_old : st.FP[p]);
    if (better)
        for (int k = int(threadIdx.x); k < n; k += 64 * W) st.P[size_t(p) * ns + k] = tour[k];
    if (threadIdx.x == 0) {
        st.F[p] = F;
        if (better) st.FP[p] = F;
        atomicAdd(reinterpret_cast<unsigned long long *>(&h->n_sweeps), (unsigned long long)sweeps);
        atomicAdd(reinterpret_cast<unsigned long long *>(&h->n_moves), (unsigned long long)moves);
    }
}

template <int MB, bool VEC4, bool HALF>
__global__ __launch_bounds__(64, DPSO_2OPT_WAVES) void k_2opt_wave(Inst I)
{
    twoopt_wave_body<MB, VEC4, HALF>(I, int(blockIdx.x));
}

template <int MB, bool VEC4, bool HALF>
__global__ __launch_bounds__(64, DPSO_2OPT_WAVES) void k_2opt_wave_batch(Batch B)
{
    int p;
    const int b = batch_item(B, int(blockIdx.x));
    if (b < 0) return;
    const Inst &I = batch_pick(B, b, p);
    twoopt_wave_body<MB, VEC4, HALF>(I, p);
}

// Two wavefronts per particle, 16-bit rows (n > 128: MB = 4, 8, 16). They are
// for launches that leave SIMDs idle, so they trade occupancy for registers:
// at least two waves per SIMD (256 VGPRs), where four would make the row loop
// spill.
#define DPSO_PAIR_WAVES 2
template <int MB>
__global__ __launch_bounds__(128, DPSO_PAIR_WAVES) void k_2opt_pair(Inst I)
{
    twoopt_wave_body<MB, true, true, 2>(I, int(blockIdx.x));
}

template <int MB>
__global__ __launch_bounds__(128, DPSO_PAIR_WAVES) void k_2opt_pair_batch(Batch B)
{
    int p;
    const int b = batch_item(B, int(blockIdx.x));
    if (b < 0) return;
    const Inst &I = batch_pick(B, b, p);
    twoopt_wave_body<MB, true, true, 2>(I, p);
}

// Four wavefronts per particle, 16-bit rows (n > 256: MB = 8, 16), for
// launches of a few hundred particles.
template <int MB>
__global__ __launch_bounds__(256, DPSO_PAIR_WAVES) void k_2opt_quad(Inst I)
{
    twoopt_wave_body<MB, true, true, 4>(I, int(blockIdx.x));
}

template <int MB>
__global__ __launch_bounds__(256, DPSO_PAIR_WAVES) void k_2opt_quad_batch(Batch B)
{
    int p;
    const int b = batch_item(B, int(blockIdx.x));
    if (b < 0) return;
    const Inst &I = batch_pick(B, b, p);
    twoopt_wave_body<MB, true, true, 4>(I, p);
}

// Instances of several 16-bit row classes (up to MBMAX columns per lane, W
// wavefronts per particle) in one launch: each workgroup runs the body of its
// own instance's class, the code it runs in that class's launch, so instances
// of different n run side by side instead of one class after another. The
// dynamic LDS is sized for MBMAX; a smaller body uses the front of it.
template <int MBMAX, int W>
__global__ __launch_bounds__(64 * W, W > 1 ? DPSO_PAIR_WAVES : DPSO_2OPT_WAVES) void k_2opt_wave_mixed(Batch B)
{
    int p;
    const int b = batch_item(B, int(blockIdx.x));
    if (b < 0) return;
    const Inst &I = batch_pick(B, b, p);
    const int n = I.st.n;  // uniform: the class bounds of exchange_class
    if constexpr (MBMAX >= 16) {
        if (n > 512) return twoopt_wave_body<16, true, true, W>(I, p);
    }
    if constexpr (MBMAX >= 8) {
        if (n > 256) return twoopt_wave_body<8, true, true, W>(I, p);
    }
    if constexpr (W == 4) {
        twoopt_wave_body<8, true, true, 4>(I, p);  // quads serve n > 256 only
    } else if constexpr (W > 1) {
        twoopt_wave_body<4, true, true, W>(I, p);  // pairs serve n > 128 only
    } else {
        if constexpr (MBMAX >= 4) {
            if (n > 128) return twoopt_wave_body<4, true, true>(I, p);
        }
        if (n > 64) return twoopt_wave_body<2, true, true>(I, p);
        twoopt_wave_body<1, true, true>(I, p);
    }
}

// Packed rows of one instance: the largest entry of D (into the header,
// cleared by the run's first launch), then H = D >> shift. Grid-stride over
// the n^2 entries; blockIdx.y picks the instance of a batch.
__device__ __forceinline__ void pack_max_body(const Inst &I)
{
    __shared__ uint32_t red[4];
    const size_t nn = size_t(I.st.n) * I.st.n;
    uint32_t mx = 0;
    for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < nn; k += size_t(gridDim.x) * blockDim.x)
        mx = max(mx, uint32_t(I.D[k]));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx = max(mx, uint32_t(__shfl_xor(int(mx), off, 64)));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < int(blockDim.x >> 6); ++w) mx = max(mx, red[w]);
        if (mx) atomicMax(&I.st.hdr->dmax, mx);
    }
}

__device__ __forceinline__ void pack_rows_body(const Inst &I)
{
    const int n = I.st.n, hs = packed_stride(n);
    const size_t total = size_t(n) * hs;
    const int shift = pack_shift(I.st.hdr->dmax);
    for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < total; k += size_t(gridDim.x) * blockDim.x) {
        const int r = int(k / hs), c = int(k - size_t(r) * hs);
        I.st.H[k] = c < n ? uint16_t(uint32_t(I.D[size_t(r) * n + c]) >> shift) : uint16_t(0);
    }
}

constexpr int kPackThreads = 256;

__global__ __launch_bounds__(kPackThreads) void k_pack_max(Inst I) { pack_max_body(I); }
__global__ __launch_bounds__(kPackThreads) void k_pack_rows(Inst I) { pack_rows_body(I); }
__global__ __launch_bounds__(kPackThreads) void k_pack_max_batch(Batch B)
{
    Inst I = B.inst[blockIdx.y];
    I.D = global_ptr(I.D);
    I.st.hdr = global_ptr(I.st.hdr);
    I.st.H = global_ptr(I.st.H);
    pack_max_body(I);
}
__global__ __launch_bounds__(kPackThreads) void k_pack_rows_batch(Batch B)
{
    Inst I = B.inst[blockIdx.y];
    I.D = global_ptr(I.D);
    I.st.hdr = global_ptr(I.st.hdr);
    I.st.H = global_ptr(I.st.H);
    pack_rows_body(I);
}

__global__ __launch_bounds__(kThreads) void k_2opt_rows(Inst I) { twoopt_rows_body(I, int(blockIdx.x)); }

__global__ __launch_bounds__(kThreads) void k_2opt_rows_batch(Batch B)
{
    int p;
    const int b = batch_item(B, int(blockIdx.x));
    if (b < 0) return;
    const Inst &I = batch_pick(B, b, p);
    twoopt_rows_body(I, p);
}

namespace {

template <int MB, bool VEC4, bool HALF = false>
hipError_t launch_wave(const Inst *one, const Batch &B, int grid, int max_ns, hipStream_t s)
{
    const size_t lds = size_t(WaveCfg<MB, VEC4>::GUARD + 2 * WaveCfg<MB, VEC4>::STRIDE) * 4 + size_t(max_ns) * 2;
    hipError_t e = allow_lds(k_2opt_wave<MB, VEC4, HALF>, lds);
    if (e == hipSuccess) e = allow_lds(k_2opt_wave_batch<MB, VEC4, HALF>, lds);
    if (e != hipSuccess || grid <= 0) return e;
    if (one)
        k_2opt_wave<MB, VEC4, HALF><<<grid, 64, lds, s>>>(*one);
    else
        k_2opt_wave_batch<MB, VEC4, HALF><<<grid, 64, lds, s>>>(B);
    return hipGetLastError();
}

template <int MBMAX, int W>
hipError_t launch_mixed(const Batch &B, int grid, int max_ns, hipStream_t s)
{
    const size_t lds = size_t(W) * (WaveCfg<MBMAX, true>::GUARD + 2 * WaveCfg<MBMAX, true>::STRIDE) * 4 +
                       size_t(max_ns) * 2;
    hipError_t e = allow_lds(k_2opt_wave_mixed<MBMAX, W>, lds);
    if (e != hipSuccess || grid <= 0) return e;
    k_2opt_wave_mixed<MBMAX, W><<<grid, 64 * W, lds, s>>>(B);
    return hipGetLastError();
}

template <int MB>
hipError_t launch_quad(const Inst *one, const Batch &B, int grid, int max_ns, hipStream_t s)
{
    const size_t lds = size_t(4) * (WaveCfg<MB, true>::GUARD + 2 * WaveCfg<MB, true>::STRIDE) * 4 +
                       size_t(max_ns) * 2;
    hipError_t e = allow_lds(k_2opt_quad<MB>, lds);
    if (e == hipSuccess) e = allow_lds(k_2opt_quad_batch<MB>, lds);
    if (e != hipSuccess || grid <= 0) return e;
    if (one)
        k_2opt_quad<MB><<<grid, 256, lds, s>>>(*one);
    else
        k_2opt_quad_batch<MB><<<grid, 256, lds, s>>>(B);
    return hipGetLastError();
}

template <int MB>
hipError_t launch_pair(const Inst *one, const Batch &B, int grid, int max_ns, hipStream_t s)
{
    const size_t lds = size_t(2) * (WaveCfg<MB, true>::GUARD + 2 * WaveCfg<MB, true>::STRIDE) * 4 +
                       size_t(max_ns) * 2;
    hipError_t e = allow_lds(k_2opt_pair<MB>, lds);
    if (e == hipSuccess) e = allow_lds(k_2opt_pair_batch<MB>, lds);
    if (e != hipSuccess || grid <= 0) return e;
    if (one)
        k_2opt_pair<MB><<<grid, 128, lds, s>>>(*one);
    else
        k_2opt_pair_batch<MB><<<grid, 128, lds, s>>>(B);
    return hipGetLastError();
}

hipError_t launch_rows(const Inst *one, const Batch &B, int grid, int max_ns, hipStream_t s)
{
    const size_t lds = size_t(max_ns) * 2 + size_t(max_ns) * 4 * 4;
    hipError_t e = allow_lds(k_2opt_rows, lds);
    if (e == hipSuccess) e = allow_lds(k_2opt_rows_batch, lds);
    if (e != hipSuccess || grid <= 0) return e;
    if (one)
        k_2opt_rows<<<grid, kThreads, lds, s>>>(*one);
    else
        k_2opt_rows_batch<<<grid, kThreads, lds, s>>>(B);
    return hipGetLastError();
}

hipError_t launch_class(int cls, const Inst *one, const Batch &B, int grid, int max_ns, hipStream_t s)
{
    switch (cls) {
    case 0: return launch_wave<1, true>(one, B, grid, max_ns, s);
    case 1: return launch_wave<2, true>(one, B, grid, max_ns, s);
    case 2: return launch_wave<4, true>(one, B, grid, max_ns, s);
    case 3: return launch_wave<8, true>(one, B, grid, max_ns, s);
    case 4: return launch_wave<16, true>(one, B, grid, max_ns, s);
    case 5: return launch_wave<1, false>(one, B, grid, max_ns, s);
    case 6: return launch_wave<2, false>(one, B, grid, max_ns, s);
    case 7: return launch_wave<4, false>(one, B, grid, max_ns, s);
    case 8: return launch_wave<8, false>(one, B, grid, max_ns, s);
    case 9: return launch_wave<16, false>(one, B, grid, max_ns, s);
    case 10: return launch_wave<1, true, true>(one, B, grid, max_ns, s);
    case 11: return launch_wave<2, true, true>(one, B, grid, max_ns, s);
    case 12: return launch_wave<4, true, true>(one, B, grid, max_ns, s);
    case 13: return launch_wave<8, true, true>(one, B, grid, max_ns, s);
    case 14: return launch_wave<16, true, true>(one, B, grid, max_ns, s);
    case 15: return launch_pair<4>(one, B, grid, max_ns, s);
    case 16: return launch_pair<8>(one, B, grid, max_ns, s);
    case 17: return launch_pair<16>(one, B, grid, max_ns, s);
    case 18: return launch_quad<8>(one, B, grid, max_ns, s);
    case 19: return launch_quad<16>(one, B, grid, max_ns, s);
    case 20: return launch_rows(one, B, grid, max_ns, s);
    default: return launch_node_swap(one, B, grid, max_ns, s);
    }
}

constexpr int kFirstHalfClass = 10;  // 16-bit rows at 1, 2, 4, 8, 16 columns per lane
constexpr int kFirstPairClass = 15;  // ... two wavefronts per particle, 4, 8, 16 columns per lane
constexpr int kFirstQuadClass = 18;  // ... four wavefronts per particle, 8, 16 columns per lane
constexpr int kRowsClass = 20;       // one workgroup per particle, int32 rows
static_assert(kExchangeClasses == kRowsClass + 2, "class table: the node-swap class last");

bool wave_half_class(int cls) { return cls >= kFirstHalfClass && cls < kFirstHalfClass + 5; }
bool pair_class(int cls) { return cls >= kFirstPairClass && cls < kFirstPairClass + 3; }
bool quad_class(int cls) { return cls >= kFirstQuadClass && cls < kFirstQuadClass + 2; }
// classes that stage 16-bit rows (their set-up packs H)
bool half_class(int cls) { return wave_half_class(cls) || pair_class(cls) || quad_class(cls); }

// blocks per instance for the packing kernels: ~16 entries per thread
int pack_blocks(int n) { return int(std::min<int64_t>(1024, (int64_t(n) * packed_stride(n) + 4095) / 4096)); }

}  // namespace

int exchange_class(int n, const int32_t *D, int neighbourhood, int rows)
{
    if (neighbourhood == DPSO_NB_NODE_SWAP) return kExchangeClasses - 1;
    if (n > 1024 || rows == DPSO_ROWS_BLOCK) return kRowsClass;
    const int mb = n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : n <= 512 ? 3 : 4;
    if (kHalf && rows == DPSO_ROWS_U16_QUAD && packed_rows(n) && n > 256) return kFirstQuadClass + mb - 3;
    if (kHalf && (rows == DPSO_ROWS_U16_PAIR || rows == DPSO_ROWS_U16_QUAD) && packed_rows(n) && n > 128)
        return kFirstPairClass + mb - 2;
    if (kHalf && (rows == DPSO_ROWS_U16 || rows == DPSO_ROWS_U16_PAIR || rows == DPSO_ROWS_U16_QUAD) &&
        packed_rows(n))
        return kFirstHalfClass + mb;
    const bool vec4 = (n & 3) == 0 && (reinterpret_cast<uintptr_t>(D) & 15) == 0;
    return vec4 ? mb : 5 + mb;
}

hipError_t launch_2opt_prepare(const Inst &I, int cls, hipStream_t s)
{
    if (!half_class(cls)) return hipSuccess;
    const dim3 grid(pack_blocks(I.st.n), 1);
    k_pack_max<<<grid, kPackThreads, 0, s>>>(I);
    k_pack_rows<<<grid, kPackThreads, 0, s>>>(I);
    return hipGetLastError();
}

hipError_t launch_batch_2opt_prepare(int cls, const Batch &members, int max_n, hipStream_t s)
{
    if (!half_class(cls) || members.count <= 0) return hipSuccess;
    const dim3 grid(pack_blocks(max_n), members.count);
    k_pack_max_batch<<<grid, kPackThreads, 0, s>>>(members);
    k_pack_rows_batch<<<grid, kPackThreads, 0, s>>>(members);
    return hipGetLastError();
}

hipError_t launch_2opt(const Inst &I, int cls, hipStream_t s)
{
    return launch_class(cls, &I, Batch{}, I.st.S, I.st.ns, s);
}

hipError_t launch_batch_2opt(int cls, const Batch &items, int total, int max_ns, hipStream_t s)
{
    return launch_class(cls, nullptr, items, total, max_ns, s);
}

int exchange_merge_group(int cls)
{
    return wave_half_class(cls) ? 1 : pair_class(cls) ? 2 : quad_class(cls) ? 3 : 0;
}

hipError_t launch_batch_2opt_mixed(int cls, const Batch &items, int total, int max_ns, hipStream_t s)
{
    if (quad_class(cls))
        return cls == kFirstQuadClass ? launch_class(cls, nullptr, items, total, max_ns, s)
                                      : launch_mixed<16, 4>(items, total, max_ns, s);
    if (pair_class(cls)) {
        switch (cls - kFirstPairClass) {
        case 0: return launch_class(cls, nullptr, items, total, max_ns, s);  // the smallest: one body
        case 1: return launch_mixed<8, 2>(items, total, max_ns, s);
        default: return launch_mixed<16, 2>(items, total, max_ns, s);
        }
    }
    if (!wave_half_class(cls)) return hipErrorInvalidValue;
    switch (cls - kFirstHalfClass) {
    case 0: return launch_class(cls, nullptr, items, total, max_ns, s);  // one column per lane: one body
    case 1: return launch_mixed<2, 1>(items, total, max_ns, s);
    case 2: return launch_mixed<4, 1>(items, total, max_ns, s);
    case 3: return launch_mixed<8, 1>(items, total, max_ns, s);
    default: return launch_mixed<16, 1>(items, total, max_ns, s);
    }
}

}  // namespace dpso
