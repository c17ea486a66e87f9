// Layout of the swarm state buffer in device memory.
//
// Structure-of-arrays, every region 256-byte aligned:
//   hdr    Header (generation counter, flags, global-best cost, counters)
//   X, P   uint16 [S][ns]   current and personal-best tours (ns = n rounded up
//                           to 64 labels, so each row starts 128-byte aligned)
//   V      uint16 [S][2][ns] velocity as the pair of tours (from, to) whose
//                           canonical difference to - from is the velocity, or
//                           (raw velocity) up to ns transpositions (a, b)
//   VL     int32  [S]       1 if particle p has a velocity, 0 if it is empty
//                           (raw velocity: the number of transpositions)
//   F, FP  int64  [S]       costs of X and P
//   G      uint16 [ns]      global-best tour
//   trace  int64  [cap]     global-best cost after each generation
//   flags  int32  [S]      mutation scratch: duplicate marks
//   keep   int32  [S]      mutation scratch: kept marks
//   H      uint16 [n][hs]  D >> shift with rows padded to hs = n rounded up to
//                          8 (zeros), the rows the 16-bit edge exchange stages,
//                          held when packed_rows(n) (else empty); rewritten by
//                          every run that uses it
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dpso {

constexpr uint32_t kMagic = 0x4f535044u;  // "DPSO"

struct Hdr {
    uint32_t magic;
    int32_t n, S, cap;
    int32_t t;         // generations completed
    int32_t stall;     // generations without improvement of the global best
    int32_t done;      // stop condition reached
    int32_t improved;  // global best improved in the current generation
    int32_t ee_ran;    // edge exchange runs in the current generation
    int32_t err;       // non-zero: state rejected by a kernel
    int32_t max_generations, stall_limit;
    int32_t velocity_cap;  // 0: velocity held as two tours; > 0: as a transposition list
    int64_t FG;        // cost of the global best
    uint64_t n_sweeps, n_moves, n_reshuffled;
    uint32_t dmax;     // largest entry of D, found at the start of each run
    int32_t pad;
};

// The edge exchange can stage 16-bit rows (H = D >> shift, padded rows of
// 2 hs bytes that start on 16 bytes) for these n, where a sweep fits one
// wavefront; the state holds H for them.
__host__ __device__ inline bool packed_rows(int32_t n) { return n >= 8 && n <= 1024; }

__host__ __device__ inline int32_t packed_stride(int32_t n) { return (n + 7) & ~7; }

// shift that brings the largest entry of D under 2^16
__host__ __device__ inline int pack_shift(uint32_t dmax)
{
    int bits = 0;
    while (bits < 32 && (dmax >> bits) != 0) ++bits;
    return bits > 16 ? bits - 16 : 0;
}

struct Layout {
    int32_t n, S, cap, ns;
    size_t hdr, X, P, V, VL, F, FP, G, trace, flags, keep, H, total;
};

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

inline Layout make_layout(int32_t n, int32_t S, int32_t cap)
{
    Layout L{};
    L.n = n; L.S = S; L.cap = cap;
    L.ns = (n + 63) & ~63;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    L.hdr = take(sizeof(Hdr));
    L.X = take(size_t(S) * L.ns * 2);
    L.P = take(size_t(S) * L.ns * 2);
    L.V = take(size_t(S) * L.ns * 4);
    L.VL = take(size_t(S) * 4);
    L.F = take(size_t(S) * 8);
    L.FP = take(size_t(S) * 8);
    L.G = take(size_t(L.ns) * 2);
    L.trace = take(size_t(cap) * 8);
    L.flags = take(size_t(S) * 4);
    L.keep = take(size_t(S) * 4);
    L.H = take(packed_rows(n) ? size_t(n) * packed_stride(n) * 2 : 0);
    L.total = o;
    return L;
}

// Device pointers into one state buffer.
struct View {
    Hdr *hdr;
    uint16_t *X, *P, *G;
    uint16_t *V;
    uint16_t *H;  // packed rows (see Layout), valid when packed_rows(n)
    int32_t *VL, *flags, *keep;
    int64_t *F, *FP, *trace;
    int32_t n, S, ns;
};

inline View make_view(void *base, const Layout &L)
{
    char *b = static_cast<char *>(base);
    View v;
    v.hdr = reinterpret_cast<Hdr *>(b + L.hdr);
    v.X = reinterpret_cast<uint16_t *>(b + L.X);
    v.P = reinterpret_cast<uint16_t *>(b + L.P);
    v.V = reinterpret_cast<uint16_t *>(b + L.V);
    v.VL = reinterpret_cast<int32_t *>(b + L.VL);
    v.F = reinterpret_cast<int64_t *>(b + L.F);
    v.FP = reinterpret_cast<int64_t *>(b + L.FP);
    v.G = reinterpret_cast<uint16_t *>(b + L.G);
    v.trace = reinterpret_cast<int64_t *>(b + L.trace);
    v.flags = reinterpret_cast<int32_t *>(b + L.flags);
    v.keep = reinterpret_cast<int32_t *>(b + L.keep);
    v.H = reinterpret_cast<uint16_t *>(b + L.H);
    v.n = L.n; v.S = L.S; v.ns = L.ns;
    return v;
}

// Swarm parameters as the kernels see them.
struct KParams {
    uint64_t seed, instance;
    uint32_t w_q16, phi1_q16, phi2_q16;
    int32_t mutation_period, ee_trigger, ee_max_moves, stall_limit, max_generations;
    int32_t det_count;  // number of nearest-neighbour seeded particles
    int32_t ee_neighbourhood, mutation_swaps, velocity_cap;
};

// One swarm as the kernels see it: its distance matrix, state and params.
struct Inst {
    const int32_t *D;
    View st;
    KParams kp;
    int32_t cap;  // trace capacity (max_generations + 1)
    int32_t pad;
};

// Many swarms in one launch: block b belongs to the instance i with
// first[i] <= b < first[i + 1] and handles item b - first[i] of it.
struct Batch {
    const Inst *inst;
    const int32_t *first;  // [count + 1]
    int32_t count;
    // XCD groups of a per-particle launch (groups == 8): workgroups are
    // handed to the eight XCDs in turn, so block b runs on XCD b mod 8 and
    // works on item xbase[b & 7] + (b >> 3) of that XCD's group while below
    // xcount[b & 7]; the members of a group are contiguous in the table, so
    // each instance's particles share one XCD's L2. groups == 0: block b is
    // item b.
    int32_t groups;
    int32_t xbase[8], xcount[8];
};

}  // namespace dpso
