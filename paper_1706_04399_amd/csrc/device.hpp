// Device helpers shared by the kernels: counter-based random draws and
// wavefront / workgroup reductions (64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "state.hpp"

namespace dpso {

enum Purpose : uint64_t { kInit = 0, kVel = 1, kMut = 2 };

// Philox4x64 with 10 rounds (Salmon et al., SC 2011). Counter words are
// (block, particle, generation, purpose); the key is (seed, instance).
struct Philox4 {
    uint64_t w0, w1, w2, w3;
};

__device__ __forceinline__ Philox4 philox4x64_10(uint64_t k0, uint64_t k1, uint64_t x0, uint64_t x1,
                                        uint64_t x2, uint64_t x3)
{
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
    constexpr uint64_t kMulB = 0xCA5A826395121157ull;
    constexpr uint64_t kBumpA = 0x9E3779B97F4A7C15ull;
    constexpr uint64_t kBumpB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t loA = x0 * kMulA, hiA = __umul64hi(x0, kMulA);
        const uint64_t loB = x2 * kMulB, hiB = __umul64hi(x2, kMulB);
        const uint64_t y0 = hiB ^ x1 ^ k0;
        const uint64_t y2 = hiA ^ x3 ^ k1;
        x0 = y0; x1 = loB; x2 = y2; x3 = loA;
        k0 += kBumpA;
        k1 += kBumpB;
    }
    return {x0, x1, x2, x3};
}

// Draw number i (32 bits) of the stream (particle, generation, purpose):
// block i / 8, 64-bit word (i % 8) / 2, low half for even i.
__device__ inline uint32_t draw_from_block(const Philox4 &b, int i)
{
    const int w = (i >> 1) & 3;
    const uint64_t word = w == 0 ? b.w0 : w == 1 ? b.w1 : w == 2 ? b.w2 : b.w3;
    return (i & 1) ? uint32_t(word >> 32) : uint32_t(word);
}

// Integer in [0, m): high word of d * m.
__device__ inline uint32_t scale_draw(uint32_t d, uint32_t m)
{
    return uint32_t((uint64_t(d) * uint64_t(m)) >> 32);
}

__device__ inline int64_t wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline uint64_t wave_min_u64(uint64_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ inline int wave_sum_i32(int v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Workgroup-wide reductions; `red` is LDS scratch of blockDim.x / 64 entries.
// Every thread of the workgroup must call them; all receive the result.
__device__ inline uint64_t block_min_u64(uint64_t v, uint64_t *red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_min_u64(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    uint64_t r = red[0];
    for (int w = 1; w < nw; ++w) r = red[w] < r ? red[w] : r;
    return r;
}

__device__ inline int64_t block_sum_i64(int64_t v, int64_t *red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum_i64(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    int64_t r = 0;
    for (int w = 0; w < nw; ++w) r += red[w];
    return r;
}

// Cost of a tour held in LDS (eq. min): sum of D over its n closing edges.
__device__ inline int64_t block_tour_cost(const int32_t *__restrict__ D, int n,
                                          const uint16_t *tour, int64_t *red)
{
    int64_t s = 0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const int a = tour[k], b = tour[k + 1 < n ? k + 1 : 0];
        s += D[size_t(a) * n + b];
    }
    return block_sum_i64(s, red);
}

// Marks p as pointing to global memory. A pointer loaded from memory (or
// rebuilt from an integer) has no known address space, so the compiler would
// access it with flat instructions, which also count against the LDS wait
// counter and so stall LDS work behind outstanding memory loads.
// The empty asm keeps the compiler from folding the two address-space
// casts back into the original pointer; p must be uniform (it is kept in
// scalar registers).
template <class T>
__device__ inline T *global_ptr(T *p)
{
    typedef __attribute__((address_space(1))) T GT;
    GT *g = (GT *)p;
    __asm__("" : "+s"(g));
    return (T *)g;
}

// Instance and local index of block b in a batched launch (binary search
// over the prefix table; uniform across the workgroup). The descriptor's
// pointers are returned marked as global.
// The item block b of a batched launch works on, or -1 for a block past
// the end of its XCD group (it does nothing).
__device__ inline int batch_item(const Batch &B, int b)
{
    if (B.groups == 0) return b;
    const int x = b & 7, k = b >> 3;
    return k < B.xcount[x] ? B.xbase[x] + k : -1;
}

__device__ inline Inst batch_pick(const Batch &B, int b, int &local)
{
    int lo = 0, hi = B.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (B.first[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    local = b - B.first[lo];
    Inst I = B.inst[lo];
    I.D = global_ptr(I.D);
    View &v = I.st;
    v.hdr = global_ptr(v.hdr);
    v.X = global_ptr(v.X);
    v.P = global_ptr(v.P);
    v.G = global_ptr(v.G);
    v.V = global_ptr(v.V);
    v.VL = global_ptr(v.VL);
    v.flags = global_ptr(v.flags);
    v.keep = global_ptr(v.keep);
    v.F = global_ptr(v.F);
    v.FP = global_ptr(v.FP);
    v.trace = global_ptr(v.trace);
    v.H = global_ptr(v.H);
    return I;
}

// Lets `kernel` take `bytes` of dynamic LDS (gfx950 has 160 KiB per CU).
template <typename Kernel>
inline hipError_t allow_lds(Kernel kernel, size_t bytes)
{
    if (bytes <= 60 * 1024) return hipSuccess;  // leaves room for static LDS
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

}  // namespace dpso
