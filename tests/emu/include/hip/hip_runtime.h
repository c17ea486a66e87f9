// Host emulation of the small part of HIP that the library's kernels and
// launchers use, for building them as ordinary x86-64 code under
// AddressSanitizer (test infrastructure; see tests/emu/build_emu.py).
//
// Every thread of a workgroup runs as a fiber on its own stack. A fiber runs
// until it reaches a point where threads interact, then yields:
//   * workgroup barriers (__syncthreads, __syncthreads_or) wait for every
//     thread of the workgroup that has not returned;
//   * wavefront operations (ballot, any, shuffles, readlane, the row rotate,
//     inverse ballot) and wavefront synchronisation points (compiler fences,
//     s_waitcnt, wave barriers) wait for every lane of the 64-lane wavefront
//     that has not returned or stopped at a workgroup barrier, and are then
//     resolved together;
//   * direct loads into LDS (global_load_lds) are queued per wavefront and
//     performed only at the next s_waitcnt whose vmcnt is 0, so a read of a
//     row buffer before that wait sees the old contents.
// Workgroups of a grid run one after another; waves of a workgroup run in an
// order chosen by EMU_ORDER (fwd, rev, or a seed for a shuffled order per
// barrier interval), so results that depend on that order reveal a missing
// barrier. Device memory is host memory; dynamic LDS is a malloc of exactly the
// requested size, so AddressSanitizer reports any access outside it.
#pragma once

#include <stddef.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <type_traits>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))
#define __restrict__ __restrict
#define HIP_SYMBOL(x) ((const void *)&(x))

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

struct uint4 { unsigned x, y, z, w; };
struct int4 { int x, y, z, w; };
inline uint4 make_uint4(unsigned a, unsigned b, unsigned c, unsigned d) { return uint4{a, b, c, d}; }
inline int4 make_int4(int a, int b, int c, int d) { return int4{a, b, c, d}; }

namespace emu {

enum Wait { kRun = 0, kWave = 1, kBarrier = 2, kDone = 3 };
enum WaveOp { kSync = 0, kBallot, kShflXor, kShflIdx, kShflUp, kReadlane, kRor1, kInvBallot, kReadFirst };

struct Lane {
    dim3 tid;
    int index = 0;     // linear thread index
    int state = kRun;
    int op = kSync;
    uint64_t a = 0, b = 0, result = 0;
    void *sp = nullptr;
    void *fake = nullptr;  // AddressSanitizer's fake stack of this fiber
    unsigned char *stack = nullptr;
    uint64_t dma_issued = 0;  // direct LDS loads this thread has issued
};

struct Dma {
    unsigned char *dst;
    const unsigned char *src;
    size_t bytes;
    int lane;      // issuing thread
    uint64_t seq;  // its issue number within that thread
};

struct BlockCtx {
    dim3 bid, bdim, gdim;
    std::vector<Lane> lanes;
    unsigned char *lds = nullptr;
    size_t lds_bytes = 0;
    std::vector<std::vector<Dma>> dma;  // per wave
    int barrier_or = 0;                 // accumulates __syncthreads_or
    int barrier_or_result = 0;
};

extern BlockCtx *g_blk;
extern Lane *g_lane;
extern std::function<void()> *g_body;

void yield_to_scheduler();
void run_grid(std::function<void()> body, dim3 grid, dim3 block, size_t dyn_lds);
void fail(const char *fmt, ...);

inline unsigned char *dyn_lds() { return g_blk->lds; }

inline uint64_t wave_op(int op, uint64_t a, uint64_t b = 0)
{
    g_lane->op = op;
    g_lane->a = a;
    g_lane->b = b;
    g_lane->state = kWave;
    yield_to_scheduler();
    return g_lane->result;
}

inline void sync_threads()
{
    g_lane->state = kBarrier;
    yield_to_scheduler();
}

template <class T>
inline uint64_t bits(T v)
{
    static_assert(sizeof(T) <= 8, "wave operand too wide");
    uint64_t u = 0;
    memcpy(&u, &v, sizeof v);
    return u;
}

template <class T>
inline T from_bits(uint64_t u)
{
    T v;
    memcpy(&v, &u, sizeof v);
    return v;
}

}  // namespace emu

#define threadIdx (::emu::g_lane->tid)
#define blockIdx (::emu::g_blk->bid)
#define blockDim (::emu::g_blk->bdim)
#define gridDim (::emu::g_blk->gdim)

inline void __syncthreads() { ::emu::sync_threads(); }
inline int __syncthreads_or(int pred)
{
    ::emu::g_blk->barrier_or |= pred != 0;
    ::emu::sync_threads();
    return ::emu::g_blk->barrier_or_result;
}

inline uint64_t __ballot(int pred) { return ::emu::wave_op(::emu::kBallot, pred != 0); }
inline int __any(int pred) { return ::emu::wave_op(::emu::kBallot, pred != 0) != 0; }

template <class T>
inline T __shfl_xor(T v, int mask, int width = 64)
{
    (void)width;
    return ::emu::from_bits<T>(::emu::wave_op(::emu::kShflXor, ::emu::bits(v), uint64_t(mask)));
}
template <class T>
inline T __shfl(T v, int src, int width = 64)
{
    (void)width;
    return ::emu::from_bits<T>(::emu::wave_op(::emu::kShflIdx, ::emu::bits(v), uint64_t(src)));
}
template <class T>
inline T __shfl_up(T v, unsigned delta, int width = 64)
{
    (void)width;
    return ::emu::from_bits<T>(::emu::wave_op(::emu::kShflUp, ::emu::bits(v), uint64_t(delta)));
}

inline int emu_amdgcn_readlane(int v, int lane)
{
    return ::emu::from_bits<int>(::emu::wave_op(::emu::kReadlane, ::emu::bits(v), uint64_t(lane)));
}
inline int emu_amdgcn_readfirstlane(int v)
{
    return ::emu::from_bits<int>(::emu::wave_op(::emu::kReadFirst, ::emu::bits(v)));
}
inline int emu_amdgcn_mov_dpp(int v, int ctrl, int, int, bool)
{
    if (ctrl != 0x13C) ::emu::fail("mov_dpp control %#x not emulated", ctrl);
    return ::emu::from_bits<int>(::emu::wave_op(::emu::kRor1, ::emu::bits(v)));
}
inline bool emu_amdgcn_inverse_ballot_w64(uint64_t mask)
{
    return ::emu::wave_op(::emu::kInvBallot, mask) != 0;
}
inline void emu_wave_sync() { ::emu::wave_op(::emu::kSync, 0); }
inline void emu_amdgcn_wave_barrier() { emu_wave_sync(); }
#define emu_amdgcn_fence(...) emu_wave_sync()

// s_waitcnt: vmcnt in bits 3:0 and 15:14 (63: no wait). At vmcnt(N) every
// direct LDS load of the calling thread but its last N lands (loads complete
// in issue order; only these loads are counted, so a wait lands no more than
// the hardware's would).
void emu_waitcnt_vmem(int keep);
inline void emu_amdgcn_s_waitcnt(int imm)
{
    const int vm = (imm & 0xF) | ((imm >> 14) & 3) << 4;
    if (vm < 63) emu_waitcnt_vmem(vm);
    emu_wave_sync();
}
// global_load_lds: lane l's `size` bytes from `src` land at lds + offset + size * l.
void emu_amdgcn_global_load_lds(const void *src, void *lds, int size, int offset, int aux);

template <class T>
inline T atomicAdd(T *p, T v) { T o = *p; *p = o + v; return o; }
inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v) { auto o = *p; *p = o + v; return o; }
template <class T>
inline T atomicMax(T *p, T v) { T o = *p; *p = o < v ? v : o; return o; }
template <class T>
inline T atomicMin(T *p, T v) { T o = *p; *p = v < o ? v : o; return o; }
template <class T>
inline T atomicExch(T *p, T v) { T o = *p; *p = v; return o; }
template <class T>
inline T atomicOr(T *p, T v) { T o = *p; *p = o | v; return o; }

inline int __ffsll(long long x) { return __builtin_ffsll(x); }
inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline uint64_t __umul64hi(uint64_t a, uint64_t b) { return uint64_t((unsigned __int128)a * b >> 64); }

template <class A, class B>
inline typename std::common_type<A, B>::type min(A a, B b)
{
    typedef typename std::common_type<A, B>::type C;
    return C(a) < C(b) ? C(a) : C(b);
}
template <class A, class B>
inline typename std::common_type<A, B>::type max(A a, B b)
{
    typedef typename std::common_type<A, B>::type C;
    return C(a) < C(b) ? C(b) : C(a);
}
inline uint32_t emu_add_sat(uint32_t a, uint32_t b)
{
    const uint64_t s = uint64_t(a) + b;
    return s > 0xFFFFFFFFull ? 0xFFFFFFFFu : uint32_t(s);
}

// ---------------------------------------------------------------- runtime

typedef int hipError_t;
constexpr hipError_t hipSuccess = 0;
constexpr hipError_t hipErrorInvalidValue = 1;
constexpr hipError_t hipErrorInvalidConfiguration = 9;
typedef void *hipStream_t;
typedef void *hipEvent_t;
typedef void *hipGraph_t;
typedef void *hipGraphExec_t;
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
enum hipStreamCaptureStatus { hipStreamCaptureStatusNone = 0, hipStreamCaptureStatusActive = 1 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1 };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };

inline const char *hipGetErrorString(hipError_t) { return "emulated HIP error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
inline hipError_t hipGetSymbolAddress(void **p, const void *sym) { *p = const_cast<void *>(sym); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t)
{
    memmove(dst, src, n);
    return hipSuccess;
}
inline hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width,
                                   size_t height, hipMemcpyKind, hipStream_t)
{
    for (size_t r = 0; r < height; ++r)
        memmove(static_cast<char *>(dst) + r * dpitch, static_cast<const char *>(src) + r * spitch, width);
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = nullptr; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
// streams and events: every launch runs to completion when it is made, so
// ordering between streams holds by construction
constexpr unsigned hipStreamNonBlocking = 1;
constexpr unsigned hipEventDisableTiming = 2;
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = nullptr; return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = nullptr; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
inline hipError_t hipStreamIsCapturing(hipStream_t, hipStreamCaptureStatus *c)
{
    *c = hipStreamCaptureStatusNone;
    return hipSuccess;
}
// kernels run as they are launched, so a capture is a no-op
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) { *g = nullptr; return hipSuccess; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t, void *, void *, size_t)
{
    *x = nullptr;
    return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }

// Largest dynamic LDS a kernel may use once allowed (gfx950: 160 KiB per
// workgroup); 64 KiB otherwise.
void emu_allow_lds(const void *kernel, int bytes);
inline hipError_t hipFuncSetAttribute(const void *kernel, hipFuncAttribute, int bytes)
{
    emu_allow_lds(kernel, bytes);
    return hipSuccess;
}
void emu_check_lds(const void *kernel, size_t bytes);

namespace emu {
template <class K, class... A>
inline void launch(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t, A... args)
{
    emu_check_lds(reinterpret_cast<const void *>(kernel), lds);
    run_grid([=]() { kernel(args...); }, grid, block, lds);
}
}  // namespace emu
