// Measured ceilings of the memory paths the swarm kernels use, for the
// benchmark's roofline report. Not part of the DPSO library: every entry
// point launches one micro-benchmark kernel on the caller's stream and
// returns the launch status; the caller times it with events.
//
//   ceil_l2_stream   16-byte reads streamed over an L2-resident buffer
//   ceil_l2_gather   random 4-byte reads over the same buffer (the access
//                    pattern of a distance-matrix gather straight from memory)
//   ceil_lds_gather  random 4-byte LDS reads within a 4 KB row per wave
//                    (the edge-exchange gather)
//   ceil_lds_gather16 random 2-byte LDS reads within a 2 KB row per wave
//                    (the gather of the 16-bit rows)
//   ceil_lds_write   16-byte LDS writes of whole 4 KB rows per wave (the
//                    edge-exchange row staging through registers)
//   ceil_lds_dma     rows of an L2-resident matrix loaded straight into LDS
//                    (global_load_lds_dwordx4), one wave per block and one
//                    row in flight (the edge-exchange row staging for rows
//                    that start on 16 bytes)
//   ceil_lds_dma16   the same for 2 KB rows of a 16-bit matrix (the staging
//                    of the 16-bit rows)
//
// Every kernel accumulates what it reads and stores only if the sum equals a
// value it never reaches, so the reads cannot be dropped and nothing is
// written. Argument checks keep every access inside the buffers.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 256;
constexpr int kRow = 1024;  // ints per LDS row (4 KB)
constexpr int kNever = 0x7e5a1c3b;

// Block b reads, on pass r, slice (b + 8r) mod nb. Blocks are dealt to the 8
// XCDs round-robin, so a slice is always read by the same XCD (its L2 keeps
// it) while a CU moves to a new slice every pass (no L1 reuse).
__global__ __launch_bounds__(kThreads) void k_stream(const int4 *__restrict__ buf, int slice, int reps,
                                                     int *sink)
{
    const int nb = gridDim.x;
    int acc = 0;
    for (int r = 0; r < reps; ++r) {
        const int4 *p = buf + size_t((blockIdx.x + 8 * r) % nb) * slice;
        for (int i = threadIdx.x; i < slice; i += 4 * kThreads) {  // slice % (4 * kThreads) == 0
            int4 v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = p[i + k * kThreads];
#pragma unroll
            for (int k = 0; k < 4; ++k) acc += v[k].x ^ v[k].y ^ v[k].z ^ v[k].w;
        }
    }
    if (acc == kNever) sink[blockIdx.x] = acc;
}

// Addresses come from a per-lane xorshift sequence, independent of the data,
// so many reads are in flight. words is a power of two.
__global__ __launch_bounds__(kThreads) void k_gather(const int *__restrict__ buf, uint32_t words, int reps,
                                                     int *sink)
{
    uint32_t s = (blockIdx.x * kThreads + threadIdx.x) * 2654435761u + 0x9e3779b9u;
    int acc = 0;
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            s ^= s << 13;
            s ^= s >> 17;
            s ^= s << 5;
            acc += buf[s & (words - 1)];
        }
    }
    if (acc == kNever) sink[blockIdx.x] = acc;
}

// One 4 KB row per wave; each lane holds 16 random column offsets and walks
// them with a per-pass stride, three VALU operations per read (as in the
// edge-exchange sweep, where a read costs a few VALU operations too).
__global__ __launch_bounds__(kThreads) void k_lds_gather(int reps, int *sink)
{
    __shared__ int row[kThreads / 64][kRow];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int k = l; k < kRow; k += 64) row[w][k] = k * 7 + w;
    __syncthreads();
    uint32_t s = (blockIdx.x * kThreads + threadIdx.x) * 2654435761u + 0x9e3779b9u;
    uint32_t col[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        s ^= s << 13;
        s ^= s >> 17;
        s ^= s << 5;
        col[k] = s;
    }
    int acc = 0;
    uint32_t off = 0;
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int k = 0; k < 16; ++k) acc += row[w][(col[k] + off) & (kRow - 1)];
        off += 97;
    }
    if (acc == kNever) sink[blockIdx.x * kThreads + threadIdx.x] = acc;
}

// The same with one 2 KB row of 16-bit entries per wave.
__global__ __launch_bounds__(kThreads) void k_lds_gather16(int reps, int *sink)
{
    __shared__ uint16_t row[kThreads / 64][kRow];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int k = l; k < kRow; k += 64) row[w][k] = uint16_t(k * 7 + w);
    __syncthreads();
    uint32_t s = (blockIdx.x * kThreads + threadIdx.x) * 2654435761u + 0x9e3779b9u;
    uint32_t col[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        s ^= s << 13;
        s ^= s >> 17;
        s ^= s << 5;
        col[k] = s;
    }
    int acc = 0;
    uint32_t off = 0;
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int k = 0; k < 16; ++k) acc += row[w][(col[k] + off) & (kRow - 1)];
        off += 97;
    }
    if (acc == kNever) sink[blockIdx.x * kThreads + threadIdx.x] = acc;
}

// Two 4 KB rows per wave written alternately with 16-byte stores.
__global__ __launch_bounds__(kThreads) void k_lds_write(int reps, int *sink)
{
    __shared__ int4 rows[kThreads / 64][2][kRow / 4];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    int4 v = make_int4(int(threadIdx.x), int(blockIdx.x), 1, 2);
    for (int r = 0; r < reps; ++r) {
        int4 *b = rows[w][r & 1];
#pragma unroll
        for (int k = 0; k < kRow / 4; k += 64) b[l + k] = v;
        v.x += 1;
        __asm__ volatile("" ::: "memory");  // every pass's stores are kept
    }
    __syncthreads();
    const int4 u = rows[(w + 1) & 3][1][(l * 5) & (kRow / 4 - 1)];
    if (u.x + u.y + u.z + u.w == kNever) sink[blockIdx.x * kThreads + threadIdx.x] = u.x;
}

// One wave per block, two 4 KB LDS buffers: row t + 1 is in flight while
// row t, landed, is read once. Rows r = (7 b + 13 t) mod rows; chunk indices
// are clamped to the row.
// CH chunks of 1 KB per row: a row of row_ints ints (CH = 4) or of
// 2 row_ints 16-bit entries (CH = 2).
template <int CH>
__global__ __launch_bounds__(64) void k_lds_dma(const int *__restrict__ mat, int rows, int row_ints, int reps,
                                               int *sink)
{
    typedef __attribute__((address_space(1))) const void GV;
    typedef __attribute__((address_space(3))) void LV;
    __shared__ __align__(16) int buf[2][256 * CH];
    const int l = threadIdx.x, q = row_ints / 4 - 1;
    int r = int((7ll * blockIdx.x) % rows), acc = 0;
    for (int k = 0; k < CH; ++k)
        __builtin_amdgcn_global_load_lds((GV *)(mat + size_t(r) * row_ints + 4 * min(l + 64 * k, q)),
                                         (LV *)(buf[0] + 256 * k), 16, 0, 0);
    for (int t = 0; t < reps; ++t) {
        r = (r + 13) % rows;
        for (int k = 0; k < CH; ++k)
            __builtin_amdgcn_global_load_lds((GV *)(mat + size_t(r) * row_ints + 4 * min(l + 64 * k, q)),
                                             (LV *)(buf[(t + 1) & 1] + 256 * k), 16, 0, 0);
        __builtin_amdgcn_s_waitcnt(0x0F70 | CH);  // vmcnt(CH): row t has landed
        acc += buf[t & 1][(l * 37 + t) & (256 * CH - 1)];
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0) before the buffer is refilled
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);
    if (acc == kNever) sink[blockIdx.x * 64 + l] = acc;
}

}  // namespace

extern "C" {

// buf: device, `bytes` >= 16 KB * blocks; blocks a positive multiple of 8;
// sink: device, >= blocks ints. A block's slice is bytes / blocks rounded
// down to 16 KB; reads 16 KB * (bytes / blocks / 16 KB) * blocks * reps bytes.
int ceil_l2_stream(const void *buf, size_t bytes, int blocks, int reps, int *sink, hipStream_t stream)
{
    if (!buf || !sink || blocks <= 0 || blocks % 8 != 0 || reps <= 0) return int(hipErrorInvalidValue);
    const size_t slice = bytes / 16 / size_t(blocks) / (4 * kThreads) * (4 * kThreads);
    if (slice == 0 || slice > 0x7fffffff) return int(hipErrorInvalidValue);
    k_stream<<<blocks, kThreads, 0, stream>>>(static_cast<const int4 *>(buf), int(slice), reps, sink);
    return int(hipGetLastError());
}

// buf: device, `words` ints, words a power of two; sink: >= blocks ints.
// Reads blocks * 256 * reps * 16 ints.
int ceil_l2_gather(const void *buf, uint32_t words, int blocks, int reps, int *sink, hipStream_t stream)
{
    if (!buf || !sink || blocks <= 0 || reps <= 0 || words == 0 || (words & (words - 1)) != 0)
        return int(hipErrorInvalidValue);
    k_gather<<<blocks, kThreads, 0, stream>>>(static_cast<const int *>(buf), words, reps, sink);
    return int(hipGetLastError());
}

// sink: >= blocks * 256 ints. Reads blocks * 256 * reps * 16 LDS ints.
int ceil_lds_gather(int blocks, int reps, int *sink, hipStream_t stream)
{
    if (!sink || blocks <= 0 || reps <= 0) return int(hipErrorInvalidValue);
    k_lds_gather<<<blocks, kThreads, 0, stream>>>(reps, sink);
    return int(hipGetLastError());
}

// sink: >= blocks * 256 ints. Reads blocks * 256 * reps * 16 LDS 16-bit words.
int ceil_lds_gather16(int blocks, int reps, int *sink, hipStream_t stream)
{
    if (!sink || blocks <= 0 || reps <= 0) return int(hipErrorInvalidValue);
    k_lds_gather16<<<blocks, kThreads, 0, stream>>>(reps, sink);
    return int(hipGetLastError());
}

// sink: >= blocks * 256 ints. Writes blocks * 4 * reps * 4096 LDS bytes.
int ceil_lds_write(int blocks, int reps, int *sink, hipStream_t stream)
{
    if (!sink || blocks <= 0 || reps <= 0) return int(hipErrorInvalidValue);
    k_lds_write<<<blocks, kThreads, 0, stream>>>(reps, sink);
    return int(hipGetLastError());
}

// mat: device, rows x row_ints ints, row_ints a multiple of 4 in [4, 1024];
// sink: >= blocks * 64 ints. Stages blocks * (reps + 1) rows of 4096 LDS
// bytes each (lanes past the row repeat its last 16 bytes).
int ceil_lds_dma(const void *mat, int rows, int row_ints, int blocks, int reps, int *sink, hipStream_t stream)
{
    if (!mat || !sink || rows <= 0 || blocks <= 0 || reps <= 0 || row_ints < 4 || row_ints > kRow ||
        row_ints % 4 != 0)
        return int(hipErrorInvalidValue);
    k_lds_dma<4><<<blocks, 64, 0, stream>>>(static_cast<const int *>(mat), rows, row_ints, reps, sink);
    return int(hipGetLastError());
}

// mat: device, rows x row_u16 16-bit entries, row_u16 a multiple of 8 in
// [8, 1024]; sink: >= blocks * 64 ints. Stages blocks * (reps + 1) rows of
// 2048 LDS bytes each (lanes past the row repeat its last 16 bytes).
int ceil_lds_dma16(const void *mat, int rows, int row_u16, int blocks, int reps, int *sink, hipStream_t stream)
{
    if (!mat || !sink || rows <= 0 || blocks <= 0 || reps <= 0 || row_u16 < 8 || row_u16 > 1024 ||
        row_u16 % 8 != 0)
        return int(hipErrorInvalidValue);
    k_lds_dma<2><<<blocks, 64, 0, stream>>>(static_cast<const int *>(mat), rows, row_u16 / 2, reps, sink);
    return int(hipGetLastError());
}

}  // extern "C"
