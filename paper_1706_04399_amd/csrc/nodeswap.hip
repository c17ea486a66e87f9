// Edge exchange with the node-swap neighbourhood (the edge-exchange kernel and
// pseudo code of Sect. 3.3: exchange the nodes at two positions, keep the
// best). Exchanging the labels at positions i < j changes only the closing
// edges that touch i or j (edge k joins positions k and k+1 mod n), so with
// e_k = D[x_k][x_k+1] and D symmetric:
//   j > i+1, (i, j) != (0, n-1):
//     delta = D[x_i-1][x_j] + D[x_i+1][x_j] + D[x_i][x_j-1] + D[x_i][x_j+1]
//             - e_i-1 - e_i - e_j-1 - e_j
//   j = i+1 (adjacent):   delta = D[x_i-1][x_j] + D[x_i][x_j+1] - e_i-1 - e_j
//   (0, n-1) (adjacent through the closing edge), n >= 3:
//                         delta = D[x_0][x_n-2] + D[x_1][x_n-1] - e_n-2 - e_0
//   n = 2:                delta = 0 (the same cycle)
// The most improving exchange is taken, ties to the smallest i then j: the
// minimum of the packed key (delta + 2^31) << 32 | i << 16 | j.
//
// One workgroup per particle. Row i of the neighbourhood reads the rows of
// D of x_i-1, x_i and x_i+1; they sit in LDS in a ring of four row buffers
// (label x_r in buffer r mod 4) while the row of x_i+2 is being staged into
// the fourth, so every row of D is read from memory once per sweep. Four
// LDS gathers per exchange.
#include "device.hpp"
#include "dpso.h"
#include "kernels.hpp"

namespace dpso {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void node_swap_body(const Inst &I, int p)
{
    const int32_t *__restrict__ D = I.D;
    const View st = I.st;
    const KParams kp = I.kp;
    Hdr *h = st.hdr;
    if (h->err || h->done || !h->ee_ran) return;
    const int n = st.n, ns = st.ns, tid = threadIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint64_t red[kThreads / 64];
    int32_t *rows = reinterpret_cast<int32_t *>(smem);  // [4][ns]
    int32_t *e = rows + 4 * ns;                          // [ns]
    uint16_t *x = reinterpret_cast<uint16_t *>(e + ns);  // [ns]

    uint16_t *xg = st.X + size_t(p) * ns;
    for (int k = tid; k < n; k += kThreads) x[k] = xg[k];
    int64_t F = st.F[p];
    const int64_t fp_old = st.FP[p];  // before the first barrier (thread 0 stores it at the end)
    int moves = 0, sweeps = 0;
    __syncthreads();
    for (;;) {
        ++sweeps;
        uint64_t best = ~0ull;
        if (n >= 2) {
            for (int k = tid; k < n; k += kThreads) e[k] = D[size_t(x[k]) * n + x[k + 1 < n ? k + 1 : 0]];
            // rows of x_n-1 (buffer 3, the predecessor of position 0), x_0, x_1
            for (int k = tid; k < n; k += kThreads) {
                rows[3 * ns + k] = D[size_t(x[n - 1]) * n + k];
                rows[k] = D[size_t(x[0]) * n + k];
                rows[ns + k] = D[size_t(x[1]) * n + k];
            }
            __syncthreads();
            for (int i = 0; i + 1 < n; ++i) {
                const int32_t *Rm = rows + ((i + 3) & 3) * ns;  // row of x_i-1
                const int32_t *R0 = rows + (i & 3) * ns;        // row of x_i
                const int32_t *Rp = rows + ((i + 1) & 3) * ns;  // row of x_i+1
                const int32_t em = e[i == 0 ? n - 1 : i - 1], ei = e[i];
                for (int j = i + 1 + tid; j < n; j += kThreads) {
                    const int xj = x[j], xn = x[j + 1 < n ? j + 1 : 0];
                    int32_t d;
                    if (n == 2)
                        d = 0;
                    else if (j == i + 1)
                        d = Rm[xj] + R0[xn] - em - e[j];
                    else if (i == 0 && j == n - 1)
                        d = R0[x[j - 1]] + Rp[xj] - e[j - 1] - ei;
                    else
                        d = Rm[xj] + Rp[xj] + R0[x[j - 1]] + R0[xn] - em - ei - e[j - 1] - e[j];
                    const uint64_t key = (uint64_t(uint32_t(d) + 0x80000000u) << 32) |
                                         (uint64_t(i) << 16) | uint64_t(j);
                    best = key < best ? key : best;
                }
                if (i + 2 < n) {  // row of x_i+2 into the buffer of x_i-2
                    const int32_t *src = D + size_t(x[i + 2]) * n;
                    int32_t *dst = rows + ((i + 2) & 3) * ns;
                    for (int k = tid; k < n; k += kThreads) dst[k] = src[k];
                }
                __syncthreads();
            }
        }
        best = block_min_u64(best, red);
        if (best == ~0ull) break;
        const int32_t d = int32_t(uint32_t(best >> 32) - 0x80000000u);
        if (d >= 0) break;
        const int bi = int((best >> 16) & 0xffffu), bj = int(best & 0xffffu);
        if (tid == 0) {
            const uint16_t a = x[bi];
            x[bi] = x[bj];
            x[bj] = a;
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

}  // namespace

__global__ __launch_bounds__(kThreads) void k_node_swap(Inst I) { node_swap_body(I, int(blockIdx.x)); }

__global__ __launch_bounds__(kThreads) void k_node_swap_batch(Batch B)
{
    int p;
    const int b = batch_item(B, int(blockIdx.x));
    if (b < 0) return;
    const Inst &I = batch_pick(B, b, p);
    node_swap_body(I, p);
}

hipError_t launch_node_swap(const Inst *one, const Batch &items, int grid, int max_ns, hipStream_t s)
{
    const size_t lds = size_t(max_ns) * (4 * 4 + 4 + 2);
    hipError_t e = allow_lds(k_node_swap, lds);
    if (e == hipSuccess) e = allow_lds(k_node_swap_batch, lds);
    if (e != hipSuccess || grid <= 0) return e;
    if (one)
        k_node_swap<<<grid, kThreads, lds, s>>>(*one);
    else
        k_node_swap_batch<<<grid, kThreads, lds, s>>>(items);
    return hipGetLastError();
}

}  // namespace dpso
