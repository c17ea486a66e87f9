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
#include "device.hpp"
#include "kernels.hpp"

namespace dpso {

namespace {
constexpr int kThreads = 256;
}

__global__ __launch_bounds__(kThreads) void k_2opt_rows(const int32_t *__restrict__ D, View st,
                                                        KParams kp)
{
    Hdr *h = st.hdr;
    if (h->err || h->done || !h->ee_ran) return;
    const int p = blockIdx.x, n = st.n, ns = st.ns, tid = threadIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint64_t red[kThreads / 64];
    uint16_t *x = reinterpret_cast<uint16_t *>(smem);
    int32_t *e = reinterpret_cast<int32_t *>(x + ns);
    int32_t *rows = e + ns;  // [3][ns]

    uint16_t *xg = st.X + size_t(p) * ns;
    for (int k = tid; k < n; k += kThreads) x[k] = xg[k];
    int64_t F = st.F[p];
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
    const bool better = F < st.FP[p];
    if (better)
        for (int k = tid; k < n; k += kThreads) st.P[size_t(p) * ns + k] = x[k];
    if (tid == 0) {
        st.F[p] = F;
        if (better) st.FP[p] = F;
        atomicAdd(reinterpret_cast<unsigned long long *>(&h->n_sweeps), (unsigned long long)sweeps);
        atomicAdd(reinterpret_cast<unsigned long long *>(&h->n_moves), (unsigned long long)moves);
    }
}

hipError_t launch_2opt(const int32_t *D, const View &st, const KParams &kp, hipStream_t s)
{
    const size_t lds = size_t(st.ns) * 2 + size_t(st.ns) * 4 * 4;
    hipError_t e = allow_lds(k_2opt_rows, lds);
    if (e != hipSuccess) return e;
    k_2opt_rows<<<st.S, kThreads, lds, s>>>(D, st, kp);
    return hipGetLastError();
}

}  // namespace dpso
