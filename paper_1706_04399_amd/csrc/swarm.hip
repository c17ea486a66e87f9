// Swarm kernels of the enhanced DPSO (pseudo code of Sect. 3.3): initial
// tours, the velocity/position move, random mutation, the global-best
// reduction and the per-generation control step.
//
// Every kernel of a generation reads the generation counter and the stop
// flags from the state header on the device, so a whole run is enqueued
// without any host round trip.
#include <algorithm>

#include "device.hpp"
#include "kernels.hpp"

namespace dpso {

namespace {

__device__ inline bool mutation_generation(const KParams &kp, int t)
{
    return kp.mutation_period > 0 && t % kp.mutation_period == 0;
}

// Fisher-Yates shuffle of the identity into `tour` (LDS) with the stream
// (p, t, purpose): for i = n-1 down to 1 exchange places i and j_i =
// uniform(i+1), uniform(m) being the high word of draw * m.
//
// The exchanges are not replayed one by one. Step i fixes place i for good,
// so tour[i] is what place j_i holds just before step i. Let T(q) be the set
// of steps i > q with j_i = q, and W(i) what place i holds just before step i
// (for i = 0: at the end). Place q starts as q and, at each step of T(q) in
// decreasing order, hands its content to that step's place and takes that
// place's content W(step). Hence
//   W(i)    = W(min T(i)), or i when T(i) is empty;
//   tour[i] = W(i) if j_i = i (and for i = 0); otherwise W(u) with u the
//             smallest step of T(j_i) above i, or j_i when there is none.
// The sets T(q) are built as per-place lists with LDS atomic exchanges (their
// order does not matter: only minima are taken; a set has about ln(n / q)
// members), and the chains of W are resolved by pointer jumping.
// `work` holds 14 * ns bytes.
constexpr uint16_t kNone = 0xffffu;

__device__ __forceinline__ void fisher_yates(uint16_t *tour, unsigned char *work, int n, int ns,
                                             const KParams &kp, int p, int t, uint64_t purpose)
{
    uint32_t *head = reinterpret_cast<uint32_t *>(work);
    uint16_t *jv = reinterpret_cast<uint16_t *>(work + size_t(ns) * 4);
    uint16_t *nxt = jv + ns, *up = nxt + ns, *wa = up + ns, *wb = wa + ns;
    for (int q = threadIdx.x; q < n; q += blockDim.x) head[q] = kNone;
    if (threadIdx.x == 0) jv[0] = 0;
    // step i uses draw n-1-i of the stream
    const int nblk = (n - 1 + 7) / 8;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        const Philox4 r = philox4x64_10(kp.seed, kp.instance, uint64_t(b), uint64_t(p), uint64_t(t), purpose);
        for (int k = 0; k < 8; ++k) {
            const int i = n - 1 - (b * 8 + k);
            if (i >= 1) jv[i] = uint16_t(scale_draw(draw_from_block(r, k), uint32_t(i + 1)));
        }
    }
    __syncthreads();
    for (int i = threadIdx.x + 1; i < n; i += blockDim.x)
        if (jv[i] < i) nxt[i] = uint16_t(atomicExch(head + jv[i], uint32_t(i)));
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        uint32_t m = kNone;
        for (uint32_t c = head[i]; c != kNone; c = nxt[c]) m = min(m, c);
        wa[i] = m == kNone ? uint16_t(i) : uint16_t(m);
        uint32_t u = kNone;
        const uint32_t q = jv[i];
        if (q < uint32_t(i))
            for (uint32_t c = head[q]; c != kNone; c = nxt[c])
                if (c > uint32_t(i)) u = min(u, c);
        up[i] = uint16_t(u);
    }
    __syncthreads();
    // every chain i -> min T(i) -> ... ends at a place with empty T; at most
    // ceil(log2 n) + 1 rounds
    for (int round = 0; round < 16; ++round) {
        int changed = 0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const uint16_t a = wa[i], c = wa[a];
            wb[i] = c;
            changed |= c != a;
        }
        uint16_t *tmp = wa; wa = wb; wb = tmp;
        if (!__syncthreads_or(changed)) break;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const uint16_t q = jv[i];
        tour[i] = (i == 0 || q == i) ? wa[i] : up[i] != kNone ? wa[up[i]] : q;
    }
    __syncthreads();
}

// Disturbance by k exchanges of the positions (uniform(n), uniform(n)),
// drawn in that order from the stream (p, t, purpose) and applied one after
// another: the mutation text's reading of a perturbation in randomly chosen
// dimensions. The workgroup draws 1024 exchanges at a time into `draws`
// (LDS, 2048 entries); one thread applies them in order.
__device__ __forceinline__ void disturb(uint16_t *tour, uint32_t *draws, int n, int k, const KParams &kp,
                                        int p, int t, uint64_t purpose)
{
    constexpr int kChunk = 1024;
    for (int a0 = 0; a0 < k; a0 += kChunk) {
        const int m = min(kChunk, k - a0), b0 = a0 / 4;  // 2 draws per exchange, 8 per block
        __syncthreads();                                // the previous chunk is applied
        for (int b = threadIdx.x; b < (2 * m + 7) / 8; b += blockDim.x) {
            const Philox4 r = philox4x64_10(kp.seed, kp.instance, uint64_t(b0 + b), uint64_t(p), uint64_t(t), purpose);
            for (int i = 0; i < 8; ++i)
                if (b * 8 + i < 2 * m) draws[b * 8 + i] = draw_from_block(r, i);
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int a = 0; a < m; ++a) {
                const int i = int(scale_draw(draws[2 * a], uint32_t(n)));
                const int j = int(scale_draw(draws[2 * a + 1], uint32_t(n)));
                const uint16_t v = tour[i];
                tour[i] = tour[j];
                tour[j] = v;
            }
    }
    __syncthreads();
}

// Writes a tour of LDS into X (and P), its cost into F (and FP); returns
// the cost to every thread.
__device__ __forceinline__ int64_t store_particle(const int32_t *__restrict__ D, View st, int p, const uint16_t *tour,
                                  bool also_pbest, int64_t *red)
{
    const int n = st.n;
    uint16_t *x = st.X + size_t(p) * st.ns;
    uint16_t *pb = st.P + size_t(p) * st.ns;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        x[k] = tour[k];
        if (also_pbest) pb[k] = tour[k];
    }
    const int64_t c = block_tour_cost(D, n, tour, red);
    if (threadIdx.x == 0) {
        st.F[p] = c;
        if (also_pbest) st.FP[p] = c;
        st.VL[p] = 0;
    }
    return c;
}

}  // namespace

// Header of a freshly initialised state.
__device__ __forceinline__ void hdr_init_body(const Inst &I)
{
    const View st = I.st;
    const int32_t cap = I.cap, max_generations = I.kp.max_generations, stall_limit = I.kp.stall_limit;
    Hdr *h = st.hdr;
    h->magic = kMagic;
    h->n = st.n;
    h->S = st.S;
    h->cap = cap;
    h->t = 0;
    h->stall = 0;
    h->done = max_generations == 0;
    h->improved = 0;
    h->ee_ran = 0;
    h->err = 0;
    h->max_generations = max_generations;
    h->stall_limit = stall_limit;
    h->velocity_cap = I.kp.velocity_cap;
    h->FG = 0;
    h->n_sweeps = h->n_moves = h->n_reshuffled = 0;
}

// Rejects a state whose header does not match the call.
__device__ __forceinline__ void hdr_check_body(const Inst &I)
{
    Hdr *h = I.st.hdr;
    if (h->magic != kMagic || h->n != I.st.n || h->S != I.st.S || h->cap != I.cap ||
        (h->velocity_cap > 0) != (I.kp.velocity_cap > 0))
        h->err = 1;
    if (threadIdx.x == 0) h->dmax = 0;  // the run's packed rows start from here
}

// One workgroup per particle. Particles below det_count take the
// nearest-neighbour tour from start floor(p * n / det_count): always the
// closest unvisited label, the smallest label on ties (the argmin runs over
// the packed key (distance, label)). The others take a Fisher-Yates shuffle
// of stream (p, 0, init). Velocities start empty, P = X.
__device__ __forceinline__ void init_body(const Inst &I, int p)
{
    const int32_t *__restrict__ D = I.D;
    const View st = I.st;
    const KParams kp = I.kp;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint64_t red64[4];
    __shared__ int64_t redi[4];
    const int n = st.n;
    uint16_t *tour = reinterpret_cast<uint16_t *>(smem);
    if (p < kp.det_count) {
        uint8_t *seen = smem + size_t(st.ns) * 2;
        int cur = int(int64_t(p) * n / kp.det_count);
        for (int k = threadIdx.x; k < n; k += blockDim.x) seen[k] = 0;
        __syncthreads();
        if (threadIdx.x == 0) {
            seen[cur] = 1;
            tour[0] = uint16_t(cur);
        }
        __syncthreads();
        for (int s = 1; s < n; ++s) {
            uint64_t best = ~0ull;
            const int32_t *row = D + size_t(cur) * n;
            for (int k = threadIdx.x; k < n; k += blockDim.x)
                if (!seen[k]) {
                    const uint64_t key = (uint64_t(uint32_t(row[k])) << 32) | uint32_t(k);
                    best = key < best ? key : best;
                }
            best = block_min_u64(best, red64);
            cur = int(uint32_t(best));
            if (threadIdx.x == 0) {
                seen[cur] = 1;
                tour[s] = uint16_t(cur);
            }
            __syncthreads();
        }
    } else {
        fisher_yates(tour, smem + size_t(st.ns) * 2, n, st.ns, kp, p, 0, kInit);
    }
    store_particle(D, st, p, tour, true, redi);
}

// ------------------------------------------------------------------ move
//
// Move of one particle (eq. velocity, eq. position):
//   b = P - x, c = G - x (canonical differences: scanning positions left to
//   right, each position holding the wrong label gets the right one by
//   exchanging the two labels), y = x + first k_w of v + first k_1 of b +
//   first k_2 of c, v <- y - x, x <- y; new cost; personal best on strict
//   improvement. k_w = floor(w |v|), k_i = floor(phi_i r_i |.|) clamped to
//   the list length, in Q16, r_i the top 16 bits of draws 0, 1 of stream
//   (p, t, vel).
//
// Nothing here scans serially. With rho(p) = position in `from` of the
// label to[p], the canonical difference exchanges labels exactly at the
// positions that are not the largest of their rho-cycle, in increasing order
// (so its length is n minus the number of cycles). After its first k
// exchanges the first k such positions hold to[p], and every other position
// s holds from[rho(r)] for the nearest predecessor r of s along rho that is
// not among them. Cycle maxima and nearest predecessors are found by pointer
// jumping (ceil(log2 n) rounds). A prefix of label exchanges acts on labels,
// so it is the label map from[q] -> cur[q] and applies to any tour; the
// three prefixes compose into y[p] = cc(cb(cw(x[p]))).
//
// A velocity is stored as the pair of tours (from, to) = (x before, y after
// the move); its transposition list is the canonical to - from.
namespace {

// Threads per particle of the move (TPB, a template argument): 64, 128, 256
// or 512; every loop takes EPT = ceil(ns / TPB) positions per thread.
constexpr int kMaxMoveThreads = 256;
constexpr uint16_t kEmit = 1u << 14;   // in rho[p]: p is not the largest of its cycle
constexpr uint16_t kFixed = 1u << 15;  // in rho[p]: p is among the first k of those
constexpr uint16_t kLabel = 0x0fff;    // labels and positions (n <= 4096)

// LDS of one particle (nl = n rounded up to 8): six uint16 arrays and two
// uint32 pointer-jumping buffers, 20 nl bytes. from / posf (the stored
// velocity's tours, used first) and x / posx (used after) share slots, so
// eight 1000-viewpoint particles fit in a CU's LDS.
struct MoveLds {
    uint16_t *x, *posx, *from, *posf, *to, *rho, *cur, *z;
    uint32_t *e0, *e1;
    int *wsum;   // 8 per-wave sums
    int *vote;   // 3 rotating flags of vote_any
    int round;   // vote count so far (identical in every thread)
};

// Workgroup-wide "is pred true anywhere", with one barrier: waves holding a
// true lane set flag r % 3, everyone reads it after the barrier, and thread 0
// clears the flag of the previous vote, which nobody reads or writes again
// before the next barrier.
__device__ inline bool vote_any(MoveLds &L, bool pred)
{
    int *flag = L.vote + L.round;
    if (__ballot(pred) != 0 && (threadIdx.x & 63) == 0) *flag = 1;
    __syncthreads();
    const bool any = *flag != 0;
    if (threadIdx.x == 0) L.vote[L.round == 0 ? 2 : L.round - 1] = 0;
    L.round = L.round == 2 ? 0 : L.round + 1;
    return any;
}

__device__ MoveLds carve_move_lds(unsigned char *base, int nl)
{
    MoveLds L;
    uint16_t *u = reinterpret_cast<uint16_t *>(base);
    uint16_t **slots[] = {&L.x, &L.posx, &L.to, &L.rho, &L.cur, &L.z};
    for (uint16_t **s : slots) {
        *s = u;
        u += nl;
    }
    L.from = L.x;
    L.posf = L.posx;
    L.e0 = reinterpret_cast<uint32_t *>(u);  // 12 nl bytes in: 16-byte aligned
    L.e1 = L.e0 + nl;
    L.wsum = reinterpret_cast<int *>(L.e1 + nl);
    L.vote = L.wsum + 8;
    L.round = 0;
    return L;
}

// Exclusive prefix count of the kEmit marks of rho[0..n) into rank[];
// returns the total. Each thread takes a contiguous chunk.
template <int TPB>
__device__ __forceinline__ int block_rank(const uint16_t *rho, uint16_t *rank, int n, int *wsum)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int chunk = (n + TPB - 1) / TPB;
    const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
    int c = 0;
    for (int p = lo; p < hi; ++p) c += (rho[p] & kEmit) != 0;
    int incl = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int base = 0, total = 0;
    for (int w = 0; w < TPB / 64; ++w) {
        base += w < wave ? wsum[w] : 0;
        total += wsum[w];
    }
    int run = base + incl - c;
    for (int p = lo; p < hi; ++p) {
        rank[p] = uint16_t(run);
        run += (rho[p] & kEmit) != 0;
    }
    __syncthreads();
    return total;
}

// The move kernel's loops visit the positions tid, tid + TPB, ... of one
// thread; EPT (elements per thread, ceil(ns / TPB) rounded up to a power of
// two) is a compile-time bound, so every loop is unrolled and the LDS reads of
// a pointer-jumping round are all in flight together.
#define DPSO_EACH(p)                                                                   \
    _Pragma("unroll") for (int e_ = 0, p = int(threadIdx.x); e_ < EPT; ++e_, p += TPB) \
        if (p < n)

// cur <- from + (first k transpositions of the canonical to - from), with
// k = pick(length). posf is the inverse of from. Returns the length, or -1
// when `whole` says the prefix is the whole list whatever its length (then
// cur = to and nothing else is computed).
template <int TPB, int EPT, class Pick>
__device__ __forceinline__ int partial_toward(const uint16_t *from, const uint16_t *posf, const uint16_t *to, int n,
                              Pick pick, bool whole, MoveLds &L)
{
    if (whole) {
        DPSO_EACH(p) L.cur[p] = to[p];
        __syncthreads();
        return -1;
    }
    uint32_t *ea = L.e0, *eb = L.e1;
    // (jump target, largest position seen) packed in one word; the window
    // starts as {p} and doubles every round. A thread keeps its own words in
    // registers; the buffers only serve the other threads' reads.
    uint32_t e[EPT];
    DPSO_EACH(p)
    {
        const uint16_t r = posf[to[p]];
        L.rho[p] = r;
        e[e_] = uint32_t(r) | (uint32_t(p) << 16);
        ea[p] = e[e_];
    }
    __syncthreads();
    // Stop when no window maximum grows: then every window's maximum equals
    // the next window's along the jumps, i.e. the whole cycle's maximum.
    for (int span = 1; span < n; span <<= 1) {
        uint32_t f[EPT];
        int grew = 0;
        DPSO_EACH(p) f[e_] = ea[e[e_] & 0xffffu];
        DPSO_EACH(p)
        {
            const uint32_t m = max(e[e_] >> 16, f[e_] >> 16);
            grew |= m != (e[e_] >> 16);
            e[e_] = (f[e_] & 0xffffu) | (m << 16);
            eb[p] = e[e_];
        }
        uint32_t *t = ea; ea = eb; eb = t;
        if (!vote_any(L, grew != 0)) break;
    }
    DPSO_EACH(p)
    if ((e[e_] >> 16) != uint32_t(p)) L.rho[p] |= kEmit;
    __syncthreads();
    uint16_t *rank = reinterpret_cast<uint16_t *>(eb);  // eb is free here
    const int len = block_rank<TPB>(L.rho, rank, n, L.wsum);
    const int k = pick(len);
    if (k <= 0 || k >= len) {
        const uint16_t *src = k <= 0 ? from : to;
        DPSO_EACH(p) L.cur[p] = src[p];
        __syncthreads();
        return len;
    }
    DPSO_EACH(p)
    if ((L.rho[p] & kEmit) && rank[p] < k) L.rho[p] |= kFixed;
    __syncthreads();
    // (successor, successor is fixed) packed in 16 bits; jump over fixed
    // successors until every pointer lands on an unfixed position. Every
    // cycle keeps its largest position unfixed, so ceil(log2 n) + 1 rounds
    // suffice; the cap only bounds the loop on a corrupted state.
    uint16_t *ja = reinterpret_cast<uint16_t *>(ea), *jb = reinterpret_cast<uint16_t *>(eb);
    uint16_t j[EPT];
    DPSO_EACH(p)
    {
        const uint16_t r = L.rho[p] & kLabel;
        j[e_] = r | (L.rho[r] & kFixed);
        ja[p] = j[e_];
    }
    __syncthreads();
    for (int round = 0; round < 20; ++round) {
        int pending = 0;
        DPSO_EACH(p)
        {
            if (j[e_] & kFixed) j[e_] = ja[j[e_] & kLabel];
            pending |= j[e_] & kFixed;
        }
        DPSO_EACH(p) jb[p] = j[e_];
        uint16_t *t = ja; ja = jb; jb = t;
        if (!vote_any(L, pending != 0)) break;
    }
    DPSO_EACH(p)
    {
        const uint16_t r = L.rho[p];
        if (r & kFixed)
            L.cur[p] = to[p];
        else
            L.cur[j[e_] & kLabel] = from[r & kLabel];
    }
    __syncthreads();
    return len;
}

__device__ inline int prefix_count(uint64_t coef_q16, uint64_t r16, int len)
{
    const uint64_t k = (coef_q16 * r16 * uint64_t(len)) >> 32;
    return k < uint64_t(len) ? int(k) : len;
}

}  // namespace

// The default move's arrays (+ sums, votes) or the raw-velocity move's 15 ns.
size_t move_lds_bytes(int n, int ns)
{
    const size_t nl = (size_t(n) + 7) & ~size_t(7);
    return std::max(nl * 2 * 6 + nl * 4 * 2 + 64, size_t(ns) * 15);
}

// The move with the velocity kept as the raw concatenation of eq. velocity
// (velocity_cap > 0): y as in the default move, and the new velocity is the
// list of the transpositions applied, in order (the stored velocity's
// prefix, then the prefixes of P - x and G - x), truncated to velocity_cap.
// The lists are walked in order, so one lane does the walking: wave 0 stages
// the tours in LDS, lane 0 applies the stored prefix, counts the cycles of
// each difference (its length is n minus that count) and scans the canonical
// difference up to its prefix length, appending and applying each emitted
// transposition; the other waves leave at once (no workgroup barrier here).
__device__ __forceinline__ void move_raw_body(const Inst &I, int part)
{
    if (threadIdx.x >= 64) return;
    const int32_t *__restrict__ D = I.D;
    const View st = I.st;
    const KParams kp = I.kp;
    const int t = st.hdr->t + 1;
    const int n = st.n, ns = st.ns, lane = threadIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *y = reinterpret_cast<uint16_t *>(smem);  // 15 ns bytes in all
    uint16_t *posy = y + ns, *cur = posy + ns, *posc = cur + ns, *T = posc + ns;
    uint8_t *seen = reinterpret_cast<uint8_t *>(T + ns);
    uint16_t *lst = reinterpret_cast<uint16_t *>(seen + ns);  // ns transpositions
    const uint16_t *xg = st.X + size_t(part) * ns;
    uint16_t *vg = st.V + size_t(part) * 2 * ns;
    const int lv = st.VL[part];
    const uint64_t w0 = philox4x64_10(kp.seed, kp.instance, 0, uint64_t(part), uint64_t(t), kVel).w0;
    const uint64_t rr[2] = {uint32_t(w0) >> 16, uint32_t(w0 >> 32) >> 16};
    const uint32_t coef[2] = {kp.phi1_q16, kp.phi2_q16};
    const uint16_t *targets[2] = {st.P + size_t(part) * ns, st.G};
    for (int k = lane; k < n; k += 64) {
        const uint16_t v = xg[k];
        y[k] = v;
        posy[v] = uint16_t(k);
    }
    for (int k = lane; k < 2 * lv; k += 64) lst[k] = vg[k];
    int len = 0;
    for (int d = 0; d < 2; ++d) {
        for (int k = lane; k < n; k += 64) {  // cur <- x, T <- P or G
            const uint16_t v = xg[k];
            cur[k] = v;
            posc[v] = uint16_t(k);
            T[k] = targets[d][k];
            seen[k] = 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane == 0) {
            if (d == 0) {  // the stored velocity's prefix
                const uint64_t kw = (uint64_t(kp.w_q16) * uint64_t(lv)) >> 16;
                len = kw < uint64_t(lv) ? int(kw) : lv;
                for (int a = 0; a < len; ++a) {
                    const uint16_t la = lst[2 * a], lb = lst[2 * a + 1];
                    const uint16_t i = posy[la], j = posy[lb];
                    y[i] = lb;
                    y[j] = la;
                    posy[la] = j;
                    posy[lb] = i;
                }
                len = min(len, kp.velocity_cap);
            }
            int cycles = 0;  // of rho(q) = position in x of T[q]
            for (int q = 0; q < n; ++q) {
                if (seen[q]) continue;
                ++cycles;
                for (int r = q; !seen[r]; r = posc[T[r]]) seen[r] = 1;
            }
            const int k = prefix_count(coef[d], rr[d], n - cycles);
            for (int q = 0, e = 0; e < k; ++q) {
                const uint16_t la = cur[q], lb = T[q];
                if (la == lb) continue;
                const uint16_t j = posc[lb];  // cur: exchange labels la (at q) and lb
                cur[q] = lb;
                cur[j] = la;
                posc[lb] = uint16_t(q);
                posc[la] = j;
                const uint16_t yi = posy[la], yj = posy[lb];  // the same exchange on y
                y[yi] = lb;
                y[yj] = la;
                posy[la] = yj;
                posy[lb] = yi;
                if (len < kp.velocity_cap) {
                    lst[2 * len] = la;
                    lst[2 * len + 1] = lb;
                    ++len;
                }
                ++e;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    len = __shfl(len, 0, 64);
    uint16_t *xo = st.X + size_t(part) * ns;
    int64_t c = 0;
    for (int k = lane; k < n; k += 64) {
        xo[k] = y[k];
        c += D[size_t(y[k]) * n + y[k + 1 < n ? k + 1 : 0]];
    }
    for (int k = lane; k < 2 * len; k += 64) vg[k] = lst[k];
    c = wave_sum_i64(c);
    const bool better = c < st.FP[part];
    if (better)
        for (int k = lane; k < n; k += 64) st.P[size_t(part) * ns + k] = y[k];
    if (lane == 0) {
        st.F[part] = c;
        st.VL[part] = len;
        if (better) st.FP[part] = c;
    }
}

template <int TPB, int EPT>
__device__ __forceinline__ void move_body(const Inst &I, int part)
{
    const int32_t *__restrict__ D = I.D;
    const View st = I.st;
    const KParams kp = I.kp;
    const Hdr *h = st.hdr;
    if (h->err || h->done) return;
    if (kp.velocity_cap > 0) {  // uniform over the workgroup
        move_raw_body(I, part);
        return;
    }
    const int t = h->t + 1;
    const int n = st.n, ns = st.ns, tid = threadIdx.x;
    // read before the first barrier: thread 0 stores the new personal-best
    // cost at the end, after the last one
    const int64_t fp_old = st.FP[part];
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t redi[TPB / 64];
    __shared__ uint64_t draw0;  // first 64-bit word of stream (part, t, vel)
    MoveLds L = carve_move_lds(smem, (n + 7) & ~7);
    if (tid < 3) L.vote[tid] = 0;  // ordered before the first vote by the barriers below

    const uint16_t *xg = st.X + size_t(part) * ns;
    const uint16_t *vref = st.V + size_t(part) * 2 * ns, *vtgt = vref + ns;
    const bool has_v = st.VL[part] != 0;
    // with few positions per thread, the personal-best and global-best rows
    // used by the later steps are read now, beside the first loads, so their
    // memory latency is not paid again in the middle of the step (neither row
    // changes before this kernel writes P at its end)
    constexpr bool kPre = EPT <= 4;
    uint16_t pre_p[kPre ? EPT : 1], pre_g[kPre ? EPT : 1];
    if constexpr (kPre) {
        DPSO_EACH(k)
        {
            pre_p[e_] = st.P[size_t(part) * ns + k];
            pre_g[e_] = st.G[k];
        }
    }
    DPSO_EACH(k)
    {
        L.z[k] = xg[k];
        if (has_v) {  // the stored velocity's tours, in the slots x / posx take later
            const uint16_t f = vref[k];
            L.from[k] = f;
            L.posf[f] = uint16_t(k);
            L.to[k] = vtgt[k];
        }
    }
    if (tid == 0) draw0 = philox4x64_10(kp.seed, kp.instance, 0, uint64_t(part), uint64_t(t), kVel).w0;
    __syncthreads();
    const uint64_t r1 = uint32_t(draw0) >> 16, r2 = uint32_t(draw0 >> 32) >> 16;
    // a coefficient product of at least one keeps the whole list: k >= |list|
    // for every length, so the cycle structure is not needed
    const bool whole_b = uint64_t(kp.phi1_q16) * r1 >= (uint64_t(1) << 32);
    const bool whole_c = uint64_t(kp.phi2_q16) * r2 >= (uint64_t(1) << 32);
    const bool whole_w = kp.w_q16 >= 65536u;
    // z <- w(z): the prefix of the stored velocity as a label map
    if (has_v) {
        partial_toward<TPB, EPT>(L.from, L.posf, L.to, n,
                            [&](int len) {
                                const uint64_t k = (uint64_t(kp.w_q16) * uint64_t(len)) >> 16;
                                return k < uint64_t(len) ? int(k) : len;
                            },
                            whole_w, L);
        DPSO_EACH(k) L.z[k] = L.cur[L.posf[L.z[k]]];
        __syncthreads();  // posf is read above; posx takes its slot now
    }
    DPSO_EACH(k)
    {
        const uint16_t v = xg[k];
        L.x[k] = v;
        L.posx[v] = uint16_t(k);
        if constexpr (kPre)
            L.to[k] = pre_p[e_];
        else
            L.to[k] = st.P[size_t(part) * ns + k];
    }
    __syncthreads();
    // z <- b(z), b the prefix of P - x
    partial_toward<TPB, EPT>(L.x, L.posx, L.to, n, [&](int len) { return prefix_count(kp.phi1_q16, r1, len); },
                        whole_b, L);
    DPSO_EACH(k)
    {
        L.z[k] = L.cur[L.posx[L.z[k]]];
        if constexpr (kPre)
            L.to[k] = pre_g[e_];
        else
            L.to[k] = st.G[k];
    }
    __syncthreads();
    // z <- c(z), c the prefix of G - x
    partial_toward<TPB, EPT>(L.x, L.posx, L.to, n, [&](int len) { return prefix_count(kp.phi2_q16, r2, len); },
                        whole_c, L);
    DPSO_EACH(k) L.z[k] = L.cur[L.posx[L.z[k]]];
    __syncthreads();
    const uint16_t *y = L.z;
    uint16_t *xo = st.X + size_t(part) * ns;
    uint16_t *wref = st.V + size_t(part) * 2 * ns, *wtgt = wref + ns;
    DPSO_EACH(k)
    {
        wref[k] = L.x[k];
        wtgt[k] = y[k];
        xo[k] = y[k];
    }
    const int64_t c = block_tour_cost(D, n, y, redi);
    const bool better = c < fp_old;
    if (better) DPSO_EACH(k) st.P[size_t(part) * ns + k] = y[k];
    if (tid == 0) {
        st.F[part] = c;
        st.VL[part] = 1;
        if (better) st.FP[part] = c;
    }
}

#undef DPSO_EACH

// Mutation step 1 (Sect. 3.2.2): particle p is a duplicate if an earlier
// particle (lower index) has the same cost and the same tour. One wave per
// particle; candidates with equal cost are found by ballot, tours compared
// 64 labels at a time.
__device__ __forceinline__ void mut_dup_body(const Inst &I, int p)
{
    const View st = I.st;
    const KParams kp = I.kp;
    const Hdr *h = st.hdr;
    if (h->err || h->done) return;
    const int t = h->t + 1;
    if (!mutation_generation(kp, t)) return;
    const int lane = threadIdx.x, n = st.n, ns = st.ns;
    const int64_t Fp = st.F[p];
    const uint16_t *xp = st.X + size_t(p) * ns;
    bool dup = false;
    for (int q0 = 0; q0 < p && !dup; q0 += 64) {
        const int q = q0 + lane;
        uint64_t cand = __ballot(q < p && st.F[q] == Fp);
        while (cand && !dup) {
            const int qq = q0 + __ffsll((unsigned long long)cand) - 1;
            cand &= cand - 1;
            const uint16_t *xq = st.X + size_t(qq) * ns;
            bool diff = false;
            for (int k = lane; k < n; k += 64) diff |= xq[k] != xp[k];
            dup = !__any(diff);
        }
    }
    if (lane == 0) st.flags[p] = dup;
}

// Mutation step 2: order by (cost, index); the first ceil(S/3)
// non-duplicates are kept.
__device__ __forceinline__ void mut_keep_body(const Inst &I, int p)
{
    const View st = I.st;
    const KParams kp = I.kp;
    const Hdr *h = st.hdr;
    if (h->err || h->done) return;
    const int t = h->t + 1;
    if (!mutation_generation(kp, t)) return;
    const int lane = threadIdx.x, S = st.S;
    if (st.flags[p]) {
        if (lane == 0) st.keep[p] = 0;
        return;
    }
    const int64_t Fp = st.F[p];
    int before = 0;
    for (int q = lane; q < S; q += 64) {
        const int64_t Fq = st.F[q];
        before += !st.flags[q] && (Fq < Fp || (Fq == Fp && q < p));
    }
    before = wave_sum_i32(before);
    if (lane == 0) st.keep[p] = before < (S + 2) / 3;
}

// Mutation step 3: every particle not kept restarts from a Fisher-Yates
// shuffle of stream (p, t, mut), or with mutation_swaps = k > 0 is disturbed
// by k random position exchanges from that stream, with an empty velocity;
// its personal best is kept and replaced only by a strictly cheaper tour.
__device__ __forceinline__ void mut_apply_body(const Inst &I, int p)
{
    const int32_t *__restrict__ D = I.D;
    const View st = I.st;
    const KParams kp = I.kp;
    const Hdr *h = st.hdr;
    if (h->err || h->done) return;
    const int t = h->t + 1;
    if (!mutation_generation(kp, t)) return;
    const int n = st.n;
    if (st.keep[p]) return;
    const int64_t fp_old = st.FP[p];  // before the first barrier (thread 0 stores it at the end)
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t redi[4];
    uint16_t *tour = reinterpret_cast<uint16_t *>(smem);
    if (kp.mutation_swaps > 0) {
        const uint16_t *xg = st.X + size_t(p) * st.ns;
        for (int k = threadIdx.x; k < n; k += blockDim.x) tour[k] = xg[k];
        disturb(tour, reinterpret_cast<uint32_t *>(smem + size_t(st.ns) * 2), n, kp.mutation_swaps, kp, p, t,
                kMut);
    } else {
        fisher_yates(tour, smem + size_t(st.ns) * 2, n, st.ns, kp, p, t, kMut);
    }
    const int64_t cf = store_particle(D, st, p, tour, false, redi);
    const bool better = cf < fp_old;
    if (better)
        for (int k = threadIdx.x; k < n; k += blockDim.x) st.P[size_t(p) * st.ns + k] = tour[k];
    if (threadIdx.x == 0) {
        if (better) st.FP[p] = cf;
        atomicAdd(reinterpret_cast<unsigned long long *>(&st.hdr->n_reshuffled), 1ull);
    }
}

// Global best (the pseudo code's step that picks the fittest particle): the
// minimum of the packed key (FP << 16 | p) gives the cheapest personal best
// with the lowest index on ties. mode 0 (initialisation) installs it
// unconditionally; mode 1 (after move and mutation) and mode 2 (after the
// edge exchange) only on a strictly lower cost. Mode 1 also decides whether
// the edge exchange runs in this generation.
template <int MODE>
__device__ __forceinline__ void gbest_body(const Inst &I)
{
    constexpr int mode = MODE;
    const View st = I.st;
    const KParams kp = I.kp;
    Hdr *h = st.hdr;
    if (h->err) return;
    if (mode != 0 && h->done) return;
    if (mode == 2 && !h->ee_ran) return;
    // read before the reduction's barriers: thread 0 stores the new cost at
    // the end, after the last one
    const int64_t fg_old = h->FG;
    __shared__ uint64_t red[16];
    uint64_t best = ~0ull;
    for (int p = threadIdx.x; p < st.S; p += blockDim.x) {
        const uint64_t key = (uint64_t(st.FP[p]) << 16) | uint64_t(p);
        best = key < best ? key : best;
    }
    best = block_min_u64(best, red);
    const int g = int(best & 0xffffu);
    const int64_t FPg = int64_t(best >> 16);
    const bool better = mode == 0 || FPg < fg_old;
    __syncthreads();
    if (better)
        for (int k = threadIdx.x; k < st.n; k += blockDim.x) st.G[k] = st.P[size_t(g) * st.ns + k];
    if (threadIdx.x == 0) {
        if (better) h->FG = FPg;
        if (mode == 0) {
            st.trace[0] = FPg;
        } else if (mode == 1) {
            h->improved = better;
            h->ee_ran = kp.ee_trigger == 2 || (kp.ee_trigger == 1 && !better);
        } else {
            h->improved |= better;
        }
    }
}

// End of a generation: advance the counter, count generations without
// improvement, record the trace and test the stop conditions.
__device__ __forceinline__ void end_body(const Inst &I)
{
    const View st = I.st;
    const KParams kp = I.kp;
    Hdr *h = st.hdr;
    if (h->err || h->done) return;
    const int t = h->t + 1;
    h->t = t;
    h->stall = h->improved ? 0 : h->stall + 1;
    st.trace[t] = h->FG;
    if (t >= kp.max_generations || (kp.stall_limit > 0 && h->stall >= kp.stall_limit)) h->done = 1;
    h->improved = 0;
    h->ee_ran = 0;
}

// ------------------------------------------------------------------ kernels
// Each body runs as a single-instance kernel (descriptor by value) and as a
// batched kernel over many instances (descriptor from a device table).

// The global best after the exchange, then the end of the generation, in one
// launch (every early return of the first part is uniform over the block).
__device__ __forceinline__ void gbest2_end_body(const Inst &I)
{
    gbest_body<2>(I);
    __syncthreads();
    if (threadIdx.x == 0) end_body(I);
}

#define DPSO_KERNELS(name, threads, call)                                                   \
    __global__ __launch_bounds__(threads) void name(Inst I)                                  \
    {                                                                                        \
        const int item = int(blockIdx.x);                                                    \
        call;                                                                                \
    }                                                                                        \
    __global__ __launch_bounds__(threads) void name##_batch(Batch B)                         \
    {                                                                                        \
        const int b = batch_item(B, int(blockIdx.x));                                        \
        if (b < 0) return;                                                                   \
        int item;                                                                            \
        const Inst &I = batch_pick(B, b, item);                                              \
        call;                                                                                \
    }

DPSO_KERNELS(k_hdr_init, 64, hdr_init_body(I))
DPSO_KERNELS(k_hdr_check, 64, hdr_check_body(I))
DPSO_KERNELS(k_init, 256, init_body(I, item))
DPSO_KERNELS(k_mut_dup, 64, mut_dup_body(I, item))
DPSO_KERNELS(k_mut_keep, 64, mut_keep_body(I, item))
DPSO_KERNELS(k_mut_apply, 256, mut_apply_body(I, item))
DPSO_KERNELS(k_gbest0, 1024, gbest_body<0>(I))
DPSO_KERNELS(k_gbest1, 1024, gbest_body<1>(I))
DPSO_KERNELS(k_gbest2, 1024, gbest_body<2>(I))
DPSO_KERNELS(k_end, 64, end_body(I))
DPSO_KERNELS(k_gbest2_end, 1024, gbest2_end_body(I))

#undef DPSO_KERNELS

// The move at TPB threads per particle and EPT positions per thread.
template <int TPB, int EPT>
__global__ __launch_bounds__(TPB) void k_move(Inst I)
{
    move_body<TPB, EPT>(I, int(blockIdx.x));
}
template <int TPB, int EPT>
__global__ __launch_bounds__(TPB) void k_move_batch(Batch B)
{
    const int b = batch_item(B, int(blockIdx.x));
    if (b < 0) return;
    int item;
    const Inst &I = batch_pick(B, b, item);
    move_body<TPB, EPT>(I, item);
}

// A batch whose instances need different positions per thread (up to
// EPTMAX) in one launch: each workgroup runs the body at its own instance's
// ceil(ns / TPB) rounded up to a power of two, the layout a launch of that
// instance alone takes, instead of the largest instance's. The dynamic LDS
// is sized for the largest.
template <int TPB, int EPTMAX>
__global__ __launch_bounds__(TPB) void k_move_batch_mixed(Batch B)
{
    const int b = batch_item(B, int(blockIdx.x));
    if (b < 0) return;
    int item;
    const Inst &I = batch_pick(B, b, item);
    const int ept = (I.st.ns + TPB - 1) / TPB;  // uniform
    if constexpr (EPTMAX >= 16) {
        if (ept > 8) return move_body<TPB, 16>(I, item);
    }
    if constexpr (EPTMAX >= 8) {
        if (ept > 4) return move_body<TPB, 8>(I, item);
    }
    if constexpr (EPTMAX >= 4) {
        if (ept > 2) return move_body<TPB, 4>(I, item);
    }
    if constexpr (EPTMAX >= 2) {
        if (ept > 1) return move_body<TPB, 2>(I, item);
    }
    move_body<TPB, 1>(I, item);
}

// ---------------------------------------------------------------- launchers

size_t init_lds_bytes(int ns) { return size_t(ns) * 2 + size_t(ns) * 14; }
// the tour, then the shuffle's work area or the disturbance's 2048 draws
size_t mut_lds_bytes(int ns) { return size_t(ns) * 2 + std::max(size_t(ns) * 14, size_t(2048 * 4)); }

namespace {

// A launch over one instance (grid = its item count) or a batch.
struct Target {
    const Inst *one;    // single instance, or null
    Batch items;        // batch: blocks enumerate particles
    Batch instances;    // batch: one block per instance
    int total_items;    // blocks of a per-particle launch
    int count;          // instances
    int max_ns;         // largest row stride (dynamic LDS sizing)
};

Target single(const Inst &I)
{
    Target t{};
    t.one = &I;
    t.total_items = I.st.S;
    t.count = 1;
    t.max_ns = I.st.ns;
    return t;
}

template <class K1, class KB>
hipError_t launch(K1 k1, KB kb, const Target &t, bool per_particle, int threads, size_t lds, hipStream_t s)
{
    hipError_t e = allow_lds(k1, lds);
    if (e == hipSuccess) e = allow_lds(kb, lds);
    if (e != hipSuccess) return e;
    const int grid = per_particle ? t.total_items : t.count;
    if (grid <= 0) return hipSuccess;
    if (t.one)
        k1<<<grid, threads, lds, s>>>(*t.one);
    else
        kb<<<grid, threads, lds, s>>>(per_particle ? t.items : t.instances);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_init_t(const Target &t, hipStream_t s)
{
    hipError_t e = launch(k_hdr_init, k_hdr_init_batch, t, false, 64, 0, s);
    if (e == hipSuccess) e = launch(k_init, k_init_batch, t, true, 256, init_lds_bytes(t.max_ns), s);
    if (e == hipSuccess) e = launch(k_gbest0, k_gbest0_batch, t, false, 1024, 0, s);
    return e;
}

hipError_t launch_check_t(const Target &t, hipStream_t s)
{
    return launch(k_hdr_check, k_hdr_check_batch, t, false, 64, 0, s);
}

namespace {

template <int TPB>
hipError_t launch_move_tpb(const Target &t, size_t lds, hipStream_t s)
{
    // a batch takes the mixed kernel: each instance at its own positions per thread
    const int ept = (t.max_ns + TPB - 1) / TPB;
    if (ept <= 1) return launch(k_move<TPB, 1>, k_move_batch<TPB, 1>, t, true, TPB, lds, s);
    if (ept <= 2) return launch(k_move<TPB, 2>, k_move_batch_mixed<TPB, 2>, t, true, TPB, lds, s);
    if (ept <= 4) return launch(k_move<TPB, 4>, k_move_batch_mixed<TPB, 4>, t, true, TPB, lds, s);
    if (ept <= 8) return launch(k_move<TPB, 8>, k_move_batch_mixed<TPB, 8>, t, true, TPB, lds, s);
    if (ept <= 16) return launch(k_move<TPB, 16>, k_move_batch_mixed<TPB, 16>, t, true, TPB, lds, s);
    return hipErrorInvalidConfiguration;  // more than 16 positions per thread
}

}  // namespace

bool move_threads_ok(int tpb, int ns)
{
    return (tpb == 64 || tpb == 128 || tpb == 256 || tpb == 512) && ns <= 16 * tpb;
}

hipError_t launch_move_t(const Target &t, int tpb, hipStream_t s)
{
    // a single instance sizes LDS by its n; a batch by its largest row stride
    const size_t lds = t.one ? move_lds_bytes(t.one->st.n, t.one->st.ns) : move_lds_bytes(t.max_ns, t.max_ns);
    if (!move_threads_ok(tpb, t.max_ns)) return hipErrorInvalidConfiguration;
    if (tpb == 64) return launch_move_tpb<64>(t, lds, s);
    if (tpb == 128) return launch_move_tpb<128>(t, lds, s);
    if (tpb == 512) return launch_move_tpb<512>(t, lds, s);
    return launch_move_tpb<256>(t, lds, s);
}

hipError_t launch_mutation_t(const Target &t, hipStream_t s)
{
    hipError_t e = launch(k_mut_dup, k_mut_dup_batch, t, true, 64, 0, s);
    if (e == hipSuccess) e = launch(k_mut_keep, k_mut_keep_batch, t, true, 64, 0, s);
    if (e == hipSuccess) e = launch(k_mut_apply, k_mut_apply_batch, t, true, 256, mut_lds_bytes(t.max_ns), s);
    return e;
}

hipError_t launch_gbest_t(const Target &t, int mode, hipStream_t s)
{
    // a single instance's reduction takes as many threads as particles (one
    // wavefront for a swarm of 64: no idle waves, no workgroup barrier work);
    // a batch's blocks serve swarms of every size
    const int threads = t.one ? std::min(1024, std::max(64, (t.one->st.S + 63) & ~63)) : 1024;
    if (mode == 0) return launch(k_gbest0, k_gbest0_batch, t, false, threads, 0, s);
    if (mode == 1) return launch(k_gbest1, k_gbest1_batch, t, false, threads, 0, s);
    if (mode == 2) return launch(k_gbest2, k_gbest2_batch, t, false, threads, 0, s);
    return launch(k_gbest2_end, k_gbest2_end_batch, t, false, threads, 0, s);  // 3: mode 2, then the end
}

hipError_t launch_end_t(const Target &t, hipStream_t s)
{
    return launch(k_end, k_end_batch, t, false, 64, 0, s);
}

// Single-instance entry points.
hipError_t launch_init(const Inst &I, hipStream_t s) { return launch_init_t(single(I), s); }
hipError_t launch_check(const Inst &I, hipStream_t s) { return launch_check_t(single(I), s); }
hipError_t launch_move(const Inst &I, int tpb, hipStream_t s) { return launch_move_t(single(I), tpb, s); }
hipError_t launch_mutation(const Inst &I, hipStream_t s) { return launch_mutation_t(single(I), s); }
hipError_t launch_gbest(const Inst &I, int mode, hipStream_t s) { return launch_gbest_t(single(I), mode, s); }
hipError_t launch_end(const Inst &I, hipStream_t s) { return launch_end_t(single(I), s); }

// Batched entry points: `items` enumerates particles, `instances` one block
// per instance.
hipError_t launch_batch_init(const Batch &items, const Batch &instances, int total, int max_ns, hipStream_t s)
{
    Target t{nullptr, items, instances, total, instances.count, max_ns};
    return launch_init_t(t, s);
}
hipError_t launch_batch_check(const Batch &items, const Batch &instances, int total, int max_ns, hipStream_t s)
{
    Target t{nullptr, items, instances, total, instances.count, max_ns};
    return launch_check_t(t, s);
}
hipError_t launch_batch_move(int tpb, const Batch &items, int total, int max_ns, hipStream_t s)
{
    Target t{nullptr, items, Batch{}, total, items.count, max_ns};
    return launch_move_t(t, tpb, s);
}
hipError_t launch_batch_mutation(const Batch &items, const Batch &instances, int total, int max_ns,
                                 hipStream_t s)
{
    Target t{nullptr, items, instances, total, instances.count, max_ns};
    return launch_mutation_t(t, s);
}
hipError_t launch_batch_gbest(const Batch &items, const Batch &instances, int total, int max_ns, int mode,
                              hipStream_t s)
{
    Target t{nullptr, items, instances, total, instances.count, max_ns};
    return launch_gbest_t(t, mode, s);
}
hipError_t launch_batch_end(const Batch &items, const Batch &instances, int total, int max_ns, hipStream_t s)
{
    Target t{nullptr, items, instances, total, instances.count, max_ns};
    return launch_end_t(t, s);
}

}  // namespace dpso
