// Travelling costs from the voxel-grid planner (Sect. 2.2): voxels of edge
// s, occupied when their centre is in the open interior of a box, inflated by
// a sphere of the UAV's size (the clearance); paths step between the 26
// neighbouring voxels at cost L = a1 alpha^2 + a2 beta^2 + a3 gamma^2 (eq.
// cost), pass through free voxels only (their end voxels may be occupied),
// and the cost of a pair is s times the least total step cost.
//
// Grid: origin = (smallest coordinate of the viewpoints and box corners) - s
// per axis, dims = (largest - origin) / s + 2; voxel (i, j, k) has index
// i + dims_x (j + dims_y k).
//
// Inflation: a voxel is occupied when some box voxel lies within squared
// voxel distance R2 = floor(clearance^2 / s^2). The squared Euclidean
// distance to the nearest box voxel is separable: three passes, one per
// axis, each take the lower envelope of the parabolas (x - q)^2 + f(q) along
// every line of the grid (Meijster, Roerdink and Hesselink's linear-time
// scan, one thread per line). Values are capped at R2 + 1, which leaves the
// test d <= R2 exact (min(C, min_q (x-q)^2 + min(f_q, C)) = min(C, min_q
// (x-q)^2 + f_q)), so the work is linear in the grid whatever the clearance.
//
// Shortest paths: one workgroup per source. The grid is stored in bricks of
// 4 x 4 x 4 voxels (64 consecutive words, padded with occupied voxels), so a
// wave of 64 lanes owns one brick, a voxel per lane. A round takes the list
// of active bricks; a wave loads its brick with a one-voxel halo into LDS and
// relaxes it to local convergence (each voxel pulls from its 26 neighbours
// the least cost plus step over those a path may pass through), writes back
// its own voxels only, and activates the neighbouring bricks that touch an
// improved voxel. Costs only decrease, so the rounds end; at the end every
// voxel is consistent with all its neighbours, which is the shortest-path
// fixed point. A brick is written only by its owner wave; halo reads that
// race with a neighbour's writes see an old or a new cost, and a new one
// re-activates the reader. Sources run in chunks that fit the workspace.
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "device.hpp"
#include "dpso.h"
#include "errors.hpp"

namespace dpso {

namespace {

constexpr int kThreads = 256;
constexpr int kSearchThreads = 1024;
constexpr int32_t kUnreached = INT32_MAX;     // cost of a voxel no path has reached
constexpr int32_t kCostCap = INT32_MAX - 1;   // saturation of a path cost (then s * cost >= D_INF)
constexpr int kMaxWeight = 1 << 20;

struct Grid {
    int64_t origin[3];
    int32_t dims[3];
    int64_t G;
};

struct Args {
    Grid g;
    int32_t s, nb, n;
    int32_t w[3];
    int64_t cap;           // R2 + 1
    int32_t bx, by, bz;    // bricks per axis
    int64_t NB;            // bricks
    const int64_t *boxes;  // [nb][6]
    const int32_t *vox;    // [n] bricked index of each viewpoint's voxel
    uint8_t *core, *occ;   // [G] linear layout
    uint8_t *occb;         // [64 NB] bricked: 0 free, 1 occupied or padding, 2 occupied viewpoint voxel
    int64_t *edt, *ev;     // [G] squared distances; per-line envelope values
    int32_t *es, *et;      // [G] per-line envelope apexes and start abscissas
    int32_t *cost;         // [chunk][64 NB] bricked costs
    int32_t *tag;          // [chunk][NB] round + 1 for which a brick was last queued
    int32_t *la, *lb;      // [chunk][NB] active brick lists
    int32_t *D;            // [n][n]
    int32_t *flag;         // range error
};

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

__device__ inline int64_t floor_div(int64_t a, int64_t b)  // b > 0
{
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}

__global__ __launch_bounds__(kThreads) void k_vox_core(Args a)
{
    const Grid g = a.g;
    for (int64_t v = int64_t(blockIdx.x) * kThreads + threadIdx.x; v < g.G; v += int64_t(gridDim.x) * kThreads) {
        const int64_t idx[3] = {v % g.dims[0], (v / g.dims[0]) % g.dims[1], v / (int64_t(g.dims[0]) * g.dims[1])};
        uint8_t in = 0;
        for (int b = 0; b < a.nb && !in; ++b) {
            bool inside = true;
            for (int ax = 0; ax < 3; ++ax) {
                const int64_t c2 = 2 * g.origin[ax] + (2 * idx[ax] + 1) * a.s;  // twice the centre
                inside &= 2 * a.boxes[6 * b + ax] < c2 && c2 < 2 * a.boxes[6 * b + 3 + ax];
            }
            in = inside;
        }
        a.core[v] = in;
    }
}

// One distance-transform pass along `axis` (0, 1, 2): thread per grid line.
// The first pass reads the box voxels (distance 0, else the cap), the last
// one writes the occupancy. The envelope of line l keeps its entry q at
// [q * lines + l], so neighbouring threads touch neighbouring words.
__global__ __launch_bounds__(kThreads) void k_vox_edt(Args a, int axis, int first, int last)
{
    const Grid g = a.g;
    const int64_t nx = g.dims[0], ny = g.dims[1], nxy = nx * ny;
    const int64_t L = g.dims[axis], lines = g.G / L;
    const int64_t stride = axis == 0 ? 1 : axis == 1 ? nx : nxy;
    const int64_t cap = a.cap;
    for (int64_t l = int64_t(blockIdx.x) * kThreads + threadIdx.x; l < lines; l += int64_t(gridDim.x) * kThreads) {
        const int64_t base = axis == 0 ? l * nx : axis == 1 ? (l % nx) + nxy * (l / nx) : l;
        int32_t *S = a.es + l, *T = a.et + l;
        int64_t *V = a.ev + l;
        auto f = [&](int64_t q) -> int64_t {
            const int64_t v = base + q * stride;
            return first ? (a.core[v] ? 0 : cap) : a.edt[v];
        };
        int64_t q = 0;
        S[0] = 0;
        T[0] = 0;
        V[0] = f(0);
        for (int64_t u = 1; u < L; ++u) {
            const int64_t fu = f(u);
            // drop the parabolas that u beats at the start of their interval
            while (q >= 0) {
                const int64_t t = T[q * lines], sq = S[q * lines];
                if ((t - sq) * (t - sq) + V[q * lines] > (t - u) * (t - u) + fu)
                    --q;
                else
                    break;
            }
            if (q < 0) {
                q = 0;
                S[0] = int32_t(u);
                T[0] = 0;
                V[0] = fu;
            } else {
                const int64_t sq = S[q * lines], vq = V[q * lines];
                const int64_t w = 1 + floor_div(u * u - sq * sq + fu - vq, 2 * (u - sq));
                if (w < L) {
                    ++q;
                    S[q * lines] = int32_t(u);
                    T[q * lines] = int32_t(w);
                    V[q * lines] = fu;
                }
            }
        }
        for (int64_t u = L - 1; u >= 0; --u) {
            const int64_t sq = S[q * lines];
            const int64_t d = min((u - sq) * (u - sq) + V[q * lines], cap);
            const int64_t v = base + u * stride;
            if (last)
                a.occ[v] = d < cap;
            else
                a.edt[v] = d;
            if (u == T[q * lines]) --q;
        }
    }
}

// Bricked occupancy: 1 for padding outside the grid.
__global__ __launch_bounds__(kThreads) void k_vox_brick(Args a)
{
    const Grid g = a.g;
    const int64_t total = 64 * a.NB;
    for (int64_t q = int64_t(blockIdx.x) * kThreads + threadIdx.x; q < total; q += int64_t(gridDim.x) * kThreads) {
        const int64_t b = q >> 6;
        const int l = int(q & 63);
        const int64_t x = (b % a.bx) * 4 + (l & 3), y = ((b / a.bx) % a.by) * 4 + ((l >> 2) & 3),
                      z = (b / (int64_t(a.bx) * a.by)) * 4 + (l >> 4);
        a.occb[q] = x < g.dims[0] && y < g.dims[1] && z < g.dims[2]
                        ? a.occ[x + g.dims[0] * (y + int64_t(g.dims[1]) * z)]
                        : uint8_t(1);
    }
}

// Occupancy 2: an occupied voxel that holds a viewpoint. Paths may end
// there but not pass through; other occupied voxels (1) are never entered.
__global__ __launch_bounds__(kThreads) void k_vox_mark(Args a)
{
    const int32_t i = int32_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i < a.n && a.occb[a.vox[i]]) a.occb[a.vox[i]] = 2;
}

// Costs are shared by the waves of one workgroup only: relaxed atomics at
// workgroup scope (plain accesses on this target) keep the racing halo reads
// defined; the barriers between rounds order everything else.
__device__ inline int32_t ld_wg(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline void st_wg(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kWaves = kSearchThreads / 64;
constexpr int kHalo = 216;  // 6 x 6 x 6: a brick and its one-voxel halo

// One workgroup per source src0 + blockIdx.x; wave w takes the active bricks
// w, w + kWaves, ... of each round's list.
__global__ __launch_bounds__(kSearchThreads) void k_vox_sssp(Args a, int32_t src0)
{
    const int blk = blockIdx.x, src = src0 + blk, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t NB = a.NB, words = 64 * NB;
    const int32_t bx = a.bx, by = a.by, bz = a.bz;
    int32_t *cost = a.cost + size_t(blk) * size_t(words);
    int32_t *tag = a.tag + size_t(blk) * size_t(NB);
    int32_t *cur = a.la + size_t(blk) * size_t(NB), *nxt = a.lb + size_t(blk) * size_t(NB);
    const uint8_t *__restrict__ occb = a.occb;
    __shared__ int32_t count[2];
    __shared__ int32_t offer[kWaves][kHalo];  // cost of a voxel a path may pass through, else kUnreached
    for (int64_t v = tid; v < words; v += kSearchThreads) cost[v] = kUnreached;
    for (int64_t v = tid; v < NB; v += kSearchThreads) tag[v] = 0;
    const int32_t s0 = a.vox[src];
    __syncthreads();
    if (tid == 0) {
        cur[0] = s0 >> 6;
        tag[s0 >> 6] = 1;
        count[0] = 1;
        count[1] = 0;
    }
    __syncthreads();
    // this lane's voxel in the brick, and its place in the halo cube
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const int p0 = (lx + 1) + 6 * ((ly + 1) + 6 * (lz + 1));
    int32_t *L = offer[wave];
    for (int32_t round = 0, c = 0;; ++round, c ^= 1) {
        const int32_t na = count[c];
        if (na == 0) break;
        const int32_t qtag = round + 2;  // queued for round + 1
        for (int32_t e = wave; e < na; e += kWaves) {
            const int32_t bb = cur[e];
            const int32_t ox = bb % bx, oy = (bb / bx) % by, oz = bb / (bx * by);
            for (int p = lane; p < kHalo; p += 64) {
                const int gx = ox * 4 + p % 6 - 1, gy = oy * 4 + (p / 6) % 6 - 1, gz = oz * 4 + p / 36 - 1;
                int32_t v = kUnreached;
                if (gx >= 0 && gx < 4 * bx && gy >= 0 && gy < 4 * by && gz >= 0 && gz < 4 * bz) {
                    const int64_t q = (int64_t((gx >> 2) + bx * ((gy >> 2) + by * (gz >> 2))) << 6) + (gx & 3) +
                                      4 * (gy & 3) + 16 * (gz & 3);
                    if (occb[q] == 0 || q == s0) v = ld_wg(cost + q);
                }
                L[p] = v;
            }
            const int64_t own = (int64_t(bb) << 6) + lane;
            const uint8_t oo = occb[own];
            const bool recv = oo != 1, pass = oo == 0 || own == s0;
            const int32_t c0 = ld_wg(cost + own);
            int32_t cc = own == s0 ? 0 : c0;  // the source enters with cost 0 in its first activation
            wave_sync();
            if (pass && cc < c0) L[p0] = cc;
            wave_sync();
            for (;;) {
                int64_t best = cc;
                if (recv) {
#pragma unroll
                    for (int k = 0; k < 26; ++k) {
                        const int q = k < 13 ? k : k + 1, di = q % 3 - 1, dj = (q / 3) % 3 - 1, dk = q / 9 - 1;
                        const int32_t v = L[p0 + di + 6 * dj + 36 * dk];
                        const int64_t step = int64_t(di ? a.w[0] : 0) + (dj ? a.w[1] : 0) + (dk ? a.w[2] : 0);
                        const int64_t t = v == kUnreached ? INT64_MAX : min(int64_t(v) + step, int64_t(kCostCap));
                        best = min(best, t);
                    }
                }
                const bool ch = best < cc;
                if (ch) {
                    cc = int32_t(best);
                    if (pass) L[p0] = cc;
                }
                wave_sync();
                if (!__any(ch)) break;
            }
            uint32_t m = 0;  // neighbouring bricks (dx, dy, dz) touched by an improved voxel
            if (cc < c0) {
                st_wg(cost + own, cc);
                for (int dz = -1; dz <= 1; ++dz) {
                    if (dz && (dz < 0 ? lz != 0 : lz != 3)) continue;
                    for (int dy = -1; dy <= 1; ++dy) {
                        if (dy && (dy < 0 ? ly != 0 : ly != 3)) continue;
                        for (int dx = -1; dx <= 1; ++dx) {
                            if (dx && (dx < 0 ? lx != 0 : lx != 3)) continue;
                            m |= 1u << ((dx + 1) + 3 * (dy + 1) + 9 * (dz + 1));
                        }
                    }
                }
            }
#pragma unroll
            for (int sh = 32; sh >= 1; sh >>= 1) m |= uint32_t(__shfl_xor(int(m), sh));
            if (lane < 27 && lane != 13 && ((m >> lane) & 1)) {
                const int nx_ = ox + lane % 3 - 1, ny_ = oy + (lane / 3) % 3 - 1, nz_ = oz + lane / 9 - 1;
                if (nx_ >= 0 && nx_ < bx && ny_ >= 0 && ny_ < by && nz_ >= 0 && nz_ < bz) {
                    const int32_t nbk = nx_ + bx * (ny_ + by * nz_);
                    if (atomicExch(tag + nbk, qtag) != qtag) nxt[atomicAdd(&count[c ^ 1], 1)] = nbk;
                }
            }
        }
        __syncthreads();
        if (tid == 0) count[c] = 0;
        int32_t *t = cur;
        cur = nxt;
        nxt = t;
        __syncthreads();
    }
    for (int32_t j = tid; j < a.n; j += kSearchThreads) {
        const int64_t d = ld_wg(cost + a.vox[j]);
        int32_t out = DPSO_D_INF;  // unreached
        if (d != kUnreached) {
            if (d * a.s < DPSO_D_INF)
                out = int32_t(d * a.s);
            else
                atomicOr(a.flag, 1);  // a finite cost at or above D_INF (a saturated one included)
        }
        a.D[size_t(src) * a.n + j] = out;
    }
}

// Grid of a scene; false if it is too large.
bool make_grid(const dpso_scene *sc, int32_t s, Grid &g)
{
    int64_t lo[3], hi[3];
    for (int ax = 0; ax < 3; ++ax) lo[ax] = hi[ax] = sc->vp_mm[ax];
    for (int32_t i = 0; i < sc->n; ++i)
        for (int ax = 0; ax < 3; ++ax) {
            lo[ax] = std::min<int64_t>(lo[ax], sc->vp_mm[3 * i + ax]);
            hi[ax] = std::max<int64_t>(hi[ax], sc->vp_mm[3 * i + ax]);
        }
    for (int32_t b = 0; b < sc->n_boxes; ++b)
        for (int ax = 0; ax < 3; ++ax) {
            lo[ax] = std::min<int64_t>(lo[ax], sc->boxes_mm[6 * b + ax]);
            hi[ax] = std::max<int64_t>(hi[ax], sc->boxes_mm[6 * b + 3 + ax]);
        }
    g.G = 1;
    for (int ax = 0; ax < 3; ++ax) {
        g.origin[ax] = lo[ax] - s;
        const int64_t d = (hi[ax] - g.origin[ax]) / s + 2;
        if (d > (1 << 20)) return false;
        g.dims[ax] = int32_t(d);
        g.G *= d;
    }
    return g.G <= (int64_t(1) << 26);
}

struct Bricks {
    int32_t b[3];
    int64_t NB;
};

Bricks bricks_of(const Grid &g)
{
    Bricks r;
    r.NB = 1;
    for (int ax = 0; ax < 3; ++ax) {
        r.b[ax] = (g.dims[ax] + 3) / 4;
        r.NB *= r.b[ax];
    }
    return r;
}

// Per-source arrays: costs (64 words a brick), tags and two brick lists.
size_t per_source_bytes(int64_t NB) { return size_t(NB) * (64 * 4 + 3 * 4); }

// Sources per chunk: 16 GiB of per-source arrays at most, at most 1024, and
// the chunks evened out (a short last chunk would cost a whole search
// latency for a few sources).
int32_t chunk_sources(int32_t n, int64_t NB)
{
    const int64_t k = std::max<int64_t>(1, (int64_t(16) << 30) / int64_t(per_source_bytes(NB)));
    const int64_t most = std::min<int64_t>({k, n, 1024});
    const int64_t chunks = (n + most - 1) / most;
    return int32_t((n + chunks - 1) / chunks);
}

// The distance transform's arrays (24 bytes per voxel) and the per-source
// arrays share one region: the transform ends before the first search.
size_t shared_bytes(const Grid &g, int64_t NB, int32_t B)
{
    const size_t G = size_t(g.G), b = size_t(B), nb = size_t(NB);
    return std::max(2 * a256(G * 8) + 2 * a256(G * 4), a256(b * nb * 64 * 4) + 3 * a256(b * nb * 4));
}

size_t work_bytes(const Grid &g, int32_t n, int32_t nb)
{
    const size_t G = size_t(g.G);
    const Bricks k = bricks_of(g);
    return a256(size_t(nb > 0 ? nb : 1) * 6 * 8) + a256(size_t(n) * 4) + 2 * a256(G) + a256(size_t(k.NB) * 64) +
           256 + shared_bytes(g, k.NB, chunk_sources(n, k.NB));
}

dpso_status check_voxel_args(const dpso_scene *sc, const dpso_voxel_params *vp, Grid &g)
{
    if (!sc || !vp) return fail(DPSO_E_INVAL, "scene and voxel parameters must be non-NULL");
    if (sc->n < 1 || !sc->vp_mm) return fail(DPSO_E_INVAL, "scene has n = %d viewpoints", sc->n);
    if (sc->n > DPSO_MAX_N) return fail(DPSO_E_RANGE, "n = %d exceeds DPSO_MAX_N", sc->n);
    if (sc->n_boxes < 0 || (sc->n_boxes > 0 && !sc->boxes_mm))
        return fail(DPSO_E_INVAL, "bad box list (n_boxes = %d)", sc->n_boxes);
    if (sc->clearance_mm < 0) return fail(DPSO_E_INVAL, "clearance must be >= 0");
    if (vp->voxel_mm < 1) return fail(DPSO_E_INVAL, "voxel_mm = %d must be >= 1", vp->voxel_mm);
    for (int ax = 0; ax < 3; ++ax)
        if (vp->weight[ax] < 1 || vp->weight[ax] > kMaxWeight)
            return fail(DPSO_E_INVAL, "step weight %d = %d outside 1..2^20", ax, vp->weight[ax]);
    const int64_t lim = int64_t(1) << 26;
    for (int64_t i = 0; i < 3 * int64_t(sc->n); ++i)
        if (sc->vp_mm[i] <= -lim || sc->vp_mm[i] >= lim)
            return fail(DPSO_E_RANGE, "viewpoint coordinate %d outside (-2^26, 2^26)", sc->vp_mm[i]);
    for (int32_t b = 0; b < sc->n_boxes; ++b)
        for (int ax = 0; ax < 3; ++ax) {
            const int64_t lo = sc->boxes_mm[6 * b + ax], hi = sc->boxes_mm[6 * b + 3 + ax];
            if (lo > hi) return fail(DPSO_E_INVAL, "box %d has lo > hi on axis %d", b, ax);
            if (lo <= -lim || hi >= lim) return fail(DPSO_E_RANGE, "box %d outside (-2^26, 2^26)", b);
        }
    if (!make_grid(sc, vp->voxel_mm, g))
        return fail(DPSO_E_RANGE, "voxel grid above 2^26 voxels or 2^20 per axis");
    return DPSO_OK;
}

}  // namespace

}  // namespace dpso

extern "C" size_t dpso_voxel_work_bytes(const dpso_scene *scene, const dpso_voxel_params *params)
{
    dpso::Grid g;
    if (dpso::check_voxel_args(scene, params, g) != DPSO_OK) return 0;
    return dpso::work_bytes(g, scene->n, scene->n_boxes);
}

extern "C" dpso_status dpso_build_dist_voxel(const dpso_scene *scene, const dpso_voxel_params *params,
                                             int32_t *d_dist, void *d_work, size_t work_bytes, void *stream)
{
    using namespace dpso;
    Grid g;
    dpso_status st = check_voxel_args(scene, params, g);
    if (st) return st;
    if (!d_dist || !d_work) return fail(DPSO_E_INVAL, "d_dist and d_work must be non-NULL");
    const int32_t n = scene->n, nb = scene->n_boxes;
    const size_t need = dpso::work_bytes(g, n, nb);
    if (work_bytes < need) return fail(DPSO_E_NOMEM, "workspace of %zu bytes, %zu needed", work_bytes, need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Bricks k = bricks_of(g);
    const int32_t B = chunk_sources(n, k.NB);
    char *w = static_cast<char *>(d_work);
    Args a{};
    a.g = g;
    a.s = params->voxel_mm;
    a.nb = nb;
    a.n = n;
    for (int ax = 0; ax < 3; ++ax) a.w[ax] = params->weight[ax];
    const int64_t c = scene->clearance_mm, sv = params->voxel_mm;
    a.cap = (c * c) / (sv * sv) + 1;
    a.bx = k.b[0];
    a.by = k.b[1];
    a.bz = k.b[2];
    a.NB = k.NB;
    size_t at = 0;
    auto take = [&](size_t bytes) { char *p = w + at; at += a256(bytes); return p; };
    int64_t *boxes = reinterpret_cast<int64_t *>(take(size_t(nb > 0 ? nb : 1) * 6 * 8));
    int32_t *vox = reinterpret_cast<int32_t *>(take(size_t(n) * 4));
    a.core = reinterpret_cast<uint8_t *>(take(size_t(g.G)));
    a.occ = reinterpret_cast<uint8_t *>(take(size_t(g.G)));
    a.occb = reinterpret_cast<uint8_t *>(take(size_t(k.NB) * 64));
    a.flag = reinterpret_cast<int32_t *>(take(4));
    char *shared = take(shared_bytes(g, k.NB, B));
    at = size_t(shared - w);
    a.edt = reinterpret_cast<int64_t *>(take(size_t(g.G) * 8));
    a.ev = reinterpret_cast<int64_t *>(take(size_t(g.G) * 8));
    a.es = reinterpret_cast<int32_t *>(take(size_t(g.G) * 4));
    a.et = reinterpret_cast<int32_t *>(take(size_t(g.G) * 4));
    at = size_t(shared - w);
    a.cost = reinterpret_cast<int32_t *>(take(size_t(B) * size_t(k.NB) * 64 * 4));
    a.tag = reinterpret_cast<int32_t *>(take(size_t(B) * size_t(k.NB) * 4));
    a.la = reinterpret_cast<int32_t *>(take(size_t(B) * size_t(k.NB) * 4));
    a.lb = reinterpret_cast<int32_t *>(take(size_t(B) * size_t(k.NB) * 4));
    a.boxes = boxes;
    a.vox = vox;
    a.D = d_dist;
    std::vector<int64_t> hb(size_t(nb > 0 ? nb : 1) * 6, 0);
    for (size_t k = 0; k < size_t(nb) * 6; ++k) hb[k] = scene->boxes_mm[k];
    std::vector<int32_t> hv(n);
    for (int32_t i = 0; i < n; ++i) {
        int64_t id[3];
        for (int ax = 0; ax < 3; ++ax) id[ax] = (int64_t(scene->vp_mm[3 * i + ax]) - g.origin[ax]) / params->voxel_mm;
        const int64_t brick = (id[0] >> 2) + k.b[0] * ((id[1] >> 2) + int64_t(k.b[1]) * (id[2] >> 2));
        hv[i] = int32_t((brick << 6) + (id[0] & 3) + 4 * (id[1] & 3) + 16 * (id[2] & 3));
    }
    const int32_t zero = 0;
    hipError_t e = hipMemcpyAsync(boxes, hb.data(), hb.size() * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(vox, hv.data(), hv.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(a.flag, &zero, 4, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail(DPSO_E_DEVICE, "voxel planner upload: %s", hipGetErrorString(e));
    const int blocks = int(std::min<int64_t>((g.G + kThreads - 1) / kThreads, 4096));
    k_vox_core<<<blocks, kThreads, 0, s>>>(a);
    for (int axis = 0; axis < 3; ++axis) {
        const int64_t lines = g.G / g.dims[axis];
        k_vox_edt<<<int(std::min<int64_t>((lines + kThreads - 1) / kThreads, 4096)), kThreads, 0, s>>>(
            a, axis, axis == 0, axis == 2);
    }
    k_vox_brick<<<int(std::min<int64_t>((64 * k.NB + kThreads - 1) / kThreads, 4096)), kThreads, 0, s>>>(a);
    k_vox_mark<<<(n + kThreads - 1) / kThreads, kThreads, 0, s>>>(a);
    for (int32_t src0 = 0; src0 < n; src0 += B)
        k_vox_sssp<<<std::min(B, n - src0), kSearchThreads, 0, s>>>(a, src0);
    int32_t flag = 0;
    if ((e = hipGetLastError()) == hipSuccess)
        e = hipMemcpyAsync(&flag, a.flag, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(DPSO_E_DEVICE, "voxel planner: %s", hipGetErrorString(e));
    if (flag) return fail(DPSO_E_RANGE, "a finite path cost reaches DPSO_D_INF");
    return ok();
}
