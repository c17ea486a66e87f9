/*
 * dpso.h - C ABI of the MI355X (gfx950) library for the enhanced discrete
 * particle swarm optimisation of UAV inspection paths (Phung, Quach, Dinh, Ha,
 * "Enhanced Discrete Particle Swarm Optimization Path Planning for UAV
 * Vision-based Surface Inspection", arXiv 1706.04399).
 *
 * The inspection path is a travelling-salesman tour over camera viewpoints
 * with obstacle-aware travelling costs (Sect. 2.3). A swarm of particles,
 * each a tour, evolves by the discrete velocity update of Sect. 3.1, random
 * mutation (Sect. 3.2.2) and complete 2-opt edge exchange (Sect. 3.2.3),
 * following the pseudo code of Sect. 3.3.
 *
 * Conventions
 *  - Labels are 0..n-1 (the paper's nodes 1..N). A tour is n labels; the
 *    return to the first node is implicit.
 *  - Distances are int32 millimetres, row-major [n][n], symmetric, zero on
 *    the diagonal, 0 <= d < DPSO_D_INF, or DPSO_D_INF for a pair with no
 *    obstacle-free path (Sect. 2.3 gives such a pair an arbitrarily large
 *    cost). Costs are
 *    int64.
 *  - Pointers prefixed d_ are device memory on the current HIP device; h_
 *    pointers and dpso_scene arrays are host memory. The caller owns every
 *    buffer and keeps it alive until the work enqueued on `stream` is done.
 *    `stream` is a hipStream_t (NULL = the null stream).
 *  - Calls that only enqueue work return before it finishes; a device fault
 *    surfaces as DPSO_E_DEVICE at a later call. Calls documented as
 *    synchronising wait for `stream`.
 *  - Errors are returned, never thrown. dpso_last_error() gives a
 *    thread-local text for the last failing call of the calling thread.
 *  - Arguments are validated before any device work is enqueued, so a
 *    rejected call has no effect.
 */
#ifndef DPSO_H
#define DPSO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dpso_status;
#define DPSO_OK 0
#define DPSO_E_INVAL (-1)  /* null pointer, bad size or parameter              */
#define DPSO_E_RANGE (-2)  /* value outside what the library supports          */
#define DPSO_E_NOMEM (-3)  /* a caller buffer is smaller than required         */
#define DPSO_E_DEVICE (-4) /* a HIP call failed (text in dpso_last_error)       */
#define DPSO_E_STATE (-5)  /* state buffer not initialised for this n / swarm  */
#define DPSO_E_ADMIT (-6)  /* a served request needs more device memory than the
                              whole serving budget (dpso_request_footprint)    */

#define DPSO_D_INF 268435455 /* 2^28 - 1 */
#define DPSO_MAX_N 4096      /* largest number of viewpoints                    */
#define DPSO_MAX_SWARM 65536 /* largest swarm                                   */
#define DPSO_MAX_GRAPH 16384 /* largest n + 8 * n_boxes (visibility-graph nodes)  */
#define DPSO_MAX_BATCH 65536 /* largest number of instances in one batched call  */

/* Edge-exchange trigger (pseudo code of Sect. 3.3: exchange when the global
 * best did not improve; ALWAYS runs it every generation). */
#define DPSO_EE_OFF 0
#define DPSO_EE_ON_STALL 1
#define DPSO_EE_ALWAYS 2

/* Edge-exchange neighbourhoods (dpso_params.ee_neighbourhood). */
#define DPSO_NB_TWO_OPT 0   /* reverse a segment: the 2-opt search of Sect. 3.2.3      */
#define DPSO_NB_NODE_SWAP 1 /* exchange the nodes at two positions: the edge-exchange
                               kernel and pseudo code of Sect. 3.3                    */

/* A scene (Sect. 2.1-2.2): viewpoint positions and axis-aligned box
 * obstacles in integer mm; boxes are inflated by clearance_mm (the UAV's
 * size). Coordinates must satisfy |c| < 2^26 after inflation, and
 * n + 8 * n_boxes <= DPSO_MAX_GRAPH. */
typedef struct {
    const int32_t *vp_mm;    /* host [n][3]: x, y, z                        */
    int32_t n;               /* 1 <= n <= DPSO_MAX_N                         */
    const int32_t *boxes_mm; /* host [n_boxes][6]: lo x, y, z, hi x, y, z   */
    int32_t n_boxes;         /* >= 0                                         */
    int32_t clearance_mm;    /* >= 0                                         */
} dpso_scene;

/* Swarm parameters (pseudo code of Sect. 3.3). Coefficients of eq. velocity
 * are Q16 fixed point: value * 65536, at most 2.0 (131072). A coefficient
 * product above one keeps the whole transposition list. */
typedef struct {
    int32_t swarm_size;      /* 1..DPSO_MAX_SWARM                                   */
    int32_t max_generations; /* generations after initialisation (>= 0)             */
    uint32_t w_q16;          /* inertia w                                           */
    uint32_t phi1_q16;       /* cognitive coefficient phi1                          */
    uint32_t phi2_q16;       /* social coefficient phi2                             */
    int32_t mutation_period; /* mutate on generations t % period == 0; 0 = never    */
    int32_t ee_trigger;      /* DPSO_EE_*                                           */
    int32_t ee_max_moves;    /* exchanges per particle per invocation; 0 = until no
                                improving exchange remains                          */
    int32_t stall_limit;     /* stop after this many generations without a better
                                global best; 0 = never                             */
    int32_t det_permille;    /* share of nearest-neighbour seeded particles (0..1000) */
    uint64_t seed;           /* Philox key word 0                                   */
    uint64_t instance;       /* Philox key word 1                                   */
    int32_t ee_neighbourhood; /* DPSO_NB_*; both take the most improving move, ties
                                 to the smallest first then second position          */
    int32_t mutation_swaps;  /* 0: mutated particles restart from a shuffle; k > 0
                                (at most 65536): they are disturbed by k exchanges of
                                random positions instead (mutation text, Sect. 3.2.2) */
    int32_t velocity_cap;    /* 0: the velocity is renormalised to y - x after each
                                move; c in 1..n: it is kept as the raw concatenation
                                of eq. velocity (operator (+), Sect. 3.1), truncated to
                                its first c transpositions. A state keeps the mode it
                                was initialised with (another mode: DPSO_E_STATE).  */
} dpso_params;

/* Progress of a swarm, read by dpso_get_info. */
typedef struct {
    int32_t n, swarm_size, trace_capacity;
    int32_t generation;      /* generations completed (0 after init)            */
    int32_t stall;           /* generations since the global best last improved */
    int32_t done;            /* max_generations or stall_limit reached          */
    int64_t best_cost;       /* cost of the global best tour                    */
    int64_t sweeps;          /* complete edge-exchange neighbourhood searches   */
    int64_t moves;           /* edge exchanges applied                          */
    int64_t reshuffled;      /* particles reshuffled or disturbed by mutation   */
} dpso_info;

/* Host view of a swarm state for dpso_export_state / dpso_import_state.
 * Arrays are row-major; velocity row p holds vlen[p] transpositions
 * (label a, label b). */
typedef struct {
    uint16_t *X;    /* [S][n] current tours          */
    uint16_t *P;    /* [S][n] personal-best tours    */
    uint16_t *V;    /* [S][n][2] velocities          */
    int32_t *vlen;  /* [S]                           */
    int64_t *F;     /* [S] cost of X                 */
    int64_t *FP;    /* [S] cost of P                 */
    uint16_t *G;    /* [n] global-best tour          */
    int64_t *trace; /* [trace_capacity] global-best cost after each generation */
    int32_t generation, stall, done;
    int64_t best_cost;
} dpso_host_state;

/* Library version string. */
const char *dpso_version(void);

/* Text of the last error returned to the calling thread ("" if none). */
const char *dpso_last_error(void);

/* Checks parameters against n without touching the device. */
dpso_status dpso_validate_params(const dpso_params *params, int32_t n);

/* Exact size of the device state buffer for n viewpoints, a swarm of
 * swarm_size and max_generations generations; 0 if the sizes are out of
 * range. The buffer holds every particle's tour, personal best and
 * velocity, costs, the global best, the cost trace and the scratch space
 * used by the generation loop, and, for 8 <= n <= 1024, the 16-bit copy of D
 * with rows padded to a multiple of 8 entries (2 n ceil8(n) bytes) that the
 * edge exchange stages (DPSO_ROWS_U16), rewritten by every run that uses it:
 * dpso_run allocates nothing. */
size_t dpso_state_bytes(int32_t n, int32_t swarm_size, int32_t max_generations);

/* Device bytes a served plan request holds while it stays resident (the
 * re-planning of criterion (iv) of Sect. 1 keeps the distance matrix and the
 * swarm on the device between requests): its swarm state
 * (dpso_state_bytes(n, swarm_size, max_generations)) and its int32 [n][n]
 * distance matrix, built with dpso_build_dist_noalloc, which needs no
 * workspace of its own. Writes *bytes (may be NULL). Returns DPSO_E_ADMIT if
 * they exceed `budget` (such a request can never be admitted), DPSO_E_INVAL
 * or DPSO_E_RANGE for parameters dpso_validate_params rejects. Host only. */
dpso_status dpso_request_footprint(int32_t n, const dpso_params *params, size_t budget, size_t *bytes);

/* A planar surface to inspect (Sect. 2.1): an axis-aligned rectangle in the
 * plane {coordinate normal_axis = lo_mm[normal_axis]} spanning lo..hi along
 * the two other axes (lo_mm[normal_axis] == hi_mm[normal_axis]); the UAV
 * views it from the side normal_sign (+1 or -1) of the plane. */
typedef struct {
    int32_t lo_mm[3], hi_mm[3];
    int32_t normal_axis;  /* 0, 1, 2 = x, y, z */
    int32_t normal_sign;  /* +1 or -1           */
} dpso_surface;

/* Camera and image requirements of the viewpoint selection (Sect. 2.1). */
typedef struct {
    int32_t resolution_px;    /* r_c: pixels along the image side          */
    int32_t feature_um;       /* s_f: smallest feature to resolve          */
    int32_t overlap_permille; /* o_p: overlap of neighbouring images, 0..999 */
    int32_t focal_um;         /* f: focal length                           */
    int32_t sensor_um;        /* s_s: sensor size along the same side       */
} dpso_camera;

/* Viewpoint selection (Sect. 2.1, eq. fov, eq. premitive, eq.
 * cameraDistance): footprint a = r_c s_f / 2, cell size p = (1 - o_p) a,
 * working distance d = a f / s_s (exact in um, then truncated to whole um).
 * Each surface is covered by a grid of cells of size p anchored at its low
 * corner, max(1, ceil(L / p)) cells along each in-plane axis of extent L (the
 * last cell may overhang); each cell centre moved d along the viewing side
 * is one viewpoint, its coordinates rounded half up to whole mm. Order:
 * surface by surface, the lower in-plane axis outer, the other inner. Host
 * function (no device work). *n_out receives the number of viewpoints; with
 * vp_mm == NULL nothing else happens (counting). Otherwise the viewpoints are
 * written to vp_mm (host [max_n][3]) if they fit, else nothing is written
 * and DPSO_E_RANGE is returned (also for a coordinate outside int32).
 * DPSO_E_INVAL for a malformed surface or camera (a cell size below 1 um). */
dpso_status dpso_viewpoints(const dpso_surface *surfaces, int32_t count, const dpso_camera *camera,
                            int32_t *vp_mm, int32_t max_n, int32_t *n_out);

/* Voxel-grid planner (Sect. 2.2, eq. cost), an alternative source of the
 * travelling costs. Voxels of edge voxel_mm cover the scene with a one-voxel
 * margin (origin = smallest viewpoint or box coordinate - voxel_mm per axis,
 * (largest - origin) / voxel_mm + 2 voxels per axis); a voxel is occupied when
 * its centre is in the open interior of a box, and so is every voxel whose
 * centre is within clearance_mm (the UAV's size) of an occupied centre. A path
 * steps between the 26 neighbouring voxels; step (a, b, c) in {-1,0,1}^3 costs
 * weight[0] a^2 + weight[1] b^2 + weight[2] c^2. It passes through free voxels
 * only; its end voxels (those holding the two viewpoints) may be occupied.
 * D[i][j] = voxel_mm * least total step cost, DPSO_D_INF if no path. */
typedef struct {
    int32_t voxel_mm;   /* voxel edge, >= 1               */
    int32_t weight[3];  /* a1, a2, a3 of eq. cost, 1..2^20 */
} dpso_voxel_params;

/* Device workspace for dpso_build_dist_voxel; 0 for invalid arguments or a
 * grid above 2^26 voxels (or 2^20 along an axis). It holds the occupancy
 * grids and the search arrays of min(n, 1024) sources searched at once, at
 * most 16 GiB of those (a larger problem runs its sources in several
 * chunks). */
size_t dpso_voxel_work_bytes(const dpso_scene *scene, const dpso_voxel_params *params);

/* Travelling costs by the voxel-grid planner: writes d_dist (device int32
 * [n][n]); d_work (device, dpso_voxel_work_bytes) is scratch. Synchronises
 * `stream`. DPSO_E_RANGE if a finite path cost reaches DPSO_D_INF (those
 * entries are DPSO_D_INF) or the grid is too large. */
dpso_status dpso_build_dist_voxel(const dpso_scene *scene, const dpso_voxel_params *params,
                                  int32_t *d_dist, void *d_work, size_t work_bytes, void *stream);

/* Checks a device matrix against the contract every swarm call relies on
 * (Sect. 2: one symmetric travelling cost per pair of viewpoints, none from a
 * viewpoint to itself; Sect. 2.3: a blocked pair costs DPSO_D_INF):
 * D[i][i] = 0, D[i][j] = D[j][i] and 0 <= D[i][j] <= DPSO_D_INF. d_dist:
 * device int32 [n][n]; d_work: device scratch of at least 8 bytes. *h_bad
 * receives the row-major index i * n + j of the first entry that breaks the
 * contract, or -1. Synchronises `stream`. DPSO_OK if the matrix holds,
 * DPSO_E_RANGE if not. The swarm calls do not run this check themselves (it
 * is a full pass over the matrix); both builders produce matrices that hold. */
dpso_status dpso_check_dist(const int32_t *d_dist, int32_t n, void *d_work, size_t work_bytes,
                            int64_t *h_bad, void *stream);

/* Bytes of device workspace dpso_build_dist needs for this scene size. */
size_t dpso_dist_work_bytes(int32_t n, int32_t n_boxes);

/* Travelling costs between all viewpoints (Sect. 2.2-2.3): the cost of the
 * shortest path in the visibility graph whose nodes are the viewpoints and
 * the corners of the inflated boxes. A straight flight is allowed iff it
 * misses the open interior of every inflated box; it costs its Euclidean
 * length rounded half up to whole mm. Writes d_dist (device int32 [n][n]).
 * d_work (device, dpso_dist_work_bytes) is scratch. Synchronises `stream`.
 * Returns DPSO_E_RANGE if a finite path cost reaches DPSO_D_INF. */
dpso_status dpso_build_dist(const dpso_scene *scene, int32_t *d_dist, void *d_work,
                            size_t work_bytes, void *stream);

/* Largest workspace of dpso_build_dist_noalloc (32 MiB): enough for visibility
 * graphs of up to 2880 nodes (n + 8 * n_boxes). */
#define DPSO_NOALLOC_WORK_BYTES 33554432

/* dpso_build_dist without a workspace argument, for callers that cannot
 * allocate device memory (serving loops, harnesses that forbid allocation).
 * The same kernels and result as dpso_build_dist; the workspace is a static
 * device buffer of DPSO_NOALLOC_WORK_BYTES that the library holds on every
 * device it runs on until the process ends. Calls nothing that allocates.
 * Returns DPSO_E_NOMEM if dpso_dist_work_bytes(n, n_boxes) exceeds
 * DPSO_NOALLOC_WORK_BYTES (checked before any device work); the other
 * errors as dpso_build_dist. Calls on one device share that buffer: calls
 * that overlap in time on one device (other host threads, other streams)
 * race and must be serialised by the caller. Synchronises `stream`, so it
 * cannot be captured into a graph. */
dpso_status dpso_build_dist_noalloc(const dpso_scene *scene, int32_t *d_dist, void *stream);

/* Initial swarm (pseudo code of Sect. 3.3, deterministic initialisation of
 * Sect. 3.2.1): the first ceil(S * det_permille / 1000) particles start from
 * nearest-neighbour tours whose start labels are spread evenly over 0..n-1
 * (smallest label on ties); the others from Philox Fisher-Yates shuffles.
 * Velocities are empty, personal bests are the particles themselves and the
 * global best is the cheapest (lowest index on ties). d_state must hold
 * dpso_state_bytes(n, S, max_generations) bytes. Enqueues only. */
dpso_status dpso_init_nn(const int32_t *d_dist, int32_t n, const dpso_params *params,
                         void *d_state, size_t state_bytes, void *stream);

/* Runs up to `generations` more generations (eq. velocity, eq. position,
 * mutation, global-best update, edge exchange), stopping early once
 * max_generations or stall_limit is reached; resumes from the generation
 * the state holds, so run(a) followed by run(b) equals run(a + b). params
 * must be those given to dpso_init_nn. Enqueues only; a state that was not
 * initialised for (n, swarm_size) is reported as DPSO_E_STATE by the next
 * dpso_get_info / dpso_get_best. When the edge exchange is on and it stages
 * 16-bit rows (see dpso_state_bytes), the run first rewrites the state's
 * copy of D (two small kernels), so D may change between runs; D must meet
 * the contract that dpso_check_dist checks. */
dpso_status dpso_run(const int32_t *d_dist, int32_t n, const dpso_params *params, void *d_state,
                     size_t state_bytes, int32_t generations, void *stream);

/* Device time of each phase of the generation loop, summed over a
 * dpso_run_profiled call (HIP events recorded on `stream` between phases). */
typedef struct {
    float ms_total;     /* first to last event                                 */
    float ms_move;      /* velocity / position update, cost, personal best     */
    float ms_mutation;  /* duplicate marking, ranking and reshuffles           */
    float ms_gbest;     /* both global-best reductions (with the edge exchange
                           on, the second one also runs the end of the
                           generation)                                         */
    float ms_exchange;  /* 2-opt edge exchange                                 */
    float ms_control;   /* end-of-generation step when it runs on its own (the
                           edge exchange off), else 0                          */
    int32_t generations;        /* generations enqueued                        */
    int32_t exchange_launches;  /* edge-exchange kernel launches               */
} dpso_phase_times;

/* dpso_run with a HIP event between the phases of every generation; fills
 * *times and synchronises `stream`. Results are identical to dpso_run. */
dpso_status dpso_run_profiled(const int32_t *d_dist, int32_t n, const dpso_params *params,
                              void *d_state, size_t state_bytes, int32_t generations,
                              dpso_phase_times *times, void *stream);

/* dpso_run with a HIP event just before and just after every edge-exchange
 * launch, and no others: times->ms_exchange receives their summed device
 * time, times->exchange_launches and times->generations the counts, the
 * other fields 0. Synchronises `stream`. Two events a generation instead of
 * dpso_run_profiled's six, for timing whole runs with the exchange kernel's
 * own duration. Results are identical to dpso_run. */
dpso_status dpso_run_timed(const int32_t *d_dist, int32_t n, const dpso_params *params, void *d_state,
                           size_t state_bytes, int32_t generations, dpso_phase_times *times, void *stream);

/* One swarm of a batch: its own distance matrix, parameters and state. */
typedef struct {
    const int32_t *d_dist;  /* device int32 [n][n]                          */
    int32_t n;
    dpso_params params;
    void *d_state;          /* dpso_state_bytes(n, swarm_size, max_generations) */
    size_t state_bytes;
} dpso_batch_item;

/* Bytes of device workspace for the tables of a batch of `count` swarms. */
size_t dpso_batch_work_bytes(int32_t count);

/* dpso_init_nn for many independent swarms (instances of different n and
 * swarm size) in one pass of batched launches. d_work (device,
 * dpso_batch_work_bytes(count)) receives the batch tables. Synchronises
 * `stream`. */
dpso_status dpso_init_batch(const dpso_batch_item *items, int32_t count, void *d_work,
                            size_t work_bytes, void *stream);

/* dpso_run for many independent swarms: every generation is one launch per
 * phase covering all instances' particles (one per move class and one per
 * edge-exchange class, the 16-bit row classes of a small batch merged into
 * one (dpso_batch_merge_set), ordered by dpso_batch_order_get), so each kernel
 * boundary synchronises the whole batch and the hardware scheduler balances
 * instances of uneven size. The launches go to `stream` as they are
 * enqueued (no graph: capturing thousands of nodes cost more than it saved).
 * Each instance's result is identical to dpso_run on it alone. Synchronises
 * `stream`. */
dpso_status dpso_run_batch(const dpso_batch_item *items, int32_t count, int32_t generations,
                           void *d_work, size_t work_bytes, void *stream);

/* Progress counters. Synchronises `stream`. */
dpso_status dpso_get_info(const void *d_state, dpso_info *info, void *stream);

/* The answer of the method: its global best (the particle with the best
 * fitness, kept across generations; pseudo code of Sect. 3.3). h_tour (host
 * [n]) receives the tour as stored, *h_cost its cost, *h_generation the
 * generations completed; h_trace (nullable, host [generation + 1]) the
 * global-best cost after each generation. Any output pointer may be NULL.
 * Synchronises `stream`. */
dpso_status dpso_get_best(const void *d_state, int32_t *h_tour, int64_t *h_cost,
                          int32_t *h_generation, int64_t *h_trace, void *stream);

/* Copies the whole swarm to host arrays (checkpoint, inspection). n and
 * swarm_size must match the state. Synchronises `stream`. */
dpso_status dpso_export_state(const void *d_state, int32_t n, int32_t swarm_size,
                              dpso_host_state *out, void *stream);

/* Replaces the swarm with host arrays (resume from a checkpoint). The state
 * must have been initialised for (n, swarm_size); trace entries
 * 0..generation are copied. Tours must be permutations of 0..n-1 and every
 * velocity a canonical difference T - x of two tours, as the method
 * produces (checked on the host; DPSO_E_INVAL otherwise). Synchronises
 * `stream`. */
dpso_status dpso_import_state(void *d_state, size_t state_bytes, int32_t n, int32_t swarm_size,
                              const dpso_host_state *in, void *stream);

/* ------------------------------------------------------------- tuning
 * How the generation loop is laid out on the GPU, per instance: threads per
 * particle in the move, and how the edge exchange stages rows of D. Every
 * configuration computes the same result bit for bit; only the speed
 * differs. The library keeps one table per device, keyed by the bucket of n
 * (n in (2^(b-1), 2^b], b = 1 .. 12) and the bucket of the particles that run
 * together (the swarm of a single-instance call, the batch's total particles
 * in a batched call: <= 128, <= 512, <= 1024, <= 2048, <= 8192, more). An
 * empty entry takes the built-in default. The table lives in process memory;
 * the Python package saves and reloads it per device. */
#define DPSO_ROWS_AUTO 0  /* the default for n                                  */
#define DPSO_ROWS_U16 1   /* one wavefront per particle, rows of the 16-bit copy
                             of D (8 <= n <= 1024), candidates checked exactly  */
#define DPSO_ROWS_I32 2   /* one wavefront per particle, int32 rows (n <= 1024)  */
#define DPSO_ROWS_BLOCK 3 /* one workgroup per particle, int32 rows (any n)     */
#define DPSO_ROWS_U16_PAIR 4 /* 16-bit rows, two wavefronts per particle, each
                                sweeping about half of the neighbourhood (for
                                128 < n <= 1024; smaller n take DPSO_ROWS_U16) */
#define DPSO_ROWS_U16_QUAD 5 /* 16-bit rows, four wavefronts per particle (for
                                256 < n <= 1024; smaller n take DPSO_ROWS_U16_PAIR) */

typedef struct {
    int32_t move_threads;  /* 64, 128, 256 or 512 threads per particle (0: default);
                              n must be at most 16 * move_threads               */
    int32_t exchange_rows; /* DPSO_ROWS_*; a form that does not serve an n of the
                              bucket falls back: U16_QUAD to U16_PAIR up to
                              n = 256, U16_PAIR to U16 up to n = 128, U16 below 8
                              to the default                                    */
} dpso_tuning;

/* The configuration the library uses for an instance of n viewpoints among
 * `particles` particles launched together, on the current device. The
 * exchange form is reported as resolved for n (never DPSO_ROWS_AUTO). Host
 * only. */
dpso_status dpso_tuning_get(int32_t n, int32_t particles, dpso_tuning *out);

/* Sets the table entry of the bucket holding (n, particles) on the current
 * device; `t` NULL clears it. DPSO_E_RANGE if move_threads cannot serve the
 * bucket's largest n, or an int32 or 16-bit wavefront form is asked for
 * above n = 1024; DPSO_E_INVAL for other values. Calls racing with runs on
 * other threads see either entry. Host only. */
dpso_status dpso_tuning_set(int32_t n, int32_t particles, const dpso_tuning *t);

/* Clears the whole table of the current device (and restores the default
 * batch order). Host only. */
dpso_status dpso_tuning_reset(void);

/* Order of the particles in each batched move and edge-exchange launch, per
 * device; results are the same in every order. */
#define DPSO_ORDER_DEFAULT 0 /* the library's choice (DPSO_ORDER_LPT)            */
#define DPSO_ORDER_INDEX 1   /* instances in the order of the batch               */
#define DPSO_ORDER_LPT 2     /* most work first (swarm x n^2 in the exchange,
                                swarm x n in the move)                             */
#define DPSO_ORDER_XCD 3     /* LPT order dealt to eight groups of balanced work,
                                one per XCD (workgroups go to the XCDs in turn), so
                                an instance's particles share one L2; falls back to
                                LPT when the groups cannot be balanced            */

/* Sets the batch order of the current device. DPSO_E_INVAL for an unknown
 * value. Host only. */
dpso_status dpso_batch_order_set(int32_t order);

/* The batch order in use on the current device (never DPSO_ORDER_DEFAULT).
 * Host only. */
int32_t dpso_batch_order_get(void);

/* Merged edge-exchange launches in batched runs, per device. Instances whose
 * exchange stages 16-bit rows (one wavefront per particle) fall into classes
 * by the columns each lane holds (n up to 64, 128, 256, 512, 1024). A batch of
 * at most `max_particles` particles runs all of them in one launch, each
 * workgroup running its own instance's class code, so instances of different
 * n run side by side; a larger batch launches the classes one after another.
 * Results are the same either way. 0 never merges; a negative value restores
 * the default. Host only. */
#define DPSO_MERGE_DEFAULT_PARTICLES 8192
dpso_status dpso_batch_merge_set(int64_t max_particles);

/* The merge limit in use on the current device. Host only. */
int64_t dpso_batch_merge_get(void);

typedef struct {
    dpso_tuning config;
    float ms;         /* best of two timed runs of `generations` generations  */
    uint64_t digest;  /* FNV-1a of the swarm after the run (tours, personal
                         bests, velocities, costs, global best, trace, counters) */
} dpso_tune_result;

/* Autotuner: times `generations` generations of the given swarm under each
 * candidate configuration (threads per particle in the move, then the
 * exchange's row form with the fastest move; the two phases are separate
 * kernels, so their times add) and records the fastest in the table entry of
 * (n, swarm_size). Every candidate starts from the same snapshot of the state
 * (kept in d_scratch, at least state_bytes) and the state is restored at the
 * end, so the call leaves d_state as it found it. The candidates' digests
 * must agree: a disagreement returns DPSO_E_STATE and records nothing.
 * results (nullable, max_results entries) receive every timed candidate in
 * order, *n_results their count, *chosen (nullable) the pick. The state must
 * be initialised and at least `generations` generations short of
 * max_generations. Synchronises `stream`. */
dpso_status dpso_autotune(const int32_t *d_dist, int32_t n, const dpso_params *params, void *d_state,
                          size_t state_bytes, int32_t generations, void *d_scratch, size_t scratch_bytes,
                          dpso_tune_result *results, int32_t max_results, int32_t *n_results,
                          dpso_tuning *chosen, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DPSO_H */
