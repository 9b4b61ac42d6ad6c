/*
 * gtmp.h -- C ABI of the MI355X (gfx950) implementation of the data-parallel
 * hot path of Global Tensor Motion Planning with a straight-line local
 * planner ("Anytime Global Tensor Motion Planning", Coumar, Le, Kingston).
 *
 * The planner:  sample a layered multipartite graph of waypoints (Sec. III-A),
 * realise every adjacent-layer edge with the straight-line local planner and
 * collision-check its interpolated states (Sec. III-B), run the min-plus
 * Bellman recursion backwards over the layers (Sec. IV-B) and follow the
 * minimisers from the start (Alg. 1, extraction).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Layers are numbered as in Alg. 1: intermediate layers m = 0..M-1, the
 *   start q0 precedes layer 0 and the goals follow layer M-1.
 * - Pointers named in the comments as "device" must point to device memory of
 *   the current HIP device; "host" pointers are read before the call returns.
 *   The caller owns every buffer; the library never allocates, frees or
 *   keeps a pointer after the call returns.
 * - Each call validates its arguments on the host first.  On an invalid
 *   argument it returns GTMP_EINVAL, enqueues nothing and writes nothing.
 *   GTMP_EHIP means a HIP launch or API call failed.  gtmp_last_error()
 *   returns a thread-local message describing the last failure.
 * - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *   the call returns without waiting for it.  Results are valid once the
 *   stream has reached the call.
 * - All floating-point work is FP32.  Samples, costs and values are float32.
 */
#ifndef GTMP_H
#define GTMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
typedef int gtmp_status;
#define GTMP_OK 0
#define GTMP_ENOPATH 1      /* informational: the graph holds no feasible chain */
#define GTMP_INCOMPLETE 2   /* informational: a round limit stopped an iterative call early */
#define GTMP_EINVAL (-1)    /* invalid argument; nothing was enqueued */
#define GTMP_EHIP (-2)      /* a HIP call failed */
#define GTMP_EWORKSPACE (-3) /* workspace too small */

/* Human-readable name of a status code (static storage). */
const char *gtmp_status_string(gtmp_status s);
/* Message of the last failure on the calling thread ("" if none). */
const char *gtmp_last_error(void);
/* Library version string. */
const char *gtmp_version(void);

/* ---------------------------------------------------------------- limits */
#define GTMP_MAX_DOF 8             /* configuration dimension d */
#define GTMP_MAX_JOINTS 8          /* revolute joints of a serial arm */
#define GTMP_MAX_ROBOT_SPHERES 64  /* collision spheres of a serial arm */
#define GTMP_MAX_H 256             /* interpolated states per edge */

/* --------------------------------------------------------------- problem */
/* Sizes and constants of one layered graph (Sec. III-A; Alg. 1 data).
 *   d        configuration dimension, 1..GTMP_MAX_DOF
 *   M        intermediate layers (>= 1)
 *   N        samples per layer (>= 1)
 *   G        goals (>= 1)
 *   H        interpolated states per edge, endpoints included (2..GTMP_MAX_H)
 *   lo, hi   sampling box, lo[j] < hi[j] for j < d
 *   penalty  cost added to an edge whose local planner fails; +INF gives the
 *            paper's absent edge (Sec. IV-B: an absent edge costs +inf)
 *   max_edge_len  length limit ell of the local planner query (Sec. III-B):
 *            an edge longer than this fails; +INF disables the limit.     */
typedef struct gtmp_problem {
    int32_t d, M, N, G, H;
    float lo[GTMP_MAX_DOF];
    float hi[GTMP_MAX_DOF];
    float penalty;
    float max_edge_len;
} gtmp_problem;

/* ----------------------------------------------------------------- robot */
#define GTMP_ROBOT_POINT 0   /* configuration = point in workspace (d == wdim) */
#define GTMP_ROBOT_DH_ARM 1  /* revolute serial arm, standard DH, sphere model  */

/* Host memory, read during the call.  For a DH arm, joint i (0-based) has the
 * link transform Rz(q_i + dh[i][3]) Tz(dh[i][2]) Tx(dh[i][0]) Rx(dh[i][1]),
 * chained from a base frame at the origin; sphere k sits on link
 * sph_link[k] (1..n_joints) at fraction sph_t[k] from frame origin
 * o_{L-1} to o_L, with radius sph_r[k].  Spheres must be listed in
 * non-decreasing link order.  A twist dh[i][1] within 1e-7 rad of 0 or
 * +-pi/2 (the FP32 value nearest pi/2 is 4.4e-8 off) is taken as exactly that angle (its cosine and sine as 1 / 0 or
 * 0 / +-1); any other twist as given.  A point robot ignores every field but
 * kind. */
typedef struct gtmp_robot {
    int32_t kind;
    int32_t n_joints;   /* == d for an arm */
    int32_t n_spheres;  /* 1..GTMP_MAX_ROBOT_SPHERES for an arm */
    int32_t reserved;
    float dh[GTMP_MAX_JOINTS][4]; /* (a, alpha, d, theta_offset) */
    int32_t sph_link[GTMP_MAX_ROBOT_SPHERES];
    float sph_t[GTMP_MAX_ROBOT_SPHERES];
    float sph_r[GTMP_MAX_ROBOT_SPHERES];
} gtmp_robot;

/* ----------------------------------------------------------------- scene */
/* Obstacles in a workspace of dimension wdim (2 or 3; a point robot needs
 * wdim == d, an arm needs wdim == 3).  Device memory:
 *   spheres [n_spheres][wdim + 1]  (centre, radius)      -- circles in 2D
 *   boxes   [n_boxes][2 * wdim]    (centre, half extents), axis-aligned
 * A configuration is in collision iff its signed distance to the union of
 * obstacles is <= 0 (Sec. III: the free space is open).  Obstacle data must
 * be finite; the results for non-finite obstacles are unspecified.        */
typedef struct gtmp_scene {
    int32_t wdim;
    int32_t n_spheres;
    const float *spheres;
    int32_t n_boxes;
    const float *boxes;
} gtmp_scene;

/* ------------------------------------------------------------ a1 sampler */
/* Uniform layer samples (Alg. 1: "uniformly sample Q"; Sec. III-A: N
 * independent samples in each of the M layers).
 * Q: device float32 [M][N][d], written.
 * Coordinate j of sample n in layer m is lo[j] + u * (hi[j] - lo[j]) rounded
 * once to float32, u = (w >> 8) * 2^-24 with w word (j mod 4) of
 * Philox4x32-10 (Salmon et al., SC'11) at key (seed mod 2^32, seed div 2^32)
 * and counter (n, m, stage mod 2^32, j div 4).  Deterministic in
 * (seed, stage); `stage` separates the stages of the anytime loops. */
gtmp_status gtmp_sample_layers(const gtmp_problem *prob, uint64_t seed, uint64_t stage, float *Q,
                               void *stream);

/* -------------------------------------------------- a2-a4 edge checking */
#define GTMP_CHECK_FAST 0  /* endpoint pre-pass + early-exit interior checks */
#define GTMP_CHECK_FULL 1  /* every state of every edge, exact signed distance */

/* Tuning knobs; zero-initialise for the defaults. */
typedef struct gtmp_edge_opts {
    int32_t mode;             /* GTMP_CHECK_FAST (default) or GTMP_CHECK_FULL */
    int32_t states_per_iter;  /* point robots: interior states per lane and iteration (1,2,4,8; 0 = auto = 8) */
    int32_t block;            /* ignored: the interior kernels run 256-thread blocks */
    int32_t blocks_per_cu;    /* resident blocks per CU for the persistent interior kernel (0 = auto:
                                 the occupancy limit, at most 3 for point robots) */
    int32_t sphere_chunks;    /* arms: 0 (auto) = each robot sphere is tested exactly against the
                                 obstacles that its per-axis obstacle bins list (a conservative
                                 filter: the same decisions as testing every obstacle) when the
                                 scene has at most 64 obstacles, else as for 2; 1, 2 or 4 = every
                                 sphere against every obstacle, the spheres in this many chunks.
                                 Point robots, full check: 0 (auto) = the same bins, four states
                                 per lane (states_per_iter ignored), when the graph has at least
                                 1024 tiles of 256 edges and the scene 1 to 96 obstacles; other
                                 values (and lazy rounds) = every state against every obstacle */
    int32_t reserved[3];
    unsigned long long *stats; /* optional device [4]: states evaluated (those a walk of each
                                  edge's interior states in the check order, stopping at the
                                  first state in contact, evaluates; evaluations are counted
                                  whole, states_per_iter at a time), edges checked in the
                                  interior pass, exact sphere-obstacle tests made behind the
                                  obstacle bins (sphere_chunks 0), [3] unused.  Added to. */
    void *ev_begin;            /* optional hipEvent_t recorded on `stream` just before the
                                  interior (fast mode) or every-state (full mode) kernel */
    void *ev_end;              /* optional hipEvent_t recorded just after it */
} gtmp_edge_opts;

/* Bytes of device workspace gtmp_edge_check_cost needs for this problem. */
gtmp_status gtmp_edge_check_workspace_size(const gtmp_problem *prob, size_t *bytes);

/* Realise and cost every candidate edge (Sec. III-B; Alg. 1 "compute cost
 * matrices C_s, C_h, C_l"; SEV local planner of Sec. V).
 * Edge (x, y) is checked at the H states x + (h/(H-1)) (y - x), h = 0..H-1;
 * it fails if a state is in collision or |y - x| > max_edge_len.  Its cost
 * is |y - x| (Euclidean, configuration space) plus `penalty` if it failed.
 *   q0      device float32 [d]
 *   goals   device float32 [G][d]
 *   Q       device float32 [M][N][d]
 *   C_s     device float32 [N]           q0 -> layer 0 vertex v
 *   C_h     device float32 [M-1][N][N]   layer m vertex u (row) -> layer m+1 vertex v (column)
 *   C_l     device float32 [N][G]        layer M-1 vertex u -> goal g
 *   minsd   device float32 [E] or NULL   minimum signed distance over the edge's states
 *           (E = N + (M-1) N^2 + N G, ordered as C_s, C_h, C_l); forces GTMP_CHECK_FULL
 *   flags   device uint8 [E] or NULL     1 = local planner failed, same order as minsd
 *   prune   device uint8 [E] or NULL     nonzero = edge pruned by a surrogate: not checked,
 *           cost |y - x| + penalty, flag 1
 *   workspace, ws_bytes   device scratch of at least gtmp_edge_check_workspace_size bytes
 *   opts    host, may be NULL
 * C_h may be NULL when M == 1. */
gtmp_status gtmp_edge_check_cost(const gtmp_problem *prob, const gtmp_robot *robot, const gtmp_scene *scene,
                                 const float *q0, const float *goals, const float *Q, float *C_s, float *C_h,
                                 float *C_l, float *minsd, uint8_t *flags, const uint8_t *prune,
                                 void *workspace, size_t ws_bytes, const gtmp_edge_opts *opts,
                                 void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * edge check as gtmp_edge_check_cost, same kernels and results, with its
 * scratch taken from a static device array of GTMP_NOALLOC_SCRATCH_BYTES
 * (32 MiB) that the library holds on every GPU it runs on until the process
 * ends.  The call allocates and frees nothing; the caller still owns the
 * inputs and outputs.  Problems whose gtmp_edge_check_workspace_size exceeds
 * GTMP_NOALLOC_SCRATCH_BYTES are rejected with GTMP_EINVAL (the arm with
 * M = 8, N = 2048 needs 30.4 MB and fits).  `stream` must belong to the
 * current device.  Every call on one GPU shares that GPU's array and leaves
 * its contents behind: calls that overlap on one GPU (concurrent streams,
 * threads) race and must be serialised by the caller. */
#define GTMP_NOALLOC_SCRATCH_BYTES (32u << 20)
gtmp_status gtmp_edge_check_cost_noalloc(const gtmp_problem *prob, const gtmp_robot *robot,
                                         const gtmp_scene *scene, const float *q0, const float *goals,
                                         const float *Q, float *C_s, float *C_h, float *C_l, float *minsd,
                                         uint8_t *flags, const uint8_t *prune, const gtmp_edge_opts *opts,
                                         void *stream);

/* Signed distance / collision flag of a batch of configurations (the state
 * test of Sec. III used by the edge check).  X device float32 [n][d];
 * sd device float32 [n] or NULL (exact signed distance); coll device
 * uint8 [n] or NULL (1 iff sd <= 0). */
gtmp_status gtmp_state_check(const gtmp_robot *robot, const gtmp_scene *scene, int32_t d, int64_t n,
                             const float *X, float *sd, uint8_t *coll, void *stream);

/* ------------------------------------------------- path shortcutting */
/* Shortcutting of planned paths, simp() of Alg. 1 ao-gtmp (Sec. IV-E); the
 * paper uses it without a definition.  Reading implemented: for each of B
 * paths of K waypoints w_0 .. w_{K-1}, the shortcut w_i -> w_j (i < j) passes
 * iff none of its H_ij = (j - i)(H - 1) + 1 states w_i + (h/(H_ij - 1))
 * (w_j - w_i), h = 0 .. H_ij - 1 (endpoints exact), collides, with the state
 * test of gtmp_state_check; a consecutive pair is thus tested at the plan's
 * own H states.  The simplified path is the shortest chain w_0 -> w_{K-1}
 * over passing shortcuts, lengths |w_j - w_i| in FP32 as the edge check
 * computes them, summed from the goal backwards; among equal costs the
 * lowest next index.  A waypoint with a non-finite coordinate fails every
 * shortcut that starts or ends at it.
 *   wp      device float32 [B][K][d], the paths (e.g. gtmp_extract_path's wp)
 *   valid   device uint8 [B][K][K], written: 1 iff i < j and w_i -> w_j passes
 *   idx     device int32 [B][K]: waypoint indices of the simplified path, then -1
 *   count   device int32 [B]: waypoints kept (0 when no chain passes)
 *   cost    device float32 [B]: its length (+inf when count is 0)
 *   out_wp  device float32 [B][K][d] or NULL: the kept waypoints, then NaN
 * Sizes: 2 <= K <= 64, 2 <= H <= GTMP_MAX_H, B K^2 <= 2^31; robot and scene
 * as for gtmp_edge_check_cost with d the configuration dimension. */
gtmp_status gtmp_simplify_paths(const gtmp_robot *robot, const gtmp_scene *scene, int32_t d, int32_t B, int32_t K,
                                int32_t H, const float *wp, uint8_t *valid, int32_t *idx, int32_t *count, float *cost,
                                float *out_wp, void *stream);

/* ------------------------------------- RRT-Connect local planner (LP) */
/* The second local planner of Sec. III / Sec. V: LP(x, y; s, ell) returns a
 * collision-free path from x to y inside the query ellipsoid
 * E(x, y; ell) = {z : |z - x| + |z - y| <= ell}, or fails.  RRT-Connect as
 * constructed in the proof of the paper's local-planner reach proposition:
 * the straight line first (that is the edge check above, so an edge it
 * passes is kept as a straight segment), then two trees rooted at x and y,
 * for iterations i = 0 .. budget-1: draw one sample, extend tree A towards
 * it by at most `step`, on success connect tree B to the new node by
 * repeated extensions, and swap the trees.  Decisions, all FP32 with a fixed
 * operation order (no fused multiply-add):
 *   ell      ell_factor * |y - x| (length summed in coordinate order)
 *   sample   attempt a (a < 4096) of iteration i: y_j = (w_j >> 8) 2^-23 - 1
 *            from Philox4x32-10 at key (seed) and counter
 *            (e, i, stage, (3 << 16) | (2a + j div 4)), e the flat edge id;
 *            accepted iff sum y_j^2 < 1 and z = c + H (r1 y_1, r2 y_2, ...) lies
 *            in the box, with the hyperspheroid map of gtmp_sample_informed
 *            for foci x, y and bound ell; the lowest accepted attempt is the
 *            sample, none = no extension in this iteration
 *   nearest  least squared distance summed in coordinate order, lowest node
 *            index on ties
 *   steer    d = sqrt(d2); d <= step: the target itself (reached); else
 *            p + (step / d) (q - p)
 *   check    states p + (h / (Hs - 1)) (q_new - p), h = 1 .. Hs - 1, with
 *            Hs = max(2, ceil(|q_new - p| / resolution) + 1); the extension
 *            fails if one collides (state test of gtmp_state_check)
 *   full     a tree holding tree_cap nodes extends no further
 * A path is the x tree's chain to the junction followed by the y tree's
 * chain to y; its cost is its length in FP32, summed over the segments from
 * x to y. */
typedef struct gtmp_rrtc_opts {
    int32_t budget;      /* s >= 1: iterations per call (one sample each) */
    int32_t tree_cap;    /* nodes per tree, 2 .. 4096, with the LDS limit 4 (2 d + 4) tree_cap + 256 <= 155648 */
    float step;          /* eta > 0: extension step (configuration units) */
    float resolution;    /* > 0, step / resolution <= 4096: spacing bound of checked states */
    float ell_factor;    /* >= 1: major axis of the query ellipsoid over |y - x| */
    int32_t reserved;
    unsigned long long *stats; /* optional device [6]: calls, successes, iterations, tree nodes, states
                                  checked, nearest-node distances evaluated.  Added to. */
} gtmp_rrtc_opts;

/* Bytes of device workspace gtmp_rrtc_repair needs for this problem. */
gtmp_status gtmp_rrtc_workspace_size(const gtmp_problem *prob, size_t *bytes);

/* Run the RRT-Connect LP on every edge whose straight line failed (flags[e]
 * == 1 as written by gtmp_edge_check_cost) with both endpoints
 * collision-free and |y - x| <= max_edge_len.  A call that succeeds replaces
 * the edge's cost by its path length and sets flags[e] = 2; a failed call
 * leaves both.  Calls are keyed by (seed, stage, e), so a call is
 * reproducible on its own (gtmp_rrtc_local_path).  Arguments as for
 * gtmp_edge_check_cost; flags device uint8 [E], required (read and
 * written); E < 2^32. */
gtmp_status gtmp_rrtc_repair(const gtmp_problem *prob, const gtmp_robot *robot, const gtmp_scene *scene,
                             const float *q0, const float *goals, const float *Q, float *C_s, float *C_h, float *C_l,
                             uint8_t *flags, uint64_t seed, uint64_t stage, const gtmp_rrtc_opts *opts,
                             void *workspace, size_t ws_bytes, void *stream);

/* The local path of edge `edge` (flat id, order C_s | C_h | C_l) by the same
 * call gtmp_rrtc_repair makes: path device float32 [2 tree_cap][d] receives
 * the waypoints from x to y, count device int32 [1] their number (0 when
 * the call fails), cost device float32 [1] the length (+inf on failure),
 * equal to the cost the repair wrote.  No workspace. */
gtmp_status gtmp_rrtc_local_path(const gtmp_problem *prob, const gtmp_robot *robot, const gtmp_scene *scene,
                                 const float *q0, const float *goals, const float *Q, uint64_t edge, uint64_t seed,
                                 uint64_t stage, const gtmp_rrtc_opts *opts, float *path, int32_t *count, float *cost,
                                 void *stream);

/* -------------------------------------------- lazy edge realisation */
/* The lazy variant the paper names as future work (realise only a subset of
 * the adjacent-layer pairs).  Every edge starts at its optimistic cost: its
 * length, or length + penalty when an endpoint collides or it exceeds
 * max_edge_len (known without a check).  Rounds of: backward sweep and
 * extraction (as gtmp_minplus_sweep / gtmp_extract_path); stop when every
 * edge of the extracted path has been checked; else the forward sweep
 * F[m][v] = min_u F[m-1][u] + C(u, v) and a straight-line check (the fast
 * mode of gtmp_edge_check_cost) of the unchecked edges of the extracted path
 * and of every unchecked edge (u, v) whose best path through it,
 * F(u) + C(u, v) + V(v), costs at most (1 + band) V_s.
 * Checked costs are the true ones and unchecked ones are lower bounds, so
 * the final path is optimal for the fully checked graph and its cost equals
 * the full check's V_s (the same FP32 edge costs summed in the same order).
 *   Q, q0, goals, C_*, V, A, V_s, a_s, idx, wp, cost  as for the plain calls
 *   flags   device uint8 [E], written: 0 free, 1 failed, 0xFF not checked
 *   band    >= 0; 0 checks only edges on currently optimal paths
 *   max_rounds  >= 1: rounds before giving up (GTMP_INCOMPLETE is returned
 *           and the path may hold unchecked edges)
 *   stats   optional device [2]: rounds, edges checked.  Added to.
 *   rounds  optional host int32 [1]: rounds run
 * The call reads one flag back per round (it synchronises `stream`). */
gtmp_status gtmp_lazy_workspace_size(const gtmp_problem *prob, size_t *bytes);
gtmp_status gtmp_plan_lazy(const gtmp_problem *prob, const gtmp_robot *robot, const gtmp_scene *scene,
                           const float *q0, const float *goals, const float *Q, float *C_s, float *C_h, float *C_l,
                           uint8_t *flags, float *V, int32_t *A, float *V_s, int32_t *a_s, int32_t *idx, float *wp,
                           float *cost, float band, int32_t max_rounds, unsigned long long *stats, int32_t *rounds,
                           void *workspace, size_t ws_bytes, const gtmp_edge_opts *edge_opts, void *stream);

/* --------------------------------------------------- a5 min-plus sweep */
/* Backward value iteration on the layered DAG (Sec. IV-B; Alg. 1):
 *   V[M-1][u] = min_g C_l[u][g] + V_g[g]
 *   V[m][u]   = min_v C_h[m][u][v] + V[m+1][v],   m = M-2 .. 0
 *   V_s       = min_u C_s[u] + V[0][u]
 * A[m][u] / a_s receive the minimiser (lowest index among equal values; -1
 * when the minimum is +inf).  One backward pass reaches the fixed point of
 * Alg. 1's repeated sweeps on this depth-(M+1) DAG.
 *   Vg      device float32 [G] or NULL (zeros: terminal cost-to-go 0)
 *   V       device float32 [M][N];  A device int32 [M][N]
 *   V_s     device float32 [1];     a_s device int32 [1]            */
gtmp_status gtmp_minplus_sweep(int32_t M, int32_t N, int32_t G, const float *C_s, const float *C_h,
                               const float *C_l, const float *Vg, float *V, int32_t *A, float *V_s,
                               int32_t *a_s, void *stream);

/* ------------------------------------------------------ a6 extraction */
/* Follow the minimisers from the start (Alg. 1 extraction; Sec. IV-B).
 *   idx   device int32 [M+1]: idx[m] = chosen vertex of layer m, idx[M] = goal
 *   wp    device float32 [M+2][d]: q0, Q[0][idx0], ..., Q[M-1][idx_{M-1}], goals[idx_M]
 *   cost  device float32 [1] = V_s
 * With no path (a_s < 0 or V_s = +inf) idx is filled with -1, wp with
 * NaN and cost with +inf. */
gtmp_status gtmp_extract_path(int32_t M, int32_t N, int32_t G, int32_t d, const int32_t *a_s,
                              const int32_t *A, const float *V_s, const float *Q, const float *q0,
                              const float *goals, int32_t *idx, float *wp, float *cost, void *stream);

/* --------------------------------------- a7 growing-budget sampler */
/* Alg. 1 expand-samples (Sec. IV-E): grow every layer from n_old to N samples,
 * layer by layer in increasing m.  Each new slot (m, n) flips the coin of the
 * sample mixture (Sec. III-A): heuristic half iff the top bit of word 0 of
 * Philox at counter (n, m, stage, 2 << 16) is set, and only when a bound
 * exists and both neighbour layers are non-empty (layer -1 = {q0}, layer M =
 * the goals; layer m-1 as already expanded, layer m+1 at its old size).  The
 * h-th heuristic slot of a layer takes the midpoint of the h-th closest
 * (layer m-1, layer m+1) pair, ranked by FP32 squared distance summed in
 * coordinate order without fused multiply-add, ties by (u, v) index; with
 * fewer pairs it falls back to the uniform half.  The uniform half draws
 * from the informed set {x : |x-q0| + |x-q_g| <= c} (goal 0) intersected with
 * the box, c = *c_best; see gtmp_sample_informed.  Without a bound (c = +inf
 * or c >= penalty) the uniform half is uniform in the box.
 *   Q_old  device float32 [M][n_old][d] (ignored when n_old == 0)
 *   Q_new  device float32 [M][N][d], written (the old samples are copied in)
 *   c_best device float32 [1]
 * Q_old and Q_new must not overlap. */
gtmp_status gtmp_expand_workspace_size(const gtmp_problem *prob, size_t *bytes);
gtmp_status gtmp_expand_samples(const gtmp_problem *prob, const float *q0, const float *goals, const float *Q_old,
                                int32_t n_old, float *Q_new, const float *c_best, uint64_t seed, uint64_t stage,
                                void *workspace, size_t ws_bytes, void *stream);

/* The same expansion with the heuristic half biased by the learned
 * surrogate (gtmp_surrogate below): of the 4 (N - n_old) closest pairs of a
 * layer (all pairs if fewer), only those whose FP32 midpoint gets a logit
 * <= tau_logit are used, in rank order; heuristic slots beyond them take
 * their uniform-half draw.  The uniform half is unchanged, so the coverage
 * and convergence results, which use only that half, still hold (Sec. III
 * Layered Sampling Model).  net->d must equal prob->d. */
struct gtmp_surrogate;
gtmp_status gtmp_expand_biased_workspace_size(const gtmp_problem *prob, size_t *bytes);
gtmp_status gtmp_expand_samples_biased(const gtmp_problem *prob, const float *q0, const float *goals,
                                       const float *Q_old, int32_t n_old, float *Q_new, const float *c_best,
                                       uint64_t seed, uint64_t stage, const struct gtmp_surrogate *net,
                                       float tau_logit, void *workspace, size_t ws_bytes, void *stream);

/* Draws of the uniform half of the growing-budget sampler for slots
 * (m, 0..count-1) at `stage`: uniform draws of the informed set of Sec. IV-E,
 * X_f(c) = {x : |x-q0| + |x-q_g| <= c} (goal 0), intersected with the box,
 * by rejection from one of two proposal regions that both contain it:
 *   R  the hyperspheroid's frame box: a cube point y kept iff |y| < 1, mapped
 *      by the direct method of Gammell et al. (2018),
 *      x = (q0 + q_g)/2 + H (c/2 y_1, r2 y_2, ...), r2 = sqrt(c^2 - c_min^2)/2,
 *      c_min = |q_g - q0|, H = I - (2/w.w) w w^T, w = e_1 - (q_g - q0)/c_min;
 *      x kept iff inside the box;
 *   C  the hyperspheroid's axis-aligned bounding box (half-extents
 *      sqrt(sum_j (H_ij r_j)^2) (1 + 2^-10)) clipped to the box: x = mid +
 *      half y, kept iff inside the box and sqrt(|x-q0|^2) + sqrt(|x-q_g|^2)
 *      <= c.
 * C is used iff its volume (product of its sides) is below R's
 * (prod 2 r_i).  Everything is FP32 with a fixed operation order (sums in
 * coordinate order, no fused multiply-add); y_i = (w_i >> 8) 2^-23 - 1 from
 * Philox words at counter (n, m, stage, (1 << 16) | (2 a + j div 4)) for
 * attempt a.  Past 16384 attempts (probability below e^-499 wherever 3 % of
 * the proposals are accepted) x is the centre (q0 + q_g)/2.  Without a bound
 * (c = +inf or c >= penalty) x is the box sample of attempt 0's words.
 *   X         device float32 [count][d]
 *   attempts  device int32 [count] or NULL: attempts used, 0 unbounded, -1 cap reached
 *   workspace device, at least 1024 bytes */
gtmp_status gtmp_sample_informed(const gtmp_problem *prob, const float *q0, const float *goals, const float *c_best,
                                 uint64_t seed, uint64_t stage, int32_t m, int32_t count, float *X, int32_t *attempts,
                                 void *workspace, void *stream);

/* ------------------------------------------------- a7 anytime policies */
#define GTMP_ANYTIME_RESTART 0 /* Anytime-GTMP: fixed (M, N), fresh samples every stage (Sec. IV-D) */
#define GTMP_ANYTIME_GROWING 1 /* AO-GTMP: growing (M, N), informed expansion (Sec. IV-E) */

typedef struct gtmp_anytime_opts {
    int32_t mode;
    int32_t max_stages;         /* stage cap (restart: the number of stages) */
    int32_t M_min, M_max;       /* growing: layer schedule */
    int32_t N_min, N_max;       /* growing: samples per layer */
    int32_t use_graph;          /* restart: capture one stage as a hipGraph and replay it */
    float bias_tau;             /* growing: logit threshold of the surrogate bias */
    const struct gtmp_surrogate *bias_net; /* growing: surrogate biasing the heuristic half
                                              (gtmp_expand_samples_biased), NULL = off */
    int32_t simplify;           /* nonzero: shortcut each stage's path (simp() of Alg. 1, by
                                   gtmp_simplify_paths); needs M + 2 <= 64 (M_max + 2 growing) */
    const struct gtmp_rrtc_opts *lp; /* non-NULL: after each stage's straight-line check, the
                                        RRT-Connect repair (gtmp_rrtc_repair, keyed by seed and
                                        the stage index); use_graph is then ignored */
} gtmp_anytime_opts;

/* Bytes of device workspace gtmp_plan_anytime needs (sizes of prob for a
 * restart plan, of (M_max, N_max) for a growing one). */
gtmp_status gtmp_anytime_workspace_size(const gtmp_problem *prob, const gtmp_anytime_opts *opts, size_t *bytes);

/* Anytime policies with one homotopy class (|K| = 1): the archive keeps the
 * lowest-cost path, a later stage replaces it only with a strictly lower
 * cost (Alg. 1 anytime-gtmp / ao-gtmp; Sec. IV-C..E).
 * Restart: stage s plans (M, N) of prob on samples drawn with key `seed` at
 * stage s (gtmp_sample_layers).  Growing: starts at (M_min, N_min); after
 * each stage N doubles (capped at N_max) while N < N_max, after which M grows
 * by one per stage with every layer resampled (a new epoch); the loop ends
 * after the stage run at (M_max, N_max) or after max_stages stages.  Each
 * growing stage expands the samples with gtmp_expand_samples at stage s,
 * bounded by the archive's cost.
 * Outputs (device): best_cost [1]; best_idx [M_max + 1] and best_wp
 * [(M_max + 2) d] for the best stage's (M); best_meta [4] = (best stage, its
 * M, its N, stages run); stage_costs [max_stages].  prob->M, N give the
 * restart sizes; prob->G, H, d, box and penalty apply to both.  The whole
 * loop is enqueued on `stream` with no host synchronisation.
 * With opts->simplify the archive holds shortcut paths (Alg. 1): restart
 * compares the stage path's cost with the archived cost and, when lower,
 * stores the shortcut of the stage path; growing shortcuts every stage path
 * first and compares shortcut lengths, so the informed sampler is bounded by
 * the best shortcut length.  A stage path that no shortcut chain realises
 * (one through failed edges) is never stored.  best_cost is then the stored
 * shortcut's length, best_wp its waypoints followed by NaN rows, best_idx
 * the layer indices of the stage path it was cut from, and stage_costs[s]
 * the cost compared at stage s (restart: the stage path's; growing: its
 * shortcut's, +inf when none). */
gtmp_status gtmp_plan_anytime(const gtmp_problem *prob, const gtmp_robot *robot, const gtmp_scene *scene,
                              const float *q0, const float *goals, uint64_t seed, const gtmp_anytime_opts *opts,
                              float *best_cost, int32_t *best_idx, float *best_wp, int32_t *best_meta,
                              float *stage_costs, void *workspace, size_t ws_bytes, const gtmp_edge_opts *edge_opts,
                              void *stream);

/* ------------------------------------------------------ a8 batched plans */
/* One independent plan of a batch.  Robot by value (host memory); scene,
 * q0 and goals are device pointers.  mode GTMP_ANYTIME_RESTART runs
 * `stages` restart stages at (problem.M, problem.N) (stages = 1 is the plain
 * planner); GTMP_ANYTIME_GROWING runs the growing schedule of
 * gtmp_plan_anytime from (M_min, N_min) to (problem.M, problem.N). */
typedef struct gtmp_plan_desc {
    gtmp_problem problem;
    gtmp_robot robot;
    gtmp_scene scene;
    const float *q0;
    const float *goals;
    uint64_t seed;
    int32_t mode;
    int32_t stages;
    int32_t M_min;
    int32_t N_min;
} gtmp_plan_desc;

typedef struct gtmp_batch_opts {
    int32_t use_graph;        /* capture the whole batch (every stage, every policy) as one hipGraph
                                 and launch it; the instantiated graph is kept and launched again by
                                 later calls with the same plans, options, outputs and workspace */
    int32_t states_per_iter;  /* interior states per lane and iteration for point robots (0 = auto = 8) */
    int32_t sphere_chunks;    /* arms: as gtmp_edge_opts.sphere_chunks; 0 (auto) uses the obstacle bins
                                 when every arm plan's scene has at most 64 obstacles */
    int32_t blocks_per_cu;    /* resident blocks per CU of the persistent kernels (0 = auto) */
    unsigned long long *stats; /* optional device [4], as gtmp_edge_opts.stats */
} gtmp_batch_opts;

/* Bytes of device workspace gtmp_plan_batch needs for these plans. */
gtmp_status gtmp_batch_workspace_size(const gtmp_plan_desc *plans, int32_t n, const gtmp_batch_opts *opts,
                                      size_t *bytes);

/* Run n independent plans through batched kernels: per stage one sampling
 * launch, one vertex launch per robot group (2D points, 3D points, arms),
 * one edge pre-pass launch, one persistent interior launch per robot group
 * over the tiles of all its plans, max-M sweep launches covering every plan
 * and one finishing launch (start row, extraction, archive).  Each plan's
 * results equal those of gtmp_plan_anytime (or of one plain plan) with the
 * same seed.  Outputs (device), plans concatenated in order:
 *   best_cost   [n]
 *   best_idx    [sum_p (M_p + 1)]        M_p = plans[p].problem.M
 *   best_wp     [sum_p (M_p + 2) d_p]
 *   best_meta   [n][4] = (best stage, its M, its N, stages run)
 *   stage_costs [n][stage_stride], stage_stride >= the largest stage count
 * A plan's best_idx / best_wp hold the best stage's chain in their first
 * M + 1 / (M + 2) d entries (M = best_meta[1]); the rest is left as it was.
 * The call writes its tables into the workspace with a synchronous copy
 * after waiting for `stream`, then enqueues the stages, or with use_graph
 * captures them into a graph and launches it, asynchronously.  With use_graph
 * a later call with byte-identical plan descriptors, options, output
 * pointers and workspace only launches the kept graph (no host tables, no
 * wait), re-uploading the tables first (with the wait) if another batch used
 * that workspace in between.  At most 64 graphs are kept per process; past
 * that a call captures, launches and waits for its graph, then releases it. */
gtmp_status gtmp_plan_batch(const gtmp_plan_desc *plans, int32_t n, const gtmp_batch_opts *opts, float *best_cost,
                            int32_t *best_idx, float *best_wp, int32_t *best_meta, float *stage_costs,
                            int32_t stage_stride, void *workspace, size_t ws_bytes, void *stream);


/* ------------------------------------- class-augmented sweep (2D robots) */
/* Class-augmented value iteration (Sec. IV-B; Prop. 2) and the class-indexed
 * archive of Anytime-GTMP (Sec. IV-D) for point robots in the plane (d = 2).
 *
 * Class label: for each of k <= 16 representative points z_i (one inside
 * each obstacle that separates classes) the signed number of crossings of the
 * path with the upward ray {(z_x, y): y > z_y}, +1 moving in +x.  Labels add
 * along concatenation, and two start-to-goal paths avoiding the obstacles
 * have equal labels iff they wind equally around every z_i (the discrete form
 * of the h-signature).  Packed as two uint64 words per label: field i is
 * byte (i mod 8) of word (i / 8), value (count + 128), fields past k at 128;
 * chains have at most 127 edges (M <= 126), so no count leaves -127..127.
 * The crossing decision is FP32 with a fixed order: u, v straddle z_x
 * ((u_x < z_x) != (v_x < z_x)) and the crossing lies above z, i.e.
 * cr = fl(fl(dx * ey) - fl(dy * ex)) < 0 when dx > 0, > 0 when dx < 0, with
 * dx = v_x - u_x, dy = v_y - u_y, ex = z_x - u_x, ey = z_y - u_y.
 *
 * Sweep: for every vertex the least cost of a chain to a goal per label,
 * keeping at most L <= 64 labels per vertex (a full list keeps the L
 * cheapest; *overflow counts dropped labels: the result is exact when it is
 * 0).  Edges with cost >= penalty are absent.  Outputs for the start vertex:
 * labels [L][2], costs [L], chains [L][M+1] (layer indices, then the goal),
 * count [1] (classes found); device pointers; reps device float [k][2]. */
gtmp_status gtmp_class_sweep_workspace_size(int32_t M, int32_t N, int32_t L, size_t *bytes);
gtmp_status gtmp_class_sweep(int32_t M, int32_t N, int32_t G, int32_t L, const float *Q, const float *q0,
                             const float *goals, const float *C_s, const float *C_h, const float *C_l, float penalty,
                             const float *reps, int32_t k, uint64_t *labels, float *costs, int32_t *chains,
                             int32_t *count, uint32_t *overflow, void *workspace, size_t ws_bytes, void *stream);

/* Anytime-GTMP with the class archive: `stages` restart stages (samples of
 * key (seed, stage), edge check, class sweep), each class's best path kept
 * (a later stage replaces an entry only with a strictly lower cost).  Archive
 * (device, capacity cap): a_labels [cap][2], a_costs [cap], a_stage [cap],
 * a_wp [cap][M+2][2] waypoints, a_count [1]; overflow [1] counts labels
 * dropped by full vertex lists or a full archive.  prob->d must be 2 and
 * scene->wdim 2 (point robot). */
gtmp_status gtmp_class_anytime_workspace_size(const gtmp_problem *prob, int32_t L, size_t *bytes);
gtmp_status gtmp_plan_classes(const gtmp_problem *prob, const gtmp_scene *scene, const float *q0, const float *goals,
                              uint64_t seed, int32_t stages, const float *reps, int32_t k, int32_t L, int32_t cap,
                              uint64_t *a_labels, float *a_costs, int32_t *a_stage, float *a_wp, int32_t *a_count,
                              uint32_t *overflow, void *workspace, size_t ws_bytes, const gtmp_edge_opts *edge_opts,
                              void *stream);

/* ------------------------------------------------- a9 learned surrogate */
/* A small ReLU MLP that predicts whether a configuration collides, used only
 * to prune edges before the exact check and to bias the heuristic half of
 * the sample mixture (the paper leaves that half to any history-dependent
 * sampler, Sec. III Layered Sampling Model; it names learned functions among
 * possible local planners, Sec. II).  Every edge it does not prune is still
 * checked exactly.
 *
 * Network: features x = [q/pi, sin(2 pi B q/pi), cos(2 pi B q/pi)] with
 * B = fourier [16][d], computed in FP64, rounded once to BF16 and
 * zero-padded to 64; four hidden
 * layers a_l = bf16(relu(bf16(W_l) a_{l-1} + b_l)) of width 256 with FP32
 * accumulation; logit z = bf16(w5) . a_4 + b5 (FP32).  Loss: mean BCE with
 * logits.  Backward with the same rounding points: dz = (sigmoid(z) - y)/n,
 * dZ_l = bf16(dA_l * [a_l > 0]), dW_l = dZ_l^T a_{l-1}, db_l = sum_b dZ_l,
 * dA_{l-1} = dZ_l bf16(W_l), all sums FP32.
 *
 * Parameters live in caller buffers: FP32 master values `params` and their
 * BF16 copy `params_bf16` (round to nearest even), one flat array each, in
 * the order W1 [256][64], b1 [256], W2 [256][256], b2, W3, b3, W4, b4,
 * w5 [256], b5 [1]; gtmp_surrogate_layout gives the offsets. */
#define GTMP_SUR_WIDTH 256
#define GTMP_SUR_IN 64
#define GTMP_SUR_FREQ 16

typedef struct gtmp_surrogate {
    int32_t d;               /* configuration dimension, 1..GTMP_MAX_DOF */
    const float *fourier;    /* device [16][d] */
    float *params;           /* device FP32 [total], 16-byte aligned */
    uint16_t *params_bf16;   /* device BF16 bits [total], 16-byte aligned */
} gtmp_surrogate;

/* offsets[0..9] = W1 b1 W2 b2 W3 b3 W4 b4 w5 b5 (elements), offsets[10] = total. */
gtmp_status gtmp_surrogate_layout(int32_t offsets[11]);

/* params_bf16 <- bf16(params) (after the caller writes new FP32 values). */
gtmp_status gtmp_surrogate_refresh_bf16(const gtmp_surrogate *net, void *stream);

/* Workspace for gtmp_surrogate_grad with a batch of n rows, and for the
 * inference calls processing up to n rows per chunk. */
gtmp_status gtmp_surrogate_workspace_size(int64_t n, size_t *bytes);

/* Logits of n configurations X [n][d] (device) -> logits [n] (device).
 * Any n >= 0; processed in chunks that fit the workspace. */
gtmp_status gtmp_surrogate_infer(const gtmp_surrogate *net, int64_t n, const float *X, float *logits,
                                 void *workspace, size_t ws_bytes, void *stream);

/* Loss and gradient of the mean BCE on one batch: X [n][d], y [n] (0/1,
 * uint8), n a positive multiple of 256.  grad [total] FP32 in the parameter
 * layout (overwritten); loss [1]; logits [n] or NULL.  Deterministic: every
 * sum runs in a fixed order. */
gtmp_status gtmp_surrogate_grad(const gtmp_surrogate *net, int32_t n, const float *X, const uint8_t *y, float *grad,
                                float *loss, float *logits, void *workspace, size_t ws_bytes, void *stream);

/* One Adam step (Kingma and Ba 2015) on params with moments m, v (FP32
 * [total], caller-zeroed before step t = 1), then params_bf16 refreshed. */
gtmp_status gtmp_surrogate_adam(const gtmp_surrogate *net, const float *grad, float *m, float *v, int32_t t, float lr,
                                float beta1, float beta2, float eps, void *stream);

/* Training states for labels: X [2n][d].  Rows 0..n-1 are uniform in the
 * box (layer 0 of gtmp_sample_layers with M = 3, N = n, key (seed, stage));
 * row n + j is the interior state h = 1 + j mod (H - 2) of the edge from
 * layer-1 sample j to layer-2 sample j (t = h / (H - 1)), H = prob->H >= 3.
 * Only prob->d, the box and H are used.  Labels come from gtmp_state_check. */
gtmp_status gtmp_surrogate_label_states(const gtmp_problem *prob, uint64_t seed, uint64_t stage, int64_t n, float *X,
                                        void *stream);

/* Prune mask of a plan's edges: prune[e] = 1 iff the logit at the edge's
 * midpoint (u + v) / 2 exceeds tau_logit.  The midpoint is exact (FP64 of
 * the FP32 endpoints); its features are formed from per-sample phase tables
 * (sin and cos of pi B x / pi for each sample x) by angle addition in FP64,
 * then rounded to BF16 as in gtmp_surrogate_infer.  Edge order as
 * gtmp_edge_check_cost (C_s | C_h | C_l).  Pass the mask to
 * gtmp_edge_check_cost, which checks every unpruned edge exactly.
 *   vcoll   device uint8 [M][N] or NULL: nonzero = the sample Q[m][n]
 *           collides (e.g. gtmp_state_check's coll output on Q).  Only the
 *           candidate edges, those whose sample endpoints are all free, are
 *           inferred; every other edge gets prune 0 (its colliding endpoint
 *           fails it in the exact check's vertex pass) and logit NaN.  NULL:
 *           every edge is a candidate.  q0 and the goals count as free.
 *   tau_logit  not NaN (+inf prunes nothing)
 *   prune   device uint8 [E], every entry written
 *   logits  device float32 [E] or NULL, every entry written
 *   workspace  device, 256-byte aligned, of
 *           gtmp_surrogate_prune_workspace_size bytes (M N int32 free lists
 *           and a fragment-ordered copy of the BF16 weights).
 * Candidates are processed by a persistent kernel in index order; nothing
 * is read back to the host. */
gtmp_status gtmp_surrogate_prune_workspace_size(const gtmp_problem *prob, size_t *bytes);
gtmp_status gtmp_surrogate_prune(const gtmp_problem *prob, const gtmp_surrogate *net, const float *q0,
                                 const float *goals, const float *Q, const uint8_t *vcoll, float tau_logit,
                                 uint8_t *prune, float *logits, void *workspace, size_t ws_bytes, void *stream);

/* Pruning threshold of the surrogate for a free-edge recall (the calibration
 * that makes the pruning conservative: at least `recall` of the free edges
 * stay unpruned).  With n_free edges of flags[e] == 0, tau is the k-th
 * smallest of their logits (0-based, NaN ordered last),
 * k = ceil(recall * n_free) - 1 (FP64) clamped to [0, n_free - 1], so that
 * pruning logit > tau keeps at least recall * n_free of them; tau = +inf when
 * no edge is free.  Found on the device by a radix select; nothing is read
 * back and no memory is cleared with memset (the call can be captured).
 *   logits    device float32 [E] (e.g. gtmp_surrogate_prune's logits output)
 *   flags     device uint8 [E], the exact checker's flags (0 = free)
 *   recall    in (0, 1]
 *   tau       device float32 [1], written
 *   workspace device, 256-byte aligned, gtmp_surrogate_threshold_workspace_size bytes */
gtmp_status gtmp_surrogate_threshold_workspace_size(size_t *bytes);
gtmp_status gtmp_surrogate_threshold(const float *logits, const uint8_t *flags, int64_t E, double recall, float *tau,
                                     void *workspace, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GTMP_H */
