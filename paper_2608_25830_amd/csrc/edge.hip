// edge.hip -- realisation and costing of every candidate edge of the layered
// graph with the straight-line local planner (Sec. III-B; Alg. 1 "compute
// cost matrices C_s, C_h, C_l"; the SEV planner of Sec. V).
//
// Fast mode (default) runs three kernels:
//   1. k_vertices   : packs q0 | Q | goals into one vertex array and tests every
//                     vertex once.  The endpoints are states h = 0 and h = H-1
//                     of every edge that touches them, so an edge with a
//                     colliding endpoint fails without further work.
//   2. k_prepass    : one thread per edge, memory bound.  Writes the
//                     provisional cost |v-u| + penalty (and flag 1) for every
//                     edge and compacts the edges that still need their
//                     interior states checked into per-tile candidate lists.
//   3. k_interior   : persistent waves.  Each lane owns one candidate edge and
//                     evaluates its interior states in bisection order,
//                     stopping at the first collision; a lane whose edge is
//                     done takes the next candidate of the wave's current tile
//                     (ballot + mbcnt), so the wave stays full however the
//                     early exits fall.  Only edges found free are written
//                     again (cost |v-u|, flag 0).
// Full mode evaluates the exact signed distance of every state of every edge
// (lanes = states, wave-level segmented min per edge) and writes minsd.
#include "edge_common.hpp"

namespace gtmp {

// Tile cursors of the interior kernel: the tiles fall into kCursors
// contiguous ranges, one per XCD of the chip (blocks are dealt to the XCDs in
// turn), each counted by its own cursor 256 bytes from the next, so that the
// waves' atomics spread over several addresses instead of queueing on one.
constexpr int kCursors = 8;
constexpr int kCursorStride = 64;  // 32-bit words between two cursors
__host__ __device__ __forceinline__ uint32_t cursor_begin(uint32_t n_tiles, uint32_t c) {
    return (uint32_t)((uint64_t)n_tiles * c / kCursors);
}

// Statistics of the interior kernel.  Every wave writes its totals (states
// evaluated, edges taken, exact tests) to its own slot with plain stores, and
// k_wave_stats_sum adds the slots to the caller's counters after the kernel:
// a persistent grid's waves all finish at about the same time, and one atomic
// add per wave on the same three words then serialised into a tail of about
// 0.1 ms.  Waves past kStatWaves, and every wave of a grid under
// kStatSlotsMinWaves (where the extra launch costs more than the atomics),
// add their totals directly.
constexpr uint32_t kStatWaves = 16384;
constexpr uint32_t kStatSlotsMinWaves = 1024;

__global__ void __launch_bounds__(256) k_wave_stats_sum(const unsigned long long *__restrict__ w, uint32_t waves,
                                                        unsigned long long *stats) {
    // one slot per thread, a block's sums added with one atomic per counter
    __shared__ unsigned long long part[3][256 / kWave];
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long acc[3] = {0, 0, 0};
    if (i < waves)
        for (int c = 0; c < 3; ++c) acc[c] = w[4 * (size_t)i + c];
    const int lane = lane_id(), wv = threadIdx.x / kWave;
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off);
        if (lane == 0) part[c][wv] = acc[c];
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long t = 0;
        for (int k = 0; k < 256 / kWave; ++k) t += part[threadIdx.x][k];
        atomicAdd(&stats[threadIdx.x], t);
    }
}

// The per-wave slots of a grid of grid_blocks blocks of 256 threads (NULL:
// its waves add to the counters directly).
static unsigned long long *wave_stat_slots(const EdgeArgs &A, unsigned grid_blocks) {
    return A.stats && (uint64_t)grid_blocks * (256 / kWave) >= kStatSlotsMinWaves ? A.wstats : nullptr;
}

static void finish_wave_stats(const EdgeArgs &A, unsigned grid_blocks, hipStream_t s) {
    if (!A.stats || !A.wstats) return;
    const uint64_t all = (uint64_t)grid_blocks * (256 / kWave);
    const uint32_t waves = (uint32_t)(all < kStatWaves ? all : kStatWaves);
    hipLaunchKernelGGL(k_wave_stats_sum, dim3((waves + 255) / 256), dim3(256), 0, s, A.wstats, waves, A.stats);
}

// A wave's totals (lane 0 calls this).
__device__ __forceinline__ void store_wave_stats(const EdgeArgs &A, unsigned long long states,
                                                 unsigned long long edges, unsigned long long tests) {
    const uint32_t wid = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (A.wstats && wid < kStatWaves) {
        A.wstats[4 * (size_t)wid + 0] = states;
        A.wstats[4 * (size_t)wid + 1] = edges;
        A.wstats[4 * (size_t)wid + 2] = tests;
    } else {
        atomicAdd(&A.stats[0], states);
        atomicAdd(&A.stats[1], edges);
        atomicAdd(&A.stats[2], tests);
    }
}

// ------------------------------------------------------------------ plan
EdgePlan make_edge_plan(const gtmp_problem &p) {
    EdgePlan e{};
    e.d = p.d; e.M = p.M; e.N = p.N; e.G = p.G; e.H = p.H;
    e.penalty = p.penalty; e.max_len = p.max_edge_len;
    e.n_vertices = 1u + (uint32_t)p.M * (uint32_t)p.N + (uint32_t)p.G;
    e.rows = 1u + (uint32_t)(p.M - 1) * (uint32_t)p.N + (uint32_t)p.G;
    e.tiles_per_row = (uint32_t)((p.N + kTile - 1) / kTile);
    e.n_tiles = e.rows * e.tiles_per_row;
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t o = 0;
    e.off_verts = o; o = up(o + sizeof(float) * (size_t)vertex_stride(p.d) * e.n_vertices);
    e.off_vflag = o; o = up(o + e.n_vertices);
    e.off_tile_off = o; o = up(o + (size_t)e.n_tiles * kTile);
    e.off_tile_cnt = o; o = up(o + sizeof(uint32_t) * (size_t)e.n_tiles);
    e.off_counter = o; o = up(o + sizeof(uint32_t) * kCursorStride * kCursors);
    e.off_wstats = o; o = up(o + sizeof(unsigned long long) * 4 * kStatWaves);
    e.off_params = o; o = up(o + sizeof(ArmParams));
    e.off_grid = o; o = up(o + sizeof(ObsGrid));
    e.total = o;
    return e;
}

int interior_order(int H, uint8_t *order) {
    // breadth-first bisection of [0, H-1]
    int n = 0;
    int qa[GTMP_MAX_H], qb[GTMP_MAX_H];
    int head = 0, tail = 0;
    qa[tail] = 0; qb[tail] = H - 1; ++tail;
    while (head < tail) {
        const int a = qa[head], b = qb[head];
        ++head;
        if (b - a < 2) continue;
        const int mid = (a + b) / 2;
        order[n++] = (uint8_t)mid;
        qa[tail] = a; qb[tail] = mid; ++tail;
        qa[tail] = mid; qb[tail] = b; ++tail;
    }
    return n;
}


// Copy of the robot table (a kernel argument) into device memory.
__global__ void k_store_params(ArmParams R, ArmParams *dst) {
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&R);
    uint32_t *d = reinterpret_cast<uint32_t *>(dst);
    constexpr int n = sizeof(ArmParams) / 4;
    for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = src[i];
}

// The robot table for the interior kernel plus the tolerance of the expanded
// sphere test: tol = 2^-19 ((reach + max|c|)^2 + (max r_o + r0)^2) over the
// sphere obstacles (one wave, lanes 0..63 of the caller).  R is only read
// (the two computed words are substituted as the table is copied), so it
// stays in kernel-argument memory rather than being copied to per-lane
// scratch.
__device__ __forceinline__ void store_params_tol_wave(const ArmParams &R, ArmParams *dst, const SceneParams &S) {
    const int lane = threadIdx.x;
    float cmax = 0.f, rmax = 0.f;
    for (int o = lane; o < S.n_sph; o += kWave) {
        const float *c = S.sph + 4 * o;
        cmax = __builtin_fmaxf(cmax, __builtin_sqrtf(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]));
        rmax = __builtin_fmaxf(rmax, __builtin_fabsf(c[3]));
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        cmax = __builtin_fmaxf(cmax, __shfl_xor(cmax, off));
        rmax = __builtin_fmaxf(rmax, __shfl_xor(rmax, off));
    }
    // rounding of the bound itself: inflate by 1e-3 relative
    const float pc = (R.reach + cmax) * 1.001f, rr = (rmax + R.r0) * 1.001f;
    const float sph_tol = 0x1p-19f * (pc * pc + rr * rr);
    // Links near the base that no obstacle can reach: an obstacle (box of
    // half-extents h around c, grown by rho) is at distance dist(0, box) - rho
    // from the base, and a sphere of link L has |centre| <= link_reach[L-1];
    // while every obstacle is farther than (link_reach + r_max) (1 + 1e-3) +
    // 1e-6, no sphere of links 1..L can touch one (the exact test's rounding
    // is far inside that margin), and the bin filter may skip them.
    float dmin = __builtin_inff(), rk_max = 0.f;
    for (int o = lane; o < S.n_sph + S.n_box; o += kWave) {
        float dd;
        if (o < S.n_sph) {
            const float *c = S.sph + 4 * o;
            dd = __builtin_sqrtf(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]) - __builtin_fabsf(c[3]);
        } else {
            const float *b = S.box + 6 * (o - S.n_sph);
            float acc = 0.f;
            for (int i = 0; i < 3; ++i) {
                const float e = __builtin_fmaxf(__builtin_fabsf(b[i]) - __builtin_fabsf(b[3 + i]), 0.f);
                acc += e * e;
            }
            dd = __builtin_sqrtf(acc);
        }
        dmin = __builtin_fminf(dmin, dd != dd ? -__builtin_inff() : dd);  // NaN data: nothing is skipped
    }
    for (int k = lane; k < R.n_spheres; k += kWave) rk_max = __builtin_fmaxf(rk_max, R.r[k]);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        dmin = __builtin_fminf(dmin, __shfl_xor(dmin, off));
        rk_max = __builtin_fmaxf(rk_max, __shfl_xor(rk_max, off));
    }
    int k_first = 0;
    for (int L = 1; L <= R.n_joints; ++L) {
        if (!(dmin > (R.link_reach[L - 1] + rk_max) * 1.001f + 1e-6f)) break;
        k_first = R.lk_end[L - 1];
    }
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&R);
    uint32_t *d = reinterpret_cast<uint32_t *>(dst);
    constexpr int n = sizeof(ArmParams) / 4;
    constexpr int w_tol = offsetof(ArmParams, sph_tol) / 4, w_first = offsetof(ArmParams, k_first) / 4;
    for (int i = lane; i < n; i += kWave)
        d[i] = i == w_tol ? __float_as_uint(sph_tol) : i == w_first ? (uint32_t)k_first : src[i];
}

__global__ void __launch_bounds__(kWave) k_store_params_tol(ArmParams R, ArmParams *dst, SceneParams S) {
    store_params_tol_wave(R, dst, S);
}

__global__ void k_zero_u32(uint32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void __launch_bounds__(kGridBuildThreads) k_build_grid(SceneParams S, int wdim, float r_max,
                                                                        ObsGrid *G) {
    build_grid_block(S, wdim, r_max, G);
}

// An arm plan's obstacle bins (block 0) and its robot table with the sphere
// test's tolerance (block 1, first wave) in one launch of two blocks:
// neither reads what the other writes.
__global__ void __launch_bounds__(kGridBuildThreads) k_build_grid_params(SceneParams S, float r_max, ObsGrid *G,
                                                                         ArmParams R, ArmParams *dst) {
    if (blockIdx.x == 0) build_grid_block(S, 3, r_max, G);
    else if (threadIdx.x < kWave) store_params_tol_wave(R, dst, S);
}

// ------------------------------------------------------------------ 1. vertices
template <int KP>
__global__ void __launch_bounds__(256) k_vertices_arm(EdgeArgs A, ArmParams R, SceneParams S, const float *q0,
                                                      const float *goals, const float *Q, float *verts,
                                                      uint8_t *vflag) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < A.n_vertices;
    const uint32_t MN = (uint32_t)A.M * (uint32_t)A.N;
    float q[GTMP_MAX_JOINTS];
#pragma unroll
    for (int j = 0; j < GTMP_MAX_JOINTS; ++j) q[j] = 0.f;
    if (valid) {
        const float *src = i == 0 ? q0 : (i <= MN ? Q + (size_t)(i - 1) * A.d : goals + (size_t)(i - 1 - MN) * A.d);
#pragma unroll
        for (int j = 0; j < GTMP_MAX_JOINTS; ++j)
            if (j < A.d) q[j] = src[j];
#pragma unroll
        for (int j = 0; j < GTMP_MAX_JOINTS; ++j) verts[(size_t)i * A.dp + j] = q[j];
    }
    const v32f o = arm_fk<GTMP_MAX_JOINTS>(R, q);
    Probes<3, KP> P;
    arm_spheres<KP>(R, o, P);
    float pr[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) pr[k] = k < R.n_spheres ? R.r[k] : 0.f;
    const float gap = R.uniform_r ? probes_min_gap<3, KP, true>(P, pr, R.r0, S)
                                  : probes_min_gap<3, KP, false>(P, pr, R.r0, S);
    if (valid) vflag[i] = gap <= 0.f ? 1 : 0;
}

// Vertex flags of an arm through the obstacle bins (the same decisions as
// k_vertices_arm).
// Waves per block of the arm vertex kernel: a plan has few vertices, so
// one-wave blocks spread them over more CUs (and hold one queue each).
constexpr int kVertexGridWaves = 1;

template <int WG>
__global__ void __launch_bounds__(kVertexGridWaves * kWave) k_vertices_arm_grid(EdgeArgs A, ArmParams R,
                                                                                const float *q0,
                                                                                const float *goals, const float *Q,
                                                                                float *verts, uint8_t *vflag) {
    __shared__ GridLds<WG> glds_raw;
    __shared__ GridQueue<WG> gque[kVertexGridWaves];  // one queue per wave of the block
    // the vertex first, so that its loads and the bins' are in flight together
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < A.n_vertices;
    const uint32_t MN = (uint32_t)A.M * (uint32_t)A.N;
    float q[GTMP_MAX_JOINTS];
#pragma unroll
    for (int j = 0; j < GTMP_MAX_JOINTS; ++j) q[j] = 0.f;
    if (valid) {
        const float *src = i == 0 ? q0 : (i <= MN ? Q + (size_t)(i - 1) * A.d : goals + (size_t)(i - 1 - MN) * A.d);
#pragma unroll
        for (int j = 0; j < GTMP_MAX_JOINTS; ++j)
            if (j < A.d) q[j] = src[j];
    }
    copy_to_lds<grid_lds_bytes<WG>(), kVertexGridWaves * kWave>(&glds_raw, A.grid, threadIdx.x);
    if (valid) {
#pragma unroll
        for (int j = 0; j < GTMP_MAX_JOINTS; ++j) verts[(size_t)i * A.dp + j] = q[j];
    }
    __syncthreads();
    const ObsGrid &G = *reinterpret_cast<const ObsGrid *>(&glds_raw);
    float inv[3], off[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        inv[k] = G.inv[k];
        off[k] = G.off[k];
    }
    uint32_t tests = 0;
    const bool hit = arm_hit_grid<WG>(R, q, G.mask, G.rec, inv, off, gque[wave_in_block()], tests, valid);
    if (valid) vflag[i] = hit ? 1 : 0;
}

template <int W>
__global__ void __launch_bounds__(256) k_vertices_point(EdgeArgs A, SceneParams S, const float *q0,
                                                        const float *goals, const float *Q, float *verts,
                                                        uint8_t *vflag) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n_vertices) return;
    const uint32_t MN = (uint32_t)A.M * (uint32_t)A.N;
    const float *src = i == 0 ? q0 : (i <= MN ? Q + (size_t)(i - 1) * W : goals + (size_t)(i - 1 - MN) * W);
    Probes<W, 1> P;
#pragma unroll
    for (int j = 0; j < GTMP_MAX_DOF; ++j) verts[(size_t)i * A.dp + j] = j < W ? src[j] : 0.f;  // zeros past W
#pragma unroll
    for (int j = 0; j < W; ++j) P.p[j][0] = src[j];
    const float pr[1] = {0.f};
    const float gap = probes_min_gap<W, 1, true>(P, pr, 0.f, S);
    vflag[i] = gap <= 0.f ? 1 : 0;
}

// ------------------------------------------------------------------ 2. pre-pass
// (prepass_block in edge_common.hpp; shared with the batched planner)
// Block 0 also resets the interior kernel's tile cursors (read by nothing
// before that kernel, which the stream orders after this one).
template <int D>
__global__ void __launch_bounds__(kTile) k_prepass(EdgeArgs A) {
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < kCursors * kCursorStride; i += kTile) A.counter[i] = 0u;
    prepass_block<D>(A, blockIdx.x);
}

static inline unsigned prepass_blocks(const EdgeArgs &A) { return prepass_block_count(A); }

// ------------------------------------------------------------------ 3. interior
// Persistent: blocks loop until the tile cursor runs past n_tiles.  Every
// wave owns its tile cursor state; lanes own edges.  For an arm the KP
// collision spheres of a state are tested in NCH chunks of KP / NCH spheres:
// fewer live probe registers buy a higher occupancy for a few per-obstacle
// set-up instructions more.

// Lazy lists of at most this many (edge, state) pairs are checked by
// k_list_states, all states side by side; longer ones by the early-exit
// interior kernel in list mode (both are launched; each returns at once when
// the list is the other's).
__device__ __forceinline__ uint64_t list_states_limit() { return 1ull << 19; }

// LIST: the edges of a lazy round's list (A.edge_list, *A.n_list of them)
// when the list is too long for k_list_states to take all their states at
// once, in chunks instead of the pre-pass tiles: chunks sized to spread the
// list over every resident wave (at least kListChunk edges, at most 64), a
// lane walking its edge's states with early exit; a collision marks the edge
// for k_list_finish (no pre-pass wrote a provisional cost).  A separate
// instantiation, so the full check's kernel carries no extra live state.
constexpr int kListChunk = 4;

template <class Model, bool UNIFORM_R, int NCH, bool LIST = false>
__global__ void __launch_bounds__(256, Model::kGrid ? (Model::kArm ? 6 : 4) : NCH == 1 ? 3 : NCH == 2 ? 4 : 5)
    k_interior(EdgeArgs A, const ArmParams *Rg, SceneParams S) {
    constexpr int D = Model::D;
    constexpr int KP = Model::KP;
    constexpr bool ARM = Model::kArm;
    constexpr bool GRID = Model::kGrid;
    constexpr int W = ARM ? 3 : D;
    constexpr int SP = ARM ? 1 : KP;  // interior states per evaluation
    static_assert(!ARM || KP % NCH == 0, "chunking must divide the sphere slots");
    // outside lazy lists the last edges are finished with their states
    // spread over the lanes (below)
    constexpr bool TAIL = !LIST;
    __shared__ float tord[GTMP_MAX_H];
    __shared__ typename std::conditional<TAIL, uint32_t[256], char>::type tail_hit;  // per wave: 64 words
    constexpr int WG = Model::kWords > 0 ? Model::kWords : 1;
    constexpr int WS = point_mask_stride<WG>();
    // arms: the grid's own mask layout; points: the maps and obstacles here,
    // the mask words in pmask, one cell's words side by side
    __shared__ typename std::conditional<GRID, GridLds<ARM ? WG : 0>, char>::type glds_raw;
    __shared__ typename std::conditional<GRID && !ARM, PointMaskLds<WG>, char>::type pmask;
    __shared__ typename std::conditional<GRID, GridQueue<WG>[256 / kWave], char>::type gque;
    const ObsGrid &glds = *reinterpret_cast<const ObsGrid *>(&glds_raw);  // the first grid_lds_bytes()
    for (int i = threadIdx.x; i < A.n_int; i += blockDim.x) tord[i] = A.tord[i];
    if constexpr (GRID) {  // the maps, the obstacles and the mask words this kernel reads
        const uint4 *src = reinterpret_cast<const uint4 *>(A.grid);
        uint4 *dst = reinterpret_cast<uint4 *>(&glds_raw);
        constexpr int n16 = (int)(grid_lds_bytes<ARM ? WG : 0>() / 16);
        for (int i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
        if constexpr (!ARM) {
            for (int i = threadIdx.x; i < W * kGridCells; i += blockDim.x) {
                const int ax = i / kGridCells, bin = i - ax * kGridCells;
#pragma unroll
                for (int wd = 0; wd < WS; ++wd) pmask.m[ax][bin][wd] = wd < WG ? A.grid->mask[wd][ax][bin] : 0u;
            }
        }
    }
    __syncthreads();
    float ginv[3] = {0.f, 0.f, 0.f}, goff[3] = {0.f, 0.f, 0.f};
    if constexpr (GRID && Model::kArm) {
        // wave-uniform and used once per link: the scales in scalar
        // registers, the offsets in vector registers (an FMA reads one
        // scalar operand)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            ginv[i] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(glds.inv[i])));
            goff[i] = glds.off[i];
        }
    } else if constexpr (GRID) {
        // point probes take both in one FMA per axis, which can read only one
        // scalar operand: vector registers avoid a copy per probe
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            ginv[i] = glds.inv[i];
            goff[i] = glds.off[i];
        }
    }

    const int lane = lane_id();
    const uint32_t wv = wave_in_block();  // a scalar: the wave's LDS areas keep scalar base addresses
    uint32_t n_tiles = A.n_tiles;
    uint32_t chunk = kWave;
    if constexpr (LIST) {
        const uint32_t n_list = uniform(*A.n_list);
        if ((uint64_t)n_list * (uint32_t)A.n_int <= list_states_limit()) {  // k_list_states took it
            if (A.stats && lane_id() == 0) store_wave_stats(A, 0, 0, 0);
            return;
        }
        const uint32_t waves = gridDim.x * (blockDim.x / kWave);
        chunk = (n_list + waves - 1) / waves;
        chunk = chunk < (uint32_t)kListChunk ? (uint32_t)kListChunk : chunk > (uint32_t)kWave ? (uint32_t)kWave : chunk;
        n_tiles = (n_list + chunk - 1) / chunk;
    }

    // wave-uniform tile state
    uint32_t tile = 0, cnt = 0, pos = 0;
    uint32_t cursor = blockIdx.x % kCursors, cursors_left = kCursors;
    RowInfo ri{};
    bool exhausted = false;
    // wave totals (wave-uniform, scalar registers): states evaluated, edges
    // taken, exact sphere-obstacle tests behind the bin filter
    unsigned long long n_states = 0, n_edges = 0;
    uint32_t n_tests = 0;

    // lane state: the edge (flat id), its start and direction, next state
    bool has = false, fresh = false;
    float u[D], dv[D];
    uint32_t e = 0, uid = 0, vid = 0;
    int j = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) { u[i] = 0.f; dv[i] = 0.f; }
    const float r0 = ARM ? Rg->r0 : 0.f;
    // gap sign of one arm state q (<= 0: in contact); `live` false: the lane
    // takes part in the wave's queue but its result is meaningless
    auto arm_gap = [&](const float (&q)[D], bool live) -> float {
        if constexpr (ARM) {
            // The robot table is re-read through a pointer the compiler cannot
            // see through, so each value is a short-lived scalar load at its
            // use instead of a register held (and spilled) across the loop.
            carm Rp = (carm)Rg;
            asm volatile("" : "+s"(Rp));
            const auto &R = *Rp;
            if constexpr (GRID) {
                uint32_t tests = 0;
                const bool hit =
                    arm_hit_grid<WG, UNIFORM_R && !LIST>(R, q, glds.mask, glds.rec, ginv, goff, gque[wv], tests, live);
                n_tests += tests;
                return hit ? -1.f : 1.f;
            } else {
                (void)live;
                const v32f o = arm_fk<D>(R, q);
                return arm_state_gap<KP, NCH, UNIFORM_R>(R, o, r0, S);
            }
        } else {
            (void)q;
            (void)live;
            return 1.f;
        }
    };
    // gap sign of the SP point states j0, j0 + 1, ... (clipped to the last
    // state) of the edge from uu along dd: <= 0 when one of them is in contact
    auto point_gap = [&](const float (&uu)[D], const float (&dd)[D], int j0, bool live) -> float {
        if constexpr (!ARM && GRID) {
            float p[W][SP];
#pragma unroll
            for (int s = 0; s < SP; ++s) {
                int jj = j0 + s;
                jj = jj < A.n_int ? jj : A.n_int - 1;
                const float t = tord[live ? jj : 0];
#pragma unroll
                for (int i = 0; i < W; ++i) p[i][s] = __builtin_fmaf(t, dd[i], uu[i]);
            }
            uint32_t tests = 0;
            const bool hit =
                point_hit_grid<W, SP, Model::kWords>(p, pmask.m, glds.rec, ginv, goff, gque[wv], tests, live);
            n_tests += tests;
            return hit ? -1.f : 1.f;
        } else if constexpr (!ARM) {
            Probes<W, KP> P;
#pragma unroll
            for (int s = 0; s < SP; ++s) {
                int jj = j0 + s;
                jj = jj < A.n_int ? jj : A.n_int - 1;
                const float t = tord[live ? jj : 0];
#pragma unroll
                for (int i = 0; i < W; ++i) P.p[i][s] = __builtin_fmaf(t, dd[i], uu[i]);
            }
            float pr[KP];
#pragma unroll
            for (int k = 0; k < KP; ++k) pr[k] = 0.f;
            return probes_min_gap<W, KP, true>(P, pr, 0.f, S);
        } else {
            (void)uu;
            (void)dd;
            (void)j0;
            (void)live;
            return 1.f;
        }
    };

    while (true) {
        // ---- refill idle lanes from the current tile, taking new tiles as needed
        // (a list chunk fills the first `chunk` lanes of the wave)
        const bool taker = !LIST || (uint32_t)lane < chunk;
        uint64_t need = ballot(!has && taker);
        int n_need = __popcll(need);
        while (n_need > 0 && !exhausted) {
            const uint32_t avail = cnt - pos;
            if (avail == 0) {
                // the tiles (lists: chunks) fall into kCursors ranges, each with
                // its own cursor; a wave starts on its block's range and moves
                // on to the next ones as they run dry
                uint32_t t = 0;
                bool got = false;
                while (cursors_left > 0) {
                    if (lane == 0) t = atomicAdd(A.counter + kCursorStride * cursor, 1u);
                    t = uniform(t) + cursor_begin(n_tiles, cursor);
                    if (t < cursor_begin(n_tiles, cursor + 1)) {
                        got = true;
                        break;
                    }
                    cursor = cursor + 1 < (uint32_t)kCursors ? cursor + 1 : 0u;
                    --cursors_left;
                }
                if (!got) {
                    exhausted = true;
                    break;
                }
                tile = t;
                if constexpr (LIST) {
                    const uint32_t left = uniform(*A.n_list) - t * chunk;
                    cnt = left < chunk ? left : chunk;
                } else {
                    ri = decode_row(A, tile / A.tiles_per_row);
                    cnt = uniform(A.tile_cnt[tile]);
                }
                pos = 0;
                continue;
            }
            const uint32_t take = avail < (uint32_t)n_need ? avail : (uint32_t)n_need;
            const int r = rank_in(need);
            if (!has && (uint32_t)r < take) {
                if constexpr (LIST) {
                    e = A.edge_list[(size_t)tile * chunk + pos + r];
                    edge_vertex_ids(A, e, uid, vid);
                } else {
                    const uint32_t seg = tile - (tile / A.tiles_per_row) * A.tiles_per_row;
                    const uint32_t n = seg * kTile + A.tile_off[(size_t)tile * kTile + pos + r];
                    uid = ri.u_base + n * ri.u_step;
                    vid = ri.v_base + n * ri.v_step;
                    e = (uint32_t)(ri.e_base + (uint64_t)n * ri.e_step);
                }
                j = 0;
                has = true;
                fresh = true;
            }
            pos += take;
            if constexpr (!LIST) {
                n_edges += take;  // lists: counted by k_list_finish
                asm volatile("" : "+s"(n_edges));
            }
            need = ballot(!has && taker);
            n_need = __popcll(need);
        }
        // the vertices of the edges just taken, loaded once after the refill
        // loop (only integers are carried around it)
        if (fresh) {
            float v[D];
            load_vertex<D>(A, uid, u);
            load_vertex<D>(A, vid, v);
#pragma unroll
            for (int i = 0; i < D; ++i) dv[i] = v[i] - u[i];
            fresh = false;
        }
        const uint64_t busy = ballot(has);
        if (busy == 0) break;  // exhausted and every lane idle
        if constexpr (TAIL) {
            if (exhausted) break;  // no tile left: the edges in progress are finished below
        }
        n_states += (unsigned long long)__popcll(busy) * SP;
        asm volatile("" : "+s"(n_states));  // wave-uniform: a scalar register pair

        // ---- evaluate the next interior state(s) of every busy lane
        float gap;
        if constexpr (ARM) {
            float q[D];
            const float t = tord[has ? j : 0];
#pragma unroll
            for (int i = 0; i < D; ++i) q[i] = __builtin_fmaf(t, dv[i], u[i]);
            gap = arm_gap(q, has);
        } else {
            gap = point_gap(u, dv, j, has);
        }
        if (has) {
            if (gap <= 0.f) {
                if constexpr (LIST) A.list_mark[e] = 2;
                has = false;  // failed: provisional cost and flag stand (lists: marked for k_list_finish)
            } else {
                j += SP;
                if (j >= A.n_int && LIST) {
                    has = false;  // free: k_list_finish writes the length
                } else if (j >= A.n_int) {
                    // free edge: its cost is the length, computed as in the pre-pass
                    float acc = 0.f;
#pragma unroll
                    for (int i = 0; i < D; ++i)
                        acc = __builtin_fmaf(dv[i], dv[i], acc);  // zero past d
                    *cost_slot(A, e) = len_sqrt(acc);
                    if (A.flags) A.flags[e] = 0;
                    has = false;
                }
            }
        }
    }
    if constexpr (TAIL) {
        // No tile is left.  Instead of each lane walking the rest of its own
        // edge while the lanes whose edges are done idle, the remaining
        // evaluations of the wave's edges (SP consecutive states each) are
        // spread over its lanes, 64 per round: an edge's in its own state
        // order, the edges in lane order.  An edge found in contact takes no
        // further round; one whose states are all free is written as the main
        // loop writes it.  The states counted are those the main loop's early
        // exit would have evaluated (up to the first evaluation in contact),
        // so the count does not depend on how the evaluations were spread.
        uint32_t *th = tail_hit + wv * kWave;  // per owner: first evaluation in contact this round
        uint32_t rem = has ? (uint32_t)(A.n_int - j) : 0u;  // states left
        uint32_t counted = 0;                                // states counted for this lane's edge
        // A pair's edge comes from its owner lane: its start and direction
        // read across lanes, or (the bin-filtered arm kernel, whose registers
        // are tighter) its endpoints re-read from the vertex array by id.
        uint32_t ue = 0, ve = 0;
        if constexpr (ARM && GRID)
            if (rem > 0) edge_vertex_ids(A, e, ue, ve);
        for (;;) {
            const uint32_t nev = (rem + (uint32_t)SP - 1) / (uint32_t)SP;  // evaluations left
            uint32_t incl = nev;  // inclusive prefix sum over the lanes
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const uint32_t y = lane_read(lane - o, incl);
                if (lane >= o) incl += y;
            }
            const uint32_t total = uniform(__builtin_amdgcn_readlane(incl, kWave - 1));
            if (total == 0) break;
            const uint32_t pre = incl - nev;
            // evaluation `lane`: owner = the last lane whose prefix is <= lane
            // (lanes after the last owner have prefix `total`, beyond every
            // live evaluation)
            const bool live = (uint32_t)lane < total;
            int own = 0;
#pragma unroll
            for (int step = kWave / 2; step > 0; step >>= 1)
                if (lane_read(own + step, pre) <= (uint32_t)lane) own += step;
            const uint32_t kk = (uint32_t)lane - lane_read(own, pre);  // the owner's evaluation kk of this round
            const int j0 = (int)(lane_read(own, (uint32_t)j) + kk * (uint32_t)SP);
            th[lane] = 0xffffffffu;
            __builtin_amdgcn_wave_barrier();
            float gap;
            if constexpr (ARM) {
                const float t = tord[live ? j0 : 0];
                float q[D];
                if constexpr (GRID) {
                    float qu[D], qv[D];
                    load_vertex<D>(A, lane_read(own, ue), qu);
                    load_vertex<D>(A, lane_read(own, ve), qv);
#pragma unroll
                    for (int i = 0; i < D; ++i) q[i] = __builtin_fmaf(t, qv[i] - qu[i], qu[i]);  // as the refill forms it
                } else {
#pragma unroll
                    for (int i = 0; i < D; ++i)
                        q[i] = __builtin_fmaf(t, __uint_as_float(lane_read(own, __float_as_uint(dv[i]))),
                                              __uint_as_float(lane_read(own, __float_as_uint(u[i]))));
                }
                gap = arm_gap(q, live);
            } else {
                float tu[D], td[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    tu[i] = __uint_as_float(lane_read(own, __float_as_uint(u[i])));
                    td[i] = __uint_as_float(lane_read(own, __float_as_uint(dv[i])));
                }
                gap = point_gap(tu, td, j0, live);
            }
            if (live && gap <= 0.f) atomicMin(&th[own], kk);
            __builtin_amdgcn_wave_barrier();
            if (rem > 0) {
                const uint32_t took = pre >= (uint32_t)kWave ? 0u : min(nev, (uint32_t)kWave - pre);
                const uint32_t first = th[lane];
                if (first != 0xffffffffu) {
                    counted += (first + 1) * (uint32_t)SP;
                    rem = 0;  // failed: provisional cost and flag stand
                } else {
                    counted += took * (uint32_t)SP;
                    const uint32_t st = min(rem, took * (uint32_t)SP);
                    rem -= st;
                    j += (int)st;
                    if (rem == 0) {  // free edge: its cost is the length, as in the main loop
                        float dd[D], acc = 0.f;
                        if constexpr (ARM && GRID) {
                            float a[D], b[D];
                            load_vertex<D>(A, ue, a);
                            load_vertex<D>(A, ve, b);
#pragma unroll
                            for (int i = 0; i < D; ++i) dd[i] = b[i] - a[i];
                        } else {
#pragma unroll
                            for (int i = 0; i < D; ++i) dd[i] = dv[i];
                        }
#pragma unroll
                        for (int i = 0; i < D; ++i) acc = __builtin_fmaf(dd[i], dd[i], acc);  // zero past d
                        *cost_slot(A, e) = len_sqrt(acc);
                        if (A.flags) A.flags[e] = 0;
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) counted += lane_read(lane ^ o, counted);
        n_states += uniform(counted);
    }
    if (A.stats && lane == 0) store_wave_stats(A, n_states, n_edges, GRID ? n_tests : 0u);
}

// Edges with H == 2 have no interior state: the pre-pass result is final
// except that every candidate edge is free.
template <int D>
__global__ void __launch_bounds__(kTile) k_finalize_no_interior(EdgeArgs A) {
    const uint32_t tile = blockIdx.x;
    const uint32_t cnt = A.tile_cnt[tile];
    if (threadIdx.x >= cnt) return;
    const uint32_t row = tile / A.tiles_per_row;
    const uint32_t seg = tile - row * A.tiles_per_row;
    const RowInfo ri = decode_row(A, row);
    const uint32_t n = seg * kTile + A.tile_off[(size_t)tile * kTile + threadIdx.x];
    float u[D], v[D];
    load_vertex<D>(A, ri.u_base + n * ri.u_step, u);
    load_vertex<D>(A, ri.v_base + n * ri.v_step, v);
    ri.c_base[(size_t)n * ri.c_step] = edge_len<D>(u, v, A.d);
    if (A.flags) A.flags[ri.e_base + (uint64_t)n * ri.e_step] = 0;
}

// ------------------------------------------------------------------ lazy lists
// The listed edges of a lazy round (flat ids of edges with free endpoints
// within the length limit), every interior state of each at once: lane =
// (listed edge, state).  A round lists few edges, mostly free, and walking an
// edge's states one after another would chain their latencies; side by side
// (without early exit: the flag is the OR over the states either way) they
// overlap.  A colliding state marks its edge (list_mark[e] = 2), and
// k_list_finish then writes every listed edge's cost and flag as the full
// check does.
constexpr int kListBlocksPerCu = 4;

template <class Model, bool UNIFORM_R, int NCH>
__global__ void __launch_bounds__(256, 3) k_list_states(EdgeArgs A, const ArmParams *Rg, SceneParams S) {
    constexpr int D = Model::D;
    constexpr int KP = Model::KP;
    constexpr bool ARM = Model::kArm;
    constexpr bool GRID = Model::kGrid;
    constexpr int W = ARM ? 3 : D;
    constexpr int WG = Model::kWords > 0 ? Model::kWords : 1;
    __shared__ float tord[GTMP_MAX_H];
    __shared__ typename std::conditional<GRID, GridLds<WG>, char>::type glds_raw;
    __shared__ typename std::conditional<GRID, GridQueue<WG>[256 / kWave], char>::type gque;
    const ObsGrid &G = *reinterpret_cast<const ObsGrid *>(&glds_raw);
    for (int i = threadIdx.x; i < A.n_int; i += blockDim.x) tord[i] = A.tord[i];
    if constexpr (GRID) {
        const uint4 *src = reinterpret_cast<const uint4 *>(A.grid);
        uint4 *dst = reinterpret_cast<uint4 *>(&glds_raw);
        for (int i = threadIdx.x; i < (int)(grid_lds_bytes<WG>() / 16); i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    float ginv[3] = {0.f, 0.f, 0.f}, goff[3] = {0.f, 0.f, 0.f};
    if constexpr (GRID) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            ginv[i] = G.inv[i];
            goff[i] = G.off[i];
        }
    }
    const int lane = lane_id();
    const uint32_t n_int = (uint32_t)A.n_int;
    const uint64_t n_items = (uint64_t)uniform(*A.n_list) * n_int;
    if (n_items > list_states_limit()) return;  // long lists: the early-exit kernel takes them
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / kWave);
    unsigned long long n_states = 0;
    uint32_t n_tests = 0;
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * kWave; base < n_items;
         base += waves * kWave) {
        const uint64_t item = base + (uint64_t)lane;
        const bool live = item < n_items;
        const uint32_t k = live ? (uint32_t)(item / n_int) : 0u, jj = live ? (uint32_t)(item - (uint64_t)k * n_int) : 0u;
        const uint32_t e = A.edge_list[k];
        uint32_t uid, vid;
        edge_vertex_ids(A, e, uid, vid);
        float u[D], v[D], q[D];
        load_vertex<D>(A, uid, u);
        load_vertex<D>(A, vid, v);
        const float t = tord[jj];
#pragma unroll
        for (int i = 0; i < D; ++i) q[i] = __builtin_fmaf(t, v[i] - u[i], u[i]);
        bool hit;
        if constexpr (ARM) {
            carm Rp = (carm)Rg;
            asm volatile("" : "+s"(Rp));
            const auto &R = *Rp;
            if constexpr (GRID) {
                hit = arm_hit_grid<Model::kWords>(R, q, G.mask, G.rec, ginv, goff, gque[wave_in_block()], n_tests,
                                                   live);
            } else {
                const v32f o = arm_fk<D>(R, q);
                hit = arm_state_gap<KP, NCH, UNIFORM_R>(R, o, R.r0, S) <= 0.f;
            }
        } else {
            Probes<W, 1> P;
#pragma unroll
            for (int i = 0; i < W; ++i) P.p[i][0] = q[i];
            const float pr[1] = {0.f};
            hit = probes_min_gap<W, 1, true>(P, pr, 0.f, S) <= 0.f;
        }
        if (live && hit) A.list_mark[e] = 2;
        n_states += (unsigned long long)__popcll(ballot(live));
    }
    if (A.stats && lane == 0) {
        atomicAdd(&A.stats[0], n_states);
        if constexpr (GRID) atomicAdd(&A.stats[2], (unsigned long long)n_tests);  // wave total
    }
}

// Costs and flags of the listed edges: length if no state collided, else
// length + penalty (the same FP32 values as the full check's).
template <int D>
__global__ void __launch_bounds__(256) k_list_finish(EdgeArgs A) {
    const uint32_t n = *A.n_list;
    if (A.stats && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&A.stats[1], (unsigned long long)n);
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const uint32_t e = A.edge_list[k];
        uint32_t uid, vid;
        edge_vertex_ids(A, e, uid, vid);
        float u[D], v[D];
        load_vertex<D>(A, uid, u);
        load_vertex<D>(A, vid, v);
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < D; ++i)
            if (i < A.d) {
                const float dv = v[i] - u[i];
                acc = __builtin_fmaf(dv, dv, acc);
            }
        const float len = len_sqrt(acc);
        const bool hit = A.list_mark[e] == 2;
        *cost_slot(A, e) = hit ? failed_cost(len, A.penalty) : len;
        if (A.flags) A.flags[e] = hit ? 1 : 0;
    }
}

// Blocks of a lazy-list launch (the kernels stride over the list).
static unsigned list_blocks() {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    return (unsigned)(cus * kListBlocksPerCu);
}

// ------------------------------------------------------------------ full mode
// Exact signed distance of every state.  Lanes are (edge, state) pairs: HP
// lanes (a power of two >= min(H, 64)) per edge, 64 / HP edges per wave; for
// H > 64 each lane strides over the states.  The per-edge minimum is a
// butterfly over the HP-lane segment.
template <int W>
__device__ __forceinline__ float state_sd_point(const float (&x)[W], const SceneParams &S) {
    return point_sd<W>(x, S);
}

__device__ __forceinline__ float state_sd_arm(const ArmParams &R, const float (&q)[GTMP_MAX_JOINTS],
                                              const SceneParams &S) {
    const v32f o = arm_fk<GTMP_MAX_JOINTS>(R, q);
    float best = __builtin_inff();
    for (int k = 0; k < R.n_spheres; ++k) {
        const int b = 3 * R.link[k];
        const float t = R.t[k];
        float c[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float lo = o[b - 3 + i];
            const float hi = o[b + i];
            c[i] = __builtin_fmaf(t, hi - lo, lo);
        }
        best = __builtin_fminf(best, point_sd<3>(c, S) - R.r[k]);
    }
    return best;
}

template <bool ARMK, int D>
__global__ void __launch_bounds__(256) k_full(EdgeArgs A, ArmParams R, SceneParams S, float *minsd, int hp_log2) {
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    const int HP = 1 << hp_log2;
    const int epw = kWave / HP;
    const int seg = lane >> hp_log2;
    const int hl = lane & (HP - 1);
    const uint64_t E = (uint64_t)A.N + (uint64_t)(A.M - 1) * A.N * A.N + (uint64_t)A.N * A.G;
    const uint64_t inner_end = (uint64_t)A.N + (uint64_t)(A.M - 1) * A.N * A.N;
    const uint64_t gw = (uint64_t)blockIdx.x * (blockDim.x / kWave) + wv;
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x / kWave);
    for (uint64_t base = gw * epw; base < E; base += nw * epw) {
        const uint64_t e = base + seg;
        const bool valid = e < E;
        uint32_t uid = 0, vid = 0;
        float *cp = A.C_s;
        if (valid) {
            if (e < (uint64_t)A.N) {
                uid = 0; vid = 1 + (uint32_t)e; cp = A.C_s + e;
            } else if (e < inner_end) {
                const uint64_t r = e - A.N;
                const uint64_t ri = r / A.N, n = r - ri * A.N;  // ri = m N + u
                const uint64_t m = ri / A.N;
                uid = 1 + (uint32_t)ri; vid = 1 + (uint32_t)((m + 1) * A.N + n); cp = A.C_h + r;
            } else {
                const uint64_t r = e - inner_end;
                const uint64_t n = r / A.G, g = r - n * A.G;
                uid = 1 + (uint32_t)((A.M - 1) * A.N + n); vid = 1 + (uint32_t)A.M * A.N + (uint32_t)g;
                cp = A.C_l + r;
            }
        }
        float u[D], v[D];
        load_vertex<D>(A, uid, u);
        load_vertex<D>(A, vid, v);
        float best = __builtin_inff();
        for (int h0 = 0; h0 < A.H; h0 += HP) {
            const int h = h0 + hl;
            const bool act = h < A.H;
            const float t = (float)(act ? h : A.H - 1) / (float)(A.H - 1);
            float sd;
            if constexpr (ARMK) {
                float q[GTMP_MAX_JOINTS];
#pragma unroll
                for (int i = 0; i < D; ++i) q[i] = __builtin_fmaf(t, v[i] - u[i], u[i]);
                sd = state_sd_arm(R, q, S);
            } else {
                float x[D];
#pragma unroll
                for (int i = 0; i < D; ++i) x[i] = __builtin_fmaf(t, v[i] - u[i], u[i]);
                sd = state_sd_point<D>(x, S);
            }
            if (act) best = __builtin_fminf(best, sd);
        }
        for (int off = HP >> 1; off > 0; off >>= 1) best = __builtin_fminf(best, __shfl_xor(best, off));
        if (valid && hl == 0) {
            const float len = edge_len<D>(u, v, A.d);
            bool failed = best <= 0.f || len > A.max_len;
            if (A.prune) failed = failed || A.prune[e] != 0;
            *cp = failed ? failed_cost(len, A.penalty) : len;
            if (A.flags) A.flags[e] = failed ? 1 : 0;
            if (minsd) minsd[e] = best;
        }
    }
}

// ------------------------------------------------------------------ state check
template <bool ARMK, int D, int KP>
__global__ void __launch_bounds__(256) k_state_check(ArmParams R, SceneParams S, int d, int64_t n, const float *X,
                                                     float *sd, uint8_t *coll) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    float x[D];
#pragma unroll
    for (int j = 0; j < D; ++j) x[j] = (valid && j < d) ? X[i * d + j] : 0.f;
    if constexpr (ARMK) {
        if (coll) {
            const v32f o = arm_fk<D>(R, x);
            Probes<3, KP> P;
            arm_spheres<KP>(R, o, P);
            float pr[KP];
#pragma unroll
            for (int k = 0; k < KP; ++k) pr[k] = k < R.n_spheres ? R.r[k] : 0.f;
            const float gap = R.uniform_r ? probes_min_gap<3, KP, true>(P, pr, R.r0, S)
                                          : probes_min_gap<3, KP, false>(P, pr, R.r0, S);
            if (valid) coll[i] = gap <= 0.f ? 1 : 0;
        }
        if (sd) {
            const float s = state_sd_arm(R, x, S);
            if (valid) sd[i] = s;
        }
    } else {
        if (coll) {
            Probes<D, 1> P;
#pragma unroll
            for (int j = 0; j < D; ++j) P.p[j][0] = x[j];
            const float pr[1] = {0.f};
            const float gap = probes_min_gap<D, 1, true>(P, pr, 0.f, S);
            if (valid) coll[i] = gap <= 0.f ? 1 : 0;
        }
        if (sd && valid) sd[i] = point_sd<D>(x, S);
    }
}

// ------------------------------------------------------------------ launchers
static int round_kp(int k) { return ((k + 7) / 8) * 8; }

// gw: mask words of the obstacle-bin filter (1 or 2), 0 for the chunked test
// of every sphere against every obstacle.
template <int KP, int NCH>
static hipError_t launch_arm_kp(const EdgeArgs &A, const ArmParams &R, const SceneParams &S, const EdgeBuffers &b,
                                const gtmp_edge_opts &o, int grid_persist, hipStream_t s, const float *q0,
                                const float *goals, const float *Q, float *verts, uint8_t *vflag, int phases,
                                int gw) {
    const unsigned vb = (A.n_vertices + 255) / 256;
    ArmParams *Rg = reinterpret_cast<ArmParams *>(static_cast<char *>(b.workspace) + A.off_params);
    float r_max = 0.f;
    for (int k = 0; k < R.n_spheres; ++k) r_max = r_max > R.r[k] ? r_max : R.r[k];
    ObsGrid *grid = const_cast<ObsGrid *>(A.grid);
    if (phases & kPhaseVertices) {
        if (gw) {
            // the bins serve the vertex flags and, later, the interior kernel
            // (which also reads the robot table written beside them)
            hipLaunchKernelGGL(k_build_grid_params, dim3(2), dim3(kGridBuildThreads), 0, s, S, r_max, grid, R, Rg);
            // one wave per block: a plan has few vertices, so small blocks spread them over more CUs
            constexpr int vt = kVertexGridWaves * kWave;
            const unsigned vb64 = (A.n_vertices + vt - 1) / vt;
            if (gw == 1)
                hipLaunchKernelGGL(k_vertices_arm_grid<1>, dim3(vb64), dim3(vt), 0, s, A, R, q0, goals, Q, verts,
                                   vflag);
            else
                hipLaunchKernelGGL(k_vertices_arm_grid<2>, dim3(vb64), dim3(vt), 0, s, A, R, q0, goals, Q, verts,
                                   vflag);
        } else {
            hipLaunchKernelGGL(k_vertices_arm<KP>, dim3(vb), dim3(256), 0, s, A, R, S, q0, goals, Q, verts, vflag);
            hipLaunchKernelGGL(k_store_params_tol, dim3(1), dim3(kWave), 0, s, R, Rg, S);
        }
    }
    if (!(phases & kPhaseEdges)) return hipGetLastError();
    if (!A.edge_list) hipLaunchKernelGGL(k_prepass<GTMP_MAX_JOINTS>, dim3(prepass_blocks(A)), dim3(kTile), 0, s, A);
    if (gw && A.n_int > 0 && !(phases & kPhaseVertices))  // an edge pass on its own: bins built afresh
        hipLaunchKernelGGL(k_build_grid, dim3(1), dim3(kGridBuildThreads), 0, s, S, 3, r_max, grid);
    if (o.ev_begin) (void)hipEventRecord((hipEvent_t)o.ev_begin, s);
    if (A.edge_list) {  // lazy round: the listed edges, states side by side
        const unsigned lb = list_blocks();
        if (A.n_int > 0) {
            if (gw == 1) {
                hipLaunchKernelGGL((k_list_states<ArmGridModel<1>, true, 1>), dim3(lb), dim3(256), 0, s, A, Rg, S);
                hipLaunchKernelGGL((k_interior<ArmGridModel<1>, true, 1, true>), dim3(grid_persist), dim3(256), 0, s, A,
                                   Rg, S);
            } else if (gw == 2) {
                hipLaunchKernelGGL((k_list_states<ArmGridModel<2>, true, 1>), dim3(lb), dim3(256), 0, s, A, Rg, S);
                hipLaunchKernelGGL((k_interior<ArmGridModel<2>, true, 1, true>), dim3(grid_persist), dim3(256), 0, s, A,
                                   Rg, S);
            } else if (R.uniform_r) {
                hipLaunchKernelGGL((k_list_states<ArmModel<KP>, true, 2>), dim3(lb), dim3(256), 0, s, A, Rg, S);
                hipLaunchKernelGGL((k_interior<ArmModel<KP>, true, 2, true>), dim3(grid_persist), dim3(256), 0, s, A, Rg,
                                   S);
            } else {
                hipLaunchKernelGGL((k_list_states<ArmModel<KP>, false, 2>), dim3(lb), dim3(256), 0, s, A, Rg, S);
                hipLaunchKernelGGL((k_interior<ArmModel<KP>, false, 2, true>), dim3(grid_persist), dim3(256), 0, s, A,
                                   Rg, S);
            }
        }
        hipLaunchKernelGGL(k_list_finish<GTMP_MAX_JOINTS>, dim3(lb), dim3(256), 0, s, A);
    } else if (A.n_int == 0) {
        hipLaunchKernelGGL(k_finalize_no_interior<GTMP_MAX_JOINTS>, dim3(A.n_tiles), dim3(kTile), 0, s, A);
    } else if (gw) {
        // robots whose spheres share one radius read the exact test's starting
        // gap from the obstacle records
        if (gw == 1 && R.uniform_r)
            hipLaunchKernelGGL((k_interior<ArmGridModel<1>, true, 1>), dim3(grid_persist), dim3(256), 0, s, A, Rg, S);
        else if (gw == 1)
            hipLaunchKernelGGL((k_interior<ArmGridModel<1>, false, 1>), dim3(grid_persist), dim3(256), 0, s, A, Rg, S);
        else if (R.uniform_r)
            hipLaunchKernelGGL((k_interior<ArmGridModel<2>, true, 1>), dim3(grid_persist), dim3(256), 0, s, A, Rg, S);
        else
            hipLaunchKernelGGL((k_interior<ArmGridModel<2>, false, 1>), dim3(grid_persist), dim3(256), 0, s, A, Rg, S);
    } else if (R.uniform_r) {
        hipLaunchKernelGGL((k_interior<ArmModel<KP>, true, NCH>), dim3(grid_persist), dim3(256), 0, s, A, Rg, S);
    } else {
        hipLaunchKernelGGL((k_interior<ArmModel<KP>, false, NCH>), dim3(grid_persist), dim3(256), 0, s, A, Rg, S);
    }
    if (o.ev_end) (void)hipEventRecord((hipEvent_t)o.ev_end, s);
    if (A.n_int > 0) finish_wave_stats(A, (unsigned)grid_persist, s);
    (void)b;
    return hipGetLastError();
}

// States per lane and evaluation of the point kernels behind the obstacle bins.
constexpr int kPointGridSp = 4;
// Fewest tiles for which the point kernels take the bins (a small graph does
// not repay building them).
constexpr int kPointGridMinTiles = 1024;
// Resident blocks per CU of the point kernels behind the bins (automatic;
// 2d-large, M 16, N 1024: 0.35 ms at four blocks against 0.38 at two and 0.60
// at one).
constexpr int kPointGridBlocksPerCuAuto = 4;
// The arm kernels take at most two mask words.
constexpr int kGridArmMaxObs = 64;

template <int W, int SPI>
static hipError_t launch_point_s(const EdgeArgs &A, const ArmParams &R, const SceneParams &S, int grid_persist,
                                 const gtmp_edge_opts &o, hipStream_t s, int gw) {
    if (o.ev_begin) (void)hipEventRecord((hipEvent_t)o.ev_begin, s);
    if (A.edge_list) {  // lazy round: the listed edges, states side by side
        const unsigned lb = list_blocks();
        if (A.n_int > 0) {
            hipLaunchKernelGGL((k_list_states<PointModel<W, 1>, true, 1>), dim3(lb), dim3(256), 0, s, A,
                               (const ArmParams *)nullptr, S);
            hipLaunchKernelGGL((k_interior<PointModel<W, 8>, true, 1, true>), dim3(grid_persist), dim3(256), 0, s, A,
                               (const ArmParams *)nullptr, S);
        }
        hipLaunchKernelGGL(k_list_finish<W>, dim3(lb), dim3(256), 0, s, A);
    } else if (A.n_int == 0) {
        hipLaunchKernelGGL(k_finalize_no_interior<W>, dim3(A.n_tiles), dim3(kTile), 0, s, A);
    } else if (gw) {
        const auto kern = gw == 1 ? k_interior<PointGridModel<W, kPointGridSp, 1>, true, 1>
                        : gw == 2 ? k_interior<PointGridModel<W, kPointGridSp, 2>, true, 1>
                                  : k_interior<PointGridModel<W, kPointGridSp, 3>, true, 1>;
        hipLaunchKernelGGL(kern, dim3(grid_persist), dim3(256), 0, s, A, (const ArmParams *)nullptr, S);
    } else {
        hipLaunchKernelGGL((k_interior<PointModel<W, SPI>, true, 1>), dim3(grid_persist), dim3(256), 0, s, A,
                           (const ArmParams *)nullptr, S);
    }
    if (o.ev_end) (void)hipEventRecord((hipEvent_t)o.ev_end, s);
    if (A.n_int > 0) finish_wave_stats(A, (unsigned)grid_persist, s);
    return hipGetLastError();
}

template <int W>
static hipError_t launch_point(const EdgeArgs &A, const ArmParams &R, const SceneParams &S, int spi,
                               int grid_persist, const gtmp_edge_opts &o, hipStream_t s, const float *q0,
                               const float *goals, const float *Q, float *verts, uint8_t *vflag, int phases,
                               int gw) {
    const unsigned vb = (A.n_vertices + 255) / 256;
    if (phases & kPhaseVertices)
        hipLaunchKernelGGL(k_vertices_point<W>, dim3(vb), dim3(256), 0, s, A, S, q0, goals, Q, verts, vflag);
    if (!(phases & kPhaseEdges)) return hipGetLastError();
    if (!A.edge_list) hipLaunchKernelGGL(k_prepass<W>, dim3(prepass_blocks(A)), dim3(kTile), 0, s, A);
    if (gw)  // the bins of the full check (lazy rounds keep the full test)
        hipLaunchKernelGGL(k_build_grid, dim3(1), dim3(kGridBuildThreads), 0, s, S, W, 0.f,
                           const_cast<ObsGrid *>(A.grid));
    switch (spi) {
        case 1: return launch_point_s<W, 1>(A, R, S, grid_persist, o, s, gw);
        case 2: return launch_point_s<W, 2>(A, R, S, grid_persist, o, s, gw);
        case 4: return launch_point_s<W, 4>(A, R, S, grid_persist, o, s, gw);
        default: return launch_point_s<W, 8>(A, R, S, grid_persist, o, s, gw);
    }
}

// Resident blocks of a persistent launch: the request, else the occupancy
// limit capped at auto_cap (cheap states make the tile cursor a point of
// contention when every resident wave claims tiles from it).
static int persistent_grid(const void *kernel, int block, int blocks_per_cu_req, uint32_t n_tiles,
                           int auto_cap = 1 << 20) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    int per_cu = blocks_per_cu_req;
    if (per_cu <= 0) {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, block, 0) != hipSuccess || occ <= 0) occ = 2;
        per_cu = occ < auto_cap ? occ : auto_cap;
    }
    // a small graph gets one wave per tile at most: thousands of idle waves
    // would only queue on the tile cursor's atomic
    const uint64_t cap = ((uint64_t)n_tiles + (block / kWave) - 1) / (block / kWave);
    const uint64_t g = (uint64_t)cus * per_cu;
    return (int)(g < cap ? g : (cap > 0 ? cap : 1));
}

// automatic launch shape of the point-robot interior kernel with the full test
// (measured on the 2D workload with 50 circles and 20 boxes: 8 states per
// lane, 6 blocks per CU: 0.70 ms against 0.73 at 3)
constexpr int kPointSpiAuto = 8;
constexpr int kPointBlocksPerCuAuto = 6;

hipError_t launch_edge_check(const EdgePlan &plan, const ArmParams *arm, const SceneParams &scene, int wdim,
                             const EdgeBuffers &b, const gtmp_edge_opts &o, hipStream_t s) {
    return launch_edge_phases(plan, arm, scene, wdim, b, o, s, nullptr, nullptr, nullptr,
                              kPhaseVertices | kPhaseEdges);
}

hipError_t launch_edge_phases(const EdgePlan &plan, const ArmParams *arm, const SceneParams &scene, int wdim,
                              const EdgeBuffers &b, const gtmp_edge_opts &o, hipStream_t s,
                              const uint32_t *edge_list, const uint32_t *n_list, uint8_t *list_mark,
                              int phases) {
    EdgeArgs A{};
    A.d = plan.d; A.M = plan.M; A.N = plan.N; A.G = plan.G; A.H = plan.H; A.dp = vertex_stride(plan.d);
    A.penalty = plan.penalty; A.max_len = plan.max_len;
    A.tiles_per_row = plan.tiles_per_row; A.n_tiles = plan.n_tiles; A.n_vertices = plan.n_vertices;
    A.prepass_rows = prepass_rows_for(plan.n_tiles);
    char *ws = static_cast<char *>(b.workspace);
    float *verts = reinterpret_cast<float *>(ws + plan.off_verts);
    uint8_t *vflag = reinterpret_cast<uint8_t *>(ws + plan.off_vflag);
    A.verts = verts; A.vflag = vflag;
    A.C_s = b.C_s; A.C_h = b.C_h; A.C_l = b.C_l; A.flags = b.flags; A.prune = b.prune;
    A.tile_off = reinterpret_cast<uint8_t *>(ws + plan.off_tile_off);
    A.tile_cnt = reinterpret_cast<uint32_t *>(ws + plan.off_tile_cnt);
    A.counter = reinterpret_cast<uint32_t *>(ws + plan.off_counter);
    A.wstats = reinterpret_cast<unsigned long long *>(ws + plan.off_wstats);
    A.edge_list = edge_list;
    A.n_list = n_list;
    A.list_mark = list_mark;
    A.stats = o.stats;
    A.off_params = plan.off_params;
    uint8_t order[GTMP_MAX_H];
    A.n_int = interior_order(plan.H, order);
    for (int i = 0; i < A.n_int; ++i) A.tord[i] = (float)order[i] / (float)(plan.H - 1);

    ArmParams R{};
    if (arm) R = *arm;

    const bool full = o.mode == GTMP_CHECK_FULL || b.minsd != nullptr;
    if (full) {
        // pack vertices (flags are not needed but the kernel is cheap)
        const unsigned vb = (A.n_vertices + 255) / 256;
        int hp = 1, hpl = 0;
        const int hcap = plan.H < kWave ? plan.H : kWave;
        while (hp < hcap) { hp <<= 1; ++hpl; }
        const uint64_t E = (uint64_t)plan.N + (uint64_t)(plan.M - 1) * plan.N * plan.N + (uint64_t)plan.N * plan.G;
        const uint64_t waves = (E + (kWave / hp) - 1) / (kWave / hp);
        uint64_t blocks = (waves + 3) / 4;
        if (blocks > 65536) blocks = 65536;
        if (arm) {
            const int kp = round_kp(R.n_spheres);
            switch (kp) {
#define GTMP_VA(K) case K: hipLaunchKernelGGL(k_vertices_arm<K>, dim3(vb), dim3(256), 0, s, A, R, scene, b.q0, b.goals, b.Q, verts, vflag); break;
                GTMP_VA(8) GTMP_VA(16) GTMP_VA(24) GTMP_VA(32) GTMP_VA(40) GTMP_VA(48) GTMP_VA(56) GTMP_VA(64)
#undef GTMP_VA
                default: return hipErrorInvalidValue;
            }
            if (o.ev_begin) (void)hipEventRecord((hipEvent_t)o.ev_begin, s);
            hipLaunchKernelGGL((k_full<true, GTMP_MAX_JOINTS>), dim3((unsigned)blocks), dim3(256), 0, s, A, R, scene,
                               b.minsd, hpl);
            if (o.ev_end) (void)hipEventRecord((hipEvent_t)o.ev_end, s);
        } else if (wdim == 2) {
            hipLaunchKernelGGL(k_vertices_point<2>, dim3(vb), dim3(256), 0, s, A, scene, b.q0, b.goals, b.Q, verts, vflag);
            if (o.ev_begin) (void)hipEventRecord((hipEvent_t)o.ev_begin, s);
            hipLaunchKernelGGL((k_full<false, 2>), dim3((unsigned)blocks), dim3(256), 0, s, A, R, scene, b.minsd, hpl);
            if (o.ev_end) (void)hipEventRecord((hipEvent_t)o.ev_end, s);
        } else {
            hipLaunchKernelGGL(k_vertices_point<3>, dim3(vb), dim3(256), 0, s, A, scene, b.q0, b.goals, b.Q, verts, vflag);
            if (o.ev_begin) (void)hipEventRecord((hipEvent_t)o.ev_begin, s);
            hipLaunchKernelGGL((k_full<false, 3>), dim3((unsigned)blocks), dim3(256), 0, s, A, R, scene, b.minsd, hpl);
            if (o.ev_end) (void)hipEventRecord((hipEvent_t)o.ev_end, s);
        }
        return hipGetLastError();
    }

    // fast mode: the tile cursors are reset by the pre-pass; a lazy round's
    // list has no pre-pass and resets them with a fill kernel (no memset
    // node, so the sequence can be captured into a graph and replayed)
    if ((phases & kPhaseEdges) && A.edge_list)
        hipLaunchKernelGGL(k_zero_u32, dim3(kCursors * kCursorStride / 256), dim3(256), 0, s, A.counter,
                           kCursors * kCursorStride);
    if (arm) {
        const int kp = round_kp(R.n_spheres);
        const int n_obs = scene.n_sph + scene.n_box;
        // automatic choice: the obstacle-bin filter whenever the masks hold
        // every obstacle, else (and on request) the chunked full test
        const int gw = o.sphere_chunks == 0 && n_obs <= kGridArmMaxObs ? grid_words(n_obs) : 0;
        const int nch = o.sphere_chunks == 1 ? 1 : o.sphere_chunks == 4 ? 4 : 2;
        A.grid = reinterpret_cast<const ObsGrid *>(ws + plan.off_grid);
        const void *kern = nullptr;
        switch (gw ? -gw : kp * 8 + nch) {
            case -1: kern = R.uniform_r ? (const void *)k_interior<ArmGridModel<1>, true, 1> : (const void *)k_interior<ArmGridModel<1>, false, 1>; break;
            case -2: kern = R.uniform_r ? (const void *)k_interior<ArmGridModel<2>, true, 1> : (const void *)k_interior<ArmGridModel<2>, false, 1>; break;
#define GTMP_KK(K, C) case K * 8 + C: kern = R.uniform_r ? (const void *)k_interior<ArmModel<K>, true, C> : (const void *)k_interior<ArmModel<K>, false, C>; break;
#define GTMP_KK3(K) GTMP_KK(K, 1) GTMP_KK(K, 2) GTMP_KK(K, 4)
            GTMP_KK3(8) GTMP_KK3(16) GTMP_KK3(24) GTMP_KK3(32) GTMP_KK3(40) GTMP_KK3(48) GTMP_KK3(56) GTMP_KK3(64)
#undef GTMP_KK3
#undef GTMP_KK
            default: return hipErrorInvalidValue;
        }
        const int grid = persistent_grid(kern, 256, o.blocks_per_cu, plan.n_tiles);
        A.wstats = wave_stat_slots(A, (unsigned)grid);
        switch (kp * 8 + nch) {
#define GTMP_LA(K, C) case K * 8 + C: return launch_arm_kp<K, C>(A, R, scene, b, o, grid, s, b.q0, b.goals, b.Q, verts, vflag, phases, gw);
#define GTMP_LA3(K) GTMP_LA(K, 1) GTMP_LA(K, 2) GTMP_LA(K, 4)
            GTMP_LA3(8) GTMP_LA3(16) GTMP_LA3(24) GTMP_LA3(32) GTMP_LA3(40) GTMP_LA3(48) GTMP_LA3(56) GTMP_LA3(64)
#undef GTMP_LA3
#undef GTMP_LA
            default: return hipErrorInvalidValue;
        }
    }
    int spi = o.states_per_iter;
    if (spi <= 0) spi = kPointSpiAuto;
    if (spi != 1 && spi != 2 && spi != 4) spi = 8;
    // automatic choice: the obstacle bins for a full check of a graph with
    // many tiles whose scene the masks hold, else (and on request) the full test
    const int n_obs = scene.n_sph + scene.n_box;
    const int gw = o.sphere_chunks == 0 && !A.edge_list && n_obs > 0 && plan.n_tiles >= kPointGridMinTiles
                       ? grid_words(n_obs) : 0;
    A.grid = reinterpret_cast<const ObsGrid *>(ws + plan.off_grid);
    if (wdim == 2) {
        const void *kern = gw == 1 ? (const void *)k_interior<PointGridModel<2, kPointGridSp, 1>, true, 1>
                         : gw == 2 ? (const void *)k_interior<PointGridModel<2, kPointGridSp, 2>, true, 1>
                         : gw == 3 ? (const void *)k_interior<PointGridModel<2, kPointGridSp, 3>, true, 1>
                         : spi == 1 ? (const void *)k_interior<PointModel<2, 1>, true, 1>
                         : spi == 2 ? (const void *)k_interior<PointModel<2, 2>, true, 1>
                         : spi == 4 ? (const void *)k_interior<PointModel<2, 4>, true, 1>
                                    : (const void *)k_interior<PointModel<2, 8>, true, 1>;
        const int grid = persistent_grid(kern, 256, o.blocks_per_cu, plan.n_tiles, gw ? kPointGridBlocksPerCuAuto : kPointBlocksPerCuAuto);
        A.wstats = wave_stat_slots(A, (unsigned)grid);
        return launch_point<2>(A, R, scene, spi, grid, o, s, b.q0, b.goals, b.Q, verts, vflag, phases, gw);
    }
    const void *kern = gw == 1 ? (const void *)k_interior<PointGridModel<3, kPointGridSp, 1>, true, 1>
                     : gw == 2 ? (const void *)k_interior<PointGridModel<3, kPointGridSp, 2>, true, 1>
                     : gw == 3 ? (const void *)k_interior<PointGridModel<3, kPointGridSp, 3>, true, 1>
                     : spi == 1 ? (const void *)k_interior<PointModel<3, 1>, true, 1>
                     : spi == 2 ? (const void *)k_interior<PointModel<3, 2>, true, 1>
                     : spi == 4 ? (const void *)k_interior<PointModel<3, 4>, true, 1>
                                : (const void *)k_interior<PointModel<3, 8>, true, 1>;
    const int grid = persistent_grid(kern, 256, o.blocks_per_cu, plan.n_tiles, gw ? kPointGridBlocksPerCuAuto : kPointBlocksPerCuAuto);
    A.wstats = wave_stat_slots(A, (unsigned)grid);
    return launch_point<3>(A, R, scene, spi, grid, o, s, b.q0, b.goals, b.Q, verts, vflag, phases, gw);
}

hipError_t launch_state_check(const ArmParams *arm, const SceneParams &scene, int wdim, int d, int64_t n,
                              const float *X, float *sd, uint8_t *coll, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    ArmParams R{};
    if (arm) {
        R = *arm;
        switch (round_kp(R.n_spheres)) {
#define GTMP_SC(K) case K: hipLaunchKernelGGL((k_state_check<true, GTMP_MAX_JOINTS, K>), dim3(blocks), dim3(256), 0, s, R, scene, d, n, X, sd, coll); break;
            GTMP_SC(8) GTMP_SC(16) GTMP_SC(24) GTMP_SC(32) GTMP_SC(40) GTMP_SC(48) GTMP_SC(56) GTMP_SC(64)
#undef GTMP_SC
            default: return hipErrorInvalidValue;
        }
    } else if (wdim == 2) {
        hipLaunchKernelGGL((k_state_check<false, 2, 1>), dim3(blocks), dim3(256), 0, s, R, scene, d, n, X, sd, coll);
    } else {
        hipLaunchKernelGGL((k_state_check<false, 3, 1>), dim3(blocks), dim3(256), 0, s, R, scene, d, n, X, sd, coll);
    }
    return hipGetLastError();
}

}  // namespace gtmp
