// batch.hip -- many independent plans (uneven N, M, d, robots and anytime
// policies) through batched kernels: one launch per step for every plan of
// the batch, and one persistent edge-interior launch per robot group over the
// tiles of all its plans.  A plan's stages follow the single-plan policies
// (Alg. 1 gtmp / anytime-gtmp / ao-gtmp), and every result equals the
// single-plan call with the same seed: the kernels run the same per-edge,
// per-row and per-plan code as the single-plan ones.
#include <map>
#include <mutex>
#include <string>

#include "edge_common.hpp"

namespace gtmp {

// Tile cursors of the batched interior kernels: a group's tiles fall into
// kBatchCursors contiguous ranges, one per XCD (blocks are dealt to the XCDs
// in turn), each counted by its own cursor 256 bytes from the next, so that
// the waves' atomics spread over several addresses.
constexpr int kBatchCursors = 8;
constexpr int kBatchCursorStride = 64;                                      // 32-bit words
constexpr int kBatchGroupCounters = kBatchCursors * kBatchCursorStride;    // one robot group
constexpr int kBatchStageCounters = 3 * kBatchGroupCounters;               // the three groups of a stage
static_assert(kBatchStageCounters % 256 == 0, "cleared by whole 256-thread blocks");
__device__ __forceinline__ uint32_t batch_cursor_begin(uint32_t n, uint32_t c) {
    return (uint32_t)((uint64_t)n * c / kBatchCursors);
}

// Per-plan, per-stage descriptor (device table, read-only during a stage).
struct BPlan {
    EdgeArgs A;          // edge check of this plan's stage (workspace, costs, tiles, t order)
    SceneParams S;
    const ArmParams *arm;  // device copy of the robot table (arms), null for points
    float grid_r_max;      // arms: largest robot sphere radius (the obstacle bins are built for it); points: 0
    int group;           // 0: 2D point, 1: 3D point, 2: arm
    uint32_t vert_base;  // first vertex of this plan in its group's vertex space
    uint32_t tile_base;  // first tile of this plan in the batch's tile space
    uint32_t gtile_base; // first tile of this plan in its group's tile space
    uint32_t pblock_base; // first pre-pass block of this plan in its group's block space
    uint32_t row_base;   // first row (layer vertex) in the batch's row space
    const float *Q, *q0, *goals;
    float *V;
    int32_t *Aidx;
    float *Vs;
    int32_t *as;
    int32_t *idx;
    float *wp;
    float *cost;
    // archive of the plan's anytime policy
    float *best_cost;
    int32_t *best_idx;
    float *best_wp;
    int32_t *best_meta;
    float *stage_costs;
    uint32_t *counter;
    int max_stages;
    // uniform sampling of this stage (restart policy); 0 = samples come from elsewhere
    int sample;
    uint32_t k0, k1, stage;
    float lo[GTMP_MAX_DOF], wd[GTMP_MAX_DOF];
};

typedef const __attribute__((address_space(4))) BPlan *cplan;

// Largest p with base(p) <= x over plans [lo, hi) (bases non-decreasing).
template <class F>
__device__ __forceinline__ int find_plan(int lo, int hi, uint64_t x, F base) {
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((uint64_t)base(mid) <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------ sampling
__global__ void __launch_bounds__(256) k_batch_sample(const BPlan *plans, int n_plans, const uint64_t *sample_base,
                                                      uint64_t total) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int p = find_plan(0, n_plans, g, [&](int i) { return sample_base[i]; });
    const BPlan &P = plans[p];
    if (!P.sample) return;
    const int d = P.A.d;
    const int nblk = (d + 3) >> 2;
    const uint64_t t = g - sample_base[p];
    const uint32_t blk = (uint32_t)(t % nblk);
    const uint64_t mn = t / nblk;
    const uint32_t n = (uint32_t)(mn % P.A.N), m = (uint32_t)(mn / P.A.N);
    const uint4 w = philox4x32_10(make_uint4(n, m, P.stage, blk), P.k0, P.k1);
    const uint32_t words[4] = {w.x, w.y, w.z, w.w};
    float *dst = const_cast<float *>(P.Q) + mn * d;
    for (int i = 0; i < 4; ++i) {
        const int j = (int)blk * 4 + i;
        if (j < d) dst[j] = __builtin_fmaf(unit_from_word(words[i]), P.wd[j], P.lo[j]);
    }
}

// ------------------------------------------------------------------ vertices
template <int GROUP, int KP>
__global__ void __launch_bounds__(256) k_batch_vertices(const BPlan *plans, int p0, int p1, uint32_t total) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = g < total;
    const int p = find_plan(p0, p1, live ? g : 0, [&](int i) { return plans[i].vert_base; });
    const BPlan &P = plans[p];
    const EdgeArgs &A = P.A;
    const uint32_t i = (live ? g : 0) - P.vert_base;
    const bool valid = live && i < A.n_vertices;
    const uint32_t MN = (uint32_t)A.M * (uint32_t)A.N;
    float *verts = const_cast<float *>(A.verts);
    uint8_t *vflag = const_cast<uint8_t *>(A.vflag);
    if constexpr (GROUP == 2) {
        float q[GTMP_MAX_JOINTS];
#pragma unroll
        for (int j = 0; j < GTMP_MAX_JOINTS; ++j) q[j] = 0.f;
        if (valid) {
            const float *src = i == 0 ? P.q0 : (i <= MN ? P.Q + (size_t)(i - 1) * A.d : P.goals + (size_t)(i - 1 - MN) * A.d);
#pragma unroll
            for (int j = 0; j < GTMP_MAX_JOINTS; ++j)
                if (j < A.d) q[j] = src[j];
#pragma unroll
            for (int j = 0; j < GTMP_MAX_JOINTS; ++j) verts[(size_t)i * A.dp + j] = q[j];
        }
        // plans of one block may differ: the robot and the scene are per lane here
        const ArmParams &R = *P.arm;
        if (valid) {
            const v32f o = arm_fk<GTMP_MAX_JOINTS>(R, q);
            float best = __builtin_inff();
            for (int k = 0; k < R.n_spheres; ++k) {
                const int b = 3 * R.link[k];
                float c[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) c[a] = __builtin_fmaf(R.t[k], o[b + a] - o[b - 3 + a], o[b - 3 + a]);
                const float r = R.r[k];
                for (int oo = 0; oo < P.S.n_sph; ++oo) {
                    const float *sp = P.S.sph + oo * 4;
                    float g2 = -(sp[3] + r) * (sp[3] + r);
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const float dl = c[a] - sp[a];
                        g2 = __builtin_fmaf(dl, dl, g2);
                    }
                    best = __builtin_fminf(best, g2);
                }
                for (int oo = 0; oo < P.S.n_box; ++oo) {
                    const float *bx = P.S.box + oo * 6;
                    float g2 = -r * r;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const float dl = c[a] - __builtin_amdgcn_fmed3f(c[a], bx[a] - bx[3 + a], bx[a] + bx[3 + a]);
                        g2 = __builtin_fmaf(dl, dl, g2);
                    }
                    best = __builtin_fminf(best, g2);
                }
            }
            vflag[i] = best <= 0.f ? 1 : 0;
        }
    } else {
        constexpr int W = GROUP == 0 ? 2 : 3;
        if (!valid) return;
        const float *src = i == 0 ? P.q0 : (i <= MN ? P.Q + (size_t)(i - 1) * W : P.goals + (size_t)(i - 1 - MN) * W);
        Probes<W, 1> Pr;
        for (int j = 0; j < GTMP_MAX_DOF; ++j) verts[(size_t)i * A.dp + j] = j < W ? src[j] : 0.f;
#pragma unroll
        for (int j = 0; j < W; ++j) Pr.p[j][0] = src[j];
        float best = __builtin_inff();
        for (int oo = 0; oo < P.S.n_sph; ++oo) {
            const float *sp = P.S.sph + oo * (W + 1);
            float g2 = -sp[W] * sp[W];
#pragma unroll
            for (int a = 0; a < W; ++a) {
                const float dl = Pr.p[a][0] - sp[a];
                g2 = __builtin_fmaf(dl, dl, g2);
            }
            best = __builtin_fminf(best, g2);
        }
        for (int oo = 0; oo < P.S.n_box; ++oo) {
            const float *bx = P.S.box + oo * 2 * W;
            float g2 = 0.f;
#pragma unroll
            for (int a = 0; a < W; ++a) {
                const float x = Pr.p[a][0];
                const float dl = x - __builtin_amdgcn_fmed3f(x, bx[a] - bx[W + a], bx[a] + bx[W + a]);
                g2 = __builtin_fmaf(dl, dl, g2);
            }
            best = __builtin_fminf(best, g2);
        }
        vflag[i] = best <= 0.f ? 1 : 0;
        (void)KP;
    }
}

// ------------------------------------------------------------------ pre-pass
// Pre-pass of the plans [p0, p1) of one robot group: the single-plan
// pre-pass (rows per block, target vertices reused along a run of rows),
// block b of the launch being block b - pblock_base of its plan.
template <int D>
__global__ void __launch_bounds__(kTile) k_batch_prepass(const BPlan *plans, int p0, int p1) {
    const uint32_t g = blockIdx.x;
    const int p = find_plan(p0, p1, g, [&](int i) { return plans[i].pblock_base; });
    prepass_block<D>(plans[p].A, g - plans[p].pblock_base);
}

// ------------------------------------------------------------------ interior (persistent)
// Lanes of a wave always hold edges of one plan: obstacles and the robot
// table are read with wave-uniform addresses.  A wave that draws a tile of
// another plan finishes its edges before it switches.
template <class Model, bool UNIFORM_R, int NCH>
__global__ void __launch_bounds__(256, Model::kGrid ? (Model::kWords > 1 ? 3 : (Model::kArm ? 5 : 4)) : NCH == 1 ? 3 : NCH == 2 ? 4 : 5)
    k_batch_interior(const BPlan *plans, int p0, int p1, uint32_t n_gtiles, uint32_t *gcounter,
                     unsigned long long *stats) {
    constexpr int D = Model::D;
    constexpr int KP = Model::KP;
    constexpr bool ARM = Model::kArm;
    constexpr bool GRID = Model::kGrid;
    constexpr int W = ARM ? 3 : D;
    constexpr int SP = ARM ? 1 : KP;
    __shared__ float tord[4][GTMP_MAX_H];
    // obstacle bins: each wave holds the mask words of its current plan in
    // LDS (arms: the grid's layout; points: the W axes a point state uses,
    // one cell's words side by side, one vector read per axis); the obstacle
    // records (read by the exact tests only) stay in device memory
    constexpr int WG = Model::kWords > 0 ? Model::kWords : 1;
    constexpr int WS = point_mask_stride<WG>();
    __shared__ typename std::conditional<GRID && ARM, GridMaskTable[4][WG], char>::type gmask;
    __shared__ typename std::conditional<GRID && !ARM, uint32_t[4][W][kGridCells][WS], char>::type pmask;
    __shared__ typename std::conditional<GRID, GridQueue<WG>[4], char>::type gque;
    const float4(*grec)[2] = nullptr;
    float ginv[3] = {0.f, 0.f, 0.f}, goff[3] = {0.f, 0.f, 0.f};
    uint32_t n_tests = 0;
    const int lane = lane_id();
    const int wv = (int)wave_in_block();

    int cur = -1;               // plan of the lanes' edges (wave uniform)
    uint32_t tile = 0, cnt = 0, pos = 0, pending = 0xffffffffu;
    uint32_t cursor = blockIdx.x % kBatchCursors, cursors_left = kBatchCursors;
    int pend_plan = -1;
    RowInfo ri{};
    bool exhausted = false;
    unsigned long long n_states = 0, n_edges = 0;
    bool has = false, fresh = false;
    float u[D], dv[D];
    uint32_t e = 0, uid = 0, vid = 0;
    int j = 0;
    int n_int = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) { u[i] = 0.f; dv[i] = 0.f; }

    while (true) {
        uint64_t need = ballot(!has);
        int n_need = __popcll(need);
        while (n_need > 0 && !exhausted) {
            const uint32_t avail = cnt - pos;
            if (avail == 0 && pending == 0xffffffffu) {
                // the group's tiles fall into kBatchCursors ranges, each with
                // its own cursor; a wave starts on its block's range and moves
                // on to the next ones as they run dry
                uint32_t t = 0;
                bool got = false;
                while (cursors_left > 0) {
                    if (lane == 0) t = atomicAdd(gcounter + kBatchCursorStride * cursor, 1u);
                    t = uniform(t) + batch_cursor_begin(n_gtiles, cursor);
                    if (t < batch_cursor_begin(n_gtiles, cursor + 1)) {
                        got = true;
                        break;
                    }
                    cursor = cursor + 1 < (uint32_t)kBatchCursors ? cursor + 1 : 0u;
                    --cursors_left;
                }
                if (!got) {
                    exhausted = true;
                    break;
                }
                pending = t;
                pend_plan = find_plan(p0, p1, t, [&](int i) { return plans[i].gtile_base; });
            }
            if (avail == 0 && pending != 0xffffffffu) {
                if (pend_plan != cur) {
                    if (ballot(has) != 0) break;  // finish the current plan's edges first
                    cur = pend_plan;
                    n_int = plans[cur].A.n_int;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    for (int i = lane; i < n_int; i += kWave) tord[wv][i] = plans[cur].A.tord[i];
                    if constexpr (GRID && ARM) {
                        const uint4 *src = reinterpret_cast<const uint4 *>(plans[cur].A.grid->mask);
                        uint4 *dst = reinterpret_cast<uint4 *>(&gmask[wv][0]);
                        constexpr int n16 = (int)(sizeof(GridMaskTable) * WG / 16);
                        for (int i = lane; i < n16; i += kWave) dst[i] = src[i];
                    } else if constexpr (GRID) {
                        const ObsGrid *G = plans[cur].A.grid;
                        for (int i = lane; i < W * kGridCells; i += kWave) {
                            const int ax = i / kGridCells, bin = i - ax * kGridCells;
#pragma unroll
                            for (int wd = 0; wd < WS; ++wd) pmask[wv][ax][bin][wd] = wd < WG ? G->mask[wd][ax][bin] : 0u;
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    if constexpr (GRID) {
                        const ObsGrid *G = plans[cur].A.grid;
                        grec = G->rec;
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            ginv[i] = G->inv[i];
                            goff[i] = G->off[i];
                        }
                    }
                }
                const EdgeArgs &A = plans[cur].A;
                tile = pending - plans[cur].gtile_base;
                pending = 0xffffffffu;
                ri = decode_row(A, tile / A.tiles_per_row);
                cnt = uniform(A.tile_cnt[tile]);
                pos = 0;
                continue;
            }
            const EdgeArgs &A = plans[cur].A;
            const uint32_t take = avail < (uint32_t)n_need ? avail : (uint32_t)n_need;
            const int r = rank_in(need);
            if (!has && (uint32_t)r < take) {
                const uint32_t seg = tile - (tile / A.tiles_per_row) * A.tiles_per_row;
                const uint32_t n = seg * kTile + A.tile_off[(size_t)tile * kTile + pos + r];
                uid = ri.u_base + n * ri.u_step;
                vid = ri.v_base + n * ri.v_step;
                e = (uint32_t)(ri.e_base + (uint64_t)n * ri.e_step);
                j = 0;
                has = true;
                fresh = true;
            }
            pos += take;
            n_edges += take;
            need = ballot(!has);
            n_need = __popcll(need);
        }
        // the vertices of the edges just taken (all of the current plan: the
        // plan changes only when no lane is busy), loaded once after the
        // refill loop, which carries only integers
        if (fresh) {
            const EdgeArgs &A = plans[cur].A;
            float v[D];
            load_vertex<D>(A, uid, u);
            load_vertex<D>(A, vid, v);
#pragma unroll
            for (int i = 0; i < D; ++i) dv[i] = v[i] - u[i];
            fresh = false;
        }
        const uint64_t busy = ballot(has);
        if (busy == 0) {
            if (exhausted) break;
            continue;  // drained: switch plans at the top of the loop
        }
        n_states += (unsigned long long)__popcll(busy) * SP;

        cplan Pp = (cplan)(plans + cur);
        asm volatile("" : "+s"(Pp));
        const SceneParams S{Pp->S.sph, Pp->S.box, Pp->S.n_sph, Pp->S.n_box};
        float gap;
        if constexpr (ARM) {
            float q[D];
            const float t = tord[wv][has ? j : 0];
#pragma unroll
            for (int i = 0; i < D; ++i) q[i] = __builtin_fmaf(t, dv[i], u[i]);
            carm Rp = (carm)Pp->arm;
            asm volatile("" : "+s"(Rp));
            const auto &R = *Rp;
            if constexpr (GRID) {
                uint32_t tests = 0;
                gap = arm_hit_grid<Model::kWords, UNIFORM_R>(R, q, gmask[wv], grec, ginv, goff, gque[wv], tests, has) ? -1.f : 1.f;
                n_tests += tests;
            } else {
                const float r0 = R.r0;
                const v32f o = arm_fk<D>(R, q);
                gap = arm_state_gap<KP, NCH, UNIFORM_R>(R, o, r0, S);
            }
        } else if constexpr (GRID) {
            float p[W][SP];
#pragma unroll
            for (int s = 0; s < SP; ++s) {
                int jj = j + s;
                jj = jj < n_int ? jj : n_int - 1;
                const float t = tord[wv][has ? jj : 0];
#pragma unroll
                for (int i = 0; i < W; ++i) p[i][s] = __builtin_fmaf(t, dv[i], u[i]);
            }
            uint32_t tests = 0;
            gap = point_hit_grid<W, SP, Model::kWords>(p, pmask[wv], grec, ginv, goff, gque[wv], tests, has) ? -1.f
                                                                                                              : 1.f;
            n_tests += tests;
        } else {
            Probes<W, KP> P;
#pragma unroll
            for (int s = 0; s < SP; ++s) {
                int jj = j + s;
                jj = jj < n_int ? jj : n_int - 1;
                const float t = tord[wv][has ? jj : 0];
#pragma unroll
                for (int i = 0; i < W; ++i) P.p[i][s] = __builtin_fmaf(t, dv[i], u[i]);
            }
            float pr[KP];
#pragma unroll
            for (int k = 0; k < KP; ++k) pr[k] = 0.f;
            gap = probes_min_gap<W, KP, true>(P, pr, 0.f, S);
        }
        if (has) {
            if (gap <= 0.f) {
                has = false;
            } else {
                j += SP;
                if (j >= n_int) {
                    const EdgeArgs &A = plans[cur].A;
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
    if (stats && lane == 0) {
        atomicAdd(&stats[0], n_states);
        atomicAdd(&stats[1], n_edges);
        if constexpr (GRID) atomicAdd(&stats[2], (unsigned long long)n_tests);  // wave total
    }
}

// Edges with H == 2: every candidate is free.
__global__ void __launch_bounds__(kTile) k_batch_no_interior(const BPlan *plans, int n_plans) {
    const uint32_t g = blockIdx.x;
    const int p = find_plan(0, n_plans, g, [&](int i) { return plans[i].tile_base; });
    const EdgeArgs &A = plans[p].A;
    if (A.n_int != 0) return;
    const uint32_t tile = g - plans[p].tile_base;
    if (threadIdx.x >= A.tile_cnt[tile]) return;
    const uint32_t row = tile / A.tiles_per_row;
    const uint32_t seg = tile - row * A.tiles_per_row;
    const RowInfo ri = decode_row(A, row);
    const uint32_t n = seg * kTile + A.tile_off[(size_t)tile * kTile + threadIdx.x];
    float u[GTMP_MAX_DOF], v[GTMP_MAX_DOF];
    load_vertex<GTMP_MAX_DOF>(A, ri.u_base + n * ri.u_step, u);
    load_vertex<GTMP_MAX_DOF>(A, ri.v_base + n * ri.v_step, v);
    ri.c_base[(size_t)n * ri.c_step] = edge_len<GTMP_MAX_DOF>(u, v, A.d);
    if (A.flags) A.flags[ri.e_base + (uint64_t)n * ri.e_step] = 0;
}

// ------------------------------------------------------------------ sweep
struct BBest {
    float v;
    int i;
};
__device__ __forceinline__ void btake(BBest &b, float v, int i) {
    if (v < b.v) { b.v = v; b.i = i; }
}
__device__ __forceinline__ BBest bwave_argmin(BBest b) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const float ov = __shfl_xor(b.v, off);
        const int oi = __shfl_xor(b.i, off);
        if (ov < b.v || (ov == b.v && (unsigned)oi < (unsigned)b.i)) { b.v = ov; b.i = oi; }
    }
    return b;
}

// Step k of the backward recursion for every plan: k = 0 is the goal layer,
// k >= 1 the inner layer m = M - 1 - k (plans with fewer layers idle).
// One wave per (plan, row).
__global__ void __launch_bounds__(256) k_batch_layer(const BPlan *plans, int n_plans, int k, uint32_t total_rows) {
    const uint32_t wave = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (wave >= total_rows) return;
    const int p = find_plan(0, n_plans, wave, [&](int i) { return plans[i].row_base; });
    const BPlan &P = plans[p];
    const EdgeArgs &A = P.A;
    const int u = (int)(wave - P.row_base);
    if (u >= A.N) return;
    const int lane = lane_id();
    const int N = A.N, M = A.M;
    if (k == 0) {
        if (lane == 0) {
            BBest b{__builtin_inff(), -1};
            for (int g = 0; g < A.G; ++g) btake(b, A.C_l[(size_t)u * A.G + g], g);
            P.V[(size_t)(M - 1) * N + u] = b.v;
            P.Aidx[(size_t)(M - 1) * N + u] = b.i;
        }
        return;
    }
    const int m = M - 1 - k;
    if (m < 0) return;
    const float *row = A.C_h + ((size_t)m * N + u) * N;
    const float *vn = P.V + (size_t)(m + 1) * N;
    BBest b{__builtin_inff(), -1};
    for (int v = lane; v < N; v += kWave) btake(b, row[v] + vn[v], v);
    b = bwave_argmin(b);
    if (lane == 0) {
        P.V[(size_t)m * N + u] = b.v;
        P.Aidx[(size_t)m * N + u] = b.i;
    }
}

// Start row, extraction and archive of every plan: one block per plan.
__global__ void __launch_bounds__(256) k_batch_finish(const BPlan *plans, int n_plans) {
    __shared__ float sv[4];
    __shared__ int si[4];
    const int p = blockIdx.x;
    if (p >= n_plans) return;
    const BPlan &P = plans[p];
    const EdgeArgs &A = P.A;
    const int N = A.N, M = A.M, d = A.d;
    BBest b{__builtin_inff(), -1};
    for (int u = threadIdx.x; u < N; u += blockDim.x) btake(b, A.C_s[u] + P.V[u], u);
    b = bwave_argmin(b);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) { sv[w] = b.v; si[w] = b.i; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    BBest r{__builtin_inff(), -1};
    for (int kk = 0; kk < 4; ++kk)
        if (sv[kk] < r.v || (sv[kk] == r.v && (unsigned)si[kk] < (unsigned)r.i)) { r.v = sv[kk]; r.i = si[kk]; }
    *P.Vs = r.v;
    *P.as = r.i;
    // extraction (Alg. 1), as k_extract
    float c = r.v;
    int i = r.i;
    bool ok = i >= 0 && i < N && c < __builtin_inff();
    int ii = i;
    for (int m = 0; m < M && ok; ++m) {
        const int nx = P.Aidx[(size_t)m * N + ii];
        ok = nx >= 0 && nx < (m + 1 < M ? N : A.G);
        ii = ok ? nx : 0;
    }
    if (!ok) {
        for (int m = 0; m <= M; ++m) P.idx[m] = -1;
        for (int kk = 0; kk < (M + 2) * d; ++kk) P.wp[kk] = __builtin_nanf("");
        c = __builtin_inff();
    } else {
        for (int jj = 0; jj < d; ++jj) P.wp[jj] = P.q0[jj];
        for (int m = 0; m < M; ++m) {
            P.idx[m] = i;
            for (int jj = 0; jj < d; ++jj) P.wp[(size_t)(m + 1) * d + jj] = P.Q[((size_t)m * N + i) * d + jj];
            i = P.Aidx[(size_t)m * N + i];
        }
        P.idx[M] = i;
        for (int jj = 0; jj < d; ++jj) P.wp[(size_t)(M + 1) * d + jj] = P.goals[(size_t)i * d + jj];
    }
    *P.cost = c;
    // archive (|K| = 1): strictly lower cost replaces
    const uint32_t stage = *P.counter;
    if ((int)stage < P.max_stages) P.stage_costs[stage] = c;
    if (c < *P.best_cost) {
        *P.best_cost = c;
        for (int m = 0; m <= M; ++m) P.best_idx[m] = P.idx[m];
        for (int kk = 0; kk < (M + 2) * d; ++kk) P.best_wp[kk] = P.wp[kk];
        P.best_meta[0] = (int32_t)stage;
        P.best_meta[1] = M;
        P.best_meta[2] = N;
    }
    P.best_meta[3] = (int32_t)stage + 1;
    *P.counter = stage + 1;
}

__global__ void k_batch_init(const BPlan *plans, int n_plans) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_plans) return;
    const BPlan &P = plans[p];
    *P.best_cost = __builtin_inff();
    P.best_meta[0] = -1;
    P.best_meta[1] = 0;
    P.best_meta[2] = 0;
    P.best_meta[3] = 0;
    *P.counter = 0;
}

// Rounding bound of the expanded sphere test per arm plan (see
// k_store_params_tol): one wave per plan of the group range [p0, p1).
__global__ void __launch_bounds__(64) k_batch_arm_tol(const BPlan *plans, int p0) {
    const BPlan &P = plans[p0 + blockIdx.x];
    float cmax = 0.f, rmax = 0.f;
    for (int o = threadIdx.x; o < P.S.n_sph; o += blockDim.x) {
        const float *c = P.S.sph + 4 * o;
        cmax = __builtin_fmaxf(cmax, __builtin_sqrtf(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]));
        rmax = __builtin_fmaxf(rmax, __builtin_fabsf(c[3]));
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        cmax = __builtin_fmaxf(cmax, __shfl_xor(cmax, off));
        rmax = __builtin_fmaxf(rmax, __shfl_xor(rmax, off));
    }
    if (threadIdx.x == 0) {
        ArmParams *R = const_cast<ArmParams *>(P.arm);
        const float pc = (R->reach + cmax) * 1.001f, rr = (rmax + R->r0) * 1.001f;
        R->sph_tol = 0x1p-19f * (pc * pc + rr * rr);
    }
}

// Obstacle bins of every arm plan of the group range [p0, p0 + gridDim.x)
// (one block per plan; the bins depend on the scene and the robot radii only).
__global__ void __launch_bounds__(kGridBuildThreads) k_batch_build_grid(const BPlan *plans, int p0, int wdim) {
    const BPlan &P = plans[p0 + blockIdx.x];
    build_grid_block(P.S, wdim, P.grid_r_max, const_cast<ObsGrid *>(P.A.grid));
}

__global__ void k_batch_zero(uint32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_store_params_n(const ArmParams *src, ArmParams *dst, int n) {
    // src is a kernel-argument-free copy path: words of n structs
    const uint32_t *s = reinterpret_cast<const uint32_t *>(src);
    uint32_t *dd = reinterpret_cast<uint32_t *>(dst);
    const size_t words = (size_t)n * (sizeof(ArmParams) / 4);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
        dd[i] = s[i];
}

// ------------------------------------------------------------------ host side
static int persistent_blocks(const void *kernel, int per_cu_req, int auto_cap = 1 << 20) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    int per_cu = per_cu_req;
    if (per_cu <= 0) {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, 256, 0) != hipSuccess || occ <= 0) occ = 2;
        per_cu = occ < auto_cap ? occ : auto_cap;
    }
    return cus * per_cu;
}

size_t batch_table_bytes() { return sizeof(BPlan); }

BatchLayout make_batch_layout(const gtmp_plan_desc *plans, int n, const gtmp_batch_opts &o) {
    BatchLayout L{};
    L.n = n;
    size_t off = 0;
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    L.plan_off.resize(n);
    L.schedules.resize(n);
    int max_stages = 0;
    for (int p = 0; p < n; ++p) {
        const gtmp_plan_desc &D = plans[p];
        std::vector<StageShape> &S = L.schedules[p];
        if (D.mode == GTMP_ANYTIME_GROWING) {
            int M = D.M_min, N = D.N_min, n_old = 0;
            for (int s = 0; s < D.stages; ++s) {
                S.push_back({M, N, n_old});
                if (M >= D.problem.M && N >= D.problem.N) break;
                if (N < D.problem.N) {
                    n_old = N;
                    N = 2 * N < D.problem.N ? 2 * N : D.problem.N;
                } else {
                    ++M;
                    n_old = 0;
                }
            }
        } else {
            for (int s = 0; s < D.stages; ++s) S.push_back({D.problem.M, D.problem.N, 0});
        }
        if ((int)S.size() > max_stages) max_stages = (int)S.size();
        const uint64_t M = D.problem.M, N = D.problem.N, d = D.problem.d, G = D.problem.G;
        PlanOffsets &P = L.plan_off[p];
        P.Q = off; off = up(off + sizeof(float) * M * N * d);
        P.Q2 = off; off = up(off + (D.mode == GTMP_ANYTIME_GROWING ? sizeof(float) * M * N * d : 0));
        P.Cs = off; off = up(off + sizeof(float) * N);
        P.Ch = off; off = up(off + sizeof(float) * (M > 1 ? M - 1 : 1) * N * N);
        P.Cl = off; off = up(off + sizeof(float) * N * G);
        P.V = off; off = up(off + sizeof(float) * M * N);
        P.A = off; off = up(off + sizeof(int32_t) * M * N);
        P.small = off; off = up(off + 256 + sizeof(int32_t) * (M + 1) + sizeof(float) * (M + 2) * d);
        const EdgePlan ep = make_edge_plan(D.problem);
        P.edge = off; off = up(off + ep.total);
        if (D.mode == GTMP_ANYTIME_GROWING) {
            const ExpandPlan xp = make_expand_plan(D.problem);
            P.expand = off; off = up(off + xp.total);
        } else {
            P.expand = 0;
        }
    }
    L.max_stages = max_stages;
    L.off_arm = off; off = up(off + sizeof(ArmParams) * (size_t)n);
    L.off_grids = off; off = up(off + sizeof(ObsGrid) * (size_t)n);
    L.off_tables = off; off = up(off + sizeof(BPlan) * (size_t)n * (size_t)max_stages);
    L.off_bases = off; off = up(off + sizeof(uint64_t) * (size_t)n * (size_t)max_stages);
    L.off_jobs = off; off = up(off + sizeof(ExpandJob) * (size_t)n * (size_t)max_stages);
    L.off_counters = off; off = up(off + sizeof(uint32_t) * kBatchStageCounters * (size_t)max_stages + 256);
    L.total = off;
    (void)o;
    return L;
}

// ------------------------------------------------------------------ graph cache
// An instantiated batch graph depends on everything the host put into its
// kernel arguments and tables: the plan descriptors (sizes, policies, seeds,
// device pointers), the options, the output buffers and the workspace.  A
// call whose key matches an earlier one launches that graph again; the
// tables it reads live in the workspace and are uploaded again only if
// another batch wrote that workspace in between.  Graphs are kept for the
// life of the process, at most kMaxBatchGraphs of them (later keys are
// captured, launched, waited for and released as before).
namespace {
struct BatchGraph {
    hipGraphExec_t exec;
    std::vector<ArmParams> arms;
    std::vector<BPlan> host;
    std::vector<uint64_t> bases;
    std::vector<ExpandJob> jobs;
};
constexpr size_t kMaxBatchGraphs = 64;
std::mutex g_batch_mu;
std::map<std::string, BatchGraph> g_batch_graphs;
std::map<const void *, std::string> g_batch_ws_owner;  // the key whose tables a workspace holds

template <class T>
void key_add(std::string &k, const T &v) {
    k.append(reinterpret_cast<const char *>(&v), sizeof(T));
}

std::string batch_key(const gtmp_plan_desc *plans, int n, const gtmp_batch_opts &o, const BatchLayout &L,
                      const BatchOut &out, const void *workspace) {
    std::string k;
    key_add(k, n);
    k.append(reinterpret_cast<const char *>(plans), sizeof(gtmp_plan_desc) * (size_t)n);
    key_add(k, o);
    key_add(k, L.total);
    key_add(k, out.best_cost);
    key_add(k, out.best_idx);
    key_add(k, out.best_wp);
    key_add(k, out.best_meta);
    key_add(k, out.stage_costs);
    key_add(k, out.stage_stride);
    key_add(k, workspace);
    return k;
}

hipError_t upload_tables(const BatchLayout &L, void *workspace, const std::vector<ArmParams> &arms,
                         const std::vector<BPlan> &host, const std::vector<uint64_t> &bases,
                         const std::vector<ExpandJob> &jobs, hipStream_t s) {
    // after the work already on the stream (which may still read an earlier
    // table) is done
    char *ws = static_cast<char *>(workspace);
    hipError_t err = hipStreamSynchronize(s);
    if (err != hipSuccess) return err;
    err = hipMemcpy(ws + L.off_arm, arms.data(), sizeof(ArmParams) * arms.size(), hipMemcpyHostToDevice);
    if (err != hipSuccess) return err;
    err = hipMemcpy(ws + L.off_tables, host.data(), sizeof(BPlan) * host.size(), hipMemcpyHostToDevice);
    if (err != hipSuccess) return err;
    err = hipMemcpy(ws + L.off_bases, bases.data(), sizeof(uint64_t) * bases.size(), hipMemcpyHostToDevice);
    if (err != hipSuccess || jobs.empty()) return err;
    return hipMemcpy(ws + L.off_jobs, jobs.data(), sizeof(ExpandJob) * jobs.size(), hipMemcpyHostToDevice);
}
}  // namespace

hipError_t launch_batch(const gtmp_plan_desc *plans, const ArmParams *arms_host, int n, const gtmp_batch_opts &o,
                        const BatchLayout &L, const BatchOut &out, void *workspace, hipStream_t s) {
    std::string key;
    if (o.use_graph) {
        key = batch_key(plans, n, o, L, out, workspace);
        std::lock_guard<std::mutex> lk(g_batch_mu);
        auto it = g_batch_graphs.find(key);
        if (it != g_batch_graphs.end()) {
            auto ow = g_batch_ws_owner.find(workspace);
            if (ow == g_batch_ws_owner.end() || ow->second != key) {
                hipError_t err = upload_tables(L, workspace, it->second.arms, it->second.host, it->second.bases,
                                               it->second.jobs, s);
                if (err != hipSuccess) return err;
                g_batch_ws_owner[workspace] = key;
            }
            return hipGraphLaunch(it->second.exec, s);
        }
    }
    char *ws = static_cast<char *>(workspace);
    ArmParams *arm_dev = reinterpret_cast<ArmParams *>(ws + L.off_arm);
    BPlan *tables = reinterpret_cast<BPlan *>(ws + L.off_tables);
    uint64_t *bases = reinterpret_cast<uint64_t *>(ws + L.off_bases);
    uint32_t *counters = reinterpret_cast<uint32_t *>(ws + L.off_counters);
    (void)arm_dev;

    // ---- host tables of every stage (plans grouped: 2D points, 3D points, arms)
    std::vector<ArmParams> arms(arms_host, arms_host + n);
    std::vector<int> group(n);
    for (int p = 0; p < n; ++p) {
        const gtmp_plan_desc &D = plans[p];
        group[p] = D.robot.kind == GTMP_ROBOT_DH_ARM ? 2 : (D.scene.wdim == 2 ? 0 : 1);
    }
    std::vector<int> order(n);
    for (int p = 0; p < n; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return group[a] < group[b]; });
    int kp = 8;
    for (int p = 0; p < n; ++p)
        if (group[p] == 2) kp = std::max(kp, ((arms[p].n_spheres + 7) / 8) * 8);
    bool uniform_r = true;
    for (int p = 0; p < n; ++p)
        if (group[p] == 2 && !arms[p].uniform_r) uniform_r = false;
    // the obstacle-bin filter for the arm group (automatic choice) when every
    // arm plan's scene fits the masks; mask words: the most any plan needs
    int grid_words = o.sphere_chunks == 0 ? 1 : 0;
    for (int p = 0; p < n && grid_words; ++p) {
        if (group[p] != 2) continue;
        const int n_obs = plans[p].scene.n_spheres + plans[p].scene.n_boxes;
        if (n_obs > 64) grid_words = 0;  // the arm kernels take at most two mask words
        else if (n_obs > 32) grid_words = 2;
    }
    // the same bins for the 2D point group when every plan's scene fits them
    // (four states per lane; states_per_iter then applies to the full test only)
    int pgrid_words = 0;
    if (o.sphere_chunks == 0) {
        int most = 1;
        for (int p = 0; p < n; ++p)
            if (group[p] == 0) most = std::max(most, plans[p].scene.n_spheres + plans[p].scene.n_boxes);
        pgrid_words = most <= kGridMaxObs ? grid_words_for(most) : 0;
    }
    ObsGrid *grids = reinterpret_cast<ObsGrid *>(ws + L.off_grids);

    struct StageInfo {
        int count;
        int g0, g1, g2, g3;       // plan index ranges per group: [g0,g1) 2D, [g1,g2) 3D, [g2,g3) arms
        uint32_t verts[3];
        uint32_t gtiles[3];
        uint32_t tiles;
        uint32_t rows;
        uint64_t samples;
        int maxM;
        uint32_t pblocks[3];
        bool any_interior, any_no_interior;
    };
    std::vector<StageInfo> info(L.max_stages);
    std::vector<BPlan> host(n * (size_t)L.max_stages);
    std::vector<uint64_t> host_bases(n * (size_t)L.max_stages);
    for (int st = 0; st < L.max_stages; ++st) {
        StageInfo I{};
        uint32_t vb[3] = {0, 0, 0}, gb[3] = {0, 0, 0}, pbb[3] = {0, 0, 0}, tb = 0, rb = 0;
        uint64_t sb = 0;
        int cnt = 0;
        int gstart[4] = {0, 0, 0, 0};
        for (int gi = 0; gi < 3; ++gi) {
            gstart[gi] = cnt;
            for (int p : order) {
                if (group[p] != gi || st >= (int)L.schedules[p].size()) continue;
                const gtmp_plan_desc &D = plans[p];
                const StageShape sh = L.schedules[p][st];
                gtmp_problem pp = D.problem;
                pp.M = sh.M;
                pp.N = sh.N;
                const EdgePlan ep = make_edge_plan(pp);
                const PlanOffsets &PO = L.plan_off[p];
                BPlan B{};
                char *ews = ws + PO.edge;
                EdgeArgs &A = B.A;
                A.d = pp.d; A.M = pp.M; A.N = pp.N; A.G = pp.G; A.H = pp.H; A.dp = vertex_stride(pp.d);
                A.penalty = pp.penalty; A.max_len = pp.max_edge_len;
                A.tiles_per_row = ep.tiles_per_row; A.n_tiles = ep.n_tiles; A.n_vertices = ep.n_vertices;
                A.prepass_rows = prepass_rows_for(ep.n_tiles);
                A.verts = reinterpret_cast<float *>(ews + ep.off_verts);
                A.vflag = reinterpret_cast<uint8_t *>(ews + ep.off_vflag);
                A.C_s = reinterpret_cast<float *>(ws + PO.Cs);
                A.C_h = reinterpret_cast<float *>(ws + PO.Ch);
                A.C_l = reinterpret_cast<float *>(ws + PO.Cl);
                A.flags = nullptr;
                A.prune = nullptr;
                A.tile_off = reinterpret_cast<uint8_t *>(ews + ep.off_tile_off);
                A.tile_cnt = reinterpret_cast<uint32_t *>(ews + ep.off_tile_cnt);
                A.counter = nullptr;
                A.stats = nullptr;
                uint8_t ordr[GTMP_MAX_H];
                A.n_int = interior_order(pp.H, ordr);
                for (int i = 0; i < A.n_int; ++i) A.tord[i] = (float)ordr[i] / (float)(pp.H - 1);
                B.S = SceneParams{D.scene.spheres, D.scene.boxes, D.scene.n_spheres, D.scene.n_boxes};
                B.arm = gi == 2 ? arm_dev + p : nullptr;
                if (gi == 0) {
                    A.grid = grids + p;  // point robot: bins for radius 0
                    B.grid_r_max = 0.f;
                }
                if (gi == 2) {
                    A.grid = grids + p;
                    float r_max = 0.f;
                    for (int k = 0; k < arms[p].n_spheres; ++k) r_max = std::max(r_max, arms[p].r[k]);
                    B.grid_r_max = r_max;
                }
                B.group = gi;
                B.vert_base = vb[gi]; vb[gi] += ep.n_vertices;
                B.gtile_base = gb[gi]; gb[gi] += ep.n_tiles;
                B.pblock_base = pbb[gi]; pbb[gi] += prepass_block_count(A);
                B.tile_base = tb; tb += ep.n_tiles;
                B.row_base = rb; rb += (uint32_t)pp.N;
                // samples: restart stages draw uniform samples into Q; growing
                // stages expand into Q / Q2 alternately (stage parity)
                float *Qa = reinterpret_cast<float *>(ws + PO.Q);
                float *Qb = reinterpret_cast<float *>(ws + PO.Q2);
                const bool grow = D.mode == GTMP_ANYTIME_GROWING;
                B.Q = grow ? ((st & 1) ? Qb : Qa) : Qa;
                B.q0 = D.q0;
                B.goals = D.goals;
                char *small = ws + PO.small;
                B.V = reinterpret_cast<float *>(ws + PO.V);
                B.Aidx = reinterpret_cast<int32_t *>(ws + PO.A);
                B.Vs = reinterpret_cast<float *>(small);
                B.as = reinterpret_cast<int32_t *>(small + 4);
                B.cost = reinterpret_cast<float *>(small + 8);
                B.idx = reinterpret_cast<int32_t *>(small + 256);
                B.wp = reinterpret_cast<float *>(small + 256 + sizeof(int32_t) * (D.problem.M + 1));
                B.best_cost = out.best_cost + p;
                B.best_idx = out.best_idx + out.idx_offset[p];
                B.best_wp = out.best_wp + out.wp_offset[p];
                B.best_meta = out.best_meta + 4 * (size_t)p;
                B.stage_costs = out.stage_costs + (size_t)p * out.stage_stride;
                B.max_stages = out.stage_stride;
                B.counter = reinterpret_cast<uint32_t *>(small + 12);
                B.sample = grow ? 0 : 1;
                B.k0 = (uint32_t)(D.seed & 0xffffffffu);
                B.k1 = (uint32_t)(D.seed >> 32);
                B.stage = (uint32_t)st;
                for (int j = 0; j < pp.d; ++j) {
                    B.lo[j] = pp.lo[j];
                    B.wd[j] = pp.hi[j] - pp.lo[j];
                }
                host[(size_t)st * n + cnt] = B;
                host_bases[(size_t)st * n + cnt] = sb;
                sb += grow ? 0 : (uint64_t)pp.M * pp.N * ((pp.d + 3) / 4);
                if (A.n_int > 0) I.any_interior = true;
                else I.any_no_interior = true;
                if (pp.M > I.maxM) I.maxM = pp.M;
                ++cnt;
            }
        }
        gstart[3] = cnt;
        I.count = cnt;
        I.g0 = gstart[0]; I.g1 = gstart[1]; I.g2 = gstart[2]; I.g3 = gstart[3];
        for (int gi = 0; gi < 3; ++gi) {
            I.verts[gi] = vb[gi];
            I.gtiles[gi] = gb[gi];
            I.pblocks[gi] = pbb[gi];
        }
        I.tiles = tb;
        I.rows = rb;
        I.samples = sb;
        info[st] = I;
    }
    // the growing plans' expansions of each stage, run together (one launch
    // per kernel and layer step for all of them)
    std::vector<ExpandJob> jobs;
    std::vector<size_t> job_begin(L.max_stages + 1, 0);
    for (int st = 0; st < L.max_stages; ++st) {
        job_begin[st] = jobs.size();
        for (int p = 0; p < n; ++p) {
            if (plans[p].mode != GTMP_ANYTIME_GROWING || st >= (int)L.schedules[p].size()) continue;
            const StageShape sh = L.schedules[p][st];
            gtmp_problem pp = plans[p].problem;
            pp.M = sh.M;
            pp.N = sh.N;
            const PlanOffsets &PO = L.plan_off[p];
            float *Qa = reinterpret_cast<float *>(ws + PO.Q);
            float *Qb = reinterpret_cast<float *>(ws + PO.Q2);
            ExpandJob J;
            fill_expand_job(J, pp, plans[p].q0, plans[p].goals, (st & 1) ? Qa : Qb, sh.n_old, (st & 1) ? Qb : Qa,
                            out.best_cost + p, plans[p].seed, (uint64_t)st, ws + PO.expand);
            jobs.push_back(J);
        }
    }
    job_begin[L.max_stages] = jobs.size();
    const ExpandJob *jobs_dev = reinterpret_cast<const ExpandJob *>(ws + L.off_jobs);

    // tables are written once, before any work is enqueued
    hipError_t err = upload_tables(L, workspace, arms, host, host_bases, jobs, s);
    if (err != hipSuccess) return err;
    {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        if (o.use_graph) g_batch_ws_owner[workspace] = key;
        else g_batch_ws_owner.erase(workspace);
    }

    // point robots: 8 states per lane and at most 3 resident blocks per CU
    // unless asked otherwise (as the single-plan launcher)
    const int spi = o.states_per_iter == 1 || o.states_per_iter == 2 || o.states_per_iter == 4 ? o.states_per_iter : 8;
    const int nch = o.sphere_chunks == 1 ? 1 : o.sphere_chunks == 4 ? 4 : 2;

    auto enqueue = [&](hipStream_t st_) -> hipError_t {
        if (info.empty()) return hipSuccess;
        // archive init over the plans of stage 0 (every plan has a stage 0)
        hipLaunchKernelGGL(k_batch_init, dim3((info[0].count + 255) / 256), dim3(256), 0, st_, tables, info[0].count);
        if (pgrid_words && info[0].g1 > info[0].g0)
            hipLaunchKernelGGL(k_batch_build_grid, dim3(info[0].g1 - info[0].g0), dim3(kGridBuildThreads), 0, st_,
                               tables, info[0].g0, 2);
        if (info[0].g3 > info[0].g2) {
            hipLaunchKernelGGL(k_batch_arm_tol, dim3(info[0].g3 - info[0].g2), dim3(64), 0, st_, tables, info[0].g2);
            if (grid_words)
                hipLaunchKernelGGL(k_batch_build_grid, dim3(info[0].g3 - info[0].g2), dim3(kGridBuildThreads), 0, st_,
                                   tables, info[0].g2, 3);
        }
        for (int st = 0; st < L.max_stages; ++st) {
            const StageInfo &I = info[st];
            const BPlan *T = tables + (size_t)st * n;
            const uint64_t *Bs = bases + (size_t)st * n;
            uint32_t *ctr = counters + kBatchStageCounters * st;  // the three groups' cursors
            hipLaunchKernelGGL(k_batch_zero, dim3(kBatchStageCounters / 256), dim3(256), 0, st_, ctr,
                               kBatchStageCounters);
            // samples
            if (I.samples > 0)
                hipLaunchKernelGGL(k_batch_sample, dim3((unsigned)((I.samples + 255) / 256)), dim3(256), 0, st_, T,
                                   I.count, Bs, I.samples);
            if (job_begin[st + 1] > job_begin[st]) {
                const std::vector<ExpandJob> stage_jobs(jobs.begin() + job_begin[st], jobs.begin() + job_begin[st + 1]);
                hipError_t e = launch_expand_jobs(jobs_dev + job_begin[st], stage_jobs, st_);
                if (e != hipSuccess) return e;
            }
            // vertices per group
            if (I.verts[0] > 0)
                hipLaunchKernelGGL((k_batch_vertices<0, 1>), dim3((I.verts[0] + 255) / 256), dim3(256), 0, st_, T,
                                   I.g0, I.g1, I.verts[0]);
            if (I.verts[1] > 0)
                hipLaunchKernelGGL((k_batch_vertices<1, 1>), dim3((I.verts[1] + 255) / 256), dim3(256), 0, st_, T,
                                   I.g1, I.g2, I.verts[1]);
            if (I.verts[2] > 0)
                hipLaunchKernelGGL((k_batch_vertices<2, 8>), dim3((I.verts[2] + 255) / 256), dim3(256), 0, st_, T,
                                   I.g2, I.g3, I.verts[2]);
            if (I.pblocks[0] > 0)
                hipLaunchKernelGGL(k_batch_prepass<2>, dim3(I.pblocks[0]), dim3(kTile), 0, st_, T, I.g0, I.g1);
            if (I.pblocks[1] > 0)
                hipLaunchKernelGGL(k_batch_prepass<3>, dim3(I.pblocks[1]), dim3(kTile), 0, st_, T, I.g1, I.g2);
            if (I.pblocks[2] > 0)
                hipLaunchKernelGGL(k_batch_prepass<GTMP_MAX_JOINTS>, dim3(I.pblocks[2]), dim3(kTile), 0, st_, T, I.g2,
                                   I.g3);
            if (I.any_no_interior)  // H = 2 plans: every candidate is free
                hipLaunchKernelGGL(k_batch_no_interior, dim3(I.tiles), dim3(kTile), 0, st_, T, I.count);
            // persistent interior per group
            if (I.gtiles[0] > 0) {
                const void *k = pgrid_words == 1 ? (const void *)k_batch_interior<PointGridModel<2, 4, 1>, true, 1>
                              : pgrid_words == 2 ? (const void *)k_batch_interior<PointGridModel<2, 4, 2>, true, 1>
                              : pgrid_words == 3 ? (const void *)k_batch_interior<PointGridModel<2, 4, 3>, true, 1>
                              : spi == 1 ? (const void *)k_batch_interior<PointModel<2, 1>, true, 1>
                              : spi == 2 ? (const void *)k_batch_interior<PointModel<2, 2>, true, 1>
                              : spi == 8 ? (const void *)k_batch_interior<PointModel<2, 8>, true, 1>
                                         : (const void *)k_batch_interior<PointModel<2, 4>, true, 1>;
                const int grid = persistent_blocks(k, o.blocks_per_cu, 3);
                void *args[] = {(void *)&T, (void *)&I.g0, (void *)&I.g1, (void *)&I.gtiles[0], (void *)&ctr,
                                (void *)&out.stats};
                hipError_t e = hipLaunchKernel(k, dim3(grid), dim3(256), args, 0, st_);
                if (e != hipSuccess) return e;
            }
            if (I.gtiles[1] > 0) {
                const void *k = (const void *)k_batch_interior<PointModel<3, 8>, true, 1>;
                const int grid = persistent_blocks(k, o.blocks_per_cu, 3);
                uint32_t *c1 = ctr + kBatchGroupCounters;
                void *args[] = {(void *)&T, (void *)&I.g1, (void *)&I.g2, (void *)&I.gtiles[1], (void *)&c1,
                                (void *)&out.stats};
                hipError_t e = hipLaunchKernel(k, dim3(grid), dim3(256), args, 0, st_);
                if (e != hipSuccess) return e;
            }
            if (I.gtiles[2] > 0) {
                const void *k = nullptr;
#define GTMP_BK1(K, C) (uniform_r ? (const void *)k_batch_interior<ArmModel<K>, true, C> : (const void *)k_batch_interior<ArmModel<K>, false, C>)
#define GTMP_BK(K) \
    if (kp == K) k = nch == 1 ? GTMP_BK1(K, 1) : nch == 4 ? GTMP_BK1(K, 4) : GTMP_BK1(K, 2);
                GTMP_BK(8) GTMP_BK(16) GTMP_BK(24) GTMP_BK(32) GTMP_BK(40) GTMP_BK(48) GTMP_BK(56) GTMP_BK(64)
#undef GTMP_BK
#undef GTMP_BK1
                if (grid_words == 1)
                    k = uniform_r ? (const void *)k_batch_interior<ArmGridModel<1>, true, 1>
                                  : (const void *)k_batch_interior<ArmGridModel<1>, false, 1>;
                if (grid_words == 2)
                    k = uniform_r ? (const void *)k_batch_interior<ArmGridModel<2>, true, 1>
                                  : (const void *)k_batch_interior<ArmGridModel<2>, false, 1>;
                if (!k) return hipErrorInvalidValue;
                const int grid = persistent_blocks(k, o.blocks_per_cu);
                uint32_t *c2 = ctr + 2 * kBatchGroupCounters;
                void *args[] = {(void *)&T, (void *)&I.g2, (void *)&I.g3, (void *)&I.gtiles[2], (void *)&c2,
                                (void *)&out.stats};
                hipError_t e = hipLaunchKernel(k, dim3(grid), dim3(256), args, 0, st_);
                if (e != hipSuccess) return e;
            }
            // backward sweep: step 0 = goal layer, step k = layer M-1-k
            const unsigned lblocks = (I.rows + 3) / 4;
            for (int k = 0; k < I.maxM; ++k)
                hipLaunchKernelGGL(k_batch_layer, dim3(lblocks), dim3(256), 0, st_, T, I.count, k, I.rows);
            hipLaunchKernelGGL(k_batch_finish, dim3(I.count), dim3(256), 0, st_, T, I.count);
        }
        return hipGetLastError();
    };

    // every stage of every policy is capturable: no memset and no host
    // read-back anywhere in the enqueued work (the growing plans' pair
    // ranking included)
    if (!o.use_graph) return enqueue(s);
    hipStream_t cs;
    err = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (err != hipSuccess) return err;
    err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (err != hipSuccess) { (void)hipStreamDestroy(cs); return err; }
    hipError_t e_ops = enqueue(cs);
    hipGraph_t g = nullptr;
    err = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (e_ops != hipSuccess) { if (g) (void)hipGraphDestroy(g); return e_ops; }
    if (err != hipSuccess) return err;
    hipGraphExec_t exec = nullptr;
    err = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (err != hipSuccess) return err;
    {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        if (g_batch_graphs.size() < kMaxBatchGraphs) {
            g_batch_graphs.emplace(key, BatchGraph{exec, std::move(arms), std::move(host), std::move(host_bases),
                                                   std::move(jobs)});
            return hipGraphLaunch(exec, s);
        }
    }
    err = hipGraphLaunch(exec, s);
    // beyond the cache: the executable graph is released once the stream has run it
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    (void)hipGraphExecDestroy(exec);
    return err;
}

}  // namespace gtmp
