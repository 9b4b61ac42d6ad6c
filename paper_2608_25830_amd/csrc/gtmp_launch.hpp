// gtmp_launch.hpp -- host-side launchers shared between the kernel sources
// and the C-ABI layer (api.hip).  Arguments have been validated by the
// caller; launchers only enqueue.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "gtmp.h"
#include "gtmp_device.hpp"

namespace gtmp {


struct EdgePlan {
    // sizes
    int d, M, N, G, H;
    float penalty, max_len;
    // derived
    uint32_t n_vertices;     // 1 + M N + G
    uint32_t rows;           // 1 + (M-1) N + G
    uint32_t tiles_per_row;  // ceil(N / kTile)
    uint32_t n_tiles;
    // workspace carve-up (byte offsets)
    size_t off_verts, off_vflag, off_tile_off, off_tile_cnt, off_counter, off_params, off_grid, off_wstats, total;
};

EdgePlan make_edge_plan(const gtmp_problem &p);

struct EdgeBuffers {
    const float *q0, *goals, *Q;
    float *C_s, *C_h, *C_l;
    float *minsd;
    uint8_t *flags;
    const uint8_t *prune;
    void *workspace;
};

hipError_t launch_edge_check(const EdgePlan &plan, const ArmParams *arm /* NULL = point robot */,
                             const SceneParams &scene, int wdim, const EdgeBuffers &b, const gtmp_edge_opts &o,
                             hipStream_t s);
// The fast-mode check in phases: kPhaseVertices packs the vertices and their
// collision flags into the workspace; kPhaseEdges runs the pre-pass and the
// interior checks.  With edge_list given (device, *n_list flat edge ids of
// edges with free endpoints within the length limit) kPhaseEdges checks those
// edges only, without a pre-pass, and writes each one's cost and flag (the
// others are left as they are); list_mark (device, per flat edge id) holds a
// value other than 2 for each listed edge and is set to 2 for those that
// collide.
constexpr int kPhaseVertices = 1, kPhaseEdges = 2;
hipError_t launch_edge_phases(const EdgePlan &plan, const ArmParams *arm, const SceneParams &scene, int wdim,
                              const EdgeBuffers &b, const gtmp_edge_opts &o, hipStream_t s,
                              const uint32_t *edge_list, const uint32_t *n_list, uint8_t *list_mark, int phases);

hipError_t launch_state_check(const ArmParams *arm, const SceneParams &scene, int wdim, int d, int64_t n,
                              const float *X, float *sd, uint8_t *coll, hipStream_t s);

hipError_t launch_sample_layers(const gtmp_problem &p, uint64_t seed, uint64_t stage, float *Q, hipStream_t s);

hipError_t launch_minplus(int M, int N, int G, const float *C_s, const float *C_h, const float *C_l,
                          const float *Vg, float *V, int32_t *A, float *V_s, int32_t *a_s, hipStream_t s);

hipError_t launch_extract(int M, int N, int G, int d, const int32_t *a_s, const int32_t *A, const float *V_s,
                          const float *Q, const float *q0, const float *goals, int32_t *idx, float *wp,
                          float *cost, hipStream_t s);

// ---- ranking of sample pairs (select.hip): the K closest pairs of U [nu][d]
// and V [nv][d] by FP32 squared distance (summed in coordinate order, no
// contraction), ties by pair index a * nv + b, as pair indices in rank order
// (K <= nu nv < 2^32).  Asynchronous, no memset.
struct RankPlan {
    uint32_t cap;  // candidate keys the final sort holds
    size_t off_state, off_hist, off_cand, total;
};
RankPlan make_rank_plan(uint32_t max_k);
hipError_t launch_rank_pairs(int d, int nu, const float *U, int nv, const float *V, uint32_t K, uint32_t *out,
                             const RankPlan &rp, void *workspace, hipStream_t s);

// ---- growing-budget sampler and anytime drivers (anytime.hip)
struct ExpandPlan {
    uint32_t max_k;  // closest pairs ranked per layer at most
    size_t off_informed, off_rank, off_sorted, off_rankws;
    // surrogate-biased heuristic half (when planned with bias)
    uint64_t bias_rows;
    size_t off_bX, off_bz, off_bfree, off_bcount, off_bws, bws_bytes;
    size_t total;
};
// One growing plan's expansion inside a batch: the arguments of
// launch_expand (no surrogate bias) with the workspace carved as
// make_expand_plan lays it out.  launch_expand_jobs runs the expansions of
// several plans together, kernel by kernel (each launch covers every plan),
// with the same kernels' device code and results as launch_expand.
struct ExpandJob {
    int d, M, N, G, n_old;
    float penalty;
    float lo[GTMP_MAX_DOF], hi[GTMP_MAX_DOF];
    uint32_t k0, k1, stage;
    const float *q0, *goals, *Q_old;
    float *Q_new;
    const float *c_dev;
    void *informed;
    int32_t *rank;
    uint32_t *sorted;
    char *rankws;
    uint32_t rank_cap;
    uint32_t rank_off_hist, rank_off_cand;
};
void fill_expand_job(ExpandJob &J, const gtmp_problem &p, const float *q0, const float *goals, const float *Q_old,
                     int n_old, float *Q_new, const float *c_dev, uint64_t seed, uint64_t stage, void *workspace);
hipError_t launch_expand_jobs(const ExpandJob *jobs_dev, const std::vector<ExpandJob> &jobs, hipStream_t s);

// closest pairs scored by the surrogate per new slot of a layer
constexpr int kBiasCandidates = 4;
struct SurNet;
ExpandPlan make_expand_plan(const gtmp_problem &p, bool bias = false);
hipError_t launch_expand(const gtmp_problem &p, const float *q0, const float *goals, const float *Q_old, int n_old,
                         float *Q_new, const float *c_dev, uint64_t seed, uint64_t stage, void *workspace,
                         hipStream_t s, const SurNet *bias = nullptr, float bias_tau = 0.f);
hipError_t launch_informed_batch(const gtmp_problem &p, const float *q0, const float *goals, const float *c_dev,
                                 uint64_t seed, uint64_t stage, uint32_t m, int count, float *X, int32_t *attempts,
                                 void *workspace, hipStream_t s);

struct AnytimePlan {
    gtmp_problem big;  // sizes the buffers are carved for
    size_t off_Q, off_Q2, off_Cs, off_Ch, off_Cl, off_V, off_A, off_small, off_counter, off_simp, off_flags, off_rrtc,
        off_edge, off_expand, total;
};
AnytimePlan make_anytime_plan(const gtmp_problem &p, const gtmp_anytime_opts &o);

struct AnytimeOut {
    float *best_cost;
    int32_t *best_idx;
    float *best_wp;
    int32_t *best_meta;
    float *stage_costs;
};
hipError_t launch_anytime(const gtmp_problem &p, const ArmParams *arm, const SceneParams &scene, int wdim,
                          const float *q0, const float *goals, uint64_t seed, const gtmp_anytime_opts &o,
                          const gtmp_edge_opts &eo, const AnytimeOut &out, void *workspace, hipStream_t s,
                          const SurNet *bias = nullptr);

// ---- class-augmented sweep and class archive (classes.hip)
struct ClassPlan {
    size_t off_lab, off_cost, off_nxt, off_cnt, off_s, total;
};
ClassPlan make_class_plan(int M, int N, int L);
hipError_t launch_class_sweep(int M, int N, int G, int L, const float *Q, const float *q0, const float *goals,
                              const float *C_s, const float *C_h, const float *C_l, float penalty, const float *reps,
                              int k, uint64_t *labels, float *costs, int32_t *chains, int32_t *count,
                              uint32_t *overflow, bool reset_overflow, void *ws, hipStream_t s);
hipError_t launch_class_archive(int M, int N, int stage, const float *Q, const float *q0, const float *goals,
                                const uint64_t *labels, const float *costs, const int32_t *chains,
                                const int32_t *count, int cap, uint64_t *a_lab, float *a_cost, int32_t *a_stage,
                                float *a_wp, int32_t *a_count, uint32_t *overflow, hipStream_t s);
struct ClassAnytimePlan {
    size_t off_Q, off_Cs, off_Ch, off_Cl, off_out, off_edge, off_class, total;
};
ClassAnytimePlan make_class_anytime_plan(const gtmp_problem &p, int L);
hipError_t launch_plan_classes(const gtmp_problem &p, const SceneParams &scene, const float *q0, const float *goals,
                               uint64_t seed, int stages, const float *reps, int k, int L, int cap, uint64_t *a_lab,
                               float *a_cost, int32_t *a_stage, float *a_wp, int32_t *a_count, uint32_t *overflow,
                               const gtmp_edge_opts &eo, void *workspace, hipStream_t s);

// ---- path shortcutting (simplify.hip)
hipError_t launch_simplify(const ArmParams *arm, const SceneParams &scene, int wdim, int d, int B, int K, int H,
                           const float *wp, uint8_t *valid, int32_t *idx, int32_t *count, float *cost, float *out_wp,
                           hipStream_t s);

// ---- RRT-Connect local planner (rrtc.hip)
struct RrtcPlan {
    size_t off_counters, off_vfree, off_cand, total;
};
RrtcPlan make_rrtc_plan(const gtmp_problem &p);
size_t rrtc_lds_bytes(int d, int cap, int obstacle_floats);
hipError_t launch_rrtc_repair(const gtmp_problem &p, const ArmParams *arm, const SceneParams &S, int wdim,
                              const float *q0, const float *goals, const float *Q, float *C_s, float *C_h, float *C_l,
                              uint8_t *flags, uint64_t seed, uint64_t stage, const gtmp_rrtc_opts &o, void *workspace,
                              hipStream_t s, const uint32_t *stage_dev = nullptr);
hipError_t launch_rrtc_path(const gtmp_problem &p, const ArmParams *arm, const SceneParams &S, int wdim,
                            const float *q0, const float *goals, const float *Q, uint64_t edge, uint64_t seed,
                            uint64_t stage, const gtmp_rrtc_opts &o, float *path, int32_t *count, float *cost,
                            hipStream_t s);

// ---- lazy edge realisation (lazy.hip)
struct LazyPlan {
    size_t off_edge, off_F, off_select, off_list, off_counters, total;
};
LazyPlan make_lazy_plan(const gtmp_problem &p);
hipError_t launch_plan_lazy(const gtmp_problem &p, const ArmParams *arm, const SceneParams &S, int wdim,
                            const float *q0, const float *goals, const float *Q, float *C_s, float *C_h, float *C_l,
                            uint8_t *flags, float *V, int32_t *Am, float *V_s, int32_t *a_s, int32_t *idx, float *wp,
                            float *cost, float band, int max_rounds, unsigned long long *stats,
                            const gtmp_edge_opts &eo, void *workspace, int *rounds_host, bool *done_host,
                            hipStream_t s);

// ---- batched plans (batch.hip)
struct StageShape {
    int M, N, n_old;
};
struct PlanOffsets {
    size_t Q, Q2, Cs, Ch, Cl, V, A, small, edge, expand;
};
struct BatchLayout {
    int n, max_stages;
    std::vector<PlanOffsets> plan_off;
    std::vector<std::vector<StageShape>> schedules;
    size_t off_arm, off_grids, off_tables, off_bases, off_jobs, off_counters, total;
};
BatchLayout make_batch_layout(const gtmp_plan_desc *plans, int n, const gtmp_batch_opts &o);
struct BatchOut {
    float *best_cost;
    int32_t *best_idx;
    float *best_wp;
    int32_t *best_meta;
    float *stage_costs;
    int stage_stride;
    std::vector<size_t> idx_offset, wp_offset;
    unsigned long long *stats;
};
hipError_t launch_batch(const gtmp_plan_desc *plans, const ArmParams *arms_host, int n, const gtmp_batch_opts &o,
                        const BatchLayout &L, const BatchOut &out, void *workspace, hipStream_t s);

// Bisection order of the interior states 1..H-2 (midpoint first, then the
// midpoints of the remaining halves, breadth first).  Returns the count.
int interior_order(int H, uint8_t *order_out);

}  // namespace gtmp
