// classes.hip -- class-augmented value iteration on the layered DAG (Sec. IV-B;
// Prop. 2) and the class-indexed archive of Anytime-GTMP (Sec. IV-D) for 2D
// point robots.
//
// Class label of an edge: its signed crossings with upward rays from up to 16
// representative obstacle points, one 8-bit field per point in a 128-bit
// label held as two 64-bit words (fields 0..7 in the first, 8..15 in the
// second).  A chain of at most 127 edges (M <= 126) crosses a ray at most 127
// times, so every count fits a field: chain labels are kept in offset binary
// (the empty label has every field at 128) and edge labels in two's
// complement, and a sum is a field-wise addition modulo 256 with no carries
// between fields (SWAR addition).  The crossing decision is taken in FP32
// with a fixed operation order; this file is compiled without contraction.
//
// Sweep: one wave per vertex u.  Lane j holds entry j of u's list (label, least
// cost of a chain from u to the goal with that label, successor).  For every
// successor v (in index order) the candidates kappa(u, v) + chi, C(u, v) +
// J(v, chi) arrive one per lane (v's entries); each is matched against u's
// entries by broadcast, a lower cost replaces the entry's, a new label is
// appended.  When a list is full, a new label replaces the costliest entry if
// it is cheaper and the overflow counter counts every label dropped: results
// are exact whenever the counter stays zero.
#include "gtmp_launch.hpp"

namespace gtmp {

constexpr int kClassMaxReps = 16;
constexpr uint64_t kByteHigh = 0x8080808080808080ull;
constexpr uint64_t kEmptyWord = 0x8080808080808080ull;  // eight fields at zero, offset binary

struct Label {
    uint64_t w[2];
};

__device__ __forceinline__ uint64_t swar_add(uint64_t x, uint64_t y) {
    return ((x & ~kByteHigh) + (y & ~kByteHigh)) ^ ((x ^ y) & kByteHigh);
}

__device__ __forceinline__ Label label_add(const Label &a, const Label &b) {
    return Label{{swar_add(a.w[0], b.w[0]), swar_add(a.w[1], b.w[1])}};
}

__device__ __forceinline__ bool label_eq(const Label &a, const Label &b) {
    return a.w[0] == b.w[0] && a.w[1] == b.w[1];
}

// Signed crossings of u -> v with the upward rays of reps[0..k), packed in
// two's complement.
__device__ __forceinline__ Label edge_label(float ux, float uy, float vx, float vy, const float *reps, int k) {
    Label lab{{0ull, 0ull}};
    for (int i = 0; i < k; ++i) {
        const float zx = reps[2 * i], zy = reps[2 * i + 1];
        if ((ux < zx) == (vx < zx)) continue;
        const float dx = vx - ux, dy = vy - uy, ex = zx - ux, ey = zy - uy;
        const float cross = dx * ey - dy * ex;
        const bool above = dx > 0.f ? cross < 0.f : cross > 0.f;
        if (!above) continue;
        const uint64_t field = dx > 0.f ? 1ull : 255ull;  // +1 or -1 mod 256
        lab.w[i >> 3] |= field << (8 * (i & 7));
    }
    return lab;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ Label readlane_label(const Label &x, int l) {
    return Label{{readlane64(x.w[0], l), readlane64(x.w[1], l)}};
}

__device__ __forceinline__ uint64_t shfl64(uint64_t x, int l) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)x, l);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ Label load_label(const uint64_t *p, size_t i) {
    const ulonglong2 v = reinterpret_cast<const ulonglong2 *>(p)[i];
    return Label{{v.x, v.y}};
}

__device__ __forceinline__ void store_label(uint64_t *p, size_t i, const Label &l) {
    reinterpret_cast<ulonglong2 *>(p)[i] = make_ulonglong2(l.w[0], l.w[1]);
}

struct ClassLists {
    uint64_t *lab;   // [M][N][L][2]
    float *cost;     // [M][N][L]
    uint32_t *nxt;   // [M][N][L]: successor << 8 | its entry
    int32_t *cnt;    // [M][N]
    uint64_t *s_lab; // start list [L][2]
    float *s_cost;
    uint32_t *s_nxt;
    int32_t *s_cnt;  // [1]
    uint32_t *overflow;  // [1] labels dropped by full lists
};

// One wave per vertex u of layer m (m = -1: the start vertex).
__global__ void __launch_bounds__(256) k_class_layer(int m, int M, int N, int G, int L, const float *__restrict__ Q,
                                                     const float *__restrict__ q0, const float *__restrict__ goals,
                                                     const float *__restrict__ C_s, const float *__restrict__ C_h,
                                                     const float *__restrict__ C_l, float penalty,
                                                     const float *__restrict__ reps, int k, ClassLists CL) {
    const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
    const int lane = lane_id();
    const int n_u = m < 0 ? 1 : N;
    if (wave >= n_u) return;
    const int u = wave;
    const float *pu = m < 0 ? q0 : Q + ((size_t)m * N + u) * 2;
    const float ux = pu[0], uy = pu[1];
    const int nv = m == M - 1 ? G : N;

    Label my_lab{{0ull, 0ull}};
    float my_cost = __builtin_inff();
    uint32_t my_nxt = 0;
    int cnt = 0;
    uint32_t dropped = 0;

    for (int v = 0; v < nv; ++v) {
        float c;
        const float *pv;
        if (m < 0) {
            c = C_s[v];
            pv = Q + (size_t)v * 2;
        } else if (m == M - 1) {
            c = C_l[(size_t)u * G + v];
            pv = goals + (size_t)v * 2;
        } else {
            c = C_h[((size_t)m * N + u) * N + v];
            pv = Q + ((size_t)(m + 1) * N + v) * 2;
        }
        c = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(c)));  // one value for the wave
        if (!(c < penalty)) continue;  // absent or failed edge
        const Label kap = edge_label(ux, uy, pv[0], pv[1], reps, k);
        // candidates: one per lane
        int n_src;
        Label cl{{0ull, 0ull}};
        float cc = __builtin_inff();
        uint32_t cn = 0;
        if (m == M - 1) {
            n_src = 1;
            if (lane == 0) {
                cl = label_add(kap, Label{{kEmptyWord, kEmptyWord}});
                cc = c;
                cn = (uint32_t)v << 8;
            }
        } else {
            const int mm = m + 1;  // successor layer (0 for the start)
            n_src = __builtin_amdgcn_readfirstlane(CL.cnt[(size_t)mm * N + v]);
            if (lane < n_src) {
                const size_t base = ((size_t)mm * N + v) * L + lane;
                cl = label_add(kap, load_label(CL.lab, base));
                cc = c + CL.cost[base];
                cn = ((uint32_t)v << 8) | (uint32_t)lane;
            }
        }
        if (n_src == 0) continue;
        // match: list lane j finds the candidate with its label (labels are
        // distinct within u's list and within one successor's candidates)
        uint64_t matched = 0;
        int src = -1;
        for (int e = 0; e < n_src; ++e) {
            const Label le = readlane_label(cl, e);
            const bool hit = lane < cnt && label_eq(my_lab, le);
            if (hit) src = e;
            if (ballot(hit) != 0) matched |= 1ull << e;
        }
        {
            const float pc = __shfl(cc, src < 0 ? 0 : src);
            const uint32_t pn = (uint32_t)__shfl((int)cn, src < 0 ? 0 : src);
            if (src >= 0 && pc < my_cost) {
                my_cost = pc;
                my_nxt = pn;
            }
        }
        // new labels: appended in candidate order while there is room
        uint64_t pending = (n_src >= 64 ? ~0ull : ((1ull << n_src) - 1ull)) & ~matched;
        const int n_new = __popcll(pending);
        if (n_new == 0) continue;
        const int room = L - cnt;
        const int n_app = n_new < room ? n_new : room;
        int asrc = -1;
        for (int idx = 0; idx < n_app; ++idx) {
            const int e = __builtin_ctzll(pending);
            pending &= pending - 1;
            if (lane == cnt + idx) asrc = e;
        }
        {
            const int from = asrc < 0 ? 0 : asrc;
            const Label pl{{shfl64(cl.w[0], from), shfl64(cl.w[1], from)}};
            const float pc = __shfl(cc, from);
            const uint32_t pn = (uint32_t)__shfl((int)cn, from);
            if (asrc >= 0) {
                my_lab = pl;
                my_cost = pc;
                my_nxt = pn;
            }
        }
        cnt += n_app;
        // full list: each remaining label replaces the costliest entry if cheaper
        while (pending != 0) {
            const int e = __builtin_ctzll(pending);
            pending &= pending - 1;
            const Label el = readlane_label(cl, e);
            const float ec = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(cc), e));
            const uint32_t en = __builtin_amdgcn_readlane(cn, e);
            float mx = lane < cnt ? my_cost : -__builtin_inff();
            int arg = lane;
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) {
                const float om = __shfl_xor(mx, off);
                const int oa = __shfl_xor(arg, off);
                if (om > mx || (om == mx && oa > arg)) {
                    mx = om;
                    arg = oa;
                }
            }
            ++dropped;  // either this label or the replaced one
            if (ec < mx && lane == arg) {
                my_lab = el;
                my_cost = ec;
                my_nxt = en;
            }
        }
    }
    // store u's list
    if (m < 0) {
        if (lane < cnt) {
            store_label(CL.s_lab, lane, my_lab);
            CL.s_cost[lane] = my_cost;
            CL.s_nxt[lane] = my_nxt;
        }
        if (lane == 0) *CL.s_cnt = cnt;
    } else {
        const size_t base = ((size_t)m * N + u) * L;
        if (lane < cnt) {
            store_label(CL.lab, base + lane, my_lab);
            CL.cost[base + lane] = my_cost;
            CL.nxt[base + lane] = my_nxt;
        }
        if (lane == 0) CL.cnt[(size_t)m * N + u] = cnt;
    }
    if (lane == 0 && dropped) atomicAdd(CL.overflow, dropped);
}

// Chains of the start list: lane e follows entry e through the layers.
__global__ void __launch_bounds__(64) k_class_extract(int M, int N, int L, ClassLists CL, uint64_t *labels,
                                                      float *costs, int32_t *chains, int32_t *count) {
    const int e = threadIdx.x;
    const int n = *CL.s_cnt;
    if (e == 0) *count = n;
    if (e >= n) return;
    labels[2 * e] = CL.s_lab[2 * e];
    labels[2 * e + 1] = CL.s_lab[2 * e + 1];
    costs[e] = CL.s_cost[e];
    uint32_t nx = CL.s_nxt[e];
    for (int m = 0; m < M; ++m) {
        const int v = (int)(nx >> 8), ent = (int)(nx & 0xffu);
        chains[(size_t)e * (M + 1) + m] = v;
        nx = CL.nxt[((size_t)m * N + v) * L + ent];
    }
    chains[(size_t)e * (M + 1) + M] = (int)(nx >> 8);
}

__global__ void k_class_reset(uint32_t *overflow) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *overflow = 0u;
}

// Class-indexed archive update (one wave): per label the lowest cost, a later
// stage replacing an entry only with a strictly lower cost; waypoints copied
// from this stage's samples.
__global__ void __launch_bounds__(64) k_class_archive(int M, int N, int stage, const float *__restrict__ Q,
                                                      const float *__restrict__ q0, const float *__restrict__ goals,
                                                      const uint64_t *labels, const float *costs,
                                                      const int32_t *chains, const int32_t *count, int cap,
                                                      uint64_t *a_lab, float *a_cost, int32_t *a_stage, float *a_wp,
                                                      int32_t *a_count, uint32_t *overflow) {
    const int lane = lane_id();
    const int n = *count;
    // the labels of one stage are distinct, so only entries of earlier stages
    // (the first na0) can match; new entries are appended after them
    const int na0 = *a_count;
    int na = na0;
    for (int e = 0; e < n; ++e) {
        const uint64_t lab0 = labels[2 * e], lab1 = labels[2 * e + 1];
        const float c = costs[e];
        int found = -1;
        for (int base = 0; base < na0; base += kWave) {
            const int j = base + lane;
            const uint64_t hit = ballot(j < na0 && a_lab[2 * j] == lab0 && a_lab[2 * j + 1] == lab1);
            if (hit != 0) {
                found = base + __builtin_ctzll(hit);
                break;
            }
        }
        int slot = -1;
        if (found >= 0) {
            if (c < a_cost[found]) slot = found;
        } else if (na < cap) {
            slot = na++;
        } else if (lane == 0) {
            atomicAdd(overflow, 1u);
        }
        if (slot < 0) continue;
        if (lane == 0) {
            a_lab[2 * slot] = lab0;
            a_lab[2 * slot + 1] = lab1;
            a_cost[slot] = c;
            a_stage[slot] = stage;
        }
        // waypoints q0, Q[0][i0], ..., Q[M-1][i_{M-1}], goal
        const int32_t *ch = chains + (size_t)e * (M + 1);
        float *wp = a_wp + (size_t)slot * (M + 2) * 2;
        for (int p = lane; p < M + 2; p += kWave) {
            const float *src = p == 0 ? q0 : (p <= M ? Q + ((size_t)(p - 1) * N + ch[p - 1]) * 2 : goals + (size_t)ch[M] * 2);
            wp[2 * p] = src[0];
            wp[2 * p + 1] = src[1];
        }
    }
    if (lane == 0) *a_count = na;
}

// ------------------------------------------------------------------ host side
static size_t up256c(size_t x) { return (x + 255) & ~size_t(255); }

ClassPlan make_class_plan(int M, int N, int L) {
    ClassPlan p{};
    size_t o = 0;
    const size_t e = (size_t)M * N * L;
    p.off_lab = o; o = up256c(o + 2 * sizeof(uint64_t) * e);
    p.off_cost = o; o = up256c(o + sizeof(float) * e);
    p.off_nxt = o; o = up256c(o + sizeof(uint32_t) * e);
    p.off_cnt = o; o = up256c(o + sizeof(int32_t) * (size_t)M * N);
    p.off_s = o; o = up256c(o + (2 * sizeof(uint64_t) + sizeof(float) + sizeof(uint32_t)) * (size_t)L + 64);
    p.total = o;
    return p;
}

static ClassLists carve_lists(const ClassPlan &p, int L, void *ws, uint32_t *overflow) {
    char *w = static_cast<char *>(ws);
    ClassLists CL{};
    CL.lab = reinterpret_cast<uint64_t *>(w + p.off_lab);
    CL.cost = reinterpret_cast<float *>(w + p.off_cost);
    CL.nxt = reinterpret_cast<uint32_t *>(w + p.off_nxt);
    CL.cnt = reinterpret_cast<int32_t *>(w + p.off_cnt);
    char *s = w + p.off_s;
    CL.s_lab = reinterpret_cast<uint64_t *>(s);
    CL.s_cost = reinterpret_cast<float *>(s + 2 * sizeof(uint64_t) * L);
    CL.s_nxt = reinterpret_cast<uint32_t *>(s + (2 * sizeof(uint64_t) + sizeof(float)) * L);
    CL.s_cnt = reinterpret_cast<int32_t *>(s + (2 * sizeof(uint64_t) + sizeof(float) + sizeof(uint32_t)) * L);
    CL.overflow = overflow;
    return CL;
}

hipError_t launch_class_sweep(int M, int N, int G, int L, const float *Q, const float *q0, const float *goals,
                              const float *C_s, const float *C_h, const float *C_l, float penalty, const float *reps,
                              int k, uint64_t *labels, float *costs, int32_t *chains, int32_t *count,
                              uint32_t *overflow, bool reset_overflow, void *ws, hipStream_t s) {
    const ClassPlan p = make_class_plan(M, N, L);
    const ClassLists CL = carve_lists(p, L, ws, overflow);
    if (reset_overflow) hipLaunchKernelGGL(k_class_reset, dim3(1), dim3(64), 0, s, overflow);
    const unsigned blocks = (unsigned)((N + 3) / 4);
    for (int m = M - 1; m >= 0; --m)
        hipLaunchKernelGGL(k_class_layer, dim3(blocks), dim3(256), 0, s, m, M, N, G, L, Q, q0, goals, C_s, C_h, C_l,
                           penalty, reps, k, CL);
    hipLaunchKernelGGL(k_class_layer, dim3(1), dim3(256), 0, s, -1, M, N, G, L, Q, q0, goals, C_s, C_h, C_l, penalty,
                       reps, k, CL);
    hipLaunchKernelGGL(k_class_extract, dim3(1), dim3(64), 0, s, M, N, L, CL, labels, costs, chains, count);
    return hipGetLastError();
}

hipError_t launch_class_archive(int M, int N, int stage, const float *Q, const float *q0, const float *goals,
                                const uint64_t *labels, const float *costs, const int32_t *chains,
                                const int32_t *count, int cap, uint64_t *a_lab, float *a_cost, int32_t *a_stage,
                                float *a_wp, int32_t *a_count, uint32_t *overflow, hipStream_t s) {
    hipLaunchKernelGGL(k_class_archive, dim3(1), dim3(64), 0, s, M, N, stage, Q, q0, goals, labels, costs, chains,
                       count, cap, a_lab, a_cost, a_stage, a_wp, a_count, overflow);
    return hipGetLastError();
}

ClassAnytimePlan make_class_anytime_plan(const gtmp_problem &p, int L) {
    ClassAnytimePlan a{};
    const uint64_t M = p.M, N = p.N, G = p.G;
    size_t o = 0;
    a.off_Q = o; o = up256c(o + sizeof(float) * M * N * 2);
    a.off_Cs = o; o = up256c(o + sizeof(float) * N);
    a.off_Ch = o; o = up256c(o + sizeof(float) * (M > 1 ? M - 1 : 1) * N * N);
    a.off_Cl = o; o = up256c(o + sizeof(float) * N * G);
    a.off_out = o; o = up256c(o + (2 * sizeof(uint64_t) + sizeof(float)) * (size_t)L + sizeof(int32_t) * (size_t)L * (M + 1) + 64);
    const EdgePlan ep = make_edge_plan(p);
    a.off_edge = o; o = up256c(o + ep.total);
    const ClassPlan cp = make_class_plan(p.M, p.N, L);
    a.off_class = o; o = up256c(o + cp.total);
    a.total = o;
    return a;
}

__global__ void k_class_archive_init(int32_t *a_count, uint32_t *overflow) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *a_count = 0;
        *overflow = 0u;
    }
}

hipError_t launch_plan_classes(const gtmp_problem &p, const SceneParams &scene, const float *q0, const float *goals,
                               uint64_t seed, int stages, const float *reps, int k, int L, int cap, uint64_t *a_lab,
                               float *a_cost, int32_t *a_stage, float *a_wp, int32_t *a_count, uint32_t *overflow,
                               const gtmp_edge_opts &eo, void *workspace, hipStream_t s) {
    const ClassAnytimePlan a = make_class_anytime_plan(p, L);
    char *ws = static_cast<char *>(workspace);
    float *Q = reinterpret_cast<float *>(ws + a.off_Q);
    float *Cs = reinterpret_cast<float *>(ws + a.off_Cs);
    float *Ch = reinterpret_cast<float *>(ws + a.off_Ch);
    float *Cl = reinterpret_cast<float *>(ws + a.off_Cl);
    char *out = ws + a.off_out;
    uint64_t *labels = reinterpret_cast<uint64_t *>(out);
    float *costs = reinterpret_cast<float *>(out + 2 * sizeof(uint64_t) * L);
    int32_t *chains = reinterpret_cast<int32_t *>(out + (2 * sizeof(uint64_t) + sizeof(float)) * L);
    int32_t *count = reinterpret_cast<int32_t *>(out + (2 * sizeof(uint64_t) + sizeof(float)) * L +
                                                 sizeof(int32_t) * (size_t)L * (p.M + 1));
    hipLaunchKernelGGL(k_class_archive_init, dim3(1), dim3(64), 0, s, a_count, overflow);
    const EdgePlan ep = make_edge_plan(p);
    gtmp_edge_opts e2 = eo;
    e2.ev_begin = nullptr;
    e2.ev_end = nullptr;
    for (int st = 0; st < stages; ++st) {
        hipError_t e = launch_sample_layers(p, seed, (uint64_t)st, Q, s);
        if (e != hipSuccess) return e;
        EdgeBuffers b{q0, goals, Q, Cs, Ch, Cl, nullptr, nullptr, nullptr, ws + a.off_edge};
        e = launch_edge_check(ep, nullptr, scene, 2, b, e2, s);
        if (e != hipSuccess) return e;
        e = launch_class_sweep(p.M, p.N, p.G, L, Q, q0, goals, Cs, Ch, Cl, p.penalty, reps, k, labels, costs, chains,
                               count, overflow, false, ws + a.off_class, s);
        if (e != hipSuccess) return e;
        e = launch_class_archive(p.M, p.N, st, Q, q0, goals, labels, costs, chains, count, cap, a_lab, a_cost, a_stage,
                                 a_wp, a_count, overflow, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace gtmp
