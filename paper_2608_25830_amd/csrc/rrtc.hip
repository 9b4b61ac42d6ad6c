// rrtc.hip -- the RRT-Connect local planner LP(x, y; s, ell) of the
// generalized GTMP graph (Sec. III; construction in the proof of the
// local-planner reach proposition of the appendix), run on every edge whose
// straight line failed while both endpoints are collision-free.
//
// One wave per call, persistent over the candidate list.  The two trees live
// in the wave's LDS (coordinates as [tree][coordinate][node], so that lanes
// reading consecutive nodes touch consecutive banks); a call is a sequence of
// wave-uniform steps, each spread over the 64 lanes:
//   sample   64 ellipsoid attempts at a time, the lowest accepted one wins
//            (the sequential result);
//   nearest  lanes stride over the tree, (squared distance, index) butterfly
//            with the lowest index on ties;
//   check    the states of the extension segment, each shared by 64 / s
//            lanes that split the obstacles between them (s states at a
//            time, a power of two), a ballot ends it at a colliding state.
// This file is compiled without floating-point contraction: sampling, nearest
// node and steering are FP32 computations with a fixed operation order (see
// include/gtmp.h), so the trees are reproducible bit for bit.
#include "edge_common.hpp"
#include "state_test.hpp"

namespace gtmp {

constexpr int kRrtcAttempts = 4096;
constexpr int kRrtcLdsObstacles = 2048;  // obstacle floats held in LDS (more: read from global memory)
enum { kTrapped = 0, kAdvanced = 1, kReached = 2 };

struct RrtcArgs {
    int d, M, N, G;
    const float *q0, *goals, *Q;
    float lo[GTMP_MAX_DOF], hi[GTMP_MAX_DOF];
    // candidates: cand[0 .. *n_cand) pulled through *cursor; cand == NULL runs
    // the single edge `single` on block 0
    const uint32_t *cand;
    const uint32_t *n_cand;
    uint32_t *cursor;
    uint32_t single;
    float *C_s, *C_h, *C_l;
    uint8_t *flags;
    int budget, cap;
    float eta, res, ell_factor;
    uint32_t k0, k1, stage;
    const uint32_t *stage_dev;  // when set, the stage is read here at kernel start (replayed graphs)
    unsigned long long *stats;  // calls, successes, iterations, nodes, states checked, nearest-node distances
    // single-edge outputs (path mode)
    float *path;
    int32_t *path_count;
    float *path_cost;
};

__device__ __forceinline__ void edge_endpoints(const RrtcArgs &A, uint32_t e, const float *&u, const float *&v) {
    const uint32_t N = (uint32_t)A.N;
    const uint64_t inner = (uint64_t)(A.M - 1) * N * N;
    if (e < N) {
        u = A.q0;
        v = A.Q + (size_t)e * A.d;
    } else if ((uint64_t)e - N < inner) {
        const uint64_t r = (uint64_t)e - N;
        const uint64_t m = r / ((uint64_t)N * N), uv = r - m * N * N;
        u = A.Q + ((size_t)m * N + uv / N) * A.d;
        v = A.Q + ((size_t)(m + 1) * N + uv % N) * A.d;
    } else {
        const uint64_t r = (uint64_t)e - N - inner;
        const uint64_t n = r / (uint64_t)A.G, g = r - n * A.G;
        u = A.Q + ((size_t)(A.M - 1) * N + n) * A.d;
        v = A.goals + (size_t)g * A.d;
    }
}

__device__ __forceinline__ float *cost_slot_of(const RrtcArgs &A, uint32_t e) {
    const uint64_t N = (uint64_t)A.N, inner_end = N + (uint64_t)(A.M - 1) * N * N;
    if (e < N) return A.C_s + e;
    if (e < inner_end) return A.C_h + (e - N);
    return A.C_l + (e - inner_end);
}

// Vertex ids of flat edge e in the order [q0 | Q[0] | ... | Q[M-1] | goals].
__device__ __forceinline__ void edge_vertex_ids(const RrtcArgs &A, uint64_t e, uint32_t &u, uint32_t &v) {
    const uint64_t N = (uint64_t)A.N, inner = (uint64_t)(A.M - 1) * N * N;
    if (e < N) {
        u = 0;
        v = 1 + (uint32_t)e;
    } else if (e - N < inner) {
        const uint64_t r = e - N, m = r / (N * N), uv = r - m * N * N;
        u = 1 + (uint32_t)(m * N + uv / N);
        v = 1 + (uint32_t)((m + 1) * N + uv % N);
    } else {
        const uint64_t r = e - N - inner, n = r / (uint64_t)A.G, g = r - n * A.G;
        u = 1 + (uint32_t)((A.M - 1) * N + n);
        v = 1 + (uint32_t)(A.M * N + g);
    }
}

__device__ __forceinline__ const float *vertex_ptr(const RrtcArgs &A, uint32_t id) {
    const uint32_t MN = (uint32_t)A.M * (uint32_t)A.N;
    if (id == 0) return A.q0;
    if (id <= MN) return A.Q + (size_t)(id - 1) * A.d;
    return A.goals + (size_t)(id - 1 - MN) * A.d;
}

__device__ __forceinline__ float f32_d2(int d, const float *a, const float *b) {
    float acc = 0.0f;
    for (int i = 0; i < d; ++i) {
        const float t = a[i] - b[i];
        acc = acc + t * t;
    }
    return acc;
}

// The wave's LDS: coordinates pos[2][d][cap], parents par[2][cap], the
// ellipsoid map (centre, H, radii) and a scratch chain for the path walk.
struct RrtcLds {
    float *pos;
    int32_t *par;
    float *H;  // [d][d]
    int32_t *chain;  // [2 cap]
};

template <bool ARM, int W, int KP>
struct RrtcCall {
    static constexpr int D = StateDim<ARM, W>::D;
    const RrtcArgs &A;
    const ArmParams &R;
    const SceneParams &S;
    RrtcLds L;
    int lane;
    uint32_t stage;
    int n0, n1;  // node counts of the x and y trees (scalars: no dynamically indexed array)
    unsigned long long it_count, states, dists;

    __device__ __forceinline__ int count(int t) const { return t ? n1 : n0; }

    __device__ __forceinline__ float &P(int t, int i, int j) const { return L.pos[((size_t)t * A.d + i) * A.cap + j]; }

    // Extend tree t towards q; returns the status and the new node in *idx.
    __device__ __forceinline__ int extend(int t, const float (&q)[GTMP_MAX_DOF], int *idx) {
        const int d = A.d;
        const int nt = count(t);
        if (nt >= A.cap) return kTrapped;
        dists += (unsigned long long)nt;
        float best = __builtin_inff();
        int bi = 0x7fffffff;
        for (int j = lane; j < nt; j += kWave) {
            float acc = 0.0f;
            for (int i = 0; i < d; ++i) {
                const float tt = P(t, i, j) - q[i];
                acc = acc + tt * tt;
            }
            if (acc < best) {  // j increases: the lowest index among equal values stays
                best = acc;
                bi = j;
            }
        }
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const float ob = __shfl_xor(best, off);
            const int oi = __shfl_xor(bi, off);
            if (ob < best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        const int near = bi;
        float p[GTMP_MAX_DOF], qn[GTMP_MAX_DOF];
        for (int i = 0; i < GTMP_MAX_DOF; ++i) p[i] = i < d ? P(t, i, near) : 0.f;
        const float dist = __builtin_sqrtf(best);
        const bool reached = dist <= A.eta;
        const float f = A.eta / dist;
        for (int i = 0; i < GTMP_MAX_DOF; ++i) qn[i] = i < d ? (reached ? q[i] : p[i] + f * (q[i] - p[i])) : 0.f;
        // the segment p -> qn at H_s states; p itself is a tree node (free).
        // spr states per round (a power of two), lps = 64 / spr lanes sharing
        // each state's obstacles
        const float len = __builtin_sqrtf(f32_d2(d, p, qn));
        int Hs = (int)__builtin_ceilf(len / A.res) + 1;
        Hs = Hs < 2 ? 2 : Hs;
        const float den = (float)(Hs - 1);
        int lg = 0;
        while ((1 << lg) < Hs - 1 && lg < 6) ++lg;
        const int spr = 1 << lg, lgl = 6 - lg, lps = 1 << lgl;
        const int sl = lane >> lgl, part = lane & (lps - 1);
        for (int h0 = 1; h0 < Hs; h0 += spr) {
            const int h = h0 + sl;
            const bool act = h < Hs;
            const float tt = (float)(act ? h : 1) / den;
            float s[D];
#pragma unroll
            for (int i = 0; i < D; ++i)
                s[i] = i < d ? (h == Hs - 1 ? qn[i] : __builtin_fmaf(tt, qn[i] - p[i], p[i])) : 0.f;
            float gap = state_gap_part<ARM, W, KP>(R, S, s, part, lps);
            for (int off = lps >> 1; off > 0; off >>= 1) gap = __builtin_fminf(gap, __shfl_xor(gap, off));
            states += (unsigned long long)(Hs - h0 < spr ? Hs - h0 : spr);
            if (ballot(act && !(gap > 0.f)) != 0) return kTrapped;
        }
        const int k = nt;
        if (lane == 0) {
            for (int i = 0; i < d; ++i) P(t, i, k) = qn[i];
            L.par[t * A.cap + k] = near;
        }
        __syncthreads();
        if (t) n1 = k + 1; else n0 = k + 1;
        *idx = k;
        return reached ? kReached : kAdvanced;
    }

    // The sample of iteration it: true and q set when an attempt passes.
    __device__ __forceinline__ bool sample(uint32_t e, uint32_t it, const float *centre, float r1, float r2,
                           float (&q)[GTMP_MAX_DOF]) const {
        const int d = A.d;
        for (int base = 0; base < kRrtcAttempts; base += kWave) {
            const uint32_t a = (uint32_t)(base + lane);
            const uint4 w0 = philox4x32_10(make_uint4(e, it, stage, (3u << 16) | (2u * a)), A.k0, A.k1);
            const uint4 w1 = philox4x32_10(make_uint4(e, it, stage, (3u << 16) | (2u * a + 1u)), A.k0, A.k1);
            float y[GTMP_MAX_DOF], x[GTMP_MAX_DOF];
            float s2 = 0.0f;
            for (int i = 0; i < GTMP_MAX_DOF; ++i) {
                const uint32_t wi = i == 0 ? w0.x : i == 1 ? w0.y : i == 2 ? w0.z : i == 3 ? w0.w
                                  : i == 4 ? w1.x : i == 5 ? w1.y : i == 6 ? w1.z : w1.w;
                y[i] = (float)(wi >> 8) * (1.0f / 8388608.0f) - 1.0f;
                if (i < d) s2 = s2 + y[i] * y[i];
            }
            bool ok = s2 < 1.0f;
            for (int r = 0; r < GTMP_MAX_DOF; ++r) {
                float acc = 0.0f;
                if (r < d) {
                    for (int c = 0; c < d; ++c) acc = acc + L.H[r * d + c] * ((c == 0 ? r1 : r2) * y[c]);
                    x[r] = centre[r] + acc;
                    ok = ok && x[r] >= A.lo[r] && x[r] <= A.hi[r];
                } else {
                    x[r] = 0.f;
                }
            }
            const uint64_t m = ballot(ok);
            if (m != 0) {
                const int src = __builtin_ctzll(m);
                for (int i = 0; i < GTMP_MAX_DOF; ++i) q[i] = __shfl(x[i], src);
                return true;
            }
        }
        return false;
    }

    // Run one call on edge e.  Returns success; the path length in *cost.
    __device__ __forceinline__ bool run(uint32_t e, float *cost) {
        const int d = A.d;
        const float *pu, *pv;
        edge_endpoints(A, e, pu, pv);
        float x[GTMP_MAX_DOF], y[GTMP_MAX_DOF];
        for (int i = 0; i < GTMP_MAX_DOF; ++i) {
            x[i] = i < d ? pu[i] : 0.f;
            y[i] = i < d ? pv[i] : 0.f;
        }
        // query ellipsoid: foci x, y, major axis ell (hyperspheroid map as in
        // the informed set of Sec. IV-E)
        const float cmin = __builtin_sqrtf(f32_d2(d, x, y));
        const float ell = A.ell_factor * cmin;
        float centre[GTMP_MAX_DOF];
        for (int i = 0; i < GTMP_MAX_DOF; ++i) centre[i] = (x[i] + y[i]) * 0.5f;
        const float r1 = ell * 0.5f;
        const float sq = ell * ell - cmin * cmin;
        const float r2 = __builtin_sqrtf(sq > 0.0f ? sq : 0.0f) * 0.5f;
        {
            float w[GTMP_MAX_DOF];
            float ww = 0.0f;
            for (int i = 0; i < d; ++i) {
                const float a = (y[i] - x[i]) / cmin;
                w[i] = (i == 0 ? 1.0f : 0.0f) - a;
                ww = ww + w[i] * w[i];
            }
            if (lane < d * d) {
                const int i = lane / d, j = lane - (lane / d) * d;
                const float delta = i == j ? 1.0f : 0.0f;
                float hv = delta;
                if (ww != 0.0f) {
                    const float s = 2.0f / ww;
                    hv = delta - (s * w[i]) * w[j];
                }
                L.H[lane] = hv;
            }
        }
        if (lane == 0) {
            for (int i = 0; i < d; ++i) {
                P(0, i, 0) = x[i];
                P(1, i, 0) = y[i];
            }
            L.par[0] = -1;
            L.par[A.cap] = -1;
        }
        __syncthreads();
        n0 = n1 = 1;
        int ta = 0;  // tree A: 0 = the x tree
        bool ok = false;
        int ax = -1, ay = -1;
        uint32_t it = 0;
        for (; it < (uint32_t)A.budget && !ok; ++it) {
            float q[GTMP_MAX_DOF];
            if (sample(e, it, centre, r1, r2, q)) {
                int ia = -1;
                if (extend(ta, q, &ia) != kTrapped) {
                    float qn[GTMP_MAX_DOF];
                    for (int i = 0; i < GTMP_MAX_DOF; ++i) qn[i] = i < d ? P(ta, i, ia) : 0.f;
                    int ib = -1, st;
                    do {
                        st = extend(1 - ta, qn, &ib);
                    } while (st == kAdvanced);
                    if (st == kReached) {
                        ok = true;
                        ax = ta == 0 ? ia : ib;
                        ay = ta == 0 ? ib : ia;
                    }
                }
            }
            ta = 1 - ta;
        }
        it_count += it;
        *cost = __builtin_inff();
        if (!ok) return false;
        // path x -> ... -> junction -> ... -> y: the x tree's chain from the
        // junction to its root (stored junction first), then the y tree's
        // chain from the junction's parent to its root; the length is summed
        // along the path from x to y
        if (lane == 0) {
            int nc = 0;
            for (int j = ax; j >= 0; j = L.par[j]) L.chain[nc++] = j;  // x tree, junction first
            const int nx = nc;
            for (int j = L.par[A.cap + ay]; j >= 0; j = L.par[A.cap + j]) L.chain[nc++] = A.cap + j;  // y tree
            // k-th waypoint of the path: x chain reversed, then the y chain
            auto node = [&](int k) { return k < nx ? L.chain[nx - 1 - k] : L.chain[k]; };
            float Lsum = 0.0f;
            for (int k = 0; k + 1 < nc; ++k) {
                const int a = node(k), b = node(k + 1);
                const int ta_ = a >= A.cap, tb_ = b >= A.cap;
                float s2 = 0.0f;
                for (int i = 0; i < d; ++i) {
                    const float tt = P(tb_, i, b - tb_ * A.cap) - P(ta_, i, a - ta_ * A.cap);
                    s2 = s2 + tt * tt;
                }
                Lsum = Lsum + __builtin_sqrtf(s2);
            }
            *cost = Lsum;
            if (A.path) {
                // waypoints in path order: the x chain reversed, then the y chain
                int np = 0;
                for (int k = nx - 1; k >= 0; --k, ++np)
                    for (int i = 0; i < d; ++i) A.path[(size_t)np * d + i] = P(0, i, L.chain[k]);
                for (int k = nx; k < nc; ++k, ++np)
                    for (int i = 0; i < d; ++i) A.path[(size_t)np * d + i] = P(1, i, L.chain[k] - A.cap);
                *A.path_count = np;
            }
        }
        *cost = __shfl(*cost, 0);
        return true;
    }
};

// OCC: waves per SIMD the register allocation is made for (2 when the trees
// are small enough for 8 blocks per CU, else 1: more registers, no spills)
template <bool ARM, int W, int KP, int OCC>
__global__ void __launch_bounds__(kWave, OCC) k_rrtc(RrtcArgs A, ArmParams R, SceneParams Sg) {
    extern __shared__ float lds[];
    const int d = A.d;
    RrtcLds L;
    L.pos = lds;
    L.par = reinterpret_cast<int32_t *>(lds + (size_t)2 * d * A.cap);
    L.H = reinterpret_cast<float *>(L.par + 2 * A.cap);
    L.chain = reinterpret_cast<int32_t *>(L.H + GTMP_MAX_DOF * GTMP_MAX_DOF);
    // obstacles copied into LDS when they fit (the extension checks read them
    // with per-lane indices)
    SceneParams S = Sg;
    {
        constexpr int PW = ARM ? 3 : W;
        const int ns = Sg.n_sph * (PW + 1), nb = Sg.n_box * 2 * PW;
        if (ns + nb <= kRrtcLdsObstacles) {
            float *obs = reinterpret_cast<float *>(L.chain + 2 * A.cap);
            for (int i = threadIdx.x; i < ns; i += kWave) obs[i] = Sg.sph[i];
            for (int i = threadIdx.x; i < nb; i += kWave) obs[ns + i] = Sg.box[i];
            S.sph = obs;
            S.box = obs + ns;
            __syncthreads();
        }
    }
    const uint32_t stage = A.stage_dev ? *A.stage_dev : A.stage;
    RrtcCall<ARM, W, KP> c{A, R, S, L, (int)threadIdx.x, stage, 1, 1, 0ull, 0ull, 0ull};
    unsigned long long calls = 0, wins = 0, nodes = 0;
    if (A.cand == nullptr) {  // one edge, path mode
        if (blockIdx.x != 0) return;
        float cost;
        const bool ok = c.run(A.single, &cost);
        if (threadIdx.x == 0) {
            *A.path_cost = cost;
            if (!ok) *A.path_count = 0;
        }
        return;
    }
    const uint32_t total = *A.n_cand;
    while (true) {
        uint32_t slot = 0;
        if (threadIdx.x == 0) slot = atomicAdd(A.cursor, 1u);
        slot = uniform(slot);
        if (slot >= total) break;
        const uint32_t e = A.cand[slot];
        float cost;
        const bool ok = c.run(e, &cost);
        ++calls;
        nodes += (unsigned long long)(c.n0 + c.n1);
        if (ok) {
            ++wins;
            if (threadIdx.x == 0) {
                *cost_slot_of(A, e) = cost;
                A.flags[e] = 2;
            }
        }
    }
    if (A.stats && threadIdx.x == 0) {
        atomicAdd(&A.stats[0], calls);
        atomicAdd(&A.stats[1], wins);
        atomicAdd(&A.stats[2], c.it_count);
        atomicAdd(&A.stats[3], nodes);
        atomicAdd(&A.stats[4], c.states);
        atomicAdd(&A.stats[5], c.dists);
    }
}

// ------------------------------------------------------------------ candidates
template <bool ARM, int W, int KP>
__global__ void __launch_bounds__(256) k_rrtc_vertices(RrtcArgs A, ArmParams R, SceneParams S, uint32_t nv,
                                                       uint8_t *vfree) {
    constexpr int D = StateDim<ARM, W>::D;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t id = i < nv ? i : nv - 1;
    const float *p = vertex_ptr(A, id);
    float q[D];
#pragma unroll
    for (int k = 0; k < D; ++k) q[k] = k < A.d ? p[k] : 0.f;
    const float gap = state_gap<ARM, W, KP>(R, S, q);
    if (i < nv) vfree[i] = gap > 0.f ? 1 : 0;
}

__global__ void k_rrtc_reset(uint32_t *counters) {
    if (threadIdx.x < 2) counters[threadIdx.x] = 0;
}

// Edges whose straight line failed with both endpoints free and within the
// length limit; appended in any order (each call is independent).
__global__ void __launch_bounds__(256) k_rrtc_collect(RrtcArgs A, const uint8_t *vfree, float max_len, uint64_t E,
                                                      uint32_t *cand, uint32_t *n_cand) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E || A.flags[e] != 1) return;
    uint32_t u, v;
    edge_vertex_ids(A, e, u, v);
    if (!vfree[u] || !vfree[v]) return;
    const float *pu = vertex_ptr(A, u), *pv = vertex_ptr(A, v);
    float a[GTMP_MAX_DOF], b[GTMP_MAX_DOF];
    for (int i = 0; i < GTMP_MAX_DOF; ++i) {
        a[i] = i < A.d ? pu[i] : 0.f;
        b[i] = i < A.d ? pv[i] : 0.f;
    }
    if (edge_len<GTMP_MAX_DOF>(a, b, A.d) > max_len) return;  // as the edge check measures it
    cand[atomicAdd(n_cand, 1u)] = (uint32_t)e;
}

// ------------------------------------------------------------------ host side
static size_t up256_r(size_t x) { return (x + 255) & ~size_t(255); }

RrtcPlan make_rrtc_plan(const gtmp_problem &p) {
    RrtcPlan r{};
    const uint64_t N = p.N, M = p.M, G = p.G;
    const uint64_t E = N + (M - 1) * N * N + N * G;
    const uint64_t nv = 1 + M * N + G;
    size_t off = 0;
    r.off_counters = off; off = up256_r(off + 64);
    r.off_vfree = off; off = up256_r(off + nv);
    r.off_cand = off; off = up256_r(off + sizeof(uint32_t) * E);
    r.total = off;
    return r;
}

size_t rrtc_lds_bytes(int d, int cap, int obstacle_floats) {
    const size_t obs = obstacle_floats <= kRrtcLdsObstacles ? (size_t)obstacle_floats : 0;
    return sizeof(float) * ((size_t)2 * d * cap + (size_t)2 * cap + GTMP_MAX_DOF * GTMP_MAX_DOF + (size_t)2 * cap + obs);
}

static RrtcArgs rrtc_args(const gtmp_problem &p, const float *q0, const float *goals, const float *Q, float *C_s,
                          float *C_h, float *C_l, uint8_t *flags, uint64_t seed, uint64_t stage, const gtmp_rrtc_opts &o) {
    RrtcArgs A{};
    A.d = p.d; A.M = p.M; A.N = p.N; A.G = p.G;
    A.q0 = q0; A.goals = goals; A.Q = Q;
    for (int i = 0; i < GTMP_MAX_DOF; ++i) {
        A.lo[i] = i < p.d ? p.lo[i] : 0.f;
        A.hi[i] = i < p.d ? p.hi[i] : 0.f;
    }
    A.C_s = C_s; A.C_h = C_h; A.C_l = C_l; A.flags = flags;
    A.budget = o.budget; A.cap = o.tree_cap;
    A.eta = o.step; A.res = o.resolution; A.ell_factor = o.ell_factor;
    A.k0 = (uint32_t)(seed & 0xffffffffu);
    A.k1 = (uint32_t)(seed >> 32);
    A.stage = (uint32_t)(stage & 0xffffffffu);
    A.stats = o.stats;
    return A;
}

template <bool ARM, int W, int KP>
static hipError_t launch_rrtc_kernels(const RrtcArgs &A, const ArmParams &R, const SceneParams &S, uint64_t E,
                                      float max_len, uint8_t *vfree, uint32_t *cand, uint32_t *counters, bool single,
                                      hipStream_t s) {
    constexpr int PW = ARM ? 3 : W;
    const size_t lds = rrtc_lds_bytes(A.d, A.cap, S.n_sph * (PW + 1) + S.n_box * 2 * PW);
    // 8 blocks (two waves per SIMD) fit in the 160 KiB of LDS of a CU?
    const bool two = lds * 8 <= 163840;
    const void *kern = two ? (const void *)k_rrtc<ARM, W, KP, 2> : (const void *)k_rrtc<ARM, W, KP, 1>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (single) {
        if (two)
            hipLaunchKernelGGL((k_rrtc<ARM, W, KP, 2>), dim3(1), dim3(kWave), lds, s, A, R, S);
        else
            hipLaunchKernelGGL((k_rrtc<ARM, W, KP, 1>), dim3(1), dim3(kWave), lds, s, A, R, S);
        return hipGetLastError();
    }
    const uint32_t nv = 1 + (uint32_t)A.M * A.N + A.G;
    hipLaunchKernelGGL((k_rrtc_vertices<ARM, W, KP>), dim3((nv + 255) / 256), dim3(256), 0, s, A, R, S, nv, vfree);
    hipLaunchKernelGGL(k_rrtc_reset, dim3(1), dim3(64), 0, s, counters);
    hipLaunchKernelGGL(k_rrtc_collect, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, s, A, vfree, max_len, E, cand,
                       counters);
    RrtcArgs B = A;
    B.cand = cand;
    B.n_cand = counters;
    B.cursor = counters + 1;
    int dev = 0, cus = 256, occ = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kWave, lds) != hipSuccess || occ <= 0) occ = 1;
    occ = occ < 16 ? occ : 16;
    if (two)
        hipLaunchKernelGGL((k_rrtc<ARM, W, KP, 2>), dim3(cus * occ), dim3(kWave), lds, s, B, R, S);
    else
        hipLaunchKernelGGL((k_rrtc<ARM, W, KP, 1>), dim3(cus * occ), dim3(kWave), lds, s, B, R, S);
    return hipGetLastError();
}

static hipError_t dispatch_rrtc(const ArmParams *arm, int wdim, const RrtcArgs &A, const SceneParams &S, uint64_t E,
                                float max_len, uint8_t *vfree, uint32_t *cand, uint32_t *counters, bool single,
                                hipStream_t s) {
    ArmParams R{};
    if (arm) {
        R = *arm;
        switch (round8(R.n_spheres)) {
#define GTMP_RC(KP) case KP: return launch_rrtc_kernels<true, 3, KP>(A, R, S, E, max_len, vfree, cand, counters, single, s);
            GTMP_RC(8) GTMP_RC(16) GTMP_RC(24) GTMP_RC(32) GTMP_RC(40) GTMP_RC(48) GTMP_RC(56) GTMP_RC(64)
#undef GTMP_RC
            default: return hipErrorInvalidValue;
        }
    }
    if (wdim == 2) return launch_rrtc_kernels<false, 2, 1>(A, R, S, E, max_len, vfree, cand, counters, single, s);
    return launch_rrtc_kernels<false, 3, 1>(A, R, S, E, max_len, vfree, cand, counters, single, s);
}

hipError_t launch_rrtc_repair(const gtmp_problem &p, const ArmParams *arm, const SceneParams &S, int wdim,
                              const float *q0, const float *goals, const float *Q, float *C_s, float *C_h, float *C_l,
                              uint8_t *flags, uint64_t seed, uint64_t stage, const gtmp_rrtc_opts &o, void *workspace,
                              hipStream_t s, const uint32_t *stage_dev) {
    const RrtcPlan plan = make_rrtc_plan(p);
    char *ws = static_cast<char *>(workspace);
    const uint64_t N = p.N, M = p.M, G = p.G;
    const uint64_t E = N + (M - 1) * N * N + N * G;
    RrtcArgs A = rrtc_args(p, q0, goals, Q, C_s, C_h, C_l, flags, seed, stage, o);
    A.stage_dev = stage_dev;
    return dispatch_rrtc(arm, wdim, A, S, E, p.max_edge_len, reinterpret_cast<uint8_t *>(ws + plan.off_vfree),
                         reinterpret_cast<uint32_t *>(ws + plan.off_cand),
                         reinterpret_cast<uint32_t *>(ws + plan.off_counters), false, s);
}

hipError_t launch_rrtc_path(const gtmp_problem &p, const ArmParams *arm, const SceneParams &S, int wdim,
                            const float *q0, const float *goals, const float *Q, uint64_t edge, uint64_t seed,
                            uint64_t stage, const gtmp_rrtc_opts &o, float *path, int32_t *count, float *cost,
                            hipStream_t s) {
    RrtcArgs A = rrtc_args(p, q0, goals, Q, nullptr, nullptr, nullptr, nullptr, seed, stage, o);
    A.stats = nullptr;
    A.single = (uint32_t)edge;
    A.path = path;
    A.path_count = count;
    A.path_cost = cost;
    return dispatch_rrtc(arm, wdim, A, S, 1, p.max_edge_len, nullptr, nullptr, nullptr, true, s);
}

}  // namespace gtmp
