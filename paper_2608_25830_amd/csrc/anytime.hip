// anytime.hip -- the two iteration policies on top of one plan (Alg. 1
// anytime-gtmp and ao-gtmp; Sec. IV-C..E) and the growing-budget sampler
// (Alg. 1 expand-samples).
//
// This file is compiled without floating-point contraction: the informed
// sampler and the ranking of sample pairs are defined as FP32 computations
// with a fixed operation order (see include/gtmp.h), so that the decisions
// they take (ball rejection, box rejection, pair order) are reproducible.
#include <map>
#include <mutex>
#include <tuple>

#include "gtmp_launch.hpp"
#include "rank.hpp"
#include "surrogate.hpp"

namespace gtmp {

// Attempt cap of one uniform-half draw.  Past it (probability below
// 0.97^16384 wherever at least 3 % of the proposals are accepted, which
// holds at every bound the workloads reach) the draw is the centre of the
// hyperspheroid, a point of the set.  2 * attempt + 1 must stay below 2^16
// (the counter's block field).
constexpr int kMaxAttempts = 16384;

struct BoxArgs {
    float lo[GTMP_MAX_DOF], hi[GTMP_MAX_DOF], wd[GTMP_MAX_DOF];
};

// ------------------------------------------------------------------ informed set
// Proposal regions of the uniform half (both contain X_f(c) n box, and each
// attempt is accepted iff its point lies in X_f(c) n box, so either gives a
// uniform draw of that set): the hyperspheroid's frame box (a cube point
// kept inside the unit ball, mapped by the direct method of Gammell et al.
// 2018, kept inside the box) or its axis-aligned bounding box clipped to the
// sampling box (a point kept iff |x - q0| + |x - q_g| <= c).  The smaller
// of the two accepts more often and is used.
struct Informed {
    float centre[GTMP_MAX_DOF];
    float H[GTMP_MAX_DOF * GTMP_MAX_DOF];
    float mid[GTMP_MAX_DOF], half[GTMP_MAX_DOF];
    float q0[GTMP_MAX_DOF], qg[GTMP_MAX_DOF];
    float r1, r2, c;
    int bounded, clipped;
};

// Hyperspheroid of the informed set X_f(c) (Sec. IV-E; Gammell et al. 2018):
// centre (q0 + q_g)/2, radii c/2 along q_g - q0 and sqrt(c^2 - c_min^2)/2
// across, orientation by the Householder reflection mapping e_1 to the unit
// vector from q0 to q_g; the bounding half-extents sqrt(sum_j (H_ij r_j)^2),
// widened by 2^-10 of themselves against FP32 rounding, clipped to the box;
// the clipped box is used iff its volume is below the frame box's
// prod 2 r_i (both multiplied in coordinate order).  Without a bound
// (c = +inf or c >= penalty) the draws are uniform in the box.
__device__ __forceinline__ void informed_prep(int d, const float *q0, const float *goals, const float *c_dev,
                                              float penalty, const BoxArgs &L, Informed *out) {
    const float c = *c_dev;
    Informed I;
    I.bounded = !(__builtin_isinf(c) || c >= penalty || c != c);
    I.c = c;
    float acc = 0.0f;
    for (int i = 0; i < d; ++i) {
        const float t = goals[i] - q0[i];
        acc = acc + t * t;
        I.q0[i] = q0[i];
        I.qg[i] = goals[i];
    }
    const float cmin = __builtin_sqrtf(acc);
    for (int i = 0; i < d; ++i) I.centre[i] = (q0[i] + goals[i]) * 0.5f;
    I.r1 = c * 0.5f;
    const float sq = c * c - cmin * cmin;
    I.r2 = __builtin_sqrtf(sq > 0.0f ? sq : 0.0f) * 0.5f;
    float w[GTMP_MAX_DOF];
    float ww = 0.0f;
    for (int i = 0; i < d; ++i) {
        const float a = (goals[i] - q0[i]) / cmin;
        w[i] = (i == 0 ? 1.0f : 0.0f) - a;
        ww = ww + w[i] * w[i];
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            const float delta = i == j ? 1.0f : 0.0f;
            if (ww == 0.0f) {
                I.H[i * d + j] = delta;
            } else {
                const float s = 2.0f / ww;
                I.H[i * d + j] = delta - (s * w[i]) * w[j];
            }
        }
    float vol_r = 1.0f, vol_c = 1.0f;
    for (int i = 0; i < d; ++i) {
        float e2 = 0.0f;
        for (int j = 0; j < d; ++j) {
            const float t = I.H[i * d + j] * (j == 0 ? I.r1 : I.r2);
            e2 = e2 + t * t;
        }
        const float e = __builtin_sqrtf(e2) * 1.0009765625f;
        const float a = I.centre[i] - e, b = I.centre[i] + e;
        const float clo = a > L.lo[i] ? a : L.lo[i];
        const float chi = b < L.hi[i] ? b : L.hi[i];
        I.mid[i] = (clo + chi) * 0.5f;
        I.half[i] = (chi - clo) * 0.5f;
        vol_r = vol_r * ((i == 0 ? I.r1 : I.r2) * 2.0f);
        vol_c = vol_c * (chi - clo);
    }
    I.clipped = vol_c < vol_r ? 1 : 0;
    *out = I;
}

__global__ void k_informed_prep(int d, const float *q0, const float *goals, const float *c_dev, float penalty,
                                BoxArgs L, Informed *out) {
    if (threadIdx.x == 0) informed_prep(d, q0, goals, c_dev, penalty, L, out);
}

__device__ __forceinline__ uint4 words(uint32_t k0, uint32_t k1, uint32_t n, uint32_t m, uint32_t stage,
                                       uint32_t stream, uint32_t blk) {
    return philox4x32_10(make_uint4(n, m, stage, (stream << 16) | blk), k0, k1);
}

__device__ __forceinline__ uint32_t pick(const uint4 &w, int i) {
    return i == 0 ? w.x : i == 1 ? w.y : i == 2 ? w.z : w.w;
}

// Attempt a of the uniform-half draw for slot (m, n): true iff accepted
// (the point lies in X_f(c) and in the box), the point in x.
__device__ __forceinline__ bool informed_attempt(int d, const float *lo, const float *hi, const Informed &I,
                                                 uint32_t k0, uint32_t k1, uint32_t stage, uint32_t m, uint32_t n,
                                                 int a, float *x) {
    float y[GTMP_MAX_DOF];
    const uint4 w0 = words(k0, k1, n, m, stage, 1u, (uint32_t)(2 * a));
    const uint4 w1 = words(k0, k1, n, m, stage, 1u, (uint32_t)(2 * a + 1));
    for (int i = 0; i < d; ++i) {
        const uint32_t wi = i < 4 ? pick(w0, i) : pick(w1, i - 4);
        y[i] = (float)(wi >> 8) * (1.0f / 8388608.0f) - 1.0f;
    }
    bool inside = true;
    if (I.clipped) {
        float s0 = 0.0f, s1 = 0.0f;
        for (int i = 0; i < d; ++i) {
            x[i] = I.mid[i] + I.half[i] * y[i];
            if (!(x[i] >= lo[i] && x[i] <= hi[i])) inside = false;
            const float t0 = x[i] - I.q0[i], t1 = x[i] - I.qg[i];
            s0 = s0 + t0 * t0;
            s1 = s1 + t1 * t1;
        }
        return inside && __builtin_sqrtf(s0) + __builtin_sqrtf(s1) <= I.c;
    }
    float s2 = 0.0f;
    for (int i = 0; i < d; ++i) s2 = s2 + y[i] * y[i];
    if (!(s2 < 1.0f)) return false;
    float z[GTMP_MAX_DOF];
    for (int i = 0; i < d; ++i) z[i] = (i == 0 ? I.r1 : I.r2) * y[i];
    for (int i = 0; i < d; ++i) {
        float acc = 0.0f;
        for (int j = 0; j < d; ++j) acc = acc + I.H[i * d + j] * z[j];
        x[i] = I.centre[i] + acc;
        if (!(x[i] >= lo[i] && x[i] <= hi[i])) inside = false;
    }
    return inside;
}

// Box sample of slot (m, n): the words of attempt 0 mapped to the box.
__device__ __forceinline__ void box_draw(int d, const float *lo, const float *wd, uint32_t k0, uint32_t k1,
                                         uint32_t stage, uint32_t m, uint32_t n, float *x) {
    const uint4 w0 = words(k0, k1, n, m, stage, 1u, 0u);
    const uint4 w1 = words(k0, k1, n, m, stage, 1u, 1u);
    for (int i = 0; i < d; ++i) {
        const uint32_t wi = i < 4 ? pick(w0, i) : pick(w1, i - 4);
        x[i] = __builtin_fmaf(unit_from_word(wi), wd[i], lo[i]);
    }
}

// One draw of the uniform half for slot (m, n): the first accepted attempt.
// Returns attempts used (0 for an unbounded draw, -1 past the attempt cap,
// where x is the centre).
__device__ int informed_draw(int d, const float *lo, const float *wd, const float *hi, const Informed &I,
                             uint32_t k0, uint32_t k1, uint32_t stage, uint32_t m, uint32_t n, float *x) {
    if (I.bounded) {
        for (int a = 0; a < kMaxAttempts; ++a) {
            float xx[GTMP_MAX_DOF];
            if (!informed_attempt(d, lo, hi, I, k0, k1, stage, m, n, a, xx)) continue;
            for (int i = 0; i < d; ++i) x[i] = xx[i];
            return a + 1;
        }
        for (int i = 0; i < d; ++i) x[i] = I.centre[i];
        return -1;
    }
    box_draw(d, lo, wd, k0, k1, stage, m, n, x);
    return 0;
}

// ------------------------------------------------------------------ expansion

// Copy the old samples of every layer into the new (wider) layout.
__device__ __forceinline__ void relayout_one(uint64_t t, int n_old, int N, int d, const float *Q_old, float *Q_new) {
    const uint64_t j = t % d, mn = t / d;
    const uint64_t n = mn % n_old, m = mn / n_old;
    Q_new[(m * N + n) * d + j] = Q_old[t];
}

__global__ void k_relayout(int M, int n_old, int N, int d, const float *Q_old, float *Q_new) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (uint64_t)M * n_old * d) relayout_one(t, n_old, N, d, Q_old, Q_new);
}

// Mixture coin and heuristic rank of the new slots of one layer (Sec. III-A
// coin flip; Alg. 1 expand-samples): rank[n] = index among this layer's
// heuristic draws, -1 for a uniform-half draw.  One block.
// (wsum, carry: the block's LDS, blockDim.x / 64 words and one)
__device__ __forceinline__ void coin_rank_block(int m, int n_old, int N, uint32_t k0, uint32_t k1, uint32_t stage,
                                                const Informed *I, int heuristic_ok, int32_t *rank, int *wsum,
                                                int &carry) {
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const bool allow = heuristic_ok && I->bounded;
    for (int base = n_old; base < N; base += blockDim.x) {
        const int n = base + threadIdx.x;
        bool heur = false;
        if (n < N && allow) {
            const uint4 w = words(k0, k1, (uint32_t)n, (uint32_t)m, stage, 2u, 0u);
            heur = (w.x >> 31) != 0;
        }
        const uint64_t mask = ballot(heur);
        const int wv = threadIdx.x / kWave;
        if (lane_id() == 0) wsum[wv] = __popcll(mask);
        __syncthreads();
        int before = carry;
        for (int k = 0; k < wv; ++k) before += wsum[k];
        if (n < N) rank[n] = heur ? before + rank_in(mask) : -1;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int k = 0; k < (int)(blockDim.x / kWave); ++k) tot += wsum[k];
            carry += tot;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(1024) k_coin_rank(int m, int n_old, int N, uint32_t k0, uint32_t k1, uint32_t stage,
                                                    const Informed *I, int heuristic_ok, int32_t *rank) {
    __shared__ int wsum[1024 / kWave];
    __shared__ int carry;
    coin_rank_block(m, n_old, N, k0, k1, stage, I, heuristic_ok, rank, wsum, carry);
}

// Fill the new slots of layer m, one wave per slot (four per block): a
// heuristic slot of rank h takes the midpoint of the h-th closest pair (a
// uniform draw when fewer pairs exist), every other slot a draw of the
// uniform half.  The draw's attempts are tested 64 at a time, one per lane,
// and the lowest accepted attempt index wins (the first set bit of the
// wave's ballot), so the result is the sequential first accepted attempt;
// the proposal of the uniform half accepts at least a few per cent of its
// attempts, so a slot nearly always needs one round.  With the surrogate
// bias the pair list is the compacted list of candidates predicted free and
// its length is read from n_avail.
constexpr int kExpandThreads = 256;
constexpr int kExpandSlots = kExpandThreads / kWave;  // slots per block
static_assert(kMaxAttempts % kWave == 0, "whole rounds of attempts");

// Slot n of layer m, by one wave.
__device__ __forceinline__ void fill_slot(int m, int n, int d, const BoxArgs &B, uint32_t k0, uint32_t k1,
                                          uint32_t stage, const Informed *Ip, const int32_t *rank,
                                          const uint32_t *sorted_pairs, uint64_t n_pairs, const uint32_t *n_avail,
                                          int nv, const float *U, const float *Vv, float *Qm) {
    const int lane = lane_id();
    const Informed I = *Ip;
    const int h = rank[n];
    const uint64_t avail = n_avail ? (uint64_t)*n_avail : n_pairs;
    if (h >= 0 && (uint64_t)h < avail) {
        if (lane == 0) {
            const uint32_t p = sorted_pairs[h];
            const uint32_t a = p / (uint32_t)nv, b = p % (uint32_t)nv;
            for (int i = 0; i < d; ++i) Qm[(size_t)n * d + i] = (U[(size_t)a * d + i] + Vv[(size_t)b * d + i]) * 0.5f;
        }
        return;
    }
    if (I.bounded) {
        for (int base = 0; base < kMaxAttempts; base += kWave) {
            const int att = base + lane;
            float x[GTMP_MAX_DOF];
            const bool ok = informed_attempt(d, B.lo, B.hi, I, k0, k1, stage, (uint32_t)m, (uint32_t)n, att, x);
            const uint64_t acc = ballot(ok);
            if (acc != 0) {  // wave-uniform
                if (lane == __builtin_ctzll(acc))
                    for (int i = 0; i < d; ++i) Qm[(size_t)n * d + i] = x[i];
                return;
            }
        }
    }
    if (lane == 0) {
        float x[GTMP_MAX_DOF];
        if (I.bounded) {  // past the attempt cap: the centre, a point of the set
            for (int i = 0; i < d; ++i) x[i] = I.centre[i];
        } else {
            box_draw(d, B.lo, B.wd, k0, k1, stage, (uint32_t)m, (uint32_t)n, x);
        }
        for (int i = 0; i < d; ++i) Qm[(size_t)n * d + i] = x[i];
    }
}

__global__ void __launch_bounds__(kExpandThreads) k_expand_layer(int m, int n_old, int N, int d, BoxArgs B, uint32_t k0,
                                                                 uint32_t k1, uint32_t stage, const Informed *Ip,
                                                                 const int32_t *rank, const uint32_t *sorted_pairs,
                                                                 uint64_t n_pairs, const uint32_t *n_avail, int nv,
                                                                 const float *U, const float *Vv, float *Qm) {
    const int n = n_old + (int)blockIdx.x * kExpandSlots + (int)(threadIdx.x / kWave);  // wave-uniform
    if (n < N) fill_slot(m, n, d, B, k0, k1, stage, Ip, rank, sorted_pairs, n_pairs, n_avail, nv, U, Vv, Qm);
}

// Surrogate bias of the heuristic half: midpoints of the K closest pairs
// (the same FP32 expression as the expansion), scored by the surrogate, and
// the pairs whose logit is at most tau compacted in rank order.
__global__ void __launch_bounds__(256) k_bias_midpoints(int d, uint64_t K, const uint32_t *sorted_pairs, int nv,
                                                        const float *U, const float *Vv, float *X) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= K) return;
    const uint32_t p = sorted_pairs[c];
    const uint32_t a = p / (uint32_t)nv, b = p % (uint32_t)nv;
    for (int i = 0; i < d; ++i) X[c * d + i] = (U[(size_t)a * d + i] + Vv[(size_t)b * d + i]) * 0.5f;
}

__global__ void __launch_bounds__(1024) k_bias_compact(uint64_t K, const float *z, float tau,
                                                       const uint32_t *sorted_pairs, uint32_t *free_pairs,
                                                       uint32_t *count) {
    __shared__ uint32_t wsum[1024 / kWave];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint64_t base = 0; base < K; base += blockDim.x) {
        const uint64_t c = base + threadIdx.x;
        const bool keep = c < K && z[c] <= tau;
        const uint64_t mask = ballot(keep);
        const int wv = threadIdx.x / kWave;
        if (lane_id() == 0) wsum[wv] = (uint32_t)__popcll(mask);
        __syncthreads();
        uint32_t before = carry;
        for (int k = 0; k < wv; ++k) before += wsum[k];
        if (keep) free_pairs[before + rank_in(mask)] = sorted_pairs[c];
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int k = 0; k < (int)(blockDim.x / kWave); ++k) tot += wsum[k];
            carry += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = carry;
}

// Standalone informed draws (for tests of the sampler): X[n][d] for slots
// (m, n), n = 0..count-1, attempts[n] as informed_draw returns it.
__global__ void k_informed_batch(int d, BoxArgs B, uint32_t k0, uint32_t k1, uint32_t stage, uint32_t m, int count,
                                 const Informed *Ip, float *X, int32_t *attempts) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= count) return;
    const Informed I = *Ip;
    float x[GTMP_MAX_DOF];
    const int a = informed_draw(d, B.lo, B.wd, B.hi, I, k0, k1, stage, m, (uint32_t)n, x);
    for (int i = 0; i < d; ++i) X[(size_t)n * d + i] = x[i];
    if (attempts) attempts[n] = a;
}

static BoxArgs box_args(const gtmp_problem &p) {
    BoxArgs B{};
    for (int j = 0; j < p.d; ++j) {
        B.lo[j] = p.lo[j];
        B.hi[j] = p.hi[j];
        B.wd[j] = p.hi[j] - p.lo[j];
    }
    return B;
}

// ------------------------------------------------------------------ workspace of the expansion
static size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

ExpandPlan make_expand_plan(const gtmp_problem &p, bool bias) {
    ExpandPlan e{};
    const uint64_t Nn = (uint64_t)p.N;
    // at most N - n_old <= N heuristic slots per layer: the N closest pairs
    // (4 N candidates with the surrogate bias)
    e.max_k = (uint32_t)((bias ? (uint64_t)kBiasCandidates : 1ull) * Nn);
    size_t o = 0;
    e.off_informed = o; o = up256(o + sizeof(Informed));
    e.off_rank = o; o = up256(o + sizeof(int32_t) * Nn);
    e.off_sorted = o; o = up256(o + sizeof(uint32_t) * e.max_k);
    const RankPlan rp = make_rank_plan(e.max_k);
    e.off_rankws = o; o = up256(o + rp.total);
    if (bias) {
        const uint64_t K = (uint64_t)kBiasCandidates * Nn;
        e.bias_rows = K;
        e.off_bX = o; o = up256(o + sizeof(float) * K * p.d);
        e.off_bz = o; o = up256(o + sizeof(float) * K);
        e.off_bfree = o; o = up256(o + sizeof(uint32_t) * K);
        e.off_bcount = o; o = up256(o + 64);
        e.bws_bytes = sur_infer_bytes((int64_t)((K + 255) / 256 * 256));
        e.off_bws = o; o = up256(o + e.bws_bytes);
    }
    e.total = o;
    return e;
}

hipError_t launch_expand(const gtmp_problem &p, const float *q0, const float *goals, const float *Q_old, int n_old,
                         float *Q_new, const float *c_dev, uint64_t seed, uint64_t stage, void *workspace,
                         hipStream_t s, const SurNet *bias, float bias_tau) {
    const ExpandPlan e = make_expand_plan(p, bias != nullptr);
    const RankPlan rp = make_rank_plan(e.max_k);
    char *ws = static_cast<char *>(workspace);
    Informed *I = reinterpret_cast<Informed *>(ws + e.off_informed);
    int32_t *rank = reinterpret_cast<int32_t *>(ws + e.off_rank);
    uint32_t *sorted_pairs = reinterpret_cast<uint32_t *>(ws + e.off_sorted);
    const int M = p.M, N = p.N, d = p.d;
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32), st = (uint32_t)stage;
    hipLaunchKernelGGL(k_informed_prep, dim3(1), dim3(64), 0, s, d, q0, goals, c_dev, p.penalty, box_args(p), I);
    if (n_old > 0) {
        const uint64_t total = (uint64_t)M * n_old * d;
        hipLaunchKernelGGL(k_relayout, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, M, n_old, N, d, Q_old,
                           Q_new);
    }
    if (n_old >= N) return hipGetLastError();
    const BoxArgs B = box_args(p);
    for (int m = 0; m < M; ++m) {
        // neighbours as Alg. 1 sees them when it reaches layer m: layer m-1
        // already expanded (q0 for m = 0), layer m+1 still at its old size
        // (the goals for m = M-1)
        const float *U = m == 0 ? q0 : Q_new + (size_t)(m - 1) * N * d;
        const int nu = m == 0 ? 1 : N;
        const float *Vv = m == M - 1 ? goals : Q_new + (size_t)(m + 1) * N * d;
        const int nv = m == M - 1 ? p.G : n_old;
        const uint64_t npairs = (uint64_t)nu * (uint64_t)nv;
        const int heuristic_ok = npairs > 0;
        hipLaunchKernelGGL(k_coin_rank, dim3(1), dim3(1024), 0, s, m, n_old, N, k0, k1, st, I, heuristic_ok, rank);
        // the closest pairs in rank order: as many as there are new slots (a
        // heuristic rank never reaches past them), or the bias candidates
        const uint64_t cap = (uint64_t)(bias ? kBiasCandidates : 1) * (uint64_t)(N - n_old);
        const uint64_t K = npairs < cap ? npairs : cap;
        const uint32_t *sorted = sorted_pairs;
        if (heuristic_ok) {
            hipError_t err = launch_rank_pairs(d, nu, U, nv, Vv, (uint32_t)K, sorted_pairs, rp, ws + e.off_rankws, s);
            if (err != hipSuccess) return err;
        }
        const uint32_t *n_avail = nullptr;
        if (heuristic_ok && bias) {
            float *bX = reinterpret_cast<float *>(ws + e.off_bX);
            float *bz = reinterpret_cast<float *>(ws + e.off_bz);
            uint32_t *bfree = reinterpret_cast<uint32_t *>(ws + e.off_bfree);
            uint32_t *bcount = reinterpret_cast<uint32_t *>(ws + e.off_bcount);
            hipLaunchKernelGGL(k_bias_midpoints, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, d, K, sorted, nv, U,
                               Vv, bX);
            hipError_t err = launch_sur_infer(*bias, (int64_t)K, bX, bz, ws + e.off_bws, e.bws_bytes, s);
            if (err != hipSuccess) return err;
            hipLaunchKernelGGL(k_bias_compact, dim3(1), dim3(1024), 0, s, K, bz, bias_tau, sorted, bfree, bcount);
            sorted = bfree;
            n_avail = bcount;
        }
        const unsigned blocks = (unsigned)((N - n_old + kExpandSlots - 1) / kExpandSlots);
        hipLaunchKernelGGL(k_expand_layer, dim3(blocks), dim3(kExpandThreads), 0, s, m, n_old, N, d, B, k0, k1, st, I,
                           rank, sorted, heuristic_ok ? K : 0, n_avail, nv, U, Vv, Q_new + (size_t)m * N * d);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ expansions of several plans
// Layer m's neighbour sets of a job, as launch_expand forms them.
struct LayerPairs {
    const float *U, *V;
    int nu, nv;
    uint64_t npairs, K;
};

__host__ __device__ inline LayerPairs layer_pairs(const ExpandJob &J, int m) {
    LayerPairs L;
    L.U = m == 0 ? J.q0 : J.Q_new + (size_t)(m - 1) * J.N * J.d;
    L.nu = m == 0 ? 1 : J.N;
    L.V = m == J.M - 1 ? J.goals : J.Q_new + (size_t)(m + 1) * J.N * J.d;
    L.nv = m == J.M - 1 ? J.G : J.n_old;
    L.npairs = (uint64_t)L.nu * (uint64_t)L.nv;
    const uint64_t cap = (uint64_t)(J.N - J.n_old);
    L.K = L.npairs < cap ? L.npairs : cap;
    return L;
}

__device__ __forceinline__ BoxArgs job_box(const ExpandJob &J) {
    BoxArgs B{};
    for (int j = 0; j < J.d; ++j) {
        B.lo[j] = J.lo[j];
        B.hi[j] = J.hi[j];
        B.wd[j] = J.hi[j] - J.lo[j];
    }
    return B;
}

__device__ __forceinline__ bool job_active(const ExpandJob &J, int m) { return m < J.M && J.n_old < J.N; }

__global__ void k_bx_prep(const ExpandJob *jobs) {
    const ExpandJob &J = jobs[blockIdx.x];
    if (threadIdx.x == 0)
        informed_prep(J.d, J.q0, J.goals, J.c_dev, J.penalty, job_box(J), static_cast<Informed *>(J.informed));
}

__global__ void __launch_bounds__(256) k_bx_relayout(const ExpandJob *jobs) {
    const ExpandJob &J = jobs[blockIdx.y];
    const uint64_t total = (uint64_t)J.M * J.n_old * J.d;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x)
        relayout_one(t, J.n_old, J.N, J.d, J.Q_old, J.Q_new);
}

__global__ void __launch_bounds__(1024) k_bx_coin(const ExpandJob *jobs, int m) {
    __shared__ int wsum[1024 / kWave];
    __shared__ int carry;
    const ExpandJob &J = jobs[blockIdx.x];
    if (!job_active(J, m)) return;
    const int heuristic_ok = layer_pairs(J, m).npairs > 0;
    coin_rank_block(m, J.n_old, J.N, J.k0, J.k1, J.stage, static_cast<const Informed *>(J.informed), heuristic_ok,
                    J.rank, wsum, carry);
}

__device__ __forceinline__ bool job_ranks_small(const ExpandJob &J, int m, LayerPairs &L) {
    if (!job_active(J, m)) return false;
    L = layer_pairs(J, m);
    return L.npairs > 0 && L.npairs <= (uint64_t)rank::kRankSortCap;
}

__device__ __forceinline__ bool job_ranks_large(const ExpandJob &J, int m, LayerPairs &L) {
    if (!job_active(J, m)) return false;
    L = layer_pairs(J, m);
    return L.npairs > (uint64_t)rank::kRankSortCap;
}

__global__ void __launch_bounds__(rank::kRankSortThreads) k_bx_rank_small(const ExpandJob *jobs, int m) {
    __shared__ uint64_t lds[rank::kRankSortCap];
    const ExpandJob &J = jobs[blockIdx.x];
    LayerPairs L;
    if (!job_ranks_small(J, m, L)) return;
    rank::rank_small_block(J.d, L.U, L.nv, L.V, (uint32_t)L.npairs, (uint32_t)L.K, J.sorted, lds);
}

__global__ void __launch_bounds__(256) k_bx_rank_init(const ExpandJob *jobs, int m) {
    const ExpandJob &J = jobs[blockIdx.x];
    LayerPairs L;
    if (!job_ranks_large(J, m, L)) return;
    rank::rank_init_block((uint32_t)L.K, reinterpret_cast<uint32_t *>(J.rankws + J.rank_off_hist),
                          reinterpret_cast<rank::RankState *>(J.rankws));
}

// The jobs whose layer pairs at one layer take the radix selection, listed
// by the host (which holds the same job table) as a kernel argument, so that
// the selection's grids have rows for those jobs only instead of for every
// job of the stage; a captured launch keeps its own copy of the list.
constexpr int kMaxListedJobs = 1024;
struct JobList {
    uint32_t all;                 // 1: every job, grid row y is job y
    uint16_t id[kMaxListedJobs];  // else grid row y is job id[y]
};
__device__ __forceinline__ uint32_t listed_job(const JobList &sel) { return sel.all ? blockIdx.y : sel.id[blockIdx.y]; }

__global__ void __launch_bounds__(256) k_bx_rank_pass(const ExpandJob *jobs, const JobList sel, int m, int pass) {
    __shared__ uint32_t h[rank::kRankBins];
    __shared__ uint32_t part[256];
    __shared__ bool last;
    const ExpandJob &J = jobs[listed_job(sel)];
    LayerPairs L;
    if (!job_ranks_large(J, m, L)) return;  // every block of the job returns alike
    rank::rank_pass_block(pass, J.d, L.U, L.nv, L.V, (uint32_t)L.npairs, (uint32_t)L.K,
                          reinterpret_cast<uint32_t *>(J.rankws + J.rank_off_hist),
                          reinterpret_cast<rank::RankState *>(J.rankws), blockIdx.x, gridDim.x, h, part, last);
}

__global__ void __launch_bounds__(256) k_bx_rank_compact(const ExpandJob *jobs, const JobList sel, int m) {
    const ExpandJob &J = jobs[listed_job(sel)];
    LayerPairs L;
    if (!job_ranks_large(J, m, L)) return;
    rank::rank_compact_block(J.d, L.U, L.nv, L.V, (uint32_t)L.npairs, reinterpret_cast<rank::RankState *>(J.rankws),
                             reinterpret_cast<uint64_t *>(J.rankws + J.rank_off_cand), J.rank_cap, blockIdx.x,
                             gridDim.x);
}

__global__ void __launch_bounds__(rank::kRankSortThreads) k_bx_rank_sort(const ExpandJob *jobs, int m) {
    __shared__ uint64_t lds[rank::kRankSortCap];
    const ExpandJob &J = jobs[blockIdx.x];
    LayerPairs L;
    if (!job_ranks_large(J, m, L)) return;
    rank::rank_sort_block((uint32_t)L.K, reinterpret_cast<const rank::RankState *>(J.rankws),
                          reinterpret_cast<uint64_t *>(J.rankws + J.rank_off_cand), J.rank_cap, J.sorted, lds);
}

__global__ void __launch_bounds__(kExpandThreads) k_bx_fill(const ExpandJob *jobs, int m) {
    const ExpandJob &J = jobs[blockIdx.y];
    if (!job_active(J, m)) return;
    const int n = J.n_old + (int)blockIdx.x * kExpandSlots + (int)(threadIdx.x / kWave);  // wave-uniform
    if (n >= J.N) return;
    const LayerPairs L = layer_pairs(J, m);
    fill_slot(m, n, J.d, job_box(J), J.k0, J.k1, J.stage, static_cast<const Informed *>(J.informed), J.rank, J.sorted,
              L.npairs > 0 ? L.K : 0, nullptr, L.nv, L.U, L.V, J.Q_new + (size_t)m * J.N * J.d);
}

void fill_expand_job(ExpandJob &J, const gtmp_problem &p, const float *q0, const float *goals, const float *Q_old,
                     int n_old, float *Q_new, const float *c_dev, uint64_t seed, uint64_t stage, void *workspace) {
    const ExpandPlan e = make_expand_plan(p, false);
    const RankPlan rp = make_rank_plan(e.max_k);
    char *ws = static_cast<char *>(workspace);
    J = ExpandJob{};
    J.d = p.d; J.M = p.M; J.N = p.N; J.G = p.G; J.n_old = n_old;
    J.penalty = p.penalty;
    for (int j = 0; j < p.d; ++j) {
        J.lo[j] = p.lo[j];
        J.hi[j] = p.hi[j];
    }
    J.k0 = (uint32_t)(seed & 0xffffffffu);
    J.k1 = (uint32_t)(seed >> 32);
    J.stage = (uint32_t)stage;
    J.q0 = q0; J.goals = goals; J.Q_old = Q_old; J.Q_new = Q_new; J.c_dev = c_dev;
    J.informed = ws + e.off_informed;
    J.rank = reinterpret_cast<int32_t *>(ws + e.off_rank);
    J.sorted = reinterpret_cast<uint32_t *>(ws + e.off_sorted);
    J.rankws = ws + e.off_rankws;
    J.rank_cap = rp.cap;
    J.rank_off_hist = (uint32_t)rp.off_hist;
    J.rank_off_cand = (uint32_t)rp.off_cand;
}

hipError_t launch_expand_jobs(const ExpandJob *jobs_dev, const std::vector<ExpandJob> &jobs, hipStream_t s) {
    const unsigned nj = (unsigned)jobs.size();
    if (nj == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bx_prep, dim3(nj), dim3(64), 0, s, jobs_dev);
    uint64_t most = 0;
    int maxM = 0;
    for (const ExpandJob &J : jobs) {
        most = std::max(most, (uint64_t)J.M * J.n_old * J.d);
        maxM = std::max(maxM, J.M);
    }
    if (most > 0)
        hipLaunchKernelGGL(k_bx_relayout, dim3((unsigned)std::min<uint64_t>((most + 255) / 256, 4096), nj), dim3(256), 0,
                           s, jobs_dev);
    JobList sel{};
    for (int m = 0; m < maxM; ++m) {
        bool any_small = false;
        uint64_t large = 0;
        int slots = 0;
        uint32_t n_large = 0;
        for (unsigned j = 0; j < nj; ++j) {
            const ExpandJob &J = jobs[j];
            if (m >= J.M || J.n_old >= J.N) continue;  // the device's job_active
            const LayerPairs L = layer_pairs(J, m);
            if (L.npairs > 0 && L.npairs <= (uint64_t)rank::kRankSortCap) any_small = true;
            if (L.npairs > (uint64_t)rank::kRankSortCap) {  // the device's job_ranks_large
                large = std::max(large, L.npairs);
                if (n_large < (uint32_t)kMaxListedJobs) sel.id[n_large] = (uint16_t)j;
                ++n_large;
            }
            slots = std::max(slots, J.N - J.n_old);
        }
        // more listed jobs than the list holds: rows for every job (the
        // others return at once, as every job's blocks do once its
        // selection is done)
        sel.all = n_large > (uint32_t)kMaxListedJobs || nj > 65536u ? 1u : 0u;
        const unsigned rows = sel.all ? nj : n_large;
        if (slots == 0) continue;
        hipLaunchKernelGGL(k_bx_coin, dim3(nj), dim3(1024), 0, s, jobs_dev, m);
        if (any_small) hipLaunchKernelGGL(k_bx_rank_small, dim3(nj), dim3(rank::kRankSortThreads), 0, s, jobs_dev, m);
        if (large > 0) {
            const unsigned bx = (unsigned)std::min<uint64_t>((large + 1023) / 1024, 1024);
            hipLaunchKernelGGL(k_bx_rank_init, dim3(nj), dim3(256), 0, s, jobs_dev, m);
            for (int pass = 0; pass < rank::kRankPasses; ++pass)
                hipLaunchKernelGGL(k_bx_rank_pass, dim3(bx, rows), dim3(256), 0, s, jobs_dev, sel, m, pass);
            hipLaunchKernelGGL(k_bx_rank_compact, dim3(bx, rows), dim3(256), 0, s, jobs_dev, sel, m);
            hipLaunchKernelGGL(k_bx_rank_sort, dim3(nj), dim3(rank::kRankSortThreads), 0, s, jobs_dev, m);
        }
        hipLaunchKernelGGL(k_bx_fill, dim3((unsigned)((slots + kExpandSlots - 1) / kExpandSlots), nj),
                           dim3(kExpandThreads), 0, s, jobs_dev, m);
    }
    return hipGetLastError();
}

hipError_t launch_informed_batch(const gtmp_problem &p, const float *q0, const float *goals, const float *c_dev,
                                 uint64_t seed, uint64_t stage, uint32_t m, int count, float *X, int32_t *attempts,
                                 void *workspace, hipStream_t s) {
    Informed *I = reinterpret_cast<Informed *>(workspace);
    hipLaunchKernelGGL(k_informed_prep, dim3(1), dim3(64), 0, s, p.d, q0, goals, c_dev, p.penalty, box_args(p), I);
    if (count > 0)
        hipLaunchKernelGGL(k_informed_batch, dim3((count + 255) / 256), dim3(256), 0, s, p.d, box_args(p),
                           (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), (uint32_t)stage, m, count, I, X,
                           attempts);
    return hipGetLastError();
}

// ------------------------------------------------------------------ one stage of a plan
// Uniform layer samples with the stage number read from device memory
// (stage = base + *counter), so that a captured stage can be replayed.
__global__ void __launch_bounds__(256) k_sample_dev_stage(int M, int N, int d, uint32_t k0, uint32_t k1,
                                                          const uint32_t *counter, uint32_t base, BoxArgs B,
                                                          float *__restrict__ Q) {
    const int nblk = (d + 3) >> 2;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (uint64_t)M * N * nblk) return;
    const uint32_t stage = base + *counter;
    const uint32_t blk = (uint32_t)(tid % nblk);
    const uint64_t mn = tid / nblk;
    const uint32_t n = (uint32_t)(mn % N), m = (uint32_t)(mn / N);
    const uint4 w = philox4x32_10(make_uint4(n, m, stage, blk), k0, k1);
    float *dst = Q + mn * d;
    for (int i = 0; i < 4; ++i) {
        const int j = (int)blk * 4 + i;
        if (j < d) dst[j] = __builtin_fmaf(unit_from_word(pick(w, i)), B.wd[j], B.lo[j]);
    }
}

// Archive update of the anytime policies with |K| = 1 (Alg. 1; Sec. IV-D):
// the best path so far; strictly better costs replace it, so ties keep the
// earlier stage.  Also records the stage's cost and advances the counter.
// Archive update of the single-class anytime loops.  Without shortcutting
// (s_cost == NULL) the stage path replaces the archived one iff its cost is
// strictly lower.  With shortcutting the compared cost is the stage path's
// (cmp_short == 0, the restart loop) or its shortcut's (cmp_short == 1, the
// growing loop), and what is stored is the shortcut, if one exists.
__global__ void k_archive(int M, int N, int d, const float *cost, const int32_t *idx, const float *wp,
                          const float *s_cost, const float *s_wp, int cmp_short, float *best_cost, int32_t *best_idx,
                          float *best_wp, int32_t *best_meta, float *stage_costs, uint32_t *counter, int max_stages) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t stage = *counter;
    const float c = s_cost && cmp_short ? *s_cost : *cost;
    if ((int)stage < max_stages) stage_costs[stage] = c;
    const bool store = c < *best_cost && (!s_cost || *s_cost < __builtin_inff());
    if (store) {
        *best_cost = s_cost ? *s_cost : c;
        const float *src = s_cost ? s_wp : wp;
        for (int m = 0; m <= M; ++m) best_idx[m] = idx[m];
        for (int k = 0; k < (M + 2) * d; ++k) best_wp[k] = src[k];
        best_meta[0] = (int32_t)stage;
        best_meta[1] = M;
        best_meta[2] = N;
    }
    best_meta[3] = (int32_t)stage + 1;
    *counter = stage + 1;
}

__global__ void k_anytime_init(float *best_cost, int32_t *best_meta, uint32_t *counter) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    *best_cost = __builtin_inff();
    best_meta[0] = -1;
    best_meta[1] = 0;
    best_meta[2] = 0;
    best_meta[3] = 0;
    *counter = 0;
}

// ------------------------------------------------------------------ drivers
// Buffers of one path's shortcutting (at most K waypoints): the shortcut
// table, then its length and kept count, the kept indices and waypoints.
namespace {
struct SimpCarve {
    uint8_t *valid;
    float *cost;
    int32_t *count, *idx;
    float *wp;
};
size_t simp_bytes(int K, int d) { return up256((size_t)K * K) + 256 + sizeof(int32_t) * K + sizeof(float) * K * d; }
SimpCarve simp_carve(char *base, int K, int d) {
    const size_t o = up256((size_t)K * K);
    return SimpCarve{reinterpret_cast<uint8_t *>(base), reinterpret_cast<float *>(base + o),
                     reinterpret_cast<int32_t *>(base + o + 4), reinterpret_cast<int32_t *>(base + o + 256),
                     reinterpret_cast<float *>(base + o + 256 + sizeof(int32_t) * K)};
}
}  // namespace

AnytimePlan make_anytime_plan(const gtmp_problem &p, const gtmp_anytime_opts &o) {
    AnytimePlan a{};
    gtmp_problem big = p;
    if (o.mode == GTMP_ANYTIME_GROWING) {
        big.M = o.M_max;
        big.N = o.N_max;
    }
    a.big = big;
    const uint64_t M = big.M, N = big.N, d = big.d, G = big.G;
    size_t off = 0;
    a.off_Q = off; off = up256(off + sizeof(float) * M * N * d);
    a.off_Q2 = off; off = up256(off + sizeof(float) * M * N * d);
    a.off_Cs = off; off = up256(off + sizeof(float) * N);
    a.off_Ch = off; off = up256(off + sizeof(float) * (M > 1 ? M - 1 : 1) * N * N);
    a.off_Cl = off; off = up256(off + sizeof(float) * N * G);
    a.off_V = off; off = up256(off + sizeof(float) * M * N);
    a.off_A = off; off = up256(off + sizeof(int32_t) * M * N);
    a.off_small = off; off = up256(off + 256 + sizeof(int32_t) * (M + 1) + sizeof(float) * (M + 2) * d);
    a.off_counter = off; off = up256(off + 64);
    if (o.simplify) {
        a.off_simp = off; off = up256(off + simp_bytes((int)M + 2, (int)d));
    }
    if (o.lp) {  // edge flags and the RRT-Connect repair's buffers
        a.off_flags = off; off = up256(off + N + (M > 1 ? M - 1 : 0) * N * N + N * G);
        a.off_rrtc = off; off = up256(off + make_rrtc_plan(big).total);
    }
    const EdgePlan ep = make_edge_plan(big);
    a.off_edge = off; off = up256(off + ep.total);
    if (o.mode == GTMP_ANYTIME_GROWING) {
        const ExpandPlan xp = make_expand_plan(big, o.bias_net != nullptr);
        a.off_expand = off; off = up256(off + xp.total);
    }
    a.total = off;
    return a;
}

namespace {
struct GraphKey {
    std::tuple<const void *, const void *, const void *, const void *, uint64_t, int, int, int, int, int, hipStream_t>
        k;
    bool operator<(const GraphKey &o) const { return k < o.k; }
};
std::mutex g_graph_mu;
std::map<GraphKey, hipGraphExec_t> g_graphs;  // kept for the life of the process
}  // namespace

hipError_t launch_anytime(const gtmp_problem &p, const ArmParams *arm, const SceneParams &scene, int wdim,
                          const float *q0, const float *goals, uint64_t seed, const gtmp_anytime_opts &o,
                          const gtmp_edge_opts &eo_in, const AnytimeOut &out, void *workspace, hipStream_t s,
                          const SurNet *bias) {
    const AnytimePlan a = make_anytime_plan(p, o);
    char *ws = static_cast<char *>(workspace);
    float *Q = reinterpret_cast<float *>(ws + a.off_Q);
    float *Q2 = reinterpret_cast<float *>(ws + a.off_Q2);
    float *Cs = reinterpret_cast<float *>(ws + a.off_Cs);
    float *Ch = reinterpret_cast<float *>(ws + a.off_Ch);
    float *Cl = reinterpret_cast<float *>(ws + a.off_Cl);
    float *V = reinterpret_cast<float *>(ws + a.off_V);
    int32_t *A = reinterpret_cast<int32_t *>(ws + a.off_A);
    char *small = ws + a.off_small;
    float *Vs = reinterpret_cast<float *>(small);
    int32_t *as = reinterpret_cast<int32_t *>(small + 4);
    float *cost = reinterpret_cast<float *>(small + 8);
    int32_t *idx = reinterpret_cast<int32_t *>(small + 256);
    float *wp = reinterpret_cast<float *>(small + 256 + sizeof(int32_t) * (a.big.M + 1));
    uint32_t *counter = reinterpret_cast<uint32_t *>(ws + a.off_counter);
    void *edge_ws = ws + a.off_edge;
    gtmp_edge_opts eo = eo_in;
    eo.ev_begin = nullptr;
    eo.ev_end = nullptr;
    const int d = p.d;
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);

    hipLaunchKernelGGL(k_anytime_init, dim3(1), dim3(64), 0, s, out.best_cost, out.best_meta, counter);

    auto one_plan = [&](const gtmp_problem &pp, const float *Qp, hipStream_t st) -> hipError_t {
        const EdgePlan ep = make_edge_plan(pp);
        uint8_t *flags = o.lp ? reinterpret_cast<uint8_t *>(ws + a.off_flags) : nullptr;
        EdgeBuffers b{q0, goals, Qp, Cs, Ch, Cl, nullptr, flags, nullptr, edge_ws};
        hipError_t e = launch_edge_check(ep, arm, scene, wdim, b, eo, st);
        if (e != hipSuccess) return e;
        if (o.lp) {  // the stage index is the device counter's value during the stage
            e = launch_rrtc_repair(pp, arm, scene, wdim, q0, goals, Qp, Cs, Ch, Cl, flags, seed, 0, *o.lp,
                                   ws + a.off_rrtc, st, counter);
            if (e != hipSuccess) return e;
        }
        e = launch_minplus(pp.M, pp.N, pp.G, Cs, Ch, Cl, nullptr, V, A, Vs, as, st);
        if (e != hipSuccess) return e;
        e = launch_extract(pp.M, pp.N, pp.G, d, as, A, Vs, Qp, q0, goals, idx, wp, cost, st);
        if (e != hipSuccess) return e;
        const float *sc = nullptr, *swp = nullptr;
        if (o.simplify) {
            const SimpCarve c = simp_carve(ws + a.off_simp, a.big.M + 2, d);
            e = launch_simplify(arm, scene, wdim, d, 1, pp.M + 2, pp.H, wp, c.valid, c.idx, c.count, c.cost, c.wp, st);
            if (e != hipSuccess) return e;
            sc = c.cost;
            swp = c.wp;
        }
        hipLaunchKernelGGL(k_archive, dim3(1), dim3(64), 0, st, pp.M, pp.N, d, cost, idx, wp, sc, swp,
                           o.mode == GTMP_ANYTIME_GROWING ? 1 : 0, out.best_cost, out.best_idx, out.best_wp,
                           out.best_meta, out.stage_costs, counter, o.max_stages);
        return hipGetLastError();
    };

    if (o.mode == GTMP_ANYTIME_RESTART) {
        const BoxArgs B = box_args(p);
        const uint64_t total = (uint64_t)p.M * p.N * ((d + 3) / 4);
        const unsigned sblocks = (unsigned)((total + 255) / 256);
        auto stage_ops = [&](hipStream_t st) -> hipError_t {
            hipLaunchKernelGGL(k_sample_dev_stage, dim3(sblocks), dim3(256), 0, st, p.M, p.N, d, k0, k1, counter, 0u, B,
                               Q);
            return one_plan(p, Q, st);
        };
        if (!o.use_graph || o.lp) {
            for (int r = 0; r < o.max_stages; ++r) {
                hipError_t e = stage_ops(s);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }
        // one stage captured on a private stream, instantiated once per
        // (buffers, sizes, stream) and replayed max_stages times on `s`
        GraphKey key{std::make_tuple((const void *)workspace, (const void *)q0, (const void *)goals,
                                     (const void *)out.best_cost, seed, p.M, p.N, p.H, (int)eo.mode,
                                     eo.sphere_chunks * 16 + eo.states_per_iter + (o.simplify ? 1 << 16 : 0), s)};
        hipGraphExec_t exec = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_graph_mu);
            auto it = g_graphs.find(key);
            if (it != g_graphs.end()) exec = it->second;
        }
        if (!exec) {
            hipStream_t cs;
            hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
            if (e != hipSuccess) return e;
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) { (void)hipStreamDestroy(cs); return e; }
            hipError_t e_ops = stage_ops(cs);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(cs, &g);
            (void)hipStreamDestroy(cs);
            if (e_ops != hipSuccess) { if (g) (void)hipGraphDestroy(g); return e_ops; }
            if (e != hipSuccess) return e;
            e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return e;
            std::lock_guard<std::mutex> lk(g_graph_mu);
            g_graphs[key] = exec;
        }
        for (int r = 0; r < o.max_stages; ++r) {
            hipError_t e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }

    // growing budget (Alg. 1 ao-gtmp): the schedule is fixed, so the whole
    // loop is enqueued without reading anything back.
    int M = o.M_min, N = o.N_min, n_old = 0;
    float *cur = Q, *nxt = Q2;
    void *xws = ws + a.off_expand;
    for (int stage = 0; stage < o.max_stages; ++stage) {
        gtmp_problem pp = p;
        pp.M = M;
        pp.N = N;
        hipError_t e = launch_expand(pp, q0, goals, cur, n_old, nxt, out.best_cost, seed, (uint64_t)stage, xws, s,
                                     bias, o.bias_tau);
        if (e != hipSuccess) return e;
        float *t = cur; cur = nxt; nxt = t;
        e = one_plan(pp, cur, s);
        if (e != hipSuccess) return e;
        if (M >= o.M_max && N >= o.N_max) break;  // the stage at the full budget has run
        if (N < o.N_max) {
            n_old = N;
            N = 2 * N < o.N_max ? 2 * N : o.N_max;
        } else {
            ++M;  // new epoch: more layers, every layer resampled
            n_old = 0;
        }
    }
    return hipSuccess;
}

}  // namespace gtmp
