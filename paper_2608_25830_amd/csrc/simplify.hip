// simplify.hip -- shortcutting of planned paths (simp() of Alg. 1 ao-gtmp;
// Sec. IV-E), which the paper uses but does not define.
//
// Reading implemented here: a path of K waypoints w_0 .. w_{K-1} keeps the
// state spacing of the plan's own edges, so the shortcut w_i -> w_j (i < j)
// is tested at H_ij = (j - i)(H - 1) + 1 states, t = h / (H_ij - 1); a
// consecutive pair is tested exactly as the plan tested its edge.  The
// simplified path is the shortest chain w_0 -> w_{K-1} over the shortcuts that
// pass (edge lengths as the edge check computes them; ties to the lowest next
// index).
//
// Two kernels, B paths per launch:
//   k_shortcut_check  one wave per ordered pair (path, i, j): lanes take 64
//                     states at a time, a ballot ends the pair at the first
//                     colliding state;
//   k_shortcut_dp     one wave per path: lane j holds the cost-to-goal of
//                     waypoint j, the backward recursion takes K - 1 wave
//                     arg-min reductions, then the chain is followed from w_0.
#include "edge_common.hpp"
#include "state_test.hpp"

namespace gtmp {

template <bool ARM, int W, int KP>
__global__ void __launch_bounds__(256) k_shortcut_check(ArmParams R, SceneParams S, int d, int B, int K, int H,
                                                        const float *__restrict__ wp, uint8_t *__restrict__ valid) {
    constexpr int D = ARM ? GTMP_MAX_JOINTS : W;
    const int lane = lane_id();
    const uint64_t KK = (uint64_t)K * K;
    const uint64_t gw = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (gw >= (uint64_t)B * KK) return;  // wave-uniform
    const uint64_t b = gw / KK;
    const int r = (int)(gw - b * KK);
    const int i = r / K, j = r - (r / K) * K;
    if (j <= i) {
        if (lane == 0) valid[gw] = 0;
        return;
    }
    const float *pu = wp + (b * K + i) * d;
    const float *pv = wp + (b * K + j) * d;
    float u[D], v[D], dv[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        u[k] = k < d ? pu[k] : 0.f;
        v[k] = k < d ? pv[k] : 0.f;
        dv[k] = v[k] - u[k];
    }
    bool finite = true;
#pragma unroll
    for (int k = 0; k < D; ++k) finite = finite && __builtin_isfinite(u[k]) && __builtin_isfinite(v[k]);
    if (!finite) {  // wave-uniform: a non-finite waypoint fails every shortcut touching it
        if (lane == 0) valid[gw] = 0;
        return;
    }
    const int Hij = (j - i) * (H - 1) + 1;
    const float den = (float)(Hij - 1);
    bool free = true;
    for (int h0 = 0; h0 < Hij; h0 += kWave) {
        const int h = h0 + lane;
        const bool act = h < Hij;
        const bool last = h == Hij - 1;  // the far endpoint itself, not u + 1 * (v - u)
        const float t = (float)(act ? h : 0) / den;
        float q[D];
#pragma unroll
        for (int k = 0; k < D; ++k) q[k] = last ? v[k] : __builtin_fmaf(t, dv[k], u[k]);
        const float gap = state_gap<ARM, W, KP>(R, S, q);
        if (ballot(act && !(gap > 0.f)) != 0) {
            free = false;
            break;
        }
    }
    if (lane == 0) valid[gw] = free ? 1 : 0;
}

__global__ void __launch_bounds__(kWave) k_shortcut_dp(int d, int K, const float *__restrict__ wp,
                                                       const uint8_t *__restrict__ valid, int32_t *idx, int32_t *count,
                                                       float *cost, float *out_wp) {
    const int lane = threadIdx.x;
    const size_t b = blockIdx.x;
    const float *Wb = wp + b * K * d;
    const uint8_t *Vb = valid + b * K * K;
    const float inf = __builtin_inff();
    float x[GTMP_MAX_DOF];
#pragma unroll
    for (int k = 0; k < GTMP_MAX_DOF; ++k) x[k] = (lane < K && k < d) ? Wb[lane * d + k] : 0.f;
    float best = lane == K - 1 ? 0.f : inf;
    int nxt = -1;
    for (int i = K - 2; i >= 0; --i) {
        float c = inf;
        if (lane > i && lane < K && Vb[i * K + lane] != 0 && best < inf) {
            float wi[GTMP_MAX_DOF];
#pragma unroll
            for (int k = 0; k < GTMP_MAX_DOF; ++k) wi[k] = k < d ? Wb[i * d + k] : 0.f;
            c = edge_len<GTMP_MAX_DOF>(wi, x, d) + best;
        }
        int a = c < inf ? lane : kWave;
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const float oc = __shfl_xor(c, off);
            const int oa = __shfl_xor(a, off);
            if (oc < c || (oc == c && oa < a)) {
                c = oc;
                a = oa;
            }
        }
        if (lane == i) {
            best = c;
            nxt = c < inf ? a : -1;
        }
    }
    const float total = __shfl(best, 0);
    int n = 0;
    if (total < inf) {
        int cur = 0;
        while (true) {  // wave-uniform walk; every step moves to a larger index
            if (lane == 0) idx[b * K + n] = cur;
            if (out_wp && lane < d) out_wp[(b * K + n) * d + lane] = Wb[cur * d + lane];
            ++n;
            if (cur == K - 1 || n == K) break;
            cur = __shfl(nxt, cur);
        }
    }
    for (int r = n + lane; r < K; r += kWave) idx[b * K + r] = -1;
    if (out_wp)
        for (int r = n * d + lane; r < K * d; r += kWave) out_wp[b * K * d + r] = __builtin_nanf("");
    if (lane == 0) {
        count[b] = n;
        cost[b] = total;
    }
}

hipError_t launch_simplify(const ArmParams *arm, const SceneParams &scene, int wdim, int d, int B, int K, int H,
                           const float *wp, uint8_t *valid, int32_t *idx, int32_t *count, float *cost, float *out_wp,
                           hipStream_t s) {
    if (B == 0) return hipSuccess;
    const uint64_t waves = (uint64_t)B * K * K;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    ArmParams R{};
    if (arm) {
        R = *arm;
        switch (round8(R.n_spheres)) {
#define GTMP_SC(KP) case KP: hipLaunchKernelGGL((k_shortcut_check<true, 3, KP>), dim3(blocks), dim3(256), 0, s, R, scene, d, B, K, H, wp, valid); break;
            GTMP_SC(8) GTMP_SC(16) GTMP_SC(24) GTMP_SC(32) GTMP_SC(40) GTMP_SC(48) GTMP_SC(56) GTMP_SC(64)
#undef GTMP_SC
            default: return hipErrorInvalidValue;
        }
    } else if (wdim == 2) {
        hipLaunchKernelGGL((k_shortcut_check<false, 2, 1>), dim3(blocks), dim3(256), 0, s, R, scene, d, B, K, H, wp,
                           valid);
    } else {
        hipLaunchKernelGGL((k_shortcut_check<false, 3, 1>), dim3(blocks), dim3(256), 0, s, R, scene, d, B, K, H, wp,
                           valid);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_shortcut_dp, dim3((unsigned)B), dim3(kWave), 0, s, d, K, wp, valid, idx, count, cost, out_wp);
    return hipGetLastError();
}

}  // namespace gtmp
