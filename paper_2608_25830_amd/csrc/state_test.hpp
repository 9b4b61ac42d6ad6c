// state_test.hpp -- collision gap of one configuration for the kernels that
// test states one lane at a time outside the edge checker (path shortcutting,
// the RRT-Connect local planner): every robot sphere at once, per-sphere radii
// or the uniform radius, difference form.  <= 0 iff the state collides.
#pragma once

#include "gtmp_launch.hpp"

namespace gtmp {

template <bool ARM, int W>
struct StateDim {
    static constexpr int D = ARM ? GTMP_MAX_JOINTS : W;
};

// Arm spheres BASE .. KP-1 in chunks of KC (fewer live registers than all
// KP at once); the minimum over chunks is the minimum over all spheres.
template <int KC, int BASE, int KP, bool UNIFORM>
__device__ __forceinline__ float arm_gap_chunked(const ArmParams &R, const v32f &o, const SceneParams &S) {
    Probes<3, KC> P;
    arm_spheres<KC, BASE>(R, o, P);
    float pr[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) pr[k] = BASE + k < R.n_spheres ? R.r[BASE + k] : 0.f;
    const float g = probes_min_gap<3, KC, UNIFORM>(P, pr, R.r0, S);
    if constexpr (BASE + KC < KP)
        return __builtin_fminf(g, arm_gap_chunked<KC, BASE + KC, KP, UNIFORM>(R, o, S));
    else
        return g;
}

template <bool ARM, int W, int KP>
__device__ __forceinline__ float state_gap(const ArmParams &R, const SceneParams &S,
                                           const float (&q)[StateDim<ARM, W>::D]) {
    if constexpr (ARM) {
        constexpr int KC = KP >= 32 ? KP / 2 : KP;
        const v32f o = arm_fk<GTMP_MAX_JOINTS>(R, q);
        return R.uniform_r ? arm_gap_chunked<KC, 0, KP, true>(R, o, S) : arm_gap_chunked<KC, 0, KP, false>(R, o, S);
    } else {
        Probes<W, 1> P;
#pragma unroll
        for (int k = 0; k < W; ++k) P.p[k][0] = q[k];
        const float pr[1] = {0.f};
        return probes_min_gap<W, 1, true>(P, pr, 0.f, S);
    }
}

// Gap of the probes P (radius pr(k), k < NP) over the obstacles o = part,
// part + nparts, ... of each kind; obstacles read with per-lane loads.
template <int PW, int NP, class PR>
__device__ __forceinline__ float probes_gap_part(const Probes<PW, NP> &P, PR pr, const SceneParams &S, int part,
                                                 int nparts) {
    float m = __builtin_inff();
    for (int ob = part; ob < S.n_sph; ob += nparts) {
        float c[PW + 1];
#pragma unroll
        for (int i = 0; i <= PW; ++i) c[i] = S.sph[ob * (PW + 1) + i];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const float Rk = c[PW] + pr(k);
            float g = -Rk * Rk;
#pragma unroll
            for (int i = 0; i < PW; ++i) {
                const float dlt = P.p[i][k] - c[i];
                g = __builtin_fmaf(dlt, dlt, g);
            }
            m = __builtin_fminf(m, g);
        }
    }
    for (int ob = part; ob < S.n_box; ob += nparts) {
        float lo[PW], hi[PW];
#pragma unroll
        for (int i = 0; i < PW; ++i) {
            const float c = S.box[ob * 2 * PW + i], h = S.box[ob * 2 * PW + PW + i];
            lo[i] = c - h;
            hi[i] = c + h;
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const float rk = pr(k);
            float g = -rk * rk;
#pragma unroll
            for (int i = 0; i < PW; ++i) {
                const float x = P.p[i][k];
                const float dlt = x - __builtin_amdgcn_fmed3f(x, lo[i], hi[i]);
                g = __builtin_fmaf(dlt, dlt, g);
            }
            m = __builtin_fminf(m, g);
        }
    }
    return m;
}

template <int KC, int BASE, int KP>
__device__ __forceinline__ float arm_gap_part(const ArmParams &R, const v32f &o, const SceneParams &S, int part,
                                              int nparts) {
    Probes<3, KC> P;
    arm_spheres<KC, BASE>(R, o, P);
    auto pr = [&](int k) { return R.uniform_r ? R.r0 : (BASE + k < R.n_spheres ? R.r[BASE + k] : 0.f); };
    const float g = probes_gap_part<3, KC>(P, pr, S, part, nparts);
    if constexpr (BASE + KC < KP)
        return __builtin_fminf(g, arm_gap_part<KC, BASE + KC, KP>(R, o, S, part, nparts));
    else
        return g;
}

// The state gap restricted to the obstacles o = part, part + nparts, ... of
// each kind: nparts lanes holding one state each compute its gap together
// (the minimum over their results), so a step that checks few states keeps
// the wave's lanes busy.
template <bool ARM, int W, int KP>
__device__ __forceinline__ float state_gap_part(const ArmParams &R, const SceneParams &S,
                                                const float (&q)[StateDim<ARM, W>::D], int part, int nparts) {
    if constexpr (ARM) {
        constexpr int KC = KP >= 32 ? KP / 2 : KP;
        const v32f o = arm_fk<GTMP_MAX_JOINTS>(R, q);
        return arm_gap_part<KC, 0, KP>(R, o, S, part, nparts);
    } else {
        Probes<W, 1> P;
#pragma unroll
        for (int i = 0; i < W; ++i) P.p[i][0] = q[i];
        return probes_gap_part<W, 1>(P, [](int) { return 0.f; }, S, part, nparts);
    }
}

// Sphere slots of an arm rounded up to the instantiated probe counts.
inline int round8(int k) { return ((k + 7) / 8) * 8; }

}  // namespace gtmp
