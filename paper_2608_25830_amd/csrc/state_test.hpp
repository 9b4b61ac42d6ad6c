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

// Sphere slots of an arm rounded up to the instantiated probe counts.
inline int round8(int k) { return ((k + 7) / 8) * 8; }

}  // namespace gtmp
