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

template <bool ARM, int W, int KP>
__device__ __forceinline__ float state_gap(const ArmParams &R, const SceneParams &S,
                                           const float (&q)[StateDim<ARM, W>::D]) {
    if constexpr (ARM) {
        const v32f o = arm_fk<GTMP_MAX_JOINTS>(R, q);
        Probes<3, KP> P;
        arm_spheres<KP>(R, o, P);
        float pr[KP];
#pragma unroll
        for (int k = 0; k < KP; ++k) pr[k] = k < R.n_spheres ? R.r[k] : 0.f;
        return R.uniform_r ? probes_min_gap<3, KP, true>(P, pr, R.r0, S) : probes_min_gap<3, KP, false>(P, pr, R.r0, S);
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
