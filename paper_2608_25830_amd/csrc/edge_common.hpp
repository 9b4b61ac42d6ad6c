// edge_common.hpp -- kernel arguments and device helpers shared by the
// single-plan edge kernels (edge.hip) and the batched ones (batch.hip).
#pragma once

#include "gtmp_launch.hpp"

namespace gtmp {

// ------------------------------------------------------------------ kernel args
struct EdgeArgs {
    int d, M, N, G, H, dp;
    float penalty, max_len;
    uint32_t tiles_per_row, n_tiles, n_vertices;
    const float *__restrict__ verts;
    const uint8_t *__restrict__ vflag;
    float *C_s, *C_h, *C_l;
    uint8_t *flags;
    const uint8_t *__restrict__ prune;
    const uint8_t *__restrict__ select;  // lazy rounds: only edges with select[e] != 0 are touched
    uint8_t *tile_off;
    uint32_t *tile_cnt;
    uint32_t *counter;  // [0] tile cursor of the interior kernel, [1] length of tile_list
    uint32_t *tile_list;  // lazy rounds: the tiles holding candidates (NULL: every tile in order)
    unsigned long long *stats;
    size_t off_params;  // workspace byte offset of the device copy of the robot table
    int n_int;
    float tord[GTMP_MAX_H];  // t = h / (H-1) of the interior states, in check order
};

// ------------------------------------------------------------------ arm state test
// Collision gap of one arm state (<= 0 iff some robot sphere touches an
// obstacle), its spheres evaluated in NCH chunks of KP / NCH.  Uniform robot
// radius: sphere obstacles in the expanded form with the difference form
// re-evaluated for the lanes within the rounding bound R.sph_tol of zero
// (wave-uniform branch), boxes in the difference form.  Otherwise every
// obstacle in the difference form with per-sphere radii.  Every lane of the
// wave must call this (it contains a ballot).
template <int KP, int NCH, bool UNIFORM_R, class AP>
__device__ __forceinline__ float arm_state_gap(const AP &R, const v32f &o, float r0, const SceneParams &S) {
    constexpr int KC = KP / NCH;
    float gap = __builtin_inff();
    float pr[KC];
    const float tol = UNIFORM_R ? R.sph_tol : 0.f;
#pragma unroll
    for (int k = 0; k < KC; ++k) pr[k] = 0.f;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        Probes<3, KC> P;
        if (ch == 0) arm_spheres<KC, 0>(R, o, P);
        else if (ch == 1) arm_spheres<KC, (NCH > 1 ? KC : 0)>(R, o, P);
        else if (ch == 2) arm_spheres<KC, (NCH > 2 ? 2 * KC : 0)>(R, o, P);
        else arm_spheres<KC, (NCH > 3 ? 3 * KC : 0)>(R, o, P);
        float g;
        if constexpr (UNIFORM_R) {
            float gs = sph_min_gap_expanded<KC>(P, r0, S);
            const bool near = __builtin_fabsf(gs) <= tol;
            if (ballot(near) != 0) {
                const float ex = probes_min_gap<3, KC, true, true, false>(P, pr, r0, S);
                if (near) gs = ex;
            }
            g = __builtin_fminf(gs, probes_min_gap<3, KC, true, false, true>(P, pr, r0, S));
        } else {
#pragma unroll
            for (int k = 0; k < KC; ++k) pr[k] = ch * KC + k < R.n_spheres ? R.r[ch * KC + k] : 0.f;
            g = probes_min_gap<3, KC, false>(P, pr, r0, S);
        }
        gap = ch == 0 ? g : __builtin_fminf(gap, g);
    }
    return gap;
}

// Row / tile decoding.  Rows enumerate the edges by their shared endpoint:
//   row 0                 : q0 -> layer 0 vertex n            (C_s[n])
//   row 1 + m N + u       : layer m vertex u -> layer m+1 vertex n  (C_h[m][u][n])
//   row 1 + (M-1) N + g   : layer M-1 vertex n -> goal g       (C_l[n][g])
// n is the varying index of the row (0..N-1).  Vertex ids index the packed
// array [q0 | Q[0][0..N) | ... | Q[M-1][0..N) | goals].
struct RowInfo {
    uint32_t u_base, u_step, v_base, v_step;  // vertex ids of (u, v) = base + n * step
    uint64_t e_base, e_step;                  // flat edge id (C_s | C_h | C_l order)
    float *c_base;                            // cost element of n = c_base + n * c_step
    uint32_t c_step;
};

__device__ __forceinline__ RowInfo decode_row(const EdgeArgs &A, uint32_t row) {
    RowInfo r;
    const uint32_t N = (uint32_t)A.N;
    const uint32_t inner_rows = (uint32_t)(A.M - 1) * N;
    if (row == 0) {
        r.u_base = 0; r.u_step = 0; r.v_base = 1; r.v_step = 1;
        r.e_base = 0; r.e_step = 1; r.c_base = A.C_s; r.c_step = 1;
    } else if (row <= inner_rows) {
        const uint32_t ri = row - 1;       // = m N + u
        const uint32_t m = ri / N;
        r.u_base = 1 + ri; r.u_step = 0;
        r.v_base = 1 + (m + 1) * N; r.v_step = 1;
        r.e_base = (uint64_t)N + (uint64_t)ri * N; r.e_step = 1;
        r.c_base = A.C_h + (size_t)ri * N; r.c_step = 1;
    } else {
        const uint32_t g = row - 1 - inner_rows;
        r.u_base = 1 + (uint32_t)(A.M - 1) * N; r.u_step = 1;
        r.v_base = 1 + (uint32_t)A.M * N + g; r.v_step = 0;
        r.e_base = (uint64_t)N + (uint64_t)inner_rows * N + g; r.e_step = (uint32_t)A.G;
        r.c_base = A.C_l + g; r.c_step = (uint32_t)A.G;
    }
    return r;
}

template <int D>
__device__ __forceinline__ void load_vertex(const EdgeArgs &A, uint32_t vid, float (&x)[D]) {
    const float *p = A.verts + (size_t)vid * A.dp;
    if constexpr (D <= 4) {
        const float4 a = *reinterpret_cast<const float4 *>(p);
        const float t[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int i = 0; i < D; ++i) x[i] = t[i];
    } else {
        const float4 a = *reinterpret_cast<const float4 *>(p);
        const float4 b = *reinterpret_cast<const float4 *>(p + 4);
        const float t[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int i = 0; i < D; ++i) x[i] = t[i];
    }
}

// Euclidean length in configuration space (FP32, fixed summation order so
// that the pre-pass and the interior kernel produce the same value).
template <int D>
__device__ __forceinline__ float edge_len(const float (&u)[D], const float (&v)[D], int d) {
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < D; ++i)
        if (i < d) {
            const float t = v[i] - u[i];
            acc = __builtin_fmaf(t, t, acc);
        }
    return __builtin_sqrtf(acc);
}

__device__ __forceinline__ float failed_cost(float len, float penalty) { return len + penalty; }

// ------------------------------------------------------------------ robot adapters
// Point robot in R^W: a state is one probe of radius 0.  Arm: a state is KP
// probes (the collision spheres) obtained by forward kinematics.
template <int W, int S>
struct PointModel {
    static constexpr bool kArm = false;
    static constexpr int D = W;
    static constexpr int KP = S;  // probes per evaluation = S states
};

template <int KPm>
struct ArmModel {
    static constexpr bool kArm = true;
    static constexpr int D = GTMP_MAX_JOINTS;
    static constexpr int KP = KPm;
};


__device__ __forceinline__ float *cost_slot(const EdgeArgs &A, uint32_t e) {
    const uint32_t N = (uint32_t)A.N;
    const uint32_t inner_end = N + (uint32_t)(A.M - 1) * N * N;
    if (e < N) return A.C_s + e;
    if (e < inner_end) return A.C_h + (e - N);
    return A.C_l + (e - inner_end);
}

}  // namespace gtmp
