// gtmp_device.hpp -- device-side building blocks of the gfx950 planner:
// counter-based RNG, the robot/obstacle collision model in the form the
// kernels evaluate it, and wave64 helpers.  Included by the kernel sources
// only; the public boundary is include/gtmp.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gtmp.h"

namespace gtmp {

constexpr int kWave = 64;

// Vertex stride (floats) of the packed vertex array used by the edge kernels:
// every vertex takes GTMP_MAX_DOF floats (zero padded), 32-byte aligned.
inline int vertex_stride(int) { return GTMP_MAX_DOF; }

constexpr int kTile = 256;  // edges per pre-pass tile (one block, one edge per thread)

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit products whose halves are mixed with the other counter words
// and the round key; the key advances by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo_a = 0xD2511F53u * c.x, hi_a = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo_b = 0xCD9E8D57u * c.z, hi_b = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi_b ^ c.y ^ k0, lo_b, hi_a ^ c.w ^ k1, lo_a);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// 24 high bits of a word as a float in [0, 1); exact in FP32.
__device__ __forceinline__ float unit_from_word(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }

// ---------------------------------------------------------------------------
// Robot model as passed by value in kernel arguments (uniform for the whole
// grid, so every field is read through the scalar unit).
// ---------------------------------------------------------------------------
// Twist kinds of a joint: (cos, sin) of the twist exactly (1, 0), (0, 1),
// (0, -1), or anything else.
constexpr int kTwistGeneral = 0, kTwistNone = 1, kTwistPlus = 2, kTwistMinus = 3;

struct ArmParams {
    int n_joints;
    int n_spheres;
    int uniform_r;  // 1 if every collision sphere has radius r0
    float r0;
    float a[GTMP_MAX_JOINTS], dz[GTMP_MAX_JOINTS], off[GTMP_MAX_JOINTS];
    float ca[GTMP_MAX_JOINTS], sa[GTMP_MAX_JOINTS];  // cos / sin of the twist
    int twist[GTMP_MAX_JOINTS];                       // kind of twist (kTwist*): exact quarter turns take no arithmetic
    int link[GTMP_MAX_ROBOT_SPHERES];
    float t[GTMP_MAX_ROBOT_SPHERES];
    float tm1[GTMP_MAX_ROBOT_SPHERES];  // t - 1: the sphere's place measured from the link's end
    float r[GTMP_MAX_ROBOT_SPHERES];
    int lk_end[GTMP_MAX_JOINTS];  // spheres of link L (1-based) are lk_end[L-2] .. lk_end[L-1]-1 (from 0 for L = 1)
    float reach;    // bound on |sphere centre|: sum of the link lengths sqrt(a^2 + d^2), rounded up
    float sph_tol;  // rounding bound of the expanded sphere test (set on the device per launch)
    float link_reach[GTMP_MAX_JOINTS];  // bound on |centre| of the spheres of link L (index L-1), rounded up
    int k_first;    // spheres below this index can touch no obstacle of the scene (set on the device; 0 = unknown)
};

// Obstacles: raw device arrays of the scene, spheres [n][wdim+1], boxes
// [n][2*wdim].  They are read with wave-uniform indices through the constant
// address space, which lets the compiler fetch them with scalar loads into
// SGPRs (read-only for the lifetime of a launch).
typedef const __attribute__((address_space(4))) float *cfp;

struct SceneParams {
    const float *sph;
    const float *box;
    int n_sph;
    int n_box;
};

__device__ __forceinline__ cfp as_const(const float *p) { return (cfp)(p); }

typedef const __attribute__((address_space(4))) struct ArmParams *carm;

// ---------------------------------------------------------------------------
// Collision test of a set of KP probe spheres against every obstacle.
// Returns min over (probe, obstacle) of |p - closest point|^2 - R^2, so the
// probe set is in collision iff the result is <= 0.  R = obstacle radius +
// probe radius for sphere obstacles, probe radius for boxes.  Obstacles are
// the outer loop: each obstacle is loaded once (scalar registers) and tested
// against all probes held in vector registers.
// ---------------------------------------------------------------------------
template <int W, int KP>
struct Probes {
    float p[W][KP];
};

// Copy a wave-uniform value into a vector register (a plain v_mov; keeps the
// compiler from folding the scalar operand back into every use).
__device__ __forceinline__ float to_vgpr(float s) {
    float v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

// s_waitcnt immediate for gfx9: lgkmcnt(0), vmcnt and expcnt left at their maxima
constexpr int kWaitLgkm0 = 0xC07F;

// SPH / BOX select the obstacle kinds tested (both by default).
template <int W, int KP, bool UNIFORM_R, bool SPH = true, bool BOX = true>
__device__ __forceinline__ float probes_min_gap(const Probes<W, KP> &P, const float (&pr)[KP], float r0,
                                                const SceneParams &S) {
    float m0 = __builtin_inff(), m1 = __builtin_inff();
    const cfp sph = as_const(S.sph);
    const cfp box = as_const(S.box);
    // Scalar loads are software pipelined: the data of obstacle o + 1 is
    // requested before obstacle o is tested, so the scalar-cache latency hides
    // behind the vector work of the current obstacle.
    if (SPH && S.n_sph > 0) {
        float c[W + 1];
#pragma unroll
        for (int i = 0; i <= W; ++i) c[i] = sph[i];
        // drain every scalar load issued so far, so that the only scalar load
        // in flight inside the loop is the prefetch of the next obstacle
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        for (int o = 0; o < S.n_sph; ++o) {
            const int on = o + 1 < S.n_sph ? o + 1 : o;
            float cn[W + 1];
#pragma unroll
            for (int i = 0; i <= W; ++i) cn[i] = sph[on * (W + 1) + i];
            __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the tests
            const float ro = c[W];
            const float R = ro + r0;
            const float nR2 = -R * R;
            float cv[W];  // VGPR copies: the per-probe subtractions then read no SGPR
#pragma unroll
            for (int i = 0; i < W; ++i) cv[i] = to_vgpr(c[i]);
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                float g;
                if (UNIFORM_R) {
                    g = nR2;
                } else {
                    const float Rk = ro + pr[k];
                    g = -Rk * Rk;
                }
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const float dlt = P.p[i][k] - cv[i];
                    g = __builtin_fmaf(dlt, dlt, g);
                }
                if (k & 1) m1 = __builtin_fminf(m1, g);
                else m0 = __builtin_fminf(m0, g);
            }
#pragma unroll
            for (int i = 0; i <= W; ++i) c[i] = cn[i];
        }
    }
    if (BOX && S.n_box > 0) {
        float b[2 * W];
#pragma unroll
        for (int i = 0; i < 2 * W; ++i) b[i] = box[i];
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        for (int o = 0; o < S.n_box; ++o) {
            const int on = o + 1 < S.n_box ? o + 1 : o;
            float bn[2 * W];
#pragma unroll
            for (int i = 0; i < 2 * W; ++i) bn[i] = box[on * 2 * W + i];
            __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the tests
            float lo[W], hi[W];
#pragma unroll
            for (int i = 0; i < W; ++i) {
                lo[i] = b[i] - b[W + i];
                hi[i] = b[i] + b[W + i];
            }
            const float nr2 = -r0 * r0;
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                float g = UNIFORM_R ? nr2 : -pr[k] * pr[k];
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const float x = P.p[i][k];
                    const float dlt = x - __builtin_amdgcn_fmed3f(x, lo[i], hi[i]);
                    g = __builtin_fmaf(dlt, dlt, g);
                }
                if (k & 1) m1 = __builtin_fminf(m1, g);
                else m0 = __builtin_fminf(m0, g);
            }
#pragma unroll
            for (int i = 0; i < 2 * W; ++i) b[i] = bn[i];
        }
    }
    return __builtin_fminf(m0, m1);
}

// Sphere obstacles only, in the expanded form
//   |p - c|^2 - R^2 = |p|^2 + p.(-2c) + (|c|^2 - R^2),
// for KC probes of the uniform radius r0: per (probe, obstacle) pair three
// FMAs and half a three-way min (two obstacles per iteration, one running
// minimum per probe); |p|^2 is added once per probe at the end.  Compared with
// the difference form this loses accuracy by cancellation when |p| and |c| are
// large against |p - c|.  With u = 2^-24 and B = (|p| + |c|)^2 + R^2 the
// rounding error of this form is below 8.1 u B and that of the difference form
// below 4 u B, so whenever the result exceeds tol = 32 u B_max in magnitude
// both forms give the same sign; callers re-evaluate the difference form for
// results within tol (B_max from a bound on |p| and the largest |c| and R).
template <int KC>
__device__ __forceinline__ float sph_min_gap_expanded(const Probes<3, KC> &P, float r0, const SceneParams &S) {
    float acc[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = __builtin_inff();
    const cfp sph = as_const(S.sph);
    const int n = S.n_sph;
    if (n > 0) {
        float c[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            c[i] = sph[i];
            c[4 + i] = sph[(n > 1 ? 4 : 0) + i];
        }
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
        for (int o = 0; o < n; o += 2) {
            // the next pair (the last obstacle repeats when n is odd: a
            // repeated minimum changes nothing)
            const int o1 = o + 2 < n ? o + 2 : o;
            const int o2 = o + 3 < n ? o + 3 : o1;
            float cn[8];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                cn[i] = sph[o1 * 4 + i];
                cn[4 + i] = sph[o2 * 4 + i];
            }
            __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the tests
            float a[2][3], t[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float cx = c[4 * h], cy = c[4 * h + 1], cz = c[4 * h + 2];
                const float R = c[4 * h + 3] + r0;
                a[h][0] = -2.f * cx;
                a[h][1] = -2.f * cy;
                a[h][2] = -2.f * cz;
                const float c2 = __builtin_fmaf(cz, cz, __builtin_fmaf(cy, cy, cx * cx));
                t[h] = c2 - R * R;
            }
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const float x = P.p[0][k], y = P.p[1][k], z = P.p[2][k];
                const float v0 = __builtin_fmaf(x, a[0][0], __builtin_fmaf(y, a[0][1], __builtin_fmaf(z, a[0][2], t[0])));
                const float v1 = __builtin_fmaf(x, a[1][0], __builtin_fmaf(y, a[1][1], __builtin_fmaf(z, a[1][2], t[1])));
                acc[k] = __builtin_fminf(acc[k], __builtin_fminf(v0, v1));
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) c[i] = cn[i];
        }
    }
    float gap = __builtin_inff();
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const float x = P.p[0][k], y = P.p[1][k], z = P.p[2][k];
        const float s2 = __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x));
        gap = __builtin_fminf(gap, s2 + acc[k]);
    }
    return gap;
}

// Exact signed distance of one workspace point to the obstacle set:
// spheres |p - c| - r, boxes |max(q,0)| + min(max_i q_i, 0), q = |p - c| - h.
template <int W>
__device__ __forceinline__ float point_sd(const float (&p)[W], const SceneParams &S) {
    float best = __builtin_inff();
    for (int o = 0; o < S.n_sph; ++o) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const float dlt = p[i] - S.sph[o * (W + 1) + i];
            acc = __builtin_fmaf(dlt, dlt, acc);
        }
        best = __builtin_fminf(best, __builtin_sqrtf(acc) - S.sph[o * (W + 1) + W]);
    }
    for (int o = 0; o < S.n_box; ++o) {
        float out = 0.f, in = -__builtin_inff();
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const float q = __builtin_fabsf(p[i] - S.box[o * 2 * W + i]) - S.box[o * 2 * W + W + i];
            const float qp = __builtin_fmaxf(q, 0.f);
            out = __builtin_fmaf(qp, qp, out);
            in = __builtin_fmaxf(in, q);
        }
        best = __builtin_fminf(best, __builtin_sqrtf(out) + __builtin_fminf(in, 0.f));
    }
    return best;
}

// ---------------------------------------------------------------------------
// Sine and cosine of a joint angle.  For |x| <= 32: Cody-Waite reduction
// r = x - k pi/2, k = rint(2x/pi), with pi/2 split into two FP32 parts
// (every product k * part is exact inside its fused multiply-add; the third
// part would move r by less than 4e-14 for |k| <= 21), then minimax
// polynomials on |r| <= pi/4 (Remez exchange on the absolute error):
// sin r = r + r^3 P(r^2), cos r = 1 + r^2 Q(r^2) with P and Q of degree 2
// (approximation errors 1.8e-9 and 3.2e-8), and the quadrant of k.  In FP32
// the results are within 1.2e-7 of the exact values over |x| <= 32, far
// inside what the collision decisions can resolve.  Arguments beyond 32 (or
// not finite) take the library sincosf in that lane only, so a state's
// result never depends on the other lanes of its wave.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void joint_sincos(float x, float &s, float &c) {
    constexpr float kTwoOverPi = 0.636619772367581f;
    constexpr float kP1 = 1.5707963705062866f;      // fl(pi/2)
    constexpr float kP2 = -4.371138828673793e-08f;  // fl(pi/2 - kP1)
    const float k = __builtin_rintf(x * kTwoOverPi);
    float r = __builtin_fmaf(-k, kP1, x);
    r = __builtin_fmaf(-k, kP2, r);
    const float z = r * r;
    // the innermost coefficients enter through scalar registers, so that no
    // vector register holds a constant for the whole kernel
    const float p2 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(-1.949563593e-04f)));
    const float q2 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(-1.359782298e-03f)));
    float ps = __builtin_fmaf(z, p2, 8.331978694e-03f);
    ps = __builtin_fmaf(z, ps, -1.666665077e-01f);
    const float sr = __builtin_fmaf(r * z, ps, r);
    float pc = __builtin_fmaf(z, q2, 4.165629297e-02f);
    pc = __builtin_fmaf(z, pc, -4.999989569e-01f);
    const float cr = __builtin_fmaf(z, pc, 1.0f);
    // quadrant n = k mod 4: sin x = (s, c, -s, -c)[n], cos x = (c, -s, -c, s)[n]
    const int n = (int)k;
    const bool swap = (n & 1) != 0;
    const float a = swap ? cr : sr, b = swap ? sr : cr;
    s = __uint_as_float(__float_as_uint(a) ^ (((uint32_t)n << 30) & 0x80000000u));
    c = __uint_as_float(__float_as_uint(b) ^ (((uint32_t)(n + 1) << 30) & 0x80000000u));
    if (!(__builtin_fabsf(x) <= 32.0f)) sincosf(x, &s, &c);
}

// ---------------------------------------------------------------------------
// Serial-arm forward kinematics, standard DH: frame i+1 = frame i *
// Rz(q_i + off_i) Tz(dz_i) Tx(a_i) Rx(alpha_i).  The frame is updated in place
// (columns x, y, z and origin p).  The origins o_0..o_J are returned packed in
// one 32-wide register vector [o_0.xyz, o_1.xyz, ...]; the sphere loop reads
// it with wave-uniform indices (the link id of a sphere is the same for every
// lane), which gfx9 serves with relative VGPR addressing.
// ---------------------------------------------------------------------------
typedef float v32f __attribute__((ext_vector_type(32)));

// Frame origins visited link by link: after joint j the visitor gets the link
// index L = j + 1 and the origins o_{L-1} (b) and o_L (p) of that link.  The
// first joint starts from the identity frame, written out (the general
// update would multiply by the frame's zeros and ones, which floating point
// cannot drop; the values are the same).
template <int D, class AP, class F>
__device__ __forceinline__ void arm_fk_visit(const AP &A, const float (&q)[D], F &&link) {
    float x0 = 1.f, x1 = 0.f, x2 = 0.f;
    float y0 = 0.f, y1 = 1.f, y2 = 0.f;
    float z0 = 0.f, z1 = 0.f, z2 = 1.f;
    float p0 = 0.f, p1 = 0.f, p2 = 0.f;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        if (j >= A.n_joints) break;
        const float b[3] = {p0, p1, p2};
        float st, ct;
        joint_sincos(q[j] + A.off[j], st, ct);
        const float ca = A.ca[j], sa = A.sa[j];
        if (j == 0) {
            x0 = ct; x1 = st; x2 = 0.f;
            p0 = A.a[0] * ct; p1 = A.a[0] * st; p2 = A.dz[0];
            y0 = -(ca * st); y1 = ca * ct; y2 = sa;
            z0 = sa * st; z1 = -(sa * ct); z2 = ca;
        } else {
            const float xn0 = ct * x0 + st * y0, xn1 = ct * x1 + st * y1, xn2 = ct * x2 + st * y2;
            p0 += A.a[j] * xn0 + A.dz[j] * z0;
            p1 += A.a[j] * xn1 + A.dz[j] * z1;
            p2 += A.a[j] * xn2 + A.dz[j] * z2;
            {
                const float yp0 = ct * y0 - st * x0, yp1 = ct * y1 - st * x1, yp2 = ct * y2 - st * x2;
                // y' = ca yp + sa z, z' = ca z - sa yp; exact quarter turns and
                // no twist give the same values without the products
                const int tw = A.twist[j];
                if (tw == kTwistNone) {
                    y0 = yp0; y1 = yp1; y2 = yp2;
                } else if (tw == kTwistPlus) {
                    y0 = z0; y1 = z1; y2 = z2;
                    z0 = -yp0; z1 = -yp1; z2 = -yp2;
                } else if (tw == kTwistMinus) {
                    y0 = -z0; y1 = -z1; y2 = -z2;
                    z0 = yp0; z1 = yp1; z2 = yp2;
                } else {
                    const float yn0 = ca * yp0 + sa * z0, yn1 = ca * yp1 + sa * z1, yn2 = ca * yp2 + sa * z2;
                    const float zn0 = ca * z0 - sa * yp0, zn1 = ca * z1 - sa * yp1, zn2 = ca * z2 - sa * yp2;
                    y0 = yn0; y1 = yn1; y2 = yn2;
                    z0 = zn0; z1 = zn1; z2 = zn2;
                }
            }
            x0 = xn0; x1 = xn1; x2 = xn2;
        }
        const float p[3] = {p0, p1, p2};
        link(j + 1, b, p);
    }
}

template <int D, class AP>
__device__ __forceinline__ v32f arm_fk(const AP &A, const float (&q)[D]) {
    v32f o;  // only o_0 .. o_J are written and read
    o[0] = 0.f;
    o[1] = 0.f;
    o[2] = 0.f;
    arm_fk_visit<D>(A, q, [&](int L, const float (&)[3], const float (&p)[3]) {
        o[3 * L + 0] = p[0];
        o[3 * L + 1] = p[1];
        o[3 * L + 2] = p[2];
    });
    return o;
}

// Collision sphere centres c_k = o_{L-1} + t_k (o_L - o_{L-1}) for spheres
// BASE .. BASE+KC-1; slots beyond n_spheres are parked far away so that they
// can never collide.
template <int KC, int BASE = 0, class AP>
__device__ __forceinline__ void arm_spheres(const AP &A, const v32f &o, Probes<3, KC> &P) {
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const int k = BASE + kk;
        if (k < A.n_spheres) {
            const int b = 3 * A.link[k];
            const float t = A.t[k];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float lo = o[b - 3 + i];
                const float hi = o[b + i];
                P.p[i][kk] = __builtin_fmaf(t, hi - lo, lo);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) P.p[i][kk] = 1.0e18f;
        }
    }
}

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ int rank_in(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// x of lane `src` (taken mod 64), for every lane.
__device__ __forceinline__ uint32_t lane_read(int src, uint32_t x) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)x);
}

// Index of the calling wave in its block, as a scalar (so that per-wave LDS
// arrays indexed by it keep their base addresses in scalar registers).
__device__ __forceinline__ uint32_t wave_in_block() { return uniform(threadIdx.x / (uint32_t)kWave); }

}  // namespace gtmp
