// edge_common.hpp -- kernel arguments and device helpers shared by the
// single-plan edge kernels (edge.hip) and the batched ones (batch.hip).
#pragma once

#include <stddef.h>

#include <type_traits>

#include "gtmp_launch.hpp"

namespace gtmp {

// ------------------------------------------------------------------ obstacle bins
// A conservative filter in front of the exact sphere test of an arm state.
// Each obstacle o is a rounded box: the points within rho_o of the box
// [lo_o, hi_o] (a sphere obstacle has lo = hi = centre and rho = its radius,
// a box has rho = 0).  A robot sphere of radius r at p can only touch it if,
// on every axis i, p_i lies in [lo_oi - E_o, hi_oi + E_o] with
// E_o = (rho_o + r_max)(1 + 2^-12).  Each axis is cut into bins by the bin
// coordinate f = x inv_i + off_i (one FP32 fused multiply-add) and the bin
// index rne(f) saturated to 0..255 (one v_cvt_pk_u8_f32, which also sends NaN
// to 0).  The obstacles span f in about [5, 250], so bins 0 and 255 catch
// everything outside and hold no obstacle.  mask[w][i][b] has bit o - 32 w
// set when obstacle o's interval on axis i reaches bin b, widened by one bin
// on each side.  The AND of the three masks of p's bins therefore holds every
// obstacle the exact test could find in contact with p: the kernel evaluates
// the exact test on those obstacles only, and its decision is the one of the
// full test.
constexpr int kGridCells = 256;
constexpr int kGridMaxObs = 96;  // three mask words

struct ObsGrid {
    float inv[4], off[4];                  // axes x, y, z (the fourth entry unused)
    float4 rec[kGridMaxObs][2];            // (lo.xyz, rho), (hi.xyz, -(rho + r_max)^2); 2D scenes: z = 0
    uint32_t mask[3][3][kGridCells];       // mask word, axis, bin (axes past the workspace list every obstacle)
};

// Mask words for a scene of n obstacles (0: too many for the bins).
inline int grid_words(int n) { return n <= 32 ? 1 : n <= 64 ? 2 : n <= kGridMaxObs ? 3 : 0; }
inline int grid_words_for(int n) { return grid_words(n); }  // (where a local variable hides grid_words)
// The part of the grid a kernel with WORDS mask words copies to LDS.
template <int WORDS>
constexpr size_t grid_lds_bytes() { return offsetof(ObsGrid, mask) + sizeof(uint32_t) * 3 * kGridCells * WORDS; }

template <int WORDS>
struct alignas(16) GridLds {
    unsigned char bytes[grid_lds_bytes<WORDS>()];
};

// Copy of the first BYTES bytes of src (global) to dst (LDS) by THREADS
// threads, tid being the caller's index among them: every 16-byte load of a
// thread is issued before its first store, so the copy waits for memory once
// rather than once per load.
// (A native vector type: an array of HIP's uint4 structs is not promoted to
// registers.)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <size_t BYTES, int THREADS>
__device__ __forceinline__ void copy_to_lds(void *dst, const void *src, int tid) {
    constexpr int n16 = (int)(BYTES / 16), iters = (n16 + THREADS - 1) / THREADS;
    const u32x4 *s = reinterpret_cast<const u32x4 *>(src);
    u32x4 *d = reinterpret_cast<u32x4 *>(dst);
    u32x4 t[iters];
#pragma unroll
    for (int i = 0; i < iters; ++i) {
        const int k = tid + i * THREADS;
        t[i] = s[k < n16 ? k : n16 - 1];  // unconditional: past the end, the last piece again
    }
#pragma unroll
    for (int i = 0; i < iters; ++i) {
        const int k = tid + i * THREADS;
        if (k < n16) d[k] = t[i];
    }
}

// Point kernels keep the mask words of one (axis, bin) cell side by side in
// LDS, padded to 1, 2 or 4 words, so that a probe reads each axis with one
// vector load.
template <int WORDS>
constexpr int point_mask_stride() { return WORDS == 3 ? 4 : WORDS; }

template <int WORDS>
struct alignas(16) PointMaskLds {
    uint32_t m[3][kGridCells][point_mask_stride<WORDS>()];  // axis, bin, word
};

__device__ __forceinline__ uint32_t grid_bin(float f) { return __builtin_amdgcn_cvt_pk_u8_f32(f, 0u, 0u); }

static_assert(sizeof(ObsGrid) % 16 == 0 && grid_lds_bytes<1>() % 16 == 0, "the grid is copied in 16-byte words");

// ------------------------------------------------------------------ kernel args
struct EdgeArgs {
    int d, M, N, G, H, dp;
    float penalty, max_len;
    uint32_t tiles_per_row, n_tiles, n_vertices;
    uint32_t prepass_rows;  // rows per pre-pass block (1..8)
    const float *__restrict__ verts;
    const uint8_t *__restrict__ vflag;
    float *C_s, *C_h, *C_l;
    uint8_t *flags;
    const uint8_t *__restrict__ prune;
    uint8_t *tile_off;
    uint32_t *tile_cnt;
    uint32_t *counter;  // [0] tile (or list chunk) cursor of the interior kernel
    const uint32_t *edge_list;  // lazy rounds: the edges to check (flat ids), *n_list of them
    const uint32_t *n_list;
    uint8_t *list_mark;         // lazy rounds: per flat edge id, set to 2 when a listed edge collides
    unsigned long long *stats;
    unsigned long long *wstats;  // [kStatWaves][4]: the interior kernel's per-wave totals, or NULL: atomics
    const ObsGrid *grid;  // arms with the bin filter: the obstacle bins of this scene
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

// The obstacle bins of a scene of dimension wdim (2 or 3) for robot spheres
// of radius <= r_max (a point robot: 0), built by one block of
// kGridBuildThreads threads (a thread per obstacle, then a wave per axis, then
// a thread per (axis, bin) cell).  The bin maps and the obstacle intervals are
// computed in FP32 with the same fused multiply-add and bin rounding the
// kernels apply to a probe centre (both monotone), and every interval is
// widened by one bin on each side, so rounding in either place cannot move a
// probe out of a bin that lists the obstacle.  An obstacle with non-finite
// data is listed in every bin, the outer two included, and takes no part in
// the bin maps; should a map still come out non-finite, every obstacle is
// listed everywhere.  Either way the exact test then sees that obstacle for
// every probe, as without the filter.  Axes past the workspace list every
// obstacle in every bin.
constexpr int kGridBuildThreads = 3 * kGridCells;  // one (axis, bin) cell per thread

__device__ __forceinline__ void build_grid_block(const SceneParams &S, int wdim, float r_max, ObsGrid *G) {
    __shared__ float lo_s[kGridMaxObs][3], hi_s[kGridMaxObs][3];
    __shared__ int wild_s[kGridMaxObs];
    __shared__ int2 span_s[3][kGridMaxObs];  // bins listed for obstacle o on each axis
    __shared__ int bad_s;
    const int n = S.n_sph + S.n_box;  // <= kGridMaxObs (checked by the launcher)
    const int tid = threadIdx.x;
    if (tid == 0) bad_s = 0;
    if (tid < n) {
        float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f}, rho;
        if (tid < S.n_sph) {
            const float *c = S.sph + (wdim + 1) * tid;
            for (int i = 0; i < wdim; ++i) lo[i] = hi[i] = c[i];
            rho = c[wdim];
        } else {
            const float *bx = S.box + 2 * wdim * (tid - S.n_sph);
            for (int i = 0; i < wdim; ++i) {
                lo[i] = bx[i] - bx[wdim + i];
                hi[i] = bx[i] + bx[wdim + i];
            }
            rho = 0.f;
        }
        G->rec[tid][0] = make_float4(lo[0], lo[1], lo[2], rho);
        // the exact test's starting gap -R^2 for probes of radius r_max,
        // formed as the test forms it (R = rho + r, gap = -R R)
        const float Rr = rho + r_max;
        G->rec[tid][1] = make_float4(hi[0], hi[1], hi[2], -Rr * Rr);
        const float ext = (__builtin_fabsf(rho) + r_max) * (1.f + 0x1p-12f);
        bool wild = !__builtin_isfinite(ext);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            lo_s[tid][i] = lo[i] - ext;
            hi_s[tid][i] = hi[i] + ext;
            wild = wild || !__builtin_isfinite(lo[i] - ext) || !__builtin_isfinite(hi[i] + ext);
        }
        wild_s[tid] = wild ? 1 : 0;
    }
    __syncthreads();
    if (tid < 3 * kWave) {  // one wave per axis: the extent of the finite obstacles
        const int ax = tid / kWave, l = tid % kWave;
        float a = __builtin_inff(), b = -__builtin_inff();
        for (int o = l; o < n; o += kWave)
            if (!wild_s[o]) {
                a = __builtin_fminf(a, lo_s[o][ax]);
                b = __builtin_fmaxf(b, hi_s[o][ax]);
            }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            a = __builtin_fminf(a, __shfl_xor(a, off));
            b = __builtin_fmaxf(b, __shfl_xor(b, off));
        }
        if (!(a <= b)) {  // no finite obstacle
            a = 0.f;
            b = 1.f;
        }
        // [a, b] -> f in [1, 254], the obstacles (four bins in) in about [5, 250]
        constexpr float kSpan = (float)(kGridCells - 3);
        const float scale = __builtin_fmaxf(1.f, __builtin_fmaxf(__builtin_fabsf(a), __builtin_fabsf(b)));
        const float span = __builtin_fmaxf(b - a, 1e-6f * scale);
        const float pad = span * (4.f / kSpan);
        a -= pad;
        b += pad;
        const float inv = kSpan / (b - a);
        const float off = __builtin_fmaf(-a, inv, 1.f);
        if (l == 0) {
            if (!__builtin_isfinite(inv) || !__builtin_isfinite(off) || !(inv > 0.f)) bad_s = 1;
            G->inv[ax] = inv;
            G->off[ax] = off;
        }
        for (int o = l; o < n; o += kWave) {  // the obstacle's bins on this axis, one bin wider on each side
            int2 sp = make_int2(0, kGridCells - 1);  // non-finite obstacle or axis past the workspace: every bin
            if (!wild_s[o] && ax < wdim) {
                sp.x = (int)grid_bin(__builtin_fmaf(lo_s[o][ax], inv, off)) - 1;
                sp.y = (int)grid_bin(__builtin_fmaf(hi_s[o][ax], inv, off)) + 1;
                sp.x = sp.x < 1 ? 1 : sp.x;
                sp.y = sp.y > kGridCells - 2 ? kGridCells - 2 : sp.y;
            }
            span_s[ax][o] = sp;
        }
    }
    if (tid == 3 * kWave) {
        G->inv[3] = 0.f;
        G->off[3] = 0.f;
    }
    __syncthreads();
    const int ax = tid / kGridCells, bin = tid - ax * kGridCells;
    uint32_t w[3] = {0u, 0u, 0u};
    const bool all = bad_s != 0;
    for (int o = 0; o < n; ++o) {
        const int2 sp = span_s[ax][o];
        if (all || (bin >= sp.x && bin <= sp.y)) w[o >> 5] |= 1u << (o & 31);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) G->mask[k][ax][bin] = w[k];
}

// Collision of one arm state through the obstacle bins (G in LDS; inv / off
// the bin maps of G held in registers).  For every robot sphere k (centre c,
// radius r_k) the obstacles of its bin masks are tested exactly as the full
// test does, R = rho_o + r_k, gap = -R^2 + sum_i (c_i - med3(c_i, lo_i, hi_i))^2
// in that order, and the state collides iff some gap is <= 0.
//
// Few spheres of a wave have a non-empty mask, so the exact tests are not
// made where the masks are found: each such sphere is appended to the wave's
// queue Qw in LDS (centre, mask, owning lane and sphere index), and whenever
// 64 entries are waiting the wave takes the 64 newest one per lane, which
// keeps every lane busy in the tests.  A lane appends nothing more once a
// drained test has found its state in contact, and a lane that is not `live`
// appends nothing at all (its result is then meaningless).  `tests` counts
// the exact tests of the whole wave, one popcount per round of the test loop:
// a wave-uniform total held in a scalar register (a per-lane count would take
// vector registers in the hot loop).
// Every lane of the wave must call this (it drains on ballots), and Qw should
// be addressed through a wave-uniform index, so that the queue's addresses
// stay in scalar registers.
constexpr int kQueue = 128;  // entries per wave: up to 63 waiting plus one probe of every lane

template <int WORDS>
struct GridQueue {
    // one array per field: the centre with the first mask word beside it in
    // one 16-byte entry (one store per probe; 2,372 bytes per wave with one
    // mask word)
    float4 c[kQueue];                                                // centre x, y, z; mask word 0 (bits)
    uint32_t m[WORDS > 1 ? WORDS - 1 : 1][WORDS > 1 ? kQueue : 1];  // mask words 1 ..
    uint16_t own[kQueue];                                            // owning lane | probe index << 8
    uint8_t hit[kWave];
};

typedef uint32_t GridMaskTable[3][kGridCells];  // one mask word: axis, bin

// The wave's side of the queue: probes are offered one per lane at a time
// (every lane of the wave takes part in each offer and drain).  Entries
// [0, tail) are waiting; a drain takes the newest 64 (the order of the tests
// does not matter: a lane collides iff any of its tests finds contact), so
// the queue needs no ring index.  rad(k) is the radius of probe k; UNI: every
// probe has the radius the bins were built for (r_max), whose starting gap
// the obstacle record holds, and entries carry no probe index.
template <int WORDS, bool UNI, class Rad>
struct GridProber {
    GridQueue<WORDS> &Q;
    const float4 (*rec)[2];
    uint32_t &tests;
    const Rad &rad;
    uint32_t tail;        // wave-uniform: entries waiting
    uint32_t hit;         // 1: this lane's state is in contact (known from a drain); an integer,
                          // not a bool, so that it stays a plain register across the loops
    uint64_t done;        // wave-uniform: the lanes that offer nothing more (hit, or not live)

    __device__ __forceinline__ GridProber(GridQueue<WORDS> &q, const float4 (*r)[2], uint32_t &t, const Rad &rd,
                                          bool live)
        : Q(q), rec(r), tests(t), rad(rd), tail(0), hit(live ? 0u : 1u), done(ballot(!live)) {
        Q.hit[lane_id()] = 0;
    }

    // Entries [first, first + n), n <= 64, one per lane.
    __device__ __forceinline__ void drain(uint32_t first, uint32_t n) {
        const int lane = lane_id();
        __builtin_amdgcn_wave_barrier();
        // words 0-1 as one 32- or 64-bit mask, word 2 beside it
        typedef typename std::conditional<WORDS == 1, uint32_t, uint64_t>::type Mask;
        Mask m = 0;
        uint32_t m2 = 0;
        float4 e = make_float4(0.f, 0.f, 0.f, 0.f);
        float pr = 0.f;
        int own = 0;
        if ((uint32_t)lane < n) {
            e = (&Q.c[first])[lane];
            const uint32_t w0 = __float_as_uint(e.w);
            if constexpr (WORDS == 1) m = (Mask)w0;
            else m = (Mask)(((uint64_t)(&Q.m[0][first])[lane] << 32) | w0);
            if constexpr (WORDS > 2) m2 = (&Q.m[WORDS > 2 ? 1 : 0][first])[lane];
            const uint32_t o = (&Q.own[first])[lane];
            own = (int)(o & 0xffu);
            if constexpr (!UNI) pr = rad(o >> 8);
        }
        for (;;) {
            const uint64_t act = ballot(m != 0 || m2 != 0);
            if (act == 0) break;
            tests += (uint32_t)__popcll(act);
            if (m != 0 || m2 != 0) {
                int o;
                if (m != 0) {
                    o = WORDS == 1 ? __builtin_ctz((uint32_t)m) : __builtin_ctzll((uint64_t)m);
                    m &= m - 1;
                } else {
                    o = 64 + __builtin_ctz(m2);
                    m2 &= m2 - 1;
                }
                const float4 a = rec[o][0], h = rec[o][1];
                float g;
                if constexpr (UNI) {
                    (void)pr;
                    g = h.w;
                } else {
                    const float Rr = a.w + pr;
                    g = -Rr * Rr;
                }
                const float c[3] = {e.x, e.y, e.z}, lo[3] = {a.x, a.y, a.z}, hi[3] = {h.x, h.y, h.z};
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const float dlt = c[i] - __builtin_amdgcn_fmed3f(c[i], lo[i], hi[i]);
                    g = __builtin_fmaf(dlt, dlt, g);
                }
                if (g <= 0.f) {
                    Q.hit[own] = 1;
                    m = 0;
                    m2 = 0;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        hit |= Q.hit[lane] != 0 ? 1u : 0u;
        done = ballot(hit != 0);
    }

    // This lane's probe k (bin mask words mw; centre(c) writes its centre,
    // evaluated only for a queued probe): queued when some obstacle is listed
    // and the lane's state is not known to collide.  The lanes to queue are
    // found as one wave-wide mask (the compare's own lane mask less `done`),
    // which is also the branch condition, so the common case of no lane
    // queueing costs one vector compare.
    template <class C>
    __device__ __forceinline__ void offer(const uint32_t (&mw)[WORDS], uint32_t k, C &&centre) {
        uint32_t any = mw[0];
#pragma unroll
        for (int wd = 1; wd < WORDS; ++wd) any |= mw[wd];
        const uint64_t wmask = ballot(any != 0) & ~done;
        if (wmask != 0) {
            if (__builtin_amdgcn_inverse_ballot_w64(wmask)) {  // any != 0 && hit == 0 in this lane
                float c[3];
                centre(c);
                const int r = rank_in(wmask);
                (&Q.c[tail])[r] = make_float4(c[0], c[1], c[2], __uint_as_float(mw[0]));
#pragma unroll
                for (int wd = 1; wd < WORDS; ++wd) (&Q.m[wd - 1][tail])[r] = mw[wd];
                (&Q.own[tail])[r] = (uint16_t)(UNI ? (uint32_t)lane_id() : (uint32_t)lane_id() | k << 8);
            }
            tail += (uint32_t)__popcll(wmask);
            if (tail >= (uint32_t)kWave) {
                tail -= (uint32_t)kWave;
                drain(tail, kWave);
            }
        }
    }

    __device__ __forceinline__ bool finish() {
        if (tail != 0) drain(0, tail);
        return hit != 0;
    }
};

// mk: the mask tables (mk[w] = word w), rec: the obstacle records; both may
// live in LDS or in device memory.  The bin coordinate of a sphere centre
// c = b + t (p - b) on axis i is taken as f = fp_i + (t - 1) (fp_i - fb_i),
// fb and fp the bin coordinates of the link's ends (o_{L-1} and o_L, each
// formed once: o_L's serves as the next link's fb); it differs from the
// coordinate of the FP32 centre, c_i inv_i + off_i, by rounding only (below
// 1e-4 of a bin for any centre within the bins' span), and every obstacle's
// bin interval is widened by a bin on each side, so the bins still list
// every obstacle the exact test can find in contact.  The centre itself,
// fma(t, p - b, b) as the full test forms it, is formed only for the
// spheres queued for an exact test.
template <int WORDS, bool UNI = false, class AP>
__device__ __forceinline__ bool arm_hit_grid(const AP &R, const float (&q)[GTMP_MAX_JOINTS],
                                             const GridMaskTable *mk, const float4 (*rec)[2],
                                             const float (&inv)[3], const float (&off)[3],
                                             GridQueue<WORDS> &Qw, uint32_t &tests, bool live) {
    // the radius of a queued sphere, read per lane when its tests are drained
    const auto rad = [&](uint32_t k) { return R.r[k]; };
    GridProber<WORDS, UNI, decltype(rad)> P(Qw, rec, tests, rad, live);
    float fb[3] = {off[0], off[1], off[2]};  // o_0 = 0
    arm_fk_visit<GTMP_MAX_JOINTS>(R, q, [&](int L, const float (&b)[3], const float (&p)[3]) {
        float fp[3], fd[3], d[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            fp[i] = __builtin_fmaf(p[i], inv[i], off[i]);
            fd[i] = fp[i] - fb[i];
            d[i] = p[i] - b[i];
            // formed once per link: kept in registers rather than re-formed
            // in every iteration of the sphere loop below
            asm volatile("" : "+v"(fp[i]), "+v"(fd[i]), "+v"(d[i]));
        }
        const int kl = L == 1 ? 0 : R.lk_end[L - 2];
        const int k0 = kl > R.k_first ? kl : R.k_first;  // spheres below k_first reach no obstacle
        const int k1 = R.lk_end[L - 1];
        // unsigned index: the parameter address is a plain increment
        for (uint32_t k = (uint32_t)k0; k < (uint32_t)k1; ++k) {
            const float tm = R.tm1[k];
            uint32_t bin[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) bin[i] = grid_bin(__builtin_fmaf(tm, fd[i], fp[i]));
            uint32_t mw[WORDS];
#pragma unroll
            for (int wd = 0; wd < WORDS; ++wd) mw[wd] = mk[wd][0][bin[0]] & mk[wd][1][bin[1]] & mk[wd][2][bin[2]];
            P.offer(mw, k, [&](float (&c)[3]) {
                const float t = R.t[k];
#pragma unroll
                for (int i = 0; i < 3; ++i) c[i] = __builtin_fmaf(t, d[i], b[i]);
            });
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) fb[i] = fp[i];
    });
    return P.finish();
}

// Collision of SP point states of dimension W (radius 0) through the obstacle
// bins: the obstacles their W bin masks list, tested exactly as the full test
// does (R = rho_o, gap = -R^2 + sum_i (p_i - med3(p_i, lo_i, hi_i))^2, the
// third axis of a 2D state at 0 on both sides, which adds nothing); true when
// some state is in contact.  and_mask(i, bin, mw) ANDs the mask words of
// bin `bin` on axis i into mw.  Every lane of the wave must call this.
template <int W, int SP, int WORDS, class AndMask>
__device__ __forceinline__ bool point_hit_grid_by(const float (&p)[W][SP], const AndMask &and_mask,
                                                  const float4 (*rec)[2], const float (&inv)[3],
                                                  const float (&off)[3], GridQueue<WORDS> &Qw, uint32_t &tests,
                                                  bool live) {
    const auto rad = [](uint32_t) { return 0.f; };
    GridProber<WORDS, true, decltype(rad)> P(Qw, rec, tests, rad, live);
#pragma unroll
    for (int s = 0; s < SP; ++s) {
        float c[3] = {0.f, 0.f, 0.f};
        uint32_t bin[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            c[i] = p[i][s];
            bin[i] = grid_bin(__builtin_fmaf(c[i], inv[i], off[i]));
        }
        uint32_t mw[WORDS];
#pragma unroll
        for (int wd = 0; wd < WORDS; ++wd) mw[wd] = ~0u;
#pragma unroll
        for (int i = 0; i < W; ++i) and_mask(i, bin[i], mw);
        P.offer(mw, 0u, [&](float (&o)[3]) {
#pragma unroll
            for (int i = 0; i < 3; ++i) o[i] = c[i];
        });
    }
    return P.finish();
}

// The masks with one cell's words side by side (one vector read per axis),
// for AX >= W axes.
template <int W, int SP, int WORDS, int AX>
__device__ __forceinline__ bool point_hit_grid(const float (&p)[W][SP],
                                               const uint32_t (&pm)[AX][kGridCells][point_mask_stride<WORDS>()],
                                               const float4 (*rec)[2], const float (&inv)[3],
                                               const float (&off)[3], GridQueue<WORDS> &Qw, uint32_t &tests,
                                               bool live) {
    auto and_mask = [&](int i, uint32_t bin, uint32_t (&mw)[WORDS]) {
        const uint32_t *cell = pm[i][bin];
        if constexpr (WORDS == 3) {
            const uint4 v = *reinterpret_cast<const uint4 *>(cell);
            mw[0] &= v.x;
            mw[1 % WORDS] &= v.y;
            mw[2 % WORDS] &= v.z;
        } else if constexpr (WORDS == 2) {
            const uint2 v = *reinterpret_cast<const uint2 *>(cell);
            mw[0] &= v.x;
            mw[1 % WORDS] &= v.y;
        } else {
            mw[0] &= cell[0];
        }
    };
    return point_hit_grid_by<W, SP, WORDS>(p, and_mask, rec, inv, off, Qw, tests, live);
}

// The masks in the grid's own layout (mk[w] = word w).
template <int W, int SP, int WORDS>
__device__ __forceinline__ bool point_hit_grid(const float (&p)[W][SP], const GridMaskTable *mk,
                                               const float4 (*rec)[2], const float (&inv)[3],
                                               const float (&off)[3], GridQueue<WORDS> &Qw, uint32_t &tests,
                                               bool live) {
    auto and_mask = [&](int i, uint32_t bin, uint32_t (&mw)[WORDS]) {
#pragma unroll
        for (int wd = 0; wd < WORDS; ++wd) mw[wd] &= mk[wd][i][bin];
    };
    return point_hit_grid_by<W, SP, WORDS>(p, and_mask, rec, inv, off, Qw, tests, live);
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

// Row info of row, given m = (row - 1) / N for an inner row (ignored for the
// others): a walk over consecutive rows carries m instead of dividing.
__device__ __forceinline__ RowInfo decode_row_m(const EdgeArgs &A, uint32_t row, uint32_t m) {
    RowInfo r;
    const uint32_t N = (uint32_t)A.N;
    const uint32_t inner_rows = (uint32_t)(A.M - 1) * N;
    if (row == 0) {
        r.u_base = 0; r.u_step = 0; r.v_base = 1; r.v_step = 1;
        r.e_base = 0; r.e_step = 1; r.c_base = A.C_s; r.c_step = 1;
    } else if (row <= inner_rows) {
        const uint32_t ri = row - 1;       // = m N + u
        r.u_base = row; r.u_step = 0;
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

// Vertex ids (u, v) of flat edge e (C_s | C_h | C_l order, rows as above);
// 32-bit arithmetic: every edge id and N^2 are below 2^32.
__device__ __forceinline__ void edge_vertex_ids(const EdgeArgs &A, uint32_t e, uint32_t &u, uint32_t &v) {
    const uint32_t N = (uint32_t)A.N, NN = N * N;
    const uint32_t inner = (uint32_t)(A.M - 1) * NN;
    if (e < N) {
        u = 0;
        v = 1 + e;
    } else if (e - N < inner) {
        const uint32_t r = e - N, m = r / NN, uv = r - m * NN, a = uv / N;
        u = 1 + m * N + a;
        v = 1 + (m + 1) * N + (uv - a * N);
    } else {
        const uint32_t r = e - N - inner, n = r / (uint32_t)A.G, g = r - n * (uint32_t)A.G;
        u = 1 + (uint32_t)(A.M - 1) * N + n;
        v = 1 + (uint32_t)A.M * N + g;
    }
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

// Square root of an edge's squared length: the hardware square root (within
// one ulp; every kernel that writes an edge length takes it, so the lengths
// agree bit for bit between them).
__device__ __forceinline__ float len_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Euclidean length in configuration space (FP32, fixed summation order so
// that the pre-pass and the interior kernel produce the same value).  The
// coordinates past d are zero in both endpoints (the packed vertex array and
// every caller fill them with zeros), so all D are summed: a zero difference
// leaves the sum exactly as it is.
template <int D>
__device__ __forceinline__ float edge_len(const float (&u)[D], const float (&v)[D], int d) {
    (void)d;
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const float t = v[i] - u[i];
        acc = __builtin_fmaf(t, t, acc);
    }
    return len_sqrt(acc);
}

__device__ __forceinline__ float failed_cost(float len, float penalty) { return len + penalty; }

// ------------------------------------------------------------------ pre-pass
// Takes x as read here: a load of x still in flight is waited for at this
// point (inside a branch that loaded it) rather than where the branches
// meet, where the wait would also cover every store issued before it.
template <int D>
__device__ __forceinline__ void settle(float (&x)[D]) {
#pragma unroll
    for (int i = 0; i < D; ++i) asm volatile("" : "+v"(x[i]));
}
__device__ __forceinline__ void settle(uint32_t &x) { asm volatile("" : "+v"(x)); }

// One block per (A.prepass_rows <= kPrepassRows consecutive rows, row
// segment): thread i takes column seg * kTile + i of every row.  Consecutive
// rows of a layer share their target vertices, so a thread loads its target
// once and reuses it while the rows' targets stay the same; the per-tile
// compaction of all the rows shares one barrier.  A row whose source vertex
// is the same for every column (all but the goal rows) reads it from LDS,
// where the block stages the sources of all its rows at once before the
// rows are costed: the block waits for memory once, not once per row.  Small
// graphs take one row per block (more blocks in flight).
constexpr int kPrepassRows = 8;
constexpr uint32_t kPrepassRowsMinTiles = 4096;  // graphs from this size take kPrepassRows rows per block

// Rows per pre-pass block of a graph of n_tiles tiles, and the blocks of a
// plan's pre-pass.
__host__ __device__ inline uint32_t prepass_rows_for(uint32_t n_tiles) {
    return n_tiles >= kPrepassRowsMinTiles ? (uint32_t)kPrepassRows : 1u;
}
__host__ __device__ inline uint32_t prepass_block_count(const EdgeArgs &A) {
    const uint32_t rows = A.n_tiles / A.tiles_per_row;
    return ((rows + A.prepass_rows - 1) / A.prepass_rows) * A.tiles_per_row;
}

// Pre-pass block b of a plan (blocks of kTile threads).
template <int D>
__device__ __forceinline__ void prepass_block(const EdgeArgs &A, uint32_t b) {
    static_assert(kTile / kWave == 4, "one 16-byte read of a row's wave counts");
    __shared__ __align__(16) uint32_t wave_cnt[kPrepassRows][kTile / kWave];
    __shared__ float src_x[kPrepassRows][D];  // uniform source vertex of each row
    __shared__ uint8_t src_fl[kPrepassRows];
    static_assert(kPrepassRows * D <= kTile, "one staging thread per source coordinate");
    const int w = threadIdx.x / kWave;
    const uint32_t seg = b % A.tiles_per_row;
    const uint32_t row0 = (b / A.tiles_per_row) * A.prepass_rows;
    const uint32_t rows = A.n_tiles / A.tiles_per_row;
    const uint32_t n = seg * kTile + threadIdx.x;
    const bool col = n < (uint32_t)A.N;
    uint32_t candbits = 0;
    float v[D];
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = 0.f;
    uint32_t vfl = 0;
    // Layer of the block's first inner row (one division per block; the rows
    // after it step m on when they cross into the next layer).
    const uint32_t N = (uint32_t)A.N, inner_rows = (uint32_t)(A.M - 1) * N;
    uint32_t m = (row0 > 0 ? row0 - 1 : 0) / N;
    // Target of the first row (issued before the staging loads, so that both
    // are in flight together).
    const RowInfo ri0 = decode_row_m(A, row0, m);
    uint32_t vb = ri0.v_base, vs = ri0.v_step;  // target pattern of the loaded v
    if (col) {
        const uint32_t vid = vb + n * vs;
        load_vertex<D>(A, vid, v);
        vfl = A.vflag[vid];
    }
    {
        // The source of row 0 and of every inner row is vertex id = row.
        const uint32_t r = threadIdx.x / D, j = threadIdx.x % D, row = row0 + r;
        if (r < (uint32_t)A.prepass_rows && row < rows && row <= inner_rows) {
            const float x = A.verts[(size_t)row * A.dp + j];
            const uint8_t f = j == 0 ? A.vflag[row] : 0;
            src_x[r][j] = x;
            if (j == 0) src_fl[r] = f;
        }
    }
    settle<D>(v);
    settle(vfl);
    __syncthreads();
    // Cost and flag of edge e (source u, target v), written through cp;
    // whether its interior still has to be checked.
    auto cost_edge = [&](const float (&u)[D], uint32_t ufl, uint64_t e, float *cp) -> bool {
        const float len = edge_len<D>(u, v, A.d);
        bool failed = (ufl | vfl) != 0 || len > A.max_len;
        if (A.prune) failed = failed || A.prune[e] != 0;
        *cp = failed_cost(len, A.penalty);
        if (A.flags) A.flags[e] = 1;
        return !failed;
    };
    const uint32_t last = row0 + kPrepassRows - 1;
    if (A.prepass_rows == kPrepassRows && row0 > 0 && last <= inner_rows && last - 1 < (m + 1) * N) {
        // Every row an inner row of layer m: sources staged, one target, the
        // row's costs N apart.
        const size_t off0 = (size_t)(row0 - 1) * N + n;
#pragma unroll
        for (int r = 0; r < kPrepassRows; ++r) {
            bool cand = false;
            if (col) {
                float u[D];
#pragma unroll
                for (int i = 0; i < D; ++i) u[i] = src_x[r][i];
                const size_t off = off0 + (size_t)r * N;
                cand = cost_edge(u, src_fl[r], (uint64_t)N + off, A.C_h + off);
            }
            candbits |= (cand ? 1u : 0u) << r;
            const uint64_t mask = ballot(cand);
            if (lane_id() == 0) wave_cnt[r][w] = (uint32_t)__popcll(mask);
        }
    } else {
#pragma unroll
        for (int r = 0; r < kPrepassRows; ++r) {
            const uint32_t row = row0 + r;
            if (r >= A.prepass_rows || row >= rows) break;
            while (row > 0 && row - 1 >= (m + 1) * N) ++m;
            const RowInfo ri = decode_row_m(A, row, m);
            bool cand = false;
            if (ri.v_base != vb || ri.v_step != vs) {
                vb = ri.v_base;
                vs = ri.v_step;
                if (col) {
                    const uint32_t vid = vb + n * vs;
                    load_vertex<D>(A, vid, v);
                    vfl = A.vflag[vid];
                    settle<D>(v);
                    settle(vfl);
                }
            }
            if (col) {
                float u[D];
                uint32_t ufl;
                if (ri.u_step == 0) {
#pragma unroll
                    for (int i = 0; i < D; ++i) u[i] = src_x[r][i];
                    ufl = src_fl[r];
                } else {
                    const uint32_t uid = ri.u_base + n * ri.u_step;
                    load_vertex<D>(A, uid, u);
                    ufl = A.vflag[uid];
                    settle<D>(u);
                    settle(ufl);
                }
                cand = cost_edge(u, ufl, ri.e_base + (uint64_t)n * ri.e_step, ri.c_base + (size_t)n * ri.c_step);
            }
            candbits |= (cand ? 1u : 0u) << r;
            const uint64_t mask = ballot(cand);
            if (lane_id() == 0) wave_cnt[r][w] = (uint32_t)__popcll(mask);
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPrepassRows; ++r) {
        const uint32_t row = row0 + r;
        if (r >= A.prepass_rows || row >= rows) break;
        const uint32_t tile = row * A.tiles_per_row + seg;
        const uint4 c4 = *reinterpret_cast<const uint4 *>(wave_cnt[r]);
        const uint32_t cnt[kTile / kWave] = {c4.x, c4.y, c4.z, c4.w};
        uint32_t base = 0, total = 0;
#pragma unroll
        for (int k = 0; k < kTile / kWave; ++k) {
            if (k < w) base += cnt[k];
            total += cnt[k];
        }
        const bool cand = (candbits >> r) & 1u;
        const uint64_t mask = ballot(cand);
        if (cand) A.tile_off[(size_t)tile * kTile + base + rank_in(mask)] = (uint8_t)threadIdx.x;
        if (threadIdx.x == 0) A.tile_cnt[tile] = total;
    }
}


// ------------------------------------------------------------------ robot adapters
// Point robot in R^W: a state is one probe of radius 0.  Arm: a state is KP
// probes (the collision spheres) obtained by forward kinematics.
template <int W, int S>
struct PointModel {
    static constexpr bool kArm = false;
    static constexpr bool kGrid = false;
    static constexpr int kWords = 0;
    static constexpr int D = W;
    static constexpr int KP = S;  // probes per evaluation = S states
};

template <int KPm>
struct ArmModel {
    static constexpr bool kArm = true;
    static constexpr bool kGrid = false;
    static constexpr int kWords = 0;
    static constexpr int D = GTMP_MAX_JOINTS;
    static constexpr int KP = KPm;
};

// Arm states tested through the obstacle bins (WORDS 32-bit mask words: up to
// 32 WORDS obstacles).
template <int WORDS>
struct ArmGridModel {
    static constexpr bool kArm = true;
    static constexpr bool kGrid = true;
    static constexpr int kWords = WORDS;
    static constexpr int D = GTMP_MAX_JOINTS;
    static constexpr int KP = 1;
};

// Point states in R^W tested through the obstacle bins, S states per
// evaluation (WORDS mask words).
template <int W, int S, int WORDS>
struct PointGridModel {
    static constexpr bool kArm = false;
    static constexpr bool kGrid = true;
    static constexpr int kWords = WORDS;
    static constexpr int D = W;
    static constexpr int KP = S;
};


__device__ __forceinline__ float *cost_slot(const EdgeArgs &A, uint32_t e) {
    const uint32_t N = (uint32_t)A.N;
    const uint32_t inner_end = N + (uint32_t)(A.M - 1) * N * N;
    if (e < N) return A.C_s + e;
    if (e < inner_end) return A.C_h + (e - N);
    return A.C_l + (e - inner_end);
}

}  // namespace gtmp
