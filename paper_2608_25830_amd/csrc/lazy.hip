// lazy.hip -- lazy edge realisation on the layered graph (the lazy variant
// that realises only a subset of adjacent-layer pairs, named as future work
// in the paper's conclusion): every edge starts at its optimistic cost (its
// length; length + penalty when an endpoint collides or it is too long), and
// rounds of
//   backward sweep -> extraction -> stop if every edge of the path is known
//   -> forward sweep -> check the unknown edges whose best path through them
//      costs at most (1 + band) V_s, and those of the extracted path
// run until the extracted path holds only checked edges.  Checked costs are
// the true ones and unchecked costs are lower bounds, so the final path is
// optimal for the fully checked graph and its cost is the same FP32 number
// the full check gives (same edge costs, same summation order).
//
// Edge status (flags): 0 free, 1 failed, 0xFF not yet checked.
#include "edge_common.hpp"

namespace gtmp {

constexpr uint8_t kUnknown = 0xFF;

struct LazyArgs {
    int d, M, N, G;
    float penalty, max_len;
    const float *verts;    // packed vertices [1 + MN + G][vertex_stride]
    const uint8_t *vflag;  // vertex collision flags
    float *C_s, *C_h, *C_l;
    uint8_t *flags;
    const float *V, *F;  // cost-to-go [M][N], cost-from-start [M][N]
    const float *V_s;
    uint8_t *select;
    uint32_t *list;      // the round's selected edges (flat ids), counters[1] of them
    uint32_t *counters;  // [0] done, [1] edges selected this round, [2] unknown edges on the path
    unsigned long long *stats;  // optional: rounds, edges selected for checking
};

__device__ __forceinline__ void lazy_vertex_ids(const LazyArgs &A, uint64_t e, uint32_t &u, uint32_t &v, float *&c) {
    const uint64_t N = A.N, inner = (uint64_t)(A.M - 1) * N * N;
    if (e < N) {
        u = 0;
        v = 1 + (uint32_t)e;
        c = A.C_s + e;
    } else if (e - N < inner) {
        const uint64_t r = e - N, m = r / (N * N), uv = r - m * N * N;
        u = 1 + (uint32_t)(m * N + uv / N);
        v = 1 + (uint32_t)((m + 1) * N + uv % N);
        c = A.C_h + r;
    } else {
        const uint64_t r = e - N - inner, n = r / (uint64_t)A.G, g = r - n * A.G;
        u = 1 + (uint32_t)((A.M - 1) * N + n);
        v = 1 + (uint32_t)(A.M * N + g);
        c = A.C_l + r;
    }
}

// Optimistic costs: the length for edges with free endpoints (status
// unknown), the failed cost for the others.
__global__ void __launch_bounds__(256) k_lazy_init(LazyArgs A, uint64_t E) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    uint32_t u, v;
    float *c;
    lazy_vertex_ids(A, e, u, v, c);
    float a[GTMP_MAX_DOF], b[GTMP_MAX_DOF];
    for (int i = 0; i < GTMP_MAX_DOF; ++i) {
        a[i] = A.verts[(size_t)u * GTMP_MAX_DOF + i];
        b[i] = A.verts[(size_t)v * GTMP_MAX_DOF + i];
    }
    const float len = edge_len<GTMP_MAX_DOF>(a, b, A.d);
    const bool failed = (A.vflag[u] | A.vflag[v]) != 0 || len > A.max_len;
    *c = failed ? failed_cost(len, A.penalty) : len;
    A.flags[e] = failed ? 1 : kUnknown;
}

// Cost from the start: F[0][v] = C_s[v]; F[m+1][v] = min_u F[m][u] + C_h[m][u][v].
// Thread (v, chunk of kFwdChunk sources u) reads a coalesced column strip and
// folds its minimum into F with an integer atomic minimum: costs are
// non-negative, and the IEEE order of non-negative floats is the unsigned
// order of their bit patterns (the minimum is exact in any order).
constexpr int kFwdChunk = 64;

__global__ void k_lazy_forward_init(LazyArgs A, float *F) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t MN = (size_t)A.M * A.N;
    if (i >= MN) return;
    F[i] = i < (size_t)A.N ? A.C_s[i] : __builtin_inff();
}

__global__ void __launch_bounds__(256) k_lazy_forward(LazyArgs A, int m, float *F) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= A.N) return;
    const int u0 = blockIdx.y * kFwdChunk;
    const int u1 = u0 + kFwdChunk < A.N ? u0 + kFwdChunk : A.N;
    const float *Fp = F + (size_t)(m - 1) * A.N;
    const float *C = A.C_h + (size_t)(m - 1) * A.N * A.N;
    float best = __builtin_inff();
    for (int u = u0; u < u1; ++u) best = __builtin_fminf(best, Fp[u] + C[(size_t)u * A.N + v]);
    atomicMin(reinterpret_cast<unsigned int *>(F + (size_t)m * A.N + v), __float_as_uint(best));
}

// Done test: the extracted path idx[0..M] (vertex per layer, then the goal)
// has no unknown edge.  With no path (idx[0] < 0) the loop is done as well.
__global__ void k_lazy_done(LazyArgs A, const int32_t *idx) {
    if (threadIdx.x != 0) return;
    uint32_t unknown = 0;
    if (idx[0] >= 0) {
        const uint64_t N = A.N;
        unknown += A.flags[idx[0]] == kUnknown;
        for (int m = 0; m + 1 < A.M; ++m) {
            const uint64_t e = N + (uint64_t)m * N * N + (uint64_t)idx[m] * N + idx[m + 1];
            unknown += A.flags[e] == kUnknown;
        }
        const uint64_t e = N + (uint64_t)(A.M - 1) * N * N + (uint64_t)idx[A.M - 1] * A.G + idx[A.M];
        unknown += A.flags[e] == kUnknown;
    }
    A.counters[0] = unknown == 0 ? 1u : 0u;
    A.counters[1] = 0;
    A.counters[2] = unknown;
}

// Selection of the round: unknown edges whose best path through them (cost
// from the start + edge + cost to go) is at most thr = (1 + band) V_s, marked
// in select and appended to the round's list.  Each block walks its
// grid-stride range twice: first selecting and counting (one atomic per block
// reserves its part of the list), then writing its selected edges into that
// part in order (the list order is immaterial to the check).
__global__ void __launch_bounds__(256) k_lazy_select(LazyArgs A, uint64_t E, float band) {
    __shared__ uint32_t part[256 / kWave];
    __shared__ uint32_t base_s;
    const uint64_t N = A.N, inner = (uint64_t)(A.M - 1) * N * N;
    const float thr = (1.0f + band) * *A.V_s;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const int w = threadIdx.x / kWave;
    uint32_t cnt = 0;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += stride) {
        bool sel = false;
        if (A.flags[e] == kUnknown) {
            float t;
            if (e < N) {
                t = A.C_s[e] + A.V[e];
            } else if (e - N < inner) {
                const uint64_t r = e - N, m = r / (N * N), uv = r - m * N * N;
                t = (A.F[m * N + uv / N] + A.C_h[r]) + A.V[(m + 1) * N + uv % N];
            } else {
                const uint64_t r = e - N - inner, n = r / (uint64_t)A.G;
                t = A.F[(uint64_t)(A.M - 1) * N + n] + A.C_l[r];
            }
            sel = t <= thr;
        }
        A.select[e] = sel ? 1 : 0;
        cnt += sel ? 1u : 0u;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if (lane_id() == 0) part[w] = cnt;
    __syncthreads();
    uint32_t tot = 0;
#pragma unroll
    for (int k = 0; k < 256 / kWave; ++k) tot += part[k];
    if (tot == 0) return;  // uniform over the block
    if (threadIdx.x == 0) base_s = atomicAdd(&A.counters[1], tot);
    __syncthreads();
    // second walk: the block's selected edges in grid-stride order, each wave
    // placing its ballot after the earlier waves' of the same step
    uint32_t next = base_s;
    for (uint64_t e0 = (uint64_t)blockIdx.x * blockDim.x; e0 < E && next < base_s + tot; e0 += stride) {
        const uint64_t e = e0 + threadIdx.x;
        const bool sel = e < E && A.select[e] != 0;
        const uint64_t mask = ballot(sel);
        __syncthreads();  // part[] of the previous step has been read by every wave
        if (lane_id() == 0) part[w] = (uint32_t)__popcll(mask);
        __syncthreads();
        uint32_t before = 0, step = 0;
#pragma unroll
        for (int k = 0; k < 256 / kWave; ++k) {
            if (k < w) before += part[k];
            step += part[k];
        }
        if (sel) A.list[next + before + rank_in(mask)] = (uint32_t)e;
        next += step;
    }
}

// The unchecked edges of the extracted path always join the round's
// selection (their through-cost equals V_s only up to the rounding of a
// different summation order), so every round checks at least one edge.
__global__ void k_lazy_mark_path(LazyArgs A, const int32_t *idx) {
    if (threadIdx.x != 0 || idx[0] < 0) return;
    const uint64_t N = A.N;
    auto mark = [&](uint64_t e) {
        if (A.flags[e] == kUnknown && A.select[e] == 0) {
            A.select[e] = 1;
            A.list[A.counters[1]++] = (uint32_t)e;
        }
    };
    mark((uint64_t)idx[0]);
    for (int m = 0; m + 1 < A.M; ++m) mark(N + (uint64_t)m * N * N + (uint64_t)idx[m] * N + idx[m + 1]);
    mark(N + (uint64_t)(A.M - 1) * N * N + (uint64_t)idx[A.M - 1] * A.G + idx[A.M]);
}

__global__ void k_lazy_count(LazyArgs A) {
    if (threadIdx.x != 0) return;
    A.stats[0] += 1;
    A.stats[1] += A.counters[1];
}

// ------------------------------------------------------------------ host side
static size_t up256_l(size_t x) { return (x + 255) & ~size_t(255); }

LazyPlan make_lazy_plan(const gtmp_problem &p) {
    LazyPlan L{};
    const uint64_t N = p.N, M = p.M, G = p.G;
    const uint64_t E = N + (M - 1) * N * N + N * G;
    const EdgePlan ep = make_edge_plan(p);
    size_t off = 0;
    L.off_edge = off; off = up256_l(off + ep.total);
    L.off_F = off; off = up256_l(off + sizeof(float) * M * N);
    L.off_select = off; off = up256_l(off + E);
    L.off_list = off; off = up256_l(off + sizeof(uint32_t) * E);
    L.off_counters = off; off = up256_l(off + 256);
    L.total = off;
    return L;
}

hipError_t launch_plan_lazy(const gtmp_problem &p, const ArmParams *arm, const SceneParams &S, int wdim,
                            const float *q0, const float *goals, const float *Q, float *C_s, float *C_h, float *C_l,
                            uint8_t *flags, float *V, int32_t *Am, float *V_s, int32_t *a_s, int32_t *idx, float *wp,
                            float *cost, float band, int max_rounds, unsigned long long *stats,
                            const gtmp_edge_opts &eo, void *workspace, int *rounds_host, bool *done_host,
                            hipStream_t s) {
    const LazyPlan plan = make_lazy_plan(p);
    const EdgePlan ep = make_edge_plan(p);
    char *ws = static_cast<char *>(workspace);
    EdgeBuffers b{q0, goals, Q, C_s, C_h, C_l, nullptr, flags, nullptr, ws + plan.off_edge};
    const uint64_t E = (uint64_t)p.N + (uint64_t)(p.M - 1) * p.N * p.N + (uint64_t)p.N * p.G;
    LazyArgs A{};
    A.d = p.d; A.M = p.M; A.N = p.N; A.G = p.G;
    A.penalty = p.penalty; A.max_len = p.max_edge_len;
    A.verts = reinterpret_cast<const float *>(ws + plan.off_edge + ep.off_verts);
    A.vflag = reinterpret_cast<const uint8_t *>(ws + plan.off_edge + ep.off_vflag);
    A.C_s = C_s; A.C_h = C_h; A.C_l = C_l; A.flags = flags;
    A.V = V;
    float *F = reinterpret_cast<float *>(ws + plan.off_F);
    A.F = F;
    A.V_s = V_s;
    A.select = reinterpret_cast<uint8_t *>(ws + plan.off_select);
    A.list = reinterpret_cast<uint32_t *>(ws + plan.off_list);
    A.counters = reinterpret_cast<uint32_t *>(ws + plan.off_counters);
    A.stats = stats;
    gtmp_edge_opts o = eo;
    o.mode = GTMP_CHECK_FAST;
    o.ev_begin = o.ev_end = nullptr;
    hipError_t e = launch_edge_phases(ep, arm, S, wdim, b, o, s, nullptr, nullptr, nullptr, kPhaseVertices);
    if (e != hipSuccess) return e;
    const unsigned eb = (unsigned)((E + 255) / 256);
    hipLaunchKernelGGL(k_lazy_init, dim3(eb), dim3(256), 0, s, A, E);
    uint32_t done = 0;
    int r = 0;
    for (;;) {
        e = launch_minplus(p.M, p.N, p.G, C_s, C_h, C_l, nullptr, V, Am, V_s, a_s, s);
        if (e != hipSuccess) return e;
        e = launch_extract(p.M, p.N, p.G, p.d, a_s, Am, V_s, Q, q0, goals, idx, wp, cost, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_lazy_done, dim3(1), dim3(64), 0, s, A, idx);
        e = hipMemcpyAsync(&done, A.counters, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (done || r >= max_rounds) break;
        const unsigned nb = (unsigned)((p.N + 255) / 256), nc = (unsigned)((p.N + kFwdChunk - 1) / kFwdChunk);
        const size_t MN = (size_t)p.M * p.N;
        hipLaunchKernelGGL(k_lazy_forward_init, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, s, A, F);
        for (int m = 1; m < p.M; ++m) hipLaunchKernelGGL(k_lazy_forward, dim3(nb, nc), dim3(256), 0, s, A, m, F);
        const unsigned sb = eb < 8192u ? eb : 8192u;
        hipLaunchKernelGGL(k_lazy_select, dim3(sb), dim3(256), 0, s, A, E, band);
        hipLaunchKernelGGL(k_lazy_mark_path, dim3(1), dim3(64), 0, s, A, idx);
        e = launch_edge_phases(ep, arm, S, wdim, b, o, s, A.list, A.counters + 1, A.select, kPhaseEdges);
        if (e != hipSuccess) return e;
        if (stats) hipLaunchKernelGGL(k_lazy_count, dim3(1), dim3(64), 0, s, A);
        ++r;
    }
    *rounds_host = r;
    *done_host = done != 0;
    return hipGetLastError();
}

}  // namespace gtmp
