// sweep.hip -- backward min-plus value iteration over the layers (Sec. IV-B;
// Alg. 1) and extraction of the minimising chain.
//
// V[M-1][u] = min_g C_l[u][g] + V_g[g]
// V[m][u]   = min_v C_h[m][u][v] + V[m+1][v]     m = M-2 .. 0
// V_s       = min_u C_s[u] + V[0][u]
// Minimisers keep the lowest index among equal values; a row whose minimum is
// +inf stores -1.  Large layers are HBM bound (one read of C_h[m]): one wave
// per row streams the row with 16-byte loads beside the cache-resident
// V[m+1]; the (value, index) pair is reduced across the wave with a
// butterfly.  Small graphs run the whole recursion in one block.
#include "gtmp_launch.hpp"

namespace gtmp {

typedef float f4v __attribute__((ext_vector_type(4)));

struct Best {
    float v;
    int i;
};

__device__ __forceinline__ void take(Best &b, float v, int i) {
    if (v < b.v) { b.v = v; b.i = i; }
}

__device__ __forceinline__ Best wave_argmin(Best b) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const float ov = __shfl_xor(b.v, off);
        const int oi = __shfl_xor(b.i, off);
        if (ov < b.v || (ov == b.v && (unsigned)oi < (unsigned)b.i)) { b.v = ov; b.i = oi; }
    }
    return b;
}

// Minimum of row[v] + vn[v] over v in [0, n), lanes striding; each lane scans
// its elements in increasing index so strict < keeps the lowest index.
__device__ __forceinline__ Best row_argmin(const float *__restrict__ row, const float *vn, int n, int lane) {
    Best b{__builtin_inff(), -1};
    if ((n & 3) == 0 && ((reinterpret_cast<uintptr_t>(row) & 15) == 0)) {
        const f4v *r4 = reinterpret_cast<const f4v *>(row);
        const f4v *v4 = reinterpret_cast<const f4v *>(vn);
        const int n4 = n >> 2;
        int k = lane;
        for (; k + 3 * kWave < n4; k += 4 * kWave) {
            f4v c[4], w[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) c[t] = __builtin_nontemporal_load(r4 + k + t * kWave);
#pragma unroll
            for (int t = 0; t < 4; ++t) w[t] = v4[k + t * kWave];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int base = 4 * (k + t * kWave);
                take(b, c[t].x + w[t].x, base + 0);
                take(b, c[t].y + w[t].y, base + 1);
                take(b, c[t].z + w[t].z, base + 2);
                take(b, c[t].w + w[t].w, base + 3);
            }
        }
        for (; k < n4; k += kWave) {
            const f4v c = __builtin_nontemporal_load(r4 + k);
            const f4v w = v4[k];
            take(b, c.x + w.x, 4 * k + 0);
            take(b, c.y + w.y, 4 * k + 1);
            take(b, c.z + w.z, 4 * k + 2);
            take(b, c.w + w.w, 4 * k + 3);
        }
    } else {
        for (int v = lane; v < n; v += kWave) take(b, row[v] + vn[v], v);
    }
    return wave_argmin(b);
}

// ---------------------------------------------------------------- goal layer
__global__ void __launch_bounds__(256) k_goal_layer(int M, int N, int G, const float *__restrict__ C_l,
                                                    const float *__restrict__ Vg, float *V, int32_t *A) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= N) return;
    Best b{__builtin_inff(), -1};
    for (int g = 0; g < G; ++g) take(b, C_l[(size_t)u * G + g] + (Vg ? Vg[g] : 0.f), g);
    V[(size_t)(M - 1) * N + u] = b.v;
    A[(size_t)(M - 1) * N + u] = b.i;
}

// ---------------------------------------------------------------- inner layer
// V[m][u] for all u.  V[m+1] (N floats, read by every wave) is read straight
// from global memory, where it stays cache-resident: no staging barrier holds
// back the first loads of the streamed rows.
__global__ void __launch_bounds__(256) k_inner_layer(int m, int N, int rows_per_wave, const float *__restrict__ C_h,
                                                     float *V, int32_t *A) {
    const float *vn = V + (size_t)(m + 1) * N;
    const int lane = lane_id();
    const int wave = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int u0 = wave * rows_per_wave;
    for (int r = 0; r < rows_per_wave; ++r) {
        const int u = u0 + r;
        if (u >= N) break;
        const Best b = row_argmin(C_h + ((size_t)m * N + u) * N, vn, N, lane);
        if (lane == 0) {
            V[(size_t)m * N + u] = b.v;
            A[(size_t)m * N + u] = b.i;
        }
    }
}

// ---------------------------------------------------------------- start
__global__ void __launch_bounds__(1024) k_start(int N, const float *__restrict__ C_s, const float *__restrict__ V0,
                                                float *V_s, int32_t *a_s) {
    __shared__ float sv[1024 / kWave];
    __shared__ int si[1024 / kWave];
    Best b{__builtin_inff(), -1};
    for (int u = threadIdx.x; u < N; u += blockDim.x) take(b, C_s[u] + V0[u], u);
    // threads stride by blockDim: within a thread indices increase; across
    // threads the butterfly keeps the lowest index among equal values
    b = wave_argmin(b);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) { sv[w] = b.v; si[w] = b.i; }
    __syncthreads();
    if (threadIdx.x == 0) {
        Best r{__builtin_inff(), -1};
        const int nw = blockDim.x / kWave;
        for (int k = 0; k < nw; ++k)
            if (sv[k] < r.v || (sv[k] == r.v && (unsigned)si[k] < (unsigned)r.i)) { r.v = sv[k]; r.i = si[k]; }
        *V_s = r.v;
        *a_s = r.i;
    }
}

// ---------------------------------------------------------------- small graphs
// Whole recursion in one block of 256 threads; only for N <= 1024 (the
// value buffers below hold one layer of at most 1024 entries each).  When C_h fits
// (kSmallStage floats) the block first loads all of it into LDS in one
// parallel burst, so the rows of a layer are not each a dependent global
// load away.
constexpr int kSmallStage = 12288;

__global__ void __launch_bounds__(256) k_sweep_small(int M, int N, int G, const float *__restrict__ C_s,
                                                     const float *__restrict__ C_h, const float *__restrict__ C_l,
                                                     const float *__restrict__ Vg, float *V, int32_t *A, float *V_s,
                                                     int32_t *a_s, int staged) {
    __shared__ __align__(16) float buf[2][1024];
    __shared__ float sv[4];
    __shared__ int si[4];
    extern __shared__ float ch_lds[];
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    float *cur = buf[0];
    float *nxt = buf[1];
    if (staged) {
        // eight independent 16-byte loads per thread in flight before their
        // LDS stores (a load-store loop would wait on every load in turn)
        const int n = (M - 1) * N * N;
        const int n4 = n >> 2;
        const f4v *src = reinterpret_cast<const f4v *>(C_h);
        f4v *dst = reinterpret_cast<f4v *>(ch_lds);
        const bool vec = (reinterpret_cast<uintptr_t>(C_h) & 15) == 0;
        if (vec) {
            for (int base = 0; base < n4; base += 8 * 256) {
                f4v t[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int i = base + k * 256 + threadIdx.x;
                    if (i < n4) t[k] = src[i];
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int i = base + k * 256 + threadIdx.x;
                    if (i < n4) dst[i] = t[k];
                }
            }
        }
        for (int i = vec ? 4 * n4 + threadIdx.x : threadIdx.x; i < n; i += blockDim.x) ch_lds[i] = C_h[i];
    }
    for (int u = threadIdx.x; u < N; u += blockDim.x) {
        Best b{__builtin_inff(), -1};
        for (int g = 0; g < G; ++g) take(b, C_l[(size_t)u * G + g] + (Vg ? Vg[g] : 0.f), g);
        V[(size_t)(M - 1) * N + u] = b.v;
        A[(size_t)(M - 1) * N + u] = b.i;
        nxt[u] = b.v;
    }
    __syncthreads();
    // staged: tpr threads per row (consecutive lanes, a power of two), each
    // scanning its columns in increasing order, then a tpr-lane butterfly;
    // otherwise one wave per row streaming from global memory
    int lg = 0;
    while ((N << (lg + 1)) <= 256 && lg < 6) ++lg;
    const int tpr = 1 << lg, sub = threadIdx.x & (tpr - 1), rows_per_pass = 256 >> lg;
    for (int m = M - 2; m >= 0; --m) {
        if (staged) {
            for (int u0 = 0; u0 < N; u0 += rows_per_pass) {
                const int u = u0 + (threadIdx.x >> lg);
                Best b{__builtin_inff(), -1};
                if (u < N) {
                    const float *row = ch_lds + ((size_t)m * N + u) * N;
                    for (int v = sub; v < N; v += tpr) take(b, row[v] + nxt[v], v);
                }
                for (int off = tpr >> 1; off > 0; off >>= 1) {
                    const float ov = __shfl_xor(b.v, off);
                    const int oi = __shfl_xor(b.i, off);
                    if (ov < b.v || (ov == b.v && (unsigned)oi < (unsigned)b.i)) { b.v = ov; b.i = oi; }
                }
                if (u < N && sub == 0) {
                    V[(size_t)m * N + u] = b.v;
                    A[(size_t)m * N + u] = b.i;
                    cur[u] = b.v;
                }
            }
        } else {
            for (int u = w; u < N; u += 4) {
                const Best b = row_argmin(C_h + ((size_t)m * N + u) * N, nxt, N, lane);
                if (lane == 0) {
                    V[(size_t)m * N + u] = b.v;
                    A[(size_t)m * N + u] = b.i;
                    cur[u] = b.v;
                }
            }
        }
        __syncthreads();
        float *t = cur; cur = nxt; nxt = t;
    }
    Best b{__builtin_inff(), -1};
    for (int u = threadIdx.x; u < N; u += blockDim.x) take(b, C_s[u] + nxt[u], u);
    b = wave_argmin(b);
    if (lane == 0) { sv[w] = b.v; si[w] = b.i; }
    __syncthreads();
    if (threadIdx.x == 0) {
        Best r{__builtin_inff(), -1};
        for (int k = 0; k < 4; ++k)
            if (sv[k] < r.v || (sv[k] == r.v && (unsigned)si[k] < (unsigned)r.i)) { r.v = sv[k]; r.i = si[k]; }
        *V_s = r.v;
        *a_s = r.i;
    }
}

hipError_t launch_minplus(int M, int N, int G, const float *C_s, const float *C_h, const float *C_l,
                          const float *Vg, float *V, int32_t *A, float *V_s, int32_t *a_s, hipStream_t s) {
    // one block only while C_h fits its LDS: streamed from memory by a single
    // block the recursion is slower than a launch per layer (measured: M 4,
    // N 128 78 us against about 20; M 16, N 256 1.0 ms)
    // (N <= 1024: the block's two value buffers hold one layer each; at M = 1
    // the staging bound alone would admit any N)
    if (N <= 1024 && (long long)(M - 1) * N * N <= kSmallStage) {
        const int staged = 1;
        const size_t lds = staged ? sizeof(float) * (size_t)(M - 1) * N * N : 0;
        hipLaunchKernelGGL(k_sweep_small, dim3(1), dim3(256), lds, s, M, N, G, C_s, C_h, C_l, Vg, V, A, V_s, a_s,
                           staged);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_goal_layer, dim3((N + 255) / 256), dim3(256), 0, s, M, N, G, C_l, Vg, V, A);
    const int rows_per_wave = N >= 4096 ? 2 : 1;
    const int waves = (N + rows_per_wave - 1) / rows_per_wave;
    const int blocks = (waves + 3) / 4;
    for (int m = M - 2; m >= 0; --m)
        hipLaunchKernelGGL(k_inner_layer, dim3(blocks), dim3(256), 0, s, m, N, rows_per_wave, C_h, V, A);
    hipLaunchKernelGGL(k_start, dim3(1), dim3(1024), 0, s, N, C_s, V, V_s, a_s);
    return hipGetLastError();
}

// ---------------------------------------------------------------- extraction
// Chains of up to this many vertices are followed once into LDS and their
// waypoints copied by every lane at once; longer ones by one thread.
constexpr int kExtractChain = 4096;

__global__ void __launch_bounds__(64) k_extract(int M, int N, int G, int d, const int32_t *a_s, const int32_t *A,
                                                const float *V_s, const float *Q, const float *q0,
                                                const float *goals, int32_t *idx, float *wp, float *cost) {
    if (blockIdx.x != 0) return;
    if (M + 1 <= kExtractChain) {
        __shared__ int32_t chain[kExtractChain];
        __shared__ int ok_s;
        if (threadIdx.x == 0) {
            const float vs = *V_s;
            int i = *a_s;
            // a minimiser outside its layer can only come from inconsistent
            // inputs; it is reported as "no path" rather than followed
            bool ok = i >= 0 && i < N && vs < __builtin_inff();
            chain[0] = i;
            for (int m = 0; m < M && ok; ++m) {
                const int nxt = A[(size_t)m * N + i];
                ok = nxt >= 0 && nxt < (m + 1 < M ? N : G);
                i = nxt;
                chain[m + 1] = i;
            }
            ok_s = ok;
            *cost = ok ? vs : __builtin_inff();
        }
        __syncthreads();
        const bool ok = ok_s != 0;
        for (int m = threadIdx.x; m <= M; m += blockDim.x) idx[m] = ok ? chain[m] : -1;
        // waypoint k: row k / d of q0 | the chosen layer samples | the goal
        const int n_wp = (M + 2) * d;
        for (int k = threadIdx.x; k < n_wp; k += blockDim.x) {
            const int row = k / d, j = k - row * d;
            float x = __builtin_nanf("");
            if (ok) {
                if (row == 0) x = q0[j];
                else if (row <= M) x = Q[((size_t)(row - 1) * N + chain[row - 1]) * d + j];
                else x = goals[(size_t)chain[M] * d + j];
            }
            wp[k] = x;
        }
        return;
    }
    if (threadIdx.x != 0) return;
    const float vs = *V_s;
    int i = *a_s;
    *cost = vs;
    if (i < 0 || !(vs < __builtin_inff())) {
        for (int m = 0; m <= M; ++m) idx[m] = -1;
        for (int k = 0; k < (M + 2) * d; ++k) wp[k] = __builtin_nanf("");
        *cost = __builtin_inff();
        return;
    }
    bool ok = i < N;
    for (int m = 0; m < M && ok; ++m) {
        const int nxt = A[(size_t)m * N + i];
        ok = nxt >= 0 && nxt < (m + 1 < M ? N : G);
        i = ok ? nxt : 0;
    }
    if (!ok) {
        for (int m = 0; m <= M; ++m) idx[m] = -1;
        for (int k = 0; k < (M + 2) * d; ++k) wp[k] = __builtin_nanf("");
        *cost = __builtin_inff();
        return;
    }
    i = *a_s;
    for (int j = 0; j < d; ++j) wp[j] = q0[j];
    for (int m = 0; m < M; ++m) {
        idx[m] = i;
        for (int j = 0; j < d; ++j) wp[(size_t)(m + 1) * d + j] = Q[((size_t)m * N + i) * d + j];
        i = A[(size_t)m * N + i];
    }
    idx[M] = i;
    for (int j = 0; j < d; ++j) wp[(size_t)(M + 1) * d + j] = goals[(size_t)i * d + j];
}

hipError_t launch_extract(int M, int N, int G, int d, const int32_t *a_s, const int32_t *A, const float *V_s,
                          const float *Q, const float *q0, const float *goals, int32_t *idx, float *wp, float *cost,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_extract, dim3(1), dim3(64), 0, s, M, N, G, d, a_s, A, V_s, Q, q0, goals, idx, wp, cost);
    return hipGetLastError();
}

}  // namespace gtmp
