// surrogate.hip -- the learned collision surrogate: a ReLU MLP on Fourier
// features of the configuration, with BF16 weights and activations and FP32
// accumulation on the matrix cores (v_mfma_f32_32x32x16_bf16), its BCE loss,
// backward pass and Adam update, and its two uses: edge pruning at the
// midpoint probe and scoring of heuristic sample candidates.
//
// Every reduction runs in a fixed order (split-K partials summed in split
// order, column sums over fixed row chunks, wave reductions by butterfly), so
// results are reproducible run to run.
#include <algorithm>

#include "surrogate.hpp"

namespace gtmp {

// ------------------------------------------------------------------ layout
SurLayout sur_layout() {
    SurLayout L{};
    int o = 0;
    const int W = GTMP_SUR_WIDTH, I = GTMP_SUR_IN;
    L.W[0] = o; o += W * I;
    L.b[0] = o; o += W;
    for (int l = 1; l < 4; ++l) {
        L.W[l] = o; o += W * W;
        L.b[l] = o; o += W;
    }
    L.w5 = o; o += W;
    L.b5 = o; o += 1;
    L.total = o;
    return L;
}

// ------------------------------------------------------------------ BF16
__device__ __forceinline__ uint16_t f2bf(float f) {
    // round to nearest, ties to even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------------ features
// Round a double to the nearest BF16 value, ties to even, in one step (no
// intermediate FP32 rounding): keep 7 of the 52 mantissa bits.  Finite
// inputs inside the FP32 normal range or zero.
__device__ __forceinline__ uint16_t d2bf(double x) {
    uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint64_t drop = 45;  // 52 - 7 mantissa bits
    u += ((1ull << (drop - 1)) - 1) + ((u >> drop) & 1ull);
    u &= ~((1ull << drop) - 1);
    return (uint16_t)(__float_as_uint((float)__longlong_as_double((long long)u)) >> 16);
}

// One thread per configuration: [q/pi, sin(2 pi B q/pi), cos(2 pi B q/pi), 0...]
// in FP64, rounded to BF16 once, 64 values.  FP64 keeps the phases (up to a
// few tens of radians) accurate enough that the BF16 rounding of a feature
// does not depend on how its value was computed.
__global__ void __launch_bounds__(256) k_features(int d, int64_t n, const float *__restrict__ X,
                                                  const float *__restrict__ Bf, uint16_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr double kPi = 3.14159265358979323846;
    double qh[GTMP_MAX_DOF];
    for (int j = 0; j < GTMP_MAX_DOF; ++j) qh[j] = j < d ? (double)X[i * d + j] / kPi : 0.0;
    uint16_t v[GTMP_SUR_IN];
#pragma unroll
    for (int k = 0; k < GTMP_SUR_IN; ++k) v[k] = 0;
    for (int j = 0; j < d; ++j) v[j] = d2bf(qh[j]);
    for (int f = 0; f < GTMP_SUR_FREQ; ++f) {
        double s = 0.0;
        for (int j = 0; j < d; ++j) s += (double)Bf[f * d + j] * qh[j];
        s *= 2.0 * kPi;
        double sn, cs;
        sincos(s, &sn, &cs);
        v[d + f] = d2bf(sn);
        v[d + GTMP_SUR_FREQ + f] = d2bf(cs);
    }
    uint4 *dst = reinterpret_cast<uint4 *>(out + i * GTMP_SUR_IN);
#pragma unroll
    for (int q = 0; q < GTMP_SUR_IN / 8; ++q) {
        uint4 w;
        w.x = v[8 * q + 0] | ((uint32_t)v[8 * q + 1] << 16);
        w.y = v[8 * q + 2] | ((uint32_t)v[8 * q + 3] << 16);
        w.z = v[8 * q + 4] | ((uint32_t)v[8 * q + 5] << 16);
        w.w = v[8 * q + 6] | ((uint32_t)v[8 * q + 7] << 16);
        dst[q] = w;
    }
}

// ------------------------------------------------------------------ GEMM (NT)
// C[m][n] = sum_k A[m][k] B[n][k], A and B BF16 row-major with K contiguous,
// K a multiple of 32 (per split).  Block tile 128 x 128, four waves of
// 64 x 64 (2 x 2 MFMA 32x32x16 tiles), K step 32 staged through LDS.
enum GemmEpi { EPI_F32 = 0, EPI_BIAS_RELU_BF16 = 1, EPI_MASK_BF16 = 2 };

constexpr int kBM = 128, kBN = 128, kBK = 32, kLdsPad = 8;
constexpr int kLdsRow = kBK + kLdsPad;  // 40 BF16 = 80 bytes per row

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_nt(int M, int N, int K_split, const uint16_t *__restrict__ A, int lda,
                                                 const uint16_t *__restrict__ B, int ldb, void *__restrict__ Cout,
                                                 int ldc, const float *__restrict__ bias,
                                                 const uint16_t *__restrict__ mask, int ldm, size_t c_split_stride) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kBM * kLdsRow];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN * kLdsRow];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    const int k_begin = blockIdx.z * K_split;
    // global -> LDS: thread loads 16 BF16 (2 x 16 B) of one row of A and of B
    const int lr = tid >> 1, lk = (tid & 1) * 16;
    const bool a_ok = m0 + lr < M, b_ok = n0 + lr < N;
    const uint16_t *a_src = A + (size_t)(a_ok ? m0 + lr : 0) * lda + k_begin + lk;
    const uint16_t *b_src = B + (size_t)(b_ok ? n0 + lr : 0) * ldb + k_begin + lk;

    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

    const uint4 zero4 = make_uint4(0u, 0u, 0u, 0u);
    for (int k0 = 0; k0 < K_split; k0 += kBK) {
        const uint4 a0 = a_ok ? *reinterpret_cast<const uint4 *>(a_src + k0) : zero4;
        const uint4 a1 = a_ok ? *reinterpret_cast<const uint4 *>(a_src + k0 + 8) : zero4;
        const uint4 b0 = b_ok ? *reinterpret_cast<const uint4 *>(b_src + k0) : zero4;
        const uint4 b1 = b_ok ? *reinterpret_cast<const uint4 *>(b_src + k0 + 8) : zero4;
        __syncthreads();  // previous tile fully consumed
        *reinterpret_cast<uint4 *>(&As[lr * kLdsRow + lk]) = a0;
        *reinterpret_cast<uint4 *>(&As[lr * kLdsRow + lk + 8]) = a1;
        *reinterpret_cast<uint4 *>(&Bs[lr * kLdsRow + lk]) = b0;
        *reinterpret_cast<uint4 *>(&Bs[lr * kLdsRow + lk + 8]) = b1;
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kBK / 16; ++s) {
            const int kk = 16 * s + 8 * (lane >> 5);
            bf16x8 af[2], bfr[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int r = wm * 64 + 32 * i + (lane & 31);
                af[i] = *reinterpret_cast<const bf16x8 *>(&As[r * kLdsRow + kk]);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int r = wn * 64 + 32 * j + (lane & 31);
                bfr[j] = *reinterpret_cast<const bf16x8 *>(&Bs[r * kLdsRow + kk]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
    }
    // epilogue: element v of tile (i, j) is row 8 (v/4) + 4 (lane/32) + v%4, column lane%32
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = n0 + wn * 64 + 32 * j + (lane & 31);
            if (col >= N) continue;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = m0 + wm * 64 + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                if (row >= M) continue;
                const float x = acc[i][j][v];
                if constexpr (EPI == EPI_F32) {
                    float *C = static_cast<float *>(Cout) + blockIdx.z * c_split_stride;
                    C[(size_t)row * ldc + col] = x;
                } else if constexpr (EPI == EPI_BIAS_RELU_BF16) {
                    const float z = x + bias[col];
                    static_cast<uint16_t *>(Cout)[(size_t)row * ldc + col] = f2bf(z > 0.f ? z : 0.f);
                } else {
                    const bool on = bf2f(mask[(size_t)row * ldm + col]) > 0.f;
                    static_cast<uint16_t *>(Cout)[(size_t)row * ldc + col] = f2bf(on ? x : 0.f);
                }
            }
        }
}

// ------------------------------------------------------------------ fused inference
// Whole network for 128 rows per block tile (inference only): features
// computed in FP64 straight into LDS, then four hidden layers whose BF16
// activations stay in LDS (one 128 x 256 tile, written back in place after a
// barrier), then the FP32 head.  Wave w owns output columns [64 w, 64 w + 64)
// of every layer: 4 x 2 tiles of 32 x 32 (v_mfma_f32_32x32x16_bf16, 128
// accumulators per lane); activation fragments come from LDS, weight
// fragments from a copy of the weights stored in fragment order (for every
// 32-column tile and 16-wide K slice, the 64 lanes' 16-byte operands side by
// side), so each weight load of a wave is one contiguous 1 KB read from L2.
// Two blocks share a CU (2 x 68 KB of LDS), so one block's feature or
// epilogue phase overlaps the other's MFMAs.  Sums run in K order as in
// k_gemm_nt.
constexpr int kFR = 128;                              // rows per block tile
constexpr int kFRow = GTMP_SUR_WIDTH + 8;             // LDS row stride (BF16), 528 bytes
constexpr int kColTiles = GTMP_SUR_WIDTH / 32;        // 32-column output tiles per layer

// Offsets (in 16-byte fragments) of the layers in the fragment-order copy.
__host__ __device__ constexpr int frag_offset(int l) {
    return l == 0 ? 0 : kColTiles * (GTMP_SUR_IN / 16) * 64 + (l - 1) * kColTiles * (GTMP_SUR_WIDTH / 16) * 64;
}
constexpr int kFragTotal = frag_offset(4);  // 16-byte fragments of the four hidden layers

// Feature order of the fused kernels' LDS rows: each of a row's two
// threads writes one half with four 16-byte stores, thread 0 [sin f0..7 |
// cos f0..7 | q/pi (8, zero past d) | 0 x 8], thread 1 [sin f8..15 |
// cos f8..15 | 0 x 16].  feature_at maps an LDS position to the input of the
// standard order [q/pi (d) | sin (16) | cos (16) | 0...], -1 for a zero; the
// first layer's weight fragments are stored in the LDS order, so the sums
// are over the same products.
__host__ __device__ inline int feature_at(int p, int d) {
    if (p < 8) return d + p;
    if (p < 16) return d + GTMP_SUR_FREQ + (p - 8);
    if (p < 24) return p - 16 < d ? p - 16 : -1;
    if (p < 32) return -1;
    if (p < 40) return d + 8 + (p - 32);
    if (p < 48) return d + GTMP_SUR_FREQ + 8 + (p - 40);
    return -1;
}

__device__ __forceinline__ uint32_t pack2(uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }

// Thread `half` of a row: sn, cs = its 8 frequencies' sines and cosines, qh
// (half 0) the d linear features; BF16-rounded and stored in the LDS order.
__device__ __forceinline__ void store_features(int d, int half, const double (&sn)[8], const double (&cs)[8],
                                               const double (&qh)[GTMP_MAX_DOF], uint16_t *row) {
    uint16_t v[32];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        v[q] = d2bf(sn[q]);
        v[8 + q] = d2bf(cs[q]);
        v[16 + q] = (half == 0 && q < d) ? d2bf(qh[q]) : (uint16_t)0;
        v[24 + q] = 0;
    }
    uint4 *dst = reinterpret_cast<uint4 *>(row + 32 * half);
#pragma unroll
    for (int c = 0; c < 4; ++c)
        dst[c] = make_uint4(pack2(v[8 * c], v[8 * c + 1]), pack2(v[8 * c + 2], v[8 * c + 3]),
                            pack2(v[8 * c + 4], v[8 * c + 5]), pack2(v[8 * c + 6], v[8 * c + 7]));
}

// Fragment f of layer l: lane = f % 64, K slice ks and column tile c from
// f / 64 = c * S + ks; it holds W_l[32 c + lane % 32][16 ks + 8 (lane / 32) ..+8].
// (Layer 1's columns in the LDS feature order of feature_at.)
__global__ void __launch_bounds__(256) k_weight_frag(int d, const uint16_t *__restrict__ P16, SurLayout L,
                                                     uint4 *__restrict__ Wf) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= kFragTotal) return;
    const int l = f < frag_offset(1) ? 0 : 1 + (f - frag_offset(1)) / (frag_offset(2) - frag_offset(1));
    const int K = l == 0 ? GTMP_SUR_IN : GTMP_SUR_WIDTH;
    const int S = K / 16;
    const int r = f - frag_offset(l);
    const int lane = r & 63, ks = (r >> 6) % S, c = (r >> 6) / S;
    const int row = 32 * c + (lane & 31), col = 16 * ks + 8 * (lane >> 5);
    const uint16_t *src = P16 + L.W[l] + (size_t)row * K;
    if (l > 0) {
        Wf[f] = *reinterpret_cast<const uint4 *>(src + col);
        return;
    }
    uint16_t w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int j = feature_at(col + k, d);
        w[k] = j < 0 ? (uint16_t)0 : src[j];
    }
    Wf[f] = make_uint4(pack2(w[0], w[1]), pack2(w[2], w[3]), pack2(w[4], w[5]), pack2(w[6], w[7]));
}

// One hidden layer on the block's LDS tile: K input columns -> 256 outputs,
// bias + ReLU, BF16, written back in place.  The MFMA computes the transposed
// product (weights as the A operand, activations as B), so each lane's
// accumulators hold four consecutive output columns of one row: they are
// converted with one packed instruction per pair and stored with one 8-byte
// LDS write.  Weight fragments are requested one K slice ahead.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

template <int K>
__device__ __forceinline__ void mlp_layer(const bf16x8 *__restrict__ Wf, const float *__restrict__ bias,
                                          uint16_t *act, int wave, int lane) {
    constexpr int S = K / 16;
    const int cl = lane & 31, kh = 8 * (lane >> 5);
    const int c0 = wave * 64;
    f32x16 acc[4][2];  // [row tile i][column tile j]
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;
    const bf16x8 *wr0 = Wf + (size_t)(2 * wave) * S * 64 + lane;
    const bf16x8 *wr1 = Wf + (size_t)(2 * wave + 1) * S * 64 + lane;
    // weight fragments requested kWPre K slices ahead (an L2 round trip is
    // longer than one slice of MFMAs); the next slice's four activation
    // fragments are read from LDS while the current slice's MFMAs run
    constexpr int kWPre = 3;
    bf16x8 w0[S], w1[S];
#pragma unroll
    for (int k = 0; k < kWPre && k < S; ++k) {
        w0[k] = wr0[64 * k];
        w1[k] = wr1[64 * k];
    }
    auto act_frag = [&](int i, int ks) {
        return *reinterpret_cast<const bf16x8 *>(&act[(32 * i + cl) * kFRow + 16 * ks + kh]);
    };
    bf16x8 a_cur[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a_cur[i] = act_frag(i, 0);
#pragma unroll
    for (int ks = 0; ks < S; ++ks) {
        if (ks + kWPre < S) {
            w0[ks + kWPre] = wr0[64 * (ks + kWPre)];
            w1[ks + kWPre] = wr1[64 * (ks + kWPre)];
        }
        bf16x8 a_nxt[4];
        if (ks + 1 < S) {
#pragma unroll
            for (int i = 0; i < 4; ++i) a_nxt[i] = act_frag(i, ks + 1);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            acc[i][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0[ks], a_cur[i], acc[i][0], 0, 0, 0);
            acc[i][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1[ks], a_cur[i], acc[i][1], 0, 0, 0);
        }
        if (ks + 1 < S) {
#pragma unroll
            for (int i = 0; i < 4; ++i) a_cur[i] = a_nxt[i];
        }
    }
    // element v of tile (i, j): output column c0 + 32 j + 8 (v/4) + 4 (lane/32) + v%4, row 32 i + lane%32
    f32x4v bq[2][4];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int g = 0; g < 4; ++g)
            bq[j][g] = *reinterpret_cast<const f32x4v *>(bias + c0 + 32 * j + 8 * g + 4 * (lane >> 5));
    __syncthreads();  // every wave has read this layer's input
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                f32x4v z;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float t = acc[i][j][4 * g + r] + bq[j][g][r];
                    z[r] = t > 0.f ? t : 0.f;
                }
                const bf16x4 o = __builtin_convertvector(z, bf16x4);
                const int col = c0 + 32 * j + 8 * g + 4 * (lane >> 5);
                *reinterpret_cast<bf16x4 *>(&act[(32 * i + cl) * kFRow + col]) = o;
            }
    __syncthreads();
}

// Features of one row into its LDS slot; two threads per row (half 0 and 1),
// each taking half of the frequencies.  qh = q / pi in FP64.
__device__ __forceinline__ void row_features(int d, const double (&qh)[GTMP_MAX_DOF], int half,
                                             const float *__restrict__ Bf, uint16_t *dst) {
    constexpr double kPi = 3.14159265358979323846;
    double sn[8], cs[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int f = half * (GTMP_SUR_FREQ / 2) + q;
        double sarg = 0.0;
        for (int j = 0; j < d; ++j) sarg += (double)Bf[f * d + j] * qh[j];
        sarg *= 2.0 * kPi;
        sincos(sarg, &sn[q], &cs[q]);
    }
    store_features(d, half, sn, cs, qh, dst);
}

// The four hidden layers and the FP32 head of the block's tile; thread
// tid < kFR gets its row's logit.  Head: two threads per row, each summing
// one half of the 256 products in K order (8 activations per LDS read);
// z = first half + second half + b5.
__device__ __forceinline__ float mlp_tile(const bf16x8 *__restrict__ Wf, const float *__restrict__ P32,
                                          const SurLayout &L, uint16_t *act, const float *w5s, float *zpart,
                                          int tid) {
    const int lane = tid & 63, wave = tid >> 6;
    mlp_layer<GTMP_SUR_IN>(Wf + frag_offset(0), P32 + L.b[0], act, wave, lane);
    mlp_layer<GTMP_SUR_WIDTH>(Wf + frag_offset(1), P32 + L.b[1], act, wave, lane);
    mlp_layer<GTMP_SUR_WIDTH>(Wf + frag_offset(2), P32 + L.b[2], act, wave, lane);
    mlp_layer<GTMP_SUR_WIDTH>(Wf + frag_offset(3), P32 + L.b[3], act, wave, lane);
    const int r = tid & (kFR - 1), half = tid >> 7;
    constexpr int kHalf = GTMP_SUR_WIDTH / 2;
    const uint4 *a = reinterpret_cast<const uint4 *>(act + r * kFRow + half * kHalf);
    const float *w = w5s + half * kHalf;
    float z = 0.f;
#pragma unroll 4
    for (int q = 0; q < kHalf / 8; ++q) {
        const uint4 v = a[q];
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            z = __builtin_fmaf(w[8 * q + 2 * h], __uint_as_float(wd[h] << 16), z);
            z = __builtin_fmaf(w[8 * q + 2 * h + 1], __uint_as_float(wd[h] & 0xffff0000u), z);
        }
    }
    if (half == 1) zpart[r] = z;
    __syncthreads();
    return half == 0 ? z + zpart[r] + P32[L.b5] : 0.f;
}

__global__ void __launch_bounds__(256, 2) k_mlp_infer(int d, int64_t n, const float *__restrict__ X,
                                                     const float *__restrict__ Bf, const bf16x8 *__restrict__ Wf,
                                                     const uint16_t *__restrict__ P16,
                                                     const float *__restrict__ P32, SurLayout L,
                                                     float *__restrict__ logits) {
    __shared__ __attribute__((aligned(16))) uint16_t act[kFR * kFRow];
    __shared__ float w5s[GTMP_SUR_WIDTH];
    __shared__ float zpart[kFR];
    const int tid = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * kFR;
    {
        const int r = tid & (kFR - 1), half = tid >> 7;
        const int64_t gr = row0 + r;
        constexpr double kPi = 3.14159265358979323846;
        double qh[GTMP_MAX_DOF];
        for (int j = 0; j < GTMP_MAX_DOF; ++j) qh[j] = (gr < n && j < d) ? (double)X[gr * d + j] / kPi : 0.0;
        row_features(d, qh, half, Bf, act + r * kFRow);
        if (tid < GTMP_SUR_WIDTH) w5s[tid] = bf2f(P16[L.w5 + tid]);
    }
    __syncthreads();
    const float z = mlp_tile(Wf, P32, L, act, w5s, zpart, tid);
    if (tid < kFR && row0 + tid < n) logits[row0 + tid] = z;
}

// ------------------------------------------------------------------ pruning
// Candidate edges: those whose two endpoints are free samples (an edge with
// a colliding endpoint fails the exact check at its vertex, so it is never
// inferred).  Per layer m the free samples in index order fl[m][0 .. nf[m]);
// candidate t lies in segment s with seg[s] <= t < seg[s + 1]: s = 0 start
// edges (q0 -> free layer-0 samples), s = 1 .. M-1 the free pairs of layers
// s-1 and s (row-major over the two free lists), s = M the edges from free
// layer M-1 samples to every goal.
__global__ void __launch_bounds__(256) k_free_lists(int N, const uint8_t *__restrict__ vcoll,
                                                    int32_t *__restrict__ fl, int32_t *__restrict__ nf) {
    __shared__ int wsum[256 / kWave];
    const int m = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int count = 0;
    for (int base = 0; base < N; base += 256) {
        const int i = base + tid;
        const bool fr = i < N && (vcoll == nullptr || vcoll[(size_t)m * N + i] == 0);
        const uint64_t bal = __ballot(fr);
        if (lane == 0) wsum[wv] = __popcll(bal);
        __syncthreads();
        int before = count;
        for (int w = 0; w < wv; ++w) before += wsum[w];
        if (fr) fl[(size_t)m * N + before + __popcll(bal & ((1ull << lane) - 1ull))] = i;
        for (int w = 0; w < 256 / kWave; ++w) count += wsum[w];
        __syncthreads();
    }
    if (tid == 0) nf[m] = count;
}

// Phase table of the probe features.  The midpoint of u and v is
// (u + v) / 2 exactly (FP64), so its phases are 2 pi B (u + v) / (2 pi) =
// a(u) + a(v) with a(x) = pi sum_j B_fj (x_j / pi), and its sines and
// cosines follow from the endpoints' by angle addition.  Row of a sample
// (kPhaseRow doubles): sin a_f (16), cos a_f (16), x_j / pi (8, zero past d).
// Rows: the free samples in free-list order ([M][N] slots), then q0, then
// the goals.
constexpr int kPhaseRow = 2 * GTMP_SUR_FREQ + GTMP_MAX_DOF;

__global__ void __launch_bounds__(256) k_sample_phases(int d, int M, int N, int G, const float *__restrict__ Q,
                                                       const float *__restrict__ q0, const float *__restrict__ goals,
                                                       const int32_t *__restrict__ fl, const int32_t *__restrict__ nf,
                                                       const float *__restrict__ Bf, double *__restrict__ T) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t MN = (int64_t)M * N;
    if (t >= MN + 1 + G) return;
    const float *x;
    if (t < MN) {
        const int m = (int)(t / N), i = (int)(t - (int64_t)m * N);
        if (i >= nf[m]) return;
        x = Q + ((size_t)m * N + fl[t]) * d;
    } else if (t == MN) {
        x = q0;
    } else {
        x = goals + (size_t)(t - MN - 1) * d;
    }
    constexpr double kPi = 3.14159265358979323846;
    double qh[GTMP_MAX_DOF];
    for (int j = 0; j < GTMP_MAX_DOF; ++j) qh[j] = j < d ? (double)x[j] / kPi : 0.0;
    double *row = T + (size_t)t * kPhaseRow;
    for (int f = 0; f < GTMP_SUR_FREQ; ++f) {
        double a = 0.0;
        for (int j = 0; j < d; ++j) a += (double)Bf[f * d + j] * qh[j];
        a *= kPi;
        double sn, cs;
        sincos(a, &sn, &cs);
        row[f] = sn;
        row[GTMP_SUR_FREQ + f] = cs;
    }
    for (int j = 0; j < GTMP_MAX_DOF; ++j) row[2 * GTMP_SUR_FREQ + j] = qh[j];
}

__global__ void k_cand_segments(int M, int G, const int32_t *__restrict__ nf, int64_t *__restrict__ seg) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t o = 0;
    seg[0] = 0;
    o += nf[0];
    seg[1] = o;
    for (int s = 1; s < M; ++s) {
        o += (int64_t)nf[s - 1] * nf[s];
        seg[s + 1] = o;
    }
    o += (int64_t)nf[M - 1] * G;
    seg[M + 1] = o;
}

__global__ void k_prune_fill(int64_t E, uint8_t *__restrict__ prune, float *__restrict__ logits) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E; i += stride) {
        prune[i] = 0;
        if (logits) logits[i] = __builtin_nanf("");
    }
}

// Endpoints of candidate t (t < total): their rows in the phase table and
// the edge's flat id.  Segment bounds and list lengths come from LDS.
template <typename IDX>
__device__ __forceinline__ void cand_rows(int64_t t, int M, int N, int G, const int64_t *seg, const int32_t *nf,
                                          const int32_t *__restrict__ fl, int64_t &ru, int64_t &rv, int64_t &e) {
    int lo = 0, hi = M;  // largest s in [0, M] with seg[s] <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const IDX loc = (IDX)(t - seg[lo]);
    const int64_t MN = (int64_t)M * N;
    if (lo == 0) {
        ru = MN;
        rv = (int64_t)loc;
        e = fl[loc];
    } else if (lo < M) {
        const int m = lo - 1;
        const IDX n1 = (IDX)nf[m + 1];
        const IDX i = loc / n1, j = loc - i * n1;
        ru = (int64_t)m * N + (int64_t)i;
        rv = (int64_t)(m + 1) * N + (int64_t)j;
        e = N + (int64_t)m * N * N + (int64_t)fl[ru] * N + fl[rv];
    } else {
        const IDX i = loc / (IDX)G, g = loc - i * (IDX)G;
        ru = (int64_t)(M - 1) * N + (int64_t)i;
        rv = MN + 1 + (int64_t)g;
        e = N + (int64_t)(M - 1) * N * N + (int64_t)fl[ru] * G + g;
    }
}

// Probe features of the midpoint of the samples with phase rows Tu and Tv:
// x_j / pi = (Tu_j + Tv_j) / 2, sin(a_u + a_v) = sin a_u cos a_v + cos a_u
// sin a_v, cos(a_u + a_v) = cos a_u cos a_v - sin a_u sin a_v (FP64), each
// rounded once to BF16; two threads per row as in row_features.
__device__ __forceinline__ void mid_features(int d, const double *__restrict__ Tu, const double *__restrict__ Tv,
                                             int half, uint16_t *dst) {
    double sn[8], cs[8], qh[GTMP_MAX_DOF];
#pragma unroll
    for (int j = 0; j < GTMP_MAX_DOF; ++j)
        qh[j] = half == 0 && j < d ? (Tu[2 * GTMP_SUR_FREQ + j] + Tv[2 * GTMP_SUR_FREQ + j]) * 0.5 : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int f = half * (GTMP_SUR_FREQ / 2) + q;
        const double su = Tu[f], cu = Tu[GTMP_SUR_FREQ + f], sv = Tv[f], cv = Tv[GTMP_SUR_FREQ + f];
        sn[q] = __builtin_fma(su, cv, cu * sv);
        cs[q] = __builtin_fma(cu, cv, -(su * sv));
    }
    store_features(d, half, sn, cs, qh, dst);
}

constexpr int kSegLds = 130;  // segment bounds kept in LDS (M <= 128)

// One block per tile of 128 candidates, launched over the upper bound E / 128
// (the candidate count is known only on the device: blocks past it return
// at once).  Blocks of one CU start at different times, so one block's
// feature or head phase overlaps the other's MFMAs.  The candidate's
// endpoints give the features of the midpoint (u + v) / 2 (from their phase
// rows) and its logit z; prune[e] = z > tau and logits[e] = z at the edge's
// flat id e (C_s | C_h | C_l order).
template <typename IDX>
__global__ void __launch_bounds__(256, 2) k_mlp_prune(int d, int M, int N, int G, const double *__restrict__ T,
                                                     const int32_t *__restrict__ fl, const int32_t *__restrict__ nf,
                                                     const int64_t *__restrict__ seg, const bf16x8 *__restrict__ Wf,
                                                     const uint16_t *__restrict__ P16, const float *__restrict__ P32,
                                                     SurLayout L, float tau,
                                                     uint8_t *__restrict__ prune, float *__restrict__ logits) {
    __shared__ __attribute__((aligned(16))) uint16_t act[kFR * kFRow];
    __shared__ float w5s[GTMP_SUR_WIDTH];
    __shared__ float zpart[kFR];
    __shared__ int64_t eid[kFR];
    __shared__ int64_t seg_s[kSegLds];
    __shared__ int32_t nf_s[kSegLds];
    const int tid = threadIdx.x;
    const int64_t total = seg[M + 1];
    const int64_t tile = blockIdx.x;
    if (tile * kFR >= total) return;  // block-uniform
    const bool in_lds = M + 2 <= kSegLds;
    if (in_lds) {
        for (int i = tid; i < M + 2; i += blockDim.x) seg_s[i] = seg[i];
        for (int i = tid; i < M; i += blockDim.x) nf_s[i] = nf[i];
    }
    if (tid < GTMP_SUR_WIDTH) w5s[tid] = bf2f(P16[L.w5 + tid]);
    __syncthreads();
    const int64_t *sg = in_lds ? seg_s : seg;
    const int32_t *nl = in_lds ? nf_s : nf;
    {
        const int r = tid & (kFR - 1), half = tid >> 7;
        const int64_t t = tile * kFR + r;
        int64_t ru = 0, rv = 0, e = -1;
        if (t < total) cand_rows<IDX>(t, M, N, G, sg, nl, fl, ru, rv, e);
        if (half == 0) eid[r] = e;
        if (e >= 0) {
            mid_features(d, T + (size_t)ru * kPhaseRow, T + (size_t)rv * kPhaseRow, half, act + r * kFRow);
        } else {
            uint4 *z4 = reinterpret_cast<uint4 *>(act + r * kFRow + 32 * half);
            for (int c = 0; c < 4; ++c) z4[c] = make_uint4(0u, 0u, 0u, 0u);
        }
    }
    __syncthreads();
    const float z = mlp_tile(Wf, P32, L, act, w5s, zpart, tid);
    if (tid < kFR) {
        const int64_t e = eid[tid];
        if (e >= 0) {
            prune[e] = z > tau ? 1 : 0;
            if (logits) logits[e] = z;
        }
    }
}

// ------------------------------------------------------------------ small kernels
// out [C][R] = in [R][C]^T, BF16, R and C multiples of 64.
__global__ void __launch_bounds__(256) k_transpose_bf16(int R, int C, const uint16_t *__restrict__ in,
                                                        uint16_t *__restrict__ out) {
    __shared__ uint16_t t[64][65];
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) t[r][tx] = in[(size_t)(r0 + r) * C + c0 + tx];
    __syncthreads();
    for (int c = ty; c < 64; c += 4) out[(size_t)(c0 + c) * R + r0 + tx] = t[tx][c];
}

// Output layer, loss and its gradient: one wave per row.
//   z = sum_k bf16(w5)[k] a4[k] + b5;  loss_b = max(z,0) - y z + log1p(exp(-|z|));
//   dz = (sigmoid(z) - y) / n
__global__ void __launch_bounds__(256) k_head(int64_t n, const uint16_t *__restrict__ A4,
                                              const uint16_t *__restrict__ w5, const float *__restrict__ b5,
                                              const uint8_t *__restrict__ y, float inv_n, float *__restrict__ logits,
                                              float *__restrict__ loss_terms, float *__restrict__ dz) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (row >= n) return;
    const int lane = lane_id();
    const uint16_t *a = A4 + row * GTMP_SUR_WIDTH;
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < GTMP_SUR_WIDTH / kWave; ++q) {
        const int k = lane * (GTMP_SUR_WIDTH / kWave) + q;
        s = __builtin_fmaf(bf2f(w5[k]), bf2f(a[k]), s);
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane != 0) return;
    const float z = s + b5[0];
    if (logits) logits[row] = z;
    if (y) {
        const float yy = y[row] ? 1.f : 0.f;
        const float az = __builtin_fabsf(z);
        const float e = __expf(-az);
        loss_terms[row] = (z > 0.f ? z : 0.f) - yy * z + log1pf(e);
        const float sig = z >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
        dz[row] = (sig - yy) * inv_n;
    }
}

// dZ4 = bf16(dz[b] bf16(w5)[k] [a4 > 0])
__global__ void __launch_bounds__(256) k_head_back(int64_t n, const float *__restrict__ dz,
                                                   const uint16_t *__restrict__ w5, const uint16_t *__restrict__ A4,
                                                   uint16_t *__restrict__ dZ) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * GTMP_SUR_WIDTH) return;
    const int64_t b = i / GTMP_SUR_WIDTH;
    const int k = (int)(i % GTMP_SUR_WIDTH);
    const float g = dz[b] * bf2f(w5[k]);
    dZ[i] = f2bf(bf2f(A4[i]) > 0.f ? g : 0.f);
}

// Column sums over fixed row chunks: part[p][c] = sum_{r in chunk p} scale[r] X[r][c]
template <typename T>
__device__ __forceinline__ float load_val(const T *p);
template <>
__device__ __forceinline__ float load_val<uint16_t>(const uint16_t *p) { return bf2f(*p); }
template <>
__device__ __forceinline__ float load_val<float>(const float *p) { return *p; }

template <typename T>
__global__ void __launch_bounds__(256) k_colsum_part(int64_t rows, int cols, int rows_per_part, const T *__restrict__ X,
                                                     const float *__restrict__ scale, float *__restrict__ part) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_part;
    const int64_t r1 = r0 + rows_per_part < rows ? r0 + rows_per_part : rows;
    float s = 0.f;
    for (int64_t r = r0; r < r1; ++r) {
        const float x = load_val<T>(X + r * cols + c);
        s = scale ? __builtin_fmaf(scale[r], x, s) : s + x;
    }
    part[(size_t)blockIdx.y * cols + c] = s;
}

// out[i] = sum_p part[p][i] in p order
__global__ void __launch_bounds__(256) k_sum_parts(int parts, int64_t len, const float *__restrict__ part,
                                                   float *__restrict__ out, float scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    float s = 0.f;
    for (int p = 0; p < parts; ++p) s += part[(size_t)p * len + i];
    out[i] = s * scale;
}

__global__ void __launch_bounds__(256) k_adam(int total, float *__restrict__ P, uint16_t *__restrict__ P16,
                                              const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float p = P[i] - lr * (mi * c1) / (__builtin_sqrtf(vi * c2) + eps);
    P[i] = p;
    P16[i] = f2bf(p);
}

__global__ void __launch_bounds__(256) k_to_bf16(int total, const float *__restrict__ P, uint16_t *__restrict__ P16) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) P16[i] = f2bf(P[i]);
}

// Training states: rows [0, n) uniform (layer 0), rows [n, 2n) interior
// lerp states of the edge (layer-1 sample j, layer-2 sample j).
__global__ void __launch_bounds__(256) k_label_states(int d, int64_t n, int H, uint32_t k0, uint32_t k1,
                                                      uint32_t stage, SurBox B, float *__restrict__ X) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * n) return;
    const int nblk = (d + 3) >> 2;
    auto sample = [&](uint32_t m, uint32_t s, float *x) {
        for (int blk = 0; blk < nblk; ++blk) {
            const uint4 w = philox4x32_10(make_uint4(s, m, stage, (uint32_t)blk), k0, k1);
            const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
            for (int q = 0; q < 4; ++q) {
                const int j = blk * 4 + q;
                if (j < d) x[j] = __builtin_fmaf(unit_from_word(ws[q]), B.wd[j], B.lo[j]);
            }
        }
    };
    float x[GTMP_MAX_DOF];
    if (i < n) {
        sample(0u, (uint32_t)i, x);
    } else {
        const int64_t j = i - n;
        float u[GTMP_MAX_DOF], v[GTMP_MAX_DOF];
        sample(1u, (uint32_t)j, u);
        sample(2u, (uint32_t)j, v);
        const int h = 1 + (int)(j % (H - 2));
        const float t = (float)h / (float)(H - 1);
        for (int q = 0; q < d; ++q) x[q] = __builtin_fmaf(t, v[q] - u[q], u[q]);
    }
    for (int q = 0; q < d; ++q) X[i * d + q] = x[q];
}

// ------------------------------------------------------------------ host side
static unsigned blocks_for(int64_t n, int per = 256) { return (unsigned)((n + per - 1) / per); }

template <int EPI>
static void gemm(int M, int N, int K, int splits, const uint16_t *A, int lda, const uint16_t *B, int ldb, void *C,
                 int ldc, const float *bias, const uint16_t *mask, int ldm, hipStream_t s) {
    const dim3 grid((unsigned)((N + kBN - 1) / kBN), (unsigned)((M + kBM - 1) / kBM), (unsigned)splits);
    hipLaunchKernelGGL(k_gemm_nt<EPI>, grid, dim3(256), 0, s, M, N, K / splits, A, lda, B, ldb, C, ldc, bias, mask,
                       ldm, (size_t)M * ldc);
}

// Workspace carve-up for n rows.
struct SurWs {
    uint4 *Wf;  // fragment-order weights (inference)
    uint16_t *X0, *A[4], *dZa, *dZb, *T1, *T2, *WT;
    float *part, *loss_terms, *dz, *logit_tmp, *Xf;
    size_t total;
};
static size_t up256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr int kSplitsMax = 32;      // split-K partials of the weight gradients
constexpr int kColParts = 64;       // row chunks of the column sums

static SurWs carve(int64_t n, void *base) {
    SurWs w{};
    char *p = static_cast<char *>(base);
    size_t o = 0;
    auto take = [&](size_t bytes) { char *q = p ? p + o : nullptr; o = up256(o + bytes); return q; };
    const size_t W = GTMP_SUR_WIDTH;
    w.X0 = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * n * GTMP_SUR_IN));
    for (int l = 0; l < 4; ++l) w.A[l] = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * n * W));
    w.dZa = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * n * W));
    w.dZb = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * n * W));
    w.T1 = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * n * W));
    w.T2 = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * n * W));
    w.WT = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * W * W));
    const size_t part_floats = std::max((size_t)kSplitsMax * W * W, (size_t)kColParts * W);
    w.part = reinterpret_cast<float *>(take(sizeof(float) * part_floats));
    w.loss_terms = reinterpret_cast<float *>(take(sizeof(float) * n));
    w.dz = reinterpret_cast<float *>(take(sizeof(float) * n));
    w.logit_tmp = reinterpret_cast<float *>(take(sizeof(float) * n));
    w.Xf = reinterpret_cast<float *>(take(sizeof(float) * n * GTMP_MAX_DOF));
    w.total = o;
    return w;
}

// Inference needs the fragment-order weights, and for chunked use the
// features, two activation buffers (layers alternate between them), the
// logits and the FP32 probe states.
static SurWs carve_infer(int64_t n, void *base) {
    SurWs w{};
    char *p = static_cast<char *>(base);
    size_t o = 0;
    auto take = [&](size_t bytes) { char *q = p ? p + o : nullptr; o = up256(o + bytes); return q; };
    w.Wf = reinterpret_cast<uint4 *>(take(sizeof(uint4) * kFragTotal));
    w.X0 = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * n * GTMP_SUR_IN));
    w.A[0] = w.A[2] = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * n * GTMP_SUR_WIDTH));
    w.A[1] = w.A[3] = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * n * GTMP_SUR_WIDTH));
    w.logit_tmp = reinterpret_cast<float *>(take(sizeof(float) * n));
    w.Xf = reinterpret_cast<float *>(take(sizeof(float) * n * GTMP_MAX_DOF));
    w.total = o;
    return w;
}

size_t sur_workspace_bytes(int64_t n) { return carve(n, nullptr).total; }

int64_t sur_rows_for(size_t bytes) {
    // largest multiple of 256 rows whose inference carve-up fits
    int64_t lo = 0, hi = 1 << 24;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (carve_infer(mid * 256, nullptr).total <= bytes) lo = mid;
        else hi = mid - 1;
    }
    return lo * 256;
}

size_t sur_infer_bytes(int64_t n) { return carve_infer(n, nullptr).total; }

// forward of rows [0, n) of X (FP32 [n][d]) into logits; activations kept in ws
static void forward(const SurNet &net, int64_t n, const float *X, const SurWs &w, float *logits, const uint8_t *y,
                    float inv_n, hipStream_t s) {
    const SurLayout L = sur_layout();
    hipLaunchKernelGGL(k_features, dim3(blocks_for(n)), dim3(256), 0, s, net.d, n, X, net.fourier, w.X0);
    const uint16_t *in = w.X0;
    int K = GTMP_SUR_IN;
    for (int l = 0; l < 4; ++l) {
        gemm<EPI_BIAS_RELU_BF16>((int)n, GTMP_SUR_WIDTH, K, 1, in, K, net.p16 + L.W[l], K, w.A[l], GTMP_SUR_WIDTH,
                                 net.p32 + L.b[l], nullptr, 0, s);
        in = w.A[l];
        K = GTMP_SUR_WIDTH;
    }
    hipLaunchKernelGGL(k_head, dim3(blocks_for(n, 4)), dim3(256), 0, s, n, w.A[3], net.p16 + L.w5, net.p32 + L.b5, y,
                       inv_n, logits, w.loss_terms, w.dz);
}

static void weight_frag(const SurNet &net, uint4 *Wf, hipStream_t s) {
    hipLaunchKernelGGL(k_weight_frag, dim3((kFragTotal + 255) / 256), dim3(256), 0, s, net.d, net.p16, sur_layout(),
                       Wf);
}

hipError_t launch_sur_infer(const SurNet &net, int64_t n, const float *X, float *logits, void *ws, size_t ws_bytes,
                            hipStream_t s) {
    (void)ws_bytes;
    if (n <= 0) return hipSuccess;
    const SurWs w = carve_infer(0, ws);
    weight_frag(net, w.Wf, s);
    // chunks bound the grid size
    constexpr int64_t kChunk = (int64_t)1 << 30;
    for (int64_t r = 0; r < n; r += kChunk) {
        const int64_t c = n - r < kChunk ? n - r : kChunk;
        hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((c + kFR - 1) / kFR)), dim3(256), 0, s, net.d, c,
                           X + r * net.d, net.fourier, reinterpret_cast<const bf16x8 *>(w.Wf), net.p16, net.p32,
                           sur_layout(), logits + r);
    }
    return hipGetLastError();
}

hipError_t launch_sur_grad(const SurNet &net, int n, const float *X, const uint8_t *y, float *grad, float *loss,
                           float *logits, void *ws, hipStream_t s) {
    const SurLayout L = sur_layout();
    const SurWs w = carve(n, ws);
    const int W = GTMP_SUR_WIDTH;
    forward(net, n, X, w, logits ? logits : w.logit_tmp, y, 1.f / (float)n, s);
    // loss = mean of the per-row terms (fixed-order sums)
    {
        const int rpp = (n + kColParts - 1) / kColParts;
        hipLaunchKernelGGL(k_colsum_part<float>, dim3(1, kColParts), dim3(256), 0, s, (int64_t)n, 1, rpp,
                           w.loss_terms, (const float *)nullptr, w.part);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, kColParts, (int64_t)1, w.part, loss,
                           1.f / (float)n);
    }
    // output layer: dW5 = sum_b dz a4, db5 = sum_b dz
    const int rpp = (n + kColParts - 1) / kColParts;
    hipLaunchKernelGGL(k_colsum_part<uint16_t>, dim3(1, kColParts), dim3(256), 0, s, (int64_t)n, W, rpp, w.A[3],
                       w.dz, w.part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, kColParts, (int64_t)W, w.part, grad + L.w5, 1.f);
    hipLaunchKernelGGL(k_colsum_part<float>, dim3(1, kColParts), dim3(256), 0, s, (int64_t)n, 1, rpp, w.dz,
                       (const float *)nullptr, w.part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, kColParts, (int64_t)1, w.part, grad + L.b5, 1.f);
    // dZ4
    uint16_t *dZ = w.dZa, *dZn = w.dZb;
    hipLaunchKernelGGL(k_head_back, dim3(blocks_for((int64_t)n * W)), dim3(256), 0, s, (int64_t)n, w.dz,
                       net.p16 + L.w5, w.A[3], dZ);
    int splits = 1;
    while (splits < kSplitsMax && n / (splits * 2) >= 256 && (n % (splits * 2 * kBK)) == 0) splits *= 2;
    for (int l = 3; l >= 0; --l) {
        const int K_in = l == 0 ? GTMP_SUR_IN : W;
        const uint16_t *A_prev = l == 0 ? w.X0 : w.A[l - 1];
        // dW_l = dZ^T A_prev: transposes put the batch dimension last
        hipLaunchKernelGGL(k_transpose_bf16, dim3(W / 64, n / 64), dim3(256), 0, s, n, W, dZ, w.T1);
        hipLaunchKernelGGL(k_transpose_bf16, dim3(K_in / 64, n / 64), dim3(256), 0, s, n, K_in, A_prev, w.T2);
        gemm<EPI_F32>(W, K_in, n, splits, w.T1, n, w.T2, n, w.part, K_in, nullptr, nullptr, 0, s);
        hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for((int64_t)W * K_in)), dim3(256), 0, s, splits,
                           (int64_t)W * K_in, w.part, grad + L.W[l], 1.f);
        // db_l = column sums of dZ (after the split-K partials are consumed)
        hipLaunchKernelGGL(k_colsum_part<uint16_t>, dim3(1, kColParts), dim3(256), 0, s, (int64_t)n, W, rpp, dZ,
                           (const float *)nullptr, w.part);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, kColParts, (int64_t)W, w.part, grad + L.b[l], 1.f);
        if (l > 0) {
            // dZ_{l-1} = bf16((dZ_l W_l) * [a_{l-1} > 0]): B operand W_l^T [K_in][W]
            hipLaunchKernelGGL(k_transpose_bf16, dim3(K_in / 64, W / 64), dim3(256), 0, s, W, K_in,
                               net.p16 + L.W[l], w.WT);
            gemm<EPI_MASK_BF16>(n, K_in, W, 1, dZ, W, w.WT, W, dZn, K_in, nullptr, A_prev, K_in, s);
            std::swap(dZ, dZn);
        }
    }
    return hipGetLastError();
}

hipError_t launch_sur_adam(const SurNet &net, const float *grad, float *m, float *v, int t, float lr, float b1,
                           float b2, float eps, hipStream_t s) {
    const int total = sur_layout().total;
    const double c1 = 1.0 / (1.0 - std::pow((double)b1, (double)t));
    const double c2 = 1.0 / (1.0 - std::pow((double)b2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(total)), dim3(256), 0, s, total, net.p32, net.p16, grad, m, v, lr, b1,
                       b2, eps, (float)c1, (float)c2);
    return hipGetLastError();
}

hipError_t launch_sur_refresh(const SurNet &net, hipStream_t s) {
    const int total = sur_layout().total;
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(total)), dim3(256), 0, s, total, net.p32, net.p16);
    return hipGetLastError();
}

hipError_t launch_sur_label_states(const gtmp_problem &p, uint64_t seed, uint64_t stage, int64_t n, float *X,
                                   hipStream_t s) {
    SurBox B{};
    for (int j = 0; j < p.d; ++j) {
        B.lo[j] = p.lo[j];
        B.wd[j] = p.hi[j] - p.lo[j];
    }
    if (n > 0)
        hipLaunchKernelGGL(k_label_states, dim3(blocks_for(2 * n)), dim3(256), 0, s, p.d, n, p.H,
                           (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), (uint32_t)stage, B, X);
    return hipGetLastError();
}

// Workspace of the pruning call: fragment-order weights, the free lists
// [M][N], their lengths [M] and the M + 2 segment bounds.
struct PruneWs {
    uint4 *Wf;
    int32_t *fl, *nf;
    double *T;
    int64_t *seg;
    size_t total;
};

static PruneWs carve_prune(const gtmp_problem &p, void *base) {
    PruneWs w{};
    char *q = static_cast<char *>(base);
    size_t o = 0;
    auto take = [&](size_t bytes) { char *r = q ? q + o : nullptr; o = up256(o + bytes); return r; };
    w.Wf = reinterpret_cast<uint4 *>(take(sizeof(uint4) * kFragTotal));
    w.fl = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)p.M * p.N));
    w.T = reinterpret_cast<double *>(take(sizeof(double) * kPhaseRow * ((size_t)p.M * p.N + 1 + p.G)));
    w.nf = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (size_t)p.M));
    w.seg = reinterpret_cast<int64_t *>(take(sizeof(int64_t) * ((size_t)p.M + 2)));
    w.total = o;
    return w;
}

size_t sur_prune_bytes(const gtmp_problem &p) { return carve_prune(p, nullptr).total; }

hipError_t launch_sur_prune(const gtmp_problem &p, const SurNet &net, const float *q0, const float *goals,
                            const float *Q, const uint8_t *vcoll, float tau, uint8_t *prune, float *logits, void *ws,
                            hipStream_t s) {
    const int64_t E = (int64_t)p.N + (int64_t)(p.M - 1) * p.N * p.N + (int64_t)p.N * p.G;
    const PruneWs w = carve_prune(p, ws);
    weight_frag(net, w.Wf, s);
    const int64_t fill_blocks = std::min<int64_t>((E + 255) / 256, 4096);
    hipLaunchKernelGGL(k_prune_fill, dim3((unsigned)fill_blocks), dim3(256), 0, s, E, prune, logits);
    hipLaunchKernelGGL(k_free_lists, dim3(p.M), dim3(256), 0, s, p.N, vcoll, w.fl, w.nf);
    const int64_t rows = (int64_t)p.M * p.N + 1 + p.G;
    hipLaunchKernelGGL(k_sample_phases, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, p.d, p.M, p.N, p.G, Q,
                       q0, goals, w.fl, w.nf, net.fourier, w.T);
    hipLaunchKernelGGL(k_cand_segments, dim3(1), dim3(64), 0, s, p.M, p.G, w.nf, w.seg);
    const int64_t grid = (E + kFR - 1) / kFR;  // candidates <= E
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    // 32-bit index arithmetic when every segment's local index fits
    const bool narrow = (uint64_t)p.N * p.N < (1ull << 32) && (uint64_t)p.N * p.G < (1ull << 32);
    const auto kern = narrow ? k_mlp_prune<uint32_t> : k_mlp_prune<uint64_t>;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), 0, s, net.d, p.M, p.N, p.G, w.T, w.fl, w.nf, w.seg,
                       reinterpret_cast<const bf16x8 *>(w.Wf), net.p16, net.p32, sur_layout(), tau, prune, logits);
    return hipGetLastError();
}

}  // namespace gtmp
