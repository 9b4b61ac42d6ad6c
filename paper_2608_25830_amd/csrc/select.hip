// select.hip -- order statistics on the device: the pruning threshold of the
// learned surrogate.
//
// The threshold keeps a stated fraction of the free edges unpruned: with
// n_free edges of flag 0 and recall r, tau is the k-th smallest free-edge
// logit (0-based), k = ceil(r n_free) - 1 clamped to [0, n_free - 1], so
// that pruning z > tau keeps at least r n_free of them.  It is found by a
// radix select on the logits' order-preserving 32-bit keys, 11 + 11 + 10
// bits: each pass histograms the digit of the keys that share the prefix
// fixed so far (LDS histogram per block, merged with global atomics) and
// one block picks the digit holding the k-th key.  Everything stays on the
// device: no host read-back, no memset (the workspace is cleared by a
// kernel), so the call can sit in a captured stream.
#include "gtmp_launch.hpp"

namespace gtmp {

namespace {

constexpr int kSelBins = 2048;
constexpr int kSelPasses = 3;
__host__ __device__ constexpr int sel_shift(int pass) { return pass == 0 ? 21 : pass == 1 ? 10 : 0; }
__host__ __device__ constexpr int sel_bits(int pass) { return pass == 2 ? 10 : 11; }

struct SelState {
    uint32_t prefix, mask;  // key bits fixed so far
    uint64_t k;             // rank sought among the keys matching the prefix
    uint32_t done;          // no free edge: tau = +inf
    uint32_t pad;
};

// Monotone map of a float to an unsigned key (NaN canonicalised to the
// largest key, as sorting puts NaN last).
__device__ __forceinline__ uint32_t float_key(float z) {
    uint32_t b = __float_as_uint(z);
    if (z != z) return 0xffffffffu;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float key_float(uint32_t k) {
    const uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(b);
}

__global__ void __launch_bounds__(256) k_sel_init(uint32_t *hist, SelState *st) {
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) hist[i] = 0;
    if (threadIdx.x == 0) *st = SelState{0u, 0u, 0ull, 0u, 0u};
}

__global__ void __launch_bounds__(256) k_sel_hist(int pass, int64_t E, const float *__restrict__ z,
                                                  const uint8_t *__restrict__ flags, uint32_t *hist,
                                                  const SelState *st) {
    __shared__ uint32_t h[kSelBins];
    if (st->done) return;  // block-uniform
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint32_t prefix = st->prefix, mask = st->mask;
    const int shift = sel_shift(pass);
    const uint32_t dmask = (1u << sel_bits(pass)) - 1u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += stride) {
        if (flags[e] != 0) continue;
        const uint32_t key = float_key(z[e]);
        if ((key & mask) == prefix) atomicAdd(&h[(key >> shift) & dmask], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// One block: the digit of pass `pass` that holds rank k; fixes it into the
// prefix and clears the histogram for the next pass.  Pass 0 also sets k
// from the free-edge count; the last pass writes tau.
__global__ void __launch_bounds__(256) k_sel_pick(int pass, double recall, uint32_t *hist, SelState *st,
                                                  float *tau) {
    __shared__ uint64_t part[256];
    if (st->done) return;
    const int nb = 1 << sel_bits(pass);
    const int per = nb / 256;  // 8 or 4 bins per thread
    uint64_t mine = 0;
    for (int j = 0; j < per; ++j) mine += hist[threadIdx.x * per + j];
    part[threadIdx.x] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t total = 0;
        for (int t = 0; t < 256; ++t) total += part[t];
        SelState s = *st;
        if (pass == 0) {
            if (total == 0) {
                s.done = 1;
                *tau = __builtin_inff();
                *st = s;
            } else {
                double kk = ceil(recall * (double)total) - 1.0;
                if (kk < 0.0) kk = 0.0;
                if (kk > (double)(total - 1)) kk = (double)(total - 1);
                s.k = (uint64_t)kk;
            }
        }
        if (!s.done) {
            uint64_t before = 0;
            int t = 0;
            // the counts add up to more than k, so both scans stop inside
            // the histogram; the bounds only guard against a broken count
            while (t < 255 && before + part[t] <= s.k) before += part[t++];
            int b = t * per;
            while (b < t * per + per - 1 && before + hist[b] <= s.k) before += hist[b++];
            s.k -= before;
            const int shift = sel_shift(pass);
            s.prefix |= (uint32_t)b << shift;
            s.mask |= (uint32_t)(nb - 1) << shift;
            *st = s;
            if (pass == kSelPasses - 1) *tau = key_float(s.prefix);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSelBins; i += blockDim.x) hist[i] = 0;
}

}  // namespace

size_t sur_threshold_bytes() { return 256 + sizeof(uint32_t) * kSelBins; }

hipError_t launch_sur_threshold(const float *logits, const uint8_t *flags, int64_t E, double recall, float *tau,
                                void *workspace, hipStream_t s) {
    char *ws = static_cast<char *>(workspace);
    SelState *st = reinterpret_cast<SelState *>(ws);
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + 256);
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, hist, st);
    int64_t blocks = (E + 255) / 256;
    blocks = blocks < 1 ? 1 : blocks > 2048 ? 2048 : blocks;
    for (int pass = 0; pass < kSelPasses; ++pass) {
        hipLaunchKernelGGL(k_sel_hist, dim3((unsigned)blocks), dim3(256), 0, s, pass, E, logits, flags, hist, st);
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, s, pass, recall, hist, st, tau);
    }
    return hipGetLastError();
}

}  // namespace gtmp
