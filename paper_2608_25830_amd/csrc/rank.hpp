// rank.hpp -- the device side of the ranking of sample pairs (closest pairs
// of two point sets), shared by the single-plan launcher (select.hip) and
// the batched expansion (anytime.hip).  Both sources are compiled without
// floating-point contraction: the pair distance is an FP32 computation with
// a fixed operation order.
#pragma once

#include "gtmp_launch.hpp"

namespace gtmp {
namespace rank {

constexpr int kRankBins = 2048;
// The K closest (u, v) pairs of two point sets in increasing order of the
// FP32 squared distance (summed in coordinate order, no contraction), ties
// by pair index a * nv + b: the order of a stable sort of all nu * nv keys.
// Each pair has the composite key (distance bits << 32) | index, distinct
// for every pair and ordered as wanted (non-negative floats order as their
// bit patterns).  Up to kRankSortCap pairs, one block sorts every key in LDS
// (one launch).  Beyond, a radix select fixes the composite key's digits
// from the top (11, 11, 11, 11, 11, 9 bits) until the digit group holding
// rank K-1, with everything below it, fits the final sort (at most K +
// kRankSortCap keys); each pass is one launch whose last block to finish
// picks the digit (blocks publish their histograms, then count themselves
// done); those keys are compacted and one block sorts them (in LDS when they
// fit, else in the candidate buffer in device memory) and writes the first K
// indices.  Keys are recomputed from the points in every pass rather than
// stored.


constexpr int kRankPasses = 6;
constexpr int kRankSortCap = 8192;  // keys sorted in LDS (64 KiB)
__host__ __device__ constexpr int rank_shift(int pass) { return pass < 5 ? 53 - 11 * pass : 0; }
__host__ __device__ constexpr int rank_bits(int pass) { return pass < 5 ? 11 : 9; }

struct RankState {
    uint64_t prefix, mask;  // digits fixed so far
    uint32_t k;             // rank sought inside the prefix group
    uint32_t before;        // keys below the prefix group
    uint32_t done;          // the group is small enough: compact and sort
    uint32_t cnt;           // compacted keys
    uint32_t blocks_done;   // blocks of the current pass that have published
    uint32_t pad;
};

__device__ __forceinline__ uint64_t pair_key(int d, const float *__restrict__ U, int nv, const float *__restrict__ V,
                                             uint32_t idx) {
    const uint32_t a = idx / (uint32_t)nv, b = idx - a * (uint32_t)nv;
    float acc = 0.0f;  // (this file is compiled without contraction)
    for (int i = 0; i < d; ++i) {
        const float x = U[(size_t)a * d + i] - V[(size_t)b * d + i];
        acc = acc + x * x;
    }
    return ((uint64_t)__float_as_uint(acc) << 32) | idx;
}

// Bitonic sort of p (a power of two) keys at a, by the whole block.
__device__ __forceinline__ void bitonic_steps(uint64_t *a, uint32_t p) {
    for (uint32_t size = 2; size <= p; size <<= 1)
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t t = threadIdx.x; t < p / 2; t += blockDim.x) {
                const uint32_t lo = 2 * t - (t & (stride - 1));
                const uint32_t hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t x = a[lo], y = a[hi];
                if ((x > y) == up) {
                    a[lo] = y;
                    a[hi] = x;
                }
            }
            __syncthreads();
        }
}

constexpr int kRankSortThreads = 1024;

// npairs <= kRankSortCap: every key sorted by one block (lds: kRankSortCap keys).
__device__ __forceinline__ void rank_small_block(int d, const float *U, int nv, const float *V, uint32_t npairs,
                                                 uint32_t K, uint32_t *out, uint64_t *lds) {
    uint32_t p = 1;
    while (p < npairs) p <<= 1;
    for (uint32_t i = threadIdx.x; i < p; i += blockDim.x) lds[i] = i < npairs ? pair_key(d, U, nv, V, i) : ~0ull;
    __syncthreads();
    bitonic_steps(lds, p);
    for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) out[i] = (uint32_t)(lds[i] & 0xffffffffu);
}

__device__ __forceinline__ void rank_init_block(uint32_t K, uint32_t *hist, RankState *st) {
    for (int i = threadIdx.x; i < kRankBins; i += blockDim.x) hist[i] = 0;
    if (threadIdx.x == 0) *st = RankState{0ull, 0ull, K - 1u, 0u, 0u, 0u, 0u, 0u};
}

// One radix-select pass: every block histograms its share of the keys in
// the prefix group, adds it to the global histogram and counts itself done;
// the last block picks the digit holding rank k, extends the prefix, clears
// the histogram and the block count for the next pass.
// (blk, nblk: this block's index among the nblk blocks of the pass; h,
// part, last: the block's LDS, kRankBins and 256 words and a flag)
__device__ __forceinline__ void rank_pass_block(int pass, int d, const float *U, int nv, const float *V,
                                                uint32_t npairs, uint32_t K, uint32_t *hist, RankState *st,
                                                uint32_t blk, uint32_t nblk, uint32_t *h, uint32_t *part,
                                                bool &last) {
    if (st->done) return;  // block-uniform
    for (int i = threadIdx.x; i < kRankBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint64_t prefix = st->prefix, mask = st->mask;
    const int shift = rank_shift(pass);
    const uint64_t dmask = (1ull << rank_bits(pass)) - 1ull;
    for (uint64_t e = (uint64_t)blk * blockDim.x + threadIdx.x; e < npairs; e += (uint64_t)nblk * blockDim.x) {
        const uint64_t c = pair_key(d, U, nv, V, (uint32_t)e);
        if ((c & mask) == prefix) atomicAdd(&h[(uint32_t)((c >> shift) & dmask)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kRankBins; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
    __threadfence();  // this block's counts are visible before it counts itself done
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(&st->blocks_done, 1u) == nblk - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    // the last block: pick the digit of rank k
    const int nb = 1 << rank_bits(pass);
    const int per = nb / 256;  // 8 or 2 bins per thread
    uint32_t mine = 0;
    for (int j = 0; j < per; ++j) mine += __atomic_load_n(&hist[threadIdx.x * per + j], __ATOMIC_RELAXED);
    part[threadIdx.x] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        RankState s = *st;
        uint32_t below = 0;
        int t = 0;
        // the counts of the prefix group add up to more than k: both scans
        // stop inside the histogram (the bounds only guard a broken count)
        while (t < 255 && below + part[t] <= s.k) below += part[t++];
        int b = t * per;
        auto count = [&](int i) { return __atomic_load_n(&hist[i], __ATOMIC_RELAXED); };  // read where added
        while (b < t * per + per - 1 && below + count(b) <= s.k) below += count(b++);
        s.k -= below;
        s.before += below;
        s.prefix |= (uint64_t)b << shift;
        s.mask |= (uint64_t)(nb - 1) << shift;
        const uint32_t group = count(b);
        if (pass == kRankPasses - 1 || (uint64_t)s.before + group <= (uint64_t)K + kRankSortCap) s.done = 1;
        s.blocks_done = 0;
        *st = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kRankBins; i += blockDim.x) hist[i] = 0;
}

__device__ __forceinline__ void rank_compact_block(int d, const float *U, int nv, const float *V, uint32_t npairs,
                                                   RankState *st, uint64_t *cand, uint32_t cap, uint32_t blk,
                                                   uint32_t nblk) {
    const uint64_t prefix = st->prefix, mask = st->mask;
    for (uint64_t e = (uint64_t)blk * blockDim.x + threadIdx.x; e < npairs; e += (uint64_t)nblk * blockDim.x) {
        const uint64_t c = pair_key(d, U, nv, V, (uint32_t)e);
        if ((c & mask) <= prefix) {
            const uint32_t slot = atomicAdd(&st->cnt, 1u);
            if (slot < cap) cand[slot] = c;
        }
    }
}

// Sort of the compacted keys (padded with ~0 to a power of two p; in LDS
// when p fits, else in place in `cand`, capacity >= p), then the K smallest
// indices.
__device__ __forceinline__ void rank_sort_block(uint32_t K, const RankState *st, uint64_t *cand, uint32_t cap,
                                                uint32_t *out, uint64_t *lds) {
    const uint32_t n = st->cnt < cap ? st->cnt : cap;
    uint32_t p = 1;
    while (p < n) p <<= 1;
    uint64_t *a = p <= (uint32_t)kRankSortCap ? lds : cand;
    for (uint32_t i = threadIdx.x; i < p; i += blockDim.x) a[i] = i < n ? cand[i] : ~0ull;
    __syncthreads();
    bitonic_steps(a, p);
    for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) out[i] = (uint32_t)(a[i] & 0xffffffffu);
}


}  // namespace rank
}  // namespace gtmp
