// sample.hip -- uniform layer samples (Alg. 1 "uniformly sample Q";
// Sec. III-A: N independent samples in each of the M intermediate layers).
// One thread produces four consecutive coordinates of one sample from one
// Philox4x32-10 block; the counter layout is documented in gtmp.h.
#include "gtmp_launch.hpp"

namespace gtmp {

__global__ void __launch_bounds__(256) k_sample_uniform(int M, int N, int d, uint32_t k0, uint32_t k1,
                                                        uint32_t stage, float4 lo_a, float4 lo_b, float4 w_a,
                                                        float4 w_b, float *__restrict__ Q) {
    const int nblk = (d + 3) >> 2;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t total = (uint64_t)M * N * nblk;
    if (tid >= total) return;
    const uint32_t blk = (uint32_t)(tid % nblk);
    const uint64_t mn = tid / nblk;
    const uint32_t n = (uint32_t)(mn % N), m = (uint32_t)(mn / N);
    const uint4 w = philox4x32_10(make_uint4(n, m, stage, blk), k0, k1);
    const uint32_t words[4] = {w.x, w.y, w.z, w.w};
    const float lo[8] = {lo_a.x, lo_a.y, lo_a.z, lo_a.w, lo_b.x, lo_b.y, lo_b.z, lo_b.w};
    const float wd[8] = {w_a.x, w_a.y, w_a.z, w_a.w, w_b.x, w_b.y, w_b.z, w_b.w};
    float *dst = Q + mn * d;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = (int)blk * 4 + i;
        if (j < d) {
            const int jj = j & 7;
            // single rounding of lo + u * width
            dst[j] = __builtin_fmaf(unit_from_word(words[i]), wd[jj], lo[jj]);
        }
    }
}

hipError_t launch_sample_layers(const gtmp_problem &p, uint64_t seed, uint64_t stage, float *Q, hipStream_t s) {
    float lo[8] = {0}, wd[8] = {0};
    for (int j = 0; j < p.d; ++j) {
        lo[j] = p.lo[j];
        wd[j] = p.hi[j] - p.lo[j];  // float32 width, as in the definition
    }
    const uint64_t total = (uint64_t)p.M * p.N * ((p.d + 3) / 4);
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sample_uniform, dim3(blocks), dim3(256), 0, s, p.M, p.N, p.d, (uint32_t)(seed & 0xffffffffu),
                       (uint32_t)(seed >> 32), (uint32_t)(stage & 0xffffffffu),
                       make_float4(lo[0], lo[1], lo[2], lo[3]), make_float4(lo[4], lo[5], lo[6], lo[7]),
                       make_float4(wd[0], wd[1], wd[2], wd[3]), make_float4(wd[4], wd[5], wd[6], wd[7]), Q);
    return hipGetLastError();
}

}  // namespace gtmp
