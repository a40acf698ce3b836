// Deterministic in-block reductions for gfx950 kernels (64-wide wavefronts):
// butterflies inside a wavefront, then the wavefront partials in wavefront
// order.  Every result depends only on the data and the block shape.
#pragma once
#include <hip/hip_runtime.h>

namespace dg {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;       // the butterfly leaves the same sum in every lane
}

// Block sum (blockDim.x a multiple of 64): butterfly inside each wavefront,
// then the wavefront partials in wavefront order.  Every thread gets the sum.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
    __syncthreads();
    return r;
}

// Block sums of kn <= K accumulators at once (one barrier pair for all):
// thread c < kn writes the sum of acc[c] to out[c * ostride].
template <int K>
__device__ __forceinline__ void block_sum_cols(const double (&acc)[K], int kn, double* sh, double* out,
                                               size_t ostride) {
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int c = 0; c < K; ++c)
        if (c < kn) {
            const double v = wave_sum(acc[c]);
            if ((threadIdx.x & 63) == 0) sh[w * K + c] = v;
        }
    __syncthreads();
    if ((int)threadIdx.x < kn) {
        double r = 0.0;
        for (int i = 0; i < nw; ++i) r += sh[i * K + threadIdx.x];
        out[threadIdx.x * ostride] = r;
    }
    __syncthreads();
}

}  // namespace dg
