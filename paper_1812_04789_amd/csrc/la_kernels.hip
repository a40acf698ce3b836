// Vector kernels for the Krylov solvers and the p-multigrid transfer
// (Sec. 6, flexible GMRES; Sec. 6.1 restriction/prolongation).
//
// Reductions are deterministic: a fixed grid of RED_BLOCKS blocks, each
// summing a fixed grid-stride subset in a fixed order and reducing its
// threads by a fixed tree, then one block per output summing the partials in
// a fixed tree.  Results are bitwise reproducible run to run and independent
// of what else shares the device.
#include "internal.h"
#include "reduce.h"

namespace dg {

namespace {
constexpr int KCH = 8;    // dot products per pass of the multi-dot
constexpr int GS_MAXK = 64;   // largest Krylov basis handled by the Arnoldi / back-solve kernels

}  // namespace

__global__ void __launch_bounds__(RED_THREADS)
    multi_dot_stage1(const double* __restrict__ X, size_t ldx, int k0, int kn, const double* __restrict__ y, size_t n,
                     double* __restrict__ partial) {
    __shared__ double sh[RED_THREADS];
    double acc[KCH];
#pragma unroll
    for (int c = 0; c < KCH; ++c) acc[c] = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double yi = y[i];
#pragma unroll
        for (int c = 0; c < KCH; ++c)
            if (c < kn) acc[c] = fma(X[(size_t)(k0 + c) * ldx + i], yi, acc[c]);
    }
    block_sum_cols<KCH>(acc, kn, sh, partial + (size_t)k0 * gridDim.x + blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(RED_THREADS) sum_stage2(const double* __restrict__ partial, int nparts,
                                                          double* __restrict__ out) {
    __shared__ double sh[RED_THREADS];
    const double* p = partial + (size_t)blockIdx.x * nparts;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += p[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// The grid depends only on n (>= 2 entries per thread, at most RED_BLOCKS
// blocks), so the summation order is a function of n alone.
static int red_blocks(size_t n) {
    size_t b = (n + (size_t)RED_THREADS * 2 - 1) / ((size_t)RED_THREADS * 2);
    if (b < 1) b = 1;
    if (b > (size_t)RED_BLOCKS) b = RED_BLOCKS;
    return (int)b;
}

hipError_t launch_multi_dot(const double* X, size_t ldx, int nx, const double* y, size_t n, double* partial,
                            double* out, hipStream_t s) {
    const int nbk = red_blocks(n);
    for (int k0 = 0; k0 < nx; k0 += KCH) {
        const int kn = (nx - k0 < KCH) ? nx - k0 : KCH;
        hipLaunchKernelGGL(multi_dot_stage1, dim3(nbk), dim3(RED_THREADS), 0, s, X, ldx, k0, kn, y, n, partial);
    }
    hipLaunchKernelGGL(sum_stage2, dim3(nx), dim3(RED_THREADS), 0, s, partial, nbk, out);
    return hipGetLastError();
}

hipError_t launch_dot(const double* x, const double* y, size_t n, double* partial, double* out, hipStream_t s) {
    return launch_multi_dot(x, n, 1, y, n, partial, out, s);
}

// The FD step of Eq. DG-mf in two launches.  Stage 1: each block's partial
// of ||v||^2 (column 0) and, when W is given (the caller has no norm of W), of
// ||W||^2 (column 1), over the grid and per-thread order of multi_dot_stage1.
// Stage 2 (one block): the sums in the order of sum_stage2, then ||v||^2,
// ||W||^2 and h = eps sqrt(1 + ||W||) / ||v|| (0 for v = 0).  Bitwise the
// results of the separate launch_dot reductions.
__global__ void __launch_bounds__(RED_THREADS)
    fd_norms_stage1(const double* __restrict__ v, const double* __restrict__ W, size_t n,
                    double* __restrict__ partial) {
    __shared__ double sh[RED_THREADS];
    const bool withw = (W != nullptr);
    double acc[2] = {0.0, 0.0};
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double vi = v[i];
        acc[0] = fma(vi, vi, acc[0]);
        if (withw) {
            const double wi = W[i];
            acc[1] = fma(wi, wi, acc[1]);
        }
    }
    block_sum_cols<2>(acc, withw ? 2 : 1, sh, partial + blockIdx.x, gridDim.x);
}
__global__ void __launch_bounds__(RED_THREADS)
    fd_step_stage2(const double* __restrict__ partial, int nparts, int withw, const double* __restrict__ nw2_in,
                   double* __restrict__ nw2_out, double eps, double* __restrict__ nv2, double* __restrict__ h) {
    __shared__ double sh[RED_THREADS];
    double a0 = 0.0, a1 = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        a0 += partial[i];
        if (withw) a1 += partial[nparts + i];
    }
    const double s2 = block_sum(a0, sh);
    const double sw = withw ? block_sum(a1, sh) : 0.0;
    if (threadIdx.x == 0) {
        nv2[0] = s2;
        if (withw) nw2_out[0] = sw;
        const double w2 = withw ? sw : nw2_in[0];
        const double nv = sqrt(s2);
        h[0] = (nv > 0.0) ? eps * sqrt(1.0 + sqrt(w2)) / nv : 0.0;
    }
}
hipError_t launch_fd_step(const double* v, const double* W, size_t n, const double* nw2_in, double* nw2_out,
                          double eps, double* partial, double* nv2, double* h, hipStream_t s) {
    if ((W == nullptr) == (nw2_in == nullptr) || (W && !nw2_out)) return hipErrorInvalidValue;
    const int nbk = red_blocks(n);
    hipLaunchKernelGGL(fd_norms_stage1, dim3(nbk), dim3(RED_THREADS), 0, s, v, W, n, partial);
    hipLaunchKernelGGL(fd_step_stage2, dim3(1), dim3(RED_THREADS), 0, s, partial, nbk, W ? 1 : 0, nw2_in, nw2_out,
                       eps, nv2, h);
    return hipGetLastError();
}

__global__ void axpby_kernel(size_t n, double a, const double* __restrict__ x, double b, const double* y,
                             double* z) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double yi = (b != 0.0) ? b * y[i] : 0.0;
        z[i] = fma(a, x[i], yi);
    }
}
static dim3 grid_for(size_t n) {
    size_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    if (g == 0) g = 1;
    return dim3((unsigned)g);
}
hipError_t launch_axpby(size_t n, double a, const double* x, double b, const double* y, double* z, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel, grid_for(n), dim3(256), 0, s, n, a, x, b, y, z);
    return hipGetLastError();
}

// y (+/-)= sum_k c[k] X_k, coefficients read from device memory
__global__ void multi_axpy_kernel(size_t n, int k, const double* __restrict__ c, int sign,
                                  const double* __restrict__ X, size_t ldx, double* __restrict__ y) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc = fma(c[j], X[(size_t)j * ldx + i], acc);
        y[i] = (sign < 0) ? y[i] - acc : y[i] + acc;
    }
}
hipError_t launch_multi_axpy(size_t n, int k, const double* c, int sign, const double* X, size_t ldx, double* y,
                             hipStream_t s) {
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(multi_axpy_kernel, grid_for(n), dim3(256), 0, s, n, k, c, sign, X, ldx, y);
    return hipGetLastError();
}

__global__ void scale_dev_kernel(size_t n, const double* __restrict__ x, const double* __restrict__ sc, int invert,
                                 double* __restrict__ y) {
    const double a = invert ? ((sc[0] != 0.0) ? 1.0 / sc[0] : 0.0) : sc[0];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = a * x[i];
}
hipError_t launch_scale_dev(size_t n, const double* x, const double* sc, int invert, double* y, hipStream_t s) {
    hipLaunchKernelGGL(scale_dev_kernel, grid_for(n), dim3(256), 0, s, n, x, sc, invert, y);
    return hipGetLastError();
}

__global__ void copy_kernel(size_t n, const double* __restrict__ x, double* __restrict__ y) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = x[i];
}
hipError_t launch_copy(size_t n, const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(copy_kernel, grid_for(n), dim3(256), 0, s, n, x, y);
    return hipGetLastError();
}
__global__ void fill_kernel(size_t n, double v, double* __restrict__ y) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = v;
}
hipError_t launch_fill(size_t n, double v, double* y, hipStream_t s) {
    hipLaunchKernelGGL(fill_kernel, grid_for(n), dim3(256), 0, s, n, v, y);
    return hipGetLastError();
}

// Restriction to the first nvc modes of every (element, equation) run.
__global__ void restrict_kernel(size_t nc, int nvf, int nvc, const double* __restrict__ fine,
                                double* __restrict__ coarse) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
        const size_t run = i / nvc;
        const int m = (int)(i % nvc);
        coarse[i] = fine[run * nvf + m];
    }
}
hipError_t launch_restrict(int ne, int nvf, int nvc, const double* fine, double* coarse, hipStream_t s) {
    const size_t nc = (size_t)ne * 5 * nvc;
    hipLaunchKernelGGL(restrict_kernel, grid_for(nc), dim3(256), 0, s, nc, nvf, nvc, fine, coarse);
    return hipGetLastError();
}
// Prolongation (zero padding of the fine modes), added to or written over fine.
__global__ void prolong_kernel(size_t nf, int nvf, int nvc, const double* __restrict__ coarse,
                               double* __restrict__ fine, int overwrite) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += stride) {
        const size_t run = i / nvf;
        const int m = (int)(i % nvf);
        const double c = (m < nvc) ? coarse[run * nvc + m] : 0.0;
        fine[i] = overwrite ? c : fine[i] + c;
    }
}
hipError_t launch_prolong_add(int ne, int nvf, int nvc, const double* coarse, double* fine, int overwrite,
                              hipStream_t s) {
    const size_t nf = (size_t)ne * 5 * nvf;
    hipLaunchKernelGGL(prolong_kernel, grid_for(nf), dim3(256), 0, s, nf, nvf, nvc, coarse, fine, overwrite);
    return hipGetLastError();
}

__global__ void nonfinite_kernel(size_t n, const double* __restrict__ x, int* flag) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if (!isfinite(x[i])) bad = 1;
    if (bad) atomicOr(flag, 1);
}
hipError_t launch_count_nonfinite(size_t n, const double* x, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(nonfinite_kernel, grid_for(n), dim3(256), 0, s, n, x, flag);
    return hipGetLastError();
}

__global__ void f64_to_f32_kernel(const double* __restrict__ x, float* __restrict__ y, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = (float)x[i];
}
// FP64 -> BF16 bits: round to FP32 (nearest even), then to BF16 (nearest even).
__global__ void f64_to_bf16_kernel(const double* __restrict__ x, unsigned short* __restrict__ y, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const unsigned int b = __float_as_uint((float)x[i]);
        const unsigned int r = b + 0x7FFFu + ((b >> 16) & 1u);
        y[i] = (unsigned short)(r >> 16);
    }
}
hipError_t launch_convert_fp64_to_bf16(const double* x, unsigned short* y, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(f64_to_bf16_kernel, grid_for(n), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

hipError_t launch_convert_fp64_to_fp32(const double* x, float* y, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(f64_to_f32_kernel, grid_for(n), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

// ---- GMRES small dense algebra on the device ---------------------------------------------
// y = R^-1 g[0:k] for the k x k upper triangle of H.  After a breakdown
// (zero new direction) the trailing columns are exactly zero: they are dropped.
__global__ void __launch_bounds__(256) backsolve_kernel(const double* H, int ldh, int k, const double* g, double* y) {
    // the k x k triangle and g staged in LDS by all threads, then one thread solves
    __shared__ double sH[GS_MAXK * GS_MAXK];
    __shared__ double sg[GS_MAXK], sy[GS_MAXK];
    for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
        const int c = t / k, i = t % k;
        sH[c * GS_MAXK + i] = H[(size_t)c * ldh + i];
    }
    for (int t = threadIdx.x; t < k; t += blockDim.x) sg[t] = g[t];
    __syncthreads();
    if (threadIdx.x == 0) {
        int ke = k;
        for (int i = 0; i < k; ++i)
            if (!(fabs(sH[i * GS_MAXK + i]) > 0.0)) { ke = i; break; }
        for (int i = ke; i < k; ++i) sy[i] = 0.0;
        for (int i = ke - 1; i >= 0; --i) {
            double s = sg[i];
            for (int c = i + 1; c < ke; ++c) s -= sH[c * GS_MAXK + i] * sy[c];
            sy[i] = s / sH[i * GS_MAXK + i];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < k; t += blockDim.x) y[t] = sy[t];
}
__global__ void init_g_kernel(double* g, int len, const double* beta2) {
    for (int i = 0; i < len; ++i) g[i] = 0.0;
    g[0] = sqrt(beta2[0]);
}

hipError_t launch_backsolve(const double* H, int ldh, int k, const double* g, double* y, hipStream_t s) {
    if (k < 1 || k > GS_MAXK) return hipErrorInvalidValue;
    hipLaunchKernelGGL(backsolve_kernel, dim3(1), dim3(256), 0, s, H, ldh, k, g, y);
    return hipGetLastError();
}
hipError_t launch_init_g(double* g, int len, const double* beta2, hipStream_t s) {
    hipLaunchKernelGGL(init_g_kernel, dim3(1), dim3(1), 0, s, g, len, beta2);
    return hipGetLastError();
}

// ---- fused classical Gram-Schmidt (applied twice) for one Arnoldi step -----------------------
// Step j, w = V[j+1], basis V[0..j]; three launches, no inter-block
// synchronisation inside a launch:
//   K1  pa = per-block partials of V_i . w                     (i <= j)
//   K2  h  = sum of pa (every block; block 0 stores H column j);
//       w -= sum_i h_i V_i ; pb = partials of V_i . w (second pass, i <= j)
//       and of w . w (column j + 1)
//   K3  h2, ||w||^2 = sums of pb (every block); the norm after the second
//       update by Pythagoras, ||w - V h2||^2 = ||w||^2 - ||h2||^2 (exact for
//       orthonormal V; after the first pass h2 is at rounding level against
//       w, so the difference keeps full relative precision), clamped at 0;
//       w <- (w - sum_i h2_i V_i) / norm; block 0: H column j += h2,
//       H[j+1,j] = norm, Givens rotation j, est = |g_{j+1}|
// Every block sums the previous launch's partials in the same fixed order,
// so all blocks hold bitwise the same coefficients and the result depends
// only on the data.  pa and pb are disjoint (K2 reads one set while writing
// the other).
constexpr int GS_CH = 16;
constexpr int GS_BLOCKS = 256;
static_assert(2 * GS_MAXK * RED_BLOCKS + (GS_MAXK + 1) * GS_BLOCKS <= RED_BLOCKS * 256,
              "the partial buffer holds the first-pass set and the second-pass set with its norm column");

// out[c] = sum_{b < nparts} part[c * nparts + b] for c < k <= 65, into LDS
// (all threads see it after the call).  A group of g threads (a power of two,
// g k <= blockDim.x, g <= 64) takes output c: thread i of the group sums
// b = i, i + g, ... into eight accumulators (b = i + g (8 m + u) into u, the
// eight loads of a round in flight together; the last partial round into
// accumulator 0), adds them pairwise, then the group reduces by butterfly.  The order depends only on
// (nparts, k, blockDim.x).
__device__ __forceinline__ void sum_parts(const double* __restrict__ part, int nparts, int k, double* out) {
    int g = 64;
    while (g > 1 && g * k > (int)blockDim.x) g >>= 1;
    const int c = threadIdx.x / g, i = threadIdx.x % g;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (c < k) {
        const double* pc = part + (size_t)c * nparts;
        int b = i;
        for (; b + 7 * g < nparts; b += 8 * g) {
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = pc[b + u * g];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += x[u];
        }
        for (; b < nparts; b += g) acc[0] += pc[b];
    }
    double a = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    for (int o = g >> 1; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (c < k && i == 0) out[c] = a;
    __syncthreads();
}

// part[c * grid + block] = partial of V_c . w over this block's entries, c < k
__device__ __forceinline__ void gs_block_dots(const double* __restrict__ V, size_t n, int k,
                                              const double* __restrict__ w, double* __restrict__ part, double* sh) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (int c0 = 0; c0 < k; c0 += GS_CH) {
        double acc[GS_CH];
#pragma unroll
        for (int c = 0; c < GS_CH; ++c) acc[c] = 0.0;
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
            const double wi = w[i];
#pragma unroll
            for (int c = 0; c < GS_CH; ++c)
                if (c0 + c < k) acc[c] = fma(V[(size_t)(c0 + c) * n + i], wi, acc[c]);
        }
        block_sum_cols<GS_CH>(acc, min(GS_CH, k - c0), sh, part + (size_t)c0 * gridDim.x + blockIdx.x, gridDim.x);
    }
}

__global__ void __launch_bounds__(RED_THREADS)
    gs_dots_kernel(const double* __restrict__ V, size_t n, int k, const double* __restrict__ w,
                   double* __restrict__ pa) {
    __shared__ double sh[RED_THREADS];
    gs_block_dots(V, n, k, w, pa, sh);
}

// K2: coefficients from the first-pass partials, w -= sum_i c_i V_i, then the
// second-pass dots (columns 0..k-1 of pout) and ||w||^2 (column k).
__global__ void __launch_bounds__(RED_THREADS)
    gs_update_kernel(const double* __restrict__ V, size_t n, int k, const double* __restrict__ pin, int np_in,
                     double* __restrict__ cout, double* __restrict__ w, double* __restrict__ pout) {
    __shared__ double sh[RED_THREADS];
    __shared__ double hs[GS_MAXK];
    sum_parts(pin, np_in, k, hs);
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < k; i += blockDim.x) cout[i] = hs[i];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    double nrm = 0.0;
    if (k <= 2 * GS_CH) {
        // one pass: the basis entries of a row stay in registers for the
        // update and the dots (the same per-thread sums as the two passes)
        double a0[GS_CH], a1[GS_CH];
#pragma unroll
        for (int c = 0; c < GS_CH; ++c) a0[c] = a1[c] = 0.0;
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
            double v[2 * GS_CH];
#pragma unroll
            for (int c = 0; c < 2 * GS_CH; ++c) v[c] = (c < k) ? V[(size_t)c * n + i] : 0.0;
            double wi = w[i];
#pragma unroll
            for (int c = 0; c < 2 * GS_CH; ++c)
                if (c < k) wi -= hs[c] * v[c];
            w[i] = wi;
            nrm = fma(wi, wi, nrm);
#pragma unroll
            for (int c = 0; c < GS_CH; ++c) {
                if (c < k) a0[c] = fma(v[c], wi, a0[c]);
                if (GS_CH + c < k) a1[c] = fma(v[GS_CH + c], wi, a1[c]);
            }
        }
        block_sum_cols<GS_CH>(a0, min(GS_CH, k), sh, pout + blockIdx.x, gridDim.x);
        if (k > GS_CH) block_sum_cols<GS_CH>(a1, k - GS_CH, sh, pout + (size_t)GS_CH * gridDim.x + blockIdx.x, gridDim.x);
    } else {
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
            double wi = w[i];
            for (int c = 0; c < k; ++c) wi -= hs[c] * V[(size_t)c * n + i];
            w[i] = wi;
            nrm = fma(wi, wi, nrm);
        }
        gs_block_dots(V, n, k, w, pout, sh);
    }
    const double sm = block_sum(nrm, sh);
    if (threadIdx.x == 0) pout[(size_t)k * gridDim.x + blockIdx.x] = sm;
}

// K3: second update and normalisation from the second-pass partials; block 0
// finishes H column j (first-pass coefficients already there) and the Givens
// rotation.
__global__ void __launch_bounds__(RED_THREADS)
    gs_update_normalise_kernel(const double* __restrict__ V, size_t n, int k, const double* __restrict__ pin,
                               int np_in, double* __restrict__ w, double* H, int ldh, double* cs, double* sn,
                               double* g, double* nrm_out, double* est) {
    __shared__ double hs[GS_MAXK + 1];
    sum_parts(pin, np_in, k + 1, hs);
    double h22 = 0.0;
    for (int c = 0; c < k; ++c) h22 = fma(hs[c], hs[c], h22);
    const double nr2 = hs[k] - h22;
    const double nr = (nr2 > 0.0) ? sqrt(nr2) : 0.0;
    const double a = (nr != 0.0) ? 1.0 / nr : 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double wi = w[i];
        for (int c = 0; c < k; ++c) wi -= hs[c] * V[(size_t)c * n + i];
        w[i] = a * wi;
    }
    if (blockIdx.x != 0) return;
    const int j = k - 1;
    __shared__ double sh_h[GS_MAXK + 1], sh_c[GS_MAXK], sh_s[GS_MAXK];
    double* h = H + (size_t)j * ldh;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        sh_h[i] = h[i] + hs[i];
        sh_c[i] = cs[i];
        sh_s[i] = sn[i];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    sh_h[j + 1] = nr;
    nrm_out[0] = nr;
    for (int i = 0; i < j; ++i) {
        const double t = sh_c[i] * sh_h[i] + sh_s[i] * sh_h[i + 1];
        sh_h[i + 1] = -sh_s[i] * sh_h[i] + sh_c[i] * sh_h[i + 1];
        sh_h[i] = t;
    }
    const double x = sh_h[j], y = sh_h[j + 1];
    const double r = hypot(x, y);
    const double c = (r > 0.0) ? x / r : 1.0, sg = (r > 0.0) ? y / r : 0.0;
    cs[j] = c;
    sn[j] = sg;
    sh_h[j] = r;
    sh_h[j + 1] = 0.0;
    for (int i = 0; i <= j + 1; ++i) h[i] = sh_h[i];
    const double gj = g[j];
    g[j + 1] = -sg * gj;
    g[j] = c * gj;
    est[0] = fabs(g[j + 1]);
}

static hipError_t arnoldi_tail(const double* V, size_t n, int j, double* H, int ldh, double* cs, double* sn,
                               double* g, double* nrm, double* est, double* partial, int np_a, hipStream_t s) {
    const int k = j + 1;
    const int nbk = red_blocks(n) < GS_BLOCKS ? red_blocks(n) : GS_BLOCKS;
    double* w = const_cast<double*>(V) + (size_t)k * n;
    double* hcol = H + (size_t)j * ldh;
    double* pa = partial;
    double* pb = partial + (size_t)GS_MAXK * RED_BLOCKS;
    hipLaunchKernelGGL(gs_update_kernel, dim3(nbk), dim3(RED_THREADS), 0, s, V, n, k, pa, np_a, hcol, w, pb);
    hipLaunchKernelGGL(gs_update_normalise_kernel, dim3(nbk), dim3(RED_THREADS), 0, s, V, n, k, pb, nbk, w, H, ldh,
                       cs, sn, g, nrm, est);
    return hipGetLastError();
}

hipError_t launch_arnoldi_cgs2(const double* V, size_t n, int j, double* H, int ldh, double* cs, double* sn,
                               double* g, double* nrm, double* est, double* partial, hipStream_t s) {
    const int k = j + 1;
    if (k > GS_MAXK) return hipErrorInvalidValue;
    // at most one block per CU: every block re-reads all partials of a set
    const int nbk = red_blocks(n) < GS_BLOCKS ? red_blocks(n) : GS_BLOCKS;
    double* w = const_cast<double*>(V) + (size_t)k * n;
    hipLaunchKernelGGL(gs_dots_kernel, dim3(nbk), dim3(RED_THREADS), 0, s, V, n, k, w, partial);
    return arnoldi_tail(V, n, j, H, ldh, cs, sn, g, nrm, est, partial, nbk, s);
}

hipError_t launch_arnoldi_cgs2_after_dots(const double* V, size_t n, int j, double* H, int ldh, double* cs,
                                          double* sn, double* g, double* nrm, double* est, double* partial, int np_a,
                                          hipStream_t s) {
    if (j + 1 > GS_MAXK || np_a < 1 || np_a > RED_BLOCKS) return hipErrorInvalidValue;
    return arnoldi_tail(V, n, j, H, ldh, cs, sn, g, nrm, est, partial, np_a, s);
}

// ---- per-case FD steps of a batch ------------------------------------------------------------
// Case c's squared norms are summed exactly as the single-case reduction of
// its n_c entries (red_blocks(n_c) blocks, the same grid stride, the same
// trees), so the step h_c is bitwise the one a single-case product uses.
int red_blocks_for(size_t n) { return red_blocks(n); }

__global__ void __launch_bounds__(RED_THREADS)
    seg_sq_stage1(const SegBlock* __restrict__ tab, const double* __restrict__ x, const double* __restrict__ y,
                  double* __restrict__ px, double* __restrict__ py) {
    __shared__ double sh[RED_THREADS];
    const SegBlock b = tab[blockIdx.x];
    const size_t stride = (size_t)b.nbk * blockDim.x;
    double ax = 0.0, ay = 0.0;
    for (size_t i = (size_t)b.lb * blockDim.x + threadIdx.x; i < b.n; i += stride) {
        const double xi = x[b.off + i], yi = y[b.off + i];
        ax = fma(xi, xi, ax);
        ay = fma(yi, yi, ay);
    }
    const double sx = block_sum(ax, sh);
    const double sy = block_sum(ay, sh);
    if (threadIdx.x == 0) {
        px[blockIdx.x] = sx;
        py[blockIdx.x] = sy;
    }
}

__global__ void __launch_bounds__(RED_THREADS)
    seg_fd_step(const int* __restrict__ first, const int* __restrict__ nbk, const double* __restrict__ px,
                const double* __restrict__ py, double eps, double* __restrict__ h) {
    __shared__ double sh[RED_THREADS];
    const int c = blockIdx.x;
    const double* a = px + first[c];
    const double* b = py + first[c];
    double ax = 0.0, ay = 0.0;
    for (int i = threadIdx.x; i < nbk[c]; i += blockDim.x) ax += a[i];
    for (int i = threadIdx.x; i < nbk[c]; i += blockDim.x) ay += b[i];
    const double nw2 = block_sum(ax, sh);
    const double nv2 = block_sum(ay, sh);
    if (threadIdx.x == 0) {
        const double nv = sqrt(nv2);
        h[c] = (nv > 0.0) ? eps * sqrt(1.0 + sqrt(nw2)) / nv : 0.0;
    }
}

hipError_t launch_seg_fd_step(const SegBlock* tab, int nblocks, const int* first, const int* nbk, int ncases,
                              const double* W, const double* v, double* px, double* py, double eps, double* h,
                              hipStream_t s) {
    if (nblocks <= 0 || ncases <= 0) return hipSuccess;
    hipLaunchKernelGGL(seg_sq_stage1, dim3(nblocks), dim3(RED_THREADS), 0, s, tab, W, v, px, py);
    hipLaunchKernelGGL(seg_fd_step, dim3(ncases), dim3(RED_THREADS), 0, s, first, nbk, px, py, eps, h);
    return hipGetLastError();
}

}  // namespace dg
