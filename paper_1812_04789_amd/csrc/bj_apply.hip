// Block-Jacobi apply of the smoother (Sec. 6.3; Alg. 2 SMOOTH): z = D^-1 r
// for every element block, either by the two triangular solves with the PLU
// factors or by a product with the explicit block inverse.  Factor storage is
// double or float, column-major: a[col*ld + row] with ld >= n for the
// triangular solves, ld = n for the inverses; vectors and the arithmetic
// of the apply are FP64.  These kernels stream the factors once per apply and
// are bound by HBM bandwidth.
#include "internal.h"

namespace dg {

// z = U^-1 L^-1 P r with TS-wide panels, one wavefront per element block:
// the TS x TS diagonal triangle is solved with cross-lane shuffles (each lane
// preloads its triangle row), the rows beyond it are updated by all lanes
// (coalesced reads of the factor columns).  With one wavefront per block all
// element blocks of a CU are resident together, so the sequential panel chain
// of one block overlaps with the factor streams of the others.  At most 128
// registers (four wavefronts per SIMD): 16 blocks per CU, e.g. a 16^3 mesh on
// 256 CUs, run in a single round.
constexpr int TS = 32;
constexpr int SOLVE_THREADS = 64;

// Factor and inverse entries are read once per apply, and the fine-level
// factors (GBs) are far larger than the 256 MB last-level cache: nontemporal
// loads stream them without evicting the vectors and operators that are
// reused.  Blocks small enough to stay cached (FP32 coarse inverses) use
// ordinary loads.
template <class T>
__device__ __forceinline__ T ld_stream(const T* p) { return __builtin_nontemporal_load(p); }

// Entry of a diagonal triangle, zero outside it.  FP64 factors read only the
// triangle's own entries (lanes outside it issue no load: the lower and the
// upper sweep each fetch their half of the tile); FP32 factors read the whole
// tile row unconditionally and mask, which measures faster for 4-byte loads.
template <class TF>
__device__ __forceinline__ TF tri_load(const TF* __restrict__ a, size_t idx, bool in) {
    if constexpr (sizeof(TF) == 8) {
        return in ? ld_stream(&a[idx]) : TF(0);
    } else {
        const TF v = ld_stream(&a[idx]);
        return in ? v : TF(0);
    }
}

// x[row] -= sum_{j < kb} a[(k0 + j) ld + row] x[k0 + j] for rows [r0, r1): the
// panel's factor entries of a row, all loads of a lane in flight at once.
// FP32 factors take four rows per lane when the leading dimension is a
// multiple of 4 (16-byte loads, the panel's columns in two halves of 16),
// else two rows when it is even (8-byte loads): fewer load instructions for
// the same bytes.  Rows past r1 that such a load covers lie inside the
// column (ld >= n) and are never used.
template <class TF>
__device__ __forceinline__ void panel_rows(const TF* __restrict__ a, int ld, int k0, int kb, int r0, int r1,
                                           double* x, int t) {
    if constexpr (sizeof(TF) == 4) {
        if ((ld & 3) == 0 && (r0 & 3) == 0) {
            typedef float f4v __attribute__((ext_vector_type(4)));
            for (int row = r0 + 4 * t; row < r1; row += 4 * SOLVE_THREADS) {
                double acc[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[u] = (row + u < r1) ? x[row + u] : 0.0;
#pragma unroll
                for (int h = 0; h < TS; h += 16) {
                    f4v av[16];
#pragma unroll
                    for (int j = 0; j < 16; ++j)
                        av[j] = ld_stream(reinterpret_cast<const f4v*>(&a[(size_t)(k0 + (h + j < kb ? h + j : 0)) * ld + row]));
#pragma unroll
                    for (int j = 0; j < 16; ++j)
                        if (h + j < kb) {
                            const double xj = x[k0 + h + j];
                            acc[0] -= (double)av[j].x * xj;
                            acc[1] -= (double)av[j].y * xj;
                            acc[2] -= (double)av[j].z * xj;
                            acc[3] -= (double)av[j].w * xj;
                        }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (row + u < r1) x[row + u] = acc[u];
            }
            return;
        }
        // (with r1 odd the last pair's second row lies in the column's
        // padding, ld > n: loaded, never used)
        if ((ld & 1) == 0 && (r0 & 1) == 0) {
            typedef float f2v __attribute__((ext_vector_type(2)));
            for (int row = r0 + 2 * t; row < r1; row += 2 * SOLVE_THREADS) {
                f2v av[TS];
#pragma unroll
                for (int j = 0; j < TS; ++j)
                    av[j] = ld_stream(reinterpret_cast<const f2v*>(&a[(size_t)(k0 + (j < kb ? j : 0)) * ld + row]));
                double acc0 = x[row], acc1 = (row + 1 < r1) ? x[row + 1] : 0.0;
#pragma unroll
                for (int j = 0; j < TS; ++j)
                    if (j < kb) {
                        const double xj = x[k0 + j];
                        acc0 -= (double)av[j].x * xj;
                        acc1 -= (double)av[j].y * xj;
                    }
                x[row] = acc0;
                if (row + 1 < r1) x[row + 1] = acc1;
            }
            return;
        }
    }
    for (int row = r0 + t; row < r1; row += SOLVE_THREADS) {
        TF av[TS];
#pragma unroll
        for (int j = 0; j < TS; ++j) av[j] = ld_stream(&a[(size_t)(k0 + (j < kb ? j : 0)) * ld + row]);
        double acc = x[row];
#pragma unroll
        for (int j = 0; j < TS; ++j)
            if (j < kb) acc -= (double)av[j] * x[k0 + j];
        x[row] = acc;
    }
}

template <class TF>
__global__ void __launch_bounds__(SOLVE_THREADS, 4)
    lu_solve_blocked_kernel(const TF* __restrict__ LU, const int* __restrict__ pos, const double* __restrict__ r,
                            double* __restrict__ z, int n, int ld) {
    extern __shared__ double x[];
    const TF* a = LU + (size_t)blockIdx.x * n * ld;        // column c at a + c ld
    const int* po = pos + (size_t)blockIdx.x * n;
    const double* rb = r + (size_t)blockIdx.x * n;
    const int t = threadIdx.x;
    const int lane = t & 63;
    for (int i = t; i < n; i += SOLVE_THREADS) x[i] = rb[po[i]];
    __syncthreads();
    // forward, unit lower
    for (int k0 = 0; k0 < n; k0 += TS) {
        const int kb = min(TS, n - k0);
        {
            // lane i holds row i of the diagonal triangle (loads issued together)
            TF lrow[TS];
            const int li = (lane < kb) ? lane : 0;
#pragma unroll
            for (int j = 0; j < TS; ++j)
                lrow[j] = tri_load(a, (size_t)(k0 + (j < kb ? j : 0)) * ld + k0 + li, j < kb && lane < kb && lane > j);
            double xi = (lane < kb) ? x[k0 + lane] : 0.0;
#pragma unroll
            for (int j = 0; j < TS - 1; ++j) {
                const double xj = __shfl(xi, j, 64);
                xi -= (double)lrow[j] * xj;
            }
            if (lane < kb) x[k0 + lane] = xi;
        }
        __syncthreads();
        panel_rows<TF>(a, ld, k0, kb, k0 + kb, n, x, t);
        __syncthreads();
    }
    // backward, upper
    const int nb0 = ((n - 1) / TS) * TS;
    for (int k0 = nb0; k0 >= 0; k0 -= TS) {
        const int kb = min(TS, n - k0);
        {
            TF urow[TS];
            const int ui = (lane < kb) ? lane : 0;
#pragma unroll
            for (int j = 0; j < TS; ++j)
                urow[j] = tri_load(a, (size_t)(k0 + (j < kb ? j : 0)) * ld + k0 + ui, j < kb && lane < kb && lane <= j);
            double xi = (lane < kb) ? x[k0 + lane] : 0.0;
#pragma unroll
            for (int j = TS - 1; j >= 0; --j) {
                if (j < kb) {
                    if (lane == j) xi /= (double)urow[j];
                    const double xj = __shfl(xi, j, 64);
                    if (lane < j) xi -= (double)urow[j] * xj;
                }
            }
            if (lane < kb) x[k0 + lane] = xi;
        }
        __syncthreads();
        panel_rows<TF>(a, ld, k0, kb, 0, k0, x, t);
        __syncthreads();
    }
    double* zb = z + (size_t)blockIdx.x * n;
    for (int i = t; i < n; i += SOLVE_THREADS) zb[i] = x[i];
}

template <class TF>
hipError_t launch_lu_solve_blocked(const TF* LU, const int* pos, const double* r, double* z, int nblk, int n, int ld,
                                   hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    if (ld < n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lu_solve_blocked_kernel<TF>, dim3(nblk), dim3(SOLVE_THREADS), n * sizeof(double), s, LU, pos,
                       r, z, n, ld);
    return hipGetLastError();
}
template hipError_t launch_lu_solve_blocked<double>(const double*, const int*, const double*, double*, int, int, int,
                                                    hipStream_t);
template hipError_t launch_lu_solve_blocked<float>(const float*, const int*, const double*, double*, int, int, int,
                                                   hipStream_t);

// z = X r per block with the explicit inverse (column-major, storage TF).
// Four wavefronts per block, wavefront w takes columns c = w (mod 4) two at a
// time; lane i accumulates rows i, i+64, ... (every column read is a
// contiguous run of rows); the four partial sums are added in a fixed order.
// FP64 accumulation.
constexpr int GEMV_THREADS = 256;
constexpr int GEMV_ROWS = 5;     // rows per lane (n <= 320)

template <class TF>
__global__ void __launch_bounds__(GEMV_THREADS)
    inv_gemv_kernel(const TF* __restrict__ X, const double* __restrict__ r, double* __restrict__ z, int n) {
    extern __shared__ double rs[];             // n entries of r, then 4 x n partial sums
    double* part = rs + n;
    const TF* xb = X + (size_t)blockIdx.x * n * n;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int i = t; i < n; i += GEMV_THREADS) rs[i] = r[(size_t)blockIdx.x * n + i];
    __syncthreads();
    double acc[GEMV_ROWS];
#pragma unroll
    for (int k = 0; k < GEMV_ROWS; ++k) acc[k] = 0.0;
    int c = w;
    for (; c + 4 < n; c += 8) {
        const double r0 = rs[c], r1 = rs[c + 4];
        const TF* c0 = xb + (size_t)c * n;
        const TF* c1 = xb + (size_t)(c + 4) * n;
#pragma unroll
        for (int k = 0; k < GEMV_ROWS; ++k) {
            const int i = lane + k * 64;
            if (i < n) {
                const TF x0 = (sizeof(TF) == 8) ? ld_stream(&c0[i]) : c0[i];
                const TF x1 = (sizeof(TF) == 8) ? ld_stream(&c1[i]) : c1[i];
                acc[k] = fma((double)x1, r1, fma((double)x0, r0, acc[k]));
            }
        }
    }
    for (; c < n; c += 4) {
        const double r0 = rs[c];
        const TF* c0 = xb + (size_t)c * n;
#pragma unroll
        for (int k = 0; k < GEMV_ROWS; ++k) {
            const int i = lane + k * 64;
            if (i < n) acc[k] = fma((double)((sizeof(TF) == 8) ? ld_stream(&c0[i]) : c0[i]), r0, acc[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < GEMV_ROWS; ++k) {
        const int i = lane + k * 64;
        if (i < n) part[w * n + i] = acc[k];
    }
    __syncthreads();
    for (int i = t; i < n; i += GEMV_THREADS)
        z[(size_t)blockIdx.x * n + i] = ((part[i] + part[n + i]) + part[2 * n + i]) + part[3 * n + i];
}

template <class TF>
hipError_t launch_inv_gemv(const TF* X, const double* r, double* z, int nblk, int n, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    if (n > 64 * GEMV_ROWS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(inv_gemv_kernel<TF>, dim3(nblk), dim3(GEMV_THREADS), 5 * n * sizeof(double), s, X, r, z, n);
    return hipGetLastError();
}
template hipError_t launch_inv_gemv<double>(const double*, const double*, double*, int, int, hipStream_t);
template hipError_t launch_inv_gemv<float>(const float*, const double*, double*, int, int, hipStream_t);

}  // namespace dg
