// Element block-Jacobi (Sec. 6.3): batched PLU with partial pivoting of the
// element diagonal blocks and the block solves z = D^-1 r used by the
// smoother.  Blocks are column-major (a[col*n + row]); one workgroup per
// block.  Factor storage type TF is double or float (vectors stay FP64 and
// the solve arithmetic is FP64).
#include "internal.h"

namespace dg {

constexpr int LU_THREADS = 256;

// Right-looking PLU.  Per step k: pivot search (max |a_ik|, lowest index on
// ties), row exchange over all columns, scaling of the multipliers, rank-1
// update of the trailing matrix with the pivot row and multiplier column
// staged in LDS.
template <class TF>
__global__ void __launch_bounds__(LU_THREADS) lu_kernel(TF* __restrict__ A, int* __restrict__ piv, int n) {
    extern __shared__ double lds[];
    double* colk = lds;          // multipliers l_ik, i > k
    double* rowk = lds + n;      // pivot row u_kj, j > k
    __shared__ double rv[LU_THREADS];
    __shared__ int ri[LU_THREADS];
    TF* a = A + (size_t)blockIdx.x * n * n;
    int* pv = piv + (size_t)blockIdx.x * n;
    const int t = threadIdx.x;
    for (int k = 0; k < n; ++k) {
        // pivot search
        double best = -1.0;
        int bi = n;
        for (int r = k + t; r < n; r += LU_THREADS) {
            const double v = fabs((double)a[(size_t)k * n + r]);
            if (v > best) { best = v; bi = r; }
        }
        rv[t] = best;
        ri[t] = bi;
        __syncthreads();
        for (int s = LU_THREADS / 2; s > 0; s >>= 1) {
            if (t < s) {
                const double v2 = rv[t + s];
                const int i2 = ri[t + s];
                if (v2 > rv[t] || (v2 == rv[t] && i2 < ri[t])) { rv[t] = v2; ri[t] = i2; }
            }
            __syncthreads();
        }
        int p = ri[0];
        if (p < k || p >= n) p = k;      // no finite candidate (NaN column): keep the row
        __syncthreads();
        if (t == 0) pv[k] = p;
        if (p != k)
            for (int j = t; j < n; j += LU_THREADS) {
                const TF x = a[(size_t)j * n + k];
                a[(size_t)j * n + k] = a[(size_t)j * n + p];
                a[(size_t)j * n + p] = x;
            }
        __syncthreads();
        const double inv = 1.0 / (double)a[(size_t)k * n + k];
        for (int r = k + 1 + t; r < n; r += LU_THREADS) {
            const TF l = (TF)((double)a[(size_t)k * n + r] * inv);
            a[(size_t)k * n + r] = l;
            colk[r] = (double)l;
        }
        for (int j = k + 1 + t; j < n; j += LU_THREADS) rowk[j] = (double)a[(size_t)j * n + k];
        __syncthreads();
        const int m = n - k - 1;
        const size_t tot = (size_t)m * m;
        for (size_t idx = t; idx < tot; idx += LU_THREADS) {
            const int j = k + 1 + (int)(idx / m);
            const int r = k + 1 + (int)(idx % m);
            TF& x = a[(size_t)j * n + r];
            x = (TF)((double)x - colk[r] * rowk[j]);
        }
        __syncthreads();
    }
}

template <class TF>
hipError_t launch_lu(TF* A, int* piv, int nblk, int n, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(lu_kernel<TF>, dim3(nblk), dim3(LU_THREADS), 2 * n * sizeof(double), s, A, piv, n);
    return hipGetLastError();
}
template hipError_t launch_lu<double>(double*, int*, int, int, hipStream_t);
template hipError_t launch_lu<float>(float*, int*, int, int, hipStream_t);

// z = U^-1 L^-1 P r per block: the right-hand side lives in LDS, the
// column-oriented substitutions read contiguous factor columns.
template <class TF>
__global__ void __launch_bounds__(LU_THREADS)
    lu_solve_kernel(const TF* __restrict__ LU, const int* __restrict__ piv, const double* __restrict__ r,
                    double* __restrict__ z, int n) {
    extern __shared__ double x[];
    const TF* a = LU + (size_t)blockIdx.x * n * n;
    const int* pv = piv + (size_t)blockIdx.x * n;
    const double* rb = r + (size_t)blockIdx.x * n;
    const int t = threadIdx.x;
    for (int i = t; i < n; i += LU_THREADS) x[i] = rb[i];
    __syncthreads();
    if (t == 0)
        for (int k = 0; k < n; ++k) {
            const int p = pv[k];
            if (p != k && p > k && p < n) {
                const double s = x[k];
                x[k] = x[p];
                x[p] = s;
            }
        }
    __syncthreads();
    for (int k = 0; k < n - 1; ++k) {           // unit lower
        const double xk = x[k];
        for (int i = k + 1 + t; i < n; i += LU_THREADS) x[i] -= (double)a[(size_t)k * n + i] * xk;
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {          // upper
        const double xk = x[k] / (double)a[(size_t)k * n + k];
        __syncthreads();
        if (t == 0) x[k] = xk;
        for (int i = t; i < k; i += LU_THREADS) x[i] -= (double)a[(size_t)k * n + i] * xk;
        __syncthreads();
    }
    double* zb = z + (size_t)blockIdx.x * n;
    for (int i = t; i < n; i += LU_THREADS) zb[i] = x[i];
}

template <class TF>
hipError_t launch_lu_solve(const TF* LU, const int* piv, const double* r, double* z, int nblk, int n,
                           hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(lu_solve_kernel<TF>, dim3(nblk), dim3(LU_THREADS), n * sizeof(double), s, LU, piv, r, z, n);
    return hipGetLastError();
}
template hipError_t launch_lu_solve<double>(const double*, const int*, const double*, double*, int, int, hipStream_t);
template hipError_t launch_lu_solve<float>(const float*, const int*, const double*, double*, int, int, hipStream_t);

// Coarse principal sub-block: rows/columns (a, i), i < nvc, of the fine block
// whose local index is a*nvf + i; output local index a*nvc + i.
template <class TF>
__global__ void extract_sub_kernel(const double* __restrict__ fine, int nbf, int nvf, int nvc, TF* __restrict__ out) {
    const int nbc = 5 * nvc;
    const double* fb = fine + (size_t)blockIdx.x * nbf * nbf;
    TF* ob = out + (size_t)blockIdx.x * nbc * nbc;
    for (int idx = threadIdx.x; idx < nbc * nbc; idx += blockDim.x) {
        const int jc = idx / nbc, ic = idx % nbc;
        const int jf = (jc / nvc) * nvf + jc % nvc, i_f = (ic / nvc) * nvf + ic % nvc;
        ob[idx] = (TF)fb[(size_t)jf * nbf + i_f];
    }
}
template <class TF>
hipError_t launch_extract_sub(const double* fine, int nbf, int nvf, int nvc, TF* out, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(extract_sub_kernel<TF>, dim3(nblk), dim3(256), 0, s, fine, nbf, nvf, nvc, out);
    return hipGetLastError();
}
template hipError_t launch_extract_sub<double>(const double*, int, int, int, double*, int, hipStream_t);
template hipError_t launch_extract_sub<float>(const double*, int, int, int, float*, int, hipStream_t);

}  // namespace dg
