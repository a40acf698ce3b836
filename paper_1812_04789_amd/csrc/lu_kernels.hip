// Element block-Jacobi (Sec. 6.3): batched PLU with partial pivoting of the
// element diagonal blocks, the simple per-block solve of the library's
// batched-LU entry point, coarse sub-block extraction and the explicit block
// inverse.  Blocks are column-major (a[col*n + row]); one workgroup per
// block.  Factor storage type TF is double or float.  The smoother's apply
// kernels are in bj_apply.hip.
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
__global__ void extract_sub_kernel(const double* __restrict__ fine, int nbf, int ldf, int nvf, int nvc,
                                   TF* __restrict__ out) {
    const int nbc = 5 * nvc;
    const double* fb = fine + (size_t)blockIdx.x * nbf * ldf;
    TF* ob = out + (size_t)blockIdx.x * nbc * nbc;
    for (int idx = threadIdx.x; idx < nbc * nbc; idx += blockDim.x) {
        const int jc = idx / nbc, ic = idx % nbc;
        const int jf = (jc / nvc) * nvf + jc % nvc, i_f = (ic / nvc) * nvf + ic % nvc;
        ob[idx] = (TF)fb[(size_t)jf * ldf + i_f];
    }
}
template <class TF>
hipError_t launch_extract_sub(const double* fine, int nbf, int ldf, int nvf, int nvc, TF* out, int nblk,
                              hipStream_t s) {
    if (ldf < nbf) return hipErrorInvalidValue;
    hipLaunchKernelGGL(extract_sub_kernel<TF>, dim3(nblk), dim3(256), 0, s, fine, nbf, ldf, nvf, nvc, out);
    return hipGetLastError();
}
template hipError_t launch_extract_sub<double>(const double*, int, int, int, int, double*, int, hipStream_t);
template hipError_t launch_extract_sub<float>(const double*, int, int, int, int, float*, int, hipStream_t);

// ---- blocked variants used by the smoother -------------------------------------------------
// Right-looking PLU with column panels.  The panel (rows k0..n-1) is factored
// in LDS (pivot search, row exchange, scaling, rank-1 updates); every other
// column then takes the panel's row exchanges and, right of the panel, its
// U12 = L11^-1 A12 entries; the trailing matrix A22 -= L21 U12 is updated on
// the matrix cores.  Pivots are the partial-pivoting choices of the unblocked
// kernel (max |a_ik|, lowest index on ties); only the summation order of the
// trailing updates differs.

// Largest |value| with the lowest row index on ties, over the block: a
// butterfly inside each wavefront, then the wavefront winners in order.
template <class TA>
__device__ __forceinline__ int block_argmax(TA v, int r, TA* sv, int* sr) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const TA v2 = __shfl_xor(v, o, 64);
        const int r2 = __shfl_xor(r, o, 64);
        if (v2 > v || (v2 == v && r2 < r)) { v = v2; r = r2; }
    }
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) { sv[w] = v; sr[w] = r; }
    __syncthreads();
    TA bv = sv[0];
    int br = sr[0];
    for (int i = 1; i < nw; ++i)
        if (sv[i] > bv || (sv[i] == bv && sr[i] < br)) { bv = sv[i]; br = sr[i]; }
    return br;
}

// A22 -= L21 U12 for one panel with 16 x 16 x 4 matrix-core instructions,
// computed as its transpose U12^T L21^T so that the lanes of a result run
// down a column of A22 (contiguous in the column-major block).  Wavefront w
// of the block takes the 16-column strips w, w + 4, ... of A22: the strip's
// U12 entries stay in registers while the wavefront walks down the strip,
// UPD_G tiles at a time (all their loads issued before the first store, so
// the memory latency of the group overlaps).  In a tile lane l holds
//   A operand:  U12[kk + l/16][c0 + l%16],
//   B operand: -L21[r0 + l%16][kk + l/16]    (LDS panel),
//   accumulator item i: row r0 + l%16 of A22, column c0 + l/16 + 4 i (FP64)
//   or c0 + 4 (l/16) + i (FP32): the two instructions order their results
//   differently across the lanes.
// The accumulator starts from the A22 tile, so each entry becomes
// a - sum_k l_k u_k accumulated in panel order.  Out-of-range rows and
// columns enter as zeros and are not stored.
constexpr int UPD_G = 2;
template <class TF, class TA, int NBW>
__device__ __forceinline__ void trailing_update_mfma(TF* __restrict__ a, const TA* P, int n, int ld, int k0, int kb,
                                                     int n2, int t) {
    typedef TA acc4 __attribute__((ext_vector_type(4)));
    static_assert(NBW % 4 == 0, "the panel width is a multiple of the instruction's K = 4");
    static_assert(LU_THREADS % 64 == 0, "whole wavefronts");
    constexpr int NK = NBW / 4;
    const int lane = t & 63, wv = t >> 6, nwv = LU_THREADS / 64;
    const int li = lane & 15, lk = lane >> 4;
    const int nt = (n2 + 15) / 16;
    TF* a22 = a + (size_t)(k0 + kb) * ld + k0 + kb;         // A22[r][c] = a22[c ld + r]
    const TA* l21 = P + kb;                                  // L21[r][k] = l21[k n + r]
    for (int st = wv; st < nt; st += nwv) {
        const int c0 = st * 16;
        const bool cok = c0 + li < n2;
        const TF* ucol = a + (size_t)(k0 + kb + (cok ? c0 + li : 0)) * ld + k0;
        TA uv[NK];
#pragma unroll
        for (int q = 0; q < NK; ++q) {
            const int k = 4 * q + lk;
            uv[q] = (cok && k < kb) ? (TA)ucol[k] : TA(0);
        }
        int cc[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) cc[i] = (sizeof(TA) == 8) ? c0 + lk + 4 * i : c0 + 4 * lk + i;
        for (int r0 = 0; r0 < n2; r0 += 16 * UPD_G) {
            acc4 acc[UPD_G];
#pragma unroll
            for (int g = 0; g < UPD_G; ++g) {
                const int r = r0 + 16 * g + li;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[g][i] = (r < n2 && cc[i] < n2) ? (TA)a22[(size_t)cc[i] * ld + r] : TA(0);
            }
#pragma unroll
            for (int g = 0; g < UPD_G; ++g) {
                const int r = r0 + 16 * g + li;
#pragma unroll
                for (int q = 0; q < NK; ++q) {
                    const int k = 4 * q + lk;
                    const TA lv = (r < n2 && k < kb) ? -l21[k * n + r] : TA(0);
                    if constexpr (sizeof(TA) == 8)
                        acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(uv[q], lv, acc[g], 0, 0, 0);
                    else
                        acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(uv[q], lv, acc[g], 0, 0, 0);
                }
            }
#pragma unroll
            for (int g = 0; g < UPD_G; ++g) {
                const int r = r0 + 16 * g + li;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (r < n2 && cc[i] < n2) a22[(size_t)cc[i] * ld + r] = (TF)acc[g][i];
            }
        }
    }
}

// TF: storage type of the blocks; TA: arithmetic of the factorisation (the
// panel in LDS and every update); NBW: panel width.  FP64 blocks: double,
// 16 columns; FP32 blocks: float arithmetic, 32 columns (the same 40 KB panel,
// half the trailing-matrix passes).
template <class TF, class TA, int NBW>
__global__ void __launch_bounds__(LU_THREADS) lu_blocked_kernel(TF* __restrict__ A, int* __restrict__ piv, int n,
                                                                int ld) {
    extern __shared__ double lds_raw[];
    TA* P = reinterpret_cast<TA*>(lds_raw);  // panel, column-major with stride n: P[c*n + r], r < m
    __shared__ TA wv[LU_THREADS / 64];
    __shared__ int wr[LU_THREADS / 64];
    __shared__ int spiv[NBW];
    // perm[r]: the row (relative to k0) whose content row r holds after the
    // panel's exchanges so far
    int* perm = reinterpret_cast<int*>(P + (size_t)NBW * n);
    TF* a = A + (size_t)blockIdx.x * n * ld;                 // column c at a + c ld
    int* pv = piv + (size_t)blockIdx.x * n;
    const int t = threadIdx.x;
    for (int k0 = 0; k0 < n; k0 += NBW) {
        const int kb = min(NBW, n - k0), m = n - k0;
        for (int r = t; r < m; r += LU_THREADS) perm[r] = r;
        for (int idx = t; idx < m * kb; idx += LU_THREADS) {
            const int c = idx / m, r = idx % m;
            P[c * n + r] = (TA)a[(size_t)(k0 + c) * ld + k0 + r];
        }
        __syncthreads();
        for (int j = 0; j < kb; ++j) {
            TA best = -1;
            int bi = m;
            for (int r = j + t; r < m; r += LU_THREADS) {
                const TA v = fabs(P[j * n + r]);
                if (v > best) { best = v; bi = r; }
            }
            int p = block_argmax<TA>(best, bi, wv, wr);
            if (p < j || p >= m) p = j;
            if (t == 0) {
                spiv[j] = p;
                pv[k0 + j] = k0 + p;
                const int x = perm[j];
                perm[j] = perm[p];
                perm[p] = x;
            }
            if (p != j && t < kb) {
                const TA x = P[t * n + j];
                P[t * n + j] = P[t * n + p];
                P[t * n + p] = x;
            }
            __syncthreads();
            const TA inv = TA(1) / P[j * n + j];
            for (int r = j + 1 + t; r < m; r += LU_THREADS) {
                const TA l = P[j * n + r] * inv;
                P[j * n + r] = l;
                for (int c = j + 1; c < kb; ++c) P[c * n + r] -= l * P[c * n + j];
            }
            __syncthreads();
        }
        // panel back to memory (rounded to the storage type)
        for (int idx = t; idx < m * kb; idx += LU_THREADS) {
            const int c = idx / m, r = idx % m;
            a[(size_t)(k0 + c) * ld + k0 + r] = (TF)P[c * n + r];
        }
        // every other column: the panel's row exchanges at once (rows 0..kb-1
        // and the pivot rows change; each column's reads come before its
        // writes) and, right of the panel, U12 = L11^-1 A12.  A group of NBW
        // lanes takes a column, lane i its row i (coalesced column segments),
        // CPI columns per group in flight; the unit-lower solve passes x_q
        // down the group by shuffles, lane i holding row i of L11 in
        // registers for the whole panel (the same operation order as a
        // per-column forward substitution).
        const int n2 = n - k0 - kb;
        {
            constexpr int GW = NBW, NG = LU_THREADS / NBW, CPI = 4;
            static_assert(64 % GW == 0, "a lane group lies inside one wavefront (shuffle width)");
            const int gi = t % GW, grp = t / GW;
            const bool rowok = gi < kb;
            TA lrow[GW];
#pragma unroll
            for (int q = 0; q < GW; ++q) lrow[q] = (rowok && q < gi) ? P[q * n + gi] : TA(0);
            const int prow = rowok ? spiv[gi] : 0;
            const bool zon = rowok && prow >= kb;
            const int ysrc = rowok ? perm[gi] : 0;
            const int zsrc = zon ? perm[prow] : 0;
            const int ncol = n - kb;                    // columns outside the panel
            for (int c0 = grp; c0 < ncol; c0 += NG * CPI) {
                TF y[CPI], z[CPI];
                TF* cols[CPI];
#pragma unroll
                for (int u = 0; u < CPI; ++u) {
                    const int cr = c0 + u * NG;
                    const int c = (cr < k0) ? cr : cr + kb;
                    cols[u] = a + (size_t)(cr < ncol ? c : 0) * ld + k0;
                    y[u] = (cr < ncol && rowok) ? cols[u][ysrc] : TF(0);
                    z[u] = (cr < ncol && zon) ? cols[u][zsrc] : TF(0);
                }
#pragma unroll
                for (int u = 0; u < CPI; ++u)
                    if (c0 + u * NG < ncol && zon) cols[u][prow] = z[u];
                TA x[CPI];
#pragma unroll
                for (int u = 0; u < CPI; ++u) x[u] = (TA)y[u];
#pragma unroll
                for (int q = 0; q < GW - 1; ++q)
#pragma unroll
                    for (int u = 0; u < CPI; ++u) {
                        const TA xq = __shfl(x[u], q, GW);
                        x[u] -= lrow[q] * xq;
                    }
#pragma unroll
                for (int u = 0; u < CPI; ++u) {
                    const int cr = c0 + u * NG;
                    if (cr < ncol && rowok) cols[u][gi] = (cr < k0) ? y[u] : (TF)x[u];
                }
            }
        }
        __syncthreads();
        if (n2 <= 0) break;
        // A22 -= L21 U12 on the matrix cores: 16 x 16 tiles of A22, one per
        // wavefront at a time, K = 4 per instruction over the panel width
        trailing_update_mfma<TF, TA, NBW>(a, P, n, ld, k0, kb, n2, t);
        __syncthreads();
    }
}

// pos[i] such that (P b)[i] = b[pos[i]] for the exchanges recorded in piv.
__global__ void __launch_bounds__(256) lu_pos_kernel(const int* __restrict__ piv, int* __restrict__ pos, int n) {
    extern __shared__ int sp[];
    const int* pv = piv + (size_t)blockIdx.x * n;
    int* po = pos + (size_t)blockIdx.x * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) sp[i] = i;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < n; ++k) {
            const int p = pv[k];
            if (p > k && p < n) {
                const int x = sp[k];
                sp[k] = sp[p];
                sp[p] = x;
            }
        }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) po[i] = sp[i];
}

template <class TF>
struct LuCfg;
template <> struct LuCfg<double> { using TA = double; static constexpr int NBW = 16; };
template <> struct LuCfg<float> { using TA = float; static constexpr int NBW = 32; };

template <class TF>
hipError_t launch_lu_blocked(TF* A, int* piv, int* pos, int nblk, int n, int ld, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    if (ld < n) return hipErrorInvalidValue;
    using C = LuCfg<TF>;
    const size_t lds = (size_t)C::NBW * n * sizeof(typename C::TA) + (size_t)n * sizeof(int);
    auto kern = lu_blocked_kernel<TF, typename C::TA, C::NBW>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(LU_THREADS), lds, s, A, piv, n, ld);
    e = hipGetLastError();
    if (e != hipSuccess || !pos) return e;
    hipLaunchKernelGGL(lu_pos_kernel, dim3(nblk), dim3(256), n * sizeof(int), s, piv, pos, n);
    return hipGetLastError();
}
template hipError_t launch_lu_blocked<double>(double*, int*, int*, int, int, int, hipStream_t);
template hipError_t launch_lu_blocked<float>(float*, int*, int*, int, int, int, hipStream_t);

// ---- explicit block inverse for the smoother apply --------------------------------------------
// X = A^-1 from the PLU factors: X starts as P I (X[c][i] = 1 iff pos[i] = c)
// and is overwritten by L^-1 then U^-1 in INV_TB-row panels over all n
// right-hand sides (panel of the factor and panel rows of X staged in LDS,
// 4x4 register tiles for the updates).  X is column-major FP64 (workspace),
// rounded to the storage type TF at the end.  Blocks up to n = 320.
constexpr int INV_TB = 24;

size_t lu_inverse_lds(int n) { return (size_t)2 * INV_TB * n * sizeof(double); }

template <class TF>
__global__ void __launch_bounds__(LU_THREADS) lu_inverse_kernel(const TF* __restrict__ LU, const int* __restrict__ pos,
                                                                double* __restrict__ Xw, TF* __restrict__ Xout, int n) {
    extern __shared__ double lds[];
    double* Fp = lds;                          // factor panel: Fp[j*n + i]
    double* Xp = lds + (size_t)INV_TB * n;     // X panel rows: Xp[j*n + c]
    const TF* a = LU + (size_t)blockIdx.x * n * n;
    const int* po = pos + (size_t)blockIdx.x * n;
    double* X = Xw + (size_t)blockIdx.x * n * n;
    const int t = threadIdx.x;
    for (size_t idx = t; idx < (size_t)n * n; idx += LU_THREADS) X[idx] = 0.0;
    __syncthreads();
    for (int i = t; i < n; i += LU_THREADS) X[(size_t)po[i] * n + i] = 1.0;
    __syncthreads();
    // forward: L (unit lower)
    for (int k0 = 0; k0 < n; k0 += INV_TB) {
        const int kb = min(INV_TB, n - k0), m = n - k0;
        for (int idx = t; idx < m * kb; idx += LU_THREADS) {
            const int j = idx / m, i = idx % m;
            Fp[j * n + i] = (double)a[(size_t)(k0 + j) * n + k0 + i];
        }
        __syncthreads();
        for (int c = t; c < n; c += LU_THREADS) {
            double x[INV_TB];
#pragma unroll
            for (int j = 0; j < INV_TB; ++j) x[j] = (j < kb) ? X[(size_t)c * n + k0 + j] : 0.0;
#pragma unroll
            for (int j = 0; j < INV_TB; ++j)
#pragma unroll
                for (int i = j + 1; i < INV_TB; ++i)
                    if (i < kb) x[i] -= Fp[j * n + i] * x[j];
#pragma unroll
            for (int j = 0; j < INV_TB; ++j)
                if (j < kb) {
                    X[(size_t)c * n + k0 + j] = x[j];
                    Xp[j * n + c] = x[j];
                }
        }
        __syncthreads();
        const int m2 = n - k0 - kb;
        if (m2 > 0) {
            const int tr = (m2 + 3) / 4, tc = (n + 3) / 4;
            for (int tile = t; tile < tr * tc; tile += LU_THREADS) {
                const int r0 = (tile % tr) * 4, c0 = (tile / tr) * 4;
                double acc[4][4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) acc[i][jj] = 0.0;
                for (int j = 0; j < kb; ++j) {
                    double lv[4], xv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) lv[i] = (r0 + i < m2) ? Fp[j * n + kb + r0 + i] : 0.0;
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) xv[jj] = (c0 + jj < n) ? Xp[j * n + c0 + jj] : 0.0;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) acc[i][jj] = fma(lv[i], xv[jj], acc[i][jj]);
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    if (c0 + jj >= n) continue;
                    double* colp = X + (size_t)(c0 + jj) * n + k0 + kb + r0;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (r0 + i < m2) colp[i] -= acc[i][jj];
                }
            }
        }
        __syncthreads();
    }
    // backward: U (upper, non-unit)
    const int nb0 = ((n - 1) / INV_TB) * INV_TB;
    for (int k0 = nb0; k0 >= 0; k0 -= INV_TB) {
        const int kb = min(INV_TB, n - k0), m = k0 + kb;
        for (int idx = t; idx < m * kb; idx += LU_THREADS) {
            const int j = idx / m, i = idx % m;
            Fp[j * n + i] = (double)a[(size_t)(k0 + j) * n + i];
        }
        __syncthreads();
        for (int c = t; c < n; c += LU_THREADS) {
            double x[INV_TB];
#pragma unroll
            for (int j = 0; j < INV_TB; ++j) x[j] = (j < kb) ? X[(size_t)c * n + k0 + j] : 0.0;
#pragma unroll
            for (int j = INV_TB - 1; j >= 0; --j) {
                if (j < kb) {
                    x[j] /= Fp[j * n + k0 + j];
#pragma unroll
                    for (int i = 0; i < j; ++i) x[i] -= Fp[j * n + k0 + i] * x[j];
                }
            }
#pragma unroll
            for (int j = 0; j < INV_TB; ++j)
                if (j < kb) {
                    X[(size_t)c * n + k0 + j] = x[j];
                    Xp[j * n + c] = x[j];
                }
        }
        __syncthreads();
        if (k0 > 0) {
            const int tr = (k0 + 3) / 4, tc = (n + 3) / 4;
            for (int tile = t; tile < tr * tc; tile += LU_THREADS) {
                const int r0 = (tile % tr) * 4, c0 = (tile / tr) * 4;
                double acc[4][4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) acc[i][jj] = 0.0;
                for (int j = 0; j < kb; ++j) {
                    double uv[4], xv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) uv[i] = (r0 + i < k0) ? Fp[j * n + r0 + i] : 0.0;
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) xv[jj] = (c0 + jj < n) ? Xp[j * n + c0 + jj] : 0.0;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) acc[i][jj] = fma(uv[i], xv[jj], acc[i][jj]);
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    if (c0 + jj >= n) continue;
                    double* colp = X + (size_t)(c0 + jj) * n + r0;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (r0 + i < k0) colp[i] -= acc[i][jj];
                }
            }
        }
        __syncthreads();
    }
    if (Xout) {
        TF* xo = Xout + (size_t)blockIdx.x * n * n;
        for (size_t idx = t; idx < (size_t)n * n; idx += LU_THREADS) xo[idx] = (TF)X[idx];
    }
}

template <class TF>
hipError_t launch_lu_inverse(const TF* LU, const int* pos, double* Xw, TF* Xout, int nblk, int n, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    const size_t lds = lu_inverse_lds(n);
    hipError_t e = hipFuncSetAttribute((const void*)lu_inverse_kernel<TF>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lu_inverse_kernel<TF>, dim3(nblk), dim3(LU_THREADS), lds, s, LU, pos, Xw, Xout, n);
    return hipGetLastError();
}
template hipError_t launch_lu_inverse<double>(const double*, const int*, double*, double*, int, int, hipStream_t);
template hipError_t launch_lu_inverse<float>(const float*, const int*, double*, float*, int, int, hipStream_t);

}  // namespace dg
