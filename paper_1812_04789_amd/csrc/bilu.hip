// Block ILU(0) in minimum-discarded-fill order (Sec. 6.3; the coarsest-level
// preconditioner of Table MGSettings) for the assembled coarsest p-multigrid
// level.  Partition-wise, as Sec. 6.3 applies it in parallel: each partition
// is one element line along x (the elements with the same y and z index),
// couplings between lines are dropped, and each line is factored and solved
// by one workgroup.
//
// Storage (FP64, blocks column-major nb x nb, nb <= BILU_MAX_N = 48: the
// degree-1 coarsest level has nb = 40):
//   d[e]        diagonal block of element e; after bilu_factor: the inverse of
//               its updated diagonal block (U_ee^-1)
//   o[e][s]     coupling block of row e to its line neighbour in slot s
//               (s = 0: across face 0, s = 1: across face 1; for a
//               two-element line both faces reach the same neighbour and
//               slot 0 holds their sum, slot 1 is zero); after bilu_factor:
//               L(e, j) for a neighbour j eliminated before e, U(e, j) for
//               one eliminated after e.
//   ord[line * nx + t]   the t-th element of a line's elimination order,
//   pos[e]               the position of e in its line's order.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace dg {
namespace {

__device__ __forceinline__ int line_nbr(const MeshDev& m, int e, int side) {
    const int i = e % m.nx;
    const int base = e - i;
    return base + (side ? (i + 1) % m.nx : (i + m.nx - 1) % m.nx);
}

// Inverse of the nb x nb column-major block at A (LDS) into X (LDS), by
// Gauss-Jordan elimination with partial pivoting on [A | I]; A is destroyed.
// One workgroup of any size; every thread calls it.
__device__ void gj_inverse(double* A, double* X, int nb, int* sp) {
    const int t = threadIdx.x, nt = blockDim.x;
    for (int k = t; k < nb * nb; k += nt) X[k] = ((k % nb) == (k / nb)) ? 1.0 : 0.0;
    __syncthreads();
    for (int c = 0; c < nb; ++c) {
        if (t == 0) {
            int p = c;
            double best = fabs(A[c * nb + c]);
            for (int r = c + 1; r < nb; ++r) {
                const double v = fabs(A[c * nb + r]);
                if (v > best) {
                    best = v;
                    p = r;
                }
            }
            *sp = p;
        }
        __syncthreads();
        const int p = *sp;
        if (p != c) {
            for (int j = t; j < nb; j += nt) {
                double a = A[j * nb + c];
                A[j * nb + c] = A[j * nb + p];
                A[j * nb + p] = a;
                double x = X[j * nb + c];
                X[j * nb + c] = X[j * nb + p];
                X[j * nb + p] = x;
            }
        }
        __syncthreads();
        const double ip = 1.0 / A[c * nb + c];
        __syncthreads();
        for (int j = t; j < nb; j += nt) {
            A[j * nb + c] *= ip;
            X[j * nb + c] *= ip;
        }
        __syncthreads();
        // eliminate column c from every other row: row r -= A[r][c] * row c
        for (int k = t; k < nb * nb; k += nt) {
            const int r = k % nb, j = k / nb;
            if (r == c) continue;
            const double f = A[c * nb + r];
            if (j != c) A[j * nb + r] = fma(-f, A[j * nb + c], A[j * nb + r]);
            X[j * nb + r] = fma(-f, X[j * nb + c], X[j * nb + r]);
        }
        __syncthreads();
        for (int r = t; r < nb; r += nt)
            if (r != c) A[c * nb + r] = 0.0;
        __syncthreads();
    }
}

// C (+)= sign * A B, nb x nb column-major; A, B, C in any memory, C distinct.
__device__ void gemm_acc(const double* A, const double* B, double* C, int nb, double sign, bool accumulate) {
    const int t = threadIdx.x, nt = blockDim.x;
    for (int k = t; k < nb * nb; k += nt) {
        const int r = k % nb, j = k / nb;
        double acc = 0.0;
        for (int i = 0; i < nb; ++i) acc = fma(A[i * nb + r], B[j * nb + i], acc);
        C[k] = accumulate ? fma(sign, acc, C[k]) : sign * acc;
    }
}

// Minimum-discarded-fill weight of every element: with its line neighbours
// xm (face 0) and xp (face 1) distinct and not coupled (lines of four or
// more), eliminating e discards A(xm,e) A(e,e)^-1 A(e,xp) and
// A(xp,e) A(e,e)^-1 A(e,xm); w = sqrt of the summed squared Frobenius norms.
// Lines of three or fewer discard nothing: w = 0.  One workgroup per element.
__global__ void __launch_bounds__(256) bilu_weight_kernel(MeshDev m, int nb, const double* __restrict__ d,
                                                          const double* __restrict__ o, double* __restrict__ w) {
    extern __shared__ double lds[];              // A, X, T: 3 nb^2
    double* A = lds;
    double* X = lds + nb * nb;
    double* T = lds + 2 * nb * nb;
    __shared__ double red[256];
    __shared__ int sp;
    const int e = blockIdx.x, t = threadIdx.x;
    const size_t nn = (size_t)nb * nb;
    if (m.nx < 4) {
        if (t == 0) w[e] = 0.0;
        return;
    }
    for (int k = t; k < nb * nb; k += blockDim.x) A[k] = d[e * nn + k];
    __syncthreads();
    gj_inverse(A, X, nb, &sp);
    const int xm = line_nbr(m, e, 0), xp = line_nbr(m, e, 1);
    double s = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        // pass 0: A(xm,e) X A(e,xp);  pass 1: A(xp,e) X A(e,xm)
        const double* Ae = o + ((size_t)e * 2 + (pass == 0 ? 1 : 0)) * nn;          // A(e, xp) / A(e, xm)
        const double* An = o + ((size_t)(pass == 0 ? xm : xp) * 2 + (pass == 0 ? 1 : 0)) * nn;   // A(xm,e) / A(xp,e)
        __syncthreads();
        gemm_acc(X, Ae, T, nb, 1.0, false);
        __syncthreads();
        for (int k = t; k < nb * nb; k += blockDim.x) {
            const int r = k % nb, j = k / nb;
            double acc = 0.0;
            for (int i = 0; i < nb; ++i) acc = fma(An[i * nb + r], T[j * nb + i], acc);
            s = fma(acc, acc, s);
        }
    }
    red[t] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) w[e] = sqrt(red[0]);
}

// Slot of element e that reaches element j, or -1.
__device__ __forceinline__ int slot_of(const MeshDev& m, int e, int j) {
    if (j == e) return -1;
    if (line_nbr(m, e, 0) == j) return 0;
    if (line_nbr(m, e, 1) == j) return 1;
    return -1;
}

// Block ILU(0) of every line in its elimination order, in place.  For each k
// in order: X = U_kk^-1 (replacing d[k]); for each later line neighbour j:
// L(j,k) = A(j,k) X (replacing the slot of j that reaches k); for later
// neighbours j, l: A(j,l) -= L(j,k) A(k,l) when j == l or j reaches l (the
// fill the pattern keeps).  The slots of k reaching later neighbours keep
// A(k,l) = U(k,l).  One workgroup per line.
__global__ void __launch_bounds__(256) bilu_factor_kernel(MeshDev m, int nb, const int* __restrict__ ord,
                                                          const int* __restrict__ pos, double* __restrict__ d,
                                                          double* __restrict__ o) {
    extern __shared__ double lds[];              // A, X, T: 3 nb^2
    double* A = lds;
    double* X = lds + nb * nb;
    double* T = lds + 2 * nb * nb;
    __shared__ int sp;
    const int line = blockIdx.x, nx = m.nx;
    const size_t nn = (size_t)nb * nb;
    for (int step = 0; step < nx; ++step) {
        const int k = ord[line * nx + step];
        for (int q = threadIdx.x; q < nb * nb; q += blockDim.x) A[q] = d[k * nn + q];
        __syncthreads();
        gj_inverse(A, X, nb, &sp);
        for (int q = threadIdx.x; q < nb * nb; q += blockDim.x) d[k * nn + q] = X[q];
        __syncthreads();
        int later[2];
        int nl = 0;
        for (int s = 0; s < 2; ++s) {
            const int j = line_nbr(m, k, s);
            if (j == k || pos[j] < pos[k]) continue;
            if (nl == 1 && later[0] == j) continue;
            later[nl++] = j;
        }
        // L(j,k) = A(j,k) X, in the slot of j that reaches k
        for (int a = 0; a < nl; ++a) {
            const int j = later[a];
            double* Ljk = o + ((size_t)j * 2 + slot_of(m, j, k)) * nn;
            gemm_acc(Ljk, X, T, nb, 1.0, false);
            __syncthreads();
            for (int q = threadIdx.x; q < nb * nb; q += blockDim.x) Ljk[q] = T[q];
            __syncthreads();
        }
        // A(j,l) -= L(j,k) A(k,l) for later j, l kept by the pattern
        for (int a = 0; a < nl; ++a) {
            const int j = later[a];
            const double* Ljk = o + ((size_t)j * 2 + slot_of(m, j, k)) * nn;
            for (int b = 0; b < nl; ++b) {
                const int l = later[b];
                double* Ajl;
                if (j == l) Ajl = d + (size_t)j * nn;
                else {
                    const int sl = slot_of(m, j, l);
                    if (sl < 0) continue;                    // fill outside the pattern: discarded
                    Ajl = o + ((size_t)j * 2 + sl) * nn;
                }
                const double* Akl = o + ((size_t)k * 2 + slot_of(m, k, l)) * nn;
                gemm_acc(Ljk, Akl, Ajl, nb, -1.0, true);
                __syncthreads();
            }
        }
    }
}

// z = (L U)^-1 r for every line: forward sweep y_k = r_k - sum L(k,j) y_j over
// earlier j, in order, into z; backward sweep z_k = U_kk^-1 (y_k - sum
// U(k,l) z_l) over later l, in reverse order.  One workgroup per line; nb
// threads per row block.
__global__ void __launch_bounds__(128) bilu_apply_kernel(MeshDev m, int nb, const int* __restrict__ ord,
                                                         const int* __restrict__ pos, const double* __restrict__ d,
                                                         const double* __restrict__ o, const double* __restrict__ r,
                                                         double* __restrict__ z) {
    __shared__ double v[BILU_MAX_N];
    const int line = blockIdx.x, nx = m.nx, t = threadIdx.x;
    const size_t nn = (size_t)nb * nb;
    for (int step = 0; step < nx; ++step) {
        const int k = ord[line * nx + step];
        if (t < nb) {
            double acc = r[(size_t)k * nb + t];
            for (int s = 0; s < 2; ++s) {
                const int j = line_nbr(m, k, s);
                if (j == k || pos[j] > pos[k]) continue;
                if (s == 1 && line_nbr(m, k, 0) == j) continue;
                const double* Lkj = o + ((size_t)k * 2 + s) * nn;
                for (int c = 0; c < nb; ++c) acc = fma(-Lkj[c * nb + t], z[(size_t)j * nb + c], acc);
            }
            z[(size_t)k * nb + t] = acc;
        }
        __syncthreads();
    }
    for (int step = nx - 1; step >= 0; --step) {
        const int k = ord[line * nx + step];
        if (t < nb) {
            double acc = z[(size_t)k * nb + t];
            for (int s = 0; s < 2; ++s) {
                const int l = line_nbr(m, k, s);
                if (l == k || pos[l] < pos[k]) continue;
                if (s == 1 && line_nbr(m, k, 0) == l) continue;
                const double* Ukl = o + ((size_t)k * 2 + s) * nn;
                for (int c = 0; c < nb; ++c) acc = fma(-Ukl[c * nb + t], z[(size_t)l * nb + c], acc);
            }
            v[t] = acc;
        }
        __syncthreads();
        if (t < nb) {
            const double* X = d + (size_t)k * nn;
            double acc = 0.0;
            for (int c = 0; c < nb; ++c) acc = fma(X[c * nb + t], v[c], acc);
            z[(size_t)k * nb + t] = acc;
        }
        __syncthreads();
    }
}

// One step of the pipelined apply: steps 0..nx-1 are the forward sweep in
// elimination order, steps nx..2nx-1 the backward sweep in reverse order.
// The step's blocks: the couplings of its element k to the line neighbours
// eliminated before k (forward: L) or after k (backward: U), then, backward,
// U_kk^-1; src/dst are line-local element indices (e = line nx + i).  ordl
// and posl are the line's order and positions (line-local, in LDS).
struct BiluStep {
    const double* blk[3];
    int nbk, ncoup;
    int src[2];
    int dst;
};

__device__ __forceinline__ BiluStep bilu_step(const MeshDev& m, const int* ordl, const int* posl,
                                              const double* __restrict__ d, const double* __restrict__ o, int line,
                                              int step, int nb) {
    const int nx = m.nx, base = line * nx;
    const bool fwd = step < nx;
    const int i = ordl[fwd ? step : 2 * nx - 1 - step];
    const int k = base + i;
    const size_t nn = (size_t)nb * nb;
    const int j0 = line_nbr(m, k, 0) - base, j1 = line_nbr(m, k, 1) - base;
    const bool use0 = j0 != i && (fwd ? posl[j0] < posl[i] : posl[j0] > posl[i]);
    const bool use1 = j1 != i && j1 != j0 && (fwd ? posl[j1] < posl[i] : posl[j1] > posl[i]);
    const double* c0 = o + ((size_t)k * 2 + 0) * nn;
    const double* c1 = o + ((size_t)k * 2 + 1) * nn;
    const double* dk = d + (size_t)k * nn;
    // the used couplings first (slot order), then, backward, U_kk^-1
    BiluStep S;
    S.ncoup = (use0 ? 1 : 0) + (use1 ? 1 : 0);
    S.nbk = S.ncoup + (fwd ? 0 : 1);
    S.blk[0] = use0 ? c0 : (use1 ? c1 : dk);
    S.blk[1] = (use0 && use1) ? c1 : dk;
    S.blk[2] = dk;
    S.src[0] = use0 ? j0 : j1;
    S.src[1] = j1;
    S.dst = i;
    return S;
}

// The same z = (L U)^-1 r with the block size fixed (NB): the line's vector,
// order and positions are held in LDS, every block product is split over
// 240 threads (NB rows x six column groups, partial sums added in group
// order), and the blocks of step s + 1 are written to LDS at the end of step
// s from registers loaded two steps earlier (two LDS buffers of three blocks,
// two register sets).  One workgroup per line.
constexpr int BILU_PIPE_NB = 40;
constexpr int BILU_PIPE_THREADS = 256;
constexpr int BILU_PIPE_GROUPS = 6;
__host__ __device__ constexpr size_t bilu_pipe_lds(int nb, int nx) {
    return (size_t)(6 * nb * nb + BILU_PIPE_GROUPS * nb + nb + nx * nb) * sizeof(double) + 2 * nx * sizeof(int);
}

template <int NB, int PER>
__device__ __forceinline__ void bilu_prefetch(const BiluStep& S, int t, double (&pre)[PER]) {
    constexpr int NN = NB * NB;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int q = t + BILU_PIPE_THREADS * u;
        const int b = q / NN;
        const double* src = (b == 0) ? S.blk[0] : ((b == 1) ? S.blk[1] : S.blk[2]);
        pre[u] = (q < 3 * NN && b < S.nbk) ? src[q - b * NN] : 0.0;
    }
}

template <int NB>
__global__ void __launch_bounds__(BILU_PIPE_THREADS) bilu_apply_pipe_kernel(
    MeshDev m, const int* __restrict__ ord, const int* __restrict__ pos, const double* __restrict__ d,
    const double* __restrict__ o, const double* __restrict__ r, double* __restrict__ z) {
    constexpr int NN = NB * NB;
    constexpr int NT = BILU_PIPE_THREADS;
    constexpr int PER = (3 * NN + NT - 1) / NT;      // prefetched entries per thread and step
    constexpr int NG = BILU_PIPE_GROUPS;
    constexpr int CW = (NB + NG - 1) / NG;            // columns per group
    static_assert(NG * NB <= NT, "one thread per (row, column group)");
    extern __shared__ double sm[];
    double* buf0 = sm;
    double* buf1 = sm + 3 * NN;
    double* part = sm + 6 * NN;                       // [group][row]
    double* vb = part + NG * NB;                      // backward: r_k - U x before U_kk^-1
    const int nx = m.nx, line = blockIdx.x, t = threadIdx.x;
    double* zl = vb + NB;                             // the line's vector [i][row]
    int* ordl = reinterpret_cast<int*>(zl + nx * NB);
    int* posl = ordl + nx;
    const int row = t % NB, g = t / NB;
    const int base = line * nx;
    const double* rl = r + (size_t)base * NB;
    for (int q = t; q < nx * NB; q += NT) zl[q] = rl[q];
    for (int q = t; q < nx; q += NT) {
        ordl[q] = ord[base + q] - base;
        posl[q] = pos[base + q];
    }
    __syncthreads();
    const int nsteps = 2 * nx;
    BiluStep S = bilu_step(m, ordl, posl, d, o, line, 0, NB);
#pragma unroll
    for (int b = 0; b < 3; ++b)
        if (b < S.nbk)
            for (int q = t; q < NN; q += NT) buf0[b * NN + q] = S.blk[b][q];
    // two register sets: at step s, set A holds step s + 1's blocks (loaded
    // two steps earlier) and set B step s + 2's; after A is written to LDS it
    // takes step s + 3's loads, and the sets swap roles
    BiluStep SA, SB;
    double preA[PER], preB[PER];
    if (nsteps > 1) {
        SA = bilu_step(m, ordl, posl, d, o, line, 1, NB);
        bilu_prefetch<NB, PER>(SA, t, preA);
    }
    if (nsteps > 2) {
        SB = bilu_step(m, ordl, posl, d, o, line, 2, NB);
        bilu_prefetch<NB, PER>(SB, t, preB);
    }
    __syncthreads();
    auto body = [&](int step, BiluStep& Sn, double (&pn)[PER]) {
        const double* cur = (step & 1) ? buf1 : buf0;
        double* nxt = (step & 1) ? buf0 : buf1;
        const bool fwd = step < nx;
        // coupling products of the step, split by column group
        if (t < NG * NB) {
            double acc = 0.0;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (s < S.ncoup) {
                    const double* B = cur + s * NN;
                    const double* x = zl + S.src[s] * NB;
#pragma unroll
                    for (int cc = 0; cc < CW; ++cc) {
                        const int c = g * CW + cc;
                        if (c < NB) acc = fma(B[c * NB + row], x[c], acc);
                    }
                }
            }
            part[g * NB + row] = acc;
        }
        __syncthreads();
        if (t < NB) {
            double y = zl[S.dst * NB + t];
#pragma unroll
            for (int gg = 0; gg < NG; ++gg) y -= part[gg * NB + t];
            if (fwd) zl[S.dst * NB + t] = y;
            else vb[t] = y;
        }
        __syncthreads();
        if (!fwd) {
            // z_k = U_kk^-1 (r_k - sum U x)
            if (t < NG * NB) {
                const double* X = cur + S.ncoup * NN;
                double acc = 0.0;
#pragma unroll
                for (int cc = 0; cc < CW; ++cc) {
                    const int c = g * CW + cc;
                    if (c < NB) acc = fma(X[c * NB + row], vb[c], acc);
                }
                part[g * NB + row] = acc;
            }
            __syncthreads();
            if (t < NB) {
                double y = 0.0;
#pragma unroll
                for (int gg = 0; gg < NG; ++gg) y += part[gg * NB + t];
                zl[S.dst * NB + t] = y;
            }
        }
        if (step + 1 < nsteps) {
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int q = t + NT * u;
                if (q < 3 * NN && q / NN < Sn.nbk) nxt[q] = pn[u];
            }
            S = Sn;
            if (step + 3 < nsteps) {
                Sn = bilu_step(m, ordl, posl, d, o, line, step + 3, NB);
                bilu_prefetch<NB, PER>(Sn, t, pn);
            }
        }
        __syncthreads();
    };
    for (int step = 0; step < nsteps; step += 2) {
        body(step, SA, preA);
        if (step + 1 < nsteps) body(step + 1, SB, preB);
    }
    double* zo = z + (size_t)base * NB;
    for (int q = t; q < nx * NB; q += NT) zo[q] = zl[q];
}

// d <- diag (copy); o[e][s] <- the coupling of e to its line neighbour in
// slot s from the face blocks off[e][f][c][r] (faces 0 and 1).
__global__ void bilu_gather_kernel(MeshDev m, int nb, const double* __restrict__ diag, const double* __restrict__ off,
                                   double* __restrict__ d, double* __restrict__ o) {
    const size_t nn = (size_t)nb * nb;
    const int e = blockIdx.x;
    const int xm = line_nbr(m, e, 0), xp = line_nbr(m, e, 1);
    const bool same = (xm == xp);
    for (size_t q = threadIdx.x; q < nn; q += blockDim.x) {
        d[e * nn + q] = diag[e * nn + q];
        const double f0 = off[((size_t)e * 6 + 0) * nn + q], f1 = off[((size_t)e * 6 + 1) * nn + q];
        o[((size_t)e * 2 + 0) * nn + q] = same ? f0 + f1 : f0;
        o[((size_t)e * 2 + 1) * nn + q] = same ? 0.0 : f1;
    }
}

}  // namespace

hipError_t launch_bilu_gather(const DGArgs& a, int nb, const double* diag, const double* off, double* d, double* o,
                              hipStream_t s) {
    if (nb > BILU_MAX_N) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bilu_gather_kernel, dim3(a.m.ne), dim3(256), 0, s, a.m, nb, diag, off, d, o);
    return hipGetLastError();
}

hipError_t launch_bilu_weights(const DGArgs& a, int nb, const double* d, const double* o, double* w, hipStream_t s) {
    if (nb > BILU_MAX_N) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bilu_weight_kernel, dim3(a.m.ne), dim3(256), 3 * nb * nb * sizeof(double), s, a.m, nb, d, o, w);
    return hipGetLastError();
}

hipError_t launch_bilu_factor(const DGArgs& a, int nb, const int* ord, const int* pos, double* d, double* o,
                              hipStream_t s) {
    if (nb > BILU_MAX_N) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bilu_factor_kernel, dim3(a.m.ne / a.m.nx), dim3(256), 3 * nb * nb * sizeof(double), s, a.m, nb,
                       ord, pos, d, o);
    return hipGetLastError();
}

hipError_t launch_bilu_apply(const DGArgs& a, int nb, const int* ord, const int* pos, const double* d,
                             const double* o, const double* r, double* z, hipStream_t s) {
    if (nb > BILU_MAX_N) return hipErrorInvalidValue;
    const size_t lds = bilu_pipe_lds(nb, a.m.nx);
    if (nb == BILU_PIPE_NB && lds <= 160 * 1024) {
        const hipError_t e = hipFuncSetAttribute((const void*)bilu_apply_pipe_kernel<BILU_PIPE_NB>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(bilu_apply_pipe_kernel<BILU_PIPE_NB>, dim3(a.m.ne / a.m.nx), dim3(BILU_PIPE_THREADS), lds,
                           s, a.m, ord, pos, d, o, r, z);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(bilu_apply_kernel, dim3(a.m.ne / a.m.nx), dim3(128), 0, s, a.m, nb, ord, pos, d, o, r, z);
    return hipGetLastError();
}

}  // namespace dg
