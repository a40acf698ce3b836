// Internal declarations of the MI355X DG library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dg.h"
#include "physics.h"

namespace dg {

constexpr int MAXP = 4;      // supported polynomial degrees 1..MAXP
constexpr int MAXN = MAXP + 1;

// 1D reference tables of degree P (n = P+1 Gauss points, orthonormal
// Legendre modes).  Index conventions: q = Gauss point, a = mode, s = end
// (0: xi = -1, 1: xi = +1).
struct Tab {
    double V[MAXN][MAXN];     // V[q][a]  = L_a(z_q)
    double Vd[MAXN][MAXN];    // Vd[q][a] = L_a'(z_q)
    double D[MAXN][MAXN];     // D[q][r]  = l_r'(z_q), collocation derivative on the Gauss points
    double w[MAXN];           // Gauss weights
    double z[MAXN];           // Gauss points
    double lag[2][MAXN];      // l_q(-1), l_q(+1): Lagrange basis of the Gauss points at the ends
    double lagd[2][MAXN];     // l_q'(-1), l_q'(+1)
    double Le[2][MAXN];       // L_a(-1), L_a(+1)
    double Lde[2][MAXN];      // L_a'(-1), L_a'(+1)
    double br2[2][MAXN];      // (sum_i L_i(+-1) L_i(z_q))^2 w_q: BR2 line weights
};

// perm offsets: tensor-mode tables of every P packed in one array
constexpr int perm_offset(int P) { return P == 1 ? 0 : P == 2 ? 8 : P == 3 ? 35 : 99; }
constexpr int PERM_TOTAL = 224;

// Host construction (tables.cpp).
void build_tables(Tab tabs[MAXP + 1], short perm[PERM_TOTAL]);
// Upload to the device constant memory of the current device (dg_kernels.hip).
hipError_t upload_tables(const Tab* tabs, const short* perm);

struct MeshDev {
    int nx, ny, nz, ne;
    double h[3];              // straight box spacing
    const double* vtx;        // device [ne][8][3] (curved only) or nullptr
};

// Kernel launch parameters shared by the DG kernels.
struct DGArgs {
    MeshDev m;
    Gas g;                    // physics.h
    int p;
    bool ns;
};

// ---- DG kernels (dg_kernels.hip) ------------------------------------------
hipError_t launch_residual(const DGArgs& a, const double* W, double* R, hipStream_t s);
hipError_t launch_jvp_fd(const DGArgs& a, const double* W, const double* RW, const double* v, const double* hbuf,
                         double shift, double* y, hipStream_t s);
hipError_t launch_jvp_exact(const DGArgs& a, const double* W, const double* v, double shift, double* y,
                            hipStream_t s);
// nbrtr: scratch of nbr_trace_size(p, ne) doubles (neighbour traces at the face points);
// blocks: ne column-major blocks of nb columns with leading dimension ld >= nb
// (block e at blocks + e nb ld)
hipError_t launch_diag_blocks(const DGArgs& a, const double* W, double shift, double* blocks, int ld, double* nbrtr,
                              hipStream_t s);
size_t nbr_trace_size(int p, int ne);
// Coarse face-coupling blocks: for every element e, face f, the (nbc x nbc)
// block dR_e[S]/dW_nb(f)[S] over the coarse-mode set S of degree pc (rows and
// columns equation-major over S), column-major.  out [ne][6][nbc][nbc].
hipError_t launch_offdiag_blocks(const DGArgs& a, const double* W, int pc, double* out, hipStream_t s);
hipError_t launch_mass(const DGArgs& a, const double* v, double* y, double scale, int accumulate, hipStream_t s);
hipError_t launch_quad_points(const DGArgs& a, double* xyz, hipStream_t s);
hipError_t launch_project(const DGArgs& a, const double* vals, double* W, hipStream_t s);
hipError_t launch_check_jacobian(const DGArgs& a, int* bad, hipStream_t s);

// Mesh and gas of a context (capi.cpp), for the batch layer.
const DGArgs& ctx_args(const dg_ctx* ctx);

// ---- batched DG operator (dg_kernels.hip) ------------------------------------
enum { M_RES = 0, M_JVP_FD = 1, M_TANGENT = 2 };     // residual, FD product, exact product
constexpr int BATCH_MAX_THREADS = 256;
struct BatchCaseDev {
    MeshDev m;
    Gas g;
    size_t off;               // first entry of the case in the batched vectors
};
struct BatchItem {
    int c;                    // case
    int e0;                   // first element of the tile
    int p;                    // degree of the case (selects the compiled path)
    int n;                    // elements in the tile (slots of (p+1)^3 threads)
};
// LDS bytes of one element slot of degree p for mode M_*.
size_t batch_slot_bytes(int p, int mode);
// One persistent launch: workgroup b runs items b, b + grid, ...; hcase[c] is
// case c's FD step (M_JVP_FD).  Every case must share (ns, curved).
hipError_t launch_batch_dg(int mode, bool ns, bool curved, const BatchCaseDev* cases, const BatchItem* items,
                           int nitems, int threads, int grid, size_t lds, const double* W, const double* V,
                           const double* RW, const double* hcase, double shift, double* out, hipStream_t s);

// ---- vector / reduction kernels (la_kernels.hip) ----------------------------
// Blocks of the deterministic reduction of n entries.
int red_blocks_for(size_t n);
// Per-case FD steps of a batch: block b of the first stage sums entries
// lb, lb + nbk*256, ... of case c (offset off, length n), as the single-case
// reduction does; h[c] = eps sqrt(1 + ||W_c||) / ||v_c|| (0 if v_c = 0).
struct SegBlock {
    int c, lb, nbk, pad;
    size_t off, n;
};
hipError_t launch_seg_fd_step(const SegBlock* tab, int nblocks, const int* first, const int* nbk, int ncases,
                              const double* W, const double* v, double* px, double* py, double eps, double* h,
                              hipStream_t s);
// Deterministic sums: fixed grid, fixed per-block order, fixed second stage.
constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;
// out[k] = <x_k, y> for k < nx (x_k = X + k*ldx), written to device out.
hipError_t launch_multi_dot(const double* X, size_t ldx, int nx, const double* y, size_t n, double* partial,
                            double* out, hipStream_t s);
hipError_t launch_dot(const double* x, const double* y, size_t n, double* partial, double* out, hipStream_t s);
// nv2 = ||v||^2 and h = eps sqrt(1 + ||W||) / ||v|| (0 if v == 0) in two
// launches, bitwise equal to the launch_dot reductions.  ||W||^2 from nw2_in
// (W null), or computed from W in the same pass into nw2_out (nw2_in null).
// partial: the context's reduction buffer.
hipError_t launch_fd_step(const double* v, const double* W, size_t n, const double* nw2_in, double* nw2_out,
                          double eps, double* partial, double* nv2, double* h, hipStream_t s);
hipError_t launch_axpby(size_t n, double a, const double* x, double b, const double* y, double* z, hipStream_t s);
// y += sum_k c[k] * X_k   (c on device), or y -= when sign < 0
hipError_t launch_multi_axpy(size_t n, int k, const double* c, int sign, const double* X, size_t ldx, double* y,
                             hipStream_t s);
// y = x * (*sc) with sc on device (sc inverted when invert != 0)
hipError_t launch_scale_dev(size_t n, const double* x, const double* sc, int invert, double* y, hipStream_t s);
hipError_t launch_copy(size_t n, const double* x, double* y, hipStream_t s);
hipError_t launch_fill(size_t n, double v, double* y, hipStream_t s);
// restriction: coarse[e][a][i] = fine[e][a][i], i < nvc; prolongation adds/overwrites
hipError_t launch_restrict(int ne, int nvf, int nvc, const double* fine, double* coarse, hipStream_t s);
hipError_t launch_prolong_add(int ne, int nvf, int nvc, const double* coarse, double* fine, int overwrite,
                              hipStream_t s);
hipError_t launch_count_nonfinite(size_t n, const double* x, int* flag, hipStream_t s);
// One Arnoldi step j (basis V[0..j], new vector in V[j+1]): classical
// Gram-Schmidt twice (the norm after the second pass from the first-pass norm
// and the second-pass coefficients), H column j, Givens rotation j,
// normalisation; est = |g_{j+1}|.  j + 1 <= 64.  partial: RED_BLOCKS * 256
// doubles (the context's reduction buffer).
hipError_t launch_arnoldi_cgs2(const double* V, size_t n, int j, double* H, int ldh, double* cs, double* sn,
                               double* g, double* nrm, double* est, double* partial, hipStream_t s);
// The same step when the first-pass partial dots V_i . w (i <= j) are already
// in partial[i * np_a + b], b < np_a <= RED_BLOCKS (launch_bsr_unit_dots).
hipError_t launch_arnoldi_cgs2_after_dots(const double* V, size_t n, int j, double* H, int ldh, double* cs,
                                          double* sn, double* g, double* nrm, double* est, double* partial, int np_a,
                                          hipStream_t s);

// ---- dense block kernels (lu_kernels.hip) ------------------------------------
template <class TF>
hipError_t launch_lu(TF* A, int* piv, int nblk, int n, hipStream_t s);
// z = D^-1 r for every block, factors in TF, vectors FP64; z may not alias r
template <class TF>
hipError_t launch_lu_solve(const TF* LU, const int* piv, const double* r, double* z, int nblk, int n,
                           hipStream_t s);
// Blocked PLU (same pivots) plus the gather index pos of the row permutation;
// the blocked solve takes pos.  Blocks are column-major with leading
// dimension ld >= n (block b at A + b n ld; rows n..ld-1 are never touched).
template <class TF>
hipError_t launch_lu_blocked(TF* A, int* piv, int* pos, int nblk, int n, int ld, hipStream_t s);
template <class TF>
hipError_t launch_lu_solve_blocked(const TF* LU, const int* pos, const double* r, double* z, int nblk, int n, int ld,
                                   hipStream_t s);
// Explicit inverse of PLU-factored blocks (n <= 320): FP64 workspace Xw
// [nblk][n][n]; Xout (TF, may be null when TF is double and Xw is used directly).
template <class TF>
hipError_t launch_lu_inverse(const TF* LU, const int* pos, double* Xw, TF* Xout, int nblk, int n, hipStream_t s);
template <class TF>
hipError_t launch_inv_gemv(const TF* X, const double* r, double* z, int nblk, int n, hipStream_t s);
constexpr int INV_MAX_N = 320;
constexpr int INV_POLICY_N = 135;     // the smoother applies an explicit inverse up to this block size
// Leading dimension of the fine-level blocks: blocks applied by the triangular
// solves (nb > INV_POLICY_N) start every column on a 128-byte line (nb = 625 at
// p = 4 becomes 640; nb = 320 is unchanged); inverse-path blocks stay packed.
inline int fine_block_ld(int nb) { return (nb > INV_POLICY_N) ? (nb + 15) / 16 * 16 : nb; }
// Extract coarse principal sub-blocks (FP64 column-major fine blocks of leading
// dimension ldf) and round to TF.
template <class TF>
hipError_t launch_extract_sub(const double* fine, int nbf, int ldf, int nvf, int nvc, TF* out, int nblk,
                              hipStream_t s);
// Block-sparse product y = K x with 7 blocks per element row (diagonal + 6
// faces), stored sliced row-major: rows padded to bsr_ldr(nbc) entries per
// block, grouped by 64 rows, 16-byte chunks of a group contiguous.  With
// nblk = 6 only the face blocks are stored and the diagonal is the identity.
__host__ __device__ inline int bsr_ldr(int nbc) { return (nbc + 7) & ~7; }
__host__ __device__ inline size_t bsr_entries(int ne, int nbc, int nblk = 7) {
    return ((size_t)ne * nbc + 63) / 64 * 64 * (size_t)nblk * (size_t)bsr_ldr(nbc);
}
// Pack the column-major diagonal [e][c][r] (nblk = 7) and face blocks
// [e][f][c][r] (FP64) into that layout, rounding to TF (BF16: nearest even).
template <class TF>
hipError_t launch_bsr_pack(const double* diag, const double* off, TF* out, int ne, int nbc, int nblk, hipStream_t s);
template <class TF>
hipError_t launch_bsr7(const DGArgs& a, const TF* A, const double* x, double* y, int nbc, hipStream_t s);
// y = x + sum_f F_{e,f} x_{nb(e,f)} over the six packed face blocks (nblk = 6).
template <class TF>
hipError_t launch_bsr_unit(const DGArgs& a, const TF* A, const double* x, double* y, int nbc, hipStream_t s);
// The same product, then the per-block partial dots of y with the k basis
// vectors Vb (stride ne nbc): part[c * np + b], c < k; np (the product's
// grid) is returned.  Deterministic (the grid depends only on ne nbc).
template <class TF>
hipError_t launch_bsr_unit_dots(const DGArgs& a, const TF* A, const double* x, double* y, int nbc, const double* Vb,
                                int k, double* part, int* np, hipStream_t s);
int bsr_grid(int ne, int nbc);
// Face blocks [e][f][c][r] (FP64, in place) <- K_{e,f} X_{nb(e,f)}, X the
// column-major block inverses [e][c][r]; nbc <= FOLD_MAX_N.
constexpr int FOLD_MAX_N = 64;
template <class TX>
hipError_t launch_fold_inverse(const DGArgs& a, int nbc, double* off, const TX* X, hipStream_t s);
hipError_t launch_convert_fp64_to_fp32(const double* x, float* y, size_t n, hipStream_t s);

// ---- block ILU(0) of the coarsest level, element lines along x (bilu.hip) -------
constexpr int BILU_MAX_N = 48;
// d [ne][nb^2] <- diag, o [ne][2][nb^2] <- the couplings to the two line
// neighbours from the face blocks off [ne][6][nb^2] (column-major blocks).
hipError_t launch_bilu_gather(const DGArgs& a, int nb, const double* diag, const double* off, double* d, double* o,
                              hipStream_t s);
// w[e]: minimum-discarded-fill weight of eliminating e with both line
// neighbours remaining (0 for lines of fewer than four elements).
hipError_t launch_bilu_weights(const DGArgs& a, int nb, const double* d, const double* o, double* w, hipStream_t s);
// Host: each line's elimination order ord[line * nx + t] and pos[e] from w.
void bilu_mdf_order(int nx, int ny, int nz, const double* w, int* ord, int* pos);
// In-place block ILU(0) of every line (d <- inverses of the updated diagonal
// blocks, o <- L or U blocks); z = (L U)^-1 r.
hipError_t launch_bilu_factor(const DGArgs& a, int nb, const int* ord, const int* pos, double* d, double* o,
                              hipStream_t s);
hipError_t launch_bilu_apply(const DGArgs& a, int nb, const int* ord, const int* pos, const double* d,
                             const double* o, const double* r, double* z, hipStream_t s);
hipError_t launch_convert_fp64_to_bf16(const double* x, unsigned short* y, size_t n, hipStream_t s);

}  // namespace dg
