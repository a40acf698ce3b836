// C ABI of the MI355X DG hot path (include/dg.h) and the host-side
// orchestration of the device kernels: p-multigrid V-cycle (Sec. 6, Alg. 2),
// block-Jacobi smoothing (Sec. 6.3), right-preconditioned GMRES on the
// coarsest level and flexible GMRES outside (Sec. 6), BDF2 + Newton
// (Sec. 4, Eq. NEWTON).  Every arithmetic step runs in a device kernel; the
// host only sequences launches and, in FGMRES and Newton, reads one scalar per
// iteration to test convergence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace dg;

namespace dg {
hipError_t launch_backsolve(const double* H, int ldh, int k, const double* g, double* y, hipStream_t s);
hipError_t launch_init_g(double* g, int len, const double* beta2, hipStream_t s);
}  // namespace dg

namespace {

struct DgError {
    dg_status st;
};

// Device buffer owned by the context.
template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    void ensure(size_t want) {
        if (want <= n) return;
        release();
        if (hipMalloc(&p, want * sizeof(T)) != hipSuccess) {
            p = nullptr;
            n = 0;
            throw DgError{DG_ENOMEM};
        }
        n = want;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

// Krylov workspace (Arnoldi basis, preconditioned directions, Hessenberg).
struct Krylov {
    int m = 0;
    size_t N = 0;
    DBuf<double> V, Z, H, cs, sn, g, y, sc;
    void ensure(int m_, size_t N_) {
        m = m_;
        N = N_;
        V.ensure((size_t)(m + 1) * N);
        Z.ensure((size_t)m * N);
        H.ensure((size_t)(m + 1) * m);
        cs.ensure(m);
        sn.ensure(m);
        g.ensure(m + 1);
        y.ensure(m);
        sc.ensure(8);
    }
    void release() {
        V.release(); Z.release(); H.release(); cs.release(); sn.release(); g.release(); y.release();
        sc.release();
    }
};

struct Level {
    int p = 0, nv = 0, nb = 0;
    int ld = 0;           // leading dimension of the factors (fine_block_ld(nb) on level 0, else nb)
    size_t ndof = 0;
    DBuf<double> f64;     // factors (FP64)
    DBuf<float> f32;      // factors (FP32)
    DBuf<int> piv, pos;
    bool use32 = false;
    bool inv = false;          // explicit inverse (nb <= INV_POLICY_N) applied by GEMV
    bool inv_done = false;     // inverse already formed during setup (folded level)
    bool fold = false;         // coarsest assembled level stored as K D^-1 (unit diagonal, 6 face blocks)
    DBuf<double> inv64;
    DBuf<float> inv32;
    DBuf<double> x, b, r, t, z;
    DBuf<double> fb, fx;       // full multigrid: this level's restricted right-hand side and iterate
    bool bilu = false;         // coarsest level preconditioned by block ILU(0) (element lines along x)
    DBuf<double> bd, bo, bw;   // block ILU(0): inverses of the updated diagonal blocks, L/U line blocks, MDF weights
    DBuf<int> bord, bpos;      // each line's elimination order and every element's position in it
    // assembled inherited operator: diagonal + 6 face blocks per element
    bool assembled = false;
    int op_prec = DG_FP64;
    DBuf<double> op64;               // packed rows (launch_bsr_pack layout)
    DBuf<float> op32;
    DBuf<unsigned short> op16;
    void release() { inv64.release(); inv32.release(); op64.release(); op32.release(); op16.release();
                     f64.release(); f32.release(); piv.release(); pos.release(); x.release(); b.release(); r.release(); t.release(); z.release();
                     fb.release(); fx.release(); bd.release(); bo.release(); bw.release(); bord.release();
                     bpos.release(); }
};

std::mutex g_tab_mu;
bool g_tab_built = false;
Tab g_tabs[MAXP + 1];
short g_perm[PERM_TOTAL];
bool g_tab_uploaded[64] = {false};

// Scratch of dg_assemble_diag_noalloc: the neighbour traces at the face points
// (nbr_trace_size(p, ne) doubles), in a file-scope device array of fixed size
// that every GPU the library runs on holds until the process ends.  Host code
// never uses `scratch` directly: its device address on each device is
// resolved once (dg_create, with that device current) into g_scratch_ptr.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = (size_t)16 << 20;        // 128 MiB
__device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];
double* g_scratch_ptr[64] = {nullptr};                              // guarded by g_tab_mu

}  // namespace

struct dg_ctx {
    int device = 0;
    hipStream_t s = nullptr;
    DGArgs a{};
    int p = 0, nv = 0, nb = 0, ne = 0;
    size_t N = 0;
    std::string err;
    DBuf<double> vtx;                       // Q1 vertices of every element (also for straight boxes)
    DBuf<double> partial, scal;
    DBuf<int> flag;
    DBuf<double> tmp1, tmp2, tmp3;          // N-vector scratch for jvp / pMG / Newton
    DBuf<double> mb_op;                     // assembled fine operator (7-block BSR rows), dg_assemble_operator
    bool mb_ready = false;
    // preconditioner
    bool pmg_ready = false;
    pmg_opts popt{};
    double shift = 0.0;
    DBuf<double> W0, RW0, blk, otmp, dtmp, nbrtr;
    std::vector<Level> lv;
    Krylov kc;                              // coarsest-level GMRES
    std::vector<Krylov> ks;                 // GMRES(BJ) smoothers of the finer levels
    Krylov kf;                              // outer FGMRES
    // Newton
    DBuf<double> RW, Ru, xN;
    DBuf<double> Rst, Est;                  // ESDIRK3: R of the completed stages (3 N), their weighted sum (N)
    // V-cycle replayed as a HIP graph (captured on a private stream after setup)
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t vc_exec = nullptr;
    DBuf<double> gin, gout;
    // per-kernel timing
    bool timing = false;
    std::vector<hipEvent_t> ev;          // pairs (start, stop)
    std::vector<int> ev_kind;
    std::vector<double> ev_bytes, ev_flops;
    size_t ev_used = 0;
};

namespace dg {
const DGArgs& ctx_args(const dg_ctx* ctx) { return ctx->a; }
}  // namespace dg

namespace {

// scalar slots in ctx->scal
enum { S_NW2 = 0, S_NV2 = 1, S_H = 2, S_TMP = 3, S_PMG_NW2 = 8, S_F_NW2 = 9, S_F_EST = 10, S_F_B2 = 11,
       S_F_R2 = 12, S_N_R2 = 13, S_N_M2 = 14, S_C0 = 16, S_COUNT = 32 };

#define CK(expr)                                                                          \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
            throw DgError{DG_EHIP};                                                       \
        }                                                                                 \
    } while (0)

void fail(dg_ctx* ctx, dg_status st, const std::string& msg) {
    ctx->err = msg;
    throw DgError{st};
}

double* sc(dg_ctx* ctx, int slot) { return ctx->scal.p + slot; }

// Bracket one launch with events when timing is on.
template <class F>
void timed(dg_ctx* ctx, int kind, double bytes, double flops, F&& launch) {
    if (!ctx->timing) {
        CK(launch());
        return;
    }
    if (2 * (ctx->ev_used + 1) > ctx->ev.size()) {
        hipEvent_t a, b;
        CK(hipEventCreate(&a));
        CK(hipEventCreate(&b));
        ctx->ev.push_back(a);
        ctx->ev.push_back(b);
        ctx->ev_kind.push_back(0);
        ctx->ev_bytes.push_back(0.0);
        ctx->ev_flops.push_back(0.0);
    }
    const size_t i = ctx->ev_used++;
    ctx->ev_kind[i] = kind;
    ctx->ev_bytes[i] = bytes;
    ctx->ev_flops[i] = flops;
    CK(hipEventRecord(ctx->ev[2 * i], ctx->s));
    CK(launch());
    CK(hipEventRecord(ctx->ev[2 * i + 1], ctx->s));
}

double read_scalar(dg_ctx* ctx, const double* dptr) {
    double v = 0.0;
    CK(hipMemcpyAsync(&v, dptr, sizeof(double), hipMemcpyDeviceToHost, ctx->s));
    CK(hipStreamSynchronize(ctx->s));
    return v;
}

void dot(dg_ctx* ctx, const double* x, const double* y, size_t n, double* out) {
    CK(launch_dot(x, y, n, ctx->partial.p, out, ctx->s));
}

// y = shift M v + (R(W + h v) - RW)/h.  nw2: device ||W||^2 (computed if null).
void jvp_fd(dg_ctx* ctx, const double* W, const double* RW, const double* v, double shift, double* y,
            const double* nw2) {
    CK(launch_fd_step(v, nw2 ? nullptr : W, ctx->N, nw2, nw2 ? nullptr : sc(ctx, S_NW2), 1e-7, ctx->partial.p,
                      sc(ctx, S_NV2), sc(ctx, S_H), ctx->s));
    timed(ctx, DG_K_JVP_FD, 32.0 * (double)ctx->N, 0.0, [&] { return launch_jvp_fd(ctx->a, W, RW, v, sc(ctx, S_H), shift, y, ctx->s); });
}

// ---- p-multigrid ------------------------------------------------------------------
void bj_apply(dg_ctx* ctx, int l, const double* r, double* z) {
    Level& L = ctx->lv[l];
    const double nbl = L.nb, sf = L.use32 ? 4.0 : 8.0;
    timed(ctx, l == 0 ? DG_K_BJ_FINE : DG_K_BJ_COARSE, ctx->ne * (sf * nbl * nbl + 16.0 * nbl),
          ctx->ne * 2.0 * nbl * nbl, [&] {
        if (L.inv)
            return L.use32 ? launch_inv_gemv<float>(L.inv32.p, r, z, ctx->ne, L.nb, ctx->s)
                           : launch_inv_gemv<double>(L.inv64.p, r, z, ctx->ne, L.nb, ctx->s);
        return L.use32 ? launch_lu_solve_blocked<float>(L.f32.p, L.pos.p, r, z, ctx->ne, L.nb, L.ld, ctx->s)
                       : launch_lu_solve_blocked<double>(L.f64.p, L.pos.p, r, z, ctx->ne, L.nb, L.ld, ctx->s);
    });
}

// y = K_l x (level operator): level 0 the FD product (Eq. DG-mf) at the
// lagged state; coarse levels the inherited P^T K_0 P applied matrix-free.
void level_op(dg_ctx* ctx, int l, const double* x, double* y) {
    if (l == 0) {
        jvp_fd(ctx, ctx->W0.p, ctx->RW0.p, x, ctx->shift, y, sc(ctx, S_PMG_NW2));
        return;
    }
    const Level& L = ctx->lv[l];
    if (L.assembled && L.fold) fail(ctx, DG_ESTATE, "folded coarsest operator used as a plain operator");
    if (L.assembled) {
        const double nbc = L.nb, sz = L.op_prec == DG_FP64 ? 8.0 : (L.op_prec == DG_FP32 ? 4.0 : 2.0);
        timed(ctx, DG_K_BSR, ctx->ne * (7.0 * nbc * nbc * sz + 16.0 * nbc), ctx->ne * 14.0 * nbc * nbc, [&] {
            if (L.op_prec == DG_FP64) return launch_bsr7<double>(ctx->a, L.op64.p, x, y, L.nb, ctx->s);
            if (L.op_prec == DG_FP32) return launch_bsr7<float>(ctx->a, L.op32.p, x, y, L.nb, ctx->s);
            return launch_bsr7<unsigned short>(ctx->a, L.op16.p, x, y, L.nb, ctx->s);
        });
        return;
    }
    CK(launch_prolong_add(ctx->ne, ctx->nv, L.nv, x, ctx->tmp1.p, 1, ctx->s));
    jvp_fd(ctx, ctx->W0.p, ctx->RW0.p, ctx->tmp1.p, ctx->shift, ctx->tmp2.p, sc(ctx, S_PMG_NW2));
    CK(launch_restrict(ctx->ne, ctx->nv, L.nv, ctx->tmp2.p, y, ctx->s));
}

void gmres_fixed_dev(dg_ctx* ctx, int l, Krylov& K, const double* b, double* x, int iters);

// Right preconditioner of a level's GMRES: block ILU(0) on a coarsest level
// that has it, element block Jacobi otherwise.
void level_prec(dg_ctx* ctx, int l, const double* r, double* z) {
    Level& L = ctx->lv[l];
    if (!L.bilu) {
        bj_apply(ctx, l, r, z);
        return;
    }
    const double nbl = L.nb;
    timed(ctx, DG_K_BJ_COARSE, ctx->ne * (5.0 * 8.0 * nbl * nbl + 16.0 * nbl), ctx->ne * 10.0 * nbl * nbl, [&] {
        return launch_bilu_apply(ctx->a, L.nb, L.bord.p, L.bpos.p, L.bd.p, L.bo.p, r, z, ctx->s);
    });
}

// SMOOTH of Alg. 2 on level l: nu damped block-Jacobi sweeps, or (smoother =
// 1) nu iterations of right-preconditioned GMRES(BJ) on the residual
// equation, x <- x + GMRES(K_l, D_l^-1, b - K_l x).
void smooth(dg_ctx* ctx, int l, double* x, const double* b, int nu, bool x_zero) {
    Level& L = ctx->lv[l];
    if (ctx->popt.smoother == 1) {
        if (nu == 0) {
            if (x_zero) CK(launch_fill(L.ndof, 0.0, x, ctx->s));
            return;
        }
        const double* r = b;
        if (!x_zero) {
            level_op(ctx, l, x, L.t.p);
            CK(launch_axpby(L.ndof, 1.0, b, -1.0, L.t.p, L.r.p, ctx->s));
            r = L.r.p;
        }
        gmres_fixed_dev(ctx, l, ctx->ks[l], r, L.z.p, nu);
        if (x_zero) CK(launch_copy(L.ndof, L.z.p, x, ctx->s));
        else CK(launch_axpby(L.ndof, 1.0, L.z.p, 1.0, x, x, ctx->s));
        return;
    }
    const double om = ctx->popt.omega;
    for (int s = 0; s < nu; ++s) {
        if (s == 0 && x_zero) {
            bj_apply(ctx, l, b, L.z.p);
            CK(launch_axpby(L.ndof, om, L.z.p, 0.0, nullptr, x, ctx->s));
        } else {
            level_op(ctx, l, x, L.t.p);
            CK(launch_axpby(L.ndof, 1.0, b, -1.0, L.t.p, L.r.p, ctx->s));
            bj_apply(ctx, l, L.r.p, L.z.p);
            CK(launch_axpby(L.ndof, om, L.z.p, 1.0, x, x, ctx->s));
        }
    }
    if (nu == 0 && x_zero) CK(launch_fill(L.ndof, 0.0, x, ctx->s));
}

// Arnoldi step j with classical Gram-Schmidt applied twice; w is in V[j+1].
void arnoldi_orth(dg_ctx* ctx, Krylov& K, int j, size_t n) {
    timed(ctx, DG_K_ARNOLDI, 24.0 * (j + 1) * (double)n + 32.0 * (double)n, 6.0 * (j + 1) * (double)n, [&] {
        return launch_arnoldi_cgs2(K.V.p, n, j, K.H.p, K.m + 1, K.cs.p, K.sn.p, K.g.p, K.sc.p + 1,
                                   K.sc.p + 2, ctx->partial.p, ctx->s);
    });
}

// y = (K D^-1) x on the folded coarsest level: x plus the six face products.
void folded_op(dg_ctx* ctx, int l, const double* x, double* y) {
    const Level& L = ctx->lv[l];
    const double nbc = L.nb, sz = L.op_prec == DG_FP64 ? 8.0 : (L.op_prec == DG_FP32 ? 4.0 : 2.0);
    timed(ctx, DG_K_BSR, ctx->ne * (6.0 * nbc * nbc * sz + 16.0 * nbc), ctx->ne * 12.0 * nbc * nbc, [&] {
        if (L.op_prec == DG_FP64) return launch_bsr_unit<double>(ctx->a, L.op64.p, x, y, L.nb, ctx->s);
        if (L.op_prec == DG_FP32) return launch_bsr_unit<float>(ctx->a, L.op32.p, x, y, L.nb, ctx->s);
        return launch_bsr_unit<unsigned short>(ctx->a, L.op16.p, x, y, L.nb, ctx->s);
    });
}

// Coarsest SOLVE: right-preconditioned GMRES(BJ) from x = 0 for exactly
// `iters` steps, all on the device (no host synchronisation).  On a folded
// level the Arnoldi process runs on K D^-1 directly (one product per step)
// and x = D^-1 (V y) at the end: the same Krylov space and iterate.
void coarse_gmres(dg_ctx* ctx, int l, const double* b, double* x, int iters) {
    Level& L = ctx->lv[l];
    Krylov& K = ctx->kc;
    const size_t n = L.ndof;
    if (L.fold) {
        dot(ctx, b, b, n, K.sc.p + 3);
        CK(launch_init_g(K.g.p, iters + 1, K.sc.p + 3, ctx->s));
        CK(launch_scale_dev(n, b, K.g.p, 1, K.V.p, ctx->s));
        const bool fuse = bsr_grid(ctx->ne, L.nb) <= RED_BLOCKS;
        const double nbc = L.nb, sz = L.op_prec == DG_FP64 ? 8.0 : (L.op_prec == DG_FP32 ? 4.0 : 2.0);
        for (int j = 0; j < iters; ++j) {
            const double* x = K.V.p + (size_t)j * n;
            double* y = K.V.p + (size_t)(j + 1) * n;
            if (!fuse) {
                folded_op(ctx, l, x, y);
                arnoldi_orth(ctx, K, j, n);
                continue;
            }
            // product and first Gram-Schmidt pass in one launch (timed as the product)
            int np = 0;
            timed(ctx, DG_K_BSR, ctx->ne * (6.0 * nbc * nbc * sz + 16.0 * nbc) + 8.0 * (j + 1) * n,
                  ctx->ne * 12.0 * nbc * nbc + 2.0 * (j + 1) * n, [&] {
                if (L.op_prec == DG_FP64)
                    return launch_bsr_unit_dots<double>(ctx->a, L.op64.p, x, y, L.nb, K.V.p, j + 1, ctx->partial.p,
                                                        &np, ctx->s);
                if (L.op_prec == DG_FP32)
                    return launch_bsr_unit_dots<float>(ctx->a, L.op32.p, x, y, L.nb, K.V.p, j + 1, ctx->partial.p,
                                                       &np, ctx->s);
                return launch_bsr_unit_dots<unsigned short>(ctx->a, L.op16.p, x, y, L.nb, K.V.p, j + 1,
                                                            ctx->partial.p, &np, ctx->s);
            });
            timed(ctx, DG_K_ARNOLDI, 16.0 * (j + 1) * (double)n + 32.0 * (double)n, 4.0 * (j + 1) * (double)n, [&] {
                return launch_arnoldi_cgs2_after_dots(K.V.p, n, j, K.H.p, K.m + 1, K.cs.p, K.sn.p, K.g.p,
                                                      K.sc.p + 1, K.sc.p + 2, ctx->partial.p, np, ctx->s);
            });
        }
        CK(launch_backsolve(K.H.p, K.m + 1, iters, K.g.p, K.y.p, ctx->s));
        CK(launch_fill(n, 0.0, L.t.p, ctx->s));
        CK(launch_multi_axpy(n, iters, K.y.p, 1, K.V.p, n, L.t.p, ctx->s));
        bj_apply(ctx, l, L.t.p, x);
        return;
    }
    gmres_fixed_dev(ctx, l, K, b, x, iters);
}

// Right-preconditioned GMRES(BJ) on level l from x = 0 for exactly `iters`
// Arnoldi steps (K sized for this level and at least `iters`), all on the device.
void gmres_fixed_dev(dg_ctx* ctx, int l, Krylov& K, const double* b, double* x, int iters) {
    const size_t n = ctx->lv[l].ndof;
    dot(ctx, b, b, n, K.sc.p + 3);
    CK(launch_init_g(K.g.p, iters + 1, K.sc.p + 3, ctx->s));
    CK(launch_scale_dev(n, b, K.g.p, 1, K.V.p, ctx->s));
    for (int j = 0; j < iters; ++j) {
        double* z = K.Z.p + (size_t)j * n;
        level_prec(ctx, l, K.V.p + (size_t)j * n, z);
        level_op(ctx, l, z, K.V.p + (size_t)(j + 1) * n);
        arnoldi_orth(ctx, K, j, n);
    }
    CK(launch_backsolve(K.H.p, K.m + 1, iters, K.g.p, K.y.p, ctx->s));
    CK(launch_fill(n, 0.0, x, ctx->s));
    CK(launch_multi_axpy(n, iters, K.y.p, 1, K.Z.p, n, x, ctx->s));
}

// Alg. 2: MG_V(l, b_l, x_l), from x_l = 0 (x_zero) or from the given x_l.
void vcycle(dg_ctx* ctx, int l, const double* b, double* x, bool x_zero = true) {
    const int Lc = (int)ctx->lv.size() - 1;
    if (l == Lc) {
        coarse_gmres(ctx, l, b, x, ctx->popt.coarsest_iters);
        return;
    }
    Level& L = ctx->lv[l];
    Level& C = ctx->lv[l + 1];
    smooth(ctx, l, x, b, ctx->popt.nu_pre, x_zero);
    level_op(ctx, l, x, L.t.p);
    CK(launch_axpby(L.ndof, 1.0, b, -1.0, L.t.p, L.r.p, ctx->s));
    CK(launch_restrict(ctx->ne, L.nv, C.nv, L.r.p, C.b.p, ctx->s));
    vcycle(ctx, l + 1, C.b.p, C.x.p);
    CK(launch_prolong_add(ctx->ne, L.nv, C.nv, C.x.p, x, 0, ctx->s));
    smooth(ctx, l, x, b, ctx->popt.nu_post, false);
}

// Alg. 1: MG_full.  b_l is the level-0 right-hand side restricted to level l;
// the coarsest level is solved from zero, then each finer level runs one
// V-cycle from the prolongation of the coarser level's result.
void fmg(dg_ctx* ctx, const double* b, double* z) {
    const int Lc = (int)ctx->lv.size() - 1;
    const int nv0 = ctx->lv[0].nv;
    Level& C = ctx->lv[Lc];
    CK(launch_restrict(ctx->ne, nv0, C.nv, b, C.fb.p, ctx->s));
    coarse_gmres(ctx, Lc, C.fb.p, C.fx.p, ctx->popt.coarsest_iters);
    for (int l = Lc - 1; l >= 0; --l) {
        Level& L = ctx->lv[l];
        Level& U = ctx->lv[l + 1];
        const double* bl = b;
        double* xl = z;
        if (l > 0) {
            CK(launch_restrict(ctx->ne, nv0, L.nv, b, L.fb.p, ctx->s));
            bl = L.fb.p;
            xl = L.fx.p;
        }
        CK(launch_prolong_add(ctx->ne, L.nv, U.nv, U.fx.p, xl, 1, ctx->s));
        vcycle(ctx, l, bl, xl, false);
    }
}

void drop_graph(dg_ctx* ctx) {
    if (ctx->vc_exec) (void)hipGraphExecDestroy(ctx->vc_exec);
    ctx->vc_exec = nullptr;
}

void pmg_apply_eager(dg_ctx* ctx, const double* r, double* z) {
    if (ctx->lv.size() == 1) bj_apply(ctx, 0, r, z);
    else if (ctx->popt.cycle == 1) fmg(ctx, r, z);
    else vcycle(ctx, 0, r, z);
}

// Capture one V-cycle from ctx->gin to ctx->gout.  The sequence of launches
// depends only on the setup, so it is recorded once per pmg_setup.
void capture_vcycle(dg_ctx* ctx) {
    if (!ctx->cap_stream) CK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    ctx->gin.ensure(ctx->N);
    ctx->gout.ensure(ctx->N);
    hipStream_t saved = ctx->s;
    ctx->s = ctx->cap_stream;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        try {
            pmg_apply_eager(ctx, ctx->gin.p, ctx->gout.p);
        } catch (...) {
            (void)hipStreamEndCapture(ctx->cap_stream, &g);
            if (g) (void)hipGraphDestroy(g);
            ctx->s = saved;
            throw;
        }
        e = hipStreamEndCapture(ctx->cap_stream, &g);
    }
    ctx->s = saved;
    CK(e);
    e = hipGraphInstantiate(&ctx->vc_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    CK(e);
}

void pmg_apply_impl(dg_ctx* ctx, const double* r, double* z) {
    if (!ctx->pmg_ready) fail(ctx, DG_ESTATE, "pmg_apply before pmg_setup");
    if (!ctx->use_graphs || ctx->timing) {
        pmg_apply_eager(ctx, r, z);
        return;
    }
    if (!ctx->vc_exec) capture_vcycle(ctx);
    CK(launch_copy(ctx->N, r, ctx->gin.p, ctx->s));
    CK(hipGraphLaunch(ctx->vc_exec, ctx->s));
    CK(launch_copy(ctx->N, ctx->gout.p, z, ctx->s));
}

void check_pmg_opts(dg_ctx* ctx, const pmg_opts* o) {
    if (!o) fail(ctx, DG_EINVAL, "null pmg_opts");
    if (o->n_levels < 1 || o->n_levels > 4) fail(ctx, DG_EINVAL, "n_levels must be 1..4");
    if (o->p_level[0] != ctx->p) fail(ctx, DG_EINVAL, "p_level[0] must equal the context degree");
    for (int l = 1; l < o->n_levels; ++l)
        if (o->p_level[l] < 1 || o->p_level[l] >= o->p_level[l - 1])
            fail(ctx, DG_EINVAL, "coarse degrees must decrease and be >= 1");
    if (o->nu_pre < 0 || o->nu_post < 0 || o->coarsest_iters < 1 || o->coarsest_iters > 63)
        fail(ctx, DG_EINVAL, "bad sweep or coarsest iteration counts");
    if (o->prec_fine != DG_FP64 && o->prec_fine != DG_FP32) fail(ctx, DG_EINVAL, "prec_fine must be FP64 or FP32");
    if (o->prec_coarse != DG_FP64 && o->prec_coarse != DG_FP32 && o->prec_coarse != DG_BF16)
        fail(ctx, DG_EINVAL, "prec_coarse must be FP64, FP32 or BF16");
    if (o->coarse_matrix_free < 0 || o->coarse_matrix_free > 2) fail(ctx, DG_EINVAL, "coarse_matrix_free must be 0, 1 or 2");
    if (o->coarsest_plain != 0 && o->coarsest_plain != 1) fail(ctx, DG_EINVAL, "coarsest_plain must be 0 or 1");
    if (o->smoother != 0 && o->smoother != 1) fail(ctx, DG_EINVAL, "smoother must be 0 (BJ sweeps) or 1 (GMRES(BJ))");
    if (o->cycle != 0 && o->cycle != 1) fail(ctx, DG_EINVAL, "cycle must be 0 (V-cycle) or 1 (full multigrid)");
    if (o->smoother == 1 && (o->nu_pre > 63 || o->nu_post > 63))
        fail(ctx, DG_EINVAL, "GMRES smoother iterations must be at most 63");
    if (o->coarsest_prec != 0 && o->coarsest_prec != 1) fail(ctx, DG_EINVAL, "coarsest_prec must be 0 (BJ) or 1 (BILU)");
    if (o->coarsest_prec == 1) {
        if (o->n_levels < 2 || o->coarse_matrix_free == 1)
            fail(ctx, DG_EINVAL, "BILU needs an assembled coarsest level (n_levels >= 2, coarse_matrix_free 0 or 2)");
        const int pc = o->p_level[o->n_levels - 1];
        if (5 * (pc + 1) * (pc + 1) * (pc + 1) > BILU_MAX_N)
            fail(ctx, DG_EINVAL, "BILU supports a degree-1 coarsest level only");
    }
}

double lu_bytes(dg_ctx* ctx, int nb, double s) { return ctx->ne * 2.0 * s * (double)nb * nb; }
double lu_flops(dg_ctx* ctx, int nb) { return ctx->ne * (2.0 / 3.0) * (double)nb * nb * nb; }

// Pack the assembled operator of level L (diagonal in dtmp unless nblk = 6,
// face blocks in otmp) at its storage precision.
void pack_operator(dg_ctx* ctx, Level& L, int nblk) {
    const size_t pk = bsr_entries(ctx->ne, L.nb, nblk);
    if (L.op_prec == DG_FP64) {
        L.op64.ensure(pk);
        CK(launch_bsr_pack<double>(ctx->dtmp.p, ctx->otmp.p, L.op64.p, ctx->ne, L.nb, nblk, ctx->s));
    } else if (L.op_prec == DG_FP32) {
        L.op32.ensure(pk);
        CK(launch_bsr_pack<float>(ctx->dtmp.p, ctx->otmp.p, L.op32.p, ctx->ne, L.nb, nblk, ctx->s));
    } else {
        L.op16.ensure(pk);
        CK(launch_bsr_pack<unsigned short>(ctx->dtmp.p, ctx->otmp.p, L.op16.p, ctx->ne, L.nb, nblk, ctx->s));
    }
}

// Explicit block inverses of level L from its PLU factors (ws: FP64
// workspace of ne nb^2 entries, used for FP32 factors only).
void form_inverse(dg_ctx* ctx, Level& L, double* ws) {
    const size_t sz = (size_t)ctx->ne * L.nb * L.nb;
    const double fl = ctx->ne * 2.0 * (double)L.nb * L.nb * L.nb;
    if (L.use32) {
        L.inv32.ensure(sz);
        timed(ctx, DG_K_LU, 4.0 * sz + 8.0 * 2.0 * sz, fl, [&] {
            return launch_lu_inverse<float>(L.f32.p, L.pos.p, ws, L.inv32.p, ctx->ne, L.nb, ctx->s);
        });
    } else {
        L.inv64.ensure(sz);
        timed(ctx, DG_K_LU, 8.0 * sz + 8.0 * 2.0 * sz, fl, [&] {
            return launch_lu_inverse<double>(L.f64.p, L.pos.p, L.inv64.p, (double*)nullptr, ctx->ne, L.nb, ctx->s);
        });
    }
    L.inv_done = true;
}

// Block ILU(0) of the coarsest level from its unpacked FP64 blocks (diagonal
// in dtmp, face blocks in otmp): line couplings gathered, minimum-discarded-
// fill weights on the device, each line's order on the host, then the
// in-place factorisation, one workgroup per line.
void bilu_setup(dg_ctx* ctx, Level& L) {
    const size_t nn = (size_t)L.nb * L.nb;
    const MeshDev& m = ctx->a.m;
    L.bd.ensure(ctx->ne * nn);
    L.bo.ensure(2 * ctx->ne * nn);
    L.bw.ensure(ctx->ne);
    L.bord.ensure(ctx->ne);
    L.bpos.ensure(ctx->ne);
    CK(launch_bilu_gather(ctx->a, L.nb, ctx->dtmp.p, ctx->otmp.p, L.bd.p, L.bo.p, ctx->s));
    CK(launch_bilu_weights(ctx->a, L.nb, L.bd.p, L.bo.p, L.bw.p, ctx->s));
    std::vector<double> w(ctx->ne);
    std::vector<int> ord(ctx->ne), pos(ctx->ne);
    CK(hipMemcpyAsync(w.data(), L.bw.p, ctx->ne * sizeof(double), hipMemcpyDeviceToHost, ctx->s));
    CK(hipStreamSynchronize(ctx->s));
    bilu_mdf_order(m.nx, m.ny, m.nz, w.data(), ord.data(), pos.data());
    CK(hipMemcpyAsync(L.bord.p, ord.data(), ctx->ne * sizeof(int), hipMemcpyHostToDevice, ctx->s));
    CK(hipMemcpyAsync(L.bpos.p, pos.data(), ctx->ne * sizeof(int), hipMemcpyHostToDevice, ctx->s));
    CK(launch_bilu_factor(ctx->a, L.nb, L.bord.p, L.bpos.p, L.bd.p, L.bo.p, ctx->s));
    CK(hipStreamSynchronize(ctx->s));                 // the host order arrays go out of scope
}

void pmg_setup_impl(dg_ctx* ctx, const double* W, double shift, const pmg_opts* o) {
    check_pmg_opts(ctx, o);
    ctx->pmg_ready = false;
    drop_graph(ctx);
    ctx->popt = *o;
    ctx->shift = shift;
    const size_t N = ctx->N;
    ctx->W0.ensure(N);
    ctx->RW0.ensure(N);
    CK(launch_copy(N, W, ctx->W0.p, ctx->s));
    CK(launch_residual(ctx->a, ctx->W0.p, ctx->RW0.p, ctx->s));
    dot(ctx, ctx->W0.p, ctx->W0.p, N, sc(ctx, S_PMG_NW2));
    const int nb = ctx->nb, ld0 = fine_block_ld(nb);
    ctx->blk.ensure((size_t)ctx->ne * nb * ld0);
    ctx->nbrtr.ensure(nbr_trace_size(ctx->p, ctx->ne));
    timed(ctx, DG_K_DIAG_BLOCKS, 8.0 * ctx->ne * (double)nb * nb + 8.0 * (double)ctx->N, 0.0, [&] { return launch_diag_blocks(ctx->a, ctx->W0.p, shift, ctx->blk.p, ld0, ctx->nbrtr.p, ctx->s); });
    for (size_t l = o->n_levels; l < ctx->lv.size(); ++l) ctx->lv[l].release();
    ctx->lv.resize(o->n_levels);
    for (int l = 0; l < o->n_levels; ++l) {
        Level& L = ctx->lv[l];
        L.p = o->p_level[l];
        L.nv = (L.p + 1) * (L.p + 1) * (L.p + 1);
        L.nb = 5 * L.nv;
        L.ld = (l == 0) ? ld0 : L.nb;
        L.ndof = (size_t)ctx->ne * L.nb;
        L.use32 = (l == 0) ? (o->prec_fine == DG_FP32) : (o->prec_coarse != DG_FP64);
        L.assembled = l > 0 && (o->coarse_matrix_free == 0 ||
                                (o->coarse_matrix_free == 2 && l == o->n_levels - 1));
        L.op_prec = o->prec_coarse;
        L.inv = L.nb <= INV_POLICY_N;
        L.inv_done = false;
        L.bilu = L.assembled && l == o->n_levels - 1 && o->coarsest_prec == 1;
        L.fold = L.assembled && l == o->n_levels - 1 && L.inv && L.nb <= FOLD_MAX_N && o->coarsest_plain == 0 &&
                 !L.bilu;
        L.piv.ensure((size_t)ctx->ne * L.nb);
        L.pos.ensure((size_t)ctx->ne * L.nb);
        L.x.ensure(L.ndof);
        L.b.ensure(L.ndof);
        L.r.ensure(L.ndof);
        L.t.ensure(L.ndof);
        L.z.ensure(L.ndof);
    }
    // coarse blocks are principal sub-blocks of the unfactored fine blocks
    for (int l = o->n_levels - 1; l >= 0; --l) {
        Level& L = ctx->lv[l];
        const size_t sz = (size_t)ctx->ne * L.nb * L.nb;
        if (L.assembled) {
            // inherited operator K_l = P^T K_0 P: diagonal sub-blocks + face-coupling blocks
            ctx->dtmp.ensure(sz);
            ctx->otmp.ensure(6 * sz);
            CK(launch_extract_sub<double>(ctx->blk.p, nb, ld0, ctx->nv, L.nv, ctx->dtmp.p, ctx->ne, ctx->s));
            CK(launch_offdiag_blocks(ctx->a, ctx->W0.p, L.p, ctx->otmp.p, ctx->s));
            if (!L.fold) pack_operator(ctx, L, 7);
            if (L.bilu) bilu_setup(ctx, L);
        }
        if (L.use32) {
            const size_t szl = (size_t)ctx->ne * L.nb * L.ld;
            L.f32.ensure(szl);
            if (l == 0) CK(launch_convert_fp64_to_fp32(ctx->blk.p, L.f32.p, szl, ctx->s));
            else CK(launch_extract_sub<float>(ctx->blk.p, nb, ld0, ctx->nv, L.nv, L.f32.p, ctx->ne, ctx->s));
            timed(ctx, DG_K_LU, lu_bytes(ctx, L.nb, 4.0), lu_flops(ctx, L.nb), [&] { return launch_lu_blocked<float>(L.f32.p, L.piv.p, L.pos.p, ctx->ne, L.nb, L.ld, ctx->s); });
        } else {
            if (l == 0) {
                timed(ctx, DG_K_LU, lu_bytes(ctx, L.nb, 8.0), lu_flops(ctx, L.nb), [&] { return launch_lu_blocked<double>(ctx->blk.p, L.piv.p, L.pos.p, ctx->ne, L.nb, L.ld, ctx->s); });
            } else {
                L.f64.ensure(sz);
                CK(launch_extract_sub<double>(ctx->blk.p, nb, ld0, ctx->nv, L.nv, L.f64.p, ctx->ne, ctx->s));
                timed(ctx, DG_K_LU, lu_bytes(ctx, L.nb, 8.0), lu_flops(ctx, L.nb), [&] { return launch_lu_blocked<double>(L.f64.p, L.piv.p, L.pos.p, ctx->ne, L.nb, L.ld, ctx->s); });
            }
        }
        if (L.fold) {
            // K D^-1: the block inverses first (FP64 workspace: the diagonal
            // sub-blocks in dtmp are not needed once factored), then the fold
            form_inverse(ctx, L, ctx->dtmp.p);
            if (L.use32) CK(launch_fold_inverse<float>(ctx->a, L.nb, ctx->otmp.p, L.inv32.p, ctx->s));
            else CK(launch_fold_inverse<double>(ctx->a, L.nb, ctx->otmp.p, L.inv64.p, ctx->s));
            pack_operator(ctx, L, 6);
        }
    }
    // level 0 FP64 factors live in blk (factored in place)
    if (!ctx->lv[0].use32) {
        std::swap(ctx->lv[0].f64.p, ctx->blk.p);
        std::swap(ctx->lv[0].f64.n, ctx->blk.n);
    }
    // explicit inverses for the smoother apply: blocks up to 135 entries.  For
    // larger blocks the inverse costs more than the PLU itself and the blocked
    // triangular solves are cheaper over the ~100 applies of one time step.
    for (int l = 0; l < o->n_levels; ++l) {
        Level& L = ctx->lv[l];
        if (!L.inv || L.inv_done) continue;
        if (L.use32) ctx->blk.ensure((size_t)ctx->ne * L.nb * L.nb);   // FP64 workspace (the FP64 blocks are no longer needed)
        form_inverse(ctx, L, ctx->blk.p);
    }
    if (o->n_levels > 1) {
        const Level& Lc = ctx->lv.back();
        ctx->kc.ensure(o->coarsest_iters, Lc.ndof);
    }
    // GMRES(BJ) smoothers: one Krylov workspace per finer level
    if (o->n_levels > 1 && o->smoother == 1) {
        if (ctx->ks.size() < (size_t)(o->n_levels - 1)) ctx->ks.resize(o->n_levels - 1);
        const int m = std::max(1, std::max(o->nu_pre, o->nu_post));
        for (int l = 0; l < o->n_levels - 1; ++l) ctx->ks[l].ensure(m, ctx->lv[l].ndof);
    }
    for (size_t l = (o->smoother == 1 ? (size_t)std::max(0, o->n_levels - 1) : 0); l < ctx->ks.size(); ++l)
        ctx->ks[l].release();
    for (Level& L : ctx->lv)
        if (!L.bilu) {
            L.bd.release(); L.bo.release(); L.bw.release(); L.bord.release(); L.bpos.release();
        }
    // full multigrid: restricted right-hand sides and iterates of the coarse levels
    for (int l = 1; l < o->n_levels; ++l) {
        Level& L = ctx->lv[l];
        if (o->cycle == 1) {
            L.fb.ensure(L.ndof);
            L.fx.ensure(L.ndof);
        } else {
            L.fb.release();
            L.fx.release();
        }
    }
    ctx->pmg_ready = true;
}

// ---- FGMRES (Sec. 6) --------------------------------------------------------------------
void fgmres_impl(dg_ctx* ctx, const double* W, const double* RW, const double* b, double* x, const fgmres_opts* o,
                 fgmres_stats* st) {
    if (!o || o->restart < 1 || o->restart > 63 || o->max_restarts < 0 || !(o->rtol > 0.0))
        fail(ctx, DG_EINVAL, "bad fgmres_opts");
    const size_t n = ctx->N;
    Krylov& K = ctx->kf;
    const int m = o->restart;
    K.ensure(m, n);
    fgmres_stats loc{};
    const double shift = ctx->pmg_ready ? ctx->shift : 0.0;
    auto op = [&](const double* v, double* y) {
        if (o->jvp_exact) timed(ctx, DG_K_JVP_EXACT, 24.0 * (double)ctx->N, 0.0, [&] { return launch_jvp_exact(ctx->a, W, v, shift, y, ctx->s); });
        else jvp_fd(ctx, W, RW, v, shift, y, sc(ctx, S_F_NW2));
    };
    if (!o->jvp_exact) dot(ctx, W, W, n, sc(ctx, S_F_NW2));
    dot(ctx, b, b, n, sc(ctx, S_F_B2));
    const double bn = std::sqrt(read_scalar(ctx, sc(ctx, S_F_B2)));
    CK(launch_fill(n, 0.0, x, ctx->s));
    if (!std::isfinite(bn)) fail(ctx, DG_ENONFINITE, "non-finite right-hand side");
    if (bn == 0.0) {
        loc.rel_res_true = loc.rel_res_est = 0.0;
        if (st) *st = loc;
        return;
    }
    double* r = ctx->tmp3.p;
    CK(launch_copy(n, b, r, ctx->s));
    double beta = bn;
    bool converged = false;
    for (int rs = 0; rs <= o->max_restarts; ++rs) {
        if (rs > 0) {
            dot(ctx, r, r, n, sc(ctx, S_F_R2));
        } else {
            CK(launch_copy(1, sc(ctx, S_F_B2), sc(ctx, S_F_R2), ctx->s));
        }
        CK(launch_init_g(K.g.p, m + 1, sc(ctx, S_F_R2), ctx->s));
        CK(launch_scale_dev(n, r, K.g.p, 1, K.V.p, ctx->s));
        int k = 0;
        for (int j = 0; j < m; ++j) {
            double* z = K.Z.p + (size_t)j * n;
            if (ctx->pmg_ready) pmg_apply_impl(ctx, K.V.p + (size_t)j * n, z);
            else CK(launch_copy(n, K.V.p + (size_t)j * n, z, ctx->s));
            op(z, K.V.p + (size_t)(j + 1) * n);
            arnoldi_orth(ctx, K, j, n);
            k = j + 1;
            loc.iters++;
            const double est = read_scalar(ctx, K.sc.p + 2);
            if (!std::isfinite(est)) fail(ctx, DG_ENONFINITE, "non-finite Krylov residual estimate");
            loc.rel_res_est = est / bn;
            if (est <= o->rtol * bn) break;
        }
        CK(launch_backsolve(K.H.p, m + 1, k, K.g.p, K.y.p, ctx->s));
        CK(launch_multi_axpy(n, k, K.y.p, 1, K.Z.p, n, x, ctx->s));
        // true residual
        op(x, ctx->tmp2.p);
        CK(launch_axpby(n, 1.0, b, -1.0, ctx->tmp2.p, r, ctx->s));
        dot(ctx, r, r, n, sc(ctx, S_F_R2));
        beta = std::sqrt(read_scalar(ctx, sc(ctx, S_F_R2)));
        loc.rel_res_true = beta / bn;
        if (!std::isfinite(beta)) fail(ctx, DG_ENONFINITE, "non-finite true residual");
        if (beta <= o->rtol * bn) {
            converged = true;
            break;
        }
        if (rs < o->max_restarts) loc.restarts++;
    }
    if (st) *st = loc;
    if (!converged) fail(ctx, DG_ENOCONV, "FGMRES did not reach rtol");
}

void ensure_scratch(dg_ctx* ctx) {
    ctx->tmp1.ensure(ctx->N);
    ctx->tmp2.ensure(ctx->N);
    ctx->tmp3.ensure(ctx->N);
}

// Newton iterations on one nonlinear system of a time step (Sec. 4, Eq.
// NEWTON): unsteady() evaluates R(W) into ctx->RW and the system's residual
// R_u(W) into ctx->Ru and returns ||R_u||; each iteration solves
// K x = -R_u by FGMRES (K linearised at the current W, shift of the lagged
// preconditioner) and sets W += x.  Stops when ||R_u|| <= rtol ||R_u(W_0)||
// or below `floor`.  Accumulates into loc; returns whether it converged.
template <class U>
bool newton_solve(dg_ctx* ctx, double* W, U&& unsteady, const fgmres_opts* fo, double rtol, int max_newton,
                  double floor, dg_step_stats& loc, double& worst, double& r0_out, double& r_out) {
    const size_t n = ctx->N;
    double r = unsteady();
    if (!std::isfinite(r)) fail(ctx, DG_ENONFINITE, "non-finite unsteady residual");
    const double r0 = r;
    bool conv = false;
    for (int k = 0; k < max_newton; ++k) {
        if (r <= rtol * r0 || r <= floor) {
            conv = true;
            break;
        }
        CK(launch_axpby(n, -1.0, ctx->Ru.p, 0.0, nullptr, ctx->tmp3.p, ctx->s));   // b = -R_u
        // fgmres uses tmp2/tmp3 internally: keep b in Ru (negated in place)
        CK(launch_copy(n, ctx->tmp3.p, ctx->Ru.p, ctx->s));
        fgmres_stats fs{};
        fgmres_impl(ctx, W, ctx->RW.p, ctx->Ru.p, ctx->xN.p, fo, &fs);
        loc.linear_iters += fs.iters;
        if (fs.rel_res_true > worst) worst = fs.rel_res_true;
        CK(launch_axpby(n, 1.0, ctx->xN.p, 1.0, W, W, ctx->s));
        loc.newton++;
        r = unsteady();
        if (!std::isfinite(r)) fail(ctx, DG_ENONFINITE, "non-finite unsteady residual");
    }
    if (!conv && (r <= rtol * r0 || r <= floor)) conv = true;
    r0_out = r0;
    r_out = r;
    return conv;
}

// 1e-14 a ||M Wn||: the rounding floor of a step's Newton residual (the size
// of the unsteady term a M W at rounding precision).
double newton_floor(dg_ctx* ctx, const double* Wn, double a) {
    CK(launch_mass(ctx->a, Wn, ctx->tmp1.p, 1.0, 0, ctx->s));
    dot(ctx, ctx->tmp1.p, ctx->tmp1.p, ctx->N, sc(ctx, S_N_M2));
    return 1e-14 * a * std::sqrt(read_scalar(ctx, sc(ctx, S_N_M2)));
}

void bdf2_impl(dg_ctx* ctx, const double* Wn, const double* Wnm1, double dt, const pmg_opts* po,
               const fgmres_opts* fo, double rtol, int max_newton, double* Wnp1, dg_step_stats* st) {
    if (!(dt > 0.0) || !(rtol > 0.0) || max_newton < 1) fail(ctx, DG_EINVAL, "bad dt / newton_rtol / max_newton");
    const size_t n = ctx->N;
    const double a = 1.5 / dt;
    if (!Wnm1) Wnm1 = Wn;
    dg_step_stats loc{};
    ctx->RW.ensure(n);
    ctx->Ru.ensure(n);
    ctx->xN.ensure(n);
    double* W = Wnp1;
    CK(launch_copy(n, Wn, W, ctx->s));
    CK(hipStreamSynchronize(ctx->s));
    auto t0 = std::chrono::steady_clock::now();
    pmg_setup_impl(ctx, Wn, a, po);
    CK(hipStreamSynchronize(ctx->s));
    auto t1 = std::chrono::steady_clock::now();
    const double floor = newton_floor(ctx, Wn, a);
    auto unsteady = [&]() -> double {
        timed(ctx, DG_K_RESIDUAL, 16.0 * (double)ctx->N, 0.0, [&] { return launch_residual(ctx->a, W, ctx->RW.p, ctx->s); });
        // t = 3 W - 4 Wn + Wnm1 ; Ru = M t / (2 dt) + RW
        CK(launch_axpby(n, 3.0, W, -4.0, Wn, ctx->tmp1.p, ctx->s));
        CK(launch_axpby(n, 1.0, Wnm1, 1.0, ctx->tmp1.p, ctx->tmp1.p, ctx->s));
        CK(launch_copy(n, ctx->RW.p, ctx->Ru.p, ctx->s));
        CK(launch_mass(ctx->a, ctx->tmp1.p, ctx->Ru.p, 0.5 / dt, 1, ctx->s));
        dot(ctx, ctx->Ru.p, ctx->Ru.p, n, sc(ctx, S_N_R2));
        return std::sqrt(read_scalar(ctx, sc(ctx, S_N_R2)));
    };
    double worst = 0.0, r0 = 0.0, r = 0.0;
    const bool conv = newton_solve(ctx, W, unsteady, fo, rtol, max_newton, floor, loc, worst, r0, r);
    CK(hipStreamSynchronize(ctx->s));
    auto t2 = std::chrono::steady_clock::now();
    loc.res0 = r0;
    loc.res_final = r;
    loc.max_rel_res_true = worst;
    loc.setup_seconds = std::chrono::duration<double>(t1 - t0).count();
    loc.solve_seconds = std::chrono::duration<double>(t2 - t1).count();
    if (st) *st = loc;
    if (!conv) fail(ctx, DG_ENOCONV, "Newton did not converge");
}

// ESDIRK3 (Sec. 4): the four-stage, third-order, explicit-first-stage,
// singly diagonally implicit Runge-Kutta scheme of Kennedy & Carpenter used
// by Bijl et al. (2002), published rational tableau; stiffly accurate.
constexpr double ESD_G = 1767732205903.0 / 4055673282236.0;
constexpr double ESD_A[4][4] = {
    {0.0, 0.0, 0.0, 0.0},
    {ESD_G, ESD_G, 0.0, 0.0},
    {2746238789719.0 / 10658868560708.0, -640167445237.0 / 6845629431997.0, ESD_G, 0.0},
    {1471266399579.0 / 7840856788654.0, -4482444167858.0 / 7529755066697.0, 11266239266428.0 / 11593286722821.0,
     ESD_G}};

// One ESDIRK3 step: W^1 = Wn; stages i = 2..4 solve
//   M (W - Wn) / (gamma dt) + sum_{j<i} (a_ij / gamma) R(W^j) + R(W) = 0
// by Newton from the previous stage (iteration matrix M/(gamma dt) + dR/dW,
// one pMG setup at Wn lagged over all stages); Wnp1 = W^4.
void esdirk3_impl(dg_ctx* ctx, const double* Wn, double dt, const pmg_opts* po, const fgmres_opts* fo, double rtol,
                  int max_newton, double* Wnp1, dg_step_stats* st) {
    if (!(dt > 0.0) || !(rtol > 0.0) || max_newton < 1) fail(ctx, DG_EINVAL, "bad dt / newton_rtol / max_newton");
    const size_t n = ctx->N;
    const double a = 1.0 / (ESD_G * dt);
    dg_step_stats loc{};
    ctx->RW.ensure(n);
    ctx->Ru.ensure(n);
    ctx->xN.ensure(n);
    ctx->Rst.ensure(3 * n);
    ctx->Est.ensure(n);
    double* W = Wnp1;
    CK(launch_copy(n, Wn, W, ctx->s));
    CK(hipStreamSynchronize(ctx->s));
    auto t0 = std::chrono::steady_clock::now();
    pmg_setup_impl(ctx, Wn, a, po);
    CK(hipStreamSynchronize(ctx->s));
    auto t1 = std::chrono::steady_clock::now();
    const double floor = newton_floor(ctx, Wn, a);
    CK(launch_copy(n, ctx->RW0.p, ctx->Rst.p, ctx->s));                 // R(W^1) = R(Wn), from the setup
    double worst = 0.0, r0 = 0.0, r = 0.0;
    bool conv = true;
    for (int i = 1; i < 4; ++i) {
        // E = sum_{j<i} (a_ij / gamma) R(W^j)
        CK(launch_axpby(n, ESD_A[i][0] / ESD_G, ctx->Rst.p, 0.0, nullptr, ctx->Est.p, ctx->s));
        for (int j = 1; j < i; ++j)
            CK(launch_axpby(n, ESD_A[i][j] / ESD_G, ctx->Rst.p + (size_t)j * n, 1.0, ctx->Est.p, ctx->Est.p, ctx->s));
        auto unsteady = [&]() -> double {
            timed(ctx, DG_K_RESIDUAL, 16.0 * (double)ctx->N, 0.0, [&] { return launch_residual(ctx->a, W, ctx->RW.p, ctx->s); });
            // Ru = a M (W - Wn) + E + RW
            CK(launch_axpby(n, 1.0, W, -1.0, Wn, ctx->tmp1.p, ctx->s));
            CK(launch_axpby(n, 1.0, ctx->RW.p, 1.0, ctx->Est.p, ctx->Ru.p, ctx->s));
            CK(launch_mass(ctx->a, ctx->tmp1.p, ctx->Ru.p, a, 1, ctx->s));
            dot(ctx, ctx->Ru.p, ctx->Ru.p, n, sc(ctx, S_N_R2));
            return std::sqrt(read_scalar(ctx, sc(ctx, S_N_R2)));
        };
        double rs0 = 0.0;
        conv = newton_solve(ctx, W, unsteady, fo, rtol, max_newton, floor, loc, worst, rs0, r) && conv;
        if (i == 1) r0 = rs0;
        if (i < 3) CK(launch_copy(n, ctx->RW.p, ctx->Rst.p + (size_t)i * n, ctx->s));
    }
    CK(hipStreamSynchronize(ctx->s));
    auto t2 = std::chrono::steady_clock::now();
    loc.res0 = r0;
    loc.res_final = r;
    loc.max_rel_res_true = worst;
    loc.setup_seconds = std::chrono::duration<double>(t1 - t0).count();
    loc.solve_seconds = std::chrono::duration<double>(t2 - t1).count();
    if (st) *st = loc;
    if (!conv) fail(ctx, DG_ENOCONV, "Newton did not converge in some stage");
}

template <class F>
dg_status guarded(dg_ctx* ctx, F&& f) {
    if (!ctx) return DG_EINVAL;
    try {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != ctx->device) (void)hipSetDevice(ctx->device);
        f();
        ctx->err.clear();
        return DG_OK;
    } catch (const DgError& e) {
        if (ctx->err.empty()) ctx->err = "error";
        return e.st;
    } catch (const std::bad_alloc&) {
        ctx->err = "host allocation failed";
        return DG_ENOMEM;
    } catch (...) {
        ctx->err = "unexpected exception";
        return DG_EINVAL;
    }
}

void need(dg_ctx* ctx, const void* p, const char* what) {
    if (!p) fail(ctx, DG_EINVAL, std::string("null pointer: ") + what);
}
void no_alias(dg_ctx* ctx, const void* out, const void* in, const char* what) {
    if (out && in && out == in) fail(ctx, DG_EINVAL, std::string("output aliases input: ") + what);
}

}  // namespace

// ============================================================================ C ABI

// ---- device memory of a context ------------------------------------------------------------
namespace {
template <class T>
double bytes_of(const DBuf<T>& b) { return (double)b.n * sizeof(T); }
double krylov_bytes(const Krylov& K) {
    return bytes_of(K.V) + bytes_of(K.Z) + bytes_of(K.H) + bytes_of(K.cs) + bytes_of(K.sn) + bytes_of(K.g) +
           bytes_of(K.y) + bytes_of(K.sc);
}
}  // namespace

extern "C" double dg_device_bytes(const dg_ctx* ctx) {
    if (!ctx) return 0.0;
    double b = bytes_of(ctx->vtx) + bytes_of(ctx->partial) + bytes_of(ctx->scal) + bytes_of(ctx->flag) +
               bytes_of(ctx->tmp1) + bytes_of(ctx->tmp2) + bytes_of(ctx->tmp3) + bytes_of(ctx->W0) +
               bytes_of(ctx->RW0) + bytes_of(ctx->blk) + bytes_of(ctx->otmp) + bytes_of(ctx->dtmp) +
               bytes_of(ctx->nbrtr) + bytes_of(ctx->RW) + bytes_of(ctx->Ru) + bytes_of(ctx->xN) +
               bytes_of(ctx->gin) + bytes_of(ctx->gout) + bytes_of(ctx->mb_op) + krylov_bytes(ctx->kc) +
               krylov_bytes(ctx->kf) + bytes_of(ctx->Rst) + bytes_of(ctx->Est);
    for (const Krylov& K : ctx->ks) b += krylov_bytes(K);
    for (const Level& L : ctx->lv)
        b += bytes_of(L.f64) + bytes_of(L.f32) + bytes_of(L.piv) + bytes_of(L.pos) + bytes_of(L.inv64) +
             bytes_of(L.inv32) + bytes_of(L.x) + bytes_of(L.b) + bytes_of(L.r) + bytes_of(L.t) + bytes_of(L.z) +
             bytes_of(L.op64) + bytes_of(L.op32) + bytes_of(L.op16) + bytes_of(L.fb) + bytes_of(L.fx) +
             bytes_of(L.bd) + bytes_of(L.bo) + bytes_of(L.bw) + bytes_of(L.bord) + bytes_of(L.bpos);
    return b;
}

// What a context of this mesh and degree allocates for one BDF2 step with
// these options (the allocations of dg_create, pmg_setup, fgmres_step and
// dg_bdf2_step, with graphs on): the admission size of the serving loop.
extern "C" double dg_footprint_bytes(const dg_mesh_desc* mesh, int p, const pmg_opts* po, const fgmres_opts* fo) {
    if (!mesh || !po || !fo || p < 1 || p > MAXP || po->n_levels < 1 || po->n_levels > 4) return -1.0;
    const double ne = (double)mesh->nx * mesh->ny * mesh->nz;
    const double nv = (p + 1.0) * (p + 1) * (p + 1), nb = 5 * nv, N = ne * nb;
    // Krylov workspace of restart m on n entries (basis V, directions Z, Hessenberg and rotations)
    auto krylov = [](double m, double n) { return (2 * m + 1) * n * 8 + ((m + 1) * m + 4 * m + 1 + 8) * 8; };
    double b = 24 * ne * 8 + (double)RED_BLOCKS * 256 * 8 + S_COUNT * 8 + 4 * 4 + 3 * N * 8;   // create
    b += 2 * N * 8 + ne * nb * fine_block_ld((int)nb) * 8 + (double)nbr_trace_size(p, (int)ne) * 8;  // W0, RW0, blocks, traces
    double tmp = 0.0;
    for (int l = 0; l < po->n_levels; ++l) {
        const int pl = po->p_level[l];
        const double nbl = 5.0 * (pl + 1) * (pl + 1) * (pl + 1), ndl = ne * nbl, sz = ne * nbl * nbl;
        const bool use32 = (l == 0) ? (po->prec_fine == DG_FP32) : (po->prec_coarse != DG_FP64);
        const bool assembled = l > 0 && (po->coarse_matrix_free == 0 ||
                                         (po->coarse_matrix_free == 2 && l == po->n_levels - 1));
        const bool fold = assembled && l == po->n_levels - 1 && nbl <= INV_POLICY_N && nbl <= FOLD_MAX_N &&
                          po->coarsest_plain == 0 && po->coarsest_prec == 0;
        b += 2 * ndl * 4 + 5 * ndl * 8;                                           // pivots, positions, vectors
        if (po->cycle == 1 && l > 0) b += 2 * ndl * 8;                           // full multigrid b_l, x_l
        if (po->coarsest_prec == 1 && l == po->n_levels - 1) b += 3 * sz * 8 + ne * 16;   // block ILU(0)
        if (po->smoother == 1 && l < po->n_levels - 1)                            // GMRES(BJ) smoother
            b += krylov(std::max(1, std::max(po->nu_pre, po->nu_post)), ndl);
        if (assembled) {
            tmp = std::max(tmp, 7 * sz * 8);
            b += (double)bsr_entries((int)ne, (int)nbl, fold ? 6 : 7) *
                 (po->prec_coarse == DG_FP64 ? 8 : (po->prec_coarse == DG_FP32 ? 4 : 2));
        }
        if (use32) b += (l == 0 ? ne * nbl * fine_block_ld((int)nbl) : sz) * 4;
        else if (l > 0) b += sz * 8;
        if (nbl <= INV_POLICY_N) b += sz * (use32 ? 4 : 8);
        if (l == po->n_levels - 1 && po->n_levels > 1)
            b += krylov(po->coarsest_iters, ndl);                                 // coarsest GMRES
    }
    b += tmp;
    if (po->prec_fine == DG_FP64) {        // level-0 factors took the block buffer: FP32 inverses need a workspace
        double ws = 0.0;
        for (int l = 1; l < po->n_levels; ++l) {
            const int pl = po->p_level[l];
            const double nbl = 5.0 * (pl + 1) * (pl + 1) * (pl + 1);
            const bool fold = l == po->n_levels - 1 && nbl <= FOLD_MAX_N && po->coarsest_plain == 0 &&
                              po->coarsest_prec == 0 && (po->coarse_matrix_free == 0 || po->coarse_matrix_free == 2);
            if (po->prec_coarse != DG_FP64 && nbl <= INV_POLICY_N && !fold) ws = std::max(ws, ne * nbl * nbl * 8);
        }
        b += ws;
    }
    b += krylov(fo->restart, N);                                                   // FGMRES
    b += 3 * N * 8 + 2 * N * 8;                                                    // Newton, graph staging
    return b;
}

extern "C" {

dg_status dg_create(const dg_mesh_desc* mesh, const dg_phys* phys, int p, void* hip_stream, dg_ctx** out) {
    if (!out) return DG_EINVAL;
    *out = nullptr;
    if (!mesh || !phys) return DG_EINVAL;
    if (p < 1 || p > MAXP) return DG_EINVAL;
    if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1) return DG_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (!(mesh->hi[d] > mesh->lo[d])) return DG_EINVAL;
    if (!(phys->gamma > 1.0) || phys->mu < 0.0 || (phys->mu > 0.0 && !(phys->Pr > 0.0)) || phys->eta < 0.0)
        return DG_EINVAL;
    const long long ne_ll = (long long)mesh->nx * mesh->ny * mesh->nz;
    if (ne_ll > (1ll << 30)) return DG_EINVAL;
    dg_ctx* ctx = new (std::nothrow) dg_ctx();
    if (!ctx) return DG_ENOMEM;
    dg_status st = DG_OK;
    try {
        CK(hipGetDevice(&ctx->device));
        {
            std::lock_guard<std::mutex> lk(g_tab_mu);
            if (!g_tab_built) {
                build_tables(g_tabs, g_perm);
                g_tab_built = true;
            }
            if (ctx->device < 0 || ctx->device >= 64) fail(ctx, DG_EINVAL, "device index out of range");
            if (!g_tab_uploaded[ctx->device]) {
                CK(upload_tables(g_tabs, g_perm));
                g_tab_uploaded[ctx->device] = true;
            }
            if (!g_scratch_ptr[ctx->device]) {
                void* ptr = nullptr;
                CK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
                g_scratch_ptr[ctx->device] = static_cast<double*>(ptr);
            }
        }
        ctx->s = (hipStream_t)hip_stream;
        ctx->p = p;
        ctx->nv = (p + 1) * (p + 1) * (p + 1);
        ctx->nb = 5 * ctx->nv;
        ctx->ne = (int)ne_ll;
        ctx->N = (size_t)ctx->ne * ctx->nb;
        MeshDev& m = ctx->a.m;
        m.nx = mesh->nx;
        m.ny = mesh->ny;
        m.nz = mesh->nz;
        m.ne = ctx->ne;
        for (int d = 0; d < 3; ++d) m.h[d] = (mesh->hi[d] - mesh->lo[d]) / (&mesh->nx)[d];
        m.vtx = nullptr;
        ctx->a.g = Gas{phys->gamma, phys->mu, phys->Pr, phys->eta};
        ctx->a.p = p;
        ctx->a.ns = phys->mu > 0.0;
        ctx->partial.ensure((size_t)RED_BLOCKS * 256);
        ctx->scal.ensure(S_COUNT);
        ctx->flag.ensure(4);
        ensure_scratch(ctx);
        std::vector<double> hv;
        const double* src = mesh->vtx;
        if (!src) {      // straight box vertices (used for the quadrature point coordinates only)
            hv.resize((size_t)ctx->ne * 24);
            for (int k = 0; k < m.nz; ++k)
                for (int j = 0; j < m.ny; ++j)
                    for (int i = 0; i < m.nx; ++i) {
                        const size_t e = (size_t)i + (size_t)m.nx * (j + (size_t)m.ny * k);
                        for (int v = 0; v < 8; ++v) {
                            const int c[3] = {i + (v & 1), j + ((v >> 1) & 1), k + ((v >> 2) & 1)};
                            for (int d = 0; d < 3; ++d) hv[e * 24 + v * 3 + d] = mesh->lo[d] + m.h[d] * c[d];
                        }
                    }
            src = hv.data();
        }
        ctx->vtx.ensure((size_t)ctx->ne * 24);
        CK(hipMemcpyAsync(ctx->vtx.p, src, (size_t)ctx->ne * 24 * sizeof(double), hipMemcpyHostToDevice, ctx->s));
        CK(hipStreamSynchronize(ctx->s));
        if (mesh->vtx) {
            m.vtx = ctx->vtx.p;
            CK(hipMemsetAsync(ctx->flag.p, 0, sizeof(int), ctx->s));
            CK(launch_check_jacobian(ctx->a, ctx->flag.p, ctx->s));
            int bad = 0;
            CK(hipMemcpyAsync(&bad, ctx->flag.p, sizeof(int), hipMemcpyDeviceToHost, ctx->s));
            CK(hipStreamSynchronize(ctx->s));
            if (bad) fail(ctx, DG_EINVAL, "non-positive Jacobian determinant at a quadrature point");
        }
    } catch (const DgError& e) {
        st = e.st;
    } catch (...) {
        st = DG_ENOMEM;
    }
    if (st != DG_OK) {
        dg_destroy(ctx);
        return st;
    }
    *out = ctx;
    return DG_OK;
}

dg_status dg_destroy(dg_ctx* ctx) {
    if (!ctx) return DG_EINVAL;
    if (ctx->s) (void)hipStreamSynchronize(ctx->s);
    else (void)hipDeviceSynchronize();
    for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
    drop_graph(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    ctx->gin.release();
    ctx->gout.release();
    ctx->vtx.release(); ctx->partial.release(); ctx->scal.release(); ctx->flag.release();
    ctx->tmp1.release(); ctx->tmp2.release(); ctx->tmp3.release();
    ctx->W0.release(); ctx->RW0.release(); ctx->blk.release(); ctx->otmp.release(); ctx->dtmp.release(); ctx->nbrtr.release();
    ctx->mb_op.release();
    for (auto& L : ctx->lv) L.release();
    ctx->kc.release(); ctx->kf.release();
    ctx->RW.release(); ctx->Ru.release(); ctx->xN.release(); ctx->Rst.release(); ctx->Est.release();
    for (auto& K : ctx->ks) K.release();
    delete ctx;
    return DG_OK;
}

size_t dg_ndof(const dg_ctx* ctx) { return ctx ? ctx->N : 0; }

const char* dg_last_error(const dg_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

dg_status dg_quad_points(dg_ctx* ctx, double* xyz) {
    return guarded(ctx, [&] {
        need(ctx, xyz, "xyz");
        DGArgs a = ctx->a;
        a.m.vtx = ctx->vtx.p;
        CK(launch_quad_points(a, xyz, ctx->s));
    });
}

dg_status dg_project(dg_ctx* ctx, const double* values, double* W) {
    return guarded(ctx, [&] {
        need(ctx, values, "values");
        need(ctx, W, "W");
        no_alias(ctx, W, values, "W/values");
        CK(launch_project(ctx->a, values, W, ctx->s));
    });
}

dg_status dg_residual(dg_ctx* ctx, const double* W, double* R) {
    return guarded(ctx, [&] {
        need(ctx, W, "W");
        need(ctx, R, "R");
        no_alias(ctx, R, W, "R/W");
        timed(ctx, DG_K_RESIDUAL, 16.0 * (double)ctx->N, 0.0, [&] { return launch_residual(ctx->a, W, R, ctx->s); });
    });
}

dg_status dg_jvp(dg_ctx* ctx, const double* W, const double* RW, const double* v, double shift, double* y) {
    return guarded(ctx, [&] {
        need(ctx, W, "W");
        need(ctx, RW, "RW");
        need(ctx, v, "v");
        need(ctx, y, "y");
        no_alias(ctx, y, W, "y/W");
        no_alias(ctx, y, v, "y/v");
        no_alias(ctx, y, RW, "y/RW");
        jvp_fd(ctx, W, RW, v, shift, y, nullptr);
    });
}

dg_status dg_jvp_exact(dg_ctx* ctx, const double* W, const double* v, double shift, double* y) {
    return guarded(ctx, [&] {
        need(ctx, W, "W");
        need(ctx, v, "v");
        need(ctx, y, "y");
        no_alias(ctx, y, W, "y/W");
        no_alias(ctx, y, v, "y/v");
        timed(ctx, DG_K_JVP_EXACT, 24.0 * (double)ctx->N, 0.0, [&] { return launch_jvp_exact(ctx->a, W, v, shift, y, ctx->s); });
    });
}

dg_status dg_mass(dg_ctx* ctx, const double* v, double* y) {
    return guarded(ctx, [&] {
        need(ctx, v, "v");
        need(ctx, y, "y");
        no_alias(ctx, y, v, "y/v");
        CK(launch_mass(ctx->a, v, y, 1.0, 0, ctx->s));
    });
}

dg_status dg_assemble_diag(dg_ctx* ctx, const double* W, double shift, double* blocks) {
    return guarded(ctx, [&] {
        need(ctx, W, "W");
        need(ctx, blocks, "blocks");
        ctx->nbrtr.ensure(nbr_trace_size(ctx->p, ctx->ne));
        CK(launch_diag_blocks(ctx->a, W, shift, blocks, ctx->nb, ctx->nbrtr.p, ctx->s));
    });
}

dg_status dg_assemble_diag_noalloc(dg_ctx* ctx, const double* W, double shift, double* blocks) {
    return guarded(ctx, [&] {
        need(ctx, W, "W");
        need(ctx, blocks, "blocks");
        if (nbr_trace_size(ctx->p, ctx->ne) > NOALLOC_SCRATCH_DOUBLES)
            fail(ctx, DG_EINVAL, "mesh too large for dg_assemble_diag_noalloc: its neighbour traces need " +
                                     std::to_string(nbr_trace_size(ctx->p, ctx->ne) * sizeof(double)) +
                                     " bytes, the fixed scratch holds " +
                                     std::to_string(NOALLOC_SCRATCH_DOUBLES * sizeof(double)));
        double* ws = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_tab_mu);
            ws = g_scratch_ptr[ctx->device];
        }
        if (!ws) fail(ctx, DG_ESTATE, "scratch address not resolved on this device");
        CK(launch_diag_blocks(ctx->a, W, shift, blocks, ctx->nb, ws, ctx->s));
    });
}

dg_status dg_assemble_coarse(dg_ctx* ctx, const double* W, int pc, double* off) {
    return guarded(ctx, [&] {
        need(ctx, W, "W");
        need(ctx, off, "off");
        if (pc < 1 || pc > ctx->p) fail(ctx, DG_EINVAL, "pc must satisfy 1 <= pc <= p");
        CK(launch_offdiag_blocks(ctx->a, W, pc, off, ctx->s));
    });
}

dg_status dg_assemble_operator(dg_ctx* ctx, const double* W, double shift) {
    return guarded(ctx, [&] {
        need(ctx, W, "W");
        ctx->mb_ready = false;
        const size_t sz = (size_t)ctx->ne * ctx->nb * ctx->nb;
        ctx->dtmp.ensure(sz);
        ctx->otmp.ensure(6 * sz);
        ctx->nbrtr.ensure(nbr_trace_size(ctx->p, ctx->ne));
        CK(launch_diag_blocks(ctx->a, W, shift, ctx->dtmp.p, ctx->nb, ctx->nbrtr.p, ctx->s));
        CK(launch_offdiag_blocks(ctx->a, W, ctx->p, ctx->otmp.p, ctx->s));
        ctx->mb_op.ensure(bsr_entries(ctx->ne, ctx->nb, 7));
        CK(launch_bsr_pack<double>(ctx->dtmp.p, ctx->otmp.p, ctx->mb_op.p, ctx->ne, ctx->nb, 7, ctx->s));
        // the unpacked blocks are dead once packed: free them (after the pack
        // has run) so the context holds only the packed operator
        CK(hipStreamSynchronize(ctx->s));
        ctx->dtmp.release();
        ctx->otmp.release();
        ctx->mb_ready = true;
    });
}

dg_status dg_jvp_assembled(dg_ctx* ctx, const double* v, double* y) {
    return guarded(ctx, [&] {
        if (!ctx->mb_ready) fail(ctx, DG_ESTATE, "dg_assemble_operator has not been called");
        need(ctx, v, "v");
        need(ctx, y, "y");
        if (v == y) fail(ctx, DG_EINVAL, "y must not alias v");
        CK(launch_bsr7<double>(ctx->a, ctx->mb_op.p, v, y, ctx->nb, ctx->s));
    });
}

dg_status dg_batched_lu(void* hip_stream, double* A, int* piv, int nblk, int n) {
    if (!A || !piv || nblk < 0 || n < 1 || n > 625) return DG_EINVAL;
    if (launch_lu_blocked<double>(A, piv, nullptr, nblk, n, n, (hipStream_t)hip_stream) != hipSuccess) return DG_EHIP;
    return DG_OK;
}

dg_status dg_batched_lu_solve(void* hip_stream, const double* LU, const int* piv, const double* b, double* x,
                              int nblk, int n) {
    if (!LU || !piv || !b || !x || b == x || nblk < 0 || n < 1 || n > 4096) return DG_EINVAL;
    if (launch_lu_solve<double>(LU, piv, b, x, nblk, n, (hipStream_t)hip_stream) != hipSuccess) return DG_EHIP;
    return DG_OK;
}

dg_status pmg_setup(dg_ctx* ctx, const double* W, double shift, const pmg_opts* opts) {
    return guarded(ctx, [&] {
        need(ctx, W, "W");
        pmg_setup_impl(ctx, W, shift, opts);
    });
}

dg_status pmg_apply(dg_ctx* ctx, const double* r, double* z) {
    return guarded(ctx, [&] {
        need(ctx, r, "r");
        need(ctx, z, "z");
        no_alias(ctx, z, r, "z/r");
        pmg_apply_impl(ctx, r, z);
    });
}

dg_status fgmres_step(dg_ctx* ctx, const double* W, const double* RW, const double* b, double* x,
                      const fgmres_opts* opts, fgmres_stats* stats) {
    return guarded(ctx, [&] {
        need(ctx, W, "W");
        need(ctx, b, "b");
        need(ctx, x, "x");
        if (!opts || !opts->jvp_exact) need(ctx, RW, "RW");
        no_alias(ctx, x, b, "x/b");
        no_alias(ctx, x, W, "x/W");
        fgmres_impl(ctx, W, RW, b, x, opts, stats);
    });
}

dg_status dg_bdf2_step(dg_ctx* ctx, const double* Wn, const double* Wnm1, double dt, const pmg_opts* popts,
                       const fgmres_opts* fopts, double newton_rtol, int max_newton, double* Wnp1,
                       dg_step_stats* stats) {
    return guarded(ctx, [&] {
        need(ctx, Wn, "Wn");
        need(ctx, Wnp1, "Wnp1");
        no_alias(ctx, Wnp1, Wn, "Wnp1/Wn");
        no_alias(ctx, Wnp1, Wnm1, "Wnp1/Wnm1");
        bdf2_impl(ctx, Wn, Wnm1, dt, popts, fopts, newton_rtol, max_newton, Wnp1, stats);
    });
}

dg_status dg_esdirk3_step(dg_ctx* ctx, const double* Wn, double dt, const pmg_opts* popts, const fgmres_opts* fopts,
                          double newton_rtol, int max_newton, double* Wnp1, dg_step_stats* stats) {
    return guarded(ctx, [&] {
        need(ctx, Wn, "Wn");
        need(ctx, Wnp1, "Wnp1");
        no_alias(ctx, Wnp1, Wn, "Wnp1/Wn");
        esdirk3_impl(ctx, Wn, dt, popts, fopts, newton_rtol, max_newton, Wnp1, stats);
    });
}

dg_status dg_use_graphs(dg_ctx* ctx, int enable) {
    return guarded(ctx, [&] {
        ctx->use_graphs = enable != 0;
        if (!ctx->use_graphs) drop_graph(ctx);
    });
}

dg_status dg_timing(dg_ctx* ctx, int enable) {
    return guarded(ctx, [&] {
        ctx->timing = enable != 0;
        ctx->ev_used = 0;
    });
}

dg_status dg_timing_read(dg_ctx* ctx, double* ms, int* counts, double* bytes, double* flops) {
    return guarded(ctx, [&] {
        need(ctx, ms, "ms");
        need(ctx, counts, "counts");
        need(ctx, bytes, "bytes");
        need(ctx, flops, "flops");
        CK(hipStreamSynchronize(ctx->s));
        for (int k = 0; k < DG_K_COUNT; ++k) {
            ms[k] = 0.0;
            counts[k] = 0;
            bytes[k] = 0.0;
            flops[k] = 0.0;
        }
        for (size_t i = 0; i < ctx->ev_used; ++i) {
            float t = 0.0f;
            CK(hipEventElapsedTime(&t, ctx->ev[2 * i], ctx->ev[2 * i + 1]));
            ms[ctx->ev_kind[i]] += t;
            counts[ctx->ev_kind[i]] += 1;
            bytes[ctx->ev_kind[i]] += ctx->ev_bytes[i];
            flops[ctx->ev_kind[i]] += ctx->ev_flops[i];
        }
        ctx->ev_used = 0;
    });
}

}  // extern "C"
