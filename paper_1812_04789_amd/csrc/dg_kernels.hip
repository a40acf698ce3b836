// Fused DG kernels for gfx950: residual R(W) (Sec. 3.1, Eq. dg_ns with the
// Roe flux and BR2, Eqs. visc_flux and re), the matrix-free product of
// Sec. 5.1 (Eq. DG-mf), its exact forward-mode counterpart, and the columns
// of the element diagonal blocks of K = a M + dR/dW (Sec. 6.3).
//
// Design (one kernel per call, no intermediate HBM traffic):
//  * one element per (p+1)^3 work-items; every work-item owns one volume
//    Gauss point; elements are packed so a workgroup is one or two wavefronts;
//  * sum-factorised interpolation modal -> Gauss values (three 1D sweeps
//    through LDS), reference gradients by the collocation derivative;
//  * each element evaluates all six of its faces: its own traces from its
//    Gauss values (Lagrange weights of the end points), the neighbour's
//    traces from the neighbour's modal coefficients (collapse along the
//    normal, two tangential sweeps), so no face data ever goes to HBM and
//    the result is deterministic;
//  * face integrands are spread onto the Gauss lines normal to the face with
//    the same end-point Lagrange weights, so volume and face terms are tested
//    by a single D^T + V^T sweep pass;
//  * the BR2 lifting uses its closed form at the face points (exact for the
//    Gauss-rule mass matrix): delta = lambda G,
//    lambda_q = J_F,q sum_c l(z_c)^2 w_c / detJ(line through q, c);
//  * curved (Q1) elements recompute the metric from the 8 vertices.
#include "internal.h"
#include "reduce.h"
#include "physics.h"

namespace dg {

__constant__ Tab c_tab[MAXP + 1];
__constant__ short c_perm[PERM_TOTAL];

hipError_t upload_tables(const Tab* tabs, const short* perm) {
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_tab), tabs, sizeof(Tab) * (MAXP + 1));
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(c_perm), perm, sizeof(short) * PERM_TOTAL);
}

// ---- geometry -----------------------------------------------------------------
// Jacobian J[d][k] = dx_d/dxi_k of the trilinear map at reference point x.
__device__ __forceinline__ void q1_jac(const double* X, double x0, double x1, double x2, double J[3][3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) J[d][0] = J[d][1] = J[d][2] = 0.0;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const double s0 = (v & 1) ? 1.0 : -1.0, s1 = (v & 2) ? 1.0 : -1.0, s2 = (v & 4) ? 1.0 : -1.0;
        const double f0 = 0.5 * (1.0 + s0 * x0), f1 = 0.5 * (1.0 + s1 * x1), f2 = 0.5 * (1.0 + s2 * x2);
        const double d0 = 0.5 * s0 * f1 * f2, d1 = 0.5 * s1 * f0 * f2, d2 = 0.5 * s2 * f0 * f1;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double xv = X[3 * v + d];
            J[d][0] = fma(d0, xv, J[d][0]);
            J[d][1] = fma(d1, xv, J[d][1]);
            J[d][2] = fma(d2, xv, J[d][2]);
        }
    }
}

__device__ __forceinline__ double q1_det(const double J[3][3]) {
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// Ji[k][d] = dxi_k/dx_d; returns det J.
__device__ __forceinline__ double q1_inv(const double J[3][3], double Ji[3][3]) {
    const double det = q1_det(J);
    const double id = 1.0 / det;
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    return det;
}

__device__ __forceinline__ int nbr_of(const MeshDev& m, int e, int f) {
    int i = e % m.nx, j = (e / m.nx) % m.ny, k = e / (m.nx * m.ny);
    const int d = f >> 1, step = (f & 1) ? 1 : -1;
    if (d == 0) i = (i + step + m.nx) % m.nx;
    else if (d == 1) j = (j + step + m.ny) % m.ny;
    else k = (k + step + m.nz) % m.nz;
    return i + m.nx * (j + m.ny * k);
}

// ---- sizes and LDS layout per element slot ------------------------------------------
template <int P>
struct Sz {
    static constexpr int N = P + 1, NQ = N * N * N, NF = N * N, NB = 5 * NQ;
};
// Face phase of the fused kernel (both process the faces in rounds of NQ face
// points, N whole faces per round, and spread each round onto the Gauss lines):
//  UP = true:  own traces from stored Gauss-point gradients (45 NQ of LDS:
//              23 KB at degree 3, seven elements per CU); degree <= 3, real
//              arithmetic.
//  UP = false: each round collapses its own faces; own trace gradients from
//              the face trace (collocation derivative on the face): 40 NQ of
//              LDS, for degree 4 and the dual-number product.
template <int P, int MODE>
struct FaceMode { static constexpr bool UP = (MODE < M_TANGENT) && (P <= 3); };
template <int P, bool UP>
struct Lay;
template <int P>
struct Lay<P, true> {
    static constexpr int NQ = Sz<P>::NQ;
    // [0, 20 NQ): interpolation buffers (15 NQ) | one round: neighbour collapse
    //             (10 NQ) + first tangential sweep (15 NQ, variables 0-2 after
    //             the collapse, 3-4 over the consumed collapse of 0-2), then
    //             face integrands (20 NQ) | test A, B (20 NQ).  40 NQ in all:
    //             eight elements per CU at degree 3.
    static constexpr int OFF_U = 20 * NQ;                                  // Gauss values (5 NQ)
    static constexpr int OFF_G = OFF_U + 5 * NQ;                           // Gauss ref. gradients (15 NQ)
    static constexpr int OFF_E = OFF_U;                                    // test-back (15 NQ, over the dead values and gradients)
    static constexpr int TOT = OFF_U + 20 * NQ;
};
template <int P>
struct Lay<P, false> {
    static constexpr int NQ = Sz<P>::NQ;
    // [0, 20 NQ): interpolation buffers (15 NQ) | one round: neighbour collapse (10 NQ)
    //             + own traces (5 NQ), then face integrands (20 NQ) | test A, B (20 NQ)
    static constexpr int OFF_U = 20 * NQ;                                  // Gauss values (5 NQ)
    static constexpr int OFF_G = OFF_U;                                    // (no stored gradients)
    static constexpr int OFF_E = OFF_U + 5 * NQ;                           // tangential sweep | test-back (15 NQ)
    static constexpr int TOT = OFF_E + 15 * NQ;
};
template <int P, int MODE>
using LayOf = Lay<P, FaceMode<P, MODE>::UP>;

template <int P, bool DUAL>
struct Launch;
template <> struct Launch<1, false> { static constexpr int EPB = 8; };
template <> struct Launch<1, true> { static constexpr int EPB = 4; };
template <> struct Launch<2, false> { static constexpr int EPB = 2; };
template <> struct Launch<2, true> { static constexpr int EPB = 2; };
template <> struct Launch<3, false> { static constexpr int EPB = 1; };
template <> struct Launch<3, true> { static constexpr int EPB = 1; };
template <> struct Launch<4, false> { static constexpr int EPB = 1; };
template <> struct Launch<4, true> { static constexpr int EPB = 1; };

// tensor index helpers: q = (i0 N + i1) N + i2, i0 <-> xi_1
template <int N>
__device__ __forceinline__ int tix(int i0, int i1, int i2) {
    return (i0 * N + i1) * N + i2;
}
template <int N>
__device__ __forceinline__ int tix_dir(int d, int a, const int ii[3]) {
    int j[3] = {ii[0], ii[1], ii[2]};
    j[d] = a;
    return (j[0] * N + j[1]) * N + j[2];
}

// dst[c][q] = sum_j M(i_dir(q), j) src[c][q with i_dir -> j] for c < NC;
// M(i,j) = Tb[i][j] (TR = false) or Tb[j][i] (TR = true).
template <int N, int NC, bool TR, class T>
__device__ __forceinline__ void sweep(const double (*Tb)[MAXN], const T* src, T* dst, int dir, const int ii[3],
                                      int q) {
    constexpr int NQ = N * N * N;
    const int i = ii[dir];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        T acc = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const double mij = TR ? Tb[j][i] : Tb[i][j];
            acc = fma(mij, src[c * NQ + tix_dir<N>(dir, j, ii)], acc);
        }
        dst[c * NQ + q] = acc;
    }
}

// Load one modal coefficient as the kernel's scalar type: W (residual),
// W + h v (FD product) or the dual number (W, v) (exact product).
template <int MODE, class T>
__device__ __forceinline__ T load_state(const double* W, const double* v, double h, size_t off) {
    const double w = W[off];
    if constexpr (MODE == M_RES) {
        return w;
    } else if constexpr (MODE == M_JVP_FD) {
        return w + h * v[off];
    } else {
        return mk<T>(w, v[off]);
    }
}

// Face integrand at one face point, seen from the + element: the Roe flux and
// the BR2 viscous flux (Eq. visc_flux with the closed-form lifting
// delta = lambda G) times the face weight, and the adjoint-consistency
// (symmetry) term mapped to reference gradients.  out[0..4] multiplies
// phi_i, out[5 + 3a + k] multiplies dphi_i/dxi_k (both summed onto R_+).
//   up, gxp: + trace and its reference gradient; um, gxm: - trace;
//   nrm: unit normal out of +;  Jip/Jim: dxi/dx on each side;
//   lam_p/lam_m: BR2 lifting factors;  sc = w_face * J_F.
// BR2 penalty and symmetry terms of a face point, added to the normal flux Fn
// (Roe + averaged viscous) to give the integrand fo[0..19] (see face_integrand):
// G+- = -1/2 F_v(u+-, [u] (x) n+), penalty eta/2 (lam+ G+ + lam- G-).n, symmetry
// -(dxi/dx) G+ on the reference gradients of the + test functions.
template <class T>
__device__ __forceinline__ void face_penalty_symmetry(const T up[5], const T um[5], const double nrm[3],
                                                      const double Jip[3][3], double lam_p, double lam_m, double sc,
                                                      const Gas& gas, const T Fn[5], T* fo) {
    T jmp[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) jmp[a] = up[a] - um[a];
    const double cp = 0.5 * gas.eta * lam_p, cm = 0.5 * gas.eta * lam_m;
    T Fs[5];
    {
        T Gm[5][3];
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int j = 0; j < 3; ++j) Gm[a][j] = 0.0;
        flux_v_rank1_acc(um, jmp, nrm, gas, -0.5, Gm);
#pragma unroll
        for (int a = 0; a < 5; ++a) Fs[a] = Fn[a] + cm * (Gm[a][0] * nrm[0] + Gm[a][1] * nrm[1] + Gm[a][2] * nrm[2]);
    }
    T Gp[5][3];
#pragma unroll
    for (int a = 0; a < 5; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j) Gp[a][j] = 0.0;
    flux_v_rank1_acc(up, jmp, nrm, gas, -0.5, Gp);
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        fo[a] = sc * (Fs[a] + cp * (Gp[a][0] * nrm[0] + Gp[a][1] * nrm[1] + Gp[a][2] * nrm[2]));
#pragma unroll
        for (int k = 0; k < 3; ++k)
            fo[5 + a * 3 + k] = -sc * (Jip[k][0] * Gp[a][0] + Jip[k][1] * Gp[a][1] + Jip[k][2] * Gp[a][2]);
    }
}

// FIX (dual-number block columns only): FIX_NBR, the neighbour's state does
// not move; FIX_OWN, this element's state does not move.  The fixed side's
// half of the averaged viscous flux then has no tangent and is skipped, so
// only the tangent parts of fo are valid.
constexpr int FIX_NONE = 0, FIX_NBR = 1, FIX_OWN = 2;
template <class T, bool NS, int FIX = FIX_NONE>
__device__ __forceinline__ void face_integrand(const T up[5], const T gxp[5][3], const T um[5], const T gxm[5][3],
                                               const double nrm[3], const double Jip[3][3], const double Jim[3][3],
                                               double lam_p, double lam_m, double sc, const Gas& gas, T* fo) {
    T Fn[5];
    roe_flux(up, um, nrm, gas.gamma, Fn);
    if constexpr (NS) {
        // averaged viscous flux, normal component only: 1/2 (F_v(u+, g+) + F_v(u-, g-)).n
        if constexpr (FIX != FIX_OWN) {
            T g[5][3];
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    g[a][j] = Jip[0][j] * gxp[a][0] + Jip[1][j] * gxp[a][1] + Jip[2][j] * gxp[a][2];
            flux_v_n_acc(up, g, gas, 0.5, nrm, Fn);
        }
        if constexpr (FIX != FIX_NBR) {
            T g[5][3];
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    g[a][j] = Jim[0][j] * gxm[a][0] + Jim[1][j] * gxm[a][1] + Jim[2][j] * gxm[a][2];
            flux_v_n_acc(um, g, gas, 0.5, nrm, Fn);
        }
        face_penalty_symmetry<T>(up, um, nrm, Jip, lam_p, lam_m, sc, gas, Fn, fo);
    } else {
#pragma unroll
        for (int a = 0; a < 5; ++a) fo[a] = sc * Fn[a];
        // no viscous flux: no terms on the reference gradients of the test functions
#pragma unroll
        for (int k = 5; k < 20; ++k) fo[k] = T(0.0);
    }
}

// One element of the DG operator (residual, FD product or exact product),
// evaluated by the NQ threads of one element slot, thread q at Gauss point q.
// S: the slot's LDS scratch (Sz<P>::TOT scalars), sdet: NQ doubles, svtx: 24
// doubles.  Every thread of the workgroup calls this together (barriers);
// threads of an inactive slot (no element) pass active = false.
template <int P, bool NS, bool CURVED, int MODE,
          class T = typename std::conditional<(MODE >= M_TANGENT), Dual, double>::type>
__device__ __forceinline__ void dg_element(const MeshDev& m, const Gas& gas, const double* __restrict__ W,
                                           const double* __restrict__ V, const double* __restrict__ RW,
                                           const double* __restrict__ hbuf, double shift, double* __restrict__ out,
                                           T* S, double* sdet, double* svtx, int e, bool active, int q) {
    using S_ = Sz<P>;
    using L_ = LayOf<P, MODE>;
    constexpr bool UP = FaceMode<P, MODE>::UP;
    constexpr int N = S_::N, NQ = S_::NQ, NF = S_::NF, NB = S_::NB;
    constexpr bool DUAL = (MODE >= M_TANGENT);
    const Tab& tb = c_tab[P];
    const short* perm = c_perm + perm_offset(P);
    double h = 0.0;
    if constexpr (MODE == M_JVP_FD) {
        h = hbuf[0];
        if (h == 0.0) {       // v == 0: y = shift M v = 0 (uniform across the grid)
            if (active)
                for (int a = 0; a < 5; ++a) out[(size_t)e * NB + a * NQ + perm[q]] = 0.0;
            return;
        }
    }
    const int ii[3] = {q / NF, (q / N) % N, q % N};

    // ---- load own modal coefficients (tensor order) --------------------------------
    if (active) {
        const size_t base = (size_t)e * NB;
        const int pm = perm[q];
#pragma unroll
        for (int a = 0; a < 5; ++a)
            S[a * NQ + q] = load_state<MODE, T>(W, V, h, base + a * NQ + pm);
        if constexpr (CURVED)
            for (int k = q; k < 24; k += NQ) svtx[k] = m.vtx[(size_t)e * 24 + k];
    }
    __syncthreads();
    // ---- interpolation to the Gauss points ---------------------------------------
    T* X1 = S + 5 * NQ;
    T* X2 = S + 10 * NQ;
    T* su = S + L_::OFF_U;
    T* sg = S + L_::OFF_G;        // UP only
    if (active) sweep<N, 5, false>(tb.V, S, X1, 0, ii, q);
    __syncthreads();
    if (active) sweep<N, 5, false>(tb.V, X1, X2, 1, ii, q);
    __syncthreads();
    if (active) sweep<N, 5, false>(tb.V, X2, su, 2, ii, q);
    __syncthreads();

    // ---- volume: gradients, metric, flux ------------------------------------------------
    T A[5][3], B[5];
    double detJ = 1.0, Ji[3][3];
    const double hx = m.h[0], hy = m.h[1], hz = m.h[2];
    if (active) {
        T u[5], gx[5][3];
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            u[a] = su[a * NQ + q];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                T acc = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) acc = fma(tb.D[ii[k]][j], su[a * NQ + tix_dir<N>(k, j, ii)], acc);
                gx[a][k] = acc;
                if constexpr (UP) sg[(a * 3 + k) * NQ + q] = acc;
            }
        }
        if constexpr (CURVED) {
            double J[3][3];
            q1_jac(svtx, tb.z[ii[0]], tb.z[ii[1]], tb.z[ii[2]], J);
            detJ = q1_inv(J, Ji);
            sdet[q] = detJ;
        } else {
            detJ = 0.125 * hx * hy * hz;
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int d = 0; d < 3; ++d) Ji[k][d] = 0.0;
            Ji[0][0] = 2.0 / hx;
            Ji[1][1] = 2.0 / hy;
            Ji[2][2] = 2.0 / hz;
        }
        const double wq = tb.w[ii[0]] * tb.w[ii[1]] * tb.w[ii[2]];
        T F[5][3];
        flux_c(u, gas.gamma - 1.0, F);
        if constexpr (NS) {
            T g[5][3];
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    g[a][j] = Ji[0][j] * gx[a][0] + Ji[1][j] * gx[a][1] + Ji[2][j] * gx[a][2];
            flux_v_acc(u, g, gas, 1.0, F);
        }
        const double c = -wq * detJ;
#pragma unroll
        for (int a = 0; a < 5; ++a) {
#pragma unroll
            for (int k = 0; k < 3; ++k) A[a][k] = c * (Ji[k][0] * F[a][0] + Ji[k][1] * F[a][1] + Ji[k][2] * F[a][2]);
            if constexpr (DUAL) B[a] = Dual(0.0, shift * wq * detJ * tan_(u[a]));
            else B[a] = 0.0;
        }
    }
    __syncthreads();

    if constexpr (UP) {
        // ---- faces --------------------------------------------------------------------
        // Rounds of NQ face points (N whole faces each, NQ = N NF); thread q takes
        // slot q = (face fl of the round, face point fq) in every stage:
        //   1  neighbour: collapse of its modal data along the normal (value and
        //      normal derivative at the shared face) -> sC;
        //   2  neighbour: first tangential sweep -> sE, variables 0-2 into
        //      [10 NQ, 19 NQ), then (after a barrier) 3-4 over the collapse of
        //      0-2 in [0, 6 NQ);
        //   3  both traces with reference gradients (own ones from the stored
        //      Gauss values and gradients), then the face integrand (registers);
        //   4  after a barrier, integrands -> sF over sC and sE, spread onto
        //      the Gauss lines.
        // Staging is component-major (sC[c * NQ + slot], ...): consecutive
        // threads touch consecutive doubles, and only one round's neighbour
        // data is held at a time.
        T* sC = S;                    // 10 NQ
        T* sF = S;                    // 20 NQ
        auto sE = [&](int a) -> T* { return (a < 3) ? S + (10 + 3 * a) * NQ : S + 3 * (a - 3) * NQ; };
#pragma unroll 1
        for (int r = 0; r * NQ < 6 * NF; ++r) {
            const int fp = r * NQ + q;
            const bool on = active && fp < 6 * NF;
            const int fl = q / NF, fq = q % NF;
            const int f = on ? fp / NF : 0;
            const int d = f >> 1, s = f & 1;
            const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
            const int qt1 = fq / N, qt2 = fq % N;
            const int sd = (d == 0) ? NF : ((d == 1) ? N : 1);
            const int st1 = (d == 0) ? N : NF, st2 = (d == 2) ? N : 1;
            const int tl = qt1 * st1 + qt2 * st2;
            if (on) {
                const int nb = nbr_of(m, e, f);
                const size_t nbase = (size_t)nb * NB;
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    T c0 = 0.0, c1 = 0.0;
#pragma unroll
                    for (int k = 0; k < N; ++k) {
                        const int pm = perm[tl + k * sd];
                        const T val = load_state<MODE, T>(W, V, h, nbase + a * NQ + pm);
                        c0 = fma(tb.Le[1 - s][k], val, c0);
                        c1 = fma(tb.Lde[1 - s][k], val, c1);
                    }
                    sC[(a * 2 + 0) * NQ + q] = c0;
                    sC[(a * 2 + 1) * NQ + q] = c1;
                }
            }
            __syncthreads();
            auto sweep1 = [&](int a) {
                T e0 = 0.0, e0d = 0.0, e1 = 0.0;
#pragma unroll
                for (int b2 = 0; b2 < N; ++b2) {
                    const int src = fl * NF + b2 * N + qt2;
                    const T cv0 = sC[(a * 2 + 0) * NQ + src];
                    e0 = fma(tb.V[qt1][b2], cv0, e0);
                    e0d = fma(tb.Vd[qt1][b2], cv0, e0d);
                    e1 = fma(tb.V[qt1][b2], sC[(a * 2 + 1) * NQ + src], e1);
                }
                T* se = sE(a);
                se[0 * NQ + q] = e0;
                se[1 * NQ + q] = e0d;
                se[2 * NQ + q] = e1;
            };
            if (on) {
#pragma unroll
                for (int a = 0; a < 3; ++a) sweep1(a);
            }
            __syncthreads();
            if (on) {
#pragma unroll
                for (int a = 3; a < 5; ++a) sweep1(a);
            }
            __syncthreads();
            T fo[20];
            if (on) {
                T um[5], gxm[5][3], up[5], gxp[5][3];
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    T v0 = 0.0, vt1 = 0.0, vt2 = 0.0, vd = 0.0;
                    const T* se = sE(a);
#pragma unroll
                    for (int c = 0; c < N; ++c) {
                        const int src = fl * NF + qt1 * N + c;
                        const T ev0 = se[0 * NQ + src];
                        v0 = fma(tb.V[qt2][c], ev0, v0);
                        vt1 = fma(tb.V[qt2][c], se[1 * NQ + src], vt1);
                        vt2 = fma(tb.Vd[qt2][c], ev0, vt2);
                        vd = fma(tb.V[qt2][c], se[2 * NQ + src], vd);
                    }
                    um[a] = v0;
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) gxm[a][kk] = (kk == d) ? vd : ((kk == t1) ? vt1 : vt2);
                }
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    T v0 = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
                    for (int k = 0; k < N; ++k) {
                        const int t = tl + k * sd;
                        const double l = tb.lag[s][k];
                        v0 = fma(l, su[a * NQ + t], v0);
                        g0 = fma(l, sg[(a * 3 + 0) * NQ + t], g0);
                        g1 = fma(l, sg[(a * 3 + 1) * NQ + t], g1);
                        g2 = fma(l, sg[(a * 3 + 2) * NQ + t], g2);
                    }
                    up[a] = v0;
                    gxp[a][0] = g0;
                    gxp[a][1] = g1;
                    gxp[a][2] = g2;
                }
                // geometry of the face point seen from both sides
                double nrm[3], JF, Jip[3][3], Jim[3][3], lam_p, lam_m;
                const double sgn = s ? 1.0 : -1.0;
                if constexpr (CURVED) {
                    const double z1 = tb.z[qt1], z2 = tb.z[qt2];
                    double xi[3];
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) xi[kk] = (kk == d) ? sgn : ((kk == t1) ? z1 : z2);
                    double J[3][3];
                    q1_jac(svtx, xi[0], xi[1], xi[2], J);
                    q1_inv(J, Jip);
                    // tangents dx/dxi_{d+1}, dx/dxi_{d+2} (cyclic): their cross product points to +xi_d
                    const int da = (d + 1) % 3, db = (d + 2) % 3;
                    double ta[3], tbv[3];
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) {
                        ta[kk] = (da == 0) ? J[kk][0] : ((da == 1) ? J[kk][1] : J[kk][2]);
                        tbv[kk] = (db == 0) ? J[kk][0] : ((db == 1) ? J[kk][1] : J[kk][2]);
                    }
                    const double cx = ta[1] * tbv[2] - ta[2] * tbv[1];
                    const double cy = ta[2] * tbv[0] - ta[0] * tbv[2];
                    const double cz = ta[0] * tbv[1] - ta[1] * tbv[0];
                    JF = sqrt(cx * cx + cy * cy + cz * cz);
                    nrm[0] = sgn * cx / JF;
                    nrm[1] = sgn * cy / JF;
                    nrm[2] = sgn * cz / JF;
                    const double* vn = m.vtx + (size_t)nbr_of(m, e, f) * 24;
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) xi[kk] = (kk == d) ? -sgn : ((kk == t1) ? z1 : z2);
                    q1_jac(vn, xi[0], xi[1], xi[2], J);
                    q1_inv(J, Jim);
                    double sp = 0.0, sm = 0.0;
                    for (int k = 0; k < N; ++k) {
                        sp += tb.br2[s][k] / sdet[tl + k * sd];
#pragma unroll
                        for (int kk = 0; kk < 3; ++kk) xi[kk] = (kk == d) ? tb.z[k] : ((kk == t1) ? z1 : z2);
                        q1_jac(vn, xi[0], xi[1], xi[2], J);
                        sm += tb.br2[1 - s][k] / q1_det(J);
                    }
                    lam_p = JF * sp;
                    lam_m = JF * sm;
                } else {
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) nrm[kk] = (kk == d) ? sgn : 0.0;
                    JF = 0.25 * ((d == 0) ? hy * hz : ((d == 1) ? hx * hz : hx * hy));
#pragma unroll
                    for (int k = 0; k < 3; ++k)
#pragma unroll
                        for (int dd = 0; dd < 3; ++dd) Jip[k][dd] = 0.0;
                    Jip[0][0] = 2.0 / hx;
                    Jip[1][1] = 2.0 / hy;
                    Jip[2][2] = 2.0 / hz;
#pragma unroll
                    for (int k = 0; k < 3; ++k)
#pragma unroll
                        for (int dd = 0; dd < 3; ++dd) Jim[k][dd] = Jip[k][dd];
                    lam_p = lam_m = 0.5 * N * N * JF / detJ;
                }
                face_integrand<T, NS>(up, gxp, um, gxm, nrm, Jip, Jim, lam_p, lam_m, tb.w[qt1] * tb.w[qt2] * JF, gas,
                                      fo);
            }
            __syncthreads();          // every thread has read its traces from sE
            if (on) {
#pragma unroll
                for (int k = 0; k < (NS ? 20 : 5); ++k) sF[k * NQ + q] = fo[k];
            }
            __syncthreads();
            if (active) {
#pragma unroll
                for (int fl2 = 0; fl2 < N; ++fl2) {
                    const int f2 = r * N + fl2;
                    if (f2 >= 6) break;
                    const int d2 = f2 >> 1, s2 = f2 & 1;
                    const int u1 = (d2 == 0) ? 1 : 0, u2 = (d2 == 2) ? 1 : 2;
                    const double l = tb.lag[s2][ii[d2]];
                    const int src = fl2 * NF + ii[u1] * N + ii[u2];
#pragma unroll
                    for (int a = 0; a < 5; ++a) {
                        B[a] = fma(l, sF[a * NQ + src], B[a]);
                        if constexpr (NS) {
#pragma unroll
                            for (int k = 0; k < 3; ++k) A[a][k] = fma(l, sF[(5 + a * 3 + k) * NQ + src], A[a][k]);
                        }
                    }
                }
            }
            __syncthreads();
        }
    } else {
        // ---- faces ------------------------------------------------------------------
        // Rounds of NQ face points (N whole faces each, NQ = N NF); thread q takes
        // slot q = (face fl of the round, face point fq) in every stage:
        //   1  neighbour: collapse of its modal data along the normal (value and
        //      normal derivative at the shared face) -> sC; own: trace of the
        //      Gauss values -> sT, normal derivative of the trace (registers);
        //   2  neighbour: first tangential sweep -> sE;
        //   3  both traces with reference gradients (own tangential derivatives
        //      by the collocation derivative on the face), then the face
        //      integrand -> sF (over sC and sT);
        //   4  spread onto the Gauss lines (faces in increasing order).
        T* sC = S;                    // 10 per slot
        T* sT = S + 10 * NQ;          // 5 per slot
        T* sE = S + L_::OFF_E;        // 15 per slot
        T* sF = S;                    // 20 per slot
        for (int r = 0; r * NQ < 6 * NF; ++r) {
            const int fp = r * NQ + q;
            const bool on = active && fp < 6 * NF;
            const int fl = q / NF, fq = q % NF;
            const int f = on ? fp / NF : 0;
            const int d = f >> 1, s = f & 1;
            const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
            const int qt1 = fq / N, qt2 = fq % N;
            const int sd = (d == 0) ? NF : ((d == 1) ? N : 1);
            const int st1 = (d == 0) ? N : NF, st2 = (d == 2) ? N : 1;
            const int tl = qt1 * st1 + qt2 * st2;
            T gdn[5];
            if (on) {
                const int nb = nbr_of(m, e, f);
                const size_t nbase = (size_t)nb * NB;
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    T c0 = 0.0, c1 = 0.0;
#pragma unroll
                    for (int k = 0; k < N; ++k) {
                        const int pm = perm[tl + k * sd];
                        const T val = load_state<MODE, T>(W, V, h, nbase + a * NQ + pm);
                        c0 = fma(tb.Le[1 - s][k], val, c0);
                        c1 = fma(tb.Lde[1 - s][k], val, c1);
                    }
                    sC[q * 10 + a * 2 + 0] = c0;
                    sC[q * 10 + a * 2 + 1] = c1;
                    T v0 = 0.0, v1 = 0.0;
#pragma unroll
                    for (int k = 0; k < N; ++k) {
                        const T uk = su[a * NQ + tl + k * sd];
                        v0 = fma(tb.lag[s][k], uk, v0);
                        v1 = fma(tb.lagd[s][k], uk, v1);
                    }
                    sT[q * 5 + a] = v0;
                    gdn[a] = v1;
                }
            }
            __syncthreads();
            if (on) {
                const int cc = qt2;
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    T e0 = 0.0, e0d = 0.0, e1 = 0.0;
#pragma unroll
                    for (int b = 0; b < N; ++b) {
                        const T* cb = sC + (fl * NF + b * N + cc) * 10 + a * 2;
                        e0 = fma(tb.V[qt1][b], cb[0], e0);
                        e0d = fma(tb.Vd[qt1][b], cb[0], e0d);
                        e1 = fma(tb.V[qt1][b], cb[1], e1);
                    }
                    T* eo = sE + q * 15 + a * 3;
                    eo[0] = e0;
                    eo[1] = e0d;
                    eo[2] = e1;
                }
            }
            __syncthreads();
            // Stage 3 evaluates the integrand into registers, each trace gradient
            // only where it is used (short live ranges), then writes it over sC/sT.
            T fo[20];
            if (on) {
                // geometry of the face point seen from both sides
                double nrm[3], JF, Jip[3][3], Jim[3][3], lam_p, lam_m;
                const double sgn = s ? 1.0 : -1.0;
                if constexpr (CURVED) {
                    const double z1 = tb.z[qt1], z2 = tb.z[qt2];
                    double xi[3];
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) xi[kk] = (kk == d) ? sgn : ((kk == t1) ? z1 : z2);
                    double J[3][3];
                    q1_jac(svtx, xi[0], xi[1], xi[2], J);
                    q1_inv(J, Jip);
                    // tangents dx/dxi_{d+1}, dx/dxi_{d+2} (cyclic): their cross product points to +xi_d
                    const int da = (d + 1) % 3, db = (d + 2) % 3;
                    double ta[3], tbv[3];
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) {
                        ta[kk] = (da == 0) ? J[kk][0] : ((da == 1) ? J[kk][1] : J[kk][2]);
                        tbv[kk] = (db == 0) ? J[kk][0] : ((db == 1) ? J[kk][1] : J[kk][2]);
                    }
                    const double cx = ta[1] * tbv[2] - ta[2] * tbv[1];
                    const double cy = ta[2] * tbv[0] - ta[0] * tbv[2];
                    const double cz = ta[0] * tbv[1] - ta[1] * tbv[0];
                    JF = sqrt(cx * cx + cy * cy + cz * cz);
                    nrm[0] = sgn * cx / JF;
                    nrm[1] = sgn * cy / JF;
                    nrm[2] = sgn * cz / JF;
                    const double* vn = m.vtx + (size_t)nbr_of(m, e, f) * 24;
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) xi[kk] = (kk == d) ? -sgn : ((kk == t1) ? z1 : z2);
                    q1_jac(vn, xi[0], xi[1], xi[2], J);
                    q1_inv(J, Jim);
                    double sp = 0.0, sm = 0.0;
                    for (int k = 0; k < N; ++k) {
                        sp += tb.br2[s][k] / sdet[tl + k * sd];
#pragma unroll
                        for (int kk = 0; kk < 3; ++kk) xi[kk] = (kk == d) ? tb.z[k] : ((kk == t1) ? z1 : z2);
                        q1_jac(vn, xi[0], xi[1], xi[2], J);
                        sm += tb.br2[1 - s][k] / q1_det(J);
                    }
                    lam_p = JF * sp;
                    lam_m = JF * sm;
                } else {
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) nrm[kk] = (kk == d) ? sgn : 0.0;
                    JF = 0.25 * ((d == 0) ? hy * hz : ((d == 1) ? hx * hz : hx * hy));
#pragma unroll
                    for (int k = 0; k < 3; ++k)
#pragma unroll
                        for (int dd = 0; dd < 3; ++dd) Jip[k][dd] = 0.0;
                    Jip[0][0] = 2.0 / hx;
                    Jip[1][1] = 2.0 / hy;
                    Jip[2][2] = 2.0 / hz;
#pragma unroll
                    for (int k = 0; k < 3; ++k)
#pragma unroll
                        for (int dd = 0; dd < 3; ++dd) Jim[k][dd] = Jip[k][dd];
                    lam_p = lam_m = 0.5 * N * N * JF / detJ;
                }
                T up[5], um[5];
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    T v0 = 0.0;
#pragma unroll
                    for (int c = 0; c < N; ++c) v0 = fma(tb.V[qt2][c], sE[(fl * NF + qt1 * N + c) * 15 + a * 3], v0);
                    um[a] = v0;
                    up[a] = sT[q * 5 + a];
                }
                T Fn[5];
                roe_flux(up, um, nrm, gas.gamma, Fn);
                const double sc = tb.w[qt1] * tb.w[qt2] * JF;
                if constexpr (NS) {
                    {   // + side: reference gradient of the own trace -> physical -> normal viscous flux
                        T g[5][3];
#pragma unroll
                        for (int a = 0; a < 5; ++a) {
                            T o1 = 0.0, o2 = 0.0;
#pragma unroll
                            for (int c = 0; c < N; ++c) {
                                o1 = fma(tb.D[qt1][c], sT[(fl * NF + c * N + qt2) * 5 + a], o1);
                                o2 = fma(tb.D[qt2][c], sT[(fl * NF + qt1 * N + c) * 5 + a], o2);
                            }
                            T gx[3];
#pragma unroll
                            for (int kk = 0; kk < 3; ++kk) gx[kk] = (kk == d) ? gdn[a] : ((kk == t1) ? o1 : o2);
#pragma unroll
                            for (int j = 0; j < 3; ++j) g[a][j] = Jip[0][j] * gx[0] + Jip[1][j] * gx[1] + Jip[2][j] * gx[2];
                        }
                        flux_v_n_acc(up, g, gas, 0.5, nrm, Fn);
                    }
                    {   // - side: neighbour trace gradient from the tangential sweep
                        T g[5][3];
#pragma unroll
                        for (int a = 0; a < 5; ++a) {
                            T vt1 = 0.0, vt2 = 0.0, vd = 0.0;
#pragma unroll
                            for (int c = 0; c < N; ++c) {
                                const T* eo = sE + (fl * NF + qt1 * N + c) * 15 + a * 3;
                                vt1 = fma(tb.V[qt2][c], eo[1], vt1);
                                vt2 = fma(tb.Vd[qt2][c], eo[0], vt2);
                                vd = fma(tb.V[qt2][c], eo[2], vd);
                            }
                            T gx[3];
#pragma unroll
                            for (int kk = 0; kk < 3; ++kk) gx[kk] = (kk == d) ? vd : ((kk == t1) ? vt1 : vt2);
#pragma unroll
                            for (int j = 0; j < 3; ++j) g[a][j] = Jim[0][j] * gx[0] + Jim[1][j] * gx[1] + Jim[2][j] * gx[2];
                        }
                        flux_v_n_acc(um, g, gas, 0.5, nrm, Fn);
                    }
                    face_penalty_symmetry<T>(up, um, nrm, Jip, lam_p, lam_m, sc, gas, Fn, fo);
                } else {
#pragma unroll
                    for (int a = 0; a < 5; ++a) fo[a] = sc * Fn[a];
                }
            }
            __syncthreads();
            if (on) {
#pragma unroll
                for (int k = 0; k < (NS ? 20 : 5); ++k) sF[q * 20 + k] = fo[k];
            }
            __syncthreads();
            if (active) {
#pragma unroll
                for (int fl2 = 0; fl2 < N; ++fl2) {
                    const int f2 = r * N + fl2;
                    if (f2 >= 6) break;
                    const int d2 = f2 >> 1, s2 = f2 & 1;
                    const int u1 = (d2 == 0) ? 1 : 0, u2 = (d2 == 2) ? 1 : 2;
                    const double l = tb.lag[s2][ii[d2]];
                    const T* fo = sF + (fl2 * NF + ii[u1] * N + ii[u2]) * 20;
#pragma unroll
                    for (int a = 0; a < 5; ++a) {
                        B[a] = fma(l, fo[a], B[a]);
                        if constexpr (NS) {
#pragma unroll
                            for (int k = 0; k < 3; ++k) A[a][k] = fma(l, fo[5 + a * 3 + k], A[a][k]);
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    // ---- test: R = V^T (x) V^T (x) V^T [B + sum_k D_k^T A_k] -------------------------------
    T* sA = S;                    // 15 NQ
    T* sB = S + 15 * NQ;          // 5 NQ
    T* H = S + L_::OFF_E;
    T* Y1 = H + 5 * NQ;
    T* Y2 = H + 10 * NQ;
    if (active) {
#pragma unroll
        for (int a = 0; a < 5; ++a) {
#pragma unroll
            for (int k = 0; k < 3; ++k) sA[(a * 3 + k) * NQ + q] = A[a][k];
            sB[a * NQ + q] = B[a];
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            T acc = sB[a * NQ + q];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int j = 0; j < N; ++j)
                    acc = fma(tb.D[j][ii[k]], sA[(a * 3 + k) * NQ + tix_dir<N>(k, j, ii)], acc);
            H[a * NQ + q] = acc;
        }
    }
    __syncthreads();
    if (active) sweep<N, 5, true>(tb.V, H, Y1, 0, ii, q);
    __syncthreads();
    if (active) sweep<N, 5, true>(tb.V, Y1, Y2, 1, ii, q);
    __syncthreads();
    T res[5];
    if (active) {
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            T acc = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) acc = fma(tb.V[j][ii[2]], Y2[a * NQ + tix_dir<N>(2, j, ii)], acc);
            res[a] = acc;
        }
    }
    // ---- output -------------------------------------------------------------------------
    const size_t base = (size_t)e * NB;
    const int pm = perm[q];
    if constexpr (MODE == M_RES) {
        if (active)
#pragma unroll
            for (int a = 0; a < 5; ++a) out[base + a * NQ + pm] = res[a];
    } else if constexpr (MODE == M_TANGENT) {
        if (active)
#pragma unroll
            for (int a = 0; a < 5; ++a) out[base + a * NQ + pm] = tan_(res[a]);
    } else {
        // y = shift M v + (R(W + h v) - R(W)) / h
        double mv[5];
        if constexpr (CURVED) {
            __syncthreads();
            T* V0 = S;
            T* V1 = S + 5 * NQ;
            T* V2 = S + 10 * NQ;
            if (active)
#pragma unroll
                for (int a = 0; a < 5; ++a) V0[a * NQ + q] = V[base + a * NQ + pm];
            __syncthreads();
            if (active) sweep<N, 5, false>(tb.V, V0, V1, 0, ii, q);
            __syncthreads();
            if (active) sweep<N, 5, false>(tb.V, V1, V2, 1, ii, q);
            __syncthreads();
            if (active) {
                const double wq = tb.w[ii[0]] * tb.w[ii[1]] * tb.w[ii[2]] * detJ;
                sweep<N, 5, false>(tb.V, V2, V0, 2, ii, q);
#pragma unroll
                for (int a = 0; a < 5; ++a) V0[a * NQ + q] = V0[a * NQ + q] * wq;
            }
            __syncthreads();
            if (active) sweep<N, 5, true>(tb.V, V0, V1, 0, ii, q);
            __syncthreads();
            if (active) sweep<N, 5, true>(tb.V, V1, V2, 1, ii, q);
            __syncthreads();
            if (active)
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    double acc = 0.0;
#pragma unroll
                    for (int j = 0; j < N; ++j) acc = fma(tb.V[j][ii[2]], V2[a * NQ + tix_dir<N>(2, j, ii)], acc);
                    mv[a] = acc;
                }
        } else {
            if (active)
#pragma unroll
                for (int a = 0; a < 5; ++a) mv[a] = detJ * V[base + a * NQ + pm];
        }
        if (active) {
            const double ih = 1.0 / h;
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                const size_t o = base + a * NQ + pm;
                out[o] = (res[a] - RW[o]) * ih + shift * mv[a];
            }
        }
    }
}

// Two waves per SIMD where the registers allow it without spilling (straight
// elements, real arithmetic, degree <= 3); one otherwise.
template <int P, bool CURVED, int MODE>
struct MinWaves { static constexpr int W = (MODE < M_TANGENT && P <= 3 && !CURVED) ? 2 : 1; };

template <int P, bool NS, bool CURVED, int MODE>
__global__ void __launch_bounds__((Launch<P, (MODE >= M_TANGENT)>::EPB * Sz<P>::NQ), (MinWaves<P, CURVED, MODE>::W))
    dg_kernel(MeshDev m, Gas gas, const double* __restrict__ W, const double* __restrict__ V,
              const double* __restrict__ RW, const double* __restrict__ hbuf, double shift,
              double* __restrict__ out) {
    using S_ = Sz<P>;
    constexpr int NQ = S_::NQ;
    constexpr bool DUAL = (MODE >= M_TANGENT);
    using T = typename std::conditional<DUAL, Dual, double>::type;
    constexpr int EPB = Launch<P, DUAL>::EPB;
    __shared__ T smem[EPB * LayOf<P, MODE>::TOT];
    __shared__ double sdet[EPB][CURVED ? NQ : 1];      // curved elements only
    __shared__ double svtx[EPB][CURVED ? 24 : 1];
    const int es = threadIdx.x / NQ, q = threadIdx.x % NQ;
    const int e = blockIdx.x * EPB + es;
    dg_element<P, NS, CURVED, MODE>(m, gas, W, V, RW, hbuf, shift, out, smem + es * LayOf<P, MODE>::TOT, sdet[es],
                                    svtx[es], e,
                                    e < m.ne, q);
}

// ---- mass matrix, projection, quadrature points, Jacobian check --------------------------
// y = scale * M v (+ y if accumulate).  Affine: M = detJ I.
template <int P, bool CURVED>
__global__ void __launch_bounds__((Launch<P, false>::EPB * Sz<P>::NQ))
    mass_kernel(MeshDev m, const double* __restrict__ v, double* __restrict__ y, double scale, int accumulate) {
    using S_ = Sz<P>;
    constexpr int N = S_::N, NQ = S_::NQ, NF = S_::NF, NB = S_::NB;
    constexpr int EPB = Launch<P, false>::EPB;
    __shared__ double smem[EPB][15 * NQ];
    __shared__ double svtx[EPB][24];
    const Tab& tb = c_tab[P];
    const short* perm = c_perm + perm_offset(P);
    const int es = threadIdx.x / NQ, q = threadIdx.x % NQ;
    const int e = blockIdx.x * EPB + es;
    const bool active = e < m.ne;
    const int ii[3] = {q / NF, (q / N) % N, q % N};
    const size_t base = (size_t)e * NB;
    const int pm = perm[q];
    double r[5];
    if constexpr (!CURVED) {
        if (!active) return;
        const double detJ = 0.125 * m.h[0] * m.h[1] * m.h[2];
        for (int a = 0; a < 5; ++a) r[a] = scale * detJ * v[base + a * NQ + pm];
    } else {
        double* V0 = smem[es];
        double* V1 = V0 + 5 * NQ;
        double* V2 = V0 + 10 * NQ;
        if (active) {
            for (int a = 0; a < 5; ++a) V0[a * NQ + q] = v[base + a * NQ + pm];
            for (int k = q; k < 24; k += NQ) svtx[es][k] = m.vtx[(size_t)e * 24 + k];
        }
        __syncthreads();
        if (active) sweep<N, 5, false>(tb.V, V0, V1, 0, ii, q);
        __syncthreads();
        if (active) sweep<N, 5, false>(tb.V, V1, V2, 1, ii, q);
        __syncthreads();
        if (active) {
            double J[3][3];
            q1_jac(svtx[es], tb.z[ii[0]], tb.z[ii[1]], tb.z[ii[2]], J);
            const double wq = tb.w[ii[0]] * tb.w[ii[1]] * tb.w[ii[2]] * q1_det(J);
            sweep<N, 5, false>(tb.V, V2, V0, 2, ii, q);
            for (int a = 0; a < 5; ++a) V0[a * NQ + q] *= wq;
        }
        __syncthreads();
        if (active) sweep<N, 5, true>(tb.V, V0, V1, 0, ii, q);
        __syncthreads();
        if (active) sweep<N, 5, true>(tb.V, V1, V2, 1, ii, q);
        __syncthreads();
        if (!active) return;
        for (int a = 0; a < 5; ++a) {
            double acc = 0.0;
            for (int j = 0; j < N; ++j) acc = fma(tb.V[j][ii[2]], V2[a * NQ + tix_dir<N>(2, j, ii)], acc);
            r[a] = scale * acc;
        }
    }
    for (int a = 0; a < 5; ++a) {
        const size_t o = base + a * NQ + pm;
        y[o] = accumulate ? y[o] + r[a] : r[a];
    }
}

// Physical Gauss point coordinates: xyz[e][q][3].
template <int P>
__global__ void quad_points_kernel(MeshDev m, double* __restrict__ xyz) {
    constexpr int N = P + 1, NQ = N * N * N, NF = N * N;
    const Tab& tb = c_tab[P];
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)m.ne * NQ) return;
    const int e = (int)(gid / NQ), q = (int)(gid % NQ);
    const double x0 = tb.z[q / NF], x1 = tb.z[(q / N) % N], x2 = tb.z[q % N];
    double X[3] = {0.0, 0.0, 0.0};
    if (m.vtx) {
        const double* vv = m.vtx + (size_t)e * 24;
        for (int v = 0; v < 8; ++v) {
            const double s0 = (v & 1) ? 1.0 : -1.0, s1 = (v & 2) ? 1.0 : -1.0, s2 = (v & 4) ? 1.0 : -1.0;
            const double Nv = 0.125 * (1.0 + s0 * x0) * (1.0 + s1 * x1) * (1.0 + s2 * x2);
            for (int d = 0; d < 3; ++d) X[d] = fma(Nv, vv[3 * v + d], X[d]);
        }
    }
    for (int d = 0; d < 3; ++d) xyz[gid * 3 + d] = X[d];
}

// W = M^-1 int phi u with the Gauss rule: since V is square and
// V^T diag(w) V = I, this is W = V^T diag(w) u_q independent of detJ.
template <int P>
__global__ void project_kernel(MeshDev m, const double* __restrict__ vals, double* __restrict__ W) {
    using S_ = Sz<P>;
    constexpr int N = S_::N, NQ = S_::NQ, NF = S_::NF, NB = S_::NB;
    constexpr int EPB = Launch<P, false>::EPB;
    __shared__ double smem[EPB][15 * NQ];
    const Tab& tb = c_tab[P];
    const short* perm = c_perm + perm_offset(P);
    const int es = threadIdx.x / NQ, q = threadIdx.x % NQ;
    const int e = blockIdx.x * EPB + es;
    const bool active = e < m.ne;
    const int ii[3] = {q / NF, (q / N) % N, q % N};
    double* V0 = smem[es];
    double* V1 = V0 + 5 * NQ;
    double* V2 = V0 + 10 * NQ;
    if (active) {
        const double wq = tb.w[ii[0]] * tb.w[ii[1]] * tb.w[ii[2]];
        for (int a = 0; a < 5; ++a) V0[a * NQ + q] = wq * vals[((size_t)e * NQ + q) * 5 + a];
    }
    __syncthreads();
    if (active) sweep<N, 5, true>(tb.V, V0, V1, 0, ii, q);
    __syncthreads();
    if (active) sweep<N, 5, true>(tb.V, V1, V2, 1, ii, q);
    __syncthreads();
    if (!active) return;
    for (int a = 0; a < 5; ++a) {
        double acc = 0.0;
        for (int j = 0; j < N; ++j) acc = fma(tb.V[j][ii[2]], V2[a * NQ + tix_dir<N>(2, j, ii)], acc);
        W[(size_t)e * NB + a * NQ + perm[q]] = acc;
    }
}

// bad[0] += 1 for every volume Gauss point or face point with detJ <= 0.
template <int P>
__global__ void check_jac_kernel(MeshDev m, int* bad) {
    constexpr int N = P + 1, NQ = N * N * N, NF = N * N;
    const Tab& tb = c_tab[P];
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)m.ne * NQ) return;
    const int e = (int)(gid / NQ), q = (int)(gid % NQ);
    double J[3][3];
    q1_jac(m.vtx + (size_t)e * 24, tb.z[q / NF], tb.z[(q / N) % N], tb.z[q % N], J);
    const double det = q1_det(J);
    if (!(det > 0.0)) atomicAdd(bad, 1);
}

// ---- host launchers -------------------------------------------------------------------------
namespace {
template <int P, int MODE>
hipError_t launch_dg(const DGArgs& a, const double* W, const double* V, const double* RW, const double* hbuf,
                     double shift, double* out, hipStream_t s) {
    constexpr bool DUAL = MODE >= M_TANGENT;
    constexpr int EPB = Launch<P, DUAL>::EPB;
    constexpr int NQ = Sz<P>::NQ;
    dim3 grid((a.m.ne + EPB - 1) / EPB);
    dim3 block(EPB * NQ);
    const bool curved = a.m.vtx != nullptr;
    if (a.ns) {
        if (curved) hipLaunchKernelGGL((dg_kernel<P, true, true, MODE>), grid, block, 0, s, a.m, a.g, W, V, RW, hbuf, shift, out);
        else hipLaunchKernelGGL((dg_kernel<P, true, false, MODE>), grid, block, 0, s, a.m, a.g, W, V, RW, hbuf, shift, out);
    } else {
        if (curved) hipLaunchKernelGGL((dg_kernel<P, false, true, MODE>), grid, block, 0, s, a.m, a.g, W, V, RW, hbuf, shift, out);
        else hipLaunchKernelGGL((dg_kernel<P, false, false, MODE>), grid, block, 0, s, a.m, a.g, W, V, RW, hbuf, shift, out);
    }
    return hipGetLastError();
}

template <int MODE>
hipError_t dispatch_dg(const DGArgs& a, const double* W, const double* V, const double* RW, const double* hbuf,
                       double shift, double* out, hipStream_t s) {
    switch (a.p) {
        case 1: return launch_dg<1, MODE>(a, W, V, RW, hbuf, shift, out, s);
        case 2: return launch_dg<2, MODE>(a, W, V, RW, hbuf, shift, out, s);
        case 3: return launch_dg<3, MODE>(a, W, V, RW, hbuf, shift, out, s);
        case 4: return launch_dg<4, MODE>(a, W, V, RW, hbuf, shift, out, s);
        default: return hipErrorInvalidValue;
    }
}

template <int P>
hipError_t launch_mass_p(const DGArgs& a, const double* v, double* y, double scale, int acc, hipStream_t s) {
    constexpr int EPB = Launch<P, false>::EPB;
    dim3 grid((a.m.ne + EPB - 1) / EPB), block(EPB * Sz<P>::NQ);
    if (a.m.vtx) hipLaunchKernelGGL((mass_kernel<P, true>), grid, block, 0, s, a.m, v, y, scale, acc);
    else hipLaunchKernelGGL((mass_kernel<P, false>), grid, block, 0, s, a.m, v, y, scale, acc);
    return hipGetLastError();
}
template <int P>
hipError_t launch_project_p(const DGArgs& a, const double* vals, double* W, hipStream_t s) {
    constexpr int EPB = Launch<P, false>::EPB;
    dim3 grid((a.m.ne + EPB - 1) / EPB), block(EPB * Sz<P>::NQ);
    hipLaunchKernelGGL((project_kernel<P>), grid, block, 0, s, a.m, vals, W);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_residual(const DGArgs& a, const double* W, double* R, hipStream_t s) {
    return dispatch_dg<M_RES>(a, W, nullptr, nullptr, nullptr, 0.0, R, s);
}
hipError_t launch_jvp_fd(const DGArgs& a, const double* W, const double* RW, const double* v, const double* hbuf,
                         double shift, double* y, hipStream_t s) {
    return dispatch_dg<M_JVP_FD>(a, W, v, RW, hbuf, shift, y, s);
}
hipError_t launch_jvp_exact(const DGArgs& a, const double* W, const double* v, double shift, double* y,
                            hipStream_t s) {
    return dispatch_dg<M_TANGENT>(a, W, v, nullptr, nullptr, shift, y, s);
}
hipError_t launch_mass(const DGArgs& a, const double* v, double* y, double scale, int accumulate, hipStream_t s) {
    switch (a.p) {
        case 1: return launch_mass_p<1>(a, v, y, scale, accumulate, s);
        case 2: return launch_mass_p<2>(a, v, y, scale, accumulate, s);
        case 3: return launch_mass_p<3>(a, v, y, scale, accumulate, s);
        case 4: return launch_mass_p<4>(a, v, y, scale, accumulate, s);
        default: return hipErrorInvalidValue;
    }
}
hipError_t launch_project(const DGArgs& a, const double* vals, double* W, hipStream_t s) {
    switch (a.p) {
        case 1: return launch_project_p<1>(a, vals, W, s);
        case 2: return launch_project_p<2>(a, vals, W, s);
        case 3: return launch_project_p<3>(a, vals, W, s);
        case 4: return launch_project_p<4>(a, vals, W, s);
        default: return hipErrorInvalidValue;
    }
}
hipError_t launch_quad_points(const DGArgs& a, double* xyz, hipStream_t s) {
    const size_t n = (size_t)a.m.ne * (a.p + 1) * (a.p + 1) * (a.p + 1);
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (a.p) {
        case 1: hipLaunchKernelGGL(quad_points_kernel<1>, grid, block, 0, s, a.m, xyz); break;
        case 2: hipLaunchKernelGGL(quad_points_kernel<2>, grid, block, 0, s, a.m, xyz); break;
        case 3: hipLaunchKernelGGL(quad_points_kernel<3>, grid, block, 0, s, a.m, xyz); break;
        case 4: hipLaunchKernelGGL(quad_points_kernel<4>, grid, block, 0, s, a.m, xyz); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
hipError_t launch_check_jacobian(const DGArgs& a, int* bad, hipStream_t s) {
    const size_t n = (size_t)a.m.ne * (a.p + 1) * (a.p + 1) * (a.p + 1);
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (a.p) {
        case 1: hipLaunchKernelGGL(check_jac_kernel<1>, grid, block, 0, s, a.m, bad); break;
        case 2: hipLaunchKernelGGL(check_jac_kernel<2>, grid, block, 0, s, a.m, bad); break;
        case 3: hipLaunchKernelGGL(check_jac_kernel<3>, grid, block, 0, s, a.m, bad); break;
        case 4: hipLaunchKernelGGL(check_jac_kernel<4>, grid, block, 0, s, a.m, bad); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- batched DG operator: one persistent launch over many cases ---------------------------
// Work item = (case, first element, degree, elements in the tile).  Each
// workgroup walks the item list with a fixed stride (item i goes to workgroup
// i mod grid), runs the degree's compile-time path on its tile (one slot of
// NQ threads per element) and moves on; results are per element, so they do
// not depend on the tiling or the grid.
size_t batch_slot_bytes(int p, int mode) {
    const bool dual = mode == M_TANGENT;
    const size_t sc = dual ? sizeof(Dual) : sizeof(double);
    switch (p) {
        case 1: return (dual ? LayOf<1, M_TANGENT>::TOT : LayOf<1, M_RES>::TOT) * sc + (Sz<1>::NQ + 24) * sizeof(double);
        case 2: return (dual ? LayOf<2, M_TANGENT>::TOT : LayOf<2, M_RES>::TOT) * sc + (Sz<2>::NQ + 24) * sizeof(double);
        case 3: return (dual ? LayOf<3, M_TANGENT>::TOT : LayOf<3, M_RES>::TOT) * sc + (Sz<3>::NQ + 24) * sizeof(double);
        case 4: return (dual ? LayOf<4, M_TANGENT>::TOT : LayOf<4, M_RES>::TOT) * sc + (Sz<4>::NQ + 24) * sizeof(double);
        default: return 0;
    }
}

template <int P, bool NS, bool CURVED, int MODE>
__device__ __forceinline__ void batch_tile(const BatchCaseDev& c, const BatchItem& w, double* dyn,
                                           const double* __restrict__ W, const double* __restrict__ V,
                                           const double* __restrict__ RW, const double* __restrict__ hcase,
                                           double shift, double* __restrict__ out) {
    using S_ = Sz<P>;
    constexpr int NQ = S_::NQ;
    using T = typename std::conditional<(MODE >= M_TANGENT), Dual, double>::type;
    const int es = threadIdx.x / NQ, q = threadIdx.x % NQ;
    const bool slot = es < w.n;
    const int esl = slot ? es : 0;
    constexpr int TOT = LayOf<P, MODE>::TOT;
    T* S = reinterpret_cast<T*>(dyn) + (size_t)esl * TOT;
    double* sdet = reinterpret_cast<double*>(reinterpret_cast<T*>(dyn) + (size_t)w.n * TOT) + esl * NQ;
    double* svtx = reinterpret_cast<double*>(reinterpret_cast<T*>(dyn) + (size_t)w.n * TOT) + w.n * NQ + esl * 24;
    const size_t o = c.off;
    const int e = w.e0 + es;
    dg_element<P, NS, CURVED, MODE>(c.m, c.g, W + o, V ? V + o : nullptr, RW ? RW + o : nullptr, hcase + w.c, shift,
                                    out + o, S, sdet, svtx, e, slot && e < c.m.ne, q);
}

template <bool NS, bool CURVED, int MODE>
__global__ void __launch_bounds__(BATCH_MAX_THREADS)
    batch_dg_kernel(const BatchCaseDev* __restrict__ cases, const BatchItem* __restrict__ items, int nitems,
                    const double* __restrict__ W, const double* __restrict__ V, const double* __restrict__ RW,
                    const double* __restrict__ hcase, double shift, double* __restrict__ out) {
    extern __shared__ double dyn[];
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BatchItem w = items[it];
        const BatchCaseDev c = cases[w.c];
        switch (w.p) {
            case 1: batch_tile<1, NS, CURVED, MODE>(c, w, dyn, W, V, RW, hcase, shift, out); break;
            case 2: batch_tile<2, NS, CURVED, MODE>(c, w, dyn, W, V, RW, hcase, shift, out); break;
            case 3: batch_tile<3, NS, CURVED, MODE>(c, w, dyn, W, V, RW, hcase, shift, out); break;
            default: batch_tile<4, NS, CURVED, MODE>(c, w, dyn, W, V, RW, hcase, shift, out); break;
        }
        __syncthreads();     // the next item reuses the LDS
    }
}

namespace {
template <bool NS, bool CURVED, int MODE>
hipError_t launch_batch_dg_t(const BatchCaseDev* cases, const BatchItem* items, int nitems, int threads, int grid,
                             size_t lds, const double* W, const double* V, const double* RW, const double* hcase,
                             double shift, double* out, hipStream_t s) {
    hipError_t e = hipFuncSetAttribute((const void*)batch_dg_kernel<NS, CURVED, MODE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((batch_dg_kernel<NS, CURVED, MODE>), dim3(grid), dim3(threads), lds, s, cases, items, nitems,
                       W, V, RW, hcase, shift, out);
    return hipGetLastError();
}
template <int MODE>
hipError_t launch_batch_dg_m(bool ns, bool curved, const BatchCaseDev* cases, const BatchItem* items, int nitems,
                             int threads, int grid, size_t lds, const double* W, const double* V, const double* RW,
                             const double* hcase, double shift, double* out, hipStream_t s) {
    if (ns) {
        if (curved) return launch_batch_dg_t<true, true, MODE>(cases, items, nitems, threads, grid, lds, W, V, RW, hcase, shift, out, s);
        return launch_batch_dg_t<true, false, MODE>(cases, items, nitems, threads, grid, lds, W, V, RW, hcase, shift, out, s);
    }
    if (curved) return launch_batch_dg_t<false, true, MODE>(cases, items, nitems, threads, grid, lds, W, V, RW, hcase, shift, out, s);
    return launch_batch_dg_t<false, false, MODE>(cases, items, nitems, threads, grid, lds, W, V, RW, hcase, shift, out, s);
}
}  // namespace

hipError_t launch_batch_dg(int mode, bool ns, bool curved, const BatchCaseDev* cases, const BatchItem* items,
                           int nitems, int threads, int grid, size_t lds, const double* W, const double* V,
                           const double* RW, const double* hcase, double shift, double* out, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (threads < 64 || threads > BATCH_MAX_THREADS || threads % 64 || grid < 1) return hipErrorInvalidValue;
    switch (mode) {
        case M_RES: return launch_batch_dg_m<M_RES>(ns, curved, cases, items, nitems, threads, grid, lds, W, V, RW, hcase, shift, out, s);
        case M_JVP_FD: return launch_batch_dg_m<M_JVP_FD>(ns, curved, cases, items, nitems, threads, grid, lds, W, V, RW, hcase, shift, out, s);
        case M_TANGENT: return launch_batch_dg_m<M_TANGENT>(ns, curved, cases, items, nitems, threads, grid, lds, W, V, RW, hcase, shift, out, s);
        default: return hipErrorInvalidValue;
    }
}

// ---- inherited coarse operators (Sec. 6.1) ---------------------------------------------------
// Geometry of face point (qt1, qt2) of face f of element e seen from both
// sides, everything from the vertex tables (curved) or the box spacing.
template <int P, bool CURVED>
__device__ __forceinline__ void face_geometry(const Tab& tb, const MeshDev& m, int e, int f, int qt1, int qt2,
                                              double nrm[3], double& JF, double Jip[3][3], double Jim[3][3],
                                              double& lam_p, double& lam_m) {
    constexpr int N = P + 1;
    const int d = f >> 1, s = f & 1;
    const int t1 = (d == 0) ? 1 : 0;
    const double sgn = s ? 1.0 : -1.0;
    if constexpr (CURVED) {
        const double z1 = tb.z[qt1], z2 = tb.z[qt2];
        const double* vo = m.vtx + (size_t)e * 24;
        const double* vn = m.vtx + (size_t)nbr_of(m, e, f) * 24;
        double xi[3], J[3][3];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) xi[kk] = (kk == d) ? sgn : ((kk == t1) ? z1 : z2);
        q1_jac(vo, xi[0], xi[1], xi[2], J);
        q1_inv(J, Jip);
        const int da = (d + 1) % 3, db = (d + 2) % 3;
        double ta[3], tbv[3];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
            ta[kk] = (da == 0) ? J[kk][0] : ((da == 1) ? J[kk][1] : J[kk][2]);
            tbv[kk] = (db == 0) ? J[kk][0] : ((db == 1) ? J[kk][1] : J[kk][2]);
        }
        const double cx = ta[1] * tbv[2] - ta[2] * tbv[1];
        const double cy = ta[2] * tbv[0] - ta[0] * tbv[2];
        const double cz = ta[0] * tbv[1] - ta[1] * tbv[0];
        JF = sqrt(cx * cx + cy * cy + cz * cz);
        nrm[0] = sgn * cx / JF;
        nrm[1] = sgn * cy / JF;
        nrm[2] = sgn * cz / JF;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) xi[kk] = (kk == d) ? -sgn : ((kk == t1) ? z1 : z2);
        q1_jac(vn, xi[0], xi[1], xi[2], J);
        q1_inv(J, Jim);
        double sp = 0.0, sm = 0.0;
        for (int k = 0; k < N; ++k) {
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) xi[kk] = (kk == d) ? tb.z[k] : ((kk == t1) ? z1 : z2);
            q1_jac(vo, xi[0], xi[1], xi[2], J);
            sp += tb.br2[s][k] / q1_det(J);
            q1_jac(vn, xi[0], xi[1], xi[2], J);
            sm += tb.br2[1 - s][k] / q1_det(J);
        }
        lam_p = JF * sp;
        lam_m = JF * sm;
    } else {
        const double hx = m.h[0], hy = m.h[1], hz = m.h[2];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) nrm[kk] = (kk == d) ? sgn : 0.0;
        JF = 0.25 * ((d == 0) ? hy * hz : ((d == 1) ? hx * hz : hx * hy));
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) Jip[k][dd] = Jim[k][dd] = 0.0;
        Jip[0][0] = Jim[0][0] = 2.0 / hx;
        Jip[1][1] = Jim[1][1] = 2.0 / hy;
        Jip[2][2] = Jim[2][2] = 2.0 / hz;
        lam_p = lam_m = 0.5 * N * N * JF / (0.125 * hx * hy * hz);
    }
}

// Basis function of tensor mode (i0,i1,i2) and its reference gradient at
// the face point (qt1, qt2) of the face with normal direction d on end s.
template <int N>
__device__ __forceinline__ void face_basis(const Tab& tb, int d, int s, int qt1, int qt2, int tq, double& v,
                                           double g[3]) {
    const int ii[3] = {tq / (N * N), (tq / N) % N, tq % N};
    const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    const int an = (d == 0) ? ii[0] : ((d == 1) ? ii[1] : ii[2]);
    const int a1 = (t1 == 0) ? ii[0] : ii[1];
    const int a2 = (t2 == 1) ? ii[1] : ii[2];
    const double ln = tb.Le[s][an], dn = tb.Lde[s][an];
    const double v1 = tb.V[qt1][a1], d1 = tb.Vd[qt1][a1];
    const double v2 = tb.V[qt2][a2], d2 = tb.Vd[qt2][a2];
    v = ln * v1 * v2;
    double gd = dn * v1 * v2, g1 = ln * d1 * v2, g2 = ln * v1 * d2;
#pragma unroll
    for (int k = 0; k < 3; ++k) g[k] = (k == d) ? gd : ((k == t1) ? g1 : g2);
}

// Coarse face-coupling blocks dR_e[S]/dW_nb[S] of face f (S = modes of
// degree <= PC, all equations): the dependence of the face-f integrand of
// element e on the neighbour's trace, linearised with dual numbers and tested
// with the coarse modes of e.  One workgroup per (element, face).  A face
// whose neighbour is the element itself (one-element periodic axis) belongs to
// the diagonal block: its block is zero here.
template <int P, int PC, bool NS, bool CURVED>
__global__ void __launch_bounds__(256) offdiag_kernel(MeshDev m, Gas gas, const double* __restrict__ W,
                                                      double* __restrict__ out) {
    constexpr int N = P + 1, NQ = N * N * N, NF = N * N, NB = 5 * NQ;
    constexpr int NC = PC + 1, NVC = NC * NC * NC, NBC = 5 * NVC;
    constexpr int CB = 256 / NF;
    const Tab& tb = c_tab[P];
    const short* perm = c_perm + perm_offset(P);
    const int e = blockIdx.x, f = blockIdx.y;
    const int d = f >> 1, s = f & 1;
    const int nb = nbr_of(m, e, f);
    const int t = threadIdx.x;
    double* ob = out + ((size_t)e * 6 + f) * NBC * NBC;
    if (nb == e) {
        for (int i = t; i < NBC * NBC; i += 256) ob[i] = 0.0;
        return;
    }
    __shared__ double sW[2][NB];
    __shared__ double sPr[NF][40];
    __shared__ double sGe[NF][26];
    __shared__ double sOut[CB * NF][20];
    __shared__ short sInv[NVC];
    for (int idx = t; idx < NB; idx += 256) {
        const int a = idx / NQ, q = idx % NQ;
        sW[0][a * NQ + q] = W[(size_t)e * NB + a * NQ + perm[q]];
        sW[1][a * NQ + q] = W[(size_t)nb * NB + a * NQ + perm[q]];
    }
    for (int q = t; q < NQ; q += 256) {
        const int h = perm[q];
        if (h < NVC) sInv[h] = (short)q;
    }
    __syncthreads();
    if (t < NF) {
        const int qt1 = t / N, qt2 = t % N;
        for (int side = 0; side < 2; ++side) {
            const int se = side == 0 ? s : 1 - s;
            for (int a = 0; a < 5; ++a) {
                double v = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
                for (int q = 0; q < NQ; ++q) {
                    double bv, bg[3];
                    face_basis<N>(tb, d, se, qt1, qt2, q, bv, bg);
                    const double w = sW[side][a * NQ + q];
                    v = fma(bv, w, v);
                    g0 = fma(bg[0], w, g0);
                    g1 = fma(bg[1], w, g1);
                    g2 = fma(bg[2], w, g2);
                }
                sPr[t][side * 20 + a] = v;
                sPr[t][side * 20 + 5 + a * 3 + 0] = g0;
                sPr[t][side * 20 + 5 + a * 3 + 1] = g1;
                sPr[t][side * 20 + 5 + a * 3 + 2] = g2;
            }
        }
        double nrm[3], JF, Jip[3][3], Jim[3][3], lp, lm;
        face_geometry<P, CURVED>(tb, m, e, f, qt1, qt2, nrm, JF, Jip, Jim, lp, lm);
        for (int k = 0; k < 3; ++k) sGe[t][k] = nrm[k];
        for (int k = 0; k < 9; ++k) {
            sGe[t][4 + k] = Jip[k / 3][k % 3];
            sGe[t][13 + k] = Jim[k / 3][k % 3];
        }
        sGe[t][3] = JF;
        sGe[t][22] = lp;
        sGe[t][23] = lm;
        sGe[t][24] = tb.w[qt1] * tb.w[qt2] * JF;
    }
    __syncthreads();
    for (int c0 = 0; c0 < NBC; c0 += CB) {
        if (t < CB * NF) {
            const int col = c0 + t / NF, fq = t % NF;
            if (col < NBC) {
                const int beta = col / NVC, jm = col % NVC;
                const int qt1 = fq / N, qt2 = fq % N;
                double bv, bg[3];
                face_basis<N>(tb, d, 1 - s, qt1, qt2, sInv[jm], bv, bg);
                Dual up[5], gxp[5][3], um[5], gxm[5][3];
                for (int a = 0; a < 5; ++a) {
                    up[a] = Dual(sPr[fq][a], 0.0);
                    um[a] = Dual(sPr[fq][20 + a], a == beta ? bv : 0.0);
                    for (int k = 0; k < 3; ++k) {
                        gxp[a][k] = Dual(sPr[fq][5 + a * 3 + k], 0.0);
                        gxm[a][k] = Dual(sPr[fq][25 + a * 3 + k], a == beta ? bg[k] : 0.0);
                    }
                }
                double nrm[3], Jip[3][3], Jim[3][3];
                for (int k = 0; k < 3; ++k) nrm[k] = sGe[fq][k];
                for (int k = 0; k < 9; ++k) {
                    Jip[k / 3][k % 3] = sGe[fq][4 + k];
                    Jim[k / 3][k % 3] = sGe[fq][13 + k];
                }
                Dual fo[20];
                face_integrand<Dual, NS, FIX_OWN>(up, gxp, um, gxm, nrm, Jip, Jim, sGe[fq][22], sGe[fq][23],
                                                  sGe[fq][24], gas, fo);
                for (int k = 0; k < 20; ++k) sOut[t][k] = fo[k].d;
            }
        }
        __syncthreads();
        for (int idx = t; idx < CB * NBC; idx += 256) {
            const int cc = idx / NBC, row = idx % NBC;
            const int col = c0 + cc;
            if (col >= NBC) continue;
            const int alpha = row / NVC, im = row % NVC;
            const int tq = sInv[im];
            double acc = 0.0;
            for (int fq = 0; fq < NF; ++fq) {
                double bv, bg[3];
                face_basis<N>(tb, d, s, fq / N, fq % N, tq, bv, bg);
                const double* so = sOut[cc * NF + fq];
                acc = fma(bv, so[alpha], acc);
                acc = fma(bg[0], so[5 + alpha * 3 + 0], acc);
                acc = fma(bg[1], so[5 + alpha * 3 + 1], acc);
                acc = fma(bg[2], so[5 + alpha * 3 + 2], acc);
            }
            ob[(size_t)col * NBC + row] = acc;
        }
        __syncthreads();
    }
}

namespace {
template <int P, int PC>
hipError_t launch_offdiag_pc(const DGArgs& a, const double* W, double* out, hipStream_t s) {
    dim3 grid(a.m.ne, 6), block(256);
    const bool curved = a.m.vtx != nullptr;
    if (a.ns) {
        if (curved) hipLaunchKernelGGL((offdiag_kernel<P, PC, true, true>), grid, block, 0, s, a.m, a.g, W, out);
        else hipLaunchKernelGGL((offdiag_kernel<P, PC, true, false>), grid, block, 0, s, a.m, a.g, W, out);
    } else {
        if (curved) hipLaunchKernelGGL((offdiag_kernel<P, PC, false, true>), grid, block, 0, s, a.m, a.g, W, out);
        else hipLaunchKernelGGL((offdiag_kernel<P, PC, false, false>), grid, block, 0, s, a.m, a.g, W, out);
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_offdiag_blocks(const DGArgs& a, const double* W, int pc, double* out, hipStream_t s) {
    switch (a.p * 10 + pc) {
        case 21: return launch_offdiag_pc<2, 1>(a, W, out, s);
        case 31: return launch_offdiag_pc<3, 1>(a, W, out, s);
        case 32: return launch_offdiag_pc<3, 2>(a, W, out, s);
        case 41: return launch_offdiag_pc<4, 1>(a, W, out, s);
        case 42: return launch_offdiag_pc<4, 2>(a, W, out, s);
        case 43: return launch_offdiag_pc<4, 3>(a, W, out, s);
        // pc = p: the face-coupling blocks of the fine operator itself
        case 11: return launch_offdiag_pc<1, 1>(a, W, out, s);
        case 22: return launch_offdiag_pc<2, 2>(a, W, out, s);
        case 33: return launch_offdiag_pc<3, 3>(a, W, out, s);
        case 44: return launch_offdiag_pc<4, 4>(a, W, out, s);
        default: return hipErrorInvalidValue;
    }
}

// ---- assembled coarse operator: sliced row-major block-sparse product ----------------------
// y_e = D_e x_e + sum_f O_{e,f} x_nb(e,f), 7 blocks per element row.  Storage:
// global row g = e nbc + r holds the row r of the 7 blocks of element e, each
// padded to ldr = roundup(nbc, 8) entries (zeros); rows are grouped by 64 (one
// wavefront) and within a group stored chunk-major: chunk k (16 bytes of the
// row) of the 64 rows is contiguous, so each 16-byte load of a wavefront is
// one contiguous 1 KB read.  Entries are FP64, FP32 or BF16 (RNE); products
// accumulate in FP64 (FP64/FP32 storage) or FP32 (BF16 storage).  The x
// blocks an element's rows need are staged in LDS once per workgroup.
__device__ __forceinline__ unsigned short bf16_rne(double v) {
    const unsigned int b = __float_as_uint((float)v);
    return (unsigned short)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
template <class SF>
__device__ __forceinline__ SF to_storage(double v) { return (SF)v; }
template <>
__device__ __forceinline__ unsigned short to_storage<unsigned short>(double v) { return bf16_rne(v); }

template <class SF>
__global__ void __launch_bounds__(256) bsr_pack_kernel(int ne, int nbc, int nblk, const double* __restrict__ diag,
                                                       const double* __restrict__ off, SF* __restrict__ out) {
    constexpr int W = 16 / sizeof(SF);
    const int ldr = bsr_ldr(nbc);
    const size_t nrows = (size_t)ne * nbc;
    const size_t total = bsr_entries(ne, nbc, nblk);
    const int nk = nblk * ldr / W;                  // 16-byte chunks per row
    const int f0 = 7 - nblk;                        // 0: slot 0 is the diagonal block; 1: faces only
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int j = (int)(i % W);
        const size_t t = i / W;
        const int lane = (int)(t % 64);
        const size_t t2 = t / 64;
        const int kc = (int)(t2 % nk);
        const size_t grp = t2 / nk;
        const size_t g = grp * 64 + lane;
        double v = 0.0;
        if (g < nrows) {
            const size_t e = g / nbc;
            const int r = (int)(g % nbc);
            const int k = kc * W + j, f = k / ldr + f0, c = k % ldr;
            if (c < nbc)
                v = (f == 0) ? diag[(e * nbc + c) * nbc + r] : off[((e * 6 + (f - 1)) * nbc + c) * nbc + r];
        }
        out[i] = to_storage<SF>(v);
    }
}

template <class SF, class AT>
__device__ __forceinline__ void bsr_chunk(const SF* p, const AT* xv, AT& acc);
template <>
__device__ __forceinline__ void bsr_chunk<double, double>(const double* p, const double* xv, double& acc) {
    // FP64 operators exceed the last-level cache: streamed with nontemporal
    // loads so the gathered vectors and the Krylov basis stay cached
    typedef double d2v __attribute__((ext_vector_type(2)));
    const d2v a = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
    acc = fma(a.x, xv[0], acc);
    acc = fma(a.y, xv[1], acc);
}
template <>
__device__ __forceinline__ void bsr_chunk<float, double>(const float* p, const double* xv, double& acc) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    acc = fma((double)a.x, xv[0], acc);
    acc = fma((double)a.y, xv[1], acc);
    acc = fma((double)a.z, xv[2], acc);
    acc = fma((double)a.w, xv[3], acc);
}
template <>
__device__ __forceinline__ void bsr_chunk<unsigned short, float>(const unsigned short* p, const float* xv,
                                                                  float& acc) {
    const uint4 a = *reinterpret_cast<const uint4*>(p);
    const unsigned int w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        acc = fmaf(__uint_as_float(w[q] << 16), xv[2 * q], acc);
        acc = fmaf(__uint_as_float(w[q] & 0xFFFF0000u), xv[2 * q + 1], acc);
    }
}

// y = K x, row g per thread.  UNIT: the stored blocks are the six face blocks
// and the diagonal block is the identity (y = x + sum of the face terms, the
// identity term added in FP64).
template <class SF, class AT, bool UNIT, bool DOTS = false>
__global__ void __launch_bounds__(256) bsr_rows_kernel(MeshDev m, int nbc, const SF* __restrict__ A,
                                                       const double* __restrict__ x, double* __restrict__ y,
                                                       const double* __restrict__ Vb = nullptr, int k = 0,
                                                       double* __restrict__ part = nullptr) {
    constexpr int NBLK = UNIT ? 6 : 7;
    extern __shared__ double smraw[];
    AT* xs = reinterpret_cast<AT*>(smraw);          // [element in range][NBLK][ldr]
    constexpr int W = 16 / sizeof(SF);
    const int ldr = bsr_ldr(nbc);
    const size_t nrows = (size_t)m.ne * nbc;
    const size_t g0 = (size_t)blockIdx.x * blockDim.x;
    const size_t glast = min(g0 + blockDim.x, nrows) - 1;
    const int e_first = (int)(g0 / nbc);
    const int nel = (int)(glast / nbc) - e_first + 1;
    const size_t g = g0 + threadIdx.x;
    // the row's entries of the first DOTS_PRE basis vectors, requested before
    // the gather so that their latency overlaps the product (the Arnoldi
    // dots at the end otherwise start with a cold round trip)
    constexpr int DOTS_PRE = 16;
    double vpre[DOTS_PRE];
    if constexpr (DOTS) {
#pragma unroll
        for (int c = 0; c < DOTS_PRE; ++c) vpre[c] = (g < nrows && c < k) ? Vb[(size_t)c * nrows + g] : 0.0;
    }
    for (int i = threadIdx.x; i < nel * NBLK * ldr; i += blockDim.x) {
        const int c = i % ldr, t = i / ldr, f = t % NBLK, le = t / NBLK;
        const int e = e_first + le;
        const int src = UNIT ? nbr_of(m, e, f) : ((f == 0) ? e : nbr_of(m, e, f - 1));
        xs[i] = (c < nbc) ? (AT)x[(size_t)src * nbc + c] : (AT)0;
    }
    __syncthreads();
    double yg = 0.0;
    if (g < nrows) {
        const int e = (int)(g / nbc);
        const AT* xe = xs + (size_t)(e - e_first) * NBLK * ldr;
        const int nk = NBLK * ldr / W;
        const SF* base = A + ((g / 64) * (size_t)nk * 64 + (g % 64)) * W;
        // four independent accumulators over interleaved chunks (loads of an
        // unrolled group in flight together), added in a fixed order
        AT acc[4] = {0, 0, 0, 0};
        int kc = 0;
        for (; kc + 4 <= nk; kc += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                bsr_chunk<SF, AT>(base + (size_t)(kc + u) * 64 * W, xe + (kc + u) * W, acc[u]);
        }
        for (; kc < nk; ++kc) bsr_chunk<SF, AT>(base + (size_t)kc * 64 * W, xe + kc * W, acc[0]);
        const AT sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        yg = UNIT ? x[g] + (double)sum : (double)sum;
        y[g] = yg;
    }
    if constexpr (DOTS) {
        // first Gram-Schmidt pass of the Arnoldi step on this block's rows
        constexpr int CH = 16;
        static_assert(CH == DOTS_PRE, "the first chunk is the prefetched one");
        __shared__ double sh[4 * CH];
        for (int c0 = 0; c0 < k; c0 += CH) {
            double dv[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c)
                dv[c] = (c0 == 0) ? vpre[c] * yg
                                  : ((g < nrows && c0 + c < k) ? Vb[(size_t)(c0 + c) * nrows + g] * yg : 0.0);
            block_sum_cols<CH>(dv, min(CH, k - c0), sh, part + (size_t)c0 * gridDim.x + blockIdx.x, gridDim.x);
        }
    }
}

template <class SF>
hipError_t launch_bsr_pack(const double* diag, const double* off, SF* out, int ne, int nbc, int nblk, hipStream_t s) {
    if (nblk != 6 && nblk != 7) return hipErrorInvalidValue;
    const size_t total = bsr_entries(ne, nbc, nblk);
    const unsigned grid = (unsigned)std::min<size_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(bsr_pack_kernel<SF>, dim3(grid), dim3(256), 0, s, ne, nbc, nblk, diag, off, out);
    return hipGetLastError();
}

template <class SF>
hipError_t launch_bsr7(const DGArgs& a, const SF* A, const double* x, double* y, int nbc, hipStream_t s) {
    using AT = typename std::conditional<std::is_same<SF, unsigned short>::value, float, double>::type;
    const size_t nrows = (size_t)a.m.ne * nbc;
    const unsigned grid = (unsigned)((nrows + 255) / 256);
    const size_t lds = (size_t)(256 / nbc + 2) * 7 * bsr_ldr(nbc) * sizeof(AT);
    if (lds > 65536) {      // fine-order blocks (nbc = 625): the gathered neighbour values exceed 64 KB
        const hipError_t e = hipFuncSetAttribute((const void*)bsr_rows_kernel<SF, AT, false>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((bsr_rows_kernel<SF, AT, false>), dim3(grid), dim3(256), lds, s, a.m, nbc, A, x, y);
    return hipGetLastError();
}

template <class SF>
hipError_t launch_bsr_unit(const DGArgs& a, const SF* A, const double* x, double* y, int nbc, hipStream_t s) {
    using AT = typename std::conditional<std::is_same<SF, unsigned short>::value, float, double>::type;
    const size_t nrows = (size_t)a.m.ne * nbc;
    const unsigned grid = (unsigned)((nrows + 255) / 256);
    const size_t lds = (size_t)(256 / nbc + 2) * 6 * bsr_ldr(nbc) * sizeof(AT);
    hipLaunchKernelGGL((bsr_rows_kernel<SF, AT, true>), dim3(grid), dim3(256), lds, s, a.m, nbc, A, x, y);
    return hipGetLastError();
}

int bsr_grid(int ne, int nbc) { return (int)(((size_t)ne * nbc + 255) / 256); }

template <class SF>
hipError_t launch_bsr_unit_dots(const DGArgs& a, const SF* A, const double* x, double* y, int nbc, const double* Vb,
                                int k, double* part, int* np, hipStream_t s) {
    using AT = typename std::conditional<std::is_same<SF, unsigned short>::value, float, double>::type;
    const unsigned grid = (unsigned)bsr_grid(a.m.ne, nbc);
    const size_t lds = (size_t)(256 / nbc + 2) * 6 * bsr_ldr(nbc) * sizeof(AT);
    hipLaunchKernelGGL((bsr_rows_kernel<SF, AT, true, true>), dim3(grid), dim3(256), lds, s, a.m, nbc, A, x, y, Vb, k,
                       part);
    *np = (int)grid;
    return hipGetLastError();
}
template hipError_t launch_bsr_unit_dots<double>(const DGArgs&, const double*, const double*, double*, int,
                                                 const double*, int, double*, int*, hipStream_t);
template hipError_t launch_bsr_unit_dots<float>(const DGArgs&, const float*, const double*, double*, int,
                                                const double*, int, double*, int*, hipStream_t);
template hipError_t launch_bsr_unit_dots<unsigned short>(const DGArgs&, const unsigned short*, const double*, double*,
                                                         int, const double*, int, double*, int*, hipStream_t);

// Right-preconditioned coarse operator K D^-1: every face block K_{e,f} is
// replaced by K_{e,f} X_{nb(e,f)}, X the neighbour's block-Jacobi inverse (the
// diagonal K_ee X_e is the identity).  In place, column-major nbc x nbc,
// one workgroup per (element, face), nbc <= FOLD_MAX_N.
template <class TX>
__global__ void __launch_bounds__(256) fold_inverse_kernel(MeshDev m, int nbc, double* __restrict__ off,
                                                           const TX* __restrict__ X) {
    __shared__ double sk[FOLD_MAX_N * FOLD_MAX_N];
    const int e = blockIdx.x / 6, f = blockIdx.x % 6;
    const size_t nn = (size_t)nbc * nbc;
    double* K = off + ((size_t)e * 6 + f) * nn;
    const TX* Xn = X + (size_t)nbr_of(m, e, f) * nn;
    for (int i = threadIdx.x; i < (int)nn; i += blockDim.x) sk[i] = K[i];
    __syncthreads();
    for (int i = threadIdx.x; i < (int)nn; i += blockDim.x) {
        const int r = i % nbc, c = i / nbc;
        const TX* xc = Xn + (size_t)c * nbc;
        double acc = 0.0;
        for (int k = 0; k < nbc; ++k) acc = fma(sk[k * nbc + r], (double)xc[k], acc);
        K[i] = acc;
    }
}

template <class TX>
hipError_t launch_fold_inverse(const DGArgs& a, int nbc, double* off, const TX* X, hipStream_t s) {
    if (nbc < 1 || nbc > FOLD_MAX_N) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fold_inverse_kernel<TX>, dim3((unsigned)a.m.ne * 6), dim3(256), 0, s, a.m, nbc, off, X);
    return hipGetLastError();
}
template hipError_t launch_fold_inverse<double>(const DGArgs&, int, double*, const double*, hipStream_t);
template hipError_t launch_fold_inverse<float>(const DGArgs&, int, double*, const float*, hipStream_t);
template hipError_t launch_bsr_unit<double>(const DGArgs&, const double*, const double*, double*, int, hipStream_t);
template hipError_t launch_bsr_unit<float>(const DGArgs&, const float*, const double*, double*, int, hipStream_t);
template hipError_t launch_bsr_unit<unsigned short>(const DGArgs&, const unsigned short*, const double*, double*,
                                                    int, hipStream_t);
template hipError_t launch_bsr_pack<double>(const double*, const double*, double*, int, int, int, hipStream_t);
template hipError_t launch_bsr_pack<float>(const double*, const double*, float*, int, int, int, hipStream_t);
template hipError_t launch_bsr_pack<unsigned short>(const double*, const double*, unsigned short*, int, int, int,
                                                    hipStream_t);
template hipError_t launch_bsr7<double>(const DGArgs&, const double*, const double*, double*, int, hipStream_t);
template hipError_t launch_bsr7<float>(const DGArgs&, const float*, const double*, double*, int, hipStream_t);
template hipError_t launch_bsr7<unsigned short>(const DGArgs&, const unsigned short*, const double*, double*, int,
                                                hipStream_t);

// ---- element diagonal blocks (Sec. 6.3) ------------------------------------------------------
// Column j = (beta, mode) of K_e = a M_e + dR_e/dW_e is the forward-mode
// derivative of the element residual when only W_e[beta][mode] moves.  The
// neighbours' traces do not move, so they are evaluated once per element
// (nbr_trace_kernel) and read as plain values; the own tangent is the basis
// function itself (value and reference gradient from the 1D tables); only
// tangent parts are carried through the face integrands and the test.
template <int P>
__global__ void __launch_bounds__(256) nbr_trace_kernel(MeshDev m, const double* __restrict__ W,
                                                        double* __restrict__ out) {
    constexpr int N = P + 1, NQ = N * N * N, NF = N * N, NB = 5 * NQ;
    const Tab& tb = c_tab[P];
    const short* perm = c_perm + perm_offset(P);
    const int e = blockIdx.x, t = threadIdx.x;
    if (t >= 6 * NF) return;
    const int f = t / NF, fq = t % NF;
    const int d = f >> 1, s = f & 1;
    const int nb = nbr_of(m, e, f);
    const double* wn = W + (size_t)nb * NB;
    double acc[20];
    for (int k = 0; k < 20; ++k) acc[k] = 0.0;
    for (int q = 0; q < NQ; ++q) {
        double bv, bg[3];
        face_basis<N>(tb, d, 1 - s, fq / N, fq % N, q, bv, bg);
        const int pm = perm[q];
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            const double w = wn[a * NQ + pm];
            acc[a] = fma(bv, w, acc[a]);
            acc[5 + a * 3 + 0] = fma(bg[0], w, acc[5 + a * 3 + 0]);
            acc[5 + a * 3 + 1] = fma(bg[1], w, acc[5 + a * 3 + 1]);
            acc[5 + a * 3 + 2] = fma(bg[2], w, acc[5 + a * 3 + 2]);
        }
    }
    double* o = out + (((size_t)e * 6 + f) * NF + fq) * 20;
    for (int k = 0; k < 20; ++k) o[k] = acc[k];
}

template <int P>
struct SzD {
    static constexpr int N = P + 1, NQ = N * N * N, NF = N * N;
    static constexpr int OFF_U = 20 * NQ;                 // [0, 20NQ): interpolation | face tangents of a round | test A/B
    static constexpr int OFF_G = OFF_U + 5 * NQ;          // Gauss values (5NQ), reference gradients (15NQ)
    static constexpr int OFF_H = OFF_G + 15 * NQ;         // test-back sweeps (15 NQ)
    static constexpr int TOT = OFF_H + 15 * NQ;
};
template <int P> struct LaunchD { static constexpr int EPB = (P == 1) ? 8 : ((P == 2) ? 2 : 1); };

// SELF: some axis has a single element, so a face's neighbour can be the
// element itself and its trace moves with the column; otherwise the
// neighbour traces are fixed and their half of the viscous average is skipped.
template <int P, bool NS, bool CURVED, bool SELF>
__global__ void __launch_bounds__((LaunchD<P>::EPB * SzD<P>::NQ))
    diag_kernel(MeshDev m, Gas gas, const double* __restrict__ W, const double* __restrict__ nbrtr, double shift,
                double* __restrict__ out, int ld) {
    using S_ = SzD<P>;
    constexpr int N = S_::N, NQ = S_::NQ, NF = S_::NF, NB = 5 * NQ;
    constexpr int EPB = LaunchD<P>::EPB;
    __shared__ double smem[EPB * S_::TOT];
    __shared__ double sdet[EPB][NQ];
    __shared__ double svtx[EPB][24];
    const Tab& tb = c_tab[P];
    const short* perm = c_perm + perm_offset(P);
    const int es = threadIdx.x / NQ, q = threadIdx.x % NQ;
    const int e = blockIdx.x * EPB + es;
    const bool active = e < m.ne;
    const int col = blockIdx.y;
    const int beta = col / NQ, hj = col % NQ;
    double* S = smem + es * S_::TOT;
    const int ii[3] = {q / NF, (q / N) % N, q % N};
    // tensor mode of column j (hierarchical index hj)
    __shared__ int stj;
    if (threadIdx.x < NQ && perm[threadIdx.x] == hj) stj = threadIdx.x;
    if (active) {
        const size_t base = (size_t)e * NB;
        const int pm = perm[q];
        for (int a = 0; a < 5; ++a) S[a * NQ + q] = W[base + a * NQ + pm];
        if constexpr (CURVED)
            for (int k = q; k < 24; k += NQ) svtx[es][k] = m.vtx[(size_t)e * 24 + k];
    }
    __syncthreads();
    const int tj = stj;
    const int jj[3] = {tj / NF, (tj / N) % N, tj % N};
    double* X1 = S + 5 * NQ;
    double* X2 = S + 10 * NQ;
    double* su = S + S_::OFF_U;
    double* sg = S + S_::OFF_G;
    if (active) sweep<N, 5, false>(tb.V, S, X1, 0, ii, q);
    __syncthreads();
    if (active) sweep<N, 5, false>(tb.V, X1, X2, 1, ii, q);
    __syncthreads();
    if (active) sweep<N, 5, false>(tb.V, X2, su, 2, ii, q);
    __syncthreads();
    double Ad[5][3], Bd[5];
    double detJ = 1.0, Ji[3][3];
    const double hx = m.h[0], hy = m.h[1], hz = m.h[2];
    if (active) {
        Dual u[5], gx[5][3];
        // tangent of column j at this Gauss point: phi_j and its reference gradient
        const double p0 = tb.V[ii[0]][jj[0]], p1 = tb.V[ii[1]][jj[1]], p2 = tb.V[ii[2]][jj[2]];
        const double phi = p0 * p1 * p2;
        const double dphi[3] = {tb.Vd[ii[0]][jj[0]] * p1 * p2, p0 * tb.Vd[ii[1]][jj[1]] * p2,
                                p0 * p1 * tb.Vd[ii[2]][jj[2]]};
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            u[a] = Dual(su[a * NQ + q], a == beta ? phi : 0.0);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) acc = fma(tb.D[ii[k]][j], su[a * NQ + tix_dir<N>(k, j, ii)], acc);
                gx[a][k] = Dual(acc, a == beta ? dphi[k] : 0.0);
                sg[(a * 3 + k) * NQ + q] = acc;
            }
        }
        if constexpr (CURVED) {
            double J[3][3];
            q1_jac(svtx[es], tb.z[ii[0]], tb.z[ii[1]], tb.z[ii[2]], J);
            detJ = q1_inv(J, Ji);
            sdet[es][q] = detJ;
        } else {
            detJ = 0.125 * hx * hy * hz;
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int d = 0; d < 3; ++d) Ji[k][d] = 0.0;
            Ji[0][0] = 2.0 / hx;
            Ji[1][1] = 2.0 / hy;
            Ji[2][2] = 2.0 / hz;
        }
        const double wq = tb.w[ii[0]] * tb.w[ii[1]] * tb.w[ii[2]];
        Dual F[5][3];
        flux_c(u, gas.gamma - 1.0, F);
        if constexpr (NS) {
            Dual g[5][3];
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    g[a][j] = Ji[0][j] * gx[a][0] + Ji[1][j] * gx[a][1] + Ji[2][j] * gx[a][2];
            flux_v_acc(u, g, gas, 1.0, F);
        }
        const double c = -wq * detJ;
#pragma unroll
        for (int a = 0; a < 5; ++a) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                Ad[a][k] = c * (Ji[k][0] * F[a][0].d + Ji[k][1] * F[a][1].d + Ji[k][2] * F[a][2].d);
            Bd[a] = (a == beta) ? shift * wq * detJ * phi : 0.0;
        }
    }
    __syncthreads();
    // rounds of NQ face points (N whole faces), tangents in [0, 20 NQ), spread per round
    double* sF = S;
    for (int r = 0; r * NQ < 6 * NF; ++r) {
        const int fp = r * NQ + q;
        if (active && fp < 6 * NF) {
            const int f = fp / NF, fq = fp % NF;
            const int d = f >> 1, s = f & 1;
            const int t1 = (d == 0) ? 1 : 0;
            const int qt1 = fq / N, qt2 = fq % N;
            const int sd = (d == 0) ? NF : ((d == 1) ? N : 1);
            const int st1 = (d == 0) ? N : NF, st2 = (d == 2) ? N : 1;
            const int tl = qt1 * st1 + qt2 * st2;
            const int nb = nbr_of(m, e, f);
            Dual up[5], gxp[5][3], um[5], gxm[5][3];
            double bvp, bgp[3];
            face_basis<N>(tb, d, s, qt1, qt2, tj, bvp, bgp);
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                double v0 = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const int tt = tl + k * sd;
                    const double l = tb.lag[s][k];
                    v0 = fma(l, su[a * NQ + tt], v0);
                    g0 = fma(l, sg[(a * 3 + 0) * NQ + tt], g0);
                    g1 = fma(l, sg[(a * 3 + 1) * NQ + tt], g1);
                    g2 = fma(l, sg[(a * 3 + 2) * NQ + tt], g2);
                }
                const bool on = a == beta;
                up[a] = Dual(v0, on ? bvp : 0.0);
                gxp[a][0] = Dual(g0, on ? bgp[0] : 0.0);
                gxp[a][1] = Dual(g1, on ? bgp[1] : 0.0);
                gxp[a][2] = Dual(g2, on ? bgp[2] : 0.0);
            }
            const bool self_nb = SELF && nb == e;
            if (self_nb) {
                // one-element periodic axis: the neighbour trace is this element's
                // trace on the opposite face, and it moves with W_e
                double bvm, bgm[3];
                face_basis<N>(tb, d, 1 - s, qt1, qt2, tj, bvm, bgm);
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    double v0 = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
                    for (int k = 0; k < N; ++k) {
                        const int tt = tl + k * sd;
                        const double l = tb.lag[1 - s][k];
                        v0 = fma(l, su[a * NQ + tt], v0);
                        g0 = fma(l, sg[(a * 3 + 0) * NQ + tt], g0);
                        g1 = fma(l, sg[(a * 3 + 1) * NQ + tt], g1);
                        g2 = fma(l, sg[(a * 3 + 2) * NQ + tt], g2);
                    }
                    const bool on = a == beta;
                    um[a] = Dual(v0, on ? bvm : 0.0);
                    gxm[a][0] = Dual(g0, on ? bgm[0] : 0.0);
                    gxm[a][1] = Dual(g1, on ? bgm[1] : 0.0);
                    gxm[a][2] = Dual(g2, on ? bgm[2] : 0.0);
                }
            } else {
                const double* nt = nbrtr + (((size_t)e * 6 + f) * NF + fq) * 20;
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    um[a] = Dual(nt[a], 0.0);
#pragma unroll
                    for (int k = 0; k < 3; ++k) gxm[a][k] = Dual(nt[5 + a * 3 + k], 0.0);
                }
            }
            double nrm[3], JF, Jip[3][3], Jim[3][3], lam_p, lam_m;
            if constexpr (CURVED) {
                face_geometry<P, true>(tb, m, e, f, qt1, qt2, nrm, JF, Jip, Jim, lam_p, lam_m);
            } else {
                face_geometry<P, false>(tb, m, e, f, qt1, qt2, nrm, JF, Jip, Jim, lam_p, lam_m);
            }
            (void)t1;
            Dual fo[20];
            if constexpr (SELF) {
                if (self_nb)
                    face_integrand<Dual, NS>(up, gxp, um, gxm, nrm, Jip, Jim, lam_p, lam_m,
                                             tb.w[qt1] * tb.w[qt2] * JF, gas, fo);
                else
                    face_integrand<Dual, NS, FIX_NBR>(up, gxp, um, gxm, nrm, Jip, Jim, lam_p, lam_m,
                                                      tb.w[qt1] * tb.w[qt2] * JF, gas, fo);
            } else {
                face_integrand<Dual, NS, FIX_NBR>(up, gxp, um, gxm, nrm, Jip, Jim, lam_p, lam_m,
                                                  tb.w[qt1] * tb.w[qt2] * JF, gas, fo);
            }
            double* so = sF + q * 20;
#pragma unroll
            for (int k = 0; k < 20; ++k) so[k] = fo[k].d;
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int fl = 0; fl < N; ++fl) {
                const int f = r * N + fl;
                if (f >= 6) break;
                const int d = f >> 1, s = f & 1;
                const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
                const double l = tb.lag[s][ii[d]];
                const double* fo = sF + (fl * NF + ii[t1] * N + ii[t2]) * 20;
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    Bd[a] = fma(l, fo[a], Bd[a]);
                    if constexpr (NS) {
#pragma unroll
                        for (int k = 0; k < 3; ++k) Ad[a][k] = fma(l, fo[5 + a * 3 + k], Ad[a][k]);
                    }
                }
            }
        }
        __syncthreads();
    }
    double* sA = S;
    double* sB = S + 15 * NQ;
    double* H = S + S_::OFF_H;
    double* Y1 = S + S_::OFF_U;         // Gauss values no longer needed
    double* Y2 = S + S_::OFF_G;
    if (active) {
#pragma unroll
        for (int a = 0; a < 5; ++a) {
#pragma unroll
            for (int k = 0; k < 3; ++k) sA[(a * 3 + k) * NQ + q] = Ad[a][k];
            sB[a * NQ + q] = Bd[a];
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            double acc = sB[a * NQ + q];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int j = 0; j < N; ++j)
                    acc = fma(tb.D[j][ii[k]], sA[(a * 3 + k) * NQ + tix_dir<N>(k, j, ii)], acc);
            H[a * NQ + q] = acc;
        }
    }
    __syncthreads();
    if (active) sweep<N, 5, true>(tb.V, H, Y1, 0, ii, q);
    __syncthreads();
    if (active) sweep<N, 5, true>(tb.V, Y1, Y2, 1, ii, q);
    __syncthreads();
    if (active) {
        const int pm = perm[q];
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) acc = fma(tb.V[j][ii[2]], Y2[a * NQ + tix_dir<N>(2, j, ii)], acc);
            out[((size_t)e * NB + col) * ld + a * NQ + pm] = acc;
        }
    }
}

// Diagonal blocks from Jacobian slices (no face couples the element to
// itself).  Column (beta, j) of K_e is the derivative of the element
// residual in the direction of basis function j in variable beta.  That
// residual sees W_e[beta] only through u_beta and its reference gradient at
// the Gauss points and through the own trace's value and reference gradient
// at the face points, and it is linear in each of these directions.  One
// workgroup per (element slot group, beta) therefore takes, once, with dual
// numbers: the derivatives of the volume flux term (15 outputs) with
// respect to u_beta and d u_beta / d xi_m at every Gauss point, and those of
// the face integrand (20 outputs) with respect to the own trace value and,
// for the averaged viscous flux (outputs 0..4, the only ones the gradient
// enters), its reference gradient at every face point: the slices.  Each
// column j is then these slices contracted with basis function j's values
// and reference gradients, spread onto the Gauss lines and tested exactly
// as in the per-column kernel.  Four dual evaluations per point and beta
// instead of one per column.
// LDS per element slot, 35 NQ + the face slices: before the columns, modal
// data and the two interpolation sweeps in [0, 15 NQ), Gauss values at
// OFF_U, reference gradients at OFF_G; for the columns, a round's face
// integrands and then the test inputs A, B in [0, 20 NQ), H and the two test
// sweeps at OFF_H (over the dead values and gradients).  Two workgroups per
// CU at degree 4.
template <int P>
struct SzS {
    static constexpr int N = P + 1, NQ = N * N * N, NF = N * N, NFP = 6 * NF;
    static constexpr int OFF_U = 15 * NQ;        // Gauss values (5NQ)
    static constexpr int OFF_G = 20 * NQ;        // reference gradients (15NQ)
    static constexpr int OFF_H = 20 * NQ;        // H, then the two test sweeps (5NQ each)
    static constexpr int OFF_FS = 35 * NQ;       // face slices, 35 per face point
    static constexpr int TOT = OFF_FS + 35 * NFP;
};
template <int P> struct LaunchS { static constexpr int EPB = (P == 1) ? 4 : ((P == 2) ? 2 : 1); };

template <int P, bool NS, bool CURVED>
__global__ void __launch_bounds__((LaunchS<P>::EPB * SzS<P>::NQ))
    diag_slices_kernel(MeshDev m, Gas gas, const double* __restrict__ W, const double* __restrict__ nbrtr,
                       double shift, double* __restrict__ out, int ld) {
    using S_ = SzS<P>;
    constexpr int N = S_::N, NQ = S_::NQ, NF = S_::NF, NFP = S_::NFP, NB = 5 * NQ;
    constexpr int EPB = LaunchS<P>::EPB;
    constexpr int NDIR = NS ? 4 : 1;         // u_beta, then d u_beta / d xi_m (viscous terms only)
    extern __shared__ double dsm[];
    __shared__ double svtx[EPB][24];
    __shared__ short sinv[NQ];              // tensor index of hierarchical mode
    const Tab& tb = c_tab[P];
    const short* perm = c_perm + perm_offset(P);
    const int es = threadIdx.x / NQ, q = threadIdx.x % NQ;
    const int e = blockIdx.x * EPB + es;
    const bool active = e < m.ne;
    const int beta = blockIdx.y;
    double* S = dsm + (size_t)es * S_::TOT;
    double* FS = S + S_::OFF_FS;
    const int ii[3] = {q / NF, (q / N) % N, q % N};
    if (threadIdx.x < NQ) sinv[perm[threadIdx.x]] = (short)threadIdx.x;
    if (active) {
        const size_t base = (size_t)e * NB;
        const int pm = perm[q];
        for (int a = 0; a < 5; ++a) S[a * NQ + q] = W[base + a * NQ + pm];
        if constexpr (CURVED)
            for (int k = q; k < 24; k += NQ) svtx[es][k] = m.vtx[(size_t)e * 24 + k];
    }
    __syncthreads();
    double* X1 = S + 5 * NQ;
    double* X2 = S + 10 * NQ;
    double* su = S + S_::OFF_U;
    double* sg = S + S_::OFF_G;
    if (active) sweep<N, 5, false>(tb.V, S, X1, 0, ii, q);
    __syncthreads();
    if (active) sweep<N, 5, false>(tb.V, X1, X2, 1, ii, q);
    __syncthreads();
    if (active) sweep<N, 5, false>(tb.V, X2, su, 2, ii, q);
    __syncthreads();
    // ---- reference gradients at the Gauss points (LDS, for the own traces)
    if (active) {
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) acc = fma(tb.D[ii[k]][j], su[a * NQ + tix_dir<N>(k, j, ii)], acc);
                sg[(a * 3 + k) * NQ + q] = acc;
            }
    }
    __syncthreads();
    // ---- face slices (LDS): per face point fs[0..19] (value direction),
    // fs[20 + 5 (m - 1) + o] (reference-gradient direction m, outputs o < 5)
    for (int r = 0; r * NQ < NFP; ++r) {
        const int fp = r * NQ + q;
        if (active && fp < NFP) {
            const int f = fp / NF, fq = fp % NF;
            const int d = f >> 1, s = f & 1;
            const int qt1 = fq / N, qt2 = fq % N;
            const int sd = (d == 0) ? NF : ((d == 1) ? N : 1);
            const int st1 = (d == 0) ? N : NF, st2 = (d == 2) ? N : 1;
            const int tl = qt1 * st1 + qt2 * st2;
            double upv[5], gpv[5][3], umv[5], gmv[5][3];
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                double v0 = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const int tt = tl + k * sd;
                    const double l = tb.lag[s][k];
                    v0 = fma(l, su[a * NQ + tt], v0);
                    g0 = fma(l, sg[(a * 3 + 0) * NQ + tt], g0);
                    g1 = fma(l, sg[(a * 3 + 1) * NQ + tt], g1);
                    g2 = fma(l, sg[(a * 3 + 2) * NQ + tt], g2);
                }
                upv[a] = v0;
                gpv[a][0] = g0;
                gpv[a][1] = g1;
                gpv[a][2] = g2;
            }
            const double* nt = nbrtr + (((size_t)e * 6 + f) * NF + fq) * 20;
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                umv[a] = nt[a];
#pragma unroll
                for (int k = 0; k < 3; ++k) gmv[a][k] = nt[5 + a * 3 + k];
            }
            double nrm[3], JF, Jip[3][3], Jim[3][3], lam_p, lam_m;
            face_geometry<P, CURVED>(tb, m, e, f, qt1, qt2, nrm, JF, Jip, Jim, lam_p, lam_m);
            const double sc = tb.w[qt1] * tb.w[qt2] * JF;
            double* fs = FS + (size_t)fp * 35;
#pragma unroll 1
            for (int dir = 0; dir < NDIR; ++dir) {
                Dual up[5], gxp[5][3], um[5], gxm[5][3];
#pragma unroll
                for (int a = 0; a < 5; ++a) {
                    up[a] = Dual(upv[a], (a == beta && dir == 0) ? 1.0 : 0.0);
                    um[a] = Dual(umv[a], 0.0);
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        gxp[a][k] = Dual(gpv[a][k], (a == beta && dir == k + 1) ? 1.0 : 0.0);
                        gxm[a][k] = Dual(gmv[a][k], 0.0);
                    }
                }
                Dual fo[20];
                face_integrand<Dual, NS, FIX_NBR>(up, gxp, um, gxm, nrm, Jip, Jim, lam_p, lam_m, sc, gas, fo);
                if (dir == 0) {
#pragma unroll
                    for (int o = 0; o < (NS ? 20 : 5); ++o) fs[o] = fo[o].d;
                } else {
#pragma unroll
                    for (int o = 0; o < 5; ++o) fs[20 + 5 * (dir - 1) + o] = fo[o].d;
                }
            }
        }
    }
    __syncthreads();
    // ---- volume slices (registers, live only from here on): vs[dir][a][k]
    double vs[NDIR][5][3];
    double wdet = 0.0;
    if (active) {
        double uv[5], gv[5][3];
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            uv[a] = su[a * NQ + q];
#pragma unroll
            for (int k = 0; k < 3; ++k) gv[a][k] = sg[(a * 3 + k) * NQ + q];
        }
        double detJ, Ji[3][3];
        if constexpr (CURVED) {
            double J[3][3];
            q1_jac(svtx[es], tb.z[ii[0]], tb.z[ii[1]], tb.z[ii[2]], J);
            detJ = q1_inv(J, Ji);
        } else {
            const double hx = m.h[0], hy = m.h[1], hz = m.h[2];
            detJ = 0.125 * hx * hy * hz;
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int d = 0; d < 3; ++d) Ji[k][d] = 0.0;
            Ji[0][0] = 2.0 / hx;
            Ji[1][1] = 2.0 / hy;
            Ji[2][2] = 2.0 / hz;
        }
        const double wq = tb.w[ii[0]] * tb.w[ii[1]] * tb.w[ii[2]];
        wdet = wq * detJ;
        const double c = -wq * detJ;
#pragma unroll
        for (int dir = 0; dir < NDIR; ++dir) {
            Dual u[5], gx[5][3];
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                u[a] = Dual(uv[a], (a == beta && dir == 0) ? 1.0 : 0.0);
#pragma unroll
                for (int k = 0; k < 3; ++k) gx[a][k] = Dual(gv[a][k], (a == beta && dir == k + 1) ? 1.0 : 0.0);
            }
            Dual F[5][3];
            flux_c(u, gas.gamma - 1.0, F);
            if constexpr (NS) {
                Dual g[5][3];
#pragma unroll
                for (int a = 0; a < 5; ++a)
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        g[a][j] = Ji[0][j] * gx[a][0] + Ji[1][j] * gx[a][1] + Ji[2][j] * gx[a][2];
                flux_v_acc(u, g, gas, 1.0, F);
            }
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    vs[dir][a][k] = c * (Ji[k][0] * F[a][0].d + Ji[k][1] * F[a][1].d + Ji[k][2] * F[a][2].d);
        }
    }
    __syncthreads();
    // ---- columns (beta, hj): slices times basis function hj, spread, test
    double* sF = S;                     // one round's face integrands, 20 per face point
    double* sA = S;
    double* sB = S + 15 * NQ;
    double* H = S + S_::OFF_H;          // Gauss values and gradients no longer needed
    double* Y1 = H + 5 * NQ;
    double* Y2 = Y1 + 5 * NQ;
#pragma unroll 1
    for (int hj = 0; hj < NQ; ++hj) {
        const int tj = sinv[hj];
        const int jj[3] = {tj / NF, (tj / N) % N, tj % N};
        const int col = beta * NQ + hj;
        double Ad[5][3], Bd[5];
        if (active) {
            const double p0 = tb.V[ii[0]][jj[0]], p1 = tb.V[ii[1]][jj[1]], p2 = tb.V[ii[2]][jj[2]];
            const double phi = p0 * p1 * p2;
            const double dphi[3] = {tb.Vd[ii[0]][jj[0]] * p1 * p2, p0 * tb.Vd[ii[1]][jj[1]] * p2,
                                    p0 * p1 * tb.Vd[ii[2]][jj[2]]};
#pragma unroll
            for (int a = 0; a < 5; ++a) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    double acc = vs[0][a][k] * phi;
                    if constexpr (NS) {
                        acc = fma(vs[1][a][k], dphi[0], acc);
                        acc = fma(vs[2][a][k], dphi[1], acc);
                        acc = fma(vs[3][a][k], dphi[2], acc);
                    }
                    Ad[a][k] = acc;
                }
                Bd[a] = (a == beta) ? shift * wdet * phi : 0.0;
            }
        }
        for (int r = 0; r * NQ < NFP; ++r) {
            const int fp = r * NQ + q;
            if (active && fp < NFP) {
                const int f = fp / NF, fq = fp % NF;
                const int d = f >> 1, s = f & 1;
                double bv, bg[3];
                face_basis<N>(tb, d, s, fq / N, fq % N, tj, bv, bg);
                const double* fs = FS + (size_t)fp * 35;
                double* so = sF + q * 20;
#pragma unroll
                for (int o = 0; o < 5; ++o) {
                    double acc = fs[o] * bv;
                    if constexpr (NS) {
                        acc = fma(fs[20 + o], bg[0], acc);
                        acc = fma(fs[25 + o], bg[1], acc);
                        acc = fma(fs[30 + o], bg[2], acc);
                    }
                    so[o] = acc;
                }
                if constexpr (NS) {
#pragma unroll
                    for (int o = 5; o < 20; ++o) so[o] = fs[o] * bv;
                }
            }
            __syncthreads();
            if (active) {
#pragma unroll
                for (int fl = 0; fl < N; ++fl) {
                    const int f = r * N + fl;
                    if (f >= 6) break;
                    const int d = f >> 1, s = f & 1;
                    const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
                    const double l = tb.lag[s][ii[d]];
                    const double* fo = sF + (fl * NF + ii[t1] * N + ii[t2]) * 20;
#pragma unroll
                    for (int a = 0; a < 5; ++a) {
                        Bd[a] = fma(l, fo[a], Bd[a]);
                        if constexpr (NS) {
#pragma unroll
                            for (int k = 0; k < 3; ++k) Ad[a][k] = fma(l, fo[5 + a * 3 + k], Ad[a][k]);
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (active) {
#pragma unroll
            for (int a = 0; a < 5; ++a) {
#pragma unroll
                for (int k = 0; k < 3; ++k) sA[(a * 3 + k) * NQ + q] = Ad[a][k];
                sB[a * NQ + q] = Bd[a];
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                double acc = sB[a * NQ + q];
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int j = 0; j < N; ++j)
                        acc = fma(tb.D[j][ii[k]], sA[(a * 3 + k) * NQ + tix_dir<N>(k, j, ii)], acc);
                H[a * NQ + q] = acc;
            }
        }
        __syncthreads();
        if (active) sweep<N, 5, true>(tb.V, H, Y1, 0, ii, q);
        __syncthreads();
        if (active) sweep<N, 5, true>(tb.V, Y1, Y2, 1, ii, q);
        __syncthreads();
        if (active) {
            const int pm = perm[q];
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) acc = fma(tb.V[j][ii[2]], Y2[a * NQ + tix_dir<N>(2, j, ii)], acc);
                out[((size_t)e * NB + col) * ld + a * NQ + pm] = acc;
            }
        }
        __syncthreads();
    }
}

namespace {
template <int P, bool SELF>
hipError_t launch_diag_k(const DGArgs& a, const double* W, double shift, double* blocks, int ld, double* nbrtr,
                         dim3 grid, dim3 block, bool curved, hipStream_t s) {
    if (a.ns) {
        if (curved) hipLaunchKernelGGL((diag_kernel<P, true, true, SELF>), grid, block, 0, s, a.m, a.g, W, nbrtr, shift, blocks, ld);
        else hipLaunchKernelGGL((diag_kernel<P, true, false, SELF>), grid, block, 0, s, a.m, a.g, W, nbrtr, shift, blocks, ld);
    } else {
        if (curved) hipLaunchKernelGGL((diag_kernel<P, false, true, SELF>), grid, block, 0, s, a.m, a.g, W, nbrtr, shift, blocks, ld);
        else hipLaunchKernelGGL((diag_kernel<P, false, false, SELF>), grid, block, 0, s, a.m, a.g, W, nbrtr, shift, blocks, ld);
    }
    return hipGetLastError();
}

template <int P, bool NS, bool CURVED>
hipError_t launch_diag_slices_k(const DGArgs& a, const double* W, double shift, double* blocks, int ld,
                                const double* nbrtr, hipStream_t s) {
    constexpr int EPB = LaunchS<P>::EPB;
    const size_t lds = (size_t)EPB * SzS<P>::TOT * sizeof(double);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void*)diag_slices_kernel<P, NS, CURVED>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    dim3 grid((a.m.ne + EPB - 1) / EPB, 5), block(EPB * SzS<P>::NQ);
    hipLaunchKernelGGL((diag_slices_kernel<P, NS, CURVED>), grid, block, lds, s, a.m, a.g, W, nbrtr, shift, blocks,
                       ld);
    return hipGetLastError();
}
template <int P>
hipError_t launch_diag_slices(const DGArgs& a, const double* W, double shift, double* blocks, int ld,
                              const double* nbrtr, bool curved, hipStream_t s) {
    if (a.ns) return curved ? launch_diag_slices_k<P, true, true>(a, W, shift, blocks, ld, nbrtr, s)
                            : launch_diag_slices_k<P, true, false>(a, W, shift, blocks, ld, nbrtr, s);
    return curved ? launch_diag_slices_k<P, false, true>(a, W, shift, blocks, ld, nbrtr, s)
                  : launch_diag_slices_k<P, false, false>(a, W, shift, blocks, ld, nbrtr, s);
}

template <int P>
hipError_t launch_diag_p(const DGArgs& a, const double* W, double shift, double* blocks, int ld, double* nbrtr,
                         hipStream_t s) {
    if (ld < 5 * (P + 1) * (P + 1) * (P + 1)) return hipErrorInvalidValue;
    constexpr int NQ = (P + 1) * (P + 1) * (P + 1);
    hipLaunchKernelGGL(nbr_trace_kernel<P>, dim3(a.m.ne), dim3(256), 0, s, a.m, W, nbrtr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    constexpr int EPB = LaunchD<P>::EPB;
    dim3 grid((a.m.ne + EPB - 1) / EPB, 5 * NQ), block(EPB * NQ);
    const bool curved = a.m.vtx != nullptr;
    const bool self = a.m.nx == 1 || a.m.ny == 1 || a.m.nz == 1;
    if (self) return launch_diag_k<P, true>(a, W, shift, blocks, ld, nbrtr, grid, block, curved, s);
    return launch_diag_slices<P>(a, W, shift, blocks, ld, nbrtr, curved, s);
}
}  // namespace

size_t nbr_trace_size(int p, int ne) { return (size_t)ne * 6 * (p + 1) * (p + 1) * 20; }

hipError_t launch_diag_blocks(const DGArgs& a, const double* W, double shift, double* blocks, int ld, double* nbrtr,
                              hipStream_t s) {
    switch (a.p) {
        case 1: return launch_diag_p<1>(a, W, shift, blocks, ld, nbrtr, s);
        case 2: return launch_diag_p<2>(a, W, shift, blocks, ld, nbrtr, s);
        case 3: return launch_diag_p<3>(a, W, shift, blocks, ld, nbrtr, s);
        case 4: return launch_diag_p<4>(a, W, shift, blocks, ld, nbrtr, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dg
