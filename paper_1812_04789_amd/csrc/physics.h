// Pointwise physics of the compressible Navier-Stokes equations (Sec. 2,
// Eq. NS) and the numerical fluxes of Sec. 3.1 (Roe, BR2), templated on the
// scalar type so that one source gives the residual (double) and its exact
// forward-mode linearisation (Dual: value + one tangent).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace dg {

__device__ __forceinline__ double fma(double a, double b, double c) { return ::fma(a, b, c); }

struct Dual {
    double v, d;
    __device__ __forceinline__ Dual() = default;
    __device__ __forceinline__ constexpr Dual(double a) : v(a), d(0.0) {}
    __device__ __forceinline__ constexpr Dual(double a, double b) : v(a), d(b) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, fma(a.v, b.d, a.d * b.v)); }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
__device__ __forceinline__ Dual operator/(double a, Dual b) {
    double q = a / b.v;
    return Dual(q, -q * b.d / b.v);
}
__device__ __forceinline__ Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
__device__ __forceinline__ Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
__device__ __forceinline__ Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
__device__ __forceinline__ Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
__device__ __forceinline__ Dual& operator+=(Dual& a, Dual b) { a.v += b.v; a.d += b.d; return a; }
__device__ __forceinline__ Dual& operator-=(Dual& a, Dual b) { a.v -= b.v; a.d -= b.d; return a; }
__device__ __forceinline__ Dual fma(Dual a, Dual b, Dual c) {
    return Dual(::fma(a.v, b.v, c.v), ::fma(a.v, b.d, ::fma(a.d, b.v, c.d)));
}
__device__ __forceinline__ Dual fma(double a, Dual b, Dual c) { return Dual(::fma(a, b.v, c.v), ::fma(a, b.d, c.d)); }
__device__ __forceinline__ Dual dsqrt(Dual a) {
    double s = sqrt(a.v);
    return Dual(s, 0.5 * a.d / s);
}
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }
// |x| with d|x|/dx := sign(x), sign(0) = 0 (no smoothing of Roe's |lambda|).
__device__ __forceinline__ Dual dabs(Dual a) {
    double s = (a.v > 0.0) ? 1.0 : ((a.v < 0.0) ? -1.0 : 0.0);
    return Dual(fabs(a.v), s * a.d);
}
__device__ __forceinline__ double dabs(double a) { return fabs(a); }
__device__ __forceinline__ double val(double a) { return a; }
__device__ __forceinline__ double val(Dual a) { return a.v; }
__device__ __forceinline__ double tan_(double) { return 0.0; }
__device__ __forceinline__ double tan_(Dual a) { return a.d; }
template <class T> __device__ __forceinline__ T mk(double v, double d);
template <> __device__ __forceinline__ double mk<double>(double v, double) { return v; }
template <> __device__ __forceinline__ Dual mk<Dual>(double v, double d) { return Dual(v, d); }

struct Gas {
    double gamma, mu, Pr, eta;
};

// Inviscid flux projected on a direction n (not necessarily unit):
// Fn = (rho vn, rho v vn + p n, rho h0 vn).
template <class T>
__device__ __forceinline__ void flux_c_dir(const T u[5], const double n[3], double gm1, T Fn[5]) {
    T ir = 1.0 / u[0];
    T vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
    T p = gm1 * (u[4] - 0.5 * (u[1] * vx + u[2] * vy + u[3] * vz));
    T vn = vx * n[0] + vy * n[1] + vz * n[2];
    Fn[0] = u[0] * vn;
    Fn[1] = u[1] * vn + p * n[0];
    Fn[2] = u[2] * vn + p * n[1];
    Fn[3] = u[3] * vn + p * n[2];
    Fn[4] = (u[4] + p) * vn;
}

// Full inviscid flux F[a][j].
template <class T>
__device__ __forceinline__ void flux_c(const T u[5], double gm1, T F[5][3]) {
    T ir = 1.0 / u[0];
    T v[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
    T p = gm1 * (u[4] - 0.5 * (u[1] * v[0] + u[2] * v[1] + u[3] * v[2]));
    T hp = u[4] + p;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        F[0][j] = u[1 + j];
        F[1][j] = u[1] * v[j];
        F[2][j] = u[2] * v[j];
        F[3][j] = u[3] * v[j];
        F[4][j] = hp * v[j];
    }
    F[1][0] += p;
    F[2][1] += p;
    F[3][2] += p;
}

// Viscous flux F_v(u, G) (G: gradient of the conservative variables,
// G[a][j] = du_a/dx_j), so that du/dt + div F_c + div F_v = 0 is Eq. NS:
// F_v = -(0, tau, tau.v - q), tau = mu(grad v + grad v^T) - 2/3 mu div v I,
// q = -(mu/Pr) grad h, h = gamma (E - |v|^2/2).  Linear in G.
// Accumulates s * F_v into F.
template <class T, class TG>
__device__ __forceinline__ void flux_v_acc(const T u[5], const TG G[5][3], const Gas& g, double s, T F[5][3]) {
    T ir = 1.0 / u[0];
    T v[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
    T E = u[4] * ir;
    T gv[3][3];
    T gE[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int i = 0; i < 3; ++i) gv[i][j] = (G[1 + i][j] - v[i] * G[0][j]) * ir;
        gE[j] = (G[4][j] - E * G[0][j]) * ir;
    }
    T div = gv[0][0] + gv[1][1] + gv[2][2];
    const double mu = g.mu;
    const double kq = g.gamma * g.mu / g.Pr;     // -q_j = (mu/Pr) dh/dx_j, dh = gamma (dE - v.dv)
    T tau[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) tau[i][j] = mu * (gv[i][j] + gv[j][i]);
    T dd = (2.0 / 3.0) * mu * div;
    tau[0][0] -= dd;
    tau[1][1] -= dd;
    tau[2][2] -= dd;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T mq = kq * (gE[j] - (v[0] * gv[0][j] + v[1] * gv[1][j] + v[2] * gv[2][j]));   // = -q_j
        T w = tau[j][0] * v[0] + tau[j][1] * v[1] + tau[j][2] * v[2] + mq;              // tau.v - q
        F[1][j] -= s * tau[0][j];
        F[2][j] -= s * tau[1][j];
        F[3][j] -= s * tau[2][j];
        F[4][j] -= s * w;
    }
}

// Normal component of the viscous flux: Fn[a] -= s * sum_j F_v(u, G)[a][j] n[j]
// (the same stress and heat flux as flux_v_acc, projected on n).
template <class T, class TG>
__device__ __forceinline__ void flux_v_n_acc(const T u[5], const TG G[5][3], const Gas& g, double s,
                                             const double n[3], T Fn[5]) {
    T ir = 1.0 / u[0];
    T v[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
    T E = u[4] * ir;
    T gv[3][3];
    T gE[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int i = 0; i < 3; ++i) gv[i][j] = (G[1 + i][j] - v[i] * G[0][j]) * ir;
        gE[j] = (G[4][j] - E * G[0][j]) * ir;
    }
    const double mu = g.mu;
    const double kq = g.gamma * g.mu / g.Pr;
    T dd = (2.0 / 3.0) * mu * (gv[0][0] + gv[1][1] + gv[2][2]);
    T wn = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        // (tau n)_i = mu sum_j (gv_ij + gv_ji) n_j - dd n_i
        T tn = -dd * n[i];
#pragma unroll
        for (int j = 0; j < 3; ++j) tn = tn + mu * (gv[i][j] + gv[j][i]) * n[j];
        Fn[1 + i] = Fn[1 + i] - s * tn;
        wn = wn + tn * v[i];
    }
    // (-q).n = kq sum_j (gE_j - v . gv_:j) n_j
    T qn = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) qn = qn + (gE[j] - (v[0] * gv[0][j] + v[1] * gv[1][j] + v[2] * gv[2][j])) * n[j];
    Fn[4] = Fn[4] - s * (wn + kq * qn);
}

// Viscous flux of a rank-one gradient G[a][j] = du[a] n[j] (the BR2 jump
// term): with a_i = (du_{1+i} - v_i du_0)/rho and b = (du_4 - E du_0)/rho the
// velocity gradient is a (x) n and the energy gradient b n, so
// tau = mu (a (x) n + n (x) a) - 2/3 mu (a.n) I and -q = kq (b - v.a) n.
// Accumulates s * F_v into F (all 3 columns) and returns nothing else.
template <class T>
__device__ __forceinline__ void flux_v_rank1_acc(const T u[5], const T du[5], const double n[3], const Gas& g,
                                                 double s, T F[5][3]) {
    T ir = 1.0 / u[0];
    T v[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
    T E = u[4] * ir;
    T av[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) av[i] = (du[1 + i] - v[i] * du[0]) * ir;
    T b = (du[4] - E * du[0]) * ir;
    const double mu = g.mu;
    const double kq = g.gamma * g.mu / g.Pr;
    T an = av[0] * n[0] + av[1] * n[1] + av[2] * n[2];
    T va = v[0] * av[0] + v[1] * av[1] + v[2] * av[2];
    T vn = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
    T dd = (2.0 / 3.0) * mu * an;
    T mqs = kq * (b - va);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        // tau_ij = mu (a_i n_j + n_i a_j) - dd delta_ij;  (tau v)_j = mu (n_j (a.v) + a_j (n.v)) - dd v_j
        F[1][j] = F[1][j] - s * (mu * (av[0] * n[j] + n[0] * av[j]) - ((j == 0) ? dd : T(0.0)));
        F[2][j] = F[2][j] - s * (mu * (av[1] * n[j] + n[1] * av[j]) - ((j == 1) ? dd : T(0.0)));
        F[3][j] = F[3][j] - s * (mu * (av[2] * n[j] + n[2] * av[j]) - ((j == 2) ? dd : T(0.0)));
        T w = mu * (n[j] * va + av[j] * vn) - dd * v[j] + mqs * n[j];
        F[4][j] = F[4][j] - s * w;
    }
}

// Roe flux through unit normal n from the + (L) side to the - (R) side:
// F = (F(uL) + F(uR)).n / 2 - |A(roe avg)| (uR - uL) / 2, waves written
// out (acoustic vn -/+ c, entropy, two shear), no entropy fix.
template <class T>
__device__ __forceinline__ void roe_flux(const T uL[5], const T uR[5], const double n[3], double gamma, T F[5]) {
    const double gm1 = gamma - 1.0;
    T FL[5], FR[5];
    flux_c_dir(uL, n, gm1, FL);
    flux_c_dir(uR, n, gm1, FR);
    T irL = 1.0 / uL[0], irR = 1.0 / uR[0];
    T vL[3] = {uL[1] * irL, uL[2] * irL, uL[3] * irL};
    T vR[3] = {uR[1] * irR, uR[2] * irR, uR[3] * irR};
    T pL = gm1 * (uL[4] - 0.5 * (uL[1] * vL[0] + uL[2] * vL[1] + uL[3] * vL[2]));
    T pR = gm1 * (uR[4] - 0.5 * (uR[1] * vR[0] + uR[2] * vR[1] + uR[3] * vR[2]));
    T HL = (uL[4] + pL) * irL, HR = (uR[4] + pR) * irR;
    T sL = dsqrt(uL[0]), sR = dsqrt(uR[0]);
    T iw = 1.0 / (sL + sR);
    T rt = sL * sR;
    T vt[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) vt[k] = (sL * vL[k] + sR * vR[k]) * iw;
    T Ht = (sL * HL + sR * HR) * iw;
    T q2 = vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2];
    T c2 = gm1 * (Ht - 0.5 * q2);
    T c = dsqrt(c2);
    T vn = vt[0] * n[0] + vt[1] * n[1] + vt[2] * n[2];
    T dr = uR[0] - uL[0];
    T dp = pR - pL;
    T dv[3] = {vR[0] - vL[0], vR[1] - vL[1], vR[2] - vL[2]};
    T dvn = dv[0] * n[0] + dv[1] * n[1] + dv[2] * n[2];
    T ic2 = 1.0 / c2;
    T a1 = (dp - rt * c * dvn) * (0.5 * ic2);
    T a5 = (dp + rt * c * dvn) * (0.5 * ic2);
    T a2 = dr - dp * ic2;
    T l1 = dabs(vn - c), l2 = dabs(vn), l5 = dabs(vn + c);
    T w1 = l1 * a1, w2 = l2 * a2, w5 = l5 * a5;
    T sh[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) sh[k] = l2 * rt * (dv[k] - dvn * n[k]);
    T D[5];
    D[0] = w1 + w2 + w5;
#pragma unroll
    for (int k = 0; k < 3; ++k) D[1 + k] = w1 * (vt[k] - c * n[k]) + w2 * vt[k] + sh[k] + w5 * (vt[k] + c * n[k]);
    D[4] = w1 * (Ht - vn * c) + w2 * (0.5 * q2) + (vt[0] * sh[0] + vt[1] * sh[1] + vt[2] * sh[2]) + w5 * (Ht + vn * c);
#pragma unroll
    for (int a = 0; a < 5; ++a) F[a] = 0.5 * (FL[a] + FR[a]) - 0.5 * D[a];
}

}  // namespace dg
