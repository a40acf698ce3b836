// Host construction of the 1D reference tables (Sec. 3: orthonormal modal
// tensor basis; (p+1)-point Gauss rule) and of the hierarchical mode order.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace dg {

namespace {

// Legendre P_k(x) and P_k'(x) for k = 0..n-1 (Bonnet recurrence).
void legendre_all(int n, double x, double* P, double* dP) {
    P[0] = 1.0;
    dP[0] = 0.0;
    if (n > 1) {
        P[1] = x;
        dP[1] = 1.0;
    }
    for (int k = 1; k + 1 < n; ++k) {
        P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
        dP[k + 1] = dP[k - 1] + (2 * k + 1) * P[k];
    }
}

// Gauss-Legendre points (ascending) and weights by Newton iteration on P_n.
void gauss_rule(int n, double* z, double* w) {
    for (int i = 0; i < n; ++i) {
        double x = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double P[16], dP[16];
        for (int it = 0; it < 100; ++it) {
            legendre_all(n + 1, x, P, dP);
            double dx = P[n] / dP[n];
            x -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        legendre_all(n + 1, x, P, dP);
        z[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dP[n] * dP[n]);
    }
}

}  // namespace

void build_tables(Tab tabs[MAXP + 1], short perm[PERM_TOTAL]) {
    std::memset(tabs, 0, sizeof(Tab) * (MAXP + 1));
    for (int P = 1; P <= MAXP; ++P) {
        const int n = P + 1;
        Tab& t = tabs[P];
        gauss_rule(n, t.z, t.w);
        auto orth = [](int a) { return std::sqrt((2.0 * a + 1.0) / 2.0); };
        double Pq[16], dPq[16];
        for (int q = 0; q < n; ++q) {
            legendre_all(n, t.z[q], Pq, dPq);
            for (int a = 0; a < n; ++a) {
                t.V[q][a] = orth(a) * Pq[a];
                t.Vd[q][a] = orth(a) * dPq[a];
            }
        }
        for (int s = 0; s < 2; ++s) {
            const double x = s ? 1.0 : -1.0;
            legendre_all(n, x, Pq, dPq);
            for (int a = 0; a < n; ++a) {
                t.Le[s][a] = orth(a) * Pq[a];
                t.Lde[s][a] = orth(a) * dPq[a];
            }
            // Lagrange basis of the Gauss points evaluated at the end x
            for (int q = 0; q < n; ++q) {
                double l = 1.0;
                for (int m = 0; m < n; ++m)
                    if (m != q) l *= (x - t.z[m]) / (t.z[q] - t.z[m]);
                t.lag[s][q] = l;
                // its derivative at the end: l_q'(x) = l_q(x) sum_{m != q} 1 / (x - z_m)
                double sd = 0.0;
                for (int m = 0; m < n; ++m)
                    if (m != q) sd += 1.0 / (x - t.z[m]);
                t.lagd[s][q] = l * sd;
            }
            // BR2 line weights: (sum_i L_i(x) L_i(z_q))^2 w_q
            for (int q = 0; q < n; ++q) {
                double k = 0.0;
                for (int a = 0; a < n; ++a) k += t.Le[s][a] * t.V[q][a];
                t.br2[s][q] = k * k * t.w[q];
            }
        }
        // collocation derivative D[q][r] = l_r'(z_q) (barycentric form)
        double c[16];
        for (int q = 0; q < n; ++q) {
            c[q] = 1.0;
            for (int m = 0; m < n; ++m)
                if (m != q) c[q] *= (t.z[q] - t.z[m]);
        }
        for (int q = 0; q < n; ++q) {
            double diag = 0.0;
            for (int r = 0; r < n; ++r) {
                if (r == q) continue;
                t.D[q][r] = (c[q] / c[r]) / (t.z[q] - t.z[r]);
                diag += 1.0 / (t.z[q] - t.z[r]);
            }
            t.D[q][q] = diag;
        }
        // hierarchical order: tensor mode (a,b,c) -> position in the layout
        std::vector<std::array<int, 3>> ms;
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b)
                for (int cc = 0; cc < n; ++cc) ms.push_back({a, b, cc});
        std::stable_sort(ms.begin(), ms.end(), [](const std::array<int, 3>& x, const std::array<int, 3>& y) {
            int sx = std::max(x[0], std::max(x[1], x[2])), sy = std::max(y[0], std::max(y[1], y[2]));
            if (sx != sy) return sx < sy;
            return x < y;
        });
        short* pp = perm + perm_offset(P);
        for (int k = 0; k < (int)ms.size(); ++k) {
            const auto& m = ms[k];
            pp[(m[0] * n + m[1]) * n + m[2]] = (short)k;
        }
    }
}

}  // namespace dg
