// Test driver for the library's host-only code, built with a host compiler
// and sanitizers by tests/test_host_sanitized.py (not part of the library).
//   host_driver tables   prints the 1D reference tables and the hierarchical
//                        mode order of every degree
//   host_driver mdf      reads "nx ny nz" and nx*ny*nz weights from stdin and
//                        prints the elimination order and positions
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.h"

static void print_row(const char* name, int P, int i, const double* v, int n) {
    std::printf("%s %d %d", name, P, i);
    for (int k = 0; k < n; ++k) std::printf(" %.17g", v[k]);
    std::printf("\n");
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    if (!std::strcmp(argv[1], "tables")) {
        static dg::Tab tabs[dg::MAXP + 1];
        static short perm[dg::PERM_TOTAL];
        dg::build_tables(tabs, perm);
        for (int P = 1; P <= dg::MAXP; ++P) {
            const int n = P + 1;
            const dg::Tab& t = tabs[P];
            print_row("z", P, 0, t.z, n);
            print_row("w", P, 0, t.w, n);
            for (int q = 0; q < n; ++q) {
                print_row("V", P, q, t.V[q], n);
                print_row("Vd", P, q, t.Vd[q], n);
                print_row("D", P, q, t.D[q], n);
            }
            for (int s = 0; s < 2; ++s) {
                print_row("lag", P, s, t.lag[s], n);
                print_row("lagd", P, s, t.lagd[s], n);
                print_row("Le", P, s, t.Le[s], n);
                print_row("Lde", P, s, t.Lde[s], n);
                print_row("br2", P, s, t.br2[s], n);
            }
            std::printf("perm %d 0", P);
            for (int k = 0; k < n * n * n; ++k) std::printf(" %d", perm[dg::perm_offset(P) + k]);
            std::printf("\n");
        }
        return 0;
    }
    if (!std::strcmp(argv[1], "mdf")) {
        int nx, ny, nz;
        if (std::scanf("%d %d %d", &nx, &ny, &nz) != 3 || nx < 1 || ny < 1 || nz < 1) return 3;
        const int ne = nx * ny * nz;
        std::vector<double> w(ne);
        for (int e = 0; e < ne; ++e)
            if (std::scanf("%lf", &w[e]) != 1) return 4;
        std::vector<int> ord(ne, -1), pos(ne, -1);
        dg::bilu_mdf_order(nx, ny, nz, w.data(), ord.data(), pos.data());
        std::printf("ord");
        for (int e = 0; e < ne; ++e) std::printf(" %d", ord[e]);
        std::printf("\npos");
        for (int e = 0; e < ne; ++e) std::printf(" %d", pos[e]);
        std::printf("\n");
        return 0;
    }
    return 2;
}
