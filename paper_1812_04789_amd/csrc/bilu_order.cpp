// Host part of the block ILU(0) of the coarsest level (Sec. 6.3): the
// minimum-discarded-fill elimination order of every element line along x.
// Host code only (no device calls), so it also builds with a plain host
// compiler (the sanitizer test of the host code).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace dg {

// Minimum-discarded-fill order of every line from the weights w (host):
// repeatedly eliminate, among the line's remaining elements, the one with
// the smallest weight, where an element whose two line neighbours are not
// both remaining discards nothing (weight 0); weights within a relative
// 1e-10 of the smallest tie, and ties go to the lowest element index.
void bilu_mdf_order(int nx, int ny, int nz, const double* w, int* ord, int* pos) {
    const int lines = ny * nz;
    std::vector<char> alive(nx);
    for (int line = 0; line < lines; ++line) {
        const int base = line * nx;
        std::fill(alive.begin(), alive.end(), 1);
        for (int step = 0; step < nx; ++step) {
            double wmin = INFINITY;
            std::vector<double> wk(nx, 0.0);
            for (int i = 0; i < nx; ++i) {
                if (!alive[i]) continue;
                const int im = (i + nx - 1) % nx, ip = (i + 1) % nx;
                const bool both = nx >= 4 && alive[im] && alive[ip];
                wk[i] = both ? w[base + i] : 0.0;
                wmin = std::min(wmin, wk[i]);
            }
            int best = -1;
            for (int i = 0; i < nx; ++i)
                if (alive[i] && wk[i] <= wmin * (1.0 + 1e-10)) {
                    best = i;
                    break;
                }
            alive[best] = 0;
            ord[base + step] = base + best;
            pos[base + best] = step;
        }
    }
}

}  // namespace dg
