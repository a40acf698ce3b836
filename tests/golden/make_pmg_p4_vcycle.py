"""Write pmg_p4_vcycle.txt: one p-multigrid V-cycle (Sec. 6, Alg. 2; inherited
coarse operators of Sec. 6.1; element block Jacobi of Sec. 6.3) with degrees
4 -> 2 -> 1, two pre- and two post-sweeps (omega = 1), a 10-step coarsest
GMRES(BJ), applied from zero to a seeded right-hand side, computed by the FP64
oracle only.  Navier-Stokes (mu = 0.02, Pr = 0.71, eta = 7) on a curved 2x2x2
periodic mesh of [0, 2pi]^3 (every node displaced by 0.1 h sin x sin y sin z),
a seeded random state, shift 20 (K = 20 M + dR/dW).

    python tests/golden/make_pmg_p4_vcycle.py      (about 6 minutes: the
                                                    p = 4 diagonal blocks by
                                                    complex step)

The file holds the right-hand side r and the V-cycle output z, [e][eq][mode]
in the oracle's hierarchical order, one value per line with 17 significant
digits."""
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_1812_04789_amd import inputs  # noqa: E402  (mesh vertices and seeded arrays only)
from oracle import mesh as omesh, dg as odg, linear as olin  # noqa: E402

N = (2, 2, 2)
P = 4
L = 2 * math.pi
SHIFT = 20.0
LEVELS = [4, 2, 1]
COARSE_ITERS = 10


def case():
    vtx = inputs.box_vertices(N, (0, 0, 0), (L, L, L), amp=0.1)
    return odg.Discretization(omesh.BoxMesh(N, (0, 0, 0), (L, L, L), vtx), P, gamma=1.4, mu=0.02, Pr=0.71, eta=7.0)


def state():
    return inputs.random_state(8, P, seed=81), inputs.random_vector(8, P, seed=82)


def main():
    D = case()
    W, r = state()
    pmg = olin.PMG(D, W, SHIFT, LEVELS, nu_pre=2, nu_post=2, omega=1.0, coarse_iters=COARSE_ITERS,
                   coarse_op="exact")
    z = pmg.apply(r)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pmg_p4_vcycle.txt")
    with open(out, "w") as f:
        f.write("# oracle V-cycle 4-2-1 (2+2 BJ sweeps, coarsest GMRES(BJ) 10), NS mu=0.02, p=4, curved 2x2x2 mesh "
                "of [0,2pi]^3, shift 20, random state seed 81\n")
        f.write("# written by tests/golden/make_pmg_p4_vcycle.py\n")
        f.write("# shape %d %d %d; first block r (seed 82), second block z\n" % r.shape)
        for a in (r, z):
            for v in a.reshape(-1):
                f.write("%.17g\n" % v)
    print("wrote", out)


if __name__ == "__main__":
    main()
