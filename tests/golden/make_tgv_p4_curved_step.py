"""Write tgv_p4_curved_step.txt: one BDF2 step (dt = 0.05) of the Taylor-Green
NS case at M = 0.01, Re = 1600, p = 4 on a curved 2x2x1 periodic mesh of
[0, 2pi]^3 (every node displaced by 0.05 h sin x sin y sin z), computed by the
FP64 oracle only (element block-Jacobi FGMRES to 1e-11, Newton to 1e-10).

    python tests/golden/make_tgv_p4_curved_step.py      (about 3-4 minutes)

The file holds the initial and final modal coefficients, [e][eq][mode] in the
oracle's hierarchical order, one value per line with 17 significant digits."""
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_1812_04789_amd import inputs  # noqa: E402  (mesh vertices and the initial field only)
from oracle import mesh as omesh, dg as odg, timestep as ots  # noqa: E402

N = (2, 2, 1)
P = 4
L = 2 * math.pi


def case():
    vtx = inputs.box_vertices(N, (0, 0, 0), (L, L, L), amp=0.05)
    return odg.Discretization(omesh.BoxMesh(N, (0, 0, 0), (L, L, L), vtx), P, gamma=1.4, mu=1.0 / 1600, Pr=0.71,
                              eta=7.0)


def main():
    D = case()
    W0 = D.project(inputs.taylor_green(D.quad_points(), mach=0.01))
    W1, st = ots.bdf2_step(D, W0, None, 0.05, precond="bj", restart=40, rtol=1e-11)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tgv_p4_curved_step.txt")
    with open(out, "w") as f:
        f.write("# oracle BDF2 step, Taylor-Green M=0.01 Re=1600, p=4, curved 2x2x1 mesh of [0,2pi]^3, dt=0.05\n")
        f.write("# written by tests/golden/make_tgv_p4_curved_step.py; Newton iterations %d\n" % st.newton)
        f.write("# shape %d %d %d; first block W^n, second block W^(n+1)\n" % W0.shape)
        for a in (W0, W1):
            for v in a.reshape(-1):
                f.write("%.17g\n" % v)
    print("wrote", out)


if __name__ == "__main__":
    main()
