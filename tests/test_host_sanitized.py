"""The library's host-only code built with a host C++ compiler under
AddressSanitizer and UndefinedBehaviorSanitizer (CPU only), run and checked
against independent references:

* the 1D reference tables of Sec. 3 (tables.cpp): Gauss points and weights
  against numpy's Gauss-Legendre rule; orthonormal Legendre values and
  derivatives at the Gauss points and at the ends against numpy's Legendre
  series; the collocation derivative and the Lagrange basis (values and
  derivatives at the ends) against numpy polynomial interpolation through
  the Gauss points; the BR2 line weights from their definition; the
  hierarchical mode order against the oracle's;
* the minimum-discarded-fill elimination order of the block ILU(0) lines
  (bilu_order.cpp, Sec. 6.3) against the oracle's mdf_order, on random
  block rings whose weights the oracle computes (lines of one to nine
  elements, several lines, ties).

Any sanitizer report fails the test (halt on the first error).
"""
import os
import shutil
import subprocess

import numpy as np
import numpy.polynomial.legendre as npleg
import numpy.polynomial.polynomial as nppoly
import pytest

from oracle import reference as oref, linear as olin

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1812_04789_amd", "csrc")
GXX = shutil.which("g++")
ROCM_INC = "/opt/rocm/include"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if GXX is None or not os.path.isdir(ROCM_INC):
        pytest.skip("no host C++ compiler or HIP headers")
    out = str(tmp_path_factory.mktemp("host") / "host_driver")
    cmd = [GXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, "-I" + CSRC,
           "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "host", "host_driver.cpp"),
           os.path.join(CSRC, "tables.cpp"), os.path.join(CSRC, "bilu_order.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def _run(driver, *args, stdin=None):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([driver, *args], input=stdin, capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def _tables(driver):
    t = {}
    for line in _run(driver, "tables").splitlines():
        f = line.split()
        name, P, i = f[0], int(f[1]), int(f[2])
        vals = [int(x) for x in f[3:]] if name == "perm" else [float(x) for x in f[3:]]
        t.setdefault((name, P), {})[i] = np.array(vals)
    return t


def _orthonormal(a, x, deriv=0):
    c = np.zeros(a + 1)
    c[a] = np.sqrt((2 * a + 1) / 2.0)
    if deriv:
        c = npleg.legder(c)
    return npleg.legval(x, c)


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_reference_tables(driver, P):
    t = _tables(driver)
    n = P + 1
    z, w = np.polynomial.legendre.leggauss(n)
    assert np.allclose(t[("z", P)][0], z, rtol=0, atol=1e-15)
    assert np.allclose(t[("w", P)][0], w, rtol=0, atol=1e-15)
    V = np.array([[_orthonormal(a, z[q]) for a in range(n)] for q in range(n)])
    Vd = np.array([[_orthonormal(a, z[q], 1) for a in range(n)] for q in range(n)])
    for q in range(n):
        assert np.allclose(t[("V", P)][q], V[q], rtol=0, atol=1e-13)
        assert np.allclose(t[("Vd", P)][q], Vd[q], rtol=0, atol=1e-12)
    # Lagrange basis of the Gauss points: l_r as a monomial series through the points
    lag = [nppoly.polyfit(z, np.eye(n)[r], n - 1) for r in range(n)]
    D = np.array([[nppoly.polyval(z[q], nppoly.polyder(lag[r])) for r in range(n)] for q in range(n)])
    for q in range(n):
        assert np.allclose(t[("D", P)][q], D[q], rtol=0, atol=1e-10)
    for s, x in ((0, -1.0), (1, 1.0)):
        assert np.allclose(t[("lag", P)][s], [nppoly.polyval(x, lag[r]) for r in range(n)], rtol=0, atol=1e-11)
        assert np.allclose(t[("lagd", P)][s], [nppoly.polyval(x, nppoly.polyder(lag[r])) for r in range(n)],
                           rtol=0, atol=1e-9)
        Le = np.array([_orthonormal(a, x) for a in range(n)])
        assert np.allclose(t[("Le", P)][s], Le, rtol=0, atol=1e-13)
        assert np.allclose(t[("Lde", P)][s], [_orthonormal(a, x, 1) for a in range(n)], rtol=0, atol=1e-12)
        br2 = (V @ Le) ** 2 * w
        assert np.allclose(t[("br2", P)][s], br2, rtol=1e-13, atol=1e-15)
    # hierarchical order: perm[(a n + b) n + c] = position of mode (a, b, c)
    order = oref.modes(P)
    perm = t[("perm", P)][0]
    for k, (a, b, c) in enumerate(order):
        assert perm[(a * n + b) * n + c] == k


def _ring_blocks(nx, ny, nz, nb, rng, tie=False):
    """Random diagonally dominant blocks with couplings between x-neighbours
    only (the line structure), as the oracle's block dictionary."""
    blocks = {}
    ne = nx * ny * nz
    for e in range(ne):
        blocks[(e, e)] = rng.standard_normal((nb, nb)) + 6.0 * np.eye(nb)
    shared = rng.standard_normal((nb, nb))
    for e in range(ne):
        i, base = e % nx, e - e % nx
        for j in {(i + 1) % nx, (i - 1) % nx}:
            o = base + j
            if o != e:
                blocks[(e, o)] = shared.copy() if tie else rng.standard_normal((nb, nb)) * rng.uniform(0.2, 2.0)
    if tie:
        for e in range(ne):
            blocks[(e, e)] = 6.0 * np.eye(nb)
    return blocks


@pytest.mark.parametrize("nx,ny,nz,tie", [(1, 2, 1, False), (2, 2, 1, False), (3, 2, 2, False), (4, 3, 1, False),
                                          (5, 2, 2, False), (8, 2, 1, False), (9, 1, 2, False), (6, 2, 1, True)])
def test_mdf_line_order_matches_oracle(driver, nx, ny, nz, tie):
    rng = np.random.default_rng(100 + nx * 10 + ny)
    nb = 3
    blocks = _ring_blocks(nx, ny, nz, nb, rng, tie)
    ne = nx * ny * nz
    part = {e: e // nx for e in range(ne)}
    order = olin.mdf_order(blocks, part)
    # the weight of each element with both line neighbours remaining (the
    # library evaluates it once on the unfactored blocks, like the oracle)
    nbr = {e: {o for o in olin.block_pattern(blocks)[e] if part[o] == part[e]} for e in range(ne)}
    w = [olin.discarded_fill(blocks, nbr, e, set(range(e - e % nx, e - e % nx + nx))) if nx >= 4 else 0.0
         for e in range(ne)]
    stdin = "%d %d %d\n%s\n" % (nx, ny, nz, " ".join("%.17g" % x for x in w))
    out = _run(driver, "mdf", stdin=stdin).splitlines()
    ord_lib = [int(x) for x in out[0].split()[1:]]
    pos_lib = [int(x) for x in out[1].split()[1:]]
    assert ord_lib == order
    for k, e in enumerate(ord_lib):
        assert pos_lib[e] == k % nx
