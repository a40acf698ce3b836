"""Pins of the oracle's reference element and geometry (CPU only).

Modal tensor-product basis and quadrature (Sec. 3, Eq. BSpace); geometry of the
periodic hexahedral mesh (Sec. 3)."""
import math
import os

import numpy as np
import pytest

from oracle import reference as ref, mesh as msh, dg
from paper_1812_04789_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gauss_golden():
    rows = {}
    ns = {"sqrt": math.sqrt}
    with open(os.path.join(GOLD, "gauss_legendre.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            n, x, w = line.split()
            rows.setdefault(int(n), []).append((eval(x, ns), eval(w, ns)))
    return rows


def test_gauss_matches_textbook_closed_forms():
    for n, vals in _gauss_golden().items():
        x, w = ref.gauss(n)
        gx = np.array([v[0] for v in vals])
        gw = np.array([v[1] for v in vals])
        assert np.allclose(x, gx, atol=1e-15, rtol=0)
        assert np.allclose(w, gw, atol=1e-15, rtol=0)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gauss_exact_to_degree_2n_minus_1(n):
    x, w = ref.gauss(n)
    for k in range(2 * n + 1):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        got = float(np.sum(w * x ** k))
        if k <= 2 * n - 1:
            assert abs(got - exact) < 1e-14
        elif k == 2 * n:
            assert abs(got - exact) > 1e-5     # the rule is not exact one degree higher


def test_legendre_values_and_derivatives():
    t = np.linspace(-1, 1, 11)
    L, dL = ref.legendre(7, t)
    for a in range(7):
        c = np.zeros(a + 1)
        c[a] = math.sqrt((2 * a + 1) / 2.0)
        P = np.polynomial.legendre.Legendre(c)
        assert np.allclose(L[a], P(t), atol=1e-14)
        assert np.allclose(dL[a], P.deriv()(t), atol=1e-12)
        # end values L_a(+-1) = (+-1)^a sqrt((2a+1)/2)
        Le, _ = ref.legendre(a + 1, np.array([-1.0, 1.0]))
        assert np.allclose(Le[a], [(-1) ** a * math.sqrt((2 * a + 1) / 2), math.sqrt((2 * a + 1) / 2)], atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_basis_orthonormal_under_the_rule(p):
    X, w = ref.volume_rule(p)
    Phi, _ = ref.basis(p, X)
    assert Phi.shape == ((p + 1) ** 3, (p + 1) ** 3)
    assert np.allclose(Phi.T @ (w[:, None] * Phi), np.eye(Phi.shape[1]), atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_hierarchical_prefix(p):
    ms = ref.modes(p)
    for q in range(p + 1):
        pre = ms[:(q + 1) ** 3]
        assert all(max(m) <= q for m in pre)
        assert len(set(pre)) == (q + 1) ** 3
    # the input module's shell table describes the same order
    assert np.array_equal(inputs.shells(p), np.array([max(m) for m in ms]))


def test_mode0_scale_is_the_constant_mode():
    Phi, _ = ref.basis(2, np.array([[0.3, -0.2, 0.9]]))
    assert abs(Phi[0, 0] * inputs.MODE0_SCALE - 1.0) < 1e-15


# ---- geometry -------------------------------------------------------------------
def _meshes():
    L = 2 * math.pi
    yield msh.BoxMesh((3, 2, 4), (0, 0, 0), (L, L, L)), L ** 3
    yield msh.BoxMesh((4, 4, 4), (0, 0, 0), (L, L, L), inputs.box_vertices((4, 4, 4), (0, 0, 0), (L, L, L), amp=0.05)), L ** 3
    yield msh.BoxMesh((3, 3, 3), (0, 0, 0), (L, L, L), inputs.box_vertices((3, 3, 3), (0, 0, 0), (L, L, L), amp=0.3)), L ** 3


@pytest.mark.parametrize("p", [1, 2])
def test_volume_and_closed_faces(p):
    for m, vol in _meshes():
        D = dg.Discretization(m, p)
        # total volume: detJ of a Q1 map is exactly integrated for p >= 1
        assert abs(np.sum(D.wq * D.detJ) - vol) < 1e-11 * vol
        # closed surface: sum over faces of int n dsigma = 0 for every element
        s = np.zeros((m.ne, 3))
        for f in range(6):
            s += np.einsum('q,eq,eqd->ed', D.wf, D.fJF[f], D.fn[f])
        assert np.abs(s).max() < 1e-12


def test_affine_metrics():
    m = msh.BoxMesh((2, 3, 4), (0, 0, 0), (2.0, 3.0, 8.0))
    D = dg.Discretization(m, 2)
    assert np.allclose(D.detJ, 1.0 * 1.0 * 2.0 / 8.0)
    assert np.allclose(D.Jinv[0, 0], np.diag([2.0, 2.0, 1.0]))
    assert np.allclose(D.M[0], np.eye(D.nv) * 0.25)


def test_faces_match_across_neighbours():
    m, _ = list(_meshes())[1]
    D = dg.Discretization(m, 2)
    L = 2 * math.pi
    for f in range(6):
        nb = m.nbr[:, f]
        xp = np.einsum('qv,evd->eqd', msh.shape_q1(D.Xf[f])[0], m.vtx)
        xm = np.einsum('qv,evd->eqd', msh.shape_q1(D.Xf[f ^ 1])[0], m.vtx[nb])
        d = (xp - xm) / L
        assert np.abs(d - np.round(d)).max() < 1e-13           # same points modulo a period
        assert np.abs(D.fn[f] + D.fn[f ^ 1][nb]).max() < 1e-13  # opposite normals
        assert np.abs(D.fJF[f] - D.fJF[f ^ 1][nb]).max() < 1e-13


def test_nonpositive_jacobian_rejected():
    L = 2 * math.pi
    V = inputs.box_vertices((2, 2, 2), (0, 0, 0), (L, L, L))
    V[0, [0, 1]] = V[0, [1, 0]]          # swap two vertices: inverted element
    with pytest.raises(ValueError):
        dg.Discretization(msh.BoxMesh((2, 2, 2), (0, 0, 0), (L, L, L), V), 1)
