"""Order of accuracy of the oracle's Navier-Stokes discretisation (CPU only):
Sec. 3.1, Eqs. dg_ns, visc_flux, re, with the Roe and BR2 fluxes.

A steady manufactured solution on the periodic box [0, 2pi]^3, varying in all
three directions, with viscosity strong enough (mu = 0.1, Re ~ 3 on the unit
length) that the BR2 terms shape the error.  The source s = div(F_c + F_v)
of the manufactured state is computed pointwise from its closed-form
derivatives: each d/dx_j of the flux column F_j is taken by a complex step in
x_j (the state and its gradient are analytic in x), so s is exact to rounding
and independent of the DG operator.  The discrete problem

    R(W) = S,   S_i = int phi_i s,

is linearised about the projection W0 of the manufactured state: the
correction x of one Newton step, K(W0) x = S - R(W0), is the discrete error
W_h - W0 up to a remainder of order |x|^2 (below 10% of |x| on these
meshes).  On a periodic box the steady operator conserves the element means:
the mean-mode rows of R sum to zero for any W, so K = dR/dW is singular and
the system is solvable only if the mean-mode entries of S - R(W) sum to zero.
The Gauss rule's quadrature error of int s leaves them at O(h^(2p+2)); they
are removed before each solve.  Each correction x is the solution of K x = b
with zero element-mean sum, obtained exactly as the solution of
(K + M E) x = b, E x keeping only the mean over elements of every mean-mode
entry (the added term vanishes on that solution and makes the operator
nonsingular): the discrete solution with the total mass, momentum and energy
of the projected manufactured state.  FGMRES, preconditioned by element block
Jacobi, solves the systems.

The L2 error of the discrete solution then falls as h^(p+1) (the paper sees
about k+1 on its 2D vortex, Table VOR_CONVP); the pin asks for p + 0.8 on
straight and curved (Q1) meshes.  A missing or negated BR2 penalty drops the
rate below 1.1 on these meshes; a missing symmetry term is
invisible at odd p (the known optimal L2 rate of the nonsymmetric form at odd
degree) and is pinned by the adjoint-consistency test instead.
"""
import math

import numpy as np
import pytest

from oracle import mesh as msh, dg, linear as lin, physics as phy
from paper_1812_04789_amd import inputs

GAMMA = 1.4
PR = 0.71
MU = 0.1
L2PI = 2 * math.pi


def _primitive(x):
    """rho, velocity and pressure of the manufactured state, and their
    gradients (closed form); x may be complex."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    s, c = np.sin, np.cos
    rho = 1 + 0.2 * s(X) * s(Y) * s(Z)
    vel = 0.3 * np.stack([s(Y) * c(Z), s(Z) * c(X), s(X) * c(Y)], -1)
    p = (1 + 0.1 * c(X + Y + Z)) / GAMMA
    zero = np.zeros_like(X)
    g_rho = 0.2 * np.stack([c(X) * s(Y) * s(Z), s(X) * c(Y) * s(Z), s(X) * s(Y) * c(Z)], -1)
    g_vel = 0.3 * np.stack([np.stack([zero, c(Y) * c(Z), -s(Y) * s(Z)], -1),
                            np.stack([-s(Z) * s(X), zero, c(Z) * c(X)], -1),
                            np.stack([c(X) * c(Y), -s(X) * s(Y), zero], -1)], -2)     # d v_i / d x_j
    g_p = -0.1 / GAMMA * np.stack([s(X + Y + Z)] * 3, -1)
    return rho, vel, p, g_rho, g_vel, g_p


def manufactured(x):
    """Conserved state (rho, rho v, rho e0) at points x (..., 3)."""
    rho, vel, p, _, _, _ = _primitive(x)
    return inputs.conserved(rho, vel, p, GAMMA)


def manufactured_gradient(x):
    """d u_a / d x_j of the conserved state, (..., 5, 3), by the product rule
    on the primitive closed forms (rho E = p/(gamma-1) + rho |v|^2 / 2)."""
    rho, vel, p, g_rho, g_vel, g_p = _primitive(x)
    G = np.zeros(x.shape[:-1] + (5, 3), dtype=np.result_type(x, float))
    G[..., 0, :] = g_rho
    G[..., 1:4, :] = vel[..., :, None] * g_rho[..., None, :] + rho[..., None, None] * g_vel
    G[..., 4, :] = (g_p / (GAMMA - 1) + 0.5 * np.sum(vel * vel, -1)[..., None] * g_rho
                    + rho[..., None] * np.einsum('...i,...ij->...j', vel, g_vel))
    return G


def source(x):
    """s = sum_j d/dx_j [F_c + F_v](u(x), grad u(x))_{:, j}, each derivative by
    a complex step of size 1e-30 in x_j."""
    h = 1e-30
    s = np.zeros(x.shape[:-1] + (5,))
    for j in range(3):
        xc = np.asarray(x, complex).copy()
        xc[..., j] += 1j * h
        u, G = manufactured(xc), manufactured_gradient(xc)
        F = phy.flux_c(u, GAMMA) + phy.flux_v(u, G, GAMMA, MU, PR)
        s += np.imag(F[..., :, j]) / h
    return s


def test_manufactured_gradient_is_the_gradient():
    """The closed-form gradient equals the complex-step derivative of the state."""
    x = np.random.default_rng(0).uniform(0, L2PI, (7, 3))
    G = manufactured_gradient(x)
    for j in range(3):
        xc = x.astype(complex)
        xc[:, j] += 1e-30j
        assert np.allclose(np.imag(manufactured(xc)) / 1e-30, G[:, :, j], rtol=1e-13, atol=1e-14)


def _steady_error(n, p, curved):
    V = inputs.box_vertices(n, (0, 0, 0), (L2PI,) * 3, amp=0.1 if curved else 0.0, phase=0.7)
    D = dg.Discretization(msh.BoxMesh(n, (0, 0, 0), (L2PI,) * 3, V), p, gamma=GAMMA, mu=MU, Pr=PR)
    W0 = D.project(manufactured(D.xq))
    S = D.mass(D.project(source(D.xq)))
    P = lin.BlockJacobi(D, W0, 1e-8)

    def mean_part(v):
        out = np.zeros_like(v)
        out[:, :, 0] = v[:, :, 0].mean(axis=0)
        return out

    b = S - D.residual(W0)
    b[:, :, 0] -= b[:, :, 0].mean(axis=0)
    op = lambda v: lin.jvp_exact(D, W0, v, 0.0) + D.mass(mean_part(v))
    x, st = lin.fgmres(op, P.apply, b, restart=300, rtol=1e-7, max_restarts=3)
    assert st.rel_res_true <= 1e-7
    assert np.abs(x[:, :, 0].mean(axis=0)).max() < 1e-6 * np.abs(x).max()
    return math.sqrt(float(np.sum(x * D.mass(x))))


@pytest.mark.parametrize("curved", [False, True])
def test_viscous_order_of_accuracy(curved):
    p = 1
    e = [_steady_error((k, k, k), p, curved) for k in (2, 4)]
    rate = math.log2(e[0] / e[1])
    assert rate >= p + 0.8, (e, rate)
