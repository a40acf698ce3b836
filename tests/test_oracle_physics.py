"""Pins of the oracle's fluxes (CPU only): Euler/NS fluxes of Eq. NS and the
Roe flux of Sec. 3.1, against identities and independent constructions."""
import numpy as np
import pytest

from oracle import physics as phy

G = 1.4


def _states(n, seed, mach=0.4):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, n)
    v = rng.uniform(-1, 1, (n, 3)) * mach
    p = rng.uniform(0.5, 2.0, n)
    E = p / (G - 1) + 0.5 * rho * np.sum(v * v, -1)
    return np.concatenate([rho[:, None], rho[:, None] * v, E[:, None]], -1)


def _normals(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 3))
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


def _jac(fun, u):
    """Complex-step Jacobian of fun: (5,) -> (5,) at u."""
    J = np.zeros((5, 5))
    for k in range(5):
        du = np.zeros(5, complex)
        du[k] = 1e-30j
        J[:, k] = np.imag(fun(u + du)) / 1e-30
    return J


def test_roe_consistency_and_conservation():
    u = _states(50, 1)
    w = _states(50, 2)
    n = _normals(50, 3)
    Fn = np.einsum('eaj,ej->ea', phy.flux_c(u, G), n)
    assert np.allclose(phy.roe(u, u, n, G), Fn, atol=1e-13, rtol=1e-13)
    assert np.allclose(phy.roe(u, w, n, G), -phy.roe(w, u, -n, G), atol=1e-13, rtol=1e-13)


def test_euler_flux_homogeneity():
    """F_c(u).n = A_n(u) u (the Euler flux is homogeneous of degree one)."""
    for u, n in zip(_states(5, 4), _normals(5, 5)):
        A = _jac(lambda x: phy.flux_c(x, G) @ n, u)
        assert np.allclose(A @ u, phy.flux_c(u, G) @ n, rtol=1e-12, atol=1e-12)


def _roe_state(uL, uR):
    """A conservative state with the Roe-averaged velocity and total enthalpy."""
    rL, vL, pL, HL = phy.primitives(uL, G)
    rR, vR, pR, HR = phy.primitives(uR, G)
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    v = (sL * vL + sR * vR) / (sL + sR)
    H = (sL * HL + sR * HR) / (sL + sR)
    E = (H + (G - 1) * 0.5 * v @ v) / G        # h0 = gamma e0 - (gamma-1)|v|^2/2 with rho = 1
    return np.concatenate([[1.0], v, [E]])


def test_roe_property_and_eigen_dissipation():
    """U-property A(u~)(uR - uL) = (F(uR) - F(uL)).n, and the flux equals
    1/2(FL + FR).n - 1/2 |A(u~)|(uR - uL) with |A| = R |Lambda| R^-1 from a
    numerical eigendecomposition of the complex-step Jacobian."""
    UL, UR, N = _states(8, 6), _states(8, 7), _normals(8, 8)
    for uL, uR, n in zip(UL, UR, N):
        ut = _roe_state(uL, uR)
        A = _jac(lambda x: phy.flux_c(x, G) @ n, ut)
        FL, FR = phy.flux_c(uL, G) @ n, phy.flux_c(uR, G) @ n
        assert np.allclose(A @ (uR - uL), FR - FL, rtol=1e-11, atol=1e-11)
        lam, R = np.linalg.eig(A)
        absA = np.real(R @ np.diag(np.abs(lam)) @ np.linalg.inv(R))
        ref = 0.5 * (FL + FR) - 0.5 * absA @ (uR - uL)
        assert np.allclose(phy.roe(uL, uR, n, G), ref, rtol=1e-10, atol=1e-10)


def test_roe_supersonic_upwinding():
    """All eigenvalues positive: the Roe flux is the upwind (L) flux."""
    uL = _states(1, 9)[0]
    rho, v, p, H = phy.primitives(uL, G)
    n = np.array([1.0, 0.0, 0.0])
    vel = np.array([3.0, 0.2, -0.1])          # Mach ~ 2.5 along n
    uL = np.concatenate([[rho], rho * vel, [p / (G - 1) + 0.5 * rho * vel @ vel]])
    uR = uL * np.array([1.05, 1.02, 1.0, 0.98, 1.03])
    assert np.allclose(phy.roe(uL, uR, n, G), phy.flux_c(uL, G) @ n, rtol=1e-13)


def _primitive_field(x, c):
    """A smooth primitive field (rho, v, p) of the point x (3,), complex-safe."""
    rho = 1.0 + c[0] * x[0] + c[1] * x[1] * x[2]
    v = np.array([0.3 + c[2] * x[1], -0.1 + c[3] * x[0] * x[2], 0.2 + c[4] * x[2]])
    p = 1.5 + c[5] * x[0] * x[1] + c[6] * x[2]
    return rho, v, p


def test_viscous_flux_against_primitive_gradients():
    """F_v from conservative gradients (quotient rule inside flux_v) equals the
    definition of Eq. NS written with primitive gradients computed directly
    (complex-step in x), including tau's -2/3 mu div v and q = -(mu/Pr) grad h."""
    mu, Pr = 0.03, 0.71
    rng = np.random.default_rng(10)
    c = rng.uniform(-0.5, 0.5, 7)
    x0 = np.array([0.3, -0.2, 0.4])

    def cons(x):
        rho, v, p = _primitive_field(x, c)
        return np.concatenate([[rho], rho * v, [p / (G - 1) + 0.5 * rho * (v @ v)]])

    def prim(x):
        rho, v, p = _primitive_field(x, c)
        return np.concatenate([v, [G / (G - 1) * p / rho]])     # v and h

    Gu = np.zeros((5, 3))
    Gp = np.zeros((4, 3))
    for j in range(3):
        dx = np.zeros(3, complex)
        dx[j] = 1e-30j
        Gu[:, j] = np.imag(cons(x0 + dx)) / 1e-30
        Gp[:, j] = np.imag(prim(x0 + dx)) / 1e-30
    u = cons(x0)
    gv = Gp[:3]
    gh = Gp[3]
    tau = mu * (gv + gv.T) - 2.0 / 3.0 * mu * np.trace(gv) * np.eye(3)
    q = -mu / Pr * gh
    v = u[1:4] / u[0]
    ref = np.zeros((5, 3))
    ref[1:4] = -tau
    ref[4] = -(tau @ v - q)
    assert np.allclose(phy.flux_v(u, Gu, G, mu, Pr), ref, rtol=1e-12, atol=1e-14)
    # properties: zero gradient gives zero flux; linear in the gradient
    assert np.all(phy.flux_v(u, np.zeros((5, 3)), G, mu, Pr) == 0)
    G2 = rng.standard_normal((5, 3))
    assert np.allclose(phy.flux_v(u, 2 * Gu - 3 * G2, G, mu, Pr),
                       2 * phy.flux_v(u, Gu, G, mu, Pr) - 3 * phy.flux_v(u, G2, G, mu, Pr), atol=1e-13)


def test_cabs_is_complex_step_safe():
    x = np.array([-2.0, 3.0]) + 1e-30j * np.array([1.0, 1.0])
    assert np.allclose(np.real(phy.cabs(x)), [2.0, 3.0])
    assert np.allclose(np.imag(phy.cabs(x)) / 1e-30, [-1.0, 1.0])
