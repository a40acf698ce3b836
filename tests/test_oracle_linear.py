"""Pins of the oracle's linearisation and solvers (CPU only): the matrix-free
product of Eq. DG-mf, block-Jacobi PLU (Sec. 6.3), p-multigrid inheritance and
V-cycle (Sec. 6, Alg. 2, Sec. 6.1), FGMRES (Sec. 6), BDF2 + Newton (Eq. NEWTON)."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import mesh as msh, dg, linear as lin, timestep as ts
from paper_1812_04789_amd import inputs

L2PI = 2 * math.pi


def _disc(n=(2, 2, 2), p=1, mu=0.02, curved=False):
    V = inputs.box_vertices(n, (0, 0, 0), (L2PI,) * 3, amp=0.1 if curved else 0.0)
    m = msh.BoxMesh(n, (0, 0, 0), (L2PI,) * 3, V)
    return dg.Discretization(m, p, mu=mu, Pr=0.71)


def _dense_K(D, W, shift):
    N = W.size
    K = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        K[:, j] = lin.jvp_exact(D, W, e.reshape(W.shape), shift).reshape(-1)
    return K


def test_exact_jvp_is_linear_and_zero_at_zero():
    D = _disc(curved=True)
    W = inputs.random_state(D.mesh.ne, 1, seed=1)
    v, w = inputs.random_vector(D.mesh.ne, 1, 2), inputs.random_vector(D.mesh.ne, 1, 3)
    Jv, Jw = lin.jvp_exact(D, W, v, 2.0), lin.jvp_exact(D, W, w, 2.0)
    assert np.allclose(lin.jvp_exact(D, W, 2 * v - 0.5 * w, 2.0), 2 * Jv - 0.5 * Jw, rtol=1e-12, atol=1e-12)
    assert np.all(lin.jvp_exact(D, W, np.zeros_like(v), 2.0) == 0)
    assert np.all(lin.jvp_fd(D, W, D.residual(W), np.zeros_like(v), 2.0) == 0)


def test_fd_jvp_v_curve():
    """(R(W+hv)-R(W))/h vs the exact action: error ~ C1 h + C2 eps/h; the
    paper's step (Eq. DG-mf, eps = 1e-7) lands near the bottom of the V."""
    D = _disc()
    W = inputs.random_state(D.mesh.ne, 1, seed=4)
    v = inputs.random_vector(D.mesh.ne, 1, 5)
    v /= lin.norm(v)
    RW = D.residual(W)
    ex = lin.jvp_exact(D, W, v, 0.0)
    hs = 10.0 ** -np.arange(2, 13)
    err = np.array([lin.norm((D.residual(W + h * v) - RW) / h - ex) / lin.norm(ex) for h in hs])
    k = int(np.argmin(err))
    assert 0 < k < len(hs) - 1
    assert np.all(np.diff(err[:k + 1]) < 0) and err[-1] > err[k] * 10
    assert err[k] < 1e-6
    paper = lin.norm(lin.jvp_fd(D, W, RW, v, 0.0) - ex) / lin.norm(ex)
    assert paper < 10 * err[k]


@pytest.mark.parametrize("n", [(3, 3, 2), (3, 1, 2)])
def test_diag_blocks_are_jacobian_blocks(n):
    """Block columns equal J e_j restricted to the element (brute force),
    including an odd periodic axis and a one-element-wide (self-neighbour) axis."""
    D = _disc(n=n, curved=False)
    W = inputs.random_state(D.mesh.ne, 1, seed=7)
    a = 1.7
    B = lin.diag_blocks(D, W, a)
    rng = np.random.default_rng(0)
    for e in rng.choice(D.mesh.ne, 3, replace=False):
        for j in rng.choice(5 * D.nv, 6, replace=False):
            ej = np.zeros_like(W)
            ej[e].reshape(-1)[j] = 1.0
            col = lin.jvp_exact(D, W, ej, a)
            assert np.allclose(B[e][:, j], col[e].reshape(-1), rtol=1e-12, atol=1e-12)


def test_plu_matches_scipy():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((4, 40, 40)) + 3 * np.eye(40)
    LU, piv = lin.lu_factor(A)
    b = rng.standard_normal((4, 40))
    for k in range(4):
        LUs, pivs = scipy.linalg.lu_factor(A[k])
        assert np.array_equal(piv[k], pivs)
        assert np.allclose(LU[k], LUs, rtol=1e-12, atol=1e-12)
    x = lin.lu_solve(LU, piv, b)
    assert np.allclose(np.einsum('kij,kj->ki', A, x), b, rtol=1e-12, atol=1e-12)


def test_transfer_operators():
    x = inputs.random_vector(5, 3, 1)
    c = lin.restrict(x, 1)
    assert np.array_equal(lin.restrict(lin.prolong(c, 64), 1), c)              # P^T P = I
    y = inputs.random_vector(5, 1, 2)
    assert abs(lin.dot(lin.prolong(y, 64), x) - lin.dot(y, c)) < 1e-12         # P = (P^T)^T


@pytest.fixture(scope="module")
def two_level():
    D = _disc(n=(2, 2, 1), p=2, mu=0.02)
    W = inputs.random_state(D.mesh.ne, 2, seed=9)
    a = 3.0 / (2 * 0.05)
    K = _dense_K(D, W, a)
    return D, W, a, K


def _prolong_matrix(D, pc):
    ne, nvf, nvc = D.mesh.ne, D.nv, lin.nv_of(pc)
    P = np.zeros((ne * 5 * nvf, ne * 5 * nvc))
    for j in range(P.shape[1]):
        e = np.zeros(ne * 5 * nvc)
        e[j] = 1.0
        P[:, j] = lin.prolong(e.reshape(ne, 5, nvc), nvf).reshape(-1)
    return P


def test_coarse_operator_is_galerkin_projection(two_level):
    """K_1 = P^T K_0 P (Sec. 6.1); its diagonal blocks are the coarse-mode
    sub-blocks of the fine diagonal blocks."""
    D, W, a, K = two_level
    pmg = lin.PMG(D, W, a, [2, 1])
    P = _prolong_matrix(D, 1)
    Kc = P.T @ K @ P
    x = inputs.random_vector(D.mesh.ne, 1, 4)
    assert np.allclose(pmg.op(1, x).reshape(-1), Kc @ x.reshape(-1), rtol=1e-11, atol=1e-10)
    nbc = 5 * 8
    for e in range(D.mesh.ne):
        blk = Kc[e * nbc:(e + 1) * nbc, e * nbc:(e + 1) * nbc]
        LU, piv = pmg.blocks[1]
        r = np.random.default_rng(e).standard_normal(nbc)
        assert np.allclose(blk @ lin.lu_solve(LU[e:e + 1], piv[e:e + 1], r[None])[0], r, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("nu", [1, 2])
def test_two_level_vcycle_closed_form(two_level, nu):
    """With the exact operator on level 0 and an exact coarsest solve, one
    V-cycle from x = 0 equals (I - E) K^-1 b with
    E = S^nu (I - P K_c^-1 P^T K) S^nu,  S = I - omega D^-1 K."""
    D, W, a, K = two_level
    omega = 0.8
    pmg = lin.PMG(D, W, a, [2, 1], nu_pre=nu, nu_post=nu, omega=omega)
    shape = W.shape
    pmg.op = lambda l, x: (K @ x.reshape(-1)).reshape(x.shape) if l == 0 else pmg_op1(x)
    P = _prolong_matrix(D, 1)
    Kc = P.T @ K @ P
    pmg_op1 = lambda x: (Kc @ x.reshape(-1)).reshape(x.shape)
    pmg.coarsest = lambda b: np.linalg.solve(Kc, b.reshape(-1)).reshape(b.shape)
    N = K.shape[0]
    Dinv = np.zeros((N, N))
    LU, piv = pmg.blocks[0]
    nb = 5 * D.nv
    for e in range(D.mesh.ne):
        Dinv[e * nb:(e + 1) * nb, e * nb:(e + 1) * nb] = np.linalg.inv(
            K[e * nb:(e + 1) * nb, e * nb:(e + 1) * nb])
    S = np.eye(N) - omega * Dinv @ K
    Sn = np.linalg.matrix_power(S, nu)
    E = Sn @ (np.eye(N) - P @ np.linalg.solve(Kc, P.T @ K)) @ Sn
    b = inputs.random_vector(D.mesh.ne, 2, 8)
    z = pmg.apply(b).reshape(-1)
    ref = (np.eye(N) - E) @ np.linalg.solve(K, b.reshape(-1))
    assert np.allclose(z, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_fgmres_identity_matches_direct_solve():
    rng = np.random.default_rng(2)
    N = 30
    A = rng.standard_normal((N, N)) + 8 * np.eye(N)
    b = rng.standard_normal(N)
    x, st = lin.fgmres(lambda v: A @ v, lambda v: v, b, restart=N, rtol=1e-13)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10)
    assert st.iters <= N and st.rel_res_true <= 1e-13


def test_gmres_iterates_minimise_over_krylov_space():
    """After k steps, FGMRES with a fixed right preconditioner P and the
    fixed-count GMRES both return argmin ||b - A x|| over x in P K_k(AP, b),
    computed independently by least squares on an orthonormalised Krylov basis."""
    rng = np.random.default_rng(4)
    N, k = 25, 6
    A = rng.standard_normal((N, N)) + 4 * np.eye(N)
    Pm = np.diag(rng.uniform(0.5, 2.0, N))
    b = rng.standard_normal(N)
    Kr = [b]
    for _ in range(k - 1):
        Kr.append(A @ Pm @ Kr[-1])
    Q, _ = np.linalg.qr(np.stack(Kr, 1))
    y, *_ = np.linalg.lstsq(A @ Pm @ Q, b, rcond=None)
    ref = Pm @ Q @ y
    x1 = lin.gmres_fixed(lambda v: A @ v, lambda v: Pm @ v, b, k)
    x2, _ = lin.fgmres(lambda v: A @ v, lambda v: Pm @ v, b, restart=k, rtol=1e-300, max_restarts=0)
    assert np.allclose(x1, ref, rtol=1e-9, atol=1e-10)
    assert np.allclose(x2, ref, rtol=1e-9, atol=1e-10)


def test_bdf2_newton_step_conserves_and_converges():
    """One BDF2 step: the mean of every conserved variable is unchanged (the
    residual conserves and W^{n-1} = W^n) and Newton converges in <= 3
    iterations with the exact Jacobian action; a uniform state is a fixed point."""
    D = _disc(n=(2, 2, 2), p=1, mu=0.01)
    Wn = inputs.random_state(D.mesh.ne, 1, seed=12, amp=0.03)
    W1, st = ts.bdf2_step(D, Wn, None, 0.1, precond="bj", restart=30, rtol=1e-10)
    assert st.newton <= 3
    assert st.res_history[-1] <= 1e-10 * st.res_history[0]
    assert all(r <= 1e-10 for r in st.rel_res_true)
    dm = (W1 - Wn)[:, :, 0].sum(0)
    assert np.abs(dm).max() < 1e-11 * np.abs(Wn[:, :, 0]).max()
    U = np.zeros_like(Wn)
    U[:, :, 0] = np.array([1.0, 0.1, 0.2, -0.1, 2.5]) * inputs.MODE0_SCALE
    U1, st = ts.bdf2_step(D, U, None, 0.1, precond="bj")
    assert st.newton == 0 and np.array_equal(U1, U)


class _LinearDecay:
    """Stub discretisation R(W) = lam M W with a fixed symmetric positive
    definite block mass matrix M (complex-safe), for pinning the time scheme
    on its own."""

    def __init__(self, ne=3, nv=8, lam=0.7, seed=0):
        rng = np.random.default_rng(seed)
        A = rng.standard_normal((ne, nv, nv))
        self.M = np.einsum('eij,ekj->eik', A, A) + nv * np.eye(nv)
        self.lam = lam

    def mass(self, v):
        return np.einsum('eij,eaj->eai', self.M, v)

    def residual(self, W):
        return self.lam * self.mass(W)


def test_bdf2_step_closed_form_with_history():
    """Sec. 4, Eq. NEWTON with the BDF2 coefficients: for R(W) = lam M W the
    step M(3W - 4W^n + W^{n-1})/(2 dt) + lam M W = 0 has the closed form
    W = (4W^n - W^{n-1}) / (3 + 2 dt lam), here with W^{n-1} != W^n.  Backward
    Euler (W = W^n / (1 + dt lam)) or a dropped history term fails it."""
    D = _LinearDecay()
    rng = np.random.default_rng(1)
    Wn = rng.standard_normal((3, 5, 8))
    Wnm1 = Wn + 0.3 * rng.standard_normal(Wn.shape)
    dt = 0.4
    W1, st = ts.bdf2_step(D, Wn, Wnm1, dt, precond=None, restart=60, rtol=1e-13, newton_tol=1e-12)
    ref = (4 * Wn - Wnm1) / (3 + 2 * dt * D.lam)
    assert st.newton >= 1
    assert np.allclose(W1, ref, rtol=1e-11, atol=1e-12)
    assert not np.allclose(W1, Wn / (1 + dt * D.lam), rtol=1e-3)


def test_bdf2_is_second_order_in_time():
    """Repeated steps of the stub integrate dW/dt = -lam W with global error
    O(dt^2): halving dt divides the error at t = 1 by about 4.  The history
    of the first step is the exact solution at t = -dt (starting from
    W^{n-1} = W^n instead is an O(dt) perturbation that caps the global
    rate at one)."""
    D = _LinearDecay(lam=1.3)
    W0 = np.random.default_rng(2).standard_normal((3, 5, 8))
    errs = []
    for nsteps in (10, 20, 40):
        dt = 1.0 / nsteps
        Wnm1, Wn = W0 * math.exp(D.lam * dt), W0
        for k in range(nsteps):
            W1, _ = ts.bdf2_step(D, Wn, Wnm1, dt, precond=None, restart=60, rtol=1e-13, newton_tol=1e-12)
            Wnm1, Wn = Wn, W1
        errs.append(np.abs(Wn - W0 * math.exp(-D.lam)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.8, (errs, rates)
