"""GPU parity of the HIP DG kernels against the CPU oracle, through the C ABI.

Residual (Sec. 3.1 Eqs. dg_ns, visc_flux, re), J.v (Sec. 5.1 Eq. DG-mf, FD and
exact), mass matrix, projection, diagonal blocks and batched PLU (Sec. 6.3).
Meshes span several elements per direction with odd and even counts, a
one-element-wide periodic axis, straight and curved Q1 elements, p = 1..4,
Euler and Navier-Stokes.

Tolerances (relative L2 over the whole vector unless stated):
  residual, exact J.v, mass, blocks: 1e-12 (same FP64 arithmetic, different
    summation order: a few hundred roundings of O(1) terms);
  FD J.v: 2e-7 against the oracle's FD product with the same step (rounding
    of R(W+hv) is amplified by 1/h ~ 1e6).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1812_04789_amd import binding, inputs          # noqa: E402
from oracle import mesh as omesh, dg as odg, linear as olin  # noqa: E402

L = 2 * math.pi


def _case(n, p, mu, curved, amp=0.15):
    vtx = inputs.box_vertices(n, (0, 0, 0), (L, L, L), amp=amp) if curved else None
    gas = dict(gamma=1.4, mu=mu, Pr=0.71, eta=7.0)
    ctx = binding.Context(n, (0, 0, 0), (L, L, L), p, vertices=vtx, **gas)
    D = odg.Discretization(omesh.BoxMesh(n, (0, 0, 0), (L, L, L), vtx), p, **gas)
    return ctx, D


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a).reshape(-1), dtype=torch.float64, device="cuda")


def _host(t, shape):
    return t.cpu().numpy().reshape(shape)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = [((3, 2, 2), 1), ((3, 2, 2), 2), ((2, 3, 2), 3), ((2, 2, 2), 4), ((3, 1, 2), 2), ((4, 3, 2), 1)]


@pytest.mark.parametrize("n,p", CASES)
@pytest.mark.parametrize("mu", [0.0, 0.02])
@pytest.mark.parametrize("curved", [False, True])
def test_residual_parity(n, p, mu, curved):
    print("residual", n, p, mu, curved, flush=True)
    ctx, D = _case(n, p, mu, curved)
    W = inputs.random_state(ctx.ne, p, seed=11 + p)
    R = _host(ctx.residual(_dev(W)), W.shape)
    Ro = D.residual(W)
    assert _rel(R, Ro) < 1e-12
    assert np.abs(R - Ro).max() < 1e-11 * np.abs(Ro).max()


@pytest.mark.parametrize("n,p", CASES[:4])
@pytest.mark.parametrize("curved", [False, True])
def test_jvp_parity(n, p, curved):
    print("jvp", n, p, curved, flush=True)
    ctx, D = _case(n, p, 0.02, curved)
    W = inputs.random_state(ctx.ne, p, seed=21 + p)
    v = inputs.random_vector(ctx.ne, p, seed=22 + p)
    a = 30.0
    Wd, vd = _dev(W), _dev(v)
    RWd = ctx.residual(Wd)
    ye = _host(ctx.jvp_exact(Wd, vd, a), W.shape)
    yo = olin.jvp_exact(D, W, v, a)
    assert _rel(ye, yo) < 1e-12
    assert np.abs(ye - yo).max() < 1e-11 * np.abs(yo).max()
    yf = _host(ctx.jvp(Wd, RWd, vd, a), W.shape)
    yfo = olin.jvp_fd(D, W, D.residual(W), v, a)
    assert _rel(yf, yfo) < 2e-7
    assert np.abs(yf - yfo).max() < 1e-6 * np.abs(yfo).max()
    assert _rel(yf, yo) < 1e-5            # FD truncation error of Eq. DG-mf itself
    # v = 0 gives y = 0 exactly
    z = ctx.jvp(Wd, RWd, torch.zeros_like(vd), a)
    assert torch.count_nonzero(z).item() == 0


@pytest.mark.parametrize("n,p,curved,mu", [((3, 2, 2), 1, True, 0.02), ((3, 2, 2), 2, False, 0.02),
                                            ((2, 3, 2), 3, True, 0.02), ((3, 1, 2), 2, True, 0.02),
                                            ((2, 2, 2), 4, False, 0.02), ((2, 2, 2), 4, True, 0.02),
                                            ((3, 2, 2), 2, True, 0.0)])
def test_matrix_based_product(n, p, curved, mu):
    """The assembled operator (diagonal blocks + fine face-coupling blocks in
    the 7-block product) applied to v equals the oracle's exact product
    shift M v + (dR/dW) v (both exact: 1e-12), on meshes with and without a
    single-element axis; before assembly the product is refused.  mu = 0:
    Euler."""
    print("matrix-based", n, p, curved, mu, flush=True)
    ctx, D = _case(n, p, mu, curved)
    W = inputs.random_state(ctx.ne, p, seed=41 + p)
    v = inputs.random_vector(ctx.ne, p, seed=42 + p)
    a = 25.0
    with pytest.raises(binding.DGError) as ei:
        ctx.jvp_assembled(_dev(v))
    assert ei.value.status == binding.DG_ESTATE
    ctx.assemble_operator(_dev(W), a)
    y = _host(ctx.jvp_assembled(_dev(v)), W.shape)
    yo = olin.jvp_exact(D, W, v, a)
    assert _rel(y, yo) < 1e-12
    assert np.abs(y - yo).max() < 1e-11 * np.abs(yo).max()


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("curved", [False, True])
def test_mass_and_projection(p, curved):
    ctx, D = _case((2, 3, 2), p, 0.0, curved)
    v = inputs.random_vector(ctx.ne, p, seed=5)
    assert _rel(_host(ctx.mass(_dev(v)), v.shape), D.mass(v)) < 1e-13
    xq = ctx.quad_points().cpu().numpy()
    assert np.abs(xq - D.quad_points()).max() < 1e-13
    vals = inputs.taylor_green(D.quad_points(), mach=0.2)
    W = _host(ctx.project(_dev(vals)), (ctx.ne, 5, ctx.nv))
    assert _rel(W, D.project(vals)) < 1e-13


# Meshes with no single-element axis take the Jacobian-slice kernel (NS: four
# derivative directions; Euler, mu = 0: one), those with one (3 x 1 x 2) the
# per-column kernel.
@pytest.mark.parametrize("n,p,curved,mu", [((3, 2, 2), 1, True, 0.02), ((2, 3, 2), 2, False, 0.02),
                                           ((3, 1, 2), 2, True, 0.02), ((2, 2, 2), 3, True, 0.02),
                                           ((2, 3, 2), 1, False, 0.02), ((3, 2, 2), 1, True, 0.0),
                                           ((2, 2, 3), 2, False, 0.0), ((2, 2, 2), 3, False, 0.0)])
def test_diag_blocks_parity(n, p, curved, mu):
    print("blocks", n, p, curved, mu, flush=True)
    ctx, D = _case(n, p, mu, curved)
    W = inputs.random_state(ctx.ne, p, seed=31)
    a = 12.0
    B = ctx.assemble_diag(_dev(W), a).cpu().numpy()        # [e][col][row]
    Bo = olin.diag_blocks(D, W, a)                         # [e][row][col]
    Bg = np.transpose(B, (0, 2, 1))
    assert np.linalg.norm(Bg - Bo) / np.linalg.norm(Bo) < 1e-12
    assert np.abs(Bg - Bo).max() < 1e-11 * np.abs(Bo).max()


@pytest.mark.parametrize("n,curved,mu", [((2, 2, 2), True, 0.02), ((3, 2, 2), True, 0.02), ((2, 2, 2), False, 0.0)])
def test_diag_blocks_p4_sampled_columns(n, curved, mu):
    """p = 4 diagonal blocks on meshes with no single-element axis (the
    block kernel of the 16^3 workloads; the last case Euler on a straight
    mesh): 24 seeded columns of every block, including the first and last,
    against the oracle's complex-step columns, element by element (1e-12 of
    the largest entry).  The oracle's full 625-column blocks would take
    minutes."""
    print("blocks p=4", n, curved, mu, flush=True)
    ctx, D = _case(n, 4, mu, curved, amp=0.1)
    W = inputs.random_state(ctx.ne, 4, seed=33)
    a = 12.0
    nb = 5 * ctx.nv
    rng = np.random.default_rng(4)
    cols = sorted(set([0, nb - 1] + [int(c) for c in rng.choice(nb, 22, replace=False)]))
    B = np.transpose(ctx.assemble_diag(_dev(W), a).cpu().numpy(), (0, 2, 1))      # [e][row][col]
    Bo = olin.diag_blocks(D, W, a, cols=cols)
    err = np.abs(B[:, :, cols] - Bo[:, :, cols]).max() / np.abs(Bo[:, :, cols]).max()
    print("  max rel err %.2e over %d columns" % (err, len(cols)), flush=True)
    assert err < 1e-12


@pytest.mark.parametrize("n,shift", [(135, 2.0), (1, 0.0), (5, 0.0), (16, 0.0), (17, 0.0), (40, 0.0), (135, 0.0),
                                     (320, 0.0), (320, 2.0)])
def test_batched_lu_parity(n, shift):
    """Blocked PLU against the oracle's partial pivoting: a single partial
    panel (n < 16), an exact panel (16), a one-row remainder (17), the block
    sizes of p = 1, 2, 3 (40, 135, 320) with ragged matrix-core tiles, and
    unshifted random matrices whose pivots leave the panel."""
    rng = np.random.default_rng(7 + n)
    nblk = 6 if n <= 135 else 3
    A = rng.standard_normal((nblk, n, n)) + shift * np.eye(n)
    LUo, pivo = olin.lu_factor(A)
    Ad = torch.tensor(np.ascontiguousarray(np.transpose(A, (0, 2, 1))), device="cuda")   # column-major
    piv = torch.zeros((nblk, n), dtype=torch.int32, device="cuda")
    binding.batched_lu(Ad, piv)
    torch.cuda.synchronize()
    assert np.array_equal(piv.cpu().numpy(), pivo)
    LU = np.transpose(Ad.cpu().numpy(), (0, 2, 1))
    assert np.abs(LU - LUo).max() < 1e-11 * max(1.0, np.abs(LUo).max())
    b = rng.standard_normal((nblk, n))
    x = torch.empty(nblk * n, dtype=torch.float64, device="cuda")
    binding.batched_lu_solve(Ad, piv, _dev(b), x)
    xo = olin.lu_solve(LUo, pivo, b)
    # two backward-stable solves differ by at most ~ n eps cond(A) relative
    cond = max(np.linalg.cond(A[i]) for i in range(nblk))
    assert _rel(x.cpu().numpy().reshape(nblk, n), xo) < 1e-15 * n * cond + 1e-14


def test_free_stream_and_conservation_on_device():
    ctx, D = _case((4, 3, 2), 3, 0.02, True, amp=0.2)
    W = np.zeros((ctx.ne, 5, ctx.nv))
    W[:, :, 0] = np.array([1.1, 0.2, -0.3, 0.1, 3.5]) * inputs.MODE0_SCALE
    R = _host(ctx.residual(_dev(W)), W.shape)
    assert np.abs(R).max() < 1e-12
    W = inputs.random_state(ctx.ne, 3, seed=9)
    R = _host(ctx.residual(_dev(W)), W.shape)
    assert np.abs(R[:, :, 0].sum(0)).max() < 1e-13 * np.abs(R).max() * ctx.ne


def test_residual_is_deterministic():
    ctx, _ = _case((4, 4, 4), 3, 0.02, True)
    W = _dev(inputs.random_state(ctx.ne, 3, seed=2))
    r1 = ctx.residual(W).clone()
    r2 = ctx.residual(W)
    assert torch.equal(r1, r2)


def test_abi_errors():
    ctx, _ = _case((2, 2, 2), 1, 0.0, False)
    W = _dev(inputs.random_state(ctx.ne, 1, seed=1))
    with pytest.raises(binding.DGError) as ei:
        ctx.residual(W, W)                                     # output aliases input
    assert ei.value.status == binding.DG_EINVAL
    with pytest.raises(binding.DGError) as ei:
        ctx.pmg_apply(W)
    assert ei.value.status == binding.DG_ESTATE
    with pytest.raises(binding.DGError):
        ctx.pmg_setup(W, 1.0, binding.pmg_opts([2, 1]))      # p_level[0] != p
    with pytest.raises(binding.DGError):
        binding.Context((2, 2, 2), (0, 0, 0), (1, 1, 1), 5)   # p out of range
    vtx = inputs.box_vertices((2, 2, 2), (0, 0, 0), (L, L, L))
    vtx[0, [0, 1]] = vtx[0, [1, 0]]
    with pytest.raises(binding.DGError):
        binding.Context((2, 2, 2), (0, 0, 0), (L, L, L), 1, vertices=vtx)
