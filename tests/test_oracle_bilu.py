"""Pins of the oracle's block ILU(0) with minimum-discarded-fill ordering
(Sec. 6.3, the coarsest-level preconditioner of Table MGSettings), CPU only."""
import math

import numpy as np
import pytest

from oracle import mesh as msh, dg, linear as lin
from paper_1812_04789_amd import inputs

L2PI = 2 * math.pi


def _random_blocks(edges, n, nb=4, seed=0, dominance=8.0):
    """Random block matrix on an undirected element graph: diagonal blocks
    made dominant, every edge (i, j) giving blocks (i, j) and (j, i)."""
    rng = np.random.default_rng(seed)
    blocks = {(i, i): rng.standard_normal((nb, nb)) + dominance * np.eye(nb) for i in range(n)}
    for i, j in edges:
        blocks[(i, j)] = rng.standard_normal((nb, nb))
        blocks[(j, i)] = rng.standard_normal((nb, nb))
    return blocks


def _dense(blocks, n, nb):
    A = np.zeros((n * nb, n * nb))
    for (i, j), b in blocks.items():
        A[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb] = b
    return A


def _factors_dense(ilu, n, nb):
    """Dense L (unit block-lower in the elimination order) and U."""
    Lm = np.zeros((n * nb, n * nb))
    Um = np.zeros((n * nb, n * nb))
    for i in range(n):
        Lm[i * nb:(i + 1) * nb, i * nb:(i + 1) * nb] = np.eye(nb)
    for (j, k), b in ilu.L.items():
        Lm[j * nb:(j + 1) * nb, k * nb:(k + 1) * nb] = b
    for (k, l), b in ilu.U.items():
        Um[k * nb:(k + 1) * nb, l * nb:(l + 1) * nb] = b
    return Lm, Um


def _box_edges(n):
    m = msh.BoxMesh(n, (0, 0, 0), (1, 1, 1))
    return sorted({(min(e, o), max(e, o)) for e in range(m.ne) for o in m.nbr[e] if o != e}), m.ne


def test_ilu0_reproduces_the_matrix_on_its_pattern():
    """The defining property of ILU(0): the product L U equals A on every
    block of A's sparsity pattern (the discarded fill lies outside it), here
    on a periodic 3x3x2 element graph in MDF order, and L U differs from A
    off the pattern (fill was discarded)."""
    edges, n = _box_edges((3, 3, 2))
    nb = 3
    blocks = _random_blocks(edges, n, nb, seed=1)
    part = {i: 0 for i in range(n)}
    ilu = lin.BlockILU0(blocks, part, lin.mdf_order(blocks, part))
    Lm, Um = _factors_dense(ilu, n, nb)
    # permuted to the elimination order, L is unit lower triangular and U
    # block upper triangular (full diagonal blocks)
    perm = np.concatenate([np.arange(k * nb, (k + 1) * nb) for k in ilu.order])
    assert np.allclose(np.triu(Lm[np.ix_(perm, perm)], 1), 0)
    Up = Um[np.ix_(perm, perm)]
    for bi in range(n):
        for bj in range(bi):
            assert not np.any(Up[bi * nb:(bi + 1) * nb, bj * nb:(bj + 1) * nb])
    LU = Lm @ Um
    A = _dense(blocks, n, nb)
    mask = np.zeros_like(A, dtype=bool)
    for (i, j) in blocks:
        mask[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb] = True
    assert np.allclose(LU[mask], A[mask], rtol=1e-12, atol=1e-12)
    assert np.abs(LU[~mask]).max() > 1e-3


def test_ilu0_is_exact_without_fill():
    """On a tree (a path) no elimination creates fill outside the pattern,
    so block ILU(0) is the exact block LU and apply() is the exact solve;
    MDF eliminates the path from an end (zero discarded fill each time)."""
    n, nb = 6, 4
    edges = [(i, i + 1) for i in range(n - 1)]
    blocks = _random_blocks(edges, n, nb, seed=2)
    part = {i: 0 for i in range(n)}
    order = lin.mdf_order(blocks, part)
    assert order == list(range(n))
    ilu = lin.BlockILU0(blocks, part, order)
    r = np.random.default_rng(3).standard_normal(n * nb)
    z = ilu.apply({i: r[i * nb:(i + 1) * nb] for i in range(n)})
    zz = np.concatenate([z[i] for i in range(n)])
    assert np.allclose(zz, np.linalg.solve(_dense(blocks, n, nb), r), rtol=1e-12, atol=1e-12)


def test_mdf_eliminates_the_weakest_coupling_first():
    """On a 4-cycle 0-1-2-3-0 every first elimination discards the fill
    between its two neighbours; the element whose couplings are weakest
    (scaled down) discards the least and goes first, then the remaining path
    is eliminated from its lowest-index end."""
    n, nb = 4, 3
    edges = [(0, 1), (1, 2), (2, 3), (0, 3)]
    blocks = _random_blocks(edges, n, nb, seed=4)
    for key in list(blocks):
        if 2 in key and key != (2, 2):
            blocks[key] = 1e-3 * blocks[key]
    part = {i: 0 for i in range(n)}
    w = {k: lin.discarded_fill(blocks, lin.block_pattern(blocks), k, set(range(n))) for k in range(n)}
    assert min(w, key=w.get) == 2
    order = lin.mdf_order(blocks, part)
    assert order[0] == 2 and order[1] == 1


def test_partitions_drop_the_couplings_between_them():
    """With every element its own partition, block ILU(0) is block Jacobi."""
    edges, n = _box_edges((2, 2, 2))
    nb = 3
    blocks = _random_blocks(edges, n, nb, seed=5)
    part = {i: i for i in range(n)}
    ilu = lin.BlockILU0(blocks, part, lin.mdf_order(blocks, part))
    r = {i: np.random.default_rng(i).standard_normal(nb) for i in range(n)}
    z = ilu.apply(r)
    for i in range(n):
        assert np.allclose(z[i], np.linalg.solve(blocks[(i, i)], r[i]), rtol=1e-13)


def test_bilu_coarsest_gmres_on_the_dg_coarse_operator():
    """On the inherited p = 1 operator of a p = 2 DG system (blocks from the
    oracle's complex-step columns), BILU-preconditioned GMRES reduces the
    residual more in 8 steps than BJ-preconditioned GMRES, with the element
    lines along x as partitions."""
    V = inputs.box_vertices((3, 2, 2), (0, 0, 0), (L2PI,) * 3, amp=0.1)
    D = dg.Discretization(msh.BoxMesh((3, 2, 2), (0, 0, 0), (L2PI,) * 3, V), 2, mu=0.02, Pr=0.71)
    W = inputs.random_state(D.mesh.ne, 2, seed=7)
    a = 20.0
    blocks = lin.coarse_blocks(D, W, a, 1)
    ne, nbc = D.mesh.ne, 5 * 8
    nx = D.mesh.n[0]
    part = {e: e // nx for e in range(ne)}
    ilu = lin.BlockILU0(blocks, part, lin.mdf_order(blocks, part))
    K = _dense(blocks, ne, nbc)
    b = np.random.default_rng(8).standard_normal(ne * nbc)
    bj = lambda v: np.concatenate([np.linalg.solve(blocks[(e, e)], v[e * nbc:(e + 1) * nbc]) for e in range(ne)])
    il = lambda v: np.concatenate([z for _, z in sorted(ilu.apply({e: v[e * nbc:(e + 1) * nbc]
                                                                     for e in range(ne)}).items())])
    res = []
    for P in (bj, il):
        x = lin.gmres_fixed(lambda v: K @ v, P, b, 8)
        res.append(np.linalg.norm(b - K @ x) / np.linalg.norm(b))
    assert res[1] < res[0]


def test_coarse_blocks_are_the_galerkin_operator():
    """coarse_blocks(D, W, a, pc) holds P^T K P (K = a M + dR/dW, P the
    prolongation) block by block: its dense assembly equals the projection of
    the dense Jacobian."""
    D = dg.Discretization(msh.BoxMesh((3, 2, 1), (0, 0, 0), (L2PI,) * 3), 2, mu=0.02, Pr=0.71)
    W = inputs.random_state(D.mesh.ne, 2, seed=9)
    a = 5.0
    blocks = lin.coarse_blocks(D, W, a, 1)
    ne, nbc, nbf = D.mesh.ne, 40, 5 * D.nv
    Kc = np.zeros((ne * nbc, ne * nbc))
    for j in range(ne * nbc):
        e = np.zeros(ne * nbc)
        e[j] = 1.0
        v = lin.prolong(e.reshape(ne, 5, 8), D.nv)
        Kc[:, j] = lin.restrict(lin.jvp_exact(D, W, v, a), 1).reshape(-1)
    assert np.allclose(_dense(blocks, ne, nbc), Kc, rtol=1e-12, atol=1e-12)
    assert nbf > nbc


def test_pmg_with_bilu_coarsest_level():
    """The V-cycle with a BILU-preconditioned coarsest GMRES is a better
    preconditioner than with block Jacobi there (fewer FGMRES iterations)
    and FGMRES reaches the same solution."""
    V = inputs.box_vertices((3, 2, 2), (0, 0, 0), (L2PI,) * 3, amp=0.1)
    D = dg.Discretization(msh.BoxMesh((3, 2, 2), (0, 0, 0), (L2PI,) * 3, V), 2, mu=0.02, Pr=0.71)
    W = inputs.random_state(D.mesh.ne, 2, seed=11)
    a = 2.0
    b = inputs.random_vector(D.mesh.ne, 2, 12)
    A = lambda v: lin.jvp_exact(D, W, v, a)
    Dblk = lin.diag_blocks(D, W, a)
    its, xs = [], []
    for cp in ("bj", "bilu"):
        pmg = lin.PMG(D, W, a, [2, 1], coarse_iters=4, Dblk=Dblk, coarsest_prec=cp)
        x, st = lin.fgmres(A, pmg.apply, b, restart=60, rtol=1e-10)
        its.append(st.iters)
        xs.append(x)
    assert its[1] <= its[0]
    assert np.allclose(xs[0], xs[1], rtol=1e-7, atol=1e-8 * np.abs(xs[0]).max())
