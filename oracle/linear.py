"""Linearisation, block-Jacobi, p-multigrid V-cycle and FGMRES.

Test infrastructure (oracle); see oracle/__init__.py.

Vectors are arrays (ne, 5, nv_l) in the modal layout of dg.py; level l keeps
the first nv_l = (p_l+1)^3 modes of every element (hierarchical order), which
is the reference-element L2 projection of Sec. 6.1 for an orthonormal basis.

Iteration matrix (Sec. 5.1, Eq. ODEDG):  K = a M + dR/dW, with a the shift
(1/(a_ii dt) in the paper's ESDIRK, 3/(2 dt) for BDF2).
"""
import numpy as np


def norm(x):
    return float(np.sqrt(np.sum(np.real(x) ** 2)))


# ---- Jacobian-vector products (Sec. 5.1, Eq. DG-mf) -------------------------
EPS_FD = 1e-7


def fd_step(W, v, eps=EPS_FD, printed=False):
    """Finite-difference step.  As printed, h = eps sqrt(1+||dW||)/||W||, which
    does not scale with dW; the reading used is the usual
    h = eps sqrt(1+||W||)/||dW|| (global Euclidean norms).  `printed=True`
    selects the printed form."""
    nW, nv = norm(W), norm(v)
    if printed:
        return eps * np.sqrt(1.0 + nv) / nW
    return eps * np.sqrt(1.0 + nW) / nv


def jvp_fd(D, W, RW, v, shift, eps=EPS_FD, printed=False):
    """y = a M v + (R(W + h v) - R(W))/h   (Eq. DG-mf).  y = a M v if v = 0."""
    nv = norm(v)
    if nv == 0.0:
        return shift * D.mass(v)
    h = fd_step(W, v, eps, printed)
    return shift * D.mass(v) + (D.residual(W + h * v) - RW) / h


H_CS = 1e-30


def jvp_exact(D, W, v, shift):
    """y = a M v + dR/dW v by complex-step differentiation:
    dR/dW v = Im R(W + i h v)/h  (exact to rounding; no cancellation)."""
    return shift * D.mass(v) + np.imag(D.residual(W + 1j * H_CS * v)) / H_CS


# ---- diagonal blocks (Sec. 6.3 block Jacobi; Sec. 6.3 selective assembly) ----
def face_colouring(mesh):
    """Greedy colouring so that no two face-neighbours share a colour (an
    element may be its own neighbour on a one-element-wide periodic axis)."""
    col = -np.ones(mesh.ne, dtype=np.int64)
    for e in range(mesh.ne):
        used = {col[o] for o in mesh.nbr[e] if o != e and col[o] >= 0}
        c = 0
        while c in used:
            c += 1
        col[e] = c
    return col


def diag_blocks(D, W, shift, cols=None):
    """Element diagonal blocks of K: Dblk[e] (nb, nb), nb = 5 nv, row/column
    index a*nv + i (equation-major, as W[e, a, i]).

    Column j of every block is Im R(W + i h e_j)/h restricted to the element,
    perturbing local DOF j of every element of one colour class at once; the
    colouring makes the restriction exact.  `cols` (optional) limits the
    evaluation to those column indices (the other columns stay zero)."""
    ne, nv = D.mesh.ne, D.nv
    nb = 5 * nv
    col = face_colouring(D.mesh)
    Dblk = np.zeros((ne, nb, nb))
    for c in range(col.max() + 1):
        sel = np.nonzero(col == c)[0]
        for j in (range(nb) if cols is None else cols):
            a, i = divmod(j, nv)
            Wc = W.astype(complex)
            Wc[sel, a, i] += 1j * H_CS
            Rc = np.imag(D.residual(Wc)) / H_CS
            Dblk[sel, :, j] = Rc[sel].reshape(len(sel), nb)
    # a M: M_e acts on each equation separately
    for a in range(5):
        Dblk[:, a * nv:(a + 1) * nv, a * nv:(a + 1) * nv] += shift * D.M
    if cols is not None:
        keep = np.zeros(nb, dtype=bool)
        keep[list(cols)] = True
        Dblk[:, :, ~keep] = 0.0
    return Dblk


# ---- dense PLU with partial pivoting (Sec. 6.3, element-wise PLU) -------------
def lu_factor(A):
    """Doolittle LU with partial pivoting of a stack of square matrices.

    Returns (LU, piv) in the LAPACK convention: at step k rows k and piv[k]
    were exchanged; LU holds U on and above the diagonal and the unit-lower
    L multipliers below it."""
    LU = np.array(A, dtype=float, copy=True)
    nbk, n, _ = LU.shape
    piv = np.zeros((nbk, n), dtype=np.int64)
    rows = np.arange(nbk)
    for k in range(n):
        r = k + np.argmax(np.abs(LU[:, k:, k]), axis=1)
        piv[:, k] = r
        tmp = LU[rows, k, :].copy()
        LU[rows, k, :] = LU[rows, r, :]
        LU[rows, r, :] = tmp
        LU[:, k + 1:, k] /= LU[:, k, k][:, None]
        LU[:, k + 1:, k + 1:] -= LU[:, k + 1:, k][:, :, None] * LU[:, k, k + 1:][:, None, :]
    return LU, piv


def lu_solve(LU, piv, b):
    """Solve A x = b for every block; b (nblk, n)."""
    x = np.array(b, dtype=float, copy=True)
    nbk, n = x.shape
    rows = np.arange(nbk)
    for k in range(n):
        r = piv[:, k]
        tmp = x[rows, k].copy()
        x[rows, k] = x[rows, r]
        x[rows, r] = tmp
    for k in range(n):                      # unit lower
        x[:, k + 1:] -= LU[:, k + 1:, k] * x[:, k][:, None]
    for k in range(n - 1, -1, -1):          # upper
        x[:, k] /= LU[:, k, k]
        x[:, :k] -= LU[:, :k, k] * x[:, k][:, None]
    return x


# ---- p-multigrid (Sec. 6, Alg. 2; Sec. 6.1 subspace inheritance) ------------
def nv_of(p):
    return (p + 1) ** 3


def restrict(x, p_coarse):
    """L2 restriction onto degree p_coarse (Sec. 6.1): with an orthonormal
    hierarchical basis, the coefficients of the coarse modes are kept."""
    return x[:, :, :nv_of(p_coarse)].copy()


def prolong(x, nv_fine):
    """Prolongation = transpose of the restriction: zero the fine modes."""
    out = np.zeros(x.shape[:2] + (nv_fine,))
    out[:, :, :x.shape[2]] = x
    return out


def sub_block_index(nv_f, nv_c):
    """Rows of a fine block that belong to the coarse space, in coarse order."""
    return np.array([a * nv_f + i for a in range(5) for i in range(nv_c)])


class PMG:
    """p-multigrid preconditioner (Sec. 6), lagged at the state W it was set up at.

    levels: polynomial degrees, finest first (e.g. [3, 2, 1]).
    Level 0 operator: the matrix-free FD product (Eq. DG-mf); coarse operators
    are the Galerkin-inherited K_l = P_l^T K_0 P_l (Sec. 6.1), applied here as
    P_l^T (K_0 (P_l x)) with the exact Jacobian action.  Coarsest SOLVE:
    right-preconditioned GMRES(BJ) for a fixed number of iterations.  The BJ
    blocks of level l are the principal coarse-mode sub-blocks of the fine
    diagonal blocks (which is what the block projection M K M^T of Sec. 6.1
    gives on the diagonal).

    smoother: "bj" = nu damped block-Jacobi sweeps x <- x + omega D^-1 (b - K x);
              "gmres" = nu iterations of right-preconditioned GMRES(BJ) on the
              residual equation, x <- x + GMRES(K, D^-1, b - K x) (the
              smoothers of Sec. 6 and Table MGSettings).
    cycle:    "v" = one V-cycle from zero (Alg. 2);
              "fmg" = the full multigrid cycle of Alg. 1 (coarsest solve, then
              a V-cycle on each finer level from the prolonged coarser result)."""

    def __init__(self, D, W, shift, levels, nu_pre=2, nu_post=2, omega=1.0, coarse_iters=30,
                 RW=None, Dblk=None, coarse_op="exact", smoother="bj", cycle="v", coarsest_prec="bj"):
        """coarse_op: "exact" applies P^T K_0 P with the exact Jacobian action
        (the inherited operator of Sec. 6.1); "fd" applies P^T K_FD P with the
        finite-difference product, a matrix-free approximation of it.
        coarsest_prec: "bj" (element block Jacobi) or "bilu" (block ILU(0) in
        minimum-discarded-fill order, Sec. 6.3 and Table MGSettings; partitions
        are the element lines along x, couplings between lines dropped) as the
        right preconditioner of the coarsest GMRES."""
        assert smoother in ("bj", "gmres") and cycle in ("v", "fmg") and coarsest_prec in ("bj", "bilu")
        self.smoother, self.cycle, self.coarsest_prec = smoother, cycle, coarsest_prec
        self.coarse_op = coarse_op
        self.D, self.W, self.shift = D, W, shift
        self.RW = D.residual(W) if RW is None else RW
        self.levels = list(levels)
        assert self.levels[0] == D.p
        self.nu_pre, self.nu_post, self.omega, self.coarse_iters = nu_pre, nu_post, omega, coarse_iters
        Dfine = diag_blocks(D, W, shift) if Dblk is None else Dblk
        self.blocks = []
        nvf = D.nv
        for p in self.levels:
            idx = sub_block_index(nvf, nv_of(p))
            self.blocks.append(lu_factor(Dfine[:, idx][:, :, idx]))
        self.bilu = None
        if coarsest_prec == "bilu" and len(self.levels) > 1:
            cb = coarse_blocks(D, W, shift, self.levels[-1])
            nx = D.mesh.n[0]
            part = {e: e // nx for e in range(D.mesh.ne)}
            self.bilu = BlockILU0(cb, part, mdf_order(cb, part))

    def op(self, l, x):
        D = self.D
        if l == 0:
            return jvp_fd(D, self.W, self.RW, x, self.shift)
        xf = prolong(x, D.nv)
        if self.coarse_op == "fd":
            return restrict(jvp_fd(D, self.W, self.RW, xf, self.shift), self.levels[l])
        return restrict(jvp_exact(D, self.W, xf, self.shift), self.levels[l])

    def bj(self, l, r):
        LU, piv = self.blocks[l]
        ne = r.shape[0]
        return lu_solve(LU, piv, r.reshape(ne, -1)).reshape(r.shape)

    def smooth(self, l, x, b, nu, x_is_zero):
        """SMOOTH of Alg. 2 on level l from x (x = 0 when x_is_zero)."""
        if self.smoother == "gmres":
            if nu == 0:
                return x
            r = b if x_is_zero else b - self.op(l, x)
            return x + gmres_fixed(lambda v: self.op(l, v), lambda v: self.bj(l, v), r, nu)
        for s in range(nu):
            if s == 0 and x_is_zero:
                x = self.omega * self.bj(l, b)          # K 0 = 0
            else:
                x = x + self.omega * self.bj(l, b - self.op(l, x))
        return x

    def coarsest_prec_apply(self, r):
        L = len(self.levels) - 1
        if self.bilu is None:
            return self.bj(L, r)
        z = self.bilu.apply({e: r[e].reshape(-1) for e in range(r.shape[0])})
        return np.stack([z[e] for e in range(r.shape[0])]).reshape(r.shape)

    def coarsest(self, b):
        L = len(self.levels) - 1
        return gmres_fixed(lambda x: self.op(L, x), self.coarsest_prec_apply, b, self.coarse_iters)

    def vcycle(self, l, b, x=None):
        """Alg. 2 MG_V(l, b, x); x = None is the zero initial guess."""
        if l == len(self.levels) - 1:
            return self.coarsest(b)
        zero = x is None
        if zero:
            x = np.zeros_like(b)
        x = self.smooth(l, x, b, self.nu_pre, zero)
        r = b - self.op(l, x)
        e = self.vcycle(l + 1, restrict(r, self.levels[l + 1]))
        x = x + prolong(e, nv_of(self.levels[l]))
        return self.smooth(l, x, b, self.nu_post, False)

    def fmg(self, b):
        """Alg. 1 MG_full: b_l is the restriction of the level-0 right-hand side
        to level l; the coarsest level is solved, then every finer level runs
        one V-cycle from the prolongation of the coarser level's result."""
        L = len(self.levels) - 1
        x = self.coarsest(restrict(b, self.levels[L]))
        for l in range(L - 1, -1, -1):
            bl = restrict(b, self.levels[l])
            x = self.vcycle(l, bl, prolong(x, nv_of(self.levels[l])))
        return x

    def apply(self, r):
        if len(self.levels) == 1:
            return self.bj(0, r)        # single grid: z = D^-1 r
        if self.cycle == "fmg":
            return self.fmg(r)
        return self.vcycle(0, r)


class BlockJacobi:
    """Single-grid element block-Jacobi preconditioner: z = D^-1 r (Sec. 6.3)."""

    def __init__(self, D, W, shift, Dblk=None):
        Dfine = diag_blocks(D, W, shift) if Dblk is None else Dblk
        self.LU, self.piv = lu_factor(Dfine)

    def apply(self, r):
        ne = r.shape[0]
        return lu_solve(self.LU, self.piv, r.reshape(ne, -1)).reshape(r.shape)


# ---- Krylov ----------------------------------------------------------------
def dot(a, b):
    return float(np.sum(a * b))


def gmres_fixed(A, Minv, b, iters):
    """Right-preconditioned GMRES from x0 = 0, exactly `iters` Arnoldi steps
    (fewer only on a lucky breakdown), modified Gram-Schmidt, least squares
    by Givens rotations.  Used as the coarsest-level SOLVE."""
    beta = norm(b)
    if beta == 0.0:
        return np.zeros_like(b)
    V = [b / beta]
    Z = []
    H = np.zeros((iters + 1, iters))
    cs, sn = np.zeros(iters), np.zeros(iters)
    g = np.zeros(iters + 1)
    g[0] = beta
    k = 0
    for j in range(iters):
        z = Minv(V[j])
        Z.append(z)
        w = A(z)
        for i in range(j + 1):
            H[i, j] = dot(w, V[i])
            w = w - H[i, j] * V[i]
        H[j + 1, j] = norm(w)
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        rr = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / rr, H[j + 1, j] / rr
        hj1 = H[j + 1, j]
        H[j, j] = rr
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        if hj1 <= 1e-14 * beta:
            break
        V.append(w / hj1)
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k]) if k else np.zeros(0)
    x = np.zeros_like(b)
    for i in range(k):
        x = x + y[i] * Z[i]
    return x


class FGMRESStats:
    def __init__(self):
        self.iters = 0
        self.restarts = 0
        self.rel_res_true = np.nan
        self.rel_res_est = np.nan
        self.history = []


def fgmres(A, prec, b, restart, rtol, max_restarts=20, x0=None):
    """Flexible GMRES(m) (Saad 1993, Sec. 6): right preconditioning with a
    preconditioner that may change between iterations (one p-multigrid cycle),
    z_j = P(v_j) stored, x = x0 + Z y.  Modified Gram-Schmidt, Givens rotations.
    Converged when the recomputed true residual ||b - A x|| <= rtol ||b||;
    otherwise restart from the current x.  Returns (x, stats)."""
    st = FGMRESStats()
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = norm(b)
    if bn == 0.0:
        st.rel_res_true = st.rel_res_est = 0.0
        return x, st
    r = b - A(x) if x0 is not None else b.copy()
    for rs in range(max_restarts + 1):
        beta = norm(r)
        st.history.append(beta / bn)
        if beta <= rtol * bn:
            st.rel_res_true = beta / bn
            return x, st
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        k = 0
        for j in range(restart):
            z = prec(V[j])
            Z.append(z)
            w = A(z)
            for i in range(j + 1):
                H[i, j] = dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = norm(w)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rr = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / rr, H[j + 1, j] / rr
            hj1 = H[j + 1, j]
            H[j, j] = rr
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            st.iters += 1
            st.rel_res_est = abs(g[j + 1]) / bn
            st.history.append(st.rel_res_est)
            if abs(g[j + 1]) <= rtol * bn or hj1 == 0.0:
                break
            V.append(w / hj1)
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        for i in range(k):
            x = x + y[i] * Z[i]
        r = b - A(x)
        st.rel_res_true = norm(r) / bn
        if st.rel_res_true <= rtol:
            return x, st
        st.restarts += 1
    return x, st


# ---- assembled inherited coarse operator (Sec. 6.1) ---------------------------------
def distance2_colouring(mesh):
    """Greedy colouring in which no two elements of one colour are face
    neighbours or share a face neighbour."""
    near = []
    for e in range(mesh.ne):
        s = {e} | set(int(o) for o in mesh.nbr[e])
        for o in list(s):
            s |= set(int(x) for x in mesh.nbr[o])
        near.append(s)
    col = -np.ones(mesh.ne, dtype=np.int64)
    for e in range(mesh.ne):
        used = {col[o] for o in near[e] if col[o] >= 0}
        c = 0
        while c in used:
            c += 1
        col[e] = c
    return col


def coarse_blocks(D, W, shift, pc):
    """Blocks of the inherited operator K_l = P^T K_0 P (Sec. 6.1) of degree pc,
    K_0 = shift M + dR/dW at W: {(i, j): block}, rows of element i and columns
    of element j over the coarse modes (equation-major, as W[e, a, i]), for
    j = i and j a face neighbour of i.  Column c of every block comes from the
    complex-step derivative of R for the coarse DOF c of all elements of one
    distance-2 colour class at once (no row element sees two perturbed
    elements)."""
    mesh = D.mesh
    nvc = nv_of(pc)
    nbc = 5 * nvc
    rows = sub_block_index(D.nv, nvc)
    col = distance2_colouring(mesh)
    blocks = {}
    for e in range(mesh.ne):
        blocks[(e, e)] = np.zeros((nbc, nbc))
        for o in mesh.nbr[e]:
            if o != e:
                blocks[(int(o), e)] = np.zeros((nbc, nbc))
    for c in range(col.max() + 1):
        sel = np.nonzero(col == c)[0]
        for j in range(nbc):
            a, i = divmod(j, nvc)
            Wc = W.astype(complex)
            Wc[sel, a, i] += 1j * H_CS
            Rc = (np.imag(D.residual(Wc)) / H_CS).reshape(mesh.ne, -1)[:, rows]
            for e in sel:
                blocks[(e, e)][:, j] = Rc[e]
                for o in set(int(x) for x in mesh.nbr[e]):
                    if o != e:
                        blocks[(o, e)][:, j] = Rc[o]
    Msub = D.M[:, :nvc, :nvc]
    for e in range(mesh.ne):
        for a in range(5):
            blocks[(e, e)][a * nvc:(a + 1) * nvc, a * nvc:(a + 1) * nvc] += shift * Msub[e]
    return blocks


# ---- block ILU(0) with minimum-discarded-fill ordering (Sec. 6.3) --------------------
# A block matrix on the element graph is held as a dict {(i, j): nb x nb array}
# with (i, i) the diagonal blocks and (i, j), j a face neighbour of i, the
# coupling blocks (row block i, column block j).  `part[i]` names the
# partition of element i: the factorisation is done on each partition's
# square block of the matrix, couplings between partitions are dropped (the
# partition-wise "BILU" of Sec. 6.3).

def block_pattern(blocks):
    """Neighbour sets {i: set(j)} of the off-diagonal blocks present."""
    nbr = {}
    for (i, j) in blocks:
        nbr.setdefault(i, set())
        if i != j:
            nbr[i].add(j)
    return nbr


def discarded_fill(blocks, nbr, k, alive):
    """Frobenius norm of the fill that eliminating k discards in ILU(0): the
    blocks A_jk A_kk^-1 A_kl for ordered pairs j != l of k's neighbours still
    to be eliminated whose (j, l) block is not in the pattern (Persson &
    Peraire's minimum-discarded-fill weight), on the unfactored blocks."""
    Dinv = np.linalg.inv(blocks[(k, k)])
    js = [j for j in sorted(nbr[k]) if j in alive]
    w = 0.0
    for j in js:
        for l in js:
            if j != l and l not in nbr[j]:
                w += float(np.sum((blocks[(j, k)] @ Dinv @ blocks[(k, l)]) ** 2))
    return np.sqrt(w)


MDF_TIE = 1e-10


def mdf_order(blocks, part):
    """Minimum-discarded-fill ordering within each partition: repeatedly
    eliminate the element whose elimination discards the least fill.  Ties
    (weights within a relative MDF_TIE of the smallest, so that rounding of
    the weights does not decide) go to the lowest element index.  Returns the
    elements in elimination order (partitions one after another, in
    increasing partition id)."""
    nbr_all = block_pattern(blocks)
    order = []
    for pid in sorted(set(part.values())):
        elems = [i for i in sorted(part) if part[i] == pid]
        nbr = {i: {j for j in nbr_all[i] if part[j] == pid} for i in elems}
        alive = set(elems)
        while alive:
            w = {k: discarded_fill(blocks, nbr, k, alive) for k in alive}
            wmin = min(w.values())
            best = min(k for k in alive if w[k] <= wmin * (1.0 + MDF_TIE))
            order.append(best)
            alive.remove(best)
    return order


class BlockILU0:
    """Block ILU(0) of the partition-wise blocks in a given elimination order
    (Sec. 6.3): for each k in order, L_jk = A_jk A_kk^-1 for the later
    neighbours j of k, and A_jl -= L_jk A_kl for later neighbours j, l of k
    whenever (j, l) is in the pattern (j == l included); other fill is
    discarded.  U keeps the updated blocks A_kk and A_kl (l later than k).
    apply(r) solves L U z = r by a forward sweep in order and a backward
    sweep in reverse order.  r and z are dicts {element: vector}."""

    def __init__(self, blocks, part, order):
        self.part = part
        self.order = list(order)
        self.pos = {k: i for i, k in enumerate(self.order)}
        nbr_all = block_pattern(blocks)
        self.nbr = {i: {j for j in nbr_all[i] if part[j] == part[i]} for i in part}
        A = {key: np.array(v, dtype=float, copy=True) for key, v in blocks.items()
             if part[key[0]] == part[key[1]]}
        self.L = {}
        for k in self.order:
            Dinv = np.linalg.inv(A[(k, k)])
            later = sorted(j for j in self.nbr[k] if self.pos[j] > self.pos[k])
            for j in later:
                self.L[(j, k)] = A[(j, k)] @ Dinv
            for j in later:
                for l in later:
                    if j == l or l in self.nbr[j]:
                        A[(j, l)] = A[(j, l)] - self.L[(j, k)] @ A[(k, l)]
        self.U = {(k, l): A[(k, l)] for k in self.order for l in [k] + sorted(self.nbr[k])
                  if self.pos[l] >= self.pos[k]}

    def apply(self, r):
        y = {}
        for k in self.order:
            v = np.array(r[k], dtype=float, copy=True)
            for j in self.nbr[k]:
                if self.pos[j] < self.pos[k]:
                    v -= self.L[(k, j)] @ y[j]
            y[k] = v
        z = {}
        for k in reversed(self.order):
            v = y[k].copy()
            for l in self.nbr[k]:
                if self.pos[l] > self.pos[k]:
                    v -= self.U[(k, l)] @ z[l]
            z[k] = np.linalg.solve(self.U[(k, k)], v)
        return z
