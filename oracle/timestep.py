"""One implicit BDF2 time step solved by Newton-Krylov.

Test infrastructure (oracle); see oracle/__init__.py.

Sec. 4, Eq. NEWTON gives the Newton iteration for an ESDIRK stage: the
iteration matrix M/(a_ii dt) + dR/dW and the unsteady residual.  With BDF2 in
place of ESDIRK3 (one step, W^{n+1} from W^n and W^{n-1}):

    R_u(W) = M (3 W - 4 W^n + W^{n-1}) / (2 dt) + R(W),
    K      = 3/(2 dt) M + dR/dW,
    Newton: K x = -R_u(W_k),  W_{k+1} = W_k + x.

The preconditioner is built once at W^n and lagged over the whole step (the
"MFL" option of Sec. 7.3).  Newton stops when ||R_u(W_k)|| <= tol ||R_u(W_0)||
(relative reading of the paper's nonlinear tolerance) or when ||R_u(W_k)||
reaches the rounding floor 1e-14 * (3/(2 dt)) ||M W^n|| (the size of the
unsteady term), at most `max_newton` iterations.  A fresh case has no W^{n-1}; it is taken equal to W^n.
"""
import numpy as np

from . import linear as lin


class StepStats:
    def __init__(self):
        self.newton = 0
        self.linear_iters = []
        self.rel_res_true = []
        self.res_history = []


def bdf2_step(D, Wn, Wnm1, dt, precond="pmg", levels=None, restart=40, rtol=1e-8,
              newton_tol=1e-10, max_newton=5, nu_pre=2, nu_post=2, omega=1.0, coarse_iters=30,
              max_restarts=20, jvp="exact", Dblk=None):
    """`jvp` selects the Krylov operator: "exact" (tangent-linear Jacobian
    action) or "fd" (the finite-difference form of Eq. DG-mf).  The FD form
    carries a relative error of about sqrt(machine eps) (1e-8..1e-7 here), so
    relative linear tolerances of 1e-8 and below need the exact action.
    `Dblk` (optional): the diagonal blocks of 3/(2 dt) M + dR/dW at W^n, if
    already computed (linear.diag_blocks), for the preconditioner."""
    a = 3.0 / (2.0 * dt)
    Wnm1 = Wn if Wnm1 is None else Wnm1
    W = Wn.copy()
    RW = D.residual(W)
    if precond == "pmg":
        P = lin.PMG(D, W, a, levels if levels is not None else [D.p], nu_pre, nu_post, omega,
                    coarse_iters, RW=RW, Dblk=Dblk)
    elif precond == "bj":
        P = lin.BlockJacobi(D, W, a, Dblk=Dblk)
    else:
        P = None
    prec = (lambda r: r) if P is None else P.apply
    st = StepStats()

    def unsteady(W, RW):
        return D.mass(3.0 * W - 4.0 * Wn + Wnm1) / (2.0 * dt) + RW

    Ru = unsteady(W, RW)
    r0 = lin.norm(Ru)
    floor = 1e-14 * a * lin.norm(D.mass(Wn))
    st.res_history.append(r0)
    for k in range(max_newton):
        rk = lin.norm(Ru)
        if rk <= newton_tol * r0 or rk <= floor:
            break
        Wk, RWk = W, RW
        if jvp == "fd":
            A = lambda v: lin.jvp_fd(D, Wk, RWk, v, a)
        else:
            A = lambda v: lin.jvp_exact(D, Wk, v, a)
        x, ls = lin.fgmres(A, prec, -Ru, restart, rtol, max_restarts)
        st.linear_iters.append(ls.iters)
        st.rel_res_true.append(ls.rel_res_true)
        W = W + x
        RW = D.residual(W)
        Ru = unsteady(W, RW)
        st.newton += 1
        st.res_history.append(lin.norm(Ru))
    return W, st


# ---- ESDIRK3 (Sec. 4) --------------------------------------------------------------
# The four-stage, third-order, explicit-first-stage singly diagonally implicit
# Runge-Kutta scheme the paper uses (its ref. [bijl2002implicit]), in the
# published rational form of its Butcher tableau (Kennedy & Carpenter's
# ESDIRK3(2)4L[2]SA, as used by Bijl et al. 2002).  The scheme is stiffly
# accurate: the last stage is W^{n+1}.
ESDIRK3_GAMMA = 1767732205903.0 / 4055673282236.0
ESDIRK3_A = [
    [0.0, 0.0, 0.0, 0.0],
    [ESDIRK3_GAMMA, ESDIRK3_GAMMA, 0.0, 0.0],
    [2746238789719.0 / 10658868560708.0, -640167445237.0 / 6845629431997.0, ESDIRK3_GAMMA, 0.0],
    [1471266399579.0 / 7840856788654.0, -4482444167858.0 / 7529755066697.0, 11266239266428.0 / 11593286722821.0,
     ESDIRK3_GAMMA],
]


def esdirk3_step(D, Wn, dt, precond="pmg", levels=None, restart=40, rtol=1e-8, newton_tol=1e-10, max_newton=5,
                 nu_pre=2, nu_post=2, omega=1.0, coarse_iters=30, max_restarts=20, smoother="bj", cycle="v",
                 Dblk=None):
    """One ESDIRK3 step (Sec. 4): stage 1 is W^1 = W^n; stage i = 2, 3, 4 solves

        M (W - W^n) / (a_ii dt) + sum_{j<i} (a_ij / a_ii) R(W^j) + R(W) = 0

    (Eq. NEWTON: iteration matrix M/(a_ii dt) + dR/dW, the same for every
    stage because a_ii = gamma) by Newton from the previous stage's solution,
    each linear system by FGMRES with the exact Jacobian action.  The
    preconditioner is built once, at W^n, and lagged over all stages (the MFL
    option of Sec. 7.3).  W^{n+1} = W^4 (stiffly accurate; the printed update
    formula of Sec. 4 is garbled).  Newton stops per stage as in bdf2_step:
    ||R_s(W_k)|| <= tol ||R_s(W_0)|| or below the rounding floor
    1e-14 ||M W^n|| / (gamma dt)."""
    A, g = ESDIRK3_A, ESDIRK3_GAMMA
    a = 1.0 / (g * dt)
    RWn = D.residual(Wn)
    if precond == "pmg":
        P = lin.PMG(D, Wn, a, levels if levels is not None else [D.p], nu_pre, nu_post, omega, coarse_iters,
                    RW=RWn, Dblk=Dblk, smoother=smoother, cycle=cycle)
    elif precond == "bj":
        P = lin.BlockJacobi(D, Wn, a, Dblk=Dblk)
    else:
        P = None
    prec = (lambda r: r) if P is None else P.apply
    st = StepStats()
    floor = 1e-14 * a * lin.norm(D.mass(Wn))
    Rstage = [RWn]
    W = Wn.copy()
    for i in range(1, 4):
        explicit = sum(A[i][j] / g * Rstage[j] for j in range(i))

        def stage_residual(W, RW):
            return D.mass(W - Wn) * a + explicit + RW

        RW = D.residual(W)
        Ru = stage_residual(W, RW)
        r0 = lin.norm(Ru)
        st.res_history.append(r0)
        for k in range(max_newton):
            rk = lin.norm(Ru)
            if rk <= newton_tol * r0 or rk <= floor:
                break
            Wk = W
            x, ls = lin.fgmres(lambda v: lin.jvp_exact(D, Wk, v, a), prec, -Ru, restart, rtol, max_restarts)
            st.linear_iters.append(ls.iters)
            st.rel_res_true.append(ls.rel_res_true)
            W = W + x
            RW = D.residual(W)
            Ru = stage_residual(W, RW)
            st.newton += 1
            st.res_history.append(lin.norm(Ru))
        Rstage.append(RW)
    return W, st
