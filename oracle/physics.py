"""Compressible Euler / Navier-Stokes fluxes and the Roe numerical flux.

Test infrastructure (oracle); see oracle/__init__.py.

Conservative state u = (rho, rho*v1, rho*v2, rho*v3, rho*e0), m = 5.  Arrays
carry the state in the last axis (..., 5); flux arrays are (..., 5, 3) with the
last axis the spatial direction; gradients of u are (..., 5, 3) with
G[..., a, j] = d u_a / d x_j.

Every function accepts complex arrays (complex-step differentiation): the only
non-analytic operation, |x|, is replaced by x*sign(Re x).
"""
import numpy as np


def cabs(x):
    """Complex-step-safe absolute value: x * sign(Re x)."""
    return x * np.sign(np.real(x))


def primitives(u, gamma):
    """rho, velocity (...,3), pressure, total enthalpy h0 (Sec. 2 closure:
    p = (gamma-1) rho e, e0 = e + |v|^2/2, h0 = e0 + p/rho)."""
    rho = u[..., 0]
    v = u[..., 1:4] / rho[..., None]
    E = u[..., 4] / rho
    p = (gamma - 1.0) * (u[..., 4] - 0.5 * rho * np.sum(v * v, axis=-1))
    H = E + p / rho
    return rho, v, p, H


def flux_c(u, gamma):
    """Inviscid flux F_c (...,5,3) of Eq. NS: (rho v, rho v(x)v + p I, rho v h0)."""
    rho, v, p, H = primitives(u, gamma)
    F = np.zeros(u.shape + (3,), dtype=np.result_type(u, float))
    eye = np.eye(3)
    F[..., 0, :] = rho[..., None] * v
    F[..., 1:4, :] = rho[..., None, None] * v[..., :, None] * v[..., None, :] + p[..., None, None] * eye
    F[..., 4, :] = rho[..., None] * H[..., None] * v
    return F


def flux_v(u, G, gamma, mu, Pr):
    """Viscous flux F_v (...,5,3) of Eq. PDE, written so that
    du/dt + div F_c + div F_v = 0 reproduces Eq. NS:
        F_v = -(0, tau, tau.v - q),
        tau = 2 mu (S - (div v)/3 I),  S = (grad v + grad v^T)/2,
        q = -(mu/Pr) grad h,  h = e + p/rho = gamma/(gamma-1) p/rho.
    G is the gradient of the conservative variables; F_v is linear in G.
    The velocity and enthalpy gradients follow from the quotient rule."""
    rho, v, p, H = primitives(u, gamma)
    E = u[..., 4] / rho
    gv = (G[..., 1:4, :] - v[..., :, None] * G[..., 0:1, :]) / rho[..., None, None]   # gv[...,i,j] = dv_i/dx_j
    gE = (G[..., 4, :] - E[..., None] * G[..., 0, :]) / rho[..., None]                # dE/dx_j
    gh = gamma * (gE - np.einsum('...i,...ij->...j', v, gv))                           # h = gamma (E - |v|^2/2)
    div = gv[..., 0, 0] + gv[..., 1, 1] + gv[..., 2, 2]
    tau = mu * (gv + np.swapaxes(gv, -1, -2)) - (2.0 / 3.0) * mu * div[..., None, None] * np.eye(3)
    q = -(mu / Pr) * gh
    F = np.zeros(u.shape + (3,), dtype=np.result_type(u, G, float))
    F[..., 1:4, :] = -tau
    F[..., 4, :] = -(np.einsum('...ji,...i->...j', tau, v) - q)
    return F


def roe(uL, uR, n, gamma):
    """Roe approximate Riemann flux (Sec. 3.1) through a face with unit normal
    n pointing from the L (interior, +) side to the R (neighbour, -) side:

        F = 1/2 (F_c(uL) + F_c(uR)).n - 1/2 |A_roe| (uR - uL),

    with |A_roe| d applied through the eigen-decomposition of the Roe-averaged
    Euler Jacobian (sqrt(rho)-weighted v and h0; c^2 = (gamma-1)(h0 - |v|^2/2)):
    acoustic waves v.n -/+ c, an entropy wave and two shear waves at v.n.
    No entropy fix (reading of the paper, which does not mention one)."""
    rL, vL, pL, HL = primitives(uL, gamma)
    rR, vR, pR, HR = primitives(uR, gamma)
    FL = np.einsum('...aj,...j->...a', flux_c(uL, gamma), n)
    FR = np.einsum('...aj,...j->...a', flux_c(uR, gamma), n)
    sL = np.sqrt(rL)
    sR = np.sqrt(rR)
    rt = sL * sR
    vt = (sL[..., None] * vL + sR[..., None] * vR) / (sL + sR)[..., None]
    Ht = (sL * HL + sR * HR) / (sL + sR)
    q2 = np.sum(vt * vt, axis=-1)
    c2 = (gamma - 1.0) * (Ht - 0.5 * q2)
    c = np.sqrt(c2)
    vn = np.sum(vt * n, axis=-1)
    dr = rR - rL
    dp = pR - pL
    dv = vR - vL
    dvn = np.sum(dv * n, axis=-1)
    # wave strengths
    a1 = (dp - rt * c * dvn) / (2.0 * c2)
    a5 = (dp + rt * c * dvn) / (2.0 * c2)
    a2 = dr - dp / c2
    a3 = rt[..., None] * (dv - dvn[..., None] * n)          # shear (vector, tangential)
    l1 = cabs(vn - c)
    l2 = cabs(vn)
    l5 = cabs(vn + c)
    D = np.zeros(uL.shape, dtype=np.result_type(uL, uR, n, float))
    # acoustic wave vn - c: eigenvector (1, v - c n, H - vn c)
    D[..., 0] += l1 * a1
    D[..., 1:4] += (l1 * a1)[..., None] * (vt - c[..., None] * n)
    D[..., 4] += l1 * a1 * (Ht - vn * c)
    # entropy wave: (1, v, |v|^2/2)
    D[..., 0] += l2 * a2
    D[..., 1:4] += (l2 * a2)[..., None] * vt
    D[..., 4] += l2 * a2 * 0.5 * q2
    # shear waves: (0, dv_t, v . dv_t)
    D[..., 1:4] += l2[..., None] * a3
    D[..., 4] += l2 * np.sum(vt * a3, axis=-1)
    # acoustic wave vn + c: (1, v + c n, H + vn c)
    D[..., 0] += l5 * a5
    D[..., 1:4] += (l5 * a5)[..., None] * (vt + c[..., None] * n)
    D[..., 4] += l5 * a5 * (Ht + vn * c)
    return 0.5 * (FL + FR) - 0.5 * D
