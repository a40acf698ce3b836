"""Seeded synthetic inputs shared by the library's callers and the tests.

This module holds no arithmetic of the DG method: it produces mesh vertex
tables, initial conditions as point functions of physical coordinates, and
seeded random arrays.  Each consumer evaluates and projects them with its own
code.  It imports nothing else from this package.

Workloads (all periodic boxes, conserved variables (rho, rho v, rho e0)):

  * isentropic vortex: the commonly published isentropic Euler vortex
    (e.g. Shu, "Essentially non-oscillatory and weighted essentially
    non-oscillatory schemes for hyperbolic conservation laws", 1998):
    free stream rho = p = T = 1 (R = 1), velocity M c_inf along x,
    vortex of strength beta centred at (xc, yc), uniform in z:
        du = -beta/(2 pi) (y - yc) exp((1 - r^2)/2),
        dv =  beta/(2 pi) (x - xc) exp((1 - r^2)/2),
        T  = 1 - (gamma - 1) beta^2 / (8 gamma pi^2) exp(1 - r^2),
        rho = T^(1/(gamma-1)),  p = rho T.
  * Taylor-Green vortex (Taylor & Green 1937, in the form used by the
    high-order CFD workshops): rho0 = V0 = L = 1, p0 = 1/(gamma M^2),
        u =  sin x cos y cos z,  v = -cos x sin y cos z,  w = 0,
        p = p0 + (cos 2x + cos 2y)(cos 2z + 2)/16,  rho = p / p0.
  * random-phase Fourier velocity field on a uniform state.
"""
import math

import numpy as np


# ---- meshes -----------------------------------------------------------------
def box_vertices(n, lo, hi, amp=0.0, phase=0.0):
    """Vertex table (ne, 8, 3) of a periodic box of n = (nx,ny,nz) hexahedra.

    Local vertex v = i + 2j + 4k of element (I,J,K) is grid node
    (I+i, J+j, K+k).  With amp != 0 every node is displaced by
    amp * h * sin(x+phase) sin(y+phase) sin(z+phase) in each coordinate
    (h = the x spacing), evaluated at the node's position wrapped into the box
    so that the copies of a node seen across a periodic boundary differ by
    exactly one period.  (With phase = 0 the nodes of a 2-element-wide
    [0, 2pi] axis sit where sin vanishes and do not move.)"""
    nx, ny, nz = (int(x) for x in n)
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    L = hi - lo
    h = L / np.array([nx, ny, nz], float)
    V = np.zeros((nx * ny * nz, 8, 3))
    for K in range(nz):
        for J in range(ny):
            for I in range(nx):
                e = I + nx * (J + ny * K)
                for v in range(8):
                    g = np.array([I + (v & 1), J + ((v >> 1) & 1), K + ((v >> 2) & 1)])
                    nn = np.array([nx, ny, nz])
                    wrap = g % nn
                    base = lo + h * wrap
                    disp = amp * h[0] * math.sin(base[0] + phase) * math.sin(base[1] + phase) * math.sin(base[2] + phase)
                    V[e, v] = base + disp + L * (g // nn)
    return V


# ---- initial conditions as point functions ------------------------------------
def conserved(rho, vel, p, gamma):
    """(rho, rho v, rho e0) from primitive point values; arrays (...,)."""
    E = p / (gamma - 1.0) + 0.5 * rho * np.sum(vel * vel, axis=-1)
    return np.concatenate([rho[..., None], rho[..., None] * vel, E[..., None]], axis=-1)


def isentropic_vortex(x, gamma=1.4, mach=0.5, beta=5.0, xc=5.0, yc=5.0):
    x = np.asarray(x, float)
    dx = x[..., 0] - xc
    dy = x[..., 1] - yc
    r2 = dx * dx + dy * dy
    f = np.exp(0.5 * (1.0 - r2))
    uinf = mach * math.sqrt(gamma)
    vel = np.zeros(x.shape)
    vel[..., 0] = uinf - beta / (2 * math.pi) * dy * f
    vel[..., 1] = beta / (2 * math.pi) * dx * f
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2) * f * f
    assert np.all(T > 0.0)
    rho = T ** (1.0 / (gamma - 1.0))
    return conserved(rho, vel, rho * T, gamma)


def taylor_green(x, gamma=1.4, mach=0.1):
    x = np.asarray(x, float)
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    p0 = 1.0 / (gamma * mach * mach)
    vel = np.zeros(x.shape)
    vel[..., 0] = np.sin(X) * np.cos(Y) * np.cos(Z)
    vel[..., 1] = -np.cos(X) * np.sin(Y) * np.cos(Z)
    p = p0 + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    rho = p / p0
    return conserved(rho, vel, p, gamma)


def fourier_phases(seed, kmax=4):
    """Integer wavevectors 1 <= |k|_inf <= kmax and seeded phases (nk, 3)."""
    ks = [(a, b, c) for a in range(-kmax, kmax + 1) for b in range(-kmax, kmax + 1)
          for c in range(-kmax, kmax + 1) if max(abs(a), abs(b), abs(c)) >= 1]
    rng = np.random.default_rng(seed)
    return np.array(ks, float), rng.uniform(0.0, 2 * math.pi, size=(len(ks), 3))


def _fourier_raw(y, ks, phases, L):
    """sum_k cos(k.y 2pi/L + phi_{k,c}) for c = 0, 1, 2, evaluated as the real
    part of sum_k e^{i phi} e^{i k1 y1'} e^{i k2 y2'} e^{i k3 y3'}, contracted
    one axis at a time (same sum, far fewer transcendental evaluations)."""
    y = np.asarray(y, float).reshape(-1, 3) * (2 * math.pi / L)
    ki = ks.astype(int)
    kmax = int(np.abs(ki).max())
    m = 2 * kmax + 1
    ax = np.arange(-kmax, kmax + 1)
    E = [np.exp(1j * np.outer(y[:, d], ax)) for d in range(3)]       # (npts, m) per axis
    out = np.empty((y.shape[0], 3))
    for c in range(3):
        C = np.zeros((m, m, m), complex)
        C[ki[:, 0] + kmax, ki[:, 1] + kmax, ki[:, 2] + kmax] = np.exp(1j * phases[:, c])
        t = E[2] @ C.reshape(m * m, m).T                                  # (npts, m*m): sum over k3
        t = np.einsum('pab,pb->pa', t.reshape(-1, m, m), E[1])            # sum over k2
        out[:, c] = np.einsum('pa,pa->p', t, E[0]).real                   # sum over k1
    return out


def fourier_velocity(x, ks, phases, amp=0.1, L=2 * math.pi):
    """sum_k cos(k.x 2pi/L + phi_{k,c}) per component, scaled so that its RMS
    over a uniform 16^3 sample grid of the box is `amp`."""
    x = np.asarray(x, float)
    g = (np.arange(16) + 0.5) * L / 16
    G = np.stack(np.meshgrid(g, g, g, indexing='ij'), axis=-1).reshape(-1, 3)
    rms = math.sqrt(float(np.mean(np.sum(_fourier_raw(G, ks, phases, L) ** 2, axis=-1))))
    return (_fourier_raw(x, ks, phases, L) * (amp / rms)).reshape(x.shape)


def fourier_state(x, ks, phases, gamma=1.4, mach=0.3, amp=0.1):
    x = np.asarray(x, float)
    rho = np.ones(x.shape[:-1])
    p = np.full(x.shape[:-1], 1.0 / (gamma * mach * mach))
    return conserved(rho, fourier_velocity(x, ks, phases, amp), p, gamma)


def fourier_state_torch(xq, ks, phases, gamma=1.4, mach=0.3, amp=0.1, L=2 * math.pi, chunk=1 << 18):
    """fourier_state evaluated with torch on the device of `xq` (points (..., 3),
    float64): the same separable sum as _fourier_raw and the same RMS scale
    (computed on the host), for preparing many large inputs quickly."""
    import torch
    g = (np.arange(16) + 0.5) * L / 16
    G = np.stack(np.meshgrid(g, g, g, indexing='ij'), axis=-1).reshape(-1, 3)
    rms = math.sqrt(float(np.mean(np.sum(_fourier_raw(G, ks, phases, L) ** 2, axis=-1))))
    scale = amp / rms
    ki = ks.astype(int)
    kmax = int(np.abs(ki).max())
    m = 2 * kmax + 1
    dev = xq.device
    ax = torch.arange(-kmax, kmax + 1, device=dev, dtype=torch.float64)
    Cs = []
    for c in range(3):
        C = np.zeros((m, m, m), complex)
        C[ki[:, 0] + kmax, ki[:, 1] + kmax, ki[:, 2] + kmax] = np.exp(1j * phases[:, c])
        Cs.append(torch.tensor(C.reshape(m * m, m).T.copy(), device=dev))
    y = xq.reshape(-1, 3).to(torch.float64) * (2 * math.pi / L)
    vel = torch.empty(y.shape[0], 3, dtype=torch.float64, device=dev)
    for a in range(0, y.shape[0], chunk):
        yy = y[a:a + chunk]
        E = [torch.exp(1j * yy[:, d:d + 1] * ax) for d in range(3)]
        for c in range(3):
            t = (E[2] @ Cs[c]).reshape(-1, m, m)
            t = (t * E[1][:, None, :]).sum(-1)
            vel[a:a + chunk, c] = (t * E[0]).sum(-1).real * scale
    rho = torch.ones(y.shape[0], dtype=torch.float64, device=dev)
    p = torch.full_like(rho, 1.0 / (gamma * mach * mach))
    En = p / (gamma - 1.0) + 0.5 * rho * (vel * vel).sum(-1)
    out = torch.cat([rho[:, None], rho[:, None] * vel, En[:, None]], dim=1)
    return out.reshape(tuple(xq.shape[:-1]) + (5,))


# ---- batch and serving workloads ------------------------------------------------
def batch_cases(count=96, seed=1812, nmin=4, nmax=12, pmin=1, pmax=4, mach=(0.05, 0.5)):
    """Independent Navier-Stokes cases on the periodic box [0, 2pi]^3: cube
    meshes n^3 with n ~ U{nmin..nmax}, degree p ~ U{pmin..pmax}, Mach
    ~ U[mach]; case i's Fourier phases use seed + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        p = int(rng.integers(pmin, pmax + 1))
        m = float(rng.uniform(*mach))
        out.append(dict(n=(n, n, n), lo=(0.0, 0.0, 0.0), hi=(2 * math.pi,) * 3, p=p, mach=m, seed=seed + i))
    return out


def serving_requests(count=2000, rate=200.0, seed=1812, nmin=2, nmax=20, degrees=(2, 3, 4)):
    """Poisson arrival stream: arrival times (s), cube meshes n^3 with n =
    round(exp U[ln nmin, ln nmax]) (elements log-uniform), p uniform over
    `degrees`, FP64 or mixed precision with probability 1/2, Mach
    ~ U[0.05, 0.5]; request i's Fourier phases use seed + i."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        p = int(degrees[int(rng.integers(0, len(degrees)))])
        mixed = bool(rng.integers(0, 2))
        m = float(rng.uniform(0.05, 0.5))
        out.append(dict(t=float(t[i]), n=(n, n, n), lo=(0.0, 0.0, 0.0), hi=(2 * math.pi,) * 3, p=p, mixed=mixed,
                        mach=m, seed=seed + i))
    return out


# ---- modal arrays for parity tests ---------------------------------------------
# Library layout: W[element][equation][mode], modes in hierarchical order
# (shell s = max(a,b,c), then (a,b,c) lexicographic); mode 0 is the constant
# mode, whose coefficient is the element mean times 2^(3/2) for the
# orthonormal Legendre basis on [-1,1]^3.
MODE0_SCALE = 2.0 ** 1.5


def shells(p):
    """Shell index max(a,b,c) of every mode in hierarchical order."""
    ms = [(a, b, c) for a in range(p + 1) for b in range(p + 1) for c in range(p + 1)]
    ms.sort(key=lambda m: (max(m), m[0], m[1], m[2]))
    return np.array([max(m) for m in ms])


def random_state(ne, p, seed, mean=(1.0, 0.2, -0.1, 0.15, 2.5), amp=0.02, decay=2.0):
    """Seeded smooth-ish modal state: a uniform mean state plus noise whose
    amplitude falls off as (1+s)^-decay with the shell s, so density and
    pressure stay positive for amp << 1."""
    rng = np.random.default_rng(seed)
    nv = (p + 1) ** 3
    W = amp * rng.standard_normal((ne, 5, nv)) / (1.0 + shells(p))[None, None, :] ** decay
    W[:, :, 0] += np.asarray(mean) * MODE0_SCALE
    return W


def random_vector(ne, p, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((ne, 5, (p + 1) ** 3))


def uniform_noise(shape, seed, amp):
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=shape)
