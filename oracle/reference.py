"""Reference element: orthonormal Legendre tensor-product modal basis on
[-1,1]^3 and Gauss-Legendre quadrature.

Test infrastructure (oracle); see oracle/__init__.py.

Paper Sec. 3: modal DG with tensor-product basis functions of degree k in each
direction on hexahedra/quadrilaterals, n_v = (k+1)^d modes per equation
(Eq. BSpace for the space).  The paper does not fix the 1D family or the
quadrature rule; the readings used here are:
  * 1D modes L_a(t) = sqrt((2a+1)/2) P_a(t) (orthonormal on [-1,1]);
  * every integral uses the (p+1)-point Gauss-Legendre rule per direction
    ((p+1)^3 in the volume, (p+1)^2 on a face);
  * modes are stored in hierarchical order: by shell s = max(a,b,c), ties by
    (a,b,c) lexicographically with a most significant.  With this order the
    modes of degree <= q form a prefix of length (q+1)^3 (used by the
    p-multigrid transfer, Sec. 6.1).
"""
import numpy as np


def legendre(n_modes, t):
    """Orthonormal Legendre values and derivatives.

    Returns (L, dL) of shape (n_modes,) + t.shape with L[a] = sqrt((2a+1)/2) P_a(t)
    using Bonnet's recurrence for P_a and P'_{a+1} = P'_{a-1} + (2a+1) P_a.
    """
    t = np.asarray(t)
    P = np.zeros((n_modes,) + t.shape, dtype=np.result_type(t, float))
    dP = np.zeros_like(P)
    P[0] = 1.0
    if n_modes > 1:
        P[1] = t
        dP[1] = 1.0
    for a in range(1, n_modes - 1):
        P[a + 1] = ((2 * a + 1) * t * P[a] - a * P[a - 1]) / (a + 1)
        dP[a + 1] = dP[a - 1] + (2 * a + 1) * P[a]
    scale = np.sqrt((2 * np.arange(n_modes) + 1) / 2.0).reshape((n_modes,) + (1,) * t.ndim)
    return P * scale, dP * scale


def gauss(n):
    """n-point Gauss-Legendre rule on [-1,1] (library routine)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def modes(p):
    """Hierarchical list of (a,b,c) triples, 0 <= a,b,c <= p."""
    out = [(a, b, c) for a in range(p + 1) for b in range(p + 1) for c in range(p + 1)]
    out.sort(key=lambda m: (max(m), m[0], m[1], m[2]))
    return out


def basis(p, X):
    """Tensor-product basis at reference points.

    X: (npts, 3).  Returns Phi (npts, nv) and dPhi (3, npts, nv) with
    Phi[q, i] = L_a(x) L_b(y) L_c(z) for mode i = (a,b,c) and dPhi[k] the
    derivative with respect to xi_k.
    """
    X = np.asarray(X)
    n = p + 1
    Lx, dLx = legendre(n, X[:, 0])
    Ly, dLy = legendre(n, X[:, 1])
    Lz, dLz = legendre(n, X[:, 2])
    ms = modes(p)
    npts = X.shape[0]
    Phi = np.zeros((npts, len(ms)))
    dPhi = np.zeros((3, npts, len(ms)))
    for i, (a, b, c) in enumerate(ms):
        Phi[:, i] = Lx[a] * Ly[b] * Lz[c]
        dPhi[0, :, i] = dLx[a] * Ly[b] * Lz[c]
        dPhi[1, :, i] = Lx[a] * dLy[b] * Lz[c]
        dPhi[2, :, i] = Lx[a] * Ly[b] * dLz[c]
    return Phi, dPhi


def volume_rule(p):
    """(p+1)^3 Gauss points (npts,3), ordered with the first coordinate slowest,
    and their weights."""
    x, w = gauss(p + 1)
    X = np.array([(x[i], x[j], x[k]) for i in range(p + 1) for j in range(p + 1) for k in range(p + 1)])
    W = np.array([w[i] * w[j] * w[k] for i in range(p + 1) for j in range(p + 1) for k in range(p + 1)])
    return X, W


# Faces are numbered f = 2*d + s: direction d in {0,1,2}, s = 0 for xi_d = -1,
# s = 1 for xi_d = +1.  A face is parametrised by the two other reference
# coordinates in increasing index order, so the two elements sharing a face on
# an aligned structured mesh see the same points in the same order.
def face_dirs(f):
    d = f // 2
    t = [k for k in range(3) if k != d]
    return d, (1.0 if f % 2 else -1.0), t


def face_rule(p, f):
    """(p+1)^2 Gauss points of face f in reference coordinates (npts,3) and weights."""
    x, w = gauss(p + 1)
    d, side, (t1, t2) = face_dirs(f)
    X = np.zeros(((p + 1) ** 2, 3))
    W = np.zeros((p + 1) ** 2)
    q = 0
    for i in range(p + 1):
        for j in range(p + 1):
            X[q, d] = side
            X[q, t1] = x[i]
            X[q, t2] = x[j]
            W[q] = w[i] * w[j]
            q += 1
    return X, W
