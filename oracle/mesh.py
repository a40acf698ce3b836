"""Periodic structured hexahedral mesh with trilinear (Q1) element maps.

Test infrastructure (oracle); see oracle/__init__.py.

Paper Sec. 3: a triangulation T_h of n_e non-overlapping elements; the face
sets and the +/- (interior / neighbour) convention.  The paper's vortex case is
periodic on every side (Sec. 7.1); every mesh here is a periodic box.

Element e = i + nx*(j + ny*k).  Local vertex v = i + 2j + 4k sits at reference
coordinates (2i-1, 2j-1, 2k-1).  The neighbour across face f (f = 2d+s, see
reference.face_dirs) is found by periodic index arithmetic; it sees the shared
face as its face f ^ 1.
"""
import numpy as np


def box_vertices(n, lo, hi):
    """Vertices (ne, 8, 3) of the undeformed box with n = (nx, ny, nz) elements."""
    nx, ny, nz = n
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    h = (hi - lo) / np.array(n)
    V = np.zeros((nx * ny * nz, 8, 3))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                e = i + nx * (j + ny * k)
                for v in range(8):
                    di, dj, dk = v & 1, (v >> 1) & 1, (v >> 2) & 1
                    V[e, v] = lo + h * np.array([i + di, j + dj, k + dk])
    return V


class BoxMesh:
    """Periodic box; `vertices` (ne, 8, 3) overrides the straight-sided map."""

    def __init__(self, n, lo, hi, vertices=None):
        self.n = tuple(int(x) for x in n)
        self.lo = np.asarray(lo, float)
        self.hi = np.asarray(hi, float)
        nx, ny, nz = self.n
        self.ne = nx * ny * nz
        self.vtx = box_vertices(self.n, lo, hi) if vertices is None else np.asarray(vertices, float).copy()
        assert self.vtx.shape == (self.ne, 8, 3)
        self.nbr = np.zeros((self.ne, 6), dtype=np.int64)
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    e = i + nx * (j + ny * k)
                    ijk = [i, j, k]
                    for f in range(6):
                        d, s = f // 2, f % 2
                        o = list(ijk)
                        o[d] = (o[d] + (1 if s else -1)) % self.n[d]
                        self.nbr[e, f] = o[0] + nx * (o[1] + ny * o[2])


def shape_q1(X):
    """Trilinear shape functions N (npts, 8) and derivatives dN (3, npts, 8)."""
    X = np.asarray(X)
    npts = X.shape[0]
    N = np.ones((npts, 8))
    dN = np.ones((3, npts, 8))
    for v in range(8):
        s = np.array([2 * (v & 1) - 1, 2 * ((v >> 1) & 1) - 1, 2 * ((v >> 2) & 1) - 1], float)
        fac = [(1.0 + s[k] * X[:, k]) / 2.0 for k in range(3)]
        N[:, v] = fac[0] * fac[1] * fac[2]
        for k in range(3):
            dN[k, :, v] = s[k] / 2.0
            for m in range(3):
                if m != k:
                    dN[k, :, v] *= fac[m]
    return N, dN


def geometry(vtx, X):
    """Physical points, Jacobian, determinant and inverse at reference points X.

    vtx: (ne, 8, 3).  Returns x (ne,npts,3), J (ne,npts,3,3) with
    J[...,d,k] = dx_d/dxi_k, detJ (ne,npts), Jinv (ne,npts,3,3) with
    Jinv[...,k,d] = dxi_k/dx_d.
    """
    N, dN = shape_q1(X)
    x = np.einsum('qv,evd->eqd', N, vtx)
    J = np.einsum('kqv,evd->eqdk', dN, vtx)
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    return x, J, detJ, Jinv


def face_geometry(vtx, X, f):
    """Outward unit normal n (ne,npts,3) and surface Jacobian J_F (ne,npts) of
    face f at its reference points X: J_F = |dx/dxi_{d+1} x dx/dxi_{d+2}|
    (cyclic order, which points towards +xi_d), n = side * cross / J_F."""
    d = f // 2
    side = 1.0 if f % 2 else -1.0
    _, J, _, _ = geometry(vtx, X)
    a = J[..., :, (d + 1) % 3]
    b = J[..., :, (d + 2) % 3]
    c = np.cross(a, b)
    JF = np.linalg.norm(c, axis=-1)
    n = side * c / JF[..., None]
    return n, JF
