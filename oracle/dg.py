"""DG spatial residual R(W) with Roe and BR2 fluxes, and the mass matrix.

Test infrastructure (oracle); see oracle/__init__.py.

Paper Sec. 3.1, Eq. dg_ns: for every element K and test function w_h,

   int_K w . du/dt  - int_K grad w : F(u, grad u)
 + int_dK w+ . Fhat(u+-, grad u+-, n+) - int_dK grad w+ : (K+ n+)(u+ - uhat) = 0,

uhat = (u+ + u-)/2.  Fhat = Fhat_c (Roe) + Fhat_v (BR2, Eq. visc_flux):

   Fhat_v = {F_v(u, grad u)} . n+ + eta_F {delta_F(u+ - u-)} . n+,

with the lifting delta_F of Eq. re.  The semi-discrete system is
M dW/dt + R(W) = 0 (Sec. 3.1), so with the modal coefficients W[e, a, i]
(element, equation, mode):

   R[e,a,i] = - sum_q w_q detJ_q grad phi_i . F_a
              + sum_faces sum_fq w_fq J_F [ phi_i Fhat_a - grad phi_i . G+_a ],

   G+ = (K+ n+)(u+ - uhat) = 1/2 K(u+)(n+ (x) [u]),   [u] = u+ - u-.

K is the diffusivity (F_v = -K grad u, Sec. 3.1), so K(u) X = -F_v(u, X) for
any gradient-shaped X.  For the neighbour element the same face gives
(K- n-)(u- - uhat) = 1/2 K(u-)(n+ (x) [u]): both lifting problems lift the
same jump with their own K.

This module evaluates every face from each of its two elements (element-centric
loop), with dense reference matrices and the lifting solved the long way
(element mass matrix, dense solve, evaluation at the face points).
"""
import numpy as np

from . import reference as ref
from . import mesh as msh
from . import physics as phy


class Discretization:
    """Reference tables and geometry for one (mesh, p, physics) triple.

    gamma, mu, Pr: gas constants (mu == 0 gives the Euler equations).
    eta: BR2 penalty eta_F; the paper only requires eta_F > number of faces
    (Sec. 3.1), read here as 7 for hexahedra.
    """

    # Switches used only by the pins that check each term matters.
    inviscid = True          # include F_c and the Roe flux
    symmetry_term = True     # include the adjoint-consistency face term

    def __init__(self, mesh, p, gamma=1.4, mu=0.0, Pr=0.72, eta=7.0):
        self.mesh = mesh
        self.p = p
        self.n = p + 1
        self.nv = self.n ** 3
        self.gamma, self.mu, self.Pr, self.eta = float(gamma), float(mu), float(Pr), float(eta)
        self.viscous = mu != 0.0
        ne = mesh.ne
        # volume
        self.Xq, self.wq = ref.volume_rule(p)
        self.Phi, self.dPhi = ref.basis(p, self.Xq)
        self.xq, _, self.detJ, self.Jinv = msh.geometry(mesh.vtx, self.Xq)
        if np.any(self.detJ <= 0):
            raise ValueError("non-positive Jacobian determinant")
        # faces
        self.Xf, self.Phif, self.dPhif, self.fJinv, self.fn, self.fJF = [], [], [], [], [], []
        for f in range(6):
            X, wf = ref.face_rule(p, f)
            self.wf = wf
            Phi, dPhi = ref.basis(p, X)
            _, _, _, Jinv = msh.geometry(mesh.vtx, X)
            n, JF = msh.face_geometry(mesh.vtx, X, f)
            self.Xf.append(X)
            self.Phif.append(Phi)
            self.dPhif.append(dPhi)
            self.fJinv.append(Jinv)
            self.fn.append(n)
            self.fJF.append(JF)
        # element mass matrices M_e = Phi^T diag(w detJ) Phi  (Sec. 3.1, block diagonal M)
        self.M = np.einsum('qi,q,eq,qj->eij', self.Phi, self.wq, self.detJ, self.Phi)
        self.Minv = np.linalg.inv(self.M)

    # ---- helpers -----------------------------------------------------------
    def ndof(self):
        return self.mesh.ne * 5 * self.nv

    def grad_phys(self, W, dPhi, Jinv):
        """Physical gradient of u at points: (ne,npts,5,3)."""
        gxi = np.einsum('kqm,eam->eqak', dPhi, W)
        return np.einsum('eqak,eqkj->eqaj', gxi, Jinv)

    def lift(self, G, f, elems):
        """BR2 lifting (Eq. re), the long way.  For each listed element, with
        its own face f, solve  int_K tau : delta = int_F tau : G dsigma  for
        delta in [V_h]^{5x3} using the element mass matrix, and return delta
        evaluated at the face points: (ne,nfq,5,3).  G (ne,nfq,5,3) is the
        integrand at the face points (here 1/2 K(u)(n+ (x) [u]))."""
        Phi = self.Phif[f]
        JF = self.fJF[f][elems]
        b = np.einsum('qi,q,eq,eqaj->eiaj', Phi, self.wf, JF, G)
        coef = np.einsum('eij,ejak->eiak', self.Minv[elems], b)
        return np.einsum('qi,eiaj->eqaj', Phi, coef)

    # ---- residual ----------------------------------------------------------
    def residual(self, W):
        """R(W) for W (ne, 5, nv); returns (ne, 5, nv).  Complex W allowed."""
        g, mu, Pr = self.gamma, self.mu, self.Pr
        mesh = self.mesh
        ne = mesh.ne
        allel = np.arange(ne)
        u = np.einsum('qm,eam->eqa', self.Phi, W)
        F = phy.flux_c(u, g) if self.inviscid else np.zeros(u.shape + (3,), dtype=u.dtype)
        if self.viscous:
            F = F + phy.flux_v(u, self.grad_phys(W, self.dPhi, self.Jinv), g, mu, Pr)
        # volume term  - sum_q w detJ (grad phi_i . F)
        gphi = np.einsum('kqm,eqkj->eqmj', self.dPhi, self.Jinv)       # dphi_m/dx_j
        R = -np.einsum('q,eq,eqmj,eqaj->eam', self.wq, self.detJ, gphi, F)
        for f in range(6):
            fo = f ^ 1
            nb = mesh.nbr[:, f]
            up = np.einsum('qm,eam->eqa', self.Phif[f], W)
            um = np.einsum('qm,eam->eqa', self.Phif[fo], W[nb])
            n = self.fn[f]
            JF = self.fJF[f]
            Fhat = phy.roe(up, um, n, g) if self.inviscid else np.zeros_like(up)
            gphi_f = np.einsum('kqm,eqkj->eqmj', self.dPhif[f], self.fJinv[f])
            if self.viscous:
                gp = self.grad_phys(W, self.dPhif[f], self.fJinv[f])
                gm = self.grad_phys(W[nb], self.dPhif[fo], self.fJinv[fo][nb])
                jump_n = (up - um)[..., :, None] * n[..., None, :]          # [u] (x) n+
                Gp = -0.5 * phy.flux_v(up, jump_n, g, mu, Pr)              # 1/2 K(u+)(n+ (x) [u])
                Gm = -0.5 * phy.flux_v(um, jump_n, g, mu, Pr)              # 1/2 K(u-)(n+ (x) [u])
                dp = self.lift(Gp, f, allel)
                dm = self.lift(Gm, fo, nb)
                Fv = 0.5 * (phy.flux_v(up, gp, g, mu, Pr) + phy.flux_v(um, gm, g, mu, Pr)) \
                    + self.eta * 0.5 * (dp + dm)
                Fhat = Fhat + np.einsum('eqaj,eqj->eqa', Fv, n)
                # adjoint-consistency (symmetry) term  - grad phi_i : G+
                if self.symmetry_term:
                    R -= np.einsum('q,eq,eqmj,eqaj->eam', self.wf, JF, gphi_f, Gp)
            R += np.einsum('q,eq,qm,eqa->eam', self.wf, JF, self.Phif[f], Fhat)
        return R

    def mass(self, v):
        """M v with the block-diagonal mass matrix (Sec. 3.1)."""
        return np.einsum('eij,eaj->eai', self.M, v)

    # ---- projection of point data ------------------------------------------
    def quad_points(self):
        """Physical coordinates of the volume Gauss points (ne, nq, 3)."""
        return self.xq

    def project(self, values):
        """L2 projection (with the volume rule) of values (ne,nq,5) given at the
        Gauss points: W = M^-1 int phi u."""
        b = np.einsum('qi,q,eq,eqa->eai', self.Phi, self.wq, self.detJ, values)
        return np.einsum('eij,eaj->eai', self.Minv, b)

    def evaluate(self, W, X=None):
        """u at reference points X (default: volume Gauss points): (ne,npts,5)."""
        if X is None:
            Phi = self.Phi
        else:
            Phi, _ = ref.basis(self.p, X)
        return np.einsum('qm,eam->eqa', Phi, W)
