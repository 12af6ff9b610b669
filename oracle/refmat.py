"""Reference-element matrices (oracle), Appendix A of the paper.

* mass      M_kl   = int_T phi_k phi_l                       (Eq. CKIter-ref-matrix)
* K^e_kl    = int_T phi_k d phi_l / d xi_e                   (Eq. CKIter-ref; the
  paper writes the index pair in the other order, K^e_lk, and sums l on both
  sides; the strong form of Eq. CKIter fixes which factor carries the
  derivative)
* stiffness int_T d phi_k / d xi_e phi_l = (K^e)^T           (Eq. 3rd term)
* V_ql      = phi_l(xi_q) (modal -> nodal) and the L2 projection
  P = M^{-1} V^T diag(w) (nodal -> modal): the nodal/modal round trip of
  Eqs. CKIter-ref-source, 3rd term and rhs term, with the volume quadrature
  points as nodes
* face traces F^f_il = phi_l(xi^f(eta_i)) and Lift^f_ki = beta_i phi_k(xi^f(eta_i))
  (Eq. 2nd term)

All integrals use the rules of :mod:`oracle.quadrature`.
"""
import torch

from .basis import Basis
from .quadrature import face_rule, time_rule, volume_rule

DT = torch.float64

REF_VERTS = torch.tensor([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0],
                          [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]], dtype=DT)
# face f is opposite local vertex 3 - f, vertices ordered for an outward normal
FACE_VERTS = ((0, 2, 1), (0, 1, 3), (0, 3, 2), (1, 2, 3))


def face_to_ref(f, eta):
    """xi^f(eta) = nu_a + eta1 (nu_b - nu_a) + eta2 (nu_c - nu_a)."""
    a, b, c = FACE_VERTS[f]
    va, vb, vc = REF_VERTS[a], REF_VERTS[b], REF_VERTS[c]
    eta = torch.as_tensor(eta, dtype=DT)
    return va + eta[..., 0:1] * (vb - va) + eta[..., 1:2] * (vc - va)


class RefElement:
    def __init__(self, N):
        self.N = N
        self.basis = Basis(N)
        self.L = self.basis.L
        self.xq, self.wq = volume_rule(N)
        self.Q = self.xq.shape[0]
        self.eta, self.beta = face_rule(N)
        self.Ns = self.eta.shape[0]
        self.tau, self.gamma = time_rule(N)
        self.Nt = self.tau.shape[0]

        self.V = self.basis.values(self.xq)                       # (Q, L)
        dV = self.basis.gradients(self.xq)                        # (Q, 3, L)
        W = torch.diag(self.wq)
        self.M = self.V.T @ W @ self.V                            # (L, L)
        self.Minv = torch.linalg.inv(self.M)
        self.P = self.Minv @ self.V.T @ W                         # (L, Q)
        # K^e_kl = int phi_k dphi_l/dxi_e
        self.K = torch.stack([self.V.T @ W @ dV[:, e, :] for e in range(3)])
        # stiffness int dphi_k/dxi_e phi_l
        self.Kstiff = self.K.transpose(1, 2).contiguous()
        self.Fown = torch.stack([self.basis.values(face_to_ref(f, self.eta))
                                 for f in range(4)])              # (4, Ns, L)
        self.Lift = torch.stack([(self.beta[:, None] * self.Fown[f]).T
                                 for f in range(4)])              # (4, L, Ns)
