"""Element geometry and face connectivity (oracle).

Affine map of element m: x = X0 + J xi, J = [x1-x0, x2-x0, x3-x0]; |J| is the
Jacobian determinant and Theta^{-1} = dxi/dx = J^{-1} (Appendix A.1,
Eq. CKIter-ref).  Each face has an outward unit normal n and area |S_f|
(Eq. 2nd term).

Face points.  The paper sums the face flux over surface quadrature points
(Eq. 2nd term) without saying where they sit.  Reading used here: both sides
of a face evaluate the flux at the same physical points, so that the flux is
single valued and the scheme conserves the wave quantities exactly.  The face
rule is laid on the face with its three vertices ordered by (periodically
identified) global vertex number; a rule point with barycentric weights
(1 - eta1 - eta2, eta1, eta2) on those ordered vertices has the same weights
on either element's copy of the vertices, which gives its coordinates on that
element's reference face, where the element's own basis is evaluated.
"""
import numpy as np
import torch

from .refmat import FACE_VERTS, face_to_ref

DT = torch.float64


class OracleMesh:
    def __init__(self, xyz, tets, face_tag, periodic_map, ref):
        xyz = np.asarray(xyz, dtype=np.float64)
        tets = np.asarray(tets, dtype=np.int64)
        self.E = tets.shape[0]
        X = torch.tensor(xyz[tets], dtype=DT)                      # (E, 4, 3)
        self.X = X
        self.X0 = X[:, 0]
        self.J = torch.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0],
                              X[:, 3] - X[:, 0]], dim=-1)           # J[m, d, e]
        self.detJ = torch.linalg.det(self.J)
        if not bool((self.detJ > 0).all()):
            raise ValueError("inverted or degenerate tetrahedron")
        self.Jinv = torch.linalg.inv(self.J)                         # Jinv[m, e, d]
        normals, areas = [], []
        for f, (a, b, c) in enumerate(FACE_VERTS):
            cr = torch.linalg.cross(X[:, b] - X[:, a], X[:, c] - X[:, a])
            ln = torch.linalg.norm(cr, dim=-1)
            normals.append(cr / ln[:, None])
            areas.append(0.5 * ln)
        self.normal = torch.stack(normals, dim=1)                    # (E, 4, 3)
        self.area = torch.stack(areas, dim=1)                        # (E, 4)
        self.face_tag = np.asarray(face_tag, dtype=np.int64)

        ids = tets if periodic_map is None else np.asarray(periodic_map)[tets]
        table = {}
        for m in range(self.E):
            for f, fv in enumerate(FACE_VERTS):
                if self.face_tag[m, f] >= 0:
                    continue
                key = tuple(sorted(int(ids[m, v]) for v in fv))
                table.setdefault(key, []).append((m, f))
        self.nbr = -np.ones((self.E, 4), dtype=np.int64)
        self.nbr_face = -np.ones((self.E, 4), dtype=np.int64)
        self.slot_map = -np.ones((self.E, 4, 3), dtype=np.int64)
        for key, lst in table.items():
            if len(lst) != 2:
                raise ValueError("interior face without exactly one neighbour")
            (m1, f1), (m2, f2) = lst
            for (m, f), (mp, fp) in (((m1, f1), (m2, f2)), ((m2, f2), (m1, f1))):
                self.nbr[m, f] = mp
                self.nbr_face[m, f] = fp
                own = [int(ids[m, v]) for v in FACE_VERTS[f]]
                oth = [int(ids[mp, v]) for v in FACE_VERTS[fp]]
                self.slot_map[m, f] = [oth.index(g) for g in own]

        # basis values at the shared face points, own side and neighbour side
        L, Ns = ref.L, ref.Ns
        eta = ref.eta
        bary = torch.stack([1.0 - eta[:, 0] - eta[:, 1], eta[:, 0], eta[:, 1]], 1)
        # order[m, f] = local face slots sorted by global vertex number
        self.order = np.zeros((self.E, 4, 3), dtype=np.int64)
        for f, fv in enumerate(FACE_VERTS):
            g = ids[:, list(fv)]
            self.order[:, f] = np.argsort(g, axis=1, kind="stable")
        cache = {}
        self.Fface = torch.zeros((self.E, 4, Ns, L), dtype=DT)
        self.xiface = torch.zeros((self.E, 4, Ns, 3), dtype=DT)
        for m in range(self.E):
            for f in range(4):
                key = (f, tuple(self.order[m, f]))
                if key not in cache:
                    loc = torch.zeros_like(bary)
                    for j, slot in enumerate(key[1]):
                        loc[:, slot] = bary[:, j]      # j-th smallest vertex sits in slot
                    xi = face_to_ref(f, loc[:, 1:3])
                    cache[key] = (xi, ref.basis.values(xi))
                self.xiface[m, f], self.Fface[m, f] = cache[key]
        nb = np.where(self.nbr >= 0, self.nbr, 0)
        nf = np.where(self.nbr_face >= 0, self.nbr_face, 0)
        self.Fnbr = self.Fface[torch.as_tensor(nb), torch.as_tensor(nf)]
