"""Oracle step of single elements of a large mesh (test helper).

The update of one element depends only on its own state and on the states of
its face neighbours (Appendix A: the predictor is element-local, the face term
couples the two sides of each face).  For a sampled element of a mesh too
large for the oracle, this builds the patch {element, its neighbours} as a
mesh of its own and runs one oracle step on it:

* vertices keep the order of their global numbers (the shared face points
  are laid out by global vertex order, so the patch reproduces them);
* the element keeps its face tags; faces of the neighbours that lead out of
  the patch are tagged absorbing (their updates are not used);
* materials and the initial condition are those of the global elements.
"""
import numpy as np

from oracle.step import OracleSolver

FACE_VERTS = ((0, 2, 1), (0, 1, 3), (0, 3, 2), (1, 2, 3))
TAG_ABSORB = 2


def face_partners(mesh):
    """(ne, 4) neighbour element of every face (-1 on boundaries)."""
    tets = mesh["tets"]
    pm = mesh["periodic_map"]
    g = tets if pm is None else pm[tets]
    ne = tets.shape[0]
    keys = np.stack([np.sort(g[:, list(fv)], axis=1) for fv in FACE_VERTS], axis=1)  # (ne,4,3)
    flat = keys.reshape(-1, 3)
    order = np.lexsort((flat[:, 2], flat[:, 1], flat[:, 0]))
    s = flat[order]
    same = np.all(s[1:] == s[:-1], axis=1)
    nbr = np.full(ne * 4, -1, dtype=np.int64)
    i = np.nonzero(same)[0]
    a, b = order[i], order[i + 1]
    nbr[a] = b // 4
    nbr[b] = a // 4
    nbr = nbr.reshape(ne, 4)
    nbr[mesh["face_tag"] != -1] = -1
    return nbr


def oracle_patch_step(w, e, nbr):
    """Oracle U^1 (L, 10) of element e after one step from the projected
    initial condition of workload w."""
    m = w.mesh
    elems = [int(e)] + [int(x) for x in nbr[e] if x >= 0]
    elems = list(dict.fromkeys(elems))
    tets_g = m["tets"][elems]
    verts = np.unique(tets_g)                        # sorted: keeps global order
    remap = {int(v): i for i, v in enumerate(verts)}
    tets = np.vectorize(remap.get)(tets_g).astype(np.int64)
    xyz = m["xyz"][verts]
    tag = np.full((len(elems), 4), TAG_ABSORB, dtype=np.int8)
    tag[0] = m["face_tag"][e]
    for k, x in enumerate(elems[1:], start=1):
        for f in range(4):
            if nbr[x, f] == e:
                tag[k, f] = -1
    pm = None
    if m["periodic_map"] is not None:
        # identified vertices: the rank of the global representative, which
        # keeps the global order of identified ids
        gp = m["periodic_map"][verts]
        pm = np.searchsorted(np.unique(gp), gp).astype(np.int64)
    mat = {k: np.asarray(v)[elems] for k, v in w.material.items()}
    S = OracleSolver(xyz, tets, tag, pm, mat, w.N, w.dt, alpha_max=w.alpha_max)
    gl = np.asarray(elems)

    def ic(x, elem):
        return w.ic(x, gl[elem])

    U0 = S.project(ic)
    U1 = S.step(U0)
    return U1[0].detach().numpy()
