"""Structured tetrahedral meshes of a cube (input data, not method).

A cube [o, o+length]^3 is cut into n^3 sub-cubes; every sub-cube is split into
the six Kuhn (Freudenthal) tetrahedra that share its main diagonal
(0,0,0)->(1,1,1).  Every sub-cube uses the same split, so the mesh is conforming
and periodic-compatible.

Conventions shared with the library interface (``include/dgd.h``):

* ``tets[e] = (v0, v1, v2, v3)`` is positively oriented:
  det[x1-x0, x2-x0, x3-x0] > 0.
* Face ``f`` of a tetrahedron is the face opposite local vertex ``3 - f``:
  f0 = (v0, v2, v1), f1 = (v0, v1, v3), f2 = (v0, v3, v2), f3 = (v1, v2, v3)
  (vertex triples ordered so that the right-hand normal points outward).
* ``face_tag[e, f]``: -1 interior (or periodic), 1 free surface, 2 absorbing.
* ``periodic_map[v]``: canonical vertex id that ``v`` is identified with (the
  copy with every grid coordinate reduced modulo n); vertices on opposite
  domain faces are glued through it.
"""
import itertools
import math

import numpy as np

FACE_VERTS = ((0, 2, 1), (0, 1, 3), (0, 3, 2), (1, 2, 3))

TAG_INTERIOR = -1
TAG_FREE = 1
TAG_ABSORB = 2


def kuhn_inradius(edge):
    """Inradius of a Kuhn tetrahedron of a cube with edge length ``edge``.

    volume edge^3/6, total face area (1 + sqrt 2) edge^2, r = 3V/A.
    """
    return edge / (2.0 * (1.0 + math.sqrt(2.0)))


def cube_mesh(n, length, periodic=False, origin=(0.0, 0.0, 0.0),
              top_free=True, z_nodes=None):
    """Return a dict with ``xyz`` (nv,3) f64, ``tets`` (ne,4) i64,
    ``face_tag`` (ne,4) i8, ``periodic_map`` (nv,) i64 or None, ``n``,
    ``length``, ``edge`` (the uniform spacing) and ``z_nodes``.

    Non-periodic meshes tag the top face z = origin_z + length as free surface
    (if ``top_free``) and the other five domain faces as absorbing.
    ``z_nodes`` (n+1 increasing heights from 0 to ``length``) replaces the
    uniform spacing along z: a mesh graded in depth (boxes instead of cubes,
    still split into six positively oriented tetrahedra); not periodic.
    """
    n = int(n)
    h = float(length) / n
    o = np.asarray(origin, dtype=np.float64)
    g = np.arange(n + 1)
    # vertex id = i + (n+1)*(j + (n+1)*k)
    kk, jj, ii = np.meshgrid(g, g, g, indexing="ij")
    ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    xyz = o[None, :] + h * ijk.astype(np.float64)
    if z_nodes is not None:
        z = np.asarray(z_nodes, dtype=np.float64)
        if periodic or z.shape != (n + 1,) or not np.all(np.diff(z) > 0) \
                or abs(z[0]) > 1e-9 * length or abs(z[-1] - length) > 1e-9 * length:
            raise ValueError("z_nodes: n+1 increasing heights from 0 to length, not periodic")
        xyz[:, 2] = o[2] + z[ijk[:, 2]]

    def vid(i, j, k):
        return i + (n + 1) * (j + (n + 1) * k)

    perms = list(itertools.permutations(range(3)))
    # cube order: i fastest, then j, then k; six tetrahedra per cube in the
    # order of ``perms`` (path 0 -> e_p0 -> e_p0 + e_p1 -> (1,1,1))
    ck, cj, ci = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)        # (ncell, 3)
    tets = np.zeros((base.shape[0], 6, 4), dtype=np.int64)
    for t, p in enumerate(perms):
        cur = base.copy()
        ids = [vid(cur[:, 0], cur[:, 1], cur[:, 2])]
        for ax in p:
            cur = cur.copy()
            cur[:, ax] += 1
            ids.append(vid(cur[:, 0], cur[:, 1], cur[:, 2]))
        inv = sum(1 for a in range(3) for b in range(a + 1, 3) if p[a] > p[b])
        if inv % 2 == 1:
            ids[1], ids[2] = ids[2], ids[1]
        tets[:, t, :] = np.stack(ids, axis=1)
    tets = tets.reshape(-1, 4)

    if periodic:
        pm = vid(ijk[:, 0] % n, ijk[:, 1] % n, ijk[:, 2] % n).astype(np.int64)
        face_tag = np.full((tets.shape[0], 4), TAG_INTERIOR, dtype=np.int8)
    else:
        pm = None
        face_tag = np.full((tets.shape[0], 4), TAG_INTERIOR, dtype=np.int8)
        vijk = ijk[tets]  # (ne, 4, 3)
        for f, fv in enumerate(FACE_VERTS):
            c = vijk[:, list(fv), :]  # (ne, 3, 3)
            for ax in range(3):
                on_lo = np.all(c[:, :, ax] == 0, axis=1)
                on_hi = np.all(c[:, :, ax] == n, axis=1)
                face_tag[on_lo, f] = TAG_ABSORB
                if ax == 2 and top_free:
                    face_tag[on_hi, f] = TAG_FREE
                else:
                    face_tag[on_hi, f] = TAG_ABSORB
    return {"xyz": xyz, "tets": tets, "face_tag": face_tag,
            "periodic_map": pm, "n": n, "length": float(length), "edge": h,
            "z_nodes": None if z_nodes is None else np.asarray(z_nodes, dtype=np.float64)}


def tet_inradius(xyz, tets):
    """Inradius 3V/A of every tetrahedron (volume over total face area)."""
    X = xyz[tets]                                              # (ne, 4, 3)
    vol = np.abs(np.einsum("ei,ei->e", np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]),
                           X[:, 3] - X[:, 0])) / 6.0
    area = np.zeros(len(tets))
    for fv in FACE_VERTS:
        a, b, c = X[:, fv[0]], X[:, fv[1]], X[:, fv[2]]
        area += 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    return 3.0 * vol / area
