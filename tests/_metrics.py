"""Error measures of a modal state against a reference (test helper).

States are (E, 10, L) modal arrays (the library's layout).  Every mesh of the
workloads is a uniform cube mesh, so |J| is the same for all elements and the
L2 norm over modes is the L2 norm over the domain (orthonormal basis).

Per quantity group (strain, velocity, alpha):

* ``l2``   relative L2 over the mesh;
* ``linf`` max |du| / max |u| over the volume quadrature points (the point
  values V U), or over the modes when no evaluation matrix is given;
* ``elem`` the largest per-element relative L2 error among the elements that
  carry the field (element norm at least ``ELEM_FLOOR`` of the largest), so
  that one bad element cannot hide in a mesh-wide norm.
"""
import numpy as np

GROUPS = {"strain": slice(0, 6), "velocity": slice(6, 9), "alpha": slice(9, 10)}
ELEM_FLOOR = 0.1
# Per-element errors of single sampled elements are held to twice the bar of
# the mesh-wide norms: in the first step from rest the velocity of an element
# is the small difference of its volume and face terms, so its FP32 rounding
# relative to its own size is up to about 1e-5 where the mesh-wide L2 is 1e-7.
ELEM_FACTOR = 2.0


def _pointwise_max(a, V, chunk=1 << 16):
    """max |V a_e| over elements and points, a (E, k, L), V (Q, L)."""
    m = 0.0
    for e0 in range(0, a.shape[0], chunk):
        pts = np.einsum("ql,ekl->ekq", V, a[e0:e0 + chunk], optimize=True)
        m = max(m, float(np.abs(pts).max()))
    return m


def errors(got, want, V=None, groups=GROUPS):
    """{group: {"l2", "linf", "elem"}} plus "all": the overall relative L2."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape and got.ndim == 3 and got.shape[1] == 10
    out = {}
    for name, s in groups.items():
        d = got[:, s] - want[:, s]
        w = want[:, s]
        nw = np.linalg.norm(w)
        r = {"l2": float(np.linalg.norm(d) / nw) if nw > 0 else float(np.linalg.norm(d))}
        if V is not None:
            mw = _pointwise_max(w, V)
            md = _pointwise_max(d, V)
        else:
            mw, md = float(np.abs(w).max()), float(np.abs(d).max())
        r["linf"] = md / mw if mw > 0 else md
        ew = np.sqrt((w ** 2).sum(axis=(1, 2)))
        ed = np.sqrt((d ** 2).sum(axis=(1, 2)))
        big = ew >= ELEM_FLOOR * ew.max() if ew.max() > 0 else np.ones_like(ew, dtype=bool)
        r["elem"] = float((ed[big] / np.maximum(ew[big], 1e-300)).max()) if ew.max() > 0 \
            else float(ed.max())
        out[name] = r
    out["all"] = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    return out


def group_scales(state):
    """Largest per-element norm of every quantity group over a whole state
    (E, 10, L)."""
    out = {}
    for k, s in GROUPS.items():
        a = state[:, s]
        out[k] = float(np.sqrt(np.einsum("ekl,ekl->e", a, a).max()))
    return out


def element_errors(g, w_, scales):
    """Relative L2 error of one element's state (L, 10) per quantity group.
    A group whose norm in this element is below 1e-2 of its largest element
    norm over the mesh (``scales``, e.g. a velocity not yet excited far from
    the pulses) is measured against that floor instead of its own norm."""
    out = {}
    for k, s in GROUPS.items():
        n = np.linalg.norm(w_[:, s])
        fl = max(n, 1e-2 * scales[k])
        out[k] = float(np.linalg.norm(g[:, s] - w_[:, s]) / fl) if fl > 0 else \
            float(np.linalg.norm(g[:, s] - w_[:, s]))
    return out


def worst(err):
    """Largest of every group's measures."""
    return max(v for g, r in err.items() if g != "all" for v in r.values())


def assert_within(err, tol, what=""):
    """Every group's l2, linf and elem below tol."""
    bad = {g: r for g, r in err.items() if g != "all" and max(r.values()) >= tol}
    assert not bad, f"{what}: above {tol:g}: {bad}"
