"""Clustered local time stepping (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's implementation steps every element with one global time step
(Section 5.1, performance discussion) and names local time stepping as the
missing piece that costs its nonlinear runs a factor 5.56 in time to
solution; it gives no scheme.  Reading used here (rate-2 clustering, as in
the clustered ADER-DG schemes the paper cites for the linear case):

* Every element has the admissible step of the global rule with its own
  wave speed, dt_e = cfl 2 r_in,e / ((2N+1) c_p,e).  With dt_0 = min dt_e,
  element e joins cluster c_e = min(C-1, floor(log2(dt_e / dt_0))) and steps
  with dt_c = 2^c dt_0; clusters of face neighbours differ by at most one
  (an element is moved down until they do).
* A step of cluster c over [t, t + dt_c]: its elements predict at t (the same
  predictor as the global step; its Taylor coefficients D^i are kept); cluster
  c - 1 then takes its two steps inside the interval; then cluster c corrects:
  - at a face whose neighbour is in cluster >= c the numerical flux is taken
    at the cluster's time points t + tau_z dt_c, the neighbour's state being
    its own Taylor expansion evaluated at those times (it predicted at an
    earlier or equal time);
  - at a face whose neighbour is in the finer cluster c - 1 the flux is the
    sum of the time-integrated fluxes that neighbour computed at the same
    face during its two steps;
  - volume and damage-source terms over [t, t + dt_c] come from the
    element's own prediction, and the update is that of the global step.
  Each face flux is computed once, at the time points of the finer side, and
  used by both sides, so the wave quantities stay conserved across cluster
  boundaries.  With one cluster the scheme is the global step.
* A point source adds its exact time integral over its element's own step
  after that element's update, as in the global step.
"""
import numpy as np
import torch

DT = torch.float64


def admissible_steps(S, cfl=0.5):
    """dt_e = cfl 2 r_in,e / ((2N+1) c_p,e) (intact moduli) for every element
    of the OracleSolver S; r_in = 3 |J| / (6 * total face area) for a tet."""
    m = S.mesh
    vol = m.detJ / 6.0
    r_in = 3.0 * vol / m.area.sum(dim=1)
    cp = torch.sqrt((S.mat["lambda0"] + 2.0 * S.mat["mu0"]) / S.mat["rho"])
    return (cfl * 2.0 * r_in / ((2 * S.N + 1) * cp)).numpy()


def make_clusters(dt_e, nbr, n_clusters):
    """(cluster per element, dt_0): rate-2 clusters with neighbours at most one
    cluster apart (moved down until they are)."""
    dt0 = float(np.min(dt_e))
    c = np.minimum(n_clusters - 1, np.floor(np.log2(dt_e / dt0) + 1e-12)).astype(np.int64)
    c = np.maximum(c, 0)
    while True:
        nb = np.where(nbr >= 0, c[np.maximum(nbr, 0)], n_clusters)   # no neighbour: no limit
        lim = nb.min(axis=1) + 1
        new = np.minimum(c, lim)
        if np.array_equal(new, c):
            return c, dt0
        c = new


class LtsSolver:
    """Clustered local time stepping around an OracleSolver S (which supplies
    the predictor, the volume/source terms, the face fluxes and the lift)."""

    def __init__(self, S, clusters, dt0, sources=None):
        self.S = S
        # point sources (oracle.sources.PointSources): each one's time integral
        # over its element's own step is added after that element's update
        self.sources = sources
        self.cl = np.asarray(clusters, dtype=np.int64)
        self.C = int(self.cl.max()) + 1
        self.dt0 = float(dt0)
        m = S.mesh
        self.nbr = m.nbr
        self.nbr_face = m.nbr_face
        ncl = np.where(self.nbr >= 0, self.cl[np.maximum(self.nbr, 0)], -10)
        if bool((np.abs(ncl - self.cl[:, None])[self.nbr >= 0] > 1).any()):
            raise ValueError("face neighbours more than one cluster apart")

    @property
    def macro_dt(self):
        return self.dt0 * 2 ** (self.C - 1)

    def _taylor(self, times):
        """State of every element at the absolute times (E,), from its kept
        prediction: sum_i (t - t_pred)^i / i! D^i."""
        h = torch.as_tensor(times - self.tp, dtype=DT)[:, None, None]
        acc = torch.zeros_like(self.D[0])
        fac = torch.ones_like(h)
        for i, Di in enumerate(self.D):
            if i > 0:
                fac = fac * h / i
            acc = acc + fac * Di
        return acc

    def macro_step(self, U, t0=0.0):
        """Advance every element by one macro step macro_dt from t0."""
        S = self.S
        self.U = U.clone()
        self.D = [torch.zeros_like(U) for _ in range(S.N + 1)]
        self.tp = np.full(S.E, t0)
        self.acc = torch.zeros((S.E, 4, S.ref.Ns, 10), dtype=DT)
        self._advance(self.C - 1, t0)
        return self.U

    def run(self, U, nmacro, t0=0.0):
        for k in range(nmacro):
            U = self.macro_step(U, t0 + k * self.macro_dt)
        return U

    def _advance(self, c, t):
        S, ref, m = self.S, self.S.ref, self.S.mesh
        dtc = self.dt0 * 2 ** c
        sel = self.cl == c
        if sel.any():
            D, _ = S.predict(self.U)
            for i in range(S.N + 1):
                self.D[i][sel] = D[i][sel]
            self.tp[sel] = t
        if c > 0:
            self._advance(c - 1, t)
            self._advance(c - 1, t + 0.5 * dtc)
        if not sel.any():
            return
        # time points of cluster c; every element's state there (only those of
        # clusters >= c are used)
        Uz = torch.stack([self._taylor(np.full(S.E, t + float(tz) * dtc)) for tz in ref.tau])
        Fint = S.face_fluxes(Uz)                       # (E, 4, Ns, 10), sum_z gamma_z F*
        I = torch.zeros_like(Fint)
        for e in np.nonzero(sel)[0]:
            for f in range(4):
                nb = self.nbr[e, f]
                if nb >= 0 and self.cl[nb] == c - 1:
                    I[e, f] = self.acc[e, f]
                    self.acc[e, f] = 0.0
                else:
                    I[e, f] = dtc * Fint[e, f]
                    if nb >= 0 and self.cl[nb] == c + 1:
                        nf = self.nbr_face[e, f]
                        self.acc[nb, nf] = self.acc[nb, nf] + dtc * Fint[nb, nf]
        face = torch.einsum("mf,i,mfik,mfip->mkp", m.area / m.detJ[:, None], ref.beta,
                            m.Fface, I)
        dt_save = S.dt
        S.dt = dtc
        vol, src = S.volume_and_source(Uz)
        S.dt = dt_save
        upd = torch.einsum("kl,mlp->mkp", ref.Minv, vol + src - face)
        idx = torch.as_tensor(np.nonzero(sel)[0])
        self.U[idx] = self.U[idx] + upd[idx]
        if self.sources is not None:
            dU = self.sources.increment(t, t + dtc)
            self.U[idx] = self.U[idx] + dU[idx]
