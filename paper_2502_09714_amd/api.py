"""Thin Python front end of the C interface (same names, argument marshalling).

Host arrays are numpy float64/int64 arrays; device arrays are torch tensors on
the current HIP device.  The solver runs on torch's current stream.
"""
import ctypes

import numpy as np

from ._lib import DGDError, FP32, FP64, BF16, NUM_KERNEL_CLASSES, c_dp, c_i8p, c_i64p, lib

PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16}


def _dp(a):
    return a.ctypes.data_as(c_dp)


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


class Simulation:
    """One solver instance (a ``dgd_handle``)."""

    def __init__(self, N, precision="fp64", stream=None):
        import torch
        self._L = lib()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        st = self._L.dgd_create(int(N), prec, ctypes.c_void_p(stream), ctypes.byref(h))
        if st != 0:
            raise DGDError(st, "dgd_create failed")
        self.h = h
        self.N = int(N)
        self.precision = prec
        Lm, Q, Ns, Nt = (ctypes.c_int() for _ in range(4))
        self._chk(self._L.dgd_sizes(self.h, ctypes.byref(Lm), ctypes.byref(Q),
                                    ctypes.byref(Ns), ctypes.byref(Nt)))
        self.L, self.Q, self.Ns, self.Nt = Lm.value, Q.value, Ns.value, Nt.value
        self.ne = 0
        self.nrec = 0

    def _chk(self, st):
        if st != 0:
            msg = self._L.dgd_last_error(self.h)
            raise DGDError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self._L.dgd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- setup -----------------------------------------------------------------
    def set_mesh(self, xyz, tets, face_tag, periodic_map=None):
        xyz = _f64(xyz)
        tets = np.ascontiguousarray(tets, dtype=np.int64)
        tag = np.ascontiguousarray(face_tag, dtype=np.int8)
        pm = None if periodic_map is None else np.ascontiguousarray(periodic_map, dtype=np.int64)
        self._chk(self._L.dgd_set_mesh(
            self.h, xyz.shape[0], _dp(xyz), tets.shape[0], tets.ctypes.data_as(c_i64p),
            tag.ctypes.data_as(c_i8p), None if pm is None else pm.ctypes.data_as(c_i64p)))
        self.ne = tets.shape[0]

    def set_material(self, rho, lambda0, mu0, gamma_r, xi0, Cd):
        arrs = [_f64(a) for a in (rho, lambda0, mu0, gamma_r, xi0, Cd)]
        self._chk(self._L.dgd_set_material(self.h, *[_dp(a) for a in arrs]))
        self.material = dict(zip(("rho", "lambda0", "mu0", "gamma_r", "xi0", "Cd"), arrs))

    def set_material_ivm(self, rho, lambda0, mu0, gamma_b, tau_b):
        """Internal-variable rheology (Eq. ivm-model) in place of the CDM law."""
        arrs = [_f64(a) for a in (rho, lambda0, mu0, gamma_b, tau_b)]
        self._chk(self._L.dgd_set_material_ivm(self.h, *[_dp(a) for a in arrs]))
        self.material = dict(zip(("rho", "lambda0", "mu0", "gamma_b", "tau_b"), arrs))

    def set_params(self, dt, alpha_max):
        self._chk(self._L.dgd_set_params(self.h, float(dt), float(alpha_max)))

    def get_quadrature_points(self, e0=0, count=None):
        count = self.ne - e0 if count is None else count
        out = np.zeros((count, self.Q, 3))
        self._chk(self._L.dgd_get_quadrature_points(self.h, int(e0), int(count), _dp(out)))
        return out

    def set_state_from_points(self, vals, e0=0):
        v = _f64(vals)
        count = v.size // (self.Q * 10)
        v = v.reshape(count, self.Q, 10)
        self._chk(self._L.dgd_set_state_from_points(self.h, int(e0), int(count), _dp(v)))

    def set_state(self, dofs):
        """dofs: numpy (ne, 10, L) or a float64 torch tensor on the device."""
        if isinstance(dofs, np.ndarray):
            d = _f64(dofs, (self.ne, 10, self.L))
            self._chk(self._L.dgd_set_state(self.h, d.ctypes.data_as(ctypes.c_void_p), 0))
        else:
            assert dofs.is_cuda and dofs.is_contiguous() and dofs.numel() == self.ne * 10 * self.L
            self._chk(self._L.dgd_set_state(self.h, ctypes.c_void_p(dofs.data_ptr()), 1))

    def get_state(self, out=None):
        if out is None:
            out = np.zeros((self.ne, 10, self.L))
        if isinstance(out, np.ndarray):
            self._chk(self._L.dgd_get_state(self.h, out.ctypes.data_as(ctypes.c_void_p), 0))
        else:
            self._chk(self._L.dgd_get_state(self.h, ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def get_point_values(self, e0=0, count=None, out=None):
        """Point values (count, Q, 10) at the volume quadrature points, FP64;
        out: None (a new numpy array) or a float64 device tensor."""
        count = self.ne - e0 if count is None else count
        if out is None:
            out = np.zeros((count, self.Q, 10))
        if isinstance(out, np.ndarray):
            assert out.dtype == np.float64 and out.size == count * self.Q * 10
            self._chk(self._L.dgd_get_point_values(self.h, int(e0), int(count),
                                                   out.ctypes.data_as(ctypes.c_void_p), 0))
        else:
            assert out.is_cuda and out.is_contiguous() and out.numel() == count * self.Q * 10
            self._chk(self._L.dgd_get_point_values(self.h, int(e0), int(count),
                                                   ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def set_time(self, t):
        self._chk(self._L.dgd_set_time(self.h, float(t)))

    def get_time(self):
        t = ctypes.c_double()
        self._chk(self._L.dgd_get_time(self.h, ctypes.byref(t)))
        return t.value

    def set_predictor(self, kind="ck", iterations=0):
        """Predictor of the step: "ck" (linearised Cauchy-Kovalevskaya) or
        "picard" (Picard iteration, `iterations` sweeps, 0 = N + 1)."""
        k = {"ck": 0, "picard": 1}[kind] if isinstance(kind, str) else int(kind)
        self._chk(self._L.dgd_set_predictor(self.h, k, int(iterations)))

    def make_clusters(self, cfl=0.5, max_clusters=8):
        """(cluster per element int32, dt0) proposed from the admissible steps."""
        cl = np.zeros(self.ne, dtype=np.int32)
        dt0 = ctypes.c_double()
        self._chk(self._L.dgd_make_clusters(self.h, float(cfl), int(max_clusters),
                                            cl.ctypes.data_as(ctypes.c_void_p), ctypes.byref(dt0)))
        return cl, dt0.value

    def set_clusters(self, cluster, dt0=0.0):
        """Local time stepping clusters (None removes them)."""
        if cluster is None:
            self._chk(self._L.dgd_set_clusters(self.h, None, 0.0))
            return
        cl = np.ascontiguousarray(cluster, dtype=np.int32)
        assert cl.shape == (self.ne,)
        self._chk(self._L.dgd_set_clusters(self.h, cl.ctypes.data_as(ctypes.c_void_p), float(dt0)))

    def step_lts(self, nmacro=1):
        self._chk(self._L.dgd_step_lts(self.h, int(nmacro)))

    def set_point_sources(self, xyz, M6, t_onset, stf_param, stf_kind):
        xyz = _f64(xyz, (-1, 3))
        n = xyz.shape[0]
        M6 = _f64(M6, (n, 6))
        on = _f64(t_onset, (n,))
        par = _f64(stf_param, (n,))
        self._chk(self._L.dgd_set_point_sources(self.h, n, _dp(xyz), _dp(M6), _dp(on), _dp(par),
                                                int(stf_kind)))

    def set_receivers(self, xyz):
        xyz = _f64(xyz, (-1, 3))
        self._chk(self._L.dgd_set_receivers(self.h, xyz.shape[0], _dp(xyz)))
        self.nrec = xyz.shape[0]

    # ---- run ------------------------------------------------------------------------
    def step(self, nsteps=1):
        self._chk(self._L.dgd_step(self.h, int(nsteps)))

    def set_check_interval(self, every):
        self._chk(self._L.dgd_set_check_interval(self.h, int(every)))

    def synchronize(self):
        self._chk(self._L.dgd_synchronize(self.h))

    def get_seismograms(self):
        n = ctypes.c_int64()
        self._chk(self._L.dgd_num_seismogram_steps(self.h, ctypes.byref(n)))
        out = np.zeros((n.value, self.nrec, 3))
        if n.value and self.nrec:
            self._chk(self._L.dgd_get_seismograms(self.h, _dp(out), None))
        return out

    def clear_seismograms(self):
        self._chk(self._L.dgd_clear_seismograms(self.h))

    def energy(self):
        e = ctypes.c_double()
        self._chk(self._L.dgd_energy(self.h, ctypes.byref(e)))
        return e.value

    def energy_noalloc(self, out):
        """dgd_energy_noalloc: the energy written to ``out``, a float64 torch
        tensor of one element on the device, without allocating."""
        import torch
        assert out.is_cuda and out.dtype == torch.float64 and out.numel() == 1
        self._chk(self._L.dgd_energy_noalloc(self.h, ctypes.c_void_p(out.data_ptr())))

    def wavespeed_change(self):
        out = np.zeros(self.ne)
        self._chk(self._L.dgd_wavespeed_change(self.h, _dp(out)))
        return out

    def set_profiling(self, on=True):
        self._chk(self._L.dgd_set_profiling(self.h, int(bool(on))))

    def get_kernel_times(self):
        """(ms[10], launches[10]) for the predictor, face fluxes, sources,
        receivers, the adjoint's predictor recomputation, faces, volume,
        receivers, the lift + update, and the volume integrals."""
        ms = np.zeros(NUM_KERNEL_CLASSES)
        n = np.zeros(NUM_KERNEL_CLASSES, dtype=np.int64)
        self._chk(self._L.dgd_get_kernel_times(self.h, _dp(ms), n.ctypes.data_as(c_i64p)))
        return ms, n

    # ---- discrete adjoint ----------------------------------------------------------
    def adjoint_step(self, state_n, lam, dl_dseis=None, grad_mu0=None, grad_cd=None):
        """One reverse step on the device (dgd_adjoint_step): float64 torch
        tensors on the device, state_n and lam (ne, 10, L), dl_dseis (nrec, 3)
        or None, grad_mu0 / grad_cd (ne,) or None.  lam is overwritten with
        lambda^n; the step's gradients are added to grad_mu0, grad_cd."""
        def ptr(t, n):
            if t is None:
                return None
            assert t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8
            assert t.is_contiguous() and t.numel() == n
            return ctypes.c_void_p(t.data_ptr())
        n = self.ne * 10 * self.L
        self._chk(self._L.dgd_adjoint_step(self.h, ptr(state_n, n), ptr(lam, n),
                                           ptr(dl_dseis, self.nrec * 3),
                                           ptr(grad_mu0, self.ne), ptr(grad_cd, self.ne)))

    def adjoint_step_host(self, lam_next):
        """(lam_n, grad_mu0, grad_cd) of one step at the current state, host
        arrays (dgd_adjoint_step_host, a test helper)."""
        lam = _f64(lam_next, (self.ne, 10, self.L))
        out = np.zeros((self.ne, 10, self.L))
        gmu = np.zeros(self.ne)
        gcd = np.zeros(self.ne)
        self._chk(self._L.dgd_adjoint_step_host(self.h, _dp(lam), _dp(out), _dp(gmu), _dp(gcd)))
        return out, gmu, gcd

    def tape_id(self):
        """Id of the kept checkpointed run (0: none)."""
        i = ctypes.c_int64()
        self._chk(self._L.dgd_tape_id(self.h, ctypes.byref(i)))
        return i.value

    def forward_checkpointed(self, nsteps, every):
        self._chk(self._L.dgd_forward_checkpointed(self.h, int(nsteps), int(every)))

    def backward(self, dl_dseis, want_u0=False):
        """(grad_mu0, grad_cd[, grad_u0]) of the last checkpointed run."""
        g = None if (self.nrec == 0 or dl_dseis is None) else _f64(dl_dseis)
        gmu = np.zeros(self.ne)
        gcd = np.zeros(self.ne)
        gu = np.zeros((self.ne, 10, self.L)) if want_u0 else None
        self._chk(self._L.dgd_backward(self.h, None if g is None else _dp(g), _dp(gmu), _dp(gcd),
                                       None if gu is None else _dp(gu)))
        return (gmu, gcd, gu) if want_u0 else (gmu, gcd)

    def release_tape(self):
        self._chk(self._L.dgd_release_tape(self.h))

    def get_time_point_states(self):
        out = np.zeros((self.ne, self.Nt, 10, self.L))
        self._chk(self._L.dgd_get_time_point_states(self.h, _dp(out)))
        return out


def from_workload(w, precision="fp64", stream=None, state=True):
    """Simulation set up with a :class:`workloads.Workload` (mesh, material,
    dt, initial condition projected on the device, sources, receivers)."""
    sim = Simulation(w.N, precision, stream)
    m = w.mesh
    sim.set_mesh(m["xyz"], m["tets"], m["face_tag"], m["periodic_map"])
    mat = w.material
    if getattr(w, "rheology", "cdm") == "ivm":
        sim.set_material_ivm(mat["rho"], mat["lambda0"], mat["mu0"], mat["gamma_b"], mat["tau_b"])
    else:
        sim.set_material(mat["rho"], mat["lambda0"], mat["mu0"], mat["gamma_r"], mat["xi0"],
                         mat["Cd"])
    sim.set_params(w.dt, w.alpha_max)
    if state:
        # evaluate the initial condition slice by slice to bound host memory
        chunk = max(1, (1 << 22) // sim.Q)
        for e0 in range(0, sim.ne, chunk):
            cnt = min(chunk, sim.ne - e0)
            x = sim.get_quadrature_points(e0, cnt)
            elem = np.repeat(np.arange(e0, e0 + cnt), sim.Q)
            sim.set_state_from_points(w.ic(x.reshape(-1, 3), elem), e0)
    if w.sources is not None:
        s = w.sources
        sim.set_point_sources(s["xyz"], s["M6"], s["t_onset"], s["stf_param"], s["stf_kind"])
    if w.receivers is not None:
        sim.set_receivers(w.receivers)
    return sim
