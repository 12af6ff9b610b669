#!/usr/bin/env python3
"""Throughput of the CDM ADER-DG step on one MI355X.

One step = one pass of the whole hot path (predictor, volume, faces,
boundaries, update, point sources, receivers) over the synthetic workload.
Default workload: the largest configuration, c5 -- 96^3 cubes x 6 =
5,308,416 tetrahedra, degree 4 (35 modes, 350 DOFs per element), 24 km box,
3 km gradient basin over rock, free top, absorbing sides, 64 subfault point
sources, 16 receivers.  The FP32 form is the headline value; the BF16-MFMA
(split operands, FP32 accumulation) and FP64 forms run the same steps and
are reported beside it with their device-memory footprint.

Precision errors: the precision-form configuration c3 (64^3 cubes x 6 =
1,572,864 tets, N = 4, lognormal moduli) is run in FP64, FP32 and BF16 from
the same initial state for --error-steps steps (default 100; the specified
1000 with --error-steps 1000), and the relative L2 and the pointwise maximum
(at the volume quadrature points) of every quantity group are reported
against the FP64 GPU state.

Prints one JSON line.  The FP64 CPU oracle is timed on a bounded sample (the
c5 recipe on a 3^3-cube mesh, a few steps, one thread and all threads).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DG DOF-updates/s on 1 GPU, FP32/BF16 vs FP64 at stated L2 error; adjoint/forward cost"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
HBM_TBS = 8.0
KERNELS = ("predict", "face_flux", "sources", "receivers",
           "adj_predict_recompute", "adj_face", "adj_volume", "adj_receivers", "lift_update",
           "volume")
STEP_KERNELS = ("predict", "volume", "face_flux", "lift_update")


def dims(N):
    L = (N + 1) * (N + 2) * (N + 3) // 6
    return L, (N + 1) ** 3, (N + 1) ** 2, N + 1


def face_counts(w):
    tag = w.mesh["face_tag"]
    nb = int((tag > 0).sum())
    return (w.ne * 4 - nb) // 2, nb          # interior faces, boundary faces


def flops_per_launch(w):
    """Algorithmic FLOPs per launch of the step kernels (dense counts of what
    the method computes; no padding, no exploited sparsity).  Pointwise costs
    per point: tangent 400, stress+flux+rate 230, LLF 470 (two normal fluxes,
    the acoustic-tensor eigenvalue, the combination), boundary flux 300."""
    N = w.N
    L, Q, Ns, Nt = dims(N)
    ne = w.ne
    ni, nb = face_counts(w)
    kp = (2 * Q * L * 10                          # nodal values at t_n
          + N * (3 * L * 10 * 10 * 2 + 3 * L * L * 10 * 2)   # CK: U A*^T, K^e contraction
          + 2 * L * Q                             # source projection at t_n
          + Nt * (N + 1) * L * 10 * 2             # Taylor sums
          + Q * 400)                              # pointwise tangent at t_n
    kv = (Nt * 2 * Q * L * 10                     # nodal values at the time points
          + 2 * 3 * L * Q * 9 + 2 * L * Q         # volume and source contractions
          + Nt * Q * 230)                         # stress, flux, damage rate per (z, q)
    trace = Nt * 2 * Ns * L * 10                  # one side's traces at all time points
    ff = ni * (2 * trace + Ns * Nt * 470 + Ns * Nt * 10 * 2) + nb * (trace + Ns * Nt * 300 + Ns * Nt * 10 * 2)
    lift = ne * (4 * 2 * L * Ns * 10 + 4 * Ns * 10 + 10 * L)
    return {"predict": kp * ne, "volume": kv * ne, "face_flux": ff, "lift_update": lift}


def bytes_per_launch(w, prec):
    """Algorithmic HBM bytes per launch (each array touched once; neighbour
    time-point states counted once, as if served from L2)."""
    L, Q, Ns, Nt = dims(w.N)
    ne = w.ne
    ni, nb = face_counts(w)
    t = 8 if prec == "fp64" else 4
    state = 9 * L * t + L * 8
    uz = Nt * 10 * L * t
    kp = ne * (state + uz + 16 * 8 + 8 * 8)             # read U, write U_z
    kv = ne * (uz + 2 * state + 16 * 8 + 8 * 8)         # read U_z and U, write the partial update
    flux = Ns * 10 * t
    ff = ne * uz + (ni + nb) * (flux + 8 * 4) + ne * (4 * 4 * 8 + 8 * 8)
    k3 = ne * (4 * flux + 2 * state + 4 * 4 * 8 + 4 * 4)
    return {"predict": kp, "volume": kv, "face_flux": ff, "lift_update": k3}


HASHED_SOURCES = ("kernels.hpp", "physics.hpp", "mfma.hpp", "dgd.hip")


def kernel_source_hash():
    """Hash of the device sources (kernels, their launch code in dgd.hip) with
    comments and blank lines removed (a comment edit does not change the
    measured code), and of the compiler flags of the build."""
    h = hashlib.sha256()
    for f in HASHED_SOURCES:
        with open(os.path.join(ROOT, "paper_2502_09714_amd", "csrc", f)) as fh:
            src = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in src.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code.strip():
                h.update((code + "\n").encode())
    with open(os.path.join(ROOT, "paper_2502_09714_amd", "build.py")) as fh:
        m = re.search(r"HIPCC_FLAGS = \[(.*?)\]", fh.read(), flags=re.S)
    flags = re.findall(r'"([^"]+)"', m.group(1)) if m else []
    h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload, prec):
    """HBM traffic per launch from a committed rocprofv3 PMC summary, if the
    kernel sources are unchanged since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{prec}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_hash:\s*(\w+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != kernel_source_hash():
        return None
    return float(b.group(1))


def load_error_table(workload, steps):
    """A precision-error table of a longer run (too long for the default
    bench) from its committed summary, if the kernel sources are unchanged
    since it was taken."""
    path = os.path.join(ROOT, "profiles", f"precision_errors_{workload}_{steps}steps.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_hash:\s*(\w+)", txt)
    t = re.search(r"^table:\s*(\{.*\})\s*$", txt, flags=re.M)
    if not m or not t or m.group(1) != kernel_source_hash():
        return None
    out = json.loads(t.group(1))
    out["source"] = os.path.relpath(path, ROOT)
    return out


def run_precision(w, prec, steps, warmup, want_state=True):
    import torch
    from paper_2502_09714_amd.api import from_workload
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    sim = from_workload(w, prec)
    sim.synchronize()
    footprint = free0 - torch.cuda.mem_get_info()[0]
    sim.set_check_interval(1 << 40)
    sim.step(warmup)
    sim.synchronize()
    sim.get_kernel_times()
    sim.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, launches = sim.get_kernel_times()
    sim.set_profiling(False)
    state = sim.get_state() if want_state else None
    out = {"seconds": t1 - t0, "ms_per_step": 1e3 * (t1 - t0) / steps,
           "device_bytes": int(footprint),
           "kernel_ms": {k: float(ms[i]) for i, k in enumerate(KERNELS)},
           "kernel_launches": {k: int(launches[i]) for i, k in enumerate(KERNELS)},
           "state": state, "L": sim.L, "ne": sim.ne}
    sim.close()
    return out


def run_adjoint(w, prec, steps, every, observed=False):
    """Checkpointed forward run (seismograms recorded) and the backward sweep
    for the misfit J = |v - v_obs|^2 / 2 (v_obs from the run with mu0 and C_d
    perturbed per element, if observed, else v_obs = 0): wall time of each and
    the per-kernel times of the backward sweep."""
    import numpy as np
    import torch
    from paper_2502_09714_amd.api import from_workload
    from workloads.configs import perturbed_material
    sim = from_workload(w, prec)
    if sim.nrec == 0:
        m = w.mesh
        cent = m["xyz"][m["tets"][[0, w.ne // 3, w.ne // 2, (2 * w.ne) // 3]]].mean(axis=1)
        sim.set_receivers(cent)
    sim.set_check_interval(1 << 40)
    U0 = sim.get_state()
    base = dict(sim.material)
    obs = 0.0
    print(f"adjoint {w.name}: set up", file=sys.stderr, flush=True)
    if observed:
        sim.set_material(**perturbed_material(base, seed=2))
        sim.step(steps)
        obs = sim.get_seismograms()
        sim.set_material(**base)
        print(f"adjoint {w.name}: observed run done", file=sys.stderr, flush=True)
    sim.set_state(U0)
    sim.clear_seismograms()
    sim.forward_checkpointed(2, 1)          # warm-up of both sweeps
    sim.backward(sim.get_seismograms())
    sim.set_state(U0)
    sim.set_time(0.0)
    sim.clear_seismograms()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.forward_checkpointed(steps, every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"adjoint {w.name}: checkpointed forward {t1 - t0:.1f} s", file=sys.stderr, flush=True)
    seis = sim.get_seismograms()
    sim.get_kernel_times()
    sim.set_profiling(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    gmu, gcd = sim.backward(seis - obs)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ms, launches = sim.get_kernel_times()
    sim.set_profiling(False)
    sim.close()
    out = {"workload": f"{w.name}: {w.ne} tets, N={w.N}, {len(seis[0])} receivers",
           "forward_s": t1 - t0, "backward_s": t3 - t2,
           "backward_over_forward": (t3 - t2) / (t1 - t0),
           "backward_kernel_ms_per_step": {k: float(ms[i]) / steps for i, k in enumerate(KERNELS)
                                           if launches[i] > 0},
           "steps": steps, "checkpoint_every": every,
           # the replay kept each segment's time-point states (else the
           # adjoint recomputes the prediction per step)
           "time_points_kept": bool(launches[KERNELS.index("adj_predict_recompute")] == 0),
           "finite": bool(np.isfinite(gmu).all() and np.isfinite(gcd).all())}
    return out, (gmu, gcd, obs, U0, base)


def fd_check(w, steps, grads, nelem, seed=31):
    """Central differences (relative step 1e-4) of the FP64 forward misfit on
    nelem elements drawn at random, against the adjoint gradients."""
    import numpy as np
    from paper_2502_09714_amd.api import from_workload
    gmu, gcd, obs, U0, base = grads
    sim = from_workload(w, "fp64", state=False)
    m = w.mesh
    if sim.nrec == 0:
        recx = m["xyz"][m["tets"][[0, w.ne // 3, w.ne // 2, (2 * w.ne) // 3]]].mean(axis=1)
        sim.set_receivers(recx)
    else:
        recx = np.asarray(w.receivers)
    sim.set_check_interval(1 << 40)

    def misfit(mat):
        sim.set_material(**mat)
        sim.set_state(U0)
        sim.set_time(0.0)
        sim.clear_seismograms()
        sim.step(steps)
        return 0.5 * float(((sim.get_seismograms() - obs) ** 2).sum())

    # elements drawn at random among those the receivers can see within the
    # run: centroid within half the distance a P wave travels in it
    cent = m["xyz"][m["tets"]].mean(axis=1)
    cp = np.sqrt((base["lambda0"] + 2 * base["mu0"]) / base["rho"]).max()
    reach = 0.5 * cp * steps * w.dt
    dist = np.min(np.linalg.norm(cent[:, None, :] - recx[None, :, :], axis=2), axis=1)
    near = np.nonzero(dist < reach)[0]
    idx = [int(e) for e in np.random.default_rng(seed).choice(near, min(nelem, len(near)),
                                                              replace=False)]
    j0 = misfit(base)
    rows = []
    for which, g in (("mu0", gmu), ("Cd", gcd)):
        for e in idx:
            h = 1e-4 * base[which][e]
            mp = {k: v.copy() for k, v in base.items()}
            mp[which][e] += h
            jp = misfit(mp)
            mp[which][e] -= 2 * h
            jm = misfit(mp)
            fd = (jp - jm) / (2 * h)
            # a difference of the misfit below ~1e-12 of the misfit itself is
            # rounding of the FP64 runs, not a derivative
            dj = abs(float(g[e])) * 2 * float(h)
            rows.append({"param": which, "element": e, "adjoint": float(g[e]), "fd": float(fd),
                         "rel_diff": abs(float(g[e]) - float(fd)) / max(abs(float(fd)), 1e-300),
                         "misfit": float(j0), "adjoint_delta_misfit": dj,
                         "resolved": bool(dj > 1e-12 * abs(float(j0)))})
            print(f"fd check: {rows[-1]}", file=sys.stderr, flush=True)
    sim.close()
    return rows


def run_lts(w, prec, nmacro, gts_ms_per_step, max_clusters=8):
    """Clustered local time stepping on the step workload: clusters proposed
    from the per-element admissible steps, nmacro macro steps timed."""
    import numpy as np
    import torch
    from paper_2502_09714_amd.api import from_workload
    sim = from_workload(w, prec)
    sim.set_check_interval(1 << 40)
    cl, dt0 = sim.make_clusters(0.5, max_clusters)
    sim.set_clusters(cl, dt0)
    C = int(cl.max()) + 1
    sim.step_lts(1)                       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step_lts(nmacro)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    sim.close()
    counts = np.bincount(cl, minlength=C)
    mdt = dt0 * 2 ** (C - 1)
    L = w.L
    # element updates per macro step: cluster c steps 2^(C-1-c) times
    upd = sum(int(counts[c]) * 2 ** (C - 1 - c) for c in range(C))
    gts_steps = mdt / w.dt
    return {"clusters": [int(x) for x in counts], "dt0": dt0, "macro_dt": mdt,
            "macro_steps": nmacro, "ms_per_macro_step": 1e3 * secs / nmacro,
            "dof_updates_per_s": upd * L * 10 * nmacro / secs,
            "simulated_s_per_wall_s": mdt * nmacro / secs,
            "global_step_simulated_s_per_wall_s": w.dt / (gts_ms_per_step * 1e-3),
            "speedup_vs_global_step": (gts_steps * gts_ms_per_step) / (1e3 * secs / nmacro),
            "work_ratio": upd / (w.ne * gts_steps)}


def run_picard(w, prec, steps, warmup):
    """Step time with the Picard-iteration predictor (N + 1 sweeps)."""
    import torch
    from paper_2502_09714_amd.api import from_workload
    sim = from_workload(w, prec)
    sim.set_predictor("picard")
    sim.set_check_interval(1 << 40)
    sim.step(warmup)
    sim.synchronize()
    sim.get_kernel_times()
    sim.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    secs = time.perf_counter() - t0
    ms, _ = sim.get_kernel_times()
    sim.close()
    return {"iterations": w.N + 1, "ms_per_step": 1e3 * secs / steps,
            "predictor_ms_per_step": float(ms[0]) / steps,
            "dof_updates_per_s": w.ne * w.L * 10 * steps / secs}


def rel_l2(a, b):
    import numpy as np
    out = {}
    for k, s in (("strain", slice(0, 6)), ("velocity", slice(6, 9)), ("alpha", slice(9, 10))):
        out[k] = float(np.linalg.norm(a[:, s] - b[:, s]) / max(np.linalg.norm(b[:, s]), 1e-300))
    out["all"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, n_sample, steps):
    """The FP64 oracle on the host's cores: the same recipe on a small cut
    (n_sample^3 cubes), `steps` steps with one thread and with all the threads
    torch uses here (the host's share of cores), after one untimed step."""
    import torch
    from oracle.step import from_workload as oracle_from
    from workloads import make_workload
    nproc = os.cpu_count() or 1
    allt = torch.get_num_threads()
    w = make_workload(name, n=n_sample)
    S = oracle_from(w)
    U = S.project(w.ic)
    U = S.step(U)                      # first call pays one-time set-up costs
    dofs = w.ne * w.L * 10
    rates, secs = {}, {}
    for th in (allt, 1):
        torch.set_num_threads(th)
        t0 = time.perf_counter()
        S.run(U, steps)
        secs[th] = time.perf_counter() - t0
        rates[th] = dofs * steps / secs[th]
    torch.set_num_threads(allt)
    return {"value": rates[allt], "unit": "DOF-updates/s", "cores": allt, "kind": "oracle",
            "one_thread_value": rates[1], "nproc": nproc, "cpu_model": cpu_model(),
            "sample": f"{name} recipe cut to {n_sample}^3 cubes x 6 = {w.ne} tets, N={w.N}: "
                      f"{steps} steps after one untimed step, {secs[allt]:.1f} s on {allt} threads "
                      f"and {secs[1]:.1f} s on 1 thread, torch float64 CPU; the rate is per "
                      f"DOF-update and carries over to the full mesh (the oracle is linear in "
                      f"the element count), i.e. extrapolated, not run at full size"}


GROUPS = (("strain", 0, 6), ("velocity", 6, 9), ("alpha", 9, 10))


def precision_errors(name, steps, precs, chunk=1 << 14):
    """Relative L2 (modal, uniform mesh) and pointwise maximum error (at the
    volume quadrature points, relative to the largest FP64 value) per quantity
    group of each precision against the FP64 GPU run, after `steps` steps from
    the same initial state (the FP64 projection of the initial condition)."""
    import torch
    from paper_2502_09714_amd.api import from_workload
    from workloads import make_workload
    w = make_workload(name)
    w.sources = None
    w.receivers = None
    ref = from_workload(w, "fp64")
    U0 = torch.empty((ref.ne, 10, ref.L), dtype=torch.float64, device="cuda")
    ref.get_state(U0)
    sims = {}
    for p in precs:
        sims[p] = from_workload(w, p, state=False)
        sims[p].set_state(U0)
    del U0
    t = {}
    for p, sim in [("fp64", ref)] + list(sims.items()):
        sim.set_check_interval(1 << 40)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            k = min(100, steps - done)
            sim.step(k)
            sim.synchronize()
            done += k
            print(f"errors {name}: {p} {done}/{steps} steps", file=sys.stderr, flush=True)
        t[p] = time.perf_counter() - t0
        print(f"errors {name}: {p} {steps} steps in {t[p]:.1f} s", file=sys.stderr, flush=True)
    Q, L = ref.Q, ref.L
    acc = {p: {g: [0.0, 0.0] for g, _, _ in GROUPS} for p in precs}   # sum d^2, max |d|
    ref_acc = {g: [0.0, 0.0] for g, _, _ in GROUPS}
    for e0 in range(0, ref.ne, chunk):
        cnt = min(chunk, ref.ne - e0)
        pr = torch.empty((cnt, Q, 10), dtype=torch.float64, device="cuda")
        ref.get_point_values(e0, cnt, pr)
        mr = torch.empty((cnt * 10 * L,), dtype=torch.float64, device="cuda")
        for p, sim in sims.items():
            pp = torch.empty_like(pr)
            sim.get_point_values(e0, cnt, pp)
            for g, a, b in GROUPS:
                acc[p][g][1] = max(acc[p][g][1], float((pp[..., a:b] - pr[..., a:b]).abs().max()))
        for g, a, b in GROUPS:
            ref_acc[g][1] = max(ref_acc[g][1], float(pr[..., a:b].abs().max()))
        del pr, mr
    Ur = torch.empty((ref.ne, 10, L), dtype=torch.float64, device="cuda")
    ref.get_state(Ur)
    for g, a, b in GROUPS:
        ref_acc[g][0] = float((Ur[:, a:b] ** 2).sum())
    for p, sim in sims.items():
        Up = torch.empty_like(Ur)
        sim.get_state(Up)
        for g, a, b in GROUPS:
            acc[p][g][0] = float(((Up[:, a:b] - Ur[:, a:b]) ** 2).sum())
        del Up
        sim.close()
    ref.close()
    out = {"workload": f"{name}: {w.mesh['n']}^3 cubes x 6 = {w.ne} tets, N={w.N}, "
                       f"{steps} steps from the same state (no sources)",
           "steps": steps, "reference": "fp64 GPU",
           "seconds": {p: round(v, 2) for p, v in t.items()}}
    for p in precs:
        out[p] = {g: {"l2": (acc[p][g][0] / ref_acc[g][0]) ** 0.5 if ref_acc[g][0] > 0 else 0.0,
                      "linf": acc[p][g][1] / ref_acc[g][1] if ref_acc[g][1] > 0 else 0.0}
                  for g, _, _ in GROUPS}
    return out


def run_ivm(args, precs, dofs):
    """Step timing of the benchmark workload with the IVM law, per precision."""
    from workloads import make_workload
    wi = make_workload(args.workload, n=args.n, rheology="ivm")
    ri = {p: run_precision(wi, p, args.steps, args.warmup, want_state="fp64" in precs)
          for p in precs}
    iv = {"workload": f"{args.workload} with the IVM law", "steps": args.steps}
    for p in precs:
        iv[f"{p}_ms_per_step"] = ri[p]["ms_per_step"]
        iv[f"{p}_dof_updates_per_s"] = dofs * args.steps / ri[p]["seconds"]
        iv[f"{p}_kernel_ms_per_step"] = {k: ri[p]["kernel_ms"][k] / args.steps
                                         for k in STEP_KERNELS}
    if "fp64" in ri:
        for p in precs:
            if p != "fp64":
                iv[f"l2_{p}_vs_fp64_gpu"] = rel_l2(ri[p]["state"], ri["fp64"]["state"])
    return iv


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--n", type=int, default=None, help="override the cube count")
    ap.add_argument("--precisions", default="fp32,bf16,fp64")
    ap.add_argument("--error-workload", default="c3",
                    help="workload of the precision-error table ('' for none)")
    ap.add_argument("--error-steps", type=int, default=100)
    ap.add_argument("--error-precisions", default="fp32,bf16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=3)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--adjoint-precisions", default="",
                    help="precisions whose checkpointed adjoint is timed on the step workload "
                         "('' for none)")
    ap.add_argument("--checkpoint-every", type=int, default=5)
    # c3 in FP32 with checkpoints every 10 steps: a segment's time-point
    # states (11 GB per step) then fit in HBM beside the checkpoints, and the
    # adjoint reads them instead of repeating the prediction
    ap.add_argument("--adjoint-runs", default="c4:400:20,c3:200:10,c3:200:20:bf16",
                    help="checkpointed adjoint runs workload:steps:every[:bf16] (FP32 "
                         "adjoint arithmetic; bf16: split-BF16 forward) ('' for none)")
    ap.add_argument("--adjoint-fd", type=int, default=0,
                    help="central differences on this many elements for the last adjoint run")
    ap.add_argument("--ivm-precisions", default="fp32",
                    help="precisions of the IVM-rheology step timing ('' for none)")
    ap.add_argument("--lts-workloads", default="c5f",
                    help="further workloads timed with local time stepping ('' for none)")
    ap.add_argument("--lts-macro-steps", type=int, default=3,
                    help="macro steps of the local-time-stepping timing (0 for none)")
    ap.add_argument("--picard-steps", type=int, default=3,
                    help="steps of the Picard-predictor timing (0 for none)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU only (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from workloads import make_workload
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calib:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1.0)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(f"copy calibration: 3 x {x.numel() * 4} bytes read + written", file=sys.stderr)

    w = make_workload(args.workload, n=args.n)
    precs = [p.strip() for p in args.precisions.split(",") if p.strip()]
    main_prec = precs[0]
    res = {}
    for p in precs:
        # the precision errors come from the c3 table below, not from these states
        res[p] = run_precision(w, p, args.steps, args.warmup, want_state=False)
        print(f"{p}: {res[p]['ms_per_step']:.3f} ms/step  kernels {res[p]['kernel_ms']}",
              file=sys.stderr, flush=True)
    L = res[main_prec]["L"]
    ne = res[main_prec]["ne"]
    dofs = ne * L * 10

    def rate(p):
        return dofs * args.steps / res[p]["seconds"]

    # dominant kernel of the headline precision
    km = res[main_prec]["kernel_ms"]
    kl = res[main_prec]["kernel_launches"]
    dom = max(STEP_KERNELS, key=lambda k: km[k])
    avg_ms = km[dom] / max(kl[dom], 1)
    flop_launch = flops_per_launch(w)[dom]
    achieved = flop_launch / (avg_ms * 1e-3) / 1e12
    traffic = load_traffic(dom, args.workload, main_prec)
    roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[main_prec],
            "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[main_prec], "traffic": traffic,
            "kernel": dom, "avg_launch_ms": avg_ms, "flop_per_launch": flop_launch,
            "algorithmic_bytes_per_launch": bytes_per_launch(w, main_prec)[dom]}
    other = {}
    for k in STEP_KERNELS:
        t = km[k] / max(kl[k], 1)
        other[k] = {"avg_launch_ms": t, "tflops": flops_per_launch(w)[k] / (t * 1e-3) / 1e12,
                    "hbm_tbs_algorithmic": bytes_per_launch(w, main_prec)[k] / (t * 1e-3) / 1e12}

    line = {
        "metric": METRIC, "value": rate(main_prec), "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res[main_prec]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "bf16-mfma/f32"}[main_prec],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w.mesh['n']}^3 cubes x 6 = {ne} tets, N={w.N} "
                               f"({L} modes, {L * 10} DOFs/element), {main_prec} with FP64 alpha",
                   "tets": ne, "degree": w.N, "dofs": dofs, "dt": w.dt,
                   "point_sources": 0 if w.sources is None else len(w.sources["xyz"]),
                   "receivers": 0 if w.receivers is None else len(w.receivers)},
        "roofline": roof,
        "kernels": other,
    }
    for p in precs:
        line[f"{p}_dof_updates_per_s"] = rate(p)
        line[f"{p}_ms_per_step"] = res[p]["ms_per_step"]
        line[f"{p}_device_bytes"] = res[p]["device_bytes"]
        line[f"{p}_kernel_ms_per_step"] = {k: res[p]["kernel_ms"][k] / args.steps for k in STEP_KERNELS}
    if "fp64" in res:
        for p in precs:
            if p != "fp64":
                line[f"speedup_{p}_vs_fp64"] = rate(p) / rate("fp64")
    if args.lts_macro_steps > 0:
        line["lts"] = run_lts(w, main_prec, args.lts_macro_steps, res[main_prec]["ms_per_step"])
        print(f"lts: {line['lts']}", file=sys.stderr, flush=True)
        for name in [q.strip() for q in args.lts_workloads.split(",") if q.strip()]:
            # a mesh where part of the elements limits the global step (c5f:
            # the c5 recipe with a band of layers 8 times thinner around the
            # fault): global step and local time stepping on the same mesh
            wl = make_workload(name)
            g = run_precision(wl, main_prec, 3, 1, want_state=False)
            ent = run_lts(wl, main_prec, args.lts_macro_steps, g["ms_per_step"])
            ent["workload"] = f"{name}: {wl.ne} tets, N={wl.N}, global step {wl.dt:.3e} s"
            ent["global_step_ms"] = g["ms_per_step"]
            line[f"lts_{name}"] = ent
            print(f"lts {name}: {ent}", file=sys.stderr, flush=True)
    if args.picard_steps > 0:
        line["picard"] = run_picard(w, main_prec, args.picard_steps, 1)
        print(f"picard: {line['picard']}", file=sys.stderr, flush=True)
    ivm_precs = [q.strip() for q in args.ivm_precisions.split(",") if q.strip()]
    if ivm_precs:
        # the same workload with the internal-variable rheology (Eq. ivm-model);
        # a failure here is reported in the line, not allowed to lose it
        try:
            line["ivm"] = run_ivm(args, ivm_precs, dofs)
        except Exception as exc:          # noqa: BLE001
            line["ivm"] = {"error": f"{type(exc).__name__}: {exc}"}
        print(f"ivm: {line['ivm']}", file=sys.stderr, flush=True)
    for p in [q.strip() for q in args.adjoint_precisions.split(",") if q.strip()]:
        a, _ = run_adjoint(w, p, args.steps, args.checkpoint_every)
        print(f"adjoint {p}: {a}", file=sys.stderr, flush=True)
        line[f"adjoint_{p}"] = a
    runs = [r.split(":") for r in args.adjoint_runs.split(",") if r.strip()]
    for i, spec in enumerate(runs):
        name, steps, every = spec[:3]
        aprec = spec[3] if len(spec) > 3 else "fp32"   # forward form; bf16: FP32 adjoint
        # checkpointed FP32 misfit gradient (mu0, C_d) against a run with the
        # perturbed model: c4 is the differentiation-form workload (82,944
        # tets, N=3, point source, 16 receivers, 400 steps, checkpoints every
        # 20), c3 the degree-4 precision-form mesh (1,572,864 tets)
        wa = make_workload(name)
        a, grads = run_adjoint(wa, aprec, int(steps), int(every), observed=True)
        if aprec == "bf16":
            a["arithmetic"] = "split-BF16 forward, FP32 adjoint"
        if args.adjoint_fd and i == len(runs) - 1:
            a["fd_check"] = fd_check(wa, int(steps), grads, args.adjoint_fd)
        print(f"adjoint {name} {aprec}: {a}", file=sys.stderr, flush=True)
        line[f"adjoint_{name}_{aprec}"] = a
    if args.error_workload:
        eprecs = [q.strip() for q in args.error_precisions.split(",") if q.strip()]
        line["precision_errors"] = precision_errors(args.error_workload, args.error_steps, eprecs)
        print(f"precision errors: {line['precision_errors']}", file=sys.stderr, flush=True)
        if args.error_steps < 1000:
            line["precision_errors_1000_steps"] = load_error_table(args.error_workload, 1000)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_sample_n, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
