#!/usr/bin/env python3
"""Throughput of the CDM ADER-DG step on one MI355X.

One step = one pass of the whole hot path (predictor, volume, faces,
boundaries, update) over the synthetic workload.  Default workload: the
mid-size configuration c2 -- 48^3 cubes x 6 = 663,552 tetrahedra, degree 3
(20 modes, 200 DOFs per element), soft basin over rock, free top, absorbing
sides, 32 Gaussian strain pulses, damage alpha0 ~ U(0, 0.05).  The FP32 form
is the headline value; FP64 and BF16-MFMA forms run the same steps and are
reported beside it with their L2 difference from the FP64 GPU state.

Prints one JSON line (see the keys below).  The FP64 CPU oracle is timed on
a bounded sample (the same recipe on a 6^3-cube mesh, 2 steps) on the host.
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
KERNELS = ("predict_volume", "face_flux", "sources", "receivers",
           "adj_predict_recompute", "adj_face", "adj_volume", "adj_receivers", "lift_update")
STEP_KERNELS = ("predict_volume", "face_flux", "lift_update")


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
    k1_mm = (2 * Q * L * 10                       # nodal values at t_n
             + N * (3 * L * 10 * 10 * 2 + 3 * L * L * 10 * 2)   # CK: U A*^T, K^e contraction
             + 2 * L * Q                          # source projection at t_n
             + Nt * (N + 1) * L * 10 * 2          # Taylor sums
             + Nt * 2 * Q * L * 10                # nodal values at the time points
             + 2 * 3 * L * Q * 9 + 2 * L * Q)     # volume and source contractions
    k1_pw = Q * 400 + Nt * Q * 230
    trace = Nt * 2 * Ns * L * 10                  # one side's traces at all time points
    ff = ni * (2 * trace + Ns * Nt * 470 + Ns * Nt * 10 * 2) + nb * (trace + Ns * Nt * 300 + Ns * Nt * 10 * 2)
    lift = ne * (4 * 2 * L * Ns * 10 + 4 * Ns * 10 + 10 * L)
    return {"predict_volume": (k1_mm + k1_pw) * ne, "face_flux": ff, "lift_update": lift}


def bytes_per_launch(w, prec):
    """Algorithmic HBM bytes per launch (each array touched once; neighbour
    time-point states counted once, as if served from L2)."""
    L, Q, Ns, Nt = dims(w.N)
    ne = w.ne
    ni, nb = face_counts(w)
    t = 8 if prec == "fp64" else 4
    state = 9 * L * t + L * 8
    uz = Nt * 10 * L * t
    k1 = ne * (state + uz + state + 16 * 8 + 8 * 8)     # read U, write U_z, write partial
    flux = Ns * 10 * t
    ff = ne * uz + (ni + nb) * (flux + 8 * 4) + ne * (4 * 4 * 8 + 8 * 8)
    k3 = ne * (4 * flux + 2 * state + 4 * 4 * 8 + 4 * 4)
    return {"predict_volume": k1, "face_flux": ff, "lift_update": k3}


def kernel_source_hash():
    """Hash of the step kernels' sources with comments and blank lines removed
    (a comment edit does not change the measured code)."""
    h = hashlib.sha256()
    for f in ("kernels.hpp", "physics.hpp", "mfma.hpp"):
        with open(os.path.join(ROOT, "paper_2502_09714_amd", "csrc", f)) as fh:
            src = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in src.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code.strip():
                h.update((code + "\n").encode())
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


def run_precision(w, prec, steps, warmup, want_state=True):
    import torch
    from paper_2502_09714_amd.api import from_workload
    sim = from_workload(w, prec)
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
    if observed:
        sim.set_material(**perturbed_material(base, seed=2))
        sim.step(steps)
        obs = sim.get_seismograms()
        sim.set_material(**base)
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
    return {"workload": f"{w.name}: {w.ne} tets, N={w.N}, {len(seis[0])} receivers",
            "forward_s": t1 - t0, "backward_s": t3 - t2,
            "backward_over_forward": (t3 - t2) / (t1 - t0),
            "backward_kernel_ms_per_step": {k: float(ms[i]) / steps for i, k in enumerate(KERNELS)
                                            if launches[i] > 0},
            "steps": steps, "checkpoint_every": every,
            "finite": bool(np.isfinite(gmu).all() and np.isfinite(gcd).all())}


def rel_l2(a, b):
    import numpy as np
    out = {}
    for k, s in (("strain", slice(0, 6)), ("velocity", slice(6, 9)), ("alpha", slice(9, 10))):
        out[k] = float(np.linalg.norm(a[:, s] - b[:, s]) / max(np.linalg.norm(b[:, s]), 1e-300))
    out["all"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return out


def cpu_baseline(name, n_sample, steps):
    import torch
    from oracle.step import from_workload as oracle_from
    from workloads import make_workload
    threads = min(16, os.cpu_count() or 1)
    torch.set_num_threads(threads)
    w = make_workload(name, n=n_sample)
    S = oracle_from(w)
    U = S.project(w.ic)
    U = S.step(U)                      # first call pays one-time set-up costs
    t0 = time.perf_counter()
    S.run(U, steps)
    dt = time.perf_counter() - t0
    dofs = w.ne * w.L * 10
    return {"value": dofs * steps / dt, "unit": "DOF-updates/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{name} recipe on {n_sample}^3 cubes x 6 = {w.ne} tets, N={w.N}, "
                      f"{steps} steps after one untimed step, {dt:.1f} s, torch float64 CPU"}


def run_ivm(args, precs, dofs):
    """Step timing of the benchmark workload with the IVM law, per precision."""
    from workloads import make_workload
    wi = make_workload(args.workload, n=args.n, rheology="ivm")
    ri = {p: run_precision(wi, p, args.steps, args.warmup) for p in precs}
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--n", type=int, default=None, help="override the cube count")
    ap.add_argument("--precisions", default="fp32,fp64,bf16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=6)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--adjoint-precisions", default="fp32,fp64",
                    help="precisions whose checkpointed adjoint is timed ('' for none)")
    ap.add_argument("--checkpoint-every", type=int, default=5)
    ap.add_argument("--adjoint-workload", default="c4",
                    help="workload of the full-length adjoint timing ('' for none)")
    ap.add_argument("--adjoint-workload-precisions", default="fp32")
    ap.add_argument("--ivm-precisions", default="fp32,fp64",
                    help="precisions of the IVM-rheology step timing ('' for none)")
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
        res[p] = run_precision(w, p, args.steps, args.warmup)
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
                   "tets": ne, "degree": w.N, "dofs": dofs, "dt": w.dt},
        "roofline": roof,
        "kernels": other,
    }
    for p in precs:
        line[f"{p}_dof_updates_per_s"] = rate(p)
        line[f"{p}_ms_per_step"] = res[p]["ms_per_step"]
    if "fp64" in res:
        for p in precs:
            if p != "fp64":
                line[f"speedup_{p}_vs_fp64"] = rate(p) / rate("fp64")
                line[f"l2_{p}_vs_fp64_gpu"] = rel_l2(res[p]["state"], res["fp64"]["state"])
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
        a = run_adjoint(w, p, args.steps, args.checkpoint_every)
        print(f"adjoint {p}: {a}", file=sys.stderr, flush=True)
        line[f"adjoint_{p}"] = a
    if args.adjoint_workload:
        # the differentiation-form workload: 82,944 tets, N=3, point source,
        # 16 receivers, 400 steps with checkpoints every 20, FP32
        wa = make_workload(args.adjoint_workload)
        for p in [q.strip() for q in args.adjoint_workload_precisions.split(",") if q.strip()]:
            a = run_adjoint(wa, p, wa.nsteps, 20, observed=True)
            print(f"adjoint {args.adjoint_workload} {p}: {a}", file=sys.stderr, flush=True)
            line[f"adjoint_{args.adjoint_workload}_{p}"] = a
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_sample_n, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
