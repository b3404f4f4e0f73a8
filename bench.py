"""Benchmark: ParaDiag solves of the 1D P1-FEM heat workload on one MI355X.

One step = one complete paradiag_solve (forward time transform, shifted
solves with the b reduction, capacitance GMRES, shifted solves, inverse
transform; plus refinement sweeps for the mixed form) of the n = 8191,
ell = 2048 problem whose inputs are already resident in HBM.  Prints ONE JSON
line.  `value` is space-time unknowns per second of the fastest form whose
error against the exact discrete solution is <= 1e-8.

The cpu_baseline leg (and only it) runs the CPU oracle: it times sequential
backward-Euler stepping on the host and measures the GPU results' error
against the exact modal solution at sampled space-time points.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VEC_PEAK_TFLOPS = 78.6    # 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
METRIC = "space-time unknowns/s at 1e-8 rel err (mixed vs FP64) + p50/p99 latency"
FLOPS_PER_UNKNOWN = 20.0       # shifted solves: real flops per real space-time unknown
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_fem1d_n8191_l2048_fp64.txt")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="fem1d",
                    choices=["fem1d", "ensemble", "serve", "alpha", "fom", "bdf", "fd2d"])
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--count", type=int, default=0, help="ensemble / stream size")
    ap.add_argument("--ensemble-precision", default="fp64", choices=["fp64", "mixed", "fp32"],
                    help="ensemble: precision of every plan (mixed plans do not batch: the "
                         "batched call solves them one after another)")
    ap.add_argument("--ensemble-autotune", action="store_true",
                    help="ensemble: plans time their tile widths at creation")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--forms", default="fp64,mixed,sine",
                    help="fp64, mixed, fp32: Algorithm 1 in that precision; alpha: "
                         "Algorithm 3 (float64) with the early-exit test; sine: Algorithm 1 "
                         "in float64 with the shifted solves in the sine basis")
    ap.add_argument("--alpha", type=float, default=1e-2,
                    help="alpha of the 'alpha' form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--serve-count", type=int, default=256,
                    help="requests of the serving stream in the default run (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=80.0,
                    help="fixed Poisson arrival rate of the serving stream (requests/s)")
    ap.add_argument("--no-2d", action="store_true",
                    help="skip the 2D (511^2, ell = 256) rows of the default run")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the library runs on exactly one GPU; --gpus %d is not supported "
              "(multi-GPU sharding is a design only)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2304_12597_amd import binding as pd
    from paper_2304_12597_amd import workloads as wl

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration(torch, dev)
        return
    if args.workload == "ensemble":
        print(json.dumps(bench_ensemble(args, torch, pd, wl, dev)))
        return
    if args.workload == "serve":
        srv = bench_serve(args, torch, pd, wl, dev, args.count or args.serve_count,
                          args.serve_rate)
        if not args.no_cpu_baseline:
            serve_errors(srv, wl)
        srv.pop("_samples", None)
        print(json.dumps(srv))
        return
    if args.workload == "alpha":
        print(json.dumps(bench_alpha(args, torch, pd, wl, dev)))
        return
    if args.workload == "fom":
        print(json.dumps(bench_fom(args, torch, pd, wl, dev)))
        return
    if args.workload == "bdf":
        print(json.dumps(bench_bdf(args, torch, pd, wl, dev)))
        return
    if args.workload == "fd2d":
        # the 2D rows alone (the forms of --forms among fp64 and mixed), e.g.
        # for a kernel trace of one form
        rows = bench_2d(args, torch, pd, wl, dev, forms_sel=args.forms.split(","))
        for r in rows["forms"].values():
            r.pop("_sample", None)
        print(json.dumps(rows))
        return
    stream = torch.cuda.current_stream(dev)
    prob = wl.cfg_fem_1d()
    nbar, ell = prob.nbar, prob.ell
    unknowns = nbar * ell
    u0 = torch.tensor(prob.u0, device=dev)
    F = torch.tensor(prob.F, device=dev)
    tol = 1e-8
    forms = {}
    kernels = {}
    results_U = {}
    for form in args.forms.split(","):
        prec = {"fp64": pd.PD_FP64, "mixed": pd.PD_MIXED, "fp32": pd.PD_FP32,
                "alpha": pd.PD_FP64, "sine": pd.PD_FP64}[form]
        extra = dict(alpha=args.alpha, early_exit=1) if form == "alpha" else {}
        if form == "sine":
            extra = dict(shifted_solver=pd.PD_SHIFTED_SINE)
        plan = pd.paradiag_plan_create(prob.n, ell, prob.tau, prob.M, prob.K, precision=prec,
                                       stream=stream.cuda_stream, **extra)
        try:
            U = torch.empty((ell, nbar), dtype=torch.float64, device=dev)
            for _ in range(args.warmup):
                pd.paradiag_solve(plan, u0, F, U, tol, allow_notconv=True)
            torch.cuda.synchronize()
            lat = []
            infos = []
            t0 = time.perf_counter()
            for _ in range(args.steps):
                a = time.perf_counter()
                infos.append(pd.paradiag_solve(plan, u0, F, U, tol, allow_notconv=True))
                lat.append(time.perf_counter() - a)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            res = pd.paradiag_residual(plan, u0, F, U)
            info = infos[-1]
            forms[form] = {
                "unknowns_per_s": unknowns * args.steps / wall,
                "ms_per_step": 1e3 * wall / args.steps,
                "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                               "p99": 1e3 * float(np.percentile(lat, 99))},
                "rel_residual": res,
                "gmres_iters": info.gmres_iters, "sweeps": info.sweeps,
                "pint_loops": info.pint_loops,
            }
            if form == "alpha":
                forms[form].update(alpha=args.alpha, early_exit=info.early_exit)
            if form == "sine":
                forms[form]["dst_rows_ms"] = time_sine_transform(torch, pd, plan, U, stream,
                                                                 args.kernel_reps)
            results_U[form] = U.cpu().numpy()
            if form not in ("alpha", "sine"):
                kernels[form] = time_stages(pd, plan, prob, u0, F, U, stream,
                                            args.kernel_reps, prec)
        finally:
            pd.paradiag_plan_destroy(plan)

    rows2d = None
    if not args.no_2d:
        rows2d = bench_2d(args, torch, pd, wl, dev)
    serving = None
    if args.serve_count > 0:
        serving = bench_serve(args, torch, pd, wl, dev, args.serve_count, args.serve_rate)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_leg(prob, results_U, forms, args.cpu_seconds)
        if rows2d is not None:
            errors_2d(rows2d, wl)
        if serving is not None:
            serve_errors(serving, wl)
    if serving is not None:
        serving.pop("_samples", None)
    if rows2d is not None:
        for r in rows2d["forms"].values():
            r.pop("_sample", None)

    # the headline is Algorithm 1 with partition/PCR shifted solves (float64
    # or mixed precision); the alpha form (Algorithm 3, a different accuracy
    # trade-off) and the sine-basis form (uniform grids only) are reported
    # beside it
    alg1 = [f for f in forms if f not in ("alpha", "sine")] or list(kernels) or list(forms)
    ok = [f for f in alg1 if forms[f].get("rel_err_vs_exact", 0.0) <= 1e-8]
    best = max(ok or alg1, key=lambda f: forms[f]["unknowns_per_s"])
    roof = None
    if best in kernels:
        k = kernels[best]
        # the capacitance product runs once per GMRES iteration
        k["stages"]["capacitance_apply"]["per_solve"] = forms[best]["gmres_iters"] * \
            max(1, forms[best]["sweeps"])
        dom = max(k["stages"], key=lambda s: k["stages"][s]["ms"] * k["stages"][s]["per_solve"])
        roof = roofline(k["stages"][dom], dom, best)
    # whole-solve algorithmic HBM traffic: 56 B per space-time unknown per
    # float64 sweep (pass A 8 + 8, pass B 8, pass C 8 + 8, pass D 8 + 8)
    solve_bytes = 56.0 * unknowns * max(1, forms[best]["sweeps"]) if best == "fp64" else None
    solve_hbm = None
    if solve_bytes is not None:
        gbs = solve_bytes / (forms[best]["ms_per_step"] * 1e-3) / 1e9
        solve_hbm = {"algorithmic_bytes_per_step": solve_bytes, "achieved": gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    line = {
        "metric": METRIC,
        "value": forms[best]["unknowns_per_s"],
        "unit": "space-time unknowns/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": forms[best]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if best == "fp64" else "c64+f64",
        "data": "synthetic",
        "config": {"workload": "heat1d-fem n=8191 ell=2048 T=1 nu=1 (16-mode source)",
                   "form": best, "tol": tol, "unknowns": unknowns},
        # the metric's latency half: the serving stream at a fixed arrival
        # rate (completion - arrival per request); the headline solve's own
        # back-to-back latencies are under forms
        "latency_ms": serving["latency_ms"] if serving else None,
        "forms": forms,
        "stages": kernels,
        "roofline": roof,
        "solve_hbm": solve_hbm,
        "workload_2d": rows2d,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def time_sine_transform(torch, pd, plan, U, stream, reps):
    """Average duration of one DST-I pass over all time rows (HIP events on
    the plan's stream)."""
    scratch = torch.empty_like(U)
    pd.paradiag_sine_transform(plan, U, scratch)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        pd.paradiag_sine_transform(plan, U, scratch)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def roofline(st, name, form):
    """Roofline entry of the dominant stage: HBM-bound stages against 8 TB/s,
    arithmetic-bound ones (intensity above the machine balance) against the
    FP64 vector peak.  `traffic` is the measured HBM bytes per launch of the
    stage's main kernel from the committed counter summary, or None when the
    kernel sources have changed since it was taken."""
    sec = st["ms"] * 1e-3
    balance = FP64_VEC_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if st["flops"] / st["bytes"] > balance:
        ach = st["flops"] / sec / 1e12
        out = {"kernel": name, "bound": "alu", "achieved": ach, "peak": FP64_VEC_PEAK_TFLOPS,
               "unit": "TFLOP/s", "frac": ach / FP64_VEC_PEAK_TFLOPS}
    else:
        ach = st["bytes"] / sec / 1e9
        out = {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}
    out["algorithmic_bytes"] = st["bytes"]
    out["algorithmic_flops"] = st["flops"]
    out["traffic"] = measured_traffic(name) if form == "fp64" else None
    return out


def measured_traffic(stage):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, copy-calibrated) of
    the stage's main kernel, if the committed summary matches the sources."""
    from paper_2304_12597_amd import build
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    rec = {}
    for ln in lines:
        parts = ln.split()
        if len(parts) >= 2 and parts[0] == "source_sha256:":
            rec["sha"] = parts[1]
        if len(parts) >= 4 and parts[0] == "stage" and parts[2] == "bytes_per_launch":
            rec[parts[1]] = float(parts[3])
    if rec.get("sha") != build.source_hash() or stage not in rec:
        return None
    return rec[stage]


def time_stages(pd, plan, prob, u0, F, U, stream, reps, prec):
    """Average duration of each stage, measured with HIP events recorded on
    the plan's stream, and its algorithmic HBM bytes per launch."""
    import torch
    nbar, ell = prob.nbar, prob.ell
    F2 = ell // 2 + 1
    cb = 16 if prec == pd.PD_FP64 else 8
    nb = pd.paradiag_spectrum_bytes(plan)
    spec = torch.empty(nb // 8, dtype=torch.float64, device=U.device)
    spec2 = torch.empty_like(spec)
    b = torch.empty(nbar, dtype=torch.float64, device=U.device)
    x = torch.empty_like(b)
    Jv = torch.empty_like(b)
    pd.paradiag_forward_transform(plan, u0, F, spec)
    pd.paradiag_shifted_solve(plan, spec, None, None, b)
    pd.paradiag_capacitance_solve(plan, b, x, 1e-9, allow_notconv=True)
    # algorithmic work per launch.  Bytes: each array read or written once.
    # Flops of a parfor of shifted solves: a Thomas-equivalent complex
    # tridiagonal solve costs about 20 real flops per real space-time unknown
    # (the half spectrum's ell/2 + 1 complex systems of nbar rows hold
    # nbar * ell real unknowns); the transforms' 2.5 log2(ell) per unknown
    # (they are HBM-bound by a wide margin).
    lg = float(np.log2(ell))
    stages = {
        "forward_transform": (lambda: pd.paradiag_forward_transform(plan, u0, F, spec2),
                              8 * nbar * ell + 8 * nbar + cb * F2 * nbar,
                              2.5 * nbar * ell * lg, 1),
        "shifted_solve_b": (lambda: pd.paradiag_shifted_solve(plan, spec, None, None, b),
                            cb * F2 * nbar + 8 * nbar, FLOPS_PER_UNKNOWN * nbar * ell, 1),
        "capacitance_apply": (lambda: pd.paradiag_capacitance_apply(plan, x, Jv),
                              16 * nbar, FLOPS_PER_UNKNOWN * nbar * ell, 0),
        "shifted_solve_y": (lambda: pd.paradiag_shifted_solve(plan, spec, x, spec2, None),
                            2 * cb * F2 * nbar + 8 * nbar, FLOPS_PER_UNKNOWN * nbar * ell, 1),
        "inverse_transform": (lambda: pd.paradiag_inverse_transform(plan, spec2, U),
                              cb * F2 * nbar + 8 * nbar * ell, 2.5 * nbar * ell * lg, 1),
    }
    out = {}
    for name, (fn, nbytes, flops, per) in stages.items():
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": ms, "bytes": nbytes, "flops": flops, "per_solve": per,
                     "GBps": nbytes / (ms * 1e-3) / 1e9,
                     "TFLOPs": flops / (ms * 1e-3) / 1e12}
    return {"stages": out}


def cpu_baseline_leg(prob, results_U, forms, seconds):
    """Oracle leg: time the CPU stepping oracle on the host, and measure the
    GPU results' error against the exact modal solution at sampled points."""
    from oracle import allatonce, modal
    rng = np.random.default_rng(123)
    tt = rng.integers(0, prob.ell, 20000)
    ii = rng.integers(0, prob.nbar, 20000)
    ref = modal.modal_sample(prob, tt, ii)
    for f, U in results_U.items():
        forms[f]["rel_err_vs_exact"] = float(np.linalg.norm(U[tt, ii] - ref)
                                             / np.linalg.norm(ref))
    reps = 0
    t0 = time.perf_counter()
    while True:
        Us = allatonce.step(prob)
        reps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    err = float(np.linalg.norm(Us[tt, ii] - ref) / np.linalg.norm(ref))
    return {"value": prob.unknowns * reps / el, "unit": "space-time unknowns/s", "cores": 1,
            "kind": "oracle",
            "sample": "sequential backward-Euler stepping (C, Thomas, 1 thread) of the full "
                      "n=8191 ell=2048 problem, repeated %d times (%.1f s)" % (reps, el),
            "oracle_rel_err_vs_exact": err}


def copy_calibration(torch, dev, gib=1, reps=5):
    """A plain device copy of known size: its FETCH_SIZE / WRITE_SIZE counter
    readings convert the counters of the ParaDiag kernels to bytes."""
    n = gib * (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "reps": reps}))


def bench_ensemble(args, torch, pd, wl, dev):
    """Independent 1D FD heat problems solved in one batched submission."""
    count = args.count or 512
    probs = wl.ensemble(count=count)
    stream = torch.cuda.current_stream(dev)
    prec = {"fp64": pd.PD_FP64, "mixed": pd.PD_MIXED, "fp32": pd.PD_FP32}[args.ensemble_precision]
    plans, u0s, Fs, Us = [], [], [], []
    try:
        for idx, p in enumerate(probs):
            if idx % 64 == 0:
                print("ensemble: creating plan %d/%d" % (idx, count), file=sys.stderr, flush=True)
            plans.append(pd.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K, precision=prec,
                                                 autotune=int(args.ensemble_autotune),
                                                 stream=stream.cuda_stream))
            u0s.append(torch.tensor(p.u0, device=dev))
            Fs.append(torch.tensor(p.F, device=dev))
            Us.append(torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev))
        unknowns = sum(p.unknowns for p in probs)
        for _ in range(args.warmup):
            pd.paradiag_solve_batch(plans, u0s, Fs, Us, 1e-8, allow_notconv=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            infos = pd.paradiag_solve_batch(plans, u0s, Fs, Us, 1e-8, allow_notconv=True)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        its = [i.gmres_iters for i in infos]
        print("ensemble: batched %.3f ms per submission" % (1e3 * wall), file=sys.stderr,
              flush=True)
        # the same problems solved one after another, for comparison
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for pl, u0, F, U in zip(plans, u0s, Fs, Us):
            pd.paradiag_solve(pl, u0, F, U, 1e-8, allow_notconv=True)
        torch.cuda.synchronize()
        seq = time.perf_counter() - t1
        out = {"metric": "space-time unknowns/s (batched ensemble)",
               "value": unknowns / wall, "unit": "space-time unknowns/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall,
               "higher_is_better": True,
               "dtype": {"fp64": "f64", "mixed": "c64+f64", "fp32": "f32"}[args.ensemble_precision],
               "data": "synthetic",
               "config": {"workload": "ensemble of %d 1D FD heat problems, n in [255,4095], "
                                      "ell in {64..1024}, nu log-uniform [1e-3,1]" % count,
                          "unknowns": unknowns, "precision": args.ensemble_precision,
                          "autotune": bool(args.ensemble_autotune)},
               "sweeps": {"min": min(i.sweeps for i in infos), "max": max(i.sweeps for i in infos)},
               "gmres_iters": {"min": min(its), "max": max(its), "mean": float(np.mean(its))},
               "one_by_one": {"ms": 1e3 * seq, "unknowns_per_s": unknowns / seq}}
        if not args.no_cpu_baseline:
            from oracle import modal
            errs = []
            rng = np.random.default_rng(0)
            for p, U in list(zip(probs, Us))[:: max(1, count // 32)]:
                tt = rng.integers(0, p.ell, 2000)
                ii = rng.integers(0, p.nbar, 2000)
                ref = modal.modal_sample(p, tt, ii)
                Uh = U.cpu().numpy()
                errs.append(float(np.linalg.norm(Uh[tt, ii] - ref) / np.linalg.norm(ref)))
            out["rel_err_vs_exact_max_sampled"] = max(errs)
        return out
    finally:
        for pl in plans:
            pd.paradiag_plan_destroy(pl)


def bench_alpha(args, torch, pd, wl, dev):
    """Algorithm 3 (alpha-circulant, with the early-exit test) against
    Algorithm 1 on an ill-conditioned 1D FD problem (nu = 1e-3, n = 4095,
    ell = 1024): capacitance iterations, time and error for a range of alpha."""
    p = wl.heat_1d("fd1", 4095, 1024, 1.0, 1e-3, np.random.default_rng(17), True)
    stream = torch.cuda.current_stream(dev)
    u0 = torch.tensor(p.u0, device=dev)
    F = torch.tensor(p.F, device=dev)
    U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev)
    tol = 1e-8
    rows, Us = [], {}
    # the alpha sweep at tol = 1e-8 (no early exit), then the early-exit test
    # at a looser tolerance, where it accepts U_1
    cases = [(a, 0, tol) for a in (1.0, 1e-1, 1e-2, 1e-3, 1e-4)] + [(1e-4, 1, 1e-5)]
    for ci, (alpha, exit_, ctol) in enumerate(cases):
        plan = pd.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K, alpha=alpha,
                                       early_exit=exit_, stream=stream.cuda_stream)
        try:
            for _ in range(args.warmup):
                pd.paradiag_solve(plan, u0, F, U, ctol, allow_notconv=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                info = pd.paradiag_solve(plan, u0, F, U, ctol, allow_notconv=True)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / args.steps
            rows.append({"alpha": alpha, "tol": ctol, "early_exit_test": exit_,
                         "ms": 1e3 * wall, "gmres_iters": info.gmres_iters,
                         "pint_loops": info.pint_loops, "early_exit": info.early_exit,
                         "rel_residual": pd.paradiag_residual(plan, u0, F, U)})
            Us[ci] = U.cpu().numpy()
        finally:
            pd.paradiag_plan_destroy(plan)
    out = {"metric": "space-time unknowns/s (alpha-circulant ParaDiag, early exit)",
           "value": p.unknowns / (1e-3 * rows[0]["ms"]), "unit": "space-time unknowns/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": rows[0]["ms"], "higher_is_better": True, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "heat1d-fd n=4095 ell=1024 T=1 nu=1e-3 (16-mode source), "
                                  "value at alpha = 1", "tol": tol, "unknowns": p.unknowns},
           "alphas": rows}
    if not args.no_cpu_baseline:
        from oracle import modal
        rng = np.random.default_rng(0)
        tt = rng.integers(0, p.ell, 20000)
        ii = rng.integers(0, p.nbar, 20000)
        ref = modal.modal_sample(p, tt, ii)
        for ci, r in enumerate(rows):
            Uh = Us[ci]
            r["rel_err_vs_exact"] = float(np.linalg.norm(Uh[tt, ii] - ref) / np.linalg.norm(ref))
    return out


def bench_fom(args, torch, pd, wl, dev):
    """The capacitance system by GMRES and by Algorithm 2 (FOM-like
    projection on K_m(K, b), residual every q steps) on three 1D FEM/FD heat
    problems: one where J_ell is close to I, one needing many steps, and the
    stiff headline problem (n = 8191, ell = 2048)."""
    cases = [("fem1", 4095, 16, 10.0), ("fd1", 127, 16, 4.0), ("fem1", 8191, 2048, 1.0)]
    stream = torch.cuda.current_stream(dev)
    tol = 1e-8
    rows, Us, probs = [], [], []
    for kind, n, ell, T in cases:
        p = wl.heat_1d(kind, n, ell, T, 1.0, np.random.default_rng(n + ell), True)
        u0 = torch.tensor(p.u0, device=dev)
        F = torch.tensor(p.F, device=dev)
        U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev)
        for name, extra in (("gmres", {}), ("fom_q1", dict(krylov=pd.PD_KRYLOV_FOM, fom_q=1)),
                            ("fom_q4", dict(krylov=pd.PD_KRYLOV_FOM, fom_q=4))):
            plan = pd.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K,
                                           stream=stream.cuda_stream, **extra)
            try:
                for _ in range(args.warmup):
                    pd.paradiag_solve(plan, u0, F, U, tol, allow_notconv=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    info = pd.paradiag_solve(plan, u0, F, U, tol, allow_notconv=True)
                torch.cuda.synchronize()
                wall = (time.perf_counter() - t0) / args.steps
                rows.append({"problem": "%s n=%d ell=%d T=%g" % (kind, n, ell, T),
                             "krylov": name, "ms": 1e3 * wall, "steps": info.gmres_iters,
                             "pint_loops": info.pint_loops,
                             "capacitance_rel_residual": info.gmres_rel_residual})
                Us.append(U.cpu().numpy())
                probs.append(p)
            finally:
                pd.paradiag_plan_destroy(plan)
    # the 2D example of Section 6.1 (f = 0, u0 = xy(x-1)(1-y), T = 1), inner
    # tolerance 1e-8 as in the paper (tol 1e-6: the capacitance stopping rule
    # is tol/100), on a 511 x 511 grid and on the grids of Table 1 as printed
    # (256^2, 512^2, 1024^2: the chirp-z DST along x)
    cases61 = [(511, 256), (256, 256), (256, 1024), (512, 512), (1024, 256)]
    for n2, ell2 in cases61:
        rows.extend(section61_rows(pd, torch, wl, stream, dev, args, n2, ell2))
    out = {"metric": "capacitance solver comparison (GMRES vs Algorithm 2)",
           "value": None, "unit": "ms per solve", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": False, "dtype": "f64",
           "data": "synthetic", "config": {"workload": "1D heat, three problems", "tol": tol},
           "rows": rows}
    return finish_fom(out, args, probs, Us)


def section61_rows(pd, torch, wl, stream, dev, args, n2, ell2):
    """GMRES and Algorithm 2 (q = 1) on the Section 6.1 example, n2^2 grid."""
    rows = []
    p2 = wl.heat_2d(n2, ell2, 1.0, 1.0, np.random.default_rng(1))
    xg = np.arange(1, n2 + 1) / (n2 + 1)
    X, Y = np.meshgrid(xg, xg)
    u02 = torch.tensor((X * Y * (X - 1) * (1 - Y)).reshape(-1), device=dev)
    F2d = torch.zeros((ell2, n2 * n2), dtype=torch.float64, device=dev)
    U2d = torch.empty((ell2, n2 * n2), dtype=torch.float64, device=dev)
    for name, extra in (("gmres", {}), ("fom_q1", dict(krylov=pd.PD_KRYLOV_FOM, fom_q=1))):
        plan = pd.paradiag_plan_create(n2, ell2, p2.tau, None, p2.K, dims=2,
                                       stream=stream.cuda_stream, **extra)
        try:
            for _ in range(args.warmup):
                pd.paradiag_solve(plan, u02, F2d, U2d, 1e-6, allow_notconv=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                info = pd.paradiag_solve(plan, u02, F2d, U2d, 1e-6, allow_notconv=True)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / args.steps
            rows.append({"problem": "2D Section 6.1: %d^2 ell=%d T=1 u0=xy(x-1)(1-y) tol=1e-6"
                                    % (n2, ell2),
                         "krylov": name, "ms": 1e3 * wall, "steps": info.gmres_iters,
                         "pint_loops": info.pint_loops,
                         "capacitance_rel_residual": info.gmres_rel_residual,
                         "unknowns_per_s": n2 * n2 * ell2 / wall})
        finally:
            pd.paradiag_plan_destroy(plan)
    del F2d, U2d
    return rows


def finish_fom(out, args, probs, Us):
    """Sampled error of the 1D rows against the exact modal solution."""
    if not args.no_cpu_baseline:
        from oracle import modal
        rng = np.random.default_rng(0)
        for r, U, p in zip(out["rows"], Us, probs):
            tt = rng.integers(0, p.ell, 4000)
            ii = rng.integers(0, p.nbar, 4000)
            ref = modal.modal_sample(p, tt, ii)
            r["rel_err_vs_exact"] = float(np.linalg.norm(U[tt, ii] - ref) / np.linalg.norm(ref))
    return out


def bench_bdf(args, torch, pd, wl, dev):
    """BDF of order s = 1..6 (Section 5) on the n = 8191, ell = 2048 P1-FEM
    workload, every starting value equal to u0: whole solves, the block
    capacitance product alone, and (cpu_baseline leg) the error against the
    per-mode BDF recurrence and the oracle's sequential stepping on a
    bounded number of steps."""
    stream = torch.cuda.current_stream(dev)
    p = wl.cfg_fem_1d()
    tol = 1e-8
    F = torch.tensor(p.F, device=dev)
    U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev)
    rows, Us = [], {}
    for s in range(1, 7):
        u0s = torch.tensor(np.tile(p.u0, (s, 1)), device=dev)
        plan = pd.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K, bdf_order=s,
                                       stream=stream.cuda_stream)
        try:
            for _ in range(args.warmup):
                pd.paradiag_solve(plan, u0s, F, U, tol)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                info = pd.paradiag_solve(plan, u0s, F, U, tol)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / args.steps
            v = torch.randn(s * p.nbar, dtype=torch.float64, device=dev)
            Jv = torch.empty_like(v)
            pd.paradiag_capacitance_apply(plan, v, Jv)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.kernel_reps):
                pd.paradiag_capacitance_apply(plan, v, Jv)
            e1.record(stream)
            torch.cuda.synchronize()
            rows.append({"s": s, "ms": 1e3 * wall, "gmres_iters": info.gmres_iters,
                         "pint_loops": info.pint_loops,
                         "unknowns_per_s": p.nbar * p.ell / wall,
                         "capacitance_product_ms": e0.elapsed_time(e1) / args.kernel_reps,
                         "capacitance_rel_residual": info.gmres_rel_residual})
            Us[s] = U.cpu().numpy()
        finally:
            pd.paradiag_plan_destroy(plan)
    # the block Galerkin method of Section 5 for J^(s) on the same workload
    # (stiff: its polynomial space needs many steps) and on a problem where
    # J^(s) is close to I
    grows = []
    mild = wl.heat_1d("fem1", 4095, 16, 10.0, 1.0, np.random.default_rng(4111), True)
    for prob, name in ((p, "n=8191 ell=2048 T=1"), (mild, "n=4095 ell=16 T=10")):
        Fp = torch.tensor(prob.F, device=dev)
        Up = torch.empty((prob.ell, prob.nbar), dtype=torch.float64, device=dev)
        for s, q in ((2, 1), (2, 4), (3, 4)):
            u0s = torch.tensor(np.tile(prob.u0, (s, 1)), device=dev)
            plan = pd.paradiag_plan_create(prob.n, prob.ell, prob.tau, prob.M, prob.K,
                                           bdf_order=s, krylov=pd.PD_KRYLOV_FOM, fom_q=q,
                                           stream=stream.cuda_stream)
            try:
                for _ in range(args.warmup):
                    pd.paradiag_solve(plan, u0s, Fp, Up, tol, allow_notconv=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    info = pd.paradiag_solve(plan, u0s, Fp, Up, tol, allow_notconv=True)
                torch.cuda.synchronize()
                wall = (time.perf_counter() - t0) / args.steps
                grows.append({"problem": "fem1 " + name, "s": s, "q": q, "ms": 1e3 * wall,
                              "block_steps": info.gmres_iters, "pint_loops": info.pint_loops,
                              "capacitance_rel_residual": info.gmres_rel_residual,
                              "_U": Up.cpu().numpy(), "_p": prob})
            finally:
                pd.paradiag_plan_destroy(plan)
    # 2D: the 511 x 511 FD workload (ell = 256, T = 0.1), GMRES
    rows2d = []
    p2 = wl.cfg_fd_2d()
    F2d = torch.tensor(p2.F, device=dev)
    U2d = torch.empty((p2.ell, p2.nbar), dtype=torch.float64, device=dev)
    for s in (1, 2, 3):
        u0s = torch.tensor(np.tile(p2.u0, (s, 1)), device=dev)
        plan = pd.paradiag_plan_create(p2.n, p2.ell, p2.tau, None, p2.K, dims=2, bdf_order=s,
                                       stream=stream.cuda_stream)
        try:
            for _ in range(args.warmup):
                pd.paradiag_solve(plan, u0s, F2d, U2d, tol)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                info = pd.paradiag_solve(plan, u0s, F2d, U2d, tol)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / args.steps
            rng = np.random.default_rng(s)
            tt = rng.integers(0, p2.ell, 4000)
            ii = rng.integers(0, p2.nbar, 4000)
            samp = U2d[torch.tensor(tt, device=dev), torch.tensor(ii, device=dev)].cpu().numpy()
            rows2d.append({"s": s, "ms": 1e3 * wall, "gmres_iters": info.gmres_iters,
                           "pint_loops": info.pint_loops,
                           "unknowns_per_s": p2.nbar * p2.ell / wall,
                           "_sample": (tt, ii, samp)})
        finally:
            pd.paradiag_plan_destroy(plan)
    out = {"metric": "BDF-s ParaDiag solves (Section 5)", "value": None,
           "unit": "ms per solve", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": False, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "heat1d-fem n=8191 ell=2048 T=1 nu=1 (16-mode source), "
                                  "u_{1-s} = ... = u_0 = u0", "tol": tol},
           "rows": rows, "block_galerkin_rows": grows, "rows_2d": rows2d,
           "config_2d": "heat2d-fd 511x511 ell=256 T=0.1 nu=1, u_{1-s} = ... = u_0 = u0"}
    if not args.no_cpu_baseline:
        from oracle import bdf
        from oracle.spatial import problem_matrices
        Msp, Ksp = problem_matrices(p)
        for r in rows:
            ref = bdf.modal_bdf(p, r["s"])
            r["rel_err_vs_exact"] = float(np.linalg.norm(Us[r["s"]] - ref) / np.linalg.norm(ref))
        for r in grows:
            ref = bdf.modal_bdf(r["_p"], r["s"])
            r["rel_err_vs_exact"] = float(np.linalg.norm(r["_U"] - ref) / np.linalg.norm(ref))
        for r in rows2d:
            tt, ii, samp = r["_sample"]
            ref = bdf.modal_bdf(p2, r["s"], (tt, ii))
            r["rel_err_vs_exact_sampled"] = float(np.linalg.norm(samp - ref) /
                                                  np.linalg.norm(ref))
        steps = 256
        t0 = time.perf_counter()
        Ucpu = bdf.step_bdf(Msp, Ksp, p.tau, 2, [p.u0] * 2, p.F[:steps])
        sec = time.perf_counter() - t0
        assert np.allclose(Ucpu, Us[2][:steps], rtol=0, atol=1e-9 * np.abs(Ucpu).max())
        out["cpu_baseline"] = {"value": p.nbar * steps / sec, "unit": "unknowns/s",
                               "cores": 1, "kind": "oracle",
                               "sample": "BDF2 sequential stepping (sparse LU), first %d of "
                                         "%d steps" % (steps, p.ell)}
    for r in grows:
        del r["_U"], r["_p"]
    for r in rows2d:
        del r["_sample"]
    return out


def bench_2d(args, torch, pd, wl, dev, forms_sel=("fp64", "mixed")):
    """The 2D workload (511 x 511 grid, ell = 256, T = 0.1): float64 and mixed
    forms, inputs resident in HBM, `steps` timed solves each.  Sampled outputs
    are kept for the cpu_baseline leg's error check."""
    stream = torch.cuda.current_stream(dev)
    p = wl.cfg_fd_2d()
    u0 = torch.tensor(p.u0, device=dev)
    F = torch.zeros((p.ell, p.nbar), dtype=torch.float64, device=dev)   # f = 0
    U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev)
    rng = np.random.default_rng(7)
    tt = rng.integers(0, p.ell, 4000)
    ii = rng.integers(0, p.nbar, 4000)
    tix, iix = torch.tensor(tt, device=dev), torch.tensor(ii, device=dev)
    steps = max(1, min(args.steps, 10))
    forms = {}
    for form, prec in (("fp64", pd.PD_FP64), ("mixed", pd.PD_MIXED)):
        if form not in forms_sel:
            continue
        plan = pd.paradiag_plan_create(p.n, p.ell, p.tau, None, p.K, dims=2, precision=prec,
                                       stream=stream.cuda_stream)
        try:
            for _ in range(min(args.warmup, 2) or 1):
                pd.paradiag_solve(plan, u0, F, U, 1e-8, allow_notconv=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                info = pd.paradiag_solve(plan, u0, F, U, 1e-8, allow_notconv=True)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / steps
            forms[form] = {"ms_per_step": 1e3 * wall, "unknowns_per_s": p.unknowns / wall,
                           "gmres_iters": info.gmres_iters, "sweeps": info.sweeps,
                           "pint_loops": info.pint_loops,
                           "rel_residual": pd.paradiag_residual(plan, u0, F, U),
                           "_sample": (tt, ii, U[tix, iix].cpu().numpy())}
        finally:
            pd.paradiag_plan_destroy(plan)
    del F, U
    return {"workload": "heat2d-fd 511x511 ell=256 T=0.1 nu=1 (f = 0)", "steps": steps,
            "unknowns": p.unknowns, "forms": forms}


def errors_2d(rows2d, wl):
    """Oracle leg: sampled error of the 2D rows against the exact modal
    solution."""
    from oracle import modal
    p = wl.cfg_fd_2d()
    for r in rows2d["forms"].values():
        tt, ii, got = r["_sample"]
        ref = modal.modal_sample(p, tt, ii)
        r["rel_err_vs_exact_sampled"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def bench_serve(args, torch, pd, wl, dev, count, rate):
    """The serving stream through the pd_server runtime: `count` mixed
    requests (70% 1D FEM n <= 16383, 30% 2D FD up to 511^2, nu log-uniform,
    mixed precision to 1e-8) arriving by a Poisson process at the fixed rate
    `rate` (requests/s), a 200 GB admission budget and 4 worker streams.  A
    fresh server (empty plan cache) serves the timed stream, so plan creation
    is inside each request's latency.  Each request's status is recorded;
    failed requests are excluded from throughput and latency and counted.
    Sampled outputs are kept for the cpu_baseline leg's error check."""
    import threading
    budget = 200 << 30
    reqs, staged = [], []
    t_stage = time.perf_counter()
    for r in wl.iter_serving_stream(count=count, rate=rate):
        p = r.problem
        u0 = torch.tensor(p.u0, device=dev)
        if p.dims == 2:
            F = torch.zeros((p.ell, p.nbar), dtype=torch.float64, device=dev)   # f = 0
        else:
            F = torch.tensor(p.F, device=dev)
        U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev)
        p.F = np.zeros((0, 0))              # the host copy is no longer needed
        reqs.append(r)
        staged.append((p, u0, F, U))
    torch.cuda.synchronize()
    stage_s = time.perf_counter() - t_stage
    print("serve: staged %d requests in %.1f s" % (count, stage_s), file=sys.stderr, flush=True)

    def submit(srv, item):
        p, u0, F, U = item
        return pd.pd_server_submit(srv, p.n, p.ell, p.tau, p.M, p.K, u0, F, U, 1e-8,
                                   dims=p.dims, precision=pd.PD_MIXED)

    # warm-up: a few requests through a separate server (module loading, the
    # device's first launches), then a fresh server for the timed stream
    srv = pd.pd_server_create(4, budget)
    try:
        for t in [submit(srv, it) for it in staged[:8]]:
            pd.pd_server_wait(srv, t, -1)
    finally:
        pd.pd_server_destroy(srv)
    arrivals = np.array([r.arrival for r in reqs])
    done_at = [0.0] * count
    status = [None] * count
    infos = [None] * count
    tickets = [None] * count
    srv = pd.pd_server_create(4, budget)
    try:
        start = time.perf_counter()

        def waiter():
            # poll every submitted, unfinished ticket, so that each completion
            # is timed when it happens, whatever the completion order
            pending = set(range(count))
            while pending:
                for i in sorted(pending):
                    if tickets[i] is None:
                        continue
                    done, st, info = pd.pd_server_wait(srv, tickets[i], 0)
                    if done:
                        done_at[i] = time.perf_counter() - start
                        status[i] = st
                        infos[i] = info
                        pending.discard(i)
                time.sleep(2e-4)
        th = threading.Thread(target=waiter)
        th.start()
        for i, it in enumerate(staged):
            now = time.perf_counter() - start
            if arrivals[i] > now:
                time.sleep(arrivals[i] - now)
            tickets[i] = submit(srv, it)
        th.join()
        stats = pd.pd_server_stats(srv)
    finally:
        pd.pd_server_destroy(srv)
    ok = [i for i in range(count) if status[i] == pd.PD_OK]
    failed = {}
    for i in range(count):
        if status[i] != pd.PD_OK:
            name = pd.STATUS_NAMES[status[i]]
            failed[name] = failed.get(name, 0) + 1
    lat = np.array([done_at[i] - arrivals[i] for i in ok])
    wall = max(done_at)
    unknowns = sum(staged[i][0].unknowns for i in ok)
    # sampled outputs of every request (for the error check)
    rng = np.random.default_rng(11)
    samples = []
    for i, (p, u0, F, U) in enumerate(staged):
        tt = rng.integers(0, p.ell, 300)
        ii = rng.integers(0, p.nbar, 300)
        got = U[torch.tensor(tt, device=dev), torch.tensor(ii, device=dev)].cpu().numpy()
        samples.append((i, tt, ii, got))
    sweeps = [infos[i].sweeps for i in ok]
    del staged
    return {"metric": "space-time unknowns/s + p50/p99 latency (serving)",
            "value": unknowns / wall, "unit": "space-time unknowns/s",
            "requests": count, "completed_ok": len(ok), "failed": failed,
            "arrival_rate_per_s": rate, "wall_s": wall,
            "requests_per_s": len(ok) / wall,
            "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                           "p99": 1e3 * float(np.percentile(lat, 99)),
                           "max": 1e3 * float(lat.max())},
            "sweeps": {"min": min(sweeps), "max": max(sweeps), "mean": float(np.mean(sweeps))},
            "config": {"workload": "Poisson stream (fixed rate) of %d requests, 70%% 1D FEM "
                                   "n<=16383 / 30%% 2D FD side<=511, nu log-uniform [1e-3,1], "
                                   "mixed precision to 1e-8, 200 GB budget, 4 worker streams, "
                                   "fresh plan cache" % count,
                       "staging_s": stage_s},
            "server": stats, "_samples": (samples, count, rate)}


def serve_errors(srv, wl):
    """Oracle leg: each served request's sampled error against the exact
    modal solution (the stream is regenerated from its seed)."""
    from oracle import modal
    samples, count, rate = srv["_samples"]
    errs = []
    for r, (i, tt, ii, got) in zip(wl.iter_serving_stream(count=count, rate=rate), samples):
        ref = modal.modal_sample(r.problem, tt, ii)
        errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
    srv["rel_err_vs_exact_sampled"] = {"max": max(errs), "median": float(np.median(errs)),
                                       "above_1e-8": int(sum(e > 1e-8 for e in errs))}


if __name__ == "__main__":
    main()
