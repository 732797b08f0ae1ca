#!/usr/bin/env python3
"""Benchmark: material-aware SA-AMG-PCG on one MI355X.

Workload: battery-like layered stack, 3D Q1 on a 128^3 hex mesh
(2,146,689 DOF), elements 10:1 flat (domain [0,10]^2 x [0,1]), 20 repeats of
three isotropic layers with log-uniform conductivities in [1e-5,1e-2],
[1e-10,1e-8], [1e-1,1], u = 0 / 1 on the bottom / top faces, FP64.

One step = the whole hot path on inputs already resident in HBM:
amg_setup (Clement tensors, strength, aggregation, prolongators, Galerkin
products, coarse factorisation) followed by amg_pcg_solve from x0 = 0 to a
true relative residual of 1e-8.  value = DOF * steps / time.  The JSON line
also carries solve-only throughput, the same solve from five seeded starts
(`seeded_x0`), the FP32-hierarchy form against the FP64 form (on this stack,
and on the 96^3 rotated-anisotropy cube, `fp32_form.aniso`), the V-cycle's
algorithmic HBM bandwidth per form, the roofline of the dominant kernel
(the finest level's fused Chebyshev SpMV: back-to-back launches between HIP
events on its stream), the 192^3 stack with 50 repeats (`layered192`: both
forms, 16 levels), the serving stream (256 requests at 20/s, n log-uniform
in [32, 128], layered or anisotropic, FP32-hierarchy form, 8 GiB budget:
p50 / p99 latency and solves/s, over all requests and over the converged
ones) and the CPU oracle's full setup and solve of the same workload,
measured on one host core, whose solution the GPU results are compared with.
"""

import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def measured_traffic():
    """Per-launch HBM bytes of the finest-level smoother from the committed
    counter passes, while the kernel's sources are the ones measured; None
    once they have changed."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "fine_smoother_layered128_traffic.md")
    try:
        kv = {}
        for line in open(path):
            if "=" in line and line.strip().split("=")[0].strip() in (
                    "traffic_bytes_per_launch", "kernel_sources", "kernel_sources_sha256"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        h = hashlib.sha256()
        for f in kv["kernel_sources"].split():
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != kv["kernel_sources_sha256"]:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(prob):
    """The oracle as it stands, single-threaded, on the same workload: its full
    setup and its PCG solve from x0 = 0 to a relative residual of 1e-8, both
    measured.  Returns the baseline record and the oracle's solution."""
    import oracle

    t0 = time.perf_counter()
    h = oracle.Hierarchy(prob)
    t1 = time.perf_counter()
    x, info = h.pcg(prob.b)
    t2 = time.perf_counter()
    rec = dict(value=prob.n / (t2 - t0), unit="DOF/s", cores=1, kind="oracle",
               sample=(f"the whole workload ({prob.n} DOF), measured: oracle setup {t1 - t0:.1f} s + PCG from x0 = 0, "
                       f"{info['iterations']} iterations to rel-res 1e-8 ({t2 - t1:.1f} s)"),
               t_setup_s=t1 - t0, t_solve_s=t2 - t1, iterations=info["iterations"], status=info["status"],
               rel_res=info["rel_res"], solve_only_dof_per_s=prob.n / (t2 - t1),
               host_cpu=cpu_model(), host_threads=os.cpu_count())
    return rec, x


def time_vcycles(h, n, reps, dev):
    """Mean duration (ms) of `reps` back-to-back V-cycles between HIP events on
    torch's current stream (the stream the V-cycle launches on)."""
    import torch

    r = torch.randn(n, dtype=torch.float64, device=dev)
    z = torch.zeros_like(r)
    for _ in range(3):
        h.vcycle(r, z)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        h.vcycle(r, z)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def achievable_bandwidth(dev, nbytes=1 << 30, reps=20):
    """What plain streaming reaches on this GPU: a read (sum), a device copy
    (read + write) and a fill of nbytes, each the mean of reps launches
    between HIP events on torch's current stream, in GB/s of bytes moved."""
    import torch

    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    out = {}
    for name, fn, moved in (("read", lambda: src.sum(), nbytes), ("copy", lambda: dst.copy_(src), 2 * nbytes),
                            ("fill", lambda: dst.fill_(2.0), nbytes)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        out[f"{name}_GBps"] = moved / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return out


def vcycle_record(h, n, reps, dev):
    st = h.stats()
    ms = time_vcycles(h, n, reps, dev)
    gbs = st["vcycle_alg_bytes"] / (ms * 1e-3) / 1e9
    kt = h.time_smoother(level=0, reps=reps)
    return {"ms": ms, "alg_bytes": st["vcycle_alg_bytes"], "alg_GBps": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS,
            "fine_smoother_us": kt["avg_ms"] * 1e3,
            "fine_smoother_GBps": kt["bytes_per_launch"] / (kt["avg_ms"] * 1e-3) / 1e9}


def layered_exact(prob):
    """Exact discrete solution of a layered stack (f = 0, z-only series resistor)."""
    kz = prob.meta["layer_k"]
    res = 1.0 / kz
    cf = np.concatenate([[0.0], np.cumsum(res)]) / res.sum()
    return cf[np.rint(prob.coords[:, 2] * prob.shape[2]).astype(int)]


def run_layered192(args, amg, dev, log):
    """The 192^3 layered stack (7,189,057 DOF, 50 repeats of three layers over
    192 elements, 20:1 flat), which needs 16 levels: per precision form, setup
    and PCG from x0 = 0 to 1e-8 timed `c4_reps` times, the V-cycle and the
    finest smoother step timed, errors against the exact discrete solution
    and between the forms."""
    import torch

    from workloads import layered_stack_3d

    log("generating layered stack 192^3, 50 repeats, 20:1")
    prob = layered_stack_3d(n=192, repeats=50, stretch=20.0, config_id=4)
    n = prob.n
    d = [torch.from_numpy(a).to(dev) for a in (prob.rowptr, prob.col, prob.val, prob.elem_nodes, prob.elem_sigma,
                                                prob.coords)]
    b = torch.from_numpy(prob.b).to(dev)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    exact = layered_exact(prob)
    out = dict(workload="layered stack 192^3 hex Q1 (7189057 DOF), 50 repeats x 3 layers, 20:1 flat, 16 levels",
               n=n, nnz=prob.nnz)
    sol = {}
    for name in ("fp64", "fp32"):
        opts = amg.options(dim=3, precision=name, max_levels=16)
        steps, setups, solves = [], [], []
        for k in range(max(1, args.c4_reps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = amg.Hierarchy(*d, opts)
            x.zero_()
            _, info = h.solve(b, x, max_iter=args.c4_max_iter, raise_on_error=False)
            torch.cuda.synchronize()
            steps.append(1e3 * (time.perf_counter() - t0))
            setups.append(1e3 * h.stats()["t_setup_s"])
            solves.append(1e3 * info["t_solve_s"])
            if k + 1 < max(1, args.c4_reps):
                h.close()
        sol[name] = x.cpu().numpy()
        st = h.stats()
        vc = vcycle_record(h, n, args.vcycles // 5 or 1, dev)
        h.close()
        step_ms = float(np.median(steps))
        out[name] = dict(status=info["status"], iterations=info["iterations"], rel_res=info["rel_res"],
                         levels=st["n"], op_complexity=st["op_complexity"],
                         t_setup_ms_stats=stats_ms(setups), t_solve_ms_stats=stats_ms(solves),
                         step_ms_stats=stats_ms(steps), dof_per_s=n / (step_ms * 1e-3),
                         solve_only_dof_per_s=n / (float(np.median(solves)) * 1e-3), vcycle=vc,
                         rel_err_vs_closed_form=float(np.linalg.norm(sol[name] - exact) / np.linalg.norm(exact)))
        log(f"192^3 {name}: {info['iterations']} it ({info['status']}), setup {np.median(setups):.0f} ms, solve "
            f"{np.median(solves):.0f} ms, V-cycle {vc['ms']:.3f} ms = {vc['frac_of_peak']:.1%} of peak")
    out["speedup_fp32_vs_fp64_solve"] = (out["fp64"]["t_solve_ms_stats"]["median"] /
                                         out["fp32"]["t_solve_ms_stats"]["median"])
    out["speedup_fp32_vs_fp64_vcycle"] = out["fp64"]["vcycle"]["ms"] / out["fp32"]["vcycle"]["ms"]
    out["rel_err_fp32_vs_fp64_form"] = float(np.linalg.norm(sol["fp32"] - sol["fp64"]) / np.linalg.norm(sol["fp64"]))
    return out


def run_serving(args, amg, log):
    """Serving stream: Poisson arrivals at `rate`/s of `num` requests, mesh n^3
    with n log-uniform in [32, 128], layered (20 repeats, 10:1) or rotated
    anisotropic, per-request seeds, FP32-hierarchy form, tol 1e-8, admitted
    under an HBM budget.  The requests are generated before the replay; each
    is submitted at its arrival time and latency is t_done - t_arrival as the
    server clocks them."""
    import threading
    from concurrent.futures import ThreadPoolExecutor

    from workloads import problem_from_request, serving_stream

    reqs = serving_stream(num=args.serve_num, rate=args.serve_rate)
    log(f"serving: generating {len(reqs)} requests")
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        probs = list(ex.map(problem_from_request, reqs))
    t_gen = time.perf_counter() - t0
    dofs = [p.n for p in probs]
    log(f"serving: generated in {t_gen:.1f}s, {sum(dofs)} DOF in total")
    # requests re-solved alone afterwards: the smallest of each kind
    check_ids = []
    for kind in ("layered", "aniso"):
        ks = [i for i, r in enumerate(reqs) if r["kind"] == kind]
        if ks:
            check_ids.append(min(ks, key=lambda i: reqs[i]["n"]))
    keep = {i: probs[i] for i in check_ids}
    srv = amg.Server(budget_bytes=int(args.serve_budget_gib * (1 << 30)), max_active=args.serve_active,
                     setup_workers=2, precision="fp32")
    # warm-up request (loads the code objects), outside the replay
    w = srv.submit(probs[check_ids[0]], max_iter=args.serve_max_iter)
    while not srv.poll(timeout_s=5.0):
        pass
    srv.result(w)
    results = {}
    done = threading.Event()
    id_of = {}

    def collect():
        while len(results) < len(probs):
            for rid in srv.poll(timeout_s=1.0):
                x, info, tl = srv.result(rid)
                i = id_of[rid]
                results[i] = (x if i in keep else None, info, tl)
                if len(results) % 32 == 0:
                    log(f"serving: {len(results)} of {len(probs)} done")
        done.set()

    th = threading.Thread(target=collect, daemon=True)
    log("serving: replaying the arrival stream")
    lateness = []
    t_start = time.perf_counter()
    th.start()
    for i, r in enumerate(reqs):
        wait = t_start + r["t_arrival"] - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        lateness.append(time.perf_counter() - t_start - r["t_arrival"])
        rid = srv.submit(probs[i], max_iter=args.serve_max_iter)
        id_of[rid] = i
        probs[i] = None  # the server holds its own copy
    done.wait()
    t_wall = time.perf_counter() - t_start
    st = srv.stats()
    srv.close()
    lat = np.array([results[i][2]["t_done"] - results[i][2]["t_arrival"] for i in range(len(reqs))])
    t_first = min(results[i][2]["t_arrival"] for i in range(len(reqs)))
    t_last = max(results[i][2]["t_done"] for i in range(len(reqs)))
    iters = np.array([results[i][1]["iterations"] for i in range(len(reqs))])
    status = {}
    for i in range(len(reqs)):
        s = results[i][1]["status"]
        status[s] = status.get(s, 0) + 1
    conv = [i for i in range(len(reqs)) if results[i][1]["status"] == "OK"]
    # the same requests alone: the one-hierarchy solver, same options
    alone = []
    for i in check_ids:
        p = keep[i]
        h = amg.Hierarchy.from_problem(p, precision="fp32")
        xa, ia = h.solve(p.b, max_iter=args.serve_max_iter, raise_on_error=False)
        h.close()
        xm = results[i][0]
        alone.append(dict(request=i, n=p.n, kind=reqs[i]["kind"], bitwise_equal=bool(np.array_equal(xa, xm)),
                          iterations_mix=results[i][1]["iterations"], iterations_alone=ia["iterations"],
                          shared_rounds_with=results[i][2]["max_batch"] - 1))
    makespan = t_last - t_first
    converged_only = None
    if conv:
        lc = lat[conv]
        converged_only = {"requests": len(conv), "solves_per_s": len(conv) / makespan,
                          "served_dof_per_s": sum(dofs[i] for i in conv) / makespan,
                          "p50_latency_s": float(np.percentile(lc, 50)), "p99_latency_s": float(np.percentile(lc, 99)),
                          "mean_latency_s": float(lc.mean())}
    # where the latency goes: waiting for admission, setup, solve (rounds)
    tl = [results[i][2] for i in range(len(reqs))]
    phases = {}
    for name, a, b in (("admission_wait", "t_arrival", "t_admit"), ("setup", "t_admit", "t_setup_done"),
                       ("solve", "t_setup_done", "t_done")):
        v = np.array([t[b] - t[a] for t in tl])
        phases[name] = {"mean_s": float(v.mean()), "p50_s": float(np.percentile(v, 50)),
                        "p99_s": float(np.percentile(v, 99))}
    out = {
        "requests": len(reqs), "rate_per_s": args.serve_rate, "budget_GiB": args.serve_budget_gib,
        "max_active": args.serve_active, "precision": "fp32-hierarchy", "tol": 1e-8, "max_iter": args.serve_max_iter,
        "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()), "max_latency_s": float(lat.max()),
        "solves_per_s": len(reqs) / makespan, "makespan_s": makespan, "served_dof_per_s": sum(dofs) / makespan,
        "status_counts": status, "converged": len(conv),
        "not_converged_requests": sorted(i for i in range(len(reqs)) if results[i][1]["status"] == "NOT_CONVERGED"),
        # the same figures over the requests that reached the tolerance only
        "converged_only": converged_only,
        "iterations": {"median": float(np.median(iters)), "p90": float(np.percentile(iters, 90)),
                       "max": int(iters.max())},
        "mean_batch": st["mean_batch"], "max_batch": st["max_batch"], "rounds": st["steps"],
        "launches": st["launches"], "peak_reserved_GiB": st["peak_reserved_bytes"] / 2**30,
        "estimate_exceeded": st["estimate_exceeded"], "failed": st["failed"],
        "submit_lateness_max_s": float(max(lateness)), "generation_s": t_gen, "replay_wall_s": t_wall,
        "latency_phases": phases,
        "alone_vs_mix": alone,
    }
    log(f"serving: p50 {out['p50_latency_s']:.2f}s p99 {out['p99_latency_s']:.2f}s, "
        f"{out['solves_per_s']:.2f} solves/s, statuses {status}, mean batch {st['mean_batch']:.1f}")
    if converged_only:
        log(f"serving, converged only: {converged_only['solves_per_s']:.2f} solves/s, p50 "
            f"{converged_only['p50_latency_s']:.2f}s p99 {converged_only['p99_latency_s']:.2f}s")
    return out


def run_compare(amg, log):
    """The paper's central comparison (material vs classical SA vs Euclidean
    distance measure, pointwise vs cut-drop) on the synthetic workloads:
    levels, operator complexity C, PCG iterations to 1e-8 and cost C x iters."""
    from workloads import (config1_checkerboard_2d, layered_stack_3d, rotated_anisotropic_3d, two_domain_2d)

    cases = [
        ("checkerboard 64^2, K in {1, 1e6}", lambda: config1_checkerboard_2d(), dict(max_coarse=100)),
        ("two-domain h=1/128 kappa=1e2", lambda: two_domain_2d(n=128, kappa=1e2), dict()),
        ("two-domain h=1/128 kappa=1e4", lambda: two_domain_2d(n=128, kappa=1e4), dict()),
        ("two-domain h=1/512 kappa=1e4", lambda: two_domain_2d(n=512, kappa=1e4), dict()),
        ("rotated anisotropy 48^3", lambda: rotated_anisotropic_3d(n=48, block=8), dict()),
        ("layered stack 64^3, 10 repeats", lambda: layered_stack_3d(n=64, repeats=10), dict()),
    ]
    rows = []
    for name, fn, kw in cases:
        prob = fn()
        for soc in ("material", "distance", "sa"):
            for drop in ("pointwise", "cut"):
                rec = dict(workload=name, dof=prob.n, soc=soc, drop=drop, theta=0.08)
                try:
                    h = amg.Hierarchy.from_problem(prob, soc=soc, drop=drop, **kw)
                except amg.AmgError as e:
                    rec.update(status=e.status)
                    rows.append(rec)
                    continue
                st = h.stats()
                x, info = h.solve(prob.b, max_iter=1000, raise_on_error=False)
                h.close()
                rec.update(status=info["status"], levels=st["levels"], op_complexity=st["op_complexity"],
                           iterations=info["iterations"], cost=st["op_complexity"] * info["iterations"],
                           t_setup_ms=1e3 * st["t_setup_s"], t_solve_ms=1e3 * info["t_solve_s"])
                rows.append(rec)
                log(f"compare: {name} {soc}/{drop}: C={st['op_complexity']:.2f} iters={info['iterations']} "
                    f"{info['status']}")
    return {"metric": "strength-of-connection comparison", "rows": rows}


SWEEP_THETAS = (0.0, 0.0025, 0.005, 0.01, 0.02, 0.04, 0.08, 0.16, 0.32, 0.64)
MODES = (("material", "pointwise"), ("material", "cut"), ("distance", "pointwise"), ("distance", "cut"),
         ("sa", "pointwise"), ("sa", "cut"))


def _solve_record(amg, prob, rec, max_iter, **kw):
    """setup + FP64 PCG to 1e-8 from zero; fills levels, C, iterations, cost, times"""
    try:
        h = amg.Hierarchy.from_problem(prob, **kw)
    except amg.AmgError as e:
        rec.update(status=e.status)
        return rec
    st = h.stats()
    _, info = h.solve(prob.b, max_iter=max_iter, raise_on_error=False)
    h.close()
    rec.update(status=info["status"], levels=st["levels"], op_complexity=st["op_complexity"],
               iterations=info["iterations"], cost=st["op_complexity"] * info["iterations"],
               t_setup_ms=1e3 * st["t_setup_s"], t_solve_ms=1e3 * info["t_solve_s"])
    return rec


def run_sweep(args, amg, log):
    """The two-domain study (section "Two domain problem", Figs. 6-7): PCG
    iterations and cost C x iterations over the drop tolerance for every
    strength measure x dropping criterion, h in {1/32, 1/128, 1/512} (h = 1 /
    elements per direction), kappa in {1, 1e2, 1e4}, coarsening down to at
    most 50 unknowns so that even the 33 x 33 node mesh has several levels."""
    from workloads import two_domain_2d

    rows = []
    for n in args.sweep_n:
        for kappa in (1.0, 1e2, 1e4):
            prob = two_domain_2d(n=n, kappa=kappa)
            for soc, drop in MODES:
                line = []
                for theta in SWEEP_THETAS:
                    rec = _solve_record(amg, prob, dict(h=f"1/{n}", dof=prob.n, kappa=kappa, soc=soc, drop=drop,
                                                         theta=theta), args.sweep_max_iter,
                                        soc=soc, drop=drop, theta=theta, max_coarse=50)
                    rows.append(rec)
                    line.append(_cell(rec))
                log(f"sweep h=1/{n} kappa={kappa:g} {soc}/{drop}: " + " ".join(line))
    for line in _sweep_tables(rows):
        log(line)
    return {"metric": "two-domain drop-tolerance sweep", "thetas": list(SWEEP_THETAS), "rows": rows}


def _cell(rec, cost=False):
    if rec.get("status") != "OK":
        return "-"
    return f"{rec['cost']:.1f}" if cost else str(rec["iterations"])


def _sweep_tables(rows):
    """markdown tables: one per (h, kappa), a row per measure/criterion, a column per theta"""
    out = []
    keys = []
    for r in rows:
        if (r["h"], r["kappa"]) not in keys:
            keys.append((r["h"], r["kappa"]))
    for cost in (False, True):
        for hh, kappa in keys:
            out.append(f"{'cost C x iterations' if cost else 'iterations'}, h = {hh}, kappa = {kappa:g}")
            out.append("| measure / criterion | " + " | ".join(f"{t:g}" for t in SWEEP_THETAS) + " |")
            out.append("|---|" + "---|" * len(SWEEP_THETAS))
            for soc, drop in MODES:
                cells = {r["theta"]: _cell(r, cost) for r in rows
                         if r["h"] == hh and r["kappa"] == kappa and r["soc"] == soc and r["drop"] == drop}
                out.append(f"| {soc} / {drop} | " + " | ".join(cells.get(t, "") for t in SWEEP_THETAS) + " |")
    return out


def run_annulus(args, amg, log):
    """The annulus parameter study (section "Anisotropic thermal diffusion",
    Table 1): material distance Laplacian with pointwise dropping, theta in
    {0.05, 0.1}, kappa = 10^0..10^4, the base mesh of 20 x 150 x 1 hexes and
    its refinements h / 2^k; iterations, levels and C."""
    from workloads import annulus_3d

    rows = []
    kappas = (1.0, 10.0, 100.0, 1e3, 1e4)
    for refine in args.annulus_refine:
        for kappa in kappas:
            t0 = time.perf_counter()
            prob = annulus_3d(refine, kappa=kappa)
            t_asm = time.perf_counter() - t0
            for theta in (0.05, 0.1):
                label = f"h/{1 << refine}" if refine else "h"
                rec = _solve_record(amg, prob, dict(refine=refine, h=label, dof=prob.n, nnz=prob.nnz, kappa=kappa,
                                                    theta=theta), args.annulus_max_iter, theta=theta,
                                    max_coarse=args.annulus_max_coarse)
                rows.append(rec)
                log(f"annulus {rec['h']} ({prob.n} DOF, assembled in {t_asm:.1f} s) kappa={kappa:g} "
                    f"theta={theta}: {rec.get('iterations')} its ({rec.get('levels')}, "
                    f"{rec.get('op_complexity', float('nan')):.2f}) {rec['status']} "
                    f"setup {rec.get('t_setup_ms', float('nan')):.0f} ms solve {rec.get('t_solve_ms', float('nan')):.0f} ms")
            del prob
    hs = [f"h/{1 << r}" if r else "h" for r in args.annulus_refine]
    for theta in (0.05, 0.1):
        log(f"theta = {theta}")
        log("| log10 kappa | " + " | ".join(hs) + " |")
        log("|---|" + "---|" * len(hs))
        for kappa in kappas:
            cells = []
            for r in args.annulus_refine:
                rec = next(x for x in rows if x["refine"] == r and x["kappa"] == kappa and x["theta"] == theta)
                cells.append(f"{rec['iterations']} ({rec['levels']}, {rec['op_complexity']:.2f})"
                             if rec["status"] == "OK" else rec["status"])
            log(f"| {math.log10(kappa):.0f} | " + " | ".join(cells) + " |")
    return {"metric": "annulus parameter study", "rows": rows}


def run_reuse(args, amg, log):
    """Setup reuse on the bench workload: a material update (the layer
    conductivities redrawn) applied with amg_update_values on the kept
    coarsening against a fresh setup, and successive right-hand sides on one
    hierarchy (setup cost amortised over K solves)."""
    import torch

    from workloads.q1 import layered_stack_3d

    dev = torch.device("cuda:0")

    def to_dev(prob):
        return dict(rowptr=torch.from_numpy(prob.rowptr).to(dev), col=torch.from_numpy(prob.col).to(dev),
                    val=torch.from_numpy(prob.val).to(dev), en=torch.from_numpy(prob.elem_nodes).to(dev),
                    es=torch.from_numpy(prob.elem_sigma).to(dev), xc=torch.from_numpy(prob.coords).to(dev),
                    b=torch.from_numpy(prob.b).to(dev))

    def setup(d, opts):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = amg.Hierarchy(d["rowptr"], d["col"], d["val"], d["en"], d["es"], d["xc"], opts)
        torch.cuda.synchronize()
        return h, time.perf_counter() - t0

    def solve(h, b):
        x = torch.zeros_like(b)
        _, info = h.solve(b, x, max_iter=args.reuse_max_iter, raise_on_error=False)
        return x, info

    log(f"reuse: generating layered stack {args.n}^3 with seeds 0 and 1")
    p0 = layered_stack_3d(n=args.n, repeats=args.repeats, stretch=args.stretch, seed=0)
    p1 = layered_stack_3d(n=args.n, repeats=args.repeats, stretch=args.stretch, seed=1)
    d0, d1 = to_dev(p0), to_dev(p1)
    del p0
    opts = amg.options(dim=3)
    h, _ = setup(d0, opts)  # warm-up of the allocator and the kernels
    h.close()
    h, t_setup0 = setup(d0, opts)
    _, i0 = solve(h, d0["b"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.update_values(d1["val"])
    t_update = time.perf_counter() - t0
    _, ir = solve(h, d1["b"])
    st_r = h.stats()
    h.close()
    f, t_setup1 = setup(d1, opts)
    _, if_ = solve(f, d1["b"])
    st_f = f.stats()
    log(f"reuse: setup {t_setup0 * 1e3:.0f} ms (seed 0, {i0['iterations']} its); update {t_update * 1e3:.0f} ms "
        f"-> {ir['iterations']} its {ir['status']}; fresh setup {t_setup1 * 1e3:.0f} ms -> {if_['iterations']} its")
    # successive right-hand sides b_k = A x_k, x_k seeded uniform, on the fresh hierarchy
    rng = np.random.default_rng(7)
    solves = []
    for k in range(args.reuse_rhs):
        xk = torch.from_numpy(rng.uniform(-1.0, 1.0, p1.n)).to(dev)
        bk = torch.empty_like(xk)
        f.level_spmv(0, xk, bk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = solve(f, bk)
        torch.cuda.synchronize()
        solves.append(dict(t_s=time.perf_counter() - t0, iterations=info["iterations"], status=info["status"]))
    f.close()
    amort = []
    for K in (1, 2, 4, 8, 16):
        if K <= len(solves):
            t = t_setup1 + sum(x["t_s"] for x in solves[:K])
            amort.append(dict(rhs=K, dof_per_s=p1.n * K / t, setup_share=t_setup1 / t))
    log("reuse: " + ", ".join(f"K={a['rhs']}: {a['dof_per_s'] / 1e6:.2f} M DOF/s (setup {100 * a['setup_share']:.0f}%)"
                               for a in amort))
    return {"metric": "setup reuse", "workload": f"layered stack {args.n}^3, {args.repeats} repeats, "
                                                 f"{args.stretch:g}:1, seeds 0 -> 1",
            "dof": p1.n, "t_setup_s": t_setup0, "t_update_s": t_update, "t_update_lib_s": st_r["t_update_s"],
            "iterations_before": i0["iterations"], "iterations_updated": ir["iterations"],
            "status_updated": ir["status"], "op_complexity_updated": st_r["op_complexity"],
            "t_setup_fresh_s": t_setup1, "iterations_fresh": if_["iterations"],
            "op_complexity_fresh": st_f["op_complexity"], "rhs_solves": solves, "amortised": amort}


def run_fp32_aniso(args, amg, dev, log):
    """FP32-hierarchy form against the FP64 form on the rotated-anisotropy
    cube (n^3 hexes, 8^3-element blocks, f ~ U(-1, 1)): the same right-hand
    side from x0 = 0, several timed solves per form on one hierarchy each."""
    import torch

    from workloads import rotated_anisotropic_3d

    log(f"generating rotated-anisotropy cube {args.aniso_n}^3")
    prob = rotated_anisotropic_3d(n=args.aniso_n, block=8)
    d = [torch.from_numpy(a).to(dev) for a in (prob.rowptr, prob.col, prob.val, prob.elem_nodes, prob.elem_sigma,
                                                prob.coords)]
    b = torch.from_numpy(prob.b).to(dev)
    x = torch.zeros(prob.n, dtype=torch.float64, device=dev)
    out = dict(workload=f"rotated anisotropy {args.aniso_n}^3, 8^3 blocks, eps 1e-3, isotropic fill 1e-4",
               n=prob.n, nnz=prob.nnz)
    sol = {}
    for name, prec in (("fp64", "fp64"), ("fp32", "fp32")):
        opts = amg.options(dim=3, precision=prec, max_levels=args.max_levels)
        torch.cuda.synchronize()
        h = amg.Hierarchy(*d, opts)
        t_setup = h.stats()["t_setup_s"]
        ts = []
        for _ in range(max(1, args.fp32_reps)):
            x.zero_()
            _, info = h.solve(b, x, max_iter=args.max_iter)
            ts.append(1e3 * info["t_solve_s"])
        sol[name] = x.cpu().numpy()
        vc = vcycle_record(h, prob.n, args.vcycles, dev)
        h.close()
        out[name] = dict(t_setup_ms=1e3 * t_setup, t_solve_ms_stats=stats_ms(np.array(ts)),
                         iterations=info["iterations"], rel_res=info["rel_res"], status=info["status"], vcycle=vc)
    m64, m32 = out["fp64"]["t_solve_ms_stats"]["median"], out["fp32"]["t_solve_ms_stats"]["median"]
    out["speedup_vs_fp64_solve"] = m64 / m32
    out["speedup_per_iteration"] = (m64 / max(1, out["fp64"]["iterations"])) / (m32 / max(1, out["fp32"]["iterations"]))
    out["speedup_vs_fp64_vcycle"] = out["fp64"]["vcycle"]["ms"] / out["fp32"]["vcycle"]["ms"]
    out["rel_err_vs_fp64_form"] = float(np.linalg.norm(sol["fp32"] - sol["fp64"]) / np.linalg.norm(sol["fp64"]))
    log(f"aniso {args.aniso_n}^3: V-cycle fp32 {out['fp32']['vcycle']['ms']:.3f} ms vs fp64 "
        f"{out['fp64']['vcycle']['ms']:.3f} ms ({out['speedup_vs_fp64_vcycle']:.2f}x)")
    log(f"aniso {args.aniso_n}^3: fp32 {m32:.1f} ms ({out['fp32']['iterations']} it) vs fp64 {m64:.1f} ms "
        f"({out['fp64']['iterations']} it): {out['speedup_vs_fp64_solve']:.2f}x, "
        f"rel err {out['rel_err_vs_fp64_form']:.1e}")
    return out


def stats_ms(v):
    """mean, standard deviation, median, min and max of a list of times (ms)"""
    v = np.asarray(v, dtype=float)
    return {"mean": float(v.mean()), "std": float(v.std(ddof=1)) if v.size > 1 else 0.0,
            "median": float(np.median(v)), "min": float(v.min()), "max": float(v.max()), "n": int(v.size)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128, help="hexes per side")
    ap.add_argument("--repeats", type=int, default=20)
    ap.add_argument("--stretch", type=float, default=10.0)
    ap.add_argument("--max-levels", type=int, default=10, help="hierarchy depth cap (the 192^3 stack needs 16)")
    ap.add_argument("--max-iter", type=int, default=1000, help="PCG iteration cap")
    ap.add_argument("--vcycles", type=int, default=100)
    ap.add_argument("--fp32-reps", type=int, default=5, help="timed FP32-form solves on one hierarchy")
    ap.add_argument("--x0-seeds", type=int, default=5, help="seeded initial guesses for the FP32/FP64 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle's full setup and solve")
    ap.add_argument("--c4-reps", type=int, default=1,
                    help="timed setup + solve runs per precision form on the 192^3 stack (0: skip)")
    ap.add_argument("--c4-max-iter", type=int, default=4000, help="PCG iteration cap on the 192^3 stack")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="one setup, a few V-cycles and a 1 GiB device copy (for counter collection), no JSON")
    ap.add_argument("--profile-precision", choices=("fp64", "fp32"), default="fp64",
                    help="--profile-kernels: precision form of the hierarchy")
    ap.add_argument("--profile-workload", choices=("layered", "aniso"), default="layered",
                    help="--profile-kernels: the layered stack (--n) or the rotated-anisotropy cube (--aniso-n)")
    ap.add_argument("--profile-vcycles", type=int, default=3, help="--profile-kernels: V-cycles after the setup")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--aniso-n", type=int, default=96,
                    help="hexes per side of the rotated-anisotropy FP32/FP64 comparison (0: skip)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--no-studies", action="store_true",
                    help="skip the strength-measure comparison, the drop-tolerance sweep and the annulus study "
                         "(about 45 s; each also runs alone with --compare, --sweep, --annulus)")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving stream (its JSON object)")
    ap.add_argument("--compare", action="store_true",
                    help="run only the strength-measure / dropping comparison (its JSON object)")
    ap.add_argument("--sweep", action="store_true",
                    help="run only the two-domain drop-tolerance sweep (its JSON object)")
    ap.add_argument("--sweep-n", type=int, nargs="+", default=[32, 128, 512],
                    help="two-domain elements per direction (h = 1/n)")
    ap.add_argument("--sweep-max-iter", type=int, default=1000)
    ap.add_argument("--annulus", action="store_true", help="run only the annulus parameter study (its JSON object)")
    ap.add_argument("--annulus-refine", type=int, nargs="+", default=[0, 1, 2, 3, 4],
                    help="refinement levels k of the annulus base mesh (element size h / 2^k)")
    ap.add_argument("--annulus-max-iter", type=int, default=1000)
    ap.add_argument("--annulus-max-coarse", type=int, default=5000, help="coarsest-level size target")
    ap.add_argument("--reuse", action="store_true",
                    help="run only the setup-reuse measurement (material update, successive right-hand sides)")
    ap.add_argument("--reuse-rhs", type=int, default=16)
    ap.add_argument("--reuse-max-iter", type=int, default=1000)
    ap.add_argument("--serve-num", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-budget-gib", type=float, default=8.0)
    ap.add_argument("--serve-active", type=int, default=32)
    ap.add_argument("--serve-max-iter", type=int, default=1000)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2602_05686_amd as amg
    from workloads.q1 import layered_stack_3d, seeded_start

    amg.load()
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.serving_only:
        print(json.dumps(run_serving(args, amg, log)), flush=True)
        return
    if args.compare:
        print(json.dumps(run_compare(amg, log)), flush=True)
        return
    if args.sweep:
        print(json.dumps(run_sweep(args, amg, log)), flush=True)
        return
    if args.annulus:
        print(json.dumps(run_annulus(args, amg, log)), flush=True)
        return
    if args.reuse:
        print(json.dumps(run_reuse(args, amg, log)), flush=True)
        return

    if args.profile_kernels and args.profile_workload == "aniso":
        from workloads import rotated_anisotropic_3d

        log(f"generating rotated-anisotropy cube {args.aniso_n}^3")
        prob = rotated_anisotropic_3d(n=args.aniso_n, block=8)
    else:
        log(f"generating layered stack {args.n}^3, {args.repeats} repeats, {args.stretch:g}:1")
        prob = layered_stack_3d(n=args.n, repeats=args.repeats, stretch=args.stretch)
    n = prob.n
    d = dict(rowptr=torch.from_numpy(prob.rowptr).to(dev), col=torch.from_numpy(prob.col).to(dev),
             val=torch.from_numpy(prob.val).to(dev), en=torch.from_numpy(prob.elem_nodes).to(dev),
             es=torch.from_numpy(prob.elem_sigma).to(dev), xc=torch.from_numpy(prob.coords).to(dev),
             b=torch.from_numpy(prob.b).to(dev))
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    opts64 = amg.options(dim=3, max_levels=args.max_levels)
    torch.cuda.synchronize()

    def step(opts):
        h = amg.Hierarchy(d["rowptr"], d["col"], d["val"], d["en"], d["es"], d["xc"], opts)
        x.zero_()
        _, info = h.solve(d["b"], x, max_iter=args.max_iter)
        return h, info

    if args.profile_kernels:
        # copy calibration: a plain copy of 1 GiB (read 1 GiB, write 1 GiB)
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        opts = amg.options(dim=3, max_levels=args.max_levels, precision=args.profile_precision)
        h = amg.Hierarchy(d["rowptr"], d["col"], d["val"], d["en"], d["es"], d["xc"], opts)
        st = h.stats()
        for lv in range(st["levels"]):
            log(f"level {lv}: n {st['n'][lv]}, nnz {st['nnz'][lv]}, nnz(P) {st['nnz_p'][lv]}")
        r = torch.randn(n, dtype=torch.float64, device=dev)
        z = torch.zeros_like(r)
        for _ in range(args.profile_vcycles):
            h.vcycle(r, z)
        torch.cuda.synchronize()
        h.close()
        log("profile run done")
        return

    log(f"warmup {args.warmup} step(s)")
    for _ in range(args.warmup):
        h, info = step(opts64)
        h.close()
    log(f"timing {args.steps} step(s)")
    infos, setups, step_ms = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        h, info = step(opts64)
        torch.cuda.synchronize()
        step_ms.append(1e3 * (time.perf_counter() - ts))
        infos.append(info)
        setups.append(h.stats()["t_setup_s"])
        if k + 1 < args.steps:
            h.close()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    ms_per_step = 1e3 * t_total / args.steps
    st = h.stats()
    t_solve = float(np.mean([i["t_solve_s"] for i in infos]))
    x64 = x.cpu().numpy()
    log(f"step {ms_per_step:.1f} ms, setup {np.mean(setups) * 1e3:.1f} ms, solve {t_solve * 1e3:.1f} ms, "
        f"iters {infos[-1]['iterations']}, levels {st['n']}")
    exact = layered_exact(prob)
    err64 = float(np.linalg.norm(x64 - exact) / np.linalg.norm(exact))

    # V-cycle bandwidth and the dominant kernel's roofline
    t_vc_ms = time_vcycles(h, n, args.vcycles, dev)
    vc_gbs = st["vcycle_alg_bytes"] / (t_vc_ms * 1e-3) / 1e9
    kt = h.time_smoother(level=0, reps=args.vcycles)
    avg_ms = kt["avg_ms"]
    achieved = kt["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
    log(f"V-cycle {t_vc_ms:.3f} ms = {vc_gbs:.0f} GB/s algorithmic; fine smoother SpMV {avg_ms * 1e3:.1f} us "
        f"= {achieved:.0f} GB/s")
    stream_bw = achievable_bandwidth(dev)
    log("plain streaming, 1 GiB: " + ", ".join(f"{k[:-5]} {v:.0f} GB/s" for k, v in stream_bw.items()))

    # the same solve from seeded initial guesses x0 ~ U(0, 1): how the exit
    # count and the throughput move with the starting point
    seeds = []
    for k in range(args.x0_seeds):
        x.copy_(torch.from_numpy(seeded_start(n, k)).to(dev))
        _, ik = h.solve(d["b"], x, max_iter=args.max_iter)
        seeds.append((ik["iterations"], 1e3 * ik["t_solve_s"]))

    fp32 = None
    if not args.no_fp32:
        opts32 = amg.options(dim=3, precision="fp32", max_levels=args.max_levels)
        h32, _ = step(opts32)
        t32 = []
        for _ in range(max(1, args.fp32_reps)):
            x.zero_()
            _, info32 = h32.solve(d["b"], x, max_iter=args.max_iter)
            t32.append(info32["t_solve_s"])
        x32 = x.cpu().numpy()
        vc32 = vcycle_record(h32, n, args.vcycles, dev)
        seeds32 = []
        for k in range(args.x0_seeds):
            x.copy_(torch.from_numpy(seeded_start(n, k)).to(dev))
            _, ik = h32.solve(d["b"], x, max_iter=args.max_iter)
            seeds32.append((ik["iterations"], 1e3 * ik["t_solve_s"]))
        h32.close()
        t32m = float(np.mean(t32))
        fp32 = dict(t_solve_s=t32m, t_solve_ms_stats=stats_ms(np.array(t32) * 1e3), iterations=info32["iterations"],
                    rel_res=info32["rel_res"], status=info32["status"], speedup_vs_fp64_solve=t_solve / t32m,
                    speedup_per_iteration=(t_solve / infos[-1]["iterations"]) /
                    (t32m / max(1, info32["iterations"])),
                    vcycle=vc32, speedup_vs_fp64_vcycle=t_vc_ms / vc32["ms"],
                    rel_err_vs_fp64_form=float(np.linalg.norm(x32 - x64) / np.linalg.norm(x64)),
                    rel_err_vs_closed_form=float(np.linalg.norm(x32 - exact) / np.linalg.norm(exact)))
        if seeds32:
            m64, m32 = float(np.median([v[1] for v in seeds])), float(np.median([v[1] for v in seeds32]))
            fp32["x0_seeds"] = {"seeds": len(seeds32), "fp64_iterations": [v[0] for v in seeds],
                                "fp32_iterations": [v[0] for v in seeds32], "fp64_t_solve_ms_median": m64,
                                "fp32_t_solve_ms_median": m32, "speedup_of_medians": m64 / m32}
        log(f"fp32 form: solve {t32m * 1e3:.1f} ms (mean of {len(t32)}), iters {info32['iterations']}, V-cycle "
            f"{vc32['ms']:.3f} ms ({t_vc_ms / vc32['ms']:.2f}x the FP64 one)")
    h.close()
    if fp32 is not None and args.aniso_n > 0:
        fp32["aniso"] = run_fp32_aniso(args, amg, dev, log)

    c4 = None
    if args.c4_reps > 0:
        del d
        torch.cuda.empty_cache()
        c4 = run_layered192(args, amg, dev, log)

    # the paper's parameter studies on their synthetic stand-ins (their own
    # JSON objects under "studies"; outside the timed region)
    studies = None
    if not args.no_studies:
        studies = {"compare": run_compare(amg, log), "sweep": run_sweep(args, amg, log),
                   "annulus": run_annulus(args, amg, log)}
    serving = None
    if not args.no_serving:
        torch.cuda.empty_cache()
        serving = run_serving(args, amg, log)

    cpu = None
    if not args.no_cpu_baseline:
        log("oracle: full setup and PCG solve on the same workload (single-threaded)")
        cpu, xo = cpu_baseline(prob)
        cpu["gpu_fp64_rel_err_vs_oracle"] = float(np.linalg.norm(x64 - xo) / np.linalg.norm(xo))
        cpu["oracle_rel_err_vs_closed_form"] = float(np.linalg.norm(xo - exact) / np.linalg.norm(exact))
        if fp32 is not None:
            fp32["rel_err_vs_fp64_oracle"] = float(np.linalg.norm(x32 - xo) / np.linalg.norm(xo))
        log(f"oracle: {cpu['iterations']} iterations, {cpu['t_setup_s']:.1f} s setup + {cpu['t_solve_s']:.1f} s "
            f"solve; GPU FP64 solution {cpu['gpu_fp64_rel_err_vs_oracle']:.1e} from the oracle's")

    traffic = measured_traffic() if args.n == 128 and args.repeats == 20 and args.stretch == 10.0 else None
    seeded = None
    if seeds:
        med = float(np.median([v[1] for v in seeds]))
        t_setup_ms = 1e3 * float(np.mean(setups))
        seeded = {"seeds": len(seeds), "iterations": [v[0] for v in seeds], "t_solve_ms_median": med,
                  "dof_per_s_setup_plus_median_solve": n / ((t_setup_ms + med) * 1e-3),
                  "solve_only_dof_per_s_median": n / (med * 1e-3)}
    out = {
        "metric": "DOF/s to rel-res 1e-8 (setup + AMG-PCG solve)",
        "value": n * args.steps / t_total,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"layered stack {args.n}^3 hex Q1 ({n} DOF), {args.repeats} repeats x 3 layers, "
                               f"{args.stretch:g}:1 flat, FP64 plain form, PCG from x0 = 0",
                   "dof": n, "nnz": prob.nnz, "theta": 0.08, "tol": 1e-8},
        "solve_only_dof_per_s": n / t_solve,
        "t_setup_ms": 1e3 * float(np.mean(setups)),
        "t_solve_ms": 1e3 * t_solve,
        "step_ms_stats": stats_ms(step_ms),
        "t_setup_ms_stats": stats_ms(np.array(setups) * 1e3),
        "t_solve_ms_stats": stats_ms(np.array([i["t_solve_s"] for i in infos]) * 1e3),
        "iterations_per_step": sorted(set(int(i["iterations"]) for i in infos)),
        "iterations": infos[-1]["iterations"],
        "rel_res_true": infos[-1]["rel_res"],
        "rel_err_vs_closed_form": err64,
        "seeded_x0": seeded,
        "levels": st["n"],
        "op_complexity": st["op_complexity"],
        "vcycle": {"ms": t_vc_ms, "alg_bytes": st["vcycle_alg_bytes"], "alg_GBps": vc_gbs,
                   "frac_of_peak": vc_gbs / HBM_PEAK_GBS},
        "roofline": {"bound": "hbm", "kernel": "k_stream<double, SMOOTH> on the finest level",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "avg_launch_us": avg_ms * 1e3, "launches": args.vcycles,
                     "alg_bytes_per_launch": kt["bytes_per_launch"],
                     # plain streaming on this GPU (1 GiB, torch kernels), beside the published peak
                     "achievable": stream_bw,
                     "frac_of_achievable_read": achieved / stream_bw["read_GBps"]},
        "fp32_form": fp32,
        "layered192": c4,
        "serving": serving,
        "studies": studies,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
