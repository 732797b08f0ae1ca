#!/usr/bin/env python3
"""Benchmark: material-aware SA-AMG-PCG on one MI355X.

Workload: battery-like layered stack, 3D Q1 on a 128^3 hex mesh
(2,146,689 DOF), elements 10:1 flat (domain [0,10]^2 x [0,1]), 20 repeats of
three isotropic layers with log-uniform conductivities in [1e-5,1e-2],
[1e-10,1e-8], [1e-1,1], u = 0 / 1 on the bottom / top faces, FP64.

One step = the whole hot path on inputs already resident in HBM:
amg_setup (Clement tensors, strength, aggregation, prolongators, Galerkin
products, coarse factorisation) followed by amg_pcg_solve to a true relative
residual of 1e-8.  value = DOF * steps / time.  The JSON line also carries
solve-only throughput, the FP32-hierarchy form against the FP64 form, the
V-cycle's algorithmic HBM bandwidth, the roofline of the dominant kernel
(the finest level's fused Chebyshev SpMV: back-to-back launches between
HIP events on its stream) and the CPU oracle timed on a bounded sample of the same recipe.
"""

import argparse
import json
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


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(prob, iterations, sample_iters):
    """The oracle as it stands, single-threaded, on a bounded sample of the
    same workload: its full setup plus `sample_iters` PCG iterations; the
    solve is scaled to the GPU run's iteration count."""
    import oracle

    t0 = time.perf_counter()
    h = oracle.Hierarchy(prob)
    t1 = time.perf_counter()
    _, info = h.pcg(prob.b, maxit=sample_iters)
    t2 = time.perf_counter()
    t_iter = (t2 - t1) / max(info["iterations"], 1)
    t_est = (t1 - t0) + t_iter * iterations
    return dict(value=prob.n / t_est, unit="DOF/s", cores=1, kind="oracle",
                sample=(f"same workload ({prob.n} DOF): full oracle setup ({t1 - t0:.1f}s) + "
                        f"{info['iterations']} PCG iterations ({t2 - t1:.1f}s, {t_iter * 1e3:.0f} ms/iteration); "
                        f"solve scaled to the GPU run's {iterations} iterations"),
                host_cpu=cpu_model(), host_threads=os.cpu_count())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128, help="hexes per side")
    ap.add_argument("--repeats", type=int, default=20)
    ap.add_argument("--stretch", type=float, default=10.0)
    ap.add_argument("--vcycles", type=int, default=50)
    ap.add_argument("--cpu-sample", type=int, default=5, help="oracle PCG iterations in the CPU sample (0: skip)")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="one setup, a few V-cycles and a 1 GiB device copy (for counter collection), no JSON")
    ap.add_argument("--no-fp32", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2602_05686_amd as amg
    from workloads.q1 import layered_stack_3d

    amg.load()
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    log(f"generating layered stack {args.n}^3, {args.repeats} repeats, {args.stretch:g}:1")
    prob = layered_stack_3d(n=args.n, repeats=args.repeats, stretch=args.stretch)
    n = prob.n
    d = dict(rowptr=torch.from_numpy(prob.rowptr).to(dev), col=torch.from_numpy(prob.col).to(dev),
             val=torch.from_numpy(prob.val).to(dev), en=torch.from_numpy(prob.elem_nodes).to(dev),
             es=torch.from_numpy(prob.elem_sigma).to(dev), xc=torch.from_numpy(prob.coords).to(dev),
             b=torch.from_numpy(prob.b).to(dev))
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    opts64 = amg.options(dim=3)
    torch.cuda.synchronize()

    def step(opts):
        h = amg.Hierarchy(d["rowptr"], d["col"], d["val"], d["en"], d["es"], d["xc"], opts)
        x.zero_()
        _, info = h.solve(d["b"], x)
        return h, info

    if args.profile_kernels:
        # copy calibration: a plain copy of 1 GiB (read 1 GiB, write 1 GiB)
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        h = amg.Hierarchy(d["rowptr"], d["col"], d["val"], d["en"], d["es"], d["xc"], opts64)
        r = torch.randn(n, dtype=torch.float64, device=dev)
        z = torch.zeros_like(r)
        for _ in range(3):
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
    infos, setups = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        h, info = step(opts64)
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

    # closed-form discrete solution of the layered stack (f = 0, z-only)
    kz = prob.meta["layer_k"]
    res = 1.0 / kz
    cf = np.concatenate([[0.0], np.cumsum(res)]) / res.sum()
    zi = np.rint(prob.coords[:, 2] * args.n).astype(int)
    exact = cf[zi]
    err64 = float(np.linalg.norm(x64 - exact) / np.linalg.norm(exact))

    # V-cycle bandwidth and the dominant kernel's roofline
    r = torch.randn(n, dtype=torch.float64, device=dev)
    z = torch.zeros_like(r)
    for _ in range(3):
        h.vcycle(r, z)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.vcycles):
        h.vcycle(r, z)
    e1.record(stream)
    torch.cuda.synchronize()
    t_vc_ms = e0.elapsed_time(e1) / args.vcycles
    vc_gbs = st["vcycle_alg_bytes"] / (t_vc_ms * 1e-3) / 1e9
    kt = h.time_smoother(level=0, reps=args.vcycles)
    avg_ms = kt["avg_ms"]
    achieved = kt["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
    log(f"V-cycle {t_vc_ms:.3f} ms = {vc_gbs:.0f} GB/s algorithmic; fine smoother SpMV {avg_ms * 1e3:.1f} us "
        f"= {achieved:.0f} GB/s")
    h.close()

    fp32 = None
    if not args.no_fp32:
        opts32 = amg.options(dim=3, precision="fp32")
        h32, _ = step(opts32)
        x.zero_()
        _, info32 = h32.solve(d["b"], x)
        x32 = x.cpu().numpy()
        h32.close()
        fp32 = dict(t_solve_s=info32["t_solve_s"], iterations=info32["iterations"], rel_res=info32["rel_res"],
                    status=info32["status"], speedup_vs_fp64_solve=t_solve / info32["t_solve_s"],
                    rel_err_vs_fp64_form=float(np.linalg.norm(x32 - x64) / np.linalg.norm(x64)),
                    rel_err_vs_closed_form=float(np.linalg.norm(x32 - exact) / np.linalg.norm(exact)))
        log(f"fp32 form: solve {info32['t_solve_s'] * 1e3:.1f} ms, iters {info32['iterations']}")

    cpu = None
    if args.cpu_sample > 0:
        log(f"oracle sample: setup + {args.cpu_sample} PCG iterations")
        cpu = cpu_baseline(prob, infos[-1]["iterations"], args.cpu_sample)

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
                               f"{args.stretch:g}:1 flat, FP64 plain form",
                   "dof": n, "nnz": prob.nnz, "theta": 0.08, "tol": 1e-8},
        "solve_only_dof_per_s": n / t_solve,
        "t_setup_ms": 1e3 * float(np.mean(setups)),
        "t_solve_ms": 1e3 * t_solve,
        "iterations": infos[-1]["iterations"],
        "rel_res_true": infos[-1]["rel_res"],
        "rel_err_vs_closed_form": err64,
        "levels": st["n"],
        "op_complexity": st["op_complexity"],
        "vcycle": {"ms": t_vc_ms, "alg_bytes": st["vcycle_alg_bytes"], "alg_GBps": vc_gbs,
                   "frac_of_peak": vc_gbs / HBM_PEAK_GBS},
        "roofline": {"bound": "hbm", "kernel": "k_stream<double, SMOOTH> on the finest level",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "avg_launch_us": avg_ms * 1e3, "launches": args.vcycles,
                     "alg_bytes_per_launch": kt["bytes_per_launch"]},
        "fp32_form": fp32,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
