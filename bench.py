#!/usr/bin/env python
"""Benchmark: cell-solves/s and seconds per converged time step at tol 1e-10,
FP32-refined OCI against FP64 OCI and GPU source iteration, on one MI355X.

Workload (default "regions4096"): the one-group slab of 4096 cells on [0, 64]
cm in 64 random regions (sigma_t ~ U[0.1, 10], c ~ U[0.5, 0.999], seed 2),
S16 (cell systems of n = 64), Q = 1 in the first 8 regions, vacuum boundaries,
zero initial flux, for each time-step size of the sweep {0.1, 0.01, 1e-3,
1e-4} s.  One benchmark step = one converged time step of every problem of
the sweep (four OCI time steps).  K steps reproduce K time steps of the
workload from zero initial flux; setup (assembly + LU + inversion on the
device) happens before the timed region and is reported separately.

value = cell-solves / s of the FP32-refined path over the timed region, a
cell-solve being one cell's 4NG system solved once in one iteration.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_HBM_TBS = 8.0          # published HBM3E peak, TB/s
MI355X_FP32_TFLOPS = 157.3    # published FP32 vector peak


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="regions4096")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the CPU-oracle sample")
    ap.add_argument("--no-comparators", action="store_true")
    return ap.parse_args()


def problems(name):
    from paper_2503_00264_amd import workloads as W
    if name == "regions4096":
        base = W.config(name)
        return base, [dict(base, dt=dt) for dt in W.REGIONS_DT_SWEEP]
    p = W.config(name)
    return p, [p]


def run_method(probs, method, precision, K, W_, tol, torch, B, profile=False):
    """Set up one solver per problem, warm up, reset, then time K steps."""
    solvers, setup_s = [], []
    for p in probs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = B.Solver(p, precision=precision, tol=tol)
        torch.cuda.synchronize()
        setup_s.append(time.perf_counter() - t0)
        solvers.append(s)
    for s in solvers:
        for _ in range(W_):
            s.step(method)
        s.set_state(None)      # back to zero initial flux and a fresh first iterate
    infos = torch.zeros((K, len(solvers), 32), dtype=torch.uint8, device=solvers[0].dev)
    if profile:
        for s in solvers:
            B.oci_profile_enable(s.h, True)
    fn = B.oci_step if method == "oci" else B.si_step
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    t0 = time.perf_counter()
    for k in range(K):
        for i, s in enumerate(solvers):
            fn(s.h, s.q, s.inc_l, s.inc_r, s.phi, None, infos[k, i])
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    kern = [B.oci_profile_read(s.h) if profile else (0.0, 0) for s in solvers]
    inf = infos.cpu().numpy()
    dec = [[B.decode_info(inf[k, i]) for i in range(len(solvers))] for k in range(K)]
    for s in solvers:
        s.close()
    its = np.array([[d["iterations"] for d in row] for row in dec])       # [K][problems]
    status = sorted({d["status"] for row in dec for d in row})
    J = probs[0]["J"]
    per_dt = []
    for i, p in enumerate(probs):
        per_dt.append(dict(dt=p["dt"], setup_s=setup_s[i],
                           iterations_per_step=float(its[:, i].mean()),
                           iterations_max=int(its[:, i].max())))
    return dict(time_s=max(gpu_ms / 1e3, 1e-12), wall_s=wall, iterations=its, J=J,
                cell_solves=int(its.sum()) * J, per_dt=per_dt, status=status, kernel=kern)


def cpu_baseline(prob, seconds):
    """The FP64 oracle (OpenMP) on a bounded sample of the same workload."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = oracle.Oracle(dict(prob), methods=("oci",))
    pp, pi = o.initial_state()
    t0 = time.perf_counter()
    its = steps = 0
    while steps < prob["steps"]:
        _, info = o.step("oci", pp, pi, q=prob["q"], tol=1e-10)
        its += info["iterations"]
        steps += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return dict(value=its * prob["J"] / dt, unit="cell-solves/s", cores=threads, kind="oracle",
                sample=f"first {steps} converged time step(s) of the dt={prob['dt']} problem "
                       f"({its} iterations x {prob['J']} cells, {dt:.1f} s, setup excluded)")


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    from paper_2503_00264_amd import binding as B
    torch.cuda.set_device(0)
    base, probs = problems(a.workload)
    N, G, J = base["N"], base["G"], base["J"]
    n = 4 * N * G

    prim = run_method(probs, "oci", B.OCI_FP32_REFINED, a.steps, a.warmup, a.tol, torch, B, profile=True)
    comp = {}
    if not a.no_comparators:
        comp["fp64"] = run_method(probs, "oci", B.OCI_FP64, a.steps, a.warmup, a.tol, torch, B, profile=True)
        comp["si"] = run_method(probs, "si", B.OCI_FP64, a.steps, a.warmup, a.tol, torch, B, profile=True)

    value = prim["cell_solves"] / prim["time_s"]
    ms_per_step = prim["time_s"] * 1e3 / a.steps

    # roofline of the dominant kernel: the persistent OCI kernel of the
    # refined path, one launch per time step.  Algorithmic bytes per
    # cell-iteration (factor stream + iterate/edge/source/flux traffic):
    #   4 n^2 + 4 n + 128 N G + 64 G
    kern_ms = sum(k[0] for k in prim["kernel"])
    launches = sum(k[1] for k in prim["kernel"])
    avg_launch_s = kern_ms / 1e3 / max(launches, 1)
    bytes_per_ci = 4 * n * n + 4 * n + 128 * N * G + 64 * G
    cell_iters_per_launch = prim["cell_solves"] / max(launches, 1)
    achieved = bytes_per_ci * cell_iters_per_launch / avg_launch_s / 1e9
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=MI355X_HBM_TBS * 1e3, unit="GB/s",
                    frac=round(achieved / (MI355X_HBM_TBS * 1e3), 4), traffic=None,
                    kernel="k_oci_step<float,64,resident>",
                    avg_launch_us=round(avg_launch_s * 1e6, 2),
                    cell_iterations_per_launch=round(cell_iters_per_launch, 1),
                    bytes_per_cell_iteration=bytes_per_ci,
                    flops_per_cell_iteration=2 * n * n,
                    achieved_tflops_fp32=round(2 * n * n * cell_iters_per_launch / avg_launch_s / 1e12, 3))

    def summary(r, label):
        """Per-method figures; seconds per converged step per dt come from the
        iteration-kernel events of that dt's problem."""
        return dict(cell_solves_per_s=r["cell_solves"] / r["time_s"],
                    s_per_converged_step={str(x["dt"]): ms / 1e3 / max(cnt, 1)
                                          for (ms, cnt), x in zip(r["kernel"], r["per_dt"])},
                    iterations_per_step={str(x["dt"]): x["iterations_per_step"] for x in r["per_dt"]},
                    setup_s={str(x["dt"]): round(x["setup_s"], 4) for x in r["per_dt"]},
                    timed_region_s=round(r["time_s"], 6),
                    kernel_ms=round(sum(k[0] for k in r["kernel"]), 3), status=r["status"], label=label)

    out = {
        "metric": "cell-solves/s and s per converged step: FP32-refined vs FP64 OCI vs SI @1e-10",
        "value": round(value, 1),
        "unit": "cell-solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 solve + f64 residual/norm/update",
        "data": "synthetic (seeded generator; no external data)",
        "config": {"workload": f"{a.workload}: J={J} N={N} G={G} n={n}, dt sweep "
                               f"{[p['dt'] for p in probs]}, tol {a.tol}, one step = one time step "
                               f"of each dt", "J": J, "N": N, "G": G, "n": n,
                   "dts": [p["dt"] for p in probs], "tol": a.tol},
        "roofline": roofline,
        "comparison": {"fp32_refined": summary(prim, "FP32 LU+inverse, FP64 residual refinement")},
    }
    for k, r in comp.items():
        out["comparison"][k] = summary(r, {"fp64": "FP64 LU+inverse OCI", "si": "FP64 source iteration sweep"}[k])
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(probs[0], a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
