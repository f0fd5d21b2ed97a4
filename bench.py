#!/usr/bin/env python
"""Benchmark: cell-solves/s and seconds per converged time step at tol 1e-10,
FP32-refined OCI against FP64 OCI and GPU source iteration, on one MI355X.

Default workload "regions4096": the one-group slab of 4096 cells on [0, 64] cm
in 64 random regions (sigma_t ~ U[0.1, 10], c ~ U[0.5, 0.999], seed 2), S16
(cell systems of n = 64), Q = 1 in the first 8 regions, vacuum boundaries,
zero initial flux, for each time-step size of the sweep {0.1, 0.01, 1e-3,
1e-4} s.  One benchmark step = one converged time step of every problem of the
sweep (four OCI time steps).  K steps reproduce K time steps of the workload
from zero initial flux (the state is reset after the W warm-up steps): each
problem's K OCI steps are one oci_run_steps call (one launch of the
register-resident kernel, which turns each converged step over to the next
itself), SI runs K si_step calls.  Setup (device assembly + LU + inversion,
then the launch-shape autotuner) happens before the timed region and is
reported separately.

Other workloads: "homogeneous64", "multigroup8192", "multigroup16384" (one
problem each), "batch64": the 64 uneven slabs advanced together by the
batched persistent launch with K graph-captured steps, against the same slabs
solved one after another in FP64, and "rosa": the two-group, highly
scattering performance problem of section 3.2 (table rosa_test; L = 100 cm,
vacuum, Q = 1, zero start) swept over the cell optical thickness delta =
Sigma_2 dx (the smaller total cross section), S8 / S16 / S32 and
dt = 10 s / 0.1 s: K converged steps of each configuration timed for
FP64 OCI, FP32-refined OCI and SI (setup outside the timed region, as in the
paper's convergence-loop runtimes).

value = cell-solves / s of the FP32-refined path over the timed region, a
cell-solve being one cell's 4NG system solved once in one iteration.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_HBM_GBS = 8000.0       # published HBM3E peak, GB/s
MI355X_FP32_TFLOPS = 157.3    # published FP32 vector peak (FP32 matrix: the same figure)
MI355X_FP64_TFLOPS = 78.6     # published FP64 vector peak (FP64 matrix: the same figure)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="regions4096")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU-oracle sample")
    ap.add_argument("--no-comparators", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--slabs", type=int, default=64, help="batch64: number of slabs")
    return ap.parse_args()


def problems(name):
    from paper_2503_00264_amd import workloads as W
    if name == "regions4096":
        base = W.config(name)
        return base, [dict(base, dt=dt) for dt in W.REGIONS_DT_SWEEP]
    p = W.config(name)
    return p, [p]


def kernel_label(cfg, fp32, np_):
    t = "float" if fp32 else "double"
    if cfg["local"] and cfg["resident"]:
        return f"k_oci_res<{t},{np_},{cfg['block']}>"
    if cfg["local"]:
        return f"k_oci_local<{t},{np_},{cfg['block']}>"
    return f"k_oci_step<{t},{np_},{'true' if cfg['resident'] else 'false'},{cfg['block']}>"


def run_method(probs, method, precision, K, W_, tol, torch, B, autotune=True):
    """Set up one solver per problem, tune, warm up, reset, then time K steps."""
    solvers, setup_s, configs = [], [], []
    B.Solver(probs[0], precision=precision, tol=tol).close()   # first-use costs out of the setup times
    for p in probs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = B.Solver(p, precision=precision, tol=tol)
        torch.cuda.synchronize()
        setup_s.append(time.perf_counter() - t0)
        if autotune and method == "oci":
            s.autotune(8)
        configs.append(s.config())
        solvers.append(s)
    for s in solvers:
        for _ in range(W_):
            s.step(method)
        s.set_state(None)      # back to zero initial flux and a fresh first iterate
    infos = torch.zeros((len(solvers), K, 24), dtype=torch.uint8, device=solvers[0].dev)
    phis = [torch.empty((K,) + tuple(s.phi.shape), dtype=torch.float64, device=s.dev) for s in solvers]
    for s in solvers:
        B.oci_profile_enable(s.h, True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    if method == "oci":
        # K time steps per problem in one call (one launch on the
        # register-resident kernel, K oci_step launches otherwise)
        for i, s in enumerate(solvers):
            B.oci_run_steps(s.h, K, s.q, s.inc_l, s.inc_r, phis[i], None, infos[i])
    else:
        for k in range(K):
            for i, s in enumerate(solvers):
                B.si_step(s.h, s.q, s.inc_l, s.inc_r, phis[i][k], None, infos[i, k])
    ev1.record()
    torch.cuda.synchronize()
    gpu_ms = ev0.elapsed_time(ev1)
    kern = [B.oci_profile_read(s.h) for s in solvers]            # (ms, steps) per problem
    launches = [1 if (method == "oci" and c["local"] and c["resident"]) else K for c in configs]
    inf = infos.cpu().numpy()
    dec = [[B.decode_info(inf[i, k]) for i in range(len(solvers))] for k in range(K)]
    for s in solvers:
        s.close()
    its = np.array([[d["iterations"] for d in row] for row in dec])       # [K][problems]
    status = sorted({d["status"] for row in dec for d in row})
    cell_solves = int(sum(its[:, i].sum() * p["J"] for i, p in enumerate(probs)))
    per = [dict(dt=p["dt"], setup_s=setup_s[i], iterations_per_step=float(its[:, i].mean()),
                iterations_max=int(its[:, i].max())) for i, p in enumerate(probs)]
    return dict(time_s=max(gpu_ms / 1e3, 1e-12), cell_solves=cell_solves, per=per, status=status,
                kernel=kern, launches=launches, configs=configs,
                setup=setup_model(probs, setup_s, precision == B.OCI_FP32_REFINED))


def summary(r, label, K, keys):
    """Per-method figures; seconds per converged step per problem come from the
    iteration-kernel events of that problem."""
    return dict(cell_solves_per_s=r["cell_solves"] / r["time_s"],
                s_per_converged_step={k: ms / 1e3 / max(cnt, 1) for (ms, cnt), k in zip(r["kernel"], keys)},
                iterations_per_step={k: x["iterations_per_step"] for x, k in zip(r["per"], keys)},
                setup_s={k: round(x["setup_s"], 4) for x, k in zip(r["per"], keys)},
                timed_region_s=round(r["time_s"], 6), ms_per_bench_step=round(r["time_s"] * 1e3 / K, 4),
                kernel_ms=round(sum(k[0] for k in r["kernel"]), 3), status=r["status"],
                launch_shape=r["configs"][0], label=label, setup=r["setup"])


def recorded_traffic(label, summary="pmc_traffic_regions4096.md", figure="HBM bytes per cell-iteration"):
    """A traffic figure of `label` from a committed PMC summary (HBM bytes per
    cell-iteration, or per algorithmic byte), valid only while the kernel
    source is the one the counters were taken on."""
    src = os.path.join(ROOT, "paper_2503_00264_amd", "csrc", "oci_step.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source sha256\[:16\]: `([0-9a-f]+)`", text)
    k = re.search(r"kernel: `([^`]+)`", text)
    t = re.search(re.escape(figure) + r": ([0-9.]+)", text)
    if not (m and k and t) or m.group(1) != digest or k.group(1) != label:
        return None
    return float(t.group(1))


def padded(n):
    np_ = 8
    while np_ < n:
        np_ *= 2
    return np_


def setup_model(probs, setup_s, fp32):
    """Cell inversion at setup: 2 np^3 flops per cell (LU + inversion, or the
    same count as blocked Gauss-Jordan), over the wall time of oci_setup
    (uploads, assembly, inversion and the SI precompute).  Cells with
    np >= 128 run the MFMA kernel; its peak is the matrix peak of the type."""
    flop = sum(2.0 * padded(4 * p["N"] * p["G"]) ** 3 * p["J"] for p in probs)
    secs = float(sum(setup_s))
    tf = flop / max(secs, 1e-12) / 1e12
    peak = MI355X_FP32_TFLOPS if fp32 else MI355X_FP64_TFLOPS
    nps = sorted({padded(4 * p["N"] * p["G"]) for p in probs})
    t = "float" if fp32 else "double"
    kern = [f"k_gj_invert<{t},{32 if fp32 else 16},{512 if q >= 512 else 256}>" if q >= 128
            else f"k_assemble_factor<{t}>" for q in nps]
    return dict(bound="mfma" if nps[-1] >= 128 else "alu", achieved=round(tf, 3), peak=peak, unit="TFLOP/s",
                frac=round(tf / peak, 4),
                seconds=round(secs, 4), flop=flop, kernels=kern,
                note="wall time of oci_setup (host uploads and synchronisation included)")


def roofline_for(prim, probs, fp32, workload=None):
    """Roofline of the dominant kernel (the persistent OCI kernel of the
    measured path: one launch per problem for all K steps when its rows are
    register-resident, one per time step otherwise).

    Streamed inverse rows: bound by memory; algorithmic bytes per
    cell-iteration are the factor stream plus iterate, edge, source and flux
    traffic, 4 n^2 + 4 n + 128 N G + 64 G (FP32 factors) or
    8 n^2 + 4 n + 96 N G + 64 G (FP64), against the HBM peak.

    Register-resident rows (k_oci_res): the factor stream is gone (the rows
    are loaded once per launch) and the kernel is bound by VALU issue; the
    algorithmic work is the 2 n^2 flops per cell-iteration of the inverse
    product, against the FP32 vector peak.  The stream model's figure is kept
    beside it (`stream_model`)."""
    p = probs[0]
    N, G = p["N"], p["G"]
    n = 4 * N * G
    np_ = padded(n)
    kern_ms = sum(k[0] for k in prim["kernel"])
    launches = sum(prim["launches"])
    avg_launch_s = kern_ms / 1e3 / max(launches, 1)
    bpc = (4 * n * n + 4 * n + 128 * N * G + 64 * G) if fp32 else (8 * n * n + 4 * n + 96 * N * G + 64 * G)
    fpc = 2 * n * n
    cpl = prim["cell_solves"] / max(launches, 1)
    gbs = bpc * cpl / avg_launch_s / 1e9
    tflops = fpc * cpl / avg_launch_s / 1e12
    label = kernel_label(prim["configs"][0], fp32, np_)
    if prim["configs"][0].get("resident"):
        tr = recorded_traffic(label)
        traffic = None if tr is None else round(tr * cpl, 1)
    else:
        # streamed rows: the counters' HBM bytes per algorithmic byte for this
        # kernel on this workload, if a summary for it is committed
        name = label.split("<")[0]
        ratio = recorded_traffic(label, f"{name}_{workload}.md", "HBM bytes per algorithmic byte") if workload else None
        traffic = None if ratio is None else round(ratio * bpc * cpl, 1)
    common = dict(kernel=label, avg_launch_us=round(avg_launch_s * 1e6, 2),
                  cell_iterations_per_launch=round(cpl, 1), bytes_per_cell_iteration=bpc,
                  flops_per_cell_iteration=fpc)
    if prim["configs"][0].get("resident"):
        peak = MI355X_FP32_TFLOPS if fp32 else MI355X_FP64_TFLOPS
        return dict(bound="alu", achieved=round(tflops, 3), peak=peak, unit="TFLOP/s",
                    frac=round(tflops / peak, 4), traffic=traffic,
                    note="inverse rows held in VGPRs for the whole step; bound by VALU issue "
                         "(the FP64 residual, reductions and address arithmetic beside the "
                         "2 n^2-flop product); traffic = HBM bytes per launch from the PMC counters",
                    stream_model=dict(achieved=round(gbs, 1), peak=MI355X_HBM_GBS, unit="GB/s",
                                      frac=round(gbs / MI355X_HBM_GBS, 4)),
                    **common)
    return dict(bound="hbm", achieved=round(gbs, 1), peak=MI355X_HBM_GBS, unit="GB/s",
                frac=round(gbs / MI355X_HBM_GBS, 4), traffic=traffic,
                note="inverse rows streamed from memory every iteration",
                achieved_tflops=round(tflops, 3), **common)


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
                       f"(J={prob['J']}, n={4 * prob['N'] * prob['G']}: {its} iterations x {prob['J']} "
                       f"cells, {dt:.1f} s, setup excluded)")


def run_batch(probs, K, W_, tol, torch, B, precision):
    """The batched launch: K steps captured once into a graph, timed replay."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bs = B.BatchSolver(probs, precision=precision, tol=tol)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    for _ in range(max(W_, 1)):
        bs.step()
    bs.rebalance()             # workgroups per slab from the measured iteration counts
    for k in range(len(probs)):
        bs.set_state(k, None)
    bs.capture(K)
    bs.stream.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(bs.stream)
    bs.replay()
    ev1.record(bs.stream)
    _, infos = bs.results()
    ms = ev0.elapsed_time(ev1)
    geo = bs.geometry()
    bs.close()
    # iterations of the last step per slab are in the infos; the total count
    # of the K steps comes from a second, eager pass with per-step infos
    return dict(time_s=ms / 1e3, setup_s=setup, infos=infos, geometry=geo)


def batch_main(a, torch, B):
    from paper_2503_00264_amd import workloads as W
    probs = W.config("batch64", n_slabs=a.slabs, steps=a.steps)
    K = a.steps
    # eager pass with per-step infos gives the iteration counts of every step
    bs = B.BatchSolver(probs, precision=B.OCI_FP32_REFINED, tol=a.tol)
    bs.step()
    bs.rebalance()
    for k in range(len(probs)):
        bs.set_state(k, None)
    its = np.zeros((K, len(probs)), dtype=np.int64)
    status = set()
    for k in range(K):
        bs.step()
        _, infos = bs.results()
        its[k] = [i["iterations"] for i in infos]
        status |= {i["status"] for i in infos}
    bs.close()
    torch.cuda.empty_cache()
    r = run_batch(probs, K, a.warmup, a.tol, torch, B, B.OCI_FP32_REFINED)
    J = np.array([p["J"] for p in probs])
    cell_solves = int((its * J[None, :]).sum())
    value = cell_solves / r["time_s"]
    # factor stream of the batched kernel: each slab's FP32-refined bytes per
    # cell-iteration (as for one slab) times its cell-iterations, over the
    # replayed graph's time (the small per-step kernels included)
    bpc = np.array([4 * n * n + 4 * n + 128 * p["N"] * p["G"] + 64 * p["G"]
                    for p, n in ((p, 4 * p["N"] * p["G"]) for p in probs)], dtype=np.float64)
    alg_bytes = float((its * J[None, :] * bpc[None, :]).sum())
    gbs = alg_bytes / r["time_s"] / 1e9
    ratio = recorded_traffic("k_oci_batch<float,256>", "k_oci_batch_batch64.md", "HBM bytes per algorithmic byte")
    traffic = None if ratio is None else round(ratio * alg_bytes / K, 1)
    out = {
        "metric": "cell-solves/s and s per converged step: FP32-refined vs FP64 OCI vs SI @1e-10",
        "value": round(value, 1), "unit": "cell-solves/s", "n_gpus": 1, "steps": K, "warmup": a.warmup,
        "ms_per_step": round(r["time_s"] * 1e3 / K, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 solve + f64 residual/norm/update",
        "data": "synthetic (seeded generator; no external data)",
        "config": {"workload": f"batch64: {len(probs)} slabs, J in [{J.min()}, {J.max()}], "
                               f"n in {sorted({4 * p['N'] * p['G'] for p in probs})}, dt 1e-3, "
                               f"{K} graph-captured batched steps", "slabs": len(probs),
                   "cells": int(J.sum())},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": MI355X_HBM_GBS, "unit": "GB/s",
                     "frac": round(gbs / MI355X_HBM_GBS, 4), "traffic": traffic, "kernel": "k_oci_batch<float,256>",
                     "avg_launch_us": round(r["time_s"] / K * 1e6, 1),
                     "note": "algorithmic factor-stream bytes of every slab's cell-iterations over the "
                             "replayed graph time (per-step bookkeeping kernels included)"},
        "batch": {"setup_s": round(r["setup_s"], 3), "workgroups": r["geometry"][0],
                  "iterations_per_step_max": int(its.max()), "status": sorted(status),
                  "setup": setup_model(probs, [r["setup_s"]], True)},
    }
    if not a.no_comparators:
        t_seq = 0.0
        cs_seq = 0
        for p in probs:
            s = B.Solver(p, precision=B.OCI_FP64, tol=a.tol)
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record()
            infos = []
            for _ in range(K):
                s.step("oci")
                infos.append(s.info.clone())
            ev1.record()
            torch.cuda.synchronize()
            t_seq += ev0.elapsed_time(ev1) / 1e3
            cs_seq += sum(B.decode_info(i.cpu().numpy())["iterations"] for i in infos) * p["J"]
            s.close()
            torch.cuda.empty_cache()
        out["comparison"] = {"fp64_sequential": {"time_s": round(t_seq, 4),
                                                 "cell_solves_per_s": cs_seq / t_seq,
                                                 "speedup_of_batched_fp32": round(t_seq / r["time_s"], 3)}}
    print(json.dumps(out), flush=True)


ROSA_DELTAS = (10.0, 4.0, 1.0, 0.4, 0.1, 0.04, 0.01)
ROSA_ORDERS = (8, 16, 32)
ROSA_DTS = (10.0, 0.1)


def rosa_main(a, torch, B):
    """The delta / quadrature / time-step sweep of the two-group problem."""
    from paper_2503_00264_amd import workloads as W
    K = a.steps
    rows = []
    cs_ref = 0
    t_ref = 0.0
    for dt in ROSA_DTS:
        for N in ROSA_ORDERS:
            for delta in ROSA_DELTAS:
                J = max(1, int(round(W.ROSA_SIGMA_MIN * W.ROSA_LENGTH / delta)))
                probs = [W.rosa(J=J, N=N, dt=dt, steps=K)]
                tune = not a.no_autotune
                r64 = run_method(probs, "oci", B.OCI_FP64, K, a.warmup, a.tol, torch, B, tune)
                rrf = run_method(probs, "oci", B.OCI_FP32_REFINED, K, a.warmup, a.tol, torch, B, tune)
                rsi = run_method(probs, "si", B.OCI_FP64, K, a.warmup, a.tol, torch, B, False)
                torch.cuda.empty_cache()
                cs_ref += rrf["cell_solves"]
                t_ref += rrf["time_s"]
                row = {"dt": dt, "N": N, "n": 8 * N, "delta": round(W.ROSA_SIGMA_MIN * W.ROSA_LENGTH / J, 5),
                       "J": J, "oci_fp64_s": round(r64["time_s"], 6), "oci_refined_s": round(rrf["time_s"], 6),
                       "si_s": round(rsi["time_s"], 6),
                       "oci_iterations_per_step": r64["per"][0]["iterations_per_step"],
                       "si_iterations_per_step": rsi["per"][0]["iterations_per_step"],
                       "speedup_fp64_oci_over_si": round(rsi["time_s"] / r64["time_s"], 3),
                       "speedup_refined_oci_over_si": round(rsi["time_s"] / rrf["time_s"], 3),
                       "status": sorted(set(r64["status"]) | set(rrf["status"]) | set(rsi["status"]))}
                rows.append(row)
                print(f"[rosa] dt={dt} S{N} delta={row['delta']} J={J}: OCI fp64 {row['oci_fp64_s'] * 1e3:.2f} ms "
                      f"refined {row['oci_refined_s'] * 1e3:.2f} ms SI {row['si_s'] * 1e3:.2f} ms "
                      f"({row['oci_iterations_per_step']:.0f} / {row['si_iterations_per_step']:.0f} iterations)",
                      file=sys.stderr, flush=True)
    best = {}
    for dt in ROSA_DTS:
        for N in ROSA_ORDERS:
            sel = [r for r in rows if r["dt"] == dt and r["N"] == N]
            top = max(sel, key=lambda r: r["speedup_fp64_oci_over_si"])
            best[f"dt={dt} S{N}"] = {"delta": top["delta"], "speedup_fp64_oci_over_si": top["speedup_fp64_oci_over_si"]}
    out = {
        "metric": "convergence-loop seconds over the delta sweep: FP64 OCI, FP32-refined OCI and SI @tol",
        "value": round(cs_ref / max(t_ref, 1e-12), 1), "unit": "cell-solves/s", "n_gpus": 1, "steps": K,
        "warmup": a.warmup, "ms_per_step": round(t_ref * 1e3 / K, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 (OCI, SI); f32 solve + f64 residual (refined)",
        "data": "synthetic (the paper's two-group material table; no external data)",
        "config": {"workload": f"rosa: two groups, L = 100 cm, S_N in {list(ROSA_ORDERS)}, "
                               f"delta = Sigma_2 dx in {list(ROSA_DELTAS)}, dt in {list(ROSA_DTS)} s, "
                               f"{K} steps each, tol {a.tol}", "tol": a.tol},
        "roofline": None,
        "sweep": rows,
        "best_delta": best,
    }
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    from paper_2503_00264_amd import binding as B
    torch.cuda.set_device(0)
    if a.workload == "batch64":
        batch_main(a, torch, B)
        return
    if a.workload == "rosa":
        rosa_main(a, torch, B)
        return
    base, probs = problems(a.workload)
    N, G, J = base["N"], base["G"], base["J"]
    n = 4 * N * G
    keys = [str(p["dt"]) for p in probs]
    tune = not a.no_autotune
    prim = run_method(probs, "oci", B.OCI_FP32_REFINED, a.steps, a.warmup, a.tol, torch, B, tune)
    comp = {}
    if not a.no_comparators:
        comp["fp64"] = run_method(probs, "oci", B.OCI_FP64, a.steps, a.warmup, a.tol, torch, B, tune)
        comp["si"] = run_method(probs, "si", B.OCI_FP64, a.steps, a.warmup, a.tol, torch, B, False)
    value = prim["cell_solves"] / prim["time_s"]
    out = {
        "metric": "cell-solves/s and s per converged step: FP32-refined vs FP64 OCI vs SI @1e-10",
        "value": round(value, 1),
        "unit": "cell-solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(prim["time_s"] * 1e3 / a.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 solve + f64 residual/norm/update",
        "data": "synthetic (seeded generator; no external data)",
        "config": {"workload": f"{a.workload}: J={J} N={N} G={G} n={n}, dt {keys}, tol {a.tol}, "
                               f"one step = one converged time step of each dt",
                   "J": J, "N": N, "G": G, "n": n, "dts": [p["dt"] for p in probs], "tol": a.tol},
        "roofline": roofline_for(prim, probs, True, a.workload),
        "comparison": {"fp32_refined": summary(prim, "FP32 LU+inverse, FP64 residual refinement", a.steps, keys)},
    }
    labels = {"fp64": "FP64 LU+inverse OCI", "si": "FP64 source iteration sweep"}
    for k, r in comp.items():
        out["comparison"][k] = summary(r, labels[k], a.steps, keys)
    if "fp64" in comp:
        out["comparison"]["fp64"]["roofline"] = roofline_for(comp["fp64"], probs, False, a.workload)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(probs[0], a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
