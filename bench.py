#!/usr/bin/env python
"""Benchmark: cell-solves/s and seconds per converged time step at tol 1e-10,
FP32-refined OCI against FP64 OCI and GPU source iteration, on one MI355X.

Default workload "batch64", the largest single-GPU configuration: 64
independent slabs (slab i drawn from numpy's PCG64 with seed [5, i]: J ~
U{256..8192} cells of 1/64 cm, S_N with N in {8, 16, 32}, G in {1, 2, 4}
groups, so cell systems of n = 4NG = 32 .. 512 unknowns; 64 random regions
per slab with the one-group or multigroup material rules; Q = 1 in the first
eighth of the regions; vacuum; zero initial flux; dt = 1e-3 s), 291943 cells
in all, advanced together by the batched persistent FP32-refined launch.  W
eager warm-up steps and the per-slab workgroup rebalance come first; then the
state is reset and K time steps, captured once into a HIP graph, are replayed
and timed (events on the batch's stream).  One benchmark step = one converged
time step of every slab.  Each step's iteration counts come from the per-step
argument sets the graph writes.  Comparators on the same GPU: the 64 slabs
solved one after another in plain FP64 OCI, and by GPU source iteration, K
steps each.  Comparison workloads (not the headline): the 4096-cell one-group
slab over its dt sweep and the 16384-cell four-group slab (FP32-refined,
FP64 and SI each).

Other workloads, one each: "regions4096" (one converged step of each problem
of the dt sweep per benchmark step), "homogeneous64", "multigroup8192",
"multigroup16384", and "rosa": the two-group, highly scattering performance
problem of section 3.2 (table rosa_test) swept over the cell optical
thickness, S8 / S16 / S32 and dt = 10 s / 0.1 s.

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
MI355X_FP32_TFLOPS = 157.3    # published FP32 peak (packed vector; FP32 matrix: the same figure)
MI355X_FP64_TFLOPS = 78.6     # published FP64 vector peak (FP64 matrix: the same figure)
# FP32 vector issue without packed instructions (the library is built with
# them disabled): 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz
MI355X_FP32_VALU_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch64")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU-oracle sample")
    ap.add_argument("--no-comparators", action="store_true")
    ap.add_argument("--comparators", default="dense,sequential,red_black",
                    help="batch64: which comparisons to run (dense, sequential, red_black)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--slabs", type=int, default=64, help="batch64: number of slabs")
    ap.add_argument("--no-comparison-workloads", action="store_true",
                    help="batch64: skip the 4096- and 16384-cell comparison workloads")
    ap.add_argument("--cpu-child", default=None, help=argparse.SUPPRESS)
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


def run_method(probs, method, precision, K, W_, tol, torch, B, autotune=True, solver=0):
    """Set up one solver per problem, tune, warm up, reset, then time K steps."""
    solvers, setup_s, configs = [], [], []
    B.Solver(probs[0], precision=precision, tol=tol, solver=solver).close()   # first-use costs out of the setup times
    for p in probs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = B.Solver(p, precision=precision, tol=tol, solver=solver)
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
                setup=setup_model(probs, setup_s, precision == B.OCI_FP32_REFINED) if solver == 0 else
                dict(seconds=round(float(sum(setup_s)), 4), note="structured setup: closed-form corner "
                     "inverses and one 2G x 2G complex capacitance inverse per cell"))


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


DENSE_SOURCES = ("oci_step.hip", "oci_device.hpp")
STRUCTURED_SOURCES = ("oci_wb.hip", "oci_device.hpp")


def source_digest(sources):
    """sha256[:16] over the named kernel sources, in order."""
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, "paper_2503_00264_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic(label, summary="pmc_traffic_regions4096.md", figure="HBM bytes per cell-iteration",
                     sources=DENSE_SOURCES):
    """A traffic figure of `label` from a committed PMC summary (HBM bytes per
    cell-iteration, or per algorithmic byte), valid only while the kernel
    sources are the ones the counters were taken on."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source sha256\[:16\]: `([0-9a-f]+)`", text)
    k = re.search(r"kernel: `([^`]+)`", text)
    t = re.search(re.escape(figure) + r": ([0-9.]+)", text)
    if not (m and k and t) or m.group(1) != source_digest(sources) or k.group(1) != label:
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
        peak = MI355X_FP32_VALU_TFLOPS if fp32 else MI355X_FP64_TFLOPS
        return dict(bound="alu", achieved=round(tflops, 3), peak=peak, unit="TFLOP/s",
                    frac=round(tflops / peak, 4), traffic=traffic,
                    note="inverse rows held in VGPRs for the whole step; bound by VALU issue "
                         "(the FP64 residual, reductions and address arithmetic beside the "
                         "2 n^2-flop product); peak = non-packed FP32 (or FP64) vector issue; "
                         "traffic = HBM bytes per launch from the PMC counters",
                    stream_model=dict(achieved=round(gbs, 1), peak=MI355X_HBM_GBS, unit="GB/s",
                                      frac=round(gbs / MI355X_HBM_GBS, 4)),
                    **common)
    return dict(bound="hbm", achieved=round(gbs, 1), peak=MI355X_HBM_GBS, unit="GB/s",
                frac=round(gbs / MI355X_HBM_GBS, 4), traffic=traffic,
                note="inverse rows streamed from memory every iteration",
                achieved_tflops=round(tflops, 3), **common)


def host_cpu():
    """CPU model, logical CPUs of the host and the ones this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def cpu_baseline(prob, seconds):
    """The FP64 oracle (OpenMP) on a bounded sample of one problem."""
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
    model, ncpu, _ = host_cpu()
    return dict(value=its * prob["J"] / dt, unit="cell-solves/s", cores=threads, kind="oracle",
                cpu_model=model, host_cpus=ncpu,
                sample=f"first {steps} converged time step(s) of the dt={prob['dt']} problem "
                       f"(J={prob['J']}, n={4 * prob['N'] * prob['G']}: {its} iterations x {prob['J']} "
                       f"cells, {dt:.1f} s, setup excluded)")


def oracle_seconds_per_cell_iteration(slabs, iters):
    """Seconds per cell-iteration of the oracle's OCI iteration (setup
    excluded), one entry per slab: `iters` fixed iterations of its first step."""
    import oracle
    out = []
    for p in slabs:
        o = oracle.Oracle(dict(p), methods=("oci",))
        pp, pi = o.initial_state()
        t0 = time.perf_counter()
        o.step("oci", pp, pi, q=p["q"], fixed_iters=iters)
        out.append((time.perf_counter() - t0) / (iters * p["J"]))
        del o
    return out


def batch_cpu_baseline(probs, its, seconds):
    """The oracle on a bounded sample of the batch: for each cell size n of the
    batch, the slab of that n with the fewest cells runs a fixed number of OCI
    iterations of its first step on every host thread, giving seconds per
    cell-iteration at that n; the batch's measured cell-iterations (per slab,
    all K steps) priced at those rates give the oracle's time for the whole
    workload, and value = the batch's cell-solves over that time.  The same
    sample on one thread (a child process with OMP_NUM_THREADS=1, fewer
    iterations) gives the one-core figure."""
    import subprocess
    model, ncpu, usable = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", usable))
    by_n = {}
    for k, p in enumerate(probs):
        n = 4 * p["N"] * p["G"]
        if n not in by_n or p["J"] < probs[by_n[n]]["J"]:
            by_n[n] = k
    ns = sorted(by_n)
    sample = [by_n[n] for n in ns]
    cell_its = its.sum(axis=0) * np.array([p["J"] for p in probs])   # per slab, all steps

    def priced(rates):
        rate_n = dict(zip(ns, rates))
        return float(sum(ci * rate_n[4 * p["N"] * p["G"]] for ci, p in zip(cell_its, probs)))

    # size the fixed iteration count to the budget from one quick probe
    probe = oracle_seconds_per_cell_iteration([probs[k] for k in sample], 2)
    per_iter = sum(r * probs[k]["J"] for r, k in zip(probe, sample))
    iters = int(max(2, min(200, seconds / max(per_iter, 1e-9))))
    t0 = time.perf_counter()
    rates = oracle_seconds_per_cell_iteration([probs[k] for k in sample], iters)
    wall = time.perf_counter() - t0
    total = priced(rates)
    out = dict(value=round(float(cell_its.sum()) / total, 1), unit="cell-solves/s", cores=threads,
               kind="oracle", cpu_model=model, host_cpus=ncpu, usable_cpus=usable,
               sample=f"{iters} fixed OCI iterations of the first step of one slab per cell size "
                      f"(slabs {sample}, n = {ns}, J = {[probs[k]['J'] for k in sample]}; {wall:.1f} s), "
                      f"setup excluded; the batch's measured cell-iterations priced at the sampled "
                      f"seconds per cell-iteration of their n ({total:.1f} s for the whole workload)",
               seconds_per_cell_iteration={str(n): r for n, r in zip(ns, rates)})
    iters1 = max(2, iters // max(threads, 1))
    arg = json.dumps(dict(slabs=sample, iters=iters1, n_slabs=len(probs)))
    env = dict(os.environ, OMP_NUM_THREADS="1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-child", arg], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode == 0:
        rates1 = json.loads(r.stdout.strip().splitlines()[-1])
        total1 = priced(rates1)
        out["one_core"] = dict(value=round(float(cell_its.sum()) / total1, 1), unit="cell-solves/s", cores=1,
                               sample=f"the same slabs, {iters1} iterations each, one thread",
                               seconds_per_cell_iteration={str(n): x for n, x in zip(ns, rates1)})
    else:
        out["one_core"] = dict(error=r.stderr.strip().splitlines()[-1:] or ["failed"])
    return out


def cpu_child(arg):
    """One-thread oracle sample (runs in a child process; no GPU)."""
    from paper_2503_00264_amd import workloads as W
    a = json.loads(arg)
    probs = W.config("batch64", n_slabs=a["n_slabs"], steps=1)
    print(json.dumps(oracle_seconds_per_cell_iteration([probs[k] for k in a["slabs"]], a["iters"])), flush=True)


def batch_step_bytes(probs, fp32=True):
    """Algorithmic bytes per cell-iteration of each slab (the factor stream of
    its cell size plus iterate, edge, source and flux traffic)."""
    return np.array([(4 * n * n + 4 * n + 128 * p["N"] * p["G"] + 64 * p["G"]) if fp32 else
                     (8 * n * n + 4 * n + 96 * p["N"] * p["G"] + 64 * p["G"])
                     for p, n in ((p, 4 * p["N"] * p["G"]) for p in probs)], dtype=np.float64)


def run_batch_graph(probs, K, W_, tol, torch, B, precision, solver=0, ordering=0):
    """The batched launch: W eager warm-up steps and the rebalance, then the
    state reset and K steps captured once into a graph, replayed and timed.
    Returns per-step iteration counts [K][slab] from the graph's own records."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bs = B.BatchSolver(probs, precision=precision, tol=tol, solver=solver, ordering=ordering)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    bs.bind_steps(K)
    for _ in range(max(W_, 1)):
        bs.step()
        bs.rebalance()         # workgroups per slab from the last step's iterations (and device times)
    for k in range(len(probs)):
        bs.set_state(k, None)
    bs.bind_steps(K)           # fresh argument sets, graph step i writes set i
    bs.capture(K)
    bs.stream.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(bs.stream)
    bs.replay()
    ev1.record(bs.stream)
    _, infos = bs.step_results()
    ms = ev0.elapsed_time(ev1)
    geo = bs.geometry()
    bs.close()
    its = np.array([[i["iterations"] for i in row] for row in infos], dtype=np.int64)
    status = sorted({i["status"] for row in infos for i in row})
    return dict(time_s=ms / 1e3, setup_s=setup, its=its, status=status, geometry=geo)


def sequential(probs, K, tol, torch, B, method, precision):
    """The slabs solved one after another, K eager steps each, each slab's
    steps timed with events; returns total seconds and cell-solves."""
    t_tot = 0.0
    cs = 0
    its = []
    for p in probs:
        s = B.Solver(p, precision=precision, tol=tol)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        infos = []
        for _ in range(K):
            s.step(method)
            infos.append(s.info.clone())
        ev1.record()
        torch.cuda.synchronize()
        t_tot += ev0.elapsed_time(ev1) / 1e3
        n_it = [B.decode_info(i.cpu().numpy())["iterations"] for i in infos]
        its.append(n_it)
        cs += sum(n_it) * p["J"]
        s.close()
        torch.cuda.empty_cache()
    its = np.array(its).T
    return dict(time_s=round(t_tot, 4), s_per_converged_step=round(t_tot / K, 5), cell_solves_per_s=cs / t_tot,
                iterations_per_step_max=int(its.max()), iterations_per_step_mean=round(float(its.mean()), 2))


def wb_staged_shape(J, N, G):
    """The library's shape rule for the staged structured body: N a power of
    two in 8..64, G in {1, 2, 4}, at most two (g, m) pairs per lane, a wave's
    rows of (I - W C)^-1 within 2 KiB and its per-cell data within 1 KiB,
    32-bit byte offsets.  A batch runs the staged body when every slab has
    such a shape."""
    if N < 8 or N > 64 or N & (N - 1) or G not in (1, 2, 4) or N * G > 128:
        return False
    lc = 1
    while lc < N * G:
        lc <<= 1
    cpw = 64 // min(lc, 64)
    return cpw * 4 * G * G <= 128 and cpw * G <= 8 and J * N * G * 32 < 2 ** 31


def batch_structured_bytes(probs):
    """Algorithmic bytes per cell-iteration of the structured solve, FP64
    words: psi_{k-1/2} (2NG), the incident and the outgoing corners (2NG
    each), the source (4G), the scalar flux read and written (4G each), the
    cell's cross sections and width (G^2 + G + 1), and its capacitance rows:
    the (2G)^2 complex words of (I - W C)^-1 for the staged body (which forms
    C t from Sigma_s), twice that for the direct body (which also reads the
    rows of C (I - W C)^-1)."""
    staged = all(wb_staged_shape(p["J"], p["N"], p["G"]) for p in probs)
    rows = 64 if staged else 128   # bytes per G^2
    return np.array([8 * (6 * p["N"] * p["G"] + 12 * p["G"] + p["G"] ** 2 + p["G"] + 1) + rows * p["G"] ** 2
                     for p in probs], dtype=np.float64)


def batch_graph_summary(r, probs, K, bytes_per_cell, label, extra=None):
    """Figures of one batched graph run: cell-solves/s, seconds per converged
    step, iterations, and the HBM roofline of its algorithmic bytes."""
    J = np.array([p["J"] for p in probs])
    cs = int((r["its"] * J[None, :]).sum())
    alg = float((r["its"] * J[None, :] * bytes_per_cell[None, :]).sum())
    gbs = alg / r["time_s"] / 1e9
    out = dict(time_s=round(r["time_s"], 4), s_per_converged_step=round(r["time_s"] / K, 5),
               cell_solves_per_s=cs / r["time_s"], cell_solves=cs, iterations_per_step_max=int(r["its"].max()),
               iterations_per_step_mean=round(float(r["its"].mean()), 2), status=r["status"],
               setup_s=round(r["setup_s"], 3), workgroups=r["geometry"][0],
               roofline={"bound": "hbm", "achieved": round(gbs, 1), "peak": MI355X_HBM_GBS, "unit": "GB/s",
                         "frac": round(gbs / MI355X_HBM_GBS, 4), "traffic": None, "kernel": label,
                         "avg_launch_us": round(r["time_s"] / K * 1e6, 1), "bytes_per_step": round(alg / K, 1)})
    if extra:
        out.update(extra)
    return out


def batch_main(a, torch, B):
    """The 64-slab batch.  Headline: the batched OCI iteration with the
    structured exact cell solve (FP64), K graph-captured steps.  Comparisons:
    the dense FP32-refined batched launch, plain FP64 OCI and GPU SI slab by
    slab, and the structured solve with red-black ordering."""
    from paper_2503_00264_amd import workloads as W
    probs = W.config("batch64", n_slabs=a.slabs, steps=a.steps)
    K = a.steps
    J = np.array([p["J"] for p in probs])
    r = run_batch_graph(probs, K, a.warmup, a.tol, torch, B, B.OCI_FP64, B.OCI_SOLVE_STRUCTURED)
    head = batch_graph_summary(r, probs, K, batch_structured_bytes(probs), "k_wb_batch<256,true>")
    roof = head.pop("roofline")
    ratio = recorded_traffic("k_wb_batch<256,true>", "k_wb_batch_batch64.md", "HBM bytes per algorithmic byte",
                             STRUCTURED_SOURCES)
    roof["traffic"] = None if ratio is None else round(ratio * roof["bytes_per_step"], 1)
    roof["note"] = ("algorithmic bytes of the structured solve per cell-iteration (psi_{k-1/2}, incident "
                    "and outgoing corners, source, scalar flux read and written, cross sections and width, "
                    "the rows of (I - W C)^-1 the staged body reads) times each slab's cell-iterations, over "
                    "the replayed graph's time per step (the per-step bookkeeping kernels included); traffic = "
                    "the committed counters' HBM bytes per algorithmic byte times this run's algorithmic bytes")
    out = {
        "metric": "cell-solves/s and s per converged step: FP32-refined vs FP64 OCI vs SI @1e-10",
        "value": round(head["cell_solves_per_s"], 1), "unit": "cell-solves/s", "n_gpus": 1, "steps": K,
        "warmup": a.warmup, "ms_per_step": round(r["time_s"] * 1e3 / K, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generator; no external data)",
        "config": {"workload": f"batch64: {len(probs)} independent slabs, {int(J.sum())} cells, J in "
                               f"[{J.min()}, {J.max()}], N in {{8,16,32}}, G in {{1,2,4}}, "
                               f"n = 4NG in {sorted({4 * p['N'] * p['G'] for p in probs})}, dt 1e-3 s, "
                               f"tol {a.tol}; one step = one converged time step of every slab, "
                               f"{K} steps captured in one HIP graph",
                   "method": "OCI (cell-wise block Jacobi), each cell system solved exactly through its "
                             "structure (closed-form corner blocks, rank-4G scattering coupling), FP64, "
                             "all slabs in one persistent launch per step",
                   "slabs": len(probs), "cells": int(J.sum()), "tol": a.tol},
        "roofline": roof,
        "s_per_converged_step": head["s_per_converged_step"],
        "batch": head,
    }
    which = set() if a.no_comparators else set(a.comparators.split(","))
    if which:
        comp = out["comparison"] = {}
    if "dense" in which:
        print("[bench] comparator: dense FP32-refined batched", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        rd = run_batch_graph(probs, K, a.warmup, a.tol, torch, B, B.OCI_FP32_REFINED)
        dense = batch_graph_summary(rd, probs, K, batch_step_bytes(probs, True), "k_oci_batch<float,256>",
                                    dict(setup=setup_model(probs, [rd["setup_s"]], True)))
        ratio = recorded_traffic("k_oci_batch<float,256>", "k_oci_batch_batch64.md",
                                 "HBM bytes per algorithmic byte")
        dense["roofline"]["traffic"] = (None if ratio is None else
                                        round(ratio * dense["roofline"]["bytes_per_step"], 1))
        dense["speedup_of_structured"] = round(rd["time_s"] / r["time_s"], 3)
        comp["dense_fp32_refined_batched"] = dense
    if "sequential" in which:
        print("[bench] comparators: FP64 OCI and GPU SI, slab by slab", file=sys.stderr, flush=True)
        fp64 = sequential(probs, K, a.tol, torch, B, "oci", B.OCI_FP64)
        fp64["speedup_of_structured"] = round(fp64["time_s"] / r["time_s"], 3)
        si = sequential(probs, K, a.tol, torch, B, "si", B.OCI_FP64)
        si["speedup_of_structured"] = round(si["time_s"] / r["time_s"], 3)
        comp["dense_fp64_sequential"] = fp64
        comp["si_sequential"] = si
    if "red_black" in which:
        print("[bench] comparator: structured red-black, batched", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        rr = run_batch_graph(probs, K, a.warmup, a.tol, torch, B, B.OCI_FP64, B.OCI_SOLVE_STRUCTURED,
                             B.OCI_ORDER_RED_BLACK)
        rb = batch_graph_summary(rr, probs, K, batch_structured_bytes(probs), "k_wb_batch<256,true>")
        rb["speedup_over_jacobi"] = round(r["time_s"] / rr["time_s"], 3)
        comp["structured_red_black_batched"] = rb
    if not a.no_comparison_workloads:
        print("[bench] comparison workloads: regions4096 and multigroup16384", file=sys.stderr, flush=True)
        cw = out.setdefault("comparison_workloads", {})
        for name, steps in (("regions4096", min(K, 20)), ("multigroup16384", 2)):
            base, wprobs = problems(name)
            keys = [str(p["dt"]) for p in wprobs]
            entry = {}
            for tag, method, prec, sol in (("fp32_refined", "oci", B.OCI_FP32_REFINED, 0),
                                           ("fp64", "oci", B.OCI_FP64, 0), ("si", "si", B.OCI_FP64, 0),
                                           ("structured_fp64", "oci", B.OCI_FP64, B.OCI_SOLVE_STRUCTURED)):
                rr = run_method(wprobs, method, prec, steps, 1, a.tol, torch, B, not a.no_autotune, sol)
                entry[tag] = summary(rr, tag, steps, keys)
                if method == "oci" and sol == 0:
                    entry[tag]["roofline"] = roofline_for(rr, wprobs, prec == B.OCI_FP32_REFINED, name)
                torch.cuda.empty_cache()
            cw[name] = dict(J=base["J"], N=base["N"], G=base["G"], n=4 * base["N"] * base["G"], steps=steps,
                            dts=[p["dt"] for p in wprobs], **entry)
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline: the oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = batch_cpu_baseline(probs, r["its"], a.cpu_seconds)
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
    if a.cpu_child:
        cpu_child(a.cpu_child)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only (one slab batch per device); --gpus must be 1", "n_gpus": a.gpus}))
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
