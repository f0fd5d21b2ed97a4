"""GPU parity at the workloads' full sizes, in the launch shapes the benchmark
uses (autotuned single-slab kernels; the batched launch for the 64 slabs).

* regions4096 (the benchmark workload), every dt of its sweep: FP64 lock-step
  against the oracle (<= 1e-12) and FP32-refined converged against the
  oracle's converged truth (<= 1e-10), three time steps each.
* multigroup8192 / multigroup16384: FP64 lock-step against the oracle for one
  step (<= 1e-12), and, for FP64 and FP32-refined converged solutions, the
  corner-balance residual of tests/balance.py (a property of the discrete
  solution that holds at any size and does not involve the oracle).
* multigroup8192 and multigroup16384 (the precision form): the FP32-refined
  and the FP64 OCI solutions of the first time step, converged to tol 1e-12 on
  the GPU, against the oracle's converged truth (tol 1e-14): <= 1e-10 and
  <= 1e-12 normwise relative, max|dphi| / max|phi|.  The pointwise relative
  error over the entries with |phi| >= 1e-8 max|phi| is printed beside it
  (the source covers an eighth of the slab and the fast group's flux spans
  many decades, so the normwise figure alone says little about the dim
  cells).  About one and two minutes of CPU work for the oracle.
* batch64: the first converged step of the batched launch (FP32-refined, the
  launch the benchmark times) against the oracle's converged truth for three
  slabs: the one-angle-group slab of smallest cells (n = 32) with the most
  cells, the slab of largest cells (n = 512) with the fewest cells, and the
  slab with the most cells whose oracle run takes seconds (J = 8038, n = 256;
  the one with more cells has n = 512 and 900 iterations, minutes of oracle
  time); the same three also satisfy the balance residual.

Residual bound: at convergence the OCI residual equals the change of the
lagged incident terms, |mu| |delta psi_edge|, which the stopping rule keeps
near tol; with tol = 1e-12 the bound used is 1e-9 x max |psi|.
"""
import numpy as np
import pytest

import balance as BAL
import oracle
from paper_2503_00264_amd import binding as B
from paper_2503_00264_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    B.lib()


def rel(a, b):
    """Normwise relative difference max|a - b| / max|b|."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def pointwise(a, b, floor=1e-8):
    """Largest |a - b| / |b| over the entries with |b| >= floor * max|b|."""
    m = np.abs(b) >= floor * np.max(np.abs(b))
    return float(np.max(np.abs(a[m] - b[m]) / np.abs(b[m])))


def announce(name, p, extra):
    print(f"\n[gpu full-size] {name}: J={p['J']} N={p['N']} G={p['G']} n={4 * p['N'] * p['G']} {extra}",
          flush=True)


@pytest.mark.parametrize("dt", W.REGIONS_DT_SWEEP)
def test_regions4096_every_dt(dt):
    p = dict(W.config("regions4096"), dt=dt)
    announce("regions4096", p, f"dt={dt}")
    o = oracle.Oracle(p, methods=("oci",))
    want_ls = o.run("oci", steps=3, fixed_iters=10)["phi"]
    s = B.Solver(p, precision=B.OCI_FP64, fixed_iters=10)
    s.autotune(4)
    got, _ = s.run(steps=3)
    s.close()
    assert rel(got, want_ls) <= 1e-12
    want = o.run("oci", steps=3, tol=1e-14)["phi"]
    s = B.Solver(p, precision=B.OCI_FP32_REFINED, tol=1e-12)
    s.autotune(4)
    got, infos = s.run(steps=3)
    s.close()
    assert all(i["status"] == 0 for i in infos)
    assert rel(got, want) <= 1e-10


def _residual_check(p, psi, psi_prev):
    r = BAL.residual(p, psi, psi_prev, q=p["q"], inc_l=p.get("inc_left"), inc_r=p.get("inc_right"))
    return float(np.max(np.abs(r)) / np.max(np.abs(psi)))


@pytest.mark.parametrize("name", ["multigroup8192", "multigroup16384"])
def test_multigroup_full_size(name):
    p = W.config(name)
    announce(name, p, "lock-step K=3 and converged residual")
    o = oracle.Oracle(p, methods=("oci",))
    want = o.run("oci", steps=1, fixed_iters=3)["phi"]
    del o
    s = B.Solver(p, precision=B.OCI_FP64, fixed_iters=3)
    got, _ = s.run(steps=1)
    s.close()
    assert rel(got, want) <= 1e-12
    for prec in (B.OCI_FP64, B.OCI_FP32_REFINED):
        s = B.Solver(p, precision=prec, tol=1e-12)
        s.autotune(4)
        s.step("oci", want_psi=True)
        info = s.last_info()
        psi = s.psi.cpu().numpy()
        s.close()
        torch.cuda.empty_cache()
        print(f"  prec={prec}: {info}", flush=True)
        assert info["status"] == 0
        assert _residual_check(p, psi, np.zeros((p["J"], p["G"], p["N"], 2))) <= 1e-9


@pytest.mark.parametrize("name", ["multigroup8192", "multigroup16384"])
def test_multigroup_converged_against_oracle(name):
    p = dict(W.config(name), steps=1)
    announce(name, p, "first step converged: FP32-refined and FP64 against the oracle")
    want = oracle.Oracle(p, methods=("oci",)).run("oci", steps=1, tol=1e-14)["phi"]
    errs = {}
    for prec in (B.OCI_FP32_REFINED, B.OCI_FP64):
        s = B.Solver(p, precision=prec, tol=1e-12)
        s.autotune(4)
        got, infos = s.run(steps=1)
        s.close()
        torch.cuda.empty_cache()
        assert infos[0]["status"] == 0, infos
        errs[prec] = rel(got, want)
        print(f"  prec={prec}: iterations {infos[0]['iterations']}, normwise relative phi error vs the "
              f"oracle {errs[prec]:.3e}, pointwise over |phi| >= 1e-8 max|phi| {pointwise(got, want):.3e}",
              flush=True)
    assert errs[B.OCI_FP32_REFINED] <= 1e-10
    assert errs[B.OCI_FP64] <= 1e-12


# batch64 slabs checked against the oracle: (index, what it stands for)
BATCH_SLABS = ((22, "n = 32, most cells of that size"), (6, "n = 512, fewest cells"),
               (12, "most cells with a seconds-long oracle run"))


def test_batch64_full_size_against_oracle():
    probs = W.config("batch64", steps=1)
    print(f"\n[gpu full-size] batch64: {len(probs)} slabs, {sum(p['J'] for p in probs)} cells, "
          f"FP32-refined batched launch, first step converged to 1e-12", flush=True)
    bs = B.BatchSolver(probs, precision=B.OCI_FP32_REFINED, tol=1e-12)
    bs.step()
    phis, infos = bs.results()
    states = {k: bs.get_state(k) for k, _ in BATCH_SLABS}
    bs.close()
    torch.cuda.empty_cache()
    assert all(i["status"] == 0 for i in infos), infos
    for k, why in BATCH_SLABS:
        p = probs[k]
        ref = oracle.Oracle(p, methods=("oci",)).run("oci", steps=1, tol=1e-14)
        err = rel(phis[k], ref["phi"][0])
        print(f"  slab {k} ({why}): J={p['J']} N={p['N']} G={p['G']}, iterations "
              f"{infos[k]['iterations']} (oracle {ref['info'][0]['iterations']}), normwise relative phi "
              f"error {err:.3e}, pointwise {pointwise(phis[k], ref['phi'][0]):.3e}", flush=True)
        assert err <= 1e-10, k
        assert rel(states[k], ref["psi_prev"]) <= 1e-10, k
