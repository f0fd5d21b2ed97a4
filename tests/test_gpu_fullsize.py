"""GPU parity at the workloads' full sizes, in the launch shapes the benchmark
uses (autotuned single-slab kernels; the batched launch for the 64 slabs).

* regions4096 (the benchmark workload), every dt of its sweep: FP64 lock-step
  against the oracle (<= 1e-12) and FP32-refined converged against the
  oracle's converged truth (<= 1e-10), three time steps each.
* multigroup8192 / multigroup16384: FP64 lock-step against the oracle for one
  step (<= 1e-12), and, for FP64 and FP32-refined converged solutions, the
  corner-balance residual of tests/balance.py (a property of the discrete
  solution that holds at any size and does not involve the oracle).
* multigroup16384, the precision form: the FP32-refined and the FP64 OCI
  solutions of the first time step, converged to tol 1e-12 on the GPU, against
  the oracle's converged truth (tol 1e-14): <= 1e-10 and <= 1e-12 normwise
  relative (printed; about two minutes of CPU work for the oracle).
* batch64: every slab of the batched launch satisfies the same residual
  property after a converged step.

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
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


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


def test_multigroup16384_precision_form_against_oracle():
    p = dict(W.config("multigroup16384"), steps=1)
    announce("multigroup16384", p, "first step converged: FP32-refined and FP64 against the oracle")
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
        print(f"  prec={prec}: iterations {infos[0]['iterations']}, max relative phi error vs the oracle "
              f"{errs[prec]:.3e}", flush=True)
    assert errs[B.OCI_FP32_REFINED] <= 1e-10
    assert errs[B.OCI_FP64] <= 1e-12


def test_batch64_full_size_residual():
    probs = W.config("batch64", steps=1)
    print(f"\n[gpu full-size] batch64: {len(probs)} slabs, {sum(p['J'] for p in probs)} cells", flush=True)
    bs = B.BatchSolver(probs, precision=B.OCI_FP32_REFINED, tol=1e-12)
    bs.step()
    _, infos = bs.results()
    states = [bs.get_state(k) for k in range(len(probs))]
    bs.close()
    torch.cuda.empty_cache()
    assert all(i["status"] == 0 for i in infos), infos
    # every slab's state after the step (psi_{k+1/2}) equals the one its own
    # single-slab solve reaches; three of those are also checked against the
    # balance equations directly
    order = sorted(range(len(probs)), key=lambda k: probs[k]["J"] * probs[k]["N"] * probs[k]["G"])
    check_res = {order[0], order[len(order) // 2], order[-1]}
    for k, p in enumerate(probs):
        s = B.Solver(p, precision=B.OCI_FP32_REFINED, tol=1e-12)
        s.step("oci", want_psi=True)
        psi = s.psi.cpu().numpy()
        s.close()
        torch.cuda.empty_cache()
        assert rel(psi[..., 2:4], states[k]) <= 1e-9, k
        if k in check_res:
            assert _residual_check(p, psi, np.zeros((p["J"], p["G"], p["N"], 2))) <= 1e-9, k
