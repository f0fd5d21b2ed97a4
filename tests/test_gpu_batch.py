"""GPU parity of the batched multi-slab path (one persistent launch for many
slabs of uneven J, N, G) and of its graph-captured steps.

Tolerances as in test_gpu_parity.py: FP64 lock-step <= 1e-12 against the
oracle run slab by slab; FP32-refined converged <= 1e-10 against the oracle's
converged truth; graph replays bitwise equal to eager batched steps.
"""
import numpy as np
import pytest

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


def small_batch(n_slabs=7, seed=5):
    """Uneven slabs drawn by the batch recipe, cut to sizes the oracle runs fast."""
    return W.batch(seed=seed, n_slabs=n_slabs, j_range=(3, 160), n_choices=(2, 6, 8, 16, 32),
                   g_choices=(1, 2, 3, 4), steps=2)


def _announce(probs, extra):
    shapes = [(p["J"], p["N"], p["G"], 4 * p["N"] * p["G"]) for p in probs]
    print(f"\n[gpu batch] {len(probs)} slabs (J, N, G, n) = {shapes} {extra}", flush=True)


def test_batch_fp64_lockstep_matches_oracle_per_slab():
    probs = [p for p in small_batch() if 4 * p["N"] * p["G"] <= 512]
    _announce(probs, "fp64 lock-step K=5, 2 steps")
    bs = B.BatchSolver(probs, precision=B.OCI_FP64, fixed_iters=5)
    got = []
    for _ in range(2):
        bs.step()
        phis, infos = bs.results()
        got.append(phis)
        assert all(i["iterations"] == 5 and i["status"] == 0 for i in infos), infos
    tot, per = bs.geometry()
    bs.close()
    assert sum(per) == tot and min(per) >= 1
    for k, p in enumerate(probs):
        want = oracle.Oracle(p).run("oci", steps=2, fixed_iters=5)["phi"]
        for s in range(2):
            assert rel(got[s][k], want[s]) <= 1e-12, (k, s)


def test_batch_refined_converges_to_oracle_per_slab():
    probs = [p for p in small_batch(seed=6) if 4 * p["N"] * p["G"] <= 512]
    _announce(probs, "fp32-refined converged, 2 steps")
    bs = B.BatchSolver(probs, precision=B.OCI_FP32_REFINED, tol=1e-12)
    bs.step()
    bs.step()
    phis, infos = bs.results()
    bs.close()
    assert all(i["status"] == 0 for i in infos), infos
    for k, p in enumerate(probs):
        want = oracle.Oracle(p).run("oci", steps=2, tol=1e-14)["phi"][-1]
        assert rel(phis[k], want) <= 1e-10, k


def test_batch_graph_replay_equals_eager():
    probs = [p for p in small_batch(seed=7) if 4 * p["N"] * p["G"] <= 512]
    _announce(probs, "graph of 2 steps replayed 3 times vs eager")
    g = B.BatchSolver(probs, precision=B.OCI_FP32_REFINED, tol=1e-10)
    e = B.BatchSolver(probs, precision=B.OCI_FP32_REFINED, tol=1e-10)
    g.capture(2)
    scratch = torch.ones(1 << 20, device="cuda")
    for r in range(3):
        g.replay()
        scratch.mul_(1.0001).add_(1.0)          # unrelated eager work between replays
        pg, ig = g.results()
        e.step()
        e.step()
        pe, ie = e.results()
        torch.cuda.synchronize()
        for k in range(len(probs)):
            assert np.array_equal(pg[k], pe[k]), (r, k)
            assert ig[k]["iterations"] == ie[k]["iterations"], (r, k)
            assert np.array_equal(g.get_state(k), e.get_state(k)), (r, k)
    g.close()
    e.close()


def test_batch_state_replacement():
    probs = [p for p in small_batch(seed=8, n_slabs=4) if 4 * p["N"] * p["G"] <= 512]
    _announce(probs, "set_state on one slab")
    rng = np.random.default_rng(3)
    k = len(probs) - 1
    psi0 = rng.uniform(0, 1, size=(probs[k]["J"], probs[k]["G"], probs[k]["N"], 2))
    bs = B.BatchSolver(probs, precision=B.OCI_FP64, fixed_iters=4)
    bs.set_state(k, psi0)
    bs.step()
    phis, _ = bs.results()
    bs.close()
    want = oracle.Oracle(probs[k]).run("oci", steps=1, fixed_iters=4, psi_init=psi0)["phi"][0]
    assert rel(phis[k], want) <= 1e-12


def test_batch_rebalance_keeps_results():
    probs = [p for p in small_batch(seed=9) if 4 * p["N"] * p["G"] <= 512]
    _announce(probs, "rebalance, then step and capture")
    a = B.BatchSolver(probs, precision=B.OCI_FP64, fixed_iters=5)
    b = B.BatchSolver(probs, precision=B.OCI_FP64, fixed_iters=5)
    a.step()
    b.step()
    before = b.geometry()
    b.rebalance()
    after = b.geometry()
    assert sum(after[1]) == after[0] and min(after[1]) >= 1
    a.step()
    b.capture(1)
    b.replay()
    pa, _ = a.results()
    pb, ib = b.results()
    a.close()
    b.close()
    assert all(i["iterations"] == 5 for i in ib)
    for k in range(len(probs)):
        assert rel(pb[k], pa[k]) <= 1e-12, (k, before, after)


# ------------------------------------------------------ structured batches
def test_structured_batch_lockstep_matches_oracle_per_slab():
    probs = [p for p in small_batch(seed=11) if p["G"] <= 8]
    _announce(probs, "structured fp64 lock-step K=5, 2 steps")
    bs = B.BatchSolver(probs, precision=B.OCI_FP64, fixed_iters=5, solver=B.OCI_SOLVE_STRUCTURED)
    got = []
    for _ in range(2):
        bs.step()
        phis, infos = bs.results()
        got.append(phis)
        assert all(i["iterations"] == 5 and i["status"] == 0 for i in infos), infos
    bs.close()
    for k, p in enumerate(probs):
        want = oracle.Oracle(p).run("oci", steps=2, fixed_iters=5)["phi"]
        for s in range(2):
            assert rel(got[s][k], want[s]) <= 1e-12, (k, s)


def test_structured_batch_converges_and_replays():
    """Converged structured batch steps (graph of 2 steps, replayed twice)
    against the oracle's converged truth per slab, and the replays against
    eager batched steps bit for bit."""
    probs = [p for p in small_batch(seed=12) if p["G"] <= 8]
    _announce(probs, "structured converged, graph of 2 steps vs eager vs oracle")
    g = B.BatchSolver(probs, precision=B.OCI_FP64, tol=1e-12, solver=B.OCI_SOLVE_STRUCTURED)
    e = B.BatchSolver(probs, precision=B.OCI_FP64, tol=1e-12, solver=B.OCI_SOLVE_STRUCTURED)
    g.capture(2)
    for r in range(2):
        g.replay()
        pg, ig = g.results()
        e.step()
        e.step()
        pe, ie = e.results()
        for k in range(len(probs)):
            assert np.array_equal(pg[k], pe[k]), (r, k)
            assert ig[k] == ie[k], (r, k)
    g.close()
    e.close()
    for k, p in enumerate(probs):
        want = oracle.Oracle(p).run("oci", steps=4, tol=1e-14)["phi"][-1]
        assert rel(pg[k], want) <= 1e-10, k


def test_batch_per_step_argument_sets():
    """Bound per-step argument sets: a graph of 3 steps writes each step's
    flux and report into its own set, equal to eager steps one by one."""
    probs = [p for p in small_batch(seed=13, n_slabs=4) if 4 * p["N"] * p["G"] <= 512]
    _announce(probs, "per-step argument sets, 3-step graph vs eager")
    g = B.BatchSolver(probs, precision=B.OCI_FP32_REFINED, tol=1e-10)
    g.bind_steps(3)
    g.capture(3)
    g.replay()
    pg, ig = g.step_results()
    g.close()
    e = B.BatchSolver(probs, precision=B.OCI_FP32_REFINED, tol=1e-10)
    for i in range(3):
        e.step()
        pe, ie = e.results()
        for k in range(len(probs)):
            assert np.array_equal(pg[i][k], pe[k]), (i, k)
            assert ig[i][k] == ie[k], (i, k)
    e.close()
