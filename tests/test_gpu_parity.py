"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances (see the design notes for the derivation):
  * FP64 OCI / SI in lock-step (the same fixed number of iterations per step
    on both sides): normwise relative difference of every step's scalar flux
    <= 1e-12.  Both sides solve the same systems; they differ only in
    rounding order (an explicit inverse against forward/back substitution,
    fused multiply-adds, tree against serial sums), each ~kappa * 1e-16 per
    solve with kappa <= ~200 for these cell matrices.
  * FP32-refined OCI converged to tol on the GPU against the oracle converged
    to 1e-14: <= 1e-10 normwise relative.  Both share the fixed point; the
    refined iteration adds a contraction of ~kappa * 6e-8 per step.
Every case prints its name, shape and seed before touching the GPU.
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


def _cases():
    return {
        # name: (problem, steps)
        "homogeneous64_n32": (W.config("homogeneous64"), 3),
        "regions512_n64": (W.regions(seed=2, J=512, N=16, n_regions=64, length=8.0, dt=0.1), 3),
        "multigroup192_n128": (W.multigroup(seed=3, J=192, N=8, G=4, n_regions=64, length=1.5,
                                            dt=1e-3), 2),
        "multigroup128_n256": (W.multigroup(seed=4, J=128, N=16, G=4, n_regions=64, length=1.0,
                                            dt=1e-3), 2),
        "multigroup40_n512": (W.multigroup(seed=5, J=40, N=32, G=4, n_regions=8, length=0.625,
                                           dt=1e-3), 2),
        "odd_N6_n24": (W.regions(seed=6, J=77, N=6, n_regions=7, length=3.0, dt=0.2), 2),
        "G3_n48": (W.multigroup(seed=7, J=45, N=4, G=3, n_regions=5, length=2.0,
                                speeds=(5.0, 1.0, 0.2), dt=0.3), 2),
        # identity-padded blocks in the large-cell setup kernel: n = 120 in a
        # 128 block, n = 192 in a 256 block
        "G3_N10_n120": (W.multigroup(seed=9, J=24, N=10, G=3, n_regions=4, length=1.0,
                                     speeds=(50.0, 5.0, 0.5), dt=0.01), 2),
        "G3_N16_n192": (W.multigroup(seed=10, J=16, N=16, G=3, n_regions=4, length=0.5,
                                     speeds=(50.0, 5.0, 0.5), dt=0.01), 2),
        "single_cell": (W.multigroup(seed=8, J=1, N=8, G=2, n_regions=1, length=0.5,
                                     speeds=(2.0, 1.0), dt=0.1), 2),
        "N2_J5": (W.homogeneous(J=5, N=2, length=1.0), 2),
        # the paper's two-group performance problem: delta = 0.91 at dt = 10 s
        # (scattering ratio near one), delta = 0.23 at dt = 0.1 s
        "rosa_S8_dt10": (W.rosa(J=50, N=8, dt=10.0), 2),
        "rosa_S16_dt0.1": (W.rosa(J=200, N=16, dt=0.1), 2),
        # 64 directions: a group spans the whole wave (the cross-lane sums
        # pair lanes 32 apart), one pair per lane (G = 1) or two (G = 2)
        "regions48_N64": (W.regions(seed=11, J=48, N=64, n_regions=6, length=2.0, dt=0.1), 2),
        "multigroup16_N64_G2": (W.multigroup(seed=12, J=16, N=64, G=2, n_regions=4, length=0.5,
                                             speeds=(20.0, 1.0), dt=0.05), 2),
    }


CASES = _cases()


def _announce(name, p, extra=""):
    print(f"\n[gpu case] {name}: J={p['J']} N={p['N']} G={p['G']} n={4 * p['N'] * p['G']} {extra}",
          flush=True)


@pytest.mark.parametrize("name", list(CASES))
def test_oci_fp64_lockstep(name):
    p, steps = CASES[name]
    K = 7
    _announce(name, p, f"oci fp64 lock-step K={K} steps={steps}")
    want = oracle.Oracle(p).run("oci", steps=steps, fixed_iters=K)["phi"]
    s = B.Solver(p, precision=B.OCI_FP64, fixed_iters=K)
    got, infos = s.run(steps=steps, want_psi=True)
    s.close()
    assert all(i["iterations"] == K and i["status"] == 0 for i in infos), infos
    assert rel(got, want) <= 1e-12


@pytest.mark.parametrize("name", ["homogeneous64_n32", "regions512_n64", "multigroup192_n128", "single_cell",
                                  "rosa_S8_dt10"])
def test_si_loop_layouts_agree(name, monkeypatch):
    """SI's iteration loop as the host-driven launch sequence, as one
    persistent launch on one workgroup and on several: the same iterates bit
    for bit (the passes do the same arithmetic in the same order; only the
    norm's summation order differs), the same iteration counts, converged and
    lock-step against the oracle."""
    p, steps = CASES[name]
    _announce(name, p, "si: launches / one / many")
    want = oracle.Oracle(p).run("si", steps=steps, fixed_iters=5)["phi"]
    ref = oracle.Oracle(p).run("si", steps=steps, tol=1e-14)["phi"]
    outs = []
    for mode in ("launches", "one", "many"):
        monkeypatch.setenv("OCI_SI_MODE", mode)
        s = B.Solver(p, precision=B.OCI_FP64, fixed_iters=5)
        got, infos = s.run(steps=steps, method="si")
        s.close()
        assert all(i["iterations"] == 5 and i["status"] == 0 for i in infos), (mode, infos)
        assert rel(got, want) <= 1e-12, mode
        s = B.Solver(p, precision=B.OCI_FP64, tol=1e-12)
        conv, cinfo = s.run(steps=steps, method="si")
        s.close()
        assert all(i["status"] == 0 for i in cinfo), (mode, cinfo)
        assert rel(conv, ref) <= 1e-10, mode
        outs.append((got, conv, [i["iterations"] for i in cinfo]))
    for got, conv, its in outs[1:]:
        assert np.array_equal(got, outs[0][0])
        assert its == outs[0][2]
        assert rel(conv, outs[0][1]) <= 1e-14


@pytest.mark.parametrize("name", ["homogeneous64_n32", "regions512_n64", "multigroup192_n128",
                                  "G3_n48", "single_cell", "N2_J5", "rosa_S8_dt10", "rosa_S16_dt0.1"])
def test_si_fp64_lockstep(name):
    p, steps = CASES[name]
    K = 5
    _announce(name, p, f"si fp64 lock-step K={K}")
    want = oracle.Oracle(p).run("si", steps=steps, fixed_iters=K)["phi"]
    s = B.Solver(p, precision=B.OCI_FP64, fixed_iters=K)
    got, infos = s.run(steps=steps, method="si")
    s.close()
    assert all(i["iterations"] == K and i["status"] == 0 for i in infos), infos
    assert rel(got, want) <= 1e-12


@pytest.mark.parametrize("name", ["homogeneous64_n32", "regions512_n64", "multigroup192_n128",
                                  "multigroup128_n256", "multigroup40_n512", "G3_n48", "G3_N10_n120",
                                  "G3_N16_n192"])
def test_oci_refined_converges_to_oracle(name):
    p, steps = CASES[name]
    _announce(name, p, "oci fp32-refined converged")
    want = oracle.Oracle(p).run("oci", steps=steps, tol=1e-14)["phi"]
    s = B.Solver(p, precision=B.OCI_FP32_REFINED, tol=1e-12)
    got, infos = s.run(steps=steps)
    s.close()
    assert all(i["status"] == 0 for i in infos), infos
    assert rel(got, want) <= 1e-10


@pytest.mark.parametrize("name,gpu_tol,oracle_tol", [("rosa_S8_dt10", 1e-11, 1e-12),
                                                    ("rosa_S16_dt0.1", 1e-12, 1e-14)])
def test_rosa_converged_to_oracle(name, gpu_tol, oracle_tol):
    """The two-group problem converged on the GPU (FP64 OCI, FP32-refined OCI
    and SI) against the oracle's converged OCI answer.  At dt = 10 s the flux
    reaches ~7, so the absolute stopping test cannot go below ~1e-13 in FP64
    (the oracle stops at 1e-12 there); the errors left are about tol / (1 -
    rho) absolute, far inside 1e-10 relative."""
    p, steps = CASES[name]
    _announce(name, p, f"rosa converged, gpu tol {gpu_tol}, oracle tol {oracle_tol}")
    want = oracle.Oracle(p).run("oci", steps=steps, tol=oracle_tol)["phi"]
    for prec, method in ((B.OCI_FP64, "oci"), (B.OCI_FP32_REFINED, "oci"), (B.OCI_FP64, "si")):
        s = B.Solver(p, precision=prec, tol=gpu_tol)
        got, infos = s.run(steps=steps, method=method)
        s.close()
        assert all(i["status"] == 0 for i in infos), (prec, method, infos)
        assert rel(got, want) <= 1e-10, (prec, method, rel(got, want))


def test_e_history_on_fourier_verification_problem():
    """e_l and rho_e after k iterations (fixed_iters = k) of FP64 OCI on the
    paper's verification problem (1000 cells, random start) equal the
    oracle's iteration history: the GPU's per-iteration convergence record
    is the one the empirical spectral-radius trace reads."""
    p = W.fourier_verification()
    _announce("fourier_verification", p, "e_l history, fp64 OCI, k in 2..40")
    o = oracle.Oracle(p, methods=("oci",))
    pp, pi = o.initial_state(p["psi_init"])
    phi, oinfo = o.step("oci", pp, pi, q=p["q"], fixed_iters=40, history=True)
    e = oinfo["e_hist"]
    # e_l is a norm of differences of fluxes that stay O(max|phi|): both sides
    # agree to its absolute rounding scale, 1e-14 max|phi| sqrt(entries)
    floor = 1e-14 * np.abs(phi).max() * np.sqrt(phi.size)
    for k in (2, 5, 10, 20, 40):
        s = B.Solver(p, precision=B.OCI_FP64, fixed_iters=k)
        _, infos = s.run(steps=1)
        s.close()
        i = infos[0]
        tol_k, tol_k1 = 1e-12 * e[k - 1] + floor, 1e-12 * e[k - 2] + floor
        assert i["iterations"] == k and i["status"] == 0, i
        assert abs(i["e_last"] - e[k - 1]) <= tol_k, (k, i["e_last"], e[k - 1])
        rho = e[k - 1] / e[k - 2]
        assert abs(i["rho_e"] - rho) <= rho * (tol_k / e[k - 1] + tol_k1 / e[k - 2]), (k, i["rho_e"], rho)


def test_oci_fp64_converged_iteration_counts_match():
    p = W.config("homogeneous64")
    _announce("homogeneous64", p, "converged, 10 steps, tol 1e-10")
    ref = oracle.Oracle(p).run("oci", tol=1e-10)
    s = B.Solver(p, precision=B.OCI_FP64, tol=1e-10)
    got, infos = s.run()
    s.close()
    assert [i["iterations"] for i in infos] == [i["iterations"] for i in ref["info"]]
    assert rel(got, ref["phi"]) <= 1e-12
    # e_l is a norm of differences of nearly equal iterates: each entry
    # carries ~1e-16 |phi| of rounding, so compare on that absolute scale
    scale = 1e-14 * np.max(np.abs(ref["phi"])) * np.sqrt(ref["phi"][0].size)
    for a, b in zip(infos, ref["info"]):
        assert abs(a["e_last"] - b["e_last"]) <= scale
        assert abs(a["rho_e"] - b["rho_e"]) <= 1e-3


def test_angular_norm_counts_match():
    p = W.regions(seed=2, J=256, N=8, n_regions=64, length=4.0, dt=0.05, steps=2)
    _announce("regions256", p, "angular norm")
    ref = oracle.Oracle(p).run("oci", tol=1e-9, norm=oracle.NORM_ANGULAR)
    s = B.Solver(p, precision=B.OCI_FP64, tol=1e-9, norm=B.OCI_NORM_ANGULAR)
    got, infos = s.run()
    s.close()
    assert [i["iterations"] for i in infos] == [i["iterations"] for i in ref["info"]]
    assert rel(got, ref["phi"]) <= 1e-12


def test_boundary_sources_and_initial_state():
    p = W.multigroup(seed=9, J=96, N=8, G=2, n_regions=8, length=2.0, speeds=(3.0, 1.0), dt=0.2,
                     steps=3)
    rng = np.random.default_rng(21)
    p["inc_left"] = rng.uniform(0, 1, size=(2, 2, 4))
    p["inc_right"] = rng.uniform(0, 1, size=(2, 2, 4))
    p["psi_init"] = rng.uniform(0, 1, size=(96, 2, 8, 2))
    _announce("boundary", p, "incident fluxes + initial state")
    for method in ("oci", "si"):
        want = oracle.Oracle(p).run(method, fixed_iters=6)
        s = B.Solver(p, precision=B.OCI_FP64, fixed_iters=6)
        got, _ = s.run(method=method)
        state = s.get_state().cpu().numpy()
        s.close()
        assert rel(got, want["phi"]) <= 1e-12
        assert rel(state, want["psi_prev"]) <= 1e-12


def test_oci_and_si_agree_on_gpu():
    p = W.regions(seed=2, J=512, N=16, n_regions=64, length=8.0, dt=0.05, steps=2)
    _announce("regions512", p, "oci vs si converged")
    a = B.Solver(p, tol=1e-13)
    pa, _ = a.run()
    a.close()
    b = B.Solver(p, tol=1e-13)
    pb, _ = b.run(method="si")
    b.close()
    assert rel(pa, pb) <= 1e-11


@pytest.mark.parametrize("prec", [B.OCI_FP64, B.OCI_FP32_REFINED])
def test_run_twice_bitwise(prec):
    p = W.regions(seed=2, J=1024, N=16, n_regions=64, length=16.0, dt=0.01, steps=3)
    _announce("regions1024", p, f"determinism prec={prec}")
    out = []
    for _ in range(2):
        s = B.Solver(p, precision=prec, tol=1e-10)
        got, infos = s.run()
        s.close()
        out.append((got, [i["iterations"] for i in infos]))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


def test_status_not_converged_and_nonfinite():
    p = W.homogeneous(J=64, N=8)
    _announce("homogeneous64", p, "statuses")
    s = B.Solver(p, max_iters=3, tol=1e-10)
    _, infos = s.run(steps=1)
    s.close()
    assert infos[0]["status"] == B.OCI_NOT_CONVERGED and infos[0]["iterations"] == 3
    q = p["q"].copy()
    q[10, 0, 2] = np.nan
    p2 = dict(p, q=q)
    s = B.Solver(p2, tol=1e-10)
    _, infos = s.run(steps=1)
    s.close()
    assert infos[0]["status"] == B.OCI_NONFINITE and infos[0]["iterations"] == 1


def test_state_roundtrip_restart():
    p = W.regions(seed=2, J=256, N=8, n_regions=64, length=4.0, dt=0.05, steps=4)
    _announce("regions256", p, "checkpoint / restart")
    a = B.Solver(p, fixed_iters=5)
    full, _ = a.run(steps=4)
    a.close()
    b = B.Solver(p, fixed_iters=5)
    b.run(steps=2)
    st = b.get_state().cpu().numpy()
    b.close()
    c = B.Solver(p, fixed_iters=5)
    c.set_state(st)
    rest, _ = c.run(steps=2)
    c.close()
    # restarting copies psi_{k+1/2} to both levels of the first iterate, so
    # with a fixed iteration count the restart is compared at its own start
    want = oracle.Oracle(p).run("oci", steps=2, fixed_iters=5, psi_init=st)["phi"]
    assert rel(rest, want) <= 1e-12
    assert rel(full[:2], oracle.Oracle(p).run("oci", steps=2, fixed_iters=5)["phi"]) <= 1e-12


@pytest.mark.parametrize("mode", [{"OCI_MODE": "global"}, {"OCI_NO_RESIDENT": "1"},
                                  {"OCI_BLOCK": "256"}, {"OCI_BAR_GROUP": "3"}, {"OCI_MAX_WG": "3"},
                                  {"OCI_MAX_WG": "3", "OCI_MODE": "global"}])
@pytest.mark.parametrize("name", ["regions512_n64", "multigroup128_n256", "odd_N6_n24"])
def test_kernel_variants_lockstep(name, mode, monkeypatch):
    """Every launch variant (global-memory kernel, streamed factors, block size,
    barrier arrival groups, several tiles per workgroup) gives the oracle's
    answer: FP64 in lock-step (<= 1e-12), and FP32-refined both in lock-step
    (iteration counts) and converged on the GPU (tol 1e-12) against the
    oracle converged to 1e-14 (<= 1e-10)."""
    for k, v in mode.items():
        monkeypatch.setenv(k, v)
    p, steps = CASES[name]
    K = 6
    _announce(name, p, f"variant {mode} K={K}")
    o = oracle.Oracle(p)
    for prec in (B.OCI_FP64, B.OCI_FP32_REFINED):
        s = B.Solver(p, precision=prec, fixed_iters=K)
        got, infos = s.run(steps=steps)
        s.close()
        assert all(i["iterations"] == K and i["status"] == 0 for i in infos), infos
        if prec == B.OCI_FP64:
            assert rel(got, o.run("oci", steps=steps, fixed_iters=K)["phi"]) <= 1e-12
    truth = o.run("oci", steps=steps, tol=1e-14)["phi"]
    s = B.Solver(p, precision=B.OCI_FP32_REFINED, tol=1e-12)
    cfg = s.config()
    got, infos = s.run(steps=steps)
    s.close()
    assert all(i["status"] == 0 for i in infos), infos
    err = rel(got, truth)
    print(f"  refined converged, shape {cfg}: normwise relative error {err:.2e}", flush=True)
    assert err <= 1e-10


@pytest.mark.parametrize("name", ["regions512_n64", "multigroup128_n256", "G3_n48"])
def test_autotune_keeps_parity(name):
    """The autotuner's chosen shape still gives the oracle's lock-step answer."""
    p, steps = CASES[name]
    _announce(name, p, "autotune then lock-step")
    for prec in (B.OCI_FP64, B.OCI_FP32_REFINED):
        s = B.Solver(p, precision=prec, fixed_iters=6)
        cfg = s.autotune(iters=4)
        print("chosen", cfg, flush=True)
        assert cfg["block"] in (256, 1024) and cfg["workgroups"] >= 1
        got, infos = s.run(steps=steps)
        s.close()
        assert all(i["iterations"] == 6 and i["status"] == 0 for i in infos), infos
        if prec == B.OCI_FP64:
            want = oracle.Oracle(p).run("oci", steps=steps, fixed_iters=6)["phi"]
            assert rel(got, want) <= 1e-12
    # the refined path in the tuned shape, converged, against the oracle's
    # converged truth
    s = B.Solver(p, precision=B.OCI_FP32_REFINED, tol=1e-12)
    cfg = s.autotune(iters=4)
    got, infos = s.run(steps=steps)
    s.close()
    assert all(i["status"] == 0 for i in infos), infos
    err = rel(got, oracle.Oracle(p).run("oci", steps=steps, tol=1e-14)["phi"])
    print(f"  refined converged in the tuned shape {cfg}: normwise relative error {err:.2e}", flush=True)
    assert err <= 1e-10


def _multi_step_cases():
    rng = np.random.default_rng(31)
    b = W.multigroup(seed=9, J=96, N=8, G=2, n_regions=8, length=2.0, speeds=(3.0, 1.0), dt=0.2,
                     steps=4)
    b["inc_left"] = rng.uniform(0, 1, size=(2, 2, 4))
    b["inc_right"] = rng.uniform(0, 1, size=(2, 2, 4))
    b["psi_init"] = rng.uniform(0, 1, size=(96, 2, 8, 2))
    return {
        "homogeneous64_n32": W.config("homogeneous64"),
        "regions512_n64": dict(CASES["regions512_n64"][0], steps=5),
        "boundary_n64": b,
        "multigroup128_n256": dict(CASES["multigroup128_n256"][0], steps=3),
        # two-group problem with 5-8 iterations per step: stopping decisions
        # fall on the iterations right after a turnover
        "rosa_S8_J114": W.rosa(J=114, N=8, dt=0.1, steps=8),
        "rosa_S4_J114": W.rosa(J=114, N=4, dt=0.1, steps=8),
    }


MULTI = _multi_step_cases()


@pytest.mark.parametrize("prec", [B.OCI_FP64, B.OCI_FP32_REFINED])
@pytest.mark.parametrize("name", list(MULTI))
def test_run_steps_equals_single_steps(name, prec):
    """Several steps in one launch (the register-resident kernel turns each
    stop over to the next step itself) give bit for bit what one call per step
    gives: fluxes, step reports and the final state."""
    p = MULTI[name]
    _announce(name, p, f"oci_run_steps vs oci_step, prec={prec}, steps={p['steps']}")
    s = B.Solver(p, precision=prec, tol=1e-10)
    want, winfo = s.run()
    wstate = s.get_state().cpu().numpy()
    resident = s.config()["resident"]
    s.close()
    s = B.Solver(p, precision=prec, tol=1e-10)
    got, ginfo = s.run_steps()
    gstate = s.get_state().cpu().numpy()
    s.close()
    if prec == B.OCI_FP32_REFINED and name != "multigroup128_n256":
        assert resident, "the multi-step launch needs the register-resident kernel here"
    assert ginfo == winfo
    assert np.array_equal(got, want)
    assert np.array_equal(gstate, wstate)


@pytest.mark.parametrize("block", ["256", "1024"])
def test_run_steps_partial_slots_across_turnovers(block, monkeypatch):
    """Twelve short steps in one launch of the register-resident kernel: the
    partial-sum slots of the iterations a turnover skips must not hand a
    value of the previous step to the next one's stopping decision (all
    workgroups then stop together, every step converges, and the results
    equal one call per step bit for bit)."""
    monkeypatch.setenv("OCI_BLOCK", block)
    p = W.rosa(J=114, N=8, dt=0.1, steps=12)
    _announce("rosa_S8_J114", p, f"oci_run_steps x12, block {block}")
    s = B.Solver(p, precision=B.OCI_FP32_REFINED, tol=1e-10)
    want, winfo = s.run()
    s.close()
    s = B.Solver(p, precision=B.OCI_FP32_REFINED, tol=1e-10)
    cfg = s.config()
    got, ginfo = s.run_steps()
    s.close()
    assert cfg["resident"] and cfg["block"] == int(block), cfg
    assert all(i["status"] == 0 for i in ginfo), ginfo
    assert ginfo == winfo
    assert np.array_equal(got, want)


def test_run_steps_lockstep_matches_oracle():
    p = dict(W.config("homogeneous64"), steps=6)
    _announce("homogeneous64", p, "oci_run_steps, fp64 lock-step K=9 against the oracle")
    want = oracle.Oracle(p).run("oci", fixed_iters=9)["phi"]
    s = B.Solver(p, precision=B.OCI_FP64, fixed_iters=9)
    resident = s.config()["resident"]
    got, infos = s.run_steps()
    s.close()
    assert resident, "n = 32 in FP64 runs the register-resident kernel"
    assert all(i["iterations"] == 9 and i["status"] == 0 for i in infos), infos
    assert rel(got, want) <= 1e-12


@pytest.mark.parametrize("case", ["not_converged", "nonfinite"])
def test_run_steps_statuses_equal_single_steps(case):
    p = dict(W.homogeneous(J=64, N=8), steps=3)
    kw = dict(tol=1e-10)
    if case == "not_converged":
        kw["max_iters"] = 3
    else:
        q = p["q"].copy()
        q[10, 0, 2] = np.nan
        p["q"] = q
    _announce("homogeneous64", p, f"oci_run_steps statuses: {case}")
    out = []
    for multi in (False, True):
        s = B.Solver(p, precision=B.OCI_FP32_REFINED, **kw)
        got, infos = s.run_steps() if multi else s.run()
        s.close()
        out.append((got, infos))
    want = B.OCI_NOT_CONVERGED if case == "not_converged" else B.OCI_NONFINITE
    assert all(i["status"] == want for i in out[1][1]), out[1][1]
    assert [(i["iterations"], i["status"]) for i in out[0][1]] == [(i["iterations"], i["status"]) for i in out[1][1]]
    assert np.array_equal(out[0][0], out[1][0], equal_nan=True)


# ---------------------------------------------------------------- structured
# The structured exact cell solve (OCI_SOLVE_STRUCTURED): the same OCI
# iteration with each cell system solved through its block structure (4x4
# corner blocks inverted in closed form, the rank-4G scattering coupling
# through a capacitance matrix).  Same bars as the dense FP64 path.

@pytest.mark.parametrize("name", list(CASES))
def test_structured_fp64_lockstep(name):
    p, steps = CASES[name]
    K = 7
    _announce(name, p, f"structured oci fp64 lock-step K={K} steps={steps}")
    want = oracle.Oracle(p).run("oci", steps=steps, fixed_iters=K)
    s = B.Solver(p, precision=B.OCI_FP64, fixed_iters=K, solver=B.OCI_SOLVE_STRUCTURED)
    got, infos = s.run(steps=steps, want_psi=True)
    state = s.get_state().cpu().numpy()
    s.close()
    assert all(i["iterations"] == K and i["status"] == 0 for i in infos), infos
    assert rel(got, want["phi"]) <= 1e-12
    assert rel(state, want["psi_prev"]) <= 1e-12


@pytest.mark.parametrize("name", ["homogeneous64_n32", "regions512_n64", "multigroup192_n128",
                                  "multigroup128_n256", "multigroup40_n512", "G3_n48", "G3_N16_n192",
                                  "rosa_S16_dt0.1"])
def test_structured_converges_to_oracle(name):
    p, steps = CASES[name]
    _announce(name, p, "structured oci converged")
    # converged answers differ from the fixed point by about tol rho / (1 - rho)
    # (absolute), so the converged bar is the refined path's 1e-10; the 1e-12
    # bar of FP64 is the lock-step test above
    ref = oracle.Oracle(p).run("oci", steps=steps, tol=1e-14)
    s = B.Solver(p, precision=B.OCI_FP64, tol=1e-12, solver=B.OCI_SOLVE_STRUCTURED)
    got, infos = s.run(steps=steps)
    s.close()
    assert all(i["status"] == 0 for i in infos), infos
    err = rel(got, ref["phi"])
    print(f"  normwise relative error {err:.2e}", flush=True)
    assert err <= 1e-10


@pytest.mark.parametrize("name", ["homogeneous64_n32", "regions512_n64", "multigroup192_n128",
                                  "multigroup128_n256", "multigroup40_n512", "single_cell", "rosa_S16_dt0.1",
                                  "regions48_N64", "multigroup16_N64_G2"])
@pytest.mark.parametrize("max_wg", [None, "2"])
def test_structured_staged_and_direct_bodies_agree(name, max_wg, monkeypatch):
    """The staged iteration body (tile inputs staged into LDS one tile ahead)
    and the direct body give the same lock-step iterates, both at the oracle's
    1e-12; with two workgroups every workgroup pipelines many tiles."""
    p, steps = CASES[name]
    K = 7
    if max_wg:
        monkeypatch.setenv("OCI_MAX_WG", max_wg)
    _announce(name, p, f"structured staged vs direct, K={K}, max_wg={max_wg}")
    want = oracle.Oracle(p).run("oci", steps=steps, fixed_iters=K)
    out = []
    for direct in ("0", "1"):
        monkeypatch.setenv("OCI_WB_DIRECT", direct)
        s = B.Solver(p, precision=B.OCI_FP64, fixed_iters=K, solver=B.OCI_SOLVE_STRUCTURED)
        assert s.config()["local"] == (1 if direct == "0" else 0)
        got, infos = s.run(steps=steps, want_psi=True)
        psi = s.psi.cpu().numpy()
        s.close()
        assert all(i["iterations"] == K and i["status"] == 0 for i in infos), infos
        assert rel(got, want["phi"]) <= 1e-12
        assert rel(psi, want["psi_iter"]) <= 1e-12
        out.append((got, psi))
    assert rel(out[0][0], out[1][0]) <= 1e-13
    assert rel(out[0][1], out[1][1]) <= 1e-13


def test_structured_iteration_counts_match_oracle():
    p = W.config("homogeneous64")
    _announce("homogeneous64", p, "structured converged, 10 steps, tol 1e-10: iteration counts")
    ref = oracle.Oracle(p).run("oci", tol=1e-10)
    s = B.Solver(p, precision=B.OCI_FP64, tol=1e-10, solver=B.OCI_SOLVE_STRUCTURED)
    got, infos = s.run()
    s.close()
    assert [i["iterations"] for i in infos] == [i["iterations"] for i in ref["info"]]
    assert rel(got, ref["phi"]) <= 1e-12


def test_structured_boundary_sources_and_initial_state():
    p = W.multigroup(seed=9, J=96, N=8, G=2, n_regions=8, length=2.0, speeds=(3.0, 1.0), dt=0.2,
                     steps=3)
    rng = np.random.default_rng(21)
    p["inc_left"] = rng.uniform(0, 1, size=(2, 2, 4))
    p["inc_right"] = rng.uniform(0, 1, size=(2, 2, 4))
    p["psi_init"] = rng.uniform(0, 1, size=(96, 2, 8, 2))
    _announce("boundary", p, "structured: incident fluxes + initial state")
    want = oracle.Oracle(p).run("oci", fixed_iters=6)
    s = B.Solver(p, precision=B.OCI_FP64, fixed_iters=6, solver=B.OCI_SOLVE_STRUCTURED)
    got, _ = s.run(want_psi=True)
    psi = s.psi.cpu().numpy()
    state = s.get_state().cpu().numpy()
    s.close()
    assert rel(got, want["phi"]) <= 1e-12
    assert rel(state, want["psi_prev"]) <= 1e-12
    assert rel(psi, want["psi_iter"]) <= 1e-12


@pytest.mark.parametrize("override", [{}, {"OCI_MAX_WG": "3"}, {"OCI_BAR_GROUP": "3"}])
def test_structured_run_steps_and_launch_shapes(override, monkeypatch):
    """Several workgroups' worth of tiles per workgroup, other barrier arrival
    groups and oci_run_steps all give the single-step answer bit for bit."""
    for k, v in override.items():
        monkeypatch.setenv(k, v)
    p = dict(CASES["regions512_n64"][0], steps=4)
    _announce("regions512_n64", p, f"structured, {override}")
    a = B.Solver(p, precision=B.OCI_FP64, tol=1e-11, solver=B.OCI_SOLVE_STRUCTURED)
    want, winfo = a.run()
    a.close()
    b = B.Solver(p, precision=B.OCI_FP64, tol=1e-11, solver=B.OCI_SOLVE_STRUCTURED)
    got, ginfo = b.run_steps()
    b.close()
    assert ginfo == winfo
    assert np.array_equal(got, want)
    ref = oracle.Oracle(p).run("oci", tol=1e-14)["phi"]
    assert rel(got, ref) <= 1e-10


def test_structured_rejects_unsupported_options():
    p = W.homogeneous(J=16, N=4)
    for kw in (dict(precision=B.OCI_FP32_REFINED), dict(norm=B.OCI_NORM_ANGULAR)):
        with pytest.raises(B.OciError) as e:
            B.Solver(p, solver=B.OCI_SOLVE_STRUCTURED, **kw)
        assert e.value.code == B.OCI_ERR_UNSUPPORTED


# ------------------------------------------------- time-dependent sources
def _time_dependent(steps=4):
    """A problem whose source and incident fluxes change every step."""
    p = W.multigroup(seed=9, J=96, N=8, G=2, n_regions=8, length=2.0, speeds=(3.0, 1.0), dt=0.2,
                     steps=steps)
    rng = np.random.default_rng(41)
    qs = [rng.uniform(0, 2, size=(96, 2, 4)) for _ in range(steps)]
    ls = [rng.uniform(0, 1, size=(2, 2, 4)) for _ in range(steps)]
    rs = [rng.uniform(0, 1, size=(2, 2, 4)) for _ in range(steps)]
    return p, qs, ls, rs


def _oracle_time_dependent(p, qs, ls, rs, **kw):
    o = oracle.Oracle(p)
    pp, pi = o.initial_state()
    out = []
    for q, l, r in zip(qs, ls, rs):
        phi, _ = o.step("oci", pp, pi, q=q, inc_l=l, inc_r=r, **kw)
        out.append(phi)
    return np.stack(out)


@pytest.mark.parametrize("prec,solver", [(B.OCI_FP64, B.OCI_SOLVE_DENSE), (B.OCI_FP32_REFINED, B.OCI_SOLVE_DENSE),
                                         (B.OCI_FP64, B.OCI_SOLVE_STRUCTURED)])
def test_capture_steps_time_dependent_sources(prec, solver):
    """Steps captured into a graph with per-step sources and incident fluxes
    equal eager oci_step calls bit for bit (two replays in a row, the second
    continuing from the first), and the oracle's lock-step answer (FP64)."""
    p, qs, ls, rs = _time_dependent()
    K = len(qs)
    _announce("time_dependent", p, f"capture {K} steps, prec={prec}, solver={solver}")
    dev = lambda a: torch.as_tensor(a).cuda()
    dq, dl, dr = [dev(x) for x in qs], [dev(x) for x in ls], [dev(x) for x in rs]
    torch.cuda.synchronize()
    kw = dict(precision=prec, solver=solver, fixed_iters=6)
    e = B.Solver(p, **kw)     # eager steps on torch's current stream, where the clones run
    want = []
    for rep in range(2):
        for k in range(K):
            B.oci_step(e.h, dq[k], dl[k], dr[k], e.phi, None, e.info)
            want.append(e.phi.clone())
    e.stream.synchronize()
    e.close()
    s = B.Solver(p, stream=torch.cuda.Stream(), **kw)
    phis = [torch.zeros_like(s.phi) for _ in range(K)]
    infos = torch.zeros(24 * K, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    B.oci_capture_steps(s.h, K, dq, dl, dr, phis, None, infos)
    got = []
    for rep in range(2):
        B.oci_replay_steps(s.h)
        s.stream.synchronize()
        got += [f.clone() for f in phis]
        inf = infos.cpu().numpy()
        assert all(B.decode_info(inf[24 * k:24 * k + 24])["iterations"] == 6 for k in range(K))
    s.close()
    for a, b in zip(got, want):
        assert torch.equal(a, b)
    if prec == B.OCI_FP64:
        ref = _oracle_time_dependent(p, qs, ls, rs, fixed_iters=6)
        assert rel(torch.stack(got[:K]).cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("prec", [B.OCI_FP64, B.OCI_FP32_REFINED])
def test_run_steps_strided_sources(prec):
    """oci_run_steps with one source and incident-flux array per step (the
    register-resident kernel turns each step over with the next step's
    arrays) equals one oci_step call per step bit for bit."""
    p, qs, ls, rs = _time_dependent(steps=5)
    K = len(qs)
    _announce("time_dependent", p, f"oci_run_steps with strides, prec={prec}")
    qa = torch.as_tensor(np.stack(qs)).cuda()
    la = torch.as_tensor(np.stack(ls)).cuda()
    ra = torch.as_tensor(np.stack(rs)).cuda()
    torch.cuda.synchronize()
    e = B.Solver(p, precision=prec, tol=1e-10)
    want, winfo = [], []
    for k in range(K):
        B.oci_step(e.h, qa[k], la[k], ra[k], e.phi, None, e.info)
        want.append(e.phi.clone())
        winfo.append(e.info.clone())
    e.stream.synchronize()
    e.close()
    s = B.Solver(p, precision=prec, tol=1e-10)
    resident = s.config()["resident"]
    phis = torch.empty((K,) + tuple(s.phi.shape), dtype=torch.float64, device="cuda")
    infos = torch.zeros((K, 24), dtype=torch.uint8, device="cuda")
    B.oci_run_steps(s.h, K, qa, la, ra, phis, None, infos, q_stride=qa[0].numel(), inc_stride=la[0].numel())
    s.stream.synchronize()
    s.close()
    if prec == B.OCI_FP32_REFINED:
        assert resident, "the multi-step launch needs the register-resident kernel here"
    assert torch.equal(phis, torch.stack(want))
    assert [B.decode_info(i.cpu().numpy()) for i in infos] == [B.decode_info(i[:24].cpu().numpy()) for i in winfo]
    if prec == B.OCI_FP64:
        ref = _oracle_time_dependent(p, qs, ls, rs, tol=1e-14)
        assert rel(phis.cpu().numpy(), ref) <= 1e-9


@pytest.mark.parametrize("name,solver", [("regions512_n64", B.OCI_SOLVE_DENSE), ("multigroup128_n256", B.OCI_SOLVE_DENSE),
                                         ("multigroup128_n256", B.OCI_SOLVE_STRUCTURED)])
def test_singular_cell_reported(name, solver, monkeypatch):
    """A cell whose matrix has a zero pivot (the setup's test hook zeroes its
    first column) makes oci_setup return OCI_ERR_SINGULAR and no handle,
    through the C ABI, for both setup kernels and the structured setup."""
    import ctypes as C
    p, _ = CASES[name]
    monkeypatch.setenv("OCI_TEST_ZERO_PIVOT_CELL", str(p["J"] // 2))
    _announce(name, p, f"singular cell, solver={solver}")
    d, keep = B.make_desc(p, solver=solver)
    nbytes = B.oci_workspace_bytes(d)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
    h = C.c_void_p(1)
    rc = B.lib().oci_setup(C.byref(d), ptr, nbytes, None, C.byref(h))
    assert rc == B.OCI_ERR_SINGULAR
    assert not h.value
    monkeypatch.delenv("OCI_TEST_ZERO_PIVOT_CELL")
    rc = B.lib().oci_setup(C.byref(d), ptr, nbytes, None, C.byref(h))
    assert rc == B.OCI_OK and h.value
    B.oci_destroy(h)


# ------------------------------- red-black ordering, periodic mesh, history
@pytest.mark.parametrize("name", ["homogeneous64_n32", "regions512_n64", "multigroup128_n256", "odd_N6_n24",
                                  "G3_N16_n192", "N2_J5", "single_cell"])
def test_structured_red_black_lockstep(name):
    """Red-black OCI (even cells from the previous iterate, then odd cells
    from the even cells' new values) against the oracle's red-black iteration
    in lock-step (<= 1e-12)."""
    p, steps = CASES[name]
    K = 6
    _announce(name, p, f"structured red-black lock-step K={K}")
    want = oracle.Oracle(p).run("oci", steps=steps, fixed_iters=K, ordering=oracle.ORDER_RED_BLACK)
    s = B.Solver(p, precision=B.OCI_FP64, fixed_iters=K, solver=B.OCI_SOLVE_STRUCTURED,
                 ordering=B.OCI_ORDER_RED_BLACK)
    got, infos = s.run(steps=steps, want_psi=True)
    psi = s.psi.cpu().numpy()
    s.close()
    assert all(i["iterations"] == K and i["status"] == 0 for i in infos), infos
    assert rel(got, want["phi"]) <= 1e-12
    assert rel(psi, want["psi_iter"]) <= 1e-12


def test_structured_red_black_converges_in_fewer_iterations():
    """Converged red-black steps reach the Jacobi answer (the same fixed
    point) in about half the iterations (the spectral radius squares)."""
    p = dict(CASES["regions512_n64"][0], steps=2)
    _announce("regions512_n64", p, "red-black vs Jacobi, converged")
    out = {}
    for ordering in (B.OCI_ORDER_JACOBI, B.OCI_ORDER_RED_BLACK):
        s = B.Solver(p, precision=B.OCI_FP64, tol=1e-12, solver=B.OCI_SOLVE_STRUCTURED, ordering=ordering)
        out[ordering] = s.run()
        s.close()
    ref = oracle.Oracle(p).run("oci", tol=1e-14)["phi"]
    for ordering, (phi, infos) in out.items():
        assert all(i["status"] == 0 for i in infos)
        assert rel(phi, ref) <= 1e-10, ordering
    ij = [i["iterations"] for i in out[B.OCI_ORDER_JACOBI][1]]
    irb = [i["iterations"] for i in out[B.OCI_ORDER_RED_BLACK][1]]
    print(f"  iterations per step: Jacobi {ij}, red-black {irb}", flush=True)
    assert all(b < 0.7 * a for a, b in zip(ij, irb))


@pytest.mark.parametrize("ordering", [B.OCI_ORDER_JACOBI, B.OCI_ORDER_RED_BLACK])
def test_periodic_history_matches_oracle_and_fourier_symbol(ordering):
    """The paper's verification setting (section 3.1) on a periodic mesh:
    homogeneous slab, Sigma = 2.5, dx = 0.1, c = 0.9, dt = 0.1, v = 4 (tau = 1),
    S8, no source and a random start.  The GPU's e_l history, filled by the
    kernel in one run, equals the oracle's (periodic mesh), and its decay
    rate, fitted while e_l stays far above its rounding floor, matches the
    spectral radius of the Fourier symbol at the mesh's wave numbers (its
    square for red-black)."""
    J = 200
    p = W.fourier_verification(J=J)
    K, lo, hi = (60, 15, 55) if ordering == B.OCI_ORDER_JACOBI else (30, 6, 26)
    _announce("fourier_verification_periodic", p, f"history, ordering {ordering}")
    o = oracle.Oracle(p, periodic=True, methods=("oci",))
    pp, pi = o.initial_state(p["psi_init"])
    _, oinfo = o.step("oci", pp, pi, q=p["q"], fixed_iters=K, history=True, ordering=ordering)
    want = oinfo["e_hist"]
    s = B.Solver(p, precision=B.OCI_FP64, fixed_iters=K, solver=B.OCI_SOLVE_STRUCTURED, ordering=ordering,
                 boundary=B.OCI_BOUNDARY_PERIODIC)
    hist = torch.full((K + 8,), -1.0, dtype=torch.float64, device="cuda")
    B.oci_set_history(s.h, hist, K)
    _, infos = s.run(steps=1)
    s.close()
    got = hist.cpu().numpy()
    assert infos[0]["iterations"] == K
    assert np.all(got[K:] == -1.0)
    floor = 1e-14 * np.sqrt(p["J"] * 4) * np.abs(want).max()
    assert np.all(np.abs(got[:K] - want) <= 1e-11 * want + floor)
    p1 = BAL.one_cell(p)
    rho = max(np.abs(np.linalg.eigvals(BAL.oci_symbol(p1, 2 * np.pi * k / J))).max() for k in range(J))
    if ordering == B.OCI_ORDER_RED_BLACK:
        rho = rho ** 2
    l = np.arange(lo, hi)
    rate = np.exp(np.polyfit(l, np.log(got[lo:hi]), 1)[0])
    print(f"  fitted rate {rate:.5f}, symbol radius {rho:.5f}, e_l from {got[lo]:.2e} to {got[hi - 1]:.2e}",
          flush=True)
    # the dominant eigenvalues are complex, so e_l oscillates about the decay
    # (section 3.1): the fitted rate lands within a few percent of the radius
    assert abs(rate - rho) < 0.05 * rho


@pytest.mark.parametrize("prec,solver", [(B.OCI_FP64, B.OCI_SOLVE_DENSE), (B.OCI_FP32_REFINED, B.OCI_SOLVE_DENSE),
                                         (B.OCI_FP64, B.OCI_SOLVE_STRUCTURED)])
def test_checkpoint_restart_is_bitwise(prec, solver):
    """Ten steps in one run equal five steps, a checkpoint (psi_{k-1/2} and
    the next first iterate), a fresh handle restored from it and five more
    steps, bit for bit: fluxes, step reports and the final state."""
    p = dict(W.multigroup(seed=9, J=96, N=8, G=2, n_regions=8, length=2.0, speeds=(3.0, 1.0), dt=0.2,
                          steps=10))
    _announce("checkpoint", p, f"10 steps vs 5 + checkpoint + 5, prec={prec}, solver={solver}")
    kw = dict(precision=prec, tol=1e-10, solver=solver)
    a = B.Solver(p, **kw)
    want, winfo = a.run(steps=10)
    wstate = a.get_state().cpu().numpy()
    a.close()
    b = B.Solver(p, **kw)
    first, _ = b.run(steps=5)
    pp, pi = b.checkpoint()
    b.close()
    c = B.Solver(p, **kw)
    c.restore(pp, pi)
    rest, rinfo = c.run(steps=5)
    rstate = c.get_state().cpu().numpy()
    c.close()
    assert np.array_equal(first, want[:5])
    assert np.array_equal(rest, want[5:])
    assert rinfo == winfo[5:]
    assert np.array_equal(rstate, wstate)
