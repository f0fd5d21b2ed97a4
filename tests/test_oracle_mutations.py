"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a flipped sign, a dropped term, a wrong index,
a transposed operand) in a copy of the oracle source, compiles that copy on
the CPU and checks that at least one pin from the battery below fails.  The
product library is not involved.
"""
import os

import numpy as np
import pytest

import balance as B
import oracle
from paper_2503_00264_amd import workloads as W

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "oci_oracle.c")).read()

MUTATIONS = {
    "sign_mu_half": ("r0[0] = d;      r0[1] = h;", "r0[0] = d;      r0[1] = -h;"),
    "sign_time_coupling": ("r2[0] = -a;", "r2[0] = a;"),
    "drop_half_a": ("r0[2] = 0.5 * a;", "r0[2] = 0.0;"),
    "abs_mu_dropped": ("const double d = 0.5 * (fabs(mu[m]) + dx * sig);  /* (|mu| + dx Sigma)/2 */",
                       "const double d = 0.5 * (mu[m] + dx * sig);"),
    "scatter_weight_index": ("A[(size_t)r * n + c] -= s * w[nn];", "A[(size_t)r * n + c] -= s * w[m];"),
    "scatter_transposed": ("const double s = 0.25 * dx * p->sigma_s[((size_t)j * G + g) * G + gp];",
                           "const double s = 0.25 * dx * p->sigma_s[((size_t)j * G + gp) * G + g];"),
    "scatter_any_corner": ("                        const int c = (gp * N + nn) * 4 + u;",
                           "                        const int c = (gp * N + nn) * 4 + (u ^ 1);"),
    "prev_time_corner": ("out[1] += a2 * psi_prev[IDX2(p, j, g, m, 1)];",
                         "out[1] += a2 * psi_prev[IDX2(p, j, g, m, 0)];"),
    "upstream_corner": ("return psi[IDX4(p, jn, g, m, lev == 0 ? 1 : 3)];",
                        "return psi[IDX4(p, jn, g, m, lev == 0 ? 0 : 2)];"),
    "incident_sign": ("c[1] -= mu[m] * ek;", "c[1] += mu[m] * ek;"),
    "incident_level": ("c[2] += mu[m] * eh;", "c[2] += mu[m] * ek;"),
    "source_factor": ("out[u] = q ? 0.25 * dx * q[((size_t)j * p->G + g) * 4 + u] : 0.0;",
                      "out[u] = q ? 0.5 * dx * q[((size_t)j * p->G + g) * 4 + u] : 0.0;"),
    "lu_no_row_swap": ("        if (p != k)\n            for (int c = 0; c < n; ++c) {",
                       "        if (0)\n            for (int c = 0; c < n; ++c) {"),
    "stop_without_rho": ("if (e < c->tol * (1.0 - e / e_prev))", "if (e < c->tol)"),
    "time_update_level": ("psi_prev[IDX2(p, j, g, m, 0)] = psi_iter[IDX4(p, j, g, m, 2)];\n                psi_prev[IDX2(p, j, g, m, 1)] = psi_iter[IDX4(p, j, g, m, 3)];\n            }\n    if (phi_out) memcpy(phi_out, phi_old, sizeof(double) * flen);\n    free(mu); free(w); free(next);",
                          "psi_prev[IDX2(p, j, g, m, 0)] = psi_iter[IDX4(p, j, g, m, 0)];\n                psi_prev[IDX2(p, j, g, m, 1)] = psi_iter[IDX4(p, j, g, m, 1)];\n            }\n    if (phi_out) memcpy(phi_out, phi_old, sizeof(double) * flen);\n    free(mu); free(w); free(next);"),
    "si_scatter_group": ("phi[((size_t)j * G + gp) * 4 + u];", "phi[((size_t)j * G + g) * 4 + u];"),
    "si_upstream_value": ("e0 = pos ? d[1] : d[0];", "e0 = pos ? d[0] : d[1];"),
    "rb_black_from_old_iterate": ("const double *src = colour == 0 ? psi_in : psi_out;",
                                  "const double *src = psi_in;"),
    "rb_black_skipped": ("for (int j = colour; j < p->J; j += 2) {", "for (int j = 0; j < p->J; j += 2) {"),
    "flux_weight": ("for (int m = 0; m < p->N; ++m) s += w[m] * psi[IDX4(p, j, g, m, u)];",
                    "for (int m = 0; m < p->N; ++m) s += psi[IDX4(p, j, g, m, u)];"),
}


def battery():
    """Run the pin battery; returns the names of the pins that failed."""
    failed = []
    p = W.multigroup(seed=7, J=6, N=4, G=2, n_regions=2, length=1.0, speeds=(3.0, 1.0),
                     dt=0.2, steps=1, source_regions=1)
    rng = np.random.default_rng(11)
    inc_l = rng.uniform(size=(2, 2, 2))
    inc_r = rng.uniform(size=(2, 2, 2))
    psi_prev = rng.uniform(size=(6, 2, 4, 2))
    x = B.direct_solve(p, psi_prev, q=p["q"], inc_l=inc_l, inc_r=inc_r)
    scale = np.max(np.abs(x))
    try:
        o = oracle.Oracle(p)
        for method in ("oci", "si"):
            pp, pi = o.initial_state(psi_prev)
            _, info = o.step(method, pp, pi, q=p["q"], inc_l=inc_l, inc_r=inc_r, tol=1e-14,
                             max_iters=3000)
            if info["status"] != 0 or np.max(np.abs(pi - x)) > 1e-11 * scale:
                failed.append(method + "_fixed_point")
            elif not np.array_equal(pp, pi[..., 2:4]):
                failed.append(method + "_time_update")
    except RuntimeError:
        failed.append("setup")
    # a second time step from the first one's state must also match
    try:
        o = oracle.Oracle(p)
        pp, pi = o.initial_state(psi_prev)
        o.step("oci", pp, pi, q=p["q"], inc_l=inc_l, inc_r=inc_r, tol=1e-14, max_iters=3000)
        x2 = B.direct_solve(p, x[..., 2:4].copy(), q=p["q"], inc_l=inc_l, inc_r=inc_r)
        o.step("oci", pp, pi, q=p["q"], inc_l=inc_l, inc_r=inc_r, tol=1e-14, max_iters=3000)
        if np.max(np.abs(pi - x2)) > 1e-11 * scale:
            failed.append("second_step")
    except RuntimeError:
        failed.append("setup2")
    # stopping rule as defined
    pr = W.homogeneous(J=32, N=4, length=32 * 0.05, c=0.99, dt=1.0)   # rho near 0.9
    o = oracle.Oracle(pr, methods=("oci",))
    pp, pi = o.initial_state()
    _, info = o.step("oci", pp, pi, q=pr["q"], tol=1e-8, history=True)
    e = info["e_hist"]
    ok = [l >= 1 and e[l] < 1e-8 * (1 - e[l] / e[l - 1]) for l in range(len(e))]
    if not (ok[-1] and not any(ok[:-1])):
        failed.append("stop_rule")
    # red-black ordering: the same fixed point, and an iteration operator whose
    # spectral radius is the square of the Jacobi one (2-cyclic coupling)
    try:
        o = oracle.Oracle(p)
        pp, pi = o.initial_state(psi_prev)
        _, info = o.step("oci", pp, pi, q=p["q"], inc_l=inc_l, inc_r=inc_r, tol=1e-14,
                         max_iters=3000, ordering=oracle.ORDER_RED_BLACK)
        if info["status"] != 0 or np.max(np.abs(pi - x)) > 1e-11 * scale:
            failed.append("rb_fixed_point")
    except RuntimeError:
        failed.append("setup_rb")
    pq = W.homogeneous(J=6, N=2, length=1.5, c=0.95, dt=0.4)
    o = oracle.Oracle(pq, periodic=True, methods=("oci",))
    nu = 6 * 2 * 4
    radius = {}
    for ordering in (oracle.ORDER_JACOBI, oracle.ORDER_RED_BLACK):
        T = np.zeros((nu, nu))
        for i in range(nu):
            e1 = np.zeros(nu)
            e1[i] = 1.0
            T[:, i] = o.oci_iterate(e1.reshape(6, 1, 2, 4), np.zeros((6, 1, 2, 2)),
                                    ordering=ordering).reshape(nu)
        radius[ordering] = np.abs(np.linalg.eigvals(T)).max()
    if abs(radius[oracle.ORDER_RED_BLACK] - radius[oracle.ORDER_JACOBI] ** 2) > 1e-10:
        failed.append("rb_spectrum")
    # pivoting: a matrix with a zero leading entry
    A = np.array([[0.0, 1.0], [1.0, 1.0]])
    LU, piv, rc = oracle.lu_factor(A)
    if rc != 0 or not np.allclose(oracle.lu_solve(LU, piv, [1.0, 2.0]), [1.0, 1.0]):
        failed.append("lu_pivot")
    return failed


def test_unmodified_oracle_passes_battery():
    assert battery() == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    assert SRC.count(old) == 1, f"mutation anchor for {name} not unique"
    path = oracle.build_variant(SRC.replace(old, new), str(tmp_path / f"mut_{name}.so"))
    with oracle.use_library(path):
        failed = battery()
    assert failed, f"planted mistake {name} was not caught"
