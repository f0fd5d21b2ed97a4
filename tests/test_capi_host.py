"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/oci.h declares, and rejects bad arguments before
launching anything."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2503_00264_amd import binding as B
from paper_2503_00264_amd import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "oci.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_binding_names():
    assert declared_functions() == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = B.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
        C.cast(getattr(L, name), C.c_void_p)


def test_status_strings():
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6):
        assert B.oci_status_string(code) != "unknown status"
    assert B.oci_status_string(99) == "unknown status"


def _desc(**over):
    p = W.homogeneous(J=16, N=4)
    d, keep = B.make_desc(p)
    for k, v in over.items():
        setattr(d, k, v)
    return d, keep


@pytest.mark.parametrize("field,value", [("J", 0), ("N", 3), ("N", 0), ("G", 0), ("dt", 0.0),
                                         ("dt", float("nan")), ("tol", -1.0), ("max_iters", 0),
                                         ("fixed_iters", -1), ("precision", 2), ("norm", 5),
                                         ("dx", None)])
def test_invalid_descriptions_rejected(field, value):
    d, keep = _desc(**{field: value})
    with pytest.raises(B.OciError) as e:
        B.oci_workspace_bytes(d)
    assert e.value.code == B.OCI_ERR_INVALID


@pytest.mark.parametrize("array,bad", [("dx", 0.0), ("dx", -1.0), ("sigma_t", -0.1),
                                       ("sigma_s", float("inf")), ("speed", 0.0)])
def test_invalid_material_data_rejected(array, bad):
    p = W.homogeneous(J=16, N=4)
    p[array] = p[array].copy()
    p[array].reshape(-1)[3 % p[array].size] = bad
    d, keep = B.make_desc(p)
    with pytest.raises(B.OciError) as e:
        B.oci_workspace_bytes(d)
    assert e.value.code == B.OCI_ERR_INVALID


def test_oversized_cell_system_unsupported():
    p = W.multigroup(seed=1, J=64, N=64, G=4, n_regions=64, speeds=(4, 3, 2, 1))
    d, keep = B.make_desc(p)
    with pytest.raises(B.OciError) as e:
        B.oci_workspace_bytes(d)
    assert e.value.code == B.OCI_ERR_UNSUPPORTED


def test_workspace_size_covers_the_factors():
    for name, prec, es in (("regions4096", B.OCI_FP64, 8), ("regions4096", B.OCI_FP32_REFINED, 4),
                           ("multigroup8192", B.OCI_FP32_REFINED, 4)):
        p = W.config(name)
        d, keep = B.make_desc(p, precision=prec)
        n = 4 * p["N"] * p["G"]
        assert B.oci_workspace_bytes(d) >= p["J"] * n * n * es + 2 * p["J"] * n * 8


def test_setup_rejects_bad_workspace_without_touching_it():
    d, keep = _desc()
    need = B.oci_workspace_bytes(d)
    h = C.c_void_p()
    L = B.lib()
    assert L.oci_setup(C.byref(d), None, need, None, C.byref(h)) == B.OCI_ERR_WORKSPACE
    assert L.oci_setup(C.byref(d), 256 + 8, need, None, C.byref(h)) == B.OCI_ERR_WORKSPACE
    assert L.oci_setup(C.byref(d), 4096, need - 1, None, C.byref(h)) == B.OCI_ERR_WORKSPACE
    assert L.oci_setup(C.byref(d), 4096, need, None, None) == B.OCI_ERR_INVALID


def test_step_calls_reject_null_handle_and_outputs():
    L = B.lib()
    assert L.oci_step(None, None, None, None, None, None, None) == B.OCI_ERR_INVALID
    assert L.si_step(None, None, None, None, None, None, None) == B.OCI_ERR_INVALID
    assert L.oci_run_steps(None, 3, None, 0, None, None, 0, None, None, None) == B.OCI_ERR_INVALID
    assert L.oci_run_steps(None, 0, None, 0, None, None, 0, None, None, None) == B.OCI_ERR_INVALID
    assert L.oci_capture_steps(None, 2, None, None, None, None, None, None) == B.OCI_ERR_INVALID
    assert L.oci_replay_steps(None) == B.OCI_ERR_INVALID
    assert L.oci_set_state(None, None) == B.OCI_ERR_INVALID
    assert L.oci_get_state(None, None) == B.OCI_ERR_INVALID
    assert L.oci_destroy(None) == B.OCI_ERR_INVALID


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(ImportError):
        B.lib()


def test_product_code_does_not_reference_the_oracle():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_2503_00264_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), os.path.join(dirpath, f)


@pytest.mark.parametrize("over", [dict(solver=2), dict(solver=-1)])
def test_unknown_solver_rejected(over):
    d, keep = _desc(**over)
    n = C.c_size_t(0)
    assert B.lib().oci_workspace_bytes(C.byref(d), C.byref(n)) == B.OCI_ERR_INVALID


@pytest.mark.parametrize("over", [dict(precision=B.OCI_FP32_REFINED), dict(norm=B.OCI_NORM_ANGULAR)])
def test_structured_solve_options_unsupported(over):
    d, keep = _desc(solver=B.OCI_SOLVE_STRUCTURED, **over)
    n = C.c_size_t(0)
    assert B.lib().oci_workspace_bytes(C.byref(d), C.byref(n)) == B.OCI_ERR_UNSUPPORTED


def test_structured_workspace_holds_no_dense_factors():
    p = W.multigroup(seed=3, J=64, N=16, G=4, n_regions=8, length=1.0, dt=1e-3)
    dense, k1 = B.make_desc(p)
    struct, k2 = B.make_desc(p, solver=B.OCI_SOLVE_STRUCTURED)
    nd, ns = B.oci_workspace_bytes(dense), B.oci_workspace_bytes(struct)
    # the dense form stores 64 cells x 256^2 FP64 words; the structured form
    # 64 cells x 16 G^2 words of capacitance rows and a double-buffered
    # [J][G][N][2] array of outgoing corners instead
    assert nd - ns == 64 * 256 * 256 * 8 - (64 * 16 * 16 * 8 + 2 * 64 * 64 * 2 * 8)
