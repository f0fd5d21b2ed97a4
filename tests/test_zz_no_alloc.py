"""The allocation-free setup, oci_setup_static, against oci_setup.

oci_setup_static runs the same setup and step kernels on a workspace held in
the library's own device memory instead of a caller-provided one.  Its time
steps must equal those of a handle from oci_setup bit for bit (same kernels,
same launch shapes); two calls in a row, the second with a smaller problem,
check that the array is taken over cleanly.  A problem too large for the
array is rejected before anything runs (host check)."""
import ctypes as C

import numpy as np
import pytest

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


def _steps(h, p, steps):
    phi = torch.empty((p["J"], p["G"], 4), dtype=torch.float64, device="cuda")
    info = torch.zeros(32, dtype=torch.uint8, device="cuda")
    q = torch.as_tensor(p["q"]).cuda()
    torch.cuda.synchronize()
    out, infos = [], []
    for _ in range(steps):
        B.oci_step(h, q, None, None, phi, None, info)
        out.append(phi.clone())
        infos.append(info.clone())
    torch.cuda.synchronize()
    return torch.stack(out).cpu().numpy(), [B.decode_info(i.cpu().numpy()) for i in infos]


@pytest.mark.parametrize("prec", [B.OCI_FP64, B.OCI_FP32_REFINED])
def test_static_setup_equals_workspace_setup_twice(prec):
    cases = [("regions512_n64", W.regions(seed=2, J=512, N=16, n_regions=64, length=8.0, dt=0.1)),
             ("homogeneous40_n16", W.homogeneous(J=40, N=4))]   # the second call is smaller
    for name, p in cases:
        print(f"\n[gpu no-alloc] {name}: J={p['J']} N={p['N']} G={p['G']} prec={prec}", flush=True)
        d, keep = B.make_desc(p, precision=prec, tol=1e-11)
        ref = B.Solver(p, precision=prec, tol=1e-11)
        want, winfo = _steps(ref.h, p, 3)
        ref.close()
        h = B.oci_setup_static(d, None)
        got, ginfo = _steps(h, p, 3)
        B.oci_destroy(h)
        assert ginfo == winfo
        assert np.array_equal(got, want)
        assert all(i["status"] == 0 for i in ginfo)


def test_static_setup_rejects_a_problem_beyond_the_array():
    p = W.regions(seed=2, J=4096, N=16, n_regions=64, length=64.0, dt=0.1)
    d, keep = B.make_desc(p)        # 128 MiB of FP64 inverses alone
    h = C.c_void_p(1)
    assert B.lib().oci_setup_static(C.byref(d), None, C.byref(h)) == B.OCI_ERR_TOO_LARGE
    assert not h.value
