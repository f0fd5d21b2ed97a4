"""FP64 CPU oracle for the OCI / SI slab transport solvers (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this package.  It wraps ``oci_oracle.c`` (plain C, built with gcc)
through ctypes and shares no code with the GPU library.

The problem dicts are the ones of ``paper_2503_00264_amd.workloads`` (plain
arrays, no method arithmetic).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oci_oracle.c")
_LIB = os.path.join(_HERE, "liboci_oracle.so")

OK, NOT_CONVERGED, NONFINITE, ERR_INVALID, ERR_SINGULAR = 0, 1, 2, -1, -3
NORM_SCALAR, NORM_ANGULAR = 0, 1
ORDER_JACOBI, ORDER_RED_BLACK = 0, 1


def build(openmp: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboci_oracle.so."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE",
           "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("J", C.c_int), ("N", C.c_int), ("G", C.c_int),
                ("dx", C.c_void_p), ("sigma_t", C.c_void_p),
                ("sigma_s", C.c_void_p), ("speed", C.c_void_p),
                ("dt", C.c_double), ("periodic", C.c_int)]


class _Control(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iters", C.c_int),
                ("fixed_iters", C.c_int), ("norm", C.c_int), ("ordering", C.c_int)]


class _Info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("status", C.c_int),
                ("e_last", C.c_double), ("rho_e", C.c_double)]


_lib = None


def build_variant(src_text: str, out_path: str) -> str:
    """Compile a modified copy of the oracle source (mutation tests only)."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE",
                    "-I", _HERE, "-o", out_path, src, "-lm"], check=True)
    return out_path


class use_library:
    """Context manager: route every oracle call through another build of it."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _load(_LIB)
    return _lib


def _load(path):
    L = C.CDLL(path)
    vp, ip = C.c_void_p, C.c_int
    P, Ctl, Inf = C.POINTER(_Problem), C.POINTER(_Control), C.POINTER(_Info)
    L.orc_gauss_legendre.argtypes = [ip, vp, vp]
    L.orc_cell_matrix.argtypes = [P, vp, vp, ip, vp]
    L.orc_lu_factor.argtypes = [ip, vp, vp]
    L.orc_lu_solve.argtypes = [ip, vp, vp, vp]
    L.orc_lu_solve.restype = None
    L.orc_oci_setup.argtypes = [P, vp, vp]
    L.orc_oci_iterate.argtypes = [P] + [vp] * 9
    L.orc_oci_iterate_rb.argtypes = [P] + [vp] * 9
    L.orc_oci_step.argtypes = [P, Ctl] + [vp] * 9 + [Inf, vp]
    L.orc_si_setup.argtypes = [P, vp, vp]
    L.orc_si_sweep.argtypes = [P] + [vp] * 9
    L.orc_si_step.argtypes = [P, Ctl] + [vp] * 9 + [Inf, vp]
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def gauss_legendre(N):
    mu = np.empty(N)
    w = np.empty(N)
    rc = lib().orc_gauss_legendre(N, _ptr(mu), _ptr(w))
    if rc:
        raise ValueError(f"gauss_legendre({N}) -> {rc}")
    return mu, w


def lu_factor(A):
    A = np.array(A, dtype=np.float64, order="C")
    n = A.shape[0]
    piv = np.empty(n, dtype=np.int32)
    rc = lib().orc_lu_factor(n, _ptr(A), _ptr(piv))
    return A, piv, rc


def lu_solve(LU, piv, b):
    b = np.array(b, dtype=np.float64)
    lib().orc_lu_solve(LU.shape[0], _ptr(LU), _ptr(piv), _ptr(b))
    return b


class Oracle:
    """Holds one problem (materials, dt) and its factors; steps OCI or SI."""

    def __init__(self, prob, periodic=False, methods=("oci", "si")):
        self.p = prob
        self.J, self.N, self.G = prob["J"], prob["N"], prob["G"]
        self.n = 4 * self.N * self.G
        self._arrs = [_f64(prob["dx"]), _f64(prob["sigma_t"]),
                      _f64(prob["sigma_s"]), _f64(prob["speed"])]
        self.cp = _Problem(self.J, self.N, self.G, *[_ptr(a) for a in self._arrs],
                           float(prob["dt"]), 1 if periodic else 0)
        self.lu = self.piv = self.lu4 = self.piv4 = None
        if "oci" in methods:
            self.lu = np.empty((self.J, self.n, self.n))
            self.piv = np.empty((self.J, self.n), dtype=np.int32)
            rc = lib().orc_oci_setup(C.byref(self.cp), _ptr(self.lu), _ptr(self.piv))
            if rc:
                raise RuntimeError(f"orc_oci_setup -> {rc}")
        if "si" in methods:
            self.lu4 = np.empty((self.J, self.G, self.N, 16))
            self.piv4 = np.empty((self.J, self.G, self.N, 4), dtype=np.int32)
            rc = lib().orc_si_setup(C.byref(self.cp), _ptr(self.lu4), _ptr(self.piv4))
            if rc:
                raise RuntimeError(f"orc_si_setup -> {rc}")

    def cell_matrix(self, j):
        mu, w = gauss_legendre(self.N)
        A = np.empty((self.n, self.n))
        lib().orc_cell_matrix(C.byref(self.cp), _ptr(mu), _ptr(w), j, _ptr(A))
        return A

    def initial_state(self, psi_init=None):
        """psi_prev [J][G][N][2] and the first iterate [J][G][N][4] (reading R3)."""
        if psi_init is None:
            psi_init = np.zeros((self.J, self.G, self.N, 2))
        psi_prev = np.array(psi_init, dtype=np.float64, order="C")
        psi_iter = np.concatenate([psi_prev, psi_prev], axis=-1).copy()
        return psi_prev, psi_iter

    def oci_iterate(self, psi_in, psi_prev, q=None, q_ang=None, inc_l=None, inc_r=None,
                    ordering=ORDER_JACOBI):
        psi_in = _f64(psi_in)
        out = np.empty_like(psi_in)
        q, q_ang, inc_l, inc_r, psi_prev = map(_f64, (q, q_ang, inc_l, inc_r, psi_prev))
        fn = lib().orc_oci_iterate_rb if ordering == ORDER_RED_BLACK else lib().orc_oci_iterate
        fn(C.byref(self.cp), _ptr(self.lu), _ptr(self.piv), _ptr(q),
                              _ptr(q_ang), _ptr(psi_prev), _ptr(inc_l), _ptr(inc_r),
                              _ptr(psi_in), _ptr(out))
        return out

    def si_sweep(self, phi_in, psi_prev, q=None, q_ang=None, inc_l=None, inc_r=None):
        phi_in = _f64(phi_in)
        out = np.empty((self.J, self.G, self.N, 4))
        q, q_ang, inc_l, inc_r, psi_prev = map(_f64, (q, q_ang, inc_l, inc_r, psi_prev))
        lib().orc_si_sweep(C.byref(self.cp), _ptr(self.lu4), _ptr(self.piv4), _ptr(q),
                           _ptr(q_ang), _ptr(psi_prev), _ptr(inc_l), _ptr(inc_r),
                           _ptr(phi_in), _ptr(out))
        return out

    def step(self, method, psi_prev, psi_iter, q=None, q_ang=None, inc_l=None,
             inc_r=None, tol=1e-10, max_iters=100000, fixed_iters=0,
             norm=NORM_SCALAR, history=False, ordering=ORDER_JACOBI):
        """One time step in place on (psi_prev, psi_iter); returns (phi, info dict)."""
        assert psi_prev.flags.c_contiguous and psi_prev.dtype == np.float64
        assert psi_iter.flags.c_contiguous and psi_iter.dtype == np.float64
        ctl = _Control(float(tol), int(max_iters), int(fixed_iters), int(norm), int(ordering))
        info = _Info()
        phi = np.empty((self.J, self.G, 4))
        cap = fixed_iters if fixed_iters > 0 else max_iters
        hist = np.full(cap, np.nan) if history else None
        q, q_ang, inc_l, inc_r = map(_f64, (q, q_ang, inc_l, inc_r))
        if method == "oci":
            fn, f, pv = lib().orc_oci_step, self.lu, self.piv
        elif method == "si":
            fn, f, pv = lib().orc_si_step, self.lu4, self.piv4
        else:
            raise ValueError(method)
        rc = fn(C.byref(self.cp), C.byref(ctl), _ptr(f), _ptr(pv), _ptr(q), _ptr(q_ang),
                _ptr(inc_l), _ptr(inc_r), _ptr(psi_prev), _ptr(psi_iter), _ptr(phi),
                C.byref(info), _ptr(hist))
        if rc < 0:
            raise RuntimeError(f"oracle {method} step -> {rc}")
        out = dict(iterations=info.iterations, status=info.status,
                   e_last=info.e_last, rho_e=info.rho_e)
        if history:
            out["e_hist"] = hist[: info.iterations].copy()
        return phi, out

    def run(self, method, steps=None, tol=1e-10, max_iters=100000, fixed_iters=None,
            norm=NORM_SCALAR, q=None, inc_l=None, inc_r=None, psi_init=None, ordering=ORDER_JACOBI):
        """Run `steps` time steps; fixed_iters may be a per-step list (lock-step)."""
        p = self.p
        steps = p["steps"] if steps is None else steps
        q = p["q"] if q is None else q
        inc_l = p.get("inc_left") if inc_l is None else inc_l
        inc_r = p.get("inc_right") if inc_r is None else inc_r
        psi_prev, psi_iter = self.initial_state(p.get("psi_init") if psi_init is None else psi_init)
        phis, infos = [], []
        for k in range(steps):
            fi = 0
            if fixed_iters is not None:
                fi = fixed_iters[k] if np.ndim(fixed_iters) else int(fixed_iters)
            phi, info = self.step(method, psi_prev, psi_iter, q=q, inc_l=inc_l, inc_r=inc_r,
                                  tol=tol, max_iters=max_iters, fixed_iters=fi, norm=norm,
                                  ordering=ordering)
            phis.append(phi)
            infos.append(info)
        return dict(phi=np.stack(phis), info=infos, psi_prev=psi_prev, psi_iter=psi_iter)
