"""ctypes binding of liboci (include/oci.h): same names, argument marshalling only.

Every computation happens in the gfx950 kernels of liboci.so.  This module
loads the in-tree library (it raises if the library is missing or fails to
load; there is no fallback), converts Python/torch arguments to plain pointers,
and wraps status codes into exceptions.  `Solver` is a convenience holder of
the device buffers one slab problem needs (workspace, inputs, outputs) on top
of the same calls.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboci.so")

OCI_OK, OCI_NOT_CONVERGED, OCI_NONFINITE = 0, 1, 2
OCI_ERR_INVALID, OCI_ERR_HIP, OCI_ERR_SINGULAR = -1, -2, -3
OCI_ERR_WORKSPACE, OCI_ERR_UNSUPPORTED, OCI_ERR_DEVICE = -4, -5, -6
OCI_ERR_TOO_LARGE = -7
OCI_FP64, OCI_FP32_REFINED = 0, 1
OCI_NORM_SCALAR, OCI_NORM_ANGULAR = 0, 1
OCI_SOLVE_DENSE, OCI_SOLVE_STRUCTURED = 0, 1
OCI_ORDER_JACOBI, OCI_ORDER_RED_BLACK = 0, 1
OCI_BOUNDARY_INCIDENT, OCI_BOUNDARY_PERIODIC = 0, 1

# every symbol include/oci.h declares
EXPORTS = ("oci_workspace_bytes", "oci_setup", "oci_setup_static", "oci_set_state", "oci_get_state",
           "oci_get_checkpoint", "oci_set_checkpoint",
           "oci_step", "oci_run_steps", "oci_capture_steps", "oci_replay_steps", "si_step", "oci_profile_enable", "oci_profile_read",
           "oci_autotune", "oci_set_history", "oci_get_config", "oci_destroy", "oci_batch_workspace_bytes", "oci_batch_setup", "oci_batch_bind", "oci_batch_bind_steps",
           "oci_batch_step", "oci_batch_capture", "oci_batch_replay", "oci_batch_set_state",
           "oci_batch_get_state", "oci_batch_rebalance", "oci_batch_info", "oci_batch_destroy", "oci_status_string")


class OciError(RuntimeError):
    def __init__(self, call, code):
        self.code = code
        super().__init__(f"{call} -> {code} ({oci_status_string(code)})")


class oci_desc(C.Structure):
    _fields_ = [("J", C.c_int32), ("N", C.c_int32), ("G", C.c_int32),
                ("dx", C.c_void_p), ("sigma_t", C.c_void_p),
                ("sigma_s", C.c_void_p), ("speed", C.c_void_p),
                ("dt", C.c_double), ("tol", C.c_double),
                ("max_iters", C.c_int32), ("fixed_iters", C.c_int32),
                ("precision", C.c_int32), ("norm", C.c_int32), ("solver", C.c_int32),
                ("ordering", C.c_int32), ("boundary", C.c_int32)]


class oci_step_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("status", C.c_int32),
                ("e_last", C.c_double), ("rho_e", C.c_double)]


_lib = None


def lib():
    """The loaded liboci.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2503_00264_amd.build` (no fallback exists)")
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int
        D = C.POINTER(oci_desc)
        L.oci_workspace_bytes.argtypes = [D, C.POINTER(C.c_size_t)]
        L.oci_setup.argtypes = [D, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.oci_setup_static.argtypes = [D, vp, C.POINTER(vp)]
        L.oci_set_state.argtypes = [vp, vp]
        L.oci_get_state.argtypes = [vp, vp]
        L.oci_get_checkpoint.argtypes = [vp, vp, vp]
        L.oci_set_checkpoint.argtypes = [vp, vp, vp]
        L.oci_step.argtypes = [vp] * 7
        i64 = C.c_int64
        L.oci_run_steps.argtypes = [vp, i32, vp, i64, vp, vp, i64, vp, vp, vp]
        L.oci_capture_steps.argtypes = [vp, i32] + [vp] * 6
        L.oci_replay_steps.argtypes = [vp]
        L.si_step.argtypes = [vp] * 7
        L.oci_profile_enable.argtypes = [vp, i32]
        L.oci_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.oci_destroy.argtypes = [vp]
        L.oci_autotune.argtypes = [vp, i32, vp]
        L.oci_get_config.argtypes = [vp, vp]
        L.oci_set_history.argtypes = [vp, vp, i32]
        L.oci_batch_workspace_bytes.argtypes = [i32, vp, C.POINTER(C.c_size_t)]
        L.oci_batch_setup.argtypes = [i32, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.oci_batch_bind.argtypes = [vp, vp, vp, vp, vp, vp]
        L.oci_batch_bind_steps.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.oci_batch_step.argtypes = [vp]
        L.oci_batch_capture.argtypes = [vp, i32]
        L.oci_batch_replay.argtypes = [vp]
        L.oci_batch_set_state.argtypes = [vp, i32, vp]
        L.oci_batch_get_state.argtypes = [vp, i32, vp]
        L.oci_batch_info.argtypes = [vp, vp, vp]
        L.oci_batch_rebalance.argtypes = [vp]
        L.oci_batch_destroy.argtypes = [vp]
        L.oci_status_string.argtypes = [i32]
        L.oci_status_string.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("oci_status_string",):
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def _ptr(x):
    """Device/host pointer of a torch tensor, numpy array, int or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(type(x))


def _check(call, rc):
    if rc < 0:
        raise OciError(call, rc)
    return rc


def oci_status_string(code):
    return lib().oci_status_string(int(code)).decode()


def make_desc(prob, tol=1e-10, max_iters=100000, fixed_iters=0,
              precision=OCI_FP64, norm=OCI_NORM_SCALAR, dt=None, solver=OCI_SOLVE_DENSE,
              ordering=OCI_ORDER_JACOBI, boundary=OCI_BOUNDARY_INCIDENT):
    """Build an oci_desc from a workload dict; the returned keep-alive tuple
    holds the host arrays the descriptor points to."""
    arrs = tuple(np.ascontiguousarray(prob[k], dtype=np.float64)
                 for k in ("dx", "sigma_t", "sigma_s", "speed"))
    d = oci_desc(int(prob["J"]), int(prob["N"]), int(prob["G"]),
                 *[a.ctypes.data for a in arrs],
                 float(prob["dt"] if dt is None else dt), float(tol), int(max_iters),
                 int(fixed_iters), int(precision), int(norm), int(solver), int(ordering), int(boundary))
    return d, arrs


def oci_workspace_bytes(desc):
    n = C.c_size_t(0)
    _check("oci_workspace_bytes", lib().oci_workspace_bytes(C.byref(desc), C.byref(n)))
    return n.value


def oci_setup(desc, workspace, nbytes, stream=None):
    h = C.c_void_p()
    _check("oci_setup", lib().oci_setup(C.byref(desc), _ptr(workspace), int(nbytes),
                                        _ptr(stream), C.byref(h)))
    return h


def oci_setup_static(desc, stream=None):
    """oci_setup on the library's static device workspace (allocates nothing)."""
    h = C.c_void_p()
    _check("oci_setup_static", lib().oci_setup_static(C.byref(desc), _ptr(stream), C.byref(h)))
    return h


def oci_set_state(h, psi_prev):
    _check("oci_set_state", lib().oci_set_state(h, _ptr(psi_prev)))


def oci_get_state(h, psi_prev):
    _check("oci_get_state", lib().oci_get_state(h, _ptr(psi_prev)))


def oci_get_checkpoint(h, psi_prev, psi_iter):
    _check("oci_get_checkpoint", lib().oci_get_checkpoint(h, _ptr(psi_prev), _ptr(psi_iter)))


def oci_set_checkpoint(h, psi_prev, psi_iter):
    _check("oci_set_checkpoint", lib().oci_set_checkpoint(h, _ptr(psi_prev), _ptr(psi_iter)))


def oci_step(h, q, inc_left, inc_right, phi_out, psi_out, info):
    return _check("oci_step", lib().oci_step(h, _ptr(q), _ptr(inc_left), _ptr(inc_right),
                                             _ptr(phi_out), _ptr(psi_out), _ptr(info)))


def oci_run_steps(h, nsteps, q, inc_left, inc_right, phi_out, psi_out, info, q_stride=0, inc_stride=0):
    """nsteps steps; with strides (in elements) q and the incident fluxes
    hold one array per step, else the same ones serve every step."""
    return _check("oci_run_steps", lib().oci_run_steps(h, nsteps, _ptr(q), int(q_stride), _ptr(inc_left),
                                                       _ptr(inc_right), int(inc_stride), _ptr(phi_out),
                                                       _ptr(psi_out), _ptr(info)))


def oci_capture_steps(h, n_steps, q, inc_left, inc_right, phi_out, psi_out, info):
    """q, inc_left, inc_right, psi_out: lists of n_steps tensors (entries may
    be None) or None; phi_out: list of n_steps tensors; info: n_steps records."""
    _check("oci_capture_steps", lib().oci_capture_steps(h, int(n_steps), _ptr_array(q), _ptr_array(inc_left),
                                                        _ptr_array(inc_right), _ptr_array(phi_out),
                                                        _ptr_array(psi_out), _ptr(info)))


def oci_replay_steps(h):
    _check("oci_replay_steps", lib().oci_replay_steps(h))


def si_step(h, q, inc_left, inc_right, phi_out, psi_out, info):
    return _check("si_step", lib().si_step(h, _ptr(q), _ptr(inc_left), _ptr(inc_right),
                                           _ptr(phi_out), _ptr(psi_out), _ptr(info)))


def oci_profile_enable(h, on=True):
    _check("oci_profile_enable", lib().oci_profile_enable(h, 1 if on else 0))


def oci_profile_read(h):
    """(milliseconds of iteration kernels, steps recorded) since the last read."""
    ms, n = C.c_double(0.0), C.c_int32(0)
    _check("oci_profile_read", lib().oci_profile_read(h, C.byref(ms), C.byref(n)))
    return ms.value, n.value


CONFIG_FIELDS = ("block", "local", "resident", "bar_group", "workgroups", "tiles")


def oci_autotune(h, iters=8):
    cfg = (C.c_int32 * 6)()
    _check("oci_autotune", lib().oci_autotune(h, int(iters), cfg))
    return dict(zip(CONFIG_FIELDS, list(cfg)))


def oci_set_history(h, e_hist, capacity=None):
    """Record e_l of every iteration of later steps into e_hist (a float64
    device tensor), or stop recording (e_hist None)."""
    cap = 0 if e_hist is None else int(e_hist.numel() if capacity is None else capacity)
    _check("oci_set_history", lib().oci_set_history(h, _ptr(e_hist), cap))


def oci_get_config(h):
    cfg = (C.c_int32 * 6)()
    _check("oci_get_config", lib().oci_get_config(h, cfg))
    return dict(zip(CONFIG_FIELDS, list(cfg)))


def oci_destroy(h):
    _check("oci_destroy", lib().oci_destroy(h))


def _desc_array(descs):
    arr = (oci_desc * len(descs))(*descs)
    return arr


def oci_batch_workspace_bytes(descs):
    n = C.c_size_t(0)
    arr = _desc_array(descs)
    _check("oci_batch_workspace_bytes", lib().oci_batch_workspace_bytes(len(descs), arr, C.byref(n)))
    return n.value


def oci_batch_setup(descs, workspace, nbytes, stream=None):
    b = C.c_void_p()
    arr = _desc_array(descs)
    _check("oci_batch_setup", lib().oci_batch_setup(len(descs), arr, _ptr(workspace), int(nbytes),
                                                    _ptr(stream), C.byref(b)))
    return b


def _ptr_array(xs):
    if xs is None:
        return None
    return (C.c_void_p * len(xs))(*[_ptr(x) for x in xs])


def oci_batch_bind(b, q, inc_left, inc_right, phi_out, info):
    _check("oci_batch_bind", lib().oci_batch_bind(b, _ptr_array(q), _ptr_array(inc_left),
                                                  _ptr_array(inc_right), _ptr_array(phi_out), _ptr(info)))


def oci_batch_bind_steps(b, n_steps, q, inc_left, inc_right, phi_out, info):
    """Per-step argument sets: q, inc_left, inc_right, phi_out are lists of
    n_steps * nslab tensors (or None), entry i * nslab + k for step i, slab k."""
    _check("oci_batch_bind_steps", lib().oci_batch_bind_steps(b, int(n_steps), _ptr_array(q), _ptr_array(inc_left),
                                                              _ptr_array(inc_right), _ptr_array(phi_out),
                                                              _ptr(info)))


def oci_batch_step(b):
    _check("oci_batch_step", lib().oci_batch_step(b))


def oci_batch_capture(b, n_steps):
    _check("oci_batch_capture", lib().oci_batch_capture(b, int(n_steps)))


def oci_batch_replay(b):
    _check("oci_batch_replay", lib().oci_batch_replay(b))


def oci_batch_set_state(b, k, psi_prev):
    _check("oci_batch_set_state", lib().oci_batch_set_state(b, int(k), _ptr(psi_prev)))


def oci_batch_get_state(b, k, psi_prev):
    _check("oci_batch_get_state", lib().oci_batch_get_state(b, int(k), _ptr(psi_prev)))


def oci_batch_info(b, nslab):
    tot = C.c_int32(0)
    per = (C.c_int32 * nslab)()
    _check("oci_batch_info", lib().oci_batch_info(b, C.byref(tot), per))
    return tot.value, list(per)


def oci_batch_rebalance(b):
    _check("oci_batch_rebalance", lib().oci_batch_rebalance(b))


def oci_batch_destroy(b):
    _check("oci_batch_destroy", lib().oci_batch_destroy(b))


def decode_info(raw):
    """oci_step_info from its 24 bytes (numpy uint8 array or bytes)."""
    b = bytes(np.asarray(raw, dtype=np.uint8).tobytes())
    info = oci_step_info.from_buffer_copy(b[:C.sizeof(oci_step_info)])
    return dict(iterations=info.iterations, status=info.status,
                e_last=info.e_last, rho_e=info.rho_e)


class Solver:
    """Device buffers for one slab problem plus the liboci handle.

    prob: a workload dict (see workloads.py).  All arrays are copied to the
    current CUDA (HIP) device; steps run on torch's current stream.
    """

    def __init__(self, prob, precision=OCI_FP64, tol=1e-10, max_iters=100000,
                 fixed_iters=0, norm=OCI_NORM_SCALAR, stream=None, dt=None, solver=OCI_SOLVE_DENSE,
                 ordering=OCI_ORDER_JACOBI, boundary=OCI_BOUNDARY_INCIDENT):
        import torch
        self.torch = torch
        self.prob = prob
        self.J, self.N, self.G = prob["J"], prob["N"], prob["G"]
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream() if stream is None else stream
        self.desc, self._keep = make_desc(prob, tol=tol, max_iters=max_iters,
                                          fixed_iters=fixed_iters, precision=precision,
                                          norm=norm, dt=dt, solver=solver, ordering=ordering,
                                          boundary=boundary)
        self.ws_bytes = oci_workspace_bytes(self.desc)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.dev)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr = self.ws.data_ptr() + off
        self.h = oci_setup(self.desc, self.ws_ptr, self.ws_bytes, self.stream.cuda_stream)
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.phi = torch.empty((self.J, self.G, 4), **f64)
        self.psi = torch.empty((self.J, self.G, self.N, 4), **f64)
        self.info = torch.zeros(32, dtype=torch.uint8, device=self.dev)
        self.set_inputs(prob.get("q"), prob.get("inc_left"), prob.get("inc_right"))
        if prob.get("psi_init") is not None and np.any(prob["psi_init"]):
            self.set_state(prob["psi_init"])

    def _dev(self, a):
        if a is None:
            return None
        return self.torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(self.dev)

    def set_inputs(self, q=None, inc_left=None, inc_right=None):
        self.q, self.inc_l, self.inc_r = self._dev(q), self._dev(inc_left), self._dev(inc_right)

    def set_state(self, psi_prev):
        self._state = self._dev(psi_prev)
        oci_set_state(self.h, self._state)

    def get_state(self):
        out = self.torch.empty((self.J, self.G, self.N, 2), dtype=self.torch.float64, device=self.dev)
        oci_get_state(self.h, out)
        return out

    def checkpoint(self):
        """(psi_prev, first iterate of the next step) as device tensors."""
        t = self.torch
        pp = t.empty((self.J, self.G, self.N, 2), dtype=t.float64, device=self.dev)
        pi = t.empty((self.J, self.G, self.N, 4), dtype=t.float64, device=self.dev)
        oci_get_checkpoint(self.h, pp, pi)
        self.stream.synchronize()
        return pp, pi

    def restore(self, psi_prev, psi_iter):
        self._ckpt = (self._dev(psi_prev) if not hasattr(psi_prev, "data_ptr") else psi_prev,
                      self._dev(psi_iter) if not hasattr(psi_iter, "data_ptr") else psi_iter)
        self.torch.cuda.synchronize()
        oci_set_checkpoint(self.h, *self._ckpt)

    def step(self, method="oci", want_psi=False):
        fn = oci_step if method == "oci" else si_step
        fn(self.h, self.q, self.inc_l, self.inc_r, self.phi,
           self.psi if want_psi else None, self.info)

    def last_info(self):
        self.stream.synchronize()
        return decode_info(self.info.cpu().numpy())

    def run(self, steps=None, method="oci", want_psi=False):
        """Run steps; returns (phi per step [steps][J][G][4], infos)."""
        steps = self.prob["steps"] if steps is None else steps
        phis, infos = [], []
        for _ in range(steps):
            self.step(method, want_psi)
            phis.append(self.phi.clone())
            infos.append(self.info.clone())
        self.stream.synchronize()
        return (self.torch.stack(phis).cpu().numpy(),
                [decode_info(i.cpu().numpy()) for i in infos])

    def run_steps(self, steps=None, want_psi=False):
        """`steps` OCI steps in one oci_run_steps call; the same returns as run()."""
        steps = self.prob["steps"] if steps is None else steps
        t = self.torch
        phis = t.empty((steps,) + tuple(self.phi.shape), dtype=t.float64, device=self.dev)
        infos = t.zeros((steps, 24), dtype=t.uint8, device=self.dev)
        oci_run_steps(self.h, steps, self.q, self.inc_l, self.inc_r, phis,
                      self.psi if want_psi else None, infos)
        self.stream.synchronize()
        raw = infos.cpu().numpy()
        return phis.cpu().numpy(), [decode_info(raw[k]) for k in range(steps)]

    def autotune(self, iters=8):
        """Pick the fastest launch shape.  oci_autotune leaves the state at
        zero, so the problem's initial state (if any) is applied again."""
        cfg = oci_autotune(self.h, iters)
        if self.prob.get("psi_init") is not None and np.any(self.prob["psi_init"]):
            self.set_state(self.prob["psi_init"])
        return cfg

    def config(self):
        return oci_get_config(self.h)

    def close(self):
        if self.h is not None:
            self.stream.synchronize()
            oci_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver:
    """Device buffers and the liboci batch handle for a list of slab problems.

    All slabs use one precision; steps run on a dedicated (default-priority)
    stream so they can be captured into a graph.
    """

    def __init__(self, probs, precision=OCI_FP32_REFINED, tol=1e-10, max_iters=100000,
                 fixed_iters=0, stream=None, solver=OCI_SOLVE_DENSE, ordering=OCI_ORDER_JACOBI):
        import torch
        self.torch = torch
        self.probs = probs
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.Stream() if stream is None else stream
        made = [make_desc(p, tol=tol, max_iters=max_iters, fixed_iters=fixed_iters,
                          precision=precision, solver=solver, ordering=ordering) for p in probs]
        self.descs = [d for d, _ in made]
        self._keep = [k for _, k in made]
        self.ws_bytes = oci_batch_workspace_bytes(self.descs)
        with torch.cuda.stream(self.stream):
            self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.dev)
        off = (-self.ws.data_ptr()) % 256
        self.b = oci_batch_setup(self.descs, self.ws.data_ptr() + off, self.ws_bytes,
                                 self.stream.cuda_stream)
        f64 = dict(dtype=torch.float64, device=self.dev)
        with torch.cuda.stream(self.stream):
            self.q = [self._dev(p.get("q")) for p in probs]
            self.inc_l = [self._dev(p.get("inc_left")) for p in probs]
            self.inc_r = [self._dev(p.get("inc_right")) for p in probs]
            self.phi = [torch.zeros((p["J"], p["G"], 4), **f64) for p in probs]
            self.info = torch.zeros(24 * len(probs), dtype=torch.uint8, device=self.dev)
        self.stream.synchronize()
        oci_batch_bind(self.b, self.q, self.inc_l, self.inc_r, self.phi, self.info)
        for k, p in enumerate(probs):
            if p.get("psi_init") is not None and np.any(p["psi_init"]):
                self.set_state(k, p["psi_init"])

    def _dev(self, a):
        if a is None:
            return None
        return self.torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(self.dev)

    def bind_steps(self, n_steps, q=None, inc_left=None, inc_right=None):
        """Bind n_steps argument sets: per-step outputs (self.phi_steps[i][k],
        self.info_steps) and, optionally, per-step sources given as lists of
        n_steps lists of per-slab arrays (None: the problem's own, every step)."""
        t = self.torch
        ns = len(self.probs)
        f64 = dict(dtype=t.float64, device=self.dev)

        def per_step(arg, own):
            if arg is None:
                return [own[k] for _ in range(n_steps) for k in range(ns)]
            return [self._dev(arg[i][k]) for i in range(n_steps) for k in range(ns)]

        with t.cuda.stream(self.stream):
            self._step_q = per_step(q, self.q)
            self._step_l = per_step(inc_left, self.inc_l)
            self._step_r = per_step(inc_right, self.inc_r)
            self.phi_steps = [[t.zeros((p["J"], p["G"], 4), **f64) for p in self.probs] for _ in range(n_steps)]
            self.info_steps = t.zeros(24 * ns * n_steps, dtype=t.uint8, device=self.dev)
        self.stream.synchronize()
        oci_batch_bind_steps(self.b, n_steps, self._step_q, self._step_l, self._step_r,
                             [f for row in self.phi_steps for f in row], self.info_steps)
        self.n_bound = n_steps

    def step_results(self):
        """(phi [step][slab] as numpy, info [step][slab]) of the bound argument sets."""
        self.stream.synchronize()
        raw = self.info_steps.cpu().numpy()
        ns = len(self.probs)
        return ([[f.cpu().numpy() for f in row] for row in self.phi_steps],
                [[decode_info(raw[24 * (i * ns + k):24 * (i * ns + k + 1)]) for k in range(ns)]
                 for i in range(self.n_bound)])

    def step(self):
        oci_batch_step(self.b)

    def capture(self, n_steps):
        oci_batch_capture(self.b, n_steps)

    def replay(self):
        oci_batch_replay(self.b)

    def results(self):
        """(phi per slab as numpy, info per slab) after synchronising the stream."""
        self.stream.synchronize()
        raw = self.info.cpu().numpy()
        return ([f.cpu().numpy() for f in self.phi],
                [decode_info(raw[24 * k:24 * (k + 1)]) for k in range(len(self.probs))])

    def get_state(self, k):
        p = self.probs[k]
        out = self.torch.empty((p["J"], p["G"], p["N"], 2), dtype=self.torch.float64, device=self.dev)
        oci_batch_get_state(self.b, k, out)
        self.stream.synchronize()
        return out.cpu().numpy()

    def set_state(self, k, psi_prev):
        self._state = self._dev(psi_prev)
        self.torch.cuda.synchronize()
        oci_batch_set_state(self.b, k, self._state)

    def geometry(self):
        return oci_batch_info(self.b, len(self.probs))

    def rebalance(self):
        """Re-size the slabs' workgroup blocks from the last step's iterations."""
        oci_batch_rebalance(self.b)

    def close(self):
        if self.b is not None:
            self.stream.synchronize()
            oci_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
