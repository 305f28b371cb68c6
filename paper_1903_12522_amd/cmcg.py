"""Python binding of libcmcg (include/cmcg.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module converts NumPy inputs to the C
structs, passes torch device pointers and a torch stream that each call orders after the
caller's current stream, and converts outputs back.
If the built library is missing, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcmcg.so")

# torch is loaded first so that libcmcg binds (by SONAME) to the HIP runtime torch already
# mapped: one HIP/HSA runtime per process, shared device memory and streams.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1903_12522_amd.build` "
                      "or __graft_entry__.build() first")
_lib = ctypes.CDLL(LIB_PATH)

OK, ENOTCONV, EINVAL, ECFL, ENOMEM, EDEVICE, EBREAKDOWN, EUNSUPPORTED = 0, 1, -1, -2, -3, -4, -5, -6
FP64, FP32_MIXED = 0, 1
OP_FORWARD, OP_FORCED, OP_ADJOINT, OP_RIESZ = 0, 1, 2, 3

_dp = ctypes.POINTER(ctypes.c_double)


MAX_SHOTS = 8


class _Shot(ctypes.Structure):
    _fields_ = [("harmonic", ctypes.c_int32), ("f_re", _dp), ("f_im", _dp),
                ("gS_re", _dp), ("gS_im", _dp), ("gD_re", _dp), ("gD_im", _dp)]


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("formulation", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("omega", ctypes.c_double),
                ("c", _dp), ("c_const", ctypes.c_double),
                ("f_re", _dp), ("f_im", _dp), ("gS_re", _dp), ("gS_im", _dp),
                ("sound_soft", ctypes.POINTER(ctypes.c_uint8)), ("gD_re", _dp), ("gD_im", _dp),
                ("face_bc", ctypes.c_int32 * 6), ("courant", ctypes.c_double),
                ("n_shots", ctypes.c_int32), ("shots", ctypes.POINTER(_Shot))]


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("device", ctypes.c_int32),
                ("hip_stream", ctypes.c_void_p), ("steps_per_launch", ctypes.c_int32),
                ("riesz_max_iter", ctypes.c_int32), ("riesz_tol", ctypes.c_double),
                ("fp64_refresh", ctypes.c_double), ("riesz_mode", ctypes.c_int32),
                ("runup_periods", ctypes.c_int32), ("output", ctypes.c_int32)]


class _Report(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("steps_per_period", ctypes.c_int32),
                ("dt", ctypes.c_double), ("rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("seconds_fwd", ctypes.c_double),
                ("seconds_adj", ctypes.c_double), ("seconds_riesz", ctypes.c_double),
                ("seconds_other", ctypes.c_double), ("grid_updates", ctypes.c_double),
                ("riesz_iterations", ctypes.c_int64), ("fp64_refreshes", ctypes.c_int32),
                ("runup_periods", ctypes.c_int32), ("seconds_runup", ctypes.c_double),
                ("dram_bytes", ctypes.c_double), ("riesz_unconverged", ctypes.c_int32),
                ("seconds_bulk_fwd", ctypes.c_double), ("seconds_bulk_adj", ctypes.c_double),
                ("bulk_launches_fwd", ctypes.c_int64), ("bulk_launches_adj", ctypes.c_int64)]


class _Info(ctypes.Structure):
    _fields_ = [("steps_per_period", ctypes.c_int32), ("dt", ctypes.c_double),
                ("T", ctypes.c_double), ("h", ctypes.c_double), ("state_len", ctypes.c_int64),
                ("field_len", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("n_fields", ctypes.c_int32), ("steps_per_launch", ctypes.c_int32),
                ("block_rows", ctypes.c_int32), ("block_waves", ctypes.c_int32)]


class _ServerOptions(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("steps_per_launch", ctypes.c_int32), ("device", ctypes.c_int32),
                ("hip_stream", ctypes.c_void_p), ("barrier_spin_limit", ctypes.c_int64)]


_H = ctypes.c_void_p
_sig = {
    "cmcg_create": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.POINTER(_Options),
                                   ctypes.POINTER(_H)]),
    "cmcg_solve": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Report)]),
    "cmcg_destroy": (None, [_H]),
    "cmcg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "cmcg_last_error": (ctypes.c_char_p, []),
    "cmcg_get_info": (ctypes.c_int, [_H, ctypes.POINTER(_Info)]),
    "cmcg_apply": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_void_p]),
    "cmcg_filter": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cmcg_step6": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cmcg_begin": (ctypes.c_int, [_H]),
    "cmcg_iterate": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(_Report)]),
    "cmcg_finish": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Report)]),
    "cmcg_get_state": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_void_p]),
    "cmcg_runup": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "cmcg_misfit": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "cmcg_server_create": (ctypes.c_int, [ctypes.POINTER(_ServerOptions), ctypes.POINTER(_H)]),
    "cmcg_server_submit": (ctypes.c_int, [_H, ctypes.POINTER(_Problem), ctypes.POINTER(_Options),
                                          ctypes.POINTER(ctypes.c_int64)]),
    "cmcg_server_step": (ctypes.c_int, [_H, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "cmcg_server_poll": (ctypes.c_int, [_H, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(_Report)]),
    "cmcg_server_stats": (ctypes.c_int, [_H, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32)]),
    "cmcg_server_destroy": (None, [_H]),
    "cmcg_server_launches": (ctypes.c_int, [_H, ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int64)]),
    "cmcg_apply_static": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.POINTER(_Options),
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_sig.keys())


class CMCGError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.cmcg_status_string(status).decode()
        detail = _lib.cmcg_last_error().decode()
        super().__init__(f"{where}: {msg} (status {status}){': ' + detail if detail else ''}")


def _check(st: int, where: str, allow_notconv: bool = False) -> int:
    if st == OK or (allow_notconv and st == ENOTCONV):
        return st
    raise CMCGError(st, where)


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _report_dict(r: _Report) -> dict:
    return {k: getattr(r, k) for k, _ in _Report._fields_}


def _concat_faces(parts, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=dtype).ravel() for p in parts]))


def _handle_stream(torch, stream, device):
    """The stream a handle runs on: the caller's non-default stream, else a dedicated one of
    default priority.  (Torch's default stream has the null handle, which the C ABI reads as
    "create your own stream": the handle's work would then be unordered with the caller's.)"""
    if stream is None or stream.cuda_stream == 0:
        stream = torch.cuda.Stream(device=device)
    return stream


class Solver:
    """One CMCG problem on the GPU.  `problem` is a cmcg_inputs.Problem.  Every call first makes
    the handle's stream wait for the caller's current stream, so device inputs written by torch
    are complete; every call returns after the handle's stream has finished."""

    def __init__(self, problem, precision: str = "fp64", tol: float = 1e-6, max_iter: int = 1000,
                 device: int = 0, steps_per_launch: int = 0, stream=None,
                 riesz_tol: float = 0.0, riesz_max_iter: int = 0, fp64_refresh: float = 0.0,
                 riesz_mode="default", runup_periods: int = 0, output="filter"):
        import torch  # device memory and streams
        self._torch = torch
        self.problem = problem
        p, self._keep = marshal_problem(problem)
        o = make_options(precision, tol, max_iter, device, steps_per_launch, riesz_tol,
                         riesz_max_iter, fp64_refresh, riesz_mode, runup_periods, output)
        self.device = device
        self.stream = _handle_stream(torch, stream, device)
        o.hip_stream = ctypes.c_void_p(self.stream.cuda_stream)
        h = _H()
        self._order()
        _check(_lib.cmcg_create(ctypes.byref(p), ctypes.byref(o), ctypes.byref(h)), "cmcg_create")
        self._h = h
        self.precision = precision
        info = _Info()
        _check(_lib.cmcg_get_info(h, ctypes.byref(info)), "cmcg_get_info")
        self.info = {k: getattr(info, k) for k, _ in _Info._fields_}
        # with several shots, the outputs stack one field per shot
        shots = getattr(problem, "shots", None)
        self.field_shape = ((len(shots),) if shots and len(shots) > 1 else ()) + \
            tuple(problem.field_shape())

    # ------------------------------------------------------------------ lifetime
    def _order(self):
        """The handle's stream waits for the caller's current stream."""
        self.stream.wait_stream(self._torch.cuda.current_stream(self.device))

    def close(self):
        if getattr(self, "_h", None):
            _lib.cmcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------ solve
    def solve(self, device_output: bool = False) -> Tuple[object, dict]:
        """Full CMCG solve; returns (u, report).  u is a complex NumPy array of the field shape
        (with several shots: one field per shot, stacked on a leading axis), or a pair of torch
        FP64 device tensors (re, im) if device_output."""
        rep = _Report()
        ure, uim, keep = self._out_buffers(device_output)
        self._order()
        st = _check(_lib.cmcg_solve(self._h, ure, uim, ctypes.byref(rep)), "cmcg_solve",
                    allow_notconv=True)
        d = _report_dict(rep)
        d["converged"] = st == OK
        return self._out_value(keep, device_output), d

    def begin(self):
        self._order()
        _check(_lib.cmcg_begin(self._h), "cmcg_begin")

    def iterate(self, iters: int) -> Tuple[bool, dict]:
        conv = ctypes.c_int32(0)
        rep = _Report()
        self._order()
        _check(_lib.cmcg_iterate(self._h, int(iters), ctypes.byref(conv), ctypes.byref(rep)),
               "cmcg_iterate")
        return bool(conv.value), _report_dict(rep)

    def finish(self, device_output: bool = False):
        rep = _Report()
        ure, uim, keep = self._out_buffers(device_output)
        self._order()
        _check(_lib.cmcg_finish(self._h, ure, uim, ctypes.byref(rep)), "cmcg_finish")
        return self._out_value(keep, device_output), _report_dict(rep)

    # ------------------------------------------------------------------ stage calls
    def apply(self, op: int, z, steps: int = 0, out=None):
        """op(z) on a packed FP64 state; z may be a NumPy array or a torch device tensor.
        Returns the same kind.  `out`: a device tensor to write into (it may be z itself)."""
        torch = self._torch
        as_np = isinstance(z, np.ndarray)
        zin = torch.as_tensor(np.ascontiguousarray(z, dtype=np.float64)).cuda() if as_np else z
        assert zin.dtype == torch.float64 and zin.is_cuda and zin.numel() == self.info["state_len"]
        assert zin.is_contiguous() or out is None
        zin = zin.contiguous()
        if out is None:
            out = torch.empty_like(zin)
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        assert out.numel() == zin.numel()
        self._order()
        # CMCG_ENOTCONV: a Riesz solve stopped at its iteration cap (kept in last_status)
        self.last_status = _check(
            _lib.cmcg_apply(self._h, int(op), int(steps), ctypes.c_void_p(zin.data_ptr()),
                            ctypes.c_void_p(out.data_ptr())), "cmcg_apply", allow_notconv=True)
        return out.cpu().numpy() if as_np else out

    def filter(self, z) -> np.ndarray:
        torch = self._torch
        zin = torch.as_tensor(np.ascontiguousarray(z, dtype=np.float64)).cuda() \
            if isinstance(z, np.ndarray) else z.contiguous()
        ure, uim, keep = self._out_buffers(False)
        self._order()
        _check(_lib.cmcg_filter(self._h, ctypes.c_void_p(zin.data_ptr()), ure, uim), "cmcg_filter")
        return self._out_value(keep, False)

    def step6(self, z) -> np.ndarray:
        """u read off a packed state without time stepping (cmcg_step6)."""
        torch = self._torch
        zin = torch.as_tensor(np.ascontiguousarray(z, dtype=np.float64)).cuda() \
            if isinstance(z, np.ndarray) else z.contiguous()
        ure, uim, keep = self._out_buffers(False)
        self._order()
        _check(_lib.cmcg_step6(self._h, ctypes.c_void_p(zin.data_ptr()), ure, uim), "cmcg_step6")
        return self._out_value(keep, False)

    def runup(self, periods: int, ramp: bool = True):
        """State (packed FP64 torch device vector) after `periods` periods of the forced scheme
        from rest, the source switched on by Mur's transient if `ramp` (cmcg_runup)."""
        torch = self._torch
        out = torch.empty(self.info["state_len"], dtype=torch.float64, device="cuda")
        self._order()
        _check(_lib.cmcg_runup(self._h, int(periods), 1 if ramp else 0,
                               ctypes.c_void_p(out.data_ptr())), "cmcg_runup")
        return out

    def misfit(self, z) -> float:
        """J(z) = 1/2 ||Phi(z) - z||_E^2 (cmcg_misfit); z a packed state (NumPy or device)."""
        torch = self._torch
        zin = torch.as_tensor(np.ascontiguousarray(z, dtype=np.float64)).cuda() \
            if isinstance(z, np.ndarray) else z.contiguous()
        J = ctypes.c_double(0.0)
        self._order()
        _check(_lib.cmcg_misfit(self._h, ctypes.c_void_p(zin.data_ptr()), ctypes.byref(J)),
               "cmcg_misfit")
        return J.value

    def state(self, which: int = 0) -> np.ndarray:
        torch = self._torch
        out = torch.empty(self.info["state_len"], dtype=torch.float64, device="cuda")
        self._order()
        _check(_lib.cmcg_get_state(self._h, int(which), ctypes.c_void_p(out.data_ptr())),
               "cmcg_get_state")
        return out.cpu().numpy()

    # ------------------------------------------------------------------ helpers
    def _out_buffers(self, device_output: bool):
        if device_output:
            torch = self._torch
            re = torch.empty(self.field_shape, dtype=torch.float64, device="cuda")
            im = torch.empty_like(re)
            return ctypes.c_void_p(re.data_ptr()), ctypes.c_void_p(im.data_ptr()), (re, im)
        re = np.empty(self.field_shape, dtype=np.float64)
        im = np.empty_like(re)
        return re.ctypes.data_as(ctypes.c_void_p), im.ctypes.data_as(ctypes.c_void_p), (re, im)

    @staticmethod
    def _out_value(keep, device_output: bool):
        if device_output:
            return keep
        return keep[0] + 1j * keep[1]


def status_string(st: int) -> str:
    return _lib.cmcg_status_string(st).decode()


def marshal_problem(problem):
    """cmcg_inputs.Problem -> (_Problem struct, list of arrays the struct points into)."""
    p = _Problem()
    p.dim = problem.dim
    p.formulation = problem.formulation
    for k in range(3):
        p.n[k] = int(problem.n[k]) if k < len(problem.n) else 1
    p.omega = float(problem.omega)
    keep = []

    def arr(x, dtype=np.float64):
        a = np.ascontiguousarray(np.asarray(x, dtype=dtype).ravel())
        keep.append(a)
        return a

    if problem.c is not None:
        p.c = _ptr(arr(problem.c))
    p.c_const = float(problem.c_const)

    def data(dst, f, gS, gD):
        # source, boundary and Dirichlet data into a _Problem or _Shot (imaginary parts only
        # when non-zero)
        if f is not None:
            f = np.asarray(f)
            dst.f_re = _ptr(arr(f.real))
            if np.iscomplexobj(f) and np.any(f.imag != 0):
                dst.f_im = _ptr(arr(f.imag))
        if gS is not None:
            g = _concat_faces(gS, np.complex128)
            dst.gS_re = _ptr(arr(g.real))
            if np.any(g.imag != 0):
                dst.gS_im = _ptr(arr(g.imag))
        if gD is not None:
            d = np.asarray(gD, dtype=np.complex128)
            dst.gD_re = _ptr(arr(d.real))
            if np.any(d.imag != 0):
                dst.gD_im = _ptr(arr(d.imag))

    data(p, problem.f, problem.gS, getattr(problem, "gD", None))
    shots = getattr(problem, "shots", None)
    if shots:
        table = (_Shot * len(shots))()
        for k, sh in enumerate(shots):
            table[k].harmonic = int(sh.harmonic)
            data(table[k], sh.f, sh.gS, sh.gD)
        keep.append(table)
        p.n_shots = len(shots)
        p.shots = ctypes.cast(table, ctypes.POINTER(_Shot))
    if problem.sound_soft is not None:
        m = arr(problem.sound_soft, np.uint8)
        p.sound_soft = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    bc = list(problem.face_bc) + [1] * 6
    for k in range(6):
        p.face_bc[k] = int(bc[k])
    p.courant = float(problem.courant)
    return p, keep


RIESZ_DEFAULT, RIESZ_SOLVE, RIESZ_VCYCLE = 0, 1, 2
_RIESZ = {"default": RIESZ_DEFAULT, "solve": RIESZ_SOLVE, "vcycle": RIESZ_VCYCLE}
OUTPUT_FILTER, OUTPUT_STEP6 = 0, 1
_OUTPUT = {"filter": OUTPUT_FILTER, "step6": OUTPUT_STEP6}


def make_options(precision="fp64", tol=1e-6, max_iter=1000, device=0, steps_per_launch=0,
                 riesz_tol=0.0, riesz_max_iter=0, fp64_refresh=0.0,
                 riesz_mode="default", runup_periods=0, output="filter") -> _Options:
    o = _Options()
    o.precision = FP64 if precision == "fp64" else FP32_MIXED
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.device = int(device)
    o.steps_per_launch = int(steps_per_launch)
    o.riesz_tol = float(riesz_tol)
    o.riesz_max_iter = int(riesz_max_iter)
    o.fp64_refresh = float(fp64_refresh)
    o.riesz_mode = _RIESZ[riesz_mode] if isinstance(riesz_mode, str) else int(riesz_mode)
    o.runup_periods = int(runup_periods)
    o.output = _OUTPUT[output] if isinstance(output, str) else int(output)
    return o


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, -1


def apply_static(problem, op: int, z, precision: str = "fp64", steps: int = 0,
                 steps_per_launch: int = 0, device: int = 0, out=None):
    """cmcg_apply_static: op(z) for a first-order problem without a handle (the library keeps
    the problem's fields in its fixed per-GPU buffer and allocates nothing).  z: a torch FP64
    device tensor of the problem's state length.  Runs on the caller's current stream and
    returns after it; returns `out` (a new tensor when None; it may be z itself)."""
    import torch
    assert z.dtype == torch.float64 and z.is_cuda and z.is_contiguous()
    if out is None:
        out = torch.empty_like(z)
    assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
    assert out.numel() == z.numel()
    p, keep = marshal_problem(problem)
    o = make_options(precision, 1e-6, 1, device, steps_per_launch)
    o.hip_stream = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    _check(_lib.cmcg_apply_static(ctypes.byref(p), ctypes.byref(o), int(op), int(steps),
                                  ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(out.data_ptr())),
           "cmcg_apply_static")
    return out


class Server:
    """Continuous-batching server for first-order 2D solves (cmcg_server_* in include/cmcg.h)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 16, steps_per_launch: int = 0,
                 device: int = 0, stream=None, barrier_spin_limit: int = 0):
        import torch
        o = _ServerOptions()
        o.hbm_budget_bytes = int(hbm_budget_bytes)
        o.max_slots = int(max_slots)
        o.steps_per_launch = int(steps_per_launch)
        o.device = int(device)
        o.barrier_spin_limit = int(barrier_spin_limit)
        self.stream = _handle_stream(torch, stream, device)
        o.hip_stream = ctypes.c_void_p(self.stream.cuda_stream)
        h = _H()
        _check(_lib.cmcg_server_create(ctypes.byref(o), ctypes.byref(h)), "cmcg_server_create")
        self._h = h
        self._shapes = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.cmcg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def submit(self, problem, precision: str = "fp32", tol: float = 1e-6,
               max_iter: int = 1000, runup_periods: int = 0, fp64_refresh: float = 0.0) -> int:
        p, keep = marshal_problem(problem)
        o = make_options(precision, tol, max_iter, runup_periods=runup_periods,
                         fp64_refresh=fp64_refresh)
        rid = ctypes.c_int64(0)
        _check(_lib.cmcg_server_submit(self._h, ctypes.byref(p), ctypes.byref(o),
                                       ctypes.byref(rid)), "cmcg_server_submit")
        self._shapes[rid.value] = problem.field_shape()
        return rid.value

    def step(self):
        a, q = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(_lib.cmcg_server_step(self._h, ctypes.byref(a), ctypes.byref(q)), "cmcg_server_step")
        return a.value, q.value

    def poll(self, rid: int):
        """Returns (state, u or None, report or None, status)."""
        state = ctypes.c_int32(0)
        shape = self._shapes[rid]
        re = np.empty(shape)
        im = np.empty(shape)
        rep = _Report()
        st = _lib.cmcg_server_poll(self._h, int(rid), ctypes.byref(state),
                                   re.ctypes.data_as(ctypes.c_void_p),
                                   im.ctypes.data_as(ctypes.c_void_p), ctypes.byref(rep))
        if state.value in (REQ_DONE, REQ_FAILED):
            # the library released the request with this poll
            self._shapes.pop(rid, None)
        if state.value == REQ_DONE:
            return state.value, re + 1j * im, _report_dict(rep), st
        return state.value, None, None, st

    def launches(self):
        """(ticks that advanced solves, kernel launches those ticks made, rounds they ran)."""
        t, n, r = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
        _check(_lib.cmcg_server_launches(self._h, ctypes.byref(t), ctypes.byref(n),
                                         ctypes.byref(r)), "cmcg_server_launches")
        return t.value, n.value, r.value

    def stats(self):
        used = ctypes.c_int64(0)
        a, q = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(_lib.cmcg_server_stats(self._h, ctypes.byref(used), ctypes.byref(a),
                                      ctypes.byref(q)), "cmcg_server_stats")
        return used.value, a.value, q.value
