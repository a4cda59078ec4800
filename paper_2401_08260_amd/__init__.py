"""ksum: sliced fast kernel summation on AMD MI355X -- Python binding.

A thin ctypes layer over the C ABI in include/ksum.h (libksum.so, built by
``paper_2401_08260_amd.build``).  Functions keep the C names and only marshal
arguments; every step of the computation runs in the HIP library.  ``Plan`` is a
convenience wrapper that takes torch tensors on the GPU and uses torch's
current stream.  Importing this module fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libksum.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                      "or `python paper_2401_08260_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)

# enums (include/ksum.h)
KSUM_GAUSSIAN, KSUM_LAPLACIAN, KSUM_NEGDIST, KSUM_MATERN = 1, 2, 3, 4
KSUM_1D_AUTO, KSUM_1D_NDFT, KSUM_1D_NFFT, KSUM_1D_SORT = 0, 1, 2, 3
KSUM_FP32, KSUM_SPLIT_BF16 = 0, 1
PRECISIONS = {"fp32": KSUM_FP32, "split_bf16": KSUM_SPLIT_BF16}
KSUM_OK, KSUM_EINVAL, KSUM_EUNSUPPORTED, KSUM_ENOMEM, KSUM_EWORKSPACE, KSUM_ENONFINITE, KSUM_EDEVICE = range(7)
KSUM_NOALLOC_SCRATCH_BYTES = 256 << 20      # static scratch of ksum_execute_noalloc, per GPU

KERNELS = {"gaussian": KSUM_GAUSSIAN, "laplacian": KSUM_LAPLACIAN, "negdist": KSUM_NEGDIST, "matern": KSUM_MATERN}
METHODS = {"auto": KSUM_1D_AUTO, "ndft": KSUM_1D_NDFT, "nfft": KSUM_1D_NFFT, "sort": KSUM_1D_SORT}


class ksum_params(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("directions", ctypes.POINTER(ctypes.c_double)), ("n_coeff", ctypes.c_int32),
                ("coeff_eps", ctypes.c_double), ("T", ctypes.c_double), ("oversample", ctypes.c_int32),
                ("window_m", ctypes.c_int32), ("method", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("slice_batch", ctypes.c_int32), ("device", ctypes.c_int32), ("check_finite", ctypes.c_int32)]


class ksum_probe(ctypes.Structure):
    _fields_ = [("z", ctypes.c_void_p), ("bounds", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("perm", ctypes.c_void_p)]


_P = ctypes.c_void_p
class ksum_request(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("d", ctypes.c_int32), ("P", ctypes.c_int32), ("kernel", ctypes.c_int),
                ("params", ksum_params), ("x", ctypes.c_void_p), ("N", ctypes.c_int64), ("y", ctypes.c_void_p),
                ("M", ctypes.c_int64), ("w", ctypes.c_void_p), ("s", ctypes.c_void_p), ("grad_s", ctypes.c_void_p),
                ("grad_x", ctypes.c_void_p), ("grad_y", ctypes.c_void_p), ("grad_w", ctypes.c_void_p),
                ("ready_event", ctypes.c_void_p)]


class ksum_completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_end", ctypes.c_double), ("ws_bytes", ctypes.c_size_t)]


class ksum_server_info(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("finished", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("running", ctypes.c_int64), ("plans", ctypes.c_int64), ("arena_bytes", ctypes.c_size_t),
                ("arena_used", ctypes.c_size_t), ("arena_peak", ctypes.c_size_t)]


_sigs = {
    "ksum_version": (ctypes.c_char_p, []),
    "ksum_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ksum_last_error": (ctypes.c_char_p, []),
    "ksum_params_default": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ksum_params)]),
    "ksum_check_params": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(ksum_params)]),
    "ksum_generate_directions": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, _P]),
    "ksum_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(ksum_params),
                                            ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "ksum_plan_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(ksum_params),
                                        ctypes.POINTER(_P)]),
    "ksum_plan_destroy": (ctypes.c_int, [_P]),
    "ksum_get_directions": (ctypes.c_int, [_P, _P]),
    "ksum_workspace_size": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "ksum_execute": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int64, _P, _P, _P, ctypes.c_size_t, _P]),
    "ksum_execute_f64in": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int64, _P, _P, _P, ctypes.c_size_t,
                                          _P]),
    "ksum_execute_probe": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int64, _P, _P, _P, ctypes.c_size_t,
                                          _P, ctypes.POINTER(ksum_probe)]),
    "ksum_execute_probe_f64in": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int64, _P, _P, _P,
                                                ctypes.c_size_t, _P, ctypes.POINTER(ksum_probe)]),
    "ksum_execute_noalloc": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int64, _P, _P, _P]),
    "ksum_backward_workspace_size": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64,
                                                    ctypes.POINTER(ctypes.c_size_t)]),
    "ksum_backward": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int64, _P, _P, _P, _P, _P, _P,
                                     ctypes.c_size_t, _P]),
    "ksum_server_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER(_P)]),
    "ksum_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(ksum_request)]),
    "ksum_server_poll": (ctypes.c_int, [_P, ctypes.POINTER(ksum_completion), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]),
    "ksum_server_drain": (ctypes.c_int, [_P]),
    "ksum_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(ksum_server_info)]),
    "ksum_server_destroy": (ctypes.c_int, [_P]),
    "ksum_set_timing": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ksum_stage_times": (ctypes.c_int, [_P, _P, _P]),
    "ksum_stage_count": (ctypes.c_int32, []),
    "ksum_stage_name": (ctypes.c_char_p, [ctypes.c_int32]),
}
for _name, (_res, _args) in _sigs.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_sigs)


class KsumError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.ksum_last_error().decode()
        super().__init__(f"{where}: {_lib.ksum_status_string(status).decode()} ({msg})")


def _check(status: int, where: str) -> None:
    if status != KSUM_OK:
        raise KsumError(status, where)


# ---------------------------------------------------------------------------
# C-named wrappers (argument marshalling only)
# ---------------------------------------------------------------------------
def ksum_version() -> str:
    return _lib.ksum_version().decode()


def ksum_status_string(status: int) -> str:
    return _lib.ksum_status_string(status).decode()


def ksum_last_error() -> str:
    return _lib.ksum_last_error().decode()


def ksum_params_default(kernel: int) -> ksum_params:
    p = ksum_params()
    _check(_lib.ksum_params_default(kernel, ctypes.byref(p)), "ksum_params_default")
    return p


def make_params(kernel: int, directions: Optional[np.ndarray] = None, **overrides) -> ksum_params:
    """Defaults for `kernel` with fields overridden by keyword (method may be a name)."""
    p = ksum_params_default(kernel)
    for k, v in overrides.items():
        if k == "method" and isinstance(v, str):
            v = METHODS[v]
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    if directions is not None:
        arr = np.ascontiguousarray(directions, dtype=np.float64)
        p._dir_keepalive = arr
        p.directions = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return p


def ksum_check_params(d: int, P: int, kernel: int, params: Optional[ksum_params] = None) -> int:
    return _lib.ksum_check_params(d, P, kernel, ctypes.byref(params) if params is not None else None)


def ksum_generate_directions(d: int, P: int, seed: int) -> np.ndarray:
    out = np.empty((P, d), dtype=np.float64)
    _check(_lib.ksum_generate_directions(d, P, seed, out.ctypes.data), "ksum_generate_directions")
    return out


def ksum_workspace_bytes(d: int, P: int, kernel: int, params: Optional[ksum_params], N: int, M: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.ksum_workspace_bytes(d, P, kernel, ctypes.byref(params) if params is not None else None, N, M,
                                     ctypes.byref(out)), "ksum_workspace_bytes")
    return out.value


def ksum_plan_create(d: int, P: int, kernel: int, params: Optional[ksum_params] = None) -> int:
    h = _P()
    _check(_lib.ksum_plan_create(d, P, kernel, ctypes.byref(params) if params is not None else None,
                                 ctypes.byref(h)), "ksum_plan_create")
    return h.value


def ksum_plan_destroy(plan: int) -> None:
    _check(_lib.ksum_plan_destroy(plan), "ksum_plan_destroy")


def ksum_get_directions(plan: int, d: int, P: int) -> np.ndarray:
    out = np.empty((P, d), dtype=np.float64)
    _check(_lib.ksum_get_directions(plan, out.ctypes.data), "ksum_get_directions")
    return out


def ksum_workspace_size(plan: int, N: int, M: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.ksum_workspace_size(plan, N, M, ctypes.byref(out)), "ksum_workspace_size")
    return out.value


def ksum_execute(plan: int, x: int, N: int, y: int, M: int, w: int, s: int, ws: int, ws_bytes: int,
                 stream: int) -> None:
    _check(_lib.ksum_execute(plan, x, N, y, M, w, s, ws, ws_bytes, stream), "ksum_execute")


def ksum_execute_f64in(plan: int, x: int, N: int, y: int, M: int, w: int, s: int, ws: int, ws_bytes: int,
                       stream: int) -> None:
    _check(_lib.ksum_execute_f64in(plan, x, N, y, M, w, s, ws, ws_bytes, stream), "ksum_execute_f64in")


def ksum_execute_probe(plan: int, x: int, N: int, y: int, M: int, w: int, s: int, ws: int, ws_bytes: int,
                       stream: int, probe: Optional[ksum_probe]) -> None:
    _check(_lib.ksum_execute_probe(plan, x, N, y, M, w, s, ws, ws_bytes, stream,
                                   ctypes.byref(probe) if probe is not None else None), "ksum_execute_probe")


def ksum_execute_probe_f64in(plan: int, x: int, N: int, y: int, M: int, w: int, s: int, ws: int,
                             ws_bytes: int, stream: int, probe: Optional[ksum_probe]) -> None:
    _check(_lib.ksum_execute_probe_f64in(plan, x, N, y, M, w, s, ws, ws_bytes, stream,
                                         ctypes.byref(probe) if probe is not None else None),
           "ksum_execute_probe_f64in")


def ksum_execute_noalloc(plan: int, x: int, N: int, y: int, M: int, w: int, s: int, stream: int) -> None:
    _check(_lib.ksum_execute_noalloc(plan, x, N, y, M, w, s, stream), "ksum_execute_noalloc")


def ksum_backward_workspace_size(plan: int, N: int, M: int) -> int:
    out = ctypes.c_size_t()
    _check(_lib.ksum_backward_workspace_size(plan, N, M, ctypes.byref(out)), "ksum_backward_workspace_size")
    return out.value


def ksum_backward(plan: int, x: int, N: int, y: int, M: int, w: int, grad_s: int, grad_x: Optional[int],
                  grad_y: Optional[int], grad_w: Optional[int], ws: int, ws_bytes: int, stream: int) -> None:
    _check(_lib.ksum_backward(plan, x, N, y, M, w, grad_s, grad_x, grad_y, grad_w, ws, ws_bytes, stream),
           "ksum_backward")


def ksum_set_timing(plan: int, enable: bool) -> None:
    _check(_lib.ksum_set_timing(plan, 1 if enable else 0), "ksum_set_timing")


def ksum_stage_count() -> int:
    return _lib.ksum_stage_count()


def ksum_stage_name(stage: int) -> str:
    return _lib.ksum_stage_name(stage).decode()


def ksum_stage_times(plan: int) -> dict:
    """{stage name: (total ms, launches)} accumulated since timing was enabled."""
    n = ksum_stage_count()
    ms = np.zeros(n, dtype=np.float64)
    calls = np.zeros(n, dtype=np.int64)
    _check(_lib.ksum_stage_times(plan, ms.ctypes.data, calls.ctypes.data), "ksum_stage_times")
    return {ksum_stage_name(i): (float(ms[i]), int(calls[i])) for i in range(n)}


# ---------------------------------------------------------------------------
# torch convenience wrapper
# ---------------------------------------------------------------------------
class Plan:
    """A ksum plan bound to torch device tensors.

    Plan(d, P, "gaussian", sigma=..., seed=..., n_coeff=..., T=..., method="nfft", ...)
    s = plan(x, y, w)        # x: (N,d), y: (M,d), w: (N,) on the plan's GPU; FP32 or FP64
    """

    def __init__(self, d: int, P: int, kernel: str, directions: Optional[np.ndarray] = None, **params):
        import torch  # noqa: F401  (device memory and streams)
        self.d, self.P = int(d), int(P)
        self.kernel = kernel
        self.kid = KERNELS[kernel]
        self.params = make_params(self.kid, directions=directions, **params)
        self.handle = ksum_plan_create(self.d, self.P, self.kid, self.params)
        self._ws = None
        self._bws = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                _lib.ksum_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    def directions(self) -> np.ndarray:
        return ksum_get_directions(self.handle, self.d, self.P)

    def workspace(self, N: int, M: int, device):
        import torch
        need = ksum_workspace_size(self.handle, N, M)
        if self._ws is None or self._ws.numel() < need or self._ws.device != device:
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=device)
        return self._ws, need

    def __call__(self, x, y, w, out=None, probe: Optional[dict] = None, stream=None):
        import torch
        N, M = x.shape[0], y.shape[0]
        if x.shape[1] != self.d or y.shape[1] != self.d or w.shape[0] != N:
            raise ValueError("shape mismatch")
        f64 = x.dtype == torch.float64
        want = torch.float64 if f64 else torch.float32
        if y.dtype != want or w.dtype != want:
            raise TypeError("x, y, w must share one dtype (float32 or float64)")
        if not (x.is_cuda and y.is_cuda and w.is_cuda):
            raise ValueError("x, y, w must be GPU tensors")
        x, y, w = x.contiguous(), y.contiguous(), w.contiguous()
        s = out if out is not None else torch.empty(M, dtype=torch.float32, device=x.device)
        ws, need = self.workspace(N, M, x.device)
        st = (stream if stream is not None else torch.cuda.current_stream(x.device)).cuda_stream
        if probe is not None:
            pr = ksum_probe(*(probe[k].data_ptr() if probe.get(k) is not None else None
                              for k in ("z", "bounds", "t", "perm")))
            fn = ksum_execute_probe_f64in if f64 else ksum_execute_probe
            fn(self.handle, x.data_ptr(), N, y.data_ptr(), M, w.data_ptr(), s.data_ptr(),
               ws.data_ptr(), ws.numel(), st, pr)
        elif f64:
            ksum_execute_f64in(self.handle, x.data_ptr(), N, y.data_ptr(), M, w.data_ptr(), s.data_ptr(),
                               ws.data_ptr(), ws.numel(), st)
        else:
            ksum_execute(self.handle, x.data_ptr(), N, y.data_ptr(), M, w.data_ptr(), s.data_ptr(),
                         ws.data_ptr(), ws.numel(), st)
        return s

    def backward(self, x, y, w, grad_s, need_x: bool = True, need_y: bool = True, need_w: bool = True,
                 stream=None):
        """(grad_x, grad_y, grad_w) of a loss with dL/ds = grad_s (FP32 tensors; None where not needed)."""
        import torch
        N, M = x.shape[0], y.shape[0]
        for t in (x, y, w, grad_s):
            if t.dtype != torch.float32 or not t.is_cuda:
                raise TypeError("backward takes FP32 GPU tensors")
        if x.shape[1] != self.d or y.shape[1] != self.d or w.shape[0] != N or grad_s.shape[0] != M:
            raise ValueError("shape mismatch")
        x, y, w, grad_s = x.contiguous(), y.contiguous(), w.contiguous(), grad_s.contiguous()
        need = ksum_backward_workspace_size(self.handle, N, M)
        if self._bws is None or self._bws.numel() < need or self._bws.device != x.device:
            self._bws = torch.empty(max(need, 256), dtype=torch.uint8, device=x.device)
        gx = torch.empty((N, self.d), dtype=torch.float32, device=x.device) if need_x else None
        gy = torch.empty((M, self.d), dtype=torch.float32, device=x.device) if need_y else None
        gw = torch.empty(N, dtype=torch.float32, device=x.device) if need_w else None
        st = (stream if stream is not None else torch.cuda.current_stream(x.device)).cuda_stream
        ksum_backward(self.handle, x.data_ptr(), N, y.data_ptr(), M, w.data_ptr(), grad_s.data_ptr(),
                      gx.data_ptr() if gx is not None else None, gy.data_ptr() if gy is not None else None,
                      gw.data_ptr() if gw is not None else None, self._bws.data_ptr(), self._bws.numel(), st)
        return gx, gy, gw


def _make_autograd():
    import torch

    class KernelSum(torch.autograd.Function):
        """s = KernelSum.apply(plan, x, y, w): the sliced kernel sum with a hand-written backward
        (ksum_backward) for gradients with respect to x, y and w."""

        @staticmethod
        def forward(ctx, plan, x, y, w):
            ctx.plan = plan
            ctx.save_for_backward(x, y, w)
            return plan(x.detach(), y.detach(), w.detach())

        @staticmethod
        def backward(ctx, grad_s):
            x, y, w = ctx.saved_tensors
            gx, gy, gw = ctx.plan.backward(x.detach(), y.detach(), w.detach(), grad_s.detach().float(),
                                           need_x=ctx.needs_input_grad[1], need_y=ctx.needs_input_grad[2],
                                           need_w=ctx.needs_input_grad[3])
            return None, gx, gy, gw

    return KernelSum


def __getattr__(name):
    if name == "KernelSum":
        cls = _make_autograd()
        globals()["KernelSum"] = cls
        return cls
    raise AttributeError(name)


class Server:
    """Continuous-batching request server (ksum_server_* of the C ABI) bound to torch tensors.

    srv = Server(slots=8, hbm_bytes=32 << 30)
    srv.submit(tag, "gaussian", d, P, x, y, w, s, params=dict(sigma=..), grad_s=None, grads=(gx, gy, gw))
    done = srv.poll()     # list of dicts {tag, status, t_submit, t_start, t_end, ws_bytes}
    """

    def __init__(self, slots: int = 8, hbm_bytes: int = 32 << 30, device: int = 0):
        h = _P()
        _check(_lib.ksum_server_create(device, slots, hbm_bytes, ctypes.byref(h)), "ksum_server_create")
        self.handle = h.value
        self._keep = {}          # tag -> tensors that must outlive the request

    def submit(self, tag: int, kernel: str, d: int, P: int, x, y, w, s, params: Optional[dict] = None,
               grad_s=None, grads=(None, None, None)) -> None:
        kid = KERNELS[kernel]
        r = ksum_request()
        r.tag = tag
        r.d, r.P, r.kernel = d, P, kid
        r.params = make_params(kid, **(params or {}))
        r.x, r.N, r.y, r.M = x.data_ptr(), x.shape[0], y.data_ptr(), y.shape[0]
        r.w, r.s = w.data_ptr(), s.data_ptr()
        gx, gy, gw = grads
        r.grad_s = grad_s.data_ptr() if grad_s is not None else None
        r.grad_x = gx.data_ptr() if gx is not None else None
        r.grad_y = gy.data_ptr() if gy is not None else None
        r.grad_w = gw.data_ptr() if gw is not None else None
        # the request waits for the work the current stream has queued so far (which may
        # still be writing its inputs)
        import torch
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(x.device))
        r.ready_event = ev.cuda_event
        self._keep[tag] = (x, y, w, s, grad_s, gx, gy, gw, ev)
        _check(_lib.ksum_server_submit(self.handle, ctypes.byref(r)), "ksum_server_submit")

    def poll(self, max_out: int = 256):
        buf = (ksum_completion * max_out)()
        n = ctypes.c_int32()
        _check(_lib.ksum_server_poll(self.handle, buf, max_out, ctypes.byref(n)), "ksum_server_poll")
        out = []
        for i in range(n.value):
            c = buf[i]
            self._keep.pop(c.tag, None)
            out.append(dict(tag=c.tag, status=c.status, t_submit=c.t_submit, t_start=c.t_start, t_end=c.t_end,
                            ws_bytes=c.ws_bytes))
        return out

    def drain(self) -> None:
        _check(_lib.ksum_server_drain(self.handle), "ksum_server_drain")

    def stats(self) -> dict:
        info = ksum_server_info()
        _check(_lib.ksum_server_stats(self.handle, ctypes.byref(info)), "ksum_server_stats")
        return {k: getattr(info, k) for k, _ in ksum_server_info._fields_}

    def close(self) -> None:
        if getattr(self, "handle", None):
            _lib.ksum_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
