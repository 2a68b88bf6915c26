"""Python binding of the serving runtime (include/lbessel_serve.h).

Argument marshalling only: the queue, admission, batching and every kernel
live in liblbessel.so.  Evaluation requests take pinned host tensors
(``torch.empty(..., pin_memory=True)``) for inputs and outputs, or GPU
tensors (submit_eval_device: no copies); vMF fit requests take a float32
feature matrix on the GPU.

    srv = Server(mode="batched")
    t = srv.submit_eval("K", v_host, x_host, out_host)
    info = srv.wait(t)                      # dict with status and timestamps
    infos = srv.replay(items)               # open-loop load replay
    srv.close()
"""
from __future__ import annotations

import ctypes

import torch

from . import KIND, LbesselError, _load

BATCHED, PLAIN = 0, 1
MODES = {"batched": BATCHED, "plain": PLAIN}
ETIMEOUT = -5


class Config(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_int64), ("streams", ctypes.c_int),
                ("mode", ctypes.c_int), ("max_batch_requests", ctypes.c_int),
                ("max_batch_elems", ctypes.c_int64), ("poll_us", ctypes.c_int),
                ("solo_elems", ctypes.c_int64)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("state", ctypes.c_int), ("batch", ctypes.c_int64),
                ("bytes", ctypes.c_int64), ("t_arrival", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "submitted", "completed", "batches", "kernel_launches", "eval_pairs", "vmf_fits",
        "arena_bytes", "arena_peak_bytes", "queue_peak", "max_batch_requests_seen")]


class ReplayItem(ctypes.Structure):
    _fields_ = [("t_arrival", ctypes.c_double), ("type", ctypes.c_int), ("kind", ctypes.c_int),
                ("precision", ctypes.c_int), ("reserved", ctypes.c_int),
                ("v", ctypes.c_void_p), ("x", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("X", ctypes.c_void_p), ("p", ctypes.c_int64),
                ("result", ctypes.c_void_p)]


_bound = False


def _lib():
    global _bound
    lib = _load()
    if _bound:
        return lib
    vp, i64, ci, cd = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    sig = {
        "lbessel_server_default_config": ([ctypes.POINTER(Config)], None),
        "lbessel_server_create": ([ctypes.POINTER(Config), ctypes.POINTER(vp)], ci),
        "lbessel_server_submit_eval": ([vp, ci, ci, vp, vp, vp, i64, ctypes.POINTER(i64)], ci),
        "lbessel_server_submit_eval_device": ([vp, ci, ci, vp, vp, vp, i64,
                                               ctypes.POINTER(i64)], ci),
        "lbessel_server_submit_vmf": ([vp, vp, i64, i64, vp, ctypes.POINTER(i64)], ci),
        "lbessel_server_wait": ([vp, i64, cd, ctypes.POINTER(RequestInfo)], ci),
        "lbessel_server_clock": ([vp], cd),
        "lbessel_server_stats": ([vp, ctypes.POINTER(Stats)], ci),
        "lbessel_server_destroy": ([vp], ci),
        "lbessel_server_replay": ([vp, ctypes.POINTER(ReplayItem), i64, cd,
                                   ctypes.POINTER(RequestInfo)], ci),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _bound = True
    return lib


def _err(status: int, what: str) -> LbesselError:
    msg = _load().lbessel_status_string(status).decode()
    return LbesselError(f"{what} failed: {msg} ({status})")


def _device(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise LbesselError(f"{name} must be a contiguous GPU tensor")
    if t.dtype not in (torch.float64, torch.float32):
        raise LbesselError(f"{name}: float64 or float32 only")
    return t


def _host(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.is_cuda or not t.is_contiguous():
        raise LbesselError(f"{name} must be a contiguous host tensor (pinned for overlap)")
    if t.dtype not in (torch.float64, torch.float32):
        raise LbesselError(f"{name}: float64 or float32 only")
    return t


class Server:
    """A lbessel request server on the current GPU."""

    def __init__(self, mode: str = "batched", arena_bytes: int | None = None,
                 streams: int | None = None, max_batch_requests: int | None = None,
                 max_batch_elems: int | None = None, poll_us: int | None = None,
                 solo_elems: int | None = None):
        lib = _lib()
        cfg = Config()
        lib.lbessel_server_default_config(ctypes.byref(cfg))
        cfg.mode = MODES[mode]
        for name, val in (("arena_bytes", arena_bytes), ("streams", streams),
                          ("max_batch_requests", max_batch_requests),
                          ("max_batch_elems", max_batch_elems), ("poll_us", poll_us),
                          ("solo_elems", solo_elems)):
            if val is not None:
                setattr(cfg, name, int(val))
        self.config = {name: getattr(cfg, name) for name, _ in Config._fields_}
        h = ctypes.c_void_p()
        rc = lib.lbessel_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != 0:
            raise _err(rc, "lbessel_server_create")
        self._h = h
        self._keep = {}   # ticket -> tensors that must outlive the request

    def submit_eval(self, kind: str, v: torch.Tensor, x: torch.Tensor, out: torch.Tensor) -> int:
        v, x, out = _host(v, "v"), _host(x, "x"), _host(out, "out")
        if not (v.dtype == x.dtype == out.dtype) or not (v.numel() == x.numel() == out.numel()):
            raise LbesselError("v, x, out must share dtype and size")
        prec = 64 if v.dtype == torch.float64 else 32
        t = ctypes.c_int64()
        rc = _lib().lbessel_server_submit_eval(self._h, KIND[kind], prec, v.data_ptr(),
                                               x.data_ptr(), out.data_ptr(), v.numel(),
                                               ctypes.byref(t))
        if rc != 0:
            raise _err(rc, "lbessel_server_submit_eval")
        self._keep[t.value] = (v, x, out)
        return t.value

    def submit_eval_device(self, kind: str, v: torch.Tensor, x: torch.Tensor,
                           out: torch.Tensor) -> int:
        """Device-resident evaluation request: v, x, out GPU tensors (the
        inputs complete on the current stream before this returns)."""
        v, x, out = _device(v, "v"), _device(x, "x"), _device(out, "out")
        if not (v.dtype == x.dtype == out.dtype) or not (v.numel() == x.numel() == out.numel()):
            raise LbesselError("v, x, out must share dtype and size")
        prec = 64 if v.dtype == torch.float64 else 32
        torch.cuda.current_stream(v.device).synchronize()   # inputs complete before submit
        t = ctypes.c_int64()
        rc = _lib().lbessel_server_submit_eval_device(self._h, KIND[kind], prec, v.data_ptr(),
                                                      x.data_ptr(), out.data_ptr(), v.numel(),
                                                      ctypes.byref(t))
        if rc != 0:
            raise _err(rc, "lbessel_server_submit_eval_device")
        self._keep[t.value] = (v, x, out)
        return t.value

    def submit_vmf(self, X: torch.Tensor, result: torch.Tensor) -> int:
        if not X.is_cuda or X.dtype != torch.float32 or X.dim() != 2 or not X.is_contiguous():
            raise LbesselError("X must be a contiguous 2-D float32 tensor on the GPU")
        if result.is_cuda or result.dtype != torch.float64 or result.numel() < 4:
            raise LbesselError("result must be a host float64 tensor of 4 elements")
        torch.cuda.current_stream(X.device).synchronize()   # X complete before submit
        t = ctypes.c_int64()
        rc = _lib().lbessel_server_submit_vmf(self._h, X.data_ptr(), X.shape[0], X.shape[1],
                                              result.data_ptr(), ctypes.byref(t))
        if rc != 0:
            raise _err(rc, "lbessel_server_submit_vmf")
        self._keep[t.value] = (X, result)
        return t.value

    def wait(self, ticket: int, timeout: float = -1.0) -> dict:
        info = RequestInfo()
        rc = _lib().lbessel_server_wait(self._h, ticket, float(timeout), ctypes.byref(info))
        if rc == ETIMEOUT:
            raise TimeoutError(f"request {ticket} not done after {timeout} s")
        self._keep.pop(ticket, None)
        if rc != 0:
            raise _err(rc, "request")
        return info.as_dict()

    def replay(self, items, timeout: float = 600.0):
        """items: list of dicts, sorted by 't' (arrival, seconds from the start):
        {'t', 'type': 'eval', 'kind', 'v', 'x', 'out'} (host tensors),
        {'t', 'type': 'eval_device', 'kind', 'v', 'x', 'out'} (GPU tensors) or
        {'t', 'type': 'vmf', 'X', 'result'}.  Returns one info dict per item."""
        arr = (ReplayItem * len(items))()
        for i, it in enumerate(items):
            r = arr[i]
            r.t_arrival = float(it["t"])
            if it["type"] in ("eval", "eval_device"):
                conv = _host if it["type"] == "eval" else _device
                v, x, out = conv(it["v"], "v"), conv(it["x"], "x"), conv(it["out"], "out")
                r.type = 0 if it["type"] == "eval" else 2
                r.kind = KIND[it["kind"]]
                r.precision = 64 if v.dtype == torch.float64 else 32
                r.v, r.x, r.out, r.n = v.data_ptr(), x.data_ptr(), out.data_ptr(), v.numel()
            else:
                X, res = it["X"], it["result"]
                r.type, r.X, r.n, r.p, r.result = 1, X.data_ptr(), X.shape[0], X.shape[1], \
                    res.data_ptr()
        infos = (RequestInfo * len(items))()
        torch.cuda.synchronize()
        rc = _lib().lbessel_server_replay(self._h, arr, len(items), float(timeout), infos)
        if rc != 0:
            raise _err(rc, "lbessel_server_replay")
        return [infos[i].as_dict() for i in range(len(items))]

    def clock(self) -> float:
        return _lib().lbessel_server_clock(self._h)

    def stats(self) -> dict:
        st = Stats()
        rc = _lib().lbessel_server_stats(self._h, ctypes.byref(st))
        if rc != 0:
            raise _err(rc, "lbessel_server_stats")
        return {name: getattr(st, name) for name, _ in Stats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib().lbessel_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
