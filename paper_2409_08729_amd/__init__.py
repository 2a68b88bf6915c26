"""Python binding of liblbessel (HIP, gfx950).

Argument marshalling only: every function checks its torch tensors, allocates
the output on the same device and calls the C-ABI entry point of the same
name on torch's current HIP stream.  All arithmetic runs in the library's
HIP kernels; there is no CPU path.  If the library is not built, or a tensor
is not on a GPU, the call raises.

log_iv(v, x), log_kv(v, x)                 log I_v(x), log K_v(x)
log_kv_integral(v, x)                      log K_v(x) with the paper's 600-node integral
log_iv_order(v, x), log_kv_order(v, x)     one scalar order (fast path for v = 0, 1)
log_iv_grad_x(v, x, g), log_kv_grad_x(..)  g * d/dx log I_v(x), log K_v(x)
vmf_log_norm(kappa, p), vmf_log_norm_grad  log C_p(kappa) and d/dkappa
LogIv, LogKv, VmfLogNorm                   torch.autograd.Function wrappers
vmf_colsum(X)                              column sums of L2-normalised rows
vmf_fit(X)                                 device kappa solve (kappa, R, kappa_0, steps)
vmf_fit_noalloc(X, result)                 the same into a caller tensor, no workspace
eval_segments(kind, vs, xs)                many arrays in one segmented launch
classify(kind, v, x), eval_branch(...),    diagnostics
eval_ungrouped(kind, v, x)
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbessel.so")

LBESSEL_OK = 0
KIND = {"I": 0, "K": 1}
BRANCHES = ("mu20", "u13", "fallback", "special")

_lib = None


class LbesselError(RuntimeError):
    pass


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LbesselError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2409_08729_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    sig = {
        "lbessel_log_iv_f64": [vp, vp, vp, i64, vp],
        "lbessel_log_iv_f32": [vp, vp, vp, i64, vp],
        "lbessel_log_kv_f64": [vp, vp, vp, i64, vp],
        "lbessel_log_kv_f32": [vp, vp, vp, i64, vp],
        "lbessel_log_kv_integral_f64": [vp, vp, vp, i64, vp],
        "lbessel_log_iv_grad_x_f64": [vp, vp, vp, vp, i64, vp],
        "lbessel_log_iv_grad_x_f32": [vp, vp, vp, vp, i64, vp],
        "lbessel_log_kv_grad_x_f64": [vp, vp, vp, vp, i64, vp],
        "lbessel_log_kv_grad_x_f32": [vp, vp, vp, vp, i64, vp],
        "lbessel_vmf_log_norm_f64": [vp, ctypes.c_double, vp, i64, vp],
        "lbessel_vmf_log_norm_f32": [vp, ctypes.c_float, vp, i64, vp],
        "lbessel_vmf_log_norm_grad_f64": [vp, ctypes.c_double, vp, i64, vp],
        "lbessel_classify": [ctypes.c_int, ctypes.c_int, vp, vp, vp, i64, vp],
        "lbessel_k_nodes": [ctypes.c_int, vp, vp, vp, i64, vp],
        "lbessel_k_terms": [ctypes.c_int, vp, vp, vp, i64, vp],
        "lbessel_elementary_f64": [ctypes.c_int, vp, vp, i64, vp],
        "lbessel_log_iv_order_f64": [ctypes.c_double, vp, vp, i64, vp],
        "lbessel_log_kv_order_f64": [ctypes.c_double, vp, vp, i64, vp],
        "lbessel_log_iv_order_f32": [ctypes.c_float, vp, vp, i64, vp],
        "lbessel_log_kv_order_f32": [ctypes.c_float, vp, vp, i64, vp],
        "lbessel_eval_variant": [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp, i64, vp,
                                 i64, vp],
        "lbessel_eval_branch_f64": [ctypes.c_int, ctypes.c_int, vp, vp, vp, i64, vp],
        "lbessel_eval_branch_f32": [ctypes.c_int, ctypes.c_int, vp, vp, vp, i64, vp],
        "lbessel_eval_ungrouped": [ctypes.c_int, ctypes.c_int, vp, vp, vp, i64, vp],
        "lbessel_vmf_colsum_f32": [vp, i64, i64, vp, vp, vp, i64, vp],
        "lbessel_vmf_fit_f32": [vp, i64, i64, vp, vp, i64, vp],
        "lbessel_vmf_fit_f32_noalloc": [vp, i64, i64, vp, vp],
        "lbessel_eval_segments": [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, i64, vp],
        "lbessel_eval_segments_inline": [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, i64,
                                         vp],
        "lbessel_abi_version": [],
        "lbessel_status_string": [ctypes.c_int],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.lbessel_status_string.restype = ctypes.c_char_p
    for name in ("lbessel_vmf_colsum_workspace", "lbessel_vmf_fit_workspace"):
        getattr(lib, name).argtypes = [i64, i64]
        getattr(lib, name).restype = i64
    lib.lbessel_eval_variant_workspace.argtypes = [i64]
    lib.lbessel_eval_variant_workspace.restype = i64
    lib.lbessel_segment_tiles.argtypes = [i64]
    lib.lbessel_segment_tiles.restype = i64
    _lib = lib
    return lib


def lib():
    """The loaded ctypes handle (raises if the library is not built)."""
    return _load()


def _check(status: int, name: str) -> None:
    if status != LBESSEL_OK:
        msg = _load().lbessel_status_string(status).decode()
        raise LbesselError(f"{name} failed: {msg} ({status})")


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def _prep(*ts: torch.Tensor):
    t0 = ts[0]
    if not isinstance(t0, torch.Tensor) or not t0.is_cuda:
        raise LbesselError("inputs must be torch tensors on a GPU (there is no CPU path)")
    if t0.dtype not in (torch.float64, torch.float32):
        raise LbesselError(f"unsupported dtype {t0.dtype}: float64 or float32 only")
    out = []
    for t in ts:
        if not isinstance(t, torch.Tensor) or t.device != t0.device or t.dtype != t0.dtype:
            raise LbesselError("all tensors must share one GPU device and one dtype")
        if t.shape != t0.shape:
            raise LbesselError(f"shape mismatch: {tuple(t.shape)} vs {tuple(t0.shape)}")
        out.append(t.contiguous())
    return out


def _suffix(t: torch.Tensor) -> str:
    return "f64" if t.dtype == torch.float64 else "f32"


def _unary(name: str, v: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    v, x = _prep(v, x)
    out = torch.empty_like(x)
    fn = f"{name}_{_suffix(x)}"
    with torch.cuda.device(x.device):
        _check(getattr(_load(), fn)(v.data_ptr(), x.data_ptr(), out.data_ptr(), x.numel(),
                                    _stream(x)), fn)
    return out


def log_iv(v: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """log I_v(x), elementwise, float64 or float32."""
    return _unary("lbessel_log_iv", v, x)


def log_kv(v: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """log K_v(x), elementwise, float64 or float32."""
    return _unary("lbessel_log_kv", v, x)


def log_kv_integral(v: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """log K_v(x), float64, with the paper's own 600-node integral as the
    small-argument branch (lbessel_log_kv_integral_f64)."""
    v, x = _prep(v, x)
    if x.dtype != torch.float64:
        raise LbesselError("log_kv_integral takes float64 tensors")
    out = torch.empty_like(x)
    with torch.cuda.device(x.device):
        _check(_load().lbessel_log_kv_integral_f64(v.data_ptr(), x.data_ptr(), out.data_ptr(),
                                                   x.numel(), _stream(x)),
               "lbessel_log_kv_integral_f64")
    return out


def _order(name: str, v: float, x: torch.Tensor) -> torch.Tensor:
    (x,) = _prep(x)
    out = torch.empty_like(x)
    fn = f"{name}_{_suffix(x)}"
    with torch.cuda.device(x.device):
        _check(getattr(_load(), fn)(float(v), x.data_ptr(), out.data_ptr(), x.numel(),
                                    _stream(x)), fn)
    return out


def log_iv_order(v: float, x: torch.Tensor) -> torch.Tensor:
    """log I_v(x) for one order v (host scalar) over the array x; orders 0 and 1
    take the polynomial fast path."""
    return _order("lbessel_log_iv_order", v, x)


def log_kv_order(v: float, x: torch.Tensor) -> torch.Tensor:
    """log K_v(x) for one order v (host scalar) over the array x; |v| in {0, 1}
    takes the polynomial fast path."""
    return _order("lbessel_log_kv_order", v, x)


def _grad(name: str, v, x, g):
    v, x, g = _prep(v, x, g)
    out = torch.empty_like(x)
    fn = f"{name}_{_suffix(x)}"
    with torch.cuda.device(x.device):
        _check(getattr(_load(), fn)(v.data_ptr(), x.data_ptr(), g.data_ptr(), out.data_ptr(),
                                    x.numel(), _stream(x)), fn)
    return out


def log_iv_grad_x(v, x, g=None):
    """g * d/dx log I_v(x) (g defaults to ones)."""
    if g is None:
        g = torch.ones_like(x)
    return _grad("lbessel_log_iv_grad_x", v, x, g)


def log_kv_grad_x(v, x, g=None):
    """g * d/dx log K_v(x) (g defaults to ones)."""
    if g is None:
        g = torch.ones_like(x)
    return _grad("lbessel_log_kv_grad_x", v, x, g)


def vmf_log_norm(kappa: torch.Tensor, p: float) -> torch.Tensor:
    """log C_p(kappa) of the von Mises-Fisher distribution on S^{p-1}."""
    (k,) = _prep(kappa)
    out = torch.empty_like(k)
    fn = f"lbessel_vmf_log_norm_{_suffix(k)}"
    with torch.cuda.device(k.device):
        _check(getattr(_load(), fn)(k.data_ptr(), float(p), out.data_ptr(), k.numel(),
                                    _stream(k)), fn)
    return out


def vmf_log_norm_grad(kappa: torch.Tensor, p: float) -> torch.Tensor:
    """d/dkappa log C_p(kappa) = -I_{p/2}(kappa) / I_{p/2-1}(kappa) (float64)."""
    (k,) = _prep(kappa)
    if k.dtype != torch.float64:
        raise LbesselError("vmf_log_norm_grad is float64 only")
    out = torch.empty_like(k)
    with torch.cuda.device(k.device):
        _check(_load().lbessel_vmf_log_norm_grad_f64(k.data_ptr(), float(p), out.data_ptr(),
                                                     k.numel(), _stream(k)),
               "lbessel_vmf_log_norm_grad_f64")
    return out


def vmf_colsum(X: torch.Tensor):
    """(colsum, sumsq): column sums (float64, (p,)) of the L2-normalised rows of
    X (N, p) float32, and their sum of squares (float64, (1,))."""
    if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dtype != torch.float32 or X.dim() != 2:
        raise LbesselError("X must be a 2-D float32 tensor on a GPU")
    X = X.contiguous()
    n, p = X.shape
    lib = _load()
    nbytes = lib.lbessel_vmf_colsum_workspace(n, p)
    if nbytes < 0:
        raise LbesselError("invalid vMF shape")
    out = torch.empty(p, dtype=torch.float64, device=X.device)
    ss = torch.empty(1, dtype=torch.float64, device=X.device)
    work = torch.empty(max(int(nbytes), 8), dtype=torch.uint8, device=X.device)
    with torch.cuda.device(X.device):
        _check(lib.lbessel_vmf_colsum_f32(X.data_ptr(), n, p, out.data_ptr(), ss.data_ptr(),
                                          work.data_ptr(), work.numel(), _stream(X)),
               "lbessel_vmf_colsum_f32")
    return out, ss


def vmf_fit(X: torch.Tensor):
    """Maximum-likelihood vMF concentration of the rows of X (N, p) float32,
    solved on the device: (kappa, R, kappa_0, newton_steps) as Python floats."""
    if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dtype != torch.float32 or X.dim() != 2:
        raise LbesselError("X must be a 2-D float32 tensor on a GPU")
    X = X.contiguous()
    n, p = X.shape
    lib = _load()
    nbytes = lib.lbessel_vmf_fit_workspace(n, p)
    if nbytes < 0:
        raise LbesselError("invalid vMF shape")
    res = torch.empty(4, dtype=torch.float64, device=X.device)
    work = torch.empty(max(int(nbytes), 8), dtype=torch.uint8, device=X.device)
    with torch.cuda.device(X.device):
        _check(lib.lbessel_vmf_fit_f32(X.data_ptr(), n, p, res.data_ptr(), work.data_ptr(),
                                       work.numel(), _stream(X)), "lbessel_vmf_fit_f32")
    k, R, k0, steps = res.cpu().tolist()
    return k, R, k0, int(steps)


def vmf_fit_noalloc(X: torch.Tensor, result: torch.Tensor) -> torch.Tensor:
    """vmf_fit into result (4 float64 on X's device: kappa, R, kappa_0,
    Newton steps), with the workspace in the library's static device buffer:
    nothing is allocated.  Calls that overlap on one GPU race."""
    if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dtype != torch.float32 or X.dim() != 2:
        raise LbesselError("X must be a 2-D float32 tensor on a GPU")
    if not X.is_contiguous():
        raise LbesselError("X must be contiguous (a copy would allocate)")
    if (not isinstance(result, torch.Tensor) or result.device != X.device
            or result.dtype != torch.float64 or result.numel() < 4 or not result.is_contiguous()):
        raise LbesselError("result must be 4 contiguous float64 on X's device")
    n, p = X.shape
    with torch.cuda.device(X.device):
        _check(_load().lbessel_vmf_fit_f32_noalloc(X.data_ptr(), n, p, result.data_ptr(),
                                                   _stream(X)), "lbessel_vmf_fit_f32_noalloc")
    return result


class Segment(ctypes.Structure):
    """lbessel_segment_t of include/lbessel.h."""
    _fields_ = [("v", ctypes.c_void_p), ("x", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("tile0", ctypes.c_int64)]


def eval_segments(kind: str, vs, xs, inline: bool = False):
    """log I or log K of several (v, x) array pairs in ONE segmented launch;
    returns the list of outputs (each equals log_iv/log_kv of that pair).
    inline: pass the segment table in the kernel arguments
    (lbessel_eval_segments_inline, at most 32 non-empty pairs) instead of a
    device copy."""
    if len(vs) != len(xs):
        raise LbesselError("vs and xs must have the same length")
    pairs = [_prep(v, x) for v, x in zip(vs, xs)]
    if not pairs:
        return []
    dev, dt = pairs[0][1].device, pairs[0][1].dtype
    if any(x.device != dev or x.dtype != dt for _, x in pairs):
        raise LbesselError("all segments must share one device and dtype")
    lib = _load()
    outs = [torch.empty_like(x) for _, x in pairs]
    table = (Segment * len(pairs))()
    tiles = 0
    k = 0
    for (v, x), o in zip(pairs, outs):
        if x.numel() == 0:
            continue
        table[k] = Segment(v.data_ptr(), x.data_ptr(), o.data_ptr(), x.numel(), tiles)
        tiles += lib.lbessel_segment_tiles(x.numel())
        k += 1
    prec = 64 if dt == torch.float64 else 32
    if inline:
        with torch.cuda.device(dev):
            _check(lib.lbessel_eval_segments_inline(KIND[kind], prec, ctypes.addressof(table), k,
                                                    tiles, _stream(pairs[0][1])),
                   "lbessel_eval_segments_inline")
            torch.cuda.current_stream(dev).synchronize()
        return outs
    host = torch.frombuffer(bytearray(bytes(table)), dtype=torch.uint8)
    dseg = host.to(dev)
    with torch.cuda.device(dev):
        _check(lib.lbessel_eval_segments(KIND[kind], prec, dseg.data_ptr(), k, tiles,
                                         _stream(dseg)), "lbessel_eval_segments")
        torch.cuda.current_stream(dev).synchronize()   # table and outputs live until here
    return outs


VARIANTS = {"default": 0, "paper_regimes": 1, "u_integral": 2, "simpson": 3, "paper": 4,
            "seven": 5}
LAYOUTS = {"grouped": 0, "naive": 1, "sorted": 2}


def eval_variant(kind: str, variant: str, layout: str, v: torch.Tensor, x: torch.Tensor,
                 work: torch.Tensor | None = None) -> torch.Tensor:
    """Forward log I / log K (float64) with one of the paper's own choices put
    back (see VARIANTS) and a chosen grouping layout (see LAYOUTS)."""
    v, x = _prep(v, x)
    if x.dtype != torch.float64:
        raise LbesselError("eval_variant is float64 only")
    lib = _load()
    out = torch.empty_like(x)
    if layout == "sorted" and work is None:
        need = lib.lbessel_eval_variant_workspace(x.numel())
        if need < 0:
            raise LbesselError("too many elements for the sorted layout")
        work = torch.empty(max(int(need), 8), dtype=torch.uint8, device=x.device)
    wp, wn = (work.data_ptr(), work.numel()) if work is not None else (None, 0)
    with torch.cuda.device(x.device):
        _check(lib.lbessel_eval_variant(KIND[kind], VARIANTS[variant], LAYOUTS[layout],
                                        v.data_ptr(), x.data_ptr(), out.data_ptr(), x.numel(),
                                        wp, wn, _stream(x)), "lbessel_eval_variant")
    return out


def classify(kind: str, v: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """Branch index per element (0 mu20, 1 u13, 2 fallback, 3 special)."""
    v, x = _prep(v, x)
    out = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
    prec = 64 if x.dtype == torch.float64 else 32
    with torch.cuda.device(x.device):
        _check(_load().lbessel_classify(KIND[kind], prec, v.data_ptr(), x.data_ptr(),
                                        out.data_ptr(), x.numel(), _stream(x)),
               "lbessel_classify")
    return out


def k_nodes(v: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """Integrand evaluations of the log K fallback per element (int32; 0 for
    elements that take another branch)."""
    v, x = _prep(v, x)
    out = torch.empty(x.shape, dtype=torch.int32, device=x.device)
    prec = 64 if x.dtype == torch.float64 else 32
    with torch.cuda.device(x.device):
        _check(_load().lbessel_k_nodes(prec, v.data_ptr(), x.data_ptr(), out.data_ptr(),
                                       x.numel(), _stream(x)), "lbessel_k_nodes")
    return out


ELEMENTARY = {"rcp": 0, "exp": 1, "exp_bounded": 2, "log": 3, "log1p": 4, "rsqrt": 5}


def elementary(op: str, a: torch.Tensor) -> torch.Tensor:
    """The library's binary64 elementary function `op` (see ELEMENTARY),
    evaluated on the device (lbessel_elementary_f64)."""
    (a,) = _prep(a)
    if a.dtype != torch.float64:
        raise LbesselError("elementary takes float64 tensors")
    out = torch.empty_like(a)
    with torch.cuda.device(a.device):
        _check(_load().lbessel_elementary_f64(ELEMENTARY[op], a.data_ptr(), out.data_ptr(),
                                              a.numel(), _stream(a)), "lbessel_elementary_f64")
    return out


def k_terms(v: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """Temme-series terms of the log K fallback per element (int32; 0 for
    elements that take another branch or sub-case)."""
    v, x = _prep(v, x)
    out = torch.empty(x.shape, dtype=torch.int32, device=x.device)
    prec = 64 if x.dtype == torch.float64 else 32
    with torch.cuda.device(x.device):
        _check(_load().lbessel_k_terms(prec, v.data_ptr(), x.data_ptr(), out.data_ptr(),
                                       x.numel(), _stream(x)), "lbessel_k_terms")
    return out


def eval_branch(kind: str, branch: int, v: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """Every element through one forced branch (float64 or float32)."""
    v, x = _prep(v, x)
    out = torch.empty_like(x)
    fn = f"lbessel_eval_branch_{_suffix(x)}"
    with torch.cuda.device(x.device):
        _check(getattr(_load(), fn)(KIND[kind], int(branch), v.data_ptr(), x.data_ptr(),
                                    out.data_ptr(), x.numel(), _stream(x)), fn)
    return out


def eval_ungrouped(kind: str, v: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """Forward evaluation without regrouping by branch (one element per thread)."""
    v, x = _prep(v, x)
    out = torch.empty_like(x)
    prec = 64 if x.dtype == torch.float64 else 32
    with torch.cuda.device(x.device):
        _check(_load().lbessel_eval_ungrouped(KIND[kind], prec, v.data_ptr(), x.data_ptr(),
                                              out.data_ptr(), x.numel(), _stream(x)),
               "lbessel_eval_ungrouped")
    return out


class LogIv(torch.autograd.Function):
    """log I_v(x) with the hand-written d/dx backward (no gradient in v)."""

    @staticmethod
    def forward(ctx, v, x):
        ctx.save_for_backward(v, x)
        return log_iv(v, x)

    @staticmethod
    def backward(ctx, g):
        v, x = ctx.saved_tensors
        if ctx.needs_input_grad[0]:
            raise LbesselError("the derivative in the order v is not provided")
        return None, log_iv_grad_x(v, x, g.contiguous())


class LogKv(torch.autograd.Function):
    """log K_v(x) with the hand-written d/dx backward (no gradient in v)."""

    @staticmethod
    def forward(ctx, v, x):
        ctx.save_for_backward(v, x)
        return log_kv(v, x)

    @staticmethod
    def backward(ctx, g):
        v, x = ctx.saved_tensors
        if ctx.needs_input_grad[0]:
            raise LbesselError("the derivative in the order v is not provided")
        return None, log_kv_grad_x(v, x, g.contiguous())


class VmfLogNorm(torch.autograd.Function):
    """log C_p(kappa) (float64) with d/dkappa = -I_{p/2}(kappa) / I_{p/2-1}(kappa)."""

    @staticmethod
    def forward(ctx, kappa, p):
        ctx.save_for_backward(kappa)
        ctx.p = float(p)
        return vmf_log_norm(kappa, p)

    @staticmethod
    def backward(ctx, g):
        (kappa,) = ctx.saved_tensors
        return g * vmf_log_norm_grad(kappa, ctx.p), None
