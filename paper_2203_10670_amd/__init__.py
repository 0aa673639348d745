"""Python binding of libfcfs: fully convolutional fractional scaling on MI355X.

Thin ctypes marshalling over the C ABI declared in ``include/fcfs.h``; every
step of the computation runs in the library's HIP kernels. PyTorch supplies
device memory (its caching allocator) and the stream work is enqueued on.

Low-level functions carry the C names (``fcfs_plan``, ``fcfs_forward``, ...)
and take plain integers / pointers. The convenience layer on top
(``Plan``, ``resize``, ``FCFSFunction``) converts torch tensors to pointers.

There is no fallback: if ``libfcfs.so`` is missing, importing this package
raises, and every call requires tensors that live on a ROCm device.
"""
from __future__ import annotations

import ctypes
import math
import os

__all__ = [
    "FcfsError", "METHODS", "PADS", "GRIDS", "DTYPES", "lib", "library_path",
    "fcfs_plan", "fcfs_plan_ex", "fcfs_plan_destroy", "fcfs_plan_query", "fcfs_plan_taps",
    "fcfs_output_size",
    "fcfs_forward", "fcfs_forward_config", "fcfs_backward_workspace", "fcfs_backward", "fcfs_status_string",
    "fcfs_backward_noalloc", "FCFS_NOALLOC_SCRATCH_BYTES",
    "fcfs_version", "Plan", "resize", "FCFSFunction",
    "fcfs_request", "fcfs_result", "fcfs_server_create", "fcfs_submit", "fcfs_poll", "fcfs_wait",
    "fcfs_release", "fcfs_server_stats", "fcfs_server_debug", "fcfs_server_destroy", "Server",
    "fcfs_server_config", "fcfs_server_replay", "fcfs_server_reset_stats",
    "device_view",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libfcfs.so")

METHODS = {"nearest": 0, "bilinear": 1, "bicubic": 2, "dw4": 3, "mix4": 4}
PADS = {"zero": 0, "replicate": 1, "reflect": 2}
GRIDS = {"half": 0, "paper": 1, "asym": 2}
DTYPES = {"f32": 0, "bf16": 1, "f16": 2}

OK, E_INVAL, E_UNSUPPORTED, E_NOMEM, E_DEVICE, E_AGAIN, E_PENDING, E_CANCELLED = range(8)
FCFS_SERVER_MAX_BATCH, FCFS_SERVER_DISCARD_OUTPUTS, FCFS_SERVER_CHUNK_WAVES = 1, 2, 3


class FcfsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (status %d)" % (where, fcfs_status_string(status), status))


def _load():
    if not os.path.exists(library_path):
        raise ImportError("libfcfs.so is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
                          "or `python paper_2203_10670_amd/build.py` first (%s)" % library_path)
    # The library must use the HIP runtime torch uses (streams and device
    # state are per runtime). torch ships its own libamdhip64, which its
    # libraries ask for by an unversioned name: loaded after the library
    # (which asks for libamdhip64.so.7 and gets the system one), torch would
    # bring a second runtime into the process. Loading torch first makes the
    # library bind to torch's runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    return ctypes.CDLL(library_path)


lib = _load()

_I, _I64, _P, _SZ = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
_PP = ctypes.POINTER(ctypes.c_void_p)


def _sig(name, args, res=_I):
    f = getattr(lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("fcfs_plan", [_I, _I, _I, _I, _PP])
_sig("fcfs_plan_ex", [_I, _I, _I, _I, _I, _I, _I, _PP])
_sig("fcfs_plan_destroy", [_P])
_sig("fcfs_plan_query", [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)])
_sig("fcfs_plan_taps", [_P, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_float)])
_sig("fcfs_output_size", [_P, _I64, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_I64)])
_sig("fcfs_forward", [_P, _I, _I64, _I64, _I64, _I64, _P, _P, _I64, _P, _P])
_sig("fcfs_forward_config", [_P, _I, _I64, _I64, _I64, _I64, ctypes.POINTER(_I), ctypes.POINTER(_I),
                             ctypes.POINTER(_I), ctypes.POINTER(_I64)])
_sig("fcfs_forward_1d", [_P, _I, _I64, _I64, _I64, _P, _P, _P])
_sig("fcfs_forward_3d_workspace", [_P, _P, _I, _I64, _I64, _I64, _I64, _I64, ctypes.POINTER(_SZ)])
_sig("fcfs_forward_3d", [_P, _P, _I, _I64, _I64, _I64, _I64, _I64, _P, _P, _P, _SZ, _P])
_sig("fcfs_backward_workspace", [_P, _I, _I64, _I64, _I64, _I64, _I64, ctypes.POINTER(_SZ)])
_sig("fcfs_backward", [_P, _I, _I64, _I64, _I64, _I64, _P, _P, _I64, _P, _P, _P, _P, _SZ, _P])
_sig("fcfs_backward_noalloc", [_P, _I, _I64, _I64, _I64, _I64, _P, _P, _I64, _P, _P, _P, _P])


class fcfs_request(ctypes.Structure):
    _fields_ = [("p", _I), ("q", _I), ("method", _I), ("pad", _I), ("dtype", _I),
                ("n", _I64), ("c", _I64), ("h", _I64), ("w", _I64),
                ("x", _P), ("seed", ctypes.c_uint64), ("y", _P)]


class fcfs_result(ctypes.Structure):
    _fields_ = [("status", _I), ("y", _P), ("h_out", _I64), ("w_out", _I64),
                ("t_arrive_us", ctypes.c_double), ("t_start_us", ctypes.c_double),
                ("t_done_us", ctypes.c_double)]


_D = ctypes.POINTER(ctypes.c_double)
_sig("fcfs_server_create", [_I, _SZ, _I, _PP])
_sig("fcfs_submit", [_P, ctypes.POINTER(fcfs_request), ctypes.POINTER(ctypes.c_uint64)])
_sig("fcfs_poll", [_P, ctypes.c_uint64, ctypes.POINTER(fcfs_result)])
_sig("fcfs_wait", [_P, ctypes.c_uint64, _I64, ctypes.POINTER(fcfs_result)])
_sig("fcfs_release", [_P, ctypes.c_uint64])
_sig("fcfs_server_stats", [_P, _D, _D, _D, _D])
_sig("fcfs_server_debug", [_P, _I, _I64])
_sig("fcfs_server_destroy", [_P])
_sig("fcfs_server_config", [_P, _I, _I64])
_sig("fcfs_server_replay", [_P, ctypes.POINTER(fcfs_request), ctypes.POINTER(ctypes.c_double), _I64,
                            ctypes.POINTER(ctypes.c_uint64)])
_sig("fcfs_server_reset_stats", [_P])
_sig("fcfs_status_string", [_I], ctypes.c_char_p)
_sig("fcfs_version", [], _I)


def _check(status: int, where: str):
    if status != OK:
        raise FcfsError(status, where)


# ------------------------------------------------------------------ C names

def fcfs_status_string(status: int) -> str:
    return lib.fcfs_status_string(status).decode()


def fcfs_version() -> int:
    return lib.fcfs_version()


def fcfs_plan(p: int, q: int, method: int, pad: int) -> int:
    h = ctypes.c_void_p()
    _check(lib.fcfs_plan(p, q, method, pad, ctypes.byref(h)), "fcfs_plan")
    return h.value


def fcfs_plan_ex(p_h: int, q_h: int, p_w: int, q_w: int, method: int, pad: int, grid: int) -> int:
    h = ctypes.c_void_p()
    _check(lib.fcfs_plan_ex(p_h, q_h, p_w, q_w, method, pad, grid, ctypes.byref(h)), "fcfs_plan_ex")
    return h.value


def fcfs_plan_destroy(plan: int) -> None:
    _check(lib.fcfs_plan_destroy(plan), "fcfs_plan_destroy")


def fcfs_plan_query(plan: int):
    p, q, t = _I(), _I(), _I()
    _check(lib.fcfs_plan_query(plan, ctypes.byref(p), ctypes.byref(q), ctypes.byref(t)), "fcfs_plan_query")
    return p.value, q.value, t.value


def fcfs_plan_taps(plan: int, axis: int, phase: int):
    """(first tap offset, [4 weights]) of one phase of one axis."""
    off = _I()
    w = (ctypes.c_float * 4)()
    _check(lib.fcfs_plan_taps(plan, axis, phase, ctypes.byref(off), w), "fcfs_plan_taps")
    return off.value, list(w)


def fcfs_output_size(plan: int, h: int, w: int):
    ho, wo = _I64(), _I64()
    _check(lib.fcfs_output_size(plan, h, w, ctypes.byref(ho), ctypes.byref(wo)), "fcfs_output_size")
    return ho.value, wo.value


def fcfs_forward(plan, dtype, n, c_in, h, w, x_ptr, weight_ptr, c_out, y_ptr, stream) -> int:
    """Returns the raw status (callers decide whether to raise)."""
    return lib.fcfs_forward(plan, dtype, n, c_in, h, w, x_ptr, weight_ptr, c_out, y_ptr, stream)


def fcfs_forward_config(plan, dtype, n, c_in, h, w):
    """(kernel_id, strip_width, band_cells, waves) of the forward launch."""
    k, tw, bc, wv = _I(), _I(), _I(), _I64()
    _check(lib.fcfs_forward_config(plan, dtype, n, c_in, h, w, ctypes.byref(k), ctypes.byref(tw),
                                   ctypes.byref(bc), ctypes.byref(wv)), "fcfs_forward_config")
    return k.value, tw.value, bc.value, wv.value


def fcfs_forward_1d(plan, dtype, n, c, l, x_ptr, y_ptr, stream) -> int:
    return lib.fcfs_forward_1d(plan, dtype, n, c, l, x_ptr, y_ptr, stream)


def fcfs_forward_3d_workspace(plan_d, plan_hw, dtype, n, c, d, h, w) -> int:
    b = _SZ()
    _check(lib.fcfs_forward_3d_workspace(plan_d, plan_hw, dtype, n, c, d, h, w, ctypes.byref(b)),
           "fcfs_forward_3d_workspace")
    return b.value


def fcfs_forward_3d(plan_d, plan_hw, dtype, n, c, d, h, w, x_ptr, y_ptr, ws_ptr, ws_bytes, stream) -> int:
    return lib.fcfs_forward_3d(plan_d, plan_hw, dtype, n, c, d, h, w, x_ptr, y_ptr, ws_ptr, ws_bytes, stream)


def fcfs_backward_workspace(plan, dtype, n, c_in, h, w, c_out) -> int:
    b = _SZ()
    _check(lib.fcfs_backward_workspace(plan, dtype, n, c_in, h, w, c_out, ctypes.byref(b)),
           "fcfs_backward_workspace")
    return b.value


def fcfs_backward(plan, dtype, n, c_in, h, w, x_ptr, weight_ptr, c_out, dy_ptr, dx_ptr, dw_ptr,
                  ws_ptr, ws_bytes, stream) -> int:
    return lib.fcfs_backward(plan, dtype, n, c_in, h, w, x_ptr, weight_ptr, c_out, dy_ptr, dx_ptr,
                             dw_ptr, ws_ptr, ws_bytes, stream)


FCFS_NOALLOC_SCRATCH_BYTES = 64 << 20


def fcfs_backward_noalloc(plan, dtype, n, c_in, h, w, x_ptr, weight_ptr, c_out, dy_ptr, dx_ptr, dw_ptr,
                          stream) -> int:
    """fcfs_backward with the library's fixed device workspace (no allocation)."""
    return lib.fcfs_backward_noalloc(plan, dtype, n, c_in, h, w, x_ptr, weight_ptr, c_out, dy_ptr, dx_ptr,
                                     dw_ptr, stream)


def fcfs_server_create(device: int, mem_budget_bytes: int, max_slots: int) -> int:
    h = ctypes.c_void_p()
    _check(lib.fcfs_server_create(device, mem_budget_bytes, max_slots, ctypes.byref(h)), "fcfs_server_create")
    return h.value


def fcfs_submit(server: int, req: fcfs_request):
    """Returns (status, ticket)."""
    t = ctypes.c_uint64()
    st = lib.fcfs_submit(server, ctypes.byref(req), ctypes.byref(t))
    return st, t.value


def fcfs_poll(server: int, ticket: int):
    r = fcfs_result()
    st = lib.fcfs_poll(server, ticket, ctypes.byref(r))
    return st, r


def fcfs_wait(server: int, ticket: int, timeout_us: int = -1):
    r = fcfs_result()
    st = lib.fcfs_wait(server, ticket, timeout_us, ctypes.byref(r))
    return st, r


def fcfs_release(server: int, ticket: int) -> int:
    return lib.fcfs_release(server, ticket)


def fcfs_server_stats(server: int):
    """(p50_us, p99_us, req_per_s, gbps)."""
    v = [ctypes.c_double() for _ in range(4)]
    _check(lib.fcfs_server_stats(server, *[ctypes.byref(x) for x in v]), "fcfs_server_stats")
    return tuple(x.value for x in v)


def fcfs_server_debug(server: int, hook: int, value: int) -> int:
    return lib.fcfs_server_debug(server, hook, value)


def fcfs_server_config(server: int, option: int, value: int) -> int:
    return lib.fcfs_server_config(server, option, value)


def fcfs_server_replay(server: int, reqs, arrival_us):
    """Submit requests at arrival offsets (µs) from a native loop; returns
    (status, tickets)."""
    n = len(reqs)
    arr = (fcfs_request * n)(*reqs)
    t = (ctypes.c_double * n)(*arrival_us)
    out = (ctypes.c_uint64 * n)()
    st = lib.fcfs_server_replay(server, arr, t, n, out)
    return st, list(out)


def fcfs_server_reset_stats(server: int) -> int:
    return lib.fcfs_server_reset_stats(server)


def fcfs_server_destroy(server: int) -> None:
    _check(lib.fcfs_server_destroy(server), "fcfs_server_destroy")


class Server:
    """Owns an fcfs serving loop on one device."""

    def __init__(self, device: int = 0, mem_budget_bytes: int = 64 << 30, max_slots: int = 256):
        self.handle = fcfs_server_create(device, mem_budget_bytes, max_slots)

    def submit(self, p, q, method="bilinear", pad="replicate", dtype="f32", shape=(1, 1, 1, 1), x=None,
               seed=0, y=None):
        """Queue a request; x / y are device tensors (or None: generated input
        from ``seed`` / server-owned output). Returns the ticket."""
        n, c, h, w = shape
        if x is not None or y is not None:
            # the server's streams do not wait for the caller's: whatever the
            # caller's stream still has to do with x or y must finish first
            t = x if x is not None else y
            _torch().cuda.current_stream(t.device).synchronize()
        req = fcfs_request(p, q, METHODS[method], PADS[pad], DTYPES[dtype], n, c, h, w,
                           None if x is None else _dev_ptr(x), seed, None if y is None else _dev_ptr(y))
        st, t = fcfs_submit(self.handle, req)
        _check(st, "fcfs_submit")
        return t

    def wait(self, ticket, timeout_us=-1):
        st, r = fcfs_wait(self.handle, ticket, timeout_us)
        _check(st, "fcfs_wait")
        return r

    def release(self, ticket):
        _check(fcfs_release(self.handle, ticket), "fcfs_release")

    def stats(self):
        return fcfs_server_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            fcfs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def device_view(ptr: int, shape, dtype: str, device=None):
    """A torch tensor over device memory owned by the library (a server
    output); valid until the ticket is released. The memory is copied."""
    torch = _torch()
    td = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[dtype]
    n = 1
    for d in shape:
        n *= d
    out = torch.empty(shape, dtype=td, device=device or "cuda")
    if n:
        _check(0 if lib_copy(out.data_ptr(), ptr, n * out.element_size()) == 0 else E_DEVICE, "copy")
    return out


def lib_copy(dst: int, src: int, nbytes: int) -> int:
    """Device-to-device copy through the HIP runtime (used to read server outputs)."""
    hip = _hip()
    return hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), ctypes.c_size_t(nbytes), 3)


_hip_lib = None


def _hip():
    global _hip_lib
    if _hip_lib is None:
        _hip_lib = ctypes.CDLL("libamdhip64.so")
        _hip_lib.hipMemcpy.argtypes = [_P, _P, _SZ, _I]
        _hip_lib.hipMemcpy.restype = _I
    return _hip_lib


# ------------------------------------------------------------------ torch layer

def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    m = {torch.float32: 0, torch.bfloat16: 1, torch.float16: 2}
    if t.dtype not in m:
        raise TypeError("unsupported dtype %s" % t.dtype)
    return m[t.dtype]


def _stream_ptr(device) -> int:
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


def _dev_ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libfcfs takes device tensors only")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous NCHW")
    return t.data_ptr()


class Plan:
    """Owns an fcfs plan handle."""

    def __init__(self, p: int, q: int, method: str = "bilinear", pad: str = "replicate",
                 grid: str = "half", pw: int | None = None, qw: int | None = None):
        self.method, self.pad, self.grid = method, pad, grid
        self.p, self.q = p, q
        self.pw = p if pw is None else pw
        self.qw = q if qw is None else qw
        self.handle = fcfs_plan_ex(p, q, self.pw, self.qw, METHODS[method], PADS[pad], GRIDS[grid])
        self.p_red, self.q_red, self.taps = fcfs_plan_query(self.handle)

    def output_size(self, h: int, w: int):
        return fcfs_output_size(self.handle, h, w)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and lib is not None:   # (module globals may be gone at interpreter exit)
            lib.fcfs_plan_destroy(h)
            self.handle = None

    # forward / backward on torch tensors -------------------------------
    def _p_width(self) -> int:
        return self.pw // math.gcd(self.pw, self.qw)

    def _check_weight(self, weight, act, c_in):
        """The C ABI reads the weight through a plain pointer whose type and
        extent follow from the method: refuse anything else here.
        Fixed methods take none; the depthwise layer an FP32
        [c_in][p_h][p_w][4][4]; the channel-mixing layer
        [p_h][p_w][c_out][c_in][4][4] in the activations' type. Returns c_out."""
        if self.method not in ("dw4", "mix4"):
            if weight is not None:
                raise ValueError("method %r takes no weight" % self.method)
            return c_in
        if weight is None:
            raise ValueError("method %r needs a weight" % self.method)
        if weight.device != act.device:
            raise ValueError("weight must be on the activations' device")
        ph, pw = self.p_red, self._p_width()
        if self.method == "dw4":
            torch = _torch()
            if weight.dtype != torch.float32:
                raise TypeError("the depthwise layer's weight must be float32, got %s" % weight.dtype)
            want = (c_in, ph, pw, 4, 4)
            if tuple(weight.shape) != want:
                raise ValueError("depthwise weight shape %s, expected %s" % (tuple(weight.shape), want))
            return c_in
        if weight.dtype != act.dtype:
            raise TypeError("the channel-mixing weight must have the activations' type %s, got %s"
                            % (act.dtype, weight.dtype))
        if weight.dim() != 6 or tuple(weight.shape[:2]) != (ph, pw) or weight.shape[3] != c_in \
                or tuple(weight.shape[4:]) != (4, 4):
            raise ValueError("channel-mixing weight shape %s, expected (%d, %d, c_out, %d, 4, 4)"
                             % (tuple(weight.shape), ph, pw, c_in))
        return int(weight.shape[2])

    def forward(self, x, weight=None, out=None):
        torch = _torch()
        n, c, h, w = x.shape
        ho, wo = self.output_size(h, w)
        c_out = self._check_weight(weight, x, c)
        if out is None:
            out = torch.empty((n, c_out, ho, wo), dtype=x.dtype, device=x.device)
        st = fcfs_forward(self.handle, _dtype_code(x), n, c, h, w, _dev_ptr(x), _dev_ptr(weight),
                          c_out, _dev_ptr(out), _stream_ptr(x.device))
        _check(st, "fcfs_forward")
        return out

    def backward(self, dy, x_shape, x=None, weight=None, need_dx=True, need_dw=False):
        torch = _torch()
        n, c, h, w = x_shape
        c_out = dy.shape[1]
        if self.method in ("dw4", "mix4") or weight is not None:
            if self._check_weight(weight, dy, c) != c_out:
                raise ValueError("dy has %d channels, the weight %d outputs" % (c_out, weight.shape[2]))
        if x is not None and (x.dtype != dy.dtype or tuple(x.shape) != tuple(x_shape)):
            raise ValueError("x must have dy's type and the shape %s" % (tuple(x_shape),))
        dx = torch.empty((n, c, h, w), dtype=dy.dtype, device=dy.device) if need_dx else None
        dw = torch.empty_like(weight, dtype=torch.float32) if need_dw else None
        code = _dtype_code(dy)
        ws_bytes = fcfs_backward_workspace(self.handle, code, n, c, h, w, c_out)
        ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dy.device)
        st = fcfs_backward(self.handle, code, n, c, h, w, _dev_ptr(x), _dev_ptr(weight), c_out,
                           _dev_ptr(dy), _dev_ptr(dx), _dev_ptr(dw), _dev_ptr(ws), ws_bytes,
                           _stream_ptr(dy.device))
        _check(st, "fcfs_backward")
        return dx, dw


_plan_cache: dict = {}


def _cached_plan(p, q, method, pad, grid, pw, qw):
    key = (p, q, method, pad, grid, pw, qw)
    pl = _plan_cache.get(key)
    if pl is None:
        pl = _plan_cache[key] = Plan(p, q, method, pad, grid, pw, qw)
    return pl


def resize(x, p: int, q: int, method: str = "bilinear", pad: str = "replicate", grid: str = "half",
           weight=None, pw: int | None = None, qw: int | None = None):
    """Rescale an NCHW device tensor by p/q (and pw/qw on the width axis)."""
    return _cached_plan(p, q, method, pad, grid, pw, qw).forward(x.contiguous(), weight)


def resize1d(x, p: int, q: int, method: str = "bilinear", pad: str = "replicate", grid: str = "half"):
    """Rescale an NCL device tensor (1D signals) by p/q."""
    torch = _torch()
    x = x.contiguous()
    n, c, l = x.shape
    pl = _cached_plan(1, 1, method, pad, grid, p, q)
    lo = pl.output_size(1, l)[1]
    y = torch.empty((n, c, lo), dtype=x.dtype, device=x.device)
    _check(fcfs_forward_1d(pl.handle, _dtype_code(x), n, c, l, _dev_ptr(x), _dev_ptr(y), _stream_ptr(x.device)),
           "fcfs_forward_1d")
    return y


def resize3d(x, factors, method: str = "bilinear", pad: str = "replicate", grid: str = "half"):
    """Rescale an NCDHW device tensor by ``factors`` = ((p_d, q_d), (p_h, q_h), (p_w, q_w))."""
    torch = _torch()
    x = x.contiguous()
    n, c, d, h, w = x.shape
    (pd, qd), (ph, qh), (pw, qw) = factors
    pl_d = _cached_plan(pd, qd, method, pad, grid, 1, 1)
    pl_hw = _cached_plan(ph, qh, method, pad, grid, pw, qw)
    do = pl_d.output_size(d, 1)[0]
    ho, wo = pl_hw.output_size(h, w)
    code = _dtype_code(x)
    y = torch.empty((n, c, do, ho, wo), dtype=x.dtype, device=x.device)
    wsb = fcfs_forward_3d_workspace(pl_d.handle, pl_hw.handle, code, n, c, d, h, w)
    ws = torch.empty(max(wsb, 4), dtype=torch.uint8, device=x.device)
    _check(fcfs_forward_3d(pl_d.handle, pl_hw.handle, code, n, c, d, h, w, _dev_ptr(x), _dev_ptr(y),
                           _dev_ptr(ws), wsb, _stream_ptr(x.device)), "fcfs_forward_3d")
    return y


def _make_function():
    torch = _torch()

    class FCFSFunction(torch.autograd.Function):
        """Differentiable FCFS layer: forward and backward run in libfcfs."""

        @staticmethod
        def forward(ctx, x, weight, plan: Plan):
            x = x.contiguous()
            w = weight.contiguous() if weight is not None else None
            ctx.plan = plan
            ctx.x_shape = tuple(x.shape)
            ctx.save_for_backward(x, w)
            return plan.forward(x, w)

        @staticmethod
        def backward(ctx, dy):
            x, w = ctx.saved_tensors
            need_dx = ctx.needs_input_grad[0]
            need_dw = w is not None and ctx.needs_input_grad[1]
            dx, dw = ctx.plan.backward(dy.contiguous(), ctx.x_shape, x=x if need_dw else None,
                                       weight=w, need_dx=need_dx, need_dw=need_dw)
            if dw is not None and dw.dtype != w.dtype:
                dw = dw.to(w.dtype)   # (the FP32 weight gradient, in the parameter's type)
            return dx, dw, None

    return FCFSFunction


class _LazyFunction:
    _cls = None

    def __getattr__(self, name):
        if _LazyFunction._cls is None:
            _LazyFunction._cls = _make_function()
        return getattr(_LazyFunction._cls, name)


FCFSFunction = _LazyFunction()
