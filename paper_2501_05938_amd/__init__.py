"""Python binding of libwf, the MI355X (gfx950) anti-diagonal wavefront sweep.

Only argument marshalling lives here: every step of the sweep runs in the HIP
kernels of libwf.so (built in-tree by ``paper_2501_05938_amd.build``).  PyTorch
tensors provide device memory and streams.  There is no CPU fallback: if the
library is missing or the device is not gfx950, calls raise.

    import torch, paper_2501_05938_amd as wf
    H = wf.solve(cost)                       # cost: (m, n) float32/int32 CUDA tensor
    last_row, last_col, final = wf.solve(cost, mode="edges")
    outs = wf.solve_batched([c0, c1, ...])

The cell rule (see include/wf.h): H[i][j] = c[i][j] + op(H[i-1][j], H[i][j-1], H[i-1][j-1]),
op = min or max, with default or explicit top (n+1 values) / left (m values) boundaries.
"""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwf.so")

WF_OK, WF_PENDING = 0, 1
STATUS = {0: "WF_OK", 1: "WF_PENDING", -1: "WF_EINVAL", -2: "WF_ENOMEM", -3: "WF_E2BIG", -4: "WF_EHIP",
          -5: "WF_ETIMEDOUT", -6: "WF_ENOTFOUND", -7: "WF_ESHUTDOWN", -8: "WF_EUNSUPPORTED"}
DTYPES = {"f32": 0, "i32": 1, "f64": 2}
RULES = {"min": 0, "max": 1}
MODES = {"full": 0, "edges": 1}


class WfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("rule", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("flags", ctypes.c_int32),
                ("cost", ctypes.c_void_p), ("ld_cost", ctypes.c_int64),
                ("out", ctypes.c_void_p), ("ld_out", ctypes.c_int64),
                ("top", ctypes.c_void_p), ("left", ctypes.c_void_p),
                ("last_row", ctypes.c_void_p), ("last_col", ctypes.c_void_p), ("final_cell", ctypes.c_void_p),
                ("seq_x", ctypes.c_void_p), ("seq_y", ctypes.c_void_p)]


COST_ABSDIFF = 1  # WF_COST_ABSDIFF


class Tuning(ctypes.Structure):
    _fields_ = [("waves_per_wg", ctypes.c_int32), ("max_wgs", ctypes.c_int32), ("order", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("rows_per_lane", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("copy_streams", ctypes.c_int32),
                ("max_wait_skip_us", ctypes.c_int32), ("staging_bytes", ctypes.c_int64),
                ("reserved", ctypes.c_int32 * 2)]


INPUT_DEVICE, INPUT_HOST, INPUT_SEED, INPUT_HOST_PINNED = 0, 1, 2, 3


class Request(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("rule", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("input_kind", ctypes.c_int32), ("input", ctypes.c_void_p), ("ld_input", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("ready_event", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("out", ctypes.c_void_p), ("ld_out", ctypes.c_int64),
                ("last_row", ctypes.c_void_p), ("last_col", ctypes.c_void_p), ("final_cell", ctypes.c_void_p),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


class StreamSample(ctypes.Structure):
    _fields_ = [("size", ctypes.c_double), ("streams", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("t_str", ctypes.c_double), ("t_non_str", ctypes.c_double), ("sum", ctypes.c_double)]


class StreamModel(ctypes.Structure):
    _fields_ = [("sum_slope", ctypes.c_double), ("sum_intercept", ctypes.c_double),
                ("split_size", ctypes.c_double), ("small", ctypes.c_double * 3), ("big", ctypes.c_double * 3)]


class FitReport(ctypes.Structure):
    _fields_ = [("r2_train", ctypes.c_double), ("r2_test", ctypes.c_double),
                ("mse_train", ctypes.c_double), ("mse_test", ctypes.c_double),
                ("n_train", ctypes.c_int64), ("n_test", ctypes.c_int64)]


# Every symbol the C header declares, with its ctypes signature.
_P = ctypes.c_void_p
_SIGS = {
    "wf_init": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_P)]),
    "wf_destroy": (ctypes.c_int, [_P]),
    "wf_solve": (ctypes.c_int, [_P, ctypes.POINTER(Problem), _P]),
    "wf_solve_batched": (ctypes.c_int, [_P, ctypes.POINTER(Problem), ctypes.c_int64, ctypes.POINTER(Tuning), _P]),
    "wf_solve_tuned": (ctypes.c_int, [_P, ctypes.POINTER(Problem), ctypes.POINTER(Tuning), _P]),
    "wf_solve_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(Problem), _P]),
    "wf_traceback": (ctypes.c_int, [_P, ctypes.POINTER(Problem), _P, _P, _P]),
    "wf_solve_each": (ctypes.c_int, [_P, ctypes.POINTER(Problem), ctypes.c_int64, ctypes.POINTER(_P), ctypes.c_int32]),
    "wf_set_watchdog": (ctypes.c_int, [_P, ctypes.c_int64]),
    "wf_check": (ctypes.c_int, [_P]),
    "wf_measure_step_ns": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    "wf_server_create": (ctypes.c_int, [_P, ctypes.POINTER(ServerOpts), ctypes.POINTER(_P)]),
    "wf_submit": (ctypes.c_int, [_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "wf_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(Result)]),
    "wf_release": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "wf_server_destroy": (ctypes.c_int, [_P]),
    "wf_server_memory": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "wf_server_done": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int64)]),
    "wf_stream_model_fit": (ctypes.c_int, [ctypes.POINTER(StreamSample), ctypes.c_int64, ctypes.c_double,
                                           ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(StreamModel),
                                           ctypes.POINTER(FitReport)]),
    "wf_stream_model_overhead": (ctypes.c_double, [ctypes.POINTER(StreamModel), ctypes.c_double, ctypes.c_int32]),
    "wf_stream_model_choose": (ctypes.c_int, [ctypes.POINTER(StreamModel), ctypes.c_double,
                                              ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "wf_last_error": (ctypes.c_char_p, []),
    "wf_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "wf_version": (ctypes.c_char_p, []),
}

_lib = None
_lock = threading.Lock()


def load_library(path: str = LIB_PATH):
    """Load libwf.so and bind every exported entry point (no GPU needed)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise RuntimeError(f"libwf.so not built ({path}); run python -m paper_2501_05938_amd.build")
            lib = ctypes.CDLL(path)
            for name, (res, args) in _SIGS.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def _check(status: int):
    if status != WF_OK:
        raise WfError(status, load_library().wf_last_error().decode(errors="replace"))


_ctx = {}


def context(device: int | None = None):
    """The per-(thread, device) libwf context."""
    import torch
    if device is None:
        device = torch.cuda.current_device()
    key = (threading.get_ident(), device)
    c = _ctx.get(key)
    if c is None:
        lib = load_library()
        h = _P()
        _check(lib.wf_init(device, ctypes.byref(h)))
        c = _ctx[key] = h
    return c


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_of(t):
    import torch
    if t.dtype == torch.float32:
        return "f32"
    if t.dtype == torch.int32:
        return "i32"
    if t.dtype == torch.float64:
        return "f64"
    raise TypeError("cost must be float32, float64 or int32")


def _ld(t, n):
    if t.dim() != 2 or t.stride(1) != 1 or t.stride(0) < n:
        raise ValueError("expected a 2-D tensor with unit column stride and row stride >= n")
    return t.stride(0)


def make_problem(cost, out=None, rule="min", top=None, left=None, mode="full",
                 last_row=None, last_col=None, final_cell=None) -> Problem:
    """Fill a wf_problem from tensors (no allocation, no launch)."""
    m, n = cost.shape
    dt = _dtype_of(cost)
    p = Problem()
    p.m, p.n = m, n
    p.dtype, p.rule, p.mode, p.flags = DTYPES[dt], RULES[rule], MODES[mode], 0
    p.cost, p.ld_cost = cost.data_ptr(), _ld(cost, n)
    if out is not None:
        p.out, p.ld_out = out.data_ptr(), _ld(out, n)
    for name, t, ln in (("top", top, n + 1), ("left", left, m)):
        if t is not None:
            if t.dtype != cost.dtype or t.dim() != 1 or t.numel() != ln or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous vector of {ln} {cost.dtype}")
            setattr(p, name, t.data_ptr())
    for name, t in (("last_row", last_row), ("last_col", last_col), ("final_cell", final_cell)):
        if t is not None:
            setattr(p, name, t.data_ptr())
    return p


def solve(cost, out=None, rule: str = "min", top=None, left=None, mode: str = "full", stream=None,
          last_row=None, last_col=None, final_cell=None, waves_per_wg: int = 0, max_wgs: int = 0,
          rows_per_lane: int = 0):
    """Sweep one grid on the GPU (asynchronous on `stream`, default: current stream).

    mode="full": returns H (m x n), written into `out` if given.
    mode="edges": returns (last_row, last_col, final_cell) tensors.
    """
    import torch
    if not cost.is_cuda:
        raise ValueError("cost must be a device tensor")
    m, n = cost.shape
    if mode == "full" and out is None:
        out = torch.empty((m, n), dtype=cost.dtype, device=cost.device)
    if mode == "edges":
        if last_row is None:
            last_row = torch.empty(n, dtype=cost.dtype, device=cost.device)
        if last_col is None:
            last_col = torch.empty(m, dtype=cost.dtype, device=cost.device)
        if final_cell is None:
            final_cell = torch.empty(1, dtype=cost.dtype, device=cost.device)
    p = make_problem(cost, out, rule, top, left, mode, last_row, last_col, final_cell)
    if waves_per_wg or max_wgs or rows_per_lane:
        t = Tuning()
        t.waves_per_wg, t.max_wgs, t.rows_per_lane = waves_per_wg, max_wgs, rows_per_lane
        _check(load_library().wf_solve_tuned(context(cost.device.index), ctypes.byref(p), ctypes.byref(t),
                                             _stream_ptr(stream)))
    else:
        _check(load_library().wf_solve(context(cost.device.index), ctypes.byref(p), _stream_ptr(stream)))
    if mode == "full":
        return out
    return last_row, last_col, final_cell


def dtw(x, y, out=None, rule: str = "min", mode: str = "full", stream=None, last_row=None, last_col=None,
        final_cell=None, waves_per_wg: int = 0, max_wgs: int = 0, rows_per_lane: int = 0):
    """Dynamic time warping of two float32 device sequences x (m) and y (n): the sweep with
    cell inputs |x[i] - y[j]| computed on the device (WF_COST_ABSDIFF), so only the
    sequences are read.  mode="full" returns D (m x n); mode="edges" returns
    (last_row, last_col, final_cell).  Asynchronous on `stream`."""
    import torch
    if not (x.is_cuda and y.is_cuda) or x.dtype != torch.float32 or y.dtype != torch.float32:
        raise ValueError("x and y must be float32 device tensors")
    if x.dim() != 1 or y.dim() != 1 or not x.is_contiguous() or not y.is_contiguous():
        raise ValueError("x and y must be contiguous vectors")
    m, n = x.numel(), y.numel()
    if mode == "full" and out is None:
        out = torch.empty((m, n), dtype=torch.float32, device=x.device)
    if mode == "edges":
        last_row = torch.empty(n, dtype=torch.float32, device=x.device) if last_row is None else last_row
        last_col = torch.empty(m, dtype=torch.float32, device=x.device) if last_col is None else last_col
        final_cell = torch.empty(1, dtype=torch.float32, device=x.device) if final_cell is None else final_cell
    p = Problem()
    p.m, p.n = m, n
    p.dtype, p.rule, p.mode, p.flags = DTYPES["f32"], RULES[rule], MODES[mode], COST_ABSDIFF
    p.cost, p.ld_cost = None, n
    p.seq_x, p.seq_y = x.data_ptr(), y.data_ptr()
    if out is not None:
        p.out, p.ld_out = out.data_ptr(), _ld(out, n)
    for name, t in (("last_row", last_row), ("last_col", last_col), ("final_cell", final_cell)):
        if t is not None:
            setattr(p, name, t.data_ptr())
    lib = load_library()
    if waves_per_wg or max_wgs or rows_per_lane:
        t = Tuning()
        t.waves_per_wg, t.max_wgs, t.rows_per_lane = waves_per_wg, max_wgs, rows_per_lane
        _check(lib.wf_solve_tuned(context(x.device.index), ctypes.byref(p), ctypes.byref(t), _stream_ptr(stream)))
    else:
        _check(lib.wf_solve(context(x.device.index), ctypes.byref(p), _stream_ptr(stream)))
    if mode == "full":
        return out
    return last_row, last_col, final_cell


def traceback(H, rule: str = "min", top=None, left=None, stream=None):
    """wf_traceback: the path of predecessor choices through the computed grid H (device,
    float32 or int32; top/left: the boundary the sweep used).  Returns (path, exit): path
    is an (L, 2) int32 device tensor of visited cells, (m-1, n-1) first; exit the (2,)
    outside predecessor the walk ended on.  Waits for the stream to read L."""
    import torch
    m, n = H.shape
    p = make_problem(H, H, rule, top, left)
    buf = torch.empty((m + n, 2), dtype=torch.int32, device=H.device)
    length = torch.empty(1, dtype=torch.int64, device=H.device)
    _check(load_library().wf_traceback(context(H.device.index), ctypes.byref(p), buf.data_ptr(),
                                       length.data_ptr(), _stream_ptr(stream)))
    if stream is not None:
        stream.synchronize()
    L = int(length.item())
    return buf[:L], buf[L]


NOALLOC_SCRATCH_BYTES = 32 << 20  # WF_NOALLOC_SCRATCH_BYTES


def solve_noalloc(cost, out, rule: str = "min", top=None, left=None, mode: str = "full", stream=None,
                  last_row=None, last_col=None, final_cell=None):
    """wf_solve_noalloc: as solve(), but the library allocates nothing for the call (its
    workspace is a fixed device array), so every output must be given.  Calls that
    overlap on one device race on that array: keep them on one stream."""
    p = make_problem(cost, out, rule, top, left, mode, last_row, last_col, final_cell)
    _check(load_library().wf_solve_noalloc(context(cost.device.index), ctypes.byref(p), _stream_ptr(stream)))
    if mode == "full":
        return out
    return last_row, last_col, final_cell


class BatchPlan:
    """A batch of grids marshalled once for repeated launches.

    The wf_problem array is built when the plan is made; run() only calls
    wf_solve_batched with it, so a batch solved again and again (a serving or
    training loop over fixed buffers) pays no per-call argument marshalling.
    The plan keeps the tensors it was made from alive.
    """

    def __init__(self, costs, outs=None, rule: str = "min", mode: str = "full",
                 waves_per_wg: int = 0, max_wgs: int = 0, order: int = 0, use_graph: int = 1,
                 rows_per_lane: int = 0):
        import torch
        if outs is None:
            outs = []
            for c in costs:
                m, n = c.shape
                if mode == "full":
                    outs.append(torch.empty((m, n), dtype=c.dtype, device=c.device))
                else:
                    outs.append((torch.empty(n, dtype=c.dtype, device=c.device),
                                 torch.empty(m, dtype=c.dtype, device=c.device),
                                 torch.empty(1, dtype=c.dtype, device=c.device)))
        arr = (Problem * len(costs))()
        for i, c in enumerate(costs):
            if mode == "full":
                arr[i] = make_problem(c, outs[i], rule, mode=mode)
            else:
                lr, lc, fc = outs[i]
                arr[i] = make_problem(c, None, rule, mode=mode, last_row=lr, last_col=lc, final_cell=fc)
        t = Tuning()
        t.waves_per_wg, t.max_wgs, t.order, t.use_graph = waves_per_wg, max_wgs, order, use_graph
        t.rows_per_lane = rows_per_lane
        self.costs, self.outs = list(costs), outs
        self._arr, self._tuning = arr, t
        self._device = costs[0].device.index if costs else None

    def run(self, stream=None):
        """Launch the batch (asynchronous on `stream`); returns the outputs."""
        _check(load_library().wf_solve_batched(context(self._device), self._arr, len(self.costs),
                                               ctypes.byref(self._tuning), _stream_ptr(stream)))
        return self.outs


class EachPlan:
    """The per-grid path over a fixed list of grids: every grid swept by its own launch
    (wf_solve_each), grid i on streams[i % len(streams)].  Arguments are marshalled
    once, so run() measures the library's launches, not Python."""

    def __init__(self, costs, outs=None, rule: str = "min"):
        import torch
        if outs is None:
            outs = [torch.empty_like(c) for c in costs]
        arr = (Problem * len(costs))()
        for i, (c, o) in enumerate(zip(costs, outs)):
            arr[i] = make_problem(c, o, rule)
        self.costs, self.outs, self._arr = list(costs), outs, arr
        self._device = costs[0].device.index if costs else None

    def run(self, streams):
        sp = (_P * len(streams))(*[s.cuda_stream for s in streams])
        _check(load_library().wf_solve_each(context(self._device), self._arr, len(self.costs), sp, len(streams)))
        return self.outs


def set_watchdog(ms: int, device: int | None = None):
    """Device watchdog of later launches on this thread's context (milliseconds)."""
    _check(load_library().wf_set_watchdog(context(device), int(ms)))


def solve_batched(costs, outs=None, rule: str = "min", mode: str = "full", stream=None,
                  waves_per_wg: int = 0, max_wgs: int = 0, order: int = 0, use_graph: int = 1,
                  rows_per_lane: int = 0):
    """Sweep many independent grids in one persistent launch.  Returns the list of outputs
    (H per grid in full mode, (last_row, last_col, final_cell) in edges mode)."""
    return BatchPlan(costs, outs, rule, mode, waves_per_wg, max_wgs, order, use_graph, rows_per_lane).run(stream)


def check(device: int | None = None):
    """Wait for the context's work; raise WfError if a device watchdog fired."""
    _check(load_library().wf_check(context(device)))


class _DeviceArray:
    """A zero-copy view of server-owned device memory for torch.as_tensor."""

    def __init__(self, ptr: int, shape, typestr: str, strides=None):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (ptr, False),
                                         "version": 2, "strides": strides}


class Server:
    """Serving front end (wf_server_* in the C ABI).

    Requests are admitted against a device-memory budget as they arrive and
    batched into persistent launches on up to `max_inflight` streams while
    earlier launches still run.  Results stay in server memory until released.

        srv = Server(budget_bytes=8 << 30)
        t = srv.submit(cost)                  # device tensor (kept alive until done) or host array
        r = srv.poll(t)                       # None while pending
        H = r["out"].clone()                  # server memory: copy it, and let the copy finish, before release
        srv.release(t)
    """

    def __init__(self, budget_bytes: int = 0, max_inflight: int = 0, max_batch: int = 0, device: int | None = None,
                 copy_streams: int = 0, staging_bytes: int = 0, max_wait_skip_us: int = 0, ctx=None):
        lib = load_library()
        o = ServerOpts()
        o.hbm_budget_bytes, o.max_inflight, o.max_batch = budget_bytes, max_inflight, max_batch
        o.copy_streams, o.staging_bytes, o.max_wait_skip_us = copy_streams, staging_bytes, max_wait_skip_us
        self._h = _P()
        _check(lib.wf_server_create(context(device) if ctx is None else ctx, ctypes.byref(o), ctypes.byref(self._h)))
        self._keep = {}
        self._events = {}  # submitting stream -> the event its device inputs' readiness is recorded in
        self._done_buf = (ctypes.c_uint64 * 4096)()

    def _submit(self, r, keep):
        t = ctypes.c_uint64()
        _check(load_library().wf_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = keep
        return t.value

    def submit(self, cost, rule: str = "min", mode: str = "full") -> int:
        """Queue one grid; `cost` is a 2-D float32/int32 device tensor (the launch waits,
        on the device, for the work already queued on the current stream, which may
        still be writing it), a pinned CPU tensor (copied by DMA), or a C-contiguous host
        numpy array / CPU tensor (copied through staging).  Returns the ticket."""
        import numpy as np
        import torch
        r = Request()
        ev = None
        if isinstance(cost, torch.Tensor) and cost.is_cuda:
            m, n = cost.shape
            r.dtype = DTYPES[_dtype_of(cost)]
            r.input_kind, r.input, r.ld_input = INPUT_DEVICE, cost.data_ptr(), _ld(cost, n)
            # One event per submitting stream, recorded again at every submit: the server's
            # wait then covers at least the work queued before this submit.
            stream = torch.cuda.current_stream(cost.device)
            ev = self._events.get(stream.cuda_stream)
            if ev is None:
                ev = self._events[stream.cuda_stream] = torch.cuda.Event()
            ev.record(stream)
            r.ready_event = ev.cuda_event
        elif isinstance(cost, torch.Tensor) and cost.is_pinned():
            m, n = cost.shape
            r.dtype = DTYPES[_dtype_of(cost)]
            r.input_kind, r.input, r.ld_input = INPUT_HOST_PINNED, cost.data_ptr(), _ld(cost, n)
        else:
            a = np.ascontiguousarray(cost.numpy() if isinstance(cost, torch.Tensor) else cost)
            if a.dtype == np.float32:
                r.dtype = 0
            elif a.dtype == np.int32:
                r.dtype = 1
            else:
                raise TypeError("cost must be float32 or int32")
            m, n = a.shape
            cost = a
            r.input_kind, r.input, r.ld_input = INPUT_HOST, a.ctypes.data, n
        r.m, r.n, r.rule, r.mode = m, n, RULES[rule], MODES[mode]
        return self._submit(r, (cost, m, n, r.dtype, mode, ev))

    def submit_seeded(self, m: int, n: int, seed: int, dtype: str = "f32", rule: str = "min",
                      mode: str = "full") -> int:
        """Queue an m x n grid whose inputs the server generates on the device from `seed`
        (SplitMix64, as wfgen.cells(seed, m, n, dtype))."""
        r = Request()
        r.m, r.n, r.dtype, r.rule, r.mode = m, n, DTYPES[dtype], RULES[rule], MODES[mode]
        r.input_kind, r.seed = INPUT_SEED, seed & 0xFFFFFFFFFFFFFFFF
        return self._submit(r, (None, m, n, r.dtype, mode, None))

    def poll(self, ticket: int):
        """None while pending; else a dict with torch views of the results and timestamps."""
        import torch
        res = Result()
        st = load_library().wf_poll(self._h, ticket, ctypes.byref(res))
        if st == WF_PENDING:
            return None
        _check(st)
        _, m, n, dt, mode, _ = self._keep[ticket]
        ts = "<f4" if dt == 0 else "<i4"

        def view(ptr, shape, strides=None):
            if not ptr or 0 in shape:
                return None
            return torch.as_tensor(_DeviceArray(ptr, shape, ts, strides), device="cuda")

        return {"out": view(res.out, (m, n), (res.ld_out * 4, 4)) if mode == "full" else None,
                "last_row": view(res.last_row, (n,)), "last_col": view(res.last_col, (m,)),
                "final_cell": view(res.final_cell, (1,)),
                "t_submit": res.t_submit, "t_admit": res.t_admit, "t_launch": res.t_launch, "t_done": res.t_done}

    def poll_times(self, ticket: int):
        """None while pending; else (t_submit, t_admit, t_launch, t_done) on the server's
        monotonic clock (the clock of time.perf_counter on Linux)."""
        res = Result()
        st = load_library().wf_poll(self._h, ticket, ctypes.byref(res))
        if st == WF_PENDING:
            return None
        _check(st)
        return res.t_submit, res.t_admit, res.t_launch, res.t_done

    def done(self):
        """Tickets finished (done or failed) since the last call, oldest first."""
        out = []
        n = ctypes.c_int64()
        while True:
            _check(load_library().wf_server_done(self._h, self._done_buf, len(self._done_buf), ctypes.byref(n)))
            out.extend(self._done_buf[:n.value])
            if n.value < len(self._done_buf):
                return out

    def release(self, ticket: int):
        _check(load_library().wf_release(self._h, ticket))
        self._keep.pop(ticket, None)

    def memory(self):
        """(bytes held for requests now, peak)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(load_library().wf_server_memory(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def close(self):
        if self._h:
            _check(load_library().wf_server_destroy(self._h))
            self._h = _P()
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


# ------------------------------------------------------------ stream-count model
def stream_model_groups(samples, split_size):
    """Point counts of the three fits wf_stream_model_fit makes from `samples`
    ((size, streams, t_str, t_non_str, sum) tuples): distinct sizes, small-regime
    overhead samples, big-regime overhead samples.  A caller needs them to draw
    the shuffles it passes in."""
    sizes = []
    for s in samples:
        if s[0] not in sizes:
            sizes.append(s[0])
    small = sum(1 for s in samples if s[1] >= 2 and s[0] <= split_size)
    big = sum(1 for s in samples if s[1] >= 2 and s[0] > split_size)
    return len(sizes), small, big


def fit_stream_model(samples, split_size, perm_sum, perm_small, perm_big):
    """Fit the model of Sections 2.3-2.4 (Eqs. 4, 5, 7) to (size, streams, t_str,
    t_non_str, sum) samples with the given 3:1-split shuffles.  Returns
    (StreamModel, [FitReport x 3]) for the sum, small and big fits."""
    lib = load_library()
    arr = (StreamSample * len(samples))()
    for i, (size, s, t_str, t_non, sm) in enumerate(samples):
        arr[i] = StreamSample(float(size), int(s), 0, float(t_str), float(t_non), float(sm))

    def iarr(p):
        a = (ctypes.c_int64 * max(len(p), 1))()
        for i, v in enumerate(p):
            a[i] = int(v)
        return a

    model = StreamModel()
    rep = (FitReport * 3)()
    _check(lib.wf_stream_model_fit(arr, len(samples), float(split_size), iarr(perm_sum), iarr(perm_small),
                                   iarr(perm_big), ctypes.byref(model), rep))
    return model, list(rep)


def choose_streams(model, size, candidates=(1, 2, 4, 8, 16, 32)):
    """Section 3's choice: (best stream count, [gap per candidate])."""
    lib = load_library()
    c = (ctypes.c_int32 * len(candidates))(*candidates)
    g = (ctypes.c_double * len(candidates))()
    best = ctypes.c_int32()
    _check(lib.wf_stream_model_choose(ctypes.byref(model), float(size), c, len(candidates), ctypes.byref(best), g))
    return best.value, list(g)


def measure_step_ns(steps: int = 1 << 22, device: int | None = None) -> float:
    """Latency of one step of the walk's dependency chain (ns), measured on the device."""
    v = ctypes.c_double()
    _check(load_library().wf_measure_step_ns(context(device), steps, ctypes.byref(v)))
    return v.value
