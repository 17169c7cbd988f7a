"""ctypes binding of libfalcon.so: argument marshalling only.

Every step of compression and decompression runs in the library's HIP
kernels; nothing here touches the data.  If the library is missing the
import fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libfalcon.so")

FALCON_FLOAT32 = 1
FALCON_FLOAT64 = 2
_STATUS = {0: "ok", 1: "invalid argument", 2: "buffer too small", 3: "corrupt stream",
           4: "device error", 5: "out of memory"}
ERR_INVALID_ARG = 1
ERR_BUFFER_TOO_SMALL = 2
ERR_CORRUPT_STREAM = 3


class FalconError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {_STATUS.get(status, status)} ({status})")
        self.status = status


class Series(ctypes.Structure):
    """falcon_series of falcon.h."""
    _fields_ = [("d_in", ctypes.c_void_p), ("n", ctypes.c_size_t), ("in_len", ctypes.c_size_t),
                ("d_out", ctypes.c_void_p), ("out_cap", ctypes.c_size_t), ("dtype", ctypes.c_int),
                ("out_len", ctypes.c_size_t)]


class PlanInfo(ctypes.Structure):
    """falcon_plan_info of falcon.h."""
    _fields_ = [("split", ctypes.c_int), ("waves_per_group", ctypes.c_int), ("grid_percent", ctypes.c_int),
                ("candidates", ctypes.c_int), ("best_ms", ctypes.c_float), ("default_ms", ctypes.c_float),
                ("graph", ctypes.c_int), ("total_chunks", ctypes.c_uint64), ("form", ctypes.c_int),
                ("from_cache", ctypes.c_int)]


class Opts(ctypes.Structure):
    """falcon_opts of falcon.h."""
    _fields_ = [("flags", ctypes.c_uint), ("compress_form", ctypes.c_int)]


OPT_BLOCKING = 1
TIMED_CALLS = 64  # FALCON_TIMED_CALLS: timed calls whose stage times the context keeps
OPT_DEVICE_LENGTHS = 2
FORMS = {"two_pass": 0, "single_pass": 1}


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("pool", ctypes.c_void_p), ("lanes", ctypes.c_int),
                ("max_batch", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("d_in", ctypes.c_void_p), ("n", ctypes.c_size_t),
                ("in_len", ctypes.c_size_t), ("dtype", ctypes.c_int), ("tag", ctypes.c_uint64)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int), ("d_out", ctypes.c_void_p),
                ("out_len", ctypes.c_size_t), ("submit_us", ctypes.c_double), ("admit_us", ctypes.c_double),
                ("complete_us", ctypes.c_double), ("dev_start_us", ctypes.c_double),
                ("dev_end_us", ctypes.c_double), ("lane", ctypes.c_int)]


OP_COMPRESS = 0
OP_DECOMPRESS = 1
PLAN_TUNE = 1
PLAN_GRAPH = 2
PLAN_SINGLE_PASS = 4
SCHEDULERS = {"event": 0, "sync": 1, "prealloc": 2}
# ablation variants of compression (Sec. 5.4.2)
VARIANTS = {"falcon": 0, "elf": 1, "sparse": 2, "dense": 3}


def _load():
    if not os.path.exists(lib_path):
        raise ImportError(
            f"{lib_path} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(lib_path)
    vp, sz, i = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    L.falcon_create.argtypes = [i, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    L.falcon_create.restype = i
    L.falcon_sync.argtypes = [vp]
    L.falcon_sync.restype = i
    L.falcon_decompress_n.argtypes = [vp, vp, sz, sz, i, vp, sz, vp]
    L.falcon_decompress_n.restype = i
    L.falcon_destroy.argtypes = [vp]
    L.falcon_destroy.restype = None
    L.falcon_compress_bound.argtypes = [sz, i]
    L.falcon_compress_bound.restype = sz
    L.falcon_compress.argtypes = [vp, vp, sz, i, vp, sz, ctypes.POINTER(sz), vp]
    L.falcon_compress_bound_variant.argtypes = [sz, i, i]
    L.falcon_compress_bound_variant.restype = sz
    L.falcon_compress_variant.argtypes = [vp, vp, sz, i, i, vp, sz, ctypes.POINTER(sz), vp]
    L.falcon_compress_variant.restype = i
    L.falcon_compress.restype = i
    L.falcon_decompress.argtypes = [vp, vp, sz, vp, sz, ctypes.POINTER(sz), vp]
    L.falcon_decompress.restype = i
    L.falcon_stream_info.argtypes = [vp, sz, ctypes.POINTER(sz), ctypes.POINTER(i)]
    L.falcon_stream_info.restype = i
    L.falcon_last_kernel_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
    L.falcon_last_kernel_ms.restype = i
    L.falcon_last_stage_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
    L.falcon_last_stage_ms.restype = i
    L.falcon_call_stage_ms.argtypes = [vp, ctypes.c_uint, ctypes.POINTER(ctypes.c_float)]
    L.falcon_call_stage_ms.restype = i
    L.falcon_compress_host.argtypes = [vp, vp, sz, i, vp, sz, ctypes.POINTER(sz)]
    L.falcon_compress_host.restype = i
    L.falcon_decompress_host.argtypes = [vp, vp, sz, vp, sz, ctypes.POINTER(sz)]
    L.falcon_decompress_host.restype = i
    L.falcon_set_pipeline.argtypes = [vp, i, sz]
    L.falcon_set_pipeline.restype = i
    L.falcon_set_pipeline_scheduler.argtypes = [vp, i]
    L.falcon_set_pipeline_scheduler.restype = i
    ps = ctypes.POINTER(Series)
    L.falcon_compress_each.argtypes = [vp, ps, sz, vp]
    L.falcon_compress_each.restype = i
    L.falcon_decompress_each.argtypes = [vp, ps, sz, vp]
    L.falcon_decompress_each.restype = i
    L.falcon_compress_batch.argtypes = [vp, ps, sz, vp]
    L.falcon_compress_batch.restype = i
    L.falcon_decompress_batch.argtypes = [vp, ps, sz, vp]
    L.falcon_decompress_batch.restype = i
    L.falcon_plan_create.argtypes = [vp, i, ps, sz, ctypes.c_uint, ctypes.POINTER(vp)]
    L.falcon_plan_create.restype = i
    L.falcon_plan_run.argtypes = [vp, ps, vp]
    L.falcon_plan_run.restype = i
    L.falcon_plan_describe.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.falcon_plan_describe.restype = i
    L.falcon_plan_destroy.argtypes = [vp]
    L.falcon_plan_destroy.restype = None
    L.falcon_server_create.argtypes = [vp, ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    L.falcon_server_create.restype = i
    L.falcon_server_submit.argtypes = [vp, ctypes.POINTER(Request)]
    L.falcon_server_submit.restype = i
    L.falcon_server_poll.argtypes = [vp, ctypes.POINTER(Completion), sz, i]
    L.falcon_server_poll.restype = sz
    L.falcon_server_release.argtypes = [vp, vp]
    L.falcon_server_release.restype = i
    L.falcon_server_in_flight.argtypes = [vp]
    L.falcon_server_in_flight.restype = ctypes.c_uint64
    L.falcon_server_destroy.argtypes = [vp]
    L.falcon_server_destroy.restype = None
    L.falcon_status_str.argtypes = [i]
    L.falcon_status_str.restype = ctypes.c_char_p
    return L


_lib = None
_lock = threading.Lock()


def lib():
    global _lib
    with _lock:
        if _lib is None:
            _lib = _load()
    return _lib


def _dtype_code(dt: torch.dtype) -> int:
    if dt == torch.float64:
        return FALCON_FLOAT64
    if dt == torch.float32:
        return FALCON_FLOAT32
    raise TypeError(f"Falcon compresses float32/float64 tensors, got {dt}")


def compress_bound(n: int, dtype: torch.dtype) -> int:
    return lib().falcon_compress_bound(n, _dtype_code(dtype))


def _stream_handle(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Codec:
    """One library context on one GPU (a stream, pinned staging, scratch).

    blocking=True (the default here) makes every device call wait for its
    work and report its own errors, as the methods below expect; with
    blocking=False the *_async methods enqueue and sync() completes them.
    form selects how compression runs ("two_pass" or "single_pass")."""

    def __init__(self, device: int | torch.device = 0, blocking: bool = True, form: str = "two_pass",
                 device_lengths: bool = False):
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.device = dev
        self.blocking = blocking
        self.device_lengths = device_lengths
        self._ctx = ctypes.c_void_p()
        opts = Opts((OPT_BLOCKING if blocking else 0) | (OPT_DEVICE_LENGTHS if device_lengths else 0), FORMS[form])
        st = lib().falcon_create(dev.index or 0, ctypes.byref(opts), ctypes.byref(self._ctx))
        if st != 0:
            raise FalconError(st, "falcon_create")
        self._pending = []

    def close(self):
        if self._ctx:
            lib().falcon_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_kernel_ms(self) -> float:
        """Duration of the last kernel this codec launched (HIP events)."""
        ms = ctypes.c_float()
        st = lib().falcon_last_kernel_ms(self._ctx, ctypes.byref(ms))
        if st != 0:
            raise FalconError(st, "falcon_last_kernel_ms")
        return ms.value

    def last_stage_ms(self) -> list:
        """Stages of the last call: [size pass, scan, write pass] for
        compression, [0, scan, decoding kernel] for decompression."""
        ms = (ctypes.c_float * 3)()
        st = lib().falcon_last_stage_ms(self._ctx, ms)
        if st != 0:
            raise FalconError(st, "falcon_last_stage_ms")
        return [ms[0], ms[1], ms[2]]

    def call_stage_ms(self, back: int) -> list:
        """falcon_call_stage_ms: the stages of the timed call made `back`
        timed calls before the last (0 = the last), for callers that enqueue
        many asynchronous calls and synchronise once."""
        ms = (ctypes.c_float * 3)()
        st = lib().falcon_call_stage_ms(self._ctx, back, ms)
        if st != 0:
            raise FalconError(st, "falcon_call_stage_ms")
        return [ms[0], ms[1], ms[2]]

    def sync(self):
        """falcon_sync: waits for the asynchronous calls made since the last
        sync; raises FalconError for an error the device found among them."""
        st = lib().falcon_sync(self._ctx)
        self._pending = []
        if st != 0:
            raise FalconError(st, "falcon_sync")

    def compress_async(self, x: torch.Tensor, out: torch.Tensor, out_len=None, stream=None):
        """Enqueues falcon_compress of x into out (a uint8 device tensor of at
        least compress_bound bytes).  Returns the length holder: a
        ctypes.c_size_t filled at sync(), or, on a device_lengths codec, the
        int64 device tensor out_len (one element) that the kernels fill."""
        code = _dtype_code(x.dtype)
        n = x.numel()
        if self.device_lengths:
            holder = out_len
            ptr = ctypes.cast(ctypes.c_void_p(out_len.data_ptr()), ctypes.POINTER(ctypes.c_size_t))
        else:
            holder = ctypes.c_size_t()
            ptr = ctypes.byref(holder)
            self._pending.append(holder)
        h = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream_handle(x.device)
        st = lib().falcon_compress(self._ctx, ctypes.c_void_p(x.data_ptr() if n else 0), n, code,
                                   ctypes.c_void_p(out.data_ptr()), out.numel(), ptr, h)
        if st != 0:
            raise FalconError(st, "falcon_compress")
        return holder

    def decompress_n_async(self, stream_bytes: torch.Tensor, n: int, dtype: torch.dtype, out: torch.Tensor,
                           stream=None):
        """Enqueues falcon_decompress_n: the stream in stream_bytes holds n
        values of dtype; they go to out.  No host access to the stream."""
        h = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream_handle(out.device)
        st = lib().falcon_decompress_n(self._ctx, ctypes.c_void_p(stream_bytes.data_ptr()), stream_bytes.numel(),
                                       n, _dtype_code(dtype), ctypes.c_void_p(out.data_ptr() if out.numel() else 0),
                                       out.numel() * out.element_size(), h)
        if st != 0:
            raise FalconError(st, "falcon_decompress_n")

    def decompress_n(self, stream_bytes: torch.Tensor, n: int, dtype: torch.dtype,
                     out: torch.Tensor | None = None) -> torch.Tensor:
        """falcon_decompress_n (the count and dtype from the caller)."""
        if out is None:
            out = torch.empty(n, dtype=dtype, device=stream_bytes.device)
        self.decompress_n_async(stream_bytes, n, dtype, out)
        if not self.blocking:
            self.sync()
        return out[:n]

    def compress(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Compresses a contiguous float32/float64 device tensor; returns the
        stream as a uint8 device tensor (a view of `out` when given)."""
        if self.device_lengths:
            raise ValueError("compress() needs a codec with host lengths")
        if not x.is_cuda or not x.is_contiguous():
            raise ValueError("compress needs a contiguous device tensor")
        code = _dtype_code(x.dtype)
        n = x.numel()
        cap = lib().falcon_compress_bound(n, code)
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=x.device)
        olen = ctypes.c_size_t()
        st = lib().falcon_compress(self._ctx, ctypes.c_void_p(x.data_ptr() if n else 0), n, code,
                                   ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.byref(olen),
                                   _stream_handle(x.device))
        if st != 0:
            raise FalconError(st, "falcon_compress")
        if not self.blocking:
            self.sync()
        return out[: olen.value]

    def compress_variant(self, x: torch.Tensor, variant: str, out: torch.Tensor | None = None) -> torch.Tensor:
        """compress() under an ablation variant: "falcon", "elf" (Elf's
        decimal places), "sparse" (every row sparse) or "dense"."""
        if not x.is_cuda or not x.is_contiguous():
            raise ValueError("compress needs a contiguous device tensor")
        code = _dtype_code(x.dtype)
        v = VARIANTS[variant]
        n = x.numel()
        cap = lib().falcon_compress_bound_variant(n, code, v)
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=x.device)
        olen = ctypes.c_size_t()
        st = lib().falcon_compress_variant(self._ctx, ctypes.c_void_p(x.data_ptr() if n else 0), n, code, v,
                                           ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.byref(olen),
                                           _stream_handle(x.device))
        if st != 0:
            raise FalconError(st, "falcon_compress_variant")
        if not self.blocking:
            self.sync()
        return out[: olen.value]

    def decompress(self, stream: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Decompresses a uint8 device tensor holding one stream."""
        if not stream.is_cuda or stream.dtype != torch.uint8 or not stream.is_contiguous():
            raise ValueError("decompress needs a contiguous uint8 device tensor")
        hdr = stream[:32].cpu().numpy() if stream.numel() >= 32 else None
        if hdr is None:
            raise FalconError(ERR_CORRUPT_STREAM, "falcon_decompress")
        n = ctypes.c_size_t()
        code = ctypes.c_int()
        st = lib().falcon_stream_info(ctypes.c_void_p(hdr.ctypes.data), 32, ctypes.byref(n), ctypes.byref(code))
        if st != 0:
            raise FalconError(st, "falcon_stream_info")
        dt = torch.float64 if code.value == FALCON_FLOAT64 else torch.float32
        if out is None:
            out = torch.empty(n.value, dtype=dt, device=stream.device)
        nout = ctypes.c_size_t()
        st = lib().falcon_decompress(self._ctx, ctypes.c_void_p(stream.data_ptr()), stream.numel(),
                                     ctypes.c_void_p(out.data_ptr() if out.numel() else 0),
                                     out.numel() * out.element_size(), ctypes.byref(nout),
                                     _stream_handle(stream.device))
        if st != 0:
            raise FalconError(st, "falcon_decompress")
        if not self.blocking:
            self.sync()
        return out[: nout.value]

    # -- host -> host through the stream pipeline ---------------------------
    def set_pipeline(self, n_streams: int = 4, batch_chunks: int = 2048):
        """Pipeline geometry: N_s streams, batch_chunks chunks per batch."""
        st = lib().falcon_set_pipeline(self._ctx, n_streams, batch_chunks)
        if st != 0:
            raise FalconError(st, "falcon_set_pipeline")

    def set_scheduler(self, kind: str = "event"):
        """Compression scheduler of the pipeline: "event" (Alg. 1),
        "sync" (Sync-Based) or "prealloc" (Pre-Allocation)."""
        code = SCHEDULERS[kind]
        st = lib().falcon_set_pipeline_scheduler(self._ctx, code)
        if st != 0:
            raise FalconError(st, "falcon_set_pipeline_scheduler")

    def compress_host(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Compresses a contiguous float32/float64 host tensor through the
        pipeline; returns the stream as a uint8 host tensor (a view of `out`
        when given; pinned when x is pinned)."""
        if x.is_cuda or not x.is_contiguous():
            raise ValueError("compress_host needs a contiguous host tensor")
        code = _dtype_code(x.dtype)
        n = x.numel()
        cap = lib().falcon_compress_bound(n, code)
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, pin_memory=x.is_pinned())
        olen = ctypes.c_size_t()
        st = lib().falcon_compress_host(self._ctx, ctypes.c_void_p(x.data_ptr() if n else 0), n, code,
                                        ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.byref(olen))
        if st != 0:
            raise FalconError(st, "falcon_compress_host")
        return out[: olen.value]

    def decompress_host(self, stream: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Decompresses a uint8 host tensor holding one stream through the
        pipeline; returns a host tensor of the stream's dtype."""
        if stream.is_cuda or stream.dtype != torch.uint8 or not stream.is_contiguous():
            raise ValueError("decompress_host needs a contiguous uint8 host tensor")
        n = ctypes.c_size_t()
        code = ctypes.c_int()
        st = lib().falcon_stream_info(ctypes.c_void_p(stream.data_ptr()), stream.numel(), ctypes.byref(n),
                                      ctypes.byref(code))
        if st != 0:
            raise FalconError(st, "falcon_stream_info")
        dt = torch.float64 if code.value == FALCON_FLOAT64 else torch.float32
        if out is None:
            out = torch.empty(n.value, dtype=dt, pin_memory=stream.is_pinned())
        nout = ctypes.c_size_t()
        st = lib().falcon_decompress_host(self._ctx, ctypes.c_void_p(stream.data_ptr()), stream.numel(),
                                          ctypes.c_void_p(out.data_ptr() if out.numel() else 0),
                                          out.numel() * out.element_size(), ctypes.byref(nout))
        if st != 0:
            raise FalconError(st, "falcon_decompress_host")
        return out[: nout.value]

    # -- many series in one launch ------------------------------------------
    def _compress_descs(self, xs, outs):
        descs = (Series * len(xs))()
        views = []
        for i, x in enumerate(xs):
            if not x.is_cuda or not x.is_contiguous():
                raise ValueError("batch compression needs contiguous device tensors")
            code = _dtype_code(x.dtype)
            cap = lib().falcon_compress_bound(x.numel(), code)
            o = outs[i] if outs is not None else torch.empty(cap, dtype=torch.uint8, device=x.device)
            descs[i] = Series(x.data_ptr() if x.numel() else None, x.numel(), 0, o.data_ptr(), o.numel(), code, 0)
            views.append(o)
        return descs, views

    def _decompress_descs(self, streams, counts, dtypes, outs):
        descs = (Series * len(streams))()
        views = []
        for i, s_ in enumerate(streams):
            if not s_.is_cuda or s_.dtype != torch.uint8 or not s_.is_contiguous():
                raise ValueError("batch decompression needs contiguous uint8 device tensors")
            code = _dtype_code(dtypes[i])
            o = outs[i] if outs is not None else torch.empty(counts[i], dtype=dtypes[i], device=s_.device)
            descs[i] = Series(s_.data_ptr(), counts[i], s_.numel(), o.data_ptr() if o.numel() else None,
                              o.numel() * o.element_size(), code, 0)
            views.append(o)
        return descs, views

    def compress_each(self, xs, outs=None):
        """The one-series-per-launch loop (falcon_compress_each): one
        asynchronous compression per tensor, one wait; returns the streams."""
        descs, views = self._compress_descs(xs, outs)
        st = lib().falcon_compress_each(self._ctx, descs, len(xs), _stream_handle(self.device))
        if st != 0:
            raise FalconError(st, "falcon_compress_each")
        return [v[: descs[i].out_len] for i, v in enumerate(views)]

    def decompress_each(self, streams, counts, dtypes, outs=None):
        """falcon_decompress_each: one asynchronous falcon_decompress_n per
        stream, one wait."""
        descs, views = self._decompress_descs(streams, counts, dtypes, outs)
        st = lib().falcon_decompress_each(self._ctx, descs, len(streams), _stream_handle(self.device))
        if st != 0:
            raise FalconError(st, "falcon_decompress_each")
        return views

    def compress_batch(self, xs, outs=None):
        """Compresses a list of float32/float64 device tensors in one launch
        sequence; returns the streams (views of `outs` when given)."""
        descs, views = self._compress_descs(xs, outs)
        st = lib().falcon_compress_batch(self._ctx, descs, len(xs), _stream_handle(self.device))
        if st != 0:
            raise FalconError(st, "falcon_compress_batch")
        return [v[: descs[i].out_len] for i, v in enumerate(views)]

    def decompress_batch(self, streams, counts, dtypes, outs=None):
        """Decompresses a list of streams (uint8 device tensors) holding
        counts[i] values of dtypes[i] each, in one launch sequence."""
        descs, views = self._decompress_descs(streams, counts, dtypes, outs)
        st = lib().falcon_decompress_batch(self._ctx, descs, len(streams), _stream_handle(self.device))
        if st != 0:
            raise FalconError(st, "falcon_decompress_batch")
        return views

    def plan_compress(self, xs, outs=None, tune=True, graph=True, single_pass=False):
        descs, views = self._compress_descs(xs, outs)
        return Plan(self, OP_COMPRESS, descs, views, tune, graph, single_pass)

    def plan_decompress(self, streams, counts, dtypes, outs=None, tune=True, graph=True):
        descs, views = self._decompress_descs(streams, counts, dtypes, outs)
        return Plan(self, OP_DECOMPRESS, descs, views, tune, graph)


class Plan:
    """A reusable batch launch (falcon_plan): fixed series buffers, tuned
    geometry, optionally replayed as a HIP graph."""

    def __init__(self, codec: Codec, op: int, descs, views, tune: bool, graph: bool, single_pass: bool = False):
        self.codec, self.op, self.descs, self.views = codec, op, descs, views
        self._p = ctypes.c_void_p()
        flags = (PLAN_TUNE if tune else 0) | (PLAN_GRAPH if graph else 0) | (PLAN_SINGLE_PASS if single_pass else 0)
        st = lib().falcon_plan_create(codec._ctx, op, descs, len(descs), flags, ctypes.byref(self._p))
        if st != 0:
            raise FalconError(st, "falcon_plan_create")

    def run(self, stream=None, fetch: bool = True):
        """Runs the plan; returns the outputs (streams trimmed to length), or
        None with fetch=False (no per-series lengths are read back into
        Python, which for thousands of series costs more than the launch)."""
        h = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        st = lib().falcon_plan_run(self._p, self.descs if fetch else None, h)
        if st != 0:
            raise FalconError(st, "falcon_plan_run")
        if not fetch:
            return None
        if self.op == OP_COMPRESS:
            return [v[: self.descs[i].out_len] for i, v in enumerate(self.views)]
        return self.views

    def info(self) -> dict:
        pi = PlanInfo()
        st = lib().falcon_plan_describe(self._p, ctypes.byref(pi))
        if st != 0:
            raise FalconError(st, "falcon_plan_describe")
        return {f: getattr(pi, f) for f, _ in PlanInfo._fields_}

    def close(self):
        if self._p:
            lib().falcon_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The request loop (falcon_server) with its output pool in a torch
    device tensor, so that completions can be viewed as tensors."""

    def __init__(self, codec: Codec, hbm_budget: int = 1 << 30, lanes: int = 4, max_batch: int = 256):
        self.codec = codec
        self.pool = torch.empty(hbm_budget, dtype=torch.uint8, device=codec.device)
        opts = ServerOpts(hbm_budget, self.pool.data_ptr(), lanes, max_batch)
        self._s = ctypes.c_void_p()
        st = lib().falcon_server_create(codec._ctx, ctypes.byref(opts), ctypes.byref(self._s))
        if st != 0:
            raise FalconError(st, "falcon_server_create")
        self._buf = (Completion * 1024)()

    def submit_compress(self, x: torch.Tensor, tag: int):
        r = Request(OP_COMPRESS, x.data_ptr() if x.numel() else None, x.numel(), 0, _dtype_code(x.dtype), tag)
        st = lib().falcon_server_submit(self._s, ctypes.byref(r))
        if st != 0:
            raise FalconError(st, "falcon_server_submit")

    def submit_decompress(self, stream: torch.Tensor, n: int, dtype: torch.dtype, tag: int):
        r = Request(OP_DECOMPRESS, stream.data_ptr(), n, stream.numel(), _dtype_code(dtype), tag)
        st = lib().falcon_server_submit(self._s, ctypes.byref(r))
        if st != 0:
            raise FalconError(st, "falcon_server_submit")

    def poll(self, wait_ms: int = 0):
        """Completions as dicts (tag, status, offset into the pool, out_len,
        submit/admit/complete times in microseconds)."""
        k = lib().falcon_server_poll(self._s, self._buf, len(self._buf), wait_ms)
        base = self.pool.data_ptr()
        out = []
        for i in range(k):
            c = self._buf[i]
            out.append({"tag": c.tag, "status": c.status, "d_out": c.d_out,
                        "offset": (c.d_out - base) if c.d_out else None, "out_len": c.out_len,
                        "submit_us": c.submit_us, "admit_us": c.admit_us, "complete_us": c.complete_us,
                        "dev_start_us": c.dev_start_us, "dev_end_us": c.dev_end_us, "lane": c.lane})
        return out

    def view(self, comp: dict, dtype: torch.dtype = torch.uint8) -> torch.Tensor:
        """The completion's output as a tensor (a view of the pool)."""
        nbytes = comp["out_len"] * (torch.empty(0, dtype=dtype).element_size() if dtype != torch.uint8 else 1)
        return self.pool[comp["offset"]: comp["offset"] + nbytes].view(dtype)

    def release(self, comp: dict):
        if comp["d_out"]:
            st = lib().falcon_server_release(self._s, ctypes.c_void_p(comp["d_out"]))
            if st != 0:
                raise FalconError(st, "falcon_server_release")

    def in_flight(self) -> int:
        return lib().falcon_server_in_flight(self._s)

    def close(self):
        if self._s:
            lib().falcon_server_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default: dict = {}


def _codec_for(device: torch.device) -> Codec:
    key = device.index or 0
    if key not in _default:
        _default[key] = Codec(key)
    return _default[key]


def compress(x: torch.Tensor) -> torch.Tensor:
    return _codec_for(x.device).compress(x)


def decompress(stream: torch.Tensor) -> torch.Tensor:
    return _codec_for(stream.device).decompress(stream)
