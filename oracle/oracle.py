"""ctypes binding of the CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's cpu_baseline leg import this
module.  The product path never does.
"""
import ctypes
import os

import numpy as np

from . import build as _build

DT_F32 = 1
DT_F64 = 2
CHUNK_N = 1025
OK, ERR_ARG, ERR_SMALL, ERR_CORRUPT = 0, 1, 2, 3
# ablation variants of Sec. 5.4.2 (Fig. 12b)
VARIANTS = {"falcon": 0, "elf": 1, "sparse": 2, "dense": 3}

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        sz = ctypes.c_size_t
        vp = ctypes.c_void_p
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_bound.argtypes = [sz, ctypes.c_int]
        L.orc_bound.restype = sz
        L.orc_fl10_f64.argtypes = [ctypes.c_double]
        L.orc_fl10_f64.restype = ctypes.c_int
        L.orc_fl10_f32.argtypes = [ctypes.c_float]
        L.orc_fl10_f32.restype = ctypes.c_int
        L.orc_dpds_f64.argtypes = [ctypes.c_double, ip, ip, ip]
        L.orc_dpds_f32.argtypes = [ctypes.c_float, ip, ip, ip]
        L.orc_encode_chunk.argtypes = [vp, sz, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(sz)]
        L.orc_encode_chunk.restype = ctypes.c_int
        L.orc_decode_chunk.argtypes = [vp, sz, ctypes.c_int, ctypes.c_int, vp]
        L.orc_decode_chunk.restype = ctypes.c_int
        L.orc_chunk_info.argtypes = [vp, sz, ctypes.c_int, ctypes.c_int, ip, ip, ip,
                                     ctypes.POINTER(ctypes.c_uint64)]
        L.orc_chunk_info.restype = ctypes.c_int
        L.orc_compress.argtypes = [vp, sz, ctypes.c_int, vp, sz, ctypes.POINTER(sz)]
        L.orc_compress.restype = ctypes.c_int
        L.orc_decompress.argtypes = [vp, sz, vp, sz, ctypes.POINTER(sz)]
        L.orc_decompress.restype = ctypes.c_int
        L.orc_validate.argtypes = [vp, sz]
        L.orc_validate.restype = ctypes.c_int
        L.orc_stream_info.argtypes = [vp, sz, ctypes.POINTER(sz), ip]
        L.orc_stream_info.restype = ctypes.c_int
        L.orc_dpds_many.argtypes = [vp, sz, ctypes.c_int, vp, vp, vp]
        L.orc_dpds_many_v.argtypes = [vp, sz, ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.orc_bound_v.argtypes = [sz, ctypes.c_int, ctypes.c_int]
        L.orc_bound_v.restype = sz
        L.orc_compress_v.argtypes = [vp, sz, ctypes.c_int, ctypes.c_int, vp, sz, ctypes.POINTER(sz)]
        L.orc_compress_v.restype = ctypes.c_int
        L.orc_encode_chunk_v.argtypes = [vp, sz, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                         ctypes.POINTER(sz)]
        L.orc_encode_chunk_v.restype = ctypes.c_int
        L.orc_fl10_many.argtypes = [vp, sz, ctypes.c_int, vp]
        _lib = L
    return _lib


def _dt(arr):
    if arr.dtype == np.float64:
        return DT_F64
    if arr.dtype == np.float32:
        return DT_F32
    raise TypeError(f"unsupported dtype {arr.dtype}")


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def fl10(a, dtype=np.float64):
    if np.dtype(dtype) == np.float64:
        return lib().orc_fl10_f64(float(a))
    return lib().orc_fl10_f32(float(np.float32(a)))


def dpds(v, dtype=np.float64):
    """Alg. 2 on one value: returns (alpha, beta, exception)."""
    a, b, e = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    if np.dtype(dtype) == np.float64:
        lib().orc_dpds_f64(float(v), a, b, e)
    else:
        lib().orc_dpds_f32(float(np.float32(v)), a, b, e)
    return a.value, b.value, bool(e.value)


def dpds_many(x: np.ndarray, variant: str = "falcon"):
    """Alg. 2 over an array: returns (alpha, beta, exception) arrays.
    variant "elf" uses the trial-and-error stopping test of Sec. 1."""
    x = np.ascontiguousarray(x)
    n = x.size
    a = np.empty(n, np.int32); b = np.empty(n, np.int32); e = np.empty(n, np.int32)
    lib().orc_dpds_many_v(_ptr(x), n, _dt(x), VARIANTS[variant], _ptr(a), _ptr(b), _ptr(e))
    return a, b, e.astype(bool)


def fl10_many(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x)
    out = np.empty(x.size, np.int32)
    lib().orc_fl10_many(_ptr(x), x.size, _dt(x), _ptr(out))
    return out


def bound(n, dtype, variant: str = "falcon"):
    return lib().orc_bound_v(n, DT_F64 if np.dtype(dtype) == np.float64 else DT_F32, VARIANTS[variant])


def compress(x: np.ndarray, variant: str = "falcon") -> bytes:
    """The stream of x; variant names an ablation of Sec. 5.4.2."""
    x = np.ascontiguousarray(x)
    dt = _dt(x)
    v = VARIANTS[variant]
    cap = lib().orc_bound_v(x.size, dt, v)
    out = np.empty(cap, np.uint8)
    n = ctypes.c_size_t()
    st = lib().orc_compress_v(_ptr(x), x.size, dt, v, _ptr(out), cap, ctypes.byref(n))
    if st != OK:
        raise RuntimeError(f"oracle compress failed: {st}")
    return out[: n.value].tobytes()


def stream_info(stream: bytes):
    buf = np.frombuffer(stream, np.uint8)
    n = ctypes.c_size_t()
    dt = ctypes.c_int()
    st = lib().orc_stream_info(_ptr(buf), buf.size, ctypes.byref(n), ctypes.byref(dt))
    if st != OK:
        raise ValueError("corrupt stream")
    return n.value, (np.float64 if dt.value == DT_F64 else np.float32)


def decompress(stream: bytes) -> np.ndarray:
    buf = np.frombuffer(stream, np.uint8)
    n, dtype = stream_info(stream)
    out = np.empty(n, dtype)
    nout = ctypes.c_size_t()
    st = lib().orc_decompress(_ptr(buf), buf.size, _ptr(out), out.nbytes, ctypes.byref(nout))
    if st != OK:
        raise ValueError(f"oracle decompress failed: {st}")
    return out


def validate(stream: bytes) -> int:
    buf = np.frombuffer(stream, np.uint8)
    return lib().orc_validate(_ptr(buf), buf.size)


def encode_chunk(vals: np.ndarray, chunk_n: int = CHUNK_N, variant: str = "falcon") -> bytes:
    vals = np.ascontiguousarray(vals)
    dt = _dt(vals)
    out = np.empty(11 + 8 + 64 * ((chunk_n - 1) // 8 + (chunk_n - 1) // 64) + 64, np.uint8)
    n = ctypes.c_size_t()
    st = lib().orc_encode_chunk_v(_ptr(vals), vals.size, dt, chunk_n, VARIANTS[variant], _ptr(out),
                                  ctypes.byref(n))
    if st != OK:
        raise ValueError(f"oracle encode_chunk failed: {st}")
    return out[: n.value].tobytes()


def decode_chunk(payload: bytes, dtype, chunk_n: int = CHUNK_N) -> np.ndarray:
    buf = np.frombuffer(payload, np.uint8)
    out = np.empty(chunk_n, dtype)
    dt = DT_F64 if np.dtype(dtype) == np.float64 else DT_F32
    st = lib().orc_decode_chunk(_ptr(buf), buf.size, dt, chunk_n, _ptr(out))
    if st != OK:
        raise ValueError(f"oracle decode_chunk failed: {st}")
    return out


def chunk_info(vals: np.ndarray, chunk_n: int = CHUNK_N):
    """(A, B, w, dense_mask) of the chunk the oracle writes for vals."""
    vals = np.ascontiguousarray(vals)
    A, B, w = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    m = ctypes.c_uint64()
    st = lib().orc_chunk_info(_ptr(vals), vals.size, _dt(vals), chunk_n, A, B, w, ctypes.byref(m))
    if st != OK:
        raise ValueError("oracle chunk_info failed")
    return A.value, B.value, w.value, m.value
