"""CPU oracle of fixed-PSNR SZ-style compression (arXiv:1805.07384).

TEST INFRASTRUCTURE ONLY.  This package wraps ``fpsz_oracle.c``, a plain,
slow, single-threaded C implementation of the method (value range, Eq. 7
error bound, uniform prequantization, Lorenzo prediction, Huffman coding,
decompression and the Eq. 4 PSNR).  It shares no code with the GPU library.
Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import it; the product path never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fpsz_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_fpsz.so")

NSYM = 1036
LMAX = 18
CHUNK = 128
HDR_BYTES = 256

OK, E_INVALID_ARG, E_NONFINITE, E_RANGE, E_CORRUPT, E_CAPACITY, E_NOMEM = range(7)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Trace(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_void_p),
        ("delta", ctypes.c_void_p),
        ("code16", ctypes.c_void_p),
        ("hist", ctypes.c_void_p),
        ("code_len", ctypes.c_void_p),
        ("code", ctypes.c_void_p),
        ("scalars", ctypes.c_double * 8),
        ("minmax", ctypes.c_double * 2),
        ("counts", ctypes.c_uint64 * 6),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.or_eb_rel.restype = ctypes.c_double
        L.or_eb_rel.argtypes = [ctypes.c_double]
        L.or_symbol.restype = ctypes.c_int
        L.or_symbol.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_uint32)]
        L.or_unsymbol.restype = ctypes.c_int32
        L.or_unsymbol.argtypes = [ctypes.c_int, ctypes.c_uint32]
        L.or_huffman_unlimited.restype = ctypes.c_int
        L.or_huffman_unlimited.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
        L.or_code_lengths.restype = None
        L.or_code_lengths.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
        L.or_code_lengths_limited.restype = None
        L.or_code_lengths_limited.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_void_p]
        L.or_canonical_codes.restype = None
        L.or_canonical_codes.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
        L.or_checksum.restype = ctypes.c_uint64
        L.or_checksum.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.or_compress.restype = ctypes.c_int
        L.or_compress.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_uint64), ctypes.c_double, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_uint64),
                                  ctypes.POINTER(_Trace)]
        L.or_decompress.restype = ctypes.c_int
        L.or_decompress.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                    ctypes.c_uint64]
        L.or_stats.restype = ctypes.c_int
        L.or_stats.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64,
                               ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_uint64)]
        L.or_compress_scaled.restype = ctypes.c_int
        L.or_compress_scaled.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.c_double,
                                         ctypes.c_int, ctypes.c_double,
                                         ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_Trace)]
        L.or_compress_closed_loop.restype = ctypes.c_int
        L.or_compress_closed_loop.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_uint64), ctypes.c_double,
                                              ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                              ctypes.POINTER(ctypes.c_uint64),
                                              ctypes.POINTER(_Trace),
                                              ctypes.POINTER(ctypes.c_double)]
        L.or_compress_inloop.restype = ctypes.c_int
        L.or_compress_inloop.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.c_double,
                                         ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_Trace)]
        L.or_compress_xform.restype = ctypes.c_int
        L.or_compress_xform.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_uint64), ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_Trace)]
        L.or_quant_sse.restype = ctypes.c_int
        L.or_quant_sse.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.or_closed_loop_scale.restype = ctypes.c_double
        L.or_closed_loop_scale.argtypes = [ctypes.c_double, ctypes.c_uint64, ctypes.c_double,
                                           ctypes.c_double]
        L.or_stage_times.restype = None
        L.or_stage_times.argtypes = [ctypes.c_void_p]
        L.or_free.restype = None
        L.or_free.argtypes = [ctypes.c_void_p]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s failed with status %d" % (what, status))
        self.status = status


def _dtype_code(a: np.ndarray) -> int:
    if a.dtype == np.float32:
        return 0
    if a.dtype == np.float64:
        return 1
    raise TypeError("oracle takes float32 or float64 fields")


def eb_rel(psnr: float) -> float:
    """Eq. 7: eb_rel = sqrt(3) * 10^(-PSNR/20)."""
    return lib().or_eb_rel(float(psnr))


def symbol(d: int):
    """Residual -> (symbol, n_extra_bits, extra_bits)."""
    ne = ctypes.c_int(0)
    ev = ctypes.c_uint32(0)
    s = lib().or_symbol(int(d), ctypes.byref(ne), ctypes.byref(ev))
    return s, ne.value, ev.value


def unsymbol(s: int, extra: int) -> int:
    return lib().or_unsymbol(int(s), int(extra))


def huffman_unlimited(weights) -> np.ndarray:
    """Textbook Huffman code lengths (no length limit)."""
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.uint64))
    out = np.zeros(len(w), dtype=np.uint8)
    lib().or_huffman_unlimited(w.ctypes.data, len(w), out.ctypes.data)
    return out


def code_lengths(hist) -> np.ndarray:
    """Format code lengths: Huffman, limited to 18 bits by rebalancing the
    number of codes per length."""
    h = np.ascontiguousarray(np.asarray(hist, dtype=np.uint32))
    out = np.zeros(len(h), dtype=np.uint8)
    lib().or_code_lengths(h.ctypes.data, len(h), out.ctypes.data)
    return out


def code_lengths_limited(hist, lmax: int) -> np.ndarray:
    """The same length-limit rule with the limit as a parameter (for tests)."""
    h = np.ascontiguousarray(np.asarray(hist, dtype=np.uint32))
    out = np.zeros(len(h), dtype=np.uint8)
    lib().or_code_lengths_limited(h.ctypes.data, len(h), int(lmax), out.ctypes.data)
    return out


def canonical_codes(lengths) -> np.ndarray:
    ln = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint8))
    out = np.zeros(len(ln), dtype=np.uint32)
    lib().or_canonical_codes(ln.ctypes.data, len(ln), out.ctypes.data)
    return out


def checksum(blob: bytes) -> int:
    b = np.frombuffer(bytes(blob), dtype=np.uint8)
    return int(lib().or_checksum(b.ctypes.data, len(b)))


def compress(x: np.ndarray, psnr: float, domain: int = 0, trace: bool = False):
    """Compress a C-ordered 1D/2D/3D float32/float64 field.

    Returns ``(blob: bytes, trace: dict | None)``.  ``domain`` 0 = GLOBAL
    Lorenzo (zero outside the field), 1 = TILE (zero outside each tile).
    """
    return _compress(x, psnr, domain, trace, mode=0)


def compress_scaled(x: np.ndarray, psnr: float, scale: float, domain: int = 0,
                    trace: bool = False):
    """Compression with eb_rel of Eq. 7 multiplied by ``scale``, recorded in
    the blob (the second pass of the closed loop at a given factor)."""
    return _compress(x, psnr, domain, trace, mode=1, scale=scale)


def compress_closed_loop(x: np.ndarray, psnr: float, domain: int = 0, trace: bool = False):
    """Closed-loop compression: the quantizer's MSE at the Eq. 7 bound gives
    one secant step eb' = eb sqrt(MSE_target / MSE_1).  Returns ``(blob,
    trace, scale)``."""
    return _compress(x, psnr, domain, trace, mode=2)


def compress_inloop(x: np.ndarray, psnr: float, trace: bool = False):
    """SZ 1.4-style in-loop compression (tile domain): each point is predicted
    from the reconstructed values of its preceding neighbours in its tile and
    the prediction error quantized; points whose code leaves the radius or
    whose reconstruction misses the bound are stored exactly."""
    return _compress(x, psnr, 1, trace, mode=3)


def compress_xform(x: np.ndarray, psnr: float, trace: bool = False):
    """Orthogonal-transform compression: 4^ndim blocks, orthonormal
    Walsh-Hadamard transform, coefficients quantized with bin 2 eb (Eq. 7),
    DC bins coded as differences within a tile.  Dimensions must be multiples
    of 4.  The trace's "q" holds the codes in stream order."""
    return _compress(x, psnr, 1, trace, mode=4)


def quant_sse(x: np.ndarray, psnr: float):
    """(SSE of the quantizer output at the Eq. 7 bound, patches exact; vr)."""
    x = np.ascontiguousarray(x)
    sse, vr = ctypes.c_double(), ctypes.c_double()
    st = lib().or_quant_sse(x.ctypes.data, _dtype_code(x), x.size, float(psnr), ctypes.byref(sse),
                            ctypes.byref(vr))
    if st != OK:
        raise OracleError(st, "or_quant_sse")
    return sse.value, vr.value


def closed_loop_scale(sse: float, n: int, vr: float, psnr: float) -> float:
    return float(lib().or_closed_loop_scale(float(sse), int(n), float(vr), float(psnr)))


def _compress(x, psnr, domain, trace, mode, scale=1.0):
    x = np.ascontiguousarray(x)
    dt = _dtype_code(x)
    dl = [int(d) for d in x.shape] + [1] * max(0, 3 - x.ndim)
    dims = (ctypes.c_uint64 * len(dl))(*dl)
    n = x.size
    tr = _Trace()
    keep = {}
    if trace:
        keep["q"] = np.zeros(n, dtype=np.int32)
        keep["delta"] = np.zeros(n, dtype=np.int32)
        keep["code16"] = np.zeros(n, dtype=np.int16)
        keep["hist"] = np.zeros(NSYM, dtype=np.uint32)
        keep["code_len"] = np.zeros(NSYM, dtype=np.uint8)
        keep["code"] = np.zeros(NSYM, dtype=np.uint32)
        for k, v in keep.items():
            setattr(tr, k, v.ctypes.data)
    out = ctypes.c_void_p()
    nb = ctypes.c_uint64(0)
    sc = ctypes.c_double(1.0)
    if mode == 0:
        st = lib().or_compress(x.ctypes.data, dt, x.ndim, dims, float(psnr), int(domain),
                               ctypes.byref(out), ctypes.byref(nb), ctypes.byref(tr))
    elif mode == 1:
        st = lib().or_compress_scaled(x.ctypes.data, dt, x.ndim, dims, float(psnr), int(domain),
                                      float(scale), ctypes.byref(out), ctypes.byref(nb),
                                      ctypes.byref(tr))
    elif mode == 4:
        st = lib().or_compress_xform(x.ctypes.data, dt, x.ndim, dims, float(psnr),
                                     ctypes.byref(out), ctypes.byref(nb), ctypes.byref(tr))
    elif mode == 3:
        st = lib().or_compress_inloop(x.ctypes.data, dt, x.ndim, dims, float(psnr),
                                      ctypes.byref(out), ctypes.byref(nb), ctypes.byref(tr))
    else:
        st = lib().or_compress_closed_loop(x.ctypes.data, dt, x.ndim, dims, float(psnr),
                                           int(domain), ctypes.byref(out), ctypes.byref(nb),
                                           ctypes.byref(tr), ctypes.byref(sc))
    if st != OK:
        raise OracleError(st, "or_compress")
    blob = ctypes.string_at(out.value, nb.value)
    lib().or_free(out)
    if not trace:
        return (blob, None, sc.value) if mode == 2 else (blob, None)
    t = dict(keep)
    t["q"] = t["q"].reshape(x.shape)
    t["delta"] = t["delta"].reshape(x.shape)
    names = ["vr", "eb_rel", "eb", "e2", "r", "e2_f", "r_f", "maxabs"]
    for i, nm in enumerate(names):
        t[nm] = tr.scalars[i]
    t["min"], t["max"] = tr.minmax[0], tr.minmax[1]
    cn = ["n_tiles", "n_chunks", "n_words", "n_exc", "n_outliers", "n_patches"]
    for i, nm in enumerate(cn):
        t[nm] = int(tr.counts[i])
    return (blob, t, sc.value) if mode == 2 else (blob, t)


def header(blob: bytes) -> dict:
    """Parse the fixed 256-byte header (for tests)."""
    b = bytes(blob)
    u64 = lambda o: int(np.frombuffer(b, np.uint64, 1, o)[0])
    f64 = lambda o: float(np.frombuffer(b, np.float64, 1, o)[0])
    ndim = b[9]
    return {
        "magic": int(np.frombuffer(b, np.uint32, 1, 0)[0]),
        "version": int(np.frombuffer(b, np.uint16, 1, 4)[0]),
        "flags": int(np.frombuffer(b, np.uint16, 1, 6)[0]),
        "dtype": b[8], "ndim": ndim,
        "dims": [u64(16 + 8 * i) for i in range(ndim)],
        "psnr": f64(56), "eb_rel": f64(64), "vr": f64(72), "eb": f64(80),
        "e2": f64(88), "r": f64(96), "min": f64(120), "max": f64(128), "n": u64(136),
        "n_tiles": u64(144), "n_chunks": u64(152), "n_words": u64(160), "n_exc": u64(168),
        "n_outliers": u64(176), "n_patches": u64(184), "bytes": u64(192), "checksum": u64(200),
        "scale": f64(216),
    }


def decompress(blob: bytes) -> np.ndarray:
    if len(blob) < HDR_BYTES:
        raise OracleError(E_CORRUPT, "or_decompress")
    h = header(blob)
    # the output is sized from the header: refuse a header that fails the
    # checksum before allocating from it
    cs = checksum(bytes(blob[:200]) + b"\0" * 8 + bytes(blob[208:]))
    if h["checksum"] != cs or h["ndim"] not in (1, 2, 3) or h["dtype"] not in (0, 1):
        raise OracleError(E_CORRUPT, "or_decompress")
    dt = np.float32 if h["dtype"] == 0 else np.float64
    out = np.zeros(h["dims"], dtype=dt)
    b = np.frombuffer(bytes(blob), dtype=np.uint8)
    st = lib().or_decompress(b.ctypes.data, len(b), out.ctypes.data, out.nbytes)
    if st != OK:
        raise OracleError(st, "or_decompress")
    return out


def stats(x: np.ndarray, y: np.ndarray, vr: float, eb: float) -> dict:
    """Eq. 4: SSE, MSE, PSNR = -20 log10(sqrt(MSE)/vr), max |e|, #(|e| > eb)."""
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y, dtype=x.dtype)
    out = (ctypes.c_double * 4)()
    nov = ctypes.c_uint64(0)
    st = lib().or_stats(x.ctypes.data, y.ctypes.data, _dtype_code(x), x.size, float(vr),
                        float(eb), out, ctypes.byref(nov))
    if st != OK:
        raise OracleError(st, "or_stats")
    return {"sse": out[0], "mse": out[1], "psnr": out[2], "max_abs_err": out[3],
            "n_over_eb": int(nov.value)}


STAGES = {0: "range", 1: "prequant", 2: "lorenzo", 3: "symbols_hist_exceptions", 4: "codebook",
          5: "encode", 6: "blob", 8: "parse_tables", 9: "decode", 10: "prefix_sums",
          11: "reconstruct", 12: "stats"}


def stage_times() -> dict:
    """Wall-clock seconds of each stage of the last compress / decompress /
    stats calls (for the benchmark's CPU baseline)."""
    out = (ctypes.c_double * 16)()
    lib().or_stage_times(out)
    return {nm: out[k] for k, nm in STAGES.items()}
