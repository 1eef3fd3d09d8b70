"""Python binding of the gfx950 library ``libfpsz.so`` (C ABI in include/fpsz.h).

Argument marshalling only: every step of compression, decompression and the
PSNR check runs in the library's HIP kernels.  torch provides device memory
and streams.  There is no fallback: if the library is missing or the device
is not gfx950 the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfpsz.so")

OK, E_INVALID_ARG, E_NONFINITE, E_RANGE, E_CORRUPT, E_CAPACITY, E_NOMEM, E_DEVICE, E_UNSUPPORTED = range(9)
F32, F64 = 0, 1
GLOBAL, TILE = 0, 1
HDR_BYTES = 256
STATIC_WORKSPACE_BYTES = 64 << 20  # FPSZ_STATIC_WORKSPACE_BYTES


class FpszError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("fpsz status %d: %s" % (status, msg))
        self.status = status


class AsyncResult(ctypes.Structure):
    """fpsz_async_result: the device-side outcome of fpsz_compress_async."""
    _fields_ = [("status", ctypes.c_uint32), ("is_const", ctypes.c_uint32),
                ("blob_bytes", ctypes.c_uint64), ("n_outliers", ctypes.c_uint64),
                ("n_patches", ctypes.c_uint64), ("vr", ctypes.c_double), ("eb", ctypes.c_double)]


ASYNC_RESULT_BYTES = ctypes.sizeof(AsyncResult)


class DecompressResult(ctypes.Structure):
    """fpsz_decompress_result: the device-side outcome of fpsz_decompress_async."""
    _fields_ = [("status", ctypes.c_uint32), ("checked", ctypes.c_uint32),
                ("sse", ctypes.c_double), ("mse", ctypes.c_double), ("psnr", ctypes.c_double),
                ("max_abs_err", ctypes.c_double), ("n_over_eb", ctypes.c_uint64)]


DECOMPRESS_RESULT_BYTES = ctypes.sizeof(DecompressResult)


def decompress_result(result: torch.Tensor) -> DecompressResult:
    """Copy a device-side fpsz_decompress_result to the host (synchronizes)."""
    raw = bytes(result[:DECOMPRESS_RESULT_BYTES].cpu().numpy().tobytes())
    return DecompressResult.from_buffer_copy(raw)


def async_result(result: torch.Tensor) -> AsyncResult:
    """Copy a device-side fpsz_async_result to the host (synchronizes)."""
    raw = bytes(result[:ASYNC_RESULT_BYTES].cpu().numpy().tobytes())
    return AsyncResult.from_buffer_copy(raw)


class Info(ctypes.Structure):
    _fields_ = [
        ("target_psnr", ctypes.c_double), ("eb_rel", ctypes.c_double), ("vr", ctypes.c_double),
        ("eb", ctypes.c_double), ("min", ctypes.c_double), ("max", ctypes.c_double),
        ("n", ctypes.c_uint64), ("n_outliers", ctypes.c_uint64), ("n_patches", ctypes.c_uint64),
        ("n_exceptions", ctypes.c_uint64), ("blob_bytes", ctypes.c_uint64),
        ("bits_per_value", ctypes.c_double), ("is_const", ctypes.c_uint32),
        ("domain", ctypes.c_uint32), ("eb_scale", ctypes.c_double),
        ("variant", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("sse", ctypes.c_double), ("mse", ctypes.c_double), ("psnr", ctypes.c_double),
                ("max_abs_err", ctypes.c_double), ("n_over_eb", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StageTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("ms", ctypes.c_double)]


class FieldDesc(ctypes.Structure):
    _fields_ = [("field_dev", ctypes.c_void_p), ("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("dims", ctypes.c_uint64 * 3), ("target_psnr", ctypes.c_double),
                ("domain", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("blob_dev", ctypes.c_void_p), ("blob_capacity", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("domain", ctypes.c_int32), ("dims", ctypes.c_uint64 * 3),
                ("target_psnr", ctypes.c_double), ("src_dev", ctypes.c_void_p),
                ("src_bytes", ctypes.c_uint64), ("dst_dev", ctypes.c_void_p),
                ("dst_capacity", ctypes.c_uint64), ("ready_event", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("reserved", ctypes.c_uint32),
                ("out_bytes", ctypes.c_uint64), ("info", Info), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {"status": self.status, "out_bytes": self.out_bytes, "info": self.info.as_dict(),
                "t_submit": self.t_submit, "t_start": self.t_start, "t_done": self.t_done}


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
                ("batched_launches", ctypes.c_uint64), ("peak_inflight", ctypes.c_uint64),
                ("peak_held_bytes", ctypes.c_uint64), ("held_bytes", ctypes.c_uint64),
                ("now", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


REQ_COMPRESS, REQ_DECOMPRESS = 0, 1

_u64p = ctypes.POINTER(ctypes.c_uint64)
_vp = ctypes.c_void_p

# name -> (restype, argtypes); every symbol declared in include/fpsz.h
SIGNATURES = {
    "fpsz_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp)]),
    "fpsz_destroy": (None, [_vp]),
    "fpsz_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "fpsz_last_error": (ctypes.c_char_p, [_vp]),
    "fpsz_version": (ctypes.c_char_p, []),
    "fpsz_eb_rel": (ctypes.c_int, [ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "fpsz_compress_workspace_bytes": (ctypes.c_int, [ctypes.c_int, _u64p, ctypes.c_int, _u64p]),
    "fpsz_decompress_workspace_bytes": (ctypes.c_int, [ctypes.c_int, _u64p, ctypes.c_int, _u64p]),
    "fpsz_verify_workspace_bytes": (ctypes.c_int, [ctypes.c_uint64, _u64p]),
    "fpsz_compress_bound": (ctypes.c_int, [ctypes.c_int, _u64p, ctypes.c_int, _u64p]),
    "fpsz_compress": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _u64p, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int, _vp, ctypes.c_uint64, _vp, ctypes.c_uint64,
                                     _u64p, ctypes.POINTER(Info), _vp]),
    "fpsz_compress_xform": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _u64p, ctypes.c_int,
                                           ctypes.c_double, _vp, ctypes.c_uint64, _vp,
                                           ctypes.c_uint64, _u64p, ctypes.POINTER(Info), _vp]),
    "fpsz_compress_inloop": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _u64p, ctypes.c_int,
                                            ctypes.c_double, _vp, ctypes.c_uint64, _vp,
                                            ctypes.c_uint64, _u64p, ctypes.POINTER(Info), _vp]),
    "fpsz_compress_closed_loop": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _u64p, ctypes.c_int,
                                                 ctypes.c_double, ctypes.c_int, _vp,
                                                 ctypes.c_uint64, _vp, ctypes.c_uint64, _u64p,
                                                 ctypes.POINTER(Info), _vp]),
    "fpsz_compress_static": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _u64p, ctypes.c_int,
                                            ctypes.c_double, ctypes.c_int, _vp, ctypes.c_uint64,
                                            _u64p, ctypes.POINTER(Info), _vp]),
    "fpsz_compress_async": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _u64p, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_int, _vp, ctypes.c_uint64,
                                           _vp, ctypes.c_uint64, _vp, _vp]),
    "fpsz_decompress_async": (ctypes.c_int, [_vp, _vp, ctypes.c_uint64, _vp, _vp, ctypes.c_uint64,
                                             _vp, ctypes.c_uint64, _vp, _vp, _vp]),
    "fpsz_blob_header": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), _u64p,
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(Info)]),
    "fpsz_decompress": (ctypes.c_int, [_vp, _vp, ctypes.c_uint64, _vp, ctypes.c_uint64, _vp,
                                       ctypes.c_uint64, _vp]),
    "fpsz_decompress_verify": (ctypes.c_int, [_vp, _vp, ctypes.c_uint64, _vp, ctypes.c_uint64, _vp,
                                              ctypes.c_uint64, _vp, ctypes.POINTER(Stats), _vp]),
    "fpsz_verify": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_double, _vp, ctypes.c_uint64, ctypes.POINTER(Stats), _vp]),
    "fpsz_compress_workspace_offset": (ctypes.c_int, [ctypes.c_int, _u64p, ctypes.c_int, ctypes.c_int,
                                                      _u64p]),
    "fpsz_set_profiling": (ctypes.c_int, [_vp, ctypes.c_int]),
    "fpsz_last_stage_times": (ctypes.c_int, [_vp, ctypes.POINTER(StageTime), ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_int)]),
    "fpsz_batch_workspace_bytes": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(FieldDesc), _u64p]),
    "fpsz_batch_create": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(FieldDesc), _vp,
                                         ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_vp)]),
    "fpsz_batch_run": (ctypes.c_int, [_vp, _vp, _u64p, ctypes.POINTER(Info),
                                      ctypes.POINTER(ctypes.c_int)]),
    "fpsz_batch_autotune": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "fpsz_batch_launch_shape": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint32)]),
    "fpsz_batch_class_count": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    "fpsz_batch_set_launch_shape": (ctypes.c_int, [_vp, ctypes.c_int,
                                                   ctypes.POINTER(ctypes.c_uint32)]),
    "fpsz_batch_destroy": (None, [_vp]),
    "fpsz_compress_batch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(FieldDesc), _vp,
                                           ctypes.c_uint64, _u64p, ctypes.POINTER(Info),
                                           ctypes.POINTER(ctypes.c_int), _vp]),
    "fpsz_server_create": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                          ctypes.c_int, ctypes.POINTER(_vp)]),
    "fpsz_server_submit": (ctypes.c_int, [_vp, ctypes.POINTER(Request), _u64p]),
    "fpsz_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(Result)]),
    "fpsz_server_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(Result)]),
    "fpsz_server_get_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ServerStats)]),
    "fpsz_server_destroy": (None, [_vp]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfpsz.so and bind every exported entry point.  Raises if the
    library was not built (run ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise FpszError(E_UNSUPPORTED, "libfpsz.so is not built: %s" % path)
        L = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dims(shape):
    d = [int(s) for s in shape] + [1] * max(0, 3 - len(shape))
    return (ctypes.c_uint64 * len(d))(*d)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("fpsz compresses float32 or float64 fields")


def eb_rel(psnr: float) -> float:
    """Eq. 7 (host): eb_rel = sqrt(3) * 10^(-PSNR/20)."""
    out = ctypes.c_double()
    st = load_library().fpsz_eb_rel(float(psnr), ctypes.byref(out))
    if st != OK:
        raise FpszError(st, "eb_rel")
    return out.value


def _ws_bytes(fn, ndim, shape, dt) -> int:
    out = ctypes.c_uint64()
    st = fn(ndim, _dims(shape), dt, ctypes.byref(out))
    if st != OK:
        raise FpszError(st, "workspace size for shape %s" % (tuple(shape),))
    return out.value


def compress_workspace_bytes(shape, dtype=torch.float32) -> int:
    dt = F32 if dtype == torch.float32 else F64
    return _ws_bytes(load_library().fpsz_compress_workspace_bytes, len(shape), shape, dt)


def decompress_workspace_bytes(shape, dtype=torch.float32) -> int:
    dt = F32 if dtype == torch.float32 else F64
    return _ws_bytes(load_library().fpsz_decompress_workspace_bytes, len(shape), shape, dt)


def compress_bound(shape, dtype=torch.float32) -> int:
    dt = F32 if dtype == torch.float32 else F64
    return _ws_bytes(load_library().fpsz_compress_bound, len(shape), shape, dt)


def workspace_offset(shape, dtype, which: int) -> int:
    dt = F32 if dtype == torch.float32 else F64
    out = ctypes.c_uint64()
    st = load_library().fpsz_compress_workspace_offset(len(shape), _dims(shape), dt, which,
                                                       ctypes.byref(out))
    if st != OK:
        raise FpszError(st, "workspace offset")
    return out.value


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


@dataclass
class Header:
    ndim: int
    shape: tuple
    dtype: torch.dtype
    info: dict


def parse_header(blob_host: bytes) -> Header:
    b = bytes(blob_host[:HDR_BYTES])
    buf = ctypes.create_string_buffer(b, len(b))
    nd = ctypes.c_int()
    dims = (ctypes.c_uint64 * 3)()
    dt = ctypes.c_int()
    info = Info()
    st = load_library().fpsz_blob_header(buf, len(b), ctypes.byref(nd), dims, ctypes.byref(dt),
                                         ctypes.byref(info))
    if st != OK:
        raise FpszError(st, "blob header")
    return Header(nd.value, tuple(int(dims[i]) for i in range(nd.value)),
                  torch.float32 if dt.value == F32 else torch.float64, info.as_dict())


class Context:
    """One library context on one HIP device."""

    def __init__(self, device: int | None = None):
        self.lib = load_library()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = _vp()
        st = self.lib.fpsz_create(self.device, ctypes.byref(h))
        if st != OK:
            raise FpszError(st, "fpsz_create(%d): %s" % (self.device,
                                                         self.lib.fpsz_status_str(st).decode()))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.fpsz_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, st, what):
        msg = self.lib.fpsz_last_error(self.handle)
        return FpszError(st, "%s: %s" % (what, msg.decode() if msg else ""))

    def set_profiling(self, on: bool = True):
        st = self.lib.fpsz_set_profiling(self.handle, 1 if on else 0)
        if st != OK:
            raise self._err(st, "fpsz_set_profiling")

    def stage_times(self):
        """[(stage, ms)] of the last call (profiling must be on)."""
        buf = (StageTime * 48)()
        n = ctypes.c_int()
        st = self.lib.fpsz_last_stage_times(self.handle, buf, 48, ctypes.byref(n))
        if st != OK:
            raise self._err(st, "fpsz_last_stage_times")
        return [(buf[i].name.decode(), buf[i].ms) for i in range(min(n.value, 48))]

    # -- raw entry points on preallocated buffers ---------------------------
    def compress_into(self, x: torch.Tensor, psnr: float, workspace: torch.Tensor,
                      blob: torch.Tensor, domain: int = GLOBAL, stream=None):
        """Compress x into the device buffer ``blob``; returns (status,
        blob_bytes, Info).  Status CAPACITY reports the size needed."""
        assert x.is_contiguous() and x.is_cuda
        nb = ctypes.c_uint64()
        info = Info()
        st = self.lib.fpsz_compress(self.handle, x.data_ptr(), x.dim(), _dims(x.shape),
                                    _dtype_code(x), float(psnr), int(domain), workspace.data_ptr(),
                                    workspace.numel() * workspace.element_size(), blob.data_ptr(),
                                    blob.numel(), ctypes.byref(nb), ctypes.byref(info),
                                    _stream(stream))
        return st, nb.value, info

    def compress_inloop_into(self, x: torch.Tensor, psnr: float, workspace: torch.Tensor,
                             blob: torch.Tensor, stream=None):
        """fpsz_compress_inloop into ``blob``; returns (status, blob_bytes, Info)."""
        assert x.is_contiguous() and x.is_cuda
        nb = ctypes.c_uint64()
        info = Info()
        st = self.lib.fpsz_compress_inloop(self.handle, x.data_ptr(), x.dim(), _dims(x.shape),
                                           _dtype_code(x), float(psnr), workspace.data_ptr(),
                                           workspace.numel() * workspace.element_size(),
                                           blob.data_ptr(), blob.numel(), ctypes.byref(nb),
                                           ctypes.byref(info), _stream(stream))
        return st, nb.value, info

    def compress_xform_into(self, x: torch.Tensor, psnr: float, workspace: torch.Tensor,
                            blob: torch.Tensor, stream=None):
        """fpsz_compress_xform into ``blob``; returns (status, blob_bytes, Info)."""
        assert x.is_contiguous() and x.is_cuda
        nb = ctypes.c_uint64()
        info = Info()
        st = self.lib.fpsz_compress_xform(self.handle, x.data_ptr(), x.dim(), _dims(x.shape),
                                          _dtype_code(x), float(psnr), workspace.data_ptr(),
                                          workspace.numel() * workspace.element_size(),
                                          blob.data_ptr(), blob.numel(), ctypes.byref(nb),
                                          ctypes.byref(info), _stream(stream))
        return st, nb.value, info

    def compress_closed_loop_into(self, x: torch.Tensor, psnr: float, workspace: torch.Tensor,
                                  blob: torch.Tensor, domain: int = GLOBAL, stream=None):
        """fpsz_compress_closed_loop into ``blob``; returns (status,
        blob_bytes, Info) with Info.eb_scale the factor applied."""
        assert x.is_contiguous() and x.is_cuda
        nb = ctypes.c_uint64()
        info = Info()
        st = self.lib.fpsz_compress_closed_loop(self.handle, x.data_ptr(), x.dim(),
                                                _dims(x.shape), _dtype_code(x), float(psnr),
                                                int(domain), workspace.data_ptr(),
                                                workspace.numel() * workspace.element_size(),
                                                blob.data_ptr(), blob.numel(), ctypes.byref(nb),
                                                ctypes.byref(info), _stream(stream))
        return st, nb.value, info

    def compress_closed_loop(self, x: torch.Tensor, psnr: float, domain: int = GLOBAL,
                             stream=None):
        """Returns (blob tensor of the blob's size, info dict)."""
        x = x.contiguous()
        ws = torch.empty(compress_workspace_bytes(x.shape, x.dtype), dtype=torch.uint8,
                         device=x.device)
        blob = torch.empty(compress_bound(x.shape, x.dtype), dtype=torch.uint8, device=x.device)
        st, nb, info = self.compress_closed_loop_into(x, psnr, ws, blob, domain, stream)
        if st != OK:
            raise self._err(st, "fpsz_compress_closed_loop")
        return blob[:nb], info.as_dict()

    def compress_static(self, x: torch.Tensor, psnr: float, blob: torch.Tensor,
                        domain: int = GLOBAL, stream=None):
        """fpsz_compress_static: compress x into ``blob`` using the library's
        static device workspace (no allocation); returns (status,
        blob_bytes, Info)."""
        assert x.is_contiguous() and x.is_cuda
        nb = ctypes.c_uint64()
        info = Info()
        st = self.lib.fpsz_compress_static(self.handle, x.data_ptr(), x.dim(), _dims(x.shape),
                                           _dtype_code(x), float(psnr), int(domain),
                                           blob.data_ptr(), blob.numel(), ctypes.byref(nb),
                                           ctypes.byref(info), _stream(stream))
        return st, nb.value, info

    def compress_async_into(self, x: torch.Tensor, psnr: float, workspace: torch.Tensor,
                            blob: torch.Tensor, result: torch.Tensor, domain: int = GLOBAL,
                            stream=None) -> int:
        """fpsz_compress_async: enqueue the compression of x into ``blob``;
        the outcome goes to ``result`` (a device uint8 tensor of
        ASYNC_RESULT_BYTES, read it with async_result()).  Returns the host
        status only; nothing is synchronized."""
        assert x.is_contiguous() and x.is_cuda
        assert result.is_cuda and result.numel() * result.element_size() >= ASYNC_RESULT_BYTES
        return self.lib.fpsz_compress_async(self.handle, x.data_ptr(), x.dim(), _dims(x.shape),
                                            _dtype_code(x), float(psnr), int(domain),
                                            workspace.data_ptr(),
                                            workspace.numel() * workspace.element_size(),
                                            blob.data_ptr(), blob.numel(), result.data_ptr(),
                                            _stream(stream))

    def decompress_async_into(self, blob: torch.Tensor, nbytes: int, header: bytes,
                              workspace: torch.Tensor, out: torch.Tensor, result: torch.Tensor,
                              orig: torch.Tensor | None = None, stream=None) -> int:
        """fpsz_decompress_async: enqueue the decompression of ``blob`` whose
        header (its first 256 bytes) the caller holds on the host; the
        outcome (and Eq. 4 against ``orig`` when given) goes to ``result`` (a
        device uint8 tensor of DECOMPRESS_RESULT_BYTES, read it with
        decompress_result()).  Returns the host status only."""
        assert len(header) >= 256
        assert result.is_cuda and result.numel() * result.element_size() >= DECOMPRESS_RESULT_BYTES
        hb = ctypes.create_string_buffer(bytes(header[:256]), 256)
        return self.lib.fpsz_decompress_async(
            self.handle, blob.data_ptr(), int(nbytes), hb, workspace.data_ptr(),
            workspace.numel() * workspace.element_size(), out.data_ptr(),
            out.numel() * out.element_size(), orig.data_ptr() if orig is not None else None,
            result.data_ptr(), _stream(stream))

    def decompress_into(self, blob: torch.Tensor, nbytes: int, workspace: torch.Tensor,
                        out: torch.Tensor, stream=None) -> int:
        return self.lib.fpsz_decompress(self.handle, blob.data_ptr(), int(nbytes), workspace.data_ptr(),
                                         workspace.numel() * workspace.element_size(), out.data_ptr(),
                                         out.numel() * out.element_size(), _stream(stream))

    def decompress_verify_into(self, blob: torch.Tensor, nbytes: int, workspace: torch.Tensor,
                               out: torch.Tensor, x: torch.Tensor, stream=None):
        """Decompress into ``out`` and check it against the original ``x`` in the
        same pass (fpsz_decompress_verify); returns (status, Stats)."""
        stats = Stats()
        st = self.lib.fpsz_decompress_verify(self.handle, blob.data_ptr(), int(nbytes),
                                             workspace.data_ptr(),
                                             workspace.numel() * workspace.element_size(),
                                             out.data_ptr(), out.numel() * out.element_size(),
                                             x.data_ptr(), ctypes.byref(stats), _stream(stream))
        return st, stats

    def verify_into(self, x: torch.Tensor, y: torch.Tensor, vr: float, eb: float,
                    workspace: torch.Tensor, stream=None):
        stats = Stats()
        st = self.lib.fpsz_verify(self.handle, x.data_ptr(), y.data_ptr(), x.numel(),
                                  _dtype_code(x), float(vr), float(eb), workspace.data_ptr(),
                                  workspace.numel() * workspace.element_size(),
                                  ctypes.byref(stats), _stream(stream))
        return st, stats

    # -- convenience API ------------------------------------------------------
    def compress(self, x: torch.Tensor, psnr: float, domain: int = GLOBAL, stream=None):
        """Returns (blob: uint8 device tensor of exactly the blob's size, info dict)."""
        x = x.contiguous()
        ws = torch.empty(compress_workspace_bytes(x.shape, x.dtype), dtype=torch.uint8,
                         device=x.device)
        cap = x.numel() * x.element_size() + (1 << 20) + x.numel() // 8
        blob = torch.empty(cap, dtype=torch.uint8, device=x.device)
        st, nb, info = self.compress_into(x, psnr, ws, blob, domain, stream)
        if st == E_CAPACITY and nb > cap:
            blob = torch.empty(nb, dtype=torch.uint8, device=x.device)
            st, nb, info = self.compress_into(x, psnr, ws, blob, domain, stream)
        if st != OK:
            raise self._err(st, "fpsz_compress")
        return blob[:nb], info.as_dict()

    def decompress(self, blob: torch.Tensor, stream=None) -> torch.Tensor:
        hdr = parse_header(blob[:HDR_BYTES].cpu().numpy().tobytes())
        out = torch.empty(hdr.shape, dtype=hdr.dtype, device=blob.device)
        ws = torch.empty(decompress_workspace_bytes(hdr.shape, hdr.dtype), dtype=torch.uint8,
                         device=blob.device)
        st = self.decompress_into(blob, blob.numel(), ws, out, stream)
        if st != OK:
            raise self._err(st, "fpsz_decompress")
        return out

    def decompress_verify(self, blob: torch.Tensor, x: torch.Tensor, stream=None):
        """Returns (reconstruction, stats dict) of one fused decompress + check pass."""
        hdr = parse_header(blob[:HDR_BYTES].cpu().numpy().tobytes())
        out = torch.empty(hdr.shape, dtype=hdr.dtype, device=blob.device)
        ws = torch.empty(decompress_workspace_bytes(hdr.shape, hdr.dtype), dtype=torch.uint8,
                         device=blob.device)
        st, stats = self.decompress_verify_into(blob, blob.numel(), ws, out, x.contiguous(), stream)
        if st != OK:
            raise self._err(st, "fpsz_decompress_verify")
        return out, stats.as_dict()

    def verify(self, x: torch.Tensor, y: torch.Tensor, vr: float, eb: float, stream=None) -> dict:
        ws_n = ctypes.c_uint64()
        self.lib.fpsz_verify_workspace_bytes(x.numel(), ctypes.byref(ws_n))
        ws = torch.empty(ws_n.value, dtype=torch.uint8, device=x.device)
        st, stats = self.verify_into(x.contiguous(), y.contiguous(), vr, eb, ws, stream)
        if st != OK:
            raise self._err(st, "fpsz_verify")
        return stats.as_dict()


def field_descs(fields, psnrs, blobs, domains=None):
    """ctypes array of fpsz_field_desc for device tensors ``fields`` (each
    contiguous float32/float64) with targets ``psnrs`` and output buffers
    ``blobs`` (uint8 device tensors)."""
    n = len(fields)
    arr = (FieldDesc * n)()
    for i, (x, p, b) in enumerate(zip(fields, psnrs, blobs)):
        assert x.is_contiguous() and x.is_cuda and b.is_cuda
        d = arr[i]
        d.field_dev = x.data_ptr()
        d.ndim = x.dim()
        d.dtype = _dtype_code(x)
        for k, v in enumerate(list(x.shape) + [1] * (3 - x.dim())):
            d.dims[k] = int(v)
        d.target_psnr = float(p)
        d.domain = int(domains[i]) if domains is not None else GLOBAL
        d.blob_dev = b.data_ptr()
        d.blob_capacity = b.numel()
    return arr


# -- persistent autotune cache (JSON) ------------------------------------------
# {"version": 1, "entries": {key: {"shapes": [[range, quant, encode, checksum]
# per field group], "best_ms": t, "fields": n}}}.  The key covers what the
# launch shapes depend on: the device, the library build and every field's
# (dtype, ndim, dims, domain) as a multiset; targets do not enter (shapes are
# bit-neutral and the timing barely depends on them).

def _device_name(device) -> str:
    try:
        p = torch.cuda.get_device_properties(device)
        return "%s/%s/%d" % (p.name, getattr(p, "gcnArchName", ""), p.multi_processor_count)
    except Exception:  # noqa: BLE001 - a name is only part of a cache key
        return "unknown"


def autotune_key(descs, device_name: str) -> str:
    import hashlib
    import json
    fields = sorted((int(d.dtype), int(d.ndim), [int(v) for v in d.dims], int(d.domain))
                    for d in descs)
    ver = load_library().fpsz_version().decode()
    blob = json.dumps({"device": device_name, "version": ver, "fields": fields},
                      sort_keys=True)
    return hashlib.sha256(blob.encode()).hexdigest()


def load_autotune_cache(path: str) -> dict:
    """Entries of a cache file; {} for a missing, unreadable or foreign file."""
    import json
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return {}
    if not isinstance(d, dict) or d.get("version") != 1 or not isinstance(d.get("entries"), dict):
        return {}
    out = {}
    for k, v in d["entries"].items():
        ok = (isinstance(v, dict) and isinstance(v.get("shapes"), list)
              and all(isinstance(s, list) and len(s) == 4 and all(isinstance(x, int) and x > 0
                                                                 for x in s)
                      for s in v["shapes"]) and isinstance(v.get("best_ms"), (int, float)))
        if ok:
            out[k] = v
    return out


def store_autotune_cache(path: str, key: str, shapes, best_ms: float):
    """Add (or replace) one entry; the file is replaced atomically."""
    import json
    import tempfile
    entries = load_autotune_cache(path)
    entries[key] = {"shapes": [[int(x) for x in s] for s in shapes], "best_ms": float(best_ms)}
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(prefix=".fpsz_autotune.", dir=d)
    with os.fdopen(fd, "w") as fh:
        json.dump({"version": 1, "entries": entries}, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def batch_workspace_bytes(descs) -> int:
    out = ctypes.c_uint64()
    st = load_library().fpsz_batch_workspace_bytes(len(descs), descs, ctypes.byref(out))
    if st != OK:
        raise FpszError(st, "batch workspace size")
    return out.value


class Batch:
    """A planned batch of fields (fpsz_batch_*).  Keeps references to the
    tensors it was created with; they must not be freed before close()."""

    def __init__(self, ctx: Context, fields, psnrs, blobs, domains=None, graph: bool = False,
                 workspace: torch.Tensor | None = None):
        self.ctx = ctx
        self.lib = ctx.lib
        self.fields, self.blobs = list(fields), list(blobs)
        self.descs = field_descs(self.fields, psnrs, self.blobs, domains)
        self.n = len(self.fields)
        need = batch_workspace_bytes(self.descs)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.fields[0].device)
        self.workspace = workspace
        h = _vp()
        st = self.lib.fpsz_batch_create(ctx.handle, self.n, self.descs, workspace.data_ptr(),
                                        workspace.numel(), 1 if graph else 0, ctypes.byref(h))
        if st != OK:
            raise ctx._err(st, "fpsz_batch_create")
        self.handle = h

    def run(self, stream=None, check: bool = True):
        """Returns (status, blob_bytes list, info list of dicts, per-field status list)."""
        nb = (ctypes.c_uint64 * self.n)()
        info = (Info * self.n)()
        sts = (ctypes.c_int * self.n)()
        st = self.lib.fpsz_batch_run(self.handle, _stream(stream), nb, info, sts)
        if check and st != OK:
            raise self.ctx._err(st, "fpsz_batch_run")
        return st, list(nb), [i.as_dict() for i in info], list(sts)

    def autotune(self, reps: int = 3, stream=None, cache: str | None = None) -> float:
        """Time launch shapes and keep the fastest (fpsz_batch_autotune).  With
        a cache file (``cache``, else $FPSZ_AUTOTUNE_CACHE when set), shapes
        found earlier for the same fields on the same device are applied
        without timing, and new ones are added to the file.  Sets
        ``self.autotune_source`` to "cache" or "timed"; returns the best batch
        time in ms (the one recorded with the shapes on a cache hit)."""
        if cache is None:
            cache = os.environ.get("FPSZ_AUTOTUNE_CACHE") or None
        key = autotune_key(self.descs, _device_name(self.fields[0].device)) if cache else None
        if key is not None:
            hit = load_autotune_cache(cache).get(key)
            if hit is not None and len(hit["shapes"]) == self.class_count():
                for c, sh in enumerate(hit["shapes"]):
                    self.set_launch_shape(c, sh)
                self.autotune_source = "cache"
                return float(hit["best_ms"])
        best = ctypes.c_double()
        st = self.lib.fpsz_batch_autotune(self.handle, _stream(stream), int(reps), ctypes.byref(best))
        if st != OK:
            raise self.ctx._err(st, "fpsz_batch_autotune")
        self.autotune_source = "timed"
        if key is not None:
            store_autotune_cache(cache, key, [self.launch_shape(c) for c in range(self.class_count())],
                                 best.value)
        return best.value

    def class_count(self) -> int:
        n = ctypes.c_int()
        st = self.lib.fpsz_batch_class_count(self.handle, ctypes.byref(n))
        if st != OK:
            raise FpszError(st, "class count")
        return n.value

    def set_launch_shape(self, cls: int, shape4):
        arr = (ctypes.c_uint32 * 4)(*[int(v) for v in shape4])
        st = self.lib.fpsz_batch_set_launch_shape(self.handle, int(cls), arr)
        if st != OK:
            raise self.ctx._err(st, "fpsz_batch_set_launch_shape")

    def launch_shape(self, cls: int = 0):
        out = (ctypes.c_uint32 * 4)()
        st = self.lib.fpsz_batch_launch_shape(self.handle, int(cls), out)
        if st != OK:
            raise FpszError(st, "launch shape")
        return list(out)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.fpsz_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """fpsz_server_*: a request loop with HBM-budget admission and continuous
    batching.  Keeps the tensors of each request alive until it is reported."""

    def __init__(self, ctx: Context, hbm_budget: int, arena_bytes: int, max_inflight: int = 64,
                 n_streams: int = 4):
        self.ctx = ctx
        self.lib = ctx.lib
        h = _vp()
        st = self.lib.fpsz_server_create(ctx.handle, int(hbm_budget), int(arena_bytes),
                                         int(max_inflight), int(n_streams), ctypes.byref(h))
        if st != OK:
            raise ctx._err(st, "fpsz_server_create")
        self.handle = h
        self._keep = {}

    def submit_compress(self, x: torch.Tensor, psnr: float, blob: torch.Tensor,
                        domain: int = GLOBAL) -> int:
        assert x.is_contiguous() and x.is_cuda
        r = Request()
        r.kind = REQ_COMPRESS
        r.ndim = x.dim()
        r.dtype = _dtype_code(x)
        r.domain = int(domain)
        for k, v in enumerate(list(x.shape) + [1] * (3 - x.dim())):
            r.dims[k] = int(v)
        r.target_psnr = float(psnr)
        r.src_dev = x.data_ptr()
        r.dst_dev = blob.data_ptr()
        r.dst_capacity = blob.numel()
        return self._submit(r, (x, blob))

    def submit_decompress(self, blob: torch.Tensor, nbytes: int, out: torch.Tensor) -> int:
        assert out.is_contiguous() and out.is_cuda
        r = Request()
        r.kind = REQ_DECOMPRESS
        r.ndim = out.dim()
        r.dtype = _dtype_code(out)
        for k, v in enumerate(list(out.shape) + [1] * (3 - out.dim())):
            r.dims[k] = int(v)
        r.src_dev = blob.data_ptr()
        r.src_bytes = int(nbytes)
        r.dst_dev = out.data_ptr()
        r.dst_capacity = out.numel() * out.element_size()
        return self._submit(r, (blob, out))

    def _submit(self, r, keep) -> int:
        # the inputs may still be in flight on torch's current stream: the
        # server's stream waits on an event recorded there after them
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream())
        r.ready_event = ev.cuda_event
        keep = keep + (ev,)
        rid = ctypes.c_uint64()
        st = self.lib.fpsz_server_submit(self.handle, ctypes.byref(r), ctypes.byref(rid))
        if st != OK:
            raise FpszError(st, "fpsz_server_submit")
        self._keep[rid.value] = keep
        return rid.value

    def poll(self, rid: int):
        """Result dict when request ``rid`` has finished, else None."""
        done = ctypes.c_int()
        res = Result()
        st = self.lib.fpsz_server_poll(self.handle, int(rid), ctypes.byref(done), ctypes.byref(res))
        if st != OK:
            raise FpszError(st, "fpsz_server_poll(%d)" % rid)
        if not done.value:
            return None
        self._keep.pop(rid, None)
        return res.as_dict()

    def wait(self, rid: int) -> dict:
        res = Result()
        st = self.lib.fpsz_server_wait(self.handle, int(rid), ctypes.byref(res))
        if st != OK:
            raise FpszError(st, "fpsz_server_wait(%d)" % rid)
        self._keep.pop(rid, None)
        return res.as_dict()

    def stats(self) -> dict:
        out = ServerStats()
        st = self.lib.fpsz_server_get_stats(self.handle, ctypes.byref(out))
        if st != OK:
            raise FpszError(st, "fpsz_server_get_stats")
        return out.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            self.lib.fpsz_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def default_context(device: int | None = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def compress(x: torch.Tensor, psnr: float, domain: int = GLOBAL):
    return default_context(x.device.index).compress(x, psnr, domain)


def decompress(blob: torch.Tensor) -> torch.Tensor:
    return default_context(blob.device.index).decompress(blob)


def verify(x: torch.Tensor, y: torch.Tensor, vr: float, eb: float) -> dict:
    return default_context(x.device.index).verify(x, y, vr, eb)
