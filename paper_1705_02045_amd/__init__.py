"""Euler characteristic curves of gray-scale images on one MI355X.

Thin ctypes binding of ``libecc.so`` (C ABI in ``include/ecc.h``): argument
marshalling only.  Every step of the computation runs in the library's HIP
kernels; PyTorch supplies device memory and the current stream.  Importing
this package fails loudly if the library is not built.
"""
from __future__ import annotations

import ctypes
import os
import pathlib

_HERE = pathlib.Path(__file__).resolve().parent
_LIBPATH = _HERE / "libecc.so"
if not _LIBPATH.exists():
    raise ImportError(f"{_LIBPATH} is missing: build it with __graft_entry__.build() (hipcc, gfx950)")
_lib = ctypes.CDLL(str(_LIBPATH))

ECC_OK = 0
ECC_E_ARG = -1
ECC_E_RANGE = -2
ECC_E_NAN = -3
ECC_E_BUFFER_TOO_SMALL = -4
ECC_E_STATE = -5
ECC_E_NOMEM = -6
ECC_E_HIP = -7
ECC_E_UNSUPPORTED = -8
STATUS_RANGE_BIT = 1

DTYPES = {"u8": 1, "u14": 2, "u16": 3, "f32": 4}
THRESHOLDS = {"u8": 256, "u14": 16384, "u16": 65536}
_ERRNAME = {v: k for k, v in globals().items() if k.startswith("ECC_E_")}


class Dims(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int64 * 4)]


class Job(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p), ("dims", Dims), ("dtype", ctypes.c_int32),
                ("chi", ctypes.c_void_p)]


class Tiling(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("tiles_per_cu", ctypes.c_int32), ("waves_x", ctypes.c_int32),
                ("ms", ctypes.c_float)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("one_launch_per_image", ctypes.c_int32),
                ("max_batch_bytes", ctypes.c_int64), ("arena_bytes", ctypes.c_int64),
                ("stream_above_bytes", ctypes.c_int64), ("chunk_bytes", ctypes.c_int64),
                ("max_inflight", ctypes.c_int32)]


class Curve(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("count", ctypes.c_int64),
                ("chi", ctypes.c_void_p), ("keys", ctypes.c_void_p)]


_vp = ctypes.c_void_p
_lib.ecc_compute.restype = ctypes.c_int
_lib.ecc_compute.argtypes = [_vp, ctypes.POINTER(Dims), ctypes.c_int, ctypes.POINTER(Curve), _vp]
_lib.ecc_compute_change_points.restype = ctypes.c_int
_lib.ecc_compute_change_points.argtypes = [_vp, ctypes.POINTER(Dims), ctypes.c_int, ctypes.POINTER(Curve), _vp]
_lib.ecc_compute_quantized.restype = ctypes.c_int
_lib.ecc_compute_quantized.argtypes = [_vp, ctypes.POINTER(Dims), ctypes.c_float, ctypes.c_float, ctypes.c_int,
                                       ctypes.POINTER(Curve), _vp]
_lib.ecc_autotune.restype = ctypes.c_int
_lib.ecc_autotune.argtypes = [_vp, ctypes.POINTER(Dims), ctypes.c_int, _vp, ctypes.POINTER(Tiling)]
_lib.ecc_tiling_for.restype = ctypes.c_int
_lib.ecc_tiling_for.argtypes = [ctypes.POINTER(Dims), ctypes.c_int, ctypes.POINTER(Tiling)]
_lib.ecc_autotune_reset.restype = None
_lib.ecc_autotune_reset.argtypes = []
_lib.ecc_autotune_save.restype = ctypes.c_int
_lib.ecc_autotune_save.argtypes = [ctypes.c_char_p]
_lib.ecc_autotune_load.restype = ctypes.c_int
_lib.ecc_autotune_load.argtypes = [ctypes.c_char_p]
_lib.ecc_release_workspaces.restype = ctypes.c_int
_lib.ecc_release_workspaces.argtypes = []
_lib.ecc_batch_autotune.restype = ctypes.c_int
_lib.ecc_batch_autotune.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float)]
_lib.ecc_compute_dual.restype = ctypes.c_int
_lib.ecc_compute_dual.argtypes = [_vp, ctypes.POINTER(Dims), ctypes.c_int, ctypes.POINTER(Curve), _vp]
_lib.ecc_compute_max_entry.restype = ctypes.c_int
_lib.ecc_compute_max_entry.argtypes = [_vp, ctypes.POINTER(Dims), ctypes.c_int, ctypes.POINTER(Curve), _vp]
_lib.ecc_compute_async.restype = ctypes.c_int
_lib.ecc_compute_async.argtypes = [_vp, ctypes.POINTER(Dims), ctypes.c_int, _vp, _vp, _vp]
_lib.ecc_compute_async_noalloc.restype = ctypes.c_int
_lib.ecc_compute_async_noalloc.argtypes = [_vp, ctypes.POINTER(Dims), ctypes.c_int, _vp, _vp, _vp]
_lib.ecc_threshold_count.restype = ctypes.c_int
_lib.ecc_threshold_count.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
_lib.ecc_stream_begin.restype = ctypes.c_int
_lib.ecc_stream_begin.argtypes = [ctypes.POINTER(Dims), ctypes.c_int, _vp, ctypes.POINTER(_vp)]
_lib.ecc_stream_push_chunk.restype = ctypes.c_int
_lib.ecc_stream_push_chunk.argtypes = [_vp, _vp, ctypes.c_int64]
_lib.ecc_stream_finish.restype = ctypes.c_int
_lib.ecc_stream_finish.argtypes = [_vp, ctypes.POINTER(Curve)]
_lib.ecc_stream_abort.restype = None
_lib.ecc_stream_abort.argtypes = [_vp]
_lib.ecc_stream_snapshot_size.restype = ctypes.c_int
_lib.ecc_stream_snapshot_size.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)]
_lib.ecc_stream_snapshot.restype = ctypes.c_int
_lib.ecc_stream_snapshot.argtypes = [_vp, _vp, ctypes.c_int64]
_lib.ecc_stream_restore.restype = ctypes.c_int
_lib.ecc_stream_restore.argtypes = [_vp, ctypes.c_int64, _vp, ctypes.POINTER(_vp)]
_lib.ecc_profile_enable.restype = ctypes.c_int
_lib.ecc_profile_enable.argtypes = [ctypes.c_int]
_lib.ecc_profile_reset.restype = ctypes.c_int
_lib.ecc_batch_create.restype = ctypes.c_int
_lib.ecc_batch_create.argtypes = [_vp, ctypes.POINTER(_vp)]
_lib.ecc_batch_run.restype = ctypes.c_int
_lib.ecc_batch_run.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
_lib.ecc_batch_destroy.restype = None
_lib.ecc_batch_destroy.argtypes = [_vp]
_lib.ecc_serve_simulate.restype = ctypes.c_int
_lib.ecc_serve_simulate.argtypes = [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                    _vp, _vp, _vp]
_lib.ecc_job_footprint.restype = ctypes.c_int
_lib.ecc_serve.restype = ctypes.c_int
_lib.ecc_serve.argtypes = [_vp, ctypes.c_int32, _vp, _vp, ctypes.POINTER(ServeConfig), _vp, _vp, _vp, _vp]
_lib.ecc_job_footprint.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)]
_lib.ecc_profile_read.restype = ctypes.c_int
_lib.ecc_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
_lib.ecc_last_error.restype = ctypes.c_char_p
_lib.ecc_version.restype = ctypes.c_char_p


class EccError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.ecc_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_ERRNAME.get(code, code)} ({code}): {msg}")
        self.code = code


def _check(code: int, where: str):
    if code != ECC_OK:
        raise EccError(code, where)


def profile_enable(on: bool = True):
    _check(_lib.ecc_profile_enable(1 if on else 0), "ecc_profile_enable")


def profile_reset():
    _check(_lib.ecc_profile_reset(), "ecc_profile_reset")


def profile_read():
    """(summed milliseconds, launches) of the per-voxel kernels since the last reset."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(_lib.ecc_profile_read(ctypes.byref(ms), ctypes.byref(n)), "ecc_profile_read")
    return ms.value, n.value


def library_path() -> str:
    return str(_LIBPATH)


def version() -> str:
    return _lib.ecc_version().decode()


def make_dims(shape) -> Dims:
    shape = tuple(int(s) for s in shape)
    d = Dims()
    d.ndim = len(shape)
    for i, s in enumerate(shape[:4]):
        d.n[i] = s
    return d


def _stream_handle(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dtype_of(t, dtype):
    import torch
    if dtype is not None:
        return dtype
    return {torch.uint8: "u8", torch.float32: "f32"}.get(t.dtype) or _raise(
        f"pass dtype= for tensors of {t.dtype} (u14 or u16 for 16-bit data)")


def _raise(msg):
    raise TypeError(msg)


def compute(image, dtype: str | None = None):
    """chi(T_t) for every threshold of a CUDA tensor (int64 tensor on the same device).

    dtype: "u8" (uint8), "u14"/"u16" (16-bit tensors, any 16-bit torch dtype
    reinterpreted as unsigned), "f32" (returns (keys, chi)).
    """
    import torch
    if not image.is_cuda:
        raise ValueError("compute() takes a device tensor")
    dtype = _dtype_of(image, dtype)
    image = image.contiguous()
    dims = make_dims(image.shape)
    dev = image.device
    with torch.cuda.device(dev):
        if dtype == "f32":
            n = image.numel()
            chi = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
            keys = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
            cv = Curve(capacity=n, count=0, chi=chi.data_ptr(), keys=keys.data_ptr())
            _check(_lib.ecc_compute(image.data_ptr(), ctypes.byref(dims), DTYPES[dtype], ctypes.byref(cv),
                                    _stream_handle(dev)), "ecc_compute")
            return keys[: cv.count], chi[: cv.count]
        m = THRESHOLDS[dtype]
        chi = torch.empty(m, dtype=torch.int64, device=dev)
        cv = Curve(capacity=m, count=0, chi=chi.data_ptr(), keys=None)
        _check(_lib.ecc_compute(image.data_ptr(), ctypes.byref(dims), DTYPES[dtype], ctypes.byref(cv),
                                _stream_handle(dev)), "ecc_compute")
        return chi


def _compute_int_variant(fn, name, image, dtype):
    import torch
    if not image.is_cuda:
        raise ValueError(f"{name}() takes a device tensor")
    image = image.contiguous()
    dims = make_dims(image.shape)
    dev = image.device
    with torch.cuda.device(dev):
        m = THRESHOLDS.get(dtype, 1)  # the library rejects non-integer dtypes
        chi = torch.empty(m, dtype=torch.int64, device=dev)
        cv = Curve(capacity=m, count=0, chi=chi.data_ptr(), keys=None)
        _check(fn(image.data_ptr(), ctypes.byref(dims), DTYPES[dtype], ctypes.byref(cv), _stream_handle(dev)),
               f"ecc_{name}")
        return chi


def compute_max_entry(image, dtype: str):
    """ecc_compute_max_entry on a CUDA tensor (integer dtypes): each cell's value
    is the maximum over its voxels.  Returns the int64 curve on the same device."""
    return _compute_int_variant(_lib.ecc_compute_max_entry, "compute_max_entry", image, dtype)


def compute_change_points(image):
    """ecc_compute_change_points on a float32 CUDA tensor: (keys, chi) at the
    distinct values where chi changes."""
    import torch
    if not image.is_cuda:
        raise ValueError("compute_change_points() takes a device tensor")
    image = image.contiguous()
    dims = make_dims(image.shape)
    dev = image.device
    n = image.numel()
    with torch.cuda.device(dev):
        chi = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
        keys = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
        cv = Curve(capacity=n, count=0, chi=chi.data_ptr(), keys=keys.data_ptr())
        _check(_lib.ecc_compute_change_points(image.data_ptr(), ctypes.byref(dims), DTYPES["f32"], ctypes.byref(cv),
                                              _stream_handle(dev)), "ecc_compute_change_points")
        return keys[: cv.count], chi[: cv.count]


def compute_quantized(image, lo: float, hi: float, bins: str):
    """ecc_compute_quantized on a float32 CUDA tensor: the integer curve of the
    image quantised to `bins` ("u8", "u14", "u16") over [lo, hi)."""
    import torch
    if not image.is_cuda:
        raise ValueError("compute_quantized() takes a device tensor")
    image = image.contiguous()
    dims = make_dims(image.shape)
    dev = image.device
    with torch.cuda.device(dev):
        m = THRESHOLDS[bins]
        chi = torch.empty(m, dtype=torch.int64, device=dev)
        cv = Curve(capacity=m, count=0, chi=chi.data_ptr(), keys=None)
        _check(_lib.ecc_compute_quantized(image.data_ptr(), ctypes.byref(dims), float(lo), float(hi), DTYPES[bins],
                                          ctypes.byref(cv), _stream_handle(dev)), "ecc_compute_quantized")
        return chi


def autotune(image, dtype: str) -> dict:
    """ecc_autotune on a device tensor: times the candidate tilings and stores
    the fastest for the image's shape; returns it."""
    import torch
    t = Tiling()
    dims = make_dims(image.shape)
    with torch.cuda.device(image.device):
        _check(_lib.ecc_autotune(image.contiguous().data_ptr(), ctypes.byref(dims), DTYPES[dtype],
                                 _stream_handle(image.device), ctypes.byref(t)), "ecc_autotune")
    return {"rows": t.rows, "tiles_per_cu": t.tiles_per_cu, "waves_x": t.waves_x, "ms": t.ms}


def tiling_for(shape, dtype: str) -> dict:
    """ecc_tiling_for: the tiling a resident launch of this shape would use."""
    t = Tiling()
    _check(_lib.ecc_tiling_for(ctypes.byref(make_dims(shape)), DTYPES[dtype], ctypes.byref(t)), "ecc_tiling_for")
    return {"rows": t.rows, "tiles_per_cu": t.tiles_per_cu, "waves_x": t.waves_x}


def autotune_reset():
    _lib.ecc_autotune_reset()


def autotune_save(path) -> int:
    """ecc_autotune_save: the stored tilings to a text file; returns the count."""
    n = _lib.ecc_autotune_save(os.fsencode(path))
    if n < 0:
        _check(n, "ecc_autotune_save")
    return n


def autotune_load(path) -> int:
    """ecc_autotune_load: adds a saved file's tilings; returns the count."""
    n = _lib.ecc_autotune_load(os.fsencode(path))
    if n < 0:
        _check(n, "ecc_autotune_load")
    return n


def release_workspaces() -> None:
    """ecc_release_workspaces: frees the per-stream device scratch kept
    between calls on the current device (waits for the device first)."""
    _check(_lib.ecc_release_workspaces(), "ecc_release_workspaces")


def compute_dual(image, dtype: str):
    """ecc_compute_dual on a CUDA tensor (u8, u14): the dual complex, voxels as
    vertices with the lower-star filtration.  Returns the int64 curve."""
    return _compute_int_variant(_lib.ecc_compute_dual, "compute_dual", image, dtype)


def compute_async(image, out_chi, dtype: str, status=None, stream=None):
    """Stream-ordered ecc_compute_async on device tensors (no host synchronisation)."""
    import torch
    dims = make_dims(image.shape)
    s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream_handle(image.device)
    _check(_lib.ecc_compute_async(image.data_ptr(), ctypes.byref(dims), DTYPES[dtype], out_chi.data_ptr(),
                                  status.data_ptr() if status is not None else None, s), "ecc_compute_async")


def compute_async_noalloc(image, out_chi, dtype: str, status=None, stream=None):
    """ecc_compute_async_noalloc on device tensors: as compute_async, with the
    library's static scratch array (no allocation); calls on one GPU must not
    overlap in time."""
    dims = make_dims(image.shape)
    s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream_handle(image.device)
    _check(_lib.ecc_compute_async_noalloc(image.data_ptr(), ctypes.byref(dims), DTYPES[dtype], out_chi.data_ptr(),
                                          status.data_ptr() if status is not None else None, s),
           "ecc_compute_async_noalloc")


def compute_host(array, dtype: str):
    """ecc_compute on a host numpy array; returns a numpy int64 curve (host output buffer)."""
    import numpy as np
    a = np.ascontiguousarray(array)
    dims = make_dims(a.shape)
    m = THRESHOLDS[dtype]
    chi = np.empty(m, dtype=np.int64)
    cv = Curve(capacity=m, count=0, chi=chi.ctypes.data, keys=None)
    _check(_lib.ecc_compute(a.ctypes.data, ctypes.byref(dims), DTYPES[dtype], ctypes.byref(cv), None),
           "ecc_compute")
    return chi


class Stream:
    """ecc_stream_begin / push_chunk / finish over axis-0 chunks."""

    def __init__(self, shape, dtype: str, stream=None):
        import torch
        self.dtype = dtype
        self._h = ctypes.c_void_p()
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else (
            _stream_handle(torch.cuda.current_device()) if torch.cuda.is_available() else None)
        _check(_lib.ecc_stream_begin(ctypes.byref(make_dims(shape)), DTYPES[dtype], s, ctypes.byref(self._h)),
               "ecc_stream_begin")

    def push(self, planes, n_planes: int | None = None):
        import numpy as np
        if isinstance(planes, np.ndarray):
            planes = np.ascontiguousarray(planes)
            ptr, n = planes.ctypes.data, planes.shape[0]
        else:
            ptr, n = planes.data_ptr(), planes.shape[0]
        _check(_lib.ecc_stream_push_chunk(self._h, ptr, int(n_planes if n_planes is not None else n)),
               "ecc_stream_push_chunk")
        self._keep = planes

    def finish(self, out=None):
        import numpy as np
        m = THRESHOLDS[self.dtype]
        chi = out if out is not None else np.empty(m, dtype=np.int64)
        ptr = chi.ctypes.data if isinstance(chi, np.ndarray) else chi.data_ptr()
        cv = Curve(capacity=m, count=0, chi=ptr, keys=None)
        h, self._h = self._h, ctypes.c_void_p()
        _check(_lib.ecc_stream_finish(h, ctypes.byref(cv)), "ecc_stream_finish")
        return chi


    def snapshot(self):
        """ecc_stream_snapshot: the stream's resume state as a numpy uint8 array."""
        import numpy as np
        n = ctypes.c_int64()
        _check(_lib.ecc_stream_snapshot_size(self._h, ctypes.byref(n)), "ecc_stream_snapshot_size")
        buf = np.empty(n.value, dtype=np.uint8)
        _check(_lib.ecc_stream_snapshot(self._h, buf.ctypes.data, n.value), "ecc_stream_snapshot")
        return buf

    @classmethod
    def restore(cls, snapshot, dtype: str, stream=None):
        """ecc_stream_restore: a stream in the state of a snapshot (numpy uint8)."""
        import numpy as np
        import torch
        buf = np.ascontiguousarray(snapshot, dtype=np.uint8)
        self = cls.__new__(cls)
        self.dtype = dtype
        self._h = ctypes.c_void_p()
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else (
            _stream_handle(torch.cuda.current_device()) if torch.cuda.is_available() else None)
        _check(_lib.ecc_stream_restore(buf.ctypes.data, buf.size, s, ctypes.byref(self._h)), "ecc_stream_restore")
        return self
    def abort(self):
        h, self._h = self._h, ctypes.c_void_p()
        _lib.ecc_stream_abort(h)


def _jobs_array(images, dtypes, chis=None):
    n = len(images)
    arr = (Job * n)()
    for i, img in enumerate(images):
        arr[i].image = img.data_ptr()
        arr[i].dims = make_dims(img.shape)
        arr[i].dtype = DTYPES[dtypes[i]]
        arr[i].chi = chis[i].data_ptr() if chis is not None else None
    return arr


class Batch:
    """ecc_batch_create / run / destroy: curves of many device images per launch."""

    def __init__(self, stream=None):
        import torch
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream_handle(torch.cuda.current_device())
        self._h = ctypes.c_void_p()
        _check(_lib.ecc_batch_create(s, ctypes.byref(self._h)), "ecc_batch_create")

    def run(self, images, dtypes, chis, status=None):
        """Enqueue; images and chis are device tensors (chis int64 of m entries each)."""
        arr = _jobs_array(images, dtypes, chis)
        _check(_lib.ecc_batch_run(self._h, len(images), ctypes.cast(arr, _vp),
                                  status.data_ptr() if status is not None else None), "ecc_batch_run")

    def serve(self, images, dtypes, arrival_s, max_batch: int, one_launch_per_image: bool = False,
              max_batch_bytes: int = 0, with_batches: bool = False):
        """ecc_serve_simulate: returns (latency seconds per request, host curves
        concatenated) and, with with_batches, the batch index of each request."""
        import numpy as np
        arr = _jobs_array(images, dtypes)
        arrival = np.ascontiguousarray(arrival_s, dtype=np.float64)
        total = sum(THRESHOLDS[d] for d in dtypes)
        chi = np.empty(total, dtype=np.int64)
        lat = np.empty(len(images), dtype=np.float64)
        bid = np.empty(len(images), dtype=np.int32)
        _check(_lib.ecc_serve_simulate(self._h, len(images), ctypes.cast(arr, _vp), arrival.ctypes.data,
                                       int(max_batch), int(max_batch_bytes), int(bool(one_launch_per_image)),
                                       chi.ctypes.data, lat.ctypes.data, bid.ctypes.data), "ecc_serve_simulate")
        return (lat, chi, bid) if with_batches else (lat, chi)

    def serve_config(self, images, dtypes, arrival_s, max_batch: int = 256, one_launch_per_image: bool = False,
                     max_batch_bytes: int = 0, arena_bytes: int = 0, stream_above_bytes: int = 0,
                     chunk_bytes: int = 0, max_inflight: int = 0, check: bool = True):
        """ecc_serve.  images: device tensors, or (arena_bytes > 0) pinned host
        tensors.  Returns (latency seconds, host curves concatenated in request
        order, batch index, per-request status code, return code); with check,
        a non-zero return code raises instead."""
        import numpy as np
        arr = _jobs_array(images, dtypes)
        arrival = np.ascontiguousarray(arrival_s, dtype=np.float64)
        total = sum(THRESHOLDS[d] for d in dtypes)
        chi = np.empty(total, dtype=np.int64)
        n = len(images)
        lat = np.empty(n, dtype=np.float64)
        bid = np.empty(n, dtype=np.int32)
        st = np.empty(n, dtype=np.int32)
        cfg = ServeConfig(max_batch=int(max_batch), one_launch_per_image=int(bool(one_launch_per_image)),
                          max_batch_bytes=int(max_batch_bytes), arena_bytes=int(arena_bytes),
                          stream_above_bytes=int(stream_above_bytes), chunk_bytes=int(chunk_bytes),
                          max_inflight=int(max_inflight))
        rc = _lib.ecc_serve(self._h, n, ctypes.cast(arr, _vp), arrival.ctypes.data, ctypes.byref(cfg),
                            chi.ctypes.data, lat.ctypes.data, bid.ctypes.data, st.ctypes.data)
        if check:
            _check(rc, "ecc_serve")
        return lat, chi, bid, st, rc

    def autotune(self, images, dtypes, chis):
        """ecc_batch_autotune: picks the context's tile depth on this batch;
        returns (min_planes, split, ms)."""
        arr = _jobs_array(images, dtypes, chis)
        mp, sp, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_float(0)
        _check(_lib.ecc_batch_autotune(self._h, len(images), ctypes.cast(arr, _vp), ctypes.byref(mp),
                                       ctypes.byref(sp), ctypes.byref(ms)), "ecc_batch_autotune")
        return mp.value, sp.value, ms.value

    @staticmethod
    def footprint(image, dtype: str) -> int:
        """ecc_job_footprint of one request (bytes)."""
        arr = _jobs_array([image], [dtype])
        out = ctypes.c_int64(0)
        _check(_lib.ecc_job_footprint(ctypes.cast(arr, _vp), ctypes.byref(out)), "ecc_job_footprint")
        return out.value

    def close(self):
        h, self._h = self._h, ctypes.c_void_p()
        if h:
            _lib.ecc_batch_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
