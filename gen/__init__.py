"""Seeded synthetic inputs shared by the CPU oracle (tests) and the GPU benchmarks.

This package only makes input bytes: it holds none of the Euler-characteristic
arithmetic.  The definitions (SplitMix64-based counter hash, i.i.d. values,
integer value noise, float value noise with Gaussian jitter) are stated in
``eccgen_host.c``.  ``libeccgen.so`` is the fast threaded implementation; the
``*_np`` functions restate the same definitions in numpy for small sizes and
exist so that tests can check the C library against a second implementation.
"""
from __future__ import annotations

import ctypes
import os
import pathlib

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
_LIB = None
GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(n, 16))


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        path = _HERE / "libeccgen.so"
        if not path.exists():
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(str(path))
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.eccgen_hash.restype = ctypes.c_uint64
        L.eccgen_hash.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        L.eccgen_iid.restype = ctypes.c_int
        L.eccgen_iid.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        L.eccgen_value_noise.restype = ctypes.c_int
        L.eccgen_value_noise.argtypes = [ctypes.c_uint64, ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.c_int]
        L.eccgen_value_noise_voxelwise.restype = ctypes.c_int
        L.eccgen_value_noise_voxelwise.argtypes = L.eccgen_value_noise.argtypes
        L.eccgen_value_noise_f32.restype = ctypes.c_int
        L.eccgen_value_noise_f32.argtypes = [ctypes.c_uint64, ctypes.c_int, i64p, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_int]
        _LIB = L
    return _LIB


def _dims(shape):
    arr = (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])
    return arr


# ----------------------------------------------------------------- C-backed
def iid(shape, bits: int, seed: int, dtype=None, nthreads: int | None = None) -> np.ndarray:
    """i.i.d. values h(seed, 0, i) >> (64 - bits) in C order."""
    dtype = np.dtype(dtype or (np.uint8 if bits <= 8 else np.uint16))
    out = np.empty(tuple(int(s) for s in shape), dtype=dtype)
    rc = lib().eccgen_iid(seed, bits, 0, out.size, out.ctypes.data, dtype.itemsize, nthreads or _threads())
    if rc:
        raise ValueError("eccgen_iid: bad arguments")
    return out


def value_noise(shape, bits: int, amp: int, seed: int, lshift: int = 4, z0: int = 0, z1: int | None = None,
                dtype=None, nthreads: int | None = None) -> np.ndarray:
    """Integer value noise (lattice 2**lshift, +-amp jitter) for planes [z0, z1) of axis 0."""
    shape = tuple(int(s) for s in shape)
    z1 = shape[0] if z1 is None else z1
    dtype = np.dtype(dtype or (np.uint8 if bits <= 8 else np.uint16))
    out = np.empty((z1 - z0,) + shape[1:], dtype=dtype)
    rc = lib().eccgen_value_noise(seed, len(shape), _dims(shape), lshift, bits, amp, z0, z1,
                                  out.ctypes.data, dtype.itemsize, nthreads or _threads())
    if rc:
        raise ValueError("eccgen_value_noise: bad arguments")
    return out


def value_noise_f32(shape, sigma: float, seed: int, lshift: int = 3, z0: int = 0, z1: int | None = None,
                    nthreads: int | None = None) -> np.ndarray:
    shape = tuple(int(s) for s in shape)
    z1 = shape[0] if z1 is None else z1
    out = np.empty((z1 - z0,) + shape[1:], dtype=np.float32)
    rc = lib().eccgen_value_noise_f32(seed, len(shape), _dims(shape), lshift, float(sigma), z0, z1,
                                      out.ctypes.data, nthreads or _threads())
    if rc:
        raise ValueError("eccgen_value_noise_f32: bad arguments")
    return out


# ------------------------------------------------------ device generator
_DEV = None


def dev_lib() -> ctypes.CDLL:
    """libeccgen_dev.so: the integer value noise made in device memory (same bytes)."""
    global _DEV
    if _DEV is None:
        path = _HERE / "libeccgen_dev.so"
        if not path.exists():
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(str(path))
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.eccgen_dev_table_entries.restype = ctypes.c_int
        L.eccgen_dev_table_entries.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                               i64p]
        L.eccgen_dev_value_noise.restype = ctypes.c_int
        L.eccgen_dev_value_noise.argtypes = [ctypes.c_uint64, ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        _DEV = L
    return _DEV


def dev_table_entries(shape, z0: int, z1: int, lshift: int = 4) -> int:
    """uint16 entries of the lattice table for planes [z0, z1) of a 3-D image."""
    n = ctypes.c_int64(0)
    if dev_lib().eccgen_dev_table_entries(len(shape), _dims(shape), lshift, z0, z1, ctypes.byref(n)):
        raise ValueError("eccgen_dev_table_entries: bad arguments")
    return n.value


def value_noise_dev(out_ptr: int, shape, bits: int, amp: int, seed: int, z0: int, z1: int, table_ptr: int,
                    table_entries: int, lshift: int = 4, elem: int = 2, stream: int = 0) -> None:
    """Enqueues planes [z0, z1) of the 3-D integer value noise into device
    memory at out_ptr (the bytes value_noise() makes), on HIP stream `stream`."""
    rc = dev_lib().eccgen_dev_value_noise(seed, len(shape), _dims(shape), lshift, bits, amp, z0, z1, out_ptr, elem,
                                          table_ptr, table_entries, stream or None)
    if rc:
        raise ValueError(f"eccgen_dev_value_noise failed ({rc})")


def cfg_u14_value_noise_dev(out_ptr: int, shape, seed: int, z0: int, z1: int, table_ptr: int, table_entries: int,
                            stream: int = 0) -> None:
    """Device-made planes [z0, z1) of cfg_u14_value_noise(shape, seed)."""
    value_noise_dev(out_ptr, shape, 14, 64, seed, z0, z1, table_ptr, table_entries, lshift=4, elem=2, stream=stream)


# ------------------------------------------------------ numpy restatements
def mix64_np(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def key_np(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        return mix64_np(np.uint64(seed) * GAMMA + np.uint64(stream))


def hash_np(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    k = key_np(seed, stream)
    with np.errstate(over="ignore"):
        return mix64_np(k + (np.asarray(idx, dtype=np.uint64) + np.uint64(1)) * GAMMA)


def iid_np(shape, bits: int, seed: int) -> np.ndarray:
    n = int(np.prod(shape))
    v = hash_np(seed, 0, np.arange(n, dtype=np.uint64)) >> np.uint64(64 - bits)
    return v.reshape(shape).astype(np.uint8 if bits <= 8 else np.uint16)


def _corners(d):
    for corner in range(1 << d):
        yield [(corner >> (d - 1 - k)) & 1 for k in range(d)]


def value_noise_np(shape, bits: int, amp: int, seed: int, lshift: int = 4) -> np.ndarray:
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    L = 1 << lshift
    N = [((s - 1) >> lshift) + 2 for s in shape]
    coords = np.indices(shape).reshape(d, -1).astype(np.int64)
    base = coords >> lshift
    r = coords & (L - 1)
    acc = np.zeros(coords.shape[1], dtype=np.uint64)
    for bitsv in _corners(d):
        node = np.zeros(coords.shape[1], dtype=np.int64)
        w = np.ones(coords.shape[1], dtype=np.uint64)
        for k in range(d):
            node = node * N[k] + base[k] + bitsv[k]
            w = w * (r[k] if bitsv[k] else (L - r[k])).astype(np.uint64)
        u = hash_np(seed, 1, node.astype(np.uint64)) >> np.uint64(64 - bits)
        acc = acc + u * w
    bv = ((acc + np.uint64(1 << (d * lshift - 1))) >> np.uint64(d * lshift)).astype(np.int64)
    hj = hash_np(seed, 2, np.arange(coords.shape[1], dtype=np.uint64))
    jit = (((hj >> np.uint64(32)) * np.uint64(2 * amp + 1)) >> np.uint64(32)).astype(np.int64) - amp
    v = np.clip(bv + jit, 0, (1 << bits) - 1)
    return v.reshape(shape).astype(np.uint8 if bits <= 8 else np.uint16)


def value_noise_f32_np(shape, sigma: float, seed: int, lshift: int = 3) -> np.ndarray:
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    L = 1 << lshift
    N = [((s - 1) >> lshift) + 2 for s in shape]
    coords = np.indices(shape).reshape(d, -1).astype(np.int64)
    base = coords >> lshift
    r = coords & (L - 1)
    acc = np.zeros(coords.shape[1], dtype=np.float64)
    for bitsv in _corners(d):
        node = np.zeros(coords.shape[1], dtype=np.int64)
        w = np.ones(coords.shape[1], dtype=np.float64)
        for k in range(d):
            node = node * N[k] + base[k] + bitsv[k]
            w = w * ((r[k] / L) if bitsv[k] else ((L - r[k]) / L))
        u = (hash_np(seed, 1, node.astype(np.uint64)) >> np.uint64(40)).astype(np.float64)
        acc = acc + u * (1.0 / 16777216.0) * w
    hj = hash_np(seed, 2, np.arange(coords.shape[1], dtype=np.uint64))
    u1 = ((hj >> np.uint64(32)).astype(np.float64) + 1.0) * (1.0 / 4294967296.0)
    u2 = (hj & np.uint64(0xFFFFFFFF)).astype(np.float64) * (1.0 / 4294967296.0)
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(6.283185307179586 * u2)
    return (acc + sigma * z).astype(np.float32).reshape(shape)


# ------------------------------------------------------- named workloads
def cfg_2d_u8_iid(shape=(256, 256), seed: int = 0) -> np.ndarray:
    """2-D uint8, i.i.d. uniform 0..255 (seed 0 for the 256x256 case)."""
    return iid(shape, 8, seed)


def cfg_u14_value_noise(shape=(1024, 1024, 1024), seed: int = 1, **kw) -> np.ndarray:
    """14-bit value noise stored as uint16: lattice 16, lattice values 0..16383, jitter +-64."""
    return value_noise(shape, 14, 64, seed, lshift=4, **kw)


def cfg_u8_value_noise(shape, seed: int) -> np.ndarray:
    """8-bit value noise: lattice 16, lattice values 0..255, jitter +-1 (the 14-bit jitter scaled by 256/16384)."""
    return value_noise(shape, 8, 1, seed, lshift=4)


def cfg_f32_value_noise(shape=(128, 128, 128, 128), seed: int = 3, sigma: float = 0.01, **kw) -> np.ndarray:
    """float32 value noise: lattice 8, values in [0,1), Gaussian jitter of standard deviation sigma."""
    return value_noise_f32(shape, sigma, seed, lshift=3, **kw)


def serving_requests(count: int, seed: int = 4, side_scale: float = 1.0):
    """Mixed request stream: request i draws h = hash(seed, 3, i); the low bit
    picks 2-D uint8 value noise (sides uniform in 32..2048) or 3-D 14-bit value
    noise (sides uniform in 16..256); further 16-bit fields of h pick the
    sides, and the request's image seed is h >> 32.  side_scale < 1 shrinks the
    side ranges proportionally (small test streams).  Returns a list of
    (dtype, shape, image_seed)."""
    h = hash_np(seed, 3, np.arange(count, dtype=np.uint64))
    out = []
    for i in range(count):
        v = int(h[i])
        f = [(v >> (8 + 16 * k)) & 0xFFFF for k in range(3)]
        if v & 1:
            lo, hi = 16, max(16, int(256 * side_scale))
            shape = tuple(lo + (x * (hi - lo + 1) >> 16) for x in f)
            out.append(("u14", shape, v >> 32))
        else:
            lo, hi = 32, max(32, int(2048 * side_scale))
            shape = tuple(lo + (x * (hi - lo + 1) >> 16) for x in f[:2])
            out.append(("u8", shape, v >> 32))
    return out


def serving_image(dtype: str, shape, image_seed: int) -> np.ndarray:
    """The image of one serving request (see serving_requests)."""
    if dtype == "u14":
        return cfg_u14_value_noise(shape, seed=image_seed)
    return cfg_u8_value_noise(shape, seed=image_seed)
