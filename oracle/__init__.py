"""ORACLE -- test infrastructure only.

Plain CPU computation of the Euler characteristic curve (ECC) of a gray-scale
image, from the definitions in Section 2 of Heiss & Wagner (arXiv 1705.02045):
every cell of the image's cubical complex is enumerated, its value is the
minimum over the voxels that contain it (sublevel set filtration), and
(-1)^dim is added at that value; the curve is the prefix sum (Section 3,
"Tracking the Changes" and "Post-Processing").  The cell loop is plain C
(``ecc_oracle.c``); this module binds it and adds the floating-point reading.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this package.  The GPU library never imports it.

``curve_max_entry`` computes the other convention for a cell's value, the
maximum over its voxels (the literal "largest gray value" reading), by the
same cell enumeration.  ``curve_dual`` enumerates the dual complex (voxels as
vertices, each cell at the maximum over its vertices).

Floating-point images (Section 3, "Other Ranges of Gray Values"): the curve is
a step function over the distinct values.  NaN is rejected; -0.0 and +0.0 are
one value (IEEE equality).  The output lists every distinct value in ascending
order with chi(T_v) right after v is included.  It is computed by replacing
each value with its rank among the distinct values (``numpy.unique``) and
running the integer computation with m = number of distinct values; a strictly
increasing relabelling commutes with taking minima, so cell values map to the
ranks of their values (the transform statement at the end of Section 3).
"""
from __future__ import annotations

import ctypes
import os
import pathlib

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        path = _HERE / "liboracle.so"
        if not path.exists():
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(str(path))
        i64p = ctypes.POINTER(ctypes.c_int64)
        for name in ("oracle_vcec", "oracle_curve", "oracle_curve_max", "oracle_curve_dual"):
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, i64p, ctypes.c_int64,
                           i64p, ctypes.c_int, ctypes.c_int64]
        L.oracle_vcec_range.restype = ctypes.c_int
        L.oracle_vcec_range.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, i64p, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int64, i64p]
        L.oracle_vcec3.restype = ctypes.c_int
        L.oracle_vcec3.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int64, i64p, ctypes.c_int]
        _LIB = L
    return _LIB


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


_ELEM = {np.dtype(np.uint8): 1, np.dtype(np.uint16): 2, np.dtype(np.uint32): 4}
DEFAULT_M = {np.dtype(np.uint8): 256, np.dtype(np.uint16): 65536}


def _prep(img: np.ndarray):
    img = np.ascontiguousarray(img)
    if img.dtype not in _ELEM:
        raise TypeError(f"oracle: unsupported dtype {img.dtype}")
    if img.ndim < 1 or img.size == 0:
        raise ValueError("oracle: empty image")
    dims = (ctypes.c_int64 * img.ndim)(*img.shape)
    return img, dims


def _check(rc: int):
    if rc == -2:
        raise ValueError("oracle: a value is >= m")
    if rc:
        raise RuntimeError(f"oracle failed ({rc})")


def vcec(img: np.ndarray, m: int | None = None, nthreads: int | None = None,
         max_bytes: int = 8 << 30) -> np.ndarray:
    """a_t = signed number of cells whose value is t, t = 0..m-1 (int64)."""
    img, dims = _prep(img)
    m = int(m if m is not None else DEFAULT_M[img.dtype])
    out = np.zeros(m, dtype=np.int64)
    rc = lib().oracle_vcec(img.ctypes.data, _ELEM[img.dtype], img.ndim, dims, m,
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           nthreads or default_threads(), max_bytes)
    _check(rc)
    return out


def curve(img: np.ndarray, m: int | None = None, nthreads: int | None = None,
          max_bytes: int = 8 << 30) -> np.ndarray:
    """chi(T_t) for t = 0..m-1 (int64).  m defaults to 256 for uint8 and 65536 for uint16."""
    img, dims = _prep(img)
    m = int(m if m is not None else DEFAULT_M[img.dtype])
    out = np.zeros(m, dtype=np.int64)
    rc = lib().oracle_curve(img.ctypes.data, _ELEM[img.dtype], img.ndim, dims, m,
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            nthreads or default_threads(), max_bytes)
    _check(rc)
    return out


def curve_max_entry(img: np.ndarray, m: int | None = None, nthreads: int | None = None,
                    max_bytes: int = 8 << 30) -> np.ndarray:
    """The "largest value" convention: each cell's value is the maximum of f
    over the voxels containing it; returns sum_{c: value(c) <= t} (-1)^dim c
    for t = 0..m-1 (int64).  These cell sets are not complexes."""
    img, dims = _prep(img)
    m = int(m if m is not None else DEFAULT_M[img.dtype])
    out = np.zeros(m, dtype=np.int64)
    rc = lib().oracle_curve_max(img.ctypes.data, _ELEM[img.dtype], img.ndim, dims, m,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                nthreads or default_threads(), max_bytes)
    _check(rc)
    return out


def curve_dual(img: np.ndarray, m: int | None = None, nthreads: int | None = None,
               max_bytes: int = 8 << 30) -> np.ndarray:
    """The dual complex (voxels as vertices, edges between voxels sharing a
    (d-1)-face, squares and cubes of such neighbours): every cell enters at
    the maximum over its vertices.  chi(T_t) for t = 0..m-1 (int64)."""
    img, dims = _prep(img)
    m = int(m if m is not None else DEFAULT_M[img.dtype])
    out = np.zeros(m, dtype=np.int64)
    rc = lib().oracle_curve_dual(img.ctypes.data, _ELEM[img.dtype], img.ndim, dims, m,
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 nthreads or default_threads(), max_bytes)
    _check(rc)
    return out


def vcec_q0_range(img: np.ndarray, m: int, q0_lo: int, q0_hi: int) -> np.ndarray:
    """Signed counts of the cells whose doubled first coordinate is in [q0_lo, q0_hi)."""
    img, dims = _prep(img)
    out = np.zeros(int(m), dtype=np.int64)
    rc = lib().oracle_vcec_range(img.ctypes.data, _ELEM[img.dtype], img.ndim, dims, int(m),
                                 int(q0_lo), int(q0_hi), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    _check(rc)
    return out


def vcec3_q0_range(img: np.ndarray, m: int, q0_lo: int, q0_hi: int, nthreads: int | None = None) -> np.ndarray:
    """vcec_q0_range for a 3-D image, by the three-loop enumeration
    (``oracle_vcec3``), on up to nthreads threads."""
    img, dims = _prep(img)
    if img.ndim != 3:
        raise ValueError("oracle: vcec3_q0_range takes 3-D images")
    out = np.zeros(int(m), dtype=np.int64)
    rc = lib().oracle_vcec3(img.ctypes.data, _ELEM[img.dtype], dims, int(m), int(q0_lo), int(q0_hi),
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nthreads or default_threads())
    _check(rc)
    return out


def canonical_float(img: np.ndarray) -> np.ndarray:
    """float32 copy with -0.0 replaced by +0.0; raises on NaN."""
    a = np.ascontiguousarray(img, dtype=np.float32)
    if np.isnan(a).any():
        raise ValueError("oracle: NaN in a float image")
    a = a + np.float32(0.0)  # -0.0 + 0.0 == +0.0 in round-to-nearest
    return a


def curve_float(img: np.ndarray, nthreads: int | None = None, max_bytes: int = 32 << 30):
    """(keys, chi): keys = ascending distinct values, chi[k] = chi(T_{keys[k]})."""
    a = canonical_float(img)
    keys, ranks = np.unique(a.ravel(), return_inverse=True)
    ranks = ranks.astype(np.uint32).reshape(a.shape)
    chi = curve(ranks, m=len(keys), nthreads=nthreads, max_bytes=max_bytes)
    return keys.astype(np.float32), chi
