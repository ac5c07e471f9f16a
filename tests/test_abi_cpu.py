"""The C-ABI library loads without a GPU, exports every symbol include/ecc.h
declares, and rejects bad arguments before touching the device."""
import ctypes
import pathlib
import re

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]


def declared_functions():
    text = (ROOT / "include" / "ecc.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ecc_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    import paper_1705_02045_amd as ecc
    lib = ctypes.CDLL(ecc.library_path())
    names = declared_functions()
    assert "ecc_compute" in names and "ecc_stream_push_chunk" in names
    for name in names:
        assert hasattr(lib, name), name


def test_threshold_counts_and_version():
    import paper_1705_02045_amd as ecc
    m = ctypes.c_int64()
    for name, want in ecc.THRESHOLDS.items():
        assert ecc._lib.ecc_threshold_count(ecc.DTYPES[name], ctypes.byref(m)) == 0 and m.value == want
    assert ecc._lib.ecc_threshold_count(ecc.DTYPES["f32"], ctypes.byref(m)) == ecc.ECC_E_ARG
    assert "gfx950" in ecc.version()


@pytest.mark.parametrize("shape", [(), (0,), (3, 0), (1, 2, 3, 4, 5)])
def test_bad_dims_rejected(shape):
    import paper_1705_02045_amd as ecc
    dims = ecc.make_dims(shape[:4]) if shape else ecc.Dims()
    if len(shape) == 5:
        dims.ndim = 5
    buf = (ctypes.c_int64 * 16384)()
    cv = ecc.Curve(capacity=16384, count=0, chi=ctypes.addressof(buf), keys=None)
    rc = ecc._lib.ecc_compute(ctypes.addressof(buf), ctypes.byref(dims), ecc.DTYPES["u14"], ctypes.byref(cv), None)
    assert rc == ecc.ECC_E_ARG
    assert ecc._lib.ecc_last_error()


def test_null_and_dtype_rejected():
    import paper_1705_02045_amd as ecc
    dims = ecc.make_dims((4, 4))
    buf = (ctypes.c_int64 * 256)()
    cv = ecc.Curve(capacity=256, count=0, chi=ctypes.addressof(buf), keys=None)
    assert ecc._lib.ecc_compute(None, ctypes.byref(dims), 1, ctypes.byref(cv), None) == ecc.ECC_E_ARG
    assert ecc._lib.ecc_compute(ctypes.addressof(buf), ctypes.byref(dims), 9, ctypes.byref(cv), None) == ecc.ECC_E_ARG
    assert ecc._lib.ecc_compute(ctypes.addressof(buf), None, 1, ctypes.byref(cv), None) == ecc.ECC_E_ARG


def test_small_capacity_reports_needed_size():
    import paper_1705_02045_amd as ecc
    dims = ecc.make_dims((4, 4))
    buf = (ctypes.c_int64 * 16)()
    cv = ecc.Curve(capacity=16, count=0, chi=ctypes.addressof(buf), keys=None)
    rc = ecc._lib.ecc_compute(ctypes.addressof(buf), ctypes.byref(dims), ecc.DTYPES["u8"], ctypes.byref(cv), None)
    assert rc == ecc.ECC_E_BUFFER_TOO_SMALL and cv.count == 256


def test_stream_argument_errors():
    import paper_1705_02045_amd as ecc
    h = ctypes.c_void_p()
    dims = ecc.make_dims((4, 5, 6))
    assert ecc._lib.ecc_stream_begin(None, ecc.DTYPES["u14"], None, ctypes.byref(h)) == ecc.ECC_E_ARG
    assert ecc._lib.ecc_stream_begin(ctypes.byref(dims), 9, None, ctypes.byref(h)) == ecc.ECC_E_ARG
    bad = ecc.make_dims((4, 0, 6))
    assert ecc._lib.ecc_stream_begin(ctypes.byref(bad), ecc.DTYPES["u8"], None, ctypes.byref(h)) == ecc.ECC_E_ARG
    assert ecc._lib.ecc_stream_push_chunk(None, None, 1) == ecc.ECC_E_ARG
    assert ecc._lib.ecc_stream_finish(None, None) == ecc.ECC_E_ARG
    ecc._lib.ecc_stream_abort(None)


def test_batch_argument_errors():
    import paper_1705_02045_amd as ecc
    assert ecc._lib.ecc_batch_create(None, None) == ecc.ECC_E_ARG
    assert ecc._lib.ecc_batch_run(None, 1, None, None) == ecc.ECC_E_ARG
    lat = (ctypes.c_double * 1)()
    arr = (ctypes.c_double * 1)()
    chi = (ctypes.c_int64 * 256)()
    assert ecc._lib.ecc_serve_simulate(None, 1, None, arr, 1, 0, 0, chi, lat, None) == ecc.ECC_E_ARG
    ecc._lib.ecc_batch_destroy(None)


def test_job_footprint():
    """Host-side sizing of a request: image bytes + count rows + changes
    vector + curve; larger images need more; no GPU involved."""
    import paper_1705_02045_amd as ecc

    def fp(shape, dtype):
        job = ecc.Job()
        job.dims = ecc.make_dims(shape)
        job.dtype = ecc.DTYPES[dtype]
        out = ctypes.c_int64(0)
        rc = ecc._lib.ecc_job_footprint(ctypes.byref(job), ctypes.byref(out))
        return rc, out.value

    rc, a = fp((300, 70), "u8")
    assert rc == 0 and a >= 300 * 70 + 2 * 256 * 8 + 256 * 4
    rc, b = fp((600, 700), "u8")
    assert rc == 0 and b > a
    rc, c = fp((16, 16, 16), "u14")
    assert rc == 0 and c >= 2 * 16 ** 3 + 2 * 16384 * 8 + 16384 * 4
    rc, w = fp((4, 4), "u16")  # count rows of 16384 bins (one window), 65536-entry changes vector and curve
    assert rc == 0 and w >= 2 * 16 + 16384 * 4 + 2 * 65536 * 8
    assert fp((4, 4), "f32")[0] == ecc.ECC_E_UNSUPPORTED
    assert ecc._lib.ecc_job_footprint(None, None) == ecc.ECC_E_ARG


def test_job_struct_layout():
    import paper_1705_02045_amd as ecc
    # image, dims (int32 + pad + 4 x int64), dtype (+ pad), chi
    assert ctypes.sizeof(ecc.Job) == 8 + 40 + 8 + 8
    assert ecc.Job.chi.offset == 56


def test_autotune_cache_save_and_load(tmp_path):
    """The tuning cache as a text file: entries load into the table that
    ecc_tiling_for reads, save writes them back, a malformed file stores
    nothing (no GPU is needed for any of it)."""
    import paper_1705_02045_amd as ecc
    ecc.autotune_reset()
    shape = (1024, 1024, 1024)
    rule = ecc.tiling_for(shape, "u14")
    assert ecc.autotune_save(tmp_path / "empty.txt") == 0 and (tmp_path / "empty.txt").read_text() == ""
    cache = tmp_path / "tiling.txt"
    cache.write_text("# tuned on one MI355X\n"
                     "ecc-tiling-v1 2 2 1024 1024 1024 4 8 8 0.61\n"
                     "\n"
                     "ecc-tiling-v1 1 1 1 300 70 2 16 16 0.01\n")
    assert ecc.autotune_load(cache) == 2
    assert ecc.tiling_for(shape, "u14") == {"rows": 4, "tiles_per_cu": 8, "waves_x": 8}
    assert ecc.tiling_for((70, 300), "u8") == {"rows": 2, "tiles_per_cu": 16, "waves_x": 16}
    out = tmp_path / "saved.txt"
    assert ecc.autotune_save(out) == 2
    assert sorted(out.read_text().split("\n")) == sorted(
        ["ecc-tiling-v1 1 1 1 300 70 2 16 16 0.01", "ecc-tiling-v1 2 2 1024 1024 1024 4 8 8 0.61", ""])
    ecc.autotune_reset()
    assert ecc.tiling_for(shape, "u14") == rule
    for bad in ["ecc-tiling-v1 2 2 1024 1024 1024 3 8 8 0.61\n",          # rows 3
                "ecc-tiling-v1 2 2 1024 1024 1024 4 8 8\n",               # a field missing
                "ecc-tiling-v1 2 2 1024 1024 1024 4 8 8 0.61 extra\n",    # one too many
                "ecc-tiling-v2 2 2 1024 1024 1024 4 8 8 0.61\n",          # unknown tag
                "ecc-tiling-v1 4 2 1024 1024 1024 4 8 8 0.61\n",          # float32: no integer tiling
                "ecc-tiling-v1 2 2 1024 1024 1024 4 8 8 0.61\ngarbage\n"]:
        cache.write_text(bad)
        with pytest.raises(ecc.EccError) as ei:
            ecc.autotune_load(cache)
        assert ei.value.code == ecc.ECC_E_ARG
        assert ecc.tiling_for(shape, "u14") == rule  # nothing stored
    with pytest.raises(ecc.EccError):
        ecc.autotune_load(tmp_path / "missing.txt")


def test_stream_restore_rejects_non_snapshots():
    """Checked before any device work: too short, wrong magic."""
    import ctypes
    import numpy as np
    import paper_1705_02045_amd as ecc
    h = ctypes.c_void_p()
    for buf in (np.zeros(8, dtype=np.uint8), np.zeros(200, dtype=np.uint8)):
        rc = ecc._lib.ecc_stream_restore(buf.ctypes.data, buf.size, None, ctypes.byref(h))
        assert rc == ecc.ECC_E_ARG and not h.value
    assert ecc._lib.ecc_stream_restore(None, 0, None, ctypes.byref(h)) == ecc.ECC_E_ARG
