"""GPU parity of the float32 path through the C ABI: keys (distinct values,
ascending, -0 folded into +0) and chi must equal the oracle's exactly."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ecc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1705_02045_amd as ecc
    return ecc


def gpu_float(ecc, img):
    t = torch.from_numpy(np.ascontiguousarray(img, dtype=np.float32)).cuda()
    keys, chi = ecc.compute(t, dtype="f32")
    return keys.cpu().numpy(), chi.cpu().numpy()


def check(ecc, img):
    rk, rc = oracle.curve_float(img)
    gk, gc = gpu_float(ecc, img)
    assert len(gk) == len(rk), f"shape {img.shape}: {len(gk)} keys, want {len(rk)}"
    # keys compared as bit patterns: -0 must come back as +0
    assert (gk.view(np.uint32) == rk.view(np.uint32)).all(), f"shape {img.shape}: keys differ"
    if not (gc == rc).all():
        bad = np.nonzero(gc != rc)[0]
        raise AssertionError(f"shape {img.shape}: {len(bad)} values differ, first {bad[:5]} "
                             f"got {gc[bad[:5]]} want {rc[bad[:5]]}")


SHAPES = [(1,), (2,), (7,), (300,), (1, 1), (5, 9), (64, 65), (2, 200), (33, 2, 70), (9, 17, 129),
          (3, 1, 70), (5, 6, 7, 8), (3, 1, 70, 4), (12, 12, 12, 12), (2, 3, 300, 5), (1, 1, 1, 1)]


@pytest.mark.parametrize("shape", SHAPES, ids=[str(s) for s in SHAPES])
def test_float_value_noise(ecc, shape):
    check(ecc, gen.value_noise_f32(shape, sigma=0.01, seed=11))


@pytest.mark.parametrize("shape", [(40, 50), (6, 7, 70), (4, 5, 6, 70)])
def test_float_many_ties(ecc, shape):
    # values on a coarse grid: long runs of equal keys across records
    img = np.round(gen.value_noise_f32(shape, sigma=0.05, seed=12) * 8) / 8
    check(ecc, img.astype(np.float32))


@pytest.mark.parametrize("shape,levels", [((40, 60, 80), 4), ((300, 700), 3), ((9, 10, 11, 120), 5),
                                          ((50, 50, 50), 1)], ids=str)
def test_float_few_values_long_slices(ecc, shape, levels):
    """A handful of values over 10^5 voxels: one sorted-key tile owns each
    value, with thousands of non-zero records each (more than a tile keeps
    in LDS), and a constant image (one key, chi = 1)."""
    rng = np.random.default_rng(13)
    img = rng.integers(0, levels, size=shape).astype(np.float32) * np.float32(0.75)
    check(ecc, img)


@pytest.mark.parametrize("shape", [(40, 40, 40, 40), (120, 130, 140)], ids=str)
def test_float_iid_noise_dense_records(ecc, shape):
    """Independent uniform values: critical points everywhere, so a tile of
    sorted keys owns hundreds to thousands of non-zero records (the long-slice
    launch, from LDS)."""
    img = np.random.default_rng(14).random(shape, dtype=np.float32)
    check(ecc, img)


def test_float_signed_zero_and_infinities(ecc):
    rng = np.random.default_rng(3)
    img = rng.choice(np.array([-0.0, 0.0, 1.5, -2.0, np.inf, -np.inf], dtype=np.float32), size=(9, 11, 70))
    check(ecc, img)
    gk, _ = gpu_float(ecc, img)
    assert not np.signbit(gk[gk == 0]).any()


def test_float_equals_integer_curve_at_present_values(ecc):
    # a strictly increasing relabelling of the values re-indexes the curve
    img = gen.cfg_u8_value_noise((20, 30, 70), seed=4)
    gk, gc = gpu_float(ecc, img.astype(np.float32))
    ref = oracle.curve(img, m=256)
    assert (gk == np.unique(img).astype(np.float32)).all()
    assert (gc == ref[np.unique(img)]).all()


def test_float_nan_rejected(ecc):
    img = gen.value_noise_f32((5, 6, 70), sigma=0.01, seed=1)
    img[3, 2, 69] = np.nan
    with pytest.raises(ecc.EccError) as e:
        gpu_float(ecc, img)
    assert e.value.code == ecc.ECC_E_NAN
    # the device status is clear again: a valid image works afterwards
    check(ecc, gen.value_noise_f32((5, 6, 70), sigma=0.01, seed=1))


def test_float_capacity_too_small(ecc):
    import ctypes
    img = gen.value_noise_f32((8, 70), sigma=0.01, seed=2)
    k = len(np.unique(img))
    t = torch.from_numpy(img).cuda()
    chi = torch.empty(k - 1, dtype=torch.int64, device="cuda")
    keys = torch.empty(k - 1, dtype=torch.float32, device="cuda")
    cv = ecc.Curve(capacity=k - 1, count=0, chi=chi.data_ptr(), keys=keys.data_ptr())
    rc = ecc._lib.ecc_compute(t.data_ptr(), ctypes.byref(ecc.make_dims(img.shape)), ecc.DTYPES["f32"],
                              ctypes.byref(cv), None)
    assert rc == ecc.ECC_E_BUFFER_TOO_SMALL and cv.count == k
    # enough room, host output buffers
    hk = np.empty(k, dtype=np.float32)
    hc = np.empty(k, dtype=np.int64)
    cv = ecc.Curve(capacity=k, count=0, chi=hc.ctypes.data, keys=hk.ctypes.data)
    rc = ecc._lib.ecc_compute(t.data_ptr(), ctypes.byref(ecc.make_dims(img.shape)), ecc.DTYPES["f32"],
                              ctypes.byref(cv), None)
    assert rc == ecc.ECC_OK and cv.count == k
    rk, rcv = oracle.curve_float(img)
    assert (hk == rk).all() and (hc == rcv).all()


def test_float_host_image(ecc):
    import ctypes
    img = gen.value_noise_f32((6, 40, 70), sigma=0.01, seed=6)
    n = img.size
    hk = np.empty(n, dtype=np.float32)
    hc = np.empty(n, dtype=np.int64)
    cv = ecc.Curve(capacity=n, count=0, chi=hc.ctypes.data, keys=hk.ctypes.data)
    rc = ecc._lib.ecc_compute(img.ctypes.data, ctypes.byref(ecc.make_dims(img.shape)), ecc.DTYPES["f32"],
                              ctypes.byref(cv), None)
    assert rc == ecc.ECC_OK
    rk, rcv = oracle.curve_float(img)
    assert cv.count == len(rk) and (hk[: cv.count] == rk).all() and (hc[: cv.count] == rcv).all()


def test_float_4d_full_size(ecc):
    # the 4-D 128^4 value-noise workload, compared in full
    img = gen.cfg_f32_value_noise((128, 128, 128, 128), seed=3)
    check(ecc, img)


def _top_bytes(img):
    """Top bytes of the order-preserving 32-bit keys of a float image (-0
    taken as +0): negative values complement all bits, others set the sign."""
    b = np.where(img == 0, np.float32(0), img).astype(np.float32).view(np.uint32)
    key = np.where(b >> 31 != 0, ~b, b | np.uint32(0x80000000))
    return np.unique(key >> 24)


# (number of sign and binade-pair groups, shape): after two passes on bits
# 0-17 the key sort joins bits 18-23 to the rank of the top byte when at most
# 16 top bytes occur (a 9-bit digit up to 8 of them, a 10-bit one up to 16),
# and takes two 7-bit passes otherwise; the shapes span several 8192-key
# tiles with a ragged last one, and one image fills a single partial tile
PLANS = [(8, (5, 8192 * 2 + 77)), (9, (5, 8192 * 2 + 77)), (16, (5, 8192 * 2 + 77)), (17, (5, 8192 * 2 + 77)),
         (1, (3, 7, 500)), (8, (11, 300)), (40, (4, 9, 1100)), (9, (3, 4, 5, 300)), (16, (6, 7, 8, 9))]


@pytest.mark.parametrize("groups,shape", PLANS, ids=[f"{g}-{s}" for g, s in PLANS])
def test_float_key_sort_plans(ecc, groups, shape):
    """Value noise with each voxel moved to one of `groups` sign and binade
    pairs at random: exactly `groups` distinct top bytes of the keys."""
    rng = np.random.default_rng(40 + groups)
    base = gen.value_noise_f32(shape, sigma=0.0, seed=21)
    base = (np.float32(1) + np.clip(base, 0, np.float32(0.999)))  # in [1, 2): exponent 127
    g = rng.integers(0, groups, size=shape)
    # group i: sign (-1)^i, exponent 127 + 2 (i // 2) - 40 (one top byte each)
    scale = np.ldexp(np.float32(1), (2 * (g // 2) - 40).astype(np.int32)).astype(np.float32)
    img = (np.where(g % 2 == 1, -base, base) * scale).astype(np.float32)
    assert len(_top_bytes(img)) == groups
    check(ecc, img)
