"""GPU parity of ecc_compute_max_entry (each cell's value is the maximum over
its voxels) against the oracle's max-entry cell enumeration, exact int64."""
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


def dev(img):
    return torch.from_numpy(img.view(np.int16) if img.dtype == np.uint16 else img).cuda()


def check(ecc, img, dtype):
    m = ecc.THRESHOLDS[dtype]
    got = ecc.compute_max_entry(dev(img), dtype).cpu().numpy()
    ref = oracle.curve_max_entry(img, m=m)
    if not (got == ref).all():
        bad = np.nonzero(got != ref)[0]
        raise AssertionError(f"{img.shape} {dtype}: {len(bad)} thresholds differ, first {bad[:5]}")
    assert ref[-1] == 1


SHAPES = [(1,), (2,), (1000,), (1, 1), (5, 9), (63, 257), (300, 1000), (17, 4097), (1, 1, 1), (2, 2, 2),
          (3, 5, 7), (9, 17, 129), (20, 129, 63), (64, 64, 64), (3, 1, 300), (100, 2, 2), (3, 5000, 700)]


@pytest.mark.parametrize("shape", SHAPES, ids=str)
def test_max_entry_u14_value_noise(ecc, shape):
    print(f"\n[gpu] max entry u14 {shape}", flush=True)
    check(ecc, gen.cfg_u14_value_noise(shape, seed=8), "u14")


@pytest.mark.parametrize("shape", SHAPES, ids=str)
def test_max_entry_u8_iid(ecc, shape):
    print(f"\n[gpu] max entry u8 {shape}", flush=True)
    check(ecc, gen.iid(shape, 8, seed=9), "u8")


SHAPES_4D = [(5, 6, 7, 8), (2, 3, 40, 5), (12, 12, 12, 12), (3, 4, 5, 70), (1, 4, 1, 9), (24, 20, 33, 17)]


@pytest.mark.parametrize("shape", SHAPES_4D, ids=str)
def test_max_entry_4d(ecc, shape):
    """Four axes longer than 1: through the float path on m - 1 - v."""
    print(f"\n[gpu] max entry 4-D {shape}", flush=True)
    check(ecc, gen.cfg_u14_value_noise(shape, seed=18), "u14")
    check(ecc, gen.iid(shape, 8, seed=19), "u8")


def test_max_entry_4d_range_error(ecc):
    img = gen.cfg_u14_value_noise((3, 4, 5, 6), seed=20)
    img[2, 3, 4, 5] = 16384
    with pytest.raises(ecc.EccError) as ei:
        ecc.compute_max_entry(dev(img), "u14")
    assert ei.value.code == ecc.ECC_E_RANGE


def test_max_entry_ties_and_extremes(ecc):
    rng = np.random.default_rng(5)
    for shape in [(7, 40, 70), (33, 65), (500,)]:
        img = rng.integers(0, 3, size=shape).astype(np.uint8) * 127  # values 0, 127, 254
        check(ecc, img, "u8")
        check(ecc, np.full(shape, 255, dtype=np.uint8), "u8")
        check(ecc, np.zeros(shape, dtype=np.uint16), "u14")
        check(ecc, np.full(shape, 16383, dtype=np.uint16), "u14")


def test_max_entry_matches_identity_with_min_path(ecc):
    """The two GPU entry points agree through max_f(t) = 1 - min_{M-f}(M-t-1)."""
    img = gen.cfg_u14_value_noise((40, 100, 130), seed=3)
    got = ecc.compute_max_entry(dev(img), "u14").cpu().numpy()
    inv = ecc.compute(dev((16383 - img.astype(np.int64)).astype(np.uint16)), "u14").cpu().numpy()
    want = 1 - np.concatenate([inv[::-1][1:], [0]])
    assert (got == want).all()


def test_max_entry_range_error_and_reuse(ecc):
    img = gen.cfg_u14_value_noise((5, 40, 70), seed=2)
    bad = img.copy()
    bad[1, 2, 3] = 16384
    with pytest.raises(ecc.EccError) as ei:
        ecc.compute_max_entry(dev(bad), "u14")
    assert ei.value.code == ecc.ECC_E_RANGE
    check(ecc, img, "u14")  # the workspace status was cleared
    with pytest.raises(ecc.EccError) as ei:
        ecc.compute_max_entry(torch.zeros(8, dtype=torch.float32, device="cuda"), "f32")
    assert ei.value.code == ecc.ECC_E_UNSUPPORTED
