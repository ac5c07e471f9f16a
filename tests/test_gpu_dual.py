"""GPU parity of ecc_compute_dual (the dual complex: voxels as vertices,
lower-star filtration) against the oracle's direct enumeration of that
complex, exact int64."""
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
    got = ecc.compute_dual(dev(img), dtype).cpu().numpy()
    ref = oracle.curve_dual(img, m=m)
    if not (got == ref).all():
        bad = np.nonzero(got != ref)[0]
        raise AssertionError(f"{img.shape} {dtype}: {len(bad)} thresholds differ, first {bad[:5]} "
                             f"got {got[bad[:5]]} want {ref[bad[:5]]}")
    assert ref[-1] == 1


SHAPES = [(1,), (2,), (1000,), (1, 1), (5, 9), (2, 2), (63, 257), (300, 1000), (17, 4097), (1, 1, 1), (2, 2, 2),
          (3, 5, 7), (1, 5, 7), (5, 1, 7), (5, 7, 1), (9, 17, 129), (20, 129, 63), (64, 64, 64), (3, 1, 300),
          (100, 2, 2), (3, 5000, 700)]


@pytest.mark.parametrize("shape", SHAPES, ids=str)
def test_dual_u14_value_noise(ecc, shape):
    print(f"\n[gpu] dual u14 {shape}", flush=True)
    check(ecc, gen.cfg_u14_value_noise(shape, seed=10), "u14")


@pytest.mark.parametrize("shape", SHAPES, ids=str)
def test_dual_u8_iid(ecc, shape):
    print(f"\n[gpu] dual u8 {shape}", flush=True)
    check(ecc, gen.iid(shape, 8, seed=11), "u8")


SHAPES_4D = [(5, 6, 7, 8), (2, 3, 40, 5), (12, 12, 12, 12), (3, 4, 5, 70), (2, 2, 2, 2), (24, 20, 33, 17)]


@pytest.mark.parametrize("shape", SHAPES_4D, ids=str)
def test_dual_4d(ecc, shape):
    """Four axes longer than 1: 81 faces, the full box through the float path."""
    print(f"\n[gpu] dual 4-D {shape}", flush=True)
    check(ecc, gen.cfg_u14_value_noise(shape, seed=21), "u14")
    check(ecc, gen.iid(shape, 8, seed=22), "u8")


def test_dual_checkerboard_and_constants(ecc):
    for shape in [(9, 10), (4, 6, 5)]:
        idx = np.indices(shape).sum(axis=0)
        check(ecc, (idx % 2).astype(np.uint8) * 200, "u8")   # isolated vertices at t < 200
        check(ecc, np.full(shape, 7, dtype=np.uint16), "u14")


def test_dual_range_error_and_reuse(ecc):
    img = gen.cfg_u14_value_noise((6, 33, 45), seed=2)
    bad = img.copy()
    bad[5, 32, 44] = 20000  # a corner voxel: it is in the volume and in three faces
    with pytest.raises(ecc.EccError) as ei:
        ecc.compute_dual(dev(bad), "u14")
    assert ei.value.code == ecc.ECC_E_RANGE
    check(ecc, img, "u14")


def test_dual_full_size_1024_cubed_u14(ecc):
    """The 1024^3 14-bit value-noise volume (seed 1) in full."""
    print("\n[gpu] dual 1024^3: generating", flush=True)
    img = gen.cfg_u14_value_noise((1024, 1024, 1024), seed=1)
    print("[gpu] oracle ...", flush=True)
    ref = oracle.curve_dual(img, m=16384)
    print("[gpu] GPU ...", flush=True)
    got = ecc.compute_dual(dev(img), "u14").cpu().numpy()
    assert (got == ref).all()
