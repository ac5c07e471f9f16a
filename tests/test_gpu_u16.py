"""GPU parity of 16-bit images (m = 65536 thresholds) against the oracle,
exact int64.  An image whose values fit one window of 16384 values is
counted in a 16384-bin workgroup histogram (guard bins where values lie
outside the window); wider ranges go through 32768-bin passes (one pass when
the values span fewer than 32768, else [0, 32768) and [32768, 65536) with
the adds outside each pass masked off).  These cases put values on and
around window and pass edges, span one to all five windows and both passes,
and run both the synchronous call (planned from the image's range) and the
stream-ordered one (passes over 0..65535)."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WIN = 16382


@pytest.fixture(scope="module")
def ecc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1705_02045_amd as ecc
    return ecc


def dev(img):
    return torch.from_numpy(img.view(np.int16)).cuda()


def check(ecc, img):
    ref = oracle.curve(img, m=65536)
    got = ecc.compute(dev(img), "u16").cpu().numpy()
    if not (got == ref).all():
        bad = np.nonzero(got != ref)[0]
        raise AssertionError(f"{img.shape}: {len(bad)} thresholds differ, first {bad[:5]} "
                             f"got {got[bad[:5]]} want {ref[bad[:5]]}")
    chi = torch.empty(65536, dtype=torch.int64, device="cuda")
    st = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    ecc.compute_async(dev(img), chi, "u16", status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert (chi.cpu().numpy() == ref).all()


SHAPES = [(1,), (1000,), (5, 9), (63, 257), (300, 1000), (3, 5, 7), (9, 17, 129), (20, 129, 63), (64, 64, 64),
          (3, 1, 300)]


@pytest.mark.parametrize("shape", SHAPES, ids=str)
def test_u16_iid_full_range(ecc, shape):
    print(f"\n[gpu] u16 iid {shape}", flush=True)
    check(ecc, gen.iid(shape, 16, seed=13))


@pytest.mark.parametrize("shape", SHAPES, ids=str)
def test_u16_value_noise(ecc, shape):
    print(f"\n[gpu] u16 value noise {shape}", flush=True)
    check(ecc, gen.value_noise(shape, 16, 256, seed=14))


def test_u16_window_edges(ecc):
    edges = [0, 1, WIN - 1, WIN, WIN + 1, WIN + 2, 2 * WIN - 1, 2 * WIN, 2 * WIN + 1, 3 * WIN, 3 * WIN + 1,
             4 * WIN - 1, 4 * WIN, 4 * WIN + 1, 65534, 65535]
    rng = np.random.default_rng(15)
    for shape in [(40, 50), (6, 20, 30), (2000,)]:
        img = rng.choice(np.array(edges, dtype=np.uint16), size=shape)
        check(ecc, img)


def test_u16_narrow_ranges(ecc):
    rng = np.random.default_rng(16)
    for lo, hi in [(50000, 50100), (WIN - 3, WIN + 3), (0, 3), (65530, 65535), (20000, 20000),
                   (100, 100 + 16383), (100, 100 + 16384), (0, 16383), (0, 16384), (40000, 65535)]:
        img = rng.integers(lo, hi + 1, size=(7, 33, 41)).astype(np.uint16)
        check(ecc, img)


def test_u16_pass_edges(ecc):
    """Values on both sides of the 32768 boundary of the two-pass form, and
    ranges whose span is just below, at and just above one pass."""
    rng = np.random.default_rng(17)
    edges = np.array([0, 1, 32766, 32767, 32768, 32769, 65534, 65535], dtype=np.uint16)
    for shape in [(40, 50), (6, 20, 30), (3000,), (9, 130, 66)]:
        check(ecc, rng.choice(edges, size=shape))
    for lo, hi in [(0, 32767), (0, 32768), (1, 32768), (32767, 65535), (32768, 65535), (16000, 48767),
                   (16000, 48768), (32760, 32775)]:
        img = rng.integers(lo, hi + 1, size=(7, 33, 42)).astype(np.uint16)
        img.flat[0], img.flat[-1] = lo, hi
        check(ecc, img)
        check(ecc, np.ascontiguousarray(img[0]))  # one plane: two axes


def test_u16_full_size_1024_cubed(ecc):
    """1024^3 16-bit value noise (lattice 16, jitter +-256, seed 1) in full."""
    print("\n[gpu] u16 1024^3: generating", flush=True)
    img = gen.value_noise((1024, 1024, 1024), 16, 256, seed=1)
    print("[gpu] oracle ...", flush=True)
    ref = oracle.curve(img, m=65536)
    print("[gpu] GPU ...", flush=True)
    got = ecc.compute(dev(img), "u16").cpu().numpy()
    assert (got == ref).all()
    assert ref[-1] == 1
