"""Derived float views on the GPU: the change points of the float curve, and
the integer curve of a quantised float image.  Both are compared exactly with
the oracle: change points are the oracle's float curve restricted to the
distinct values where chi changes; quantised curves are the oracle's integer
curve of the same bins, computed here in float32 by the formula the ABI
states, and are also checked against the float curve they sample."""
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


def steps_of(keys, chi):
    prev = np.concatenate([[0], chi[:-1]])
    keep = chi != prev
    return keys[keep], chi[keep]


def f32_images():
    rng = np.random.default_rng(21)
    out = [gen.cfg_f32_value_noise(s, seed=22) for s in [(1000,), (40, 33), (9, 17, 20), (6, 7, 8, 9)]]
    a = gen.cfg_f32_value_noise((12, 40, 30), seed=23)
    a[rng.random(a.shape) < 0.05] = np.inf
    a[rng.random(a.shape) < 0.05] = -np.inf
    a[rng.random(a.shape) < 0.05] = -0.0
    out.append(a)
    out.append(np.round(gen.cfg_f32_value_noise((30, 31, 32), seed=24) * 8) / 8)  # many ties
    return out


@pytest.mark.parametrize("k", range(6))
def test_change_points(ecc, k):
    img = f32_images()[k]
    print(f"\n[gpu] change points {img.shape}", flush=True)
    keys, chi = ecc.compute_change_points(torch.from_numpy(img).cuda())
    rk, rc = steps_of(*oracle.curve_float(img))
    assert (keys.cpu().numpy() == rk).all() and (chi.cpu().numpy() == rc).all()


def test_change_points_full_128_4d(ecc):
    """The 4-D 128^4 float32 volume (seed 3): the change points are the full
    curve's (checked against the oracle in full elsewhere) where chi changes."""
    img = gen.cfg_f32_value_noise((128, 128, 128, 128), seed=3)
    t = torch.from_numpy(img).cuda()
    keys, chi = ecc.compute(t, "f32")
    rk, rc = steps_of(keys.cpu().numpy(), chi.cpu().numpy())
    sk, sc = ecc.compute_change_points(t)
    assert len(sk) == len(rk) < len(keys)
    assert (sk.cpu().numpy() == rk).all() and (sc.cpu().numpy() == rc).all()


def quantize_np(img, lo, hi, m):
    width = np.float32(hi) - np.float32(lo)
    scale = np.float32(m) / width
    with np.errstate(invalid="ignore", over="ignore"):
        x = (img.astype(np.float32) - np.float32(lo)) * scale
        q = np.where(~(x >= 0), 0, np.where(x >= np.float32(m), m - 1, np.trunc(np.nan_to_num(x, posinf=0))))
    return q.astype(np.uint8 if m == 256 else np.uint16)


@pytest.mark.parametrize("bins", ["u8", "u14", "u16"])
@pytest.mark.parametrize("k", range(6))
def test_quantized(ecc, bins, k):
    img = f32_images()[k]
    m = ecc.THRESHOLDS[bins]
    lo, hi = -0.05, 1.05
    print(f"\n[gpu] quantised {bins} {img.shape}", flush=True)
    got = ecc.compute_quantized(torch.from_numpy(img).cuda(), lo, hi, bins).cpu().numpy()
    q = quantize_np(img, lo, hi, m)
    assert (got == oracle.curve(q, m=m)).all()
    # the bins' sublevel sets are the image's: chi[t] = float curve at the
    # largest value whose bin is <= t
    keys, fchi = oracle.curve_float(img)
    kb = quantize_np(keys, lo, hi, m).astype(np.int64)
    last = np.searchsorted(kb, np.arange(m), side="right") - 1
    want = np.where(last >= 0, fchi[np.maximum(last, 0)], 0)
    assert (got == want).all()


def test_quantized_errors(ecc):
    img = gen.cfg_f32_value_noise((5, 6, 7), seed=1)
    t = torch.from_numpy(img).cuda()
    with pytest.raises(ecc.EccError) as ei:
        ecc.compute_quantized(t, 1.0, 1.0, "u8")
    assert ei.value.code == ecc.ECC_E_ARG
    bad = img.copy()
    bad[1, 2, 3] = np.nan
    with pytest.raises(ecc.EccError) as ei:
        ecc.compute_quantized(torch.from_numpy(bad).cuda(), 0.0, 1.0, "u14")
    assert ei.value.code == ecc.ECC_E_NAN
    got = ecc.compute_quantized(t, 0.0, 1.0, "u14").cpu().numpy()  # the NaN flag was cleared
    assert (got == oracle.curve(quantize_np(img, 0.0, 1.0, 16384), m=16384)).all()
