"""The tile-shape tuners: ecc_autotune stores a tiling per image shape that
later launches of that shape use, ecc_batch_autotune a tile depth per batch
context; curves stay exactly the oracle's under every tiling chosen."""
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


@pytest.mark.parametrize("shape,dtype", [((64, 96, 130), "u14"), ((700, 900), "u8"), ((3, 2000, 1500), "u14"),
                                         ((100000,), "u8")], ids=str)
def test_autotune_then_compute(ecc, shape, dtype):
    img = gen.cfg_u14_value_noise(shape, seed=31) if dtype == "u14" else gen.iid(shape, 8, seed=31)
    t = dev(img)
    ecc.autotune_reset()
    before = ecc.tiling_for(shape, dtype)
    best = ecc.autotune(t, dtype)
    assert best["rows"] in (2, 4) and best["tiles_per_cu"] in (4, 8, 16) and best["waves_x"] in (8, 16)
    assert best["ms"] > 0
    now = ecc.tiling_for(shape, dtype)
    assert now["rows"] == best["rows"] and now["tiles_per_cu"] == best["tiles_per_cu"]
    got = ecc.compute(t, dtype).cpu().numpy()
    assert (got == oracle.curve(img, m=ecc.THRESHOLDS[dtype])).all()
    ecc.autotune_reset()
    assert ecc.tiling_for(shape, dtype) == before


def test_autotune_rejects_bad_values_and_host_images(ecc):
    img = gen.cfg_u14_value_noise((6, 40, 50), seed=2)
    bad = img.copy()
    bad[3, 4, 5] = 16384
    ecc.autotune_reset()
    before = ecc.tiling_for(img.shape, "u14")
    with pytest.raises(ecc.EccError) as ei:
        ecc.autotune(dev(bad), "u14")
    assert ei.value.code == ecc.ECC_E_RANGE
    assert ecc.tiling_for(img.shape, "u14") == before  # nothing stored
    assert (ecc.compute(dev(img), "u14").cpu().numpy() == oracle.curve(img, m=16384)).all()


def test_batch_autotune(ecc):
    specs = [("u8", (300, 1200)), ("u14", (40, 64, 64)), ("u14", (120, 30, 50)), ("u8", (2000, 64)),
             ("u14", (9, 17, 129))]
    imgs = [gen.serving_image(d, s, 60 + i) for i, (d, s) in enumerate(specs)]
    dimgs = [dev(a) for a in imgs]
    b = ecc.Batch()
    chis = [torch.empty(ecc.THRESHOLDS[d], dtype=torch.int64, device="cuda") for d, _ in specs]
    mp, sp, ms = b.autotune(dimgs, [d for d, _ in specs], chis)
    assert mp in (16, 32, 64, 128) and sp in (2, 4, 8) and ms > 0
    chis = [torch.full((ecc.THRESHOLDS[d],), -5, dtype=torch.int64, device="cuda") for d, _ in specs]
    b.run(dimgs, [d for d, _ in specs], chis)
    torch.cuda.synchronize()
    for (d, s), img, c in zip(specs, imgs, chis):
        assert (c.cpu().numpy() == oracle.curve(img, m=ecc.THRESHOLDS[d])).all(), f"{d} {s}"
    b.close()


def test_autotune_cache_round_trip(ecc, tmp_path):
    """A tiling tuned on the GPU, saved, forgotten and loaded back is the one
    later launches use; every curve stays the oracle's."""
    img = gen.cfg_u14_value_noise((40, 300, 260), seed=32)
    t = dev(img)
    ecc.autotune_reset()
    best = ecc.autotune(t, "u14")
    path = tmp_path / "tiling.txt"
    assert ecc.autotune_save(path) == 1
    ecc.autotune_reset()
    assert ecc.autotune_load(path) == 1
    got = ecc.tiling_for(img.shape, "u14")
    assert got == {k: best[k] for k in ("rows", "tiles_per_cu", "waves_x")}
    assert (ecc.compute(t, "u14").cpu().numpy() == oracle.curve(img, m=16384)).all()
    ecc.autotune_reset()
