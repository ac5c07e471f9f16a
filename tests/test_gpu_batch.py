"""GPU parity of the batched integer path and of the serving replay: every
image's curve must equal the oracle's exactly."""
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


MIXED = [("u8", (32, 32)), ("u14", (16, 16, 16)), ("u8", (300, 70)), ("u14", (9, 17, 129)), ("u8", (1, 1)),
         ("u14", (3, 1, 300)), ("u8", (200,)), ("u14", (70, 130, 66)), ("u8", (5, 2, 300)), ("u14", (2, 2)),
         ("u8", (129, 2049)), ("u14", (100, 64, 64))]


def run_batch(ecc, b, specs, seed0=0, status=None):
    imgs = [gen.serving_image(d, s, seed0 + i) for i, (d, s) in enumerate(specs)]
    dimgs = [dev(a) for a in imgs]
    chis = [torch.full((ecc.THRESHOLDS[d],), -7, dtype=torch.int64, device="cuda") for d, _ in specs]
    b.run(dimgs, [d for d, _ in specs], chis, status)
    torch.cuda.synchronize()
    return imgs, [c.cpu().numpy() for c in chis]


def test_batch_mixed(ecc):
    b = ecc.Batch()
    imgs, got = run_batch(ecc, b, MIXED)
    for (d, s), img, g in zip(MIXED, imgs, got):
        ref = oracle.curve(img, m=ecc.THRESHOLDS[d])
        assert (g == ref).all(), f"{d} {s}"
    # a second, smaller batch on the same context reuses its scratch
    imgs, got = run_batch(ecc, b, MIXED[3:6], seed0=50)
    for (d, s), img, g in zip(MIXED[3:6], imgs, got):
        assert (g == oracle.curve(img, m=ecc.THRESHOLDS[d])).all(), f"{d} {s}"
    b.close()


def test_batch_range_error_is_per_image(ecc):
    b = ecc.Batch()
    specs = [("u14", (5, 40, 70)), ("u14", (6, 30, 65)), ("u8", (40, 70))]
    imgs = [gen.serving_image(d, s, 7 + i) for i, (d, s) in enumerate(specs)]
    imgs[1][2, 3, 4] = 20000
    chis = [torch.full((ecc.THRESHOLDS[d],), -7, dtype=torch.int64, device="cuda") for d, _ in specs]
    status = torch.full((3,), 99, dtype=torch.int32, device="cuda")
    b.run([dev(a) for a in imgs], [d for d, _ in specs], chis, status)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    assert list(st) == [0, ecc.STATUS_RANGE_BIT, 0]
    assert (chis[1].cpu().numpy() == -7).all()
    for i in (0, 2):
        assert (chis[i].cpu().numpy() == oracle.curve(imgs[i], m=ecc.THRESHOLDS[specs[i][0]])).all()
    # the flagged image's status does not leak into the next run
    imgs2, got2 = run_batch(ecc, b, specs[:2], seed0=30)
    for (d, s), img, g in zip(specs[:2], imgs2, got2):
        assert (g == oracle.curve(img, m=ecc.THRESHOLDS[d])).all()
    b.close()


@pytest.mark.parametrize("one_launch", [False, True], ids=["batched", "per_image"])
def test_serve_replay(ecc, one_launch):
    reqs = gen.serving_requests(48, seed=4, side_scale=0.25)
    imgs = [gen.serving_image(*r) for r in reqs]
    dimgs = [dev(a) for a in imgs]
    dtypes = [r[0] for r in reqs]
    arrival = np.cumsum(np.random.default_rng(1).exponential(2e-4, size=len(reqs)))
    b = ecc.Batch()
    lat, chi = b.serve(dimgs, dtypes, arrival, max_batch=16, one_launch_per_image=one_launch)
    b.close()
    assert (lat > 0).all()
    off = 0
    for (d, s, _), img in zip(reqs, imgs):
        m = ecc.THRESHOLDS[d]
        assert (chi[off:off + m] == oracle.curve(img, m=m)).all(), f"{d} {s}"
        off += m


def test_serving_stream_sample_full_sides(ecc):
    # requests of the full-size mix (sides up to 2048 / 256), a sample of them
    reqs = gen.serving_requests(4096, seed=4)[:24]
    imgs = [gen.serving_image(*r) for r in reqs]
    b = ecc.Batch()
    chis = [torch.empty(ecc.THRESHOLDS[r[0]], dtype=torch.int64, device="cuda") for r in reqs]
    b.run([dev(a) for a in imgs], [r[0] for r in reqs], chis)
    torch.cuda.synchronize()
    for r, img, c in zip(reqs, imgs, chis):
        assert (c.cpu().numpy() == oracle.curve(img, m=ecc.THRESHOLDS[r[0]])).all(), f"{r}"
    b.close()


@pytest.mark.parametrize("graph", ["1", "0"], ids=["graph", "direct"])
def test_batch_runs_replay_and_vary(ecc, monkeypatch, graph):
    """Many runs on one context: the ring's four slots are reused, so each
    slot's captured graph replays with new tables (more and fewer images,
    other dtypes and sizes), with eager work on the device between runs;
    every run is checked against the oracle.  Also through the direct
    launches (no graph)."""
    monkeypatch.setenv("ECC_BATCH_GRAPH", graph)
    b = ecc.Batch()
    for r in range(10):
        specs = MIXED[r % 4::2] if r % 3 else MIXED[: 2 + r]
        print(f"\n[gpu] batch run {r} ({graph}): {len(specs)} images", flush=True)
        imgs, got = run_batch(ecc, b, specs, seed0=200 + 17 * r)
        for (d, s), img, g in zip(specs, imgs, got):
            assert (g == oracle.curve(img, m=ecc.THRESHOLDS[d])).all(), f"run {r}: {d} {s}"
        ecc.compute(dev(gen.cfg_u14_value_noise((20, 30, 40), seed=r)), "u14")  # eager work between runs
    b.close()


def test_serve_admission_by_footprint(ecc):
    """All requests arrive at once; a byte budget of three median footprints
    splits them into consecutive batches whose footprints fit the budget (a
    larger request runs alone); every curve matches the oracle."""
    reqs = gen.serving_requests(40, seed=9, side_scale=0.2)
    imgs = [gen.serving_image(*r) for r in reqs]
    dimgs = [dev(a) for a in imgs]
    dtypes = [r[0] for r in reqs]
    foot = np.array([ecc.Batch.footprint(t, d) for t, d in zip(dimgs, dtypes)])
    budget = int(3 * np.median(foot))
    b = ecc.Batch()
    lat, chi, bid = b.serve(dimgs, dtypes, np.zeros(len(reqs)), max_batch=64, max_batch_bytes=budget,
                            with_batches=True)
    b.close()
    assert (np.diff(bid) >= 0).all() and (np.diff(bid) <= 1).all() and bid[0] == 0
    assert bid[-1] >= 2  # the budget did split the stream
    for k in range(bid[-1] + 1):
        sel = bid == k
        assert sel.sum() == 1 or foot[sel].sum() <= budget
    off = 0
    for (d, s, _), img in zip(reqs, imgs):
        m = ecc.THRESHOLDS[d]
        assert (chi[off:off + m] == oracle.curve(img, m=m)).all(), f"{d} {s}"
        off += m


def test_batch_with_16bit_jobs(ecc):
    """16-bit jobs (m = 65536) ride in a batch next to u8/u14 jobs: they run as
    windowed launches of their own after the persistent kernel, on the same
    stream; a batch of 16-bit jobs only has no persistent launch."""
    rng = np.random.default_rng(33)
    imgs = [gen.serving_image("u8", (40, 70), 1), gen.iid((9, 40, 70), 16, seed=34),
            gen.serving_image("u14", (16, 30, 20), 2), gen.value_noise((20, 60, 80), 16, 256, seed=35),
            (30000 + rng.integers(0, 5, size=(33, 65))).astype(np.uint16)]
    dtypes = ["u8", "u16", "u14", "u16", "u16"]
    b = ecc.Batch()
    for sel in (range(5), [1, 3, 4]):
        chis = [torch.full((ecc.THRESHOLDS[dtypes[i]],), -7, dtype=torch.int64, device="cuda") for i in sel]
        status = torch.full((len(sel),), 99, dtype=torch.int32, device="cuda")
        b.run([dev(imgs[i]) for i in sel], [dtypes[i] for i in sel], chis, status)
        torch.cuda.synchronize()
        assert (status.cpu().numpy() == 0).all()
        for i, c in zip(sel, chis):
            assert (c.cpu().numpy() == oracle.curve(imgs[i], m=ecc.THRESHOLDS[dtypes[i]])).all(), i
    b.close()
