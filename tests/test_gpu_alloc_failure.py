"""Allocation failures, forced from the host through the library's injection
hook (ECC_FAIL_ALLOC=k: the k-th and later allocations fail as out of
memory): each call reports ECC_E_NOMEM, leaves the caller's output alone,
frees what it had taken, and the next call without the hook succeeds."""
import ctypes

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


def img_u14(shape, seed):
    a = gen.cfg_u14_value_noise(shape, seed=seed)
    return a, torch.from_numpy(a.view(np.int16)).cuda()


def compute_raw(ecc, t, shape, out, stream):
    cv = ecc.Curve(capacity=out.size, count=0, chi=out.ctypes.data, keys=None)
    return ecc._lib.ecc_compute(t.data_ptr(), ctypes.byref(ecc.make_dims(shape)), ecc.DTYPES["u14"],
                                ctypes.byref(cv), ctypes.c_void_p(stream.cuda_stream))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_compute_on_fresh_stream(ecc, monkeypatch, k):
    """A call on a new stream allocates its workspace (status block, pinned
    status word, curve staging, count rows, ...): the k-th allocation fails."""
    a, t = img_u14((20, 30, 40), seed=3)
    out = np.full(16384, -3, dtype=np.int64)
    s = torch.cuda.Stream()
    monkeypatch.setenv("ECC_FAIL_ALLOC", str(k))
    assert compute_raw(ecc, t, a.shape, out, s) == ecc.ECC_E_NOMEM
    assert (out == -3).all()
    monkeypatch.delenv("ECC_FAIL_ALLOC")
    assert compute_raw(ecc, t, a.shape, out, s) == ecc.ECC_OK
    assert (out == oracle.curve(a, m=16384)).all()


@pytest.mark.parametrize("k", [1, 3, 5])
def test_stream_begin_and_push(ecc, monkeypatch, k):
    """Streaming: a failure in ecc_stream_begin (carry buffers, changes
    vector, status) or at the first push (staging of a host chunk, count
    rows) is ECC_E_NOMEM; a fresh stream afterwards gives the oracle's curve."""
    a, t = img_u14((12, 40, 70), seed=4)
    parts = [a[:6].view(np.int16).copy(), a[6:].view(np.int16).copy()]
    monkeypatch.setenv("ECC_FAIL_ALLOC", str(k))
    holder = []
    with pytest.raises(ecc.EccError) as ei:
        holder.append(ecc.Stream(a.shape, "u14"))
        for p in parts:
            holder[0].push(p)
        holder[0].finish()
    assert ei.value.code == ecc.ECC_E_NOMEM
    for st in holder:
        st.abort()
    monkeypatch.delenv("ECC_FAIL_ALLOC")
    st = ecc.Stream(a.shape, "u14")
    for p in parts:
        st.push(p)
    assert (st.finish() == oracle.curve(a, m=16384)).all()


def test_batch_and_serve(ecc, monkeypatch):
    """A batch context whose descriptor tables and scratch cannot be
    allocated reports ECC_E_NOMEM from run and from serve; the same context
    works once allocation succeeds again."""
    specs = [("u8", (40, 70)), ("u14", (9, 17, 129)), ("u14", (5, 30, 66))]
    imgs = [gen.serving_image(d, s, 60 + i) for i, (d, s) in enumerate(specs)]
    dev = [torch.from_numpy(x.view(np.int16) if x.dtype == np.uint16 else x).cuda() for x in imgs]
    dtypes = [d for d, _ in specs]
    b = ecc.Batch()
    chis = [torch.full((ecc.THRESHOLDS[d],), -7, dtype=torch.int64, device="cuda") for d in dtypes]
    monkeypatch.setenv("ECC_FAIL_ALLOC", "1")
    with pytest.raises(ecc.EccError) as ei:
        b.run(dev, dtypes, chis)
    assert ei.value.code == ecc.ECC_E_NOMEM
    monkeypatch.setenv("ECC_FAIL_ALLOC", "2")
    lat, chi, bid, st, rc = b.serve_config(dev, dtypes, np.zeros(3), max_batch=4, check=False)
    assert rc == ecc.ECC_E_NOMEM
    monkeypatch.delenv("ECC_FAIL_ALLOC")
    b.run(dev, dtypes, chis)
    torch.cuda.synchronize()
    for (d, _), x, c in zip(specs, imgs, chis):
        assert (c.cpu().numpy() == oracle.curve(x, m=ecc.THRESHOLDS[d])).all()
    b.close()


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("kind", ["host", "device", "4d"])
def test_stream_failed_push_is_pushed_again(ecc, monkeypatch, k, kind):
    """A push whose k-th allocation fails reports ECC_E_NOMEM having added
    nothing: the same chunk pushed again (allocation working), then the rest,
    gives the oracle's curve (Sec. 3, "Streaming": a chunk's changes are
    added once)."""
    shape = (7, 9, 10, 70) if kind == "4d" else (12, 40, 70)
    a, t = img_u14(shape, seed=5)
    parts = [a[:5], a[5:]]
    src = [torch.from_numpy(np.ascontiguousarray(p).view(np.int16)) for p in parts]
    if kind != "host":
        src = [s.cuda() for s in src]
    st = ecc.Stream(a.shape, "u14")
    monkeypatch.setenv("ECC_FAIL_ALLOC", str(k))
    failed = False
    try:
        st.push(src[0])
    except ecc.EccError as e:
        assert e.code == ecc.ECC_E_NOMEM
        failed = True
    monkeypatch.delenv("ECC_FAIL_ALLOC")
    if failed:
        st.push(src[0])
    st.push(src[1])
    torch.cuda.synchronize()
    assert (st.finish() == oracle.curve(a, m=16384)).all()
