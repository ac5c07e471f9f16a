"""ecc_compute_async_noalloc (the entry point for callers that cannot
allocate: its scratch is the library's static device array) against
ecc_compute_async on the same device images: identical int64 curves and
status words, on consecutive calls whose second input is smaller, so that
the array's leftover contents from a larger call must not leak into a
smaller one."""
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


def dev_u14(shape, seed):
    """Value-noise volume made by the device generator (the host generator's bytes)."""
    ent = gen.dev_table_entries(shape, 0, shape[0])
    table = torch.empty(ent, dtype=torch.int16, device="cuda")
    out = torch.empty(shape, dtype=torch.int16, device="cuda")
    gen.cfg_u14_value_noise_dev(out.data_ptr(), shape, seed, 0, shape[0], table.data_ptr(), ent,
                                stream=torch.cuda.current_stream().cuda_stream)
    return out


def both(ecc, img, dtype):
    """(no-alloc curve, its status, async curve, its status) on the current stream."""
    m = ecc.THRESHOLDS[dtype]
    a = torch.full((m,), -7, dtype=torch.int64, device="cuda")
    b = torch.full((m,), -9, dtype=torch.int64, device="cuda")
    sa = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    sb = torch.full((1,), 88, dtype=torch.int32, device="cuda")
    ecc.compute_async_noalloc(img, a, dtype, status=sa)
    ecc.compute_async(img, b, dtype, status=sb)
    torch.cuda.synchronize()
    return a.cpu().numpy(), int(sa.item()), b.cpu().numpy(), int(sb.item())


def check_pair(ecc, img, dtype, ref=None):
    a, sa, b, sb = both(ecc, img, dtype)
    assert sa == 0 and sb == 0, (sa, sb)
    assert (a == b).all(), f"{dtype} {tuple(img.shape)}: curves differ at {np.nonzero(a != b)[0][:5]}"
    if ref is not None:
        assert (a == ref).all()


def test_u14_large_then_small(ecc):
    """The 1024^3 headline volume (1024 workgroups of count rows), then a
    small volume (a few rows): the second call must not see the first's rows."""
    print("\n[gpu] no-alloc: u14 1024^3 then (40, 48, 72)", flush=True)
    check_pair(ecc, dev_u14((1024, 1024, 1024), 1), "u14")
    small = gen.cfg_u14_value_noise((40, 48, 72), seed=1)
    check_pair(ecc, torch.from_numpy(small.view(np.int16)).cuda(), "u14", oracle.curve(small, m=16384))


def test_u14_capped_grid(ecc):
    """62 planes of 8192^2 (8.3 GB): the size rule asks for 4096 workgroups,
    the no-alloc form caps them at 1024 (four tiles each); same curve."""
    print("\n[gpu] no-alloc: u14 (62, 8192, 8192)", flush=True)
    vol = dev_u14((62, 8192, 8192), 2)
    check_pair(ecc, vol, "u14")
    del vol
    check_pair(ecc, dev_u14((5, 64, 130), 3), "u14")


def test_u8_and_u16_large_then_small(ecc):
    print("\n[gpu] no-alloc: u8 2-D and 3-D", flush=True)
    big8 = gen.iid((512, 3000), 8, seed=3)
    check_pair(ecc, torch.from_numpy(big8).cuda(), "u8", oracle.curve(big8, m=256))
    small8 = gen.cfg_2d_u8_iid((256, 256), seed=0)
    check_pair(ecc, torch.from_numpy(small8).cuda(), "u8", oracle.curve(small8, m=256))
    print("[gpu] no-alloc: u16 full range, then a smaller image", flush=True)
    big16 = gen.value_noise((33, 64, 130), 16, 256, seed=4)
    check_pair(ecc, torch.from_numpy(big16.view(np.int16)).cuda(), "u16", oracle.curve(big16, m=65536))
    small16 = gen.value_noise((3, 7, 9), 16, 256, seed=5)
    check_pair(ecc, torch.from_numpy(small16.view(np.int16)).cuda(), "u16", oracle.curve(small16, m=65536))


def test_range_error_then_valid(ecc):
    """A 14-bit image holding 20000: the status word reports it and the curve
    is left alone; the next, valid call reports 0 (the array's status words
    are cleared per call)."""
    print("\n[gpu] no-alloc: range error, then a valid image", flush=True)
    img = gen.cfg_u14_value_noise((6, 30, 66), seed=9)
    img[3, 4, 5] = 20000
    t = torch.from_numpy(img.view(np.int16)).cuda()
    chi = torch.full((16384,), -5, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ecc.compute_async_noalloc(t, chi, "u14", status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == ecc.STATUS_RANGE_BIT
    assert (chi.cpu().numpy() == -5).all()
    good = gen.cfg_u14_value_noise((6, 30, 66), seed=9)
    check_pair(ecc, torch.from_numpy(good.view(np.int16)).cuda(), "u14", oracle.curve(good, m=16384))
