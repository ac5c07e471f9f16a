"""ecc_release_workspaces: the per-stream device scratch kept between calls
is freed and grown again on the next call, with the same curves (the
oracle's on a small image), also when work is still in flight."""
import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ecc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1705_02045_amd as ecc
    return ecc


def test_release_then_compute_again(ecc):
    img = gen.cfg_u14_value_noise((40, 70, 90), seed=51)
    ref = oracle.curve(img, m=16384)
    t = torch.from_numpy(img.view(np.int16)).cuda()
    assert (ecc.compute(t, "u14").cpu().numpy() == ref).all()
    ecc.release_workspaces()
    assert (ecc.compute(t, "u14").cpu().numpy() == ref).all()
    ecc.release_workspaces()
    ecc.release_workspaces()  # nothing held: still fine
    assert (ecc.compute(t, "u14").cpu().numpy() == ref).all()


def test_release_returns_float_scratch(ecc):
    """The float path's scratch (keys, records, sort buffers: tens of bytes
    per voxel) of a 4-D float32 image goes back to the device."""
    shape = (48, 48, 48, 48)
    img = gen.value_noise_f32(shape, sigma=0.01, seed=52)
    t = torch.from_numpy(img).cuda()
    keys, chi = ecc.compute(t, "f32")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ecc.release_workspaces()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 - free0 >= 16 * img.size, (free0, free1)
    keys2, chi2 = ecc.compute(t, "f32")
    assert torch.equal(keys, keys2) and torch.equal(chi, chi2)


def test_release_waits_for_work_in_flight(ecc):
    img = gen.cfg_u14_value_noise((64, 128, 128), seed=53)
    ref = oracle.curve(img, m=16384)
    t = torch.from_numpy(img.view(np.int16)).cuda()
    s = torch.cuda.Stream()
    chi = torch.empty(16384, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(s):
        for _ in range(4):
            ecc.compute_async(t, chi, "u14", status=st, stream=s)
    ecc.release_workspaces()  # waits for the launches above before freeing their scratch
    assert int(st.item()) == 0 and (chi.cpu().numpy() == ref).all()
    with torch.cuda.stream(s):
        ecc.compute_async(t, chi, "u14", status=st, stream=s)
    s.synchronize()
    assert int(st.item()) == 0 and (chi.cpu().numpy() == ref).all()
