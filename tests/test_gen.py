"""Input generators: the C library against its numpy restatement and the published SplitMix64 outputs."""
import numpy as np
import pytest

import gen


def test_splitmix64_published_sequence():
    # SplitMix64 started at state 0 returns 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f
    g = int(gen.GAMMA)
    outs = [int(gen.mix64_np(np.uint64((k * g) % 2**64))) for k in (1, 2, 3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_hash_c_matches_numpy():
    for seed, stream, i in [(0, 0, 0), (1, 2, 12345), (7, 1, 2**40 + 3)]:
        assert gen.lib().eccgen_hash(seed, stream, i) == int(gen.hash_np(seed, stream, np.array([i]))[0])


@pytest.mark.parametrize("shape", [(37,), (17, 33), (9, 20, 35), (5, 6, 7, 9)])
def test_value_noise_c_matches_numpy(shape):
    assert (gen.value_noise(shape, 14, 64, 1) == gen.value_noise_np(shape, 14, 64, 1)).all()
    assert (gen.value_noise(shape, 8, 1, 4) == gen.value_noise_np(shape, 8, 1, 4)).all()
    assert (gen.value_noise_f32(shape, 0.01, 3) == gen.value_noise_f32_np(shape, 0.01, 3)).all()


def test_iid_c_matches_numpy():
    assert (gen.iid((5, 7, 3), 8, 0) == gen.iid_np((5, 7, 3), 8, 0)).all()
    assert (gen.iid((11, 13), 14, 9) == gen.iid_np((11, 13), 14, 9)).all()


def test_plane_ranges_concatenate():
    shape = (20, 33, 17)
    full = gen.value_noise(shape, 14, 64, 2)
    parts = [gen.value_noise(shape, 14, 64, 2, z0=a, z1=b) for a, b in [(0, 5), (5, 11), (11, 20)]]
    assert (np.concatenate(parts) == full).all()


def test_ranges_and_statistics():
    v = gen.cfg_u14_value_noise((64, 64, 64), seed=1)
    assert v.dtype == np.uint16 and v.max() <= 16383
    # the jitter is uniform on [-64, 64]: its mean is 0 and its extremes are reached
    h = gen.hash_np(5, 2, np.arange(200000, dtype=np.uint64))
    j = (((h >> np.uint64(32)) * np.uint64(129)) >> np.uint64(32)).astype(np.int64) - 64
    assert j.min() == -64 and j.max() == 64 and abs(j.mean()) < 0.5
    u = gen.cfg_2d_u8_iid()
    assert u.shape == (256, 256) and u.dtype == np.uint8 and u.min() == 0 and u.max() == 255
    f = gen.cfg_f32_value_noise((16, 16, 16, 16))
    assert f.dtype == np.float32 and -0.2 < f.min() and f.max() < 1.2


def test_device_generator_library_exports():
    """libeccgen_dev.so loads here (no GPU needed) and sizes its lattice table:
    node planes z0 >> 4 .. ((z1 - 1) >> 4) + 1, each ((n1 - 1) >> 4) + 2 by
    ((n2 - 1) >> 4) + 2 nodes."""
    L = gen.dev_lib()
    assert hasattr(L, "eccgen_dev_value_noise")
    assert gen.dev_table_entries((2600, 14450, 14450), 0, 64) == 5 * 905 * 905
    assert gen.dev_table_entries((2600, 14450, 14450), 100, 200) == (12 - 6 + 2) * 905 * 905
    assert gen.dev_table_entries((5, 1, 1), 4, 5) == 2 * 2 * 2
    with pytest.raises(ValueError):
        gen.dev_table_entries((5, 6), 0, 5)  # 3-D only
    with pytest.raises(ValueError):
        gen.dev_table_entries((5, 6, 7), 3, 3)  # empty range


@pytest.mark.parametrize("shape,lshift,bits,amp,z0,z1", [
    ((9, 20, 35), 4, 14, 64, 0, 9), ((37, 1, 300), 4, 14, 64, 3, 30), ((3, 17, 2), 2, 8, 1, 1, 3),
    ((700, 1, 2049), 4, 8, 1, 0, 700), ((65, 1, 33), 3, 16, 256, 10, 60),
    ((20, 33, 17), 3, 16, 256, 5, 19), ((2, 70, 1), 4, 14, 64, 0, 2), ((5, 5, 129), 5, 12, 7, 2, 5)], ids=str)
def test_value_noise_rows_match_voxelwise(shape, lshift, bits, amp, z0, z1):
    """The 3-D and 2-D row forms of the generator write the per-voxel form's bytes."""
    dtype = np.uint8 if bits <= 8 else np.uint16
    if shape[1] == 1:  # also as a 2-D image
        s2 = (shape[0], shape[2])
        f2 = gen.value_noise(s2, bits, amp, 12, lshift=lshift, z0=z0, z1=z1)
        g2 = np.empty_like(f2)
        assert gen.lib().eccgen_value_noise_voxelwise(12, 2, gen._dims(s2), lshift, bits, amp, z0, z1, g2.ctypes.data,
                                                      np.dtype(dtype).itemsize, 2) == 0
        assert (f2 == g2).all()
    fast = gen.value_noise(shape, bits, amp, 11, lshift=lshift, z0=z0, z1=z1)
    slow = np.empty_like(fast)
    rc = gen.lib().eccgen_value_noise_voxelwise(11, 3, gen._dims(shape), lshift, bits, amp, z0, z1,
                                               slow.ctypes.data, np.dtype(dtype).itemsize, 3)
    assert rc == 0 and (fast == slow).all()
    if z0 == 0 and z1 == shape[0]:
        assert (fast == gen.value_noise_np(shape, bits, amp, 11, lshift=lshift)).all()
