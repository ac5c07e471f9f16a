"""GPU parity of the integer path through the C ABI: every curve must equal
the oracle's exactly (int64)."""
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


def gpu_curve(ecc, img, dtype):
    t = torch.from_numpy(img.view(np.int16) if img.dtype == np.uint16 else img).cuda()
    return ecc.compute(t, dtype=dtype).cpu().numpy()


def check(ecc, img, dtype):
    m = ecc.THRESHOLDS[dtype]
    ref = oracle.curve(img, m=m)
    got = gpu_curve(ecc, img, dtype)
    if not (got == ref).all():
        bad = np.nonzero(got != ref)[0]
        raise AssertionError(f"shape {img.shape} {dtype}: {len(bad)} thresholds differ, first {bad[:5]} "
                             f"got {got[bad[:5]]} want {ref[bad[:5]]}")


SHAPES_3D = [(1, 1, 1), (2, 2, 2), (3, 5, 7), (5, 64, 64), (4, 63, 65), (7, 66, 130), (9, 17, 129),
             (33, 40, 200), (20, 129, 63), (64, 64, 64), (3, 1, 300), (100, 2, 2), (2, 300, 1)]


@pytest.mark.parametrize("shape", SHAPES_3D, ids=str)
def test_u14_value_noise_3d(ecc, shape):
    print(f"\n[gpu] u14 value noise {shape}", flush=True)
    check(ecc, gen.cfg_u14_value_noise(shape, seed=1), "u14")


@pytest.mark.parametrize("shape", SHAPES_3D, ids=str)
def test_u8_iid_3d(ecc, shape):
    print(f"\n[gpu] u8 iid {shape}", flush=True)
    check(ecc, gen.iid(shape, 8, seed=7), "u8")


@pytest.mark.parametrize("shape", [(1, 1), (1, 2), (2, 1), (5, 9), (64, 64), (63, 257), (256, 256), (300, 1000),
                                   (1000, 3), (17, 4097)], ids=str)
def test_2d(ecc, shape):
    print(f"\n[gpu] 2-D {shape}", flush=True)
    check(ecc, gen.iid(shape, 8, seed=0), "u8")
    check(ecc, gen.cfg_u8_value_noise(shape, seed=4), "u8")
    check(ecc, gen.cfg_u14_value_noise(shape, seed=5), "u14")


@pytest.mark.parametrize("n", [1, 2, 3, 64, 65, 1000, 100003])
def test_1d(ecc, n):
    print(f"\n[gpu] 1-D {n}", flush=True)
    check(ecc, gen.iid((n,), 8, seed=3), "u8")
    check(ecc, gen.iid((n,), 14, seed=3), "u14")


def test_ties_and_constants(ecc):
    rng = np.random.default_rng(5)
    for shape in [(6, 70, 70), (3, 3, 3), (1, 130, 2)]:
        check(ecc, rng.integers(0, 2, size=shape).astype(np.uint8), "u8")
        check(ecc, rng.integers(0, 3, size=shape).astype(np.uint16), "u14")
        check(ecc, np.full(shape, 16383, dtype=np.uint16), "u14")
        check(ecc, np.zeros(shape, dtype=np.uint8), "u8")
        z, y, x = np.indices(shape)
        check(ecc, ((x + y + z) % 2).astype(np.uint8), "u8")


def test_size_one_axes_match_lower_dimension(ecc):
    img = gen.cfg_u14_value_noise((37, 53), seed=9)
    a = gpu_curve(ecc, img, "u14")
    for shape in [(37, 1, 53), (1, 37, 53), (37, 53, 1), (1, 37, 1, 53)]:
        assert (gpu_curve(ecc, img.reshape(shape), "u14") == a).all(), shape


def test_host_input_and_host_output(ecc):
    img = gen.cfg_u14_value_noise((12, 70, 90), seed=2)
    assert (ecc.compute_host(img, "u14") == oracle.curve(img, m=16384)).all()


def test_async_with_status(ecc):
    img = gen.cfg_u14_value_noise((16, 80, 96), seed=3)
    t = torch.from_numpy(img.view(np.int16)).cuda()
    out = torch.zeros(16384, dtype=torch.int64, device="cuda")
    st = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    ecc.compute_async(t, out, "u14", status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert (out.cpu().numpy() == oracle.curve(img, m=16384)).all()


def test_range_error_leaves_output_untouched(ecc):
    img = gen.cfg_u14_value_noise((8, 40, 40), seed=3)
    img[3, 17, 5] = 16384
    t = torch.from_numpy(img.view(np.int16)).cuda()
    out = torch.full((16384,), -5, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ecc.compute_async(t, out, "u14", status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == ecc.STATUS_RANGE_BIT
    assert (out.cpu().numpy() == -5).all()
    with pytest.raises(ecc.EccError) as ei:
        ecc.compute(t, dtype="u14")
    assert ei.value.code == ecc.ECC_E_RANGE


def test_repeated_calls_reuse_workspace(ecc):
    for shape in [(40, 100, 100), (3, 5, 7), (40, 100, 100), (2, 2000, 300)]:
        check(ecc, gen.cfg_u14_value_noise(shape, seed=11), "u14")


@pytest.mark.parametrize("shape,dtype", [((3, 5000, 700), "u14"), ((4, 2048, 2048), "u8"), ((20, 3000, 1000), "u14"),
                                         ((3, 2100000), "u8")], ids=str)
def test_several_tiles_per_workgroup(ecc, shape, dtype):
    """Planes with more tiles than the device holds workgroups: each workgroup
    walks a run of consecutive tiles into one histogram (2500 tiles in runs of
    3 with a short last run; 2048 in runs of 2 over a permuted grid; 1500 in
    runs of 2 over an unpermuted grid; a 2-D image of 1026 row segments)."""
    print(f"\n[gpu] several tiles per workgroup {shape} {dtype}", flush=True)
    img = gen.cfg_u14_value_noise(shape, seed=12) if dtype == "u14" else gen.iid(shape, 8, seed=12)
    check(ecc, img, dtype)


def test_full_size_1024_cubed_u14(ecc):
    """The 3-D 14-bit value-noise volume of 1024^3 voxels (seed 1), compared in full."""
    print("\n[gpu] 1024^3 u14 value noise seed 1: generating", flush=True)
    img = gen.cfg_u14_value_noise((1024, 1024, 1024), seed=1)
    print("[gpu] oracle ...", flush=True)
    ref = oracle.curve(img, m=16384)
    print("[gpu] GPU ...", flush=True)
    got = gpu_curve(ecc, img, "u14")
    assert (got == ref).all()
    assert ref[-1] == 1


def test_full_size_256_squared_u8(ecc):
    """2-D 256x256 uint8 i.i.d. image (seed 0)."""
    img = gen.cfg_2d_u8_iid((256, 256), seed=0)
    check(ecc, img, "u8")


@pytest.mark.parametrize("shape", [(3, 4, 5, 6), (2, 9, 17, 33), (5, 5, 5, 5), (12, 16, 20, 24)], ids=str)
def test_4d_integer_images(ecc, shape):
    """Four axes longer than 1: exact through the float path (the curve is
    the float step function read at every integer threshold)."""
    print(f"\n[gpu] 4-D integer {shape}", flush=True)
    check(ecc, gen.iid(shape, 8, seed=41), "u8")
    check(ecc, gen.value_noise(shape, 14, 64, seed=42), "u14")
    img16 = gen.iid(shape, 16, seed=43)
    got = ecc.compute(torch.from_numpy(img16.view(np.int16)).cuda(), dtype="u16").cpu().numpy()
    assert (got == oracle.curve(img16, m=65536)).all()
    host = gen.iid(shape, 8, seed=44)
    assert (ecc.compute_host(host, "u8") == oracle.curve(host, m=256)).all()


def test_4d_integer_range_error(ecc):
    img = gen.value_noise((3, 4, 5, 6), 14, 64, seed=45)
    img[1, 2, 3, 4] = 16384
    with pytest.raises(ecc.EccError) as ei:
        gpu_curve(ecc, img, "u14")
    assert ei.value.code == ecc.ECC_E_RANGE


ROW_PAIR_SHAPES = [(6, 34, 258), (5, 70, 194), (11, 9, 1026), (3, 130, 132), (2, 3, 4098), (4, 65, 450)]


@pytest.mark.parametrize("tiling", [{}, {"ECC_INT_ROWS": "4"}, {"ECC_INT_PD": "2"},
                                    {"ECC_INT_ROWS": "4", "ECC_INT_PD": "2"}, {"ECC_INT_PAIR": "0"}], ids=str)
@pytest.mark.parametrize("shape", ROW_PAIR_SHAPES, ids=str)
def test_row_pair_layout(ecc, shape, tiling, monkeypatch):
    """16-bit images with even rows: interior waves read aligned dwords and
    form (x-1, x) pairs with a wave shift; waves start at odd columns and
    column 0 goes to the spare lane of each row's last wave.  Several interior
    waves per row, ragged last waves, two and four rows per wave, one and two
    planes of look-ahead, and the same shapes without row pairs; the
    largest-value convention and 16-bit windows use the same loads."""
    for k, v in tiling.items():
        monkeypatch.setenv(k, v)
    print(f"\n[gpu] row pairs {shape} {tiling}", flush=True)
    img = gen.cfg_u14_value_noise(shape, seed=21)
    check(ecc, img, "u14")
    t = torch.from_numpy(img.view(np.int16)).cuda()
    assert (ecc.compute_max_entry(t, "u14").cpu().numpy() == oracle.curve_max_entry(img, m=16384)).all()
    img16 = gen.iid(shape, 16, seed=22)
    got16 = ecc.compute(torch.from_numpy(img16.view(np.int16)).cuda(), dtype="u16").cpu().numpy()
    assert (got16 == oracle.curve(img16, m=65536)).all()


@pytest.mark.parametrize("shape", [(5, 34, 258), (4, 20, 130)], ids=str)
def test_row_pairs_need_aligned_buffers(ecc, shape):
    """Row pairs need 4-byte aligned rows: an image that starts 2 bytes into
    its allocation (even rows, so every row start is 2 mod 4) takes the
    element loads instead, with the same curve; so does the aligned copy."""
    img = gen.cfg_u14_value_noise(shape, seed=31)
    flat = torch.zeros(img.size + 2, dtype=torch.int16, device="cuda")
    flat[1:1 + img.size] = torch.from_numpy(img.view(np.int16).ravel()).cuda()
    view = flat[1:1 + img.size].view(shape)
    assert view.data_ptr() % 4 == 2
    print(f"\n[gpu] row pairs, base 2 mod 4 {shape}", flush=True)
    ref = oracle.curve(img, m=16384)
    assert (ecc.compute(view, "u14").cpu().numpy() == ref).all()
    assert (ecc.compute(view.clone(), "u14").cpu().numpy() == ref).all()


def test_random_shapes_both_conventions(ecc):
    """40 seeded random 3-D shapes (extents 1..23 x 1..69 x 2..400, mostly
    even rows, so most interior waves take row pairs and the edge waves vary):
    the smallest- and largest-value curves equal the oracle's."""
    rng = np.random.default_rng(2027)
    done = 0
    while done < 40:
        n2 = int(rng.integers(2, 400))
        n1 = int(rng.integers(1, 70))
        n0 = int(rng.integers(1, 24))
        if rng.random() < 0.6:
            n2 += n2 & 1
        seed = int(rng.integers(0, 1 << 30))
        shape = (n0, n1, n2)
        print(f"\n[gpu] random shape {shape} seed {seed}", flush=True)
        img = gen.cfg_u14_value_noise(shape, seed=seed)
        t = torch.from_numpy(img.view(np.int16)).cuda()
        assert (ecc.compute(t, "u14").cpu().numpy() == oracle.curve(img, m=16384)).all(), shape
        assert (ecc.compute_max_entry(t, "u14").cpu().numpy() == oracle.curve_max_entry(img, m=16384)).all(), shape
        done += 1
