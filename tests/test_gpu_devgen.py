"""The device-made value noise and the streamed runs over it.

The 3-D 14-bit volume of 2600 planes of 14450 x 14450 voxels (seed 2, about
1.09 TB) exists only slab by slab in device memory.  Checked here:
  - the device generator writes the host generator's bytes (sampled planes of
    that volume, small shapes with odd rows and both element sizes);
  - its first planes, streamed from device slabs, give the oracle's curve;
  - the whole volume streamed in 64-plane slabs (the benchmark's launch
    configuration), and in ragged 100-plane slabs, gives the oracle's curve
    element by element, stored by tests/golden/make_large_goldens.py (the
    oracle over host-made chunks with a one-plane collar; Sec. 3,
    "Streaming": chunks add up);
  - the 1024 x 8192 x 8192 volume (128 GiB), resident and pushed from pinned
    host chunks, gives the oracle's curve, stored by
    tests/golden/make_large_goldens.py (the oracle over host-made chunks with
    a one-plane collar)."""
import hashlib
import importlib.util
import pathlib

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TB_SHAPE = (2600, 14450, 14450)
TB_SEED = 2
GOLDEN = pathlib.Path(__file__).parent / "golden"


def stored_curve(shape, seed):
    """The oracle's curve of the 14-bit value-noise volume, from its stored
    changes vector (checked against the stored digest of the curve)."""
    spec = importlib.util.spec_from_file_location("mlg", GOLDEN / "make_large_goldens.py")
    mlg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mlg)
    shp, sd, vcec, digest = mlg.read_stream(GOLDEN / mlg.stream_name(shape, seed))
    assert shp == tuple(shape) and sd == seed
    chi = np.cumsum(vcec)
    assert hashlib.sha256(chi.astype("<i8").tobytes()).hexdigest() == digest
    return chi


def assert_curve(got, want, what):
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, f"{what}: {len(bad)} thresholds differ, first {bad[:5]} got {got[bad[:5]]} want {want[bad[:5]]}"


@pytest.fixture(scope="module")
def ecc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1705_02045_amd as ecc
    return ecc


def dev_planes(shape, seed, z0, z1, bits=14, amp=64, elem=2):
    ent = gen.dev_table_entries(shape, z0, z1)
    table = torch.empty(ent, dtype=torch.int16, device="cuda")
    out = torch.empty((z1 - z0,) + tuple(shape[1:]), dtype=torch.int16 if elem == 2 else torch.uint8,
                      device="cuda")
    gen.value_noise_dev(out.data_ptr(), shape, bits, amp, seed, z0, z1, table.data_ptr(), ent, elem=elem,
                        stream=torch.cuda.current_stream().cuda_stream)
    return out


@pytest.mark.parametrize("shape,z0,z1", [((37, 53, 70), 0, 37), ((37, 53, 70), 5, 21), ((37, 53, 70), 16, 33),
                                         ((9, 11, 33), 0, 9), ((20, 1, 1), 3, 20), ((3, 17, 2), 1, 3)], ids=str)
def test_device_generator_matches_host_small(ecc, shape, z0, z1):
    got = dev_planes(shape, 5, z0, z1).cpu().numpy().view(np.uint16)
    assert (got == gen.value_noise(shape, 14, 64, 5, z0=z0, z1=z1)).all()
    got8 = dev_planes(shape, 6, z0, z1, bits=8, amp=1, elem=1).cpu().numpy()
    assert (got8 == gen.value_noise(shape, 8, 1, 6, z0=z0, z1=z1)).all()


@pytest.mark.parametrize("z0,z1", [(0, 1), (1023, 1025), (2599, 2600)], ids=str)
def test_device_generator_matches_host_full_width(ecc, z0, z1):
    print(f"\n[gpu] device generator planes [{z0}, {z1}) of {TB_SHAPE}", flush=True)
    got = dev_planes(TB_SHAPE, TB_SEED, z0, z1)
    want = gen.cfg_u14_value_noise(TB_SHAPE, seed=TB_SEED, z0=z0, z1=z1)
    assert bool((got == torch.from_numpy(want.view(np.int16)).cuda()).all())


def stream_device(ecc, shape, seed, slab, planes=None, cuts=None):
    """Streams planes [0, planes) of the value-noise volume of `shape` from
    device-made slabs (of `slab` planes, or between the given cuts); returns
    (curve, smallest value seen)."""
    planes = shape[0] if planes is None else planes
    full = (planes,) + tuple(shape[1:])
    cuts = list(range(0, planes, slab)) + [planes] if cuts is None else cuts
    spans = list(zip(cuts[:-1], cuts[1:]))
    ent = max(gen.dev_table_entries(shape, z0, z1) for z0, z1 in spans)
    width = max(z1 - z0 for z0, z1 in spans)
    table = torch.empty(ent, dtype=torch.int16, device="cuda")
    bufs = [torch.empty((width,) + tuple(shape[1:]), dtype=torch.int16, device="cuda") for _ in range(2)]
    s = torch.cuda.current_stream().cuda_stream
    st = ecc.Stream(full, "u14")
    lo = None
    for k, (z0, z1) in enumerate(spans):
        b = bufs[k % 2]
        gen.cfg_u14_value_noise_dev(b.data_ptr(), shape, seed, z0, z1, table.data_ptr(), table.numel(), stream=s)
        m = b[: z1 - z0].amin()  # 14-bit values: the int16 view is non-negative
        lo = m if lo is None else torch.minimum(lo, m)
        st.push(b, z1 - z0)
    return st.finish(), int(lo)


def test_stream_device_slabs_first_planes_vs_oracle(ecc):
    """Planes [0, 11) of the 1.09 TB volume (2.3 G voxels, 4.6 GB) against the
    oracle on the host bytes: resident (one launch of more than 4 GiB, four
    rows per wave), streamed as 1 + 10 planes (the second launch reads its
    first planes from the carry buffer, four rows per wave) and in slabs of
    4 planes (two rows per wave)."""
    planes = 11
    print("\n[gpu] first 11 planes of the TB volume: streamed 1 + 10", flush=True)
    got_a, _ = stream_device(ecc, TB_SHAPE, TB_SEED, 0, planes, cuts=[0, 1, planes])
    print("[gpu] streamed in slabs of 4", flush=True)
    got_b, _ = stream_device(ecc, TB_SHAPE, TB_SEED, 4, planes)
    print("[gpu] resident", flush=True)
    vol = dev_planes(TB_SHAPE, TB_SEED, 0, planes)
    got_c = ecc.compute(vol, "u14").cpu().numpy()
    del vol
    img = gen.cfg_u14_value_noise(TB_SHAPE, seed=TB_SEED, z0=0, z1=planes)
    print("[gpu] oracle ...", flush=True)
    ref = oracle.curve(img, m=16384)
    assert (got_a == ref).all()
    assert (got_b == ref).all()
    assert (got_c == ref).all()
    assert ref[-1] == 1


def test_stream_device_full_volume_vs_oracle(ecc):
    """The whole 2600 x 14450 x 14450 volume in 64-plane slabs, then in ragged
    slabs of 100 planes: both equal the oracle's stored curve element by
    element (and chi = 0 below the smallest value)."""
    want = stored_curve(TB_SHAPE, TB_SEED)
    print("\n[gpu] full TB volume, 64-plane slabs", flush=True)
    a, lo = stream_device(ecc, TB_SHAPE, TB_SEED, 64)
    assert_curve(a, want, "64-plane slabs")
    print("[gpu] full TB volume, 100-plane slabs", flush=True)
    b, lo2 = stream_device(ecc, TB_SHAPE, TB_SEED, 100)
    assert_curve(b, want, "100-plane slabs")
    assert lo == lo2 and (a[:lo] == 0).all()


def test_stream_host_full_size_vs_oracle(ecc):
    """The host-staged case at full size: 1024 planes of 8192 x 8192 (seed 2,
    128 GiB) made on the device; its curve computed resident in HBM, then the
    same bytes pushed from pinned host chunks of 16 planes: both equal the
    oracle's stored curve element by element."""
    shape = (1024, 8192, 8192)
    ref = stored_curve(shape, 2)
    print(f"\n[gpu] host-staged {shape}: device generation", flush=True)
    vol = torch.empty(shape, dtype=torch.int16, device="cuda")
    ent = gen.dev_table_entries(shape, 0, shape[0])
    table = torch.empty(ent, dtype=torch.int16, device="cuda")
    gen.cfg_u14_value_noise_dev(vol.data_ptr(), shape, 2, 0, shape[0], table.data_ptr(), ent,
                                stream=torch.cuda.current_stream().cuda_stream)
    del table
    print("[gpu] resident curve", flush=True)
    resident = ecc.compute(vol, "u14").cpu().numpy()
    assert_curve(resident, ref, "resident 128 GiB")
    print("[gpu] host-staged push", flush=True)
    ring = [torch.empty((16,) + shape[1:], dtype=torch.int16).pin_memory() for _ in range(2)]
    st = ecc.Stream(shape, "u14")
    for k, z0 in enumerate(range(0, shape[0], 16)):
        ring[k % 2].copy_(vol[z0:z0 + 16])
        st.push(ring[k % 2])
    got = st.finish()
    assert_curve(got, ref, "host-staged 128 GiB")
