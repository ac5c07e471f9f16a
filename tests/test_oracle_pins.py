"""The oracle pinned to things other than itself.

- golden/: small images whose curves were derived by hand (each file cites the
  passage its reasoning uses);
- brute-force Z/2 homology of the closure of {f <= t} (a different construction
  of T_t), with beta_0 and beta_(d-1) also checked against scipy labelling;
- textbook reductions: runs in 1-D, components minus holes in 2-D;
- closed forms: empty complex below the minimum, contractible box at the top,
  constant images, a single voxel;
- invariants: flips, axis permutations, strictly increasing relabelling,
  splitting axis 0 into chunks each read with a one-voxel collar.
"""
import itertools
import pathlib

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from homology import betti, betti_cells, dual_cells

GOLDEN = pathlib.Path(__file__).parent / "golden"


def load_fixture(path):
    rec = {"rule": "min"}
    for line in path.read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        key, val = line.split(":", 1)
        key = key.strip()
        rec[key] = val.strip() if key == "rule" else [int(x) for x in val.split()]
    img = np.array(rec["values"], dtype=np.uint8).reshape(rec["shape"])
    return img, rec["m"][0], np.array(rec["chi"], dtype=np.int64), rec["rule"]


# hand-derived fixtures (the stored oracle results of the full-size
# workloads, stream_*.txt and serving_*.txt, are read by the GPU tests)
HAND_FIXTURES = sorted(p for p in GOLDEN.glob("*.txt") if not p.name.startswith(("stream_", "serving_")))


@pytest.mark.parametrize("path", HAND_FIXTURES, ids=lambda p: p.stem)
def test_golden_fixture(path):
    img, m, chi, rule = load_fixture(path)
    fn = {"min": oracle.curve, "max": oracle.curve_max_entry, "dual": oracle.curve_dual}[rule]
    assert (fn(img, m=m) == chi).all()


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_max_entry_identity_and_closed_forms(d):
    """Largest-value convention against the minimum one: min(M - f) = M - max f
    over every cell's voxels, so the max-convention count up to t is the
    complement, within the whole box (chi = 1), of the min-convention
    complex of M - f at M - t - 1:  max_f(t) = 1 - min_{M-f}(M - t - 1)."""
    rng = np.random.default_rng(40 + d)
    for _ in range(6):
        shape = tuple(int(x) for x in rng.integers(1, 6, size=d))
        m = int(rng.integers(2, 9))
        img = rand_img(rng, shape, m)
        got = oracle.curve_max_entry(img, m=m)
        inv = oracle.curve((m - 1 - img.astype(np.int64)).astype(img.dtype), m=m)
        want = 1 - np.concatenate([inv[::-1][1:], [0]])  # want[t] = 1 - inv[M - t - 1], inv[-1] = 0
        assert (got == want).all()
        lo, hi = int(img.min()), int(img.max())
        assert (got[:lo] == 0).all()
        assert (got[hi:] == 1).all()
        c = int(rng.integers(0, m))
        const = np.full(shape, c, dtype=img.dtype)
        assert (oracle.curve_max_entry(const, m=m) == (np.arange(m) >= c)).all()


def rand_img(rng, shape, m):
    return rng.integers(0, m, size=shape).astype(np.uint8 if m <= 256 else np.uint16)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
def test_closed_forms(d):
    rng = np.random.default_rng(d)
    for _ in range(6):
        shape = tuple(int(x) for x in rng.integers(1, 6, size=d))
        m = int(rng.integers(2, 9))
        img = rand_img(rng, shape, m)
        chi = oracle.curve(img, m=m)
        lo, hi = int(img.min()), int(img.max())
        assert (chi[:lo] == 0).all()          # empty complex below the minimum
        assert (chi[hi:] == 1).all()          # the full box is contractible
        c = int(rng.integers(0, m))
        const = np.full(shape, c, dtype=img.dtype)
        assert (oracle.curve(const, m=m) == (np.arange(m) >= c)).all()


def test_single_voxel_every_dimension():
    for d in range(1, 7):
        img = np.full((1,) * d, 2, dtype=np.uint8)
        assert (oracle.curve(img, m=4) == [0, 0, 1, 1]).all()


def _holes(mask):
    d = mask.ndim
    comp = np.pad(~mask, 1, constant_values=True)
    _, k = ndi.label(comp, structure=ndi.generate_binary_structure(d, 1))
    return k - 1


@pytest.mark.parametrize("shape,m,trials", [((8, 8), 4, 12), ((5, 7), 3, 12), ((4, 4, 4), 3, 6),
                                            ((3, 4, 5), 4, 6), ((9,), 4, 10)])
def test_homology_brute_force(shape, m, trials):
    rng = np.random.default_rng(sum(shape) * 31 + m)
    d = len(shape)
    for _ in range(trials):
        img = rand_img(rng, shape, m)
        chi = oracle.curve(img, m=m)
        for t in range(m):
            mask = img <= t
            beta, n = betti(mask)
            assert chi[t] == sum((-1) ** k * b for k, b in enumerate(beta))
            assert chi[t] == sum((-1) ** k * c for k, c in enumerate(n))
            assert all(b >= 0 for b in beta) and beta[d] == 0
            _, comps = ndi.label(mask, structure=np.ones((3,) * d))
            assert beta[0] == comps                    # (3^d - 1)-connectivity
            if d >= 2:
                assert beta[d - 1] == _holes(mask)     # Alexander duality


def test_1d_runs():
    rng = np.random.default_rng(11)
    for _ in range(50):
        n = int(rng.integers(1, 60))
        m = int(rng.integers(1, 10))
        img = rand_img(rng, (n,), m)
        chi = oracle.curve(img, m=m)
        for t in range(m):
            mask = (img <= t).astype(np.int8)
            runs = int(mask[0]) + int(np.sum((mask[1:] == 1) & (mask[:-1] == 0)))
            assert chi[t] == runs


def test_2d_components_minus_holes():
    rng = np.random.default_rng(12)
    import gen
    imgs = [rand_img(rng, (40, 37), 6) for _ in range(4)]
    imgs.append(gen.cfg_u8_value_noise((48, 64), seed=4) // 32)
    for img in imgs:
        m = int(img.max()) + 1
        chi = oracle.curve(img.astype(np.uint8), m=m)
        for t in range(m):
            mask = img <= t
            _, comps = ndi.label(mask, structure=np.ones((3, 3)))
            assert chi[t] == comps - _holes(mask)


def test_3d_tunnels_nonnegative():
    rng = np.random.default_rng(13)
    for _ in range(3):
        img = rand_img(rng, (12, 10, 11), 5)
        chi = oracle.curve(img, m=5)
        for t in range(5):
            mask = img <= t
            _, b0 = ndi.label(mask, structure=np.ones((3, 3, 3)))
            b2 = _holes(mask)
            assert b0 + b2 - chi[t] >= 0


@pytest.mark.parametrize("d", [2, 3, 4])
def test_flip_and_permutation_invariance(d):
    rng = np.random.default_rng(20 + d)
    shape = tuple(int(x) for x in rng.integers(2, 7, size=d))
    img = rand_img(rng, shape, 7)
    ref = oracle.curve(img, m=7)
    for ax in range(d):
        assert (oracle.curve(np.flip(img, ax), m=7) == ref).all()
    for perm in itertools.permutations(range(d)):
        assert (oracle.curve(np.transpose(img, perm), m=7) == ref).all()


def test_monotone_relabel():
    rng = np.random.default_rng(30)
    img = rand_img(rng, (9, 8, 7), 10)
    table = np.cumsum(rng.integers(1, 5, size=10))  # strictly increasing map 0..9 -> ...
    m2 = int(table[-1]) + 1
    img2 = table[img].astype(np.uint16)
    c1 = oracle.curve(img, m=10)
    c2 = oracle.curve(img2, m=m2)
    for t in range(10):
        hi = table[t + 1] if t + 1 < 10 else m2
        assert (c2[table[t]:hi] == c1[t]).all()
    assert (c2[: table[0]] == 0).all()


@pytest.mark.parametrize("shape", [(10, 6, 5), (7, 9), (6, 3, 4, 3)])
def test_chunks_with_collar_sum_to_whole(shape):
    """Each chunk of axis-0 planes, read with a one-voxel collar below it, yields
    the signed counts of its own cells; the parts add up (Sec. 3, Streaming and
    Processing one Chunk)."""
    rng = np.random.default_rng(40)
    m = 6
    img = rand_img(rng, shape, m)
    whole = oracle.vcec(img, m=m)
    n0 = shape[0]
    for cuts in [(0, n0), (0, 1, n0), (0, 3, 4, n0), tuple(range(n0 + 1))]:
        total = np.zeros(m, np.int64)
        for z0, z1 in zip(cuts[:-1], cuts[1:]):
            lo = max(z0 - 1, 0)
            sub = np.ascontiguousarray(img[lo:z1])
            q_lo = 2 * (z0 - lo)
            q_hi = 2 * (z1 - lo) + (1 if z1 == n0 else 0)
            total += oracle.vcec_q0_range(sub, m, q_lo, q_hi)
        assert (total == whole).all(), cuts


def test_threads_do_not_change_result():
    rng = np.random.default_rng(41)
    img = rand_img(rng, (17, 13, 11), 50)
    ref = oracle.curve(img, m=50, nthreads=1)
    for t in (2, 3, 7, 16):
        assert (oracle.curve(img, m=50, nthreads=t) == ref).all()


def test_value_out_of_range_is_rejected():
    with pytest.raises(ValueError):
        oracle.curve(np.array([[0, 5]], dtype=np.uint8), m=5)


def test_float_reading_matches_integer_curve():
    rng = np.random.default_rng(50)
    img = rand_img(rng, (6, 7, 5), 40)
    keys, chi = oracle.curve_float(img.astype(np.float32))
    ref = oracle.curve(img, m=40)
    assert (keys == np.unique(img).astype(np.float32)).all()
    assert (chi == ref[np.unique(img)]).all()


def test_float_signed_zero_and_nan():
    img = np.array([[-0.0, 1.0], [0.0, -np.inf]], dtype=np.float32)
    keys, chi = oracle.curve_float(img)
    assert list(keys) == [-np.inf, 0.0, 1.0] and not np.signbit(keys[1])
    # T_{-inf}: one pixel; T_0: three pixels of a 2x2 block (connected); T_1: full
    assert list(chi) == [1, 1, 1]
    with pytest.raises(ValueError):
        oracle.curve_float(np.array([1.0, np.nan], dtype=np.float32))


@pytest.mark.parametrize("shape,m,trials", [((8, 8), 4, 10), ((5, 7), 3, 10), ((4, 4, 4), 3, 5),
                                            ((3, 4, 5), 4, 5), ((9,), 4, 10), ((1, 6), 3, 5)])
def test_dual_homology_brute_force(shape, m, trials):
    """Dual complex (voxels as vertices): Z/2 homology of the cells spanned by
    {f <= t}; beta_0 = components under 2d-connectivity (scipy's default
    structuring element), beta_(d-1) = bounded components of the complement
    under full (3^d - 1) connectivity (the dual adjacency pair)."""
    rng = np.random.default_rng(sum(shape) * 37 + m)
    d = len(shape)
    for _ in range(trials):
        img = rand_img(rng, shape, m)
        chi = oracle.curve_dual(img, m=m)
        for t in range(m):
            mask = img <= t
            beta, n = betti_cells(dual_cells(mask), d)
            assert chi[t] == sum((-1) ** k * b for k, b in enumerate(beta))
            assert chi[t] == sum((-1) ** k * c for k, c in enumerate(n))
            assert all(b >= 0 for b in beta) and beta[d] == 0
            _, comps = ndi.label(mask, structure=ndi.generate_binary_structure(d, 1))
            assert beta[0] == comps
            if d >= 2:
                comp = np.pad(~mask, 1, constant_values=True)
                _, k = ndi.label(comp, structure=np.ones((3,) * d))
                assert beta[d - 1] == k - 1


def box_faces(shape):
    """Every face of the box of voxel indices: (codimension, index per axis or
    None for a free axis); fixed axes take the first or the last index."""
    d = len(shape)
    for fixed in itertools.product((None, 0, 1), repeat=d):
        yield sum(f is not None for f in fixed), tuple(
            None if f is None else (0 if f == 0 else shape[k] - 1) for k, f in enumerate(fixed))


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_dual_from_max_entry_of_faces(d):
    """The dual complex's cells are the largest-value convention's cells away
    from the box's outer boundary, with dimension d - dim; inclusion-exclusion
    over the box's faces: dual(f) = (-1)^d sum_F (-1)^codim(F) max_entry(f|F)
    (a 0-dimensional face contributes [f(corner) <= t])."""
    rng = np.random.default_rng(60 + d)
    for _ in range(5):
        shape = tuple(int(x) for x in rng.integers(1, 6, size=d))
        m = int(rng.integers(2, 9))
        img = rand_img(rng, shape, m)
        acc = np.zeros(m, dtype=np.int64)
        for codim, idx in box_faces(shape):
            sub = img[tuple(slice(None) if i is None else i for i in idx)]
            if sub.ndim == 0:
                a = (np.arange(m) >= int(sub)).astype(np.int64)
            else:
                a = oracle.curve_max_entry(np.ascontiguousarray(sub), m=m)
            acc += (-1) ** codim * a
        assert (oracle.curve_dual(img, m=m) == (-1) ** d * acc).all()


@pytest.mark.parametrize("shape,m", [((4, 4, 4), 3), ((3, 4, 5), 4), ((1, 6, 2), 5), ((5, 1, 1), 4)])
def test_vcec3_homology_brute_force(shape, m):
    """The three-loop enumeration against Z/2 homology of {f <= t} for every t
    (the same pin as the general enumeration's)."""
    rng = np.random.default_rng(sum(shape) * 17 + m)
    for _ in range(4):
        img = rand_img(rng, shape, m)
        chi = np.cumsum(oracle.vcec3_q0_range(img, m, 0, 2 * shape[0] + 1, nthreads=2))
        for t in range(m):
            beta, _ = betti(img <= t)
            assert chi[t] == sum((-1) ** k * b for k, b in enumerate(beta))


@pytest.mark.parametrize("shape,elem", [((9, 13, 11), np.uint8), ((6, 1, 40), np.uint16), ((2, 33, 3), np.uint32),
                                        ((1, 1, 1), np.uint16), ((12, 7, 2), np.uint16)], ids=str)
def test_vcec3_matches_general_enumeration(shape, elem):
    """oracle_vcec3 counts the same cells as the d-dimensional enumeration, on
    every q_0 range tried (whole, a prefix, a suffix, single layers), for every
    thread count."""
    rng = np.random.default_rng(int(np.prod(shape)) + 5)
    m = 37
    img = rng.integers(0, m, size=shape).astype(elem)
    top = 2 * shape[0] + 1
    for lo, hi in [(0, top), (0, 3), (2, top), (1, 2), (top - 1, top), (3, 3)]:
        want = oracle.vcec_q0_range(img, m, lo, hi)
        for threads in (1, 3, 8):
            assert (oracle.vcec3_q0_range(img, m, lo, hi, nthreads=threads) == want).all(), (lo, hi, threads)


def test_large_golden_chunks_sum_to_whole():
    """The chunking of the script that writes the full-size stored curves:
    value-noise chunks with a one-plane collar add up to the whole volume's
    changes vector, for chunk lengths that divide the planes and ragged ones."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("mlg", GOLDEN / "make_large_goldens.py")
    mlg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mlg)
    import gen
    shape = (23, 17, 30)
    whole = oracle.vcec(gen.cfg_u14_value_noise(shape, seed=2), m=16384)
    for chunk in (1, 4, 5, 23, 40):
        total = np.zeros(16384, np.int64)
        for z0 in range(0, shape[0], chunk):
            total += mlg.chunk_vcec(shape, 2, z0, min(z0 + chunk, shape[0]), 2)
        assert (total == whole).all(), chunk
