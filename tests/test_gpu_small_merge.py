"""GPU parity, exact int64, of 8-bit curves around the one-workgroup merge:
2-D u8 images whose per-workgroup rows number from 1 to 65 (the merge of at
most 64 rows runs in one workgroup, more rows take the three-kernel merge),
in the smallest-value and largest-value conventions and the dual complex,
each against the oracle."""
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


# n0 x 100 planes of one 64-column segment pair: n0 < 8 planes give n0
# workgroups, from 8 planes on each workgroup walks 8 (rows = ceil(n0 / 8))
ROWS_CASES = [(1, 1), (7, 7), (9, 2), (56, 7), (57, 8), (63, 8), (64, 8), (497, 63), (504, 63), (505, 64),
              (512, 64), (513, 65), (520, 65)]


@pytest.mark.parametrize("n0,rows", ROWS_CASES, ids=lambda x: str(x))
def test_u8_curves_around_small_merge(ecc, n0, rows):
    assert rows == (n0 if n0 < 8 else -(-n0 // 8))
    print(f"\n[gpu] small merge u8 ({n0}, 100), {rows} rows", flush=True)
    img = gen.iid((n0, 100), 8, seed=40 + n0)
    t = torch.from_numpy(img).cuda()
    got = ecc.compute(t, "u8").cpu().numpy()
    assert (got == oracle.curve(img, m=256)).all()
    got = ecc.compute_max_entry(t, "u8").cpu().numpy()
    assert (got == oracle.curve_max_entry(img, m=256)).all()
    got = ecc.compute_dual(t, "u8").cpu().numpy()
    assert (got == oracle.curve_dual(img, m=256)).all()


def test_u8_small_merge_repeated_calls_keep_status_clear(ecc):
    """Consecutive calls of both merge forms on one stream: each starts
    from a clear status word and writes its whole curve."""
    imgs = [gen.iid((n0, 100), 8, seed=90 + n0) for n0 in (20, 700, 3, 513, 64)]
    for img in imgs * 2:
        t = torch.from_numpy(img).cuda()
        assert (ecc.compute(t, "u8").cpu().numpy() == oracle.curve(img, m=256)).all()
