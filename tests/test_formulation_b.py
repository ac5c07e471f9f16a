"""Second CPU formulation (per-axis minimum fields + 1-D ownership along axis 0)
against the cell-enumerating oracle, d = 1..4, including axes of length 1."""
import numpy as np
import pytest

import gen
import oracle
from formulation_b import vcec_b


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_matches_oracle_random(d):
    rng = np.random.default_rng(100 + d)
    for _ in range(40):
        hi = {1: 40, 2: 12, 3: 7, 4: 5}[d]
        shape = tuple(int(x) for x in rng.integers(1, hi, size=d))
        m = int(rng.integers(1, 12))
        img = rng.integers(0, m, size=shape).astype(np.uint8)
        assert (vcec_b(img, m) == oracle.vcec(img, m=m)).all(), shape


def test_matches_oracle_value_noise_3d():
    img = gen.cfg_u14_value_noise((40, 33, 47), seed=1)
    assert (vcec_b(img, 16384) == oracle.vcec(img, m=16384)).all()
