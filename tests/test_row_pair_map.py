"""The row-pair layout of the integer kernel, checked on the host.

Interior waves of 16-bit images with an even row length read each row as
aligned dwords (tile_body / pair_offsets in ecc_int.hip): wave k of a row starts at
column 64 k + 1, lane l has column x0 + l, and the lane of column n2 (in the
last wave, an edge wave) takes column 0.  An interior ("full") wave, with
x0 + 63 <= n2 - 2, loads the dword at column x & ~1; for odd x that dword is
the pair (x-1, x), for even x the value at x-1 is the previous lane's own
value (its column is x-1).  This restates those formulas and checks, for many row
lengths and waves per workgroup:
  - every column [0, n2) is owned by exactly one lane;
  - every dword load of a full wave is 4-byte aligned and inside its row;
  - lane 0 of a full wave has an odd column (it never needs the lane before);
  - an even column's left neighbour is the previous lane's column.
"""
import pytest


def lane_map(n2, wx_cap):
    xs = -(-n2 // 64)
    wx = min(xs, wx_cap)
    tiles_x = -(-n2 // (64 * wx))
    for tx in range(tiles_x):
        for wxi in range(wx):
            x0 = (tx * wx + wxi) * 64 + 1
            if x0 >= n2:
                continue
            full = x0 + 63 <= n2 - 2
            for lane in range(64):
                x = x0 + lane
                if x == n2:
                    x = 0
                yield x0, full, lane, x


@pytest.mark.parametrize("wx_cap", [1, 2, 3, 8, 16])
def test_row_pair_map(wx_cap):
    for n2 in list(range(2, 700, 2)) + [1022, 1024, 1026, 4096, 8192, 14450]:
        owner = {}
        for x0, full, lane, x in lane_map(n2, wx_cap):
            if full:
                assert 1 <= x <= n2 - 2
                col = x & ~1
                assert (2 * col) % 4 == 0 and 2 * col + 4 <= 2 * n2
                if lane == 0:
                    assert x % 2 == 1
                if x % 2 == 0:
                    assert lane >= 1 and x0 + lane - 1 == x - 1
                else:
                    assert col == x - 1
            if x < n2:
                assert x not in owner, (n2, x)
                owner[x] = lane
        assert sorted(owner) == list(range(n2)), n2
