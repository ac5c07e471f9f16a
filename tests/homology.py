"""Brute-force Z/2 homology of thresholded images (test helper, tiny inputs only).

T_t is built here as the CLOSURE of the voxels with value <= t: every face of
every such voxel cube.  For the dual complex (voxels as vertices) the cells
spanned by the vertices with value <= t are built directly.  This is a different construction from the oracle's
(which gives each cell the minimum value of its incident voxels); the two
agree only if the sublevel sets of Sec. 2 are exactly these closures.
Betti numbers come from ranks of boundary matrices over GF(2), computed by
Gaussian elimination on Python-int bitsets.
"""
import itertools

import numpy as np


def closure_cells(mask: np.ndarray):
    """Cells (doubled coordinates) of the union of closed voxel cubes where mask is True."""
    d = mask.ndim
    cells = set()
    for p in zip(*np.nonzero(mask)):
        for s in itertools.product((-1, 0, 1), repeat=d):
            cells.add(tuple(2 * pi + 1 + si for pi, si in zip(p, s)))
    return cells


def boundary(cell):
    """Faces of codimension 1: move one odd (interval) coordinate by +-1."""
    out = []
    for k, qk in enumerate(cell):
        if qk % 2:
            for dq in (-1, 1):
                c = list(cell)
                c[k] = qk + dq
                out.append(tuple(c))
    return out


def gf2_rank(rows):
    """Rank over GF(2) of a list of int bitsets."""
    pivots = {}
    rank = 0
    for r in rows:
        while r:
            top = r.bit_length() - 1
            if top in pivots:
                r ^= pivots[top]
            else:
                pivots[top] = r
                rank += 1
                break
    return rank


def dual_cells(mask: np.ndarray):
    """Cells of the dual complex spanned by the voxels where mask is True: the
    voxels are vertices; doubled coordinate p_k even = voxel index p_k/2, odd =
    the pair of neighbours (p_k-1)/2, (p_k+1)/2; a cell is present iff all its
    vertices are."""
    d = mask.ndim
    cells = set()
    for p in itertools.product(*[range(2 * n - 1) for n in mask.shape]):
        verts = itertools.product(*[(q // 2,) if q % 2 == 0 else (q // 2, q // 2 + 1) for q in p])
        if all(mask[v] for v in verts):
            cells.add(p)
    return cells


def betti(mask: np.ndarray):
    """(betti numbers beta_0..beta_d, cell counts n_0..n_d) of the closure of mask."""
    return betti_cells(closure_cells(mask), mask.ndim)


def betti_cells(cells, d: int):
    """(betti numbers, cell counts) of a cubical complex given by its cells in
    doubled coordinates (odd coordinate = interval factor)."""
    by_dim = [[] for _ in range(d + 1)]
    for c in cells:
        by_dim[sum(q % 2 for q in c)].append(c)
    index = [{c: i for i, c in enumerate(sorted(cs))} for cs in by_dim]
    ranks = [0] * (d + 2)
    for k in range(1, d + 1):
        rows = []
        for c in by_dim[k]:
            bits = 0
            for f in boundary(c):
                assert f in index[k - 1], "the cells are not a complex"
                bits ^= 1 << index[k - 1][f]
            rows.append(bits)
        ranks[k] = gf2_rank(rows)
        if k >= 2:
            # boundary of boundary is zero: every (k-2)-face appears an even number of times
            for c in by_dim[k]:
                acc = {}
                for f in boundary(c):
                    for g in boundary(f):
                        acc[g] = acc.get(g, 0) ^ 1
                assert not any(acc.values()), "dd != 0"
    n = [len(cs) for cs in by_dim]
    beta = [n[k] - ranks[k] - ranks[k + 1] for k in range(d + 1)]
    return beta, n
