"""A second CPU formulation of the VCEC (tests only, numpy, mid-size inputs).

Cells are grouped by which in-plane axes (all axes but the first) are
singletons: for each such set S the cell values on the voxel grid are the
2-window minima of f along the axes in S.  Along the first axis every line of
such a field is a 1-D complex (edges = the field values, vertices = minima of
neighbouring edges); each vertex is charged to the lower of its two edges, so
edge i carries (-1) plus the vertices it owns: c_{i-1} - c_i with
c_i = [g_{i+1} < g_i], c_{-1} = 1, c_{n-1} = 0.  Positions on the far
boundary of an in-plane axis i not in S are dropped together with the
matching positions of the field for S + {i} (the two lines are equal and
carry opposite signs).  Signs are (-1)^(number of interval axes).

It is derived from the same definitions as the oracle but shares no code with
it and does not enumerate cells, so agreement is a cross-check of both.
"""
import itertools

import numpy as np


def vcec_b(f: np.ndarray, m: int) -> np.ndarray:
    f = np.asarray(f).astype(np.int64)
    d = f.ndim
    n = f.shape
    nin = d - 1
    a = np.zeros(m, np.int64)
    big = np.int64(1) << 40
    for S in itertools.product((0, 1), repeat=nin):
        F = f
        for i, s in enumerate(S):
            if s:
                ax = i + 1
                prev = np.concatenate([np.take(F, [0], axis=ax), np.take(F, np.arange(n[ax] - 1), axis=ax)],
                                      axis=ax)
                F = np.minimum(F, prev)
        sign = (-1) ** (nin - sum(S))
        sl = [slice(None)] + [slice(None) if s else slice(0, n[i + 1] - 1) for i, s in enumerate(S)]
        G = F[tuple(sl)]
        if G.size == 0:
            continue
        pad = np.full((1,) + G.shape[1:], big)
        Gp = np.concatenate([pad, G, pad], axis=0)
        c = (Gp[1:] < Gp[:-1]).astype(np.int64)
        e = c[:-1] - c[1:]
        np.add.at(a, G.ravel(), sign * e.ravel())
    return a
