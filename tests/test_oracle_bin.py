"""Pins of the oracle's binning and canonical sort (connectivity rebuilt every
coupling step, Sec. 2.2) against brute force and library routines."""
import numpy as np
import pytest

import workload as W


def brute_cell(pos, box, nb):
    """Containing cell by testing the particle against the bounds of every cell.

    Cell i along an axis covers [i h, (i+1) h); the last cell also owns x = L.
    Positions outside [0, L] are first clamped into the box.
    """
    out = np.empty(pos.shape[0], dtype=np.int64)
    edges = [np.arange(nb[a] + 1) * (box[a] / nb[a]) for a in range(3)]
    for p in range(pos.shape[0]):
        idx = []
        for a in range(3):
            x = min(max(pos[p, a], 0.0), box[a]) if np.isfinite(pos[p, a]) else 0.0
            lo, hi = edges[a][:-1], edges[a][1:]
            inside = np.nonzero((lo <= x) & ((x < hi) | ((np.arange(nb[a]) == nb[a] - 1) & (x <= box[a]))))[0]
            idx.append(int(inside[0]))
        out[p] = idx[0] + nb[0] * (idx[1] + nb[1] * idx[2])
    return out


def test_bin_brute_force_cube8(orc):
    w = W.WORKLOADS["cube8_ngp_fp64"]
    pos, _, _ = W.particles(w)
    cell, nout = orc.bin_particles(pos, w.grid.box, w.grid.nb, prec32=False)
    assert nout == 0
    np.testing.assert_array_equal(cell, brute_cell(pos, w.grid.box, w.grid.nb))


@pytest.mark.parametrize("prec32", [False, True])
def test_bin_faces_walls_and_outside(orc, prec32):
    box, nb = (1.0, 0.75, 2.0), (4, 3, 8)
    h = [box[a] / nb[a] for a in range(3)]
    pts = []
    for a in range(3):  # every face plane along each axis, incl. x = 0 and x = L
        for i in range(nb[a] + 1):
            p = [0.3 * box[0], 0.4 * box[1], 0.55 * box[2]]
            p[a] = i * h[a]
            pts.append(p)
    pts += [[-0.1, 0.2, 0.2], [1.5, 0.2, 0.2], [0.2, 0.2, 9.0], [np.nan, 0.1, 0.1], [0.1, -np.inf, 0.1]]
    pts = np.array(pts, dtype=np.float32 if prec32 else np.float64)
    cell, nout = orc.bin_particles(pts, box, nb, prec32)
    assert nout == 5
    np.testing.assert_array_equal(cell, brute_cell(pts.astype(np.float64), box, nb))


def test_sort_matches_stable_argsort(orc):
    rng = np.random.default_rng(5)
    ncell = 97
    cell = rng.integers(0, ncell, 5000).astype(np.int32)
    perm, count, start = orc.sort_cells(cell, ncell)
    np.testing.assert_array_equal(perm, np.argsort(cell, kind="stable"))
    np.testing.assert_array_equal(count, np.bincount(cell, minlength=ncell))
    np.testing.assert_array_equal(start, np.concatenate([[0], np.cumsum(count)]))
    # canonical order: ascending (cell, id)
    key = cell[perm].astype(np.int64) * 10 ** 6 + perm
    assert np.all(np.diff(key) > 0)


def test_sort_empty_and_single_cell(orc):
    perm, count, start = orc.sort_cells(np.zeros(0, np.int32), 5)
    assert perm.size == 0 and np.all(count == 0) and np.all(start == 0)
    perm, count, start = orc.sort_cells(np.zeros(7, np.int32), 1)
    np.testing.assert_array_equal(perm, np.arange(7))
    assert count[0] == 7 and list(start) == [0, 7]
