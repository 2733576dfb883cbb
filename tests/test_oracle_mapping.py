"""Pins of the oracle's FE <-> FFT mapping by nearest Gauss point (Sec. 3 and
Table 1; compared with interpolation in Sec. 5).

* Points placed at cell centres own those cells (distance 0).
* Two points on a line along x split the grid at their bisector; a cell
  centre exactly on it (an exact tie in floating point) goes to the lower
  index, and to the other point when the two are listed the other way round.
  This fixes the cell-centre convention and the axis order too.
* Nearest distances agree with scipy's k-d tree, and the indices wherever
  the nearest point is unique.
* Back to the points: the counts times the means give back the sum over the
  cells; a point with an empty domain takes the cell that contains it.
"""

import numpy as np
from scipy.spatial import cKDTree

from oracle import mapping as om


def test_points_at_cell_centres_own_their_cells():
    shape, dx = (6, 7, 8), 0.5
    rng = np.random.default_rng(1)
    cells = rng.choice(np.prod(shape), size=40, replace=False)
    cen = om.cell_centres(shape, dx).reshape(-1, 3)
    far = np.array([[100.0, 100.0, 100.0]])
    pts = np.concatenate([far, cen[cells]])
    cp = om.voronoi_cells(pts, shape, dx).ravel()
    np.testing.assert_array_equal(cp[cells], np.arange(1, 41))
    assert not np.any(cp == 0)


def test_bisector_and_tie_rule():
    shape, dx = (3, 4, 9), 1.0
    a = np.array([2.5, 1.3, 0.7])
    b = np.array([6.5, 1.3, 0.7])      # bisector x = 4.5: the centre of column i = 4
    cp = om.voronoi_cells(np.stack([a, b]), shape, dx)
    i = np.arange(shape[2])
    expect = np.where(i <= 4, 0, 1)
    np.testing.assert_array_equal(cp, np.broadcast_to(expect, shape))
    cp2 = om.voronoi_cells(np.stack([b, a]), shape, dx)
    expect2 = np.where(i >= 4, 0, 1)
    np.testing.assert_array_equal(cp2, np.broadcast_to(expect2, shape))


def test_nearest_distances_match_kdtree():
    shape, dx = (10, 12, 14), 1.0
    rng = np.random.default_rng(2)
    pts = rng.uniform(-3.0, 17.0, size=(500, 3))
    cp = om.voronoi_cells(pts, shape, dx).ravel()
    cen = om.cell_centres(shape, dx).reshape(-1, 3)
    d_tree, i_tree = cKDTree(pts).query(cen, k=2)
    d_ours = np.sqrt(((pts[cp] - cen) ** 2).sum(axis=1))
    np.testing.assert_allclose(d_ours, d_tree[:, 0], rtol=0, atol=1e-12)
    unique = d_tree[:, 1] - d_tree[:, 0] > 1e-9
    np.testing.assert_array_equal(cp[unique], i_tree[unique, 0])


def test_back_map_conserves_and_falls_back():
    shape, dx = (4, 5, 6), 1.0
    rng = np.random.default_rng(3)
    pts = rng.uniform(0.0, 4.0, size=(400, 3)) * np.array([1.5, 1.25, 1.0])   # denser than the grid
    cp = om.voronoi_cells(pts, shape, dx)
    vals = rng.normal(size=(2,) + shape)
    out, cnt = om.to_points(cp, vals, pts, dx)
    for c in range(2):
        np.testing.assert_allclose((out[c] * cnt)[cnt > 0].sum(), vals[c].sum(), rtol=1e-12)
    empty = np.flatnonzero(cnt == 0)
    assert empty.size > 0
    for p in empty[:20]:
        i, j, k = (np.floor(pts[p] / dx)).astype(int)
        np.testing.assert_array_equal(out[:, p], vals[:, k, j, i])
    # and the forward map carries a point's value to every cell of its domain
    pv = rng.normal(size=(3, pts.shape[0]))
    cv = om.to_cells(cp, pv)
    np.testing.assert_array_equal(cv[:, cp == 7], np.repeat(pv[:, 7:8], (cp == 7).sum(), axis=1))
