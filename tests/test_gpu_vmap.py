"""GPU: the FE <-> FFT mapping by nearest Gauss point through the C ABI
against the oracle's brute force. The cell -> point map is index work:
bit-exact, ties included. The transfer to the cells is a copy: bit-exact.
The mean back to the points sums in FP64 in ascending cell order, as the
oracle's bincount does, then divides once: bit-exact too.
"""

import numpy as np
import pytest

from oracle import mapping as om
from paper_2302_13612_amd import binding, inputs

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def run(points, shape, dx, ncomp=3, seed=0):
    import torch
    pts = torch.from_numpy(np.ascontiguousarray(points, dtype=np.float64)).cuda()
    vm = binding.VoronoiMap(pts, shape, dx)
    cp = vm.cell_point.cpu().numpy()
    rng = np.random.default_rng(seed)
    pv = rng.normal(size=(ncomp, points.shape[0])).astype(np.float32)
    cv = vm.to_cells(torch.from_numpy(pv).cuda()).cpu().numpy()
    cells = rng.normal(size=(ncomp,) + tuple(shape)).astype(np.float32)
    back = vm.to_points(torch.from_numpy(cells).cuda()).cpu().numpy()
    return cp, pv, cv, cells, back


def check(points, shape, dx, label, ncomp=3):
    log(f"\n[vmap] {label}: grid {shape}, {points.shape[0]} points")
    cp, pv, cv, cells, back = run(points, shape, dx, ncomp)
    cp_o = om.voronoi_cells(points, shape, dx)
    mism = int((cp != cp_o).sum())
    log(f"  cell->point mismatches {mism}")
    assert mism == 0
    np.testing.assert_array_equal(cv, om.to_cells(cp_o, pv))
    back_o, _ = om.to_points(cp_o, cells.astype(np.float64), points, dx)
    np.testing.assert_array_equal(back, back_o.astype(np.float32))


def test_random_points_ragged_grid():
    rng = np.random.default_rng(1)
    shape, dx = (28, 20, 24), 0.1
    pts = rng.uniform(-0.5, 3.3, size=(3000, 3))
    check(pts, shape, dx, "random, some outside the grid")


def test_exact_ties_on_cell_corners():
    # every cell centre is equidistant from its eight corners: ties decide
    shape, dx = (6, 7, 8), 1.0
    z, y, x = np.meshgrid(np.arange(7), np.arange(8), np.arange(9), indexing="ij")
    pts = np.stack([x, y, z], axis=-1).reshape(-1, 3).astype(np.float64)
    rng = np.random.default_rng(2)
    check(pts[rng.permutation(pts.shape[0])], shape, dx, "corner lattice, shuffled")


def test_pillar_mesh_with_pad():
    dx = 5e-8
    shape = (64, 40, 40)
    check(inputs.pillar_gauss_points(shape, dx, elem=2.5), shape, dx, "pillar mesh", ncomp=6)


def test_points_denser_than_cells():
    rng = np.random.default_rng(3)
    shape, dx = (8, 10, 12), 1.0
    pts = rng.uniform(0.0, 1.0, size=(5000, 3)) * np.array([12.0, 10.0, 8.0])
    check(pts, shape, dx, "denser than the grid")


@pytest.mark.parametrize("case", ["one", "duplicates", "plane"])
def test_degenerate_point_sets(case):
    shape, dx = (9, 11, 13), 1.0
    rng = np.random.default_rng(4)
    if case == "one":
        pts = np.array([[4.2, 3.3, 100.0]])
    elif case == "duplicates":
        pts = np.repeat(np.array([[2.0, 5.0, 4.0], [9.5, 1.0, 7.0]]), 50, axis=0)[rng.permutation(100)]
    else:
        pts = np.concatenate([rng.uniform(0, 13, size=(200, 2)), np.full((200, 1), 4.5)], axis=1)
    check(pts, shape, dx, case)


def test_rejects_non_finite_points():
    import torch
    pts = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    pts[3, 1] = float("nan")
    with pytest.raises(binding.PfError):
        binding.VoronoiMap(pts, (4, 4, 4), 1.0)


def test_full_size_sampled_cells():
    """128 x 128 x 256 with the bench's pillar mesh: sampled cells against a
    brute-force search over every point."""
    import torch
    dx = 5e-8
    shape = (256, 128, 128)
    pts = inputs.pillar_gauss_points(shape, dx, elem=4.0)
    vm = binding.VoronoiMap(torch.from_numpy(pts).cuda(), shape, dx)
    cp = vm.cell_point.cpu().numpy().ravel()
    rng = np.random.default_rng(5)
    sample = rng.choice(cp.size, size=400, replace=False)
    cen = om.cell_centres(shape, dx).reshape(-1, 3)[sample]
    for s, c in zip(sample, cen):
        d2 = (pts[:, 0] - c[0]) ** 2
        d2 = d2 + (pts[:, 1] - c[1]) ** 2
        d2 = d2 + (pts[:, 2] - c[2]) ** 2
        assert cp[s] == int(np.argmin(d2)), s
    log(f"\n[vmap] full size {shape}, {pts.shape[0]} points: 400 sampled cells exact")


def test_few_points_own_a_large_grid():
    """Domains of hundreds of thousands of cells each (the per-point cell
    lists come from a stable radix sort, not a per-list sort)."""
    pts = np.array([[10.0, 100.0, 64.0], [120.0, 20.0, 5.0], [60.0, 60.0, 120.0]])
    check(pts, (128, 128, 128), 1.0, "three points, 128^3", ncomp=2)


def test_to_cells_unaligned_and_ragged():
    """The gather's vector path needs 16-byte aligned arrays and a cell count
    divisible by 4; other arrays take the scalar path, with the same result."""
    import torch
    rng = np.random.default_rng(6)
    shape, dx = (5, 6, 7), 1.0                  # 210 cells: not a multiple of 4
    pts = rng.uniform(0, 7, size=(40, 3))
    vm = binding.VoronoiMap(torch.from_numpy(pts).cuda(), shape, dx)
    pv = torch.from_numpy(rng.normal(size=(2, 40)).astype(np.float32)).cuda()
    expect = om.to_cells(om.voronoi_cells(pts, shape, dx), pv.cpu().numpy())
    np.testing.assert_array_equal(vm.to_cells(pv).cpu().numpy(), expect)
    shape2 = (4, 6, 8)                          # 192 cells, then an output offset by one float
    vm2 = binding.VoronoiMap(torch.from_numpy(pts).cuda(), shape2, dx)
    buf = torch.empty(2 * 192 + 1, dtype=torch.float32, device="cuda")
    out = buf[1:].view((2,) + shape2)
    vm2.to_cells(pv, out=out)
    expect2 = om.to_cells(om.voronoi_cells(pts, shape2, dx), pv.cpu().numpy())
    np.testing.assert_array_equal(out.cpu().numpy(), expect2)
