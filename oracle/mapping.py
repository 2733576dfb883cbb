"""FE <-> FFT mapping by nearest Gauss point (oracle, test only).

Sec. 3: the Gauss points of the finite-element mesh seed a Voronoi
tessellation of the FFT grid; each FFT cell lies in one domain and takes the
data of that Gauss point (the phase-field source rate, or here any per-point
field such as the plastic strain). Table 1 ends by mapping the volume
fractions back from the cells to the Gauss points; Sec. 5 compares this
"VoronoiMap" with an inverse-distance interpolation and keeps it.

Readings (the paper does not fix them):
* Cell (i, j, k) (x fastest) has its centre at ((i + 1/2) dx, (j + 1/2) dx,
  (k + 1/2) dx) in the frame of the Gauss points; distances are Euclidean and
  not periodic (the finite-element body does not wrap around).
* Ties go to the lower Gauss-point index. The squared distance is
  (px - cx)^2 + (py - cy)^2 + (pz - cz)^2, summed in that order in FP64: it
  decides an index, so every implementation must form it the same way.
* Back to the points: a Gauss point takes the mean of the cells of its
  domain; a point whose domain holds no cell centre (points denser than the
  grid) takes the cell containing it (clamped to the grid).
"""

import numpy as np


def cell_centres(shape, dx):
    """(nz, ny, nx, 3) centres (x, y, z) of the grid cells."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([(x + 0.5) * dx, (y + 0.5) * dx, (z + 0.5) * dx], axis=-1)


def voronoi_cells(points, shape, dx, chunk=4096):
    """Index (int32, (nz, ny, nx)) of the Gauss point nearest to each cell
    centre, by brute force over all points (ties: lowest index)."""
    p = np.asarray(points, dtype=np.float64)
    c = cell_centres(shape, dx).reshape(-1, 3)
    out = np.empty(c.shape[0], dtype=np.int32)
    for s in range(0, c.shape[0], chunk):
        cc = c[s:s + chunk]
        d2 = (p[None, :, 0] - cc[:, None, 0]) ** 2
        d2 = d2 + (p[None, :, 1] - cc[:, None, 1]) ** 2
        d2 = d2 + (p[None, :, 2] - cc[:, None, 2]) ** 2
        out[s:s + chunk] = np.argmin(d2, axis=1)   # first minimum: lowest index
    return out.reshape(shape)


def to_cells(cell_point, point_values):
    """point_values (ncomp, n_points) -> cell values (ncomp, nz, ny, nx)."""
    v = np.asarray(point_values)
    return v[:, cell_point]


def containing_cell(points, shape, dx):
    """Flat index of the cell containing each point, clamped to the grid."""
    nz, ny, nx = shape
    p = np.asarray(points, dtype=np.float64)
    i = np.clip(np.floor(p[:, 0] / dx).astype(np.int64), 0, nx - 1)
    j = np.clip(np.floor(p[:, 1] / dx).astype(np.int64), 0, ny - 1)
    k = np.clip(np.floor(p[:, 2] / dx).astype(np.int64), 0, nz - 1)
    return (k * ny + j) * nx + i


def to_points(cell_point, cell_values, points, dx):
    """cell_values (ncomp, nz, ny, nx) -> point values (ncomp, n_points):
    the mean over each point's domain, or its containing cell."""
    cv = np.asarray(cell_values, dtype=np.float64)
    ncomp = cv.shape[0]
    shape = cv.shape[1:]
    n = np.asarray(points).shape[0]
    idx = cell_point.ravel()
    cnt = np.bincount(idx, minlength=n).astype(np.float64)
    inside = containing_cell(points, shape, dx)
    out = np.empty((ncomp, n))
    for c in range(ncomp):
        s = np.bincount(idx, weights=cv[c].ravel(), minlength=n)
        mean = np.divide(s, cnt, out=np.zeros(n), where=cnt > 0)
        out[c] = np.where(cnt > 0, mean, cv[c].ravel()[inside])
    return out, cnt.astype(np.int64)
