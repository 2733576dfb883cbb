"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random numbers and builds input arrays (initial twin
nuclei, grain maps, grain orientations, plastic-strain fields, loads). It holds
none of the method's arithmetic: no stiffness, eigenstrain, Green's operator
or update. Every array is produced in float64 and rounded once to float32 for
the fields the GPU path consumes; callers hand the same float32 values (as
float64) to any checker.

Workload recipes (grids follow the paper's FFT grids: a 1:1:2 box like the
64x64x128 micro-pillar grid of Sec. 4.2, and polycrystals as in Sec. 5):
* single_crystal_sphere: 32^3, one spherical nucleus, homogeneous stiffness.
* single_crystal_lamellae: 128x128x256, three disc-shaped nuclei, parent/twin
  stiffness contrast, Gaussian-random-field plastic strain, ramped load.
* polycrystal: 256^3, 64 periodic Voronoi grains with uniformly random
  orientations, six twin variants, nuclei at 5% of the grain-pair
  interfaces, Gaussian-random-field plastic strain, fixed load.
* rve_batch: an ensemble of 256 single-crystal cubes of edge 32, 48, 64 or 96
  (uniform), each with a random orientation, homogeneous stiffness, one to
  four spherical nuclei and its own uniaxial strain along x.
"""

import numpy as np

VOIGT_NAMES = ("xx", "yy", "zz", "yz", "xz", "xy")


def rng_for(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ------------------------------------------------------------- nuclei
def sphere(shape, center, radius):
    """Boolean ball of voxel-centre indices within radius (periodic)."""
    nz, ny, nx = shape
    z = np.arange(nz)[:, None, None]
    y = np.arange(ny)[None, :, None]
    x = np.arange(nx)[None, None, :]
    cz, cy, cx = center

    def pd(a, c, n):
        d = np.abs(a - c)
        return np.minimum(d, n - d)

    r2 = pd(z, cz, nz) ** 2 + pd(y, cy, ny) ** 2 + pd(x, cx, nx) ** 2
    return r2 <= radius * radius


def disc(shape, center, normal_xyz, radius, half_thickness):
    """Boolean periodic disc: |d.n| <= half_thickness and |d - (d.n)n| <= radius."""
    nz, ny, nx = shape
    n = np.asarray(normal_xyz, float)
    n = n / np.linalg.norm(n)
    cz, cy, cx = center

    def pd(a, c, N):
        d = a - c
        return (d + N / 2.0) % N - N / 2.0

    dz = pd(np.arange(nz)[:, None, None], cz, nz)
    dy = pd(np.arange(ny)[None, :, None], cy, ny)
    dx = pd(np.arange(nx)[None, None, :], cx, nx)
    along = dx * n[0] + dy * n[1] + dz * n[2]
    r2 = dx * dx + dy * dy + dz * dz - along * along
    return (np.abs(along) <= half_thickness) & (r2 <= radius * radius)


# ----------------------------------------------------- plastic strain
def gaussian_random_field(shape, corr_len, rng):
    """Zero-mean, unit-RMS periodic field with covariance exp(-r^2/(2 l^2))
    (spectral filter exp(-|k|^2 l^2 / 4), k in rad/voxel)."""
    white = rng.standard_normal(shape)
    nz, ny, nx = shape
    kz = 2 * np.pi * np.fft.fftfreq(nz)[:, None, None]
    ky = 2 * np.pi * np.fft.fftfreq(ny)[None, :, None]
    kx = 2 * np.pi * np.fft.rfftfreq(nx)[None, None, :]
    filt = np.exp(-(kx * kx + ky * ky + kz * kz) * corr_len * corr_len / 4.0)
    f = np.fft.irfftn(np.fft.rfftn(white) * filt, s=shape, axes=(0, 1, 2))
    f -= f.mean()
    return f / np.sqrt((f * f).mean())


def plastic_strain_grf(shape, corr_len, rms, rng):
    """(6, nz, ny, nx) float32 traceless plastic strain, tensor-Voigt order.

    Three unit fields for the normal components are projected to zero trace
    and rescaled by sqrt(3/2); three more give the shears; every component has
    the given RMS and zero mean.
    """
    d = np.stack([gaussian_random_field(shape, corr_len, rng) for _ in range(3)])
    d = (d - d.mean(axis=0, keepdims=True)) * np.sqrt(1.5)
    s = np.stack([gaussian_random_field(shape, corr_len, rng) for _ in range(3)])
    e = np.concatenate([d, s]) * rms
    e -= e.mean(axis=(1, 2, 3), keepdims=True)
    return e.astype(np.float32)


# ------------------------------------------------------- microstructure
def random_rotations(n, rng):
    """n uniformly random rotation matrices (Shoemake's quaternion method),
    mapping crystal-frame vectors to sample-frame vectors."""
    u1, u2, u3 = rng.random((3, n))
    q0 = np.sqrt(1 - u1) * np.sin(2 * np.pi * u2)
    q1 = np.sqrt(1 - u1) * np.cos(2 * np.pi * u2)
    q2 = np.sqrt(u1) * np.sin(2 * np.pi * u3)
    q3 = np.sqrt(u1) * np.cos(2 * np.pi * u3)
    w, x, y, z = q3, q0, q1, q2
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def rotation_to_bunge(R):
    """Bunge (phi1, Phi, phi2) in radians of a crystal->sample rotation R
    (g = R^T maps sample to crystal)."""
    g = np.asarray(R).T
    Phi = np.arccos(np.clip(g[2, 2], -1.0, 1.0))
    if abs(np.sin(Phi)) > 1e-12:
        phi1 = np.arctan2(g[2, 0], -g[2, 1])
        phi2 = np.arctan2(g[0, 2], g[1, 2])
    else:
        phi1 = np.arctan2(g[0, 1], g[0, 0])
        phi2 = 0.0
    return phi1 % (2 * np.pi), Phi, phi2 % (2 * np.pi)


def voronoi_grains(shape, n_grains, rng):
    """Periodic Voronoi map (uint8 grain id per voxel, seeds uniform in the box)."""
    from scipy.spatial import cKDTree
    nz, ny, nx = shape
    seeds = rng.random((n_grains, 3)) * np.array([nz, ny, nx])
    tree = cKDTree(seeds, boxsize=[nz, ny, nx])
    gid = np.empty(shape, dtype=np.uint8)
    yy, xx = np.meshgrid(np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    for z in range(nz):
        pts = np.stack([np.full(yy.size, z + 0.5), yy.ravel(), xx.ravel()], axis=1)
        pts %= np.array([nz, ny, nx])
        _, idx = tree.query(pts)
        gid[z] = idx.reshape(ny, nx)
    return gid


def grain_pair_interfaces(gid):
    """Unique (g1 < g2) pairs of grains that touch across a voxel face, with
    one list of boundary voxels (flat indices) per pair."""
    pairs = {}
    for axis in range(3):
        nb = np.roll(gid, -1, axis=axis)
        diff = gid != nb
        idx = np.flatnonzero(diff)
        a = gid.ravel()[idx]
        b = nb.ravel()[idx]
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        for key in np.unique(lo.astype(np.int64) * 256 + hi):
            sel = idx[(lo.astype(np.int64) * 256 + hi) == key]
            pairs.setdefault((int(key // 256), int(key % 256)), []).append(sel)
    return {k: np.concatenate(v) for k, v in sorted(pairs.items())}


def boundary_nuclei(gid, n_var, fraction, radius, rng, grain_variant=None):
    """eta0 (n_var, ...) with spheres centred on random boundary voxels of a
    random `fraction` (at least one) of the grain-pair interfaces, each of the
    variant grain_variant[g] of the grain g of its centre voxel (a random
    variant without it; the draw is made either way, so both choices place
    the same spheres). A voxel already inside a nucleus keeps its first
    variant."""
    shape = gid.shape
    pairs = grain_pair_interfaces(gid)
    keys = list(pairs.keys())
    n_pick = max(1, int(round(fraction * len(keys))))
    chosen = rng.choice(len(keys), size=n_pick, replace=False)
    eta = np.zeros((n_var,) + shape, dtype=np.float64)
    taken = np.zeros(shape, dtype=bool)
    for c in sorted(chosen):
        vox = pairs[keys[c]]
        flat = vox[rng.integers(len(vox))]
        center = np.unravel_index(flat, shape)
        var = int(rng.integers(n_var))
        if grain_variant is not None:
            var = int(grain_variant[gid[center]])
        ball = sphere(shape, center, radius) & ~taken
        eta[var][ball] = 1.0
        taken |= ball
    return eta.astype(np.float32), n_pick, len(keys)


# -------------------------------------------------------------- recipes
MG_PARAMS = dict(A=1e7, kappa=1e-9, L=1.2e-5, dt=2e-4, dx=5e-8)


def single_crystal_sphere(n=32, radius=4, strain=-2e-3, steps=200):
    """32^3 homogeneous single crystal, c || z, load along x = [10-10]."""
    shape = (n, n, n)
    c = n // 2
    eta0 = sphere(shape, (c, c, c), radius)[None].astype(np.float32)
    eps_bar = np.zeros(6)
    eps_bar[0] = strain
    return dict(
        name="single_crystal_sphere", shape=shape, n_var=1, variant_ids=[0],
        rotations=np.eye(3)[None], homogeneous=True, gid=None,
        eta0=eta0, eps_p=None, steps=steps,
        eps_bar=eps_bar, sig_bar=np.zeros(6),
        stress_mask=np.array([False, True, True, True, True, True]),
        ms_tol=1e-6, ms_max_iter=1, **MG_PARAMS)


# crystal x=[10-10] -> sample z (long axis), crystal z=[0001] -> sample x.
PILLAR_ROTATION = np.array([[0.0, 0.0, 1.0],
                            [0.0, -1.0, 0.0],
                            [1.0, 0.0, 0.0]])


def single_crystal_lamellae(shape=(256, 128, 128), seed=2, corr_len=8.0,
                            rms=1e-3, final_strain=-4e-3, steps=2000,
                            n_nuclei=3, radius=12.0, half_thickness=2.0):
    """Single crystal with parent/twin contrast, loaded along its long axis z."""
    rng = rng_for(seed)
    eps_p = plastic_strain_grf(shape, corr_len, rms, rng)
    eta = np.zeros(shape, dtype=bool)
    normal = (0.7276, 0.0, 0.6860)    # disc normal (x, y, z), sample frame
    for _ in range(n_nuclei):
        center = tuple(rng.random(3) * np.array(shape))
        eta |= disc(shape, center, normal, radius, half_thickness)
    return dict(
        name="single_crystal_lamellae", shape=shape, n_var=1, variant_ids=[0],
        rotations=PILLAR_ROTATION[None], homogeneous=False, gid=None,
        eta0=eta[None].astype(np.float32), eps_p=eps_p, steps=steps,
        final_strain=final_strain,
        stress_mask=np.array([True, True, False, True, True, True]),
        ms_tol=1e-6, ms_max_iter=50, **MG_PARAMS)


def ramp_load(cfg, n):
    """Load of step n (0-based) of the ramped single-crystal recipe."""
    eps_bar = np.zeros(6)
    eps_bar[2] = cfg["final_strain"] * (n + 1) / cfg["steps"]
    return eps_bar, np.zeros(6)


def polycrystal(shape=(256, 256, 256), n_grains=64, seed=3, n_var=6,
                nuc_fraction=0.05, radius=3, rms=2e-3, corr_len=8.0,
                strain=-5e-3, steps=1000, variant_for=None):
    """Voronoi polycrystal with all six twin variants per voxel.

    variant_for: optional callable (rotations (G, 3, 3), eps_bar (6,)) ->
    the variant (0..n_var-1) each grain's nuclei take, e.g. its largest
    Schmid factor under the load; the caller computes it with its own
    crystallography (this module holds none). Without it each nucleus takes
    a random variant."""
    rng = rng_for(seed)
    gid = voronoi_grains(shape, n_grains, rng)
    rot = random_rotations(n_grains, rng)
    eps_bar = np.zeros(6)
    eps_bar[0] = strain
    gv = None if variant_for is None else np.asarray(variant_for(rot, eps_bar), dtype=np.int64)
    eta0, n_nuc, n_pairs = boundary_nuclei(gid, n_var, nuc_fraction, radius, rng, gv)
    eps_p = plastic_strain_grf(shape, corr_len, rms, rng)
    # Six variants couple through the elastic energy: the largest eigenvalue of
    # the Gram matrix eps0_a : C : eps0_b of the Mg variants is ~1.5e9 J/m^3,
    # so the explicit update needs L dt (2A + 1.5e9) < 2; dt = 4e-5 s keeps the
    # same margin (~0.75) as the single-variant recipes at dt = 2e-4 s.
    params = dict(MG_PARAMS, dt=4e-5)
    return dict(
        name="polycrystal", shape=shape, n_var=n_var, variant_ids=list(range(n_var)),
        rotations=rot, homogeneous=False, gid=gid, n_grains=n_grains,
        eta0=eta0, eps_p=eps_p, steps=steps, n_nuclei=n_nuc, n_interfaces=n_pairs,
        eps_bar=eps_bar, sig_bar=np.zeros(6),
        stress_mask=np.array([False, True, True, True, True, True]),
        ms_tol=1e-6, ms_max_iter=50, **params)


def rve_batch(n_inst=256, seed=4, sizes=(32, 48, 64, 96), radius=4.0, max_nuclei=4,
              strain_range=(-5e-3, -1e-3), steps=512, save_every=16):
    """Ensemble of independent single-crystal cubes (one twin variant each,
    chosen by the caller: the one most favoured by compression along x)."""
    rng = rng_for(seed)
    insts = []
    for _ in range(n_inst):
        n = int(sizes[rng.integers(len(sizes))])
        shape = (n, n, n)
        R = random_rotations(1, rng)[0]
        k = int(rng.integers(1, max_nuclei + 1))
        eta = np.zeros(shape, dtype=bool)
        for _ in range(k):
            eta |= sphere(shape, tuple(rng.random(3) * n), radius)
        eps_bar = np.zeros(6)
        eps_bar[0] = rng.uniform(*strain_range)
        insts.append(dict(shape=shape, rotation=R, eta0=eta[None].astype(np.float32), eps_bar=eps_bar,
                          n_nuclei=k))
    return dict(
        name="rve_batch", instances=insts, n_var=1, homogeneous=True, gid=None, eps_p=None,
        steps=steps, save_every=save_every, sig_bar=np.zeros(6),
        stress_mask=np.array([False, True, True, True, True, True]),
        ms_tol=1e-6, ms_max_iter=1, **MG_PARAMS)


def pillar_gauss_points(shape, dx, pad=4, elem=2.5, jitter=0.2, seed=8):
    """Gauss points of a hexahedral finite-element mesh of a micro-pillar
    inside the FFT box (the box extends beyond the body by `pad` cells on
    every side, as the paper's pad layer does): elements of about `elem` cells
    per edge on a lattice whose interior nodes are jittered by up to
    `jitter` of an element edge, 2x2x2 Gauss points per element at the
    reference coordinates +-1/sqrt(3) mapped trilinearly. Returns (n, 3)
    float64 coordinates in metres (x, y, z), cell (i, j, k) centred at
    ((i + 1/2) dx, ...)."""
    rng = rng_for(seed)
    nz, ny, nx = shape
    lo = np.array([pad, pad, pad], dtype=np.float64) * dx
    hi = np.array([nx - pad, ny - pad, nz - pad], dtype=np.float64) * dx
    ne = np.maximum(1, np.round((hi - lo) / (elem * dx)).astype(int))
    axes = [np.linspace(lo[d], hi[d], ne[d] + 1) for d in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    nodes = np.stack([X, Y, Z], axis=-1)
    h = (hi - lo) / ne
    inner = np.zeros(nodes.shape[:3], dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    nodes[inner] += rng.uniform(-jitter, jitter, size=(inner.sum(), 3)) * h
    g = 1.0 / np.sqrt(3.0)
    pts = []
    for a in (-g, g):
        for b in (-g, g):
            for c in (-g, g):
                # trilinear map of the reference point (a, b, c) in every element
                xi = np.array([(1 - a) / 2, (1 + a) / 2])
                eta = np.array([(1 - b) / 2, (1 + b) / 2])
                zeta = np.array([(1 - c) / 2, (1 + c) / 2])
                p = 0.0
                for u in range(2):
                    for v in range(2):
                        for w in range(2):
                            p = p + xi[u] * eta[v] * zeta[w] * nodes[u:u + ne[0], v:v + ne[1], w:w + ne[2]]
                pts.append(p.reshape(-1, 3))
    return np.concatenate(pts, axis=0)


def pad_mobility(shape, pad=4, m_pad=1e-3):
    """Relative mobility of a specimen inside a pad layer of `pad` cells on
    every side (Sec. 4: very low mobility in the pad): 1 inside, m_pad in the
    pad. float32 (nz, ny, nx)."""
    m = np.full(shape, m_pad, dtype=np.float32)
    m[pad:shape[0] - pad, pad:shape[1] - pad, pad:shape[2] - pad] = 1.0
    return m
