"""Host checks of the seeded synthetic workload generators."""

import numpy as np

from paper_2302_13612_amd import inputs


def test_grf_plastic_strain_statistics():
    e = inputs.plastic_strain_grf((16, 24, 32), 4.0, 2e-3, inputs.rng_for(1)).astype(np.float64)
    assert e.shape == (6, 16, 24, 32) and e.dtype == np.float64
    np.testing.assert_allclose(e[:3].sum(axis=0), 0.0, atol=1e-9)          # traceless
    np.testing.assert_allclose(e.mean(axis=(1, 2, 3)), 0.0, atol=1e-9)     # zero mean
    rms = np.sqrt((e ** 2).mean(axis=(1, 2, 3)))
    np.testing.assert_allclose(rms[3:], 2e-3, rtol=1e-5)
    np.testing.assert_allclose(rms[:3], 2e-3, rtol=0.25)


def test_rotations_are_proper_and_uniformish():
    R = inputs.random_rotations(2000, inputs.rng_for(2))
    np.testing.assert_allclose(np.einsum("nij,nkj->nik", R, R), np.broadcast_to(np.eye(3), R.shape), atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)
    # uniform rotations: E[R] = 0
    assert np.abs(R.mean(axis=0)).max() < 0.05
    phi1, Phi, phi2 = inputs.rotation_to_bunge(R[0])
    assert 0 <= phi1 < 2 * np.pi and 0 <= Phi <= np.pi


def test_voronoi_and_boundary_nuclei():
    rng = inputs.rng_for(3)
    gid = inputs.voronoi_grains((16, 16, 16), 8, rng)
    assert gid.dtype == np.uint8 and set(np.unique(gid)) <= set(range(8))
    pairs = inputs.grain_pair_interfaces(gid)
    assert len(pairs) >= 4
    eta, n_pick, n_pairs = inputs.boundary_nuclei(gid, 6, 0.05, 2, rng)
    assert n_pick == max(1, int(round(0.05 * n_pairs)))
    assert eta.shape == (6, 16, 16, 16)
    assert eta.sum(axis=0).max() == 1.0                           # no overlap
    assert set(np.unique(eta)) <= {0.0, 1.0}


def test_recipes_shapes():
    c = inputs.single_crystal_sphere()
    assert c["eta0"].shape == (1, 32, 32, 32) and c["eta0"].sum() == 257   # 4-voxel ball
    c = inputs.single_crystal_lamellae(shape=(32, 16, 16), radius=4.0)
    assert c["eps_p"].shape == (6, 32, 16, 16) and c["eta0"].any()
    e, s = inputs.ramp_load(c, c["steps"] - 1)
    assert e[2] == c["final_strain"]
