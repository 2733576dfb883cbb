"""GPU: grids with the largest supported axes (192 = 2^6 3, 384 = 2^7 3 and
512 = 2^9) in each role (x: the fused real-to-complex passes, y, z: the
Green's operator and the Allen-Cahn divide), against the FP64 oracle.

Every one of these lengths is run as z, as y and as x in the polycrystal step
and in the spectral path; the other two axes stay small so that the oracle
finishes in seconds. The transform test covers every new length on every
axis.
Tolerances as for the other step parity tests: f max-abs <= 1e-4, stress
relative L2 <= 1e-5.
"""

import numpy as np
import pytest

from tests import cases
from tests.test_gpu_fft import make_solver
from tests.test_gpu_step import compare

pytestmark = pytest.mark.gpu

FFT_SHAPES = [(512, 48, 32), (32, 512, 48), (48, 32, 512), (384, 32, 192), (192, 384, 32),
              (32, 192, 384)]


@pytest.mark.parametrize("shape", FFT_SHAPES)
def test_transform_large_axes(shape):
    import torch
    print(f"\n[fft] shape={shape}", flush=True)
    solver = make_solver(shape)
    rng = np.random.default_rng(sum(shape) + 1)
    x = rng.standard_normal((2,) + shape).astype(np.float32)
    spec = solver.fft_forward(torch.from_numpy(x).cuda())
    back = solver.fft_inverse(spec)
    torch.cuda.synchronize()
    ref = np.fft.rfftn(x.astype(np.float64), axes=(1, 2, 3))
    got = spec.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    rel2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    d_back = np.abs(back.cpu().numpy() - x).max() / np.abs(x).max()
    print(f"  forward max {err:.2e} rel-L2 {rel2:.2e}; round trip max {d_back:.2e}", flush=True)
    solver.close()
    assert rel2 < 2e-7 and err < 2e-6
    assert d_back < 2e-6


# every large length in every role: 512 as z, y, x; 384 as z, y, x; 192 as z, y, x
@pytest.mark.parametrize("shape,n_var", [((512, 32, 32), 6), ((32, 512, 32), 2), ((32, 32, 512), 6),
                                         ((384, 32, 48), 2), ((32, 384, 32), 2), ((32, 48, 384), 2),
                                         ((192, 32, 48), 6), ((32, 192, 48), 6), ((32, 32, 192), 6)])
def test_polycrystal_large_axis(shape, n_var):
    cfg = cases.small_polycrystal(shape=shape, n_grains=6, seed=21, n_var=n_var)
    compare(cfg, 2, f"polycrystal {shape} {n_var} variants")


@pytest.mark.parametrize("shape", [(512, 32, 32), (32, 512, 32), (32, 32, 512), (384, 48, 32), (32, 384, 32),
                                   (32, 48, 384), (192, 32, 32), (32, 192, 48), (32, 32, 192)])
def test_spectral_path_large_axis(shape):
    """The homogeneous spectral path (one rotated stiffness, closed-form
    mechanics per wavevector) with a large axis in each role, 10 steps of a
    sphere nucleus, against the oracle."""
    from paper_2302_13612_amd import inputs
    from tests.test_gpu_batch import spectral_vs_oracle
    batch = inputs.rve_batch(n_inst=2, seed=17, sizes=(32,))
    cfg = cases.batch_instance_cfg(batch, 1)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (z - nz // 2) ** 2 + (y - ny // 2) ** 2 + (x - nx // 2) ** 2
    cfg.update(shape=shape, eta0=(r2 <= 16).astype(np.float32)[None])
    spectral_vs_oracle(cfg, 10, f"rotated sphere {shape}")
