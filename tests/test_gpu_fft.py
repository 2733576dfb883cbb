"""GPU: the library's 3D real-to-complex transforms against the FP64 FFT of
the same float32 input (the convention every spectral step of the oracle
uses), on grids with ragged spectral tiles and radix-3 axes."""

import numpy as np
import pytest

from tests import cases

pytestmark = pytest.mark.gpu

SHAPES = [(32, 32, 32), (48, 64, 32), (32, 48, 96), (96, 32, 64), (64, 128, 48), (256, 32, 128),
          (32, 256, 256)]


def make_solver(shape, n_var=1):
    from paper_2302_13612_amd import inputs
    cfg = inputs.single_crystal_sphere()
    cfg = dict(cfg, shape=shape, eta0=np.zeros((n_var,) + shape, np.float32), variant_ids=[0] * n_var,
               n_var=n_var)
    solver, _ = cases.gpu_solver(cfg)
    return solver


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_and_inverse_transform(shape):
    import torch
    print(f"\n[fft] shape={shape}", flush=True)
    solver = make_solver(shape)
    rng = np.random.default_rng(sum(shape))
    x = rng.standard_normal((3,) + shape).astype(np.float32)
    spec = solver.fft_forward(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    ref = np.fft.rfftn(x.astype(np.float64), axes=(1, 2, 3))
    got = spec.cpu().numpy()
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    rel2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"  forward max {err:.2e} rel-L2 {rel2:.2e}", flush=True)
    assert rel2 < 2e-7 and err < 2e-6
    back = solver.fft_inverse(spec).cpu().numpy()
    err_b = np.abs(back - x).max() / np.abs(x).max()
    print(f"  round trip max {err_b:.2e}", flush=True)
    assert err_b < 2e-6
    # inverse of an exact spectrum against the FP64 inverse
    inv = solver.fft_inverse(torch.from_numpy(ref.astype(np.complex64)).cuda()).cpu().numpy()
    assert np.abs(inv - x).max() / np.abs(x).max() < 2e-6
    solver.close()
