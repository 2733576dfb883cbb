"""GPU: the gradients the learned stepper is trained with (the training
model in FP32 on the device) against the oracle's hand-written FP64 backward
pass: relative L2 error per parameter tensor <= 1e-4 (FP32 transforms and
sums over 1,920 voxels)."""

import pytest

from tests.test_surrogate_model import _grad_case

pytestmark = pytest.mark.gpu


def test_device_training_gradients_match_the_oracle_backward():
    import torch
    errs = _grad_case(torch, "cuda", torch.float32)
    print("\n[fno grad] rel L2 per tensor: " + ", ".join(f"{k} {e:.1e}" for k, e in errs.items()), flush=True)
    for k, e in errs.items():
        assert e <= 1e-4, (k, e)
