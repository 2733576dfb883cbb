"""The PyTorch model of the learned stepper (tests/fno_torch_model.py)
computes the oracle's network (CPU, float64), and PyTorch autograd through it
reproduces the oracle's hand-written backward: a third, independent
derivation that the library's training kernels are checked against."""

import numpy as np

from oracle import fno as ofno
from tests import fno_torch_model as surrogate


def test_torch_model_matches_oracle_forward():
    import torch
    p = ofno.init_params(width=32, modes=4, hidden=128, n_layers=4, seed=7, scale_spec=0.01)
    model = surrogate.make_model(torch, modes=4).double()
    surrogate.load_params(model, p, torch)
    rng = np.random.default_rng(8)
    eta = rng.random((16, 12, 10))
    cond = rng.normal(size=7)
    with torch.no_grad():
        got = model(torch.as_tensor(eta)[None], torch.as_tensor(cond)[None])[0].numpy()
    np.testing.assert_allclose(got, ofno.forward(p, eta, cond), rtol=1e-10, atol=1e-12)
    back = surrogate.to_params(model)
    for k in ("P", "W", "Q1"):
        np.testing.assert_array_equal(back[k], p[k])
    np.testing.assert_array_equal(back["R"], p["R"])


def _grad_case(torch, device, dtype, seed=3, native=False):
    p = ofno.init_params(width=8, modes=3, hidden=10, n_layers=2, seed=seed, scale_spec=0.2)
    model = surrogate.make_model(torch, width=8, modes=3, hidden=10, n_layers=2, native=native)
    model = model.to(device=device, dtype=dtype)
    surrogate.load_params(model, p, torch)
    rng = np.random.default_rng(seed + 1)
    eta = rng.random((16, 12, 10))
    cond = rng.normal(size=7)
    w = rng.normal(size=eta.shape)
    as_t = lambda a: torch.as_tensor(a, dtype=dtype, device=device)  # noqa: E731
    loss = (model(as_t(eta)[None], as_t(cond)[None])[0] * as_t(w)).sum()
    loss.backward()
    ref = ofno.backward(p, eta, cond, w)
    out = {}
    for k in ("P", "p", "W", "b", "Q1", "q1", "Q2", "q2"):
        g = getattr(model, k).grad.detach().double().cpu().numpy().reshape(ref[k].shape)
        out[k] = np.linalg.norm(g - ref[k]) / np.linalg.norm(ref[k])
    gR = model.R.grad.detach().double().cpu().numpy()
    out["R"] = np.linalg.norm((gR[..., 0] + 1j * gR[..., 1]) - ref["R"]) / np.linalg.norm(ref["R"])
    return out


def test_training_gradients_match_the_oracle_backward():
    # PyTorch autograd (float64, CPU) against the hand-written FP64 backward
    import torch
    errs = _grad_case(torch, "cpu", torch.float64)
    for k, e in errs.items():
        assert e <= 1e-10, (k, e)
