"""The training model of the learned stepper computes the checker's network
(CPU, float64): trained weights mean the same thing in the library."""

import numpy as np

from oracle import fno as ofno
from paper_2302_13612_amd import surrogate


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
