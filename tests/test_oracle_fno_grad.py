"""Pins of the oracle's hand-written FNO backward pass (the gradients the
learned stepper is trained with): every parameter's gradient of
L = sum_x w(x) f~(x) against central finite differences of the FP64 forward
pass, on a grid small enough to perturb each sampled entry (real and
imaginary parts of R separately), and the adjoint identity of the truncated
spectral convolution."""

import numpy as np

from oracle import fno

SHAPE = (8, 6, 8)
WIDTH, MODES, HIDDEN, LAYERS = 4, 2, 5, 2


def setup(seed=0):
    rng = np.random.default_rng(seed)
    params = fno.init_params(width=WIDTH, modes=MODES, hidden=HIDDEN, n_layers=LAYERS, seed=seed,
                             scale_spec=0.3)
    eta = rng.random(SHAPE)
    cond = rng.normal(size=fno.N_COND)
    w = rng.normal(size=SHAPE)
    return rng, params, eta, cond, w


def loss(params, eta, cond, w):
    return float((w * fno.forward(params, eta, cond)).sum())


def test_gradients_match_central_differences():
    rng, params, eta, cond, w = setup()
    g = fno.backward(params, eta, cond, w)
    h = 1e-6
    for key, val in params.items():
        flat = val.reshape(-1)
        picks = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        parts = (1.0, 1j) if np.iscomplexobj(val) else (1.0,)
        for idx in picks:
            for unit in parts:
                plus = {k: v.copy() for k, v in params.items()}
                minus = {k: v.copy() for k, v in params.items()}
                plus[key].reshape(-1)[idx] += h * unit
                minus[key].reshape(-1)[idx] -= h * unit
                fd = (loss(plus, eta, cond, w) - loss(minus, eta, cond, w)) / (2 * h)
                an = g[key].reshape(-1)[idx]
                an = an.real if unit == 1.0 else an.imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (key, idx, unit, fd, an)


def test_spectral_convolution_adjoint_identity():
    rng, params, _, _, _ = setup(3)
    R = params["R"][0]
    v = rng.normal(size=(WIDTH,) + SHAPE)
    dy = rng.normal(size=(WIDTH,) + SHAPE)
    dv, dR = fno.spectral_conv_adjoint(dy, R, v)
    # <dy, K v> = <dv, v>: the input gradient of a linear map is its adjoint
    lhs = (dy * fno.spectral_conv(v, R)).sum()
    assert abs(lhs - (dv * v).sum()) <= 1e-10 * max(1.0, abs(lhs))
    # the map is linear in R: <dR, R> (real-pair inner product) = <dy, K v>
    assert abs((dR.real * R.real + dR.imag * R.imag).sum() - lhs) <= 1e-10 * max(1.0, abs(lhs))
