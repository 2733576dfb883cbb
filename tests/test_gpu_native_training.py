"""GPU: training of the learned stepper in the library's kernels alone
(surrogate.NativeTrainer: lift, Fourier layers, projection, mean-square loss,
weight gradients as outer sums, Adam). Against the checker: the prediction
against its FP64 forward and every parameter gradient of the loss against
its hand-written backward pass driven by the same loss gradient, two samples
of a 16 x 12 x 10 grid with different conditioning (relative L2 <= 1e-4);
one Adam step against the textbook update written out; and a short run on a
fixed mini-batch lowers the loss."""

import numpy as np
import pytest

from oracle import fno as ofno
from paper_2302_13612_amd import binding, surrogate

pytestmark = pytest.mark.gpu

SHAPE = (16, 12, 10)


def setup(seed=5):
    import torch
    p = ofno.init_params(width=8, modes=3, hidden=10, n_layers=2, seed=seed, scale_spec=0.2)
    rng = np.random.default_rng(seed)
    eta = rng.random((2,) + SHAPE)
    cond = rng.normal(size=(2, ofno.N_COND))
    target = eta + 0.3 * rng.normal(size=eta.shape)
    t = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")  # noqa: E731
    return p, eta, cond, target, t(eta), t(cond), t(target)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def test_gradients_match_the_oracle_backward():
    import torch
    p, eta, cond, target, et, ct, tt = setup()
    tr = surrogate.NativeTrainer(torch, binding, p, "cuda")
    out, loss = tr.gradients(et, ct, tt)
    scale = 2.0 / eta.size
    ref = None
    outs = []
    for b in range(2):
        o = ofno.forward(p, eta[b], cond[b])
        outs.append(o)
        gb = ofno.backward(p, eta[b], cond[b], scale * (o - target[b]))
        ref = gb if ref is None else {k: ref[k] + gb[k] for k in ref}
    e_out = rel(out.cpu().numpy(), np.stack(outs))
    errs = {}
    for k in surrogate.NativeTrainer.KEYS:
        g = tr.g[k].double().cpu().numpy()
        if k == "R":
            g = g[..., 0] + 1j * g[..., 1]
        errs[k] = rel(g.reshape(ref[k].shape), ref[k])
    print(f"\n[native training] prediction {e_out:.1e}; gradients " +
          ", ".join(f"{k} {e:.1e}" for k, e in errs.items()), flush=True)
    assert e_out <= 1e-5
    assert abs(loss - float(np.mean((np.stack(outs) - target) ** 2))) <= 1e-5 * loss
    for k, e in errs.items():
        assert e <= 1e-4, (k, e)


def test_adam_step_matches_the_update_written_out():
    import ctypes
    import torch
    rng = np.random.default_rng(2)
    w, g, m, v = (rng.normal(size=1000) for _ in range(4))
    v = np.abs(v)
    t = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")  # noqa: E731
    wt, gt, mt, vt = t(w), t(g), t(m), t(v)
    lib = binding.load()
    lr, b1, b2, eps, step = 1e-2, 0.9, 0.999, 1e-8, 3
    assert lib.pf_nt_adam(1000, wt.data_ptr(), gt.data_ptr(), mt.data_ptr(), vt.data_ptr(), lr, b1, b2, eps, step,
                          None) == 0
    torch.cuda.synchronize()
    m1 = b1 * m + (1 - b1) * g
    v1 = b2 * v + (1 - b2) * g * g
    w1 = w - lr * (m1 / (1 - b1 ** step)) / (np.sqrt(v1 / (1 - b2 ** step)) + eps)
    np.testing.assert_allclose(mt.cpu().numpy(), m1, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(vt.cpu().numpy(), v1, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(wt.cpu().numpy(), w1, rtol=1e-5, atol=1e-6)
    assert ctypes  # the call above went through the C ABI


def test_short_run_lowers_the_loss():
    # a learnable target (the order parameter shifted by 0.2): PyTorch's Adam on
    # the same network takes the loss from 1.5e-2 to 2.7e-5 in 40 steps (float64, CPU)
    import torch
    p, eta, cond, _, et, ct, _ = setup(6)
    tt = et + 0.2
    tr = surrogate.NativeTrainer(torch, binding, p, "cuda")
    _, l0 = tr.gradients(et, ct, tt)
    for _ in range(40):
        tr.adam(5e-3)
        _, l1 = tr.gradients(et, ct, tt)
    print(f"\n[native training] loss {l0:.3e} -> {l1:.3e} in 40 Adam steps", flush=True)
    assert l1 < 1e-2 * l0
