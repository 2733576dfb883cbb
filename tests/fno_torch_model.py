"""PyTorch model of the learned stepper (tests only): the same network as the
oracle's forward and the library's pf_fno_forward, built from PyTorch modules,
so that PyTorch autograd gives a third, independent set of gradients to check
the oracle's hand-written backward and the library's training kernels
against. native=True takes the spectral convolution of every layer from the
library (binding.spectral_conv) instead of torch.fft."""

import numpy as np


def make_model(torch, width=32, modes=12, hidden=128, n_layers=4, n_cond=7, seed=0, native=False):
    """The network as PyTorch modules. native: the spectral convolution of
    every layer (forward and backward) runs in the library's kernels
    (binding.spectral_conv); otherwise in torch.fft."""
    nn = torch.nn
    F = torch.nn.functional

    def kept(n, m, device):
        return torch.cat([torch.arange(m, device=device), torch.arange(n - m, n, device=device)])

    class TorchFno(nn.Module):
        def __init__(self):
            super().__init__()
            g = torch.Generator().manual_seed(seed)
            cin = 1 + n_cond
            self.m = modes
            self.P = nn.Parameter(torch.randn(width, cin, generator=g) / cin ** 0.5)
            self.p = nn.Parameter(torch.zeros(width))
            self.W = nn.Parameter(torch.randn(n_layers, width, width, generator=g) / width ** 0.5)
            self.b = nn.Parameter(torch.zeros(n_layers, width))
            scale = 1.0 / (width * width)
            self.R = nn.Parameter(scale * torch.rand(n_layers, width, width, 2 * modes, 2 * modes, modes, 2,
                                                     generator=g))
            self.Q1 = nn.Parameter(torch.randn(hidden, width, generator=g) / width ** 0.5)
            self.q1 = nn.Parameter(torch.zeros(hidden))
            self.Q2 = nn.Parameter(torch.randn(1, hidden, generator=g) * 1e-3 / hidden ** 0.5)
            self.q2 = nn.Parameter(torch.zeros(1))

        def forward(self, eta, cond):
            """eta (B, nz, ny, nx), cond (B, n_cond) -> predicted eta."""
            B, nz, ny, nx = eta.shape
            m = self.m
            const = cond @ self.P[:, 1:].T + self.p                      # (B, C)
            v = self.P[:, 0].view(1, -1, 1, 1, 1) * eta[:, None] + const[:, :, None, None, None]
            iz, iy = kept(nz, m, eta.device), kept(ny, m, eta.device)
            for l in range(self.W.shape[0]):
                if native:
                    from paper_2302_13612_amd import binding
                    kv = binding.spectral_conv(v, self.R[l], m)
                else:
                    Vh = torch.fft.rfftn(v, dim=(2, 3, 4))
                    sub = Vh[:, :, iz][:, :, :, iy][..., :m]
                    Rc = torch.view_as_complex(self.R[l])
                    out_sub = torch.einsum("bizyx,oizyx->bozyx", sub, Rc)
                    spec = torch.zeros((B, Rc.shape[0], nz, ny, nx // 2 + 1), dtype=Vh.dtype, device=eta.device)
                    spec[:, :, iz[:, None], iy[None, :], :m] = out_sub
                    kv = torch.fft.irfftn(spec, s=(nz, ny, nx), dim=(2, 3, 4))
                local = torch.einsum("oi,bizyx->bozyx", self.W[l], v) + self.b[l].view(1, -1, 1, 1, 1)
                v = F.gelu(local + kv)
            h = F.gelu(torch.einsum("hi,bizyx->bhzyx", self.Q1, v) + self.q1.view(1, -1, 1, 1, 1))
            d = torch.einsum("oh,bhzyx->bozyx", self.Q2, h)[:, 0] + self.q2
            return eta + d

    return TorchFno()


def to_params(model):
    """Weights in the checker's / library binding's layout (float64, R complex)."""
    g = lambda t: t.detach().double().cpu().numpy()  # noqa: E731
    R = g(model.R)
    return {"P": g(model.P), "p": g(model.p), "W": g(model.W), "b": g(model.b),
            "R": R[..., 0] + 1j * R[..., 1], "Q1": g(model.Q1), "q1": g(model.q1), "Q2": g(model.Q2),
            "q2": g(model.q2)}


def load_params(model, params, torch):
    with torch.no_grad():
        for k in ("P", "p", "W", "b", "Q1", "q1", "Q2", "q2"):
            getattr(model, k).copy_(torch.as_tensor(np.asarray(params[k]).reshape(getattr(model, k).shape)))
        R = np.asarray(params["R"])
        model.R.copy_(torch.as_tensor(np.stack([R.real, R.imag], axis=-1)))
