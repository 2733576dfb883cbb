"""GPU: the allocation-free outer sum (pf_nt_outer_sum_noalloc) against the
workspace entry point (pf_nt_outer_sum) through the C ABI: bit for bit on
three calls in a row (the second smaller than the first, accumulating into
its output; the third without Y), and PF_ENOMEM, with nothing launched, for
partials beyond the library's fixed 16 MiB array."""

import ctypes

import numpy as np
import pytest

from paper_2302_13612_amd import binding

pytestmark = pytest.mark.gpu


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _with_workspace(lib, torch, B, MA, MC, nvox, X, Y, out, acc):
    n = ctypes.c_size_t()
    assert lib.pf_nt_outer_workspace(B, MA, MC, nvox, ctypes.byref(n)) == binding.PF_OK
    work = torch.empty(n.value // 4, dtype=torch.float32, device="cuda")
    rc = lib.pf_nt_outer_sum(B, MA, MC, nvox, X.data_ptr(), Y.data_ptr() if Y is not None else None,
                             out.data_ptr(), acc, work.data_ptr(), n.value, _stream(torch))
    assert rc == binding.PF_OK


def _no_alloc(lib, torch, B, MA, MC, nvox, X, Y, out, acc):
    return lib.pf_nt_outer_sum_noalloc(B, MA, MC, nvox, X.data_ptr(), Y.data_ptr() if Y is not None else None,
                                       out.data_ptr(), acc, _stream(torch))


def test_outer_sum_no_alloc_matches_workspace_entry():
    import torch
    lib = binding.load()
    g = torch.Generator(device="cpu").manual_seed(21)
    calls = [  # (B, MA, MC, nvox, with Y, accumulate)
        (6, 128, 32, 40000, True, 0),   # ragged voxel chunk, 1 MiB of partials
        (2, 20, 7, 5000, True, 1),      # smaller, ragged channel tiles, accumulating
        (3, 32, 1, 9000, False, 0),     # Y NULL: sums of X
    ]
    for i, (B, MA, MC, nvox, with_y, acc) in enumerate(calls):
        print(f"\n[no-alloc] call {i}: B={B} MA={MA} MC={MC} nvox={nvox} Y={with_y} accumulate={acc}", flush=True)
        X = torch.randn((B, MA, nvox), generator=g).cuda()
        Y = torch.randn((B, MC, nvox), generator=g).cuda() if with_y else None
        start = torch.randn((MA, MC), generator=g).cuda()
        ref = start.clone()
        got = start.clone()
        _with_workspace(lib, torch, B, MA, MC, nvox, X, Y, ref, acc)
        assert _no_alloc(lib, torch, B, MA, MC, nvox, X, Y, got, acc) == binding.PF_OK
        torch.cuda.synchronize()
        r, o = ref.cpu().numpy(), got.cpu().numpy()
        assert np.isfinite(o).all()
        assert np.array_equal(r, o), np.abs(r - o).max()
        # the sums themselves, against float64 on the host
        Xh = X.double().cpu().numpy()
        Yh = Y.double().cpu().numpy() if with_y else np.ones((B, MC, nvox))
        exp = np.einsum("bai,bci->ac", Xh, Yh) + (start.double().cpu().numpy() if acc else 0.0)
        np.testing.assert_allclose(o, exp, rtol=1e-4, atol=1e-3 * np.sqrt(B * nvox))


def test_outer_sum_no_alloc_rejects_partials_beyond_its_array():
    import torch
    lib = binding.load()
    X = torch.zeros(16, device="cuda")
    out = torch.zeros(16, device="cuda")
    # 8192 channel pairs x 64 samples x 10 chunks > 4 Mi floats: refused on
    # the host before any launch
    rc = lib.pf_nt_outer_sum_noalloc(64, 128, 64, 40000, X.data_ptr(), X.data_ptr(), out.data_ptr(), 0,
                                     _stream(torch))
    assert rc == binding.PF_ENOMEM
