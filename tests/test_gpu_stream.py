"""GPU: the library's streaming copy (the bench's attainable-bandwidth
reference) moves every byte, bit for bit, for sizes below, at and above one
full grid of 65536 x 512 lanes, on torch's current stream."""

import pytest

from paper_2302_13612_amd import binding

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n16", [1, 513, 65536 * 512, 65536 * 512 + 7 * 512 + 3])
def test_stream_copy_bit_exact(n16):
    import torch
    g = torch.Generator(device="cuda").manual_seed(n16)
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (4 * n16,), dtype=torch.int32, device="cuda", generator=g)
    dst = torch.zeros_like(src)
    binding.stream_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
