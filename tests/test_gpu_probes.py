"""The two bandwidth references of the C ABI on the device: the streaming copy
moves every byte, and the plain read flags a non-finite value and nothing
else (its loads are live)."""
import pytest
import torch

import paper_2601_03806_amd as gmf
from gpu_common import say

pytestmark = pytest.mark.gpu


def test_copy_and_read_probes():
    say("copy and read probes, 1 MiB + 16 B")
    n = (1 << 18) + 4   # floats: 1 MiB plus one 16-byte vector (a ragged last workgroup)
    g = torch.Generator().manual_seed(7)
    a = torch.randn(n, generator=g, dtype=torch.float32).cuda()
    b = torch.zeros_like(a)
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    gmf.copy_probe(a.data_ptr(), b.data_ptr(), 4 * n, s)
    gmf.read_probe(b.data_ptr(), 4 * n, flag.data_ptr(), s)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert int(flag.item()) == 0
    # a non-finite value in the last vector is seen
    b[n - 1] = float("inf")
    torch.cuda.synchronize()
    gmf.read_probe(b.data_ptr(), 4 * n, flag.data_ptr(), s)
    torch.cuda.synchronize()
    assert int(flag.item()) == 1
