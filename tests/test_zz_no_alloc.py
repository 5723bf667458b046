"""The allocation-free noise probe (gmf_noise_probe_noalloc, staged in a fixed
device array) against gmf_noise_probe (device buffers allocated per call):
bit-identical Philox words and normals in both precisions, on two calls in a
row with the second smaller, on a torch stream and on the legacy stream; at
the maximum size; NULL outputs; and the size limit rejected."""
import numpy as np
import pytest

import paper_2601_03806_amd as gmf
from gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [gmf.FP64, gmf.FP32_SHIFTED])
def test_noalloc_probe_equals_probe(precision):
    import torch
    stream = torch.cuda.Stream()
    # two calls in a row, the second smaller (the array keeps the first call's values beyond it)
    for seed, step, node0, count, st in ((7, 1234, 100, gmf.PROBE_MAX_NODES, stream),
                                         (0xDEADBEEFCAFEF00D, (5 << 32) + 3, 4_000_000_000, 1000, None),
                                         (3, 0, 0, 1, stream)):
        say(f"noalloc probe prec={precision} seed={seed} step={step} node0={node0} count={count}")
        w_ref, n_ref = gmf.noise_probe(seed, step, node0, count, precision)
        w, n = gmf.noise_probe_noalloc(seed, step, node0, count, precision, stream=st)
        assert np.array_equal(w, w_ref)
        assert np.array_equal(n.view(np.uint64), n_ref.view(np.uint64))


def test_noalloc_probe_null_outputs_and_limit():
    import ctypes
    lib = gmf.lib()
    say("noalloc probe NULL outputs and limit")
    words = np.zeros(24 * 64, np.uint32)
    rc = lib.gmf_noise_probe_noalloc(11, 5, 0, 64, gmf.FP64, words.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                     None, None)
    assert rc == gmf.GMF_OK
    w_ref, _ = gmf.noise_probe(11, 5, 0, 64)
    assert np.array_equal(words.reshape(64, 6, 4), w_ref)
    assert lib.gmf_noise_probe_noalloc(11, 5, 0, 64, gmf.FP64, None, None, None) == gmf.GMF_OK
    with pytest.raises(gmf.GmfError) as e:
        gmf.noise_probe_noalloc(1, 0, 0, gmf.PROBE_MAX_NODES + 1)
    assert e.value.code == gmf.GMF_EINVAL
