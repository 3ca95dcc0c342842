"""The network forward that allocates nothing (sf_lrnet_forward_noalloc) against
sf_lrnet_forward, called through the C ABI: two calls in a row, the second on a
smaller input (its scratch keeps the first call's contents, which the second
must overwrite), each bit-equal to the workspace entry point's logits."""
import ctypes as ct
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1801_04720_amd import _lib, lrnet  # noqa: E402

from gpu_util import DEV, dev, host  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(prm, feat):
    B, H, W, _ = feat.shape
    out = torch.full((B, H, W), float("nan"), dtype=torch.float32, device=DEV)
    P = lambda t: ct.c_void_p(t.data_ptr())  # noqa: E731
    _lib.check(_lib.lib().sf_lrnet_forward_noalloc(P(prm), P(feat), B, H, W, P(out),
                                                   ct.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return out


def test_forward_noalloc_equals_workspace_forward():
    rng = np.random.default_rng(77)
    cases = [(2, 70, 130, 1), (1, 19, 45, 2)]  # the second smaller, with other weights
    for B, H, W, seed in cases:
        say("noalloc forward", B, H, W)
        prm = dev(lrnet.init_params(seed))
        feat = dev(rng.uniform(0, 1.5, (B, H, W, 4)).astype(np.float32))
        got = host(_noalloc(prm, feat)).copy()
        ref = host(lrnet.forward(prm, feat))
        torch.cuda.synchronize()
        assert np.array_equal(got, ref)


def test_forward_noalloc_rejects_bad_arguments():
    prm = dev(lrnet.init_params(0))
    feat = dev(np.zeros((1, 4, 4, 4), np.float32))
    out = torch.empty((1, 4, 4), dtype=torch.float32, device=DEV)
    P = lambda t: ct.c_void_p(t.data_ptr())  # noqa: E731
    L = _lib.lib()
    assert L.sf_lrnet_forward_noalloc(P(prm), P(feat), 0, 4, 4, P(out), None) == 1
    assert L.sf_lrnet_forward_noalloc(None, P(feat), 1, 4, 4, P(out), None) == 1
    assert L.sf_lrnet_forward_noalloc(P(prm), P(feat), 70000, 4, 4, P(out), None) == 1
