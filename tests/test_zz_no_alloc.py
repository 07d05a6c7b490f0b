"""bcv_mlp_forward_noalloc (inference on caller-owned device arrays with the library's fixed
workspace, for callers that cannot allocate) against bcv_mlp_forward (host arrays, per-call
device buffers): the same kernels in the same order, so the outputs must be identical. Two calls in
a row, the second with a smaller input, so the second runs over a workspace that still holds the
first call's activations; then a call at the workspace's row limit and one beyond it."""

import sys

import numpy as np
import pytest

sys.path.insert(0, __import__("os").path.dirname(__file__))

import paper_2112_00864_amd as bcv  # noqa: E402

pytestmark = pytest.mark.gpu


def announce(*a):
    print("[gpu]", *a, flush=True)


def test_forward_noalloc_matches_forward():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    net = bcv.mlp_create(width=128, seed=3)
    rng = np.random.default_rng(21)
    net.set_params(rng.uniform(-0.3, 0.3, net.num_params()).astype(np.float32))
    for n in (5000, 777, 8192):
        announce("forward_noalloc n=%d width=128" % n)
        X = rng.uniform(-1, 1, (n, 6)).astype(np.float32)
        ref = net.forward(X)
        Xd = torch.tensor(X, device="cuda:0")
        Yd = torch.full((n, 2), float("nan"), dtype=torch.float32, device="cuda:0")
        net.forward_noalloc(Xd, Yd)
        torch.cuda.synchronize()
        Y = Yd.cpu().numpy()
        announce("n=%d max |diff| %.3e" % (n, float(np.max(np.abs(Y - ref)))))
        assert np.all(np.isfinite(Y))
        assert np.array_equal(Y, ref)
    # beyond the workspace: a clear error, nothing launched
    Xd = torch.zeros((8193, 6), dtype=torch.float32, device="cuda:0")
    Yd = torch.zeros((8193, 2), dtype=torch.float32, device="cuda:0")
    with pytest.raises(bcv.BCVError) as e:
        net.forward_noalloc(Xd, Yd)
    assert e.value.status == bcv.EINVAL and "workspace" in str(e.value)
    # empty input: nothing to do
    net.forward_noalloc(torch.zeros((0, 6), dtype=torch.float32, device="cuda:0"),
                        torch.zeros((0, 2), dtype=torch.float32, device="cuda:0"))
