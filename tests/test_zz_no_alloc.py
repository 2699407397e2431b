"""The allocation-free training entry point (workspace in the library's
static device array) through the C ABI: two calls in a row, the second on a
smaller input, each bit-identical to rewl_mlp_train with a caller-owned
workspace on the same records and starting parameters."""
import sys

import numpy as np
import pytest
from helpers import progress

pytestmark = pytest.mark.gpu


_say = progress


def _records(n, seed):
    rng = np.random.default_rng(seed)
    h = rng.normal(size=(n, 3))
    h *= (rng.random((n, 1)) / np.linalg.norm(h, axis=1, keepdims=True))
    s = h + 0.3 * rng.normal(size=(n, 3))
    s /= np.linalg.norm(s, axis=1, keepdims=True)
    rec = np.zeros((n, 8), dtype=np.float32)
    rec[:, :3] = h
    rec[:, 3] = rng.uniform(-1, 0, size=n)
    rec[:, 4:7] = s
    return rec


def test_train_static_equals_train_with_workspace():
    import torch
    from paper_1411_4212_amd import learned, rewl
    dev = torch.device("cuda:0")
    for call, (n, batch, epochs, seed) in enumerate([(20000, 4096, 3, 11), (3000, 512, 2, 12)]):
        _say("no-alloc training call", call, "n", n, "batch", batch)
        rec = torch.from_numpy(_records(n, seed)).to(dev)
        p0 = learned.init_params(seed, dev)
        pa, pb = p0.clone(), p0.clone()
        ws = torch.empty(rewl.rewl_mlp_workspace_bytes(batch), dtype=torch.uint8, device=dev)
        la = rewl.rewl_mlp_train(rec.data_ptr(), n, epochs, batch, 2e-3, 99, pa.data_ptr(), ws.data_ptr())
        lb = rewl.rewl_mlp_train_static(rec.data_ptr(), n, epochs, batch, 2e-3, 99, pb.data_ptr())
        torch.cuda.synchronize()
        _say("losses", la.tolist(), lb.tolist())
        assert np.array_equal(la.view(np.uint32), lb.view(np.uint32))
        a, b = pa.cpu().numpy(), pb.cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        assert not np.array_equal(a, p0.cpu().numpy())


def test_train_static_rejects_large_batch():
    import torch
    from paper_1411_4212_amd import learned, rewl
    dev = torch.device("cuda:0")
    rec = torch.from_numpy(_records(100, 1)).to(dev)
    p = learned.init_params(1, dev)
    with pytest.raises(rewl.RewlError) as e:
        rewl.rewl_mlp_train_static(rec.data_ptr(), 100, 1, 8193, 1e-3, 1, p.data_ptr())
    assert e.value.code == -4
