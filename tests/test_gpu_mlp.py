"""Learned-proposal kernels against the FP64 reference (oracle/vmf_mlp.py)."""
import sys

import numpy as np
import pytest
from helpers import progress

pytestmark = pytest.mark.gpu


_say = progress


def _records(n, seed):
    rng = np.random.default_rng(seed)
    X = np.concatenate([rng.normal(scale=0.4, size=(n, 3)), rng.uniform(-1, 0.2, size=(n, 1))], axis=1)
    S = rng.normal(size=(n, 3))
    S /= np.linalg.norm(S, axis=1, keepdims=True)
    R = np.zeros((n, 8), dtype=np.float32)
    R[:, :4] = X
    R[:, 4:7] = S
    return R


def _bf16(a):
    """Round float32 values to bfloat16 (nearest, ties to even), back as float."""
    a = np.asarray(a, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _emulated_outputs(theta, X):
    """The inference path's arithmetic: BF16 weights and inputs, products
    summed in FP32 or better, FP32 bias, ReLU, activations rounded to BF16
    before the next layer."""
    from oracle import vmf_mlp as V
    p = V.unpack(theta)
    x = _bf16(X)
    a1 = np.maximum(x @ _bf16(p["W1"]).T + p["b1"].astype(np.float32), 0)
    a2 = np.maximum(_bf16(a1) @ _bf16(p["W2"]).T + p["b2"].astype(np.float32), 0)
    return _bf16(a2) @ _bf16(p["W3"]).T + p["b3"].astype(np.float32)


def test_loss_and_gradient_match_fp64_reference():
    """Mean NLL and its gradient from the FP32 device kernels equal the FP64
    analytic reference on 300 records (ragged last block)."""
    import torch
    from oracle import vmf_mlp as V
    from paper_1411_4212_amd import learned
    theta = V.init_params(3) * 0.8
    R = _records(300, 1)
    L_ref, g_ref = V.loss_grad(theta, R[:, :4].astype(np.float64), R[:, 4:7].astype(np.float64))
    dev = torch.device("cuda", 0)
    L, g = learned.loss_grad(torch.tensor(R, device=dev), torch.tensor(theta.astype(np.float32), device=dev))
    g = g.cpu().numpy().astype(np.float64)
    _say("loss", L, L_ref, "grad err", np.max(np.abs(g - g_ref)), np.max(np.abs(g_ref)))
    assert abs(L - L_ref) <= 1e-5 * abs(L_ref) + 1e-6
    assert np.max(np.abs(g - g_ref)) <= 2e-4 * np.max(np.abs(g_ref))


def test_inference_matches_bf16_emulation():
    """ln q from the packed BF16 MFMA network equals the FP64 density of the
    emulated BF16 outputs, and the draw equals the reference sampler fed the
    same outputs and uniforms (this pins the lane layout, the K-slot
    permutation and the packing)."""
    import torch
    from oracle import vmf_mlp as V
    from paper_1411_4212_amd import learned
    rng = np.random.default_rng(4)
    theta = V.init_params(9) * 1.5
    n = 1000
    R = _records(n, 2)
    X, S = R[:, :4].astype(np.float64), R[:, 4:7].astype(np.float64)
    U = rng.random((n, 3))
    U[:, 1] = np.maximum(U[:, 1], 1e-6)
    Ud = rng.normal(size=(n, 3))
    Ud /= np.linalg.norm(Ud, axis=1, keepdims=True)
    dev = torch.device("cuda", 0)
    t = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device=dev)
    lnq, samp, lnq_samp = learned.evaluate(t(theta), t(X), t(S), t(U), t(Ud))
    lnq, samp, lnq_samp = lnq.cpu().numpy(), samp.cpu().numpy(), lnq_samp.cpu().numpy()
    out = _emulated_outputs(theta, X)
    ref = V.log_q(out, S)
    _say("lnq max err", np.max(np.abs(lnq - ref)))
    assert np.max(np.abs(lnq - ref)) < 5e-3
    ref_s = V.sample(out, U[:, 0], U[:, 1], U[:, 2], Ud)
    close = np.max(np.abs(samp - ref_s), axis=1) < 2e-3
    _say("sample agreement", close.mean())
    assert close.mean() > 0.995
    assert np.allclose(np.linalg.norm(samp, axis=1), 1.0, atol=1e-4)
    assert np.max(np.abs(lnq_samp - V.log_q(out, samp.astype(np.float64)))) < 5e-3


def test_training_fits_a_teacher():
    """Records drawn from a teacher network's q: training from scratch with
    the device Adam kernels lowers the NLL to near the teacher's own."""
    import torch
    from oracle import vmf_mlp as V
    from paper_1411_4212_amd import learned
    rng = np.random.default_rng(8)
    teacher = V.init_params(21)
    n = 60000
    X = np.concatenate([rng.normal(scale=0.5, size=(n, 3)), rng.uniform(-1, 0, size=(n, 1))], axis=1)
    out, _ = V.forward(teacher, X)
    Ud = rng.normal(size=(n, 3))
    Ud /= np.linalg.norm(Ud, axis=1, keepdims=True)
    S = V.sample(out, rng.random(n), np.maximum(rng.random(n), 1e-9), rng.random(n), Ud)
    R = np.zeros((n, 8), dtype=np.float32)
    R[:, :4], R[:, 4:7] = X, S
    nll_teacher = -np.mean(V.log_q(out, S))
    dev = torch.device("cuda", 0)
    params = learned.init_params(5, dev)
    Rt = torch.tensor(R, device=dev)
    L0, _ = learned.loss_grad(Rt, params)
    losses = learned.train(Rt, params, epochs=30, batch=1024, lr=3e-3, seed=1)
    L1, _ = learned.loss_grad(Rt, params)
    _say("NLL start %.4f end %.4f teacher %.4f" % (L0, L1, nll_teacher), losses[::5])
    assert L1 < L0 - 0.1
    assert L1 < nll_teacher + 0.15
