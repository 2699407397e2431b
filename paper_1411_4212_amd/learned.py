"""Learned proposal: train the MLP on harvested records (device kernels of
librewl) and hand it to a run.  Argument marshalling only."""
import numpy as np

from . import rewl


def init_params(seed=0, device="cuda"):
    """He-uniform weights, zero biases, FP32 on the device, in the parameter
    order of include/rewl.h."""
    import torch
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in [(64, 4), (64, None), (64, 64), (64, None), (12, 64), (12, None)]:
        if cols is None:
            parts.append(np.zeros(rows))
        else:
            lim = np.sqrt(6.0 / cols)
            parts.append(rng.uniform(-lim, lim, size=rows * cols))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == rewl.rewl_mlp_param_count()
    return torch.tensor(theta, device=device)


def train(records, params, epochs=4, batch=4096, lr=1e-3, seed=0):
    """Adam on device records (n, 8) float32; updates params in place;
    returns the per-epoch mean minibatch loss."""
    import torch
    n = records.shape[0]
    ws = torch.empty(rewl.rewl_mlp_workspace_bytes(batch), dtype=torch.uint8, device=records.device)
    stream = torch.cuda.current_stream(records.device).cuda_stream
    return rewl.rewl_mlp_train(records.data_ptr(), n, epochs, batch, lr, seed, params.data_ptr(),
                               ws.data_ptr(), stream)


def loss_grad(records, params):
    import torch
    n = records.shape[0]
    ws = torch.empty(rewl.rewl_mlp_workspace_bytes(n), dtype=torch.uint8, device=records.device)
    g = torch.empty_like(params)
    stream = torch.cuda.current_stream(records.device).cuda_stream
    L = rewl.rewl_mlp_loss_grad(records.data_ptr(), n, params.data_ptr(), g.data_ptr(), ws.data_ptr(),
                                stream)
    return L, g


def evaluate(params, x, s, u, udir):
    """ln q(s|x), a draw from q(.|x) and its ln q, via the packed BF16 MFMA
    network (all device tensors, float32)."""
    import torch
    dev = params.device
    packed = torch.empty(rewl.rewl_mlp_packed_bytes(), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    rewl.rewl_mlp_pack(params.data_ptr(), packed.data_ptr(), stream)
    n = x.shape[0]
    lnq_s = torch.empty(n, dtype=torch.float32, device=dev)
    samp = torch.empty(n, 3, dtype=torch.float32, device=dev)
    lnq_samp = torch.empty(n, dtype=torch.float32, device=dev)
    rewl.rewl_mlp_eval(packed.data_ptr(), x.data_ptr(), s.data_ptr(), u.data_ptr(), udir.data_ptr(),
                       lnq_s.data_ptr(), samp.data_ptr(), lnq_samp.data_ptr(), n, stream)
    return lnq_s, samp, lnq_samp
