"""GPU predictor-network kernels against the FP64 reference at identical
BF16-rounded weights: forward values, loss and gradients (<= 1e-3 relative),
and a short Adam training run that must reduce the loss."""
import numpy as np
import pytest

from oracle.mlp import MlpRef
from paper_1607_03884_amd.mlp import Mlp, init_params
from tests.parity import banner

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims", [[15, 128, 128, 44], [55, 128, 128, 164], [152, 256, 256, 455]])
def test_forward_and_gradients_match_reference(dims):
    import torch
    banner(f"mlp forward/grad {dims}")
    rng = np.random.default_rng(7)
    p = init_params(dims, 11) + rng.normal(0, 0.01, size=sum(
        o * i + o for i, o in zip(dims[:-1], dims[1:]))).astype(np.float32)
    B = 700
    x = rng.standard_normal((B, dims[0])).astype(np.float32)
    t = rng.standard_normal((B, dims[-1])).astype(np.float32)
    mask = (rng.uniform(size=B) > 0.1).astype(np.float32)
    w = rng.uniform(0.5, 2.0, dims[-1]).astype(np.float32)
    net = Mlp(dims)
    net.set_params(p)
    dev = torch.device("cuda:0")
    tx, tt, tm, tw = (torch.from_numpy(a).to(dev) for a in (x, t, mask, w))
    y = net.forward(tx).cpu().numpy()
    ref = MlpRef(dims, p)
    yr = ref.forward(x)
    scale = np.abs(yr).max()
    assert np.abs(y - yr).max() <= 1e-4 * scale
    loss, g = net.grads(tx, tt, tm, tw)
    lr, gr = ref.loss_and_grad(x, t, mask, w)
    assert abs(loss.item() - lr) <= 1e-4 * lr
    g = g.cpu().numpy()
    err = np.abs(g - gr) / (np.abs(gr) + 1e-3 * np.abs(gr).max())
    print(f"max grad rel err {err.max():.2e}")
    assert err.max() <= 1e-3


def test_training_reduces_loss():
    import torch
    banner("mlp training")
    dims = [15, 64, 64, 8]
    rng = np.random.default_rng(9)
    B = 4096
    x = rng.standard_normal((B, 15)).astype(np.float32)
    A = rng.standard_normal((15, 8)).astype(np.float32)
    t = np.tanh(x @ A).astype(np.float32)
    dev = torch.device("cuda:0")
    tx, tt = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    tm = torch.ones(B, dtype=torch.float32, device=dev)
    tw = torch.ones(8, dtype=torch.float32, device=dev)
    net = Mlp(dims)
    net.set_params(init_params(dims, 5))
    loss0, _ = net.grads(tx, tt, tm, tw)
    out = torch.empty(1, dtype=torch.float32, device=dev)
    for _ in range(300):
        net.train_step(tx, tt, tm, tw, 1.0 / B, 3e-3, out)
    loss1, _ = net.grads(tx, tt, tm, tw)
    print(f"loss {loss0.item():.4f} -> {loss1.item():.4f}")
    assert loss1.item() < 0.1 * loss0.item()
