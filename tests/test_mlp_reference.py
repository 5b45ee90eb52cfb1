"""Pins of the FP64 reference network: backpropagated gradients against
central finite differences (rounding off, so the map is smooth), the GELU
derivative against a difference quotient, and BF16 rounding against exact
cases (representable values, ties to even)."""
import numpy as np

from oracle.mlp import MlpRef, bf16_round, gelu, gelu_grad
from paper_1607_03884_amd.mlp import init_params


def test_bf16_rounding():
    x = np.array([1.0, 1.5, -2.25, 3.0e-3], dtype=np.float32)
    assert np.array_equal(bf16_round(np.array([1.0, 1.5, -2.25], np.float32)), [1.0, 1.5, -2.25])
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert bf16_round(np.array([1.0 + 2.0 ** -8], np.float32))[0] == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even -> 1 + 2^-6
    assert bf16_round(np.array([1.0 + 3 * 2.0 ** -8], np.float32))[0] == 1.0 + 2.0 ** -6
    assert np.all(np.abs(bf16_round(x) - x) <= np.abs(x) * 2.0 ** -8)


def test_gelu_derivative():
    z = np.linspace(-6, 6, 101)
    d = 1e-6
    assert np.abs((gelu(z + d) - gelu(z - d)) / (2 * d) - gelu_grad(z)).max() < 1e-8


def test_reference_gradient_matches_finite_differences():
    dims = [7, 9, 6, 4]
    p = init_params(dims, 3).astype(np.float64) + 0.01
    rng = np.random.default_rng(4)
    x = rng.standard_normal((11, 7))
    t = rng.standard_normal((11, 4))
    mask = (rng.uniform(size=11) > 0.2).astype(float)
    w = rng.uniform(0.5, 2.0, 4)
    ref = MlpRef(dims, p.astype(np.float32), round_bf16=False)
    ref.master = p
    from oracle.mlp import unpack
    ref.layers = unpack(dims, p)
    loss, g = ref.loss_and_grad(x, t, mask, w)
    for i in rng.choice(p.size, 40, replace=False):
        e = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += e
        pm[i] -= e
        rp = MlpRef(dims, pp.astype(np.float32), round_bf16=False)
        rp.layers = unpack(dims, pp)
        rm = MlpRef(dims, pm.astype(np.float32), round_bf16=False)
        rm.layers = unpack(dims, pm)
        fd = (rp.loss_and_grad(x, t, mask, w)[0] - rm.loss_and_grad(x, t, mask, w)[0]) / (2 * e)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i]))
