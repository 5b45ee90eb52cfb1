"""FP64 reference of the predictor network (test infrastructure only).

A multilayer perceptron with GELU hidden layers (x Phi(x), erf form) and a
linear output; weights rounded to BF16 (round-to-nearest-even) before use;
loss = sum_b mask_b sum_o w_o (y - t)^2 / sum_b mask_b; gradients by the
chain rule written out layer by layer.  Used to check the GPU network's
forward values and gradients.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest BF16 (ties to even), as float64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(dims, flat):
    out, o = [], 0
    for din, dout in zip(dims[:-1], dims[1:]):
        W = flat[o:o + din * dout].reshape(dout, din)
        o += din * dout
        b = flat[o:o + dout]
        o += dout
        out.append((W, b))
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


class MlpRef:
    def __init__(self, dims, params, round_bf16: bool = True):
        self.dims = list(dims)
        p = np.asarray(params, dtype=np.float32)
        self.master = p.astype(np.float64)
        w = bf16_round(p) if round_bf16 else self.master
        # biases are not rounded (added in FP32)
        layers = unpack(self.dims, w)
        raw = unpack(self.dims, self.master)
        self.layers = [(W, braw) for (W, _), (_, braw) in zip(layers, raw)]

    def forward(self, x, keep=False):
        a = np.asarray(x, dtype=np.float64)
        acts, pres = [a], []
        for i, (W, b) in enumerate(self.layers):
            z = a @ W.T + b
            pres.append(z)
            a = gelu(z) if i + 1 < len(self.layers) else z
            acts.append(a)
        return (a, acts, pres) if keep else a

    def loss_and_grad(self, x, t, mask, w):
        y, acts, pres = self.forward(x, keep=True)
        mask = np.asarray(mask, dtype=np.float64)
        w = np.asarray(w, dtype=np.float64)
        cnt = mask.sum()
        d = y - t
        loss = float((mask[:, None] * w[None, :] * d * d).sum() / cnt)
        g = 2.0 * mask[:, None] * w[None, :] * d / cnt
        grads = []
        for i in range(len(self.layers) - 1, -1, -1):
            W, _ = self.layers[i]
            if i + 1 < len(self.layers):
                g = g * gelu_grad(pres[i])
            grads.append((g.T @ acts[i], g.sum(axis=0)))
            g = g @ W
        flat = []
        for gW, gb in reversed(grads):
            flat += [gW.ravel(), gb]
        return loss, np.concatenate(flat)
