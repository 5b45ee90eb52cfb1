"""Learned stage/step predictor: features, targets, training, file format.

Input features of a state (T, Y, P): [T / 1000, ln(P / 1 atm), Y_1..Y_K],
standardised.  Targets: for each Radau stage i and component c of the first
accepted step, symlog(z_ic / sc_c) with sc_c = atol + rtol |y0_c| and
symlog(v) = sign(v) ln(1 + |v|); log10(h_first / dt); log10(step attempts).
Targets are standardised; the network predicts the standardised values.
The integrator starts the first step from the predicted h and stage values
and keeps them only if Newton converges (see the library's "predictor"
option).  One weight set per global step size.
"""
from __future__ import annotations

import math
import os
import time
from typing import Dict

import numpy as np

from . import configs
from .mlp import Mlp, init_params

P_ATM = 101325.0


def features(states: np.ndarray, K: int) -> np.ndarray:
    T, Y, P = states[:, 0], states[:, 1:K + 1], states[:, K + 1]
    return np.concatenate([(T / 1000.0)[:, None], np.log(P / P_ATM)[:, None], Y], axis=1)


def targets(states, z_first, h_first, nstep, dt, atol, rtol, K):
    N = K + 1
    y0 = states[:, :N]
    sc = atol + rtol * np.abs(y0)
    v = z_first / sc[:, None, :]
    zt = (np.sign(v) * np.log1p(np.abs(v))).reshape(len(states), 3 * N)
    ht = np.log10(np.maximum(h_first, 1e-300) / dt)
    st = np.log10(np.maximum(nstep, 1))
    return np.concatenate([zt, ht[:, None], st[:, None]], axis=1)


def write(path: str, mech: str, K: int, dt: float, dims, in_shift, in_scale, out_shift, out_scale, params):
    f = lambda a: " ".join(repr(float(x)) for x in a)
    lines = ["rkpred 1", f"mech {mech} K {K} dt {dt!r}", "dims " + str(len(dims)) + " " + " ".join(map(str, dims)),
             "in_shift " + f(in_shift), "in_scale " + f(in_scale), "out_shift " + f(out_shift),
             "out_scale " + f(out_scale), f"params {len(params)}"]
    for i in range(0, len(params), 16):
        lines.append(f(params[i:i + 16]))
    lines.append("end")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def path_for(mech: str, dt: float) -> str:
    return os.path.join(configs.DATA_DIR, f"{mech}_predictor_dt{dt:g}.rkp")


def train(mech: str, dt: float, data: Dict[str, np.ndarray], hidden=(128, 128), epochs=40, batch=4096,
          lr=2e-3, seed=3001, out_path=None, log=print) -> dict:
    import torch
    K = configs.MECHS[mech].n_species
    N = K + 1
    ok = data["status"] == 0
    X = features(data["states"], K)[ok]
    Tg = targets(data["states"], data["z_first"], data["h_first"], data["nstep"], dt, float(data["atol"]),
                 float(data["rtol"]), K)[ok]
    in_shift, in_scale = X.mean(0), np.maximum(X.std(0), 1e-6)
    out_shift, out_scale = Tg.mean(0), np.maximum(Tg.std(0), 1e-6)
    Xn = ((X - in_shift) / in_scale).astype(np.float32)
    Tn = ((Tg - out_shift) / out_scale).astype(np.float32)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(Xn))
    nval = len(Xn) // 10
    val, tr = perm[:nval], perm[nval:]
    dims = [X.shape[1], *hidden, Tg.shape[1]]
    net = Mlp(dims)
    net.set_params(init_params(dims, seed))
    dev = torch.device("cuda:0")
    Xt = torch.from_numpy(Xn[tr]).to(dev)
    Ttr = torch.from_numpy(Tn[tr]).to(dev)
    w = np.concatenate([np.full(3 * N, 1.0 / (3 * N)), [1.0, 0.5]]).astype(np.float32)
    wt = torch.from_numpy(w).to(dev)
    ones = torch.ones(batch, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ntr = len(tr)
    epochs = max(epochs, math.ceil(1700 * batch / ntr))    # at least ~1,700 updates on small sets
    steps = epochs * (ntr // batch)
    t0 = time.time()
    k = 0
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(ntr)).to(dev)
        for b in range(ntr // batch):
            idx = order[b * batch:(b + 1) * batch]
            xb, tb = Xt[idx].contiguous(), Ttr[idx].contiguous()
            lr_k = 1e-4 + 0.5 * (lr - 1e-4) * (1 + math.cos(math.pi * k / steps))
            net.train_step(xb, tb, ones, wt, 1.0 / batch, lr_k, loss)
            k += 1
        if ep % 10 == 9 or ep == epochs - 1:
            torch.cuda.synchronize()
            log(f"epoch {ep + 1}: batch loss {loss.item():.4f} ({time.time() - t0:.1f} s)")
    # validation, in target units
    yv = net.forward(torch.from_numpy(Xn[val]).to(dev)).cpu().numpy() * out_scale + out_shift
    tv = Tg[val]
    rep = {"z_rmse_symlog": float(np.sqrt(np.mean((yv[:, :3 * N] - tv[:, :3 * N]) ** 2))),
           "log10_h_rmse": float(np.sqrt(np.mean((yv[:, 3 * N] - tv[:, 3 * N]) ** 2))),
           "log10_steps_rmse": float(np.sqrt(np.mean((yv[:, 3 * N + 1] - tv[:, 3 * N + 1]) ** 2))),
           "log10_h_std": float(tv[:, 3 * N].std()), "log10_steps_std": float(tv[:, 3 * N + 1].std()),
           "n_train": int(ntr), "n_val": int(nval), "dims": dims, "steps": steps}
    log(f"validation: {rep}")
    params = net.get_params()
    write(out_path or path_for(mech, dt), mech, K, dt, dims, in_shift, in_scale, out_shift, out_scale, params)
    return rep


if __name__ == "__main__":
    # python -m paper_1607_03884_amd.predictor <mech> [output directory] [dt,...] [hidden widths]
    # e.g. "M53", or "M150 paper_1607_03884_amd/data 1e-4 256,256" (the 150-species file)
    import json
    import sys
    mech = sys.argv[1] if len(sys.argv) > 1 else "M13"
    outdir = sys.argv[2] if len(sys.argv) > 2 else configs.DATA_DIR
    dts = tuple(float(v) for v in sys.argv[3].split(",")) if len(sys.argv) > 3 else (configs.DT_SMALL, configs.DT_LARGE)
    hidden = tuple(int(v) for v in sys.argv[4].split(",")) if len(sys.argv) > 4 else (128, 128)
    os.makedirs(outdir, exist_ok=True)
    for dt in dts:
        src = os.path.join(configs.DATA_DIR, f"{mech}_train_dt{dt:g}.npz")
        d = dict(np.load(src, allow_pickle=False))
        out = os.path.join(outdir, os.path.basename(path_for(mech, dt)))
        rep = train(mech, dt, d, hidden=hidden, out_path=out, log=lambda s: print(s, flush=True))
        with open(out + ".json", "w") as fh:
            json.dump(rep, fh, indent=1)
        print(f"{mech} dt={dt:g}: wrote {out}", flush=True)
