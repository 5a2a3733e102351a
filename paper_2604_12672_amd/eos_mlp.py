"""Learned initial guess for the temperature inversion of the gas+radiation
EOS (offline training; not part of the timed step).

The guess T0 = 10^MLP(log10 rho, log10 e_int) comes from a 2 -> 64 -> 64 -> 1
ReLU network.  On the GPU a separate guess kernel evaluates it before each
stage: layer 1 on v_mfma_f32_32x32x8_bf16, layer 2 on
v_mfma_f32_32x32x16_bf16 (FP32 accumulation), layer 3 as BF16 dot products
on the vector unit (v_dot2c_f32_bf16); the same kernel then polishes the
guess by the FP64 Newton iteration (which fixes T to the 1e-11 tolerance
whatever the guess), with the bracketed solve as fallback, and the stage
starts from the polished temperature.

Training data: log-uniform rho in [1e-2, 1e2] and T in [1e5, 1e8] (seeded),
e_int from the forward EOS e = R T/((gamma-1) mu) + a T^4/rho; inputs and
target mapped affinely to [-1, 1]; Adam on the mean squared error in float32
(torch on the CPU).  Export: W2, W3 rounded to BF16 (round to nearest even);
W1 and all biases kept in FP32 (the kernel carries W1 and b1 as hi/lo BF16
pairs through the first MFMA, and b2, b3 in the FP32 accumulator).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "data", "eos_mlp_gasrad.json")
HIDDEN = 64


# --------------------------------------------------------------------------
# BF16 helpers (round to nearest even)
# --------------------------------------------------------------------------

def bf16_bits(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    return (u >> 16).astype(np.uint16)


def bf16_value(bits):
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32)


def bf16_round(x):
    return bf16_value(bf16_bits(x))


# --------------------------------------------------------------------------
# samples
# --------------------------------------------------------------------------

def eos_e(params, rho, T):
    """Forward EOS: specific internal energy e(rho, T) (eq. erad)."""
    rmu = params["rgas"] / params["mu"]
    return rmu * T / (params["gamma"] - 1.0) + params["arad"] * T ** 4 / rho


def sample(params, n, seed=5, rho_range=(1e-2, 1e2), t_range=(1e5, 1e8)):
    rng = np.random.default_rng(seed)
    lr = rng.uniform(math.log10(rho_range[0]), math.log10(rho_range[1]), size=n)
    lt = rng.uniform(math.log10(t_range[0]), math.log10(t_range[1]), size=n)
    rho, T = 10.0 ** lr, 10.0 ** lt
    return rho, eos_e(params, rho, T), T


class MLPGuess:
    """Weights and affine input/output maps of the guess network."""

    def __init__(self, w1, b1, w2, b2, w3, b3, norm):
        self.w1 = np.asarray(w1, np.float32)   # [64, 2]
        self.b1 = np.asarray(b1, np.float32)   # [64]
        self.w2 = np.asarray(w2, np.float32)   # [64 out, 64 in], BF16-representable
        self.b2 = np.asarray(b2, np.float32)   # [64]
        self.w3 = np.asarray(w3, np.float32)   # [64], BF16-representable
        self.b3 = float(b3)
        # x0 = (log10 rho - c_rho) * s_rho, x1 = (log10 e - c_e) * s_e,
        # log10 T = y / s_T + c_T
        self.norm = [float(v) for v in norm]   # c_rho, s_rho, c_e, s_e, c_T, s_T

    # -- inference as the kernel evaluates it ---------------------------------
    def inputs(self, rho, e):
        c0, s0, c1, s1, _, _ = self.norm
        x0 = np.clip(((np.log10(rho) - c0) * s0).astype(np.float32), -1, 1)
        x1 = np.clip(((np.log10(e) - c1) * s1).astype(np.float32), -1, 1)
        return x0, x1

    def predict_log10T(self, rho, e):
        """Emulates the kernel: layer 1 with hi/lo BF16 splits of inputs,
        W1 and b1; BF16 activations and W2, W3; FP32 accumulation."""
        x0, x1 = self.inputs(np.asarray(rho, np.float64), np.asarray(e, np.float64))
        x0h = bf16_round(x0)
        x0l = bf16_round(x0 - x0h)
        x1h = bf16_round(x1)
        x1l = bf16_round(x1 - x1h)
        w = self.w1
        w0h, w1h = bf16_round(w[:, 0]), bf16_round(w[:, 1])
        w0l, w1l = bf16_round(w[:, 0] - w0h), bf16_round(w[:, 1] - w1h)
        bh = bf16_round(self.b1)
        bl = bf16_round(self.b1 - bh)
        h1 = (np.outer(x0h, w0h) + np.outer(x0h, w0l) + np.outer(x0l, w0h) +
              np.outer(x1h, w1h) + np.outer(x1h, w1l) + np.outer(x1l, w1h) + bh + bl)
        h1 = bf16_round(np.maximum(h1.astype(np.float32), 0))
        h2 = h1 @ self.w2.T + self.b2
        h2 = bf16_round(np.maximum(h2.astype(np.float32), 0))
        y = h2 @ self.w3 + self.b3
        _, _, _, _, cT, sT = self.norm
        return y.astype(np.float64) / sT + cT

    def predict_T(self, rho, e):
        return 10.0 ** self.predict_log10T(rho, e)

    # -- storage --------------------------------------------------------------
    def to_json(self):
        return {"w1": self.w1.tolist(), "b1": self.b1.tolist(),
                "w2_bf16": bf16_bits(self.w2).astype(int).tolist(), "b2": self.b2.tolist(),
                "w3_bf16": bf16_bits(self.w3).astype(int).tolist(), "b3": self.b3,
                "norm": self.norm}

    @classmethod
    def from_json(cls, d):
        return cls(d["w1"], d["b1"], bf16_value(np.asarray(d["w2_bf16"], np.uint16)), d["b2"],
                   bf16_value(np.asarray(d["w3_bf16"], np.uint16)), d["b3"], d["norm"])

    def save(self, path=DEFAULT_PATH, meta=None):
        os.makedirs(os.path.dirname(path), exist_ok=True)
        d = self.to_json()
        if meta:
            d["meta"] = meta
        with open(path, "w") as f:
            json.dump(d, f)

    @classmethod
    def load(cls, path=DEFAULT_PATH):
        with open(path) as f:
            return cls.from_json(json.load(f))

    def ctypes_args(self):
        """Arrays for mhd_set_eos_mlp: w1 [64][2] f32, b1 [64] f32,
        w2 [64][64] bf16 bits, b2 [64] f32, w3 [64] bf16 bits, b3, norm [6]."""
        return (np.ascontiguousarray(self.w1, np.float32), np.ascontiguousarray(self.b1, np.float32),
                np.ascontiguousarray(bf16_bits(self.w2)), np.ascontiguousarray(self.b2, np.float32),
                np.ascontiguousarray(bf16_bits(self.w3)), float(self.b3),
                np.ascontiguousarray(self.norm, np.float64))


def train(params, n=1_000_000, n_val=100_000, seed=5, epochs=24, batch=8192, lr=3e-3,
          threads=None, verbose=True):
    """Train the guess network on samples of the forward EOS."""
    import torch
    if threads:
        torch.set_num_threads(threads)
    torch.manual_seed(seed)
    rho, e, T = sample(params, n + n_val, seed=seed)
    lr_, le, lt = np.log10(rho), np.log10(e), np.log10(T)
    c0, s0 = 0.0, 0.5                                   # log10 rho in [-2, 2]
    c1 = 0.5 * (le.min() + le.max())
    s1 = 2.0 / (le.max() - le.min())
    cT, sT = 6.5, 1.0 / 1.5                             # log10 T in [5, 8]
    X = np.stack([(lr_ - c0) * s0, (le - c1) * s1], 1).astype(np.float32)
    Y = ((lt - cT) * sT).astype(np.float32)[:, None]
    Xt, Yt = torch.from_numpy(X[:n]), torch.from_numpy(Y[:n])
    Xv, Yv = torch.from_numpy(X[n:]), torch.from_numpy(Y[n:])
    net = torch.nn.Sequential(torch.nn.Linear(2, HIDDEN), torch.nn.ReLU(),
                              torch.nn.Linear(HIDDEN, HIDDEN), torch.nn.ReLU(),
                              torch.nn.Linear(HIDDEN, 1))
    opt = torch.optim.Adam(net.parameters(), lr=lr)
    steps = epochs * (n // batch)
    sched = torch.optim.lr_scheduler.OneCycleLR(opt, max_lr=lr, total_steps=steps)
    for ep in range(epochs):
        perm = torch.randperm(n)
        for i in range(n // batch):
            idx = perm[i * batch:(i + 1) * batch]
            opt.zero_grad()
            loss = torch.mean((net(Xt[idx]) - Yt[idx]) ** 2)
            loss.backward()
            opt.step()
            sched.step()
        if verbose and (ep % 4 == 3 or ep == epochs - 1):
            with torch.no_grad():
                err = (net(Xv) - Yv).abs().max().item() / sT
            print(f"epoch {ep + 1}: train mse {loss.item():.3e}, max |dlog10 T| (val) {err:.3e}",
                  flush=True)
    l1, l2, l3 = net[0], net[2], net[4]
    m = MLPGuess(l1.weight.detach().numpy(), l1.bias.detach().numpy(),
                 bf16_round(l2.weight.detach().numpy()), l2.bias.detach().numpy(),
                 bf16_round(l3.weight.detach().numpy()[0]), float(l3.bias.detach().numpy()[0]),
                 [c0, s0, c1, s1, cT, sT])
    dv = np.abs(m.predict_log10T(rho[n:], e[n:]) - lt[n:])
    stats = {"samples": n, "holdout": n_val, "seed": seed, "epochs": epochs,
             "holdout_max_abs_dlog10T": float(dv.max()),
             "holdout_mean_abs_dlog10T": float(dv.mean())}
    if verbose:
        print("quantised guess on holdout:", stats, flush=True)
    return m, stats


if __name__ == "__main__":
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2604_12672_amd import workloads as wl
    p = wl.gasrad_params(1, 1, 1)
    model, st = train(p)
    model.save(meta=st)
    print("saved", DEFAULT_PATH)
