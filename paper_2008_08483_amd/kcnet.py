"""The approximate ln K_c network of Sec. 2.3 (Architecture 2): weights,
training, and the training set.

The network maps the standardized log temperature through N_L hidden layers
of N_H elu neurons (Eqs. 12 and 14) and a linear readout to the N_R
standardized ln K_c; standardization is by the training set's mean and
standard deviation (input and every output separately), as Sec. 2.3 does.
Training is supervised regression with the mean-squared error of the
standardized outputs on temperatures drawn uniformly from a range known in
advance (Sec. 3.1: 10^6 samples per mechanism).  The paper does not give its
optimizer settings; ``train`` uses Adam with a cosine-decayed learning rate.

Training runs in PyTorch (CPU or GPU); inference of a trained network runs
in the library's kernel (``annkin.KcNet``, ``annkin.eval_lnkc_net``,
``annkin.eval_source_net``).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class KcNetWeights:
    """Weights of an Architecture-2 network (float64 arrays).

    ``weights``: N_L + 1 matrices, [1, N_H], [N_H, N_H] ... [N_H, N_R], used as
    X W; ``biases``: the matching vectors; ``x_mean``, ``x_std``: the input's
    standardization; ``y_mean``, ``y_std`` [N_R]: the outputs'."""

    weights: list
    biases: list
    x_mean: float
    x_std: float
    y_mean: np.ndarray
    y_std: np.ndarray
    history: list = field(default_factory=list)   # mean loss per epoch

    @property
    def n_layers(self) -> int:
        return len(self.weights) - 1

    @property
    def n_hidden(self) -> int:
        return int(self.weights[0].shape[1])

    @property
    def n_out(self) -> int:
        return int(self.weights[-1].shape[1])

    def save(self, path: str) -> None:
        arrays = {f"W{l}": w for l, w in enumerate(self.weights)}
        arrays.update({f"B{l}": b for l, b in enumerate(self.biases)})
        np.savez(path, n_layers=self.n_layers, x_mean=self.x_mean, x_std=self.x_std,
                 y_mean=self.y_mean, y_std=self.y_std, history=np.asarray(self.history),
                 **arrays)

    @staticmethod
    def load(path: str) -> "KcNetWeights":
        z = np.load(path, allow_pickle=False)
        nl = int(z["n_layers"])
        return KcNetWeights([z[f"W{l}"] for l in range(nl + 1)],
                            [z[f"B{l}"] for l in range(nl + 1)], float(z["x_mean"]),
                            float(z["x_std"]), z["y_mean"], z["y_std"], list(z["history"]))


def random_weights(n_layers: int, n_hidden: int, n_out: int, seed: int = 0,
                   x_mean: float = 7.3, x_std: float = 0.6) -> KcNetWeights:
    """An untrained network with Glorot-uniform weights and small random
    biases and output scales (for tests and timing)."""
    rng = np.random.default_rng(seed)
    dims = [1] + [n_hidden] * n_layers + [n_out]
    W, B = [], []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = math.sqrt(6.0 / (a + b))
        W.append(rng.uniform(-lim, lim, (a, b)))
        B.append(rng.uniform(-0.1, 0.1, b))
    return KcNetWeights(W, B, x_mean, x_std, rng.normal(0.0, 20.0, n_out),
                        rng.uniform(1.0, 30.0, n_out))


def training_set(mech, n: int = 1_000_000, T_range=(300.0, 3000.0), seed: int = 0,
                 chunk: int = 1 << 18):
    """(T [n], ln K_c [N_R, n]) with T uniform in ``T_range``, ln K_c from the
    library's Gibbs and stoichiometric layers (``annkin.eval_lnkc``, FP64)
    for the mechanism ``mech`` (an ``annkin.Mechanism``), on its GPU."""
    import torch

    from . import annkin
    g = torch.Generator(device="cpu").manual_seed(seed)
    T = torch.empty(n, dtype=torch.float64).uniform_(*T_range, generator=g)
    out = np.empty((mech.n_reactions, n))
    dev = torch.device("cuda", mech.device)
    for a in range(0, n, chunk):
        Tc = T[a:a + chunk].to(dev)
        out[:, a:a + chunk] = annkin.eval_lnkc(mech, Tc).cpu().numpy()
    return T.numpy(), out


def train(T, lnK, n_layers: int, n_hidden: int, epochs: int = 60, batch: int = 4096,
          lr: float = 3e-3, seed: int = 0, device=None, log_every: int = 0) -> KcNetWeights:
    """Fit an Architecture-2 network to (T [n], ln K_c [N_R, n]): MSE of the
    standardized outputs, Adam, the learning rate decayed by a cosine to 1 %
    of ``lr`` over ``epochs``, minibatches of ``batch`` drawn in a seeded
    random order."""
    import torch

    torch.manual_seed(seed)
    dev = torch.device(device) if device is not None else torch.device("cpu")
    x = np.log(np.asarray(T, np.float64))
    y = np.asarray(lnK, np.float64).T          # [n, N_R]
    x_mean, x_std = float(x.mean()), float(x.std())
    y_mean, y_std = y.mean(axis=0), y.std(axis=0)
    y_std = np.where(y_std > 0, y_std, 1.0)
    X = torch.tensor((x - x_mean) / x_std, dtype=torch.float32, device=dev)[:, None]
    Yt = torch.tensor((y - y_mean) / y_std, dtype=torch.float32, device=dev)
    n, nr = Yt.shape
    layers = []
    d = 1
    for _ in range(n_layers):
        layers += [torch.nn.Linear(d, n_hidden), torch.nn.ELU()]
        d = n_hidden
    layers.append(torch.nn.Linear(d, nr))
    model = torch.nn.Sequential(*layers).to(dev)
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    steps = max(1, epochs * ((n + batch - 1) // batch))
    sched = torch.optim.lr_scheduler.LambdaLR(
        opt, lambda s: 0.01 + 0.99 * 0.5 * (1.0 + math.cos(math.pi * min(s, steps) / steps)))
    gen = torch.Generator(device="cpu").manual_seed(seed)
    history = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(dev)
        tot = 0.0
        for a in range(0, n, batch):
            idx = perm[a:a + batch]
            loss = torch.mean((model(X[idx]) - Yt[idx]) ** 2)
            opt.zero_grad(set_to_none=True)
            loss.backward()
            opt.step()
            sched.step()
            tot += float(loss.detach()) * idx.numel()
        history.append(tot / n)
        if log_every and (ep + 1) % log_every == 0:
            print(f"epoch {ep + 1}: mse {history[-1]:.3e}", flush=True)
    lin = [m for m in model if isinstance(m, torch.nn.Linear)]
    W = [m.weight.detach().double().cpu().numpy().T.copy() for m in lin]
    B = [m.bias.detach().double().cpu().numpy().copy() for m in lin]
    return KcNetWeights(W, B, x_mean, x_std, y_mean, y_std, history)
