"""Learned warm start for the solver (the network runs in the HIP library).

The network maps an image to a starting multiplier field mu0 and starting
controls eps0 for ``abc_solve``; it is trained on pairs (image, final mu and
eps) produced by the plain method itself.  The warm solve uses the predicted
multiplier with the cold controls by default (``use_eps`` adds the predicted
controls).  The plain cold-started solve stays the reference: both solves run
the solver's own stopping rule (the Lagrangian gap of Sec. 4.1, or the
iteration cap), and the warm result is accepted only when its final TV energy
is within a relative tolerance of the cold solve's (or below it); otherwise
the cold solve is the answer.  Orchestration only; every arithmetic step is a
library call.
"""
from __future__ import annotations

import os
import time
from dataclasses import dataclass

import numpy as np

from . import binding as B
from .synth import voronoi_image, wsnet_init


def make_dataset(n: int, size: int, seed0: int, params: B.Params, batch: int = 64, device="cuda"):
    """n images of size x size (RGB Voronoi: 4-16 regions, sigma U[0.02, 0.1],
    image i seeded seed0 + i), each solved by the plain method; returns device
    tensors (x n x H x W x 3, mu n x H x W x 6, eps n x K x 2)."""
    import torch
    xs, mus, epss = [], [], []
    for s0 in range(0, n, batch):
        imgs, eps_l, mu_l = [], [], []
        for i in range(s0, min(n, s0 + batch)):
            r = np.random.default_rng(seed0 + i)
            regions = int(r.integers(4, 17))
            sigma = float(r.uniform(0.02, 0.1))
            imgs.append(torch.as_tensor(voronoi_image(size, size, 3, regions, sigma, seed0 + i), device=device))
            eps_l.append(torch.full((params.K, 2), params.eps_init, dtype=torch.float32, device=device))
            mu_l.append(torch.zeros((size, size, 2, 3), dtype=torch.float32, device=device))
        B.abc_solve_batched(imgs, params, eps=eps_l, mu=mu_l)
        xs += imgs
        mus += [m.reshape(size, size, 6) for m in mu_l]
        epss += eps_l
    return torch.stack(xs), torch.stack(mus), torch.stack(epss)


# Weights trained by train_warmstart.py for K = 50 (provenance in wsnet_k50.json).
TRAINED_K50 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "wsnet_k50.npy")


@dataclass
class TrainLog:
    losses: list
    seconds: float


class WarmStart:
    def __init__(self, K: int, box: B.Params, seed: int = 0, device="cuda"):
        import torch
        self.K, self.box = K, box
        self.params = torch.as_tensor(wsnet_init(K, seed), device=device)
        assert self.params.numel() == B.abc_wsnet_param_count(K)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0

    @classmethod
    def load(cls, path: str, K: int, box: B.Params, device="cuda"):
        """A network with the FP32 weights stored at path (a flat .npy)."""
        import torch
        ws = cls(K, box, device=device)
        w = np.load(path, allow_pickle=False)
        if w.shape != tuple(ws.params.shape):
            raise ValueError(f"{path}: {w.shape[0]} parameters, the network for K={K} has {ws.params.numel()}")
        ws.params.copy_(torch.as_tensor(w, device=device))
        return ws

    def predict(self, x):
        """(mu0 B x H x W x 2 x 3, eps0 B x K x 2) for images x (B x H x W x 3)."""
        mu0, eps0 = B.abc_wsnet_forward(self.params, x.contiguous(), self.K, self.box)
        return mu0.reshape(x.shape[0], x.shape[1], x.shape[2], 2, 3), eps0

    def train(self, x, mu, eps, epochs: int, batch: int, lr: float, w_eps: float = 1.0, seed: int = 0,
              lr_decay: float = 1.0) -> TrainLog:
        import torch
        n = x.shape[0]
        rng = np.random.default_rng(seed)
        grad = torch.empty_like(self.params)
        losses = []
        t0 = time.perf_counter()
        for ep in range(epochs):
            order = rng.permutation(n)
            ep_loss = []
            for s in range(0, n - batch + 1, batch):
                idx = torch.as_tensor(order[s:s + batch], device=x.device)
                loss, _ = B.abc_wsnet_loss_grad(self.params, x[idx].contiguous(), mu[idx].contiguous(),
                                                eps[idx].contiguous(), self.K, self.box, w_eps, grad=grad)
                self.t += 1
                B.abc_wsnet_adam(self.params, grad, self.m, self.v, self.t, lr)
                ep_loss.append(loss)
            losses.append(float(np.mean(ep_loss)))
            lr *= lr_decay
        torch.cuda.synchronize()
        return TrainLog(losses, time.perf_counter() - t0)

    def solve(self, img, params: B.Params, cold=None, rel_tol: float = 1e-4, use_eps: bool = False):
        """Warm solve of one image (H x W x 3): predicted start, then the plain
        solver with its own stopping rule.  The result stands when its final
        TV energy is within rel_tol of the cold solve's (or lower) and finite;
        otherwise the cold solve is the answer and its time is added.
        ``cold``: an earlier ``cold_solve`` result (computed here if None).
        ``use_eps``: start from the predicted controls as well; by default only
        the predicted multiplier is used and the controls start cold (on
        held-out images the predicted controls leave the energy well above the
        solved one, while the predicted multiplier shortens the multiplier loop)."""
        import torch
        t0 = time.perf_counter()
        mu0, eps0 = self.predict(img[None])
        if use_eps:
            e0 = eps0[0].contiguous()
        else:
            e0 = torch.full((params.K, 2), params.eps_init, dtype=torch.float32, device=img.device)
        out = B.abc_solve(img, params, eps=e0, mu=mu0[0].contiguous())
        torch.cuda.synchronize()
        t_warm = time.perf_counter() - t0
        st = out["stats"]
        c = cold if cold is not None else cold_solve(img, params)
        ok = np.isfinite(st["K"]) and st["K"] <= c["K"] * (1 + rel_tol) and bool(torch.isfinite(out["c"]).all())
        res = {"accepted": ok, "outer_iters": st["outer_iters"], "dal_iters": st["inner_iters"], "seconds": t_warm,
               "K": st["K"], "fallback": False}
        if not ok:
            res.update(fallback=True, seconds=t_warm + c["seconds"], K=c["K"],
                       dal_iters=st["inner_iters"] + c["dal_iters"], outer_iters=st["outer_iters"] + c["outer_iters"])
        return res


def cold_solve(img, params: B.Params, keep_state: bool = False):
    """Plain solve from eps_init, mu = 0 with the solver's stopping rule; with
    keep_state also its final controls and multiplier."""
    import torch
    H, W, C = img.shape
    eps = torch.full((params.K, 2), params.eps_init, dtype=torch.float32, device=img.device)
    mu = torch.zeros((H, W, 2, C), dtype=torch.float32, device=img.device)
    t0 = time.perf_counter()
    out = B.abc_solve(img, params, eps=eps, mu=mu)
    torch.cuda.synchronize()
    st = out["stats"]
    res = {"K": st["K"], "seconds": time.perf_counter() - t0, "outer_iters": st["outer_iters"],
           "dal_iters": st["inner_iters"], "outer_log": out["outer_log"][:st["outer_iters"]].tolist()}
    if keep_state:
        res.update(eps=eps, mu=mu)
    return res


def ideal_warm_solve(img, params: B.Params, cold):
    """Upper bound for any predictor: start from the cold solve's own final
    controls and multiplier and run the same stopping rule."""
    import torch
    t0 = time.perf_counter()
    out = B.abc_solve(img, params, eps=cold["eps"].clone(), mu=cold["mu"].clone())
    torch.cuda.synchronize()
    return {"outer_iters": out["stats"]["outer_iters"], "dal_iters": out["stats"]["inner_iters"],
            "seconds": time.perf_counter() - t0, "K": out["stats"]["K"]}
