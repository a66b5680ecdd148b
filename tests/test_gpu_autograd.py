"""Differentiable form: autograd.Function whose backward is the adjoint kernel,
with trajectory checkpointing.  Workload: 2048 x 2048 x 31 smooth-spectrum
Voronoi image, R = 2, K = 100, a checkpoint every 10 steps; the gradient is
compared with the FP64 oracle's on a 64 x 64 crop of that image, and the full
size is checked through properties that hold exactly at any size."""
import numpy as np
import pytest

import paper_2510_16154_amd as A
from paper_2510_16154_amd.autograd import agent_dynamics
from paper_2510_16154_amd.workloads import HYPER2048 as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def relinf(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


def rel2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _eps(K, seed):
    rng = np.random.default_rng(seed)
    return np.column_stack([rng.uniform(20.0, 400.0, K), rng.uniform(20.0, 200.0, K)])


@pytest.fixture(scope="module")
def full_image():
    return wl.image()


def test_crop_gradient_matches_oracle(orc, full_image):
    print("[case] 64x64x31 crop, K=100, ckpt 10", flush=True)
    crop = np.ascontiguousarray(full_image[992:1056, 992:1056])
    K = wl.K
    eps = _eps(K, 2003)
    w = np.random.default_rng(2003).normal(size=crop.shape)
    gp = A.Params(K=K, R=wl.R, ckpt_every=10)
    c0 = T(crop).requires_grad_(True)
    e = T(eps).requires_grad_(True)
    cK = agent_dynamics(c0, e, gp)
    loss = (cK * T(w)).sum()
    loss.backward()
    op = orc.Params(K=K, R=wl.R)
    traj = orc.forward_sweep(crop, op, eps)
    p0, ge = orc.adjoint_sweep(traj, op, w, eps)
    assert relinf(N(cK), traj[-1]) < 1e-5
    assert relinf(N(c0.grad), p0) < 1e-4
    assert rel2(N(e.grad), ge) < 1e-4


def test_checkpointed_backward_equals_full_trajectory_bitwise():
    H, W, C, K = 96, 80, 31, 30
    from paper_2510_16154_amd.synth import voronoi_image
    img = voronoi_image(H, W, C, 6, 0.05, 7, spectra=True)
    eps = T(_eps(K, 8))
    w = T(np.random.default_rng(9).normal(size=img.shape))
    grads = []
    for ck in (0, 10, 7):
        c0 = T(img).requires_grad_(True)
        e = eps.clone().requires_grad_(True)
        (agent_dynamics(c0, e, A.Params(K=K, R=2, ckpt_every=ck)) * w).sum().backward()
        grads.append((N(c0.grad), N(e.grad)))
    for g in grads[1:]:
        assert np.array_equal(g[0], grads[0][0]) and np.array_equal(g[1], grads[0][1])


def test_full_size_properties(full_image):
    """At 2048 x 2048 x 31 (K = 100, checkpoint every 10): the dynamics conserve
    every channel's sum, and the adjoint of l = sum(c^K) is exactly 1 at every
    pixel with a zero control gradient (its differences p_j - p_i vanish)."""
    print("[case] full 2048x2048x31 K=100 ckpt 10", flush=True)
    K = wl.K
    gp = A.Params(K=K, R=wl.R, ckpt_every=10)
    c0 = T(full_image).requires_grad_(True)
    e = T(_eps(K, 2003)).requires_grad_(True)
    cK = agent_dynamics(c0, e, gp)
    s0 = torch.sum(c0.detach().double(), dim=(0, 1))
    s1 = torch.sum(cK.detach().double(), dim=(0, 1))
    assert float(torch.max(torch.abs(s1 - s0) / torch.abs(s0))) < 1e-5
    cK.sum().backward()
    assert bool(torch.all(c0.grad == 1.0))
    assert bool(torch.all(e.grad == 0.0))
    assert bool(torch.isfinite(cK).all())
