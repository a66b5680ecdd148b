"""Images past 2^31 elements (the header allows H W C <= 4e9, every element
index in 32 unsigned bits): one forward and one adjoint sweep through the C
ABI, compared with the FP64 oracle at sampled pixels (corners, both sides of
element index 2^31, around patches, random ones), each from an oracle crop
(tests/crop_checks.py; the crop method itself is checked against whole-image
oracle runs in test_crop_sampling.py), and the control gradient against the
sum of the oracle's patch crops.  The image is constant outside six small
patches of hashed colours (amplitude 0.5 sqrt(3 / C), so that with eps_c in
[2, 8] most colour differences stay inside the kernel's support); the adjoint
seed p^K is hashed everywhere.  Both are made from element indices
(synth.hashed_block), on the GPU for the whole image and on the CPU for the
crops.  eps_x is N^2 times U(0.01, 0.05): at these sizes a control inside the
paper's box would leave the spatial term of the kernel argument below 1e-5.

The terminal condition and the primal/dual step are checked the same way on
images that are 0.5 with v = mu = 0 outside the patches (crops with rho,
gamma, alpha and v rescaled to the crop's pixel spacing, tests/crop_checks.py).

Tolerances as in the other parity tests: 1e-4 relative L-infinity over the
sampled fields, 1e-4 relative l2 on eps dl/deps, 1e-5 on energies."""
import numpy as np
import pytest

import paper_2510_16154_amd as A
from paper_2510_16154_amd.synth import hashed_block, patched_block
from tests.crop_checks import (ENERGY_KEYS, boundary_pixels, patch_gradient, pd_patch_energies, pd_sampled,
                               sampled_values)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-4
ENERGY_TOL = 1e-5

CASES = [
    # N (square image), C, R, K; every case has 2.15e9-2.19e9 elements (8.6-8.8 GB per field)
    (27000, 3, 5, 2),   # one lane per pixel, two pixels per thread
    (8400, 31, 2, 2),   # eight channels per lane, four lanes per pixel
    (46400, 1, 3, 2),   # more than 2^31 pixels as well
]


def relinf(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


def rel2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def patches_for(N, C, side=6):
    """Four corners, the middle and around element index 2^31."""
    q = (1 << 31) // C
    by, bx = min(q // N, N - side), min(max(q % N - side // 2, 0), N - side)
    return [(0, 0, side), (N - side, N - side, side), (0, N - side, side), (N - side, 0, side),
            (N // 2, N // 3, side), (by, bx, side)]


def sample_pixels(N, C, patches, rng):
    pixels = boundary_pixels(N, C)
    for py, px, sd in patches:
        pixels += [(py, px), (py + sd // 2, px + sd - 1), (min(py + sd + 1, N - 1), px)]
    return pixels + [tuple(int(v) for v in p) for p in rng.integers(0, N, size=(8, 2))]


@pytest.mark.parametrize("N,C,R,K", CASES)
def test_past_two_to_the_31_elements(orc, N, C, R, K):
    assert 2 ** 31 < N * N * C <= 4e9
    print(f"[case] max size N={N} C={C} R={R} K={K}: {N * N * C / 1e9:.2f}e9 elements", flush=True)
    patches = patches_for(N, C)
    seed_c, seed_p = 101 + C, 202 + C
    amp = 0.5 * np.sqrt(3.0 / C)
    rng = np.random.default_rng(N + C)
    eps = np.stack([N * N * rng.uniform(0.01, 0.05, K), rng.uniform(2.0, 8.0, K)], axis=1)
    s = 1.0 / (2 * R + 1) ** 2
    gp = A.Params(K=K, R=R, inv_norm=s)

    dev = "cuda"
    c0 = patched_block(0, N, 0, N, N, C, seed_c, patches, amp=amp, device=dev)
    gK = torch.empty((N, N, C), dtype=torch.float32, device=dev)
    rows = max(1, (1 << 26) // (N * C))
    for r0 in range(0, N, rows):
        h = min(rows, N - r0)
        gK[r0:r0 + h] = hashed_block(r0, h, 0, N, N, C, seed_p, device=dev)
    e_gpu = torch.as_tensor(eps.astype(np.float32), device=dev)
    traj = A.abc_forward_dynamics(c0, e_gpu, gp)
    g0, geps = A.abc_adjoint_dynamics(traj, e_gpu, gp, gK)
    torch.cuda.synchronize()
    print("  sweeps done", flush=True)

    pixels = sample_pixels(N, C, patches, rng)
    got_c = np.stack([traj[K, y, x].cpu().numpy() for y, x in pixels]).astype(np.float64)
    got_p = np.stack([g0[y, x].cpu().numpy() for y, x in pixels]).astype(np.float64)
    got_e = geps.cpu().numpy().astype(np.float64)
    del traj, g0, geps, gK, c0
    torch.cuda.empty_cache()

    # oracle inputs come from the generator on the CPU, not from the device
    def block_c0(y0, h, x0, w):
        return patched_block(y0, h, x0, w, N, C, seed_c, patches, amp=amp).numpy().astype(np.float64)

    def block_pK(y0, h, x0, w):
        return hashed_block(y0, h, x0, w, N, C, seed_p).numpy().astype(np.float64)

    want_c, want_p = sampled_values(orc, block_c0, block_pK, pixels, N, R, K, eps, s)
    want_e = patch_gradient(orc, block_c0, block_pK, patches, N, R, K, eps, s)
    start = np.stack([block_c0(y, 1, x, 1)[0, 0] for y, x in pixels])
    moved = np.abs(want_c - start).max()
    # eps dl/deps (the gradient in log eps) weighs both columns alike: eps_x is
    # about 1e7 here and its gradient about 1e-9
    got_l, want_l = got_e * eps, want_e * eps
    print(f"  c^K {relinf(got_c, want_c):.2e} (largest move {moved:.2e})  p^0 {relinf(got_p, want_p):.2e}  "
          f"eps dl/deps {rel2(got_l, want_l):.2e} (columns {np.linalg.norm(want_l, axis=0)})", flush=True)
    assert moved > 1e-4
    assert relinf(got_c, want_c) < FIELD_TOL / 10
    assert relinf(got_p, want_p) < FIELD_TOL
    assert np.all(np.linalg.norm(want_l, axis=0) > 0)
    assert rel2(got_l, want_l) < FIELD_TOL


@pytest.mark.parametrize("N,C", [(N, C) for N, C, _, _ in CASES])
def test_terminal_and_pd_step_past_two_to_the_31_elements(orc, N, C):
    print(f"[case] max size terminal + pd step N={N} C={C}: {N * N * C / 1e9:.2f}e9 elements", flush=True)
    patches = patches_for(N, C)
    amp = 0.5 * np.sqrt(3.0 / C)
    alpha, rho, gamma = 3000.0, 1e-2, 1e-2
    gp = A.Params(alpha=alpha, rho=rho, gamma=gamma)

    def blocks(y0, h, x0, w, device="cpu"):
        cK = patched_block(y0, h, x0, w, N, C, 21, patches, amp=amp, device=device)
        c0 = patched_block(y0, h, x0, w, N, C, 22, patches, amp=amp, device=device)
        v = patched_block(y0, h, x0, w, N, 2 * C, 23, patches, background=0.0, amp=1.0, device=device)
        mu = patched_block(y0, h, x0, w, N, 2 * C, 24, patches, background=0.0, amp=1.0, device=device)
        return cK, c0, v.view(h, w, 2, C), mu.view(h, w, 2, C)

    cK, c0, v, mu = blocks(0, N, 0, N, device="cuda")
    gK, Lt = A.abc_pd_terminal(cK, c0, v, mu, gp)
    st = A.abc_pd_step(cK, c0, v, mu, gp, update_mu=True)
    torch.cuda.synchronize()
    print("  terminal and pd step done", flush=True)
    pixels = sample_pixels(N, C, patches, np.random.default_rng(N + C + 1))
    got = [np.stack([f[y, x].cpu().numpy() for y, x in pixels]).astype(np.float64) for f in (gK, v, mu)]
    del cK, c0, v, mu, gK
    torch.cuda.empty_cache()

    # oracle inputs come from the generator on the CPU, not from the device
    def cpu_blocks(y0, h, x0, w):
        return tuple(t.numpy().astype(np.float64) for t in blocks(y0, h, x0, w))

    want = pd_sampled(orc, cpu_blocks, pixels, N, alpha, rho, gamma)
    Lt_w, E = pd_patch_energies(orc, cpu_blocks, patches, N, alpha, rho, gamma)
    errs = [relinf(g, w) for g, w in zip(got, want)]
    rel = {k: abs(st[k] - E[k]) / abs(E[k]) for k in ENERGY_KEYS + ("r_abs", "r_rel")}
    print(f"  p^K {errs[0]:.2e}  v {errs[1]:.2e}  mu {errs[2]:.2e}  L~ {abs(Lt - Lt_w) / abs(Lt_w):.2e}  "
          + "  ".join(f"{k} {e:.1e}" for k, e in rel.items()), flush=True)
    assert all(np.max(np.abs(w)) > 0 for w in want)
    assert max(errs) < FIELD_TOL
    assert abs(Lt - Lt_w) <= ENERGY_TOL * abs(Lt_w)
    assert max(rel.values()) < ENERGY_TOL
