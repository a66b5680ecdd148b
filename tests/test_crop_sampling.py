"""The sampling behind the maximum-size GPU tests, checked on the CPU: oracle
crops (eps_x, or rho, gamma, alpha and v, rescaled to the crop's pixel
spacing) reproduce the oracle's own values on the whole image, pixel by pixel
and for the control gradient and the energies summed over patch crops, to
FP64 rounding."""
import numpy as np
import pytest

from paper_2510_16154_amd.synth import hashed_block, patched_block
from tests.crop_checks import (ENERGY_KEYS, boundary_pixels, patch_gradient, pd_patch_energies, pd_sampled,
                               sampled_values)


@pytest.mark.parametrize("N,C,R,K", [(120, 3, 2, 2), (96, 5, 1, 3)])
def test_crops_reproduce_the_whole_image(orc, N, C, R, K):
    side = 4
    patches = [(0, 0, side), (N // 2 - 2, N // 2 + 1, side), (N - side, N - side, side), (0, N - side - 3, side)]
    seed_c, seed_p = 11, 12

    def block_c0(y0, h, x0, w):
        return patched_block(y0, h, x0, w, N, C, seed_c, patches).numpy().astype(np.float64)

    def block_pK(y0, h, x0, w):
        return hashed_block(y0, h, x0, w, N, C, seed_p).numpy().astype(np.float64)

    rng = np.random.default_rng(5)
    eps = np.stack([N * N * rng.uniform(0.01, 0.05, K), rng.uniform(2.0, 8.0, K)], axis=1)
    s = 1.0 / (2 * R + 1) ** 2
    c0, pK = block_c0(0, N, 0, N), block_pK(0, N, 0, N)
    P = orc.Params(K=K, R=R, s=s)
    traj = orc.forward_sweep(c0, P, eps)
    p0, ge = orc.adjoint_sweep(traj, P, pK, eps)
    # the spatial term matters: the control gradient has both components
    assert np.all(np.abs(ge) > 1e-8 * np.abs(ge).max())

    pixels = [(y % N, x % N) for y, x in boundary_pixels(N, C)]
    pixels += [(1, 2), (N // 2, N // 2 + 2), (N - 2, N - 3), (3, N - 4)]
    pixels += [tuple(v) for v in rng.integers(0, N, size=(8, 2))]
    cK_s, p0_s = sampled_values(orc, block_c0, block_pK, pixels, N, R, K, eps, s)
    want_c = np.array([traj[K, y, x] for y, x in pixels])
    want_p = np.array([p0[y, x] for y, x in pixels])
    assert np.max(np.abs(cK_s - want_c)) <= 1e-13 * np.max(np.abs(want_c))
    assert np.max(np.abs(p0_s - want_p)) <= 1e-13 * np.max(np.abs(want_p))
    # pixels near the patches have moved, so the check is not of constants only
    assert np.any(np.abs(want_c - 0.5) > 1e-3)

    ge_s = patch_gradient(orc, block_c0, block_pK, patches, N, R, K, eps, s)
    assert np.max(np.abs(ge_s - ge)) <= 1e-11 * np.max(np.abs(ge))


def test_a_crop_with_the_unscaled_control_does_not(orc):
    """A plausible slip, the crop run with the image's own eps_x, fails the comparison."""
    N, C, R, K = 120, 3, 2, 2
    patches = [(50, 50, 4)]
    c0 = patched_block(0, N, 0, N, N, C, 11, patches).numpy().astype(np.float64)
    pK = hashed_block(0, N, 0, N, N, C, 12).numpy().astype(np.float64)
    eps = np.array([[0.03 * N * N, 4.0]] * K)
    s = 1.0 / (2 * R + 1) ** 2
    P = orc.Params(K=K, R=R, s=s)
    traj = orc.forward_sweep(c0, P, eps)
    y, x, w = 52, 49, 2 * 2 * K * R + 1
    y0, x0 = y - w // 2, x - w // 2
    crop = orc.forward_sweep(c0[y0:y0 + w, x0:x0 + w], P, eps)
    assert np.max(np.abs(crop[K, y - y0, x - x0] - traj[K, y, x])) > 1e-6


def pd_blocks(N, C, patches, amp=0.5):
    """(cK, c0, v, mu) blocks of an image that is 0.5 (cK = c0) with v = mu = 0
    outside the patches and hashed inside them."""
    def blocks(y0, h, x0, w):
        cK = patched_block(y0, h, x0, w, N, C, 21, patches, amp=amp)
        c0 = patched_block(y0, h, x0, w, N, C, 22, patches, amp=amp)
        v = patched_block(y0, h, x0, w, N, 2 * C, 23, patches, background=0.0, amp=1.0)
        mu = patched_block(y0, h, x0, w, N, 2 * C, 24, patches, background=0.0, amp=1.0)
        return tuple(t.numpy().astype(np.float64) for t in (cK, c0, v.view(h, w, 2, C), mu.view(h, w, 2, C)))
    return blocks


@pytest.mark.parametrize("N,C", [(120, 3), (90, 2)])
def test_pd_crops_reproduce_the_whole_image(orc, N, C):
    side = 5
    patches = [(0, 0, side), (N // 2, N // 2 - 3, side), (N - side, N - side, side), (N - side - 1, 2, side)]
    blocks = pd_blocks(N, C, patches)
    alpha, rho, gamma = 3000.0, 1e-2, 1e-2
    cK, c0, v, mu = blocks(0, N, 0, N)
    P = orc.Params(alpha=alpha, rho=rho, gamma=gamma)
    pK, Lt = orc.terminal(cK, c0, v, mu, P)
    vn, mun, E = orc.pd_step(cK, c0, v, mu, P, update_mu=True)
    # both branches of the shrinkage occur: among the pixels with grad# c != 0,
    # some end with v = 0 and some with v != 0
    nv = np.linalg.norm(vn.reshape(N * N, -1), axis=1)
    moving = np.linalg.norm(orc.grad(cK).reshape(N * N, -1), axis=1) > 0
    assert np.any(nv[moving] == 0) and np.any(nv[moving] > 0)

    pixels = [(y % N, x % N) for y, x in boundary_pixels(N, C)]
    pixels += [(1, 1), (N // 2 + 1, N // 2 - 4), (N - 1, N - 2), (N - side - 2, 3), (0, 5)]
    pixels += [tuple(int(t) for t in p) for p in np.random.default_rng(3).integers(0, N, size=(8, 2))]
    sp, sv, sm = pd_sampled(orc, blocks, pixels, N, alpha, rho, gamma)
    for got, full in ((sp, pK), (sv, vn), (sm, mun)):
        want = np.array([full[y, x] for y, x in pixels])
        assert np.max(np.abs(got - want)) <= 1e-12 * max(np.max(np.abs(want)), 1e-300)
    assert np.max(np.abs(sp)) > 0 and np.max(np.abs(sv)) > 0

    Lt_s, tot = pd_patch_energies(orc, blocks, patches, N, alpha, rho, gamma)
    assert abs(Lt_s - Lt) <= 1e-12 * abs(Lt)
    for k in ENERGY_KEYS + ("sq_vg", "sq_g", "sq_v", "r_abs", "r_rel"):
        assert abs(tot[k] - E[k]) <= 1e-12 * abs(E[k]), k
