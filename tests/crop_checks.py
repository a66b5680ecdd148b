"""Oracle values of single pixels of images too large for the oracle.

The sweeps of eq. MAsystem are local: one Euler step moves a pixel by its
(2R+1)^2 window, so after K steps c^K at a pixel depends only on c^0 within
K R of it, and the adjoint p^0 (Sec. 3.1) only on c^0 and p^K within 2 K R.
A square crop of side w around the pixel, clamped into the image, therefore
reproduces the pixel's values exactly, provided every pair keeps its kernel
argument: positions are normalised by the image size (dx = 1/W, dy = 1/H,
Def. 3.1), so on an N x N image the crop runs with eps_x (w / N)^2 in place of
eps_x, and the crop's dl/deps_x is scaled back by (w / N)^2.

The terminal condition and the primal/dual step (eq. admm_terminal, eq.
soft_threshold, eq. dual_ascent) reach one pixel further through the central
differences of grad#, and the gradient scales with the pixel count: on a crop
of side w, lam = w / N, grad# is lam times the image's.  Running the crop with
rho / lam, gamma / lam, alpha lam and the input v times lam gives the same
q = mu + rho (v - grad# c) and shrinkage threshold relative to a, so the crop's
v is lam v, its mu the image's mu, its p^K the image's divided by lam, and
every energy (TV, fidelity, L, L~) the image's divided by lam, while the raw
sums of squares behind the residuals are the image's times lam^2.

The control gradient is a sum over all pairs; on an image that is constant
outside a few far-apart patches, every pair with c_j != c_i lies near a patch
(D = 0 elsewhere, and constant regions stay constant), so the image's gradient
is the sum of the gradients of crops around the patches.
"""
import numpy as np


def crop_box(y: int, x: int, rho: int, N: int):
    """Square box of side 2 rho + 1 around (y, x), shifted into the N x N image."""
    w = 2 * rho + 1
    assert N >= w
    return min(max(y - rho, 0), N - w), min(max(x - rho, 0), N - w), w


def patch_box(py: int, px: int, side: int, margin: int, N: int):
    """Square box of side side + 2 margin around a patch, shifted into the image."""
    w = side + 2 * margin
    assert N >= w
    return min(max(py - margin, 0), N - w), min(max(px - margin, 0), N - w), w


def crop_sweeps(orc, c0, pK, N: int, R: int, K: int, eps, s: float):
    """Oracle forward and adjoint sweeps on a square crop (c0, pK: w x w x C) of
    an N x N image.  Returns (trajectory, p^0, dl/deps) in the image's controls."""
    w = c0.shape[0]
    f = (w / N) ** 2
    e = np.array(eps, dtype=np.float64).reshape(K, 2).copy()
    e[:, 0] *= f
    P = orc.Params(K=K, R=R, s=s)
    traj = orc.forward_sweep(c0, P, e)
    p0, ge = orc.adjoint_sweep(traj, P, pK, e)
    ge[:, 0] *= f
    return traj, p0, ge


def sampled_values(orc, block_c0, block_pK, pixels, N: int, R: int, K: int, eps, s: float):
    """c^K and p^0 of the oracle at each (y, x) of ``pixels`` (n x C each), from
    crops made by block_c0(y0, h, x0, w) and block_pK(y0, h, x0, w)."""
    cK, p0 = [], []
    for y, x in pixels:
        y0, x0, w = crop_box(y, x, 2 * K * R, N)
        traj, q0, _ = crop_sweeps(orc, block_c0(y0, w, x0, w), block_pK(y0, w, x0, w), N, R, K, eps, s)
        cK.append(traj[K, y - y0, x - x0])
        p0.append(q0[y - y0, x - x0])
    return np.array(cK), np.array(p0)


def patch_gradient(orc, block_c0, block_pK, patches, N: int, R: int, K: int, eps, s: float):
    """dl/deps of an N x N image that is constant outside ``patches`` ((py, px,
    side), far apart), summed over crops around the patches."""
    margin = 3 * K * R + R
    total = np.zeros((K, 2))
    for py, px, side in patches:
        y0, x0, w = patch_box(py, px, side, margin, N)
        total += crop_sweeps(orc, block_c0(y0, w, x0, w), block_pK(y0, w, x0, w), N, R, K, eps, s)[2]
    return total


def boundary_pixels(N: int, C: int):
    """Pixels on both sides of element index 2^31 of an N x N x C image, the
    corners and the last pixel."""
    p = (1 << 31) // C
    out = [(0, 0), (0, N - 1), (N - 1, 0), (N - 1, N - 1), (N // 2, N // 2)]
    for q in (p - 1, p, p + 1):
        out.append((q // N, q % N))
    return out


ENERGY_KEYS = ("TV", "fid", "K", "L", "Ltilde")
SQUARE_KEYS = ("sq_vg", "sq_g", "sq_v")


def crop_pd(orc, cK, c0, v, mu, N: int, alpha: float, rho: float, gamma: float):
    """Oracle terminal condition and primal/dual step (multiplier update on) on a
    square crop of an N x N image (cK, c0: w x w x C; v, mu: w x w x 2 x C), in
    the image's units: (p^K, L~, v, mu, energies)."""
    lam = cK.shape[0] / N
    P = orc.Params(alpha=alpha * lam, rho=rho / lam, gamma=gamma / lam)
    pK, Lt = orc.terminal(cK, c0, v * lam, mu, P)
    vn, mun, E = orc.pd_step(cK, c0, v * lam, mu, P, update_mu=True)
    E = dict(E)
    for k in ENERGY_KEYS:
        E[k] *= lam
    for k in SQUARE_KEYS:
        E[k] /= lam * lam
    return pK * lam, Lt * lam, vn / lam, mun, E


def pd_sampled(orc, blocks, pixels, N: int, alpha: float, rho: float, gamma: float):
    """(p^K, v, mu) of the oracle at each pixel of ``pixels``; ``blocks(y0, h, x0,
    w)`` returns the crop's (cK, c0, v, mu)."""
    out = ([], [], [])
    for y, x in pixels:
        y0, x0, w = crop_box(y, x, 4, N)
        pK, _, vn, mun, _ = crop_pd(orc, *blocks(y0, w, x0, w), N, alpha, rho, gamma)
        for lst, f in zip(out, (pK, vn, mun)):
            lst.append(f[y - y0, x - x0])
    return tuple(np.array(o) for o in out)


def pd_patch_energies(orc, blocks, patches, N: int, alpha: float, rho: float, gamma: float):
    """L~ before the step and the energies and residuals after it, of an N x N
    image whose terms vanish outside ``patches`` (cK = c0 and v = mu = 0 there),
    summed over crops around the patches."""
    side = max(sd for _, _, sd in patches)
    tot = {k: 0.0 for k in ENERGY_KEYS + SQUARE_KEYS}
    Lt = 0.0
    for py, px, _ in patches:
        y0, x0, w = patch_box(py, px, side, 3, N)
        _, lt, _, _, E = crop_pd(orc, *blocks(y0, w, x0, w), N, alpha, rho, gamma)
        Lt += lt
        for k in tot:
            tot[k] += E[k]
    tot["r_abs"] = float(np.sqrt(tot["sq_vg"] / (N * N)))
    tot["r_rel"] = float(np.sqrt(tot["sq_vg"]) / max(np.sqrt(tot["sq_g"]), np.sqrt(tot["sq_v"]), 1e-30))
    return Lt, tot
