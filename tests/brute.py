"""Brute-force checkers for tiny images, written independently of the oracle.

These follow the paper's formulas as printed wherever they are unambiguous:
all-pairs sums with 1/N (eq. MAsystem), dense Jacobians from the printed
partial derivatives (Sec. 3.1), the reflective index rule of Def. 3.1 applied
literally on the paper's 1-based vectorised indexing, the printed divergence
and wide Laplacian (eq. discrete_divergence, eq. discrete_laplacian), and a
numerical minimisation for the shrinkage step (Sec. 4.1).  They are slow
(O(N^2)) and meant for images of at most 8 x 8 pixels.
"""
from __future__ import annotations

import numpy as np


# --- kernel, written from Wendland's C^2 function (cited at eq. kernel) ---
def wendland(r):
    r = np.asarray(r, dtype=np.float64)
    t = np.clip(1.0 - r, 0.0, None)
    out = (1.0 + 4.0 * r) * t ** 4
    return np.where((r >= 0) & (r <= 1), out, 0.0)


def wendland_d(r, h=None):
    """Derivative of the kernel: from its expanded polynomial (default) or, when
    ``h`` is given, by a central difference of ``wendland``."""
    r = np.asarray(r, dtype=np.float64)
    if h is None:
        # analytic derivative of (1+4r)(1-r)^4 expanded as a polynomial in r
        # (1+4r)(1 - 4r + 6r^2 - 4r^3 + r^4) = 1 - 10 r^2 + 20 r^3 - 15 r^4 + 4 r^5
        d = -20.0 * r + 60.0 * r ** 2 - 60.0 * r ** 3 + 20.0 * r ** 4
        return np.where((r >= 0) & (r <= 1), d, 0.0)
    return (wendland(r + h) - wendland(r - h)) / (2 * h)


# --- agents ---
def positions(H, W):
    """Normalised agent coordinates (x_i, y_i) in the paper's vectorised order
    (row-major, row 0 first); shape (N, 2)."""
    q, r = np.meshgrid(np.arange(W), np.arange(H))
    return np.stack([q.ravel() / W, r.ravel() / H], axis=1)


def rhs_allpairs(c, ex, ec, s=None):
    """F_i = s sum_{j=1..N} phi(r_ij) (c_j - c_i) over ALL agents (eq. MAsystem, s = 1/N)."""
    H, W, C = c.shape
    N = H * W
    X = positions(H, W)
    cf = c.reshape(N, C)
    s = 1.0 / N if s is None else s
    F = np.zeros((N, C))
    for i in range(N):
        for j in range(N):
            dxy = X[j] - X[i]
            dc = cf[j] - cf[i]
            rij = 0.5 * ex * (dxy @ dxy) + 0.5 * ec * (dc @ dc)
            F[i] += wendland(rij) * dc
    return (s * F).reshape(H, W, C)


def euler_allpairs(c, ex, ec, dt, s=None):
    return c + dt * rhs_allpairs(c, ex, ec, s)


def jacobian_paper_c1(c, ex, ec, s=None):
    """Dense dF/dc for C = 1 from the printed formulas of Sec. 3.1:
    k != i: (1/N)[phi'(r_ik) ec (c_k - c_i)^2 + phi(r_ik)],
    k == i: -(1/N) sum_j [phi'(r_ij) ec (c_j - c_i)^2 + phi(r_ij)].
    The diagonal sum skips j = i: that summand of F_i, phi(r_ii)(c_i - c_i),
    is identically zero, so it has no derivative (the printed sum runs over
    all j, which would add -phi(0)/N)."""
    H, W, C = c.shape
    assert C == 1
    N = H * W
    X = positions(H, W)
    cf = c.reshape(N)
    s = 1.0 / N if s is None else s
    J = np.zeros((N, N))
    for i in range(N):
        for k in range(N):
            dxy = X[k] - X[i]
            d = cf[k] - cf[i]
            rik = 0.5 * ex * (dxy @ dxy) + 0.5 * ec * d * d
            val = s * (wendland_d(rik) * ec * d * d + wendland(rik))
            if k != i:
                J[i, k] += val
                J[i, i] -= val
    return J


def deps_paper_c1(c, ex, ec, s=None):
    """dF_i/d eps_x and dF_i/d eps_c for C = 1 as printed in Sec. 3.1."""
    H, W, C = c.shape
    assert C == 1
    N = H * W
    X = positions(H, W)
    cf = c.reshape(N)
    s = 1.0 / N if s is None else s
    Fx = np.zeros(N)
    Fc = np.zeros(N)
    for i in range(N):
        for j in range(N):
            dxy = X[j] - X[i]
            d = cf[j] - cf[i]
            rij = 0.5 * ex * (dxy @ dxy) + 0.5 * ec * d * d
            Fx[i] += 0.5 * s * wendland_d(rij) * (dxy @ dxy) * d
            Fc[i] += 0.5 * s * wendland_d(rij) * d ** 3
    return Fx, Fc


# --- discrete operators with the paper's literal index rules ---
def grad_paper(c):
    """grad# of Def. 3.1 on the 1-based vectorised image with the reflective rule:
    i+1 -> i-1 if i = 0 mod N_C; i-1 -> i+1 if i = 1 mod N_C;
    i+N_C -> i-N_C if i > N - N_C; i-N_C -> i+N_C if i <= N_C."""
    H, W, C = c.shape
    N = H * W
    cf = c.reshape(N, C)
    dx, dy = 1.0 / W, 1.0 / H
    g = np.zeros((H, W, 2, C))
    for i in range(1, N + 1):
        ip, im = i + 1, i - 1
        if i % W == 0:
            ip = i - 1
        if i % W == 1 % W:
            im = i + 1
        if W == 1:
            ip = im = i
        iu, idn = i + W, i - W
        if i > N - W:
            iu = i - W
        if i <= W:
            idn = i + W
        if H == 1:
            iu = idn = i
        r, q = divmod(i - 1, W)
        g[r, q, 0] = (cf[ip - 1] - cf[im - 1]) / (2 * dx)
        g[r, q, 1] = (cf[iu - 1] - cf[idn - 1]) / (2 * dy)
    return g


def div_paper(w):
    """div# of eq. discrete_divergence with the same reflective rule (literal)."""
    H, W, _, C = w.shape
    N = H * W
    wf = w.reshape(N, 2, C)
    dx, dy = 1.0 / W, 1.0 / H
    out = np.zeros((H, W, C))
    for i in range(1, N + 1):
        ip, im = i + 1, i - 1
        if i % W == 0:
            ip = i - 1
        if i % W == 1 % W:
            im = i + 1
        iu, idn = i + W, i - W
        if i > N - W:
            iu = i - W
        if i <= W:
            idn = i + W
        r, q = divmod(i - 1, W)
        out[r, q] = (wf[ip - 1, 0] - wf[im - 1, 0]) / (2 * dx) + (wf[iu - 1, 1] - wf[idn - 1, 1]) / (2 * dy)
    return out


def wide_laplacian_interior(c):
    """Delta# of eq. discrete_laplacian at pixels at least 2 away from every border
    (where no boundary rule is involved); NaN elsewhere."""
    H, W, C = c.shape
    dx, dy = 1.0 / W, 1.0 / H
    out = np.full((H, W, C), np.nan)
    for r in range(2, H - 2):
        for q in range(2, W - 2):
            out[r, q] = ((c[r, q + 2] - 2 * c[r, q] + c[r, q - 2]) / (2 * dx) ** 2
                         + (c[r + 2, q] - 2 * c[r, q] + c[r - 2, q]) / (2 * dy) ** 2)
    return out


def shrink_bruteforce(a, rho):
    """argmin_w rho/2 |w - a|^2 + |w| by numerical minimisation (no closed form)."""
    from scipy.optimize import minimize

    a = np.asarray(a, dtype=np.float64)

    def f(w):
        return 0.5 * rho * np.sum((w - a) ** 2) + np.sqrt(np.sum(w * w))

    best = None
    for start in (np.zeros_like(a), a.copy(), 0.5 * a):
        res = minimize(f, start, method="Nelder-Mead",
                       options={"xatol": 1e-12, "fatol": 1e-14, "maxiter": 40000, "maxfev": 80000})
        if best is None or res.fun < best.fun:
            best = res
    return best.x, best.fun


# --- dense operators for the end-to-end brute-force solve (C = 1) ---
def grad_matrix(H, W):
    """Dense (2N x N) matrix of grad# built column by column from grad_paper."""
    N = H * W
    D = np.zeros((2 * N, N))
    for k in range(N):
        e = np.zeros((H, W, 1))
        e.reshape(N)[k] = 1.0
        g = grad_paper(e)  # (H, W, 2, 1)
        D[:N, k] = g[:, :, 0, 0].ravel()
        D[N:, k] = g[:, :, 1, 0].ravel()
    return D


def solve_bruteforce(c0, K, dt, eps0, alpha, rho, gamma, M, P, emin, emax, sigma0=1.0, b=0.5,
                     cA=1e-4, max_ls=40, quadratic=False):
    """Alg. 2 with the Alg. 1 control argmin on a tiny grey image, all-pairs dynamics
    (s = 1/N), dense Jacobians and dense grad#.  Returns (c^K, eps, v, mu, taus).
    With ``quadratic`` the DAL loop runs once on J of Def. 3.2 (v = mu = 0, rho = 1,
    no multiplier updates)."""
    if quadratic:
        rho, M = 1.0, 1
    H, W, C = c0.shape
    assert C == 1
    N = H * W
    area = 1.0 / (H * W)
    D = grad_matrix(H, W)
    x0 = c0.reshape(N).astype(np.float64)

    def sweep(eps):
        traj = [x0.copy()]
        for k in range(K):
            ck = traj[-1].reshape(H, W, 1)
            traj.append(euler_allpairs(ck, eps[k, 0], eps[k, 1], dt).reshape(N))
        return traj

    def norms2(w):  # per-pixel squared norm of a (2N,) field
        return w[:N] ** 2 + w[N:] ** 2

    def Ltilde(x, v, mu):
        sh = v - D @ x + mu / rho
        return area * np.sum(0.5 * rho * norms2(sh) + np.sqrt(norms2(v)) + 0.5 * alpha * (x - x0) ** 2)

    def dLtilde(x, v, mu):
        sh = v - D @ x + mu / rho
        return area * (-rho * (D.T @ sh) + alpha * (x - x0))

    def shrink(x, mu):
        a = D @ x - mu / rho
        na = np.sqrt(norms2(a))
        fac = np.where(na > 1.0 / rho, (na - 1.0 / rho) / np.where(na > 0, na, 1.0), 0.0)
        return a * np.concatenate([fac, fac])

    def gradient(traj, eps, v, mu):
        p = dLtilde(traj[-1], v, mu)
        G = np.zeros((K, 2))
        for k in range(K - 1, -1, -1):
            ck = traj[k].reshape(H, W, 1)
            Fx, Fc = deps_paper_c1(ck, eps[k, 0], eps[k, 1])
            G[k, 0] = dt * np.dot(p, Fx)
            G[k, 1] = dt * np.dot(p, Fc)
            J = jacobian_paper_c1(ck, eps[k, 0], eps[k, 1])
            p = p + dt * (J.T @ p)
        return G / dt

    eps = np.array(eps0, dtype=np.float64).reshape(K, 2).copy()
    lo = np.array(emin, dtype=np.float64)
    hi = np.array(emax, dtype=np.float64)
    mu = np.zeros(2 * N)
    traj = sweep(eps)
    v = np.zeros(2 * N) if quadratic else shrink(traj[-1], mu)
    sigma = sigma0
    taus = np.zeros((M, P))

    def trial(tau, G, phi0):
        e = np.clip(eps - tau * G, lo, hi)
        tr = sweep(e)
        ph = Ltilde(tr[-1], v, mu)
        return ph <= phi0 + cA * dt * np.sum(G * (e - eps)), e, tr

    for j in range(M):
        for it in range(P):
            phi0 = Ltilde(traj[-1], v, mu)
            G = gradient(traj, eps, v, mu)
            if not np.any(G != 0):
                break
            tau = sigma
            ok, e, tr = trial(tau, G, phi0)
            n = 1
            best = None
            if ok:
                best = (tau, e, tr)
                while n < max_ls:
                    if np.array_equal(np.clip(eps - (tau / b) * G, lo, hi), best[1]):
                        break
                    tau = tau / b
                    ok, e, tr = trial(tau, G, phi0)
                    n += 1
                    if not ok:
                        break
                    best = (tau, e, tr)
            else:
                while n < max_ls:
                    tau = tau * b
                    ok, e, tr = trial(tau, G, phi0)
                    n += 1
                    if ok:
                        best = (tau, e, tr)
                        break
            if best is None:
                break
            sigma, eps, traj = best
            taus[j, it] = sigma
        if quadratic:
            break
        g = D @ traj[-1]
        v = shrink(traj[-1], mu)
        mu = mu + gamma * (v - g)
    return traj[-1].reshape(H, W, 1), eps, v, mu, taus
