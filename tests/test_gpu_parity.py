"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances: relative L-infinity 1e-4 on colour fields and adjoint fields,
1e-5 on energies; the control gradient within 1e-4 in relative l2.  FP32 on
the GPU, FP64 in the oracle.  Sizes span several tiles with ragged tails;
the full 512 x 512 x 3 (R = 5, K = 50) sweep is compared as a whole.
"""
import dataclasses

import numpy as np
import pytest

import paper_2510_16154_amd as A
from paper_2510_16154_amd.synth import voronoi_image
from tests.solve_checks import grad_errors, own_step_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-4
ENERGY_TOL = 1e-5


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def relinf(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


def rel2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def rand_eps(K, seed, lo=2.0, hi=200.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=(K, 2))


def both_params(orc, H, W, **kw):
    gp = A.Params(**kw)
    op = orc.Params(K=gp.K, R=gp.R, s=gp.inv_norm, alpha=gp.alpha, rho=gp.rho, gamma=gp.gamma,
                    max_outer=gp.max_outer, max_inner=gp.max_inner, max_ls=gp.max_ls, tol_alm=gp.tol_alm,
                    tol_dal=gp.tol_dal, tol_gap=gp.tol_gap)
    return gp, op


FWD_CASES = [
    # H, W, C, R, K, seed
    (32, 32, 3, 2, 20, 1),
    (37, 53, 3, 2, 6, 2),
    (40, 70, 1, 3, 5, 3),
    (33, 29, 4, 1, 5, 4),
    (19, 23, 5, 2, 4, 5),
    (24, 40, 2, 5, 4, 6),
    (16, 18, 31, 2, 3, 7),
    (21, 19, 3, 7, 3, 8),
    (1, 40, 3, 2, 4, 9),
    (40, 1, 3, 2, 4, 10),
    (2, 2, 1, 1, 3, 11),
    (50, 45, 3, 0, 3, 12),
    (9, 12, 64, 2, 2, 13),
    # 16 to 64 channels at radius 1-3 run on the lanes-per-pixel kernels
    (37, 45, 16, 1, 3, 14),
    (70, 33, 31, 3, 3, 15),
    (45, 70, 32, 2, 3, 16),
    (20, 21, 17, 2, 3, 17),
    (33, 40, 40, 1, 2, 18),
    (1, 50, 31, 2, 2, 19),
    # lanes whose 8 channels run past C (two lanes per pixel), eight channels per
    # pixel slot with the runtime radius, and an odd height with two pixels per thread
    (23, 37, 12, 2, 3, 20),
    (29, 31, 7, 4, 3, 21),
    (17, 9, 3, 4, 3, 22),
    (25, 30, 2, 9, 2, 23),
    # the transposed step's two thread layers at every compile-time radius, 2 and 4 channels
    (35, 41, 4, 5, 3, 24),
    (26, 19, 2, 1, 3, 25),
    (19, 50, 4, 3, 2, 26),
]


@pytest.mark.parametrize("H,W,C,R,K,seed", FWD_CASES)
def test_forward_and_adjoint_match_oracle(orc, H, W, C, R, K, seed):
    print(f"[case] fwd/adj H={H} W={W} C={C} R={R} K={K}", flush=True)
    c0 = voronoi_image(H, W, C, 3, 0.05, seed)
    eps = rand_eps(K, seed)
    gp, op = both_params(orc, H, W, K=K, R=R)
    traj = A.abc_forward_dynamics(T(c0), T(eps), gp)
    want = orc.forward_sweep(c0, op, eps)
    got = N(traj)
    assert relinf(got, want) < FIELD_TOL / 10
    gK = np.random.default_rng(seed + 100).normal(size=(H, W, C))
    g0, geps = A.abc_adjoint_dynamics(traj, T(eps), gp, T(gK))
    p0, ge = orc.adjoint_sweep(want, op, gK, eps)
    assert relinf(N(g0), p0) < FIELD_TOL
    if np.linalg.norm(ge) > 0:
        assert rel2(N(geps), ge) < FIELD_TOL
    else:
        assert np.all(N(geps) == 0)


# Controls at the corners of the box E = [2, 1100]^2 (Sec. 3.2), the same for every
# step or alternating between corners: eps_x = 2 keeps the kernel argument of the
# nearest neighbours within 1e-3 of t = 1, eps_c = 1100 cuts most pairs off at the
# edge of the support (all of them at 31 channels, where the gradient is exactly 0).
# At (2, 1100) with 6 channels the gradient (norm 2.7e-7) is carried by pairs near
# t = 0, where t = 1 - r is a difference of numbers close to 1 and FP32 leaves it a
# relative error of about 2^-24 / t; the gradient's relative error is 5.7e-5 there,
# the largest of these cases, and the same in a plain FP32 evaluation of the sums.
BOX_CORNERS = [(2.0, 2.0), (2.0, 1100.0), (1100.0, 2.0), (1100.0, 1100.0), None]


@pytest.mark.parametrize("C,R", [(3, 5), (6, 3), (31, 2)])
@pytest.mark.parametrize("corner", BOX_CORNERS)
def test_forward_and_adjoint_at_the_corners_of_the_control_box(orc, C, R, corner):
    H, W, K = 48, 40, 4
    print(f"[case] box corner {corner} C={C} R={R}", flush=True)
    c0 = voronoi_image(H, W, C, 4, 0.05, 31)
    if corner is None:
        eps = np.array([[2.0, 1100.0], [1100.0, 2.0], [2.0, 2.0], [1100.0, 1100.0]])
    else:
        eps = np.tile(corner, (K, 1))
    gp, op = both_params(orc, H, W, K=K, R=R)
    traj = A.abc_forward_dynamics(T(c0), T(eps), gp)
    want = orc.forward_sweep(c0, op, eps)
    assert relinf(N(traj), want) < FIELD_TOL / 10
    gK = np.random.default_rng(131).normal(size=(H, W, C))
    g0, geps = A.abc_adjoint_dynamics(traj, T(eps), gp, T(gK))
    p0, ge = orc.adjoint_sweep(want, op, gK, eps)
    print(f"  errors: c^K {relinf(N(traj), want):.2e} p^0 {relinf(N(g0), p0):.2e} "
          f"dl/deps {rel2(N(geps), ge):.2e} (|dl/deps| {np.linalg.norm(ge):.2e})", flush=True)
    assert relinf(N(g0), p0) < FIELD_TOL
    if np.linalg.norm(ge) > 0:
        assert rel2(N(geps), ge) < FIELD_TOL
    else:
        assert np.all(N(geps) == 0)


@pytest.mark.parametrize("C,R,tiles", [
    (3, 2, [(32, 16), (32, 8), (16, 16), (64, 4), (8, 16), (128, 2), (16, 8)]),
    (3, 5, [(32, 16), (64, 8), (16, 8), (32, 4)]),
    (31, 2, [(32, 8), (16, 16), (16, 8), (8, 8), (64, 4)]),
    (64, 1, [(16, 8), (8, 8), (8, 16), (32, 4)]),
])
def test_tile_shape_does_not_change_a_single_bit(orc, C, R, tiles):
    H, W, K = 45, 77, 4
    c0 = voronoi_image(H, W, C, 4, 0.05, 21)
    eps = rand_eps(K, 21)
    gK = T(np.random.default_rng(22).normal(size=(H, W, C)))
    ref = None
    for tx, ty in tiles:
        gp = A.Params(K=K, R=R, tile_x=tx, tile_y=ty)
        traj = A.abc_forward_dynamics(T(c0), T(eps), gp)
        g0, _ = A.abc_adjoint_dynamics(traj, T(eps), gp, gK)
        cur = (N(traj), N(g0))
        if ref is None:
            ref = cur
        else:
            assert np.array_equal(cur[0], ref[0]) and np.array_equal(cur[1], ref[1]), (tx, ty)


@pytest.mark.parametrize("C", [3, 31])
def test_constant_image_is_a_bitwise_fixed_point(C):
    c0 = np.full((40, 36, C), 0.4375, dtype=np.float32)
    gp = A.Params(K=5, R=3)
    traj = N(A.abc_forward_dynamics(T(c0), T(rand_eps(5, 1)), gp))
    assert np.all(traj == 0.4375)


# C = 3 and 31 with v, mu given take the pixel kernels' condition-free channel
# loops; 5 channels (padded to 8), 1 channel on a 2-pixel-wide image and NULL
# v, mu take the general loops.
@pytest.mark.parametrize("H,W,C,with_vmu", [(37, 45, 3, True), (29, 33, 5, True), (23, 17, 31, True),
                                            (31, 26, 3, False), (19, 2, 1, True)])
def test_terminal_and_pd_step_match_oracle(orc, H, W, C, with_vmu):
    print(f"[case] terminal/pd H={H} W={W} C={C} v,mu={'given' if with_vmu else 'NULL'}", flush=True)
    rng = np.random.default_rng(31 + C)
    c0 = voronoi_image(H, W, C, 4, 0.05, 31)
    c = np.clip(c0 + rng.normal(scale=0.02, size=c0.shape), 0, 1).astype(np.float32)
    v = rng.normal(scale=20.0, size=(H, W, 2, C)).astype(np.float32)
    mu = rng.normal(scale=0.5, size=(H, W, 2, C)).astype(np.float32)
    if not with_vmu:
        v[:] = 0.0
        mu[:] = 0.0
    gp, op = both_params(orc, H, W, alpha=40.0)
    gK, Lt = A.abc_pd_terminal(T(c), T(c0), T(v) if with_vmu else None, T(mu) if with_vmu else None, gp)
    pK, Lt_o = orc.terminal(c, c0, v, mu, op)
    assert relinf(N(gK), pK) < FIELD_TOL
    assert abs(Lt - Lt_o) / abs(Lt_o) < ENERGY_TOL
    if not with_vmu:
        return
    vt, mt = T(v), T(mu)
    st = A.abc_pd_step(T(c), T(c0), vt, mt, gp, update_mu=True)
    vo, mo, E = orc.pd_step(c, c0, v, mu, op, update_mu=True)
    assert relinf(N(vt), vo) < FIELD_TOL and relinf(N(mt), mo) < FIELD_TOL
    for key in ("TV", "fid", "K", "L", "Ltilde", "r_abs", "r_rel"):
        assert abs(st[key] - E[key]) <= ENERGY_TOL * abs(E[key]), key


def _solve_both(orc, c0, **kw):
    H, W, _ = c0.shape
    gp, op = both_params(orc, H, W, **kw)
    ref = orc.solve(c0, op)
    return gp, op, ref


@pytest.mark.parametrize("alpha,M,P", [(3000.0, 5, 50), (20.0, 2, 10)])
def test_solve_with_replayed_controls_matches_oracle(orc, alpha, M, P):
    """32 x 32 x 3 Voronoi image, R = 2, K = 20.  The accepted steps reach
    tau ~ 1e13-1e15, which turns FP32 rounding of the control gradient into
    large control differences, so the arithmetic of the loop is compared with
    the oracle's accepted controls replayed: every forward sweep, terminal
    condition, objective, shrinkage and multiplier update of the 5 x 50
    schedule runs on the GPU, and the GPU's own gradient at every DAL step is
    compared with the oracle's."""
    print(f"[case] solve control replay alpha={alpha} M={M} P={P}", flush=True)
    c0 = voronoi_image(32, 32, 3, 4, 0.05, 1001)
    gp, op, ref = _solve_both(orc, c0, K=20, R=2, alpha=alpha, max_outer=M, max_inner=P)
    eps = T(np.full((20, 2), 57.0))
    mu = torch.zeros((32, 32, 2, 3), dtype=torch.float32, device="cuda")
    out = A.abc_solve(T(c0), gp, eps=eps, mu=mu, decisions=ref["decisions"], eps_replay=ref["eps_log"])
    assert np.array_equal(out["decisions"], ref["decisions"])
    e_c = relinf(N(out["c"]), ref["c"])
    e_v = relinf(N(out["v"]), ref["v"]) if np.max(np.abs(ref["v"])) > 0 else float(np.max(np.abs(N(out["v"]))))
    e_mu = relinf(N(mu), ref["mu"])
    st, so = out["stats"], ref["stats"]
    e_E = {key: abs(st[key] - so[key]) / abs(so[key]) for key in ("K", "TV", "fid", "L")}
    g_err = grad_errors(out["grad_log"], ref["grad_log"])
    steps = own_step_errors(out, ref)
    print(f"[solve] c {e_c:.2e} v {e_v:.2e} mu {e_mu:.2e} energies {e_E} grad max {g_err.max():.2e} "
          f"over {g_err.size} iterations; own step: formula {steps[:, 0].max():.2e}, "
          f"vs oracle {steps[:, 1].max():.2e} (bound {steps[:, 2].max():.2e})", flush=True)
    assert e_c < FIELD_TOL and e_mu < FIELD_TOL
    assert e_v < FIELD_TOL or np.max(np.abs(ref["v"])) == 0
    for key, e in e_E.items():
        assert e < ENERGY_TOL, key
    assert g_err.size > 0 and g_err.max() < FIELD_TOL
    # the GPU's own projected step Pi_E(eps - tau G), logged while the oracle's controls
    # are taken: the projection formula on its own gradient, and the oracle's step within
    # what the gradient difference allows through the 1-Lipschitz projection
    assert steps.shape[0] == np.count_nonzero(ref["decisions"])
    assert np.all(steps[:, 0] <= 1e-12 * 1100.0)
    assert np.all(steps[:, 1] <= steps[:, 2] * (1 + 1e-9) + 1e-9)


def test_solve_with_replayed_steps_follows_the_schedule(orc):
    """Replaying only the step sizes: the GPU computes its own controls from its
    FP32 gradient.  Reported, and the energy checked loosely (the step sizes
    amplify gradient rounding, see the control-replay test)."""
    c0 = voronoi_image(32, 32, 3, 4, 0.05, 1001)
    gp, op, ref = _solve_both(orc, c0, K=20, R=2, alpha=3000.0, max_outer=5, max_inner=50)
    out = A.abc_solve(T(c0), gp, decisions=ref["decisions"])
    assert np.array_equal(out["decisions"], ref["decisions"])
    e_c = relinf(N(out["c"]), ref["c"])
    e_K = abs(out["stats"]["K"] - ref["stats"]["K"]) / ref["stats"]["K"]
    print(f"[solve] step replay: c {e_c:.2e} K {e_K:.2e}", flush=True)
    assert e_K < 1e-2


ARMIJO_MARGIN = 1e-5


def test_free_running_solve_tracks_the_oracle(orc):
    """Alg. 1 running on its own on both sides (two-way projected Armijo, Sec. 3.2):
    every DAL iteration before the first one whose Armijo test the oracle passes
    or fails by less than 1e-5 of the objective (an FP32 near-tie) must take the
    oracle's decision (accepted tau and number of trials) and reach its controls
    Pi_E(eps - tau G) and objective.  40 x 36 x 3 Voronoi image, alpha = 20,
    sigma0 = 1e7, K = 12, 2 x 8 iterations; the stretch holds expanding and
    backtracking searches."""
    c0 = voronoi_image(40, 36, 3, 5, 0.05, 7)
    gp, op = both_params(orc, 40, 36, K=12, R=2, alpha=20.0, max_outer=2, max_inner=8)
    gp = gp.replace(sigma0=1e7)
    op.sigma0 = 1e7
    ref = orc.solve(c0, op)
    out = A.abc_solve(T(c0), gp)
    dec_o, tr = ref["decisions"].ravel(), ref["trace"].reshape(-1, 4)
    dec_g, ph = out["decisions"].ravel(), out["phi_log"].reshape(-1, 5)
    ran = np.nonzero(tr[:, 2] > 0)[0]
    close = [s for s in ran if tr[s, 3] < ARMIJO_MARGIN]
    stop = close[0] if close else ran[-1] + 1
    stretch = [s for s in ran if s < stop]
    # branch of each search in the stretch: expanding (tau above the previous step) or backtracking
    sigma, kinds = op.sigma0, []
    for s_ in stretch:
        kinds.append("e" if dec_o[s_] > sigma else ("b" if dec_o[s_] < sigma else "s"))
        sigma = dec_o[s_] if dec_o[s_] > 0 else sigma
    e_g = out["eps_log"].reshape(-1, 12, 2)
    e_o = ref["eps_log"].reshape(-1, 12, 2)
    e_err = [float(np.max(np.abs(e_g[s_] - e_o[s_]) / np.abs(e_o[s_]))) for s_ in stretch]
    phi_err = [abs(ph[s_, 0] - tr[s_, 0]) / abs(tr[s_, 0]) for s_ in stretch]
    print(f"[solve] free running: {len(stretch)} iterations before the first near-tie ({''.join(kinds)}); "
          f"controls {max(e_err):.2e}, objective {max(phi_err):.2e}", flush=True)
    assert len(stretch) >= 6 and "e" in kinds and "b" in kinds
    for s_ in stretch:
        assert dec_g[s_] == dec_o[s_], s_
        assert ph[s_, 2] == tr[s_, 2], s_
    assert max(e_err) < FIELD_TOL
    assert max(phi_err) < ENERGY_TOL


def test_dal_stationarity_stop_matches_oracle(orc):
    """The inner loop ends at the first DAL iteration with |Phi_new - Phi| < tol_dal
    |Phi| (convergence remark, Sec. 3.2): under control replay of the full
    schedule the GPU's own test stops at the oracle's iteration (slot 7 of 20
    here; the ratios before it are 3.5 times tol_dal or more, the stopping one
    half of it)."""
    c0 = voronoi_image(40, 36, 3, 5, 0.05, 7)
    kw = dict(K=12, R=2, alpha=20.0, max_outer=1, max_inner=20)
    gp, op = both_params(orc, 40, 36, **kw)
    gp = gp.replace(sigma0=1e7)
    op.sigma0 = 1e7
    full = orc.solve(c0, op)
    op.tol_dal = 1.5e-4
    ref = orc.solve(c0, op)
    n_ref = ref["stats"]["inner_iters"]
    assert 3 <= n_ref < 20
    out = A.abc_solve(T(c0), gp.replace(tol_dal=1.5e-4), decisions=full["decisions"], eps_replay=full["eps_log"])
    assert out["stats"]["inner_iters"] == n_ref
    assert np.array_equal(out["decisions"], ref["decisions"])
    assert relinf(N(out["c"]), ref["c"]) < FIELD_TOL


def test_alm_residual_stop_matches_oracle(orc):
    """The multiplier loop ends once r_rel = |v - grad c| / max(|grad c|, |v|) <
    tol_alm: under control replay of a 12-iteration schedule the GPU stops at
    the oracle's iteration (the 5th here: r_rel 0.0241 before it, 0.0165 at it,
    tol_alm 0.02).  rho = gamma = 1, so that the shrinkage leaves v nonzero on
    this small image."""
    c0 = voronoi_image(40, 36, 3, 5, 0.05, 7)
    kw = dict(K=12, R=2, alpha=20.0, rho=1.0, gamma=1.0, max_outer=12, max_inner=3)
    gp, op = both_params(orc, 40, 36, **kw)
    gp = gp.replace(sigma0=1e7)
    op.sigma0 = 1e7
    full = orc.solve(c0, op)
    op.tol_alm = 0.02
    ref = orc.solve(c0, op)
    assert ref["stats"]["outer_iters"] == 5 and ref["stats"]["r_rel"] < 0.02
    out = A.abc_solve(T(c0), gp.replace(tol_alm=0.02), decisions=full["decisions"], eps_replay=full["eps_log"])
    assert out["stats"]["outer_iters"] == 5 and out["status"] == A.ABC_OK
    # r_rel after each multiplier iteration: |v - grad c| is a few percent of |grad c|
    # here, so FP32 differences of 1e-6 in v and grad c show up 30-100 times larger
    r_o = np.array([orc.solve(c0, dataclasses.replace(op, max_outer=m, tol_alm=0.0))["stats"]["r_rel"]
                    for m in range(1, 6)])
    r_g = out["outer_log"][:5, 2]
    print(f"[solve] r_rel per multiplier iteration: gpu {r_g}, oracle {r_o}", flush=True)
    assert np.max(np.abs(r_g - r_o) / r_o) < 1e-3
    assert relinf(N(out["c"]), ref["c"]) < FIELD_TOL


def test_constant_image_solve_returns_input():
    c0 = np.full((24, 20, 3), 0.25, dtype=np.float32)
    out = A.abc_solve(T(c0), A.Params(K=5, R=2, max_outer=2, max_inner=3))
    assert np.all(N(out["c"]) == 0.25)
    assert out["stats"]["K"] == 0.0 and out["stats"]["r_rel"] == 0.0


def test_nonfinite_input_is_reported():
    c0 = np.full((16, 16, 3), 0.5, dtype=np.float32)
    c0[3, 4, 1] = np.nan
    with pytest.raises(A.AbcError) as e:
        A.abc_solve(T(c0), A.Params(K=3, R=2, max_outer=1, max_inner=1))
    assert e.value.code == A.ABC_ENONFINITE


def test_runs_are_deterministic():
    c0 = voronoi_image(64, 48, 3, 5, 0.05, 41)
    gp = A.Params(K=10, R=3)
    eps = T(rand_eps(10, 41))
    a = A.abc_forward_dynamics(T(c0), eps, gp)
    b = A.abc_forward_dynamics(T(c0), eps, gp)
    gK = T(np.random.default_rng(42).normal(size=c0.shape))
    ga, ea = A.abc_adjoint_dynamics(a, eps, gp, gK)
    gb, eb = A.abc_adjoint_dynamics(b, eps, gp, gK)
    assert torch.equal(a, b) and torch.equal(ga, gb) and torch.equal(ea, eb)


def test_full_size_512_sweep_matches_oracle(orc):
    """512 x 512 x 3, R = 5, K = 50 (the benchmark workload): whole trajectory
    end state, adjoint field and control gradient against the oracle."""
    from paper_2510_16154_amd.workloads import VORONOI512 as wl
    print("[case] full-size 512x512x3 R=5 K=50 sweep", flush=True)
    c0 = wl.image()
    eps = rand_eps(wl.K, 1002, lo=20.0, hi=400.0)
    gp, op = both_params(orc, wl.H, wl.W, K=wl.K, R=wl.R)
    traj = A.abc_forward_dynamics(T(c0), T(eps), gp)
    gK = np.random.default_rng(7).normal(size=c0.shape)
    g0, geps = A.abc_adjoint_dynamics(traj, T(eps), gp, T(gK))
    want = orc.forward_sweep(c0, op, eps)
    assert relinf(N(traj[-1]), want[-1]) < FIELD_TOL / 10
    p0, ge = orc.adjoint_sweep(want, op, gK, eps)
    assert relinf(N(g0), p0) < FIELD_TOL
    assert rel2(N(geps), ge) < FIELD_TOL


def test_quadratic_cost_dal_with_replayed_controls_matches_oracle(orc):
    """Alg. 1 alone on the quadratic cost J of Def. 3.2 (32 x 32 x 3, R = 2, K = 20,
    alpha = 20, 10 DAL iterations), oracle controls replayed as above."""
    c0 = voronoi_image(32, 32, 3, 4, 0.05, 1001)
    gp, op = both_params(orc, 32, 32, K=20, R=2, alpha=20.0, max_outer=1, max_inner=10)
    gp = gp.replace(cost=A.ABC_COST_QUADRATIC)
    op.cost = 1
    ref = orc.solve(c0, op)
    assert np.count_nonzero(ref["decisions"]) >= 3
    out = A.abc_solve(T(c0), gp, decisions=ref["decisions"], eps_replay=ref["eps_log"])
    assert relinf(N(out["c"]), ref["c"]) < FIELD_TOL
    assert np.all(N(out["v"]) == 0)
    for key in ("K", "TV", "fid", "Ltilde"):
        assert abs(out["stats"][key] - ref["stats"][key]) <= ENERGY_TOL * abs(ref["stats"][key]), key
    g_err = grad_errors(out["grad_log"], ref["grad_log"])
    assert g_err.size > 0 and g_err.max() < FIELD_TOL
    steps = own_step_errors(out, ref)
    assert np.all(steps[:, 0] <= 1e-12 * 1100.0)
    assert np.all(steps[:, 1] <= steps[:, 2] * (1 + 1e-9) + 1e-9)
    # free-running: J decreases monotonically over the accepted steps
    free = A.abc_solve(T(c0), gp)
    ph = free["phi_log"][0]
    taken = free["decisions"][0] > 0
    assert taken.any() and np.all(ph[taken, 1] <= ph[taken, 0])


def test_high_resolution_transfer_matches_oracle(orc):
    """Sec. 4.3: controls solved on a 32 x 32 image, applied to its 2x upsampled
    version with one forward sweep (window 2R, normalisation s/4)."""
    from paper_2510_16154_amd.transfer import transfer, transfer_params
    c_lo = voronoi_image(32, 32, 3, 4, 0.05, 1001)
    gp = A.Params(K=20, R=2, alpha=20.0, max_outer=1, max_inner=4)
    eps = T(np.full((20, 2), 57.0))
    A.abc_solve(T(c_lo), gp, eps=eps)
    c_hi = np.repeat(np.repeat(c_lo, 2, axis=0), 2, axis=1)
    got = N(transfer(T(c_hi), eps, gp, 32, 32, 2))
    ph = transfer_params(gp, 32, 32, 2)
    assert ph.R == 4 and abs(ph.inv_norm - 1.0 / 100.0) < 1e-9
    want = orc.forward_sweep(c_hi, orc.Params(K=20, R=4, s=ph.inv_norm), N(eps))[-1]
    assert relinf(got, want) < FIELD_TOL / 10


@pytest.mark.parametrize("C", [1, 3])
def test_unwindowed_paper_sum_matches_oracle(orc, C):
    """eq. MAsystem literally: a window covering the whole 16 x 16 image and s = 1/N
    (the oracle's windowed sum equals the all-pairs sum there, see the CPU pins)."""
    H = W = 16
    c0 = voronoi_image(H, W, C, 3, 0.05, 77)
    eps = rand_eps(6, 78, lo=2.0, hi=60.0)
    gp, op = both_params(orc, H, W, K=6, R=15, inv_norm=1.0 / (H * W))
    traj = A.abc_forward_dynamics(T(c0), T(eps), gp)
    want = orc.forward_sweep(c0, op, eps)
    assert relinf(N(traj), want) < FIELD_TOL / 10
    gK = np.random.default_rng(79).normal(size=c0.shape)
    g0, geps = A.abc_adjoint_dynamics(traj, T(eps), gp, T(gK))
    p0, ge = orc.adjoint_sweep(want, op, gK, eps)
    assert relinf(N(g0), p0) < FIELD_TOL and rel2(N(geps), ge) < FIELD_TOL



@pytest.mark.parametrize("H,W,C,emin", [(40, 56, 3, 20.0), (24, 20, 1, 2.0), (24, 20, 5, 2.0),
                                         (30, 33, 31, 6.0)])
def test_support_radius_mode_matches_oracle(orc, H, W, C, emin):
    """R = ABC_RADIUS_SUPPORT: the library takes the window of the kernel's support at
    the box's lower bound eps_x >= emin (eq. kernel vanishes for r >= 1), here beyond
    radius 16: the tiled runtime-radius kernels run where the tile's halo fits the LDS
    (C = 1, 3, 5 here), the direct kernels where it does not (C = 31); at emin = 2 the
    window is the whole image.  With s = 1/N that is the un-windowed sum of
    eq. MAsystem."""
    R = A.abc_support_radius(H, W, emin)
    assert R > A.ABC_MAX_RADIUS
    print(f"support radius case H={H} W={W} C={C} emin={emin} R={R}", flush=True)
    c0 = voronoi_image(H, W, C, 4, 0.05, 90 + C)
    eps = rand_eps(5, 91, lo=emin, hi=300.0)
    gp = A.Params(K=5, R=A.ABC_RADIUS_SUPPORT, inv_norm=1.0 / (H * W), eps_min=(emin, 2.0))
    op = orc.Params(K=5, R=R, s=1.0 / (H * W))
    traj = A.abc_forward_dynamics(T(c0), T(eps), gp)
    want = orc.forward_sweep(c0, op, eps)
    assert relinf(N(traj), want) < FIELD_TOL / 10
    gK = np.random.default_rng(92).normal(size=c0.shape)
    g0, geps = A.abc_adjoint_dynamics(traj, T(eps), gp, T(gK))
    p0, ge = orc.adjoint_sweep(want, op, gK, eps)
    assert relinf(N(g0), p0) < FIELD_TOL and rel2(N(geps), ge) < FIELD_TOL
    # the same radius given explicitly runs the same kernels: the same bits
    traj2 = A.abc_forward_dynamics(T(c0), T(eps), gp.replace(R=R))
    assert torch.equal(traj, traj2)


@pytest.mark.parametrize("H,W,C,R", [(61, 70, 3, 40), (45, 37, 3, 60), (100, 90, 1, 99), (40, 44, 8, 20),
                                      (33, 35, 16, 17), (9, 130, 5, 129)])
def test_direct_kernels_match_oracle(orc, H, W, C, R):
    """Radii whose tile halo does not fit the LDS run the direct kernels (8 x 8 pixel
    blocks, the window's rows dealt out to the waves): windows cut by the image and
    windows covering it (no per-pair window test), blocks past the image's edge, 1 to 16
    channels.  At 1 and 3 channels two tiles whose halos do not fit give the same bits:
    the direct kernels do not depend on the tile asked for."""
    print(f"[case] direct H={H} W={W} C={C} R={R}", flush=True)
    c0 = voronoi_image(H, W, C, 4, 0.05, 70 + C)
    eps = rand_eps(3, 71, lo=2.0, hi=60.0)
    gp, op = both_params(orc, H, W, K=3, R=R)
    traj = A.abc_forward_dynamics(T(c0), T(eps), gp)
    want = orc.forward_sweep(c0, op, eps)
    assert relinf(N(traj), want) < FIELD_TOL / 10
    gK = np.random.default_rng(72).normal(size=c0.shape)
    g0, geps = A.abc_adjoint_dynamics(traj, T(eps), gp, T(gK))
    p0, ge = orc.adjoint_sweep(want, op, gK, eps)
    print(f"  errors: c^K {relinf(N(traj), want):.2e} p^0 {relinf(N(g0), p0):.2e} dl/deps {rel2(N(geps), ge):.2e}",
          flush=True)
    assert relinf(N(g0), p0) < FIELD_TOL and rel2(N(geps), ge) < FIELD_TOL
    if C > 3:
        return
    runs = []
    for tx, ty in ((32, 16), (64, 8)):  # both halos too large for the LDS at these radii
        q = gp.replace(tile_x=tx, tile_y=ty, adj_tile_x=tx, adj_tile_y=ty)
        tr = A.abc_forward_dynamics(T(c0), T(eps), q)
        runs.append((tr,) + A.abc_adjoint_dynamics(tr, T(eps), q, T(gK)))
    assert all(torch.equal(a, b) for a, b in zip(*runs))


def test_support_radius_solve_matches_oracle(orc):
    """A short solve with R = ABC_RADIUS_SUPPORT on a 20 x 20 image with the paper's box
    (eps_x >= 2: the window is the whole image, s = 1/N by the default rule) against the
    oracle at that radius, controls replayed."""
    H = W = 20
    c0 = voronoi_image(H, W, 3, 4, 0.05, 93)
    gp, op = both_params(orc, H, W, K=8, R=A.ABC_RADIUS_SUPPORT, alpha=50.0, max_outer=2, max_inner=3)
    op.R = A.abc_support_radius(H, W, gp.eps_min[0])
    assert op.R == 19
    ref = orc.solve(c0, op)
    out = A.abc_solve(T(c0), gp, decisions=ref["decisions"], eps_replay=ref["eps_log"])
    assert relinf(N(out["c"]), ref["c"]) < FIELD_TOL
    assert abs(out["stats"]["K"] - ref["stats"]["K"]) <= 1e-5 * abs(ref["stats"]["K"])


def test_gap_stop_matches_oracle(orc):
    """The Lagrangian-gap stop (Sec. 4.1) ends the GPU solve at the same multiplier
    iteration as the oracle's when the controls are replayed."""
    c0 = voronoi_image(32, 32, 3, 4, 0.05, 1001)
    gp, op = both_params(orc, 32, 32, K=20, R=2, alpha=3000.0, max_outer=8, max_inner=4, tol_gap=0.25)
    ref = orc.solve(c0, op)
    assert 1 < ref["stats"]["outer_iters"] < 8
    out = A.abc_solve(T(c0), gp, decisions=ref["decisions"], eps_replay=ref["eps_log"])
    assert out["stats"]["outer_iters"] == ref["stats"]["outer_iters"]
    assert relinf(N(out["c"]), ref["c"]) < FIELD_TOL


@pytest.mark.parametrize("K,ckpt", [(1, 0), (3, 0), (5, 2)])
def test_adjoint_in_place_equals_separate_output(K, ckpt):
    """dl/dc^0 may overwrite dl/dc^K (g0 == gK): same bits as a separate output,
    for a single step, several steps and a checkpointed trajectory."""
    H, W, C, R = 37, 29, 3, 3
    c0 = voronoi_image(H, W, C, 3, 0.05, 31)
    eps = rand_eps(K, 31)
    gp = A.Params(K=K, R=R, ckpt_every=ckpt)
    traj = A.abc_forward_dynamics(T(c0), T(eps), gp)
    gK = T(np.random.default_rng(32).normal(size=(H, W, C)))
    g_sep, ge_sep = A.abc_adjoint_dynamics(traj, T(eps), gp, gK.clone())
    g_in = gK.clone()
    g_out, ge_in = A.abc_adjoint_dynamics(traj, T(eps), gp, g_in, g0=g_in)
    torch.cuda.synchronize()
    assert g_out.data_ptr() == g_in.data_ptr()
    assert torch.equal(g_in, g_sep) and torch.equal(ge_in, ge_sep)
