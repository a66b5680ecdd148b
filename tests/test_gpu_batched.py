"""Batched form: many images of uneven sizes solved in lockstep rounds with one
multi-image launch per Euler step.  Same arithmetic per image as abc_solve,
so with the same tile shape every image's result matches its own solve bit for
bit."""
import numpy as np
import pytest

import paper_2510_16154_amd as A
from paper_2510_16154_amd.synth import voronoi_image

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


SHAPES = [(40, 57), (33, 33), (71, 24), (16, 90), (64, 48)]


@pytest.mark.parametrize("cost", [A.ABC_COST_TV, A.ABC_COST_QUADRATIC])
def test_batched_equals_individual_solves(cost):
    print(f"[case] batched vs individual, cost={cost}", flush=True)
    imgs = [voronoi_image(h, w, 3, 4, 0.05, 500 + i) for i, (h, w) in enumerate(SHAPES)]
    gp = A.Params(K=10, R=2, alpha=20.0, max_outer=2, max_inner=4, tile_x=32, tile_y=8, cost=cost)
    eps_b = [T(np.full((10, 2), 57.0)) for _ in imgs]
    mu_b = [torch.zeros((h, w, 2, 3), dtype=torch.float32, device="cuda") for h, w in SHAPES]
    outs, stats, fin = A.abc_solve_batched([T(x) for x in imgs], gp, eps=eps_b, mu=mu_b)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(fin)) and np.all(fin > 0)
    for i, x in enumerate(imgs):
        e = T(np.full((10, 2), 57.0))
        m = torch.zeros_like(mu_b[i])
        ref = A.abc_solve(T(x), gp, eps=e, mu=m)
        assert torch.equal(outs[i], ref["c"]), i
        assert torch.equal(eps_b[i], e), i
        assert torch.equal(mu_b[i], m), i
        for key in ("K", "TV", "fid", "L", "Ltilde", "r_rel", "inner_iters", "ls_evals", "outer_iters"):
            assert stats[i][key] == ref["stats"][key], (i, key)


def test_batched_handles_one_image_and_early_inner_exit():
    c0 = np.full((20, 30, 3), 0.5, dtype=np.float32)  # constant: G = 0 ends every inner loop at once
    other = voronoi_image(25, 35, 3, 4, 0.05, 9)
    gp = A.Params(K=5, R=2, alpha=20.0, max_outer=2, max_inner=3)
    outs, stats, _ = A.abc_solve_batched([T(c0), T(other)], gp)
    assert torch.all(outs[0] == 0.5)
    assert stats[0]["ls_evals"] == 0 and stats[1]["ls_evals"] > 0


def test_batched_wide_channels_equal_individual_solves_and_graphs():
    """31 channels at radius 2 run on the lanes-per-pixel kernels, batched and single."""
    print("[case] batched vs individual, C=31", flush=True)
    shapes = [(40, 57), (33, 33), (16, 90)]
    imgs = [voronoi_image(h, w, 31, 4, 0.05, 700 + i, spectra=True) for i, (h, w) in enumerate(shapes)]
    gp = A.Params(K=6, R=2, alpha=20.0, max_outer=2, max_inner=3, tile_x=16, tile_y=16)
    outs, stats, _ = A.abc_solve_batched([T(x) for x in imgs], gp)
    torch.cuda.synchronize()
    for i, x in enumerate(imgs):
        ref = A.abc_solve(T(x), gp)
        assert torch.equal(outs[i], ref["c"]), i
        for key in ("K", "L", "inner_iters", "ls_evals", "outer_iters"):
            assert stats[i][key] == ref["stats"][key], (i, key)
    direct, _, _ = A.abc_solve_batched([T(x) for x in imgs], gp.replace(flags=A.ABC_FLAG_NO_GRAPHS))
    for x, y in zip(outs, direct):
        assert torch.equal(x, y)


@pytest.mark.parametrize("R,C,tile", [(7, 3, (32, 16)), (4, 2, (16, 16)), (3, 6, (32, 8)), (5, 4, (32, 16)),
                                      (1, 1, (64, 4)), (3, 1, (16, 8))])
def test_batched_default_and_runtime_radius_tiles_equal_individual_solves(R, C, tile):
    """Two pixels per thread with a compile-time (R <= 5, the transposed step's window
    split over two thread layers) and a runtime radius (R = 7), and one pixel per
    thread for 6 channels, each in the batched launch and alone; 1 to 6 channels."""
    print(f"[case] batched vs individual, R={R} C={C} tile={tile}", flush=True)
    shapes = [(40, 57), (33, 33), (71, 24)]
    imgs = [voronoi_image(h, w, C, 4, 0.05, 800 + i) for i, (h, w) in enumerate(shapes)]
    gp = A.Params(K=5, R=R, alpha=20.0, max_outer=2, max_inner=2, tile_x=tile[0], tile_y=tile[1])
    outs, stats, _ = A.abc_solve_batched([T(x) for x in imgs], gp)
    torch.cuda.synchronize()
    for i, x in enumerate(imgs):
        ref = A.abc_solve(T(x), gp)
        assert torch.equal(outs[i], ref["c"]), i
        for key in ("K", "L", "inner_iters", "ls_evals", "outer_iters"):
            assert stats[i][key] == ref["stats"][key], (i, key)


@pytest.mark.parametrize("C,cost", [(3, A.ABC_COST_TV), (3, A.ABC_COST_QUADRATIC), (31, A.ABC_COST_TV)])
def test_batched_images_match_the_oracle_under_control_replay(orc, C, cost):
    """Every image of an uneven batch against its own FP64 oracle solve (Alg. 2
    around Alg. 1, or Alg. 1 alone on the quadratic cost), with each image's
    accepted controls replayed as in the single-image parity tests: final field
    1e-4, energies 1e-5, the control gradient of every DAL iteration 1e-4
    (relative l2), and the GPU's own projected step from its gradient."""
    from tests.solve_checks import grad_errors, own_step_errors
    print(f"[case] batched vs oracle, C={C} cost={cost}", flush=True)
    shapes = [(40, 57), (33, 33), (16, 90), (27, 44)] if C == 3 else [(24, 30), (17, 33), (30, 16)]
    K = 10 if C == 3 else 5
    # 31 noisy bands put every pair of pixels outside the kernel's support at sigma = 0.05
    # (G = 0 from the start), so the spectral images carry less noise
    noise = 0.05 if C == 3 else 0.01
    imgs = [voronoi_image(h, w, C, 4, noise, 900 + i, spectra=C > 3) for i, (h, w) in enumerate(shapes)]
    gp = A.Params(K=K, R=2, alpha=20.0, max_outer=2, max_inner=4, cost=cost)
    refs = []
    for x in imgs:
        op = orc.Params(K=K, R=2, alpha=20.0, max_outer=2, max_inner=4, cost=1 if cost else 0)
        refs.append(orc.solve(x, op))
    outs, stats, _, logs = A.abc_solve_batched(
        [T(x) for x in imgs], gp, eps=[T(np.full((K, 2), 57.0)) for _ in imgs],
        decisions=[r["decisions"] for r in refs], eps_replay=[r["eps_log"] for r in refs], want_logs=True)
    torch.cuda.synchronize()
    for i, (x, ref) in enumerate(zip(imgs, refs)):
        assert np.count_nonzero(ref["decisions"]) >= 2, i
        c = outs[i].cpu().numpy().astype(np.float64)
        e_c = np.max(np.abs(c - ref["c"])) / np.max(np.abs(ref["c"]))
        g_err = grad_errors(logs[i]["grad_log"], ref["grad_log"])
        steps = own_step_errors(logs[i], ref)
        print(f"[batched] image {i} {shapes[i]}: c {e_c:.2e} grad {g_err.max():.2e} "
              f"own step {steps[:, 1].max():.2e} (bound {steps[:, 2].max():.2e})", flush=True)
        assert np.array_equal(logs[i]["decisions"], ref["decisions"]), i
        assert e_c < 1e-4, i
        keys = ("K", "TV", "fid", "Ltilde") if cost else ("K", "TV", "fid", "L", "Ltilde")
        for key in keys:
            assert abs(stats[i][key] - ref["stats"][key]) <= 1e-5 * abs(ref["stats"][key]), (i, key)
        assert g_err.size > 0 and g_err.max() < 1e-4, i
        assert np.all(steps[:, 0] <= 1e-12 * 1100.0), i
        assert np.all(steps[:, 1] <= steps[:, 2] * (1 + 1e-9) + 1e-9), i


@pytest.mark.parametrize("C,R,spectra", [(3, 5, False), (31, 2, True), (3, 7, False)])
def test_persistent_sweeps_equal_one_workgroup_per_tile(C, R, spectra):
    """ABC_FLAG_PERSISTENT: each Euler step as a grid of as many workgroups as the
    GPU holds, taking the tiles of all images from per-step counters, gives the
    same bits as one workgroup per tile (one-lane, lanes-per-pixel and
    runtime-radius kernels)."""
    print(f"[case] persistent batched C={C} R={R}", flush=True)
    shapes = [(96, 130), (33, 57), (150, 41), (64, 64)] if C == 3 else [(40, 57), (33, 70)]
    imgs = [T(voronoi_image(h, w, C, 4, 0.05 if C == 3 else 0.01, 600 + i, spectra=spectra))
            for i, (h, w) in enumerate(shapes)]
    gp = A.Params(K=6, R=R, alpha=20.0, max_outer=2, max_inner=3)
    a, sa, _ = A.abc_solve_batched(imgs, gp)
    b, sb, _ = A.abc_solve_batched(imgs, gp.replace(flags=A.ABC_FLAG_PERSISTENT))
    torch.cuda.synchronize()
    for i in range(len(imgs)):
        assert torch.equal(a[i], b[i]), i
        for key in ("K", "L", "inner_iters", "ls_evals", "outer_iters"):
            assert sa[i][key] == sb[i][key], (i, key)


def test_autotuned_batch_equals_a_solve_with_the_tuned_tiles():
    """ABC_FLAG_AUTOTUNE: the batched solve times the tile candidates on its largest
    image and uses the fastest; its results equal the default tiles' bit for bit
    (each pixel sums its window in a fixed order, so only the time depends on
    the tile), and the workspace query leaves room for any candidate."""
    shapes = [(96, 130), (33, 57), (150, 41)]
    imgs = [T(voronoi_image(h, w, 3, 4, 0.05, 650 + i)) for i, (h, w) in enumerate(shapes)]
    gp = A.Params(K=5, R=5, alpha=20.0, max_outer=1, max_inner=2)
    tuned_p = gp.replace(flags=A.ABC_FLAG_AUTOTUNE)
    assert A.abc_workspace_bytes_batched(shapes, 3, tuned_p) >= A.abc_workspace_bytes_batched(shapes, 3, gp)
    a, _, _ = A.abc_solve_batched(imgs, tuned_p)
    again, _, _ = A.abc_solve_batched(imgs, tuned_p)  # the tuned tiles come from the process cache now
    b, _, _ = A.abc_solve_batched(imgs, gp)
    torch.cuda.synchronize()
    for i in range(len(imgs)):
        assert torch.equal(a[i], b[i]) and torch.equal(again[i], b[i]), i


def test_full_batch_in_the_bench_configuration_equals_sampled_solves():
    """The 64-image batch at its full size (sides 128-1024, 20 Mpx, R = 5, K = 50,
    5 x 10 schedule) in the configuration the batched line times (persistent
    sweeps, tuned tiles): the smallest, the largest and a middle image equal their
    own abc_solve bit for bit, with the same iteration counts."""
    from paper_2510_16154_amd.workloads import BATCH64 as wb
    print("[case] full 64-image batch, persistent and tuned", flush=True)
    host = wb.images()
    imgs = [T(x) for x in host]
    gp = wb.params(flags=A.ABC_FLAG_PERSISTENT | A.ABC_FLAG_AUTOTUNE)
    outs, stats, fin = A.abc_solve_batched(imgs, gp)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(fin)) and np.all(fin > 0)
    sizes = [x.shape[0] * x.shape[1] for x in host]
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), len(host) // 2})
    for i in picks:
        print(f"[case] image {i} of the batch, {host[i].shape}", flush=True)
        ref = A.abc_solve(imgs[i], wb.params())
        assert torch.equal(outs[i], ref["c"]), i
        for key in ("K", "L", "r_rel", "inner_iters", "ls_evals", "outer_iters"):
            assert stats[i][key] == ref["stats"][key], (i, key)
