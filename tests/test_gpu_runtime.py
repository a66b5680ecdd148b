"""Runtime pieces around the kernels: captured sweep graphs (replayed many
times with eager work in between must equal direct launches bit for bit) and
the tile autotuner with its JSON cache."""
import json
import os

import numpy as np
import pytest

import paper_2510_16154_amd as A
from paper_2510_16154_amd.synth import voronoi_image

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


@pytest.mark.parametrize("cost", [A.ABC_COST_TV, A.ABC_COST_QUADRATIC])
def test_graph_replay_equals_direct_launches(cost):
    c0 = voronoi_image(48, 40, 3, 4, 0.05, 3)
    base = A.Params(K=12, R=3, alpha=20.0, max_outer=2, max_inner=6, cost=cost)
    outs = []
    for flags in (0, A.ABC_FLAG_NO_GRAPHS, 0):
        e = T(np.full((12, 2), 57.0))
        o = A.abc_solve(T(c0), base.replace(flags=flags), eps=e)
        outs.append((o["c"], e, o["decisions"], o["stats"]))
    for o in outs[1:]:
        assert torch.equal(o[0], outs[0][0]) and torch.equal(o[1], outs[0][1])
        assert np.array_equal(o[2], outs[0][2])
        assert o[3]["K"] == outs[0][3]["K"] and o[3]["ls_evals"] == outs[0][3]["ls_evals"]


def test_batched_graph_replay_equals_direct_launches():
    imgs = [T(voronoi_image(h, w, 3, 4, 0.05, 40 + h)) for h, w in [(40, 30), (26, 61), (50, 50)]]
    base = A.Params(K=8, R=2, alpha=20.0, max_outer=2, max_inner=4)
    a, sa, _ = A.abc_solve_batched(imgs, base)
    b, sb, _ = A.abc_solve_batched(imgs, base.replace(flags=A.ABC_FLAG_NO_GRAPHS))
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert [s["ls_evals"] for s in sa] == [s["ls_evals"] for s in sb]


def test_autotuner_picks_admissible_tiles_and_caches(tmp_path):
    c0 = T(voronoi_image(256, 192, 3, 6, 0.05, 5))
    p = A.Params(K=6, R=5)
    cache = str(tmp_path / "tiles.json")
    tuned, us = A.abc_autotune(c0, p, cache_path=cache)
    print(f"[tune] fwd {tuned.tile_x}x{tuned.tile_y} {us[0]:.1f} us, adj {tuned.adj_tile_x}x{tuned.adj_tile_y} "
          f"{us[1]:.1f} us", flush=True)
    assert us[0] > 0 and us[1] > 0
    # two pixels per thread at C = 3, R = 5: 64 to 256 threads hold 128 to 512 pixels
    assert tuned.tile_x * tuned.tile_y in (128, 256, 512) and tuned.adj_tile_x * tuned.adj_tile_y in (128, 256, 512)
    assert tuned.tile_y % 2 == 0 and tuned.adj_tile_y % 2 == 0
    data = json.load(open(cache))
    assert len(data) == 1 and list(data.values())[0]["fwd"] == [tuned.tile_x, tuned.tile_y]
    again, us2 = A.abc_autotune(c0, p, cache_path=cache)
    assert us2 == (0.0, 0.0)
    assert (again.tile_x, again.tile_y, again.adj_tile_x, again.adj_tile_y) == \
        (tuned.tile_x, tuned.tile_y, tuned.adj_tile_x, tuned.adj_tile_y)
    eps = T(np.random.default_rng(1).uniform(20, 300, size=(6, 2)))
    ref = A.abc_forward_dynamics(c0, eps, p)
    got = A.abc_forward_dynamics(c0, eps, tuned)
    assert torch.equal(ref, got)
    gK = T(np.random.default_rng(2).normal(size=(256, 192, 3)))
    g_ref, _ = A.abc_adjoint_dynamics(ref, eps, p, gK)
    g_got, _ = A.abc_adjoint_dynamics(got, eps, tuned, gK)
    assert torch.equal(g_ref, g_got)


def test_autotuner_with_wide_channels():
    c0 = T(voronoi_image(96, 130, 31, 6, 0.05, 6, spectra=True))
    p = A.Params(K=4, R=2)
    tuned, us = A.abc_autotune(c0, p)
    print(f"[tune C=31] fwd {tuned.tile_x}x{tuned.tile_y} {us[0]:.1f} us, adj {tuned.adj_tile_x}x{tuned.adj_tile_y} "
          f"{us[1]:.1f} us", flush=True)
    assert us[0] > 0 and us[1] > 0
    eps = T(np.random.default_rng(3).uniform(20, 300, size=(4, 2)))
    ref = A.abc_forward_dynamics(c0, eps, p)
    got = A.abc_forward_dynamics(c0, eps, tuned)
    assert torch.equal(ref, got)
    gK = T(np.random.default_rng(4).normal(size=(96, 130, 31)))
    g_ref, e_ref = A.abc_adjoint_dynamics(ref, eps, p, gK)
    g_got, e_got = A.abc_adjoint_dynamics(got, eps, tuned, gK)
    assert torch.equal(g_ref, g_got)
