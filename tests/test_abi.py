"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/abc.h, and validates arguments before touching the GPU."""
import ctypes as ct
import json
import os
import subprocess

import pytest

import paper_2510_16154_amd as A
from paper_2510_16154_amd import binding as B

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_library_exports_every_declared_symbol():
    names = B.exported_names()
    assert len(names) >= 10
    L = B.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert f" T {n}" in out, n


def test_library_leaves_no_symbol_of_its_own_unresolved():
    """A helper declared for the other translation units but defined inside an
    anonymous namespace links into a shared library as an undefined symbol and
    fails only when first called; every abc:: symbol must be defined."""
    out = subprocess.run(["nm", "-DC", "--undefined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    assert [ln for ln in out.splitlines() if "abc::" in ln or " abc_" in ln] == []


def test_default_params_carry_the_papers_values():
    g = json.load(open(os.path.join(GOLD, "paper_parameters.json")))
    p = A.abc_default_params()
    assert p.dt == g["dt"]["value"]
    assert p.eps_min == (g["eps_box"]["value"][0],) * 2 and p.eps_max == (g["eps_box"]["value"][1],) * 2
    assert p.eps_init == g["eps_init"]["value"]
    assert (p.sigma0, p.armijo_b, p.armijo_c) == (g["sigma0"]["value"], g["armijo_b"]["value"],
                                                 g["armijo_c"]["value"])
    assert p.rho == pytest.approx(g["rho"]["value"], rel=1e-7)
    assert p.gamma == pytest.approx(g["gamma"]["value"], rel=1e-7)
    assert A.abc_version() >= 100


def test_workspace_sizes_and_slots():
    p = A.Params(K=50, R=5)
    ws = A.abc_workspace_bytes(A.ABC_WS_SOLVE, 512, 512, 3, p)
    field = 512 * 512 * 3 * 4
    assert ws >= 3 * 51 * field  # three trajectories
    assert A.abc_workspace_bytes(A.ABC_WS_FORWARD, 512, 512, 3, p) == 0
    assert A.abc_workspace_bytes(A.ABC_WS_FORWARD, 512, 512, 3, p.replace(ckpt_every=10)) >= 2 * field
    assert A.abc_traj_slots(p) == 51
    assert A.abc_traj_slots(p.replace(K=100, ckpt_every=10)) == 11
    assert A.abc_traj_slots(p.replace(K=95, ckpt_every=10)) == 11


@pytest.mark.parametrize("bad", [dict(K=0), dict(R=-2), dict(R=32768), dict(dt=0.0), dict(rho=0.0),
                                 dict(eps_min=(5.0, 2.0), eps_max=(4.0, 1100.0)), dict(max_ls=0),
                                 dict(armijo_b=1.0), dict(ckpt_every=-1), dict(tile_x=7, tile_y=3)])
def test_invalid_parameters_are_rejected_on_the_host(bad):
    with pytest.raises(A.AbcError) as e:
        A.abc_workspace_bytes(A.ABC_WS_SOLVE, 32, 32, 3, A.Params().replace(**bad))
    assert e.value.code == A.ABC_EINVAL


@pytest.mark.parametrize("C,R,tile,ok", [
    (3, 5, (32, 16), True), (3, 5, (32, 8), True), (3, 5, (16, 8), True),
    (3, 5, (64, 1), False),  # two pixels per thread: the height must be even
    (3, 5, (16, 4), False),  # 32 threads: not a whole wave
    (3, 5, (64, 16), False),  # 512 threads
    (2, 9, (32, 16), True), (6, 3, (32, 8), True), (6, 3, (64, 1), True),  # 6 channels: one pixel per thread
    (31, 2, (16, 16), True), (31, 2, (32, 16), False),  # 4 lanes per pixel: 1024 and 2048 threads
])
def test_tile_rule_on_the_host(C, R, tile, ok):
    p = A.Params(K=4, R=R, tile_x=tile[0], tile_y=tile[1])
    if ok:
        assert A.abc_workspace_bytes(A.ABC_WS_SOLVE, 40, 40, C, p) > 0
    else:
        with pytest.raises(A.AbcError) as e:
            A.abc_workspace_bytes(A.ABC_WS_SOLVE, 40, 40, C, p)
        assert e.value.code == A.ABC_EINVAL and "tile" in str(e.value)


@pytest.mark.parametrize("shape", [(0, 4, 3), (4, 0, 3), (4, 4, 0), (4, 4, 65), (70000, 70000, 1), (1, 2**31 - 1, 2)])
def test_invalid_shapes_are_rejected_before_any_launch(shape):
    L = B.lib()
    p = A.Params().to_c()
    H, W, C = shape
    dummy = ct.c_void_p(16)  # never dereferenced: validation fails first
    rc = L.abc_forward_dynamics(dummy, H, W, C, dummy, ct.byref(p), dummy, None, 0, None)
    assert rc == A.ABC_EINVAL
    assert "must" in L.abc_last_error().decode()
    rc = L.abc_solve(dummy, H, W, C, ct.byref(p), None, None, None, dummy, dummy, 1 << 30, None, None, None)
    assert rc == A.ABC_EINVAL


def test_null_pointers_are_rejected():
    L = B.lib()
    p = A.Params().to_c()
    assert L.abc_forward_dynamics(None, 8, 8, 3, None, ct.byref(p), None, None, 0, None) == A.ABC_EINVAL
    assert L.abc_solve(None, 8, 8, 3, ct.byref(p), None, None, None, None, None, 0, None, None,
                       None) == A.ABC_EINVAL
    assert L.abc_pd_step(None, None, 8, 8, 3, ct.byref(p), None, None, 1, None, None, 0, None) == A.ABC_EINVAL


def test_batched_entry_points_reject_an_empty_batch_and_bad_images():
    L = B.lib()
    p = A.Params(K=4, R=2).to_c()
    nb = ct.c_size_t(0)
    H, W = (ct.c_int32 * 1)(8), (ct.c_int32 * 1)(8)
    assert L.abc_workspace_bytes_batched(H, W, 0, 3, ct.byref(p), ct.byref(nb)) == A.ABC_EINVAL
    assert L.abc_solve_batched(None, 0, 3, ct.byref(p), None, 0, None, None, None, None) == A.ABC_EINVAL
    assert "n >= 1" in L.abc_last_error().decode()
    for shapes in ([(32, 32), (0, 8)], [(32, 32), (8, -1)], [(70000, 70000)]):
        with pytest.raises(A.AbcError) as e:
            A.abc_workspace_bytes_batched(shapes, 3, A.Params(K=4, R=2))
        assert e.value.code == A.ABC_EINVAL


def test_support_radius_on_the_host():
    # R* = min(ceil(sqrt(2 / eps_x_min) max(H, W)), max(H, W) - 1)
    assert A.abc_support_radius(512, 512, 1100.0) == 22  # 21.83 rounded up
    assert A.abc_support_radius(512, 512, 2.0) == 511  # the whole image
    assert A.abc_support_radius(40, 56, 20.0) == 18
    assert A.abc_support_radius(56, 40, 20.0) == 18  # square window: the longer side
    assert A.abc_support_radius(7, 3, 0.0) == 6
    assert A.abc_support_radius(1, 1, 57.0) == 0
    for bad in [(0, 8, 2.0), (8, 0, 2.0), (8, 8, -1.0), (8, 8, float("nan"))]:
        with pytest.raises(A.AbcError) as e:
            A.abc_support_radius(*bad)
        assert e.value.code == A.ABC_EINVAL
    # the support mode sizes workspaces as the radius it resolves to; past radius 16 a tile that leaves fewer than
    # 8 waves per CU runs the direct kernels
    p = A.Params(K=4, R=A.ABC_RADIUS_SUPPORT, eps_min=(20.0, 2.0))
    for kind in (A.ABC_WS_SOLVE, A.ABC_WS_ADJOINT):
        assert A.abc_workspace_bytes(kind, 40, 56, 3, p) == A.abc_workspace_bytes(kind, 40, 56, 3, p.replace(R=18))
    assert A.abc_workspace_bytes(A.ABC_WS_SOLVE, 40, 40, 3, A.Params(K=4, R=200, tile_x=32, tile_y=16)) > 0
    # the batched solve keeps to the tiled kernels
    for R in (A.ABC_RADIUS_SUPPORT, 17):
        with pytest.raises(A.AbcError) as e:
            A.abc_workspace_bytes_batched([(32, 32), (40, 48)], 3, A.Params(K=4, R=R))
        assert e.value.code == A.ABC_EINVAL


def test_segment_entry_points_check_arguments_on_the_host():
    L = B.lib()
    assert B.abc_segment_workspace_bytes(64, 48, 3) >= 64 * 48 * (4 + 1 + 4 * 4 + 8 + 8 * (2 + 2 * 3))
    n = ct.c_size_t()
    assert L.abc_segment_workspace_bytes(0, 8, 3, ct.byref(n)) == A.ABC_EINVAL
    assert L.abc_segment_workspace_bytes(8, 8, 65, ct.byref(n)) == A.ABC_EINVAL
    st = B.AbcSegStats()
    dummy = ct.c_void_p(16)
    assert L.abc_segment(None, dummy, 8, 8, 3, ct.c_float(0.02), None, None, ct.byref(st), dummy, 1 << 30,
                         None) == A.ABC_EINVAL
    assert L.abc_segment(dummy, dummy, 8, 8, 3, ct.c_float(float("nan")), None, None, ct.byref(st), dummy,
                         1 << 30, None) == A.ABC_EINVAL
    need = B.abc_segment_workspace_bytes(8, 8, 3)
    assert L.abc_segment(dummy, dummy, 8, 8, 3, ct.c_float(0.02), None, None, ct.byref(st), dummy, need - 1,
                         None) == A.ABC_EINVAL


def test_params_struct_is_converted_once_and_follows_assignments():
    p = A.Params(K=50, R=5)
    c = p.to_c()
    assert p.to_c() is c and (c.K, c.R) == (50, 5)
    p.K = 9
    assert p.to_c() is not c and p.to_c().K == 9 and c.K == 50
    p.eps_min = [3, 4]
    assert p.eps_min == (3.0, 4.0) and tuple(p.to_c().eps_min) == (3.0, 4.0)
    q = p.replace(R=2)
    assert q.to_c().R == 2 and p.to_c().R == 5
    assert p == A.Params(K=9, R=5, eps_min=(3.0, 4.0))
