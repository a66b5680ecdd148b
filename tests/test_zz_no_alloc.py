"""The allocation-free adjoint entry point (abc_adjoint_dynamics_noalloc, for
callers that cannot allocate device memory) against abc_adjoint_dynamics on
the same inputs: bit for bit, on two calls in a row whose second input is
smaller (the shared scratch keeps the first call's contents), and sizes
beyond its scratch rejected before any launch."""
import numpy as np
import pytest

import paper_2510_16154_amd as A
from paper_2510_16154_amd.synth import voronoi_image

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def _case(H, W, C, K, R, seed, ckpt=0):
    c0 = voronoi_image(H, W, C, 5, 0.05, seed)
    eps = T(np.random.default_rng(seed).uniform(2.0, 300.0, size=(K, 2)))
    gp = A.Params(K=K, R=R, ckpt_every=ckpt)
    traj = A.abc_forward_dynamics(T(c0), eps, gp)
    gK = T(np.random.default_rng(seed + 1).normal(size=(H, W, C)))
    return gp, traj, eps, gK


@pytest.mark.parametrize("ckpt", [0, 4])
def test_noalloc_adjoint_equals_the_workspace_entry_point_on_two_calls(ckpt):
    # the first call fills the scratch with a larger problem, the second one reuses it
    for (H, W, C, K, R, seed) in [(300, 260, 3, 12, 5, 1), (97, 131, 3, 9, 3, 2)]:
        print(f"[case] noalloc adjoint H={H} W={W} C={C} K={K} R={R} ckpt={ckpt}", flush=True)
        gp, traj, eps, gK = _case(H, W, C, K, R, seed, ckpt)
        g_ref, e_ref = A.abc_adjoint_dynamics(traj, eps, gp, gK)
        g0 = torch.full_like(gK, float("nan"))
        geps = torch.full((K, 2), float("nan"), dtype=torch.float32, device="cuda")
        A.abc_adjoint_dynamics_noalloc(traj, eps, gp, gK, g0, geps)
        torch.cuda.synchronize()
        assert torch.equal(g0, g_ref) and torch.equal(geps, e_ref)


def test_noalloc_adjoint_wide_channels_and_zero_radius():
    for (H, W, C, K, R, seed) in [(70, 66, 31, 4, 2, 3), (40, 30, 3, 3, 0, 4)]:
        print(f"[case] noalloc adjoint H={H} W={W} C={C} K={K} R={R}", flush=True)
        gp, traj, eps, gK = _case(H, W, C, K, R, seed)
        g_ref, e_ref = A.abc_adjoint_dynamics(traj, eps, gp, gK)
        g0 = torch.full_like(gK, float("nan"))
        geps = torch.full((K, 2), float("nan"), dtype=torch.float32, device="cuda")
        A.abc_adjoint_dynamics_noalloc(traj, eps, gp, gK, g0, geps)
        torch.cuda.synchronize()
        assert torch.equal(g0, g_ref) and torch.equal(geps, e_ref)


def test_noalloc_adjoint_rejects_shapes_beyond_its_scratch():
    """1200 x 1200 x 3 at K = 50 needs more than the 32 MiB scratch: the host check
    returns ABC_EINVAL before anything is launched (the pointers are never used)."""
    gp = A.Params(K=50, R=5)
    assert A.abc_workspace_bytes(A.ABC_WS_ADJOINT, 1200, 1200, 3, gp) > (32 << 20)
    x = torch.zeros(1, dtype=torch.float32, device="cuda")
    p = gp.to_c()
    L = A.binding.lib()
    rc = L.abc_adjoint_dynamics_noalloc(x.data_ptr(), 1200, 1200, 3, x.data_ptr(), A.binding.ct.byref(p),
                                        x.data_ptr(), x.data_ptr(), x.data_ptr(), None)
    assert rc == A.ABC_EINVAL
    assert b"scratch" in L.abc_last_error()
