"""Pins of the FP64 warm-start network oracle: the bfloat16 rounding rule,
convolution against scipy's correlation, the written-out backward pass
against central finite differences, and the unit-ball head."""
import numpy as np
import pytest

from oracle import wsnet as O
from paper_2510_16154_amd.synth import wsnet_init


def test_bf16_rounding_follows_the_format():
    one = 1.0
    u = 2.0 ** -7  # bfloat16 spacing at 1 (7 stored mantissa bits)
    cases = [(one, one), (one + u / 2, one), (one + 1.5 * u, one + 2 * u), (one + u / 2 + 2 ** -20, one + u),
             (-3.0, -3.0), (0.0, 0.0), (2.0 ** -130, 2.0 ** -130)]
    for x, want in cases:
        assert O.bf16_round(np.array([x]))[0] == want, x
    r = np.random.default_rng(0).normal(size=1000)
    b = O.bf16_round(r)
    assert np.all(np.abs(b - r) <= np.abs(r) * 2.0 ** -8 * (1 + 1e-12))
    bits = b.astype(np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)


def test_convolution_matches_scipy_correlation():
    from scipy.signal import correlate
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 7, 9, 2))
    Wm = rng.normal(size=(9 * 2, 3))
    b = rng.normal(size=3)
    y = O.conv(x, Wm, b, rnd=False)
    for co in range(3):
        want = np.full((7, 9), b[co])
        for ci in range(2):
            k = np.array([Wm[t * 2 + ci, co] for t in range(9)]).reshape(3, 3)
            want += correlate(x[0, :, :, ci], k, mode="same")
        assert np.allclose(y[0, :, :, co], want, atol=1e-12)


def test_im2col_adjoint():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 6, 4, 3))
    c = rng.normal(size=(2 * 6 * 4, 27))
    assert np.isclose(np.sum(O.im2col(x) * c), np.sum(x * O.col2im(c, x.shape)), rtol=1e-13)


def test_backward_matches_finite_differences():
    K = 2
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, size=(2, 8, 6, 3))
    params = wsnet_init(K, 4).astype(np.float64) * 3.0
    params += rng.normal(scale=0.05, size=params.size)  # nonzero biases too
    mu_t = rng.normal(scale=0.5, size=(2, 8, 6, 6))
    eps_t = rng.uniform(2, 1100, size=(2, K, 2))
    box = ((2.0, 2.0), (1100.0, 1100.0))
    loss, g = O.loss_grad(params, x, mu_t, eps_t, K, *box, w_eps=0.7, bf16=False)
    offs, wl, bl, n = O.layout(K)
    pick = list(rng.choice(n, size=60, replace=False)) + [offs[0][0], offs[4][1], wl, n - 1]
    for i in pick:
        h = 1e-6 * max(1.0, abs(params[i]))
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (O.loss_grad(pp, x, mu_t, eps_t, K, *box, 0.7, bf16=False)[0]
              - O.loss_grad(pm, x, mu_t, eps_t, K, *box, 0.7, bf16=False)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_mu_head_stays_in_the_unit_ball():
    K = 3
    x = np.random.default_rng(5).uniform(size=(1, 10, 12, 3))
    params = wsnet_init(K, 6).astype(np.float64) * 3.0
    mu, eps, _ = O.forward(params, x, K, (2.0, 2.0), (1100.0, 1100.0))
    assert np.all(np.sqrt(np.sum(mu ** 2, axis=3)) <= 1.0 + 1e-12)
    assert np.all((eps >= 2.0) & (eps <= 1100.0))


def test_control_head_reads_the_box_on_a_log_scale():
    """With the head's weights at zero, e = sigmoid(b) per output: b = 0 gives the
    geometric mean of the box, a large |b| its ends; a target at the geometric
    mean then costs nothing, and one at eps_max costs (1 - 1/2)^2 w_eps."""
    K = 2
    x = np.random.default_rng(7).uniform(size=(1, 6, 8, 3))
    params = wsnet_init(K, 8).astype(np.float64)
    offs, wl, bl, n = O.layout(K)
    params[wl:bl] = 0.0
    lo, hi = (2.0, 3.0), (1100.0, 300.0)
    for b, want in ((0.0, np.sqrt(np.multiply(lo, hi))), (60.0, np.array(hi)), (-60.0, np.array(lo))):
        params[bl:n] = b
        _, eps, _ = O.forward(params, x, K, lo, hi)
        assert np.allclose(eps.reshape(K, 2), want[None, :], rtol=1e-12)
    params[bl:n] = 0.0
    mu, _, _ = O.forward(params, x, K, lo, hi, bf16=False)
    for eps_t, cost in ((np.sqrt(np.multiply(lo, hi)), 0.0), (np.array(hi), 0.25)):
        loss, _ = O.loss_grad(params, x, mu, np.tile(eps_t, (1, K, 1)), K, lo, hi, w_eps=0.5, bf16=False)
        assert loss == pytest.approx(0.5 * cost, abs=1e-12)
