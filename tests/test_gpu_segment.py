"""GPU parity of the segmentation scores of Sec. 4.4: watershed labels bit for
bit against the oracle (both sides take every comparison on the same FP32
relief), IRV / IRC / VS within 1e-10 relative (the oracle sums in FP64, the
GPU in 2^-92-scaled fixed-point integers, the same bits on every run)."""
import numpy as np
import pytest

import paper_2510_16154_amd as A
from oracle import oracle as O
from paper_2510_16154_amd.synth import voronoi_image

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SCORE_TOL = 1e-10


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def check_scores(st, ref):
    for key in ("irv", "irc", "vs"):
        a, b = st[key], ref[key]
        if np.isnan(b):
            assert np.isnan(a), key
        elif b == 0.0 or np.isinf(b):
            assert a == b, key
        else:
            assert abs(a - b) <= SCORE_TOL * abs(b), (key, a, b)


def run_case(c, c0, theta=0.02):
    print(f"segment case shape={c.shape} theta={theta}", flush=True)
    lab, st = A.abc_segment(T(c), T(c0), theta)
    ref = O.segment(c, c0, theta)
    got = lab.cpu().numpy()
    assert st["k"] == ref["k"]
    np.testing.assert_array_equal(got, ref["labels"])
    check_scores(st, ref)
    return st


def quantised(H, W, C, levels, seed):
    rng = np.random.default_rng(seed)
    return (np.round(rng.uniform(size=(H, W, C)) * levels) / levels).astype(np.float32)


@pytest.mark.parametrize("H,W,C,kind", [
    (64, 80, 3, "clean"), (97, 131, 3, "noisy"), (37, 53, 1, "quantised"), (1, 300, 3, "noisy"),
    (300, 1, 2, "quantised"), (2, 2, 3, "noisy"), (128, 128, 31, "clean"), (45, 260, 4, "gradient")])
def test_watershed_and_scores_match_oracle(H, W, C, kind):
    if kind == "clean":
        c = voronoi_image(H, W, C, 9, 0.0, 2001)
    elif kind == "noisy":
        c = voronoi_image(H, W, C, 7, 0.03, 2002)
    elif kind == "gradient":
        c = voronoi_image(H, W, C, 6, 0.004, 2003, gradient_amp=0.1)
    else:
        c = quantised(H, W, C, 3, 2004)
    c0 = voronoi_image(H, W, C, 7, 0.05, 2005)
    for theta in (0.02, 0.15):
        run_case(c, c0, theta)


def test_constant_field_is_one_segment():
    c = np.full((33, 47, 3), 0.25, np.float32)
    st = run_case(c, voronoi_image(33, 47, 3, 5, 0.05, 2006))
    assert st["k"] == 1 and np.isnan(st["irc"]) and np.isnan(st["vs"])


def test_no_marker_fallback():
    st = run_case(quantised(20, 30, 3, 5, 2007), quantised(20, 30, 3, 5, 2008), theta=0.0)
    assert st["k"] == 1


def test_given_labels_are_scored():
    img, gt = voronoi_image(120, 90, 3, 8, 0.04, 2009, return_labels=True)
    gt = gt.astype(np.int32)
    _, st = A.abc_segment(T(img), T(img), labels=torch.as_tensor(gt, device="cuda"))
    ref = O.seg_metrics(img, img, gt)
    assert st["k"] == int(gt.max()) + 1
    check_scores(st, ref)
    # one label per pixel on a small image: IRV = 0, IRC = least distance between two pixels
    small = img[:16, :16].copy()
    lab = np.arange(256, dtype=np.int32).reshape(16, 16)
    _, st = A.abc_segment(T(small), T(small), labels=torch.as_tensor(lab, device="cuda"))
    check_scores(st, O.seg_metrics(small, small, lab))


def test_out_of_range_labels_are_rejected():
    img = voronoi_image(8, 8, 3, 2, 0.0, 2010)
    bad = torch.full((8, 8), 64, dtype=torch.int32, device="cuda")
    with pytest.raises(A.AbcError):
        A.abc_segment(T(img), T(img), labels=bad)


def test_repeat_calls_give_identical_labels_and_score_bits():
    c = voronoi_image(150, 170, 3, 10, 0.02, 2011)
    c0 = voronoi_image(150, 170, 3, 9, 0.05, 2012)
    a, sa = A.abc_segment(T(c), T(c0))
    for _ in range(3):
        b, sb = A.abc_segment(T(c), T(c0))
        assert torch.equal(a, b)
        for key in ("irv", "irc", "vs"):
            assert np.float64(sa[key]).tobytes() == np.float64(sb[key]).tobytes(), key
    # many small labels, so that many runs of pixels add into each label sum
    lab = (np.arange(150 * 170).reshape(150, 170) // 7 % 211).astype(np.int32)
    L = torch.as_tensor(lab, device="cuda")
    _, s1 = A.abc_segment(T(c), T(c0), labels=L)
    _, s2 = A.abc_segment(T(c), T(c0), labels=L)
    assert np.float64(s1["irv"]).tobytes() == np.float64(s2["irv"]).tobytes()
    assert np.float64(s1["irc"]).tobytes() == np.float64(s2["irc"]).tobytes()
    check_scores(s1, O.seg_metrics(c, c0, lab))


def test_values_far_from_one_keep_the_tolerance():
    # the fixed-point scale follows the largest |value|: images scaled by 2^40 and 2^-40
    # give the scores scaled by the same powers (IRV by the square), to the same tolerance
    c = voronoi_image(60, 70, 3, 6, 0.02, 2013)
    c0 = voronoi_image(60, 70, 3, 6, 0.05, 2014)
    for f in (2.0 ** 40, 2.0 ** -40):
        cs, c0s = (c * f).astype(np.float32), (c0 * f).astype(np.float32)
        lab, st = A.abc_segment(T(cs), T(c0s), 0.02 * f)
        ref = O.segment(cs, c0s, 0.02 * f)
        np.testing.assert_array_equal(lab.cpu().numpy(), ref["labels"])
        check_scores(st, ref)


@pytest.mark.parametrize("where", ["c", "c0"])
@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_input_is_rejected(where, bad):
    c = voronoi_image(20, 24, 3, 4, 0.02, 2015)
    c0 = c.copy()
    (c if where == "c" else c0)[5, 7, 1] = bad
    with pytest.raises(A.AbcError) as e:
        A.abc_segment(T(c), T(c0))
    assert e.value.code == A.ABC_ENONFINITE


def test_solver_output_at_full_size():
    # the use in the paper: labels of a solved image, scored against the input
    from paper_2510_16154_amd.workloads import VORONOI512 as wl
    c0 = wl.image()
    out = A.abc_solve(T(c0), wl.params(max_outer=2, max_inner=3, tol_alm=0.0))
    c = out["c"].cpu().numpy()
    st = run_case(c, c0)
    assert st["k"] >= 2
