"""Pins of the segmentation oracle (watershed labelling and the metrics of
Sec. 4.4) against independent algorithms, library routines, closed forms
and a hand-worked example.  CPU only."""
from __future__ import annotations

import heapq
import itertools

import numpy as np
import pytest
from scipy import ndimage
from scipy.spatial.distance import pdist

from oracle import oracle as O
from paper_2510_16154_amd.synth import voronoi_image


def prim_watershed(c, theta):
    """Independent check of the forest: Prim's algorithm grown from all markers
    at once (a virtual root joined to every marker pixel).  With a strict
    order on the edges the minimum spanning tree is unique, so Prim and
    Kruskal must give the same forest and hence the same labels."""
    H, W, _ = c.shape
    g2 = O.seg_relief(c)
    th2 = np.float32(theta) * np.float32(theta)
    mark = g2 < th2
    if not mark.any():
        mark = np.zeros_like(mark)
        mark.flat[int(np.argmin(g2))] = True
    comp, k = ndimage.label(mark, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    # scipy numbers components in raster order of their first pixel, from 1
    lab = comp.astype(np.int64) - 1
    heap = []

    def push_edges(p):
        r, q = divmod(p, W)
        for rr, qq in ((r, q - 1), (r, q + 1), (r - 1, q), (r + 1, q)):
            if 0 <= rr < H and 0 <= qq < W:
                j = rr * W + qq
                if lab.flat[j] < 0:
                    a, b = min(p, j), max(p, j)
                    eid = 2 * a + (1 if b == a + W else 0)
                    w = max(g2.flat[p], g2.flat[j])
                    heapq.heappush(heap, (float(w), eid, p, j))

    for p in range(H * W):
        if lab.flat[p] >= 0:
            push_edges(p)
    while heap:
        _, _, p, j = heapq.heappop(heap)
        if lab.flat[j] >= 0:
            continue
        lab.flat[j] = lab.flat[p]
        push_edges(j)
    return lab.astype(np.int32), k


@pytest.mark.parametrize("seed,H,W,C,levels", [(1, 6, 7, 1, 4), (2, 9, 5, 3, 3), (3, 12, 12, 2, 0),
                                               (4, 1, 17, 1, 5), (5, 15, 1, 3, 0), (6, 10, 11, 3, 2)])
def test_watershed_matches_prim(seed, H, W, C, levels):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, 1, size=(H, W, C))
    if levels:
        c = np.round(c * levels) / levels  # plateaus: many equal weights, order decided by edge index
    c = c.astype(np.float32)
    for theta in (0.02, 0.2, 0.6):
        lab, k = O.seg_watershed(c, theta)
        ref, kr = prim_watershed(c, theta)
        assert k == kr
        np.testing.assert_array_equal(lab, ref)


def test_markers_are_connected_components():
    c = voronoi_image(30, 40, 3, 6, 0.02, 11)
    lab, k = O.seg_watershed(c, 0.02)
    g2 = O.seg_relief(c)
    mark = g2 < np.float32(0.02) * np.float32(0.02)
    comp, n = ndimage.label(mark, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    assert k == n
    np.testing.assert_array_equal(lab[mark], comp[mark] - 1)
    # every label owns at least its marker pixels; labels are 0..k-1
    assert set(np.unique(lab)) == set(range(k))


def test_relief_closed_forms():
    H, W = 5, 8
    q = np.arange(W, dtype=np.float32)
    ramp = np.broadcast_to((0.125 * q)[None, :, None], (H, W, 1)).astype(np.float32)
    g2 = O.seg_relief(ramp)
    # central difference of a ramp of slope 1/8 per pixel is 1/8; zero on the first/last column
    np.testing.assert_array_equal(g2[:, 1:-1], np.float32(1 / 64))
    np.testing.assert_array_equal(g2[:, [0, -1]], 0.0)
    np.testing.assert_array_equal(O.seg_relief(np.full((4, 6, 3), 0.3, np.float32)), 0.0)


def test_constant_image_is_one_segment():
    lab, k = O.seg_watershed(np.full((7, 9, 3), 0.4, np.float32), 0.02)
    assert k == 1 and (lab == 0).all()


def test_no_marker_fallback():
    c = np.random.default_rng(3).uniform(size=(6, 6, 1)).astype(np.float32)
    lab, k = O.seg_watershed(c, 0.0)  # nothing lies below 0: the lowest pixel is the only marker
    assert k == 1 and (lab == 0).all()


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_watershed_recovers_ground_truth_up_to_edge_band(seed):
    img, gt = voronoi_image(48, 56, 3, 6, 0.0, seed, return_labels=True)
    lab, k = O.seg_watershed(img, 0.02)
    present = np.unique(gt)
    assert k == len(present)
    # each label maps to one true region; disagreements only on pixels next to a true boundary
    mapping = {j: np.bincount(gt[lab == j]).argmax() for j in range(k)}
    assert sorted(mapping.values()) == sorted(present.tolist())
    mapped = np.vectorize(mapping.get)(lab)
    H, W = gt.shape
    near = np.zeros_like(gt, dtype=bool)
    pad = np.pad(gt, 1, mode="edge")
    for dr, dq in itertools.product((-1, 0, 1), repeat=2):
        near |= pad[1 + dr:1 + dr + H, 1 + dq:1 + dq + W] != gt
    assert not ((mapped != gt) & ~near).any()


def test_metrics_hand_worked_example():
    # 2 x 2 grey image, labels [[0, 0], [1, 1]]:
    #   region 0 holds 0 and 0.5 (mean 0.25, squared deviations 0.0625 + 0.0625),
    #   region 1 holds 1 and 1 (no deviation)  ->  IRV = 0.125 / 4 = 0.03125;
    #   processed = original: means 0.25 and 1  ->  IRC = 0.75, VS = 0.03125 / 0.75.
    c0 = np.array([[[0.0], [0.5]], [[1.0], [1.0]]], np.float32)
    lab = np.array([[0, 0], [1, 1]], np.int32)
    m = O.seg_metrics(c0, c0, lab)
    assert m["irv"] == 0.03125 and m["irc"] == 0.75
    assert m["vs"] == pytest.approx(0.03125 / 0.75, rel=1e-15)


def test_metrics_single_region_is_total_variance():
    c0 = np.random.default_rng(4).uniform(size=(13, 17, 3)).astype(np.float32)
    m = O.seg_metrics(c0, c0, np.zeros((13, 17), np.int32))
    assert m["irv"] == pytest.approx(sum(np.var(c0[..., ch].astype(np.float64)) for ch in range(3)), rel=1e-12)
    assert np.isnan(m["irc"]) and np.isnan(m["vs"])


def test_metrics_pixel_regions():
    c0 = np.random.default_rng(5).uniform(size=(6, 7, 2)).astype(np.float32)
    lab = np.arange(42, dtype=np.int32).reshape(6, 7)
    m = O.seg_metrics(c0, c0, lab)
    assert m["irv"] == 0.0
    assert m["irc"] == pytest.approx(pdist(c0.reshape(-1, 2).astype(np.float64)).min(), rel=1e-14)
    assert m["vs"] == 0.0


def test_metrics_piecewise_constant_ground_truth():
    rng = np.random.default_rng(6)
    colours = rng.uniform(size=(5, 3))
    gt = np.zeros((20, 30), np.int32)
    gt[:, 10:] = 1
    gt[8:, 20:] = 2
    gt[15:, :5] = 4  # label 3 stays empty
    img = colours[gt].astype(np.float32)
    m = O.seg_metrics(img, img, gt, k=5)
    assert m["irv"] == 0.0
    used = colours[[0, 1, 2, 4]].astype(np.float32).astype(np.float64)
    assert m["irc"] == pytest.approx(pdist(used).min(), rel=1e-14)
    # renaming the regions changes nothing
    perm = np.array([3, 0, 4, 1, 2], np.int32)
    m2 = O.seg_metrics(img, img, perm[gt], k=5)
    assert m2["irv"] == m["irv"] and m2["irc"] == pytest.approx(m["irc"], rel=1e-15)


def test_metrics_original_versus_processed():
    # IRV uses the original image, IRC the processed one
    rng = np.random.default_rng(8)
    c0 = rng.uniform(size=(8, 8, 1)).astype(np.float32)
    lab = (np.arange(64) % 2).reshape(8, 8).astype(np.int32)
    proc = np.where(lab[..., None] == 0, 0.2, 0.7).astype(np.float32)
    m = O.seg_metrics(proc, c0, lab)
    assert m["irc"] == pytest.approx(0.5, rel=1e-7)
    ref = sum(((c0[lab == j, 0].astype(np.float64) - c0[lab == j, 0].astype(np.float64).mean()) ** 2).sum()
              for j in (0, 1)) / 64
    assert m["irv"] == pytest.approx(ref, rel=1e-12)


def test_metrics_reject_out_of_range_labels():
    c0 = np.zeros((3, 3, 1), np.float32)
    with pytest.raises(ValueError):
        O.seg_metrics(c0, c0, np.full((3, 3), 2, np.int32), k=2)
