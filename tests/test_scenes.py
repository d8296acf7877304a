"""Pins for the synthetic scene generator (inputs shared by oracle and GPU)."""
import numpy as np

import scenes
from scenes.generator import project


def _planted(scene, a=0, b=1):
    A, B = scene.images[a], scene.images[b]
    pos_b = {int(g): k for k, g in enumerate(B.gt) if g >= 0}
    ia = [k for k, g in enumerate(A.gt) if g >= 0 and int(g) in pos_b]
    ib = [pos_b[int(A.gt[k])] for k in ia]
    return np.array(ia), np.array(ib)


def test_f_direction_noise_free_correspondences():
    """x_b^T F x_a = 0 for exact projections, in the a -> b direction (eq. 1)."""
    s = scenes.make_two_view_2k()
    X = s.points[:200]
    xa, za = project(s.cams[0], X)
    xb, zb = project(s.cams[1], X)
    assert (za > 0).all() and (zb > 0).all()
    ha = np.c_[xa, np.ones(len(xa))]
    hb = np.c_[xb, np.ones(len(xb))]
    lines = ha @ s.F.T                     # l_b = F x_a
    dist = np.abs(np.sum(hb * lines, axis=1)) / np.hypot(lines[:, 0], lines[:, 1])
    assert dist.max() <= 1e-9
    # The transposed convention must not also hold (catches a swapped F).
    lines_t = ha @ s.F
    dist_t = np.abs(np.sum(hb * lines_t, axis=1)) / np.hypot(lines_t[:, 0], lines_t[:, 1])
    assert np.median(dist_t) > 1.0


def test_f_rank_two_and_epipole():
    s = scenes.make_two_view_2k()
    sv = np.linalg.svd(s.F, compute_uv=False)
    assert sv[2] <= 1e-12 * sv[0]
    # The epipole of image b is the projection of camera a's centre.
    ca = s.cams[0].center
    e_b, _ = project(s.cams[1], ca[None, :])
    e_h = np.r_[e_b[0], 1.0]
    assert np.abs(s.F.T @ e_h).max() <= 1e-12 * np.abs(s.F).max() * np.abs(e_h).max()
    # For cameras 15 deg apart on a circle looking at its centre the epipole
    # lies f cot(7.5 deg) from the principal point, horizontally.
    assert abs(abs(e_b[0, 0] - 512.0) - 1000.0 / np.tan(np.deg2rad(7.5))) < 1e-6
    assert abs(e_b[0, 1] - 384.0) < 1e-6


def test_descriptor_model_and_counts():
    s = scenes.make_two_view_2k()
    for im in s.images:
        assert im.n == 2000
        assert im.desc.dtype == np.uint8 and im.desc.max() <= 127
        assert im.xy.dtype == np.float32
        assert (im.xy[:, 0] >= 0).all() and (im.xy[:, 0] < 1024).all()
        assert (im.xy[:, 1] >= 0).all() and (im.xy[:, 1] < 768).all()
        assert (im.gt >= 0).sum() == 1500   # the whole box is in view at radius 20
    # True correspondences: descriptor difference is the two views' noise.
    ia, ib = _planted(s)
    da = s.images[0].desc[ia].astype(np.int32)
    db = s.images[1].desc[ib].astype(np.int32)
    diff = np.abs(da - db)
    assert diff.max() <= 12
    D = ((da - db) ** 2).sum(1)
    # E[D_true] = 128 * Var(U{-6..6} - U{-6..6}) = 128 * 28, reduced by clipping at 0.
    assert 2500 < D.mean() < 3800


def test_keypoint_noise_statistics():
    s = scenes.make_two_view_16k()
    A = s.images[0]
    t = A.gt >= 0
    xy_p, _ = project(s.cams[0], s.points[A.gt[t]])
    r = A.xy[t] - xy_p
    assert abs(r.mean()) < 0.02
    assert 0.48 < r.std() < 0.52
    assert abs(t.mean() - 0.4) < 0.01


def test_seeds_reproducible():
    a = scenes.make_two_view_2k(seed=0)
    b = scenes.make_two_view_2k(seed=0)
    c = scenes.make_two_view_2k(seed=1)
    assert np.array_equal(a.images[0].desc, b.images[0].desc)
    assert np.array_equal(a.images[1].xy, b.images[1].xy)
    assert not np.array_equal(a.images[0].desc, c.images[0].desc)


def test_multiview_visibility_and_pairs():
    scene, pairs = scenes.make_arc_batch()
    assert scene.n_images == 60 and len(pairs) == 500
    assert scene.n_features.min() >= 2000 and scene.n_features.max() <= 20000
    im = scene.image(3)
    assert im.n == scene.n_features[3]
    vis = set(scene.visible_ids(3).tolist())
    assert set(im.gt[im.gt >= 0].tolist()) <= vis
    az = np.linspace(-90.0, 90.0, 60)
    for a, b, band in pairs:
        assert a != b and 5.0 <= abs(az[a] - az[b]) <= 30.0 and band == 4.0


def test_materialize_threads_equal_sequential():
    """Images generated on a thread pool are byte-identical to one-by-one
    generation (each image has its own seeded generator; the BLAS products of
    the projection are serialised)."""
    # 200k points: products this large are the ones the BLAS runs on its own
    # threads, where concurrent calls went wrong.
    centers = scenes.generator._ring(24, 20.0, 0.0)
    seq = scenes.make_multiview_scene(centers, 1000, 3000, seed=4)
    par = scenes.make_multiview_scene(centers, 1000, 3000, seed=4)
    scenes.materialize(par, workers=8)
    for i in range(seq.n_images):
        a, b = seq.image(i), par.image(i)
        assert np.array_equal(a.xy, b.xy) and np.array_equal(a.desc, b.desc)
        assert np.array_equal(a.gt, b.gt)
    reqs = scenes.stress_requests(par, 50, seed=2)
    assert len(reqs) == len(set((a, b) for a, b, _ in reqs)) == 50
    assert all(2.0 <= d <= 8.0 for _, _, d in reqs)
