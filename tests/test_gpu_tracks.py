"""Tracks and triangulation (sfm_tracks, sfm_triangulate) through the C ABI.

The matches of a 12-camera scene's covisible pairs (batched form) become the
match graph; GPU labels must equal the oracle's exactly (smallest node id per
component).  GPU points must fit their equations as well as the oracle's
least-squares points (residuals) and agree with them closely; tracks whose
observations are all true features of one 3D point land near it."""
import numpy as np
import pytest

import scenes
from oracle import tracks as tr
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_06235_amd as sfm
    sfm.lib()
    return sfm


@pytest.fixture(scope="module")
def graph(sfm):
    centers = scenes.generator._ring(12, 20.0, 0.0)
    sc = scenes.make_multiview_scene(centers, 1000, 4000, n_points=20_000, seed=3)
    images = [(sc.image(k).xy, sc.image(k).desc) for k in range(sc.n_images)]
    pairs = [(a, b, 4.0) for a, b in scenes.covisible_pairs(sc, top_k=4)]
    Fs = np.stack([sc.F(a, b) for a, b, _ in pairs])
    m = sfm.Matcher().register(images)
    out = m.match(pairs, Fs, form="batched")
    off = np.concatenate([[0], np.cumsum([xy.shape[0] for xy, _ in images])])
    edges = []
    for k, (a, b, _) in enumerate(pairs):
        q, mt, _, _ = out.pair(k)
        edges.append(np.stack([off[a] + q, off[b] + mt], axis=1))
    edges = np.concatenate(edges).astype(np.int32)
    node_image = np.repeat(np.arange(len(images)), np.diff(off)).astype(np.int32)
    node_xy = np.concatenate([xy for xy, _ in images]).astype(np.float32)
    gt = np.concatenate([sc.image(k).gt for k in range(sc.n_images)])
    P = np.stack([c.K @ np.hstack([c.R, c.t[:, None]]) for c in sc.cams])
    say(f"  {int(off[-1])} observations, {edges.shape[0]} matches over {len(pairs)} pairs")
    return m, int(off[-1]), edges, node_image, node_xy, gt, P, sc.points


def test_tracks_equal_oracle(sfm, graph):
    import torch
    m, n, edges, *_ = graph
    label = torch.empty(n, dtype=torch.int32, device="cuda")
    d_edges = torch.as_tensor(edges).cuda()
    sfm.sfm_tracks(m.ctx, n, d_edges, label)
    sfm.sfm_sync(m.ctx)
    got = label.cpu().numpy()
    ref = tr.tracks(n, edges)
    assert np.array_equal(got, ref)
    # The same labels with the edges shuffled and reversed.
    rng = np.random.default_rng(41)
    e2 = edges[rng.permutation(edges.shape[0])][:, ::-1].copy()
    sfm.sfm_tracks(m.ctx, n, torch.as_tensor(e2).cuda(), label)
    sfm.sfm_sync(m.ctx)
    assert np.array_equal(label.cpu().numpy(), ref)
    sizes = np.bincount(ref)
    say(f"  {int((sizes >= 2).sum())} tracks of 2+ observations, longest {int(sizes.max())}")


def test_triangulation_matches_oracle(sfm, graph):
    import torch
    m, n, edges, node_image, node_xy, gt, P, points = graph
    label = torch.empty(n, dtype=torch.int32, device="cuda")
    sfm.sfm_tracks(m.ctx, n, torch.as_tensor(edges).cuda(), label)
    X = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    n_obs = torch.empty(n, dtype=torch.int32, device="cuda")
    sfm.sfm_triangulate(m.ctx, label, torch.as_tensor(node_image).cuda(),
                        torch.as_tensor(node_xy).cuda(), torch.as_tensor(P).cuda(), X, n_obs)
    sfm.sfm_sync(m.ctx)
    lab = label.cpu().numpy()
    Xg, ng = X.cpu().numpy(), n_obs.cpu().numpy()
    Xo, no = tr.triangulate(lab, node_image, node_xy, P)
    roots = np.flatnonzero(lab == np.arange(n))
    assert np.array_equal(ng[roots], no[roots])
    multi = roots[no[roots] >= 2]
    ok = np.isfinite(Xg[multi]).all(axis=1)
    assert ok.mean() > 0.99
    order = np.argsort(lab, kind="stable")
    groups = np.split(order, np.flatnonzero(np.diff(lab[order])) + 1)
    by_root = {int(lab[g[0]]): g for g in groups}
    close = worse = 0
    for r in multi[ok]:
        g = by_root[int(r)]
        rows = []
        for i in g:
            p = P[node_image[i]]
            rows += [node_xy[i, 0] * p[2] - p[0], node_xy[i, 1] * p[2] - p[1]]
        A = np.asarray(rows)
        res = lambda x: np.linalg.norm(A[:, :3] @ x + A[:, 3])  # noqa
        # The GPU point fits its equations as well as the least-squares point.
        if res(Xg[r]) > res(Xo[r]) * (1 + 1e-6) + 1e-9:
            worse += 1
        if np.linalg.norm(Xg[r] - Xo[r]) <= 1e-6 * (1 + np.linalg.norm(Xo[r])):
            close += 1
    say(f"  {len(multi)} tracks triangulated; {close} within 1e-6 of the oracle, {worse} worse fits")
    assert worse == 0
    assert close >= 0.99 * ok.sum()
    # Tracks whose observations are all true features of one point.
    true_err = []
    for r in multi[ok]:
        ids = gt[by_root[int(r)]]
        if ids[0] >= 0 and (ids == ids[0]).all():
            true_err.append(np.linalg.norm(Xg[r] - points[ids[0]]))
    say(f"  {len(true_err)} all-true tracks: median error {np.median(true_err):.4f}")
    assert len(true_err) > 100 and np.median(true_err) < 0.1


def test_bad_edges_raise(sfm, graph):
    import torch
    m, n, *_ = graph
    label = torch.empty(n, dtype=torch.int32, device="cuda")
    bad = torch.as_tensor(np.array([[0, 1], [2, n + 5]], np.int32)).cuda()
    with pytest.raises(sfm.SfmError) as e:
        sfm.sfm_tracks(m.ctx, n, bad, label)
        sfm.sfm_sync(m.ctx)
    assert e.value.status == sfm.SFM_EKERNEL


def test_tracks_large_graphs_equal_oracle(sfm):
    """Graphs large enough for many concurrent finds: the 500-pair batch's
    match graph and a million nodes in long shuffled chains.  The labelling
    pass once let a path-halving write replace a finished label with a
    non-root ancestor on the batch's graph."""
    import torch
    import bench
    images, pairs, Fs, _ = bench.arc_batch_workload()
    m = sfm.Matcher().register(images)
    out = m.match(pairs, Fs, form="batched")
    off = np.concatenate([[0], np.cumsum([xy.shape[0] for xy, _ in images])])
    edges = []
    for k, (a, b, _) in enumerate(pairs):
        q, mt, _, _ = out.pair(k)
        edges.append(np.stack([off[a] + q, off[b] + mt], axis=1))
    batch_edges = np.concatenate(edges).astype(np.int32)
    rng = np.random.default_rng(11)
    n2 = 1_000_000
    perm = rng.permutation(n2).astype(np.int32)
    cuts = np.sort(rng.choice(np.arange(1, n2), size=2_000, replace=False))
    chain = np.ones(n2 - 1, bool)
    chain[cuts - 1] = False                      # no edge across a cut
    e2 = np.stack([perm[:-1][chain], perm[1:][chain]], axis=1)
    seg = np.searchsorted(cuts, np.arange(n2), side="right")
    a = rng.integers(0, n2, size=200_000)
    starts = np.concatenate([[0], cuts])
    ends = np.concatenate([cuts, [n2]])
    b = starts[seg[a]] + (rng.integers(0, 1 << 30, size=a.size) % (ends[seg[a]] - starts[seg[a]]))
    e2 = np.concatenate([e2, np.stack([perm[a], perm[b]], axis=1)])
    e2 = e2[rng.permutation(e2.shape[0])].astype(np.int32)
    for n, e, what in ((int(off[-1]), batch_edges, "batch graph"), (n2, e2, "chains")):
        ref = tr.tracks(n, e)
        d_edges = torch.as_tensor(e).cuda()
        label = torch.empty(n, dtype=torch.int32, device="cuda")
        for rep in range(3):
            label.fill_(-1)
            sfm.sfm_tracks(m.ctx, n, d_edges, label)
            sfm.sfm_sync(m.ctx)
            got = label.cpu().numpy()
            bad = np.nonzero(got != ref)[0]
            assert bad.size == 0, f"{what}, run {rep}: {bad.size} labels differ, first {bad[:5]}"
        say(f"  {what}: {n} nodes, {e.shape[0]} edges, {np.unique(ref).size} components")
    m.close()


def test_bad_image_index_raises(sfm, graph):
    """An image index out of range raises the error flag; the node is left
    out of its track's list, so no list overflows."""
    import torch
    m, n, edges, node_image, node_xy, _, P, _ = graph
    label = torch.empty(n, dtype=torch.int32, device="cuda")
    sfm.sfm_tracks(m.ctx, n, torch.as_tensor(edges).cuda(), label)
    sfm.sfm_sync(m.ctx)
    bad_img = node_image.copy()
    bad_img[int(edges[0, 0])] = P.shape[0] + 3
    d = {k: torch.as_tensor(v).cuda() for k, v in (("img", bad_img), ("xy", node_xy), ("P", P))}
    X = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    n_obs = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(sfm.SfmError) as e:
        sfm.sfm_triangulate(m.ctx, label, d["img"], d["xy"], d["P"], X, n_obs)
        sfm.sfm_sync(m.ctx)
    assert e.value.status == sfm.SFM_EKERNEL
    # The context still works.
    d["img"] = torch.as_tensor(node_image).cuda()
    sfm.sfm_triangulate(m.ctx, label, d["img"], d["xy"], d["P"], X, n_obs)
    sfm.sfm_sync(m.ctx)
