"""The grid search of Section 6.2.1 (sfm_grid_match) against the oracle.

Every floating-point decision of the grid search is IEEE double in a fixed
order on both sides, so each query's C' size, nearest index, D1, D2 and
decision must equal the oracle's exactly."""
import numpy as np
import pytest

import scenes
from tests.fixtures import translation_F
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


def _per_query(out, q_off, p):
    s, e = int(q_off[p]), int(q_off[p + 1])
    return {"match": out.all_match[s:e].cpu().numpy(), "d1": out.all_d1[s:e].cpu().numpy(),
            "d2": out.all_d2[s:e].cpu().numpy(), "count": out.all_count[s:e].cpu().numpy()}


def _check(out, images, pairs, Fs, want, queries=None):
    q_off = np.concatenate([[0], np.cumsum([images[a][0].shape[0] for a, _, _ in pairs])])
    for p in range(len(pairs)):
        g = _per_query(out, q_off, p)
        w = want[p]
        qs = np.arange(images[pairs[p][0]][0].shape[0]) if queries is None else queries[p]
        for k in ("match", "d1", "d2", "count"):
            bad = np.nonzero(g[k][qs] != w[k])[0]
            assert bad.size == 0, f"pair {p}: {k} differs on {bad.size} queries, first {qs[bad[:5]]}"
        q, _, _, _ = out.pair(p)
        if queries is None:
            assert np.array_equal(q, np.nonzero(w["accept"])[0]), f"pair {p}: accepted set"
        else:
            acc = np.zeros(images[pairs[p][0]][0].shape[0], bool)
            acc[q] = True
            assert np.array_equal(acc[qs], w["accept"]), f"pair {p}: accepted set"


def test_grid_two_view_equals_oracle(sfm):
    from oracle.grid import grid_match
    sc = scenes.make_two_view_2k()
    images = [(im.xy, im.desc) for im in sc.images]
    m = sfm.Matcher().register(images)
    for d in (2.0, 4.0, 7.5):
        pairs = [(0, 1, d)]
        out = m.match(pairs, [sc.F], form="grid", emit_all=True)
        want = grid_match(images, pairs, [sc.F])
        _check(out, images, pairs, [sc.F], want)
        say(f"  two-view d={d}: {int(out.offset[1])} matches, mean |C'| "
            f"{want[0]['count'].mean():.1f}")
    m.close()


def test_grid_batch_equals_oracle(sfm):
    """Pairs of a 12-view arc with several d, an empty target image and
    ragged sizes."""
    from oracle.grid import grid_match
    centers = [(20 * np.sin(a), 0.0, 20 * np.cos(a)) for a in np.deg2rad(np.linspace(-30, 30, 8))]
    scene = scenes.make_multiview_scene(centers, 700, 2500, seed=9)
    images = [(scene.image(k).xy, scene.image(k).desc) for k in range(8)]
    images.append((np.zeros((0, 2), np.float32), np.zeros((0, 128), np.uint8)))
    pairs = [(0, 1, 4.0), (1, 0, 2.5), (2, 5, 6.0), (3, 4, 4.0), (6, 7, 3.0), (7, 2, 9.0),
             (0, 8, 4.0), (4, 3, 1.5)]
    Fs = np.stack([scene.F(a, b) if b < 8 else scene.F(a, 1) for a, b, _ in pairs])
    m = sfm.Matcher().register(images)
    out = m.match(pairs, Fs, form="grid", emit_all=True)
    want = grid_match(images, pairs, Fs)
    _check(out, images, pairs, Fs, want)
    n = int(out.offset[len(pairs)])
    say(f"  batch of {len(pairs)} pairs: {n} matches")
    m.close()


def test_grid_full_batch_sampled_and_recall(sfm):
    """The 500-pair batch with d = 4: 200 queries of five pairs against the
    oracle; agreement with the exact band on every pair."""
    import bench
    from oracle.grid import grid_match
    images, pairs, Fs, _ = bench.arc_batch_workload()
    m = sfm.Matcher().register(images)
    out = m.match(pairs, Fs, form="grid", emit_all=True)
    exact = m.match(pairs, Fs, form="batched")
    sample = [0, 7, 123, 311, 499]
    rng = np.random.default_rng(3)
    qsel = [np.sort(rng.choice(images[pairs[p][0]][0].shape[0], 200, replace=False))
            for p in sample]
    want = grid_match(images, [pairs[p] for p in sample], Fs[sample], queries=qsel)
    q_off = np.concatenate([[0], np.cumsum([images[a][0].shape[0] for a, _, _ in pairs])])
    for t, p in enumerate(sample):
        g = _per_query(out, q_off, p)
        for k in ("match", "d1", "d2", "count"):
            assert np.array_equal(g[k][qsel[t]], want[t][k]), f"pair {p}: {k} differs"
    # Agreement with the exact band: matches found by both, per pair summed.
    both = total_exact = total_grid = 0
    for p in range(len(pairs)):
        qe, me, _, _ = exact.pair(p)
        qg, mg, _, _ = out.pair(p)
        e = set(zip(qe.tolist(), me.tolist()))
        gset = set(zip(qg.tolist(), mg.tolist()))
        both += len(e & gset)
        total_exact += len(e)
        total_grid += len(gset)
    say(f"  grid d=4 vs exact band 4: {total_grid} vs {total_exact} matches, "
        f"{both / max(1, total_exact):.3f} of the exact ones found")
    assert both / total_exact > 0.8
    m.close()


def test_grid_errors(sfm):
    sc = scenes.make_two_view_2k()
    images = [(im.xy, im.desc) for im in sc.images]
    rng = np.random.default_rng(0)
    big = (rng.uniform(0, 1000, size=(70000, 2)).astype(np.float32),
           rng.integers(0, 128, size=(70000, 128), dtype=np.uint8))
    m = sfm.Matcher().register(images + [big])
    for d, status in ((0.0, sfm.SFM_EINVAL), (float("inf"), sfm.SFM_EINVAL),
                      (0.05, sfm.SFM_ECAPACITY)):
        with pytest.raises(sfm.SfmError) as e:
            m.match([(0, 1, d)], [sc.F], form="grid")
        assert e.value.status == status
    with pytest.raises(sfm.SfmError) as e:
        m.match([(0, 2, 4.0)], [sc.F], form="grid")
    assert e.value.status == sfm.SFM_ECAPACITY
    out = m.match([], np.zeros((0, 3, 3)), form="grid")
    assert int(out.offset[0]) == 0
    out = m.match([(0, 1, 4.0)], [sc.F], form="grid")      # still usable
    assert int(out.offset[1]) > 0
    m.close()


def test_grid_grouped_equals_oracle(sfm):
    """The 2-px query grouping of Section 6.2.2: per-query results and the
    number of groups equal the oracle's, on the two-view pair and a ragged
    batch; grouping off again gives the ungrouped results."""
    from oracle.grid import grid_match, query_groups
    sc = scenes.make_two_view_2k()
    centers = [(20 * np.sin(a), 0.0, 20 * np.cos(a)) for a in np.deg2rad(np.linspace(-30, 30, 6))]
    scene = scenes.make_multiview_scene(centers, 700, 2500, seed=4)
    images = [(im.xy, im.desc) for im in sc.images]
    images += [(scene.image(k).xy, scene.image(k).desc) for k in range(6)]
    images.append((np.zeros((0, 2), np.float32), np.zeros((0, 128), np.uint8)))
    pairs = [(0, 1, 4.0), (2, 3, 4.0), (4, 7, 3.0), (5, 2, 6.0), (6, 5, 4.0), (2, 8, 4.0),
             (3, 4, 2.5)]
    Fs = [sc.F] + [scene.F(a - 2, b - 2 if b < 8 else 1) for a, b, _ in pairs[1:]]
    Fs = np.stack(Fs)
    m = sfm.Matcher().register(images)
    with pytest.raises(sfm.SfmError):
        sfm.sfm_set_grid_grouping(m.ctx, -1.0)
    for px, lead in ((2.0, False), (0.5, False), (2.0, True)):
        sfm.sfm_set_grid_grouping(m.ctx, px, lead)
        out = m.match(pairs, Fs, form="grid", emit_all=True)
        want = grid_match(images, pairs, Fs, group_px=px, to_leader=lead)
        _check(out, images, pairs, Fs, want)
        groups = sum(len(query_groups(images[a][0], images[b][0], Fs[p], px, lead)[1])
                     for p, (a, b, _) in enumerate(pairs))
        assert sfm.sfm_grid_groups(m.ctx) == groups
        nq = sum(images[a][0].shape[0] for a, _, _ in pairs)
        say(f"  grouped px={px} to_leader={lead}: {groups} groups for {nq} queries, "
            f"{int(out.offset[len(pairs)])} matches")
    sfm.sfm_set_grid_grouping(m.ctx, 0.0)
    out = m.match(pairs, Fs, form="grid", emit_all=True)
    _check(out, images, pairs, Fs, grid_match(images, pairs, Fs))
    m.close()


def test_grid_grouped_many_pairs_equals_oracle(sfm):
    """More than 256 pairs in one grouped call: the grouping sort's pair key
    spans two digits; per-query results and the group count equal the
    oracle's."""
    from oracle.grid import grid_match, query_groups
    centers = [(20 * np.sin(a), 0.0, 20 * np.cos(a)) for a in np.deg2rad(np.linspace(-25, 25, 6))]
    scene = scenes.make_multiview_scene(centers, 60, 140, seed=6)
    images = [(scene.image(k).xy, scene.image(k).desc) for k in range(6)]
    base = [(a, b) for a in range(6) for b in range(6) if a != b]
    pairs = [(a, b, (2.0, 3.0, 4.0, 6.0)[i % 4]) for i, (a, b) in enumerate(base * 9)]
    assert len(pairs) > 256
    Fs = np.stack([scene.F(a, b) for a, b, _ in pairs])
    m = sfm.Matcher().register(images)
    sfm.sfm_set_grid_grouping(m.ctx, 2.0, False)
    out = m.match(pairs, Fs, form="grid", emit_all=True)
    want = grid_match(images, pairs, Fs, group_px=2.0, to_leader=False)
    _check(out, images, pairs, Fs, want)
    groups = sum(len(query_groups(images[a][0], images[b][0], Fs[p], 2.0, False)[1])
                 for p, (a, b, _) in enumerate(pairs))
    assert sfm.sfm_grid_groups(m.ctx) == groups
    say(f"  grouped, {len(pairs)} pairs: {groups} groups")
    m.close()


def test_grid_candidate_overflow_raises_and_context_recovers(sfm):
    """A query with more than 1,024 grid candidates C' (the LDS list of one
    query): the kernel keeps the first 1,024 and raises the device error
    flag, which sfm_sync reports as SFM_EKERNEL; the context then matches
    exactly again."""
    from oracle.grid import grid_match
    rng = np.random.default_rng(3)
    n_b = 20000
    # b's features fill a 2-px strip; lines y' = y (translation along x).
    xy_b = np.stack([rng.uniform(0, 1000, n_b), rng.uniform(500, 502, n_b)], 1).astype(np.float32)
    desc_b = rng.integers(0, 128, (n_b, 128), dtype=np.uint8)
    xy_a = np.array([[100.0, 501.0], [600.0, 501.5], [900.0, 100.0]], np.float32)
    desc_a = rng.integers(0, 128, (3, 128), dtype=np.uint8)
    sc = scenes.make_two_view_2k()
    images = [(xy_a, desc_a), (xy_b, desc_b)] + [(im.xy, im.desc) for im in sc.images]
    m = sfm.Matcher().register(images)
    with pytest.raises(sfm.SfmError) as e:
        m.match([(0, 1, 8.0)], [translation_F((1.0, 0.0, 0.0))], form="grid")
    assert e.value.status == sfm.SFM_EKERNEL
    pairs = [(2, 3, 4.0)]
    Fs = np.stack([sc.F])
    out = m.match(pairs, Fs, form="grid", emit_all=True)
    _check(out, images, pairs, Fs, grid_match(images, pairs, Fs))
    say("  grid C' overflow: SFM_EKERNEL, then exact")
    m.close()
