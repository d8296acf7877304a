"""Staged coarse matching (sfm_preemptive_match, Section 4) against the oracle.

Images list their features by decreasing scale, as the entry point requires;
the oracle ranks them by scale on its own.  Every pair's rows (query, match,
D1, D2), its comparison count and the stages it ran must equal the oracle's
exactly: all distances are integers and no band is involved."""
import numpy as np
import pytest

import scenes
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


def _truncate(img, n):
    return scenes.Image(img.xy[:n], img.desc[:n], img.gt[:n], img.scale[:n])


@pytest.fixture(scope="module")
def small_scene():
    """12 views on a 180 deg arc, 1.5k-6k features; two cut below 1000
    features (still in scale order) and one without features."""
    centers = [(20 * np.sin(a), 0.0, 20 * np.cos(a)) for a in np.deg2rad(np.linspace(-90, 90, 12))]
    scene = scenes.make_multiview_scene(centers, 1500, 6000, seed=5)
    imgs = [scenes.by_scale(scene.image(k)) for k in range(12)]
    imgs[3] = _truncate(imgs[3], 800)
    imgs[7] = _truncate(imgs[7], 999)
    imgs[10] = _truncate(imgs[10], 0)
    pairs = [(a, b, 0.0) for a in range(12) for b in range(a + 1, 12)]
    pairs += [(b, a, 0.0) for a, b, _ in pairs[:12]]
    return imgs, pairs


def _run(sfm, m, pairs, **cfg):
    out = m.buffers(pairs)
    stages = sfm.sfm_preemptive_match(m.ctx, pairs, out, cfg=sfm.preemptive_cfg(**cfg))
    return out, stages


def _compare(out, stages, want, tag):
    ncmp = out.n_comparisons.cpu().numpy()
    for p, w in enumerate(want):
        q, mt, d1, d2 = out.pair(p)
        assert stages[p] == w["stages"], f"{tag} pair {p}: stages {stages[p]} != {w['stages']}"
        for name, got in (("query", q), ("match", mt), ("d1", d1), ("d2", d2)):
            assert np.array_equal(got, w[name]), f"{tag} pair {p}: {name} differs"
        assert int(ncmp[p]) == w["n_comparisons"], f"{tag} pair {p}: comparisons differ"


CONFIGS = [
    dict(),                                                     # the paper's 10% / 20% / > 4 / 1000
    dict(query_pct=15, target_pct=30, min_matches=2, enough=40),
    dict(query_pct=60, target_pct=25, min_matches=0, small_image=0),
]


@pytest.mark.parametrize("ci", range(len(CONFIGS)))
def test_preemptive_equals_oracle(sfm, small_scene, ci):
    from oracle.preemptive import preemptive_match
    imgs, pairs = small_scene
    cfg = CONFIGS[ci]
    say(f"  preemptive config {cfg}: {len(pairs)} pairs")
    m = sfm.Matcher().register([(im.xy, im.desc) for im in imgs])
    out, stages = _run(sfm, m, pairs, **cfg)
    want = preemptive_match([(im.xy, im.desc, im.scale) for im in imgs], pairs, **cfg)
    _compare(out, stages, want, f"config {ci}")
    kinds = np.bincount(stages, minlength=3)
    say(f"    stages whole/1/2 = {kinds.tolist()}, {int(out.offset[len(pairs)])} matches")
    if ci == 0:
        assert kinds[0] > 0 and kinds[1] > 0 and kinds[2] > 0
    m.close()


def test_preemptive_edges_and_errors(sfm, small_scene):
    import torch
    imgs, pairs = small_scene
    m = sfm.Matcher().register([(im.xy, im.desc) for im in imgs])
    out = m.buffers([])
    out.offset.fill_(-1)
    assert len(sfm.sfm_preemptive_match(m.ctx, [], out)) == 0
    assert int(out.offset[0]) == 0
    out = m.buffers(pairs[:3])
    with pytest.raises(sfm.SfmError) as e:
        sfm.sfm_preemptive_match(m.ctx, pairs[:3], out, opt=sfm.options(emit_all=True))
    assert e.value.status == sfm.SFM_EINVAL
    with pytest.raises(sfm.SfmError) as e:
        sfm.sfm_preemptive_match(m.ctx, pairs[:3], out, cfg=sfm.preemptive_cfg(query_pct=0))
    assert e.value.status == sfm.SFM_EINVAL
    with pytest.raises(sfm.SfmError) as e:
        sfm.sfm_preemptive_match(m.ctx, [(0, 12)], out)
    assert e.value.status == sfm.SFM_EINVAL
    small = sfm.MatchBuffers(10, 3, "cuda:0")
    with pytest.raises(sfm.SfmError) as e:
        sfm.sfm_preemptive_match(m.ctx, pairs[:3], small)
    assert e.value.status == sfm.SFM_ECAPACITY
    # The context still works afterwards, and ordinary matching is unaffected.
    st = sfm.sfm_preemptive_match(m.ctx, pairs[:3], out)
    assert len(st) == 3
    bf = m.match(pairs[:3], None, form="bruteforce")
    assert int(bf.offset[3]) >= 0
    torch.cuda.synchronize()
    m.close()


def test_preemptive_full_batch_sampled(sfm):
    """All 1,770 unordered pairs of the 60-view arc (2k-20k features per
    image): the launch the benchmark times; six pairs against the oracle,
    properties that hold at any size on all of them."""
    from oracle.preemptive import preemptive_match, stage_sizes
    scene, _ = scenes.make_arc_batch()
    scenes.materialize(scene)
    imgs = [scenes.by_scale(scene.image(k)) for k in range(scene.n_images)]
    pairs = [(a, b, 0.0) for a in range(60) for b in range(a + 1, 60)]
    say(f"  full batch: {len(pairs)} pairs")
    m = sfm.Matcher().register([(im.xy, im.desc) for im in imgs])
    out, stages = _run(sfm, m, pairs)
    off = out.offset.cpu().numpy()
    q_all = out.query.cpu().numpy()
    for p, (a, b, _) in enumerate(pairs):
        whole, q, r, q2 = stage_sizes(imgs[a].n, imgs[b].n)
        rows = q_all[off[p]:off[p + 1]]
        n1 = int(np.sum(rows < q))
        assert np.all(np.diff(rows) > 0)
        assert stages[p] == (2 if n1 > 4 else 1)
        assert rows.size == 0 or rows[-1] < (q + q2 if stages[p] == 2 else q)
    sample = [0, 1, 300, 901, 1500, 1769]
    want = preemptive_match([(im.xy, im.desc, im.scale) for im in imgs],
                            [pairs[p] for p in sample])
    ncmp = out.n_comparisons.cpu().numpy()
    for w, p in zip(want, sample):
        q, mt, d1, d2 = out.pair(p)
        assert stages[p] == w["stages"]
        assert np.array_equal(q, w["query"]) and np.array_equal(mt, w["match"])
        assert np.array_equal(d1, w["d1"]) and np.array_equal(d2, w["d2"])
        assert int(ncmp[p]) == w["n_comparisons"]
    say(f"    stages 1/2 = {np.bincount(stages, minlength=3)[1:].tolist()}, "
        f"{int(off[-1])} matches")
    m.close()
