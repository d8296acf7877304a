"""Tuning parameters change speed, never results: every (group_tiles,
features_per_bin) setting matches the oracle on a multi-pair batch, and
sfm_autotune times all settings and keeps one of them."""
import numpy as np
import pytest

import scenes
from tests.gpu_util import compare_all, say

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
def batch():
    """10 cameras on a 90 deg arc, 1k-6k features (ragged tiles and groups)."""
    centers = scenes.generator._ring(10, 20.0, 0.0, az0=-45.0, span=90.0, endpoint=True)
    scene = scenes.make_multiview_scene(centers, 1000, 6000, n_points=30_000, seed=4)
    images = [(scene.image(k).xy, scene.image(k).desc) for k in range(scene.n_images)]
    pairs = [(a, b, 4.0) for a, b in scenes.covisible_pairs(scene, top_k=3)][:24]
    Fs = np.stack([scene.F(a, b) for a, b, _ in pairs])
    return images, pairs, Fs


@pytest.fixture(scope="module")
def oracle_result(oracle_lib, batch):
    images, pairs, Fs = batch
    return oracle_lib.match(images, pairs, Fs)


@pytest.mark.parametrize("group_tiles", [4, 8])
@pytest.mark.parametrize("features_per_bin", [1, 4, 8, 16, 64])
def test_every_tuning_matches_oracle(sfm, batch, oracle_result, group_tiles, features_per_bin):
    images, pairs, Fs = batch
    m = sfm.Matcher().register(images)
    sfm.sfm_set_tuning(m.ctx, group_tiles, features_per_bin)
    assert sfm.sfm_get_tuning(m.ctx) == (group_tiles, features_per_bin)
    for form in ("batched", "plain"):
        out = m.match(pairs, Fs, form=form, emit_all=True)
        clean, bl = compare_all(out, oracle_result, len(pairs))
        assert clean > 0
    m.close()


def test_tuning_rejects_bad_values(sfm, batch):
    images, _, _ = batch
    m = sfm.Matcher().register(images)
    for t, f in ((3, 8), (0, 8), (2, 8), (16, 8), (8, 0), (8, 2000)):
        with pytest.raises(sfm.SfmError) as e:
            sfm.sfm_set_tuning(m.ctx, t, f)
        assert e.value.status == sfm.SFM_EINVAL
    assert sfm.sfm_get_tuning(m.ctx) == (8, 8)
    m.close()


def test_autotune(sfm, batch, oracle_result):
    images, pairs, Fs = batch
    m = sfm.Matcher().register(images)
    times = sfm.sfm_autotune(m.ctx, pairs, Fs, repeats=2)
    say("  autotune ms: " + ", ".join(f"{k}: {v:.3f}" for k, v in times.items()))
    assert len(times) == 6 and all(v > 0 for v in times.values())
    best = sfm.sfm_get_tuning(m.ctx)
    assert times[best] == min(times.values())
    out = m.match(pairs, Fs, form="batched", emit_all=True)
    compare_all(out, oracle_result, len(pairs))
    m.close()


def test_autotune_cache(sfm, batch, tmp_path):
    """sfm_autotune_cached tunes a new batch shape and stores the winner; a
    later call with the same shape reads it back without timing anything; a
    new shape adds an entry.  The file stays valid JSON."""
    import json
    images, pairs, Fs = batch
    path = str(tmp_path / "tune.json")
    m = sfm.Matcher().register(images)
    hit, times = sfm.sfm_autotune_cached(m.ctx, pairs, Fs, path, repeats=1)
    assert not hit and len(times) == 6
    best = sfm.sfm_get_tuning(m.ctx)
    entries = json.loads(open(path).read())
    assert len(entries) == 1
    (key, rec), = entries.items()
    assert (rec["group_tiles"], rec["features_per_bin"]) == best and "gfx" in key
    m2 = sfm.Matcher().register(images)
    sfm.sfm_set_tuning(m2.ctx, *((4, 16) if best != (4, 16) else (8, 8)))
    hit2, t2 = sfm.sfm_autotune_cached(m2.ctx, pairs, Fs, path)
    assert hit2 and t2 is None and sfm.sfm_get_tuning(m2.ctx) == best
    hit3, _ = sfm.sfm_autotune_cached(m2.ctx, pairs[:2], Fs[:2], path, repeats=1)
    assert not hit3 and len(json.loads(open(path).read())) == 2
    say(f"  tuning cache: {key} -> {best}")
    m.close()
    m2.close()
