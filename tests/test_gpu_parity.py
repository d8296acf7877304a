"""GPU parity: the HIP library (through its C ABI) against the CPU oracle."""
import numpy as np
import pytest

import scenes
from tests.fixtures import load_hand_fixture, random_pair, translation_F
from tests.gpu_util import (FP32_ERR_PX, check_borderline_counts, compare_all, gpu_per_query,
                            say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_06235_amd as sfm
    sfm.lib()   # raises when the library is not built
    return sfm


def run_both(sfm, oracle, images, pairs, Fs, form="batched", **kw):
    say(f"  [{form}] pairs={len(pairs)} sizes={[(images[a][0].shape[0], images[b][0].shape[0]) for a, b, _ in pairs[:4]]}")
    m = sfm.Matcher().register(images)
    out = m.match(pairs, Fs, form=form, emit_all=True, **kw)
    ores = oracle.match(images, pairs, Fs, ignore_band=(form == "bruteforce"), **kw)
    return m, out, ores


def test_hand_fixture_gpu(sfm):
    xy_a, desc_a, xy_b, desc_b, F, band, expect = load_hand_fixture()
    for form in ("batched", "plain"):
        m = sfm.Matcher().register([(xy_a, desc_a), (xy_b, desc_b)])
        out = m.match([(0, 1, band)], [F], form=form, emit_all=True)
        g = gpu_per_query(out, [0, len(xy_a)], 0)
        acc = {int(q) for q in out.pair(0)[0]}
        got = [(i, int(g["match"][i]), int(g["d1"][i]), int(g["d2"][i]), int(g["count"][i]),
                int(i in acc)) for i in range(len(expect))]
        assert got == expect, form


@pytest.mark.parametrize("form", ["batched", "plain"])
def test_two_view_2k_parity(sfm, oracle_lib, form):
    s = scenes.make_two_view_2k()
    imgs = [(im.xy, im.desc) for im in s.images]
    _, out, ores = run_both(sfm, oracle_lib, imgs, s.pairs, [s.F], form)
    n, bl = compare_all(out, ores, 1)
    gbl = check_borderline_counts(out, oracle_lib, imgs, s.pairs, [s.F])
    say(f"  2-view 2k {form}: {n} queries exact ({bl} with a candidate within 1e-3 px of the "
        f"edge), {int(gbl[0])} slots decided in FP64, comparisons {int(ores.n_comparisons[0])}")


@pytest.mark.parametrize("margin", [0.0, 0.05, 0.5])
def test_recheck_margin(sfm, oracle_lib, margin):
    """A wide margin sends many slots through the FP64 re-decision (results
    unchanged, counts bracketed by the oracle's); margin 0 decides in FP32 only
    and reports no borderline slot."""
    s = scenes.make_two_view_2k()
    imgs = [(im.xy, im.desc) for im in s.images]
    m = sfm.Matcher().register(imgs)
    out = m.match(s.pairs, [s.F], emit_all=True, recheck_margin_px=margin)
    ores = oracle_lib.match(imgs, s.pairs, [s.F])
    if margin == 0.0:
        assert int(out.n_borderline[0]) == 0
        # FP32 alone may differ only on queries with a candidate within the FP32 error.
        tight = oracle_lib.match(imgs, s.pairs, [s.F], borderline_px=2 * FP32_ERR_PX)
        g = gpu_per_query(out, ores.q_off, 0)
        clean = tight.pair(0)["borderline"] == 0
        for k in ("match", "d1", "d2", "count"):
            assert np.array_equal(g[k][clean], ores.pair(0)[k][clean]), k
    else:
        compare_all(out, ores, 1)
        gbl = check_borderline_counts(out, oracle_lib, imgs, s.pairs, [s.F], margin=margin)
        say(f"  margin {margin}: {int(gbl[0])} slots decided in FP64, results exact")
        assert gbl[0] > 100
    m.close()


def test_two_view_16k_parity_and_fp32_error(sfm, oracle_lib):
    """Full 16k x 16k pair: bit-exact, borderline counts bracketed, and the
    FP32 distance within 1e-4 px of the FP64 one on every evaluated slot
    within 2d."""
    s = scenes.make_two_view_16k()
    imgs = [(im.xy, im.desc) for im in s.images]
    m, out, ores = run_both(sfm, oracle_lib, imgs, s.pairs, [s.F])
    n, bl = compare_all(out, ores, 1)
    gbl = check_borderline_counts(out, oracle_lib, imgs, s.pairs, [s.F])
    err, nslots = sfm.sfm_band_error(m.ctx, s.pairs, [s.F])
    say(f"  2-view 16k: {n} exact ({bl} with a candidate within 1e-3 px), {int(gbl[0])} slots "
        f"decided in FP64; max |e32 - e64| = {err:.3e} px over {nslots} slots within 2d")
    assert nslots > int(ores.n_comparisons[0])
    assert 0.0 < err <= FP32_ERR_PX


def test_arc_batch_sample_batched_vs_plain(sfm, oracle_lib):
    scene, pairs = scenes.make_arc_batch()
    rng = np.random.default_rng(5)
    sel = sorted(rng.choice(len(pairs), size=24, replace=False))
    sub = [pairs[k] for k in sel]
    used = sorted({a for a, _, _ in sub} | {b for _, b, _ in sub})
    remap = {k: i for i, k in enumerate(used)}
    imgs = [(scene.image(k).xy, scene.image(k).desc) for k in used]
    sp = [(remap[a], remap[b], band) for a, b, band in sub]
    Fs = [scene.F(a, b) for a, b, _ in sub]
    m = sfm.Matcher().register(imgs)
    ores = oracle_lib.match(imgs, sp, Fs)
    outs = {}
    for form in ("batched", "plain"):
        say(f"  arc batch sample {form}")
        outs[form] = m.match(sp, Fs, form=form, emit_all=True)
        n, bl = compare_all(outs[form], ores, len(sp))
        say(f"  arc batch sample {form}: {n} exact ({bl} with a candidate within 1e-3 px)")
    check_borderline_counts(outs["batched"], oracle_lib, imgs, sp, Fs)
    for k in ("query", "match", "d1", "d2", "offset", "n_comparisons", "n_borderline",
              "all_count"):
        a, b = getattr(outs["batched"], k).cpu(), getattr(outs["plain"], k).cpu()
        n = int(outs["batched"].offset[-1]) if k in ("query", "match", "d1", "d2") else a.shape[0]
        assert np.array_equal(a[:n].numpy(), b[:n].numpy()), k


def test_arc_batch_full_as_benchmarked(sfm, oracle_lib):
    """The whole 500-pair batch in the launch configuration bench.py times
    (one batched call on a PairBatch, default tuning, no per-query outputs):
    every pair against the oracle."""
    import bench
    import torch
    images, pairs, Fs, _ = bench.arc_batch_workload()
    m = sfm.Matcher().register(images)
    out = m.buffers(pairs)
    batch = sfm.PairBatch(pairs, Fs)
    st = torch.cuda.current_stream()
    sfm.sfm_guided_match(m.ctx, batch, None, out, sfm.options(), st)
    sfm.sfm_sync(m.ctx, st)
    say(f"  500-pair batch: {int(out.offset[-1])} matches, tuning {sfm.sfm_get_tuning(m.ctx)}")
    ores = oracle_lib.match(images, pairs, Fs)
    n, bl = compare_all(out, ores, len(pairs))
    gbl = check_borderline_counts(out, oracle_lib, images, pairs, Fs)
    err, nslots = sfm.sfm_band_error(m.ctx, batch)
    say(f"  500-pair batch: {n} queries exact ({bl} with a candidate within 1e-3 px), "
        f"{int(gbl.sum())} slots decided in FP64; max |e32 - e64| = {err:.3e} px over {nslots} "
        f"slots within 2d")
    assert 0.0 < err <= FP32_ERR_PX
    m.close()


def test_bruteforce_equals_infinite_band(sfm, oracle_lib):
    xy_a, desc_a, xy_b, desc_b, F = random_pair(1500, 1800, seed=21)
    imgs = [(xy_a, desc_a), (xy_b, desc_b)]
    m = sfm.Matcher().register(imgs)
    bf = m.match([(0, 1, 4.0)], None, form="bruteforce", emit_all=True)
    inf = m.match([(0, 1, np.inf)], [F], emit_all=True)
    ores = oracle_lib.match(imgs, [(0, 1, np.inf)], [F])
    compare_all(bf, ores, 1)
    compare_all(inf, ores, 1)
    assert int(bf.n_comparisons[0]) == 1500 * 1800


@pytest.mark.parametrize("na,nb", [(0, 50), (50, 0), (1, 1), (31, 2), (33, 700), (97, 1), (2100, 3000)])
def test_ragged_and_empty(sfm, oracle_lib, na, nb):
    xy_a, desc_a, xy_b, desc_b, F = random_pair(na, nb, seed=na * 7 + nb)
    imgs = [(xy_a, desc_a), (xy_b, desc_b)]
    for band in (4.0, 30.0):
        _, out, ores = run_both(sfm, oracle_lib, imgs, [(0, 1, band), (1, 0, band)],
                                [F, F.T])
        compare_all(out, ores, 2)


def test_long_candidate_ranges_and_ties(sfm, oracle_lib):
    """Bands wide enough that one query tile spans more than 1024 candidates,
    and coarse descriptors with many exact distance ties."""
    xy_a, desc_a, xy_b, desc_b, F = random_pair(3000, 9000, seed=33, spread=0.05)
    desc_a //= 16
    desc_b //= 16
    imgs = [(xy_a, desc_a), (xy_b, desc_b)]
    _, out, ores = run_both(sfm, oracle_lib, imgs, [(0, 1, 80.0), (0, 1, 3.0)], [F, F])
    compare_all(out, ores, 2)


@pytest.mark.parametrize("e", [(300.0, 200.0, 1.0), (1.0, 0.3, 0.0), (0.0, 1.0, 0.0),
                               (-40.0, 380.0, 1.0), (5e7, 1e3, 1.0)])
def test_epipole_positions(sfm, oracle_lib, e):
    """Epipole inside the image (full scan), at infinity (parallel lines), just
    outside, and very far away."""
    F = translation_F(e)
    xy_a, desc_a, xy_b, desc_b, _ = random_pair(1200, 2500, seed=44)
    imgs = [(xy_a, desc_a), (xy_b, desc_b)]
    _, out, ores = run_both(sfm, oracle_lib, imgs, [(0, 1, 4.0), (0, 1, 12.0)], [F, F])
    compare_all(out, ores, 2)


def test_scaled_f_and_options(sfm, oracle_lib):
    s = scenes.make_two_view_2k()
    imgs = [(im.xy, im.desc) for im in s.images]
    Fs = [s.F * -3.7, s.F * 1e-6]
    pairs = [(0, 1, 4.0), (0, 1, 6.5)]
    _, out, ores = run_both(sfm, oracle_lib, imgs, pairs, Fs, ratio_num=81, ratio_den=100,
                            accept_single=True)
    compare_all(out, ores, 2)


def test_determinism(sfm):
    s = scenes.make_two_view_16k()
    m = sfm.Matcher().register([(im.xy, im.desc) for im in s.images])
    a = m.match(s.pairs, [s.F], emit_all=True)
    b = m.match(s.pairs, [s.F], emit_all=True)
    n = int(a.offset[-1])
    assert n == int(b.offset[-1]) and n > 0
    for k in ("query", "match", "d1", "d2"):
        assert np.array_equal(getattr(a, k)[:n].cpu().numpy(), getattr(b, k)[:n].cpu().numpy()), k
    for k in ("offset", "n_comparisons", "all_match", "all_d1", "all_d2", "all_count"):
        assert np.array_equal(getattr(a, k).cpu().numpy(), getattr(b, k).cpu().numpy()), k


def test_fast_path_equals_counting_path(sfm):
    """Without emit_all the kernel skips per-query counts; outputs must not change."""
    scene, pairs = scenes.make_arc_batch()
    sub = pairs[:10]
    used = sorted({a for a, _, _ in sub} | {b for _, b, _ in sub})
    remap = {k: i for i, k in enumerate(used)}
    m = sfm.Matcher().register([(scene.image(k).xy, scene.image(k).desc) for k in used])
    sp = [(remap[a], remap[b], band) for a, b, band in sub]
    Fs = [scene.F(a, b) for a, b, _ in sub]
    a = m.match(sp, Fs, emit_all=True)
    b = m.match(sp, Fs, emit_all=False)
    n = int(a.offset[-1])
    assert int(b.offset[-1]) == n
    for k in ("query", "match", "d1", "d2"):
        assert np.array_equal(getattr(a, k)[:n].cpu().numpy(), getattr(b, k)[:n].cpu().numpy())
    assert np.array_equal(a.n_comparisons.cpu().numpy(), b.n_comparisons.cpu().numpy())


def test_invalid_inputs_rejected(sfm):
    import torch
    m = sfm.Matcher()
    bad = np.zeros((4, 128), np.uint8)
    bad[2, 5] = 128
    with pytest.raises(sfm.SfmError) as ei:
        m.register([(np.zeros((4, 2), np.float32), bad)])
    assert ei.value.status == sfm.SFM_EINVAL
    xy_a, desc_a, xy_b, desc_b, F = random_pair(10, 10, seed=1)
    m.register([(xy_a, desc_a), (xy_b, desc_b)])
    for pairs, Fs in [([(0, 2, 4.0)], [F]), ([(0, 1, -1.0)], [F]), ([(0, 1, np.nan)], [F]),
                      ([(0, 1, 4.0)], [np.zeros((3, 3))]), ([(0, 1, 4.0)], [F * np.nan])]:
        with pytest.raises(sfm.SfmError) as ei:
            m.match(pairs, Fs)
        assert ei.value.status == sfm.SFM_EINVAL
    out = sfm.MatchBuffers(5, 1, "cuda:0")
    with pytest.raises(sfm.SfmError) as ei:
        m.match([(0, 1, 4.0)], [F], out=out)
    assert ei.value.status == sfm.SFM_ECAPACITY
    small = sfm.Matcher(workspace_budget_bytes=1024).register([(xy_a, desc_a), (xy_b, desc_b)])
    with pytest.raises(sfm.SfmError) as ei:
        small.match([(0, 1, 4.0)], [F])
    assert ei.value.status == sfm.SFM_ECAPACITY
    # The context still works after errors.
    ok = m.match([(0, 1, 4.0)], [F])
    assert int(ok.offset[-1]) >= 0
    torch.cuda.synchronize()
