"""Exhaustive matching (sfm_bruteforce_match) against the oracle at an infinite
band, bit-exact on every query: ragged and empty sizes around the 256-query
blocks and 1024-target slices of the work items, many pairs of different sizes
in one call, exact distance ties inside and across slices (the lowest index in
b must win and D2 must equal D1), the ratio options, and the 16,000-feature
pair of the context comparison."""
import numpy as np
import pytest

from tests.fixtures import random_pair
from tests.gpu_util import compare_all, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_06235_amd as sfm
    sfm.lib()   # raises when the library is not built
    return sfm


def run(sfm, oracle, imgs, pairs, emit_all=True, **kw):
    """Exhaustive matching of `pairs` (a, b) on the GPU and in the oracle."""
    say(f"  exhaustive: {len(pairs)} pairs, sizes "
        f"{[(imgs[a][0].shape[0], imgs[b][0].shape[0]) for a, b in pairs[:6]]} emit_all={emit_all} {kw}")
    F = random_pair(1, 1, seed=0)[4]
    m = sfm.Matcher().register(imgs)
    out = m.match([(a, b, 0.0) for a, b in pairs], None, form="bruteforce", emit_all=emit_all, **kw)
    ores = oracle.match(imgs, [(a, b, np.inf) for a, b in pairs], np.stack([F] * len(pairs)),
                        ignore_band=True, **kw)
    n, _ = compare_all(out, ores, len(pairs))
    m.close()
    return n, ores


def image(n, seed, coarse=False):
    xy_a, desc_a, _, _, _ = random_pair(n, 0, seed=seed)
    if coarse:
        desc_a //= 16
    return (xy_a, desc_a)


def test_exhaustive_ragged_sizes(sfm, oracle_lib):
    sizes = [0, 1, 2, 31, 33, 255, 256, 257, 700, 1023, 1024, 1025, 2049, 3000]
    imgs = [image(n, seed=100 + k) for k, n in enumerate(sizes)]
    rng = np.random.default_rng(5)
    pairs = [(0, 5), (5, 0), (1, 1), (1, 2), (2, 1), (3, 9), (9, 10), (10, 11), (11, 12),
             (12, 13), (13, 12), (7, 8), (8, 7), (6, 11)]
    pairs += [tuple(int(x) for x in rng.integers(0, len(sizes), 2)) for _ in range(26)]
    n, _ = run(sfm, oracle_lib, imgs, pairs)
    say(f"  ragged sizes: {n} queries exact over {len(pairs)} pairs")
    run(sfm, oracle_lib, imgs, pairs[:14], emit_all=False)


def test_exhaustive_ties_across_slices(sfm, oracle_lib):
    """Coarse descriptors (values 0..7) tie on most distances; planted copies
    of target rows in later slices tie the smallest distance across slices."""
    qa = image(600, seed=7, coarse=True)
    tb = image(4100, seed=8, coarse=True)
    xa, da = qa[0], qa[1].copy()
    xb, db = tb[0], tb[1].copy()
    for src, dst in ((10, 1030), (10, 2050), (10, 4099), (500, 1024), (999, 3072)):
        db[dst] = db[src]
    for k, src in enumerate((10, 500, 999, 1030, 4099)):
        da[k] = db[src]               # D1 = 0, shared by the copies
    n, ores = run(sfm, oracle_lib, [(xa, da), (xb, db)], [(0, 1), (1, 0)])
    o = ores.pair(0)
    assert o["match"][0] == 10 and o["d1"][0] == 0 and o["d2"][0] == 0
    assert o["match"][1] == 500 and o["match"][2] == 999
    say(f"  ties across slices: {n} queries exact")


def test_exhaustive_many_pairs(sfm, oracle_lib):
    """More pairs than one workgroup resets counters for, and more than the
    emission kernel sums in one pass."""
    rng = np.random.default_rng(11)
    sizes = rng.integers(20, 400, 48)
    imgs = [image(int(n), seed=200 + k) for k, n in enumerate(sizes)]
    pairs = [tuple(int(x) for x in rng.integers(0, len(sizes), 2)) for _ in range(1100)]
    n, _ = run(sfm, oracle_lib, imgs, pairs)
    say(f"  {len(pairs)} pairs: {n} queries exact")


@pytest.mark.parametrize("kw", [dict(ratio_num=80, ratio_den=100, accept_single=True),
                                dict(ratio_num=1, ratio_den=1)])
def test_exhaustive_ratio_options(sfm, oracle_lib, kw):
    imgs = [image(n, seed=300 + k) for k, n in enumerate([1, 1200, 3, 2100])]
    run(sfm, oracle_lib, imgs, [(1, 0), (0, 1), (1, 2), (3, 1), (1, 3), (2, 2)], **kw)


def test_exhaustive_16k_pair(sfm, oracle_lib):
    """The context pair (16,000 features per image), every query against the oracle."""
    import scenes
    s = scenes.make_two_view_16k()
    imgs = [(im.xy, im.desc) for im in s.images]
    n, ores = run(sfm, oracle_lib, imgs, [(0, 1)])
    say(f"  16k pair: {n} queries exact, {int(ores.n_accepted[0])} accepted")
