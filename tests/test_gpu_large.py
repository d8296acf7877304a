"""Large targets: the paths that only images beyond ~25k features take.

* 3,000 queries against 70,000 targets: the bin count clamps at 8192, the
  target sort no longer fits the LDS permutation (direct scatter), and the
  third and later rounds of items recompute their keys.
* 40,000 x 40,000 (the largest serving images): full-size query sort and
  tiles, checked on every query.
Both against the oracle, every query bit-exact, with the FP32 distance error
measured on the evaluated slots."""
import numpy as np
import pytest

from tests.fixtures import random_pair
from tests.gpu_util import FP32_ERR_PX, compare_all, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_06235_amd as sfm
    sfm.lib()
    return sfm


def _run(sfm, oracle_lib, n_a, n_b, seed, band):
    xy_a, desc_a, xy_b, desc_b, F = random_pair(n_a, n_b, seed, spread=0.6)
    images = [(xy_a, desc_a), (xy_b, desc_b)]
    pairs = [(0, 1, band)]
    say(f"  {n_a} x {n_b}, band {band}")
    ores = oracle_lib.match(images, pairs, [F])
    m = sfm.Matcher().register(images)
    for form in ("batched", "plain"):
        out = m.match(pairs, [F], form=form, emit_all=True)
        n, bl = compare_all(out, ores, 1)
        say(f"    {form}: {n} exact ({bl} with a candidate within 1e-3 px of the edge), "
            f"{int(out.n_borderline[0])} slots decided in FP64, "
            f"comparisons {int(ores.n_comparisons[0])}")
    err, nslots = sfm.sfm_band_error(m.ctx, pairs, [F])
    say(f"    max |e32 - e64| = {err:.3e} px over {nslots} slots within 2d")
    assert err <= FP32_ERR_PX
    m.close()


def test_70k_targets(sfm, oracle_lib):
    _run(sfm, oracle_lib, 3000, 70000, seed=21, band=3.0)


def test_40k_by_40k(sfm, oracle_lib):
    _run(sfm, oracle_lib, 40000, 40000, seed=22, band=2.0)
