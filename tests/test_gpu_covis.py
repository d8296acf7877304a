"""Candidate images (sfm_candidate_images) through the C ABI against the
oracle: bit-exact ranked lists, shared counts and unique pairs, on random
edge cases and on the three-ring (300 images) and ten-ring (1,000 images)
scenes' coarse-model visibility, with each counting method (co-observer
histogram, bit-matrix product) and the automatic choice."""
import numpy as np
import pytest

import scenes
from oracle import covis
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


def _run(sfm, m, lists, npts, T, k, with_pairs=True):
    import torch
    off, pts = scenes.visibility_csr(lists)
    d_off = torch.as_tensor(off).cuda()
    d_pts = torch.as_tensor(pts if pts.size else np.zeros(0, np.int32)).cuda()
    out = sfm.CandidateBuffers(len(lists), k, with_pairs=with_pairs)
    sfm.sfm_candidate_images(m.ctx, d_off, d_pts, npts, T, k, out)
    sfm.sfm_sync(m.ctx)
    return out


def _check(sfm, m, lists, npts, T, k):
    out = _run(sfm, m, lists, npts, T, k)
    ref, ref_pairs = covis.candidate_images(lists, npts, T, k)
    got = out.lists()
    for q in range(len(lists)):
        assert got[q] == ref[q], f"image {q}: {got[q][:5]} vs {ref[q][:5]}"
    assert [tuple(p) for p in out.unique_pairs().tolist()] == ref_pairs
    return ref_pairs


@pytest.mark.parametrize("method", [1, 2, 0])
def test_random_and_edge_cases(sfm, method):
    m = sfm.Matcher()
    sfm.sfm_set_covis_method(m.ctx, method)
    rng = np.random.default_rng(21)
    for trial in range(12):
        n = int(rng.integers(1, 70))
        npts = int(rng.integers(1, 3000))
        lists = []
        for i in range(n):
            size = int(rng.integers(0, min(npts, 600) + 1)) if rng.random() > 0.1 else 0
            lists.append(np.sort(rng.choice(npts, size=size, replace=False)).astype(np.int32))
        T = int(rng.integers(0, 10))
        k = int(rng.integers(0, n + 3))
        _check(sfm, m, lists, npts, T, k)
    # One image; points seen by one image only; top_k beyond the image count.
    _check(sfm, m, [np.arange(10, dtype=np.int32)], 10, 0, 3)
    _check(sfm, m, [np.arange(5, dtype=np.int32), np.arange(5, 10, dtype=np.int32)], 10, 0, 5)
    m.close()


@pytest.mark.parametrize("method", [1, 2])
def test_bad_inputs(sfm, method):
    m = sfm.Matcher()
    sfm.sfm_set_covis_method(m.ctx, method)
    with pytest.raises(sfm.SfmError) as e:
        _run(sfm, m, [np.zeros(0, np.int32)] * 4097, 10, 8, 2)
    assert e.value.status == sfm.SFM_EINVAL
    with pytest.raises(sfm.SfmError) as e:
        _run(sfm, m, [np.arange(5, dtype=np.int32)] * 3, 10, -1, 2)
    assert e.value.status == sfm.SFM_EINVAL
    with pytest.raises(sfm.SfmError) as e:
        sfm.sfm_set_covis_method(m.ctx, 3)
    assert e.value.status == sfm.SFM_EINVAL
    # A point id past n_points: the kernels' own checks raise the error flag.
    with pytest.raises(sfm.SfmError) as e:
        _run(sfm, m, [np.array([1, 2, 50], np.int32), np.array([1, 2], np.int32)], 10, 0, 2)
    assert e.value.status == sfm.SFM_EKERNEL
    # The context still works afterwards.
    _check(sfm, m, [np.arange(5, dtype=np.int32), np.arange(3, 9, dtype=np.int32)], 10, 0, 1)
    m.close()


@pytest.mark.parametrize("rings,top_k,method", [(3, 30, 1), (3, 30, 2), (10, 100, 1), (10, 100, 2)])
def test_scenes(sfm, rings, top_k, method):
    sc = scenes.make_three_rings() if rings == 3 else scenes.make_ten_rings()
    scenes.materialize(sc, workers=16)
    lists = scenes.visibility_lists(sc)
    npts = sc.points.shape[0]
    m = sfm.Matcher()
    sfm.sfm_set_covis_method(m.ctx, method)
    pairs = _check(sfm, m, lists, npts, 8, top_k)
    say(f"  {sc.n_images} images, {sum(len(p) for p in lists)} observations, "
        f"top {top_k}, method {method}: {len(pairs)} unique pairs, bit-exact")
    m.close()
