"""Stress serving: the 1,000-camera scene (10 rings x 100, 8k-40k features per
image, about 2.65 GB of descriptors resident on the device) and 20,000
covisible-pair requests in 10 bursts of 2,000, each burst released at once
when the server has admitted the previous one; band half-widths are drawn per
request from 2-8 px, so both the sizes and the bands of a launch are uneven.

Every served result must equal the batched form on the same burst (rows and
comparison counts); a sample equals the pair run alone (plain form), and the
two smallest requests and six random ones equal the oracle on every query."""
import time

import numpy as np
import pytest

import scenes
from tests.gpu_util import compare_rows, say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

N_REQUESTS = 20_000
BURST = 2_000


@pytest.fixture(scope="module")
def sfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_06235_amd as sfm
    sfm.lib()
    return sfm


@pytest.fixture(scope="module")
def stress(sfm):
    t = time.time()
    sc = scenes.make_ten_rings()
    say(f"  stress scene: {sc.n_images} cameras, generating images")
    scenes.materialize(sc, workers=16,
                       progress=lambda k, n: say(f"    {k}/{n} images ({time.time() - t:.0f} s)"))
    reqs = scenes.stress_requests(sc, N_REQUESTS)
    Fs = np.stack([sc.F(a, b) for a, b, _ in reqs])
    images = [(sc.image(k).xy, sc.image(k).desc) for k in range(sc.n_images)]
    nfeat = sum(xy.shape[0] for xy, _ in images)
    say(f"  {nfeat} features ({nfeat * 136 / 1e9:.2f} GB with keypoints), "
        f"{len(reqs)} requests, scene ready in {time.time() - t:.0f} s")
    m = sfm.Matcher().register(images)
    yield images, reqs, Fs, m
    m.close()


def _serve(sfm, m, reqs, Fs, cap):
    """All requests in bursts; returns the results in request order."""
    sfm.sfm_server_start(m.ctx, max_batch_pairs=256, max_inflight=2)
    tickets = []
    try:
        for s in range(0, len(reqs), BURST):
            e = min(s + BURST, len(reqs))
            tickets += [int(t) for t in sfm.sfm_server_submit_batch(m.ctx, reqs[s:e], Fs[s:e])]
            # The next burst is released once this one is admitted (launched).
            t_end = time.time() + 120
            while sfm.sfm_server_stats(m.ctx)["launched"] < len(tickets):
                assert time.time() < t_end, "burst not admitted within 120 s"
                time.sleep(0.0005)
        res = []
        for t in tickets:
            r = sfm.sfm_server_poll(m.ctx, t, cap, timeout_ms=120_000)
            assert r is not None, "result not ready within 120 s"
            res.append(r)
        stats = sfm.sfm_server_stats(m.ctx)
    finally:
        sfm.sfm_server_stop(m.ctx)
    return res, stats


def test_stress_bursts_equal_batched_alone_and_oracle(sfm, oracle_lib, stress):
    images, reqs, Fs, m = stress
    cap = max(m.n_features(a) for a, _, _ in reqs)
    res, stats = _serve(sfm, m, reqs, Fs, cap)
    assert all(r["status"] == sfm.SFM_OK for r in res)
    t0 = min(r["arrival_ns"] for r in res)
    t1 = max(r["done_ns"] for r in res)
    cmp_total = sum(r["n_comparisons"] for r in res)
    say(f"  served {len(res)} requests in {stats['launches']} launches, "
        f"{(t1 - t0) / 1e6:.1f} ms wall, {cmp_total / ((t1 - t0) / 1e9):.3e} comparisons/s")

    # Every result against the batched form of its burst.
    for s in range(0, len(reqs), BURST):
        e = min(s + BURST, len(reqs))
        out = m.match(reqs[s:e], Fs[s:e], form="batched")
        off = out.offset.cpu().numpy()
        host = [t[:int(off[-1])].cpu().numpy() for t in (out.query, out.match, out.d1, out.d2)]
        ncmp = out.n_comparisons[:e - s].cpu().numpy()
        for p in range(e - s):
            r = res[s + p]
            lo, hi = int(off[p]), int(off[p + 1])
            for key, arr in zip(("query", "match", "d1", "d2"), host):
                assert np.array_equal(r[key], arr[lo:hi]), f"request {s + p}: {key} differs"
            assert r["n_comparisons"] == int(ncmp[p]), f"request {s + p}: comparisons differ"
        del out

    # A sample alone, one pair per launch.
    rng = np.random.default_rng(3)
    for k in rng.choice(len(reqs), size=16, replace=False):
        q, mt, d1, d2 = m.match([reqs[k]], Fs[k:k + 1], form="plain").pair(0)
        r = res[k]
        assert np.array_equal(r["query"], q) and np.array_equal(r["match"], mt)
        assert np.array_equal(r["d1"], d1) and np.array_equal(r["d2"], d2)

    # The two smallest requests and six drawn at random against the oracle
    # (every query).
    sizes = [images[a][0].shape[0] * images[b][0].shape[0] for a, b, _ in reqs]
    picks = list(np.argsort(sizes)[:2]) + list(np.random.default_rng(4).choice(len(reqs), 6,
                                                                             replace=False))
    for k in picks:
        a, b, band = reqs[k]
        o = oracle_lib.match([images[a], images[b]], [(0, 1, band)], Fs[k:k + 1]).pair(0)
        compare_rows(res[k]["query"], res[k]["match"], res[k]["d1"], res[k]["d2"], o,
                     what=f"request {k}: ")
        say(f"  request {k} ({images[a][0].shape[0]} x {images[b][0].shape[0]}, band {band:.2f}): "
            f"all {o['match'].shape[0]} queries equal the oracle")
