"""Serving on the scene of bench.py's serving run: 300 cameras on three rings
(4k-25k features per image, descriptors resident), requests drawn from
ground-truth covisibility (>= 8 shared points, top 30 per image), band 4 px,
arriving as an open-loop Poisson stream at 1,000 pairs/s.  Every served
result equals the batched form of the same pairs (rows and comparison
counts), and four equal the oracle on every query."""
import time

import numpy as np
import pytest

import scenes
from tests.gpu_util import compare_rows, say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


@pytest.fixture(scope="module")
def sfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_06235_amd as sfm
    sfm.lib()
    return sfm


def test_three_rings_open_loop_equals_batched_and_oracle(sfm, oracle_lib):
    t = time.time()
    sc = scenes.make_three_rings()
    scenes.materialize(sc, workers=16)
    pool = [(a, b, 4.0) for a, b in scenes.covisible_pairs(sc)]
    images = [(sc.image(k).xy, sc.image(k).desc) for k in range(sc.n_images)]
    say(f"  serving scene: {len(images)} cameras, {len(pool)} covisible pairs, "
        f"ready in {time.time() - t:.0f} s")
    arrivals = scenes.poisson_arrivals(1000.0, 0.3, seed=7)
    rng = np.random.default_rng(7)
    reqs = [pool[k] for k in rng.integers(0, len(pool), size=len(arrivals))]
    Fs = np.stack([sc.F(a, b) for a, b, _ in reqs])
    m = sfm.Matcher().register(images)
    cap = max(m.n_features(a) for a, _, _ in reqs)
    sfm.sfm_server_start(m.ctx, max_batch_pairs=256, max_inflight=2)
    try:
        t0 = sfm.sfm_server_now_ns() + 2_000_000
        tickets = []
        for at, r, F in zip(arrivals, reqs, Fs):
            due = t0 + int(at * 1e9)
            while sfm.sfm_server_now_ns() < due:
                pass
            tickets.append(sfm.sfm_server_submit(m.ctx, r, F, due))
        res = [sfm.sfm_server_poll(m.ctx, tk, cap, timeout_ms=60_000) for tk in tickets]
    finally:
        sfm.sfm_server_stop(m.ctx)
    assert all(r is not None and r["status"] == sfm.SFM_OK for r in res)
    lat = np.array([(r["done_ns"] - r["arrival_ns"]) / 1e6 for r in res])
    say(f"  {len(res)} requests: p50 {np.percentile(lat, 50):.3f} ms, "
        f"p99 {np.percentile(lat, 99):.3f} ms")

    out = m.match(reqs, Fs, form="batched")
    off = out.offset.cpu().numpy()
    host = [x[:int(off[-1])].cpu().numpy() for x in (out.query, out.match, out.d1, out.d2)]
    ncmp = out.n_comparisons[:len(reqs)].cpu().numpy()
    for k, r in enumerate(res):
        lo, hi = int(off[k]), int(off[k + 1])
        for key, arr in zip(("query", "match", "d1", "d2"), host):
            assert np.array_equal(r[key], arr[lo:hi]), f"request {k}: {key} differs"
        assert r["n_comparisons"] == int(ncmp[k])

    for k in np.random.default_rng(8).choice(len(reqs), 4, replace=False):
        a, b, band = reqs[k]
        o = oracle_lib.match([images[a], images[b]], [(0, 1, band)], Fs[k:k + 1]).pair(0)
        compare_rows(res[k]["query"], res[k]["match"], res[k]["d1"], res[k]["d2"], o,
                     what=f"request {k}: ")
    m.close()
