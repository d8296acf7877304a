"""Serving loop (sfm_server_*) through the C ABI: results equal the batched
form (itself checked against the oracle) and the oracle directly; error
paths; an open-loop Poisson stream completes with sane latencies."""
import numpy as np
import pytest

import scenes
from tests.gpu_util import compare_rows, say

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
def ring():
    """12 cameras on a ring, 20k points, 1k-4k features; covisible pairs."""
    centers = scenes.generator._ring(12, 20.0, 0.0)
    scene = scenes.make_multiview_scene(centers, 1000, 4000, n_points=20_000, seed=3)
    images = [(scene.image(k).xy, scene.image(k).desc) for k in range(scene.n_images)]
    pairs = [(a, b, 4.0) for a, b in scenes.covisible_pairs(scene, top_k=4)]
    Fs = np.stack([scene.F(a, b) for a, b, _ in pairs])
    say(f"  ring scene: {len(images)} images, {len(pairs)} pairs")
    return images, pairs, Fs


def collect(sfm, ctx, tickets, capacity):
    out = []
    for t in tickets:
        r = sfm.sfm_server_poll(ctx, t, capacity, timeout_ms=60_000)
        assert r is not None, "result not ready within 60 s"
        out.append(r)
    return out


def test_server_equals_batched_and_oracle(sfm, oracle_lib, ring):
    images, pairs, Fs = ring
    m = sfm.Matcher().register(images)
    ref = m.match(pairs, Fs, form="batched")
    cap = max(m.n_features(a) for a, _, _ in pairs)
    sfm.sfm_server_start(m.ctx, max_batch_pairs=5, max_inflight=2)
    try:
        tickets = [sfm.sfm_server_submit(m.ctx, p, F) for p, F in zip(pairs, Fs)]
        res = collect(sfm, m.ctx, tickets, cap)
        stats = sfm.sfm_server_stats(m.ctx)
    finally:
        sfm.sfm_server_stop(m.ctx)
    say(f"  {stats['launches']} launches for {stats['launched']} requests")
    assert stats["launched"] == len(pairs)
    assert stats["launches"] >= (len(pairs) + 4) // 5
    ncmp = ref.n_comparisons.cpu().numpy()
    for k, r in enumerate(res):
        assert r["status"] == sfm.SFM_OK
        q, mt, d1, d2 = ref.pair(k)
        assert np.array_equal(r["query"], q) and np.array_equal(r["match"], mt)
        assert np.array_equal(r["d1"], d1) and np.array_equal(r["d2"], d2)
        assert r["n_comparisons"] == int(ncmp[k])
        assert r["done_ns"] >= r["arrival_ns"] > 0
    # Two requests straight against the oracle (every query).
    for k in (0, len(pairs) - 1):
        o = oracle_lib.match(images, [pairs[k]], Fs[k:k + 1]).pair(0)
        compare_rows(res[k]["query"], res[k]["match"], res[k]["d1"], res[k]["d2"], o,
                     what=f"request {k}: ")


def test_server_errors(sfm, ring):
    images, pairs, Fs = ring
    m = sfm.Matcher().register(images)
    with pytest.raises(sfm.SfmError) as e:
        sfm.sfm_server_submit(m.ctx, pairs[0], Fs[0])
    assert e.value.status == sfm.SFM_EBUSY           # no server yet
    sfm.sfm_server_start(m.ctx, max_batch_pairs=4)
    try:
        with pytest.raises(sfm.SfmError) as e:
            sfm.sfm_server_start(m.ctx)
        assert e.value.status == sfm.SFM_EBUSY
        for bad_pair, bad_F in (((0, len(images), 4.0), Fs[0]), ((0, 1, -1.0), Fs[0]),
                                (pairs[0], np.zeros(9)), (pairs[0], np.full(9, np.nan))):
            with pytest.raises(sfm.SfmError) as e:
                sfm.sfm_server_submit(m.ctx, bad_pair, bad_F)
            assert e.value.status == sfm.SFM_EINVAL
        with pytest.raises(sfm.SfmError) as e:
            sfm.sfm_server_poll(m.ctx, 10**9, 16, timeout_ms=0)
        assert e.value.status == sfm.SFM_ENOTFOUND
        # A burst with one bad request queues nothing; an empty burst is a no-op.
        before = sfm.sfm_server_stats(m.ctx)
        with pytest.raises(sfm.SfmError) as e:
            sfm.sfm_server_submit_batch(m.ctx, [pairs[0], (0, 1, -2.0), pairs[1]], Fs[:3])
        assert e.value.status == sfm.SFM_EINVAL
        assert sfm.sfm_server_submit_batch(m.ctx, [], np.zeros((0, 9))).size == 0
        after = sfm.sfm_server_stats(m.ctx)
        assert after["launched"] + after["waiting"] == before["launched"] + before["waiting"]
        t = sfm.sfm_server_submit(m.ctx, pairs[0], Fs[0])
        # Too small a buffer: reported, and the result stays collectable.
        with pytest.raises(sfm.SfmError) as e:
            sfm.sfm_server_poll(m.ctx, t, 0, timeout_ms=60_000)
        assert e.value.status == sfm.SFM_ECAPACITY
        r = sfm.sfm_server_poll(m.ctx, t, m.n_features(pairs[0][0]), timeout_ms=0)
        assert r is not None and r["status"] == sfm.SFM_OK and r["query"].size > 0
        with pytest.raises(sfm.SfmError) as e:
            sfm.sfm_server_poll(m.ctx, t, 16, timeout_ms=0)
        assert e.value.status == sfm.SFM_ENOTFOUND    # collected once
    finally:
        sfm.sfm_server_stop(m.ctx)
    with pytest.raises(sfm.SfmError) as e:
        sfm.sfm_server_stop(m.ctx)
    assert e.value.status == sfm.SFM_EBUSY


def test_server_open_loop(sfm, ring):
    """300 requests at 1,000 pairs/s (Poisson, open loop): every result
    arrives, arrival <= done, and a stop with requests in flight drains them."""
    images, pairs, Fs = ring
    m = sfm.Matcher().register(images)
    cap = max(m.n_features(a) for a, _, _ in pairs)
    arrivals = scenes.poisson_arrivals(1000.0, 0.3, seed=5)
    rng = np.random.default_rng(5)
    pick = rng.integers(0, len(pairs), size=len(arrivals))
    sfm.sfm_server_start(m.ctx, max_batch_pairs=64, max_inflight=2)
    tickets = []
    try:
        t0 = sfm.sfm_server_now_ns() + 2_000_000
        for t, k in zip(arrivals, pick):
            due = t0 + int(t * 1e9)
            while sfm.sfm_server_now_ns() < due:
                pass
            tickets.append(sfm.sfm_server_submit(m.ctx, pairs[k], Fs[k], due))
        res = collect(sfm, m.ctx, tickets, cap)
        # A last burst that stop() must drain.
        for k in range(8):
            sfm.sfm_server_submit(m.ctx, pairs[k % len(pairs)], Fs[k % len(pairs)])
    finally:
        sfm.sfm_server_stop(m.ctx)
    lat = np.array([(r["done_ns"] - r["arrival_ns"]) / 1e6 for r in res])
    say(f"  {len(res)} requests: p50 {np.percentile(lat, 50):.3f} ms, p99 {np.percentile(lat, 99):.3f} ms")
    assert all(r["status"] == sfm.SFM_OK for r in res)
    assert np.all(lat > 0)


@pytest.mark.parametrize("max_batch_pairs,max_inflight", [(1, 1), (3, 4), (64, 8)])
def test_server_configurations(sfm, ring, max_batch_pairs, max_inflight):
    """Batch and slot limits change batching, never results."""
    images, pairs, Fs = ring
    m = sfm.Matcher().register(images)
    ref = m.match(pairs, Fs, form="batched")
    cap = max(m.n_features(a) for a, _, _ in pairs)
    sfm.sfm_server_start(m.ctx, max_batch_pairs=max_batch_pairs, max_inflight=max_inflight)
    try:
        tickets = [sfm.sfm_server_submit(m.ctx, p, F) for p, F in zip(pairs, Fs)]
        res = collect(sfm, m.ctx, tickets, cap)
        stats = sfm.sfm_server_stats(m.ctx)
    finally:
        sfm.sfm_server_stop(m.ctx)
    assert stats["launches"] >= (len(pairs) + max_batch_pairs - 1) // max_batch_pairs
    for k, r in enumerate(res):
        q, mt, d1, d2 = ref.pair(k)
        assert r["status"] == sfm.SFM_OK
        assert np.array_equal(r["query"], q) and np.array_equal(r["match"], mt)
        assert np.array_equal(r["d1"], d1) and np.array_equal(r["d2"], d2)


def test_server_capacity_and_empty_images(sfm, ring):
    """A request larger than a slot fails alone with SFM_ECAPACITY; pairs with
    an empty image succeed with no matches; the rest are unaffected."""
    images, pairs, Fs = ring
    empty = (np.zeros((0, 2), np.float32), np.zeros((0, 128), np.uint8))
    m = sfm.Matcher().register(images + [empty])
    e = len(images)
    small = min(m.n_features(a) for a, _, _ in pairs)
    big = max(range(len(pairs)), key=lambda k: m.n_features(pairs[k][0]))
    ok = min(range(len(pairs)), key=lambda k: m.n_features(pairs[k][0]))
    sfm.sfm_server_start(m.ctx, max_batch_pairs=4, max_batch_queries=small)
    try:
        t_big = sfm.sfm_server_submit(m.ctx, pairs[big], Fs[big])
        t_ok = sfm.sfm_server_submit(m.ctx, pairs[ok], Fs[ok])
        t_e1 = sfm.sfm_server_submit(m.ctx, (e, 0, 4.0), Fs[0])
        t_e2 = sfm.sfm_server_submit(m.ctx, (0, e, 4.0), Fs[0])
        r_big = sfm.sfm_server_poll(m.ctx, t_big, small, timeout_ms=60_000)
        r_ok = sfm.sfm_server_poll(m.ctx, t_ok, small, timeout_ms=60_000)
        r_e1 = sfm.sfm_server_poll(m.ctx, t_e1, small, timeout_ms=60_000)
        r_e2 = sfm.sfm_server_poll(m.ctx, t_e2, small, timeout_ms=60_000)
    finally:
        sfm.sfm_server_stop(m.ctx)
    if m.n_features(pairs[big][0]) > small:
        assert r_big["status"] == sfm.SFM_ECAPACITY
    assert r_ok["status"] == sfm.SFM_OK
    q, mt, _, _ = m.match([pairs[ok]], Fs[ok:ok + 1], form="batched").pair(0)
    assert np.array_equal(r_ok["query"], q) and np.array_equal(r_ok["match"], mt)
    for r in (r_e1, r_e2):
        assert r["status"] == sfm.SFM_OK and r["query"].size == 0 and r["n_comparisons"] == 0


def test_server_burst_submit(sfm, ring):
    """A burst submitted in one call: consecutive tickets, one arrival time,
    results equal the batched form."""
    images, pairs, Fs = ring
    m = sfm.Matcher().register(images)
    ref = m.match(pairs, Fs, form="batched")
    cap = max(m.n_features(a) for a, _, _ in pairs)
    sfm.sfm_server_start(m.ctx, max_batch_pairs=7, max_inflight=3)
    try:
        tickets = sfm.sfm_server_submit_batch(m.ctx, pairs, Fs)
        res = collect(sfm, m.ctx, [int(t) for t in tickets], cap)
    finally:
        sfm.sfm_server_stop(m.ctx)
    assert np.array_equal(np.diff(tickets.astype(np.int64)), np.ones(len(pairs) - 1))
    assert len({r["arrival_ns"] for r in res}) == 1
    for k, r in enumerate(res):
        q, mt, d1, d2 = ref.pair(k)
        assert r["status"] == sfm.SFM_OK
        assert np.array_equal(r["query"], q) and np.array_equal(r["match"], mt)
        assert np.array_equal(r["d1"], d1) and np.array_equal(r["d2"], d2)


def test_server_admission_by_workspace_budget(sfm, ring):
    """A context whose workspace budget holds about three requests: a burst of
    every pair is split into launches that fit, none fails, and the results
    equal the batched form on a context with the default budget."""
    images, pairs, Fs = ring
    ref_m = sfm.Matcher().register(images)
    ref = ref_m.match(pairs, Fs, form="batched")
    sizes = [sfm.sfm_workspace_size(ref_m.ctx, [p]) for p in pairs]
    per = max(sizes)
    m = sfm.Matcher(workspace_budget_bytes=3 * per).register(images)
    cap = max(m.n_features(a) for a, _, _ in pairs)
    sfm.sfm_server_start(m.ctx, max_batch_pairs=256, max_inflight=2)
    try:
        tickets = sfm.sfm_server_submit_batch(m.ctx, pairs, Fs)
        res = collect(sfm, m.ctx, [int(t) for t in tickets], cap)
        stats = sfm.sfm_server_stats(m.ctx)
    finally:
        sfm.sfm_server_stop(m.ctx)
    say(f"  budget {3 * per} B: {len(pairs)} requests in {stats['launches']} launches")
    # Every launch fitted the budget (none failed), so the burst took at
    # least about its summed workspace over the budget.
    assert stats["launches"] >= max(2, sum(sizes) // (3 * per) // 2)
    for k, r in enumerate(res):
        q, mt, d1, d2 = ref.pair(k)
        assert r["status"] == sfm.SFM_OK, (k, r["status"])
        assert np.array_equal(r["query"], q) and np.array_equal(r["match"], mt)
        assert np.array_equal(r["d1"], d1) and np.array_equal(r["d2"], d2)
    # A request larger than the whole budget fails alone.
    small = sfm.Matcher(workspace_budget_bytes=per // 4).register(images)
    sfm.sfm_server_start(small.ctx, max_batch_pairs=8)
    try:
        t = sfm.sfm_server_submit(small.ctx, pairs[0], Fs[0])
        r = sfm.sfm_server_poll(small.ctx, t, cap, timeout_ms=60_000)
    finally:
        sfm.sfm_server_stop(small.ctx)
    assert r["status"] == sfm.SFM_ECAPACITY
    for mm in (m, small, ref_m):
        mm.close()


def test_server_stop_while_polling(sfm, ring):
    """A thread blocked in poll while another stops the server gets either its
    result or SFM_EBUSY, never a crash; stop drains what was submitted."""
    import threading
    images, pairs, Fs = ring
    m = sfm.Matcher().register(images)
    cap = max(m.n_features(a) for a, _, _ in pairs)
    outcomes = []
    for trial in range(3):
        sfm.sfm_server_start(m.ctx, max_batch_pairs=4, max_inflight=1)
        tickets = [int(t) for t in sfm.sfm_server_submit_batch(m.ctx, pairs, Fs)]

        def poller():
            for t in tickets:
                try:
                    r = sfm.sfm_server_poll(m.ctx, t, cap, timeout_ms=-1)
                    outcomes.append(r["status"])
                except sfm.SfmError as e:
                    outcomes.append(e.status)

        th = threading.Thread(target=poller)
        th.start()
        sfm.sfm_server_stop(m.ctx)
        th.join(timeout=60)
        assert not th.is_alive()
    assert set(outcomes) <= {sfm.SFM_OK, sfm.SFM_EBUSY}
    say(f"  {outcomes.count(sfm.SFM_OK)} collected, {outcomes.count(sfm.SFM_EBUSY)} after stop")
    m.close()


def test_server_concurrent_clients(sfm, ring):
    """Four client threads submit and collect at once."""
    import threading
    images, pairs, Fs = ring
    m = sfm.Matcher().register(images)
    ref = m.match(pairs, Fs, form="batched")
    cap = max(m.n_features(a) for a, _, _ in pairs)
    errors = []
    sfm.sfm_server_start(m.ctx, max_batch_pairs=16, max_inflight=2)

    def client(offset):
        try:
            for k in range(offset, len(pairs), 4):
                t = sfm.sfm_server_submit(m.ctx, pairs[k], Fs[k])
                r = sfm.sfm_server_poll(m.ctx, t, cap, timeout_ms=60_000)
                q, mt, d1, d2 = ref.pair(k)
                if not (r["status"] == sfm.SFM_OK and np.array_equal(r["query"], q)
                        and np.array_equal(r["match"], mt)):
                    errors.append(k)
        except Exception as exc:   # surfaced below
            errors.append(repr(exc))

    threads = [threading.Thread(target=client, args=(i,)) for i in range(4)]
    try:
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=120)
    finally:
        sfm.sfm_server_stop(m.ctx)
    assert not errors, errors
