"""Pins of the staged-matching oracle (Section 4) to what the paper fixes.

Descriptors are uniform random bytes, for which the ratio test accepts no
pair by chance (the nearest and second-nearest of hundreds of random
neighbours lie within a few percent of each other, far from the 0.64 ratio
of squared distances).  Planted matches are exact copies of a feature of a
into b, so each is accepted with D1 = 0 and the expected result of every
rule of the scheme is known without running any matcher: which stage a
planted feature falls in follows from its scale rank alone.  Features are
stored in shuffled order, so the scale ranking itself is under test."""
import numpy as np

from oracle.preemptive import preemptive_match, stage_sizes


def test_stage_sizes_follow_the_percentages():
    # 10% of the queries, 20% of the targets, the next 10% in stage 2.
    assert stage_sizes(1000, 1000) == (False, 100, 200, 100)
    assert stage_sizes(5000, 12000) == (False, 500, 2400, 500)
    # Rounded up.
    assert stage_sizes(1001, 1003) == (False, 101, 201, 101)
    # Fewer than 1000 features in either image: all features, one stage.
    assert stage_sizes(999, 5000) == (True, 999, 5000, 0)
    assert stage_sizes(5000, 999) == (True, 5000, 999, 0)
    # Stage 2 is cut at the end of the image.
    assert stage_sizes(10, 10, query_pct=60, small_image=0) == (False, 6, 2, 4)
    assert stage_sizes(0, 10, small_image=0) == (False, 0, 2, 0)


def _pair(rng, na, nb):
    da = rng.integers(0, 128, size=(na, 128), dtype=np.uint8)
    db = rng.integers(0, 128, size=(nb, 128), dtype=np.uint8)
    sa = rng.permutation(na).astype(np.float32)          # distinct scales, shuffled
    sb = rng.permutation(nb).astype(np.float32)
    xy = lambda n: rng.uniform(0, 1000, size=(n, 2)).astype(np.float32)
    return [xy(na), da, sa], [xy(nb), db, sb]


def _by_rank(scale, lo, hi):
    """Features whose scale rank (0 = largest) lies in [lo, hi)."""
    rank = np.empty(len(scale), np.int64)
    rank[np.argsort(-scale, kind="stable")] = np.arange(len(scale))
    return np.nonzero((rank >= lo) & (rank < hi))[0]


def _plant(rng, A, B, a_lo, a_hi, b_lo, b_hi, k, used):
    """Copy k features of a (scale rank in [a_lo, a_hi)) onto k features of b
    (rank in [b_lo, b_hi)); returns the planted (i, j)."""
    ia = rng.permutation([i for i in _by_rank(A[2], a_lo, a_hi) if i not in used[0]])[:k]
    jb = rng.permutation([j for j in _by_rank(B[2], b_lo, b_hi) if j not in used[1]])[:k]
    for i, j in zip(ia, jb):
        B[1][j] = A[1][i]
        used[0].add(int(i)); used[1].add(int(j))
    return {(int(i), int(j)) for i, j in zip(ia, jb)}


def _found(res):
    assert np.all(res["d1"] == 0)
    return set(zip(res["query"].tolist(), res["match"].tolist()))


def _setup(seed, k1, k2, na=2000, nb=2400):
    rng = np.random.default_rng(seed)
    A, B = _pair(rng, na, nb)
    used = (set(), set())
    q, r = na // 10, nb // 5
    p1 = _plant(rng, A, B, 0, q, 0, r, k1, used)              # stage 1
    p2 = _plant(rng, A, B, q, 2 * q, 0, r, k2, used)          # stage 2
    miss_b = _plant(rng, A, B, 0, q, r, nb, 3, used)          # target outside the 20%
    miss_a = _plant(rng, A, B, 2 * q, na, 0, r, 3, used)      # query beyond stage 2
    return A, B, p1, p2, miss_b | miss_a


def test_no_match_among_random_descriptors():
    rng = np.random.default_rng(3)
    A, B = _pair(rng, 1500, 1500)
    res = preemptive_match([A, B], [(0, 1)], min_matches=-1)[0]
    assert res["stages"] == 2 and len(res["query"]) == 0
    assert res["n_comparisons"] == 2 * 150 * 300


def test_four_matches_do_not_open_stage_two():
    A, B, p1, p2, miss = _setup(1, 4, 6)
    res = preemptive_match([A, B], [(0, 1)])[0]
    assert res["stages"] == 1
    assert _found(res) == p1
    assert res["n_comparisons"] == 200 * 480


def test_five_matches_open_stage_two():
    A, B, p1, p2, miss = _setup(2, 5, 6)
    res = preemptive_match([A, B], [(0, 1)])[0]
    assert res["stages"] == 2
    assert _found(res) == p1 | p2
    # Stage-1 rows first, each stage in scale-rank order of its queries.
    rank = np.empty(2000, np.int64)
    rank[np.argsort(-A[2], kind="stable")] = np.arange(2000)
    r = rank[res["query"]]
    assert np.all(np.diff(r) > 0) and np.all(r[:5] < 200) and np.all(r[5:] >= 200)
    assert res["n_comparisons"] == 2 * 200 * 480


def test_enough_matches_stop_early():
    A, B, p1, p2, miss = _setup(4, 7, 6)
    res = preemptive_match([A, B], [(0, 1)], enough=7)[0]
    assert res["stages"] == 1 and _found(res) == p1
    res = preemptive_match([A, B], [(0, 1)], enough=8)[0]
    assert res["stages"] == 2 and _found(res) == p1 | p2


def test_small_image_is_matched_whole():
    A, B, p1, p2, miss = _setup(5, 2, 3, na=900, nb=2400)
    res = preemptive_match([A, B], [(0, 1)])[0]
    assert res["stages"] == 0
    assert _found(res) == p1 | p2 | miss
    assert res["n_comparisons"] == 900 * 2400
    # Rows in the scale-rank order of their queries, as for staged pairs.
    rank = np.empty(900, np.int64)
    rank[np.argsort(-A[2], kind="stable")] = np.arange(900)
    assert np.all(np.diff(rank[res["query"]]) > 0)


def test_pair_direction_and_several_pairs():
    A, B, p1, p2, miss = _setup(6, 5, 2)
    res = preemptive_match([A, B], [(0, 1), (1, 0), (0, 0)])
    assert _found(res[0]) == p1 | p2
    # b -> a: b's top 10% (then the next 10%) against a's top 20%.
    ra = set(_by_rank(A[2], 0, 400).tolist())
    b1, b2 = set(_by_rank(B[2], 0, 240).tolist()), set(_by_rank(B[2], 240, 480).tolist())
    want1 = {(j, i) for i, j in p1 | p2 | miss if j in b1 and i in ra}
    want2 = {(j, i) for i, j in p1 | p2 | miss if j in b2 and i in ra}
    assert res[1]["stages"] == (2 if len(want1) > 4 else 1)
    assert _found(res[1]) == (want1 | want2 if len(want1) > 4 else want1)
    # A pair of an image with itself: every stage-1 query finds itself.
    assert res[2]["stages"] == 2
    assert len(res[2]["query"]) == 400
    assert np.array_equal(res[2]["query"], res[2]["match"])


def test_edge_cases():
    """An image without features is below any positive size limit: its pairs
    are matched whole and find nothing.  With query_pct = 100 stage 1 takes
    every query, so stage 2 has none and never runs."""
    rng = np.random.default_rng(8)
    A, B = _pair(rng, 1200, 1500)
    empty = [np.zeros((0, 2), np.float32), np.zeros((0, 128), np.uint8), np.zeros(0, np.float32)]
    r = preemptive_match([A, B, empty], [(0, 2), (2, 1)])
    assert [x["stages"] for x in r] == [0, 0]
    assert all(len(x["query"]) == 0 and x["n_comparisons"] == 0 for x in r)
    for i in range(10):                          # ten planted copies among the top 100%
        B[1][i] = A[1][i]
    r = preemptive_match([A, B], [(0, 1)], query_pct=100, target_pct=100, min_matches=0)[0]
    assert r["stages"] == 1 and len(r["query"]) == 10
    assert r["n_comparisons"] == 1200 * 1500
