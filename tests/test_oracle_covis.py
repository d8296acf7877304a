"""Pins for the candidate-image oracle (Section 6.1) against what the
definitions fix, by other means than the oracle's sparse product."""
import itertools

import numpy as np

from oracle import covis


def _planted():
    """Image 0 observes points 0..99; image i (1..5) shares exactly
    (9, 8, 12, 12, 20)[i-1] of them and observes other, private points."""
    shared = [9, 8, 12, 12, 20]
    lists = [list(range(100))]
    nxt = 1000
    for m in shared:
        own = list(range(m)) + list(range(nxt, nxt + 30))
        nxt += 30
        lists.append(own)
    return lists, nxt


def test_planted_threshold_ranking_and_ties():
    lists, npts = _planted()
    out, pairs = covis.candidate_images(lists, npts, threshold=8, top_k=3)
    # 8 shared points is not more than T = 8; 12 and 12 tie: lower index first.
    assert out[0] == [(5, 20), (3, 12), (4, 12)]
    out10, pairs10 = covis.candidate_images(lists, npts, threshold=8, top_k=10)
    assert out10[0] == [(5, 20), (3, 12), (4, 12), (1, 9)]
    # Images 1..5 share their first m points with each other as well.
    assert (1, 5) in pairs10 and (0, 2) not in pairs10


def _brute(lists, threshold, top_k):
    n = len(lists)
    sets = [set(p) for p in lists]
    out = []
    for q in range(n):
        cand = [(i, len(sets[q] & sets[i])) for i in range(n) if i != q]
        cand = [c for c in cand if c[1] > threshold]
        cand.sort(key=lambda c: (-c[1], c[0]))
        out.append(cand[:top_k])
    pairs = sorted({tuple(sorted((q, i))) for q in range(n) for i, _ in out[q]})
    return out, pairs


def test_against_set_intersection_brute_force():
    rng = np.random.default_rng(11)
    for trial in range(20):
        n = int(rng.integers(1, 14))
        npts = int(rng.integers(1, 80))
        lists = [sorted(rng.choice(npts, size=int(rng.integers(0, npts + 1)), replace=False))
                 for _ in range(n)]
        T = int(rng.integers(0, 6))
        k = int(rng.integers(0, n + 2))
        assert covis.candidate_images(lists, npts, T, k) == _brute(lists, T, k)


def test_counts_closed_forms():
    lists = [[0, 1, 2, 3], [2, 3, 4], [], [3]]
    C = covis.covisible_counts(lists, 5)
    assert C.tolist() == [[4, 2, 0, 1], [2, 3, 0, 1], [0, 0, 0, 0], [1, 1, 0, 1]]


def test_full_lists_are_symmetric():
    rng = np.random.default_rng(12)
    lists = [sorted(rng.choice(40, size=15, replace=False)) for _ in range(9)]
    out, pairs = covis.candidate_images(lists, 40, threshold=3, top_k=100)
    for q, i in itertools.permutations(range(9), 2):
        assert (i in [c for c, _ in out[q]]) == (q in [c for c, _ in out[i]])
    assert pairs == sorted({(min(q, i), max(q, i)) for q in range(9) for i, _ in out[q]})
