"""Staged matching of coarse features -- TEST INFRASTRUCTURE.

Only tests/ and the benchmark's CPU-baseline leg may use this module.  It
restates the hybrid scheme of Section 4 (after the preemptive matching the
related-work section describes) and shares no code with the GPU library:

* the features of each image are ranked by decreasing scale (ties keep their
  order: numpy's stable sort), so "the first x%" is the x% of highest scale;
* if either image of the pair has fewer than `small_image` features (1000 in
  the paper), all features of a are matched against all of b, in one stage;
* otherwise stage 1 matches the first q = ceil(n_a * query_pct / 100) ranked
  features of a (10%) against the first r = ceil(n_b * target_pct / 100) of b
  (20%);
* stage 2 matches the next min(q, n_a - q) ranked features of a against the
  same r features of b, only if stage 1 accepted more than `min_matches` (4);
* the paper allows stopping once enough matches for the geometry are found
  but gives no number: `enough` > 0 skips stage 2 when stage 1 already
  accepted that many (0, the default, never stops early);
* a stage is exhaustive two-nearest-neighbour matching with the ratio test,
  the oracle's own `match` with the band ignored, on the selected features.

Percentages are integers and rounded up, so both implementations compute the
same subset sizes.  Rows are reported in the caller's feature indexing: stage
1's rows, then stage 2's, each in the order of the query's scale rank.
"""
from __future__ import annotations

import numpy as np

from . import match as _match


def stage_sizes(na: int, nb: int, query_pct=10, target_pct=20, small_image=1000):
    """(whole, q, r, q2): the queries of stage 1, the targets, and the queries
    of stage 2 (0 for a pair matched whole, which takes q = n_a, r = n_b)."""
    if na < small_image or nb < small_image:
        return True, na, nb, 0
    q = -(-na * query_pct // 100)
    r = -(-nb * target_pct // 100)
    return False, q, r, min(q, na - q)


def _stage(a_img, b_img, qsel, rsel, ratio_num, ratio_den, accept_single):
    """Exhaustive matching of a's features qsel against b's rsel; rows in
    the order of qsel, indices mapped back to the full images."""
    xa, da = a_img[0][qsel], a_img[1][qsel]
    xb, db = b_img[0][rsel], b_img[1][rsel]
    res = _match([(xa, da), (xb, db)], [(0, 1, np.inf)], np.eye(3)[None],
                 ratio_num=ratio_num, ratio_den=ratio_den, accept_single=accept_single,
                 ignore_band=True)
    q, m, d1, d2 = res.matches(0)
    return qsel[q], rsel[m], d1, d2, int(res.n_comparisons[0])


def preemptive_match(images, pairs, query_pct=10, target_pct=20, min_matches=4, enough=0,
                     small_image=1000, ratio_num=64, ratio_den=100, accept_single=False):
    """images: list of (xy (n,2), desc (n,128) uint8, scale (n,)); pairs: list
    of (a, b, ...).  Per pair a dict: stages (0 whole, 1, 2), query, match, d1,
    d2 (int arrays, rows as described above) and n_comparisons."""
    out = []
    for pr in pairs:
        a, b = int(pr[0]), int(pr[1])
        A, B = images[a], images[b]
        na, nb = A[0].shape[0], B[0].shape[0]
        rank_a = np.argsort(-np.asarray(A[2]), kind="stable")
        rank_b = np.argsort(-np.asarray(B[2]), kind="stable")
        whole, q, r, q2 = stage_sizes(na, nb, query_pct, target_pct, small_image)
        kw = dict(ratio_num=ratio_num, ratio_den=ratio_den, accept_single=accept_single)
        s1 = _stage(A, B, rank_a[:q], rank_b[:r], **kw)
        n1 = len(s1[0])
        run2 = (not whole and q2 > 0 and n1 > min_matches
                and not (enough > 0 and n1 >= enough))
        parts = [s1]
        if run2:
            parts.append(_stage(A, B, rank_a[q:q + q2], rank_b[:r], **kw))
        out.append({
            "stages": 0 if whole else (2 if run2 else 1),
            "query": np.concatenate([p[0] for p in parts]).astype(np.int64),
            "match": np.concatenate([p[1] for p in parts]).astype(np.int64),
            "d1": np.concatenate([p[2] for p in parts]).astype(np.int64),
            "d2": np.concatenate([p[3] for p in parts]).astype(np.int64),
            "n_comparisons": sum(p[4] for p in parts),
        })
    return out
