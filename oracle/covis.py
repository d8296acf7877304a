"""Candidate images from point-camera covisibility -- TEST INFRASTRUCTURE.

Only tests/ and the benchmark's CPU-baseline leg may use this module.  It
restates Section 6.1 directly and shares no code with the GPU library:

* P_cv(I_i, I_j) is the set of coarse-model points that both images observe;
  its size for every pair is the (i, j) entry of V V^T, V the 0/1
  image-by-point incidence (a sparse matrix product, exact in integers);
* S_q, the candidates of query image q, are the other images i with
  |P_cv(I_q, I_i)| > T;
* they are ranked by |P_cv| (equal counts: lower image index first -- the
  paper does not say; this is the reading both sides use) and cut to top_k;
* the pairs to match are the unique unordered pairs {q, i}, i in S_q.
"""
from __future__ import annotations

import numpy as np
from scipy import sparse


def covisible_counts(vis_lists, n_points: int) -> np.ndarray:
    """|P_cv(I_i, I_j)| for all i, j (the diagonal is |Points(I_i)|)."""
    n = len(vis_lists)
    rows = np.concatenate([np.full(len(p), i, dtype=np.int64) for i, p in enumerate(vis_lists)]) \
        if n else np.zeros(0, np.int64)
    cols = np.concatenate([np.asarray(p, dtype=np.int64) for p in vis_lists]) \
        if n else np.zeros(0, np.int64)
    V = sparse.csr_matrix((np.ones(rows.shape[0], dtype=np.int64), (rows, cols)),
                          shape=(n, n_points))
    return np.asarray((V @ V.T).todense(), dtype=np.int64)


def candidate_images(vis_lists, n_points: int, threshold: int, top_k: int):
    """Per query image q: [(image, shared points), ...] in rank order; and the
    sorted list of unique pairs (i, j), i < j."""
    C = covisible_counts(vis_lists, n_points)
    n = len(vis_lists)
    lists = []
    for q in range(n):
        S = np.array([i for i in range(n) if i != q and C[q, i] > threshold], dtype=np.int64)
        order = np.lexsort((S, -C[q, S])) if S.size else S   # count descending, then index
        ranked = S[order][:top_k]
        lists.append([(int(i), int(C[q, i])) for i in ranked])
    pairs = sorted({(min(q, i), max(q, i)) for q in range(n) for i, _ in lists[q]})
    return lists, pairs
