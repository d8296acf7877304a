"""Helpers for GPU-vs-oracle parity checks.

Every comparison is bit-exact on every query: the library decides FP32
distances within its recheck margin of the band edge again in FP64 with the
definition's operations, so no query is excused."""
import sys

import numpy as np

INT32_MAX = 2**31 - 1
FP32_ERR_PX = 1e-4   # bound on the FP32 epipolar-distance error (measured by sfm_band_error)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_per_query(out, q_off, p):
    s, e = int(q_off[p]), int(q_off[p + 1])
    return {"match": out.all_match[s:e].cpu().numpy(), "d1": out.all_d1[s:e].cpu().numpy(),
            "d2": out.all_d2[s:e].cpu().numpy(), "count": out.all_count[s:e].cpu().numpy()}


def _first_diff(a, b):
    bad = np.nonzero(a != b)[0]
    return f"{bad.size} differ, first at {bad[:5]}: gpu {a[bad[:5]]} oracle {b[bad[:5]]}"


def compare_rows(q, m, d1, d2, o, what=""):
    """Accepted rows (ascending query) against oracle pair dict o, exactly."""
    assert np.all(np.diff(q) > 0), f"{what}queries not strictly ascending"
    oq = np.nonzero(o["accept"])[0]
    assert q.shape == oq.shape and np.array_equal(q, oq), \
        f"{what}accepted query set differs ({q.size} vs {oq.size})"
    assert np.array_equal(m, o["match"][oq]), f"{what}match: " + _first_diff(m, o["match"][oq])
    assert np.array_equal(d1, o["d1"][oq]), f"{what}d1: " + _first_diff(d1, o["d1"][oq])
    assert np.array_equal(d2, o["d2"][oq]), f"{what}d2: " + _first_diff(d2, o["d2"][oq])


def compare_pair(out, ores, p, check_counts=True):
    """Pair p of the GPU output against the oracle, bit-exact on every query.
    Returns (queries compared, queries with an oracle-borderline candidate)."""
    o = ores.pair(p)
    compare_rows(*out.pair(p), o, what=f"pair {p}: ")
    if out.emit_all:
        g = gpu_per_query(out, ores.q_off, p)
        for k in ("match", "d1", "d2") + (("count",) if check_counts else ()):
            assert np.array_equal(g[k], o[k]), f"pair {p}: {k}: " + _first_diff(g[k], o[k])
    return int(o["match"].shape[0]), int((o["borderline"] > 0).sum())


def compare_all(out, ores, n_pairs, check_counts=True):
    """Every pair exact, and every pair's comparison count equal.
    Returns (queries compared, queries with an oracle-borderline candidate)."""
    tot = tot_bl = 0
    cmp_gpu = out.n_comparisons[:n_pairs].cpu().numpy()
    for p in range(n_pairs):
        c, b = compare_pair(out, ores, p, check_counts)
        tot += c
        tot_bl += b
        if check_counts:
            assert int(cmp_gpu[p]) == int(ores.n_comparisons[p]), \
                f"pair {p}: comparisons {int(cmp_gpu[p])} vs {int(ores.n_comparisons[p])}"
    return tot, tot_bl


def check_borderline_counts(out, oracle, images, pairs, Fs, margin=1e-3, err=FP32_ERR_PX):
    """The GPU's per-pair count of slots decided in FP64 (FP32 distance within
    `margin` of d) lies between the oracle's FP64 borderline counts at
    margin - 2 err and margin + 2 err.  Returns the GPU counts."""
    n = len(pairs)
    gpu = out.n_borderline[:n].cpu().numpy()
    lo = oracle.match(images, pairs, Fs, borderline_px=max(0.0, margin - 2 * err)).n_borderline
    hi = oracle.match(images, pairs, Fs, borderline_px=margin + 2 * err).n_borderline
    assert np.all(lo <= gpu) and np.all(gpu <= hi), \
        f"borderline counts outside the bracket: {list(zip(lo, gpu, hi))[:8]}"
    return gpu
