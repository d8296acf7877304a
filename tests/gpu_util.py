"""Helpers for GPU-vs-oracle parity checks."""
import sys

import numpy as np

INT32_MAX = 2**31 - 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_per_query(out, q_off, p):
    s, e = int(q_off[p]), int(q_off[p + 1])
    return {"match": out.all_match[s:e].cpu().numpy(), "d1": out.all_d1[s:e].cpu().numpy(),
            "d2": out.all_d2[s:e].cpu().numpy(), "count": out.all_count[s:e].cpu().numpy()}


def compare_pair(out, ores, p, check_counts=True):
    """Bit-exact comparison of pair p except queries with a borderline candidate.

    Returns (number of queries compared, number excused as borderline)."""
    o = ores.pair(p)
    q, m, d1, d2 = out.pair(p)
    # Output rows are in ascending query order.
    assert np.all(np.diff(q) > 0), "queries not strictly ascending"
    clean = o["borderline"] == 0
    oq = np.nonzero(o["accept"])[0]
    keep = clean[q] if len(q) else np.zeros(0, bool)
    okeep = clean[oq]
    assert np.array_equal(q[keep], oq[okeep]), "accepted query set differs"
    assert np.array_equal(m[keep], o["match"][oq[okeep]]), "match index differs"
    assert np.array_equal(d1[keep], o["d1"][oq[okeep]]), "d1 differs"
    assert np.array_equal(d2[keep], o["d2"][oq[okeep]]), "d2 differs"
    if out.emit_all:
        g = gpu_per_query(out, ores.q_off, p)
        for k in ("match", "d1", "d2") + (("count",) if check_counts else ()):
            bad = np.nonzero(g[k][clean] != o[k][clean])[0]
            assert bad.size == 0, f"{k} differs on {bad.size} clean queries, first {np.nonzero(clean)[0][bad[:5]]}"
        # Borderline queries: counts may differ by at most their borderline candidates.
        if check_counts:
            diff = np.abs(g["count"].astype(np.int64) - o["count"])
            assert np.all(diff <= o["borderline"])
    return int(clean.sum()), int((~clean).sum())


def compare_all(out, ores, n_pairs, check_counts=True):
    tot_clean = tot_bl = 0
    cmp_gpu = out.n_comparisons[:n_pairs].cpu().numpy()
    for p in range(n_pairs):
        c, b = compare_pair(out, ores, p, check_counts)
        tot_clean += c
        tot_bl += b
        if check_counts:
            assert abs(int(cmp_gpu[p]) - int(ores.n_comparisons[p])) <= int(ores.n_borderline[p])
            if ores.n_borderline[p] == 0:
                assert int(cmp_gpu[p]) == int(ores.n_comparisons[p])
    return tot_clean, tot_bl
