"""Pins of the CPU oracle against the paper's definitions, closed forms,
special cases and an independent brute force (no GPU needed)."""
import numpy as np
import pytest

import scenes
from tests import bruteforce_np
from tests.fixtures import load_hand_fixture, random_pair, translation_F

INF = 2**31 - 1


def run(oracle, xy_a, desc_a, xy_b, desc_b, F, band, **kw):
    r = oracle.match([(xy_a, desc_a), (xy_b, desc_b)], [(0, 1, band)], [F], **kw)
    return r.pair(0), r


# --- worked example -----------------------------------------------------------------

def test_hand_fixture(oracle_lib):
    xy_a, desc_a, xy_b, desc_b, F, band, expect = load_hand_fixture()
    p, _ = run(oracle_lib, xy_a, desc_a, xy_b, desc_b, F, band)
    got = [(i, int(p["match"][i]), int(p["d1"][i]), int(p["d2"][i]), int(p["count"][i]),
            int(p["accept"][i])) for i in range(len(expect))]
    assert got == expect


# --- band predicate, eqs. (2)-(3) ---------------------------------------------------

@pytest.mark.parametrize("d", [4.0, 2.5, 8.0])
def test_band_inclusive_closed_form(oracle_lib, d):
    """Axis-aligned line y' = y: targets at exactly d are in, d + 2^-10 are out."""
    F = translation_F((1.0, 0.0, 0.0))
    y = 300.0
    offs = [0.0, d, -d, d - 2**-10, -(d - 2**-10), d + 2**-10, -(d + 2**-10), 3 * d]
    xy_b = np.array([[100.0 + 10 * k, y + o] for k, o in enumerate(offs)], np.float32)
    assert np.all(xy_b[:, 1].astype(np.float64) - y == np.array(offs))   # exact in float32
    xy_a = np.array([[50.0, y]], np.float32)
    desc_a = np.zeros((1, 128), np.uint8)
    desc_b = np.zeros((len(offs), 128), np.uint8)
    for k in range(len(offs)):
        desc_b[k, 0] = k + 1       # distinct distances (k+1)^2
    p, _ = run(oracle_lib, xy_a, desc_a, xy_b, desc_b, F, d)
    assert p["count"][0] == 5                 # 0, +-d, +-(d - 2^-10)
    assert p["match"][0] == 0 and p["d1"][0] == 1 and p["d2"][0] == 4
    for k, want in [(0, 0.0), (1, d), (2, d), (5, d + 2**-10)]:
        assert oracle_lib.epipolar_distance(F, 50.0, y, *xy_b[k]) == want


@pytest.mark.parametrize("d", [4.0, 2.5])
def test_borderline_counter_closed_form(oracle_lib, d):
    """The borderline count: targets whose FP64 distance e satisfies
    |e - d| <= borderline_px (inclusive), on both sides of the line, members
    of the band or not.  Axis-aligned line y' = y; every offset below is a
    multiple of 2^-15, so y + offset is exact in float32 and e equals |offset|
    exactly.  Catches counting members only, a strict comparison, and a
    wrong margin."""
    F = translation_F((1.0, 0.0, 0.0))
    y = 300.0
    m, u = 2**-10, 2**-15
    offs = [d, -d,                      # on the edge
            d + m, -(d + m),            # out of the band, exactly m away: counted
            d - m, -(d - m),            # in the band, exactly m away: counted
            d + m + u, -(d - m - u),    # one ulp beyond m: not counted
            d + m - u, d + 2**-11,      # out of the band, within m: counted
            0.0, 3 * d]                 # far from the edge
    counted = [1, 1, 1, 1, 1, 1, 0, 0, 1, 1, 0, 0]
    members = [1, 1, 0, 0, 1, 1, 0, 1, 0, 0, 1, 0]
    xy_b = np.array([[100.0 + 10 * k, y + o] for k, o in enumerate(offs)], np.float32)
    assert np.all(xy_b[:, 1].astype(np.float64) - y == np.array(offs))   # exact in float32
    for k, o in enumerate(offs):
        assert oracle_lib.epipolar_distance(F, 50.0, y, *xy_b[k]) == abs(o)
    xy_a = np.array([[50.0, y], [60.0, y]], np.float32)
    desc_a = np.zeros((2, 128), np.uint8)
    desc_b = np.zeros((len(offs), 128), np.uint8)
    desc_b[:, 0] = np.arange(1, len(offs) + 1)
    for px, want in [(m, sum(counted)), (1e-3, sum(counted)), (0.0, 2), (m - u, 4),
                     (2 * d - u, len(offs) - 1), (2 * d, len(offs))]:
        p, r = run(oracle_lib, xy_a, desc_a, xy_b, desc_b, F, d, borderline_px=px)
        assert list(p["borderline"]) == [want, want], px
        assert int(r.n_borderline[0]) == 2 * want
        assert list(p["count"]) == [sum(members)] * 2


def test_band_general_line_and_sign(oracle_lib):
    """Pure translation with a finite epipole e: the line of p passes through e
    (textbook F = [e]_x); targets on it are candidates, targets 5 px off it are not."""
    e = np.array([-3000.0, 200.0, 1.0])
    F = translation_F(e)
    p = np.array([400.0, 300.0])
    u = (p - e[:2]) / np.linalg.norm(p - e[:2])
    nrm = np.array([-u[1], u[0]])
    on = [e[:2] + u * s for s in (3300.0, 3500.0, 3800.0)]
    off = [q + sgn * 5.0 * nrm for q, sgn in zip(on, (1, -1, 1))]
    xy_b = np.array(on + off, np.float32)
    for q in on:
        assert oracle_lib.epipolar_distance(F, *p, *q.astype(np.float32)) < 1e-3
    for q in off:
        assert abs(oracle_lib.epipolar_distance(F, *p, *q.astype(np.float32)) - 5.0) < 1e-3
    desc_b = np.zeros((6, 128), np.uint8)
    desc_b[:, 0] = [3, 4, 5, 0, 0, 0]         # off-line targets are the best descriptors
    p_, _ = run(oracle_lib, np.array([p], np.float32), np.zeros((1, 128), np.uint8),
                xy_b, desc_b, F, 4.0)
    assert p_["count"][0] == 3 and p_["match"][0] == 0 and p_["d1"][0] == 9 and p_["d2"][0] == 16


def test_transposed_f_is_detected(oracle_lib):
    """Noise-free planted correspondences are at distance ~0 from l = F x_a."""
    s = scenes.make_pair_scene(300, 300, seed=3)
    from scenes.generator import project
    X = s.points[:50]
    xa, _ = project(s.cams[0], X)
    xb, _ = project(s.cams[1], X)
    d = [oracle_lib.epipolar_distance(s.F, *np.float32(xa[k]), *np.float32(xb[k]))
         for k in range(50)]
    assert max(d) < 1e-3     # float32 rounding of the inputs only
    dt = [oracle_lib.epipolar_distance(s.F.T, *np.float32(xa[k]), *np.float32(xb[k]))
          for k in range(50)]
    assert np.median(dt) > 1.0


def test_scale_invariance_of_f(oracle_lib):
    xy_a, desc_a, xy_b, desc_b, F = random_pair(300, 400, seed=5)
    ref, rr = run(oracle_lib, xy_a, desc_a, xy_b, desc_b, F, 4.0)
    for lam in (-3.7, 1e-6, 1e6):
        got, rg = run(oracle_lib, xy_a, desc_a, xy_b, desc_b, lam * F, 4.0)
        clean = (ref["borderline"] == 0) & (got["borderline"] == 0)
        for k in ("match", "d1", "d2", "count", "accept"):
            assert np.array_equal(ref[k][clean], got[k][clean]), (lam, k)
        assert clean.mean() > 0.9


def test_query_at_epipole_has_no_candidates(oracle_lib):
    """F e_a = 0: the query at the epipole of a has the degenerate line (0, 0, 0)."""
    e = (100.0, 50.0, 1.0)
    F = translation_F(e)
    xy_a = np.array([[100.0, 50.0], [300.0, 50.0]], np.float32)
    xy_b = np.array([[200.0, 50.0], [400.0, 50.5], [10.0, 10.0]], np.float32)
    p, _ = run(oracle_lib, xy_a, np.zeros((2, 128), np.uint8), xy_b,
               np.zeros((3, 128), np.uint8), F, 4.0)
    assert p["count"][0] == 0 and p["match"][0] == -1 and not p["accept"][0]
    assert p["count"][1] == 2


# --- distances -------------------------------------------------------------------------

def test_distance_closed_forms(oracle_lib):
    z = np.zeros(128, np.uint8)
    m = np.full(128, 127, np.uint8)
    assert oracle_lib.desc_dist(z, z) == 0
    assert oracle_lib.desc_dist(m, m) == 0
    assert oracle_lib.desc_dist(z, m) == 128 * 127 * 127 == 2064512
    for k in (0, 63, 127):
        for v in (1, 50, 127):
            o = z.copy()
            o[k] = v
            assert oracle_lib.desc_dist(z, o) == v * v
            assert oracle_lib.desc_dist(o, z) == v * v
    rng = np.random.default_rng(0)
    a = rng.integers(0, 128, 128, dtype=np.uint8)
    b = rng.integers(0, 128, 128, dtype=np.uint8)
    assert oracle_lib.desc_dist(a, b) == int(((a.astype(int) - b.astype(int)) ** 2).sum())


# --- selection, ties, ratio (Section 6.2.2, Appendix A step 4) -----------------------

@pytest.mark.parametrize("seed", range(6))
def test_against_sorting_bruteforce(oracle_lib, seed):
    n_a, n_b = [(64, 64), (17, 50), (64, 3), (40, 64), (1, 64), (64, 1)][seed]
    xy_a, desc_a, xy_b, desc_b, F = random_pair(n_a, n_b, seed=100 + seed, spread=0.05)
    # Coarse descriptors make many exact ties; a wide band gives many candidates.
    desc_a //= 8
    desc_b //= 8
    for band in (40.0, 200.0):
        p, _ = run(oracle_lib, xy_a, desc_a, xy_b, desc_b, F, band)
        ref = bruteforce_np.match_pair(xy_a, desc_a, xy_b, desc_b, F, band)
        got = list(zip(p["match"].tolist(), p["d1"].tolist(), p["d2"].tolist(),
                       p["count"].tolist(), p["accept"].tolist()))
        assert got == [tuple(r) for r in ref]


def test_planted_ties_lowest_index(oracle_lib):
    F = translation_F((1.0, 0.0, 0.0))
    xy_a = np.array([[0.0, 10.0]], np.float32)
    xy_b = np.array([[5.0, 10.0], [1.0, 11.0], [2.0, 9.0], [3.0, 10.5]], np.float32)
    desc_a = np.zeros((1, 128), np.uint8)
    desc_b = np.zeros((4, 128), np.uint8)
    desc_b[:, 0] = [9, 3, 3, 3]      # three-way tie at D = 9, indices 1, 2, 3
    p, _ = run(oracle_lib, xy_a, desc_a, xy_b, desc_b, F, 4.0)
    assert (p["match"][0], p["d1"][0], p["d2"][0], p["count"][0]) == (1, 9, 9, 4)
    assert not p["accept"][0]


@pytest.mark.parametrize("d2_vec,accept", [((4,), False), ((3, 2, 1, 1), True)])
def test_ratio_boundary(oracle_lib, d2_vec, accept):
    """D1 = 16 vs D2 = 25 is exactly ratio 0.8 (rejected); D1 = 15 vs 25 passes."""
    F = translation_F((1.0, 0.0, 0.0))
    xy_a = np.array([[0.0, 10.0]], np.float32)
    xy_b = np.array([[1.0, 10.0], [2.0, 10.0]], np.float32)
    desc_a = np.zeros((1, 128), np.uint8)
    desc_b = np.zeros((2, 128), np.uint8)
    desc_b[0, :len(d2_vec)] = d2_vec
    desc_b[1, 0] = 5
    p, _ = run(oracle_lib, xy_a, desc_a, xy_b, desc_b, F, 4.0)
    assert p["d2"][0] == 25 and p["d1"][0] == sum(v * v for v in d2_vec)
    assert bool(p["accept"][0]) == accept


def test_single_candidate_policy(oracle_lib):
    F = translation_F((1.0, 0.0, 0.0))
    xy_a = np.array([[0.0, 10.0]], np.float32)
    xy_b = np.array([[1.0, 10.0], [2.0, 100.0]], np.float32)
    z = np.zeros((1, 128), np.uint8)
    p, _ = run(oracle_lib, xy_a, z, xy_b, np.zeros((2, 128), np.uint8), F, 4.0)
    assert p["count"][0] == 1 and p["d2"][0] == INF and not p["accept"][0]
    p, _ = run(oracle_lib, xy_a, z, xy_b, np.zeros((2, 128), np.uint8), F, 4.0,
               accept_single=True)
    assert p["accept"][0]


# --- whole-method special cases -------------------------------------------------------

def test_infinite_band_is_exhaustive_matching(oracle_lib):
    """d = inf reduces to plain 2-NN ratio matching over every target feature."""
    xy_a, desc_a, xy_b, desc_b, F = random_pair(60, 64, seed=9)
    p, _ = run(oracle_lib, xy_a, desc_a, xy_b, desc_b, F, np.inf)
    q, _ = run(oracle_lib, xy_a, desc_a, xy_b, desc_b, F, 4.0, ignore_band=True)
    ref = bruteforce_np.match_pair(xy_a, desc_a, xy_b, desc_b, F, 0.0, ignore_band=True)
    assert (p["count"] == 64).all()
    for k in ("match", "d1", "d2", "count", "accept"):
        assert np.array_equal(p[k], q[k])
    assert list(zip(p["match"].tolist(), p["d1"].tolist(), p["d2"].tolist())) == \
        [(r[0], r[1], r[2]) for r in ref]


def test_zero_band_on_noisy_data_is_empty(oracle_lib):
    s = scenes.make_two_view_2k()
    r = oracle_lib.match([(im.xy, im.desc) for im in s.images], [(0, 1, 0.0)], [s.F])
    assert r.n_comparisons[0] == 0 and r.n_accepted[0] == 0


def test_planted_match_recovery_two_view(oracle_lib):
    """Recall of in-band true correspondences and precision of accepted matches."""
    s = scenes.make_two_view_2k()
    A, B = s.images
    r = oracle_lib.match([(A.xy, A.desc), (B.xy, B.desc)], s.pairs, [s.F])
    q, m, d1, d2 = r.matches(0)
    correct = (A.gt[q] >= 0) & (A.gt[q] == B.gt[m])
    assert correct.mean() >= 0.99
    pos_b = {int(g): k for k, g in enumerate(B.gt) if g >= 0}
    inband = [i for i, g in enumerate(A.gt)
              if g >= 0 and int(g) in pos_b and oracle_lib.epipolar_distance(
                  s.F, *A.xy[i], *B.xy[pos_b[int(g)]]) <= 4.0]
    found = set(q[correct].tolist())
    assert len(found & set(inband)) / len(inband) >= 0.99
    assert r.n_comparisons[0] > 40000


def test_repetitive_structure_guided_keeps_match(oracle_lib):
    """A near-duplicate of the true partner placed outside the band fails the
    ratio test of exhaustive matching but not guided matching (Section 6.2.3)."""
    s = scenes.make_two_view_2k()
    A, B = s.images
    pos_b = {int(g): k for k, g in enumerate(B.gt) if g >= 0}
    i = next(k for k, g in enumerate(A.gt) if g >= 0 and int(g) in pos_b)
    j = pos_b[int(A.gt[i])]
    xy_b = np.vstack([B.xy, [[B.xy[j, 0], (B.xy[j, 1] + 200.0) % 768]]]).astype(np.float32)
    desc_b = np.vstack([B.desc, B.desc[j:j + 1]])
    imgs = [(A.xy[i:i + 1], A.desc[i:i + 1]), (xy_b, desc_b)]
    g = oracle_lib.match(imgs, [(0, 1, 4.0)], [s.F]).pair(0)
    x = oracle_lib.match(imgs, [(0, 1, np.inf)], [s.F]).pair(0)
    assert g["accept"][0] and g["match"][0] == j
    assert not x["accept"][0] and x["d1"][0] == x["d2"][0]


def test_invalid_arguments_rejected(oracle_lib):
    xy = np.zeros((1, 2), np.float32)
    d = np.zeros((1, 128), np.uint8)
    with pytest.raises(ValueError):
        oracle_lib.match([(xy, d)], [(0, 3, 4.0)], [np.eye(3)])
    with pytest.raises(ValueError):
        oracle_lib.match([(xy, d)], [(0, 0, -1.0)], [np.eye(3)])
    with pytest.raises(ValueError):
        oracle_lib.match([(xy, d)], [(0, 0, float("nan"))], [np.eye(3)])


def test_thread_count_does_not_change_results(oracle_lib):
    xy_a, desc_a, xy_b, desc_b, F = random_pair(700, 500, seed=11)
    a, _ = run(oracle_lib, xy_a, desc_a, xy_b, desc_b, F, 6.0, n_threads=1)
    b, _ = run(oracle_lib, xy_a, desc_a, xy_b, desc_b, F, 6.0, n_threads=5)
    for k in a:
        assert np.array_equal(a[k], b[k])
