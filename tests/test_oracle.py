"""Pins for the CPU oracle (no GPU).

Each check ties the oracle to something other than itself: a hand-worked
example (tests/golden/hand_example.txt), textbook brute force in pure Python,
library routines (numpy windows, scipy distances, numpy sorting, math.isqrt),
a sqrt-free form of the ring test derived independently, and the containment
property that makes exact-mode RIANN equal brute force (every reference at
distance <= R from the query lies in every key ring, by the triangle
inequality).  `test_planted_faults` plants each deliberate mistake the oracle
knows about and checks that at least one pin fails.
"""
import math
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import gen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hand_example.txt")


def _gold():
    rows = {}
    bounds = []
    with open(GOLD) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            if k == "bounds":
                bounds.append(tuple(int(x) for x in v))
            elif k.startswith("riann_"):
                rows[k] = dict(zip(v[0::2], (int(x) for x in v[1::2])))
            else:
                rows[k] = [int(x) for x in v]
    rows["bounds"] = bounds
    return rows


# ---------------------------------------------------------------- helpers
def py_ssd(a, b):
    return sum((int(x) - int(y)) ** 2 for x, y in zip(a, b))


def py_bf(Q, R):
    out = []
    for q in Q:
        best, arg = None, -1
        for r, ref in enumerate(R):
            d = py_ssd(q, ref)
            if best is None or d < best:
                best, arg = d, r
        out.append((arg, best))
    return out


def lib_bf(Q, R):
    """Exact NN via scipy's squared-euclidean distances (float64 is exact for
    these integer magnitudes) and numpy's first-occurrence argmin."""
    d = cdist(Q.astype(np.float64), R.astype(np.float64), "sqeuclidean")
    return d.argmin(1).astype(np.int32), d.min(1).astype(np.uint32)


def in_ring_exact(a, b, c):
    """|sqrt(a) - sqrt(b)| <= sqrt(c) decided without square roots.
    Upper side: sqrt(a) <= sqrt(b) + sqrt(c)  <=>  a-b-c <= 0 or (a-b-c)^2 <= 4bc.
    Lower side: sqrt(b) <= sqrt(a) + sqrt(c)  <=>  b-a-c <= 0 or (b-a-c)^2 <= 4ac."""
    u = a - b - c
    up = u <= 0 or u * u <= 4 * b * c
    w = b - a - c
    down = w <= 0 or w * w <= 4 * a * c
    return up and down


def small_case(seed, n=96, K=6, H=20, W=22, p=4, C=1, s=1, dup=0):
    rng = np.random.default_rng(seed)
    tex = gen.texture(rng, H, W, C)
    frame = np.clip(np.rint(tex + rng.normal(0, 2, tex.shape)), 0, 255).astype(np.uint8)
    rtex = gen.texture(rng, H + 10, W + 10, C)
    rframe = np.clip(np.rint(rtex), 0, 255).astype(np.uint8)
    ref = gen.reference_from_frame(rframe, n, p, 1, rng)
    if dup:
        ref[rng.choice(n, dup, replace=False)] = ref[rng.choice(n, dup, replace=False)]
    keys = gen.choose_keys(n, K, rng)
    return frame, ref, keys, rng


# ---------------------------------------------------------------- extraction
def test_query_counts():
    assert oracle.field_shape(64, 64, 8, 1) == (57, 57)           # 3,249
    h, w = oracle.field_shape(720, 1280, 8, 1)
    assert h * w == 907_649
    h, w = oracle.field_shape(1080, 1920, 8, 1)
    assert h * w == 2_052_649
    h, w = oracle.field_shape(2160, 3840, 12, 2)
    assert h * w == 2_058_625
    h, w = oracle.field_shape(360, 640, 12, 2)
    assert h * w == 55_125
    h, w = oracle.field_shape(360, 640, 8, 1)
    assert h * w == 223_449


@pytest.mark.parametrize("H,W,C,p,s", [(9, 11, 1, 4, 1), (13, 10, 3, 3, 2),
                                       (16, 16, 1, 8, 1), (15, 20, 2, 5, 3)])
def test_extract_matches_numpy_windows(H, W, C, p, s):
    rng = np.random.default_rng(H * W + C)
    f = rng.integers(0, 256, (H, W, C), dtype=np.uint8)
    got = oracle.extract(f, p, s)
    win = np.lib.stride_tricks.sliding_window_view(f, (p, p, C))[::s, ::s, 0]
    want = win.reshape(-1, p * p * C)
    assert got.shape == want.shape
    np.testing.assert_array_equal(got, want)


def test_extract_position_code():
    # pixel value encodes its position, so any transposition or offset shows
    H, W = 12, 9
    f = (np.arange(H)[:, None] * 16 + np.arange(W)[None, :]).astype(np.uint8)[:, :, None]
    P = oracle.extract(f, 3, 2)
    hq, wq = oracle.field_shape(H, W, 3, 2)
    for qy in range(hq):
        for qx in range(wq):
            q = P[qy * wq + qx]
            for dy in range(3):
                for dx in range(3):
                    assert q[dy * 3 + dx] == (2 * qy + dy) * 16 + (2 * qx + dx)


def test_hand_example_extract_and_nn():
    g = _gold()
    f = np.array(g["frame"], np.uint8).reshape(g["H"][0], g["W"][0], 1)
    P = oracle.extract(f, g["p"][0], g["s"][0])
    for i in range(4):
        assert list(P[i]) == g[f"q{i}"]
    ref = np.array([g[f"r{i}"] for i in range(4)], np.uint8)
    idx, d = oracle.brute_force(P, ref)
    assert list(idx) == g["nn_idx"]
    assert list(d) == g["nn_ssd"]


# ---------------------------------------------------------------- distances
def test_ssd_extremes_and_python():
    z = np.zeros(64, np.uint8)
    o = np.full(64, 255, np.uint8)
    assert oracle.ssd(z, o) == 4_161_600          # 255^2 * 64
    assert oracle.ssd(np.zeros(192, np.uint8), np.full(192, 255, np.uint8)) == 12_484_800
    rng = np.random.default_rng(1)
    for D in (1, 7, 64, 144, 192):
        a = rng.integers(0, 256, D, dtype=np.uint8)
        b = rng.integers(0, 256, D, dtype=np.uint8)
        assert oracle.ssd(a, b) == py_ssd(a, b)


def test_bf_matches_pure_python():
    rng = np.random.default_rng(2)
    Q = rng.integers(0, 256, (7, 9), dtype=np.uint8)
    R = rng.integers(0, 256, (23, 9), dtype=np.uint8)
    R[5] = R[17]                                   # duplicate pair
    Q[3] = R[17]                                   # exact hit on the duplicate
    idx, d = oracle.brute_force(Q, R)
    for i, (a, b) in enumerate(py_bf(Q, R)):
        assert idx[i] == a and d[i] == b
    assert idx[3] == 5 and d[3] == 0               # lowest index among ties


def test_bf_matches_scipy():
    frame, ref, _, _ = small_case(3, n=300)
    P = oracle.extract(frame, 4, 1)
    idx, d = oracle.brute_force(P, ref)
    li, ld = lib_bf(P, ref)
    np.testing.assert_array_equal(idx, li)
    np.testing.assert_array_equal(d, ld)


def test_bf_constant_frame():
    f = np.full((10, 10, 1), 77, np.uint8)
    ref = np.random.default_rng(4).integers(0, 256, (50, 16), dtype=np.uint8)
    ref[31] = 77
    ref[44] = 77
    idx, d = oracle.brute_force(oracle.extract(f, 4, 1), ref)
    assert (idx == 31).all() and (d == 0).all()


# ---------------------------------------------------------------- ring bounds
def test_isqrt():
    edge = [0, 1, 2, 3, 4, 15, 16, 17, 10**12, (2**26 - 1) ** 2, (2**26 - 1) ** 2 - 1,
            (2**26) ** 2, 4 * 12_484_800 * 12_484_800, 2**53 - 1]
    rng = np.random.default_rng(5)
    vals = edge + [int(x) for x in rng.integers(0, 2**53, 2000, dtype=np.int64)]
    for x in vals:
        assert oracle.isqrt(x) == math.isqrt(x), x
    for r in rng.integers(1, 2**26, 500):
        r = int(r)
        for x in (r * r - 1, r * r, r * r + 1):
            assert oracle.isqrt(x) == math.isqrt(x)


def test_ring_bounds_hand():
    for b, c, lo, hi in _gold()["bounds"]:
        assert oracle.ring_bounds(b, c) == (lo, hi)
    assert oracle.ring_bounds(123, None) == (0, oracle.INF)


def test_ring_bounds_exhaustive_small():
    for b in range(0, 40):
        for c in range(0, 40):
            lo, hi = oracle.ring_bounds(b, c)
            for a in range(0, 200):
                assert (lo <= a <= hi) == in_ring_exact(a, b, c), (a, b, c)


def test_ring_bounds_random_large():
    rng = np.random.default_rng(6)
    M = 12_484_800
    for _ in range(20000):
        b, c = (int(x) for x in rng.integers(0, M + 1, 2))
        lo, hi = oracle.ring_bounds(b, c)
        for a in (lo - 1, lo, lo + 1, hi - 1, hi, hi + 1,
                  int(rng.integers(0, 2 * M))):
            if a < 0:
                continue
            assert (lo <= a <= hi) == in_ring_exact(a, b, c), (a, b, c)


# ---------------------------------------------------------------- tables
def test_tables_hand():
    g = _gold()
    ref = np.array([g[f"r{i}"] for i in range(4)], np.uint8)
    t = oracle.Tables(ref, np.array(g["keys"], np.int32))
    for r in range(4):
        assert list(t.Piv[r]) == g[f"piv{r}"]
    assert list(t.T[0]) == g["T0"] and list(t.P[0]) == g["P0"]
    assert list(t.T[1]) == g["T1"] and list(t.P[1]) == g["P1"]


def test_tables_match_numpy_sort():
    _, ref, keys, _ = small_case(7, n=257, K=5, dup=20)
    t = oracle.Tables(ref, keys)
    d = cdist(ref.astype(np.float64), ref[keys].astype(np.float64), "sqeuclidean")
    np.testing.assert_array_equal(t.Piv, d.astype(np.uint32))
    for k in range(len(keys)):
        order = np.lexsort((np.arange(len(ref)), d[:, k]))   # by value, then index
        np.testing.assert_array_equal(t.P[k], order)
        np.testing.assert_array_equal(t.T[k], d[order, k].astype(np.uint32))


# ---------------------------------------------------------------- RIANN
def test_riann_hand():
    g = _gold()
    f = np.array(g["frame"], np.uint8).reshape(3, 3, 1)
    P = oracle.extract(f, 2, 1)
    ref = np.array([g[f"r{i}"] for i in range(4)], np.uint8)
    t = oracle.Tables(ref, np.array(g["keys"], np.int32))
    out = t.riann(P[1:2], np.array([0], np.int32))
    want = g["riann_q1_prev0"]
    for k in ("idx", "ssd", "mstar", "kstar", "nsurv"):
        assert int(out[k][0]) == want[k], k


@pytest.mark.parametrize("seed,K,mode", [(10, 6, "random"), (11, 1, "random"),
                                         (12, 0, "random"), (13, 6, "noprior"),
                                         (14, 6, "exact"), (15, 6, "mixed"),
                                         (16, 96, "random"), (17, 3, "dups")])
def test_riann_equals_brute_force(seed, K, mode):
    frame, ref, keys, rng = small_case(seed, n=96, K=K, dup=12 if mode == "dups" else 0)
    if K == 96:
        keys = np.arange(96, dtype=np.int32)
    P = oracle.extract(frame, 4, 1)
    bi, bd = oracle.brute_force(P, ref)
    hq, wq = oracle.field_shape(frame.shape[0], frame.shape[1], 4, 1)
    if mode == "noprior":
        prev = np.full(len(P), -1, np.int32)
    elif mode == "exact":
        prev = bi.copy()
    elif mode == "mixed":
        prev = gen.random_field(hq, wq, len(ref), rng, no_prior_p=0.3).reshape(-1)
        prev[rng.random(len(P)) < 0.2] = len(ref) + 5          # out of range
    else:
        prev = gen.random_field(hq, wq, len(ref), rng).reshape(-1)
    t = oracle.Tables(ref, keys)
    out = t.riann(P, prev)
    np.testing.assert_array_equal(out["idx"], bi)
    np.testing.assert_array_equal(out["ssd"], bd)
    bad = (prev < 0) | (prev >= len(ref))
    np.testing.assert_array_equal(out["noprior"].astype(bool), bad)
    if K == 0:
        assert (out["nsurv"] == len(ref)).all() and (out["mstar"] == len(ref)).all()
    assert (out["nsurv"] <= out["mstar"]).all()
    assert (out["nsurv"] >= 1).all()


def test_containment_and_prev_in_candidates():
    frame, ref, keys, rng = small_case(20, n=128, K=8, dup=8)
    P = oracle.extract(frame, 4, 1)
    t = oracle.Tables(ref, keys)
    D = cdist(P.astype(np.float64), ref.astype(np.float64), "sqeuclidean")
    for i in rng.choice(len(P), 60, replace=False):
        pv = int(rng.integers(0, len(ref)))
        S = set(t.candidates(P[i], pv).tolist())
        c = D[i, pv]
        # every reference within the radius is a candidate; so is r_prev
        within = set(np.nonzero(D[i] <= c)[0].tolist())
        assert within <= S
        assert pv in S
        # and every candidate lies in every key ring (exact sqrt-free test)
        for r in S:
            for k, kk in enumerate(keys):
                assert in_ring_exact(int(t.Piv[r, k]), int(D[i, kk]), int(c))


def test_riann_zero_radius():
    # previous match is an exact copy of the query: S = references at the
    # same key distances as the query (R = 0), and the answer has ssd 0
    frame, ref, keys, rng = small_case(21, n=80, K=5)
    P = oracle.extract(frame, 4, 1)
    ref = ref.copy()
    ref[17] = P[33]
    ref[50] = P[33]
    t = oracle.Tables(ref, keys)
    out = t.riann(P[33:34], np.array([50], np.int32))
    assert out["idx"][0] == 17 and out["ssd"][0] == 0
    S = t.candidates(P[33], 50)
    for r in S:
        assert (t.Piv[r] == t.Piv[17]).all()


def test_riann_workload_tiny_frames():
    wl = gen.make_workload("tiny")
    t = oracle.Tables(wl.ref, wl.keys)
    hq, wq = oracle.field_shape(64, 64, 8, 1)
    prev = np.full(hq * wq, -1, np.int32)
    for fr in range(3):
        P = oracle.extract(wl.frame(fr), 8, 1)
        assert len(P) == 3249
        bi, bd = oracle.brute_force(P, wl.ref)
        out = t.riann(P, prev)
        np.testing.assert_array_equal(out["idx"], bi)
        np.testing.assert_array_equal(out["ssd"], bd)
        prev = out["idx"]


# ---------------------------------------------------------------- k-NN fields
def test_knn_bf_matches_numpy_sort():
    """k nearest by exhaustive search against a numpy lexsort of all SSDs by
    (SSD, index); k = 1 reduces to the 1-NN brute force."""
    rng = np.random.default_rng(8)
    ref = rng.integers(0, 256, (300, 12), dtype=np.uint8)
    ref[[10, 20, 250]] = ref[5]                 # equal distances: index order
    q = np.concatenate([rng.integers(0, 256, (40, 12), dtype=np.uint8), ref[[5, 7]]])
    d = ((q[:, None, :].astype(np.int64) - ref[None, :, :].astype(np.int64)) ** 2).sum(-1)
    for k in (1, 3, 8):
        idx, dd = oracle.knn_brute_force(q, ref, k)
        for i in range(len(q)):
            order = np.lexsort((np.arange(len(ref)), d[i]))[:k]
            assert list(idx[i]) == list(order)
            assert list(dd[i]) == list(d[i][order])
    assert list(oracle.knn_brute_force(ref[[5]], ref, 4)[0][0]) == [5, 10, 20, 250]
    b1, d1 = oracle.brute_force(q, ref)
    k1, kd1 = oracle.knn_brute_force(q, ref, 1)
    np.testing.assert_array_equal(k1[:, 0], b1)
    np.testing.assert_array_equal(kd1[:, 0], d1)


@pytest.mark.parametrize("K", [0, 1, 5])
def test_knn_riann_equals_brute_force(K):
    """With the radius taken as the largest SSD to k distinct previous
    matches, the k nearest lie in every ring (containment): the k-NN ring
    search equals the exhaustive one for random, partly invalid, duplicated
    and exact previous fields."""
    rng = np.random.default_rng(40 + K)
    ref = rng.integers(0, 256, (400, 16), dtype=np.uint8)
    keys = np.sort(rng.choice(400, K, replace=False))
    t = oracle.Tables(ref, keys)
    q = np.clip(ref[rng.integers(0, 400, 120)].astype(np.int32) +
                rng.integers(-20, 21, (120, 16)), 0, 255).astype(np.uint8)
    k = 4
    bi, bd = oracle.knn_brute_force(q, ref, k)
    prevs = [rng.integers(0, 400, (120, k)).astype(np.int32)]
    p2 = prevs[0].copy()
    p2[::3, 1] = -1                                # no prior
    p2[1::3, 2] = p2[1::3, 0]                      # duplicates: no radius either
    prevs += [p2, bi.copy()]
    for pv in prevs:
        gi, gd = t.knn(q, pv, k)
        np.testing.assert_array_equal(gi, bi)
        np.testing.assert_array_equal(gd, bd)


# ---------------------------------------------------------------- paper mode
def test_splitmix_published_vector():
    """SplitMix64 (Steele, Lea and Flood 2014): the first outputs for seeds 0
    and 1 of the published generator."""
    assert oracle.splitmix(0) == 0xE220A8397B1DCDAF
    assert oracle.splitmix(1) == 0x910A2DEC89025CC1


def _paper(ref, q, prev, L, seed=3, t=1):
    pt = oracle.PaperTables(np.asarray(ref, np.uint8).reshape(len(ref), -1))
    return pt, pt.search(np.asarray(q, np.uint8).reshape(len(q), -1),
                         np.asarray(prev, np.int32), L=L, seed=seed, t=t)


def test_paper_hand_examples():
    """1-pixel patches worked by hand (alpha = 1/4: 9c <= 16a <= 25c), refs
    0, 12, 20, 40, 10.  q = 16, r_i = ref 0: c = 256, the ring of ref 0 is
    a in [144, 400], both ends closed, so 12 (a = 144) and 20 (a = 400) join
    r_i; the best is 12 (SSD 16, lower index than 20).  q = 12, r_i = ref 4
    (10): c = 4, the ring a in [2.25, 6.25] holds 12 (a = 4): exact match.
    q = 11, r_i = ref 4: c = 1, the ring a in [0.5625, 1.5625] is empty, so
    S = {r_i}.  With L = 1 that member is drawn as anchor; its own ring
    excludes it (a = 0), the intersection would be empty, so S is kept."""
    ref = [[0], [12], [20], [40], [10]]
    pt, r = _paper(ref, [[16], [12], [11]], [0, 4, 4], L=20)
    assert list(r["idx"]) == [1, 1, 4] and list(r["ssd"]) == [16, 0, 1]
    assert list(r["iters"]) == [0, 0, 0]
    _, r1 = _paper(ref, [[11]], [4], L=1)
    assert list(r1["idx"]) == [4] and list(r1["iters"]) == [1]
    assert pt.tv[0].tolist() == [0, 100, 144, 400, 1600]
    assert pt.tp[0].tolist() == [0, 4, 1, 2, 3]


def _paper_golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_anchor_example.txt")
    g = {"iters": {}}
    with open(path) as f:
        for line in f:
            w = line.split()
            if not w or w[0].startswith("#"):
                continue
            if w[0] == "iters":
                # "iters first A [second B] N"
                key = (int(w[2]),) if w[3] != "second" else (int(w[2]), int(w[4]))
                g["iters"][key] = int(w[-1])
            elif w[0] == "answer":
                g["answer"] = (int(w[2]), int(w[4]))
            else:
                g[w[0]] = [int(x) for x in w[1:]]
    return g


def _draw(seed, t, q, it):
    """The anchor draw: the published SplitMix64 output function (pinned
    above) chained over (seed, frame, query, iteration)."""
    m = 2**64 - 1
    x = oracle.splitmix(seed & m)
    x = oracle.splitmix((x ^ t) & m)
    x = oracle.splitmix((x ^ q) & m)
    return oracle.splitmix((x ^ it) & m)


def test_paper_anchor_loop_golden():
    """The anchor loop of Algorithm 1 against the hand-worked example in
    tests/golden/paper_anchor_example.txt: r_i's ring holds 7 of the 10
    references (8 members with r_i, L = 3), and anchors other than r_i,
    each with its own radius d_k != d_i, remove members until fewer than L
    remain.  The answer is the exact copy whatever the draws; the anchor
    count follows the hand-worked transitions from the first two draws.
    Many queries (each its own draws) walk every kind of path."""
    g = _paper_golden()
    ref = np.array(g["ref"], np.uint8).reshape(-1, 1)
    Q = 48
    q = np.full((Q, 1), g["q"][0], np.uint8)
    prev = np.full(Q, g["prev"][0], np.int32)
    S0 = g["S0"]
    S1_after_ri = [m for m in S0 if m != g["prev"][0]]
    seen = set()
    for seed, t in ((5, 1), (150807953, 7)):
        _, r = _paper(ref, q, prev, L=g["L"][0], seed=seed, t=t)
        for i in range(Q):
            first = S0[_draw(seed, t, i, 0) % len(S0)]
            if first == g["prev"][0]:
                second = S1_after_ri[_draw(seed, t, i, 1) % len(S1_after_ri)]
                key = (first, second)
            else:
                key = (first,)
            seen.add(key)
            assert (int(r["idx"][i]), int(r["ssd"][i])) == g["answer"], (seed, t, i)
            assert int(r["iters"][i]) == g["iters"][key], (seed, t, i, key)
    # the queries reach three-anchor paths and two-anchor paths that start
    # with an anchor other than r_i
    assert any(g["iters"][k] == 3 for k in seen)
    assert any(k[0] != g["prev"][0] and g["iters"][k] == 2 for k in seen)


def test_paper_without_anchors_is_the_first_ring():
    """With L above n no anchor is drawn: the answer is the (SSD, index)
    minimum over r_i and the references whose distance to r_i lies in the
    fat ring, computed here from numpy distances."""
    rng = np.random.default_rng(21)
    ref = rng.integers(0, 256, (150, 9), dtype=np.uint8)
    q = rng.integers(0, 256, (60, 9), dtype=np.uint8)
    prev = rng.integers(0, 150, 60)
    _, r = _paper(ref, q, prev, L=1000)
    R = ref.astype(np.int64)
    for i in range(60):
        c = int(((q[i].astype(np.int64) - R[prev[i]]) ** 2).sum())
        a = ((R - R[prev[i]]) ** 2).sum(1)
        S = set(np.nonzero((9 * c <= 16 * a) & (16 * a <= 25 * c))[0]) | {int(prev[i])}
        S = sorted(S)
        d = ((R[S] - q[i].astype(np.int64)) ** 2).sum(1)
        j = int(np.lexsort((S, d))[0])
        assert r["idx"][i] == S[j] and r["ssd"][i] == d[j] and r["iters"][i] == 0


def test_paper_invariants_and_determinism():
    """The answer lies in r_i's first ring or is r_i; runs are reproducible
    for a seed; the anchor count only grows when |S| >= L was reached."""
    wl = gen.make_workload("tiny", frames=2)
    P = oracle.extract(wl.frame(1), 8, 1)[:400]
    rng = np.random.default_rng(2)
    prev = rng.integers(0, len(wl.ref), len(P)).astype(np.int32)
    pt = oracle.PaperTables(wl.ref)
    a = pt.search(P, prev, L=20, seed=11, t=1)
    b = pt.search(P, prev, L=20, seed=11, t=1)
    assert all(np.array_equal(a[k], b[k]) for k in a)
    R = wl.ref.astype(np.int64)
    for i in range(0, 400, 7):
        c = int(((P[i].astype(np.int64) - R[prev[i]]) ** 2).sum())
        ai = int(pt.dm[prev[i], a["idx"][i]])
        assert a["idx"][i] == prev[i] or (9 * c <= 16 * ai <= 25 * c)
    assert a["iters"].max() > 0
    bi, bd = oracle.brute_force(P, wl.ref)
    assert np.all(a["ssd"] >= bd)


# ---------------------------------------------------------------- 3D patches
def test_extract3d_position_code():
    """Spatio-temporal patches: frame t holds the value 50*t + (y*W + x) % 50
    at (y, x), so every byte names its frame and position; checked against
    the definition element by element, with T = 1 reducing to the 2D case."""
    H, W, T, p, s = 9, 11, 3, 3, 2
    yy, xx = np.mgrid[0:H, 0:W]
    frames = [((50 * t + (yy * W + xx) % 50) % 256).astype(np.uint8) for t in range(T)]
    P = oracle.extract3d(frames, p, s)
    hq, wq = oracle.field_shape(H, W, p, s)
    assert P.shape == (hq * wq, p * p * T)
    for q in (0, 5, hq * wq - 1):
        i, j = divmod(q, wq)
        k = 0
        for dy in range(p):
            for dx in range(p):
                for t in range(T):
                    assert P[q, k] == frames[t][s * i + dy, s * j + dx]
                    k += 1
    np.testing.assert_array_equal(oracle.extract3d(frames[:1], p, s), oracle.extract(frames[0], p, s))


# ---------------------------------------------------------------- reconstruction
def test_reconstruct_hand_example():
    """Sec. 4 reconstruction worked by hand: 3x3 frame, 2x2 patches, stride
    1, references all-0 and all-4, field [[0, 1], [1, 1]].  Each pixel is the
    mean of the patches covering it; E against an all-4 frame is
    sqrt((16 + 4 + 4 + 1) / (9 * 16)) = 5/12."""
    app = np.array([[0] * 4, [4] * 4], np.uint8)
    field = np.array([[0, 1], [1, 1]], np.int32)
    gt = np.full((3, 3), 4, np.uint8)
    r = oracle.reconstruct(field, app, 2, 1, 3, 3, gt=gt)
    np.testing.assert_array_equal(r["f_r"][:, :, 0], [[0, 2, 4], [2, 3, 4], [4, 4, 4]])
    np.testing.assert_array_equal(r["count"], [[1, 2, 1], [2, 4, 2], [1, 2, 1]])
    assert r["sq_err"] == 25.0 and r["sq_gt"] == 144.0 and r["values"] == 9
    assert abs(r["E"] - 5.0 / 12.0) < 1e-15


def test_reconstruct_field_entries_outside_the_set():
    """Field entries outside [0, n) name no reference and contribute no
    patch (worked by hand): 3x3 frame, 2x2 patches, references all-0 and
    all-4 (n = 2), field [[0, -1], [7, 1]].  Only the top-left patch (0s)
    and the bottom-right patch (4s) are placed; the centre pixel averages
    them to 2, pixels (0, 2) and (2, 0) stay uncovered."""
    app = np.array([[0] * 4, [4] * 4], np.uint8)
    field = np.array([[0, -1], [7, 1]], np.int32)
    gt = np.full((3, 3), 4, np.uint8)
    r = oracle.reconstruct(field, app, 2, 1, 3, 3, gt=gt)
    np.testing.assert_array_equal(r["count"], [[1, 1, 0], [1, 2, 1], [0, 1, 1]])
    np.testing.assert_array_equal(r["f_r"][:, :, 0], [[0, 0, 0], [0, 2, 4], [0, 4, 4]])
    # covered pixels: errors 4, 4, 4, 2, 0, 0, 0 -> 16 * 3 + 4 = 52 over 7 values
    assert r["sq_err"] == 52.0 and r["sq_gt"] == 112.0 and r["values"] == 7


@pytest.mark.parametrize("H,W,p,s", [(9, 13, 3, 1), (20, 17, 4, 2), (16, 16, 8, 3), (5, 5, 5, 1)])
def test_reconstruct_identity_and_coverage(H, W, p, s):
    """Replacing every patch by itself gives the frame back on every covered
    pixel (E = 0); the coverage count is the product of the row and column
    counts #{i : s*i <= y <= s*i + p - 1}."""
    rng = np.random.default_rng(H * W + p)
    f = rng.integers(0, 256, (H, W), dtype=np.uint8)
    P = oracle.extract(f, p, s)
    hq, wq = oracle.field_shape(H, W, p, s)
    r = oracle.reconstruct(np.arange(hq * wq, dtype=np.int32).reshape(hq, wq), P, p, s, H, W,
                           gt=f)
    cy = np.array([sum(1 for i in range(hq) if s * i <= y <= s * i + p - 1) for y in range(H)])
    cx = np.array([sum(1 for j in range(wq) if s * j <= x <= s * j + p - 1) for x in range(W)])
    np.testing.assert_array_equal(r["count"], np.outer(cy, cx))
    cov = r["count"] > 0
    np.testing.assert_array_equal(r["f_r"][:, :, 0][cov], f[cov].astype(np.float32))
    assert np.all(r["f_r"][:, :, 0][~cov] == 0)
    assert r["E"] == 0.0 and r["values"] == int(cov.sum())


def test_reconstruct_transformed_references():
    """Patch replacement with a transformed reference set (Sec. 5): matching
    on gray patches, replacing with 3-channel versions whose channel c is
    (c+1) * value // 4; with every patch matched to itself the output is
    that transform of the frame, channel by channel."""
    rng = np.random.default_rng(3)
    f = rng.integers(0, 256, (12, 10), dtype=np.uint8)
    P = oracle.extract(f, 4, 2)
    hq, wq = oracle.field_shape(12, 10, 4, 2)
    app = np.stack([(P.astype(np.int32) * (c + 1)) // 4 for c in range(3)],
                   axis=-1).reshape(len(P), -1).astype(np.uint8)
    r = oracle.reconstruct(np.arange(hq * wq, dtype=np.int32).reshape(hq, wq), app, 4, 2, 12, 10)
    cov = r["count"] > 0
    for c in range(3):
        want = (f.astype(np.int32) * (c + 1)) // 4
        np.testing.assert_array_equal(r["f_r"][:, :, c][cov], want[cov].astype(np.float32))


# ---------------------------------------------------------------- planted faults
def _pins_pass():
    """Cheap versions of the pins above; True when all hold."""
    try:
        test_extract_position_code()
        test_extract_matches_numpy_windows(13, 10, 3, 3, 2)
        test_hand_example_extract_and_nn()
        test_bf_matches_pure_python()
        test_ring_bounds_hand()
        test_ring_bounds_exhaustive_small()
        test_tables_hand()
        test_riann_hand()
        test_riann_equals_brute_force(10, 6, "random")
        test_reconstruct_hand_example()
        test_extract3d_position_code()
        test_knn_riann_equals_brute_force(5)
        test_paper_hand_examples()
        test_paper_anchor_loop_golden()
        test_reconstruct_field_entries_outside_the_set()
    except AssertionError:
        return False
    return True


@pytest.mark.parametrize("fault", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13])
def test_planted_faults(fault):
    assert _pins_pass()
    oracle.set_fault(fault)
    try:
        caught = not _pins_pass()
    finally:
        oracle.set_fault(0)
    assert caught, f"planted fault {fault} was not caught by any pin"
    assert _pins_pass()
