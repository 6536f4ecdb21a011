"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Fields and SSDs must match the oracle's exact nearest neighbours bit for bit
(integer work: no tolerance).  Ring statistics must equal the oracle's
per-query counts summed the same way.
"""
import os
import tempfile

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def riann():
    import paper_1508_07953_amd as r
    return r


def to_dev(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def host(t):
    return t.cpu().numpy().reshape(-1)


def check_exact(out, ssd, P, ref, what=""):
    bi, bd = oracle.brute_force(P, ref)
    gi, gd = host(out), host(ssd).astype(np.uint32)
    bad = np.nonzero((gi != bi) | (gd != bd))[0]
    assert bad.size == 0, (f"{what}: {bad.size}/{bi.size} differ; first q={bad[0]} "
                           f"got ({gi[bad[0]]},{gd[bad[0]]}) want ({bi[bad[0]]},{bd[bad[0]]})")
    return bi, bd


def print_case(name):
    print(f"[gpu case] {name}", flush=True)


# ------------------------------------------------------------------ tiny video
def test_tiny_sequence_exact_and_stats(torch_dev, riann):
    torch, dev = torch_dev
    print_case("tiny sequence")
    wl = gen.make_workload("tiny")
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1,
                            flags=riann.FLAG_EXACT_MSTAR)
    tabs = oracle.Tables(wl.ref, wl.keys)
    thr = idx.params.dense_threshold
    prev = None
    want = dict(queries=0, ring=0, mstar=0, surv=0, mstar_ring=0, noprior=0)
    for t in range(wl.frames):
        f = wl.frame(t)
        P = oracle.extract(f, 8, 1)
        fd = to_dev(torch, dev, f)
        if prev is None:
            out, ssd = idx.full_search(fd)
            want["queries"] += len(P)
        else:
            out, ssd = idx.match_frame(fd, prev=prev)
            o = tabs.riann(P, host(prev))
            ring = (o["mstar"] <= thr) & (o["noprior"] == 0)
            want["queries"] += len(P)
            want["ring"] += int(ring.sum())
            want["mstar"] += int(o["mstar"].sum())
            want["surv"] += int(o["nsurv"][ring].sum())
            want["mstar_ring"] += int(o["mstar"][ring].sum())
            want["noprior"] += int(o["noprior"].sum())
        torch.cuda.synchronize()
        check_exact(out, ssd, P, wl.ref, f"frame {t}")
        prev = out.clone()
    st = idx.stats()
    assert st["frames"] == wl.frames
    assert st["queries"] == want["queries"]
    assert st["ring_queries"] == want["ring"]
    assert st["dense_queries"] == want["queries"] - want["ring"]
    assert st["sum_mstar"] == want["mstar"]
    assert st["sum_survivors"] == want["surv"]
    assert st["sum_mstar_ring"] == want["mstar_ring"]
    assert st["no_prior"] == want["noprior"]
    assert st["bound_routed"] == 0
    ring_phase = want["queries"] - 3249                 # frame 0 is a full search
    assert st["dense_routed"] == ring_phase - want["ring"]
    # every query with a prior searches at least one key's ring: two binary
    # searches, each ending in one line read
    assert st["bsearch_probes"] >= 2 * (ring_phase - want["noprior"])
    idx.close()


@pytest.mark.parametrize("thr", [0, 64, 1 << 30])
@pytest.mark.parametrize("prev_kind", ["random", "noprior", "mixed", "exact"])
def test_tiny_routes_and_prev(torch_dev, riann, thr, prev_kind):
    torch, dev = torch_dev
    print_case(f"tiny thr={thr} prev={prev_kind}")
    wl = gen.make_workload("tiny")
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1,
                            dense_threshold=thr)
    f = wl.frame(3)
    P = oracle.extract(f, 8, 1)
    rng = np.random.default_rng(99)
    if prev_kind == "random":
        prev = gen.random_field(57, 57, len(wl.ref), rng)
    elif prev_kind == "noprior":
        prev = np.full((57, 57), -1, np.int32)
    elif prev_kind == "mixed":
        prev = gen.random_field(57, 57, len(wl.ref), rng, no_prior_p=0.2)
        prev[rng.random((57, 57)) < 0.1] = len(wl.ref) + 7
    else:
        prev = oracle.brute_force(P, wl.ref)[0].reshape(57, 57)
    out, ssd = idx.match_frame(to_dev(torch, dev, f), prev=to_dev(torch, dev, prev))
    torch.cuda.synchronize()
    check_exact(out, ssd, P, wl.ref, f"thr={thr} prev={prev_kind}")
    idx.close()


# ------------------------------------------------------------------ shapes
SHAPES = [
    # p, C, s, n, K, H, W
    (3, 1, 1, 100, 4, 19, 23),
    (8, 3, 1, 500, 8, 40, 37),
    (12, 1, 2, 777, 12, 50, 61),
    (5, 2, 3, 64, 0, 30, 30),
    (16, 1, 1, 300, 5, 40, 40),
    (2, 1, 1, 33, 3, 9, 10),
    (8, 1, 1, 1, 1, 8, 8),
    (4, 3, 1, 2100, 64, 23, 29),
]


@pytest.mark.parametrize("flags", [0, 1, 4])      # default, column dense, gather scan
@pytest.mark.parametrize("p,C,s,n,K,H,W", SHAPES)
def test_shapes_exact(torch_dev, riann, p, C, s, n, K, H, W, flags):
    torch, dev = torch_dev
    print_case(f"shape p={p} C={C} s={s} n={n} K={K} H={H} W={W} flags={flags}")
    rng = np.random.default_rng(p * 1000 + n)
    big = np.clip(np.rint(gen.texture(rng, max(H, p + 40), max(W, p + 40), C)), 0, 255)
    big = big.astype(np.uint8)
    hq0, wq0 = oracle.field_shape(big.shape[0], big.shape[1], p, 1)
    n_eff = min(n, hq0 * wq0)
    ref = gen.reference_from_frame(big, n_eff, p, 1, rng)
    keys = gen.choose_keys(n_eff, min(K, n_eff), rng)
    f = np.clip(np.rint(gen.texture(rng, H, W, C) + rng.normal(0, 3, (H, W, C))), 0, 255)
    f = f.astype(np.uint8)
    P = oracle.extract(f, p, s)
    hq, wq = oracle.field_shape(H, W, p, s)
    for thr in (-1, 1 << 30):
        idx = riann.Index.build(ref, keys, patch=p, channels=C, stride=s, dense_threshold=thr,
                                flags=flags)
        fd = to_dev(torch, dev, f)
        out, ssd = idx.full_search(fd)
        torch.cuda.synchronize()
        bi, _ = check_exact(out, ssd, P, ref, "full")
        prev = gen.random_field(hq, wq, n_eff, rng, no_prior_p=0.1)
        out2, ssd2 = idx.match_frame(fd, prev=to_dev(torch, dev, prev))
        torch.cuda.synchronize()
        check_exact(out2, ssd2, P, ref, f"ring thr={thr}")
        out3, ssd3 = idx.match_frame(fd, prev=out)
        torch.cuda.synchronize()
        check_exact(out3, ssd3, P, ref, f"ring(prev=exact) thr={thr}")
        out4, ssd4 = idx.match_frame(fd, prev=None)
        torch.cuda.synchronize()
        check_exact(out4, ssd4, P, ref, f"ring(no prev) thr={thr}")
        idx.close()


@pytest.mark.parametrize("flags", [0, 1])
def test_ties_and_constant_frame(torch_dev, riann, flags):
    torch, dev = torch_dev
    print_case("ties")
    rng = np.random.default_rng(5)
    ref = rng.integers(0, 256, (300, 64), dtype=np.uint8)
    ref[[7, 100, 250]] = 90               # three identical constant patches
    ref[[3, 200]] = ref[150]              # duplicates of a textured patch
    f = np.full((20, 24, 1), 90, np.uint8)
    f[10:18, 14:22, 0] = ref[150].reshape(8, 8)
    P = oracle.extract(f, 8, 1)
    for thr in (-1, 0, 1 << 30):
        idx = riann.Index.build(ref, [150, 7, 42, 250], patch=8, channels=1, stride=1,
                                dense_threshold=thr, flags=flags)
        fd = to_dev(torch, dev, f)
        out, ssd = idx.full_search(fd)
        torch.cuda.synchronize()
        bi, bd = check_exact(out, ssd, P, ref, "full ties")
        assert bi[0] == 7 and bd[0] == 0
        hq, wq = oracle.field_shape(20, 24, 8, 1)
        assert bi[10 * wq + 14] == 3 and bd[10 * wq + 14] == 0   # lowest of 3, 150, 200
        prev = np.full((hq, wq), 250, np.int32)
        out2, ssd2 = idx.match_frame(fd, prev=to_dev(torch, dev, prev))
        torch.cuda.synchronize()
        check_exact(out2, ssd2, P, ref, "ring ties")
        idx.close()


def test_pitched_frame(torch_dev, riann):
    torch, dev = torch_dev
    print_case("pitch")
    wl = gen.make_workload("tiny")
    f = wl.frame(2)
    wide = np.zeros((64, 100, 1), np.uint8)
    wide[:, 10:74] = f
    wd = to_dev(torch, dev, wide)
    view = wd[:, 10:74]
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    out, ssd = idx.full_search(view)
    out2, ssd2 = idx.match_frame(view, prev=out)
    torch.cuda.synchronize()
    P = oracle.extract(f, 8, 1)
    check_exact(out, ssd, P, wl.ref, "pitched full")
    check_exact(out2, ssd2, P, wl.ref, "pitched ring")
    idx.close()


def test_repeat_determinism(torch_dev, riann):
    torch, dev = torch_dev
    print_case("determinism")
    wl = gen.make_workload("tiny")
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    fd = to_dev(torch, dev, wl.frame(4))
    rng = np.random.default_rng(3)
    prev = to_dev(torch, dev, gen.random_field(57, 57, 1024, rng))
    res = []
    for _ in range(5):
        o, s = idx.match_frame(fd, prev=prev)
        res.append((host(o).copy(), host(s).copy()))
    for o, s in res[1:]:
        assert np.array_equal(o, res[0][0]) and np.array_equal(s, res[0][1])
    idx.close()


def test_errors(torch_dev, riann):
    torch, dev = torch_dev
    print_case("errors")
    wl = gen.make_workload("tiny")
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    fd = to_dev(torch, dev, wl.frame(0))
    buf = torch.zeros((57, 57), dtype=torch.int32, device=dev)
    with pytest.raises(riann.RiannError) as e:
        idx.match_frame(fd, prev=buf, out=buf)
    assert e.value.status == riann.RIANN_E_INVALID
    small = torch.zeros((4, 4), dtype=torch.uint8, device=dev)
    with pytest.raises(riann.RiannError):
        idx.full_search(small)
    with pytest.raises(riann.RiannError):
        riann.Index.build(wl.ref, [1, 1], patch=8)
    with pytest.raises(riann.RiannError):
        riann.Index.build(wl.ref, [5000], patch=8)
    # batch items are checked before any launch: an undersized or mistyped
    # output or previous field
    good = torch.empty((57, 57), dtype=torch.int32, device=dev)
    sentinel = torch.full((57, 57), -5, dtype=torch.int32, device=dev)
    bad_items = [dict(out=torch.empty((56, 57), dtype=torch.int32, device=dev)),
                 dict(out=torch.empty((57, 57), dtype=torch.int64, device=dev)),
                 dict(out=good, ssd=torch.empty((57, 57, 2), dtype=torch.int32, device=dev)),
                 dict(out=good, prev=torch.empty((57, 56), dtype=torch.int32, device=dev))]
    for bad in bad_items:
        with pytest.raises(ValueError):
            idx.match_batch([dict(frame=fd, out=sentinel), dict(frame=fd, **bad)])
    torch.cuda.synchronize()
    assert bool((sentinel == -5).all())         # nothing was launched
    idx.close()


def test_profiling_levels(torch_dev, riann):
    """Every kernel is timed at the full level, only the dense search at the
    dense level; turning profiling on resets the totals; other levels are
    rejected; results are unchanged while timing."""
    torch, dev = torch_dev
    print_case("profiling levels")
    wl = gen.make_workload("tiny")
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    f0, f1 = wl.frame(0), wl.frame(1)
    d0, d1 = to_dev(torch, dev, f0), to_dev(torch, dev, f1)
    idx.set_profiling(True)
    o0, _ = idx.full_search(d0)
    o1, s1 = idx.match_frame(d1, prev=o0)
    p = idx.profile()
    # the ring kernel scans its own ring queries in the default layout; the
    # full search of an 8x8 gray frame cuts its patches in the dense kernel
    assert all(p[k]["launches"] == 1 for k in ("ring", "dense", "full")), p
    assert p["scan"]["launches"] == 0 and p["extract"]["launches"] == 1, p
    g = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1,
                          flags=riann.FLAG_GATHER_SCAN)
    g.set_profiling(True)
    g.match_frame(d1, prev=o0)
    pg = g.profile()
    assert all(pg[k]["launches"] == 1 for k in ("ring", "scan", "dense", "extract")), pg
    g.close()
    # threshold 0: every query with a prior goes dense on m* >= 1, no ring
    # launch, and (8x8 gray) no extraction launch either
    z = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1, dense_threshold=0)
    z.set_profiling(True)
    oz, sz = z.match_frame(d1, prev=o0)
    pz = z.profile()
    assert pz["ring"]["launches"] == 0 and pz["scan"]["launches"] == 0, pz
    assert pz["extract"]["launches"] == 0 and pz["dense"]["launches"] == 1, pz
    torch.cuda.synchronize()
    check_exact(oz, sz, oracle.extract(f1, 8, 1), wl.ref, "threshold 0 frame")
    z.close()
    assert all(p[k]["ms"] > 0 for k in ("dense", "full", "extract")), p
    idx.set_profiling("dense")
    idx.match_frame(d1, prev=o0)
    idx.full_search(d0)
    p = idx.profile()
    assert p["dense"]["launches"] == 1 and p["full"]["launches"] == 1, p
    assert all(p[k]["launches"] == 0 for k in ("ring", "scan", "extract")), p
    idx.set_profiling(False)
    assert riann.lib().riann_set_profiling(idx._h, 7) == riann.RIANN_E_INVALID
    torch.cuda.synchronize()
    check_exact(o1, s1, oracle.extract(f1, 8, 1), wl.ref, "profiled frame")
    idx.close()


def test_save_load_roundtrip(torch_dev, riann):
    torch, dev = torch_dev
    print_case("save/load")
    wl = gen.make_workload("tiny")
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    fd = to_dev(torch, dev, wl.frame(5))
    rng = np.random.default_rng(8)
    prev = to_dev(torch, dev, gen.random_field(57, 57, 1024, rng))
    o1, s1 = idx.match_frame(fd, prev=prev)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "idx.bin")
        idx.save(path)
        idx2 = riann.Index.load(path)
        o2, s2 = idx2.match_frame(fd, prev=prev)
        torch.cuda.synchronize()
        assert np.array_equal(host(o1), host(o2)) and np.array_equal(host(s1), host(s2))
        assert idx2.params.n_ref == 1024 and idx2.params.n_keys == len(wl.keys)
        idx2.close()
    idx.close()


def test_batch_matches_single(torch_dev, riann):
    torch, dev = torch_dev
    print_case("batch")
    wl = gen.make_workload("tiny")
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    rng = np.random.default_rng(4)
    frames = [wl.frame(t) for t in range(3)]
    frames.append(np.ascontiguousarray(frames[1][:40, :50]))
    items, singles = [], []
    for i, f in enumerate(frames):
        fd = to_dev(torch, dev, f)
        hq, wq = oracle.field_shape(f.shape[0], f.shape[1], 8, 1)
        prev = to_dev(torch, dev, gen.random_field(hq, wq, 1024, rng, no_prior_p=0.2))
        out = torch.empty((hq, wq), dtype=torch.int32, device=dev)
        ssd = torch.empty((hq, wq), dtype=torch.int32, device=dev)
        mode = riann.MODE_FULL if i == 0 else riann.MODE_RING
        items.append(dict(frame=fd, prev=prev, out=out, ssd=ssd, mode=mode))
        if mode == riann.MODE_FULL:
            singles.append(idx.full_search(fd))
        else:
            singles.append(idx.match_frame(fd, prev=prev))
    idx.match_batch(items)
    torch.cuda.synchronize()
    for it, (o, s), f in zip(items, singles, frames):
        assert np.array_equal(host(it["out"]), host(o))
        assert np.array_equal(host(it["ssd"]), host(s))
        check_exact(it["out"], it["ssd"], oracle.extract(f, 8, 1), wl.ref, "batch")
    idx.close()


# ------------------------------------------------------------------ full size, sampled
def test_hd720_sampled(torch_dev, riann):
    torch, dev = torch_dev
    print_case("hd720 sampled")
    wl = gen.make_workload("hd720", frames=3)
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    rng = np.random.default_rng(11)
    prev = None
    for t in range(3):
        f = wl.frame(t)
        fd = to_dev(torch, dev, f)
        if prev is None:
            out, ssd = idx.full_search(fd)
        else:
            out, ssd = idx.match_frame(fd, prev=prev)
        torch.cuda.synchronize()
        P = oracle.extract(f, 8, 1)
        assert len(P) == 907_649
        sel = np.sort(rng.choice(len(P), 65_536, replace=False))
        sel = np.concatenate([sel, [0, len(P) - 1]])
        bi, bd = oracle.brute_force(P[sel], wl.ref)
        gi, gd = host(out)[sel], host(ssd)[sel].astype(np.uint32)
        assert np.array_equal(gi, bi) and np.array_equal(gd, bd), f"frame {t}"
        prev = out.clone()
    idx.close()


def test_batch_many_uneven_frames(torch_dev, riann):
    """More frames than one launch holds, mixed sizes and modes, ssd omitted
    on some: every field equals the oracle's brute force."""
    torch, dev = torch_dev
    print_case("batch many uneven")
    wl = gen.make_workload("tiny")
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    rng = np.random.default_rng(21)
    base = [wl.frame(t) for t in range(4)]
    items, frames = [], []
    for i in range(45):
        h = int(rng.integers(8, 65))
        w_ = int(rng.integers(8, 65))
        y0 = int(rng.integers(0, 65 - h))
        x0 = int(rng.integers(0, 65 - w_))
        f = np.ascontiguousarray(base[i % 4][y0:y0 + h, x0:x0 + w_])
        frames.append(f)
        hq, wq = oracle.field_shape(h, w_, 8, 1)
        it = dict(frame=to_dev(torch, dev, f),
                  out=torch.full((hq, wq), -7, dtype=torch.int32, device=dev),
                  mode=riann.MODE_FULL if i % 5 == 0 else riann.MODE_RING)
        if i % 3:
            it["ssd"] = torch.empty((hq, wq), dtype=torch.int32, device=dev)
        if i % 4:
            it["prev"] = to_dev(torch, dev, gen.random_field(hq, wq, 1024, rng, no_prior_p=0.2))
        items.append(it)
    idx.match_batch(items)
    torch.cuda.synchronize()
    for i, (it, f) in enumerate(zip(items, frames)):
        P = oracle.extract(f, 8, 1)
        bi, bd = oracle.brute_force(P, wl.ref)
        assert np.array_equal(host(it["out"]), bi), f"frame {i}"
        if "ssd" in it:
            assert np.array_equal(host(it["ssd"]).astype(np.uint32), bd), f"frame {i}"
    # overlapping outputs of two frames are rejected before any launch
    o = items[1]["out"]
    bad = [dict(frame=items[1]["frame"], out=o, mode=riann.MODE_RING),
           dict(frame=items[1]["frame"], out=o, mode=riann.MODE_RING)]
    with pytest.raises(riann.RiannError):
        idx.match_batch(bad)
    idx.close()


@pytest.mark.parametrize("name,nsamp", [("fhd_rgb", 1500), ("uhd_mix", 800)])
def test_large_workloads_sampled(torch_dev, riann, name, nsamp):
    """1080p RGB (D=192, n=65,536) and 4K 12x12 stride-2 (D=144, n=262,144):
    frame 0 full search and frame 1 ring search at full size, with the
    launch configuration the benchmark uses; sampled queries vs brute force,
    plus every query of the first and last rows of the field."""
    torch, dev = torch_dev
    print_case(f"{name} sampled")
    wl = gen.make_workload(name, frames=2)
    idx = riann.Index.build(wl.ref, wl.keys, patch=wl.patch, channels=wl.channels,
                            stride=wl.stride)
    rng = np.random.default_rng(13)
    prev = None
    for t in range(2):
        f = wl.frame(t)
        fd = to_dev(torch, dev, f)
        if prev is None:
            out, ssd = idx.full_search(fd)
        else:
            out, ssd = idx.match_frame(fd, prev=prev)
        torch.cuda.synchronize()
        hq, wq = idx.field_shape(f.shape[0], f.shape[1])
        sel = np.sort(rng.choice(hq * wq, nsamp, replace=False))
        sel = np.unique(np.concatenate([sel, np.arange(min(wq, 200)),
                                        hq * wq - 1 - np.arange(min(wq, 200))]))
        ys, xs = (sel // wq) * wl.stride, (sel % wq) * wl.stride
        P = gen.patches_at(f, ys, xs, wl.patch)
        bi, bd = oracle.brute_force(P, wl.ref)
        gi, gd = host(out)[sel], host(ssd)[sel].astype(np.uint32)
        assert np.array_equal(gi, bi) and np.array_equal(gd, bd), f"{name} frame {t}"
        prev = out.clone()
    idx.close()


@pytest.mark.parametrize("name", ["hd720", "tiny", "fhd_rgb"])
def test_row_and_column_dense_agree_everywhere(torch_dev, riann, name):
    """Whole-frame full search by the row-layout dense kernel (class-ordered
    references, candidate check) and by the column-layout kernel (index-order
    keys): identical at every query; a sample also against brute force."""
    torch, dev = torch_dev
    print_case(f"row vs column dense {name}")
    wl = gen.make_workload(name, frames=2)
    a = riann.Index.build(wl.ref, wl.keys, patch=wl.patch, channels=wl.channels,
                          stride=wl.stride)
    b = riann.Index.build(wl.ref, wl.keys, patch=wl.patch, channels=wl.channels,
                          stride=wl.stride, flags=riann.FLAG_COLUMN_DENSE)
    f = wl.frame(1)
    fd = to_dev(torch, dev, f)
    oa, sa = a.full_search(fd)
    ob, sb = b.full_search(fd)
    torch.cuda.synchronize()
    assert torch.equal(oa, ob) and torch.equal(sa, sb)
    rng = np.random.default_rng(17)
    P = oracle.extract(f, wl.patch, wl.stride)
    sel = np.sort(rng.choice(len(P), min(len(P), 2000), replace=False))
    bi, bd = oracle.brute_force(P[sel], wl.ref)
    assert np.array_equal(host(oa)[sel], bi) and np.array_equal(host(sa)[sel].astype(np.uint32), bd)
    a.close()
    b.close()


def test_tuned_threshold_keeps_results(torch_dev, riann, tmp_path, monkeypatch):
    """The autotuner only moves the ring/dense routing threshold: the field
    after tuning equals brute force, and the cached choice is re-applied."""
    from paper_1508_07953_amd import tune
    torch, dev = torch_dev
    print_case("autotuned threshold")
    monkeypatch.setenv("RIANN_TUNE_CACHE", str(tmp_path / "tune.json"))
    wl = gen.make_workload("tiny", frames=3)
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    f = [to_dev(torch, dev, wl.frame(t)) for t in range(3)]
    p0, _ = idx.full_search(f[0])
    p1, _ = idx.match_frame(f[1], prev=p0)
    r = tune.tune_threshold(idx, [f[1], f[2]], [p0, p1], candidates=(0, 32, 1 << 30),
                            repeats=1)
    assert not r["cached"] and r["threshold"] in (0, 32, int(idx.params.n_ref))
    out, ssd = idx.match_frame(f[2], prev=p1)
    torch.cuda.synchronize()
    check_exact(out, ssd, oracle.extract(wl.frame(2), 8, 1), wl.ref, "tuned")
    idx.set_dense_threshold(7)
    r2 = tune.tune_threshold(idx, [f[1]], [p0])
    assert r2["cached"] and idx.params.dense_threshold == r["threshold"]
    idx.close()


@pytest.mark.parametrize("flags", [0, 1])
def test_minimum_split_over_two_tiles(torch_dev, riann, flags):
    """References whose SSDs to a query differ by one share the row layout's
    half-distance Y; placed in different tiles they must be resolved across
    both tiles (and at equal SSD the lower index wins)."""
    torch, dev = torch_dev
    print_case(f"two-tile minimum flags={flags}")
    rng = np.random.default_rng(23)
    n = 600
    ref = rng.integers(0, 256, (n, 64), dtype=np.uint8)
    q = rng.integers(20, 236, (4, 64), dtype=np.uint8)

    def near(p, d):                       # SSD(p, near(p, d)) == d for d <= 3
        r = p.astype(np.int64).copy()
        r[:d] += 1
        return r.astype(np.uint8)
    # query 0: SSD 1 in tile 2, SSD 2 in tile 9; query 1: SSD 2 in tile 3, 3 in tile 12;
    # query 2: SSD 0 in tiles 5 and 17 (exact tie: lower index); query 3: SSD 1 then 0
    plan = [(0, 70, 1), (0, 300, 2), (1, 100, 2), (1, 390, 3), (2, 170, 0), (2, 550, 0),
            (3, 40, 1), (3, 500, 0)]
    for qi, r, d in plan:
        ref[r] = near(q[qi], d)
    f = np.zeros((8, 4 * 8, 1), np.uint8)
    for qi in range(4):
        f[:, 8 * qi:8 * qi + 8, 0] = q[qi].reshape(8, 8)
    P = oracle.extract(f, 8, 1)
    idx = riann.Index.build(ref, [0, 1, 2], patch=8, channels=1, stride=1, flags=flags)
    out, ssd = idx.full_search(to_dev(torch, dev, f))
    torch.cuda.synchronize()
    bi, bd = check_exact(out, ssd, P, ref, "two-tile")
    assert list(bi[[0, 8, 16, 24]]) == [70, 100, 170, 500]
    assert list(bd[[0, 8, 16, 24]]) == [1, 2, 0, 0]
    idx.close()


def test_spatiotemporal_patches(torch_dev, riann):
    """p x p x T space-time patches (the 3D extension of Sec. 1): frames
    t-2..t stacked on the device, matched by an index over 3D reference
    patches, equal the oracle's brute force over its own 3D extraction."""
    torch, dev = torch_dev
    print_case("space-time patches T=3")
    T, p = 3, 6
    wl = gen.make_workload("tiny", frames=6)
    other = gen.make_video("tiny", frames=T, second=True)
    R3 = oracle.extract3d([other.frame(t) for t in range(T)], p, 1)
    rng = np.random.default_rng(31)
    ref = R3[np.sort(rng.choice(len(R3), 700, replace=False))]
    keys = np.sort(rng.choice(len(ref), 6, replace=False))
    idx = riann.Index.build(ref, keys, patch=p, channels=T, stride=1)
    frames = [to_dev(torch, dev, wl.frame(t)) for t in range(6)]
    prev = None
    for t in range(T - 1, 6):
        st = riann.stack_frames(frames[t - T + 1:t + 1])
        torch.cuda.synchronize()
        want_stack = np.stack([wl.frame(k)[:, :, 0] for k in range(t - T + 1, t + 1)], axis=-1)
        assert np.array_equal(st.cpu().numpy(), want_stack)
        if prev is None:
            out, ssd = idx.full_search(st)
        else:
            out, ssd = idx.match_frame(st, prev=prev)
        P = oracle.extract3d([wl.frame(k) for k in range(t - T + 1, t + 1)], p, 1)
        check_exact(out, ssd, P, ref, f"3D t={t}")
        prev = out.clone()
    idx.close()


def _near(p, d):
    """A patch at SSD d (<= 3 changed bytes) from p."""
    r = p.astype(np.int64).copy()
    r[:d] += 1
    return r.astype(np.uint8)


def _with_sum_parity(q, par):
    q = q.copy()
    if int(q.astype(np.int64).sum()) % 2 != par:
        q[-1] += 1
    return q


@pytest.mark.parametrize("flags", [0, 1])
def test_class_order_ties(torch_dev, riann, flags):
    """The row layout orders references by the parity of Rc (even first).
    For one query a reference's class is fixed by its SSD's parity, and SSDs
    s and s + 1 share the half-distance Y when s - Qc is even: here the
    smaller SSD always belongs to the later index, in the other class, and
    equal SSDs (one class) must still resolve to the lower index."""
    torch, dev = torch_dev
    print_case("class-order ties")
    rng = np.random.default_rng(41)
    n = 700
    ref = rng.integers(0, 256, (n, 64), dtype=np.uint8)
    q = rng.integers(20, 236, (4, 64), dtype=np.uint8)
    q[0] = _with_sum_parity(q[0], 0)     # X(2) even: SSD 2 and 3 share Y
    q[1] = _with_sum_parity(q[1], 1)     # X(1) even: SSD 1 and 2 share Y
    q[2] = _with_sum_parity(q[2], 0)     # X(0) even: SSD 0 and 1 share Y
    q[3] = _with_sum_parity(q[3], 1)     # X(0) odd: SSD 0 alone
    plan = [(0, 30, 3), (0, 600, 2), (1, 50, 2), (1, 650, 1),
            (2, 10, 1), (2, 60, 0), (2, 200, 0), (3, 90, 0), (3, 95, 1), (3, 400, 0)]
    for qi, r, d in plan:
        ref[r] = _near(q[qi], d)
    f = np.zeros((8, 4 * 8, 1), np.uint8)
    for qi in range(4):
        f[:, 8 * qi:8 * qi + 8, 0] = q[qi].reshape(8, 8)
    P = oracle.extract(f, 8, 1)
    idx = riann.Index.build(ref, [0, 1, 2], patch=8, channels=1, stride=1, flags=flags,
                            dense_threshold=-1)
    fd = to_dev(torch, dev, f)
    out, ssd = idx.full_search(fd)
    torch.cuda.synchronize()
    bi, bd = check_exact(out, ssd, P, ref, "class ties")
    assert list(bi[[0, 8, 16, 24]]) == [600, 650, 60, 90]
    assert list(bd[[0, 8, 16, 24]]) == [2, 1, 0, 0]
    hq, wq = oracle.field_shape(8, 32, 8, 1)
    prev = rng.integers(0, n, (hq, wq)).astype(np.int32)
    out2, ssd2 = idx.match_frame(fd, prev=to_dev(torch, dev, prev))
    torch.cuda.synchronize()
    check_exact(out2, ssd2, P, ref, "class ties, ring frame")
    idx.close()


def test_row_layout_two_key_segments(torch_dev, riann):
    """n = 40,000 at D = 64: more tiles than one 10-bit tile field keys, so
    each query's running key is folded into its (Y, tile) minimum between two
    segments (and small frames also split the range over blocks, merged by
    the resolve kernel); a duplicate in the second segment must lose to its
    lower-index twin."""
    torch, dev = torch_dev
    print_case("row layout split n=40000")
    rng = np.random.default_rng(43)
    n = 40000
    ref = rng.integers(0, 256, (n, 64), dtype=np.uint8)
    base = rng.integers(0, 256, (32, 48, 1), dtype=np.uint8)
    R0 = oracle.extract(base, 8, 1)
    ref[5] = R0[100]
    ref[39000] = R0[100]
    ref[20001] = R0[700]
    ref[39999] = R0[707]
    f = np.clip(base.astype(np.int32) + rng.integers(-1, 2, base.shape), 0, 255).astype(np.uint8)
    f[:8, :8] = base[:8, :8]
    P = oracle.extract(f, 8, 1)
    idx = riann.Index.build(ref, [0, 7, 9000, 30000], patch=8, channels=1, stride=1,
                            dense_threshold=-1)
    fd = to_dev(torch, dev, f)
    out, ssd = idx.full_search(fd)
    torch.cuda.synchronize()
    bi, bd = check_exact(out, ssd, P, ref, "split full")
    hq, wq = oracle.field_shape(32, 48, 8, 1)
    prev = rng.integers(-1, n, (hq, wq)).astype(np.int32)
    out2, ssd2 = idx.match_frame(fd, prev=to_dev(torch, dev, prev))
    torch.cuda.synchronize()
    check_exact(out2, ssd2, P, ref, "split ring")
    idx.close()


def test_row_layout_three_key_segments(torch_dev, riann):
    """n = 140,000 at D = 32: three segments of 2,048 tiles (11-bit tile
    field); duplicates in the first and last segments resolve to the lower
    index, and a reference that only the last segment holds is found."""
    torch, dev = torch_dev
    print_case("n=140000 D=32 three key segments")
    rng = np.random.default_rng(47)
    n = 140000
    ref = rng.integers(0, 256, (n, 32), dtype=np.uint8)
    base = rng.integers(0, 256, (20, 24, 2), dtype=np.uint8)
    R0 = oracle.extract(base, 4, 1)
    ref[139999] = R0[40]
    ref[77] = R0[41]
    ref[5] = R0[42]
    ref[139998] = R0[42]
    P = oracle.extract(base, 4, 1)
    idx = riann.Index.build(ref, [0, 1], patch=4, channels=2, stride=1, dense_threshold=-1)
    out, ssd = idx.full_search(to_dev(torch, dev, base))
    torch.cuda.synchronize()
    bi, bd = check_exact(out, ssd, P, ref, "n=140000")
    assert bi[40] == 139999 and bd[40] == 0
    assert bi[42] == 5 and bd[42] == 0
    b2 = riann.Index.build(ref, [0, 1], patch=4, channels=2, stride=1,
                           flags=riann.FLAG_COLUMN_DENSE)
    o2, s2 = b2.full_search(to_dev(torch, dev, base))
    torch.cuda.synchronize()
    assert torch.equal(out, o2) and torch.equal(ssd, s2)
    b2.close()
    idx.close()


RING_CASES = [  # p, C, K, n: the ring phase's register-bound (K <= 16, Dp <= 64) and general paths
    (8, 1, 8, 1500),
    (4, 2, 16, 2000),
    (8, 1, 24, 1800),
    (6, 1, 40, 1200),
    (8, 3, 8, 900),
    (8, 3, 32, 1300),
]


@pytest.mark.parametrize("scan", ["rows", "gather"])
@pytest.mark.parametrize("p,C,K,n", RING_CASES)
def test_ring_stats_both_paths(torch_dev, riann, p, C, K, n, scan):
    """Per-key bucket bounds must leave m* and the survivor counts exactly
    the oracle's (all K rings evaluated), whichever key-selection path runs;
    every query with a prior is sent to the ring scan, so a wrong k* or range
    would also break the exact field.  Both scan layouts: the ring-ordered
    pivot rows (default, row lengths 8/16/32/48 words here) and the gather
    through the sorted list's index."""
    torch, dev = torch_dev
    print_case(f"ring stats p={p} C={C} K={K} n={n} scan={scan}")
    rng = np.random.default_rng(1000 * p + K)
    H, W = 30, 41
    base = rng.integers(0, 256, (H + 40, W + 40, C), dtype=np.uint8)
    f = np.clip(base[2:H + 2, 1:W + 1].astype(np.int32) + rng.integers(-4, 5, (H, W, C)),
                0, 255).astype(np.uint8)
    R = oracle.extract(base, p, 1)
    ref = R[np.sort(rng.choice(len(R), n, replace=False))]
    ref[11] = ref[3]
    keys = np.sort(rng.choice(n, K, replace=False))
    idx = riann.Index.build(ref, keys, patch=p, channels=C, stride=1, dense_threshold=n,
                            flags=riann.FLAG_GATHER_SCAN if scan == "gather" else 0)
    P = oracle.extract(f, p, 1)
    hq, wq = oracle.field_shape(H, W, p, 1)
    prev = rng.integers(-1, n, (hq, wq)).astype(np.int32)
    prev[::3] = oracle.brute_force(P[::1], ref)[0].reshape(hq, wq)[::3]   # some exact priors
    idx.reset_stats()
    out, ssd = idx.match_frame(to_dev(torch, dev, f), prev=to_dev(torch, dev, prev))
    torch.cuda.synchronize()
    check_exact(out, ssd, P, ref, "ring stats")
    o = oracle.Tables(ref, keys).riann(P, prev.reshape(-1))
    ring = o["noprior"] == 0
    st = idx.stats()
    assert st["sum_mstar"] == int(o["mstar"].sum())
    assert st["ring_queries"] == int(ring.sum())
    assert st["sum_survivors"] == int(o["nsurv"][ring].sum())
    assert st["no_prior"] == int(o["noprior"].sum())
    assert st["bound_routed"] == 0          # threshold n: no ring bound exceeds it
    idx.close()


@pytest.mark.parametrize("p,C,K,n", [(8, 1, 16, 1500), (8, 3, 32, 1300)])
@pytest.mark.parametrize("thr", [0, 8, 64, 300])
def test_bound_routing_keeps_routing(torch_dev, riann, p, C, K, n, thr):
    """By default a query whose ring-size lower bounds all exceed the
    threshold goes dense without its exact m*.  The field, the ring/dense
    split, the ring-scanned m* and survivor sums stay exactly the oracle's;
    the m* left out of the sum belong to bound-routed queries, each above the
    threshold.  With the exact-m* flag nothing is bound-routed and the sum is
    the oracle's."""
    torch, dev = torch_dev
    print_case(f"bound routing p={p} C={C} K={K} n={n} thr={thr}")
    rng = np.random.default_rng(7000 + 10 * K + thr)
    H, W = 30, 41
    base = rng.integers(0, 256, (H + 40, W + 40, C), dtype=np.uint8)
    f = np.clip(base[2:H + 2, 1:W + 1].astype(np.int32) + rng.integers(-4, 5, (H, W, C)),
                0, 255).astype(np.uint8)
    R = oracle.extract(base, p, 1)
    ref = R[np.sort(rng.choice(len(R), n, replace=False))]
    keys = np.sort(rng.choice(n, K, replace=False))
    P = oracle.extract(f, p, 1)
    hq, wq = oracle.field_shape(H, W, p, 1)
    prev = rng.integers(-1, n, (hq, wq)).astype(np.int32)
    prev[::2] = oracle.brute_force(P, ref)[0].reshape(hq, wq)[::2]      # tight rings too
    o = oracle.Tables(ref, keys).riann(P, prev.reshape(-1))
    ring = (o["mstar"] <= thr) & (o["noprior"] == 0)
    total = int(o["mstar"].sum())
    for flags in (0, riann.FLAG_EXACT_MSTAR):
        idx = riann.Index.build(ref, keys, patch=p, channels=C, stride=1, dense_threshold=thr,
                                flags=flags)
        out, ssd = idx.match_frame(to_dev(torch, dev, f), prev=to_dev(torch, dev, prev))
        torch.cuda.synchronize()
        check_exact(out, ssd, P, ref, f"bound routing flags={flags}")
        st = idx.stats()
        assert st["ring_queries"] == int(ring.sum())
        assert st["dense_queries"] == len(P) - int(ring.sum())
        assert st["sum_mstar_ring"] == int(o["mstar"][ring].sum())
        assert st["sum_survivors"] == int(o["nsurv"][ring].sum())
        assert st["no_prior"] == int(o["noprior"].sum())
        b = st["bound_routed"]
        if flags:
            assert b == 0 and st["sum_mstar"] == total
        else:
            assert b <= st["dense_queries"] - st["no_prior"]
            assert total - st["sum_mstar"] >= (thr + 1) * b
            assert (b == 0) == (st["sum_mstar"] == total)
            if thr == 0:
                # m* >= 1 for every query with a prior (its nearest neighbour
                # lies in every ring): all of them go dense on that bound
                assert b == len(P) - st["no_prior"]
                assert st["ring_queries"] == 0 and st["sum_mstar"] == n * st["no_prior"]
        idx.close()
