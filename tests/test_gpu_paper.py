"""GPU parity of the paper's approximate search (Algorithm 1, alpha = 1/4,
random anchors, L): the HIP path must reproduce the oracle's transcription
bit for bit -- the match, its SSD and the number of anchors drawn -- since
both draw anchors from the same counter-based SplitMix64 chain and apply the
same integer ring test.  (Against values printed in the paper this mode is
unpinned: the paper prints none.)"""
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


def dev(torch, d, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(d)


def print_case(name):
    print(f"[gpu case] {name}", flush=True)


def check(torch, out, ssd, iters, want, what):
    torch.cuda.synchronize()
    gi = out.cpu().numpy().reshape(-1)
    gd = ssd.cpu().numpy().reshape(-1).astype(np.uint32)
    gn = iters.cpu().numpy().reshape(-1)
    bad = np.nonzero((gi != want["idx"]) | (gd != want["ssd"]) | (gn != want["iters"]))[0]
    assert bad.size == 0, (f"{what}: {bad.size}/{gi.size} differ; first {bad[0]}: got "
                           f"({gi[bad[0]]},{gd[bad[0]]},{gn[bad[0]]}) want ({want['idx'][bad[0]]},"
                           f"{want['ssd'][bad[0]]},{want['iters'][bad[0]]})")


@pytest.mark.parametrize("L", [20, 3])
def test_paper_tiny_sequence(torch_dev, riann, L):
    """The tiny video from a random initial field (drawn by the generator),
    each later frame from the oracle's previous field."""
    torch, d = torch_dev
    print_case(f"paper tiny L={L}")
    wl = gen.make_workload("tiny", frames=6)
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    idx.build_paper_tables()
    pt = oracle.PaperTables(wl.ref)
    prev = None
    for t in range(6):
        f = wl.frame(t)
        P = oracle.extract(f, 8, 1)
        pv = np.full(len(P), -1, np.int32) if prev is None else prev
        want = pt.search(P, pv, L=L, seed=99, t=t)
        out, ssd, iters = idx.match_paper(dev(torch, d, f),
                                          prev=None if prev is None else dev(torch, d, prev.reshape(57, 57)),
                                          L=L, seed=99, t=t)
        check(torch, out, ssd, iters, want, f"t={t}")
        prev = want["idx"]
    assert want["iters"].max() > 0
    idx.close()


SHAPES = [  # p, C, s, n, H, W, L
    (4, 2, 1, 700, 30, 41, 20),     # D = 32
    (4, 6, 2, 500, 40, 33, 5),      # D = 96
    (8, 3, 1, 900, 20, 70, 20),     # D = 192
    (16, 1, 3, 300, 50, 47, 1),     # D = 256, L = 1
    (8, 1, 1, 1500, 24, 90, 1000),  # no anchors at all
]


@pytest.mark.parametrize("p,C,s,n,H,W,L", SHAPES)
def test_paper_shapes(torch_dev, riann, p, C, s, n, H, W, L):
    torch, d = torch_dev
    print_case(f"paper shape p={p} C={C} s={s} n={n} L={L}")
    rng = np.random.default_rng(p * 7 + n)
    base = rng.integers(0, 256, (H + 8, W + 8, C), dtype=np.uint8)
    f = np.clip(base[1:H + 1, 1:W + 1].astype(np.int32) + rng.integers(-5, 6, (H, W, C)),
                0, 255).astype(np.uint8)
    R = oracle.extract(base, p, 1)
    ref = R[np.sort(rng.choice(len(R), n, replace=False))]
    ref[9] = ref[4]                                   # duplicates
    idx = riann.Index.build(ref, [0], patch=p, channels=C, stride=s)
    idx.build_paper_tables()
    pt = oracle.PaperTables(ref)
    P = oracle.extract(f, p, s)
    hq, wq = oracle.field_shape(H, W, p, s)
    prev = rng.integers(-3, n, len(P)).astype(np.int32)   # some entries invalid: drawn
    want = pt.search(P, prev, L=L, seed=5, t=3)
    out, ssd, iters = idx.match_paper(dev(torch, d, f), prev=dev(torch, d, prev.reshape(hq, wq)),
                                      L=L, seed=5, t=3)
    check(torch, out, ssd, iters, want, "shape")
    idx.close()


def test_paper_errors(torch_dev, riann):
    torch, d = torch_dev
    rng = np.random.default_rng(0)
    idx = riann.Index.build(rng.integers(0, 256, (50, 64), dtype=np.uint8), [0], patch=8)
    f = dev(torch, d, rng.integers(0, 256, (16, 16, 1), dtype=np.uint8))
    with pytest.raises(riann.RiannError):
        idx.match_paper(f)                              # tables not built
    idx.build_paper_tables()
    with pytest.raises(riann.RiannError):
        idx.match_paper(f, L=0)
    idx.close()
    big = riann.Index.build(rng.integers(0, 256, (32769, 4), dtype=np.uint8), [0], patch=2)
    with pytest.raises(riann.RiannError):
        big.build_paper_tables()                        # n above 32768
    big.close()


def test_paper_anchor_golden(torch_dev, riann):
    """The hand-worked anchor-loop example (tests/golden/paper_anchor_example.txt):
    1-pixel patches, q = 100 on every query of a 1 x 48 frame, previous
    match the reference of value 0.  Every query must return the exact copy
    (index 4, SSD 0) and draw the same anchors as the oracle."""
    torch, d = torch_dev
    print_case("paper anchor golden")
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_anchor_example.txt")
    vals = {}
    with open(path) as f:
        for line in f:
            w = line.split()
            if w and w[0] in ("ref", "q", "prev", "L"):
                vals[w[0]] = [int(x) for x in w[1:]]
    ref = np.array(vals["ref"], np.uint8).reshape(-1, 1)
    Q = 48
    idx = riann.Index.build(ref, [], patch=1, channels=1, stride=1)
    idx.build_paper_tables()
    pt = oracle.PaperTables(ref)
    frame = np.full((1, Q), vals["q"][0], np.uint8)
    prev = np.full((1, Q), vals["prev"][0], np.int32)
    for seed, t in ((5, 1), (150807953, 7)):
        out, ssd, iters = idx.match_paper(dev(torch, d, frame), prev=dev(torch, d, prev),
                                          L=vals["L"][0], seed=seed, t=t)
        want = pt.search(frame.reshape(Q, 1), prev.reshape(-1), L=vals["L"][0], seed=seed, t=t)
        assert np.all(want["idx"] == 4) and np.all(want["ssd"] == 0)
        check(torch, out, ssd, iters, want, f"anchor golden seed {seed}")
    idx.close()
