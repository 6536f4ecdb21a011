"""GPU parity of exact k-NN fields (riann_match_knn) against the CPU oracle:
every query's k indices and SSDs must equal the oracle's exhaustive k-NN bit
for bit (integer work), in ascending (SSD, index) order, whatever the
previous field and whichever path (ring scan or dense search) answers it."""
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


def check_knn(torch, out, ssd, P, ref, k, what, sel=None):
    torch.cuda.synchronize()
    gi = out.cpu().numpy().reshape(-1, k)
    gd = ssd.cpu().numpy().reshape(-1, k).astype(np.uint32)
    if sel is not None:
        gi, gd, P = gi[sel], gd[sel], P[sel]
    bi, bd = oracle.knn_brute_force(P, ref, k)
    bad = np.nonzero((gi != bi).any(1) | (gd != bd).any(1))[0]
    assert bad.size == 0, (f"{what}: {bad.size}/{len(bi)} queries differ; first {bad[0]}: "
                           f"got {gi[bad[0]]} {gd[bad[0]]} want {bi[bad[0]]} {bd[bad[0]]}")
    return bi, bd


@pytest.mark.parametrize("k", [2, 4, 5, 8])
@pytest.mark.parametrize("thr", [0, 64, 1 << 30])
def test_knn_tiny_sequence(torch_dev, riann, k, thr):
    """The tiny video: frame 0 exhaustive, then ring frames whose previous
    k-NN field is the oracle's; threshold 0 sends every query to the dense
    search, 2^30 every query with a radius to the ring scan."""
    torch, d = torch_dev
    print_case(f"knn tiny k={k} thr={thr}")
    wl = gen.make_workload("tiny", frames=4)
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1, dense_threshold=thr)
    f0 = wl.frame(0)
    out, ssd = idx.match_knn(dev(torch, d, f0), k, full=True)
    prev, _ = check_knn(torch, out, ssd, oracle.extract(f0, 8, 1), wl.ref, k, "full")
    for t in range(1, 4):
        f = wl.frame(t)
        P = oracle.extract(f, 8, 1)
        out, ssd = idx.match_knn(dev(torch, d, f), k, prev=dev(torch, d, prev.reshape(57, 57, k)))
        prev, _ = check_knn(torch, out, ssd, P, wl.ref, k, f"ring t={t}")
    idx.close()


@pytest.mark.parametrize("kind", ["random", "invalid", "duplicate", "exact"])
def test_knn_previous_field_kinds(torch_dev, riann, kind):
    """Any previous field gives the exact answer: random indices, entries
    outside [0, n), repeated indices (both mean no radius), the exact k-NN."""
    torch, d = torch_dev
    print_case(f"knn prev {kind}")
    k = 3
    wl = gen.make_workload("tiny", frames=2)
    f = wl.frame(1)
    P = oracle.extract(f, 8, 1)
    rng = np.random.default_rng(12)
    n = len(wl.ref)
    if kind == "exact":
        prev, _ = oracle.knn_brute_force(P, wl.ref, k)
    else:
        prev = rng.integers(0, n, (len(P), k)).astype(np.int32)
        if kind == "invalid":
            prev[::2, 1] = -1
            prev[1::4, 0] = n
        if kind == "duplicate":
            prev[:, 2] = prev[:, 0]
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1, dense_threshold=256)
    out, ssd = idx.match_knn(dev(torch, d, f), k, prev=dev(torch, d, prev.reshape(57, 57, k)))
    check_knn(torch, out, ssd, P, wl.ref, k, kind)
    idx.close()


SHAPES = [  # p, C, s, n, K, H, W, k
    (4, 2, 1, 900, 5, 30, 41, 3),     # D = 32
    (4, 6, 2, 500, 8, 40, 33, 6),     # D = 96
    (8, 3, 1, 700, 4, 20, 70, 2),     # D = 192
    (16, 1, 3, 300, 0, 50, 47, 8),    # D = 256, no key points
]


@pytest.mark.parametrize("flags", [0, 1])
@pytest.mark.parametrize("p,C,s,n,K,H,W,k", SHAPES)
def test_knn_shapes(torch_dev, riann, p, C, s, n, K, H, W, k, flags):
    """Row layout (default) and column layout (flag 1) alike."""
    torch, d = torch_dev
    print_case(f"knn shape p={p} C={C} s={s} n={n} K={K} k={k} flags={flags}")
    rng = np.random.default_rng(p * 100 + n)
    base = rng.integers(0, 256, (H + 8, W + 8, C), dtype=np.uint8)
    f = base[:H, :W].copy()
    f2 = np.clip(base[1:H + 1, 2:W + 2].astype(np.int32) + rng.integers(-6, 7, (H, W, C)),
                 0, 255).astype(np.uint8)
    R = oracle.extract(base, p, 1)
    ref = R[np.sort(rng.choice(len(R), n, replace=False))]
    ref[7] = ref[3]                                        # duplicates: index order
    keys = np.sort(rng.choice(n, K, replace=False))
    idx = riann.Index.build(ref, keys, patch=p, channels=C, stride=s, dense_threshold=100,
                            flags=flags)
    hq, wq = oracle.field_shape(H, W, p, s)
    out, ssd = idx.match_knn(dev(torch, d, f), k, full=True)
    prev, _ = check_knn(torch, out, ssd, oracle.extract(f, p, s), ref, k, "full")
    out, ssd = idx.match_knn(dev(torch, d, f2), k, prev=dev(torch, d, prev.reshape(hq, wq, k)))
    check_knn(torch, out, ssd, oracle.extract(f2, p, s), ref, k, "ring")
    idx.close()


def test_knn_hd720_sampled(torch_dev, riann):
    """Full 720p frame, n = 16,384 (the largest set the 32-bit k-NN key
    takes at D = 64), k = 4: exhaustive frame, then a ring frame whose
    previous field is a seeded random one; 2,000 sampled queries each."""
    torch, d = torch_dev
    print_case("knn hd720 sampled")
    k = 4
    wl = gen.make_workload("hd720", frames=2)
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    rng = np.random.default_rng(5)
    for t, full in ((0, True), (1, False)):
        f = wl.frame(t)
        P = oracle.extract(f, 8, 1)
        hq, wq = oracle.field_shape(f.shape[0], f.shape[1], 8, 1)
        prev = None if full else dev(torch, d, rng.integers(0, len(wl.ref), (hq, wq, k),
                                                            dtype=np.int32))
        out, ssd = idx.match_knn(dev(torch, d, f), k, prev=prev, full=full)
        sel = np.sort(rng.choice(len(P), 2000, replace=False))
        check_knn(torch, out, ssd, P, wl.ref, k, f"hd720 t={t}", sel=sel)
    idx.close()


def test_knn_errors(torch_dev, riann):
    torch, d = torch_dev
    rng = np.random.default_rng(1)
    f = dev(torch, d, rng.integers(0, 256, (16, 16, 1), dtype=np.uint8))
    small = riann.Index.build(rng.integers(0, 256, (5, 64), dtype=np.uint8), [0], patch=8)
    with pytest.raises(riann.RiannError):
        small.match_knn(f, 6, full=True)                   # k > n
    with pytest.raises(riann.RiannError):
        small.match_knn(f, 9, full=True)                   # k > 8
    small.close()
    # n = 16,385 at D = 64: beyond the column layout's 32-bit keys, within
    # the row layout's one key segment
    ref = rng.integers(0, 256, (16385, 64), dtype=np.uint8)
    mid = riann.Index.build(ref, [0], patch=8)
    out, ssd = mid.match_knn(f, 3, full=True)
    check_knn(torch, out, ssd, oracle.extract(f.cpu().numpy(), 8, 1), ref, 3, "n=16385")
    mid.close()
    col = riann.Index.build(ref, [0], patch=8, flags=riann.FLAG_COLUMN_DENSE)
    with pytest.raises(riann.RiannError):
        col.match_knn(f, 2, full=True)                     # column key range exceeded
    col.close()
    big = riann.Index.build(rng.integers(0, 256, (33000, 64), dtype=np.uint8), [0], patch=8)
    with pytest.raises(riann.RiannError):
        big.match_knn(f, 2, full=True)                     # both key ranges exceeded
    out, ssd = big.match_knn(f, 1, full=True)              # k = 1 has no limit
    torch.cuda.synchronize()
    big.close()


@pytest.mark.parametrize("k", [2, 4, 8])
def test_knn_row_and_column_agree_hd720(torch_dev, riann, k):
    """Whole 720p frame, exhaustive k-NN by the row layout (k smallest
    class-ordered tiles, rechecked exactly) and by the column layout
    (32-bit index-order keys): identical fields and SSDs everywhere."""
    torch, d = torch_dev
    print_case(f"knn row vs column hd720 k={k}")
    wl = gen.make_workload("hd720", frames=2)
    a = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    b = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1,
                          flags=riann.FLAG_COLUMN_DENSE)
    f = dev(torch, d, wl.frame(1))
    oa, sa = a.match_knn(f, k, full=True)
    ob, sb = b.match_knn(f, k, full=True)
    torch.cuda.synchronize()
    assert torch.equal(oa, ob) and torch.equal(sa, sb)
    a.close()
    b.close()


def test_knn_class_order_ties(torch_dev, riann):
    """Duplicates and SSD neighbours that share the row layout's half
    distance Y across the two Rc classes: the k nearest still come in
    (SSD, index) order."""
    torch, d = torch_dev
    print_case("knn class-order ties")
    rng = np.random.default_rng(23)
    n = 900
    ref = rng.integers(0, 256, (n, 64), dtype=np.uint8)
    q = rng.integers(20, 236, (2, 64), dtype=np.uint8)
    for qi, base in ((0, 0), (1, 400)):
        for j, dd in enumerate((0, 1, 1, 2, 2, 3, 0, 1)):
            r = q[qi].astype(np.int64).copy()
            r[:dd] += 1
            if j % 2:
                r[-1] -= 1 if dd else 0
            ref[base + 37 * j + 5] = np.clip(r, 0, 255).astype(np.uint8)
    f = np.zeros((8, 16, 1), np.uint8)
    f[:, :8, 0] = q[0].reshape(8, 8)
    f[:, 8:, 0] = q[1].reshape(8, 8)
    idx = riann.Index.build(ref, [0, 1], patch=8)
    for k in (2, 5, 8):
        out, ssd = idx.match_knn(dev(torch, d, f), k, full=True)
        check_knn(torch, out, ssd, oracle.extract(f, 8, 1), ref, k, f"ties k={k}")
    idx.close()
