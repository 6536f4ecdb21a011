"""GPU parity of frame reconstruction (Sec. 4) and patch replacement with
transformed references (Sec. 5): the HIP kernel through the C ABI against the
CPU oracle on the same fields.  f_R is one float division of exact integer
sums on both sides, so it must match bit for bit; E and its sums are fp64
reductions in different orders, compared to a relative 1e-12.
"""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
RTOL_E = 1e-12


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


def check(torch, out, err, want):
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert got.dtype == np.float32 and got.shape == want["f_r"].shape
    bad = np.nonzero(got != want["f_r"])
    assert bad[0].size == 0, f"{bad[0].size} values differ, first at {[b[0] for b in bad]}"
    if err is not None:
        e = err.cpu().numpy()
        assert abs(e[0] - want["E"]) <= RTOL_E * max(want["E"], 1e-300)
        assert abs(e[1] - want["sq_err"]) <= RTOL_E * max(want["sq_err"], 1e-300)
        assert abs(e[2] - want["sq_gt"]) <= RTOL_E * want["sq_gt"]
        assert int(e[3]) == want["values"]


def print_case(name):
    print(f"[gpu case] {name}", flush=True)


def test_reconstruct_tiny_nn_field(torch_dev, riann):
    """The tiny video's frame 1 rebuilt from its exact NN field (the
    oracle's brute force), with E against the frame itself."""
    torch, d = torch_dev
    print_case("recon tiny")
    wl = gen.make_workload("tiny", frames=2)
    f = wl.frame(1)
    P = oracle.extract(f, 8, 1)
    bi, _ = oracle.brute_force(P, wl.ref)
    hq, wq = oracle.field_shape(f.shape[0], f.shape[1], 8, 1)
    field = bi.reshape(hq, wq)
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    out, err = idx.reconstruct(dev(torch, d, field), f.shape[0], f.shape[1], gt=dev(torch, d, f))
    want = oracle.reconstruct(field, wl.ref, 8, 1, f.shape[0], f.shape[1], gt=f)
    check(torch, out, err, want)
    assert 0.0 < want["E"] < 0.5
    idx.close()


SHAPES = [  # p, C, s, H, W, n, Ca (app channels; None = the references)
    (8, 1, 1, 37, 131, 300, None),
    (4, 3, 2, 50, 70, 200, None),
    (3, 1, 3, 29, 200, 100, 3),
    (16, 1, 1, 40, 80, 64, 1),
    (2, 2, 1, 17, 65, 50, 4),
    (5, 1, 2, 16, 64, 120, 2),
]


@pytest.mark.parametrize("p,C,s,H,W,n,Ca", SHAPES)
def test_reconstruct_shapes_random_fields(torch_dev, riann, p, C, s, H, W, n, Ca):
    """Seeded random fields (any valid field is a legal input) over ragged
    frame sizes, strides, channel counts and transformed appearance sets."""
    torch, d = torch_dev
    print_case(f"recon p={p} C={C} s={s} H={H} W={W} n={n} Ca={Ca}")
    rng = np.random.default_rng(p * 1000 + H)
    ref = rng.integers(0, 256, (n, p * p * C), dtype=np.uint8)
    idx = riann.Index.build(ref, [0], patch=p, channels=C, stride=s)
    hq, wq = oracle.field_shape(H, W, p, s)
    field = rng.integers(0, n, (hq, wq), dtype=np.int32)
    ca = C if Ca is None else Ca
    app = ref if Ca is None else rng.integers(0, 256, (n, p * p * Ca), dtype=np.uint8)
    gt = rng.integers(0, 256, (H, W, ca), dtype=np.uint8)
    out, err = idx.reconstruct(dev(torch, d, field), H, W,
                               app=None if Ca is None else dev(torch, d, app),
                               gt=dev(torch, d, gt))
    want = oracle.reconstruct(field, app, p, s, H, W, gt=gt)
    check(torch, out, err, want)
    # without an error request only f_R is produced
    out2, err2 = idx.reconstruct(dev(torch, d, field), H, W,
                                 app=None if Ca is None else dev(torch, d, app))
    assert err2 is None
    check(torch, out2, None, want)
    idx.close()


def test_reconstruct_hd720_full_frame(torch_dev, riann):
    """Full 1280x720 frame, 8x8 patches, n = 16,384: every pixel against the
    oracle, on a seeded random field, twice in a row (deterministic E)."""
    torch, d = torch_dev
    print_case("recon hd720")
    wl = gen.make_workload("hd720", frames=1)
    f = wl.frame(0)
    H, W = f.shape[:2]
    hq, wq = oracle.field_shape(H, W, 8, 1)
    field = np.random.default_rng(99).integers(0, len(wl.ref), (hq, wq), dtype=np.int32)
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    fd, gd = dev(torch, d, field), dev(torch, d, f)
    out, err = idx.reconstruct(fd, H, W, gt=gd)
    want = oracle.reconstruct(field, wl.ref, 8, 1, H, W, gt=f)
    check(torch, out, err, want)
    _, err_b = idx.reconstruct(fd, H, W, gt=gd)
    torch.cuda.synchronize()
    assert torch.equal(err, err_b)
    idx.close()


def test_reconstruct_field_entries_outside_the_set(torch_dev, riann):
    """Entries outside [0, n) contribute no patch: a field with a single
    valid entry rebuilds that patch in its window and 0 elsewhere."""
    torch, d = torch_dev
    print_case("recon invalid entries")
    rng = np.random.default_rng(4)
    ref = rng.integers(1, 256, (10, 16), dtype=np.uint8)
    idx = riann.Index.build(ref, [0], patch=4, channels=1, stride=1)
    field = np.full((7, 9), -1, np.int32)
    field[2, 3] = 6
    field[5, 0] = 10          # == n: outside the set
    field[0, 8] = -7
    field[6, 6] = 9
    gt = rng.integers(0, 256, (10, 12), dtype=np.uint8)
    out, err = idx.reconstruct(dev(torch, d, field), 10, 12, gt=dev(torch, d, gt))
    torch.cuda.synchronize()
    got = out.cpu().numpy()[:, :, 0]
    want = np.zeros((10, 12), np.float32)
    want[2:6, 3:7] = ref[6].reshape(4, 4)
    want[6:10, 6:10] = ref[9].reshape(4, 4)
    np.testing.assert_array_equal(got, want)
    # and the oracle, which skips the same entries
    check(torch, out, err, oracle.reconstruct(field, ref, 4, 1, 10, 12, gt=gt))
    idx.close()


def test_reconstruct_errors(torch_dev, riann):
    torch, d = torch_dev
    ref = np.zeros((4, 16), np.uint8)
    idx = riann.Index.build(ref, [0], patch=4, channels=1, stride=1)
    field = dev(torch, d, np.zeros((3, 3), np.int32))
    with pytest.raises(riann.RiannError):
        idx.reconstruct(field, 3, 6)                    # frame smaller than a patch
    with pytest.raises(riann.RiannError):              # app channels out of range
        idx.reconstruct(field, 6, 6, app=dev(torch, d, np.zeros((4, 16 * 5), np.uint8)))
    idx.close()
