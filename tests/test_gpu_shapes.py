"""Every block shape of the row-layout dense search that the library builds
(the autotuner's choices) against the oracle's brute force, through the C
ABI: exhaustive and ring frames at every patch width, the class-order ties,
and whole 720p and 1080p RGB frames (whole and split query chunks) against
the default shape.  Integer work: fields and SSDs bit for bit."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1508_07953_amd as riann
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch, riann, torch.device("cuda:0")


def print_case(name):
    print(f"[gpu case] {name}", flush=True)


def host(t):
    return t.cpu().numpy().reshape(-1)


def exact(out, ssd, P, ref, what):
    bi, bd = oracle.brute_force(P, ref)
    gi, gd = host(out), host(ssd).astype(np.uint32)
    bad = np.nonzero((gi != bi) | (gd != bd))[0]
    assert bad.size == 0, (f"{what}: {bad.size}/{len(P)} differ; first q={bad[0]} got "
                           f"({gi[bad[0]]},{gd[bad[0]]}) want ({bi[bad[0]]},{bd[bad[0]]})")


# p, C -> Dp 32, 64, 96, 128, 160, 192, 224, 256
WIDTHS = [(4, 2), (8, 1), (9, 1), (11, 1), (12, 1), (8, 3), (14, 1), (16, 1)]


@pytest.mark.parametrize("p,C", WIDTHS)
def test_every_shape_exact(env, p, C):
    torch, riann, dev = env
    rng = np.random.default_rng(100 * p + C)
    H, W = 45, 83
    big = np.clip(np.rint(gen.texture(rng, H + 40, W + 40, C)), 0, 255).astype(np.uint8)
    n = 1500
    ref = gen.reference_from_frame(big, n, p, 1, rng)
    ref[7] = ref[900]                       # a duplicate: ties to the lower index
    keys = gen.choose_keys(n, 8, rng)
    f = np.clip(np.rint(big[3:H + 3, 2:W + 2].astype(np.float64) +
                        rng.normal(0, 3, (H, W, C))), 0, 255).astype(np.uint8)
    P = oracle.extract(f, p, 1)
    hq, wq = oracle.field_shape(H, W, p, 1)
    idx = riann.Index.build(ref, keys, patch=p, channels=C, stride=1, dense_threshold=0)
    shapes, cur = idx.dense_shapes()
    assert cur == 0 and len(shapes) >= 2
    fd = torch.from_numpy(f).to(dev)
    prev = torch.from_numpy(gen.random_field(hq, wq, n, rng, no_prior_p=0.1)).to(dev)
    for wv, cl in shapes:
        print_case(f"shape p={p} C={C} {wv}x{cl}")
        idx.set_dense_shape(wv, cl)
        assert idx.dense_shapes()[0][idx.dense_shapes()[1]] == (wv, cl)
        out, ssd = idx.full_search(fd)
        torch.cuda.synchronize()
        exact(out, ssd, P, ref, f"full {wv}x{cl}")
        out2, ssd2 = idx.match_frame(fd, prev=prev)    # threshold 0: every query dense
        torch.cuda.synchronize()
        exact(out2, ssd2, P, ref, f"ring frame {wv}x{cl}")
    with pytest.raises(riann.RiannError) as e:
        idx.set_dense_shape(5, 5)
    assert e.value.status == riann.RIANN_E_UNSUPPORTED
    idx.set_dense_shape(0, 0)
    assert idx.dense_shapes()[1] == 0
    idx.close()


@pytest.mark.parametrize("name,nsamp", [("hd720", 4096), ("fhd_rgb", 2048)])
def test_every_shape_whole_frame(env, name, nsamp):
    """A whole frame's chunks exceed the resident blocks, so each shape runs
    whole chunks and a split last round (different chunk sizes per shape):
    every shape's field equals the default shape's, sampled against brute
    force."""
    torch, riann, dev = env
    wl = gen.make_workload(name, frames=1)
    f = wl.frame(0)
    idx = riann.Index.build(wl.ref, wl.keys, patch=wl.patch, channels=wl.channels,
                            stride=wl.stride)
    fd = torch.from_numpy(f).to(dev)
    base_o, base_s = idx.full_search(fd)
    torch.cuda.synchronize()
    hq, wq = idx.field_shape(f.shape[0], f.shape[1])
    rng = np.random.default_rng(5)
    sel = np.unique(np.concatenate([rng.choice(hq * wq, nsamp, replace=False),
                                    [0, hq * wq - 1]]))
    bi, bd = oracle.brute_force(gen.patches_at(f, sel // wq, sel % wq, wl.patch), wl.ref)
    assert np.array_equal(host(base_o)[sel], bi) and np.array_equal(
        host(base_s)[sel].astype(np.uint32), bd)
    shapes, _ = idx.dense_shapes()
    for wv, cl in shapes[1:]:
        print_case(f"{name} whole frame {wv}x{cl}")
        idx.set_dense_shape(wv, cl)
        o, s = idx.full_search(fd)
        torch.cuda.synchronize()
        assert torch.equal(o, base_o) and torch.equal(s, base_s), f"{wv}x{cl}"
    idx.close()


def test_tuner_picks_a_built_shape(env, tmp_path, monkeypatch):
    torch, riann, dev = env
    from paper_1508_07953_amd import tune
    print_case("tune_shape")
    monkeypatch.setenv("RIANN_TUNE_CACHE", str(tmp_path / "tune.json"))
    wl = gen.make_workload("tiny")
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    frames = [torch.from_numpy(wl.frame(t)).to(dev) for t in range(2)]
    r = tune.tune_shape(idx, frames, repeats=1)
    shapes, cur = idx.dense_shapes()
    assert not r["cached"] and tuple(r["shape"]) == shapes[cur]
    assert set(r["ms"]) == {f"{w}x{c}" for w, c in shapes}
    r2 = tune.tune_shape(idx, frames)
    assert r2["cached"] and r2["shape"] == r["shape"]
    out, ssd = idx.full_search(frames[1])
    torch.cuda.synchronize()
    exact(out, ssd, oracle.extract(wl.frame(1), 8, 1), wl.ref, "tuned shape")
    idx.close()
