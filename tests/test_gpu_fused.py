"""GPU parity of the dense search that cuts its own query patches from the
frame (8x8 one-channel patches, one frame, every query dense: a full search
or a ring frame at routing threshold 0), against the oracle's brute force:
frame rows at every byte alignment (views offset by 0-3 bytes into a wider
buffer), strides 1-3, ragged sizes, previous fields with missing entries, the
routing counts the kernel takes itself, and a whole 720p frame on sampled
queries.  Integer work: fields and SSDs bit for bit."""
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


def host(t):
    return t.cpu().numpy().reshape(-1)


def exact(out, ssd, P, ref, what):
    bi, bd = oracle.brute_force(P, ref)
    gi, gd = host(out), host(ssd).astype(np.uint32)
    bad = np.nonzero((gi != bi) | (gd != bd))[0]
    assert bad.size == 0, (f"{what}: {bad.size}/{bi.size} differ; first q={bad[0]} "
                           f"got ({gi[bad[0]]},{gd[bad[0]]}) want ({bi[bad[0]]},{bd[bad[0]]})")


@pytest.mark.parametrize("s", [1, 2, 3])
@pytest.mark.parametrize("off", [0, 1, 2, 3])
def test_fused_alignment_stride(env, s, off):
    torch, riann, dev = env
    print(f"[gpu case] fused patches stride={s} offset={off}", flush=True)
    rng = np.random.default_rng(900 + 10 * s + off)
    H, W, n, K = 53, 77, 1100, 12
    base = np.clip(np.rint(gen.texture(rng, H + 20, W + 20, 1)), 0, 255).astype(np.uint8)
    f = np.ascontiguousarray(base[3:3 + H, 5:5 + W])
    ref = gen.reference_from_frame(base, n, 8, 1, rng)
    keys = gen.choose_keys(n, K, rng)
    wide = np.zeros((H, W + 13, 1), np.uint8)
    wide[:, off:off + W] = f
    view = torch.from_numpy(wide).to(dev)[:, off:off + W]
    idx = riann.Index.build(ref, keys, patch=8, channels=1, stride=s, dense_threshold=0)
    idx.set_profiling(True)
    P = oracle.extract(f, 8, s)
    out, ssd = idx.full_search(view)
    torch.cuda.synchronize()
    exact(out, ssd, P, ref, f"full s={s} off={off}")
    prev = out.clone()
    pv = host(prev).copy()
    miss = rng.random(pv.size) < 0.2
    pv[miss] = -1
    pv[rng.random(pv.size) < 0.05] = n + 7            # out of range: no prior either
    nop = int(((pv < 0) | (pv >= n)).sum())
    prev = torch.from_numpy(pv.reshape(prev.shape)).to(dev)
    idx.reset_stats()
    out2, ssd2 = idx.match_frame(view, prev=prev)
    torch.cuda.synchronize()
    exact(out2, ssd2, P, ref, f"ring thr=0 s={s} off={off}")
    st = idx.stats()
    assert st["queries"] == len(P) and st["ring_queries"] == 0
    assert st["dense_queries"] == len(P)
    assert st["no_prior"] == nop
    assert st["bound_routed"] == len(P) - nop
    assert st["sum_mstar"] == n * nop
    prof = idx.profile()
    assert prof["extract"]["launches"] == 0, prof     # the dense kernel cut the patches
    idx.close()


def test_fused_720p_frame_sampled(env):
    torch, riann, dev = env
    print("[gpu case] fused 720p threshold 0", flush=True)
    wl = gen.make_workload("hd720", frames=3)
    f0, f1 = wl.frame(1), wl.frame(2)
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1, dense_threshold=0)
    d0, d1 = torch.from_numpy(f0).to(dev), torch.from_numpy(f1).to(dev)
    o0, _ = idx.full_search(d0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    pv = host(o0).copy()
    pv[rng.random(pv.size) < 0.1] = -1
    nop = int((pv < 0).sum())
    prev = torch.from_numpy(pv.reshape(o0.shape)).to(dev)
    idx.reset_stats()
    out, ssd = idx.match_frame(d1, prev=prev)
    torch.cuda.synchronize()
    hq, wq = out.shape
    sel = np.unique(np.concatenate([rng.choice(hq * wq, 65536, replace=False),
                                    np.arange(wq), hq * wq - 1 - np.arange(wq)]))
    P = gen.patches_at(f1, (sel // wq), (sel % wq), 8)
    bi, bd = oracle.brute_force(P, wl.ref)
    gi, gd = host(out)[sel], host(ssd)[sel].astype(np.uint32)
    bad = np.nonzero((gi != bi) | (gd != bd))[0]
    assert bad.size == 0, f"{bad.size}/{sel.size} sampled queries differ"
    st = idx.stats()
    assert st["queries"] == hq * wq and st["no_prior"] == nop
    assert st["bound_routed"] == hq * wq - nop and st["ring_queries"] == 0
    idx.close()
