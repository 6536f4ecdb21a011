"""GPU parity of the dense search's last round, against the oracle's brute
force: a launch with more query chunks than resident blocks runs a last round
of at most an eighth of the slots as paired half-size blocks whose
wavefronts split the reference tiles and merge their minima in LDS.  Frame
sizes put the chunk count just past one round (a ragged last chunk), at the
largest paired last round, and one chunk beyond it (run whole); each case
runs a full search (patches cut in the dense kernel), a ring frame at the
default routing threshold and at threshold 0 (its routing counts as well) and a
two-frame batch (patches from the extraction kernel), and compares the last chunks' queries, all of them, plus a sample of
the rest.  Integer work: fields and SSDs bit for bit."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

BLOCK_Q = 512            # queries per chunk of the default 8x8 gray block shape


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1508_07953_amd as riann
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch, riann, torch.device("cuda:0")


def host(t):
    return t.cpu().numpy().reshape(-1)


def check(frame, out, ssd, ref, sel, what):
    hq, wq = out.shape
    P = gen.patches_at(frame, sel // wq, sel % wq, 8)
    bi, bd = oracle.brute_force(P, ref)
    gi, gd = host(out)[sel], host(ssd)[sel].astype(np.uint32)
    bad = np.nonzero((gi != bi) | (gd != bd))[0]
    assert bad.size == 0, (f"{what}: {bad.size}/{sel.size} differ; first q={sel[bad[0]]} "
                           f"got ({gi[bad[0]]},{gd[bad[0]]}) want ({bi[bad[0]]},{bd[bad[0]]})")


def selection(Q, tail_q, rng):
    """Every query of the last tail_q, and 8,192 of the others."""
    t0 = max(0, Q - tail_q)
    rest = rng.choice(t0, min(t0, 8192), replace=False) if t0 else np.zeros(0, np.int64)
    return np.unique(np.concatenate([np.arange(t0, Q), rest])).astype(np.int64)


# (H, W): 385 x 1023 queries = 770 chunks; 433 x 1021 = 864 chunks; 433 x
# 1022 = 865 chunks (with 768 resident blocks: last rounds of 2, 96 and 97);
# 257 x 1024 = 514 chunks (one round) -- in the other block shapes the last
# round of 1,028 chunks of 256 queries on 1,024 slots, 257 of 1,024 on 256
# and 513 of 768 on 512 (first size) are paired as well
@pytest.mark.parametrize("H,W", [(392, 1030), (440, 1028), (440, 1029), (264, 1031)])
def test_last_round(env, H, W):
    torch, riann, dev = env
    print(f"[gpu case] last round H={H} W={W}", flush=True)
    wl = gen.make_workload("hd720", H=H, W=W, frames=3)
    f = [wl.frame(t) for t in range(3)]
    d = [torch.from_numpy(x).to(dev) for x in f]
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    rng = np.random.default_rng(H * 7 + W)
    hq, wq = H - 7, W - 7
    Q = hq * wq
    chunks = -(-Q // BLOCK_Q)
    tail_q = (chunks % 768 + 1) * BLOCK_Q if chunks > 768 else Q
    sel = selection(Q, min(Q, tail_q, 100_000), rng)

    o1, s1 = idx.full_search(d[1])
    torch.cuda.synchronize()
    check(f[1], o1, s1, wl.ref, sel, "full search")

    idx.reset_stats()
    o2, s2 = idx.match_frame(d[2], prev=o1)
    torch.cuda.synchronize()
    check(f[2], o2, s2, wl.ref, sel, "ring frame")
    st = idx.stats()
    assert st["queries"] == Q and st["ring_queries"] + st["dense_queries"] == Q

    # threshold 0: every query dense, patches cut and routing counted by the
    # dense kernel itself (one wavefront of each pair counts)
    thr = idx.params.dense_threshold
    idx.set_dense_threshold(0)
    pv = host(o1).copy()
    pv[rng.random(pv.size) < 0.1] = -1
    nop = int((pv < 0).sum())
    idx.reset_stats()
    o3, s3 = idx.match_frame(d[2], prev=torch.from_numpy(pv.reshape(o1.shape)).to(dev))
    torch.cuda.synchronize()
    check(f[2], o3, s3, wl.ref, sel, "ring frame, threshold 0")
    st = idx.stats()
    assert st["queries"] == Q and st["dense_queries"] == Q and st["no_prior"] == nop
    assert st["bound_routed"] == Q - nop and st["ring_queries"] == 0
    idx.set_dense_threshold(thr)

    # two frames in one launch: 2 Q queries, patches from the extraction kernel
    outs = [torch.empty((hq, wq), dtype=torch.int32, device=dev) for _ in range(2)]
    ssds = [torch.empty((hq, wq), dtype=torch.int32, device=dev) for _ in range(2)]
    idx.match_batch([dict(frame=d[1], out=outs[0], ssd=ssds[0], mode=riann.MODE_FULL),
                     dict(frame=d[2], out=outs[1], ssd=ssds[1], prev=o1,
                          mode=riann.MODE_RING)])
    torch.cuda.synchronize()
    bchunks = -(-2 * Q // BLOCK_Q)
    btail = (bchunks % 768 + 1) * BLOCK_Q if bchunks > 768 else 2 * Q
    sel2 = selection(Q, min(Q, btail, 100_000), rng)
    check(f[1], outs[0], ssds[0], wl.ref, sel, "batch frame 0")
    check(f[2], outs[1], ssds[1], wl.ref, sel2, "batch frame 1")

    # every other block shape: the same field as the default's (checked above)
    shapes, _ = idx.dense_shapes()
    for wv, cl in shapes[1:]:
        print(f"[gpu case] last round H={H} W={W} shape {wv}x{cl}", flush=True)
        idx.set_dense_shape(wv, cl)
        o, s = idx.full_search(d[1])
        torch.cuda.synchronize()
        assert torch.equal(o, o1) and torch.equal(s, s1), f"shape {wv}x{cl}"
    idx.close()
