"""GPU parity at the workloads' own sizes, through the C ABI, against the CPU
oracle.

* 720p: one whole frame with every query through the ring path (routing
  threshold n), compared with the oracle's brute force at every query, and
  the ring statistics (sum of m*, sum of |S|) with the oracle's exact-mode
  RIANN run on the same previous field; another frame at the default routing
  on 65,536 sampled queries.
* 1080p RGB (n = 65,536, K = 32) and 4K 12x12 stride 2 (n = 262,144,
  K = 48): the ring path forced (threshold n), so the smallest-ring search,
  the ring scan and the survivor check run at full n, on sampled queries.
* The uneven batch: one riann_match_batch of a 4K frame together with four
  640x360 frames, eager and captured in a HIP graph (replayed with new
  frames), sampled against brute force.
* The serving mix: 640x360 / 1280x720 / 1920x1080 RGB streams through the
  server, each field identical to the stream's plain per-frame search and
  sampled against brute force.

Integer work: fields and SSDs must match bit for bit.
"""
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


def sample(rng, hq, wq, m):
    """m random field positions plus the first and last field rows."""
    sel = rng.choice(hq * wq, min(m, hq * wq), replace=False)
    edge = np.concatenate([np.arange(min(wq, 256)), hq * wq - 1 - np.arange(min(wq, 256))])
    return np.unique(np.concatenate([sel, edge]))


def check_sampled(out, ssd, frame, ref, p, s, wq, sel, what):
    ys, xs = (sel // wq) * s, (sel % wq) * s
    P = gen.patches_at(frame, ys, xs, p)
    bi, bd = oracle.brute_force(P, ref)
    gi, gd = host(out)[sel], host(ssd)[sel].astype(np.uint32)
    bad = np.nonzero((gi != bi) | (gd != bd))[0]
    assert bad.size == 0, (f"{what}: {bad.size}/{sel.size} sampled queries differ; first "
                           f"q={sel[bad[0]]} got ({gi[bad[0]]},{gd[bad[0]]}) want "
                           f"({bi[bad[0]]},{bd[bad[0]]})")


def test_hd720_whole_ring_frame_and_stats(env):
    torch, riann, dev = env
    print_case("hd720 whole frame, ring path")
    wl = gen.make_workload("hd720", frames=3)
    n = len(wl.ref)
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1,
                            flags=riann.FLAG_EXACT_MSTAR)
    f0, f1, f2 = (wl.frame(t) for t in range(3))
    d0, d1, d2 = (torch.from_numpy(f).to(dev) for f in (f0, f1, f2))
    prev, _ = idx.full_search(d0)
    idx.set_dense_threshold(n)               # every query through the ring scan
    idx.reset_stats()
    out, ssd = idx.match_frame(d1, prev=prev)
    st = idx.stats()
    P = oracle.extract(f1, 8, 1)
    assert len(P) == 907_649
    bi, bd = oracle.brute_force(P, wl.ref)
    gi, gd = host(out), host(ssd).astype(np.uint32)
    bad = np.nonzero((gi != bi) | (gd != bd))[0]
    assert bad.size == 0, f"{bad.size} of {len(P)} queries differ, first {bad[:5]}"
    # ring statistics: the oracle's exact-mode RIANN with the same previous field
    o = oracle.Tables(wl.ref, wl.keys).riann(P, host(prev))
    assert np.array_equal(o["idx"], bi) and np.array_equal(o["ssd"], bd)
    assert st["ring_queries"] == len(P) - int(o["noprior"].sum())
    assert st["dense_queries"] == int(o["noprior"].sum()) == st["dense_routed"]
    assert st["sum_mstar"] == int(o["mstar"].sum()) == st["sum_mstar_ring"]
    assert st["sum_survivors"] == int(o["nsurv"].sum())
    assert st["bound_routed"] == 0
    # every evaluated ring costs two searches of at least one line read each
    assert st["bsearch_probes"] >= 2 * st["ring_queries"]
    print(f"  mean m* {st['sum_mstar'] / len(P):.0f}, mean |S| "
          f"{st['sum_survivors'] / len(P):.0f}, probes/query {st['bsearch_probes'] / len(P):.1f}",
          flush=True)
    # the next frame at the default routing, 65,536 sampled queries
    idx.set_dense_threshold(max(64, n // 16))      # the library's default routing
    out2, ssd2 = idx.match_frame(d2, prev=out)
    torch.cuda.synchronize()
    rng = np.random.default_rng(41)
    hq, wq = idx.field_shape(720, 1280)
    check_sampled(out2, ssd2, f2, wl.ref, 8, 1, wq, sample(rng, hq, wq, 65_536), "hd720 frame 2")
    idx.close()


@pytest.mark.parametrize("name,rows,nsamp", [("fhd_rgb", None, 65_536),
                                             ("uhd_mix", 200, 32_768)])
def test_large_ring_path_forced(env, name, rows, nsamp):
    """The ring path at full n: frame 0 full search, frame 1 with every
    query ring-scanned (threshold n).  The 4K case runs a 3840 x 200 band of
    the frames (the scan of every 4K query at n = 262,144 takes seconds)."""
    torch, riann, dev = env
    print_case(f"{name} ring path forced")
    wl = gen.make_workload(name, frames=2)
    n = len(wl.ref)
    idx = riann.Index.build(wl.ref, wl.keys, patch=wl.patch, channels=wl.channels,
                            stride=wl.stride, flags=riann.FLAG_EXACT_MSTAR)
    fr = [wl.frame(t) for t in range(2)]
    if rows is not None:
        fr = [np.ascontiguousarray(f[:rows]) for f in fr]
    d = [torch.from_numpy(f).to(dev) for f in fr]
    H, W = fr[0].shape[:2]
    hq, wq = idx.field_shape(H, W)
    prev, _ = idx.full_search(d[0])
    idx.set_dense_threshold(n)
    idx.reset_stats()
    out, ssd = idx.match_frame(d[1], prev=prev)
    st = idx.stats()
    assert st["ring_queries"] + st["dense_queries"] == hq * wq
    assert st["dense_queries"] == st["no_prior"]
    print(f"  {hq * wq} queries, mean m* {st['sum_mstar'] / (hq * wq):.0f} of {n}, mean |S| "
          f"{st['sum_survivors'] / max(1, st['ring_queries']):.0f}", flush=True)
    rng = np.random.default_rng(43)
    sel = sample(rng, hq, wq, nsamp)
    check_sampled(out, ssd, fr[1], wl.ref, wl.patch, wl.stride, wq, sel, f"{name} frame 1")
    # the ring statistics of the sampled queries, from the oracle's RIANN
    ys, xs = (sel // wq) * wl.stride, (sel % wq) * wl.stride
    o = oracle.Tables(wl.ref, wl.keys).riann(gen.patches_at(fr[1], ys, xs, wl.patch),
                                             host(prev)[sel])
    assert np.array_equal(o["idx"], host(out)[sel])
    idx.close()


def test_uneven_batch_4k_and_360p_eager_and_graph(env):
    """One riann_match_batch of a 3840x2160 frame and four 640x360 frames
    (12x12 patches, stride 2, n = 262,144, K = 48): frame 0 of each video by
    full search, frame 1 by the ring path with the batch's own previous
    fields; eager, then captured in a HIP graph and replayed with frame 2."""
    torch, riann, dev = env
    print_case("uneven batch 4K + 4 x 360p, eager and graph")
    wl = gen.make_workload("uhd_mix", frames=3)
    vids = [wl.video] + [gen.make_video("uhd_mix", stream=1 + i, H=360, W=640, frames=3)
                         for i in range(4)]
    frames = [[v.frame(t) for t in range(3)] for v in vids]
    idx = riann.Index.build(wl.ref, wl.keys, patch=12, channels=1, stride=2)
    shapes = [idx.field_shape(f[0].shape[0], f[0].shape[1]) for f in frames]
    outs = [[torch.empty(s, dtype=torch.int32, device=dev) for _ in range(3)] for s in shapes]
    ssds = [[torch.empty(s, dtype=torch.int32, device=dev) for _ in range(3)] for s in shapes]
    dframes = [[torch.from_numpy(f).to(dev) for f in fv] for fv in frames]

    def items(t, mode):
        it = []
        for v in range(len(vids)):
            d = dict(frame=dframes[v][t], out=outs[v][t], ssd=ssds[v][t], mode=mode)
            if mode == riann.MODE_RING:
                d["prev"] = outs[v][t - 1]
            it.append(d)
        return it

    idx.match_batch(items(0, riann.MODE_FULL))
    idx.match_batch(items(1, riann.MODE_RING))
    torch.cuda.synchronize()
    rng = np.random.default_rng(47)
    for v in range(len(vids)):
        hq, wq = shapes[v]
        m = 8_192 if v == 0 else 2_048
        for t in (0, 1):
            check_sampled(outs[v][t], ssds[v][t], frames[v][t], wl.ref, 12, 2, wq,
                          sample(rng, hq, wq, m), f"video {v} frame {t}")
    # graph: capture the ring batch of frame 2 on a warmed stream, replay it
    s = torch.cuda.Stream()
    f_in = [torch.empty_like(dframes[v][2]) for v in range(len(vids))]
    with torch.cuda.stream(s):
        cap = []
        for v in range(len(vids)):
            f_in[v].copy_(dframes[v][1])
            cap.append(dict(frame=f_in[v], out=outs[v][2], ssd=ssds[v][2], prev=outs[v][0],
                            mode=riann.MODE_RING))
        idx.match_batch(cap, stream=s)              # warm-up: sizes the stream's scratch
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        idx.match_batch(cap, stream=s)
    eager = [idx.match_frame(dframes[v][2], prev=outs[v][0]) for v in range(len(vids))]
    torch.cuda.synchronize()
    for rep in range(3):
        for v in range(len(vids)):
            f_in[v].copy_(dframes[v][2])
            outs[v][2].fill_(-3)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for v in range(len(vids)):
            assert torch.equal(outs[v][2], eager[v][0]), f"replay {rep} video {v}"
            assert torch.equal(ssds[v][2], eager[v][1]), f"replay {rep} video {v}"
    for v in range(len(vids)):
        hq, wq = shapes[v]
        check_sampled(outs[v][2], ssds[v][2], frames[v][2], wl.ref, 12, 2, wq,
                      sample(rng, hq, wq, 4_096 if v == 0 else 1_024), f"graph video {v}")
    idx.close()


def test_serving_mix_at_size(env):
    """Three RGB streams of the serving workload's sizes (640x360, 1280x720,
    1920x1080; n = 65,536, K = 32) through the server in one mix: every
    field equals the stream's plain per-frame search, and frames are sampled
    against brute force."""
    torch, riann, dev = env
    from paper_1508_07953_amd import serve
    print_case("serving mix 360p/720p/1080p RGB")
    wl = gen.make_workload("serving")
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=3, stride=1)
    nfr = 3
    vids = [gen.make_video("serving", stream=s, H=gen.serving_stream_shape(s)[0],
                           W=gen.serving_stream_shape(s)[1], frames=nfr) for s in range(3)]
    frames = [[v.frame(t) for t in range(nfr)] for v in vids]
    dframes = [[torch.from_numpy(f).to(dev) for f in fv] for fv in frames]
    plain = []
    for fv in dframes:
        prev, res = None, []
        for f in fv:
            o, s_ = idx.full_search(f) if prev is None else idx.match_frame(f, prev=prev)
            res.append((o, s_))
            prev = o
        plain.append(res)
    torch.cuda.synchronize()
    srv = serve.Server(idx, max_batch=8, inflight=2)
    sids = [srv.open_stream(*gen.serving_stream_shape(s)) for s in range(3)]
    got = {}
    for t in range(nfr):
        n0 = len(srv.completed)
        for si, fv in zip(sids, frames):
            # host frames in pinned memory, as live streams deliver them
            srv.submit(si, torch.from_numpy(fv[t]).pin_memory())
        srv.drain()
        for c in srv.completed[n0:]:
            got[(c.stream, c.seq)] = (c.field.clone(), c.ssd.clone())
    torch.cuda.synchronize()
    for k, si in enumerate(sids):
        for t in range(nfr):
            o, s_ = got[(si, t)]
            assert torch.equal(o, plain[k][t][0]) and torch.equal(s_, plain[k][t][1]), (k, t)
    rng = np.random.default_rng(53)
    for k, t, m in ((0, 2, 16_384), (1, 1, 16_384), (2, 2, 32_768)):
        H, W = gen.serving_stream_shape(k)
        hq, wq = idx.field_shape(H, W)
        o, s_ = got[(sids[k], t)]
        check_sampled(o, s_, frames[k][t], wl.ref, 8, 1, wq, sample(rng, hq, wq, m),
                      f"stream {k} frame {t}")
    idx.close()
