"""GPU tests of the continuous-batching server: each stream's fields are the
same alone and in the mix (exact, tolerance 0), admission by memory budget,
closing a stream while a frame is in flight."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1508_07953_amd as riann
    from paper_1508_07953_amd import serve
    assert torch.cuda.is_available()
    return torch, riann, serve, torch.device("cuda:0")


def _streams(rng, n):
    """n small RGB streams of different sizes, 4 frames each."""
    out = []
    for i in range(n):
        H = int(rng.integers(24, 70))
        W = int(rng.integers(24, 90))
        v = gen.DriftVideo(4, H, W, 3, 4, speed=0.5, stream=100 + i)
        out.append([v.frame(t) for t in range(4)])
    return out


def _ref_rgb(rng, n=700, K=12):
    tex = np.clip(np.rint(gen.texture(rng, 60, 80, 3)), 0, 255).astype(np.uint8)
    ref = gen.reference_from_frame(tex, n, 8, 1, rng)
    return ref, gen.choose_keys(n, K, rng)


@pytest.mark.parametrize("concurrent", ["auto", False, True])
def test_alone_equals_mix(env, concurrent):
    torch, riann, serve, dev = env
    print(f"[gpu case] serving alone vs mix concurrent={concurrent}", flush=True)
    rng = np.random.default_rng(31)
    ref, keys = _ref_rgb(rng)
    idx = riann.Index.build(ref, keys, patch=8, channels=3, stride=1)
    vids = _streams(rng, 7)
    dframes = [[torch.from_numpy(f).to(dev) for f in v] for v in vids]
    # alone: plain per-frame calls, one stream after another
    alone = []
    for v in dframes:
        fields, prev = [], None
        for t, f in enumerate(v):
            if prev is None:
                o, s = idx.full_search(f)
            else:
                o, s = idx.match_frame(f, prev=prev)
            torch.cuda.synchronize()
            fields.append((o.cpu().numpy().copy(), s.cpu().numpy().copy()))
            prev = o
        alone.append(fields)
    # mix: all streams through the server, frames submitted interleaved
    # batches of at most 3 frames, two batches in flight at once
    srv = serve.Server(idx, max_batch=3, inflight=2, concurrent=concurrent)
    sids = [srv.open_stream(v[0].shape[0], v[0].shape[1]) for v in vids]
    got = {}
    for t in range(4):
        n0 = len(srv.completed)
        for si, v in zip(sids, dframes):
            srv.submit(si, v[t])
            if t % 2:
                srv.step()          # batches formed with and without a backlog
        srv.drain()
        for c in srv.completed[n0:]:
            got[(c.stream, c.seq)] = (c.field.cpu().numpy().copy(), c.ssd.cpu().numpy().copy())
    for k, si in enumerate(sids):
        for t in range(4):
            o, s = got[(si, t)]
            assert np.array_equal(o, alone[k][t][0]), (k, t)
            assert np.array_equal(s, alone[k][t][1]), (k, t)
    # and the fields are the exact NN
    for k in (0, 3):
        for t in (0, 2):
            bi, bd = oracle.brute_force(oracle.extract(vids[k][t], 8, 1), ref)
            assert np.array_equal(got[(sids[k], t)][0].reshape(-1), bi)
    idx.close()


def test_admission_and_close(env):
    torch, riann, serve, dev = env
    print("[gpu case] serving admission", flush=True)
    rng = np.random.default_rng(32)
    ref, keys = _ref_rgb(rng, n=300, K=6)
    idx = riann.Index.build(ref, keys, patch=8, channels=3, stride=1)
    vids = []
    for i in range(4):
        v = gen.DriftVideo(4, 40, 56, 3, 2, speed=0.5, stream=200 + i)
        vids.append([v.frame(t) for t in range(2)])
    dframes = [[torch.from_numpy(f).to(dev) for f in v] for v in vids]
    # budget: exactly what two active streams need -- the index once, two
    # streams' buffers and, per HIP stream of the server, the scratch of a
    # batch of their two frames
    probe = serve.Server(idx)
    probe.open_stream(40, 56)
    probe.open_stream(40, 56)
    budget = probe.device_bytes()
    hq, wq = idx.field_shape(40, 56)
    two_frames = riann.footprint(300, 6, 8, 3, 1, 8, 8 + 2 * hq * wq - 1) - riann.footprint(
        300, 6, 8, 3, 1)
    assert len(probe.hip_streams) == 2              # the default: two batches in flight
    assert budget == (probe.index_bytes + 2 * probe.stream_bytes(40, 56) +
                      len(probe.hip_streams) * two_frames)
    assert probe.index_bytes == riann.footprint(300, 6, 8, 3, 1)
    srv = serve.Server(idx, memory_budget=budget)
    sids = [srv.open_stream(40, 56) for _ in vids]
    assert srv.active_streams == 2 and len(srv.waiting) == 2
    # a stream that cannot fit even alone is rejected outright
    with pytest.raises(riann.RiannError):
        srv.open_stream(400, 560)
    for si, v in zip(sids, dframes):
        srv.submit(si, v[0])
        srv.submit(si, v[1])
    srv.step()                      # frame 0 of streams 0 and 1 in flight
    srv.close_stream(sids[0])       # freed once its frame finishes; frame 1 dropped
    for _ in range(1000):
        srv.step()
        srv._collect(block=bool(srv._batches))
        s1 = srv.streams.get(sids[1])
        if s1 is not None and not s1.busy and not s1.queue:
            srv.close_stream(sids[1])
        if srv.pending() == 0:
            break
    done = {(c.stream, c.seq) for c in srv.completed}
    assert (sids[0], 0) in done and (sids[0], 1) not in done
    for si in sids[1:]:
        assert (si, 0) in done and (si, 1) in done, si
    assert srv.active_streams <= 2
    idx.close()


def test_unreferenced_and_host_frames(env):
    """Frames the caller does not keep (a fresh device copy per submit, the
    caller's memory churning meanwhile) and frames in pinned host memory
    (copied on the server's copy stream) give the exact field of every
    frame, checked against the oracle's brute force."""
    torch, riann, serve, dev = env
    print("[gpu case] serving unreferenced and host frames", flush=True)
    rng = np.random.default_rng(33)
    ref, keys = _ref_rgb(rng, n=500, K=8)
    idx = riann.Index.build(ref, keys, patch=8, channels=3, stride=1)
    vids = _streams(rng, 6)
    srv = serve.Server(idx, max_batch=4, inflight=2)
    sids = [srv.open_stream(v[0].shape[0], v[0].shape[1]) for v in vids]
    got = {}
    for t in range(4):
        n0 = len(srv.completed)
        for k, (si, v) in enumerate(zip(sids, vids)):
            if k % 2 == 0:
                srv.submit(si, torch.from_numpy(v[t]).to(dev))      # no reference kept
            else:
                srv.submit(si, torch.from_numpy(v[t]).pin_memory())
            # churn the caching allocator: same-size blocks freed and reused
            junk = [torch.full(v[t].shape, 255, dtype=torch.uint8, device=dev)
                    for _ in range(3)]
            del junk
            srv.step()
        srv.drain()
        for c in srv.completed[n0:]:
            got[(c.stream, c.seq)] = (c.field.cpu().numpy().copy(), c.ssd.cpu().numpy().copy())
    for k, si in enumerate(sids):
        for t in range(4):
            bi, bd = oracle.brute_force(oracle.extract(vids[k][t], 8, 1), ref)
            o, s = got[(si, t)]
            assert np.array_equal(o.reshape(-1), bi), (k, t)
            assert np.array_equal(s.reshape(-1).astype(np.uint32), bd), (k, t)
    idx.close()


@pytest.mark.parametrize("plain", [False, True])
def test_host_frames_and_host_results(env, plain):
    """Frames in pinned host memory and results delivered to pinned host
    memory (host_results), in the plain setting (one frame at a time) and
    the serving one: every field and SSD map on the host equals the oracle's
    brute force, and a completion's host tensors are not device tensors."""
    torch, riann, serve, dev = env
    print(f"[gpu case] serving host results plain={plain}", flush=True)
    rng = np.random.default_rng(35)
    ref, keys = _ref_rgb(rng, n=600, K=10)
    idx = riann.Index.build(ref, keys, patch=8, channels=3, stride=1)
    vids = _streams(rng, 5)
    srv = (serve.Server(idx, max_batch=1, inflight=1, host_results=True) if plain else
           serve.Server(idx, max_batch=8, inflight=2, host_results=True))
    sids = [srv.open_stream(v[0].shape[0], v[0].shape[1]) for v in vids]
    got = {}
    for t in range(4):
        n0 = len(srv.completed)
        for si, v in zip(sids, vids):
            srv.submit(si, torch.from_numpy(v[t]).pin_memory())
            srv.step()
        srv.drain()
        for c in srv.completed[n0:]:
            assert not c.field.is_cuda and not c.ssd.is_cuda
            got[(c.stream, c.seq)] = (c.field.numpy().copy(), c.ssd.numpy().copy())
    for k, si in enumerate(sids):
        for t in range(4):
            bi, bd = oracle.brute_force(oracle.extract(vids[k][t], 8, 1), ref)
            o, s = got[(si, t)]
            assert np.array_equal(o.reshape(-1), bi), (k, t)
            assert np.array_equal(s.reshape(-1).astype(np.uint32), bd), (k, t)
    idx.close()


def test_backlog_grows_batches(env):
    """With a backlog the batch cap grows to the ready queries' share per batch
    in flight (up to backlog_batch_queries); without one the base cap holds.
    Fields stay exact either way."""
    torch, riann, serve, dev = env
    print("[gpu case] serving backlog batch cap", flush=True)
    rng = np.random.default_rng(37)
    ref, keys = _ref_rgb(rng, n=500, K=8)
    idx = riann.Index.build(ref, keys, patch=8, channels=3, stride=1)
    vids = _streams(rng, 8)
    qs = [idx.field_shape(v[0].shape[0], v[0].shape[1]) for v in vids]
    qmax = max(h * w for h, w in qs)
    for grow in (True, False):
        srv = serve.Server(idx, max_batch=40, inflight=2, max_batch_queries=qmax,
                           backlog_batch_queries=10 ** 7 if grow else None)
        sids = [srv.open_stream(v[0].shape[0], v[0].shape[1]) for v in vids]
        for si, v in zip(sids, vids):
            srv.submit(si, torch.from_numpy(v[0]).to(dev))
        srv.step()
        qmap = {si: h * w for si, (h, w) in zip(sids, qs)}
        batch_q = [sum(qmap[m[0]] for m in b[2]) for b in srv._batches]
        total = sum(qmap.values())
        if grow:
            # eight ready frames, two batches in flight: the first batch's cap
            # is half the ready queries, above the base cap
            assert batch_q[0] > qmax and batch_q[0] <= max(qmax, total // 2), batch_q
        else:
            assert all(bq <= qmax for bq in batch_q), batch_q
        srv.drain()
        for c in srv.completed:
            k = sids.index(c.stream)
            bi, bd = oracle.brute_force(oracle.extract(vids[k][0], 8, 1), ref)
            assert np.array_equal(c.field.cpu().numpy().reshape(-1), bi)
            assert np.array_equal(c.ssd.cpu().numpy().reshape(-1).astype(np.uint32), bd)
    idx.close()
