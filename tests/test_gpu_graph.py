"""HIP graph capture of the per-frame search: after one warm-up call on the
capture stream (which sizes that stream's scratch), a whole match call is
captured once and replayed per frame with new inputs copied into the
captured buffers.  Every replay must equal the eager result, with eager work
and synchronisations between the replays."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def test_match_frame_graph_replays(capsys):
    import torch
    import paper_1508_07953_amd as riann
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    print("[gpu case] graph capture of match_frame", flush=True)
    wl = gen.make_workload("tiny", frames=8)
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    frames = [torch.from_numpy(wl.frame(t)).to(dev) for t in range(8)]
    f_in = torch.empty_like(frames[0])
    prev_in = torch.empty((57, 57), dtype=torch.int32, device=dev)
    out_g = torch.empty_like(prev_in)
    ssd_g = torch.empty_like(prev_in)
    s = torch.cuda.Stream()
    f0, _ = idx.full_search(frames[0])
    torch.cuda.synchronize()
    with torch.cuda.stream(s):                    # warm-up on the capture stream
        f_in.copy_(frames[1])
        prev_in.copy_(f0)
        idx.match_frame(f_in, prev=prev_in, out=out_g, ssd=ssd_g, stream=s)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        idx.match_frame(f_in, prev=prev_in, out=out_g, ssd=ssd_g, stream=s)
    prev = f0
    for t in range(1, 8):
        want, want_ssd = idx.match_frame(frames[t], prev=prev)     # eager
        torch.cuda.synchronize()
        f_in.copy_(frames[t])
        prev_in.copy_(prev)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_g, want) and torch.equal(ssd_g, want_ssd), f"replay {t}"
        P = oracle.extract(wl.frame(t), 8, 1)
        bi, bd = oracle.brute_force(P, wl.ref)
        assert np.array_equal(out_g.cpu().numpy().reshape(-1), bi)
        assert np.array_equal(ssd_g.cpu().numpy().reshape(-1).astype(np.uint32), bd)
        prev = want.clone()
    idx.close()
