"""riann_match_frame_noalloc (the entry point that allocates nothing) against
riann_match_frame, through the C ABI: two calls in a row, the second on a
smaller frame, each bit-exact against the allocating call and against the
oracle's brute force; then a frame beyond the static scratch is refused.

Integer work: fields and SSDs must match bit for bit."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def print_case(name):
    print(f"[gpu case] {name}", flush=True)


def test_noalloc_matches_match_frame_twice_then_smaller():
    import torch
    import paper_1508_07953_amd as riann
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    dev = torch.device("cuda:0")
    print_case("noalloc: 360p-size gray frame, then a smaller ragged one")
    wl = gen.make_workload("hd720", frames=3)
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=1, stride=1)
    # a 640 x 360 window of the 720p video, then a 203 x 317 window of the next frame
    shapes = [(360, 640), (203, 317)]
    f0 = np.ascontiguousarray(wl.frame(0)[:360, :640])
    prev, _ = idx.full_search(torch.from_numpy(f0).to(dev))
    rng = np.random.default_rng(71)
    for call, (H, W) in enumerate(shapes):
        f = np.ascontiguousarray(wl.frame(1 + call)[:H, :W])
        fd = torch.from_numpy(f).to(dev)
        hq, wq = idx.field_shape(H, W)
        p = prev[:hq, :wq].contiguous()
        # every fourth entry without prior, so both routes run
        p.view(-1)[::4] = -1
        want_o, want_s = idx.match_frame(fd, prev=p)
        out = torch.full((hq, wq), -7, dtype=torch.int32, device=dev)
        ssd = torch.full((hq, wq), -7, dtype=torch.int32, device=dev)
        idx.match_frame_noalloc(fd, p, out, ssd)
        torch.cuda.synchronize()
        assert torch.equal(out, want_o), f"call {call}: field differs from match_frame"
        assert torch.equal(ssd, want_s), f"call {call}: ssd differs from match_frame"
        sel = rng.choice(hq * wq, min(4096, hq * wq), replace=False)
        sel = np.unique(np.concatenate([sel, [0, hq * wq - 1]]))
        ys, xs = sel // wq, sel % wq
        bi, bd = oracle.brute_force(gen.patches_at(f, ys, xs, 8), wl.ref)
        gi = out.cpu().numpy().reshape(-1)[sel]
        gd = ssd.cpu().numpy().reshape(-1)[sel].astype(np.uint32)
        assert np.array_equal(gi, bi) and np.array_equal(gd, bd), f"call {call}: vs oracle"
        prev = torch.zeros((360 - 7, 640 - 7), dtype=torch.int32, device=dev)
        prev[:hq, :wq] = out
    # a full 720p gray frame needs more scratch than the static array holds
    big = torch.from_numpy(wl.frame(2)).to(dev)
    hq, wq = idx.field_shape(720, 1280)
    o = torch.empty((hq, wq), dtype=torch.int32, device=dev)
    s_ = torch.empty_like(o)
    with pytest.raises(riann.RiannError) as ei:
        idx.match_frame_noalloc(big, None, o, s_)
    assert ei.value.status == riann.RIANN_E_UNSUPPORTED
    assert "scratch" in str(ei.value)
    idx.close()
