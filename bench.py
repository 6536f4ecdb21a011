#!/usr/bin/env python3
"""Benchmark of the exact RIANN search on one MI355X.

Workload (the 720p configuration): 1280x720 gray frames of the tiled
affine-motion generator (<= 1 px/frame per 64x64 tile, 10% of tiles re-seeded
every frame), all 8x8 patches at stride 1 (907,649 queries per frame),
reference set of 16,384 patches, 16 key points.  Frame 0 is answered by the
full search (untimed set-up); every timed step matches the next frame with
the previous frame's field as `prev` -- one pass of the whole per-frame path
(ring phase, ring scan, dense search of routed queries).  Frames are resident
in HBM before timing starts.

Prints one JSON line (rank 0) with throughput, latency percentiles, the
dominant kernel's roofline figures (HIP-event timing inside the timed region)
and a CPU-oracle baseline timed on this host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "query patches/sec and frames/sec at 720p + p99 frame latency (serving vs plain)"
WORKLOAD_DESC = {
    "hd720": "hd720: 1280x720 gray, 8x8 patches stride 1, %d queries/frame, n=16384 reference "
             "patches, K=16 key points, tiled affine motion, 10%% tiles re-seeded per frame",
    "fhd_rgb": "fhd_rgb: 1920x1080 RGB, 8x8x3 patches stride 1, %d queries/frame, n=65536, "
               "K=32, drifting texture, full search at scene cuts",
    "uhd_mix": "uhd_mix: 3840x2160 gray, 12x12 patches stride 2, %d queries/frame, n=262144, "
               "K=48, 20%% high-motion tiles, full search at scene cuts",
}
INT8_PEAK_TOPS = 5000.0   # MI355X dense int8 matrix peak, tera-ops/s
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def dense_traffic_bytes(workload, layout, shape):
    """HBM bytes per frame of the dense step (row kernel plus its resolve
    pass) from the committed rocprofv3 counter summary, or None when there is
    none for this workload, layout and block shape, or a kernel source changed
    since it was taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", f"{workload}_dense_traffic.json")) as f:
            rec = json.load(f)
        if rec.get("dense_layout") != layout or list(rec.get("shape", [])) != list(shape):
            return None
        for name, want in rec["sources_sha256"].items():
            with open(os.path.join(ROOT, "paper_1508_07953_amd", "csrc", name), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != want:
                    return None
    except (OSError, ValueError, KeyError, TypeError):
        return None
    return rec["bytes_per_frame"]


def cpu_baseline(wl, f0, f1, target_s):
    """Oracle exact-mode RIANN timed on the host's cores on a sample of one
    frame's queries; its previous field is the oracle's own brute force."""
    import gen
    import oracle
    p, s = wl.patch, wl.stride
    P0 = oracle.extract(f0, p, s)
    P1 = oracle.extract(f1, p, s)
    Q = len(P1)
    tabs = oracle.Tables(wl.ref, wl.keys)
    rng = np.random.default_rng(7)
    m = 2048
    elapsed, done = 0.0, 0
    while True:
        sel = rng.choice(Q, size=min(m, Q), replace=False)
        t0 = time.perf_counter()
        prev, _ = oracle.brute_force(P0[sel], wl.ref)
        dt_bf = time.perf_counter() - t0
        t0 = time.perf_counter()
        tabs.riann(P1[sel], prev)
        dt = time.perf_counter() - t0
        elapsed, done = dt, len(sel)
        if dt >= target_s * 0.5 or len(sel) >= Q:
            break
        m = int(min(Q, max(2 * m, m * target_s / max(dt, 1e-3))))
    cores = oracle.set_threads(0)
    # the same search on one core, on a smaller part of the sample
    sel1 = sel[: max(1, min(len(sel) // 10, 16384))]
    prev1, _ = oracle.brute_force(P0[sel1], wl.ref)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    tabs.riann(P1[sel1], prev1)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(cores)
    # the small configuration (64x64 frames, 1,024 references, 8 keys): every
    # frame, frame 0 by brute force, then exact-mode RIANN from its own fields
    tw = gen.make_workload("tiny")
    ttabs = oracle.Tables(tw.ref, tw.keys)
    tq, prev_t, t0 = 0, None, time.perf_counter()
    for t in range(tw.frames):
        Pt = oracle.extract(tw.frame(t), tw.patch, tw.stride)
        prev_t = (oracle.brute_force(Pt, tw.ref)[0] if prev_t is None
                  else ttabs.riann(Pt, prev_t)["idx"])
        tq += len(Pt)
    dt_tiny = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f
                          if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": done / elapsed, "unit": "patches/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} random queries of frame 1 ({Q} per frame), exact-mode RIANN "
                      f"with the oracle's brute-force field of frame 0 as prev; "
                      f"{elapsed:.2f} s wall, table build excluded",
            "single_core_value": len(sel1) / dt1,
            "single_core_sample": f"{len(sel1)} of the same queries on 1 thread, {dt1:.2f} s",
            "brute_force_value": done / dt_bf,
            "brute_force_sample": f"the oracle's brute force on the same {done} queries of "
                                  f"frame 0, {dt_bf:.2f} s",
            "tiny_value": tq / dt_tiny,
            "tiny_sample": f"every frame of the 64x64 workload ({tw.frames} frames, {tq} "
                           f"queries; frame 0 by brute force, then exact-mode RIANN from "
                           f"its own fields), {dt_tiny:.2f} s, table build excluded",
            "cpu_model": model}


def paper_mode(idx, frames, hq, wq, dev, log_fn, nframes=12, timed=6):
    """The paper's approximate Algorithm 1 (alpha = 1/4, L = 20, random
    anchors) on the same frames, started from a random field: time per frame
    once converged, and accuracy against the exact field of each frame."""
    import torch
    t0 = time.time()
    idx.build_paper_tables()
    build_s = time.time() - t0
    log_fn(f"paper tables built in {build_s:.1f}s")
    nframes = min(nframes, len(frames) - 1)
    timed = min(timed, nframes)
    prev = None
    outs = [torch.empty((hq, wq), dtype=torch.int32, device=dev) for _ in range(2)]
    ssd = torch.empty((hq, wq), dtype=torch.int32, device=dev)
    iters = torch.empty((hq, wq), dtype=torch.int32, device=dev)
    ex_out = torch.empty_like(ssd)
    ex_ssd = torch.empty_like(ssd)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms, exact, ratio, anchors = [], [], [], []
    for t in range(1, nframes + 1):
        cur = outs[t % 2]
        torch.cuda.synchronize()
        e0.record()
        idx.match_paper(frames[t], prev=prev, L=20, seed=150807953, t=t, out=cur, ssd=ssd,
                        iters=iters)
        e1.record()
        e1.synchronize()
        if t > nframes - timed:
            ms.append(e0.elapsed_time(e1))
            idx.full_search(frames[t], out=ex_out, ssd=ex_ssd)
            torch.cuda.synchronize()
            exact.append(float((cur == ex_out).float().mean().item()))
            ratio.append(float(ssd.double().mean().item() / ex_ssd.double().mean().item()))
            anchors.append(float(iters.double().mean().item()))
        prev = cur
    m = float(np.mean(ms))
    return {"L": 20, "alpha": 0.25, "ms_per_frame": m, "patches_per_s": hq * wq / (m * 1e-3),
            "exact_fraction": float(np.mean(exact)), "mean_ssd_ratio_vs_exact": float(np.mean(ratio)),
            "mean_anchors": float(np.mean(anchors)), "table_build_s": build_s,
            "frames": f"{nframes} from a random field, last {timed} timed"}


def extras(args, result, idx, wl, frames, field, H, Wd, hq, wq, Q, K, W, dev, stream, log):
    """Figures beside the headline: reconstruction (Sec. 4) with E, exact
    k-NN fields, and the paper's approximate search."""
    import torch
    import paper_1508_07953_amd as riann
    rf, rg = field, frames[W + K]
    out_r, err_r = idx.reconstruct(rf, H, Wd, gt=rg)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nrep = 20
    e0.record(stream)
    for _ in range(nrep):
        idx.reconstruct(rf, H, Wd, gt=rg, out=out_r)
    e1.record(stream)
    e1.synchronize()
    ms_r = e0.elapsed_time(e1) / nrep
    Cc = wl.channels
    rbytes = Q * 4 + H * Wd * Cc * (1 + 4) + int(idx.params.n_ref) * wl.D
    result["reconstruct"] = {"ms": ms_r, "E": float(err_r[0].item()),
                             "algorithmic_bytes": rbytes,
                             "GBps": rbytes / (ms_r * 1e-3) / 1e9,
                             "note": "field 4 B/query + frame 1 B and output 4 B per value + "
                                     "appearance set once; gathers served by L2"}
    # exact k-NN fields (k = 4) on the same frames, where the key range allows
    try:
        kk = 4
        kout = [torch.empty((hq, wq, kk), dtype=torch.int32, device=dev) for _ in range(2)]
        kss = torch.empty((hq, wq, kk), dtype=torch.int32, device=dev)
        idx.match_knn(frames[0], kk, full=True, out=kout[0], ssd=kss)
        torch.cuda.synchronize()
        e0.record(stream)
        idx.match_knn(frames[0], kk, full=True, out=kout[0], ssd=kss)
        e1.record(stream)
        e1.synchronize()
        full_ms = e0.elapsed_time(e1)
        nk = min(10, K)
        kc = 0
        e0.record(stream)
        for i in range(nk):
            idx.match_knn(frames[W + 1 + i], kk, prev=kout[kc], out=kout[1 - kc], ssd=kss)
            kc = 1 - kc
        e1.record(stream)
        e1.synchronize()
        result["knn"] = {"k": kk, "full_frame_ms": full_ms,
                         "ring_frame_ms": e0.elapsed_time(e1) / nk, "frames": nk}
    except riann.RiannError as ex:
        result["knn"] = {"k": 4, "unsupported": str(ex)}
    if not args.no_paper_mode:
        result["paper_mode"] = paper_mode(idx, frames, hq, wq, dev, log)


def ring_path_forced(idx, wl, frames, field, t0, nframes, hq, wq, log_fn):
    """The ring path carrying every query: routing threshold n, so each query
    with a prior goes through the smallest-ring search (k_ring), the ring
    scan and the survivor check (k_scan) -- nothing is routed to the dense
    search.  Every kernel is bracketed by HIP events on the launch stream;
    algorithmic bytes come from the device counters (sum of m*, sum of |S|)."""
    import torch
    n, D = int(idx.params.n_ref), wl.D
    Dp = (D + 31) // 32 * 32
    Kn = len(wl.keys)
    kr = 0 if Kn == 0 else (8 if Kn <= 8 else (Kn + 15) // 16 * 16)
    thr0 = int(idx.params.dense_threshold)
    idx.set_dense_threshold(n)
    outs = [torch.empty_like(field), torch.empty_like(field)]
    ssd = torch.empty_like(field)
    # frame t0's field by the full search; a warm-up ring frame; then the
    # timed frames, each with the field before it as prev
    idx.full_search(frames[t0], out=outs[0], ssd=ssd)
    idx.match_frame(frames[t0 + 1], prev=outs[0], out=outs[1], ssd=ssd)
    torch.cuda.synchronize()
    idx.reset_stats()
    idx.set_profiling(True)
    cur = 0
    w0 = time.perf_counter()
    for i in range(nframes):
        idx.match_frame(frames[t0 + 1 + i], prev=outs[cur], out=outs[1 - cur], ssd=ssd)
        cur = 1 - cur
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    prof = idx.profile()
    idx.set_profiling(False)
    st = idx.stats()
    idx.set_dense_threshold(thr0)
    Q = hq * wq
    rq = st["ring_queries"]
    per = {}
    # k_scan: per ring query its record, list entry, patch, Qc and the match
    # written; per candidate of the smallest ring its pivot row (contiguous in
    # the ring-ordered layout); per survivor its index and reference row
    sb = (rq * (16 + 4 + Dp + 4 + 8) + st["sum_mstar_ring"] * 4 * kr +
          st["sum_survivors"] * (4 + Dp)) / nframes
    for k in ("extract", "ring", "scan", "dense"):
        if prof[k]["launches"]:
            per[k] = prof[k]["ms"] / prof[k]["launches"]
    # the ring phase: patch + Qc + prev + the previous match's row + record
    # per query; the binary searches' line reads counted apart (probes)
    rb = Q * (Dp + 4 + 4 + Dp + 16)
    inline = "scan" not in per            # the ring kernel scanned its own ring queries
    scan_kernel = "k_ring (ring phase, then the ring scan of its own queries)" if inline \
        else "k_scan"
    scan_ms = per["ring"] if inline else per["scan"]
    scan_bytes = sb + (rb if inline else 0)
    res = {"threshold": n, "frames": nframes, "ms_per_frame": 1e3 * wall / nframes,
           "kernels_ms_per_frame": per,
           "ring_queries_per_frame": rq / nframes, "no_prior_per_frame": st["no_prior"] / nframes,
           "mean_mstar": st["sum_mstar_ring"] / max(1, rq),
           "mean_survivors": st["sum_survivors"] / max(1, rq),
           "probes_per_query": st["bsearch_probes"] / max(1, rq),
           "ring_scan": {"kernel": scan_kernel, "algorithmic_bytes": scan_bytes, "ms": scan_ms,
                         "GBps": scan_bytes / (scan_ms * 1e-3) / 1e9,
                         "algorithmic_frac_of_hbm_peak":
                             scan_bytes / (scan_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "layout": "ring-ordered pivot rows, %d words per entry" % kr,
                         "note": "per ring query 32 B + patch; per candidate of the smallest "
                                 "ring its pivot row; per survivor its index and row"
                                 + ("; plus the ring phase's bytes per query" if inline else "")
                                 + "; algorithmic bytes, much of them served by L2 and the "
                                   "Infinity Cache: the bytes fetched beyond L2 come from the "
                                   "FETCH_SIZE counter (profiles/hd720_hbm_traffic.txt)"}}
    log_fn(f"ring path forced: {res['ms_per_frame']:.2f} ms/frame, ring scan "
           f"{res['ring_scan']['GBps']:.0f} GB/s, mean m* {res['mean_mstar']:.0f}")
    return res


def uhd_batch_graph(dev, steps, log_fn):
    """The uneven batch: one 3840x2160 gray frame and four 640x360 gray
    frames per step (12x12 patches at stride 2, n = 262,144, K = 48), all
    five in one riann_match_batch, captured once as a HIP graph and replayed
    with each step's frames copied into the captured input buffers.  Beside
    it the same steps eagerly as one batch, and as five separate per-frame
    calls.  Frame 0 of every video is a full search; the 4K video's scene
    cuts (every 50 frames) fall outside the timed steps."""
    import torch
    import gen
    import paper_1508_07953_amd as riann
    t0 = time.time()
    nfr = steps + 2
    wl = gen.make_workload("uhd_mix", frames=nfr)
    vids = [wl.video] + [gen.make_video("uhd_mix", stream=1 + i, H=360, W=640, frames=nfr)
                         for i in range(4)]
    frames = [[torch.from_numpy(v.frame(t)).to(dev) for t in range(nfr)] for v in vids]
    idx = riann.Index.build(wl.ref, wl.keys, patch=12, channels=1, stride=2)
    log_fn(f"uhd batch: frames and index in {time.time() - t0:.1f}s")
    shapes = [idx.field_shape(int(f[0].shape[0]), int(f[0].shape[1])) for f in frames]
    Q = sum(h * w for h, w in shapes)
    outs = [[torch.empty(s, dtype=torch.int32, device=dev) for _ in range(2)] for s in shapes]
    ssds = [torch.empty(s, dtype=torch.int32, device=dev) for s in shapes]
    f_in = [torch.empty_like(frames[v][0]) for v in range(len(vids))]

    def items(src, par, mode=riann.MODE_RING):
        it = []
        for v in range(len(vids)):
            d = dict(frame=src[v], out=outs[v][1 - par], ssd=ssds[v], mode=mode)
            if mode == riann.MODE_RING:
                d["prev"] = outs[v][par]
            it.append(d)
        return it

    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for v in range(len(vids)):
            f_in[v].copy_(frames[v][0])
        idx.match_batch(items(f_in, 1, riann.MODE_FULL), stream=s)     # fields in outs[.][0]
        idx.match_batch(items(f_in, 0), stream=s)                      # warm-up, both parities
        idx.match_batch(items(f_in, 1), stream=s)
    s.synchronize()
    graphs = []
    for par in (0, 1):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            idx.match_batch(items(f_in, par), stream=s)
        graphs.append(g)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(run_step):
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            e0.record(s)
            for i in range(steps):
                run_step(1 + i, i % 2)
            e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1) / steps

    def graph_step(t, par):
        for v in range(len(vids)):
            f_in[v].copy_(frames[v][t])
        graphs[par].replay()

    def batch_step(t, par):
        idx.match_batch(items([frames[v][t] for v in range(len(vids))], par), stream=s)

    def single_step(t, par):
        for v in range(len(vids)):
            idx.match_frame(frames[v][t], prev=outs[v][par], out=outs[v][1 - par], ssd=ssds[v],
                            stream=s)

    res = {"workload": "one 3840x2160 + four 640x360 gray frames per step, 12x12 patches, "
                       "stride 2, n=262144, K=48, %d queries per step" % Q,
           "steps": steps}
    # two rounds in turn, the better of each kept (the first steps of a run
    # can meet lower clocks)
    for _ in range(2):
        for name, fn in (("separate_frames", single_step), ("batch_eager", batch_step),
                         ("graph", graph_step)):
            ms = timed(fn)
            if name not in res or ms < res[name]["ms_per_step"]:
                res[name] = {"ms_per_step": ms, "patches_per_s": Q / (ms * 1e-3)}
    # the graph's fields of the last step equal the eager per-frame search's
    last = steps % 2
    g_out = [outs[v][last].clone() for v in range(len(vids))]
    timed(single_step)
    res["graph_equals_eager"] = all(torch.equal(g_out[v], outs[v][last])
                                    for v in range(len(vids)))
    idx.close()
    log_fn(f"uhd batch: graph {res['graph']['ms_per_step']:.2f} ms/step, eager batch "
           f"{res['batch_eager']['ms_per_step']:.2f}, separate "
           f"{res['separate_frames']['ms_per_step']:.2f}")
    return res


def serving_compare(dev, streams, frames_per_stream, seconds, log_fn, shape_of=None,
                    label=None):
    """Serving (continuous batching) vs plain (one frame at a time) on a
    scaled serving workload: `streams` RGB streams, stream id mod 3 ->
    640x360 / 1280x720 / 1920x1080, 8x8x3 patches, one shared reference set
    of 65,536 patches with 32 key points, Poisson arrivals at 30 fps per
    stream.  As live streams deliver them, frames arrive in pinned host
    memory and every field and distance map goes back to pinned host memory
    (host_results): plain copies, searches and copies back one frame at a
    time; serving overlaps each batch's copies with the search of another.
    Frames are pre-generated (each stream cycles through `frames_per_stream`
    distinct frames; every result is exact, so the cycle only changes ring
    sizes, not correctness)."""
    import torch
    import gen
    import paper_1508_07953_amd as riann
    from paper_1508_07953_amd import serve

    shape_of = shape_of or gen.serving_stream_shape
    wl = gen.make_workload("serving")
    idx = riann.Index.build(wl.ref, wl.keys, patch=8, channels=3, stride=1)
    t0 = time.time()
    frames = []
    for s in range(streams):
        H, W = shape_of(s)
        v = gen.make_video("serving", stream=s, H=H, W=W, frames=frames_per_stream)
        frames.append([torch.from_numpy(v.frame(k)).pin_memory()
                       for k in range(frames_per_stream)])
    log_fn(f"serving: generated {streams} x {frames_per_stream} frames in {time.time() - t0:.1f}s")

    def frame_of(s, k):
        return frames[s][k % frames_per_stream]

    def run(max_batch, inflight, trace, scale, concurrent="auto"):
        srv = serve.Server(idx, max_batch=max_batch, inflight=inflight, host_results=True,
                           concurrent=concurrent)
        sids = {s: srv.open_stream(*shape_of(s)) for s in range(streams)}
        # warm the per-stream scratch and kernels
        for s in range(streams):
            srv.submit(sids[s], frame_of(s, 0), full=True)
        srv.drain()
        srv.completed.clear()
        r = serve.replay(srv, trace, frame_of, sids, time_scale=scale)
        per_res = {}
        for c in srv.completed:
            H, W = shape_of(c.stream)
            per_res.setdefault(f"{W}x{H}", []).append(c.latency * 1e3)
        r["p99_ms_by_resolution"] = {k: float(np.percentile(v, 99)) for k, v in per_res.items()}
        q = sum(idx.field_shape(*shape_of(s))[0] *
                idx.field_shape(*shape_of(s))[1] for s in range(streams))
        r["patches_per_s"] = r["frames_per_s"] * q / streams
        return r

    # throughput at saturation: every frame of the trace is there from the
    # start, six per stream; plain and serving alternate twice and each
    # reports the mean of its two windows (the windows' own rates are kept)
    sat_trace = [(0.0, s, k) for k in range(1, 7) for s in range(streams)]

    def mean_of(a, b):
        r = dict(a)
        r["frames_per_s"] = 0.5 * (a["frames_per_s"] + b["frames_per_s"])
        r["patches_per_s"] = 0.5 * (a["patches_per_s"] + b["patches_per_s"])
        r["window_frames_per_s"] = [a["frames_per_s"], b["frames_per_s"]]
        return r

    # the server's default: two batches side by side on two HIP streams
    # while frames are left waiting (here always), back to back otherwise
    plain_a = run(1, 1, sat_trace, 1.0)
    serve_a = run(40, 2, sat_trace, 1.0)
    plain_b = run(1, 1, sat_trace, 1.0)
    serve_b = run(40, 2, sat_trace, 1.0)
    plain_sat, serve_sat = mean_of(plain_a, plain_b), mean_of(serve_a, serve_b)
    # batches always back to back on one HIP stream; always side by side
    serve_sat_seq = run(40, 2, sat_trace, 1.0, concurrent=False)
    serve_sat_cc = run(40, 2, sat_trace, 1.0, concurrent=True)
    # latency at a sustainable rate: lambda * 30 fps per stream with lambda
    # set to ~70% of the serving capacity measured above
    cap_fps = serve_sat["frames_per_s"]
    lam = min(1.0, 0.7 * cap_fps / (30.0 * streams))
    trace = gen.poisson_trace(streams, 30.0 * lam, seconds)
    trace = [(t, s, k + 1) for (t, s, k) in trace]
    plain_lat = run(1, 1, trace, 1.0)
    serve_lat = run(40, 2, trace, 1.0)
    serve_lat_seq = run(40, 2, trace, 1.0, concurrent=False)
    # latency-first setting: one batch in flight, each batch takes everything
    # ready when the previous one completes
    serve_lat1 = run(40, 1, trace, 1.0)
    serve_lat_cc = run(40, 2, trace, 1.0, concurrent=True)
    idx.close()
    return {"workload": label or (f"{streams} RGB streams (360p/720p/1080p by id mod 3), "
                                  "8x8x3 patches, n=65536, K=32, Poisson arrivals"),
            "io": "frames from pinned host memory, fields and SSD maps back to pinned host memory",
            "serving_mode": "two batches in flight, side by side on two HIP streams while "
                            "frames wait beyond the batch, else back to back (concurrent='auto')",
            "saturation": {"plain": plain_sat, "serving": serve_sat,
                           "serving_back_to_back": serve_sat_seq,
                           "serving_side_by_side": serve_sat_cc},
            "lambda": lam, "offered_fps": 30.0 * lam * streams, "trace_seconds": seconds,
            "at_lambda": {"plain": plain_lat, "serving": serve_lat,
                          "serving_back_to_back": serve_lat_seq,
                          "serving_one_in_flight": serve_lat1,
                          "serving_side_by_side": serve_lat_cc}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-profile", action="store_true",
                    help="do not record per-kernel HIP events in the timed region")
    ap.add_argument("--workload", default="hd720", choices=["hd720", "fhd_rgb", "uhd_mix"],
                    help="per-frame workload of the timed loop (hd720 is the headline)")
    ap.add_argument("--dense-layout", default="auto", choices=["auto", "column"],
                    help="auto: references as MFMA rows (the library default); column: "
                         "queries as MFMA rows (RIANN_FLAG_COLUMN_DENSE)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the library's default routing threshold and block shape")
    ap.add_argument("--dense-shape", default="", metavar="WAVES,COLS",
                    help="use this dense block shape instead of autotuning it (e.g. 4,4)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed per-frame path: no reconstruction, k-NN or paper-mode "
                         "figures (used for kernel traces and counters)")
    ap.add_argument("--no-paper-mode", action="store_true",
                    help="skip the paper's approximate search (needs n x n tables)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving-vs-plain comparison")
    ap.add_argument("--serving-streams", type=int, default=64)
    ap.add_argument("--serving-seconds", type=float, default=8.0)
    ap.add_argument("--ring-forced-frames", type=int, default=3,
                    help="frames matched with every query on the ring path (threshold n) "
                         "after the timed region; 0 skips")
    ap.add_argument("--uhd-batch-steps", type=int, default=6,
                    help="steps of the 4K + 4 x 640x360 batch as one captured HIP graph; "
                         "0 skips")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="after the timed region, run one plain device copy of this many "
                         "MiB (reference point for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the search shards by frames/streams "
              "with no exchange, and this build measures one GPU's share only "
              "(--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    import gen
    import paper_1508_07953_amd as riann

    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    nframes = W + K + 1
    t0 = time.time()
    wl = gen.make_workload(args.workload, frames=max(nframes, 60))
    frames_h = [wl.frame(t) for t in range(nframes)]
    log(f"generated {nframes} frames in {time.time() - t0:.1f}s")
    frames = [torch.from_numpy(f).to(dev) for f in frames_h]
    H, Wd = frames_h[0].shape[:2]
    idx = riann.Index.build(wl.ref, wl.keys, patch=wl.patch, channels=wl.channels,
                            stride=wl.stride,
                            flags=riann.FLAG_COLUMN_DENSE if args.dense_layout == "column" else 0)
    hq, wq = idx.field_shape(H, Wd)
    Q = hq * wq
    bufs = [torch.empty((hq, wq), dtype=torch.int32, device=dev) for _ in range(2)]
    ssd = torch.empty((hq, wq), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    idx.full_search(frames[0], out=bufs[0], ssd=ssd)
    cur = 0
    def step(t):
        if wl.is_cut(t):
            idx.full_search(frames[t], out=bufs[1 - cur], ssd=ssd)
        else:
            idx.match_frame(frames[t], prev=bufs[cur], out=bufs[1 - cur], ssd=ssd)

    for t in range(1, W + 1):
        step(t)
        cur = 1 - cur
    torch.cuda.synchronize()
    tuned = None
    if not args.no_tune:
        # routing threshold picked by measurement on the warm-up frames (set-up,
        # outside the timed region); frames 1.. with the fields before them
        from paper_1508_07953_amd import tune
        fr, pv = [], []
        f_prev = torch.empty((hq, wq), dtype=torch.int32, device=dev)
        idx.full_search(frames[0], out=f_prev)
        for t in range(1, min(W, 3) + 1):
            o = torch.empty_like(f_prev)
            idx.match_frame(frames[t], prev=f_prev, out=o)
            fr.append(frames[t])
            pv.append(f_prev)
            f_prev = o
        if args.dense_shape:
            wv, cl = (int(x) for x in args.dense_shape.split(","))
            idx.set_dense_shape(wv, cl)
            shape = {"shape": [wv, cl], "ms": None}
        else:
            shape = tune.tune_shape(idx, fr, use_cache=False, write_cache=False)
        log(f"dense block shape {shape['shape']}: {shape['ms']}")
        tuned = tune.tune_threshold(idx, fr, pv, use_cache=False, write_cache=False)
        tuned["shape"] = shape
        log(f"tuned dense threshold {tuned['threshold']}: {tuned['ms']}")
        torch.cuda.synchronize()
    idx.reset_stats()
    if not args.no_profile:
        # inside the timed region only the dense step carries event markers
        # (the roofline figure); the other kernels are timed afterwards
        idx.set_profiling("dense")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(K)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(K):
        t = W + 1 + i
        evs[i][0].record(stream)
        step(t)
        evs[i][1].record(stream)
        cur = 1 - cur
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    wall = t_end - t_start
    prof = idx.profile() if not args.no_profile else None
    idx.set_profiling(False)
    st = idx.stats()
    # the same frames by the exhaustive search alone (no ring phase), right
    # after the timed region and timed the same way (a step's events, the
    # dense step's events): the same exact field, so this is what the ring
    # phase costs or buys on this workload
    fo = torch.empty((hq, wq), dtype=torch.int32, device=dev)
    fs = torch.empty((hq, wq), dtype=torch.int32, device=dev)
    if not args.no_profile:
        idx.set_profiling("dense")
    fevs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(K)]
    torch.cuda.synchronize()
    f_start = time.perf_counter()
    for i in range(K):
        fevs[i][0].record(stream)
        idx.full_search(frames[W + 1 + i], out=fo, ssd=fs)
        fevs[i][1].record(stream)
    torch.cuda.synchronize()
    f_wall = time.perf_counter() - f_start
    idx.set_profiling(False)
    flat = np.array([a.elapsed_time(b) for a, b in fevs])
    full_every = {"ms_per_frame": 1000.0 * f_wall / K, "frames": K,
                  "p50_frame_ms": float(np.percentile(flat, 50)),
                  "note": "riann_full_search on the timed frames right after the timed region, "
                          "timed the same way: the same exact field without the ring phase"}
    prof_all = None
    if not args.no_profile:
        # per-kernel breakdown: an untimed pass over the first timed frames
        # again, every kernel bracketed by events
        idx.set_profiling(True)
        for i in range(min(K, 10)):
            step(W + 1 + i)
            cur = 1 - cur
        prof_all = idx.profile()
        idx.set_profiling(False)
        torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in evs])

    result = {
        "metric": METRIC,
        "value": K * Q / wall,
        "unit": "patches/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1000.0 * wall / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_DESC[args.workload] % Q,
                   "frames_timed": K, "mode": "plain (one frame at a time)",
                   "dense_layout": args.dense_layout},
        "frames_per_s": K / wall,
        "full_search_every_frame": full_every,
        "p50_frame_ms": float(np.percentile(lat, 50)),
        "p99_frame_ms": float(np.percentile(lat, 99)),
        "routing": {"ring_queries": st["ring_queries"], "dense_queries": st["dense_queries"],
                    "bound_routed": st["bound_routed"],
                    "mean_mstar_evaluated": st["sum_mstar"] / max(1, st["queries"] - st["bound_routed"]),
                    "dense_threshold": int(idx.params.dense_threshold),
                    "autotune_ms_per_frame": tuned["ms"] if tuned else None,
                    "dense_shape": (tuned["shape"]["shape"] if tuned else
                                    list(idx.dense_shapes()[0][idx.dense_shapes()[1]])),
                    "dense_shape_ms_per_full_frame": tuned["shape"]["ms"] if tuned else None},
    }
    if prof is not None:
        n, D = int(idx.params.n_ref), wl.D
        # the dense search runs on routed queries and on whole cut frames
        launches = prof["dense"]["launches"] + prof["full"]["launches"]
        dense_q_per_launch = st["dense_queries"] / max(1, launches)
        ms_per_launch = (prof["dense"]["ms"] + prof["full"]["ms"]) / max(1, launches)
        ops = 2.0 * dense_q_per_launch * n * D
        achieved = ops / (ms_per_launch * 1e-3) / 1e12
        rows = args.dense_layout == "auto"
        kname = ("k_dense_rows (int8 MFMA, references as rows, own candidate check)" if rows else
                 "k_dense (int8 MFMA, queries as rows)")
        result["roofline"] = {"bound": "mfma", "kernel": kname,
                              "achieved": achieved, "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                              "frac": achieved / INT8_PEAK_TOPS,
                              "traffic": dense_traffic_bytes(
                                  args.workload, args.dense_layout,
                                  idx.dense_shapes()[0][idx.dense_shapes()[1]]),
                              "ms_per_launch": ms_per_launch,
                              "ops_per_launch": ops}
        result["kernels_ms_per_frame"] = {k: v["ms"] / max(1, v["launches"])
                                          for k, v in prof_all.items() if v["launches"]}
        result["kernels_note"] = ("dense: HIP events in the timed region; every kernel: an "
                                  "untimed pass over 10 of the frames after it")
        # the other per-frame kernels against the HBM roofline (algorithmic
        # bytes per frame; both are bound elsewhere, see the notes)
        Dp = (wl.D + 31) // 32 * 32
        sec = {}
        thr = int(idx.params.dense_threshold)
        if not prof_all["ring"]["launches"] and thr == 0:
            sec["k_ring"] = {"launched": False,
                             "note": "threshold 0: a query with a previous match has m* >= 1 "
                                     "(its nearest neighbour lies in every ring), so the "
                                     "extraction kernel routes it to the dense search on that "
                                     "bound alone and no ring kernel is launched"}
        if prof_all["ring"]["launches"]:
            # the ring kernel reads every route code; the queries the
            # extraction kernel left to it also their patch, Qc, prev, the
            # previous match's row and Rc, and write a record
            left = max(0, st["queries"] - st["bound_routed"] - st["no_prior"]) / K
            rb = Q + left * (Dp + 4 + 4 + Dp + 4 + 16)
            rms = prof_all["ring"]["ms"] / prof_all["ring"]["launches"]
            sec["k_ring"] = {"bound": "latency", "algorithmic_bytes": rb, "ms": rms,
                             "queries_left_per_frame": left,
                             "GBps": rb / (rms * 1e-3) / 1e9,
                             "note": "route codes of every query, then the exact smallest-ring "
                                     "search of the queries the extraction kernel left (binary "
                                     "searches: latency), and their ring scan"}
        if not prof_all["extract"]["launches"]:
            sec["k_extract"] = {"launched": False,
                                "note": "every query goes dense and the patch is 8x8 gray: the "
                                        "dense kernel cuts each query patch from the frame "
                                        "itself (and counts the routing), no extraction launch"}
        if prof_all["extract"]["launches"]:
            # extraction (frame once; patch, Qc, frame id, route code written)
            # and routing (prev entry, the previous match's row and Rc read)
            # (at threshold 0 only the previous match's index: every query
            # with one is routed dense on m* >= 1)
            eb = H * Wd * wl.channels + Q * (Dp + 4 + 1 + 1) + Q * (4 + (Dp + 4 if thr else 0))
            ems = prof_all["extract"]["ms"] / prof_all["extract"]["launches"]
            sec["k_extract"] = {"bound": "hbm" if thr == 0 else "hbm+valu",
                                "algorithmic_bytes": eb, "ms": ems,
                                "GBps": eb / (ems * 1e-3) / 1e9,
                                "hbm_frac": eb / (ems * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                "note": "frame read once, encoded patch + Qc + frame id + route "
                                        "code written, the previous match's index read"
                                        + ("" if thr == 0 else
                                           "; per query the previous match's row and Rc read, "
                                           "K key distances and ring bounds computed (VALU)")}
        if prof_all["scan"]["launches"] and st["ring_queries"]:
            # ring-routed queries: record, list entry, patch, Qc read and the
            # match written; the smallest ring's P entries and pivot rows; the
            # survivors' rows (device counters, summed over the timed frames)
            Kp = (len(wl.keys) + 3) // 4 * 4
            sb = (st["ring_queries"] * (16 + 4 + Dp + 4 + 8) +
                  st["sum_mstar_ring"] * (4 + 4 * Kp) + st["sum_survivors"] * Dp) / K
            sms = prof_all["scan"]["ms"] / prof_all["scan"]["launches"]
            sec["k_scan"] = {"bound": "hbm", "algorithmic_bytes": sb, "ms": sms,
                             "GBps": sb / (sms * 1e-3) / 1e9,
                             "hbm_frac": sb / (sms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "ring_queries_per_frame": st["ring_queries"] / K,
                             "note": "per ring query 32 B + patch; per candidate of the "
                                     "smallest ring 4 B index + the Kp-word pivot row; per "
                                     "survivor its row"}
        result["secondary_kernels"] = sec
    if args.ring_forced_frames > 0 and W + 1 + args.ring_forced_frames < nframes + 1:
        result["ring_path_forced"] = ring_path_forced(
            idx, wl, frames, bufs[cur], W, min(args.ring_forced_frames, nframes - W - 1),
            hq, wq, log)
    if not args.no_extras:
        extras(args, result, idx, wl, frames, bufs[cur], H, Wd, hq, wq, Q, K, W, dev, stream, log)
    if args.uhd_batch_steps > 0:
        result["uhd_batch_graph"] = uhd_batch_graph(dev, args.uhd_batch_steps, log)
    if not args.no_serving:
        result["serving_vs_plain"] = serving_compare(dev, args.serving_streams, 3,
                                                     args.serving_seconds, log)
        # small frames only: one frame no longer fills the GPU, batching does
        result["serving_vs_plain_360p"] = serving_compare(
            dev, 24, 3, args.serving_seconds, log, shape_of=lambda s: (360, 640),
            label="24 RGB 640x360 streams, 8x8x3 patches, n=65536, K=32, Poisson arrivals")
    if args.copy_calibration > 0:
        nb = args.copy_calibration << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = nb
        del src, dst
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(wl, frames_h[0], frames_h[1], args.cpu_seconds)
    idx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
