"""Autotuner for the dense search's block shape and the ring/dense routing
threshold.

Which path answers a query never changes its result (both are exact); it
only changes the time.  The break-even ring size depends on the reference-set
size, the patch dimension, the number of key points and how wide the rings of
the actual video are (Sec. 3.3: more temporal change, more candidates), so it
is measured rather than modelled: each candidate threshold is timed on real
frames with HIP events and the fastest is kept.  The same holds for the
dense search's block shape (wavefronts per block, 32-query column blocks per
wavefront, i.e. queries per wavefront): the shapes built for the patch width
are timed on the exhaustive search of real frames.  Results are cached in a
JSON file keyed by (device architecture, patch, channels, stride, n, K).
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Sequence

DEFAULT_CANDIDATES = (0, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096)


def cache_path() -> str:
    return os.environ.get("RIANN_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "riann", "tune.json"))


def cache_key(index, arch: str) -> str:
    p = index.params
    return f"{arch}:p{p.patch}c{p.channels}s{p.stride}:n{p.n_ref}:K{p.n_keys}"


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, rec: dict) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        data = _load_cache()
        data[key] = rec
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune_threshold(index, frames: Sequence, prevs: Sequence,
                   candidates: Optional[Sequence[int]] = None, repeats: int = 2,
                   use_cache: bool = True, write_cache: bool = True,
                   arch: Optional[str] = None) -> Dict:
    """Times `index.match_frame(frames[i], prev=prevs[i])` for each candidate
    threshold and sets the fastest on the index.  Returns
    {"threshold": best, "ms": {threshold: mean ms per frame}, "cached": bool}.
    `arch` (e.g. "gfx950") defaults to the frames' device."""
    import torch
    if arch is None:
        arch = torch.cuda.get_device_properties(frames[0].device).gcnArchName.split(":")[0]
    key = cache_key(index, arch)
    if use_cache:
        rec = _load_cache().get(key)
        if rec is not None:
            index.set_dense_threshold(int(rec["threshold"]))
            return dict(rec, cached=True)
    n = int(index.params.n_ref)
    cands: List[int] = sorted({int(c) for c in (candidates or DEFAULT_CANDIDATES) if c <= n})
    outs = [torch.empty_like(p) for p in prevs]
    ms: Dict[int, float] = {}
    stream = torch.cuda.current_stream()
    for thr in cands:
        index.set_dense_threshold(thr)
        for f, p, o in zip(frames, prevs, outs):          # warm-up
            index.match_frame(f, prev=p, out=o)
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(repeats):
            for f, p, o in zip(frames, prevs, outs):
                index.match_frame(f, prev=p, out=o)
        end.record(stream)
        end.synchronize()
        ms[thr] = start.elapsed_time(end) / (repeats * len(frames))
    best = min(ms, key=lambda t: (ms[t], t))
    index.set_dense_threshold(best)
    rec = {"threshold": best, "ms": {str(k): v for k, v in ms.items()}}
    if write_cache:
        _store(key, rec)
    return dict(rec, cached=False)


def tune_shape(index, frames: Sequence, repeats: int = 2, use_cache: bool = True,
               write_cache: bool = True, arch: Optional[str] = None) -> Dict:
    """Times `index.full_search(frames[i])` (every query through the dense
    search) at each block shape the library built for the index's patch
    width and sets the fastest.  Returns {"shape": (waves, cols), "ms":
    {"WxC": mean ms per frame}, "cached": bool}."""
    import torch
    if arch is None:
        arch = torch.cuda.get_device_properties(frames[0].device).gcnArchName.split(":")[0]
    key = cache_key(index, arch) + ":shape"
    if use_cache:
        rec = _load_cache().get(key)
        if rec is not None:
            index.set_dense_shape(*rec["shape"])
            return dict(rec, cached=True)
    shapes, _ = index.dense_shapes()
    outs = [index.full_search(f) for f in frames]
    ms: Dict[str, float] = {}
    stream = torch.cuda.current_stream()
    for wv, cl in shapes:
        index.set_dense_shape(wv, cl)
        for f, (o, d) in zip(frames, outs):               # warm-up
            index.full_search(f, out=o, ssd=d)
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(repeats):
            for f, (o, d) in zip(frames, outs):
                index.full_search(f, out=o, ssd=d)
        end.record(stream)
        end.synchronize()
        ms[f"{wv}x{cl}"] = start.elapsed_time(end) / (repeats * len(frames))
    best = min(shapes, key=lambda sh: (ms[f"{sh[0]}x{sh[1]}"], shapes.index(sh)))
    index.set_dense_shape(*best)
    rec = {"shape": list(best), "ms": ms}
    if write_cache:
        _store(key, rec)
    return dict(rec, cached=False)
