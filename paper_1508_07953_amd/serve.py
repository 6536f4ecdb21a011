"""Continuous batching of many live video streams over one index.

The paper's setting is a live stream of frames matched in real time against a
fixed reference set (Sec. 1, Fig. 1); frame t of a stream needs frame t-1's
field as its previous match (Algorithm 1).  A `Server` keeps every stream's
previous field resident on the device, admits streams while their device
memory fits a budget, and forms batches from whatever frames are ready --
at most one frame per stream in flight, since frame t+1 depends on frame t's
field.  Each batch is one `riann_match_batch` submission; batches formed while
others run are queued behind them on the device (concurrent=False), run side
by side on separate HIP streams (True), or (the default, "auto") run side by
side only while frames are left waiting after the batch is formed, so a
backlog fills the GPU through the tail of each launch while a short queue
keeps each batch's latency that of running alone.  A batch holds at most
max_batch_queries queries, a cap that grows with a backlog (up to
backlog_batch_queries): larger launches amortise the ragged last round of
their query chunks.  Every result is exact, so a stream's fields are the same
alone and in any mix.

`Server(..., max_batch=1, inflight=1)` is the plain mode: one frame at a time,
each finished before the next starts.

Frames may be device tensors or host tensors (pinned host memory for
asynchronous copies).  Host frames are copied into the stream's device frame
buffer on a copy stream of the server's own, so the copies of one batch
overlap the search of the batch before it.  With host_results=True every
field and distance map is also delivered to pinned host memory, copied on a
second copy stream of the server's own once its batch has run, so those
copies overlap the next batch's search too; a frame completes when its
field is on the host.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Deque, Dict, List, Optional, Tuple

import numpy as np

from . import MODE_FULL, MODE_RING, Index, RiannError, footprint


@dataclasses.dataclass
class Completion:
    stream: int
    seq: int            # frame number within the stream
    arrival: float      # host time the frame was submitted (s)
    done: float         # host time its completion was observed (s)
    field: object       # (Hq, Wq) int32 tensor holding the field, on the device
                        # or with host_results in pinned host memory (valid
                        # until the stream's frame after next is launched)
    ssd: object

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Stream:
    def __init__(self, sid, H, W, hq, wq, device, torch, channels, host_results=False):
        self.sid, self.H, self.W = sid, H, W
        self.fields = [torch.full((hq, wq), -1, dtype=torch.int32, device=device)
                       for _ in range(2)]
        self.ssd = [torch.empty((hq, wq), dtype=torch.int32, device=device) for _ in range(2)]
        # pinned host copies of the results (host_results), one per device slot
        self.fields_h = [torch.empty((hq, wq), dtype=torch.int32, pin_memory=True)
                         for _ in range(2)] if host_results else None
        self.ssd_h = [torch.empty((hq, wq), dtype=torch.int32, pin_memory=True)
                      for _ in range(2)] if host_results else None
        # device copy of the frame in flight when frames arrive in host memory
        # (one buffer: a stream has at most one frame in flight)
        self.dframe = torch.empty((H, W, channels), dtype=torch.uint8, device=device)
        self.cur = 0            # fields[cur] holds the latest finished field
        self.has_field = False
        self.seq = 0
        self.queue: Deque[Tuple[object, float, bool]] = collections.deque()
        self.busy = False
        self.closing = False


class Server:
    """Continuous-batching front end of an `Index` (see the module doc)."""

    def __init__(self, index: Index, max_batch: int = 40, inflight: int = 2,
                 memory_budget: Optional[int] = None, device=None,
                 max_batch_queries: Optional[int] = 1_000_000, concurrent="auto",
                 host_results: bool = False,
                 backlog_batch_queries: Optional[int] = 8_400_000):
        import torch
        self.torch = torch
        self.index = index
        self.max_batch = max(1, int(max_batch))
        self.inflight = max(1, int(inflight))
        # concurrent=False: batches queue back to back on one HIP stream (no
        # idle gap between them, no sharing slowdown); True: each in-flight
        # batch gets its own HIP stream and they run side by side; "auto":
        # side by side while a backlog is left after forming the batch (the
        # next batch's blocks fill the CUs the last round of a launch leaves
        # idle), back to back otherwise
        if concurrent != "auto":
            if concurrent not in (False, True):
                raise ValueError("concurrent must be False, True or 'auto'")
            concurrent = bool(concurrent)
        self.concurrent = concurrent
        # a batch completes as a whole, so its size bounds the latency of the
        # small frames in it: stop adding frames once it holds this many
        # queries (a lone larger frame still goes alone)
        self.max_batch_queries = max_batch_queries
        # with a backlog the cap grows to the ready queries' share per batch
        # in flight, up to this many: each dense launch then covers more
        # frames and the ragged last round of its query chunks weighs less
        # (saturation throughput +4 % at 2 M queries, +8 % at 8 M on the
        # 360p/720p/1080p mix), while a short queue keeps the small cap
        self.backlog_batch_queries = backlog_batch_queries
        self.device = device if device is not None else torch.device("cuda")
        self.hip_streams = [torch.cuda.Stream(device=self.device)
                            for _ in range(self.inflight if concurrent else 1)]
        self._last_hs = self.hip_streams[0]    # stream of the newest batch
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.host_results = host_results
        self.result_stream = torch.cuda.Stream(device=self.device) if host_results else None
        self.budget = memory_budget
        p = index.params
        self._fp = (p.n_ref, p.n_keys, p.patch, p.channels, p.stride)
        self.index_bytes = footprint(*self._fp)
        self.used = self.index_bytes          # index + every active stream's buffers
        self.streams: Dict[int, _Stream] = {}
        self.waiting: Deque[Tuple[int, int, int]] = collections.deque()  # (sid, H, W)
        self._pending_queues: Dict[int, Deque] = {}   # frames of waiting streams
        self._next_sid = 0
        # in flight: (completion event, HIP stream, [(sid, seq, arrival, slot)],
        # frames referenced until completion)
        self._batches: List[Tuple[object, object, List[Tuple[int, int, float, int]], list]] = []
        self.completed: List[Completion] = []

    # ------------------------------------------------------------ admission
    def stream_bytes(self, H: int, W: int) -> int:
        """Device bytes a stream holds: two fields, two distance maps and
        its device frame buffer."""
        hq, wq = self.index.field_shape(H, W)
        return 4 * 4 * hq * wq + H * W * int(self.index.params.channels)

    def _scratch_bytes(self, frame_queries: List[int]) -> int:
        """Search scratch of the server: each HIP stream the server launches
        on keeps scratch for the largest batch it can form from streams with
        these per-frame query counts -- one frame per stream, at most
        max_batch frames, and at most max_batch_queries unless one frame is
        larger (it goes alone)."""
        if not frame_queries:
            return 0
        qs = sorted(frame_queries, reverse=True)
        q = sum(qs[:self.max_batch])
        cap = self._largest_cap()
        if cap is not None:
            q = min(q, max(cap, qs[0]))
        p = self.index.params
        # the scratch of q queries: a 1 x q field (one patch row of width
        # patch + (q - 1) * stride)
        per = footprint(*self._fp, p.patch, p.patch + (q - 1) * p.stride) - self.index_bytes
        return len(self.hip_streams) * per

    def _queries(self, H, W) -> int:
        hq, wq = self.index.field_shape(H, W)
        return hq * wq

    def device_bytes(self, extra: Optional[Tuple[int, int]] = None) -> int:
        """Device bytes the server needs with its active streams (and one
        more stream of size `extra`): the index once, every stream's
        buffers, and the scratch of the largest batch per HIP stream."""
        shapes = [(s.H, s.W) for s in self.streams.values()]
        if extra is not None:
            shapes.append(extra)
        total = self.index_bytes + sum(self.stream_bytes(H, W) for H, W in shapes)
        return total + self._scratch_bytes([self._queries(H, W) for H, W in shapes])

    def open_stream(self, H: int, W: int) -> int:
        """Returns a stream id.  The stream is active at once if its memory
        fits the budget, otherwise it waits for memory (frames can be
        submitted meanwhile; they queue).  A stream that could not fit even
        with no other stream active is rejected (RiannError)."""
        if self.budget is not None:
            alone = (self.index_bytes + self.stream_bytes(H, W) +
                     self._scratch_bytes([self._queries(H, W)]))
            if alone > self.budget:
                raise RiannError(-2, f"a {H}x{W} stream needs {alone} device bytes alone, "
                                     f"above the budget of {self.budget}")
        sid = self._next_sid
        self._next_sid += 1
        if self._fits(H, W):
            self._activate(sid, H, W)
        else:
            self.waiting.append((sid, H, W))
            self._pending_queues[sid] = collections.deque()
        return sid

    def _fits(self, H, W) -> bool:
        if self.budget is None:
            return True
        return self.device_bytes(extra=(H, W)) <= self.budget

    def _activate(self, sid, H, W):
        hq, wq = self.index.field_shape(H, W)
        st = _Stream(sid, H, W, hq, wq, self.device, self.torch, int(self.index.params.channels),
                     self.host_results)
        pq = self._pending_queues.pop(sid, None)
        if pq:
            st.queue.extend(pq)
        self.streams[sid] = st
        self.used += self.stream_bytes(H, W)

    def close_stream(self, sid: int) -> None:
        """Frees the stream once its in-flight frame (if any) has finished."""
        st = self.streams.get(sid)
        if st is None:
            self.waiting = collections.deque(w for w in self.waiting if w[0] != sid)
            self._pending_queues.pop(sid, None)
            return
        st.closing = True
        st.queue.clear()
        if not st.busy:
            self._free(sid)

    def _free(self, sid):
        st = self.streams.pop(sid)
        self.used -= self.stream_bytes(st.H, st.W)
        while self.waiting and self._fits(self.waiting[0][1], self.waiting[0][2]):
            w = self.waiting.popleft()
            self._activate(*w)

    @property
    def active_streams(self) -> int:
        return len(self.streams)

    # ------------------------------------------------------------ frames
    def submit(self, sid: int, frame, arrival: Optional[float] = None,
               full: bool = False) -> None:
        """Queue one frame (H, W, C) uint8 of stream `sid`, in device memory
        or in host memory (pinned for an asynchronous copy).  The server
        keeps a reference until the frame's batch has completed.  `full`
        asks for the exhaustive search (first frame, scene cut)."""
        t = time.perf_counter() if arrival is None else arrival
        st = self.streams.get(sid)
        if st is None:
            pq = self._pending_queues
            if sid not in pq:
                raise KeyError(f"unknown stream {sid}")
            pq[sid].append((frame, t, full))
            return
        if st.closing:
            raise RiannError(-1, f"stream {sid} is closing")
        st.queue.append((frame, t, full))

    def pending(self) -> int:
        n = sum(len(s.queue) for s in self.streams.values())
        n += sum(len(q) for q in self._pending_queues.values())
        return n + sum(len(b[2]) for b in self._batches)

    def _largest_cap(self) -> Optional[int]:
        """The largest query cap a batch can get (None: no cap)."""
        if self.max_batch_queries is None:
            return None
        return max(self.max_batch_queries, self.backlog_batch_queries or 0)

    def _batch_cap(self, ready) -> Optional[int]:
        """The query cap of the next batch: the base cap, raised with a
        backlog to the ready queries' share per batch in flight."""
        if self.max_batch_queries is None:
            return None
        cap = self.max_batch_queries
        if self.backlog_batch_queries:
            rq = sum(self._queries(s.H, s.W) for s in ready)
            cap = max(cap, min(self.backlog_batch_queries, rq // self.inflight))
        return cap

    def _launch(self) -> bool:
        if len(self._batches) >= self.inflight:
            return False
        ready = [s for s in self.streams.values() if not s.busy and s.queue]
        if not ready:
            return False
        ready.sort(key=lambda s: s.queue[0][1])          # oldest arrival first
        cap = self._batch_cap(ready)
        picked, q = [], 0
        for s in ready:
            hq, wq = self.index.field_shape(s.H, s.W)
            if picked and (len(picked) >= self.max_batch or
                           (cap is not None and q + hq * wq > cap)):
                break
            picked.append(s)
            q += hq * wq
        backlog = len(ready) > len(picked)
        ready = picked
        side_by_side = self.concurrent is True or (self.concurrent == "auto" and backlog)
        if side_by_side:
            in_use = {id(b[1]) for b in self._batches}
            hs = next(x for x in self.hip_streams if id(x) not in in_use)
        elif self._batches:
            hs = self._last_hs                    # queue behind the newest batch
        else:
            hs = self.hip_streams[0]
        self._last_hs = hs
        torch = self.torch
        items, meta, keep = [], [], []
        copies = False
        for s in ready:
            frame, t_arr, full = s.queue.popleft()
            if not frame.is_cuda:
                # host frame: into the stream's device buffer on the copy
                # stream (the stream has no frame in flight, so the buffer is free)
                with torch.cuda.stream(self.copy_stream):
                    s.dframe.copy_(frame.reshape(s.dframe.shape), non_blocking=True)
                copies = True
                keep.append(frame)                    # until the copy has run
                dframe = s.dframe
            else:
                dframe = frame
                keep.append(frame)                    # until the batch has run
            nxt = 1 - s.cur
            mode = MODE_FULL if (full or not s.has_field) else MODE_RING
            it = dict(frame=dframe, out=s.fields[nxt], ssd=s.ssd[nxt], mode=mode)
            if mode == MODE_RING:
                it["prev"] = s.fields[s.cur]
            items.append(it)
            meta.append((s.sid, s.seq, t_arr, nxt))
            s.seq += 1
            s.busy = True
        # device frames were produced on the current stream, host frames were
        # copied on the copy stream: order the batch after both
        hs.wait_stream(torch.cuda.current_stream(self.device))
        if copies:
            hs.wait_stream(self.copy_stream)
        self.index.match_batch(items, stream=hs)
        ev = torch.cuda.Event()
        if self.host_results:
            # the results to pinned host memory on the result stream, after
            # the batch, while the next batch's search runs on hs
            rs = self.result_stream
            rs.wait_stream(hs)
            with torch.cuda.stream(rs):
                for (sid, _, _, nxt), s in zip(meta, ready):
                    s.fields_h[nxt].copy_(s.fields[nxt], non_blocking=True)
                    s.ssd_h[nxt].copy_(s.ssd[nxt], non_blocking=True)
            ev.record(rs)
        else:
            ev.record(hs)
        self._batches.append((ev, hs, meta, keep))
        return True

    def _collect(self, block: bool = False) -> int:
        done = 0
        keep = []
        for ev, hs, meta, frames in self._batches:
            if block and not keep:
                ev.synchronize()
            if ev.query():
                t = time.perf_counter()
                for sid, seq, t_arr, nxt in meta:
                    st = self.streams[sid]
                    st.cur = nxt
                    st.has_field = True
                    st.busy = False
                    if self.host_results:
                        self.completed.append(Completion(sid, seq, t_arr, t, st.fields_h[nxt],
                                                         st.ssd_h[nxt]))
                    else:
                        self.completed.append(Completion(sid, seq, t_arr, t, st.fields[nxt],
                                                         st.ssd[nxt]))
                    if st.closing:
                        self._free(sid)
                done += 1
            else:
                keep.append((ev, hs, meta, frames))
        self._batches = keep
        return done

    def step(self, block: bool = False) -> int:
        """Collect finished batches, then launch as many batches as there are
        free HIP streams.  Returns the number of batches launched."""
        self._collect(block=block and len(self._batches) >= self.inflight)
        n = 0
        while self._launch():
            n += 1
        return n

    def _stuck(self) -> bool:
        """Frames wait, nothing runs and nothing can be launched: only
        streams waiting for memory hold frames, and no active stream will
        free any unless the caller closes one."""
        return (not self._batches and self.pending() > 0 and
                not any(s.queue for s in self.streams.values()))

    def drain(self) -> None:
        while self.pending():
            if not self.step():
                if self._stuck():
                    raise RiannError(-2, "frames of streams waiting for memory remain; close "
                                         "active streams to admit them")
                self._collect(block=True)


def replay(server: Server, trace: List[Tuple[float, int, int]], frame_of: Callable,
           stream_ids: Dict[int, int], time_scale: float = 1.0,
           on_done: Optional[Callable[[Completion], None]] = None,
           full_of: Optional[Callable[[int, int], bool]] = None) -> Dict[str, float]:
    """Replays an arrival trace [(t, stream, frame_index)] in real time
    (t / time_scale seconds after start), submitting frame_of(stream, k) to
    `server` as it arrives.  Returns throughput and latency figures."""
    torch = server.torch
    trace = sorted(trace)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i = 0
    n_done0 = len(server.completed)
    while i < len(trace) or server.pending():
        now = time.perf_counter() - t0
        while i < len(trace) and trace[i][0] / time_scale <= now:
            t_arr, s, k = trace[i]
            full = full_of(s, k) if full_of else False
            server.submit(stream_ids[s], frame_of(s, k), arrival=t0 + t_arr / time_scale,
                          full=full)
            i += 1
        launched = server.step()
        if i >= len(trace) and server._stuck():
            raise RiannError(-2, "frames of streams waiting for memory remain; close "
                                 "active streams to admit them")
        if on_done is not None:
            for c in server.completed[n_done0:]:
                on_done(c)
            n_done0 = len(server.completed)
        if not launched and i < len(trace):
            nxt = trace[i][0] / time_scale - (time.perf_counter() - t0)
            if nxt > 0 and not server._batches:
                time.sleep(min(nxt, 0.002))
        elif not launched and server._batches:
            server._collect(block=False)
    torch.cuda.synchronize()
    server._collect(block=False)
    if on_done is not None:
        for c in server.completed[n_done0:]:
            on_done(c)
    t1 = time.perf_counter()
    lat = np.array([c.latency for c in server.completed]) * 1e3
    return {"frames": len(server.completed), "wall_s": t1 - t0,
            "frames_per_s": len(server.completed) / (t1 - t0),
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else 0.0,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else 0.0}
