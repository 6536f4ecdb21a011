"""RIANN exact ANN fields on AMD Instinct MI355X -- Python binding.

Thin ctypes layer over libriann.so (C ABI in include/riann.h).  It only
marshals arguments: every step of the search runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and streams.

    idx = Index.build(ref, keys, patch=8, channels=1, stride=1)
    out, ssd = idx.full_search(frame0)                 # frame 0 / scene cut
    out, ssd = idx.match_frame(frame1, prev=out)       # ring-intersection search

Frames are CUDA (HIP) uint8 tensors of shape (H, W) or (H, W, C); fields are
int32 (Hq, Wq) with Hq = (H - p) // s + 1, Wq = (W - p) // s + 1.

The library must be built (``__graft_entry__.build()`` or
``python paper_1508_07953_amd/_build.py``); importing this package without it
raises ImportError -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libriann.so")

RIANN_OK, RIANN_E_INVALID, RIANN_E_NOMEM, RIANN_E_DEVICE, RIANN_E_UNSUPPORTED, RIANN_E_IO = (
    0, -1, -2, -3, -4, -5)
MODE_RING, MODE_FULL = 0, 1
FLAG_COLUMN_DENSE = 1
FLAG_EXACT_MSTAR = 2
FLAG_GATHER_SCAN = 4
PROFILE_ALL, PROFILE_DENSE = 1, 2

# every symbol include/riann.h declares
EXPORTS = ["riann_build", "riann_match_frame", "riann_full_search", "riann_match_batch",
           "riann_footprint", "riann_get_stats", "riann_reset_stats", "riann_get_params",
           "riann_save", "riann_load", "riann_destroy", "riann_last_error", "riann_version",
           "riann_set_profiling", "riann_get_profile", "riann_set_dense_threshold",
           "riann_reconstruct", "riann_stack_frames", "riann_match_knn",
           "riann_build_paper_tables", "riann_match_paper", "riann_match_frame_noalloc",
           "riann_set_dense_shape", "riann_get_dense_shapes"]
KERNELS = ["ring", "scan", "dense", "full", "extract"]


class RiannError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"riann status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("patch", C.c_int32), ("channels", C.c_int32), ("stride", C.c_int32),
                ("n_keys", C.c_int32), ("n_ref", C.c_int64), ("dense_threshold", C.c_int64),
                ("flags", C.c_uint32), ("reserved", C.c_uint32)]


class FrameDesc(C.Structure):
    _fields_ = [("frame", C.c_void_p), ("H", C.c_int32), ("W", C.c_int32),
                ("pitch", C.c_int64), ("prev", C.c_void_p), ("out", C.c_void_p),
                ("ssd", C.c_void_p), ("mode", C.c_int32), ("reserved", C.c_int32)]


class Profile(C.Structure):
    _fields_ = [("launches", C.c_uint64 * 5), ("ms", C.c_double * 5)]


class Stats(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in
                ("frames", "queries", "ring_queries", "dense_queries", "no_prior",
                 "sum_mstar", "sum_survivors", "sum_mstar_ring", "bound_routed",
                 "dense_routed", "bsearch_probes")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    # torch ships its own HIP runtime.  Loading torch first makes the library
    # bind to that same runtime; loaded the other way round, the process would
    # hold two HIP/HSA runtimes and the second to start finds no device.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.riann_build.argtypes = [vp, vp, C.POINTER(Params), vp, C.POINTER(vp)]
    L.riann_match_frame.argtypes = [vp, vp, i32, i32, i64, vp, vp, vp, vp]
    L.riann_match_frame_noalloc.argtypes = [vp, vp, i32, i32, i64, vp, vp, vp, vp]
    L.riann_full_search.argtypes = [vp, vp, i32, i32, i64, vp, vp, vp]
    L.riann_match_batch.argtypes = [vp, C.POINTER(FrameDesc), i32, vp]
    L.riann_footprint.argtypes = [C.POINTER(Params), i32, i32, C.POINTER(i64)]
    L.riann_get_stats.argtypes = [vp, C.POINTER(Stats)]
    L.riann_reset_stats.argtypes = [vp]
    L.riann_get_params.argtypes = [vp, C.POINTER(Params)]
    L.riann_save.argtypes = [vp, C.c_char_p]
    L.riann_load.argtypes = [C.c_char_p, vp, C.POINTER(vp)]
    L.riann_destroy.argtypes = [vp]
    L.riann_set_profiling.argtypes = [vp, C.c_int]
    L.riann_set_dense_threshold.argtypes = [vp, i64]
    L.riann_set_dense_shape.argtypes = [vp, i32, i32]
    L.riann_get_dense_shapes.argtypes = [vp, vp, vp, i32, vp, vp]
    L.riann_get_profile.argtypes = [vp, C.POINTER(Profile)]
    L.riann_reconstruct.argtypes = [vp, vp, i32, i32, vp, i32, vp, vp, i64, vp, vp]
    L.riann_match_knn.argtypes = [vp, vp, i32, i32, i64, i32, vp, vp, vp, i32, vp]
    L.riann_build_paper_tables.argtypes = [vp, vp]
    L.riann_match_paper.argtypes = [vp, vp, i32, i32, i64, vp, vp, vp, vp, i32, C.c_uint64,
                                    C.c_uint64, vp]
    L.riann_stack_frames.argtypes = [C.POINTER(vp), i32, i32, i32, i32, i64, vp, vp]
    L.riann_last_error.argtypes = []
    L.riann_last_error.restype = C.c_char_p
    L.riann_version.argtypes = []
    L.riann_version.restype = C.c_uint32
    for name in EXPORTS:
        if name not in ("riann_last_error", "riann_version"):
            getattr(L, name).restype = C.c_int
    return L


_lib = _load()


def lib():
    return _lib


def _check(status: int) -> None:
    if status != RIANN_OK:
        raise RiannError(status, _lib.riann_last_error().decode(errors="replace"))


def _stream_ptr(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) or None


def field_shape(H: int, W: int, patch: int, stride: int) -> Tuple[int, int]:
    return (H - patch) // stride + 1, (W - patch) // stride + 1


def make_params(n_ref: int, n_keys: int, patch: int, channels: int, stride: int,
                dense_threshold: int = -1, flags: int = 0) -> Params:
    return Params(patch, channels, stride, n_keys, n_ref, dense_threshold, flags, 0)


def footprint(n_ref: int, n_keys: int, patch: int, channels: int, stride: int,
              H: int = 0, W: int = 0) -> int:
    """Device bytes of an index plus one stream's scratch for H x W frames."""
    b = C.c_int64()
    p = make_params(n_ref, n_keys, patch, channels, stride)
    _check(_lib.riann_footprint(C.byref(p), H, W, C.byref(b)))
    return int(b.value)


def _frame_geom(frame, channels: int):
    """(H, W, pitch) of a uint8 device tensor (H, W) or (H, W, C)."""
    import torch
    if frame.dtype != torch.uint8 or not frame.is_cuda:
        raise TypeError("frame must be a uint8 device tensor")
    if frame.dim() == 2:
        frame = frame.unsqueeze(-1)
    if frame.dim() != 3 or frame.shape[2] != channels:
        raise ValueError(f"frame must be (H, W, {channels})")
    if frame.stride(2) != 1 or frame.stride(1) != channels:
        raise ValueError("frame rows must be contiguous (H, W, C) with C innermost")
    return int(frame.shape[0]), int(frame.shape[1]), int(frame.stride(0))


def stack_frames(frames, out=None, stream=None):
    """T device frames (each (H, W) or (H, W, C) uint8, oldest first) -> one
    (H, W, T*C) frame whose p x p patches are the p x p x T space-time
    patches in (dy, dx, t, c) order (riann_stack_frames)."""
    import torch
    T = len(frames)
    if T < 1:
        raise ValueError("need at least one frame")
    C0 = 1 if frames[0].dim() == 2 else int(frames[0].shape[2])
    geo = [_frame_geom(f, C0) for f in frames]
    H, W, pitch = geo[0]
    if any(g != geo[0] for g in geo):
        raise ValueError("frames must share shape and row pitch")
    if out is None:
        out = torch.empty((H, W, T * C0), dtype=torch.uint8, device=frames[0].device)
    arr = (C.c_void_p * T)(*[f.data_ptr() for f in frames])
    _check(_lib.riann_stack_frames(arr, T, H, W, C0, pitch, out.data_ptr(), _stream_ptr(stream)))
    return out


class Index:
    """A built reference index (owns device tables)."""

    def __init__(self, handle: int, params: Params):
        self._h = C.c_void_p(handle)
        self.params = params

    # ---------------------------------------------------------------- build
    @classmethod
    def build(cls, ref: np.ndarray, keys: Sequence[int], patch: int, channels: int = 1,
              stride: int = 1, dense_threshold: int = -1, stream=None,
              flags: int = 0) -> "Index":
        ref = np.ascontiguousarray(ref, dtype=np.uint8)
        keys = np.ascontiguousarray(np.asarray(keys, dtype=np.int32))
        if ref.ndim != 2 or ref.shape[1] != patch * patch * channels:
            raise ValueError("ref must be (n, patch*patch*channels) uint8")
        p = make_params(ref.shape[0], len(keys), patch, channels, stride, dense_threshold, flags)
        h = C.c_void_p()
        _check(_lib.riann_build(ref.ctypes.data, keys.ctypes.data if len(keys) else None,
                                C.byref(p), _stream_ptr(stream), C.byref(h)))
        q = Params()
        _check(_lib.riann_get_params(h, C.byref(q)))
        return cls(h.value, q)

    @classmethod
    def load(cls, path: str, stream=None) -> "Index":
        h = C.c_void_p()
        _check(_lib.riann_load(path.encode(), _stream_ptr(stream), C.byref(h)))
        q = Params()
        _check(_lib.riann_get_params(h, C.byref(q)))
        return cls(h.value, q)

    def save(self, path: str) -> None:
        _check(_lib.riann_save(self._h, path.encode()))

    def close(self) -> None:
        if self._h is not None and self._h.value:
            _check(_lib.riann_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- queries
    @property
    def handle(self) -> int:
        return self._h.value

    def field_shape(self, H: int, W: int) -> Tuple[int, int]:
        return field_shape(H, W, self.params.patch, self.params.stride)

    def _outputs(self, H, W, device, out, ssd):
        import torch
        hq, wq = self.field_shape(H, W)
        if hq <= 0 or wq <= 0:
            # let the library report the shape error; nothing is written
            hq, wq = 1, 1
        if out is None:
            out = torch.empty((hq, wq), dtype=torch.int32, device=device)
        if ssd is None:
            ssd = torch.empty((hq, wq), dtype=torch.int32, device=device)
        for t in (out, ssd):
            if t.numel() != hq * wq or not t.is_contiguous() or t.element_size() != 4:
                raise ValueError("out/ssd must be contiguous 4-byte (Hq, Wq) tensors")
        return out, ssd

    def match_frame(self, frame, prev=None, out=None, ssd=None, stream=None):
        """Ring-intersection search of one frame given the previous field."""
        H, W, pitch = _frame_geom(frame, self.params.channels)
        out, ssd = self._outputs(H, W, frame.device, out, ssd)
        if prev is not None:
            if prev.numel() != out.numel() or not prev.is_contiguous() or prev.element_size() != 4:
                raise ValueError("prev must be a contiguous int32 (Hq, Wq) tensor")
        _check(_lib.riann_match_frame(self._h, frame.data_ptr(), H, W, pitch,
                                      prev.data_ptr() if prev is not None else None,
                                      out.data_ptr(), ssd.data_ptr(), _stream_ptr(stream)))
        return out, ssd

    def match_frame_noalloc(self, frame, prev, out, ssd, stream=None):
        """match_frame through the entry point that allocates nothing: the
        caller supplies out and ssd, and the library's scratch is its static
        per-GPU array (frames up to its size only; calls that overlap on one
        GPU race)."""
        H, W, pitch = _frame_geom(frame, self.params.channels)
        hq, wq = self.field_shape(H, W)
        for name, t in (("out", out), ("ssd", ssd), ("prev", prev)):
            if t is None:
                if name == "prev":
                    continue
                raise ValueError(f"{name} must be given (this call allocates nothing)")
            if (t.numel() != max(hq, 0) * max(wq, 0) or not t.is_contiguous()
                    or t.element_size() != 4 or t.device != frame.device):
                raise ValueError(f"{name} must be a contiguous 4-byte ({hq}, {wq}) tensor on "
                                 "the frame's device")
        _check(_lib.riann_match_frame_noalloc(self._h, frame.data_ptr(), H, W, pitch,
                                              prev.data_ptr() if prev is not None else None,
                                              out.data_ptr(), ssd.data_ptr(),
                                              _stream_ptr(stream)))
        return out, ssd

    def match_knn(self, frame, k: int, prev=None, full: bool = False, out=None, ssd=None,
                  stream=None):
        """Exact k-NN field (Hq, Wq, k), ascending (SSD, index) per query;
        `prev` is the previous frame's (Hq, Wq, k) field (ring mode)."""
        import torch
        H, W, pitch = _frame_geom(frame, self.params.channels)
        hq, wq = self.field_shape(max(H, 1), max(W, 1))
        hq, wq = max(hq, 1), max(wq, 1)
        if out is None:
            out = torch.empty((hq, wq, k), dtype=torch.int32, device=frame.device)
        if ssd is None:
            ssd = torch.empty((hq, wq, k), dtype=torch.int32, device=frame.device)
        if prev is not None and (prev.numel() != out.numel() or not prev.is_contiguous()
                                 or prev.element_size() != 4):
            raise ValueError("prev must be a contiguous int32 (Hq, Wq, k) tensor")
        _check(_lib.riann_match_knn(self._h, frame.data_ptr(), H, W, pitch, int(k),
                                    prev.data_ptr() if prev is not None and not full else None,
                                    out.data_ptr(), ssd.data_ptr(),
                                    MODE_FULL if full else MODE_RING, _stream_ptr(stream)))
        return out, ssd

    def build_paper_tables(self, stream=None) -> None:
        """n x n sorted distance tables for match_paper (synchronous)."""
        _check(_lib.riann_build_paper_tables(self._h, _stream_ptr(stream)))

    def match_paper(self, frame, prev=None, L: int = 20, seed: int = 0, t: int = 0,
                    out=None, ssd=None, iters=None, stream=None):
        """The paper's approximate search (Algorithm 1, alpha = 1/4) of one
        frame; returns (out, ssd, iters) with iters the anchors per query."""
        import torch
        H, W, pitch = _frame_geom(frame, self.params.channels)
        out, ssd = self._outputs(H, W, frame.device, out, ssd)
        if iters is None:
            iters = torch.empty_like(out)
        if prev is not None and (prev.numel() != out.numel() or not prev.is_contiguous()
                                 or prev.element_size() != 4):
            raise ValueError("prev must be a contiguous int32 (Hq, Wq) tensor")
        _check(_lib.riann_match_paper(self._h, frame.data_ptr(), H, W, pitch,
                                      prev.data_ptr() if prev is not None else None,
                                      out.data_ptr(), ssd.data_ptr(), iters.data_ptr(), int(L),
                                      C.c_uint64(seed & (2**64 - 1)), C.c_uint64(t),
                                      _stream_ptr(stream)))
        return out, ssd, iters

    def full_search(self, frame, out=None, ssd=None, stream=None):
        """Exact exhaustive search of one frame (first frame, scene cuts)."""
        H, W, pitch = _frame_geom(frame, self.params.channels)
        out, ssd = self._outputs(H, W, frame.device, out, ssd)
        _check(_lib.riann_full_search(self._h, frame.data_ptr(), H, W, pitch, out.data_ptr(),
                                      ssd.data_ptr(), _stream_ptr(stream)))
        return out, ssd

    def reconstruct(self, field, H: int, W: int, app=None, gt=None, out=None, with_error=True,
                    stream=None):
        """Frame rebuilt from `field` (Sec. 4): every query patch replaced by
        its match -- or by row field[i, j] of `app`, an (n, p*p*Ca) uint8
        device tensor of transformed references (Sec. 5) -- and overlapping
        patches averaged.  Returns (out (H, W, Ca) float32, err) where err is
        a device float64 tensor {E, sum (gt-out)^2, sum gt^2, values} when
        `gt` (H, W[, Ca] uint8 device frame) is given and with_error, else None."""
        import torch
        p = self.params
        if field.dtype != torch.int32 or not field.is_cuda or not field.is_contiguous():
            raise TypeError("field must be a contiguous int32 device tensor")
        if app is not None:
            if app.dtype != torch.uint8 or not app.is_cuda or not app.is_contiguous():
                raise TypeError("app must be a contiguous uint8 device tensor")
            ca = app.shape[1] // (p.patch * p.patch)
        else:
            ca = p.channels
        gp = 0
        if gt is not None:
            _, _, gp = _frame_geom(gt, ca)
        if out is None:
            out = torch.empty((H, W, ca), dtype=torch.float32, device=field.device)
        err = (torch.empty(4, dtype=torch.float64, device=field.device)
               if gt is not None and with_error else None)
        _check(_lib.riann_reconstruct(self._h, field.data_ptr(), H, W,
                                      app.data_ptr() if app is not None else None, ca,
                                      out.data_ptr(), gt.data_ptr() if gt is not None else None,
                                      gp, err.data_ptr() if err is not None else None,
                                      _stream_ptr(stream)))
        return out, err

    def _batch_desc(self, it: dict) -> FrameDesc:
        """Checks one batch item (the C ABI cannot see device buffer sizes)
        and returns its descriptor."""
        frame = it["frame"]
        H, W, pitch = _frame_geom(frame, self.params.channels)
        hq, wq = self.field_shape(H, W)
        mode = int(it.get("mode", MODE_RING))
        if mode not in (MODE_RING, MODE_FULL):
            raise ValueError(f"mode must be MODE_RING or MODE_FULL, got {mode}")
        out, ssd, prev = it["out"], it.get("ssd"), it.get("prev")
        if mode != MODE_RING:
            prev = None                     # the full search ignores a previous field
        for name, t in (("out", out), ("ssd", ssd), ("prev", prev)):
            if t is None:
                continue
            if (t.numel() != max(hq, 0) * max(wq, 0) or not t.is_contiguous()
                    or t.element_size() != 4 or t.device != frame.device):
                raise ValueError(f"{name} must be a contiguous 4-byte ({hq}, {wq}) tensor on "
                                 f"the frame's device")
        return FrameDesc(frame.data_ptr(), H, W, pitch,
                         prev.data_ptr() if prev is not None else None, out.data_ptr(),
                         ssd.data_ptr() if ssd is not None else None, mode, 0)

    def match_batch(self, items: List[dict], stream=None) -> None:
        """items: dicts with frame, out, ssd (optional), prev (optional; ignored
        in MODE_FULL), mode.  Every item is checked before anything is launched."""
        descs = [self._batch_desc(it) for it in items]
        arr = (FrameDesc * len(descs))(*descs)
        _check(_lib.riann_match_batch(self._h, arr, len(descs), _stream_ptr(stream)))

    def stats(self) -> dict:
        s = Stats()
        _check(_lib.riann_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    def reset_stats(self) -> None:
        _check(_lib.riann_reset_stats(self._h))

    def set_dense_threshold(self, threshold: int) -> None:
        """Routing threshold for later launches (a performance knob only)."""
        _check(_lib.riann_set_dense_threshold(self._h, int(threshold)))
        self.params.dense_threshold = int(threshold)

    def dense_shapes(self) -> Tuple[List[Tuple[int, int]], int]:
        """Block shapes (waves, cols) of the row-layout dense search built for
        this patch width (default first) and the index of the one in use."""
        wv, cl = (C.c_int32 * 16)(), (C.c_int32 * 16)()
        cnt, cur = C.c_int32(), C.c_int32()
        _check(_lib.riann_get_dense_shapes(self._h, wv, cl, 16, C.byref(cnt), C.byref(cur)))
        return [(int(wv[i]), int(cl[i])) for i in range(min(cnt.value, 16))], int(cur.value)

    def set_dense_shape(self, waves: int, cols: int) -> None:
        """Block shape of the dense search for later launches (a performance
        knob only); (0, 0) is the default."""
        _check(_lib.riann_set_dense_shape(self._h, int(waves), int(cols)))

    def set_profiling(self, enable=True) -> None:
        """True: time every kernel; "dense": only the dense search; False: off.
        Turning it on resets the totals."""
        level = PROFILE_DENSE if enable == "dense" else (PROFILE_ALL if enable else 0)
        _check(_lib.riann_set_profiling(self._h, level))

    def profile(self) -> dict:
        """Per-kernel launch counts and total milliseconds (HIP events)."""
        p = Profile()
        _check(_lib.riann_get_profile(self._h, C.byref(p)))
        return {k: dict(launches=int(p.launches[i]), ms=float(p.ms[i]))
                for i, k in enumerate(KERNELS)}
