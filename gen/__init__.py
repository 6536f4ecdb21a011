"""Seeded synthetic inputs for the RIANN workloads.

This module only makes inputs: textures, moving frames, reference patch sets,
key-point indices, scene-cut flags and arrival traces.  It holds none of the
search method's arithmetic (no distances, no tables, no matching), so both the
CPU oracle and the GPU path can consume its output without sharing any code.

The paper evaluates on Hollywood2 videos (Sec. 4, "Empirical evaluation"),
which are not available here; these seeded generators stand in for them with
the shapes, sizes and motion structure of the five workloads:

  tiny      8 x 64x64 gray, 0.5 px/frame drift, 8x8 patches, n=1024,  K=8
  hd720     60 x 1280x720 gray, per-tile affine motion (<=1 px/frame),
            10% of tiles re-seeded every frame, n=16384, K=16
  fhd_rgb   120 x 1920x1080x3, drift, scene cut every 30 frames,
            8x8x3 patches, n=65536, K=32
  serving   64 RGB streams of mixed resolution, Poisson arrivals at 30 fps,
            shared reference n=65536, K=32
  uhd_mix   3840x2160 gray, 12x12 patches at stride 2, 20% high-motion tiles,
            a cut every 50 frames, batched with 640x360 frames, n=262144, K=48

Texture: U[0,255] noise, Gaussian blur with sigma 2 (truncated at 4 sigma,
reflecting borders), no contrast stretch.  Frames: bilinear resampling of the
texture under the motion, plus N(0, 2^2) pixel noise, rounded half-to-even,
clipped to [0, 255] and stored as uint8 (H x W x C, row-major, channels last).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Tuple

import numpy as np
from scipy import ndimage

BASE_SEED = 150807953
BLUR_SIGMA = 2.0
NOISE_SIGMA = 2.0

# Workload table: (name, patch, channels, stride, n_ref, n_keys)
WORKLOADS: Dict[str, dict] = {
    "tiny": dict(patch=8, channels=1, stride=1, n_ref=1024, n_keys=8,
                 H=64, W=64, frames=8, seed_offset=1),
    "hd720": dict(patch=8, channels=1, stride=1, n_ref=16384, n_keys=16,
                  H=720, W=1280, frames=60, seed_offset=2),
    "fhd_rgb": dict(patch=8, channels=3, stride=1, n_ref=65536, n_keys=32,
                    H=1080, W=1920, frames=120, seed_offset=3, cut_every=30),
    "serving": dict(patch=8, channels=3, stride=1, n_ref=65536, n_keys=32,
                    streams=64, fps=30.0, seed_offset=4),
    "uhd_mix": dict(patch=12, channels=1, stride=2, n_ref=262144, n_keys=48,
                    H=2160, W=3840, frames=100, seed_offset=5, cut_every=50,
                    small=(360, 640)),
}


def _rng(seed_offset: int, purpose: int, extra: int = 0) -> np.random.Generator:
    """Independent child generator per (workload, purpose, extra) triple."""
    ss = np.random.SeedSequence([BASE_SEED + seed_offset, purpose, extra])
    return np.random.default_rng(ss)


# purposes
P_TEXTURE, P_REFERENCE, P_KEYS, P_NOISE, P_MOTION, P_RESEED, P_TRACE = range(7)


def texture(rng: np.random.Generator, h: int, w: int, c: int = 1) -> np.ndarray:
    """Blurred uniform-noise texture, float64 (h, w, c)."""
    out = np.empty((h, w, c), np.float64)
    for ch in range(c):
        t = rng.uniform(0.0, 255.0, size=(h, w))
        out[:, :, ch] = ndimage.gaussian_filter(t, BLUR_SIGMA, mode="reflect",
                                                truncate=4.0)
    return out


def _finish(img: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Add pixel noise, round half to even, clip, cast to uint8."""
    noisy = img + rng.normal(0.0, NOISE_SIGMA, size=img.shape)
    return np.clip(np.rint(noisy), 0, 255).astype(np.uint8)


def _shift_x(tex: np.ndarray, y0: int, x0: float, h: int, w: int) -> np.ndarray:
    """Bilinear sample tex[y0:y0+h, x0:x0+w] at a fractional x offset."""
    xi = int(np.floor(x0))
    fx = x0 - xi
    a = tex[y0:y0 + h, xi:xi + w]
    if fx == 0.0:
        return a.copy()
    b = tex[y0:y0 + h, xi + 1:xi + 1 + w]
    return (1.0 - fx) * a + fx * b


# --------------------------------------------------------------------------
# drifting-texture video (tiny, fhd_rgb, serving streams)
# --------------------------------------------------------------------------
class DriftVideo:
    """Texture translated along +x at `speed` px/frame, optional hard cuts.

    Frame t shows texture(x - speed * t'), where t' counts frames since the
    last cut; each cut starts a fresh texture (new seed).
    """

    def __init__(self, seed_offset: int, H: int, W: int, C: int, frames: int,
                 speed: float = 0.5, cut_every: Optional[int] = None,
                 stream: int = 0):
        self.so, self.H, self.W, self.C = seed_offset, H, W, C
        self.frames, self.speed, self.cut_every = frames, speed, cut_every
        self.stream = stream
        span = frames if cut_every is None else min(frames, cut_every)
        self.margin = int(np.ceil(speed * span)) + 4
        self._tex: Dict[int, np.ndarray] = {}

    def shot(self, t: int) -> Tuple[int, int]:
        if self.cut_every is None:
            return 0, t
        return t // self.cut_every, t % self.cut_every

    def is_cut(self, t: int) -> bool:
        return t == 0 or (self.cut_every is not None and t % self.cut_every == 0)

    def _texture(self, shot: int) -> np.ndarray:
        if shot not in self._tex:
            rng = _rng(self.so, P_TEXTURE, self.stream * 1000 + shot)
            self._tex = {shot: texture(rng, self.H + 2, self.W + self.margin + 2,
                                       self.C)}
        return self._tex[shot]

    def frame(self, t: int) -> np.ndarray:
        shot, tl = self.shot(t)
        tex = self._texture(shot)
        img = _shift_x(tex, 1, 1 + self.margin - self.speed * tl, self.H, self.W)
        rng = _rng(self.so, P_NOISE, self.stream * 100000 + t)
        return _finish(img, rng)


# --------------------------------------------------------------------------
# tiled affine-motion video (hd720, uhd_mix)
# --------------------------------------------------------------------------
class TiledVideo:
    """Frame made of 64x64 tiles, each a texture under its own affine motion.

    Each tile's displacement at frame t (frames since its shot started) is
    t * (A @ (x - cx, y - cy) + b), with the per-frame displacement bounded
    by `slow` px everywhere in the tile (or `fast` px for high-motion tiles).
    Every frame t >= 1, each tile is re-seeded with probability `reseed_p`:
    it gets a fresh texture and keeps it afterwards.  A hard cut replaces
    every tile's texture and motion.
    """
    TILE = 64

    def __init__(self, seed_offset: int, H: int, W: int, frames: int,
                 slow: float = 1.0, fast: float = 0.0, fast_p: float = 0.0,
                 reseed_p: float = 0.0, cut_every: Optional[int] = None,
                 stream: int = 0):
        self.so, self.H, self.W, self.frames = seed_offset, H, W, frames
        self.slow, self.fast, self.fast_p = slow, fast, fast_p
        self.reseed_p, self.cut_every, self.stream = reseed_p, cut_every, stream
        self.ty = (H + self.TILE - 1) // self.TILE
        self.tx = (W + self.TILE - 1) // self.TILE
        nt = self.ty * self.tx
        span = frames if cut_every is None else min(frames, cut_every)
        vmax = max(slow, fast)
        self.margin = int(np.ceil(vmax * span)) + 4
        # textures large enough for the whole drift, or (for fast motion over
        # long shots) a smaller periodic texture sampled with wrap-around
        self.wrap = self.TILE + 2 * self.margin > 256
        self.canvas = 128 if self.wrap else self.TILE + 2 * self.margin
        self._state_t = -1
        self._tex: List[np.ndarray] = [None] * nt  # type: ignore
        self._t0 = np.zeros(nt, np.int64)           # frame the texture started
        self._A = np.zeros((nt, 2, 2))
        self._b = np.zeros((nt, 2))

    def is_cut(self, t: int) -> bool:
        return t == 0 or (self.cut_every is not None and t % self.cut_every == 0)

    def _new_motion(self, rng: np.random.Generator, i: int, shot: int) -> None:
        fast = rng.random() < self.fast_p
        vmax = self.fast if fast else self.slow
        A = rng.uniform(-1.0, 1.0, size=(2, 2)) * 0.01
        ang = rng.uniform(0.0, 2.0 * np.pi)
        b = rng.uniform(0.2, 1.0) * np.array([np.cos(ang), np.sin(ang)])
        h = self.TILE / 2.0
        corners = np.array([[-h, -h], [-h, h], [h, -h], [h, h]])
        peak = np.max(np.linalg.norm(corners @ A.T + b, axis=1))
        scale = vmax / peak if peak > 0 else 0.0
        self._A[i], self._b[i] = A * scale, b * scale

    def _new_texture(self, i: int, key: int) -> None:
        rng = _rng(self.so, P_TEXTURE, (self.stream * 10**7) + key)
        s = self.canvas
        if self.wrap:
            t = rng.uniform(0.0, 255.0, size=(s, s))
            self._tex[i] = ndimage.gaussian_filter(t, BLUR_SIGMA, mode="wrap",
                                                   truncate=4.0).astype(np.float32)
        else:
            self._tex[i] = texture(rng, s, s, 1)[:, :, 0]

    def _advance(self, t: int) -> None:
        """Bring tile state (textures, motions, start frames) up to frame t."""
        if t < self._state_t:
            self._state_t = -1
        nt = self.ty * self.tx
        while self._state_t < t:
            u = self._state_t + 1
            if self.is_cut(u):
                shot = 0 if self.cut_every is None else u // self.cut_every
                rng = _rng(self.so, P_MOTION, self.stream * 10**5 + shot)
                for i in range(nt):
                    self._new_motion(rng, i, shot)
                    self._new_texture(i, u * nt + i)
                    self._t0[i] = u
            elif self.reseed_p > 0.0:
                rng = _rng(self.so, P_RESEED, self.stream * 10**5 + u)
                hit = np.nonzero(rng.random(nt) < self.reseed_p)[0]
                for i in hit:
                    self._new_texture(int(i), u * nt + int(i))
            self._state_t = u

    def frame(self, t: int) -> np.ndarray:
        self._advance(t)
        T = self.TILE
        img = np.empty((self.H, self.W), np.float64)
        yy, xx = np.mgrid[0:T, 0:T].astype(np.float64)
        rel = np.stack([xx - T / 2.0, yy - T / 2.0], axis=-1)
        for ty in range(self.ty):
            for tx in range(self.tx):
                i = ty * self.tx + tx
                h = min(T, self.H - ty * T)
                w = min(T, self.W - tx * T)
                tl = t - (0 if self.cut_every is None
                          else (t // self.cut_every) * self.cut_every)
                disp = tl * (rel @ self._A[i].T + self._b[i])
                if self.wrap:
                    cx = xx - disp[..., 0]
                    cy = yy - disp[..., 1]
                    v = ndimage.map_coordinates(self._tex[i], [cy[:h, :w], cx[:h, :w]],
                                                order=1, mode="grid-wrap")
                else:
                    cx = self.margin + xx - disp[..., 0]
                    cy = self.margin + yy - disp[..., 1]
                    v = ndimage.map_coordinates(self._tex[i], [cy[:h, :w], cx[:h, :w]],
                                                order=1, mode="nearest")
                img[ty * T:ty * T + h, tx * T:tx * T + w] = v
        rng = _rng(self.so, P_NOISE, self.stream * 100000 + t)
        return _finish(img[:, :, None], rng)


# --------------------------------------------------------------------------
# reference sets and key points
# --------------------------------------------------------------------------
def patches_at(frame: np.ndarray, ys: np.ndarray, xs: np.ndarray, p: int) -> np.ndarray:
    """Copy p x p x C windows with top-left corners (ys, xs), flattened in
    (dy, dx, c) order -> (len, p*p*C) uint8."""
    H, W, C = frame.shape
    out = np.empty((len(ys), p * p * C), np.uint8)
    for i, (y, x) in enumerate(zip(ys, xs)):
        out[i] = frame[y:y + p, x:x + p, :].reshape(-1)
    return out


def reference_from_frame(frame: np.ndarray, n: int, p: int, stride: int,
                         rng: np.random.Generator) -> np.ndarray:
    """n patches at distinct random window positions of `frame`."""
    H, W, C = frame.shape
    hq, wq = (H - p) // stride + 1, (W - p) // stride + 1
    if n > hq * wq:
        raise ValueError("reference set larger than the frame's window count")
    pos = np.sort(rng.choice(hq * wq, size=n, replace=False))
    ys, xs = (pos // wq) * stride, (pos % wq) * stride
    # vectorised gather of windows
    win = np.lib.stride_tricks.sliding_window_view(frame, (p, p, C))[:, :, 0]
    return np.ascontiguousarray(win[ys, xs].reshape(n, p * p * C))


def choose_keys(n: int, k: int, rng: np.random.Generator) -> np.ndarray:
    """k distinct reference indices drawn without replacement, sorted."""
    if k == 0:
        return np.zeros(0, np.int32)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)


@dataclasses.dataclass
class Workload:
    name: str
    patch: int
    channels: int
    stride: int
    ref: np.ndarray          # (n, D) uint8
    keys: np.ndarray         # (K,) int32
    video: object            # DriftVideo | TiledVideo
    frames: int

    @property
    def D(self) -> int:
        return self.patch * self.patch * self.channels

    def frame(self, t: int) -> np.ndarray:
        return self.video.frame(t)

    def is_cut(self, t: int) -> bool:
        return self.video.is_cut(t)


def make_video(name: str, stream: int = 0, H: Optional[int] = None,
               W: Optional[int] = None, frames: Optional[int] = None,
               second: bool = False):
    """The query video of a workload (second=True: an independent video of
    the same generator, used to draw reference patches)."""
    cfg = WORKLOADS[name]
    so = cfg["seed_offset"] + (1000 if second else 0)
    if name == "tiny":
        return DriftVideo(so, H or cfg["H"], W or cfg["W"], 1, frames or cfg["frames"],
                          speed=0.5, stream=stream)
    if name == "hd720":
        return TiledVideo(so, H or cfg["H"], W or cfg["W"], frames or cfg["frames"],
                          slow=1.0, reseed_p=0.1, stream=stream)
    if name == "fhd_rgb":
        return DriftVideo(so, H or cfg["H"], W or cfg["W"], 3, frames or cfg["frames"],
                          speed=0.5, cut_every=cfg["cut_every"], stream=stream)
    if name == "serving":
        return DriftVideo(so, H or 360, W or 640, 3, frames or 300, speed=0.5,
                          stream=stream)
    if name == "uhd_mix":
        return TiledVideo(so, H or cfg["H"], W or cfg["W"], frames or cfg["frames"],
                          slow=1.0, fast=8.0, fast_p=0.2, cut_every=cfg["cut_every"],
                          stream=stream)
    raise KeyError(name)


def make_workload(name: str, n_ref: Optional[int] = None, n_keys: Optional[int] = None,
                  H: Optional[int] = None, W: Optional[int] = None,
                  frames: Optional[int] = None) -> Workload:
    """Query video, reference set (from frame 0 of a second video of the same
    generator) and key points of a named workload.  Sizes may be overridden
    for small test cases."""
    cfg = WORKLOADS[name]
    p, C, s = cfg["patch"], cfg["channels"], cfg["stride"]
    n = cfg["n_ref"] if n_ref is None else n_ref
    K = cfg["n_keys"] if n_keys is None else n_keys
    if name == "serving":
        rv = DriftVideo(cfg["seed_offset"] + 1000, H or 1080, W or 1920, 3, 1)
    else:
        rv = make_video(name, H=H, W=W, frames=1, second=True)
    ref = reference_from_frame(rv.frame(0), n, p, 1,
                               _rng(cfg["seed_offset"], P_REFERENCE))
    keys = choose_keys(n, K, _rng(cfg["seed_offset"], P_KEYS, K))
    video = make_video(name, H=H, W=W, frames=frames)
    return Workload(name, p, C, s, ref, keys, video, video.frames)


def random_field(hq: int, wq: int, n: int, rng: np.random.Generator,
                 no_prior_p: float = 0.0) -> np.ndarray:
    """Uniform previous field over [0, n) (the paper's random initial field,
    shifted to 0-based indices), optionally with -1 "no prior" entries."""
    f = rng.integers(0, n, size=(hq, wq)).astype(np.int32)
    if no_prior_p > 0.0:
        f[rng.random((hq, wq)) < no_prior_p] = -1
    return f


def poisson_trace(n_streams: int, fps: float, duration_s: float,
                  seed_offset: int = WORKLOADS["serving"]["seed_offset"]
                  ) -> List[Tuple[float, int, int]]:
    """Merged Poisson arrival trace: (time_s, stream, frame_index) sorted by time."""
    ev = []
    for s in range(n_streams):
        rng = _rng(seed_offset, P_TRACE, s)
        t, k = 0.0, 0
        while True:
            t += rng.exponential(1.0 / fps)
            if t > duration_s:
                break
            ev.append((t, s, k))
            k += 1
    ev.sort()
    return ev


def serving_stream_shape(stream: int) -> Tuple[int, int]:
    """Stream id mod 3 -> 640x360, 1280x720, 1920x1080 (H, W)."""
    return [(360, 640), (720, 1280), (1080, 1920)][stream % 3]
