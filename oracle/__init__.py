"""CPU oracle for RIANN ANN fields -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never links or calls it, and it
shares no code with the GPU path: the C source `riann_oracle.c` has its own
patch extraction, distances, table build, integer square root, binary search
and reductions (see its header for what each function follows in the paper).

This module only marshals numpy arrays into that C library; all arithmetic is
in the C file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "riann_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
INF = (1 << 64) - 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        # x86-64-v3 (AVX2): every host the library runs on has it; -march=native
        # would tie the build to the build host's CPU
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-shared",
                               "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        u8p, i32p, u32p, i64p, u64p = (C.POINTER(C.c_uint8), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_uint32), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_uint64))
        L.orc_set_fault.argtypes = [C.c_int]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = C.c_int
        L.orc_extract.argtypes = [u8p, C.c_int, C.c_int, C.c_int, C.c_int64,
                                  C.c_int, C.c_int, u8p]
        L.orc_ssd.argtypes = [u8p, u8p, C.c_int]
        L.orc_ssd.restype = C.c_uint64
        L.orc_bf.argtypes = [u8p, C.c_int64, u8p, C.c_int64, C.c_int, i32p, u32p]
        L.orc_isqrt.argtypes = [C.c_uint64]
        L.orc_isqrt.restype = C.c_uint64
        L.orc_ring_bounds.argtypes = [C.c_uint64, C.c_uint64, u64p, u64p]
        L.orc_build.argtypes = [u8p, C.c_int64, C.c_int, i32p, C.c_int, u32p, i32p, u32p]
        L.orc_riann.argtypes = [u8p, C.c_int64, u8p, C.c_int64, C.c_int, i32p, C.c_int,
                                u32p, i32p, u32p, i32p, i32p, u32p, i64p, i32p, i64p,
                                u8p]
        L.orc_riann_candidates.argtypes = [u8p, u8p, C.c_int64, C.c_int, i32p, C.c_int,
                                           u32p, i32p, u32p, C.c_int32, i32p, C.c_int64]
        L.orc_riann_candidates.restype = C.c_int64
        L.orc_knn_bf.argtypes = [u8p, C.c_int64, u8p, C.c_int64, C.c_int, C.c_int, i32p, u32p]
        L.orc_knn_riann.argtypes = [u8p, C.c_int64, u8p, C.c_int64, C.c_int, i32p, C.c_int,
                                    u32p, i32p, u32p, i32p, C.c_int, i32p, u32p]
        L.orc_splitmix.argtypes = [C.c_uint64]
        L.orc_splitmix.restype = C.c_uint64
        L.orc_paper_tables.argtypes = [u8p, C.c_int64, C.c_int, u32p, u32p, i32p]
        L.orc_paper.argtypes = [u8p, C.c_int64, u8p, C.c_int64, C.c_int, u32p, u32p, i32p, i32p,
                                C.c_int, C.c_uint64, C.c_uint64, C.c_int64, i32p, u32p, i32p]
        L.orc_extract3d.argtypes = [C.POINTER(u8p), C.c_int, C.c_int, C.c_int, C.c_int,
                                    C.c_int, C.c_int, u8p]
        L.orc_reconstruct.argtypes = [i32p, C.c_int, C.c_int, u8p, C.c_int64, C.c_int, C.c_int,
                                      C.c_int, C.c_int, C.c_int, u32p, u32p, C.POINTER(C.c_float),
                                      u8p, C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray], t):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(t))


def set_fault(code: int) -> None:
    """Plant deliberate mistake `code` in the oracle (0 = correct)."""
    lib().orc_set_fault(int(code))


def set_threads(n: int) -> int:
    """Worker threads of the oracle's parallel loops (0: keep); returns the
    count in effect."""
    return int(lib().orc_set_threads(int(n)))


def field_shape(H: int, W: int, p: int, s: int) -> Tuple[int, int]:
    return (H - p) // s + 1, (W - p) // s + 1


def extract(frame: np.ndarray, p: int, s: int) -> np.ndarray:
    """frame (H, W, C) uint8 -> (Hq*Wq, p*p*C) patches, (dy, dx, c) order."""
    f = np.ascontiguousarray(frame, dtype=np.uint8)
    if f.ndim == 2:
        f = f[:, :, None]
    H, W, Cc = f.shape
    hq, wq = field_shape(H, W, p, s)
    out = np.empty((hq * wq, p * p * Cc), np.uint8)
    lib().orc_extract(_p(f, C.c_uint8), H, W, Cc, W * Cc, p, s, _p(out, C.c_uint8))
    return out


def extract3d(frames, p: int, s: int) -> np.ndarray:
    """T frames (each (H, W) or (H, W, C) uint8, oldest first) ->
    (Hq*Wq, p*p*T*C) spatio-temporal patches, (dy, dx, t, c) order."""
    fs = [np.ascontiguousarray(f if f.ndim == 3 else f[:, :, None], np.uint8) for f in frames]
    H, W, Cc = fs[0].shape
    assert all(f.shape == fs[0].shape for f in fs)
    T = len(fs)
    hq, wq = field_shape(H, W, p, s)
    out = np.empty((hq * wq, p * p * T * Cc), np.uint8)
    ptrs = (C.POINTER(C.c_uint8) * T)(*[_p(f, C.c_uint8) for f in fs])
    lib().orc_extract3d(ptrs, T, H, W, Cc, p, s, _p(out, C.c_uint8))
    return out


def ssd(a: np.ndarray, b: np.ndarray) -> int:
    a = np.ascontiguousarray(a, np.uint8)
    b = np.ascontiguousarray(b, np.uint8)
    return int(lib().orc_ssd(_p(a, C.c_uint8), _p(b, C.c_uint8), a.size))


def brute_force(patches: np.ndarray, ref: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Exact NN of each patch in ref: (idx int32, ssd uint32), ties -> lowest."""
    q = np.ascontiguousarray(patches, np.uint8)
    r = np.ascontiguousarray(ref, np.uint8)
    Q, D = q.shape
    idx = np.empty(Q, np.int32)
    d = np.empty(Q, np.uint32)
    lib().orc_bf(_p(q, C.c_uint8), Q, _p(r, C.c_uint8), r.shape[0], D,
                 _p(idx, C.c_int32), _p(d, C.c_uint32))
    return idx, d


def reconstruct(field: np.ndarray, app: np.ndarray, p: int, s: int, H: int, W: int,
                gt: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """Average of the matched (or transformed) patches over the frame
    (Sec. 4); field entries outside [0, len(app)) contribute nothing.
    Returns f_R (H, W, Ca) float32, the per-pixel sum and count, and, when
    gt (H, W[, Ca]) uint8 is given, E and its parts."""
    fld = np.ascontiguousarray(field, np.int32)
    hq, wq = fld.shape
    a = np.ascontiguousarray(app, np.uint8)
    Ca = a.shape[1] // (p * p)
    assert a.shape[1] == p * p * Ca
    sm = np.empty((H, W, Ca), np.uint32)
    cnt = np.empty((H, W), np.uint32)
    fr = np.empty((H, W, Ca), np.float32)
    err = np.zeros(4, np.float64)
    g = None if gt is None else np.ascontiguousarray(gt, np.uint8).reshape(H, W, Ca)
    lib().orc_reconstruct(_p(fld, C.c_int32), hq, wq, _p(a, C.c_uint8), len(a), p, Ca, s, H, W,
                          _p(sm, C.c_uint32), _p(cnt, C.c_uint32), _p(fr, C.c_float),
                          _p(g, C.c_uint8), _p(err, C.c_double))
    out = {"f_r": fr, "sum": sm, "count": cnt}
    if g is not None:
        out.update(E=float(err[0]), sq_err=float(err[1]), sq_gt=float(err[2]),
                   values=int(err[3]))
    return out


def knn_brute_force(patches: np.ndarray, ref: np.ndarray, k: int) -> Tuple[np.ndarray, np.ndarray]:
    """Exact k nearest neighbours of each patch: (Q, k) idx int32 and ssd
    uint32, each row ascending by (SSD, index)."""
    q = np.ascontiguousarray(patches, np.uint8)
    r = np.ascontiguousarray(ref, np.uint8)
    Q, D = q.shape
    assert 1 <= k <= min(64, r.shape[0])
    idx = np.empty((Q, k), np.int32)
    d = np.empty((Q, k), np.uint32)
    lib().orc_knn_bf(_p(q, C.c_uint8), Q, _p(r, C.c_uint8), r.shape[0], D, k,
                     _p(idx, C.c_int32), _p(d, C.c_uint32))
    return idx, d


def splitmix(x: int) -> int:
    """SplitMix64 output for state x (the counter-based anchor generator)."""
    return int(lib().orc_splitmix(C.c_uint64(x & (2**64 - 1))))


class PaperTables:
    """The paper's pre-processing for Algorithm 1 (Sec. 3.3): the n x n SSD
    matrix of the references and each row sorted by (value, index)."""

    def __init__(self, ref: np.ndarray):
        self.ref = np.ascontiguousarray(ref, np.uint8)
        n, self.D = self.ref.shape
        self.n = n
        self.dm = np.empty((n, n), np.uint32)
        self.tv = np.empty((n, n), np.uint32)
        self.tp = np.empty((n, n), np.int32)
        lib().orc_paper_tables(_p(self.ref, C.c_uint8), n, self.D, _p(self.dm, C.c_uint32),
                               _p(self.tv, C.c_uint32), _p(self.tp, C.c_int32))

    def search(self, patches: np.ndarray, prev: np.ndarray, L: int = 20, seed: int = 0,
               t: int = 0, qbase: int = 0) -> Dict[str, np.ndarray]:
        """Algorithm 1 for every patch (approximate; see orc_paper)."""
        q = np.ascontiguousarray(patches, np.uint8)
        pv = np.ascontiguousarray(prev, np.int32).reshape(-1)
        Q = q.shape[0]
        assert pv.size == Q and q.shape[1] == self.D
        out = dict(idx=np.empty(Q, np.int32), ssd=np.empty(Q, np.uint32),
                   iters=np.empty(Q, np.int32))
        lib().orc_paper(_p(q, C.c_uint8), Q, _p(self.ref, C.c_uint8), self.n, self.D,
                        _p(self.dm, C.c_uint32), _p(self.tv, C.c_uint32), _p(self.tp, C.c_int32),
                        _p(pv, C.c_int32), int(L), C.c_uint64(seed), C.c_uint64(t),
                        int(qbase), _p(out["idx"], C.c_int32), _p(out["ssd"], C.c_uint32),
                        _p(out["iters"], C.c_int32))
        return out


def isqrt(x: int) -> int:
    return int(lib().orc_isqrt(C.c_uint64(x)))


def ring_bounds(b: int, c: Optional[int]) -> Tuple[int, int]:
    """Integer ring [lo, hi] of a key for query distance b and radius^2 c
    (c=None: no radius -> (0, INF))."""
    lo, hi = C.c_uint64(), C.c_uint64()
    lib().orc_ring_bounds(C.c_uint64(b), C.c_uint64(INF if c is None else c),
                          C.byref(lo), C.byref(hi))
    return lo.value, hi.value


class Tables:
    """Sorted key-distance tables of a reference set (pre-processing)."""

    def __init__(self, ref: np.ndarray, keys: np.ndarray):
        self.ref = np.ascontiguousarray(ref, np.uint8)
        self.keys = np.ascontiguousarray(keys, np.int32)
        self.n, self.D = self.ref.shape
        self.K = len(self.keys)
        n, K = self.n, self.K
        self.T = np.empty((K, n), np.uint32)
        self.P = np.empty((K, n), np.int32)
        self.Piv = np.empty((n, max(K, 1)), np.uint32)
        lib().orc_build(_p(self.ref, C.c_uint8), n, self.D, _p(self.keys, C.c_int32), K,
                        _p(self.T, C.c_uint32), _p(self.P, C.c_int32),
                        _p(self.Piv, C.c_uint32))

    def riann(self, patches: np.ndarray, prev: np.ndarray) -> Dict[str, np.ndarray]:
        """Exact-mode RIANN for every patch with previous matches `prev`."""
        q = np.ascontiguousarray(patches, np.uint8)
        pv = np.ascontiguousarray(prev, np.int32).reshape(-1)
        Q = q.shape[0]
        assert pv.size == Q and q.shape[1] == self.D
        out = dict(idx=np.empty(Q, np.int32), ssd=np.empty(Q, np.uint32),
                   mstar=np.empty(Q, np.int64), kstar=np.empty(Q, np.int32),
                   nsurv=np.empty(Q, np.int64), noprior=np.empty(Q, np.uint8))
        lib().orc_riann(_p(q, C.c_uint8), Q, _p(self.ref, C.c_uint8), self.n, self.D,
                        _p(self.keys, C.c_int32), self.K, _p(self.T, C.c_uint32),
                        _p(self.P, C.c_int32), _p(self.Piv, C.c_uint32),
                        _p(pv, C.c_int32), _p(out["idx"], C.c_int32),
                        _p(out["ssd"], C.c_uint32), _p(out["mstar"], C.c_int64),
                        _p(out["kstar"], C.c_int32), _p(out["nsurv"], C.c_int64),
                        _p(out["noprior"], C.c_uint8))
        return out

    def knn(self, patches: np.ndarray, prev: np.ndarray, k: int) -> Tuple[np.ndarray, np.ndarray]:
        """Exact-mode RIANN k-NN with previous k-NN matches `prev` (Q, k)."""
        q = np.ascontiguousarray(patches, np.uint8)
        pv = np.ascontiguousarray(prev, np.int32).reshape(-1)
        Q = q.shape[0]
        assert pv.size == Q * k and q.shape[1] == self.D and 1 <= k <= min(64, self.n)
        idx = np.empty((Q, k), np.int32)
        d = np.empty((Q, k), np.uint32)
        lib().orc_knn_riann(_p(q, C.c_uint8), Q, _p(self.ref, C.c_uint8), self.n, self.D,
                            _p(self.keys, C.c_int32), self.K, _p(self.T, C.c_uint32),
                            _p(self.P, C.c_int32), _p(self.Piv, C.c_uint32), _p(pv, C.c_int32),
                            k, _p(idx, C.c_int32), _p(d, C.c_uint32))
        return idx, d

    def candidates(self, patch: np.ndarray, prev: int) -> np.ndarray:
        q = np.ascontiguousarray(patch, np.uint8).reshape(-1)
        cap = self.n
        out = np.empty(cap, np.int32)
        cnt = lib().orc_riann_candidates(_p(q, C.c_uint8), _p(self.ref, C.c_uint8),
                                         self.n, self.D, _p(self.keys, C.c_int32),
                                         self.K, _p(self.T, C.c_uint32),
                                         _p(self.P, C.c_int32), _p(self.Piv, C.c_uint32),
                                         int(prev), _p(out, C.c_int32), cap)
        if cnt < 0:
            raise ValueError("too many keys for the candidate dump")
        return out[:cnt].copy()
