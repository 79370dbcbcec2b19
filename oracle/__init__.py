"""CPU oracle for the KNN filtering stage -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and its
binding in ``paper_2404_10631_amd``) never imports it, and it imports nothing
from there.

The arithmetic lives in ``knn_oracle.c`` (plain C, built with
``gcc -O2 -ffp-contract=off -fopenmp``); this module only marshals numpy arrays.
What it computes follows Sec. II.C.3 of the paper (Eq. 1 distance, Eq. 2
averaging, argmax class map) with the search window of Sec. III.A.3; the exact
binary32 evaluation order is stated at the top of ``knn_oracle.c``.

Every function here is pinned by ``tests/test_oracle_pins.py`` (lattice cases,
exact dyadic cases, the lambda = 0 library-sort reduction, K = 1 identity, the
R = 0 row-mean closed form, error bounds against exact arithmetic).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knn_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libknn_oracle.so")

ORC_OK = 0
ORC_EINVAL = -1
ORC_ENOMEM = -2

_lib = None


class OracleError(RuntimeError):
    """Raised when the oracle rejects its arguments."""

    def __init__(self, status: int):
        super().__init__(f"knn oracle returned status {status}")
        self.status = status


def build(force: bool = True) -> str:
    """Compile ``knn_oracle.c`` into ``libknn_oracle.so`` next to it."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = [
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra",
            "-o", _LIB_PATH + ".tmp", _SRC, "-lm",
        ]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    fp = ctypes.POINTER(ctypes.c_float)
    ip = ctypes.POINTER(ctypes.c_int32)
    c_int, c_float = ctypes.c_int, ctypes.c_float
    lib.knn_oracle_filter.restype = c_int
    lib.knn_oracle_filter.argtypes = [c_int, c_int, c_int, c_int, c_int, c_float,
                                      fp, fp, fp, ip, ip, fp, c_int]
    lib.knn_oracle_pixels.restype = c_int
    lib.knn_oracle_pixels.argtypes = [c_int, c_int, c_int, c_int, c_int, c_float,
                                      fp, fp, ip, c_int, fp, ip, ip, fp, c_int]
    lib.knn_oracle_max_threads.restype = c_int
    lib.knn_oracle_max_threads.argtypes = []
    _lib = lib
    return lib


def _fptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _iptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def max_threads() -> int:
    return int(_load().knn_oracle_max_threads())


def _prep(pc1, prob):
    pc1 = np.ascontiguousarray(pc1, dtype=np.float32)
    prob = np.ascontiguousarray(prob, dtype=np.float32)
    if pc1.ndim != 2 or prob.ndim != 3 or prob.shape[:2] != pc1.shape:
        raise ValueError("pc1 must be (H, W) and prob (H, W, C)")
    return pc1, prob


def knn_filter(pc1, prob, K: int, R: int, lam: float, with_nbr: bool = True,
               nthreads: int | None = None):
    """Whole-frame oracle.

    Returns (out_prob (H,W,C) f32, out_class (H,W) i32, nbr (H,W,K) i32 or None,
    dist (H,W,K) f32 or None).
    """
    pc1, prob = _prep(pc1, prob)
    H, W = pc1.shape
    C = prob.shape[2]
    out_prob = np.empty((H, W, C), np.float32)
    out_class = np.empty((H, W), np.int32)
    nbr = np.empty((H, W, K), np.int32) if with_nbr and K > 0 else None
    dist = np.empty((H, W, K), np.float32) if with_nbr and K > 0 else None
    nt = max_threads() if nthreads is None else int(nthreads)
    st = _load().knn_oracle_filter(H, W, C, int(K), int(R), float(np.float32(lam)),
                                   _fptr(pc1), _fptr(prob), _fptr(out_prob),
                                   _iptr(out_class), _iptr(nbr), _fptr(dist), nt)
    if st != ORC_OK:
        raise OracleError(st)
    return out_prob, out_class, nbr, dist


def knn_pixels(pc1, prob, K: int, R: int, lam: float, pix, with_nbr: bool = True,
               nthreads: int | None = None):
    """Oracle for the listed pixels only (linear indices r*W + c).

    Returns (out_prob (n,C), out_class (n,), nbr (n,K) or None, dist (n,K) or None).
    """
    pc1, prob = _prep(pc1, prob)
    H, W = pc1.shape
    C = prob.shape[2]
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1)
    n = pix.shape[0]
    out_prob = np.empty((n, C), np.float32)
    out_class = np.empty((n,), np.int32)
    nbr = np.empty((n, K), np.int32) if with_nbr and K > 0 else None
    dist = np.empty((n, K), np.float32) if with_nbr and K > 0 else None
    nt = max_threads() if nthreads is None else int(nthreads)
    st = _load().knn_oracle_pixels(H, W, C, int(K), int(R), float(np.float32(lam)),
                                   _fptr(pc1), _fptr(prob), _iptr(pix), n,
                                   _fptr(out_prob), _iptr(out_class), _iptr(nbr),
                                   _fptr(dist), nt)
    if st != ORC_OK:
        raise OracleError(st)
    return out_prob, out_class, nbr, dist
