"""Host PIpScShuf: the paper's parallel in-place shuffle on the host's CPU
cores (C++ with OpenMP tasks), a same-machine CPU baseline for the GPU
library.  It follows arXiv 2302.03317 Sec. 3-5 (RoughScatter, FineScatter
with TwoSweep, parallel RoughScatter by binary fork-join, k = 64 / 256, a
Fisher-Yates base case of 2^18 items) with its own generator (a 128-bit MCG
with PCG's XSL-RR output).  Its permutations are uniform but are not the GPU
library's: the GPU library never calls this code and this code never stands
in for it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pipscshuf.cpp")
_LIB = os.path.join(_HERE, "libpipscshuf.so")


def build(force: bool = False) -> str:
    """Compile the library next to its source (g++, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        u32, u64, vp, i = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
        L.pipscshuf_shuffle_ex.argtypes = [vp, u64, u32, u64, i, u32, u32, u64, u64]
        L.pipscshuf_shuffle_ex.restype = i
        L.pipscshuf_fisher_yates.argtypes = [vp, u64, u32, u64]
        L.pipscshuf_fisher_yates.restype = i
        _lib = L
    return _lib


def _geometry(arr: np.ndarray):
    if not arr.flags.c_contiguous:
        raise ValueError("array must be C-contiguous")
    n = arr.shape[0]
    w = arr.itemsize * (int(np.prod(arr.shape[1:])) if arr.ndim > 1 else 1)
    return n, w


def shuffle(arr: np.ndarray, seed: int, threads: int = 0, kappa_small: int = 0, kappa_large: int = 0,
            base_case: int = 0, par_cutoff: int = 0) -> np.ndarray:
    """Shuffle in place on `threads` host threads (0: all).  The keyword
    parameters override the paper's settings (0 keeps them) for tests."""
    n, w = _geometry(arr)
    rc = lib().pipscshuf_shuffle_ex(arr.ctypes.data, n, w, seed & (2**64 - 1), threads, kappa_small,
                                    kappa_large, base_case, par_cutoff)
    if rc != 0:
        raise ValueError(f"pipscshuf_shuffle_ex failed ({rc})")
    return arr


def fisher_yates(arr: np.ndarray, seed: int) -> np.ndarray:
    """Sequential Fisher-Yates with the same generator (one thread)."""
    n, w = _geometry(arr)
    rc = lib().pipscshuf_fisher_yates(arr.ctypes.data, n, w, seed & (2**64 - 1))
    if rc != 0:
        raise ValueError(f"pipscshuf_fisher_yates failed ({rc})")
    return arr
