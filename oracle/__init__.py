"""CPU oracle for the in-place ScatterShuffle definition (version 1).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and ``bench.py``'s ``cpu_baseline`` leg may import it; the product path never
does, and it shares no code with the HIP library.

Two independent renditions of the same definition live here:

* ``css_oracle.c`` (loaded through ctypes) -- used for parity at every size;
* ``spec.py`` -- a pure-Python transcription for small inputs, used to
  cross-check the C rendition.

Paper: M. Penschuck, "Engineering Shared-Memory Parallel Shuffling to Generate
Random Permutations In-Place", arXiv 2302.03317.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "css_oracle.c")
_LIB = os.path.join(_HERE, "libcss_oracle.so")


def build(force: bool = False) -> str:
    """Compile the C oracle into a shared library next to its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-Wall", "-Wextra", "-pthread", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB)
    return _LIB


@dataclass(frozen=True)
class Params:
    """Parameters that are part of the permutation's definition.

    tile: T, the most elements one tile holds; kmax_log2: largest bucket-count
    exponent (1..8); n0: base-case size; lmax: recursion cap."""

    tile: int
    kmax_log2: int = 8
    n0: int = 64
    lmax: int = 32


class _CParams(ctypes.Structure):
    _fields_ = [
        ("tile", ctypes.c_uint64),
        ("kmax_log2", ctypes.c_uint32),
        ("n0", ctypes.c_uint32),
        ("lmax", ctypes.c_uint32),
    ]


class _CRng(ctypes.Structure):
    pass


_LABEL_FN = ctypes.CFUNCTYPE(ctypes.c_uint32, ctypes.POINTER(_CRng), ctypes.c_uint32, ctypes.c_uint64,
                             ctypes.c_uint32)
_DRAW_FN = ctypes.CFUNCTYPE(ctypes.c_uint64, ctypes.POINTER(_CRng), ctypes.c_uint32, ctypes.c_uint64,
                            ctypes.c_uint64)
_CRng._fields_ = [
    ("label", _LABEL_FN),
    ("draw", _DRAW_FN),
    ("seed", ctypes.c_uint64),
    ("stream_id", ctypes.c_uint32),
    ("ctx", ctypes.c_void_p),
]


def _crng(label_fn, draw_fn) -> tuple:
    """A randomness provider whose labels and draws come from Python
    callables label_fn(level, pos, kappa) and draw_fn(level, pos, bound)."""
    lf = _LABEL_FN(lambda _s, level, pos, kappa: int(label_fn(level, pos, kappa)))
    df = _DRAW_FN(lambda _s, level, pos, bound: int(draw_fn(level, pos, bound)))
    return _CRng(lf, df, 0, 0, None), (lf, df)


def _cparams(p: Params) -> _CParams:
    return _CParams(p.tile, p.kmax_log2, p.n0, p.lmax)


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = ctypes.CDLL(path)
        u32, u64, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
        L.css_philox4x32_10.argtypes = [vp, vp, vp]
        L.css_philox4x32_10.restype = None
        L.css_label.argtypes = [u64, u32, u32, u64, u32]
        L.css_label.restype = u32
        L.css_draw.argtypes = [u64, u32, u32, u64, u64]
        L.css_draw.restype = u64
        L.css_lemire_step.argtypes = [u32, u64, ctypes.POINTER(u64)]
        L.css_lemire_step.restype = ctypes.c_int
        L.css_lemire_histogram.argtypes = [u64, vp]
        L.css_lemire_histogram.restype = None
        L.css_lemire16_histogram.argtypes = [u32, vp]
        L.css_lemire16_histogram.restype = None
        L.css_kappa.argtypes = [u64, ctypes.c_int, ctypes.POINTER(_CParams)]
        L.css_kappa.restype = u32
        L.css_check_params.argtypes = [ctypes.POINTER(_CParams)]
        L.css_check_params.restype = ctypes.c_int
        L.css_level.argtypes = [vp, u64, u32, u64, ctypes.c_int, vp]
        L.css_level.restype = ctypes.c_int
        L.css_shuffle.argtypes = [vp, u64, u32, u64, u32, ctypes.POINTER(_CParams)]
        L.css_shuffle.restype = ctypes.c_int
        L.css_shuffle_mt.argtypes = [vp, u64, u32, u64, u32, ctypes.POINTER(_CParams), u32]
        L.css_shuffle_mt.restype = ctypes.c_int
        L.css_shuffle_rng.argtypes = [vp, u64, u32, ctypes.POINTER(_CRng), ctypes.POINTER(_CParams)]
        L.css_shuffle_rng.restype = ctypes.c_int
        L.css_fy_dest.argtypes = [ctypes.POINTER(_CRng), u32, u64, u64, vp]
        L.css_fy_dest.restype = ctypes.c_int
        L.css_fisher_yates.argtypes = [vp, u64, u32, u64, u32]
        L.css_fisher_yates.restype = ctypes.c_int
        L.css_enumerate.argtypes = [u32, ctypes.POINTER(_CParams), vp, ctypes.POINTER(u64)]
        L.css_enumerate.restype = ctypes.c_int
        L.css_perm_histogram.argtypes = [u32, u64, u64, ctypes.POINTER(_CParams), vp]
        L.css_perm_histogram.restype = ctypes.c_int
        L.css_position_histogram.argtypes = [u32, u64, u64, ctypes.POINTER(_CParams), vp]
        L.css_position_histogram.restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def philox4x32_10(ctr, key) -> tuple:
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().css_philox4x32_10(c, k, o)
    return tuple(o)


def label(seed: int, stream_id: int, level: int, pos: int, kappa: int) -> int:
    return lib().css_label(seed, stream_id, level, pos, kappa)


def draw(seed: int, stream_id: int, level: int, pos: int, bound: int) -> int:
    return lib().css_draw(seed, stream_id, level, pos, bound)


def lemire_step(word: int, bound: int):
    out = ctypes.c_uint64()
    ok = lib().css_lemire_step(word, bound, ctypes.byref(out))
    return int(out.value) if ok else None


def lemire_histogram(bound: int) -> np.ndarray:
    counts = np.zeros(bound, dtype=np.uint64)
    lib().css_lemire_histogram(bound, counts.ctypes.data)
    return counts


def lemire16_histogram(bound: int) -> np.ndarray:
    counts = np.zeros(bound, dtype=np.uint64)
    lib().css_lemire16_histogram(bound, counts.ctypes.data)
    return counts


def kappa(m: int, hbm_regime: bool, p: Params) -> int:
    cp = _cparams(p)
    return lib().css_kappa(m, int(hbm_regime), ctypes.byref(cp))


def check_params(p: Params) -> bool:
    cp = _cparams(p)
    return lib().css_check_params(ctypes.byref(cp)) == 0


def level_dest(labels, kappa_: int, tile: int, hbm_regime: bool) -> np.ndarray:
    """Destinations of one IpSc level with the given labels (relative)."""
    lab = np.ascontiguousarray(labels, dtype=np.uint8)
    dest = np.zeros(lab.size, dtype=np.uint64)
    _check(
        lib().css_level(lab.ctypes.data, lab.size, kappa_, tile, int(hbm_regime), dest.ctypes.data),
        "css_level",
    )
    return dest


def shuffle(arr: np.ndarray, seed: int, p: Params, stream_id: int = 0, threads: int = 1) -> np.ndarray:
    """Shuffle a contiguous numpy array in place (element = one row's bytes).

    threads > 1 computes the top level's labels and solves its independent
    buckets on that many host threads; the result does not depend on it."""
    if not arr.flags.c_contiguous:
        raise ValueError("array must be C-contiguous")
    n = arr.shape[0] if arr.ndim else 0
    w = arr.itemsize * (int(np.prod(arr.shape[1:])) if arr.ndim > 1 else 1)
    cp = _cparams(p)
    _check(lib().css_shuffle_mt(arr.ctypes.data, n, w, seed, stream_id, ctypes.byref(cp), max(1, threads)),
           "css_shuffle_mt")
    return arr


def shuffle_scripted(arr: np.ndarray, p: Params, label_fn, draw_fn) -> np.ndarray:
    """The oracle's shuffle with labels and draws supplied by Python callables
    label_fn(level, pos, kappa) and draw_fn(level, pos, bound) (for hand-worked
    examples); in place on a contiguous array."""
    n = arr.shape[0]
    w = arr.itemsize * (int(np.prod(arr.shape[1:])) if arr.ndim > 1 else 1)
    rng, keep = _crng(label_fn, draw_fn)
    cp = _cparams(p)
    _check(lib().css_shuffle_rng(arr.ctypes.data, n, w, ctypes.byref(rng), ctypes.byref(cp)), "css_shuffle_rng")
    del keep
    return arr


def fy_dest_scripted(m: int, level: int, base: int, draw_fn) -> np.ndarray:
    """Fisher-Yates destination map of m items at (level, absolute start
    `base`) with draws from draw_fn(level, pos, bound)."""
    dest = np.zeros(max(m, 1), dtype=np.uint64)
    rng, keep = _crng(lambda *_: 0, draw_fn)
    _check(lib().css_fy_dest(ctypes.byref(rng), level, base, m, dest.ctypes.data), "css_fy_dest")
    del keep
    return dest[:m]


def fisher_yates(arr: np.ndarray, seed: int, stream_id: int = 0) -> np.ndarray:
    """Plain sequential Fisher-Yates with the oracle's level-0 draws."""
    n = arr.shape[0]
    w = arr.itemsize * (int(np.prod(arr.shape[1:])) if arr.ndim > 1 else 1)
    _check(lib().css_fisher_yates(arr.ctypes.data, n, w, seed, stream_id), "css_fisher_yates")
    return arr


def enumerate_outcomes(m: int, p: Params):
    """Exact probability of every permutation of m <= 8 items (lexicographic
    rank order) over all label and draw outcomes, plus the path count."""
    import math

    prob = np.zeros(math.factorial(m), dtype=np.float64)
    paths = ctypes.c_uint64()
    cp = _cparams(p)
    _check(lib().css_enumerate(m, ctypes.byref(cp), prob.ctypes.data, ctypes.byref(paths)), "css_enumerate")
    return prob, int(paths.value)


def perm_histogram(m: int, seed0: int, nseeds: int, p: Params) -> np.ndarray:
    """Counts of each permutation (lexicographic rank) of 0..m-1 over seeds."""
    import math

    counts = np.zeros(math.factorial(m), dtype=np.uint64)
    cp = _cparams(p)
    _check(lib().css_perm_histogram(m, seed0, nseeds, ctypes.byref(cp), counts.ctypes.data), "css_perm_histogram")
    return counts


def position_histogram(n: int, seed0: int, nseeds: int, p: Params) -> np.ndarray:
    """counts[i, j]: how often item i ended at position j over the seeds."""
    counts = np.zeros((n, n), dtype=np.uint64)
    cp = _cparams(p)
    _check(lib().css_position_histogram(n, seed0, nseeds, ctypes.byref(cp), counts.ctypes.data), "css_position_histogram")
    return counts


def params_from_table(path: str, workload: str, elem_bytes: int) -> tuple:
    """(Params, table version) recorded for `workload` at this width in a
    parameter table (JSON written by the library's autotuner).  The oracle
    reads the file itself and takes only the four numbers of the entry; they
    are inputs of the definition like a seed (the permutation is a function
    of them), and check_params must accept them."""
    import json

    with open(path) as fh:
        table = json.load(fh)
    for e in table["entries"]:
        if e["workload"] == workload and int(e["elem_bytes"]) == elem_bytes:
            q = e["params"]
            p = Params(tile=int(q["tile"]), kmax_log2=int(q["kmax_log2"]), n0=int(q["n0"]), lmax=int(q["lmax"]))
            if not check_params(p):
                raise ValueError(f"{path}: parameters of {workload} are outside the definition's ranges")
            return p, int(table["version"])
    raise KeyError(f"{path} has no entry for {workload} at {elem_bytes} bytes")


def default_params(n: int, elem_bytes: int) -> Params:
    """The default parameters for (n, elem_bytes): a 64 KiB tile."""
    tile_bytes = 65536
    return Params(tile=tile_bytes // elem_bytes, kmax_log2=8, n0=64, lmax=32)
