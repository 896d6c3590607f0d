"""In-place parallel ScatterShuffle on one MI355X (gfx950).

A thin ctypes binding over ``libipscshuf.so`` (C ABI declared in
``include/ipscshuf.h``).  Every step of the shuffle runs in the library's HIP
kernels; this module only marshals arguments.  PyTorch is used for device
memory and streams.  There is no CPU fallback: without the built library the
calls raise.

The permutation follows arXiv 2302.03317 (Penschuck): ScatterShuffle with
RoughScatter and a FineScatter-style fix-up, recursing to Fisher-Yates.
"""
from __future__ import annotations

import atexit
import ctypes
import os
from dataclasses import dataclass

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libipscshuf.so")

SHUF_OK = 0
SHUF_EINVAL = -1
SHUF_ENOMEM = -2
SHUF_EHIP = -3
SHUF_EUNSUPPORTED = -4


class ShuffleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} (code {code})")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [
        ("tile", ctypes.c_uint32),
        ("kmax_log2", ctypes.c_uint32),
        ("n0", ctypes.c_uint32),
        ("lmax", ctypes.c_uint32),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("tiled_levels", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("tiles", ctypes.c_uint64),
        ("movers", ctypes.c_uint64),
        ("leaves", ctypes.c_uint64),
        ("fy_fallback", ctypes.c_uint64),
        ("workspace_bytes", ctypes.c_uint64),
    ]


class _KernelTime(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("launches", ctypes.c_uint64), ("bytes", ctypes.c_double)]


class _Array(ctypes.Structure):
    _fields_ = [
        ("ptr", ctypes.c_void_p),
        ("n", ctypes.c_uint64),
        ("seed", ctypes.c_uint64),
        ("stream_id", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


KERNEL_KINDS = ("rough", "tables", "gather", "scatter", "leaf", "fy_fallback")


@dataclass(frozen=True)
class Params:
    """tile: elements per tile; kmax_log2: max bucket-count exponent;
    n0: base-case size; lmax: recursion cap."""

    tile: int
    kmax_log2: int = 8
    n0: int = 64
    lmax: int = 32


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                "(there is no CPU fallback)"
            )
        L = ctypes.CDLL(LIB_PATH)
        u32, u64, vp, i = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
        L.shuffle_definition_version.argtypes = []
        L.shuffle_definition_version.restype = u32
        L.shuffle_rank_method.argtypes = []
        L.shuffle_rank_method.restype = i
        L.shuf_default_params.argtypes = [u64, u32, ctypes.POINTER(_Params)]
        L.shuf_default_params.restype = i
        L.shuffle_inplace.argtypes = [vp, u64, u32, u64, vp]
        L.shuffle_inplace.restype = i
        L.shuffle_inplace_ex.argtypes = [vp, u64, u32, u64, u32, ctypes.POINTER(_Params), vp]
        L.shuffle_inplace_ex.restype = i
        L.shuffle_batched.argtypes = [vp, ctypes.POINTER(u64), u64, u32, u64, vp]
        L.shuffle_batched.restype = i
        L.shuffle_batched_ex.argtypes = [vp, ctypes.POINTER(u64), u64, u32, u64, ctypes.POINTER(_Params), vp]
        L.shuffle_batched_ex.restype = i
        L.shuffle_workspace_bytes.argtypes = [u64, u32, u64, u32, ctypes.POINTER(_Params),
                                              ctypes.POINTER(u64), vp]
        L.shuffle_workspace_bytes.restype = i
        L.shuffle_inplace_ws.argtypes = [vp, u64, u32, u64, u32, ctypes.POINTER(_Params), vp, u64, vp]
        L.shuffle_inplace_ws.restype = i
        L.shuffle_many.argtypes = [ctypes.POINTER(_Array), u64, u32, vp]
        L.shuffle_many.restype = i
        L.shuf_session_create.argtypes = [u32, ctypes.POINTER(vp)]
        L.shuf_session_create.restype = i
        L.shuf_session_submit.argtypes = [vp, ctypes.POINTER(_Array), ctypes.POINTER(u64)]
        L.shuf_session_submit.restype = i
        L.shuf_session_step.argtypes = [vp, vp, ctypes.POINTER(u64), u64, ctypes.POINTER(u64)]
        L.shuf_session_step.restype = i
        L.shuf_session_inflight.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.shuf_session_inflight.restype = i
        L.shuf_session_set_budget.argtypes = [vp, u64]
        L.shuf_session_set_budget.restype = i
        L.shuf_session_queued.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.shuf_session_queued.restype = i
        L.shuf_session_destroy.argtypes = [vp]
        L.shuf_session_destroy.restype = i
        L.shuffle_strerror.argtypes = [i]
        L.shuffle_strerror.restype = ctypes.c_char_p
        L.shuffle_last_stats.argtypes = [ctypes.POINTER(_Stats)]
        L.shuffle_last_stats.restype = i
        L.shuffle_timing_enable.argtypes = [i]
        L.shuffle_timing_enable.restype = i
        L.shuffle_timing_read.argtypes = [ctypes.POINTER(_KernelTime)]
        L.shuffle_timing_read.restype = i
        L.shuffle_inplace_noalloc.argtypes = [vp, u64, u32, u64, u32, ctypes.POINTER(_Params), vp]
        L.shuffle_inplace_noalloc.restype = i
        L.shuffle_batched_async.argtypes = [vp, vp, u64, u32, u64, ctypes.POINTER(_Params), u64, vp, u64, vp]
        L.shuffle_batched_async.restype = i
        L.shuffle_batched_async_workspace_bytes.argtypes = [u64, u64, u32, ctypes.POINTER(_Params),
                                                            ctypes.POINTER(u64)]
        L.shuffle_batched_async_workspace_bytes.restype = i
        L.shuffle_batched_async_max_elems.argtypes = [u32, ctypes.POINTER(_Params)]
        L.shuffle_batched_async_max_elems.restype = u64
        L.shuffle_release.argtypes = []
        L.shuffle_release.restype = i
        _lib = L
        # free the library's pools while the HIP runtime and torch are still up
        atexit.register(release)
    return _lib


def release() -> None:
    """Free the library's device pools, pinned staging and timing events
    (they are allocated again by the next call)."""
    if _lib is not None:
        _lib.shuffle_release()


def strerror(code: int) -> str:
    return lib().shuffle_strerror(code).decode()


def definition_version() -> int:
    return int(lib().shuffle_definition_version())


def rank_method() -> int:
    """1: stable ranks by LDS atomics, 0: by ballots, -1: no call on this device yet."""
    return int(lib().shuffle_rank_method())


def default_params(n: int, elem_bytes: int) -> Params:
    p = _Params()
    rc = lib().shuf_default_params(n, elem_bytes, ctypes.byref(p))
    if rc != SHUF_OK:
        raise ShuffleError(rc, "shuf_default_params")
    return Params(p.tile, p.kmax_log2, p.n0, p.lmax)


def _stream_handle(tensor, stream):
    if stream is not None:
        return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream(tensor.device).cuda_stream)


def _geometry(tensor):
    if not tensor.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not tensor.is_contiguous():
        raise ValueError("tensor must be contiguous")
    n = tensor.shape[0] if tensor.dim() > 0 else 0
    row = 1
    for s in tensor.shape[1:]:
        row *= s
    return n, tensor.element_size() * row


def shuffle_inplace(tensor, seed: int, stream=None) -> None:
    """Shuffle the rows of a contiguous GPU tensor in place (row = one element
    of 4, 8 or 16 bytes), stream id 0, default parameters."""
    n, w = _geometry(tensor)
    rc = lib().shuffle_inplace(
        ctypes.c_void_p(tensor.data_ptr()), n, w, seed & (2**64 - 1), _stream_handle(tensor, stream)
    )
    if rc != SHUF_OK:
        raise ShuffleError(rc, "shuffle_inplace")


def shuffle_inplace_ex(tensor, seed: int, stream_id: int = 0, params: Params | None = None,
                       stream=None) -> None:
    """Shuffle with an explicit stream id and parameters."""
    n, w = _geometry(tensor)
    p = params if params is not None else default_params(n, w)
    cp = _Params(p.tile, p.kmax_log2, p.n0, p.lmax)
    rc = lib().shuffle_inplace_ex(
        ctypes.c_void_p(tensor.data_ptr()), n, w, seed & (2**64 - 1), stream_id, ctypes.byref(cp),
        _stream_handle(tensor, stream),
    )
    if rc != SHUF_OK:
        raise ShuffleError(rc, "shuffle_inplace_ex")


def workspace_bytes(n: int, elem_bytes: int, seed: int, stream_id: int = 0,
                    params: Params | None = None, stream=None) -> int:
    """Exact device workspace shuffle_inplace_ws needs for these arguments."""
    p = params if params is not None else default_params(n, elem_bytes)
    cp = _Params(p.tile, p.kmax_log2, p.n0, p.lmax)
    out = ctypes.c_uint64()
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    sh = ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    rc = lib().shuffle_workspace_bytes(n, elem_bytes, seed & (2**64 - 1), stream_id, ctypes.byref(cp),
                                       ctypes.byref(out), sh)
    if rc != SHUF_OK:
        raise ShuffleError(rc, "shuffle_workspace_bytes")
    return int(out.value)


def shuffle_inplace_ws(tensor, seed: int, workspace, stream_id: int = 0,
                       params: Params | None = None, stream=None) -> None:
    """Shuffle with every per-level device buffer taken from `workspace` (a
    GPU tensor of at least workspace_bytes(...) bytes)."""
    n, w = _geometry(tensor)
    p = params if params is not None else default_params(n, w)
    cp = _Params(p.tile, p.kmax_log2, p.n0, p.lmax)
    wb = workspace.numel() * workspace.element_size()
    rc = lib().shuffle_inplace_ws(
        ctypes.c_void_p(tensor.data_ptr()), n, w, seed & (2**64 - 1), stream_id, ctypes.byref(cp),
        ctypes.c_void_p(workspace.data_ptr()), wb, _stream_handle(tensor, stream),
    )
    if rc != SHUF_OK:
        raise ShuffleError(rc, "shuffle_inplace_ws")


def _cparams_or_null(params: Params | None):
    if params is None:
        return None
    return ctypes.byref(_Params(params.tile, params.kmax_log2, params.n0, params.lmax))


def batched_async_workspace_bytes(count: int, total_elems: int, elem_bytes: int,
                                  params: Params | None = None) -> int:
    out = ctypes.c_uint64()
    rc = lib().shuffle_batched_async_workspace_bytes(count, total_elems, elem_bytes, _cparams_or_null(params),
                                                     ctypes.byref(out))
    if rc != SHUF_OK:
        raise ShuffleError(rc, "shuffle_batched_async_workspace_bytes")
    return int(out.value)


def batched_async_max_elems(elem_bytes: int, params: Params | None = None) -> int:
    return int(lib().shuffle_batched_async_max_elems(elem_bytes, _cparams_or_null(params)))


def shuffle_batched_async(tensor, offsets, seed: int, workspace, total_elems: int | None = None,
                          stream=None, params: Params | None = None) -> None:
    """Enqueue the batched shuffle of `tensor` (rows [offsets[j], offsets[j+1])
    form array j) on the stream without synchronising: `offsets` is a device
    int64 tensor of count + 1 entries, `workspace` a device tensor of at least
    batched_async_workspace_bytes(..., params) bytes whose first int32 reads 0
    after the stream has completed if the device found no error.  `params`
    (default: the defaults) apply to every array."""
    n, w = _geometry(tensor)
    count = offsets.numel() - 1
    total = n if total_elems is None else int(total_elems)
    wb = workspace.numel() * workspace.element_size()
    rc = lib().shuffle_batched_async(
        ctypes.c_void_p(tensor.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), count, w, seed & (2**64 - 1),
        _cparams_or_null(params), total, ctypes.c_void_p(workspace.data_ptr()), wb,
        _stream_handle(tensor, stream),
    )
    if rc != SHUF_OK:
        raise ShuffleError(rc, "shuffle_batched_async")


def shuffle_inplace_noalloc(tensor, seed: int, stream_id: int = 0, params: Params | None = None,
                            stream=None) -> None:
    """shuffle_inplace_ex without any device allocation: every buffer comes
    from the library's static device array (arrays up to 48 MiB)."""
    n, w = _geometry(tensor)
    p = params if params is not None else default_params(n, w)
    cp = _Params(p.tile, p.kmax_log2, p.n0, p.lmax)
    rc = lib().shuffle_inplace_noalloc(
        ctypes.c_void_p(tensor.data_ptr()), n, w, seed & (2**64 - 1), stream_id, ctypes.byref(cp),
        _stream_handle(tensor, stream),
    )
    if rc != SHUF_OK:
        raise ShuffleError(rc, "shuffle_inplace_noalloc")


def shuffle_batched(tensor, offsets, seed: int, stream=None, params: Params | None = None) -> None:
    """Shuffle the arrays packed in `tensor` (rows [offsets[j], offsets[j+1])
    form array j) in place, each with stream id j and `params` (default: the
    defaults)."""
    n, w = _geometry(tensor)
    offs = [int(o) for o in offsets]
    if len(offs) < 1 or offs[-1] > n:
        raise ValueError("offsets must end within the tensor")
    arr = (ctypes.c_uint64 * len(offs))(*offs)
    rc = lib().shuffle_batched_ex(
        ctypes.c_void_p(tensor.data_ptr()), arr, len(offs) - 1, w, seed & (2**64 - 1),
        _cparams_or_null(params), _stream_handle(tensor, stream),
    )
    if rc != SHUF_OK:
        raise ShuffleError(rc, "shuffle_batched")


def _array(tensor, seed: int, stream_id: int) -> _Array:
    n, w = _geometry(tensor)
    return _Array(ctypes.c_void_p(tensor.data_ptr()), n, seed & (2**64 - 1), stream_id & (2**32 - 1), 0), w


def shuffle_many(tensors, seeds, stream_ids, stream=None) -> None:
    """Shuffle several GPU tensors (same row width, any allocations) in place,
    tensor j with seeds[j] and stream_ids[j] and default parameters, all in
    shared launches."""
    tensors = list(tensors)
    if not tensors:
        return
    arrs = []
    width = None
    for t, sd, sid in zip(tensors, seeds, stream_ids, strict=True):
        a, w = _array(t, sd, sid)
        if width is None:
            width = w
        elif w != width:
            raise ValueError("all tensors must have the same row width")
        arrs.append(a)
    buf = (_Array * len(arrs))(*arrs)
    rc = lib().shuffle_many(buf, len(arrs), width, _stream_handle(tensors[0], stream))
    if rc != SHUF_OK:
        raise ShuffleError(rc, "shuffle_many")


class Session:
    """Continuous batching: submit(tensor, seed, stream_id) queues a request;
    step() advances every request in flight by one recursion level (new
    requests join at the next step) and returns the tickets completed."""

    def __init__(self, elem_bytes: int, device=None):
        import torch

        self._torch = torch
        self.elem_bytes = elem_bytes
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib().shuf_session_create(elem_bytes, ctypes.byref(h))
        if rc != SHUF_OK:
            raise ShuffleError(rc, "shuf_session_create")
        self._h = h
        self._keep = {}  # ticket -> tensor, kept alive while in flight

    def submit(self, tensor, seed: int, stream_id: int = 0) -> int:
        a, w = _array(tensor, seed, stream_id)
        if w != self.elem_bytes:
            raise ValueError(f"row width {w} != session width {self.elem_bytes}")
        t = ctypes.c_uint64()
        rc = lib().shuf_session_submit(self._h, ctypes.byref(a), ctypes.byref(t))
        if rc != SHUF_OK:
            raise ShuffleError(rc, "shuf_session_submit")
        self._keep[int(t.value)] = tensor
        return int(t.value)

    def step(self, stream=None, cap: int = 4096) -> list:
        done = (ctypes.c_uint64 * cap)()
        nd = ctypes.c_uint64()
        if stream is None:
            stream = self._torch.cuda.current_stream(self.device)
        sh = ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        with self._torch.cuda.device(self.device):
            rc = lib().shuf_session_step(self._h, sh, done, cap, ctypes.byref(nd))
        if rc != SHUF_OK:
            raise ShuffleError(rc, "shuf_session_step")
        out = [int(done[i]) for i in range(nd.value)]
        for t in out:
            self._keep.pop(t, None)
        return out

    def set_budget(self, nbytes: int) -> None:
        """Admit requests only while the admitted ones' charges (data plus the
        library's workspace for each) fit `nbytes` (0: no limit)."""
        rc = lib().shuf_session_set_budget(self._h, int(nbytes))
        if rc != SHUF_OK:
            raise ShuffleError(rc, "shuf_session_set_budget")

    def queued(self) -> tuple:
        """(requests waiting for admission, bytes charged to admitted ones)."""
        q, u = ctypes.c_uint64(), ctypes.c_uint64()
        rc = lib().shuf_session_queued(self._h, ctypes.byref(q), ctypes.byref(u))
        if rc != SHUF_OK:
            raise ShuffleError(rc, "shuf_session_queued")
        return int(q.value), int(u.value)

    def inflight(self) -> tuple:
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        rc = lib().shuf_session_inflight(self._h, ctypes.byref(a), ctypes.byref(b))
        if rc != SHUF_OK:
            raise ShuffleError(rc, "shuf_session_inflight")
        return int(a.value), int(b.value)

    def close(self) -> None:
        if self._h:
            with self._torch.cuda.device(self.device):
                lib().shuf_session_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def last_stats() -> dict:
    s = _Stats()
    rc = lib().shuffle_last_stats(ctypes.byref(s))
    if rc != SHUF_OK:
        raise ShuffleError(rc, "shuffle_last_stats")
    return {f: int(getattr(s, f)) for f, _ in _Stats._fields_ if f != "reserved"}


def timing_enable(on: bool = True) -> None:
    """Start (and clear) or stop per-kernel HIP-event timing on the current device."""
    rc = lib().shuffle_timing_enable(1 if on else 0)
    if rc != SHUF_OK:
        raise ShuffleError(rc, "shuffle_timing_enable")


def timing_read() -> dict:
    """{kind: {"ms", "launches", "bytes"}} accumulated since timing_enable()."""
    arr = (_KernelTime * len(KERNEL_KINDS))()
    rc = lib().shuffle_timing_read(arr)
    if rc != SHUF_OK:
        raise ShuffleError(rc, "shuffle_timing_read")
    return {k: {"ms": arr[i].ms, "launches": int(arr[i].launches), "bytes": arr[i].bytes}
            for i, k in enumerate(KERNEL_KINDS)}


def raw_call(name: str, *args) -> int:
    """Call a C entry point with raw arguments (for argument-error tests)."""
    return getattr(lib(), name)(*args)
