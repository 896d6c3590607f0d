"""CPU-side checks of the C ABI library: it loads, exports every function the
header declares, and its host-only functions behave (no GPU work)."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ipscshuf.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_][a-z_0-9]*)\s*\(", text, flags=re.M)))


def _lib():
    import paper_2302_03317_amd as shuf

    if not os.path.exists(shuf.LIB_PATH):
        pytest.skip("library not built")
    return shuf


def test_header_declares_entry_points():
    names = _declared_functions()
    for n in ["shuffle_inplace", "shuffle_inplace_ex", "shuffle_batched", "shuf_default_params",
              "shuffle_strerror", "shuffle_definition_version", "shuffle_last_stats"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    shuf = _lib()
    lib = ctypes.CDLL(shuf.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_host_only_functions():
    shuf = _lib()
    assert shuf.definition_version() == 1
    assert shuf.strerror(0) == "success"
    assert "unsupported" in shuf.strerror(-4)
    for w in (4, 8, 16):
        p = shuf.default_params(1 << 20, w)
        # the defaults are part of the definition; the oracle writes them down independently
        q = oracle.default_params(1 << 20, w)
        assert (p.tile, p.kmax_log2, p.n0, p.lmax) == (q.tile, q.kmax_log2, q.n0, q.lmax)
    with pytest.raises(shuf.ShuffleError):
        shuf.default_params(10, 3)


def test_invalid_arguments_rejected_without_gpu():
    """Argument checks run before any HIP call, so they work on a CPU host."""
    shuf = _lib()
    null = ctypes.c_void_p(0)
    assert shuf.raw_call("shuffle_inplace", null, 10, 4, 1, null) == shuf.SHUF_EINVAL
    assert shuf.raw_call("shuffle_inplace", null, 10, 5, 1, null) == shuf.SHUF_EINVAL
    assert shuf.raw_call("shuffle_inplace", null, 1, 4, 1, null) == 0
    p = shuf._Params(3, 2, 1, 1)
    assert shuf.raw_call("shuffle_inplace_ex", null, 10, 4, 1, 0, ctypes.byref(p), null) == shuf.SHUF_EINVAL
    offs = (ctypes.c_uint64 * 3)(0, 5, 4)
    assert shuf.raw_call("shuffle_batched", null, offs, 2, 4, 1, null) == shuf.SHUF_EINVAL


def test_multi_array_and_session_argument_checks_without_gpu():
    """shuffle_many and the session calls validate arguments before any HIP call."""
    shuf = _lib()
    lib = shuf.lib()
    null = ctypes.c_void_p(0)
    assert lib.shuffle_many(None, 3, 4, null) == shuf.SHUF_EINVAL
    assert lib.shuffle_many(None, 0, 5, null) == shuf.SHUF_EINVAL
    bad = (shuf._Array * 2)(shuf._Array(None, 10, 1, 0, 0), shuf._Array(None, 1, 1, 1, 0))
    assert lib.shuffle_many(bad, 2, 4, null) == shuf.SHUF_EINVAL       # NULL ptr with n > 1
    odd = (shuf._Array * 1)(shuf._Array(ctypes.c_void_p(0x1002), 10, 1, 0, 0))
    assert lib.shuffle_many(odd, 1, 4, null) == shuf.SHUF_EINVAL       # misaligned
    big = (shuf._Array * 1)(shuf._Array(ctypes.c_void_p(0x1000), 1 << 41, 1, 0, 0))
    assert lib.shuffle_many(big, 1, 4, null) == shuf.SHUF_EUNSUPPORTED
    trivial = (shuf._Array * 2)(shuf._Array(None, 0, 1, 0, 0), shuf._Array(None, 1, 1, 1, 0))
    assert lib.shuffle_many(trivial, 2, 8, null) == 0                  # nothing to do
    t = ctypes.c_uint64()
    a = shuf._Array(null, 10, 1, 0, 0)
    assert lib.shuf_session_submit(None, ctypes.byref(a), ctypes.byref(t)) == shuf.SHUF_EINVAL
    nd = ctypes.c_uint64()
    assert lib.shuf_session_step(None, null, None, 0, ctypes.byref(nd)) == shuf.SHUF_EINVAL
    assert lib.shuf_session_inflight(None, ctypes.byref(nd), None) == shuf.SHUF_EINVAL
    assert lib.shuf_session_create(3, None) == shuf.SHUF_EINVAL
    assert lib.shuf_session_destroy(None) == shuf.SHUF_EINVAL


def test_workspace_calls_argument_checks_without_gpu():
    shuf = _lib()
    lib = shuf.lib()
    null = ctypes.c_void_p(0)
    p = shuf._Params(16384, 8, 64, 32)
    out = ctypes.c_uint64(123)
    assert lib.shuffle_workspace_bytes(1000, 4, 1, 0, ctypes.byref(p), None, null) == shuf.SHUF_EINVAL
    assert lib.shuffle_workspace_bytes(1000, 3, 1, 0, ctypes.byref(p), ctypes.byref(out), null) == shuf.SHUF_EINVAL
    assert lib.shuffle_workspace_bytes(1000, 4, 1, 0, None, ctypes.byref(out), null) == shuf.SHUF_EINVAL
    assert lib.shuffle_workspace_bytes(1, 4, 1, 0, ctypes.byref(p), ctypes.byref(out), null) == 0
    assert out.value == 0
    ptr = ctypes.c_void_p(0x10000)
    ws = ctypes.c_void_p(0x20000)
    assert lib.shuffle_inplace_ws(ptr, 1000, 4, 1, 0, ctypes.byref(p), ctypes.c_void_p(0x20010), 4096, null) == shuf.SHUF_EINVAL
    assert lib.shuffle_inplace_ws(ptr, 1000, 4, 1, 0, ctypes.byref(p), null, 4096, null) == shuf.SHUF_EINVAL
    assert lib.shuffle_inplace_ws(ctypes.c_void_p(0x10002), 1000, 4, 1, 0, ctypes.byref(p), ws, 4096, null) == shuf.SHUF_EINVAL
    assert lib.shuffle_inplace_ws(null, 1, 4, 1, 0, ctypes.byref(p), null, 0, null) == 0
