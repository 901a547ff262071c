"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/geonet.h, and rejects bad input on the host
before touching a device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import synth
from paper_0908_3934_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "geonet.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:net_status|void|size_t|const char\s*\*)\s*(net_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libgeonet.so not built")
    return _abi.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("net_build", "net_step_n", "net_observe", "net_free", "net_last_error", "net_set_allocator"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.check_output(["nm", "-D", "--defined-only", _abi.LIB_PATH]).decode()
    exported = set(re.findall(r" T (net_\w+)$", out, re.M))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        assert getattr(lib, n) is not None
    # the Python binding declares exactly the header's functions
    assert set(_abi.SIGNATURES) == set(declared_functions())


def _desc(spec, keep):
    d = _abi.NetDesc()

    def arr(x, dt):
        a = np.ascontiguousarray(x, dtype=dt)
        keep.append(a)
        return a.ctypes.data

    d.n_nodes, d.dims = spec.n, spec.dims
    d.pos_um = arr(spec.pos_um, np.float64)
    d.n_edges = spec.n_edges
    d.src, d.dst = arr(spec.src, np.int32), arr(spec.dst, np.int32)
    d.weight = arr(spec.weight, np.float32)
    d.v_um_per_ms, d.dt_ms, d.tau_ms = spec.v_um_per_ms, spec.dt_ms, spec.tau_ms
    d.v_th, d.n_ref, d.frame_den = 1.0, 20, 1000
    return d


def _build(lib, descs, n=None):
    h = C.c_void_p()
    arr = (_abi.NetDesc * len(descs))(*descs)
    st = lib.net_build(arr, len(descs) if n is None else n, None, None, C.byref(h))
    return st, h


def test_host_side_rejections(lib):
    keep = []
    base = synth.config0_like(64, 1)
    st, h = _build(lib, [_desc(base, keep)], n=0)
    assert st == _abi.NET_E_ARG and not h.value
    assert b"n_nets" in lib.net_last_error()

    bad = synth.config0_like(64, 1)
    bad.src = bad.src.copy()
    bad.src[0] = bad.dst[0]                        # self-loop
    st, h = _build(lib, [_desc(bad, keep)])
    assert st == _abi.NET_E_ARG and b"self-loop" in lib.net_last_error()

    oob = synth.config0_like(64, 1)
    oob.dst = oob.dst.copy()
    oob.dst[3] = 64
    st, h = _build(lib, [_desc(oob, keep)])
    assert st == _abi.NET_E_ARG and b"out of range" in lib.net_last_error()

    far = synth.NetSpec(name="far", pos_um=np.array([[0.0, 0.0], [2600.0, 0.0]]), src=np.array([0], np.int32),
                        dst=np.array([1], np.int32), weight=np.array([0.5], np.float32))
    st, h = _build(lib, [_desc(far, keep)])
    assert st == _abi.NET_E_RANGE and b"255" in lib.net_last_error()

    dup = synth.NetSpec(name="dup", pos_um=np.zeros((3, 2)), src=np.array([0, 0], np.int32),
                        dst=np.array([1, 1], np.int32), weight=np.array([0.5, 0.5], np.float32))
    st, h = _build(lib, [_desc(dup, keep)])
    assert st == _abi.NET_E_ARG and b"duplicate" in lib.net_last_error()

    d0, d1 = _desc(base, keep), _desc(base, keep)
    d1.dt_ms = 0.2
    st, h = _build(lib, [d0, d1])
    assert st == _abi.NET_E_ARG and b"dt" in lib.net_last_error()


def test_null_handles(lib):
    assert lib.net_step_n(None, 1, None, None) == _abi.NET_E_ARG
    assert lib.net_observe(None, 1, None, None, 0, None) == _abi.NET_E_ARG
    info = _abi.Info()
    assert lib.net_info(None, C.byref(info)) == _abi.NET_E_ARG
    lib.net_free(None)
    st = lib.net_set_allocator(_abi.ALLOC_FN(lambda n, s, c: None), C.cast(None, _abi.RELEASE_FN), None)
    assert st == _abi.NET_E_ARG
    assert lib.net_build(None, 1, None, None, None) == _abi.NET_E_ARG
