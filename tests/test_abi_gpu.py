"""Error conventions of the C-ABI on the GPU, with every condition forced
from the host (nothing faults): an allocator that runs out part-way through
net_build and net_mlp_create (NET_E_OOM, no handle, every block handed back),
and a handle marked as after a device fault (NET_E_STATE on every later
call)."""
import ctypes as C

import numpy as np
import pytest

import synth
from paper_0908_3934_amd import _abi

pytestmark = pytest.mark.gpu


class FailingAllocator:
    """Device allocator (PyTorch's caching allocator underneath) that returns
    NULL from the `fail_at`-th call on, counting what it hands out and gets
    back."""

    def __init__(self, fail_at):
        import torch
        self.torch = torch
        self.fail_at = fail_at
        self.calls = 0
        self.live = {}
        self.released = 0
        self.alloc_cb = _abi.ALLOC_FN(self._alloc)
        self.release_cb = _abi.RELEASE_FN(self._release)

    def _alloc(self, nbytes, stream, ctx):
        self.calls += 1
        if self.calls > self.fail_at:
            return None
        p = self.torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        self.live[int(p)] = int(nbytes)
        return p

    def _release(self, ptr, stream, ctx):
        self.live.pop(int(ptr))
        self.released += 1
        self.torch.cuda.caching_allocator_delete(int(ptr))


@pytest.fixture
def lib():
    import torch
    import paper_0908_3934_amd as gn
    assert torch.cuda.is_available()
    L = gn.library()
    yield L
    # restore the binding's allocator (or hipMalloc when none was registered)
    if gn._alloc_cb is not None:
        L.net_set_allocator(gn._alloc_cb, gn._release_cb, None)
    else:
        L.net_set_allocator(C.cast(None, _abi.ALLOC_FN), C.cast(None, _abi.RELEASE_FN), None)


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
    d.v_th, d.n_ref, d.frame_num, d.frame_den = 1.0, 20, 3, 1000
    d.noise_sigma, d.seed, d.tau_c_ms = 0.05, 7, 500.0
    return d


def _build_with(lib, fa, spec, frame_capacity=16):
    keep = []
    assert lib.net_set_allocator(fa.alloc_cb, fa.release_cb, None) == _abi.NET_OK
    opts = _abi.BuildOpts()
    opts.frame_capacity = frame_capacity
    h = C.c_void_p(12345)
    st = lib.net_build((_abi.NetDesc * 1)(_desc(spec, keep)), 1, C.byref(opts), None, C.byref(h))
    return st, h


def test_build_out_of_memory_at_every_allocation(lib):
    """Count the allocations of a successful build, then make each one of
    them fail in turn: NET_E_OOM, no handle, every earlier block released."""
    import torch
    spec = synth.config0_like(300, 5)
    ok = FailingAllocator(10 ** 6)
    st, h = _build_with(lib, ok, spec)
    assert st == _abi.NET_OK and h.value
    n = ok.calls
    assert n >= 8
    assert lib.net_step_n(h, 50, None, None) == _abi.NET_OK
    torch.cuda.synchronize()
    lib.net_free(h)
    assert not ok.live and ok.released == n
    for fail_at in range(n):
        fa = FailingAllocator(fail_at)
        st, h = _build_with(lib, fa, spec)
        torch.cuda.synchronize()
        assert st == _abi.NET_E_OOM, (fail_at, st, lib.net_last_error())
        assert b"allocation failed" in lib.net_last_error()
        assert not h.value
        assert fa.calls == fail_at + 1
        assert not fa.live and fa.released == fail_at        # every block handed back


def test_mlp_create_out_of_memory_at_every_allocation(lib):
    ok = FailingAllocator(10 ** 6)
    assert lib.net_set_allocator(ok.alloc_cb, ok.release_cb, None) == _abi.NET_OK
    h = C.c_void_p()
    assert lib.net_mlp_create(C.byref(h)) == _abi.NET_OK and h.value
    n = ok.calls
    lib.net_mlp_free(h)
    assert n >= 10 and not ok.live and ok.released == n
    for fail_at in range(n):
        fa = FailingAllocator(fail_at)
        assert lib.net_set_allocator(fa.alloc_cb, fa.release_cb, None) == _abi.NET_OK
        h = C.c_void_p(777)
        st = lib.net_mlp_create(C.byref(h))
        assert st == _abi.NET_E_OOM and not h.value
        assert fa.calls == fail_at + 1
        assert not fa.live and fa.released == fail_at


def test_state_error_after_device_fault(lib):
    import torch
    keep = []
    h = C.c_void_p()
    assert lib.net_build((_abi.NetDesc * 1)(_desc(synth.config0_like(100, 3), keep)), 1, None, None,
                         C.byref(h)) == _abi.NET_OK
    assert lib.net_step_n(h, 10, None, None) == _abi.NET_OK
    assert lib.net_simulate_device_error(h) == _abi.NET_OK
    assert lib.net_step_n(h, 10, None, None) == _abi.NET_E_STATE
    assert b"unusable" in lib.net_last_error()
    out = torch.zeros(100, device="cuda")
    assert lib.net_observe(h, 1, None, out.data_ptr(), 400, None) == _abi.NET_E_STATE
    assert lib.net_timing_begin(h, 4, 1) == _abi.NET_E_STATE
    info = _abi.Info()
    assert lib.net_info(h, C.byref(info)) == _abi.NET_OK          # still answers, still frees
    lib.net_free(h)
    assert lib.net_simulate_device_error(None) == _abi.NET_E_ARG


def test_autotune_cache_reuses_shape():
    """A second autotuned build of the same ensemble in this process takes the
    shape the first one chose (the process keeps its tuning results), and
    steps to the same bits."""
    import torch
    import time
    import paper_0908_3934_amd as gn
    specs = [synth.config0_like(n, synth.config_seed(3, 970 + k), w0=0.36) for k, n in enumerate([100, 260, 70])]
    for s in specs:
        s.noise_sigma = 0.05
    t0 = time.perf_counter()
    a = gn.Net(specs, flags=gn.NET_BUILD_AUTOTUNE)
    t1 = time.perf_counter()
    b = gn.Net(specs, flags=gn.NET_BUILD_AUTOTUNE)
    t2 = time.perf_counter()
    ia, ib = a.info(), b.info()
    print("autotuned builds: %.3f s then %.3f s; shape %d x %d" % (t1 - t0, t2 - t1, ia["ensemble_blocks"],
                                                                   ia["ensemble_threads"]), flush=True)
    assert ia["autotuned"] == ib["autotuned"] == 1
    assert (ia["ensemble_blocks"], ia["ensemble_threads"]) == (ib["ensemble_blocks"], ib["ensemble_threads"])
    ra = a.step(500, raster=True)
    rb = b.step(500, raster=True)
    torch.cuda.synchronize()
    assert torch.equal(ra["raster"], rb["raster"])
    a.close()
    b.close()
