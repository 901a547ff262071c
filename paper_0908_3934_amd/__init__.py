"""geonet on MI355X: Python binding of the C-ABI library (include/geonet.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of ``libgeonet.so``; PyTorch supplies device memory (its caching
allocator is registered with the library) and streams.  The binding fails
loudly when the library is missing -- there is no CPU fallback.

Networks are described by objects with the attributes of ``synth.NetSpec``
(positions, src/dst/weight arrays, model constants).
"""
from __future__ import annotations

import ctypes as C
from typing import Iterable, List, Optional, Sequence

import numpy as np

from . import _abi
from ._abi import (NET_BUILD_AUTOTUNE, NET_BUILD_DELIVER_NONTEMPORAL, NET_BUILD_DELIVER_PIPELINE,
                   NET_BUILD_DELIVER_STREAM_WEIGHTS, NET_BUILD_SUMMARY_HALF, NET_BUILD_DELIVER_COMPACT, NET_BUILD_FUSED_STEP,
                   NET_BUILD_DELIVER_PACKED, NET_BUILD_REORDER, NET_BUILD_GRAPH, NET_BUILD_PUSH,
                   NET_BUILD_DELIVER_UNROLL2, NET_BUILD_NO_LDS_SUMMARY, NET_BUILD_PER_STEP, NET_BUILD_SINGLE_LAUNCH,
                   NET_OBS_CALCIUM, NET_OBS_FLUOR, NET_OBS_FRAMES, NET_OBS_REF, NET_OBS_WEIGHTS,
                   NET_OBS_V, NET_OK, NET_W_INEXACT)

__all__ = ["Net", "Mlp", "GeonetError", "NET_OBS_V", "NET_OBS_REF", "NET_OBS_CALCIUM", "NET_OBS_FRAMES",
           "NET_OBS_FLUOR", "NET_OBS_WEIGHTS", "NET_BUILD_NO_LDS_SUMMARY", "NET_BUILD_DELIVER_STREAM_WEIGHTS",
           "NET_BUILD_DELIVER_NONTEMPORAL", "NET_BUILD_DELIVER_UNROLL2", "NET_BUILD_PER_STEP",
           "NET_BUILD_SINGLE_LAUNCH", "NET_BUILD_AUTOTUNE", "NET_BUILD_DELIVER_PIPELINE",
           "NET_BUILD_SUMMARY_HALF", "NET_BUILD_DELIVER_COMPACT", "NET_BUILD_FUSED_STEP", "NET_BUILD_DELIVER_PACKED",
           "NET_BUILD_REORDER", "NET_BUILD_GRAPH", "NET_BUILD_PUSH",
           "library"]


class GeonetError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__("%s failed (status %d): %s" % (where, status, msg))
        self.status = status


def library():
    return _abi.load()


def _check(st: int, where: str):
    if st != NET_OK and st != NET_W_INEXACT:
        raise GeonetError(st, where, library().net_last_error().decode())
    return st


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# PyTorch caching allocator as the library's device allocator.
_alloc_cb = None
_release_cb = None


def _register_torch_allocator():
    global _alloc_cb, _release_cb
    if _alloc_cb is not None:
        return
    import torch

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:
            return None

    def _release(ptr, stream, ctx):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    _alloc_cb = _abi.ALLOC_FN(_alloc)
    _release_cb = _abi.RELEASE_FN(_release)
    _check(library().net_set_allocator(_alloc_cb, _release_cb, None), "net_set_allocator")


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class Net:
    """One network or an ensemble of independent networks on the GPU."""

    def __init__(self, specs, frame_capacity: int = 0, stream=None, block_threads: int = 0,
                 blocks_per_cu: int = 0, flags: int = 0, torch_allocator: bool = True):
        import torch
        lib = library()
        if not torch.cuda.is_available():
            raise RuntimeError("geonet needs a ROCm GPU; none is visible")
        if torch_allocator:
            _register_torch_allocator()
        if not isinstance(specs, (list, tuple)):
            specs = [specs]
        self.specs = list(specs)
        keep: List[np.ndarray] = []

        def arr(x, dt):
            if x is None:
                return None
            a = np.ascontiguousarray(x, dtype=dt)
            keep.append(a)
            return a

        descs = (_abi.NetDesc * len(specs))()
        for k, s in enumerate(specs):
            d = descs[k]
            d.n_nodes = s.n
            d.dims = s.dims
            d.pos_um = _ptr(arr(s.pos_um, np.float64))
            d.n_edges = s.n_edges
            d.src = _ptr(arr(s.src, np.int32))
            d.dst = _ptr(arr(s.dst, np.int32))
            d.weight = _ptr(arr(s.weight, np.float32))
            d.delay_steps = _ptr(arr(s.delay_steps, np.uint8))
            d.v_um_per_ms = s.v_um_per_ms
            d.dt_ms = s.dt_ms
            d.tau_ms = s.tau_ms
            d.v_rest = s.v_rest
            d.v_reset = s.v_reset
            d.v_th = s.v_th
            d.n_ref = s.n_ref
            d.drive_rate_hz = _ptr(arr(s.drive_rate_hz, np.float32))
            d.drive_amp = s.drive_amp
            d.i_ext = _ptr(arr(s.i_ext, np.float32))
            d.noise_sigma = s.noise_sigma
            d.seed = s.seed
            d.v0 = _ptr(arr(s.v0, np.float32))
            d.tau_c_ms = s.tau_c_ms
            d.frame_num = s.frame_num
            d.frame_den = s.frame_den
            if getattr(s, "plastic", 0):
                d.plastic = 1
                d.stdp_alpha, d.stdp_beta = s.stdp_alpha, s.stdp_beta
            d.model = getattr(s, "model", 0)
            if d.model == _abi.NET_MODEL_HODGKIN_HUXLEY:
                d.hh_C, d.hh_gna, d.hh_gk, d.hh_gl = s.hh_C, s.hh_gna, s.hh_gk, s.hh_gl
                d.hh_ena, d.hh_ek, d.hh_el = s.hh_ena, s.hh_ek, s.hh_el
            if d.model:
                d.psc = s.psc
                d.iz_C, d.iz_k, d.iz_vr, d.iz_vt = s.iz_C, s.iz_k, s.iz_vr, s.iz_vt
                d.iz_a, d.iz_b, d.iz_d = s.iz_a, s.iz_b, s.iz_d
                d.psc_rate = s.psc_rate
                d.w0 = _ptr(arr(s.w0_iz, np.float32))
        opts = _abi.BuildOpts(frame_capacity, block_threads, blocks_per_cu, flags)
        h = C.c_void_p()
        self._stream = _stream_handle(stream)
        st = lib.net_build(descs, len(specs), C.byref(opts), self._stream, C.byref(h))
        self.build_status = _check(st, "net_build")
        self.h = h
        del keep
        inf = self.info()
        self.n_total = inf["n_total"]
        self.raster_words = inf["raster_words"]
        self.frame_capacity = frame_capacity

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None) and self.h.value:
            library().net_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        out = _abi.Info()
        _check(library().net_info(self.h, C.byref(out)), "net_info")
        return {name: getattr(out, name) for name, _ in _abi.Info._fields_}

    def node_offsets(self) -> np.ndarray:
        out = np.zeros(len(self.specs) + 1, dtype=np.int64)
        _check(library().net_node_offsets(self.h, out.ctypes.data), "net_node_offsets")
        return out

    @property
    def t(self) -> int:
        return self.info()["t"]

    def step(self, n_steps: int, raster=False, v=False, inp=False, stream=None):
        """Advance n_steps.  raster/v/inp: True to allocate a record tensor,
        a device tensor of the right shape to fill, or False."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())

        def out(x, shape, dtype):
            if x is False or x is None:
                return None
            if x is True:
                return torch.zeros(shape, dtype=dtype, device=dev)
            assert x.is_cuda and x.is_contiguous() and tuple(x.shape) == tuple(shape) and x.dtype == dtype
            return x

        r = out(raster, (n_steps, self.raster_words), torch.int64)
        vv = out(v, (n_steps, self.n_total), torch.float32)
        ii = out(inp, (n_steps, self.n_total), torch.float32)
        rec = _abi.Record(r.data_ptr() if r is not None else None, vv.data_ptr() if vv is not None else None,
                          ii.data_ptr() if ii is not None else None)
        s = self._stream if stream is None else _stream_handle(stream)
        _check(library().net_step_n(self.h, n_steps, C.byref(rec), s), "net_step_n")
        return {"raster": r, "v": vv, "input": ii}

    def timing_begin(self, max_launches: int, every: int = 1):
        """Bind kernel-start/end HIP events to up to max_launches launches,
        one launch of each kernel kind in every `every`."""
        _check(library().net_timing_begin(self.h, max_launches, every), "net_timing_begin")

    def timing_end(self) -> dict:
        out = _abi.Timing()
        _check(library().net_timing_end(self.h, C.byref(out)), "net_timing_end")
        return {name: getattr(out, name) for name, _ in _abi.Timing._fields_}

    def observe(self, what: int, frames: int = 0, gain: float = 1.0, offset: float = 0.0, gamma: float = 0.0,
                stream=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        if what in (NET_OBS_FRAMES, NET_OBS_FLUOR):
            out = torch.empty((frames, self.n_total), dtype=torch.float32, device=dev)
        elif what == NET_OBS_REF:
            out = torch.empty(self.n_total, dtype=torch.int32, device=dev)
        elif what == NET_OBS_WEIGHTS:
            out = torch.empty(max(self.info()["n_edges"], 1), dtype=torch.float32, device=dev)
        else:
            out = torch.empty(self.n_total, dtype=torch.float32, device=dev)
        params = None
        if what == NET_OBS_FLUOR:
            params = _abi.FluorParams(gain, offset, gamma, 0)
        s = self._stream if stream is None else _stream_handle(stream)
        _check(library().net_observe(self.h, what, C.byref(params) if params is not None else None,
                                     out.data_ptr(), out.numel() * 4, s), "net_observe")
        return out


class Mlp:
    """Edge-scoring MLP 64 -> 256 -> 256 -> 1 on the GPU (see include/geonet.h)."""

    N_PARAMS = _abi.MLP_PARAMS

    def __init__(self, params: Optional[np.ndarray] = None, torch_allocator: bool = True):
        import torch
        lib = library()
        if not torch.cuda.is_available():
            raise RuntimeError("geonet needs a ROCm GPU; none is visible")
        if torch_allocator:
            _register_torch_allocator()
        h = C.c_void_p()
        self._check(lib.net_mlp_create(C.byref(h)), "net_mlp_create")
        self.h = h
        if params is not None:
            self.set_params(params)

    @staticmethod
    def _check(st, where):
        if st != NET_OK:
            raise GeonetError(st, where, library().net_mlp_last_error().decode())

    @staticmethod
    def init_params(seed: int = 0) -> np.ndarray:
        """He-uniform initial weights, zero biases."""
        rng = np.random.default_rng(seed)
        p = np.zeros(_abi.MLP_PARAMS, dtype=np.float32)
        i, h = _abi.MLP_IN, _abi.MLP_H
        o = 0
        p[o:o + i * h] = rng.uniform(-1, 1, i * h) * np.sqrt(6.0 / i); o += i * h + h
        p[o:o + h * h] = rng.uniform(-1, 1, h * h) * np.sqrt(6.0 / h); o += h * h + h
        p[o:o + h] = rng.uniform(-1, 1, h) * np.sqrt(3.0 / h)
        return p

    def set_params(self, params: np.ndarray):
        a = np.ascontiguousarray(params, dtype=np.float32)
        self._check(library().net_mlp_set_params(self.h, a.ctypes.data, a.size), "net_mlp_set_params")

    def set_input_norm(self, shift, scale):
        a = np.ascontiguousarray(shift, dtype=np.float32)
        b = np.ascontiguousarray(scale, dtype=np.float32)
        assert a.size == _abi.MLP_IN and b.size == _abi.MLP_IN
        self._check(library().net_mlp_set_input_norm(self.h, a.ctypes.data, b.ctypes.data), "net_mlp_set_input_norm")

    def fit_input_norm(self, x, stream=None):
        """Standardisation fitted on the GPU to features x (torch float32 [rows][64])."""
        import torch
        assert x.is_cuda and x.dtype == torch.float32 and x.shape[1] == _abi.MLP_IN and x.is_contiguous()
        self._check(library().net_mlp_fit_input_norm(self.h, x.data_ptr(), x.shape[0], _stream_handle(stream)),
                    "net_mlp_fit_input_norm")

    def get_input_norm(self):
        shift = np.zeros(_abi.MLP_IN, dtype=np.float32)
        scale = np.zeros(_abi.MLP_IN, dtype=np.float32)
        self._check(library().net_mlp_get_input_norm(self.h, shift.ctypes.data, scale.ctypes.data),
                    "net_mlp_get_input_norm")
        return shift, scale

    def train_epoch(self, x, y, batch: int, lr: float, seed: int, epoch: int, losses=None, stream=None):
        """One shuffled pass over the rows, one Adam step per batch (the last may be smaller)."""
        import torch
        assert x.is_cuda and x.dtype == torch.float32 and x.shape[1] == _abi.MLP_IN and x.is_contiguous()
        assert y.is_cuda and y.dtype == torch.float32 and y.shape[0] == x.shape[0] and y.is_contiguous()
        self._check(library().net_mlp_train_epoch(self.h, x.data_ptr(), y.data_ptr(), x.shape[0], int(batch),
                                                  float(lr), int(seed) & 0xFFFFFFFFFFFFFFFF, int(epoch) & 0xFFFFFFFF,
                                                  losses.data_ptr() if losses is not None else None,
                                                  _stream_handle(stream)), "net_mlp_train_epoch")

    def get_params(self) -> np.ndarray:
        out = np.zeros(_abi.MLP_PARAMS, dtype=np.float32)
        self._check(library().net_mlp_get_params(self.h, out.ctypes.data, out.size), "net_mlp_get_params")
        return out

    def forward(self, x, stream=None):
        import torch
        assert x.is_cuda and x.dtype == torch.float32 and x.shape[1] == _abi.MLP_IN and x.is_contiguous()
        out = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        self._check(library().net_mlp_forward(self.h, x.data_ptr(), x.shape[0], out.data_ptr(),
                                              _stream_handle(stream)), "net_mlp_forward")
        return out

    def grad(self, x, y, stream=None):
        import torch
        g = torch.empty(_abi.MLP_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        self._check(library().net_mlp_grad(self.h, x.data_ptr(), y.data_ptr(), x.shape[0], g.data_ptr(),
                                           loss.data_ptr(), _stream_handle(stream)), "net_mlp_grad")
        return g, loss

    def train_step(self, x, y, lr: float, loss=None, stream=None):
        self._check(library().net_mlp_train_step(self.h, x.data_ptr(), y.data_ptr(), x.shape[0], float(lr),
                                                 loss.data_ptr() if loss is not None else None,
                                                 _stream_handle(stream)), "net_mlp_train_step")

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            library().net_mlp_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def shuffle_indices(n: int, seed: int, epoch: int, stream=None):
    """The permutation of [0, n) the scorer's training epochs visit rows in
    (torch int64 [n] on the GPU)."""
    import torch
    out = torch.empty(max(int(n), 1), dtype=torch.int64, device="cuda")
    st = library().net_shuffle_indices(int(n), int(seed) & 0xFFFFFFFFFFFFFFFF, int(epoch) & 0xFFFFFFFF,
                                       out.data_ptr(), _stream_handle(stream))
    if st != NET_OK:
        raise GeonetError(st, "net_shuffle_indices", library().net_mlp_last_error().decode())
    return out[:int(n)]


def unpack_raster(words, n: int) -> np.ndarray:
    """[T, W] int64 raster words -> [T, n] uint8 spike matrix (host)."""
    import torch
    w = words.cpu().numpy() if hasattr(words, "cpu") else np.asarray(words)
    b = np.unpackbits(w.view(np.uint8).reshape(w.shape[0], -1), axis=1, bitorder="little")
    return b[:, :n]
