"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
library: its C source (``oracle.c``) is compiled with gcc on its own, and it
reads only the seeded inputs made by ``synth``.

What it computes is listed, with the paper passages it follows, at the top of
``oracle.c``; ``dense.py`` holds a second, brute-force formulation for tiny
networks, and ``mlp.py`` / ``metrics.py`` the scorer-side references.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_c = ctypes
_vp = _c.c_void_p


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = _c.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [_vp, _vp, _vp]
        L.orc_philox4x32_10.restype = None
        L.orc_box_muller.argtypes = [_c.c_uint32, _c.c_uint32]
        L.orc_box_muller.restype = _c.c_double
        L.orc_u01_24.argtypes = [_c.c_uint32]
        L.orc_u01_24.restype = _c.c_double
        L.orc_drive_threshold.argtypes = [_c.c_double, _c.c_double]
        L.orc_drive_threshold.restype = _c.c_uint32
        L.orc_delay_steps.argtypes = [_vp, _vp, _c.c_int, _c.c_double, _c.c_double]
        L.orc_delay_steps.restype = _c.c_int32
        L.orc_create.restype = _vp
        L.orc_create.argtypes = [_c.c_int32, _c.c_int32, _vp, _c.c_int64, _vp, _vp, _vp, _vp,
                                 _c.c_double, _c.c_double, _c.c_double, _c.c_double, _c.c_double,
                                 _c.c_double, _c.c_int32, _vp, _c.c_double, _vp, _c.c_double,
                                 _c.c_uint64, _vp, _c.c_double, _c.c_int64, _c.c_int64, _c.c_int64]
        L.orc_free.argtypes = [_vp]
        L.orc_free.restype = None
        L.orc_step_n.argtypes = [_vp, _c.c_int64, _vp, _vp, _vp, _vp]
        L.orc_step_n.restype = None
        for name in ("orc_time", "orc_delivered", "orc_frames_done"):
            getattr(L, name).argtypes = [_vp]
            getattr(L, name).restype = _c.c_int64
        for name in ("orc_get_v", "orc_get_ref", "orc_get_c"):
            getattr(L, name).argtypes = [_vp, _vp]
            getattr(L, name).restype = None
        L.orc_get_frames.argtypes = [_vp, _vp, _c.c_int64]
        L.orc_get_frames.restype = _c.c_int64
        L.orc_edge_delay.argtypes = [_vp, _c.c_int32, _c.c_int32]
        L.orc_edge_delay.restype = _c.c_int32
        L.orc_fluorescence.argtypes = [_vp, _c.c_int64, _c.c_int32, _c.c_int64, _c.c_double,
                                       _c.c_double, _c.c_double, _c.c_uint64, _vp]
        L.orc_fluorescence.restype = None
        L.orc_set_izhikevich.argtypes = [_vp, _c.c_int32, _vp, _c.c_double, _vp]
        L.orc_set_izhikevich.restype = _c.c_int32
        L.orc_get_izh.argtypes = [_vp, _vp, _vp, _vp]
        L.orc_get_izh.restype = None
        L.orc_set_hodgkin_huxley.argtypes = [_vp, _c.c_int32, _vp, _c.c_double]
        L.orc_set_hodgkin_huxley.restype = _c.c_int32
        L.orc_get_hh.argtypes = [_vp, _vp, _vp, _vp]
        L.orc_get_hh.restype = None
        L.orc_set_stdp.argtypes = [_vp, _c.c_double, _c.c_double]
        L.orc_set_stdp.restype = _c.c_int32
        L.orc_get_weights.argtypes = [_vp, _vp, _vp, _c.c_int64, _vp]
        L.orc_get_weights.restype = None
        L.orc_set_threads.argtypes = [_c.c_int32]
        L.orc_set_threads.restype = None
        L.orc_get_threads.argtypes = []
        L.orc_get_threads.restype = _c.c_int32
        _lib = L
    return _lib


def set_threads(k: int) -> None:
    """Threads for the per-vertex loops of the simulation oracle (default 1).
    Results are bit-identical for any count (the spike push stays serial)."""
    _load().orc_set_threads(int(k))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def test_threads() -> int:
    """Thread count tests use for large oracle runs: the CPUs this process
    may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def philox4x32_10(ctr, key) -> np.ndarray:
    L = _load()
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    L.orc_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def box_muller(a: int, b: int) -> float:
    return _load().orc_box_muller(a, b)


def u01_24(a: int) -> float:
    return _load().orc_u01_24(a)


def drive_threshold(rate_hz: float, dt_ms: float) -> int:
    return int(_load().orc_drive_threshold(rate_hz, dt_ms))


def delay_steps(xi, xj, v_um_per_ms: float, dt_ms: float) -> int:
    a = np.ascontiguousarray(xi, dtype=np.float64)
    b = np.ascontiguousarray(xj, dtype=np.float64)
    return int(_load().orc_delay_steps(a.ctypes.data, b.ctypes.data, a.shape[0], v_um_per_ms, dt_ms))


class OracleNet:
    """One network advanced by the FP64 oracle."""

    def __init__(self, spec, frames_cap: int = 0):
        L = _load()
        self._keep = []

        def arr(x, dt):
            if x is None:
                return None
            a = np.ascontiguousarray(x, dtype=dt)
            self._keep.append(a)
            return a

        self.n = spec.n
        pos = arr(spec.pos_um, np.float64)
        src = arr(spec.src, np.int32)
        dst = arr(spec.dst, np.int32)
        w = arr(spec.weight, np.float32)
        dl = arr(spec.delay_steps, np.uint8)
        rate = arr(spec.drive_rate_hz, np.float32)
        iext = arr(spec.i_ext, np.float32)
        v0 = arr(spec.v0, np.float32)
        self.frames_cap = frames_cap
        self.h = L.orc_create(spec.n, spec.dims, _ptr(pos), spec.n_edges, _ptr(src), _ptr(dst), _ptr(w),
                              _ptr(dl), spec.v_um_per_ms, spec.dt_ms, spec.tau_ms, spec.v_rest,
                              spec.v_reset, spec.v_th, spec.n_ref, _ptr(rate), spec.drive_amp, _ptr(iext),
                              spec.noise_sigma, spec.seed, _ptr(v0), spec.tau_c_ms, spec.frame_num,
                              spec.frame_den, frames_cap)
        if not self.h:
            raise ValueError("oracle rejected the network (bad edge or delay > 255)")
        self._L = L
        self.model = getattr(spec, "model", 0)
        if self.model == 1:
            iz = np.array([spec.iz_C, spec.iz_k, spec.iz_vr, spec.iz_vt, spec.iz_a, spec.iz_b, spec.iz_d],
                          dtype=np.float64)
            if not np.array_equal(iz.astype(np.float32).astype(np.float64), iz) or \
                    float(np.float32(spec.psc_rate)) != spec.psc_rate:
                raise ValueError("Izhikevich constants must be FP32 values (the library takes them as FP32)")
            w0 = arr(getattr(spec, "w0_iz", None), np.float32)
            if L.orc_set_izhikevich(self.h, int(spec.psc), iz.ctypes.data, float(spec.psc_rate), _ptr(w0)) != 0:
                raise ValueError("oracle rejected the Izhikevich parameters")
        if getattr(spec, "plastic", 0):
            a_, b_ = float(spec.stdp_alpha), float(spec.stdp_beta)
            if float(np.float32(a_)) != a_ or float(np.float32(b_)) != b_:
                raise ValueError("STDP rates must be FP32 values (the library takes them as FP32)")
            if L.orc_set_stdp(self.h, a_, b_) != 0:
                raise ValueError("oracle rejected STDP (LIF only, weights multiples of 2^-20)")
        if self.model == 2:
            hh = np.array([spec.hh_C, spec.hh_gna, spec.hh_gk, spec.hh_gl, spec.hh_ena, spec.hh_ek, spec.hh_el],
                          dtype=np.float64)
            if not np.array_equal(hh.astype(np.float32).astype(np.float64), hh) or \
                    float(np.float32(spec.psc_rate)) != spec.psc_rate:
                raise ValueError("Hodgkin-Huxley constants must be FP32 values (the library takes them as FP32)")
            if L.orc_set_hodgkin_huxley(self.h, int(spec.psc), hh.ctypes.data, float(spec.psc_rate)) != 0:
                raise ValueError("oracle rejected the Hodgkin-Huxley parameters")

    def close(self):
        if self.h:
            self._L.orc_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self) -> int:
        return int(self._L.orc_time(self.h))

    @property
    def delivered(self) -> int:
        return int(self._L.orc_delivered(self.h))

    def step(self, n_steps: int, raster: bool = True, v: bool = False, inp: bool = False,
             force_raster: Optional[np.ndarray] = None):
        n = self.n
        r = np.zeros((n_steps, n), dtype=np.uint8) if raster else None
        vr = np.zeros((n_steps, n), dtype=np.float64) if v else None
        ir = np.zeros((n_steps, n), dtype=np.float64) if inp else None
        fr = None
        if force_raster is not None:
            fr = np.ascontiguousarray(force_raster, dtype=np.uint8)
            assert fr.shape == (n_steps, n)
        self._L.orc_step_n(self.h, n_steps, _ptr(r), _ptr(vr), _ptr(ir), _ptr(fr))
        return {"raster": r, "v": vr, "input": ir}

    def v(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.float64)
        self._L.orc_get_v(self.h, out.ctypes.data)
        return out

    def ref(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.int32)
        self._L.orc_get_ref(self.h, out.ctypes.data)
        return out

    def izhikevich_state(self):
        """(W, r, p) of every vertex (Izhikevich networks)."""
        W, r, p = (np.zeros(self.n, dtype=np.float64) for _ in range(3))
        self._L.orc_get_izh(self.h, W.ctypes.data, r.ctypes.data, p.ctypes.data)
        return W, r, p

    def weights(self, src, dst) -> np.ndarray:
        """Current weight of each edge (src[e] -> dst[e])."""
        a = np.ascontiguousarray(src, dtype=np.int32)
        b = np.ascontiguousarray(dst, dtype=np.int32)
        out = np.zeros(a.shape[0], dtype=np.float64)
        self._L.orc_get_weights(self.h, a.ctypes.data, b.ctypes.data, a.shape[0], out.ctypes.data)
        return out

    def gates(self):
        """(m, n, h) of every vertex (Hodgkin-Huxley networks)."""
        m, n, h = (np.zeros(self.n, dtype=np.float64) for _ in range(3))
        self._L.orc_get_hh(self.h, m.ctypes.data, n.ctypes.data, h.ctypes.data)
        return m, n, h

    def calcium(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.float64)
        self._L.orc_get_c(self.h, out.ctypes.data)
        return out

    def frames(self) -> np.ndarray:
        nf = int(self._L.orc_frames_done(self.h))
        nf = min(nf, self.frames_cap)
        out = np.zeros((max(nf, 0), self.n), dtype=np.float64)
        if nf > 0:
            self._L.orc_get_frames(self.h, out.ctypes.data, nf)
        return out

    def edge_delay(self, src: int, dst: int) -> int:
        return int(self._L.orc_edge_delay(self.h, src, dst))


def fluorescence(cbar: np.ndarray, gain: float, offset: float, gamma: float, seed: int,
                 frame0: int = 0) -> np.ndarray:
    cb = np.ascontiguousarray(cbar, dtype=np.float64)
    nf, n = cb.shape
    out = np.zeros_like(cb)
    _load().orc_fluorescence(cb.ctypes.data, nf, n, frame0, gain, offset, gamma, seed, out.ctypes.data)
    return out
