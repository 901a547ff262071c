"""ctypes declarations mirroring include/geonet.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgeonet.so")

NET_OK = 0
NET_W_INEXACT = 1
NET_E_ARG = -1
NET_E_RANGE = -2
NET_E_OOM = -3
NET_E_DEVICE = -4
NET_E_STATE = -5
NET_E_UNSUPPORTED = -6

NET_BUILD_NO_LDS_SUMMARY = 1
NET_BUILD_DELIVER_STREAM_WEIGHTS = 2
NET_BUILD_DELIVER_NONTEMPORAL = 4
NET_BUILD_PER_STEP = 8
NET_BUILD_DELIVER_UNROLL2 = 16
NET_BUILD_SINGLE_LAUNCH = 32
NET_BUILD_DELIVER_PIPELINE = 128
NET_BUILD_SUMMARY_HALF = 256
NET_BUILD_DELIVER_COMPACT = 512
NET_BUILD_FUSED_STEP = 1024
NET_BUILD_DELIVER_PACKED = 2048
NET_BUILD_AUTOTUNE = 64
NET_BUILD_REORDER = 4096
NET_BUILD_GRAPH = 8192
NET_BUILD_PUSH = 16384

NET_MODEL_LIF = 0
NET_MODEL_IZHIKEVICH = 1
NET_MODEL_HODGKIN_HUXLEY = 2
NET_PSC_NONE = 0
NET_PSC_EXP = 1
NET_PSC_ALPHA = 2

NET_OBS_V = 1
NET_OBS_REF = 2
NET_OBS_CALCIUM = 3
NET_OBS_FRAMES = 4
NET_OBS_FLUOR = 5
NET_OBS_WEIGHTS = 6

_vp = C.c_void_p


class NetDesc(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32), ("dims", C.c_int32), ("pos_um", _vp), ("n_edges", C.c_int64),
        ("src", _vp), ("dst", _vp), ("weight", _vp), ("delay_steps", _vp),
        ("v_um_per_ms", C.c_double), ("dt_ms", C.c_double), ("tau_ms", C.c_float),
        ("v_rest", C.c_float), ("v_reset", C.c_float), ("v_th", C.c_float), ("n_ref", C.c_int32),
        ("drive_rate_hz", _vp), ("drive_amp", C.c_float), ("i_ext", _vp), ("noise_sigma", C.c_float),
        ("seed", C.c_uint64), ("v0", _vp), ("tau_c_ms", C.c_float), ("frame_num", C.c_int32),
        ("frame_den", C.c_int32), ("model", C.c_int32), ("psc", C.c_int32), ("iz_C", C.c_float),
        ("iz_k", C.c_float), ("iz_vr", C.c_float), ("iz_vt", C.c_float), ("iz_a", C.c_float),
        ("iz_b", C.c_float), ("iz_d", C.c_float), ("psc_rate", C.c_float), ("w0", _vp),
        ("hh_C", C.c_float), ("hh_gna", C.c_float), ("hh_gk", C.c_float), ("hh_gl", C.c_float),
        ("hh_ena", C.c_float), ("hh_ek", C.c_float), ("hh_el", C.c_float),
        ("plastic", C.c_int32), ("stdp_alpha", C.c_float), ("stdp_beta", C.c_float),
    ]


class BuildOpts(C.Structure):
    _fields_ = [("frame_capacity", C.c_int32), ("block_threads", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("flags", C.c_int32)]


class Record(C.Structure):
    _fields_ = [("raster", _vp), ("v", _vp), ("input", _vp)]


class Info(C.Structure):
    _fields_ = [
        ("n_total", C.c_int64), ("n_edges", C.c_int64), ("n_edges_stored", C.c_int64),
        ("n_nets", C.c_int32), ("max_delay", C.c_int32), ("raster_words", C.c_int64), ("t", C.c_int64),
        ("frames_done", C.c_int64), ("exact", C.c_int32), ("summary_window", C.c_int32), ("lds_summary", C.c_int32),
        ("deliver_blocks", C.c_int32), ("deliver_threads", C.c_int32), ("device_bytes", C.c_int64),
        ("deliver_flags", C.c_int32), ("ensemble_blocks", C.c_int32), ("ensemble_threads", C.c_int32),
        ("autotuned", C.c_int32), ("ensemble_stream", C.c_int32),
    ]


class Timing(C.Structure):
    _fields_ = [("deliver_ms", C.c_double), ("update_ms", C.c_double), ("ensemble_ms", C.c_double),
                ("deliver_launches", C.c_int64), ("update_launches", C.c_int64),
                ("ensemble_launches", C.c_int64), ("steps", C.c_int64), ("step_ms", C.c_double),
                ("step_launches", C.c_int64)]


class FluorParams(C.Structure):
    _fields_ = [("gain", C.c_float), ("offset", C.c_float), ("gamma", C.c_float), ("pad", C.c_int32)]


class ObsDesc(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32), ("n_frames", C.c_int32), ("fluor", _vp), ("n_pairs", C.c_int64),
        ("pairs", _vp), ("pair_dist_um", _vp), ("gain", C.c_float), ("offset", C.c_float), ("gamma", C.c_float),
        ("dt_ms", C.c_double), ("tau_c_ms", C.c_float), ("frame_num", C.c_int32), ("frame_den", C.c_int32),
        ("drive_rate_hz", _vp), ("drive_amp", C.c_float), ("control_seed", C.c_uint64),
        ("tau_ms", C.c_float), ("v_rest", C.c_float), ("v_reset", C.c_float), ("v_th", C.c_float),
        ("noise_sigma", C.c_float), ("w_assumed", C.c_float), ("n_ref", C.c_int32), ("w_source", _vp),
    ]


class SimfitOpts(C.Structure):
    _fields_ = [("realisations", C.c_int32), ("sweeps", C.c_int32), ("init_fraction", C.c_float),
                ("min_gain", C.c_float), ("fit_seed", C.c_uint64)]


NET_EST_SCORER = 1
NET_EST_SIMFIT = 2
NET_EST_AUTO = 3

ALLOC_FN = C.CFUNCTYPE(_vp, C.c_size_t, _vp, _vp)
RELEASE_FN = C.CFUNCTYPE(None, _vp, _vp, _vp)

# name -> (restype, argtypes)
SIGNATURES = {
    "net_set_allocator": (C.c_int, [ALLOC_FN, RELEASE_FN, _vp]),
    "net_build": (C.c_int, [C.POINTER(NetDesc), C.c_int32, C.POINTER(BuildOpts), _vp, C.POINTER(_vp)]),
    "net_step_n": (C.c_int, [_vp, C.c_int64, C.POINTER(Record), _vp]),
    "net_observe": (C.c_int, [_vp, C.c_int32, _vp, _vp, C.c_int64, _vp]),
    "net_info": (C.c_int, [_vp, C.POINTER(Info)]),
    "net_node_offsets": (C.c_int, [_vp, _vp]),
    "net_timing_begin": (C.c_int, [_vp, C.c_int64, C.c_int32]),
    "net_timing_end": (C.c_int, [_vp, C.POINTER(Timing)]),
    "net_free": (None, [_vp]),
    "net_last_error": (C.c_char_p, []),
    "net_mlp_create": (C.c_int, [C.POINTER(_vp)]),
    "net_mlp_set_params": (C.c_int, [_vp, _vp, C.c_int64]),
    "net_mlp_get_params": (C.c_int, [_vp, _vp, C.c_int64]),
    "net_mlp_set_input_norm": (C.c_int, [_vp, _vp, _vp]),
    "net_features": (C.c_int, [_vp, _vp, _vp]),
    "net_estimate": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp, _vp]),
    "net_estimate_last_error": (C.c_char_p, []),
    "net_mlp_forward": (C.c_int, [_vp, _vp, C.c_int64, _vp, _vp]),
    "net_mlp_grad": (C.c_int, [_vp, _vp, _vp, C.c_int64, _vp, _vp, _vp]),
    "net_mlp_train_step": (C.c_int, [_vp, _vp, _vp, C.c_int64, C.c_float, _vp, _vp]),
    "net_mlp_fit_input_norm": (C.c_int, [_vp, _vp, C.c_int64, _vp]),
    "net_mlp_get_input_norm": (C.c_int, [_vp, _vp, _vp]),
    "net_mlp_train_epoch": (C.c_int, [_vp, _vp, _vp, C.c_int64, C.c_int64, C.c_float, C.c_uint64, C.c_uint32, _vp,
                                      _vp]),
    "net_shuffle_indices": (C.c_int, [C.c_int64, C.c_uint64, C.c_uint32, _vp, _vp]),
    "net_mlp_free": (None, [_vp]),
    "net_simulate_device_error": (C.c_int, [_vp]),
    "net_features_noalloc": (C.c_int, [_vp, _vp, _vp]),
    "net_features_noalloc_scratch_bytes": (C.c_size_t, [C.c_int32, C.c_int32]),
    "net_mlp_last_error": (C.c_char_p, []),
}

MLP_PARAMS = 82689
MLP_IN, MLP_H = 64, 256

_lib = None


def load() -> C.CDLL:
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgeonet.so is not built; run paper_0908_3934_amd/build.py "
                               "(or __graft_entry__.build()) first")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib
