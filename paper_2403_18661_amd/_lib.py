"""ctypes declarations of libaframe_mi.so (the C ABI in include/aframe_mi.h)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaframe_mi.so")

c_i64 = ctypes.c_int64
c_dbl = ctypes.c_double
c_vp = ctypes.c_void_p
c_sz = ctypes.c_size_t
c_int = ctypes.c_int


class NetDesc(ctypes.Structure):
    _fields_ = [("in_ch", ctypes.c_int32), ("stem_ch", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("stem_stride", ctypes.c_int32), ("stem_pool", ctypes.c_int32), ("n_stages", ctypes.c_int32),
                ("widths", ctypes.c_int32 * 8), ("blocks", ctypes.c_int32 * 8), ("window", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("fs", ctypes.c_double), ("prescale", ctypes.c_double), ("nperseg", c_i64), ("noverlap", c_i64),
                ("psd_len", c_i64), ("psd_hop", c_i64), ("fduration", ctypes.c_double),
                ("highpass", ctypes.c_double), ("stride", c_i64), ("integrate_width", c_i64), ("block", c_i64),
                ("max_chunk", c_i64), ("max_tick", c_i64), ("max_streams", c_i64), ("score_batch", c_i64),
                ("hbm_budget", c_sz)]


# name -> (restype, argtypes); the list is also the set of exported symbols
SIGNATURES = {
    "af_last_error": (ctypes.c_char_p, []),
    "af_version": (ctypes.c_char_p, []),
    "af_init": (c_int, []),
    "af_psd_workspace_bytes": (c_sz, [c_i64, c_i64, c_i64, c_i64, c_i64, c_i64]),
    "af_psd_estimate": (c_int, [c_vp, c_int, c_i64, c_i64, c_i64, c_dbl, c_dbl, c_i64, c_i64, c_i64, c_i64,
                                c_i64, c_vp, c_vp, c_sz, c_vp]),
    "af_whiten_workspace_bytes": (c_sz, [c_i64, c_i64, c_i64]),
    "af_whiten": (c_int, [c_vp, c_int, c_i64, c_i64, c_i64, c_dbl, c_dbl, c_vp, c_i64, c_i64, c_i64, c_dbl,
                          c_dbl, c_i64, c_i64, c_vp, c_i64, c_vp, c_sz, c_vp]),
    "af_whiten_noalloc": (c_int, [c_vp, c_int, c_i64, c_i64, c_i64, c_dbl, c_dbl, c_vp, c_i64, c_i64, c_i64, c_dbl,
                                  c_dbl, c_i64, c_i64, c_vp, c_i64, c_vp]),
    "af_whiten_response": (c_int, [c_vp, c_i64, c_i64, c_i64, c_dbl, c_dbl, c_dbl, c_vp, c_sz, c_vp]),
    "af_whiten_apply": (c_int, [c_vp, c_int, c_i64, c_i64, c_i64, c_dbl, c_dbl, c_vp, c_sz, c_i64, c_i64, c_dbl,
                                c_i64, c_i64, c_vp, c_i64, c_vp]),
    "af_net_create": (c_int, [ctypes.POINTER(NetDesc), c_vp, c_i64, c_int, ctypes.POINTER(c_vp)]),
    "af_net_create_gn": (c_int, [ctypes.POINTER(NetDesc), ctypes.c_int32, c_vp, c_i64, c_int, ctypes.POINTER(c_vp)]),
    "af_net_destroy": (None, [c_vp]),
    "af_net_calibrate": (c_int, [c_vp, c_vp, c_i64, c_i64, c_i64, c_i64, c_i64, c_vp, c_sz, c_vp]),
    "af_net_macs": (c_i64, [c_vp]),
    "af_score_workspace_bytes": (c_sz, [c_vp, c_i64]),
    "af_net_n_layers": (c_i64, [c_vp]),
    "af_net_fused": (c_int, [c_vp]),
    "af_net_autotune": (c_int, [c_vp, c_i64, c_vp, c_sz, c_vp, ctypes.POINTER(c_i64)]),
    "af_cluster_workspace_bytes": (c_sz, [c_i64]),
    "af_cluster": (c_int, [c_vp, c_i64, c_vp, c_i64, c_i64, c_vp, c_vp, c_i64, c_vp, c_vp, c_sz, c_vp]),
    "af_far_workspace_bytes": (c_sz, [c_i64]),
    "af_far": (c_int, [c_vp, c_i64, c_dbl, c_vp, c_i64, c_vp, c_vp, c_sz, c_vp]),
    "af_project": (c_int, [c_vp, c_vp, c_i64, c_i64, c_dbl, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "af_snr_rescale": (c_int, [c_vp, c_i64, c_i64, c_i64, c_dbl, c_vp, c_i64, c_dbl, c_dbl, c_vp, c_vp, c_vp]),
    "af_net_set_layer_tile": (c_int, [c_vp, c_i64, ctypes.c_int32]),
    "af_net_layer_tile": (c_int, [c_vp, c_i64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "af_net_set_fused": (c_int, [c_vp, c_int]),
    "af_net_fused_tile": (c_int, [c_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32)]),
    "af_net_set_fused_tile": (c_int, [c_vp, ctypes.c_int32]),
    "af_net_profile_begin": (c_int, [c_vp]),
    "af_net_profile_end": (c_int, [c_vp, c_i64, c_vp, c_vp, c_vp]),
    "af_score_windows": (c_int, [c_vp, c_vp, c_i64, c_i64, c_i64, c_i64, c_i64, c_vp, c_i64, c_vp, c_vp,
                                 c_sz, c_vp]),
    "af_integrate": (c_int, [c_vp, c_i64, c_i64, c_vp, c_vp, c_vp]),
    "af_timeslide_prepare": (c_int, [c_vp, c_vp, c_vp, c_i64, c_vp, c_i64, c_i64, c_i64, c_vp, c_sz, c_vp]),
    "af_score_timeslides_prepared": (c_int, [c_vp, c_vp, c_i64, c_i64, c_i64, c_i64, c_i64, c_i64, c_i64, c_vp,
                                             c_vp, c_sz, c_vp]),
    "af_graph_begin": (c_int, [c_vp]),
    "af_graph_end": (c_int, [c_vp, ctypes.POINTER(c_vp)]),
    "af_graph_launch": (c_int, [c_vp, c_vp]),
    "af_graph_destroy": (None, [c_vp]),
    "af_server_default_config": (None, [ctypes.POINTER(ServerConfig)]),
    "af_server_create": (c_int, [c_vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(c_vp)]),
    "af_server_destroy": (None, [c_vp]),
    "af_server_stream_bytes": (c_sz, [c_vp]),
    "af_server_shared_bytes": (c_sz, [c_vp]),
    "af_server_admit": (c_int, [c_vp, ctypes.POINTER(c_i64)]),
    "af_server_release": (c_int, [c_vp, c_i64]),
    "af_server_push": (c_int, [c_vp, c_i64, c_vp, c_i64]),
    "af_server_tick": (c_int, [c_vp, ctypes.POINTER(c_i64)]),
    "af_server_poll": (c_int, [c_vp, c_i64, c_vp, c_i64, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64), c_vp, c_i64,
                               ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
    "af_server_stats": (c_int, [c_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(c_i64), ctypes.POINTER(c_i64), c_int]),
    "af_timeslide_n_windows": (c_i64, [c_vp, c_i64, c_i64, c_i64, c_i64]),
    "af_timeslide_workspace_bytes": (c_sz, [c_vp, c_i64, c_i64, c_i64]),
    "af_score_timeslides": (c_int, [c_vp, c_vp, c_i64, c_i64, c_i64, c_vp, c_vp, c_i64, c_vp, c_i64, c_i64, c_vp,
                                    c_vp, c_sz, c_vp]),
}

_lib = None


def lib():
    """Load the library (once).  Raises ImportError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2403_18661_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class AframeError(RuntimeError):
    pass


STATUS = {0: "AF_OK", -1: "AF_EINVAL", -2: "AF_ENOMEM", -3: "AF_EHIP", -4: "AF_EUNSUPPORTED", -5: "AF_EBUDGET"}


def check(status):
    if status != 0:
        msg = lib().af_last_error().decode()
        raise AframeError(f"{STATUS.get(status, status)}: {msg}")
