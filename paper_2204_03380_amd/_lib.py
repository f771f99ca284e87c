"""ctypes loader for librtm.so (the HIP library).  Raises if the library is
missing: there is no fallback path."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtm.so")

RTM_OK = 0
RTM_EINVAL = -1
RTM_ECFL = -2
RTM_ERANGE = -3
RTM_EWORKSPACE = -4
RTM_EHIP = -5
RTM_ENUMERIC = -6

RTM_OP_RBC_PAD = 0
RTM_OP_MODEL = 1
RTM_OP_RTM = 2
RTM_OP_VJP = 3
RTM_OP_STORAGE = 4
RTM_TUNE_EXACT = 0x100

RTM_F_SKIP_CHECK = 0x1
RTM_F_NO_REINJECT = 0x2

# Every symbol declared in include/rtm.h and include/unet.h.
EXPORTS = (
    "rtm_abi_version", "rtm_last_error", "rtm_set_tuning", "rtm_get_tuning", "rtm_set_tuning2d",
    "rtm_get_tuning2d", "rtm_set_steps_per_launch", "rtm_get_steps_per_launch", "rtm_set_tuning3d",
    "rtm_get_tuning3d", "rtm_set_tile_order3d", "rtm_get_tile_order3d", "rtm_timing_enable", "rtm_timing_read",
    "rtm_workspace_bytes", "rtm_rbc_pad", "rtm_rbc_pad_ex", "rtm_pad_adjoint_ex",
    "rtm_pad_adjoint", "rtm_model_shot", "rtm_rtm_shot", "rtm_nyquist_stride", "rtm_storage_count",
    "rtm_storage_shot", "rtm_model_shot_vjp", "rtm_batch_plan", "rtm_batch_run",
    "rtm_batch_free", "rtm_window_extract", "rtm_window_accumulate", "rtm_misfit_ws_bytes", "rtm_l2_misfit",
    "rtm_stream_copy", "rtm_rtm_shot_noalloc", "rtm_set_persist_wait", "rtm_get_persist_wait",
    "unet_weight_pack", "unet_weight_pack_many", "unet_conv3d_fwd", "unet_conv3d_dgrad", "unet_conv3d_dgrad_relu", "unet_wgrad_ws_bytes",
    "unet_conv3d_wgrad", "unet_conv3d_wgrad_partial", "unet_wgrad_reduce_many", "unet_embed", "unet_pool2", "unet_up2", "unet_up2_bwd", "unet_up2_bwd_relu",
    "unet_relu_grad", "unet_mse_ws_bytes", "unet_mse",
    "unet_adam", "unet_set_conv_lds", "unet_get_conv_lds",
)

RTM_F_ACCUMULATE = 0x4
RTM_F_GRAPH = 0x8
RTM_F_CHECK_FINITE = 0x10
RTM_F_PERSISTENT = 0x20


class RtmGrid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("nb", ctypes.c_int32), ("nx", ctypes.c_int64),
                ("ny", ctypes.c_int64), ("nz", ctypes.c_int64), ("h", ctypes.c_double)]


class RtmShotDesc(ctypes.Structure):
    _fields_ = [("grid", RtmGrid), ("v_pad", ctypes.c_void_p), ("wavelet", ctypes.c_void_p),
                ("src", ctypes.c_float * 3), ("nrec", ctypes.c_int32), ("rec", ctypes.c_void_p),
                ("traces_in", ctypes.c_void_p), ("traces_out", ctypes.c_void_p), ("image", ctypes.c_void_p),
                ("grad_v_pad", ctypes.c_void_p)]


class UnetConvDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("d", ctypes.c_int32), ("h", ctypes.c_int32), ("w", ctypes.c_int32),
                ("cin", ctypes.c_int32), ("cout", ctypes.c_int32)]


class UnetPackItem(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("cin", ctypes.c_int32), ("cout", ctypes.c_int32), ("w_fwd", ctypes.c_void_p),
                ("w_bwd", ctypes.c_void_p)]


UNET_PACK_MAX = 16


class UnetWgradItem(ctypes.Structure):
    _fields_ = [("desc", UnetConvDesc), ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t),
                ("dw", ctypes.c_void_p), ("db", ctypes.c_void_p)]


UNET_WGRAD_MAX = 16


class RtmRbcOpts(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("v_cap", ctypes.c_float), ("flags", ctypes.c_uint32),
                ("taper_alpha", ctypes.c_double)]


RTM_RBC_TAPER = 0x1
RTM_RBC_FREE_SURFACE = 0x2


class RtmProbe(ctypes.Structure):
    _fields_ = [("snap_k", ctypes.c_int32), ("snap_p", ctypes.c_void_p), ("snap_mu", ctypes.c_void_p)]


_lib = None


def load():
    """The loaded library (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} not found: build it with `python -m paper_2204_03380_amd.build` "
                      "(no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, F, U32, U64, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                        ctypes.c_float, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t)
    G = ctypes.POINTER(RtmGrid)
    C = ctypes.POINTER(UnetConvDesc)
    sig = {
        "rtm_abi_version": ([], ctypes.c_int),
        "rtm_last_error": ([], ctypes.c_char_p),
        "rtm_set_tuning": ([ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "rtm_get_tuning": ([ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "rtm_set_tuning2d": ([ctypes.c_int] * 4, ctypes.c_int),
        "rtm_get_tuning2d": ([ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 3, ctypes.c_int),
        "rtm_set_steps_per_launch": ([ctypes.c_int] * 2, ctypes.c_int),
        "rtm_get_steps_per_launch": ([ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "rtm_set_tuning3d": ([ctypes.c_int] * 4, ctypes.c_int),
        "rtm_get_tuning3d": ([ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 3, ctypes.c_int),
        "rtm_set_tile_order3d": ([ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "rtm_get_tile_order3d": ([ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "rtm_timing_enable": ([ctypes.c_int], ctypes.c_int),
        "rtm_timing_read": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "rtm_workspace_bytes": ([G, ctypes.c_int, I32, I32, ctypes.POINTER(SZ)], ctypes.c_int),
        "rtm_rbc_pad": ([G, P, U64, F, P, P, SZ, P], ctypes.c_int),
        "rtm_pad_adjoint": ([G, P, U64, F, P, P, P, SZ, P], ctypes.c_int),
        "rtm_rbc_pad_ex": ([G, P, ctypes.POINTER(RtmRbcOpts), P, P, SZ, P], ctypes.c_int),
        "rtm_pad_adjoint_ex": ([G, P, ctypes.POINTER(RtmRbcOpts), P, P, P, SZ, P], ctypes.c_int),
        "rtm_model_shot": ([G, P, D, I32, P, P, I32, P, P, P, P, U32, P, SZ, P], ctypes.c_int),
        "rtm_rtm_shot": ([G, P, D, I32, P, P, I32, P, P, F, P, P, P, ctypes.POINTER(RtmProbe), U32, P, SZ, P],
                         ctypes.c_int),
        "rtm_nyquist_stride": ([D, D, D, ctypes.POINTER(I32)], ctypes.c_int),
        "rtm_storage_count": ([I32, I32, I32, ctypes.POINTER(I64)], ctypes.c_int),
        "rtm_storage_shot": ([G, P, D, I32, P, P, I32, P, P, I32, I32, F, P, P, P, P, SZ, U32, P, SZ, P],
                             ctypes.c_int),
        "rtm_model_shot_vjp": ([G, P, D, I32, P, P, I32, P, P, P, P, U32, P, SZ, P], ctypes.c_int),
        "rtm_batch_plan": ([ctypes.c_int, I32, ctypes.POINTER(RtmShotDesc), D, I32, F, U32,
                            ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(SZ)], ctypes.c_int),
        "rtm_batch_run": ([P, P, SZ, P], ctypes.c_int),
        "rtm_batch_free": ([P], ctypes.c_int),
        "rtm_window_extract": ([I64, I64, I64, I64, P, P, P], ctypes.c_int),
        "rtm_misfit_ws_bytes": ([ctypes.POINTER(SZ)], ctypes.c_int),
        "rtm_l2_misfit": ([I64, P, P, P, P, P, SZ, P], ctypes.c_int),
        "rtm_window_accumulate": ([I64, I64, I64, I64, P, P, P], ctypes.c_int),
        "rtm_stream_copy": ([P, P, SZ, ctypes.c_int, P], ctypes.c_int),
        "rtm_set_persist_wait": ([D], ctypes.c_int),
        "rtm_get_persist_wait": ([ctypes.POINTER(D)], ctypes.c_int),
        "rtm_rtm_shot_noalloc": ([G, P, D, I32, P, P, I32, P, P, F, P, P, P, U32, P], ctypes.c_int),
        "unet_weight_pack": ([C, P, P, P, P], ctypes.c_int),
        "unet_weight_pack_many": ([ctypes.c_int32, ctypes.POINTER(UnetPackItem), P], ctypes.c_int),
        "unet_conv3d_fwd": ([C, P, P, P, I32, P, P, I32, P, P, P], ctypes.c_int),
        "unet_conv3d_dgrad": ([C, P, P, P, P], ctypes.c_int),
        "unet_conv3d_dgrad_relu": ([C, P, P, P, P, P, P], ctypes.c_int),
        "unet_wgrad_ws_bytes": ([C, ctypes.POINTER(SZ)], ctypes.c_int),
        "unet_conv3d_wgrad": ([C, P, P, P, P, P, SZ, P], ctypes.c_int),
        "unet_conv3d_wgrad_partial": ([C, P, P, P, SZ, P], ctypes.c_int),
        "unet_wgrad_reduce_many": ([ctypes.c_int32, ctypes.POINTER(UnetWgradItem), P], ctypes.c_int),
        "unet_embed": ([I64, I32, P, F, P, P], ctypes.c_int),
        "unet_pool2": ([I32] * 5 + [P, P, P], ctypes.c_int),
        "unet_up2": ([I32] * 5 + [P, P, P], ctypes.c_int),
        "unet_up2_bwd": ([I32] * 5 + [P, P, P], ctypes.c_int),
        "unet_up2_bwd_relu": ([I32] * 5 + [P, P, P, P, P], ctypes.c_int),
        "unet_relu_grad": ([I32] * 5 + [P, P, P, P, P, P], ctypes.c_int),
        "unet_mse_ws_bytes": ([I64, ctypes.POINTER(SZ)], ctypes.c_int),
        "unet_mse": ([I64, I32, P, P, P, P, P, ctypes.POINTER(D), P, SZ, P], ctypes.c_int),
        "unet_adam": ([I64, P, P, P, P, D, D, D, D, I32, P], ctypes.c_int),
        "unet_set_conv_lds": ([I32], ctypes.c_int),
        "unet_get_conv_lds": ([ctypes.POINTER(I32)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class RtmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"librtm status {status}: {message}")
        self.status = status


def check(status):
    if status != RTM_OK:
        msg = load().rtm_last_error()
        raise RtmError(status, msg.decode() if msg else "")
    return status
