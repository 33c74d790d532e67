"""ctypes view of libpsvd.so (the C ABI of include/psvd.h).

Argument marshalling only: every numerical step runs in the HIP library.
Loading fails loudly when the library has not been built; there is no
fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsvd.so")

PSVD_OK = 0
STATUS = {
    0: "PSVD_OK", -1: "PSVD_E_INVAL", -2: "PSVD_E_SHAPE", -3: "PSVD_E_DTYPE", -4: "PSVD_E_NOMEM",
    -5: "PSVD_E_NONFINITE", -6: "PSVD_E_NOCONV", -7: "PSVD_E_BREAKDOWN", -8: "PSVD_E_DEVICE", -9: "PSVD_E_STATE",
}
globals().update({name: code for code, name in STATUS.items()})   # PSVD_E_INVAL = -1, ...
PSVD_F32, PSVD_F64 = 1, 2
DETERMINISTIC, RANDOMIZED = 0, 1
PREC_FP64, PREC_FP32, PREC_MIXED, PREC_BF16 = 0, 1, 2, 3
OPT_ASYNC, OPT_NO_FALLBACK, OPT_PROFILE, OPT_OMEGA_BF16, OPT_GRAPH = 1, 2, 4, 8, 16
KERNEL_CLASSES = ["fused_bf16", "fused_f32", "lift", "tn", "nn", "small", "small_svd", "split", "split3", "wide"]

EXPORTS = [
    "psvd_default_options", "psvd_initialize", "psvd_incorporate_data", "psvd_rank", "psvd_singular_values",
    "psvd_modes", "psvd_modes_ptr", "psvd_get_omega", "psvd_stats", "psvd_last_error", "psvd_status_string",
    "psvd_finalize", "psvd_reset_stats", "psvd_apmos_batched", "psvd_stream_backward", "psvd_loss_grad",
    "psvd_save_state", "psvd_load_state", "psvd_rsvd", "psvd_pstream_initialize", "psvd_pstream_incorporate",
    "psvd_pstream_modes_ptr", "psvd_pstream_modes", "psvd_rsvd_noalloc", "psvd_apmos_low_rank",
    "psvd_set_tuning",
]


class Options(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int32), ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("stream", ctypes.c_void_p), ("max_sweeps", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("tile_rows", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32), ("panel_width", ctypes.c_int32),
        ("split_m", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("batches", ctypes.c_int64), ("fallbacks", ctypes.c_int64), ("last_sweeps", ctypes.c_int32),
        ("last_path", ctypes.c_int32), ("last_update_ms", ctypes.c_double),
        ("kernel_launches", ctypes.c_int64 * 10), ("kernel_ms", ctypes.c_double * 10),
    ]


class PsvdError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        super().__init__(f"{STATUS.get(code, code)}: {msg}" if msg else STATUS.get(code, str(code)))


_lib = None


def load():
    """Load libpsvd.so (raises if it is missing: no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or paper_2108_08845_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    H = ctypes.c_void_p
    lib.psvd_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.psvd_default_options.restype = None
    lib.psvd_initialize.argtypes = [ctypes.POINTER(H), i64, i32, ctypes.c_double, i32, i32, ctypes.POINTER(Options)]
    lib.psvd_incorporate_data.argtypes = [H, vp, i64, i64, i64, i32]
    lib.psvd_rank.argtypes = [H, ctypes.POINTER(i32)]
    lib.psvd_singular_values.argtypes = [H, dp, i32, ctypes.POINTER(i32)]
    lib.psvd_modes.argtypes = [H, vp, i64, i32]
    lib.psvd_modes_ptr.argtypes = [H, ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(i32)]
    lib.psvd_get_omega.argtypes = [H, i64, i64, dp]
    lib.psvd_stats.argtypes = [H, ctypes.POINTER(Stats)]
    lib.psvd_set_tuning.argtypes = [H, i32, i32, i32, i32]
    lib.psvd_reset_stats.argtypes = [H]
    lib.psvd_last_error.argtypes = [H]
    lib.psvd_last_error.restype = ctypes.c_char_p
    lib.psvd_status_string.argtypes = [ctypes.c_int]
    lib.psvd_status_string.restype = ctypes.c_char_p
    lib.psvd_finalize.argtypes = [H]
    lib.psvd_finalize.restype = None
    lib.psvd_apmos_batched.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(i64), i64, i32,
                                       i32, i32, ctypes.POINTER(vp), ctypes.POINTER(i64), dp, dp, vp]
    lib.psvd_apmos_low_rank.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(i64), i64, i32,
                                        i32, i32, i32, ctypes.c_uint64, ctypes.POINTER(vp), ctypes.POINTER(i64), dp, dp,
                                        vp]
    lib.psvd_stream_backward.argtypes = [vp, i64, i64, i32, i32, i64, i32, ctypes.c_double, vp, dp, vp, vp]
    lib.psvd_loss_grad.argtypes = [vp, i64, i64, i32, i32, i64, i32, ctypes.c_double, dp, dp, vp, vp]
    lib.psvd_save_state.argtypes = [H, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    lib.psvd_load_state.argtypes = [H, vp, ctypes.c_size_t]
    lib.psvd_rsvd.argtypes = [vp, i64, i64, i64, i32, i32, i32, i32, ctypes.c_uint64, i32, vp, i64, vp, i64, i32, dp,
                              ctypes.POINTER(i32), vp]
    lib.psvd_rsvd_noalloc.argtypes = lib.psvd_rsvd.argtypes
    lib.psvd_pstream_initialize.argtypes = [ctypes.POINTER(H), i32, ctypes.POINTER(i64), i32, ctypes.c_double, i32,
                                            ctypes.POINTER(Options)]
    lib.psvd_pstream_incorporate.argtypes = [H, ctypes.POINTER(vp), ctypes.POINTER(i64), i64, i32]
    lib.psvd_pstream_modes_ptr.argtypes = [H, i32, ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(i32)]
    lib.psvd_pstream_modes.argtypes = [H, i32, vp, i64]
    _lib = lib
    return lib


def check(rc, handle=None, what=""):
    if rc != PSVD_OK:
        msg = ""
        if handle is not None:
            msg = load().psvd_last_error(handle).decode()
        raise PsvdError(rc, f"{what} {msg}".strip())
