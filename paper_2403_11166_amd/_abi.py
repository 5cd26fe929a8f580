"""ctypes declarations of the C ABI in include/pencil.h.

Argument marshalling only: every computation runs in libpencil.so's HIP
kernels.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpencil.so")

c_u64p = ctypes.POINTER(ctypes.c_uint64)
c_i64p = ctypes.POINTER(ctypes.c_int64)

PENCIL_OK, PENCIL_EINVAL, PENCIL_ENOMEM, PENCIL_EHIP, PENCIL_ENOISE, PENCIL_EUNSUPPORTED = range(6)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ENOISE", 5: "EUNSUPPORTED"}
X_FWD, DY_DX, X_DW, DY_DW = 0, 1, 2, 3
OP_FWD, OP_DX, OP_DW = 0, 1, 2


class Params(ctypes.Structure):
    _fields_ = [("log2_n", ctypes.c_uint32), ("num_limbs", ctypes.c_uint32), ("prime_bits", ctypes.c_uint32),
                ("flood_bits", ctypes.c_uint32), ("primes", ctypes.c_uint64 * 4), ("t", ctypes.c_uint64),
                ("seed", ctypes.c_uint64)]


class Layer(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("kind", "batch", "c_in", "c_out", "h", "w", "k", "pad", "stride")]


class Tile(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("m", "r", "k", "oh", "ow", "kh", "kw")]

    def astuple(self):
        return (self.m, self.r, self.k, self.oh, self.ow, self.kh, self.kw)


class Plan(ctypes.Structure):
    _fields_ = [("fwd", Tile), ("dx", Tile), ("dw", Tile), ("sched", ctypes.c_int32 * 3)]


class Sizes(ctypes.Structure):
    _fields_ = [("ct_bytes", ctypes.c_uint64), ("n_ct", ctypes.c_uint64 * 4), ("n_out", ctypes.c_uint64 * 3),
                ("n_pt", ctypes.c_uint64 * 3), ("n_products", ctypes.c_uint64 * 3),
                ("ws_fwd_bytes", ctypes.c_uint64), ("ws_bwd_bytes", ctypes.c_uint64),
                ("ws_dec_bytes", ctypes.c_uint64), ("ws_enc_bytes", ctypes.c_uint64)]


class Info(ctypes.Structure):
    _fields_ = [("log2_n", ctypes.c_uint32), ("num_limbs", ctypes.c_uint32), ("flood_bits", ctypes.c_uint32),
                ("ntt_loge", ctypes.c_uint32), ("primes", ctypes.c_uint64 * 4), ("psi", ctypes.c_uint64 * 4),
                ("t", ctypes.c_uint64), ("seed", ctypes.c_uint64)]


class Noise(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("product_bits", "flood_bits", "budget_bits", "margin_bits",
                                               "smudge_bits")]


class StepIO(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("ct_x1", "ct_dy_dx", "ct_x_dw", "ct_dy_dw", "x0", "dy0", "w", "bias",
                                                "ct_y", "ct_dx", "ct_dw", "y0", "dx0", "dw_mask")]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


# name -> (restype, argtypes)
SIGNATURES = {
    "pencil_ctx_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_void_p)]),
    "pencil_ctx_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pencil_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "pencil_ctx_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Info)]),
    "pencil_export_keys": (ctypes.c_int, [ctypes.c_void_p, c_i64p, c_u64p]),
    "pencil_plan_auto": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Layer), ctypes.POINTER(Plan)]),
    "pencil_layout": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Layer), ctypes.POINTER(Plan),
                                     ctypes.POINTER(Sizes)]),
    "pencil_encrypt": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Layer), ctypes.POINTER(Plan), ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                      ctypes.c_void_p]),
    "pencil_linear_fwd": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Layer), ctypes.POINTER(Plan)]
                          + [ctypes.c_void_p] * 7 + [ctypes.c_uint64, ctypes.c_void_p]),
    "pencil_linear_fwd_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Layer), ctypes.POINTER(Plan)]
                                  + [ctypes.c_void_p] * 6 + [ctypes.c_uint64, ctypes.c_void_p]),
    "pencil_linear_bwd": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Layer), ctypes.POINTER(Plan)]
                          + [ctypes.c_void_p] * 11 + [ctypes.c_uint64, ctypes.c_void_p]),
    "pencil_decrypt": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Layer), ctypes.POINTER(Plan), ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pencil_decrypt_checked": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Layer), ctypes.POINTER(Plan),
                                              ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "pencil_plan_auto_n": (ctypes.c_int, [ctypes.c_uint32, ctypes.POINTER(Layer), ctypes.POINTER(Plan)]),
    "pencil_probe_mul32": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "pencil_noise_bound": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(Layer), ctypes.POINTER(Plan),
                                          ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(Noise)]),
    "pencil_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "pencil_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(KernelStat), ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_int)]),
    "pencil_zt_linear": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Layer), ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pencil_zt_combine": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pencil_zt_combine_outer": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "pencil_zt_encode": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "pencil_zt_decode": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "pencil_zt_share": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_uint64,
                                       ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pencil_bias_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Layer), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "pencil_dp_noise": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                       ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]),
    "pencil_stride_map": (ctypes.c_int, [ctypes.POINTER(Layer), ctypes.POINTER(Layer)]),
    "pencil_stride_relayout": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Layer), ctypes.c_int, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p]),
    "pencil_step_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Layer),
                                          ctypes.POINTER(Plan), ctypes.c_int, ctypes.c_uint32,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "pencil_step_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pencil_step_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "pencil_step_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "pencil_step_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(StepIO), ctypes.c_void_p]),
    "pencil_step_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "pencil_step_graph_capture": (ctypes.c_int, [ctypes.c_void_p]),
    "pencil_step_set_nonce": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "pencil_step_graph_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pencil_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Layer), ctypes.POINTER(Plan),
                                       ctypes.c_char_p]),
    "pencil_ntt_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "pencil_ntt_inverse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
}

_lib = None


def load(path=LIB_PATH):
    """Load libpencil.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2403_11166_amd.build` "
                           "(there is no fallback: every step runs in the HIP library)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PencilError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pencil status {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, ctx_handle=None):
    if status != PENCIL_OK:
        msg = load().pencil_last_error(ctx_handle)
        raise PencilError(status, msg.decode() if msg else "")
