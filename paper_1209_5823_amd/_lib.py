"""ctypes binding of libsvconv.so (the C ABI in include/svconv.h).

Loading fails loudly (ImportError) when the library has not been built:
there is no fallback implementation.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsvconv.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, ENOTSPD = 0, -1, -2, -3, -4, -5
FP32, BF16, FP16, BF16X3, FP16X2, FP16X3 = 0, 1, 2, 3, 4, 5
FORM_BASIS, FORM_REGROUPED, FORM_SEPARABLE, FORM_SEPARABLE_REGROUPED = 0, 1, 2, 3

PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp16": FP16, "bf16x3": BF16X3,
              "fp16x2": FP16X2, "fp16x3": FP16X3}
FORMS = {"basis": FORM_BASIS, "regrouped": FORM_REGROUPED, "separable": FORM_SEPARABLE,
         "separable_regrouped": FORM_SEPARABLE_REGROUPED}

_vp = ctypes.c_void_p
_i = ctypes.c_int

# name -> (restype, argtypes); mirrors include/svconv.h
SIGNATURES = {
    "svconv_plan_create": (_i, [ctypes.POINTER(_vp), _i, _i, _i, _i,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i), _i, _i]),
    "svconv_plan_create_dfb": (_i, [ctypes.POINTER(_vp), _i, _i, _i, _i, _i]),
    "svconv_plan_set_frame": (_i, [_vp, _i, _i, _i, _i]),
    "svconv_plan_set_stream": (_i, [_vp, _vp]),
    "svconv_plan_set_precision": (_i, [_vp, _i]),
    "svconv_plan_set_form": (_i, [_vp, _i]),
    "svconv_plan_set_pedestal": (_i, [_vp, ctypes.c_float]),
    "svconv_plan_sizes": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "svconv_plan_get_basis": (_i, [_vp, ctypes.POINTER(ctypes.c_double)]),
    "svconv_plan_destroy": (_i, [_vp]),
    "svconv_forward": (_i, [_vp, _vp, _vp, _vp]),
    "svconv_difference": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "svconv_backward": (_i, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "svconv_loss_grad": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "svconv_normal_matrix": (_i, [_vp, _vp, _vp, _vp]),
    "svconv_cholesky_factor": (_i, [_vp, _vp, _i]),
    "svconv_cholesky_solve": (_i, [_vp, _vp, _vp, _vp, _i]),
    "svconv_gn_step": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]),
    "svconv_normal_equations": (_i, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "svconv_ls_step": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]),
    "svconv_stamp_mask": (_i, [_vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _i, _i,
                               _i, _vp, ctypes.POINTER(_i)]),
    "svconv_plan_set_background": (_i, [_vp, _i]),
    "svconv_add_background": (_i, [_vp, _vp, _vp]),
    "svconv_pcg_fit": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _vp, _vp, _vp,
                            ctypes.POINTER(ctypes.c_double)]),
    "svconv_host_alloc": (_i, [ctypes.c_size_t, ctypes.POINTER(_vp)]),
    "svconv_host_free": (_i, [_vp]),
    "svconv_pipeline_create": (_i, [_vp, _i, ctypes.POINTER(_vp)]),
    "svconv_pipeline_run": (_i, [_vp, _i, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                 ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "svconv_pipeline_destroy": (_i, [_vp]),
    "svconv_difference_noalloc": (_i, [_i, _i, _i, _i, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(_i), _i, _i, ctypes.c_float, _vp, _vp, _vp, _vp,
                                       _vp]),
    "svconv_strerror": (ctypes.c_char_p, [_i]),
    "svconv_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """The loaded library; raises ImportError if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsvconv.so is not built (run __graft_entry__.build() or "
                              "python -m paper_1209_5823_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class SvconvError(RuntimeError):
    def __init__(self, status, where):
        lib = load()
        detail = lib.svconv_last_error().decode()
        msg = "%s: %s (%d)%s" % (where, lib.svconv_strerror(status).decode(), status,
                                 (": " + detail) if detail else "")
        super().__init__(msg)
        self.status = status


def check(status, where):
    if status != OK:
        raise SvconvError(status, where)
    return status
