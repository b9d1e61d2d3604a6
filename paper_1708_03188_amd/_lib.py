"""ctypes loader for the in-tree libsgm.so.  Fails loudly when it is missing."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgm.so")

SGM_OK = 0
SGM_SHEN_DIRICHLET, SGM_SHEN_BIHARMONIC, SGM_CHEBYSHEV, SGM_SHEN_NEUMANN = 1, 2, 3, 4
SGM_LEGENDRE, SGM_LEG_DIRICHLET, SGM_LEG_NEUMANN, SGM_LEG_BIHARMONIC = 5, 6, 7, 8
SGM_R2C, SGM_C2C = 1, 2


class SgmError(RuntimeError):
    pass


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("basis", ctypes.c_int), ("N", ctypes.c_int), ("M1", ctypes.c_int),
        ("M2", ctypes.c_int), ("kind_last", ctypes.c_int), ("Ly", ctypes.c_double), ("Lz", ctypes.c_double),
        ("autotune", ctypes.c_int),
    ]


class GLDesc(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int), ("N", ctypes.POINTER(ctypes.c_int)), ("L", ctypes.c_double), ("b", ctypes.c_double),
        ("c", ctypes.c_double), ("dt", ctypes.c_double), ("scheme", ctypes.c_int), ("graph", ctypes.c_int),
        ("tune", ctypes.c_int),
    ]


class FNODesc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int), ("W", ctypes.c_int), ("width", ctypes.c_int), ("modes", ctypes.c_int),
                ("layers", ctypes.c_int), ("hidden", ctypes.c_int), ("max_batch", ctypes.c_int)]


class FNOStats(ctypes.Structure):
    _fields_ = [("n_checked", ctypes.c_int), ("n_fallback", ctypes.c_int), ("max_rel_l2", ctypes.c_float),
                ("mean_rel_l2", ctypes.c_float), ("n_batch_fallback", ctypes.c_int), ("n_replaced", ctypes.c_int)]


SGM_RK4, SGM_IFRK4 = 1, 2
_lib = None

_vp = ctypes.c_void_p
_SIGS = {
    "sgm_version": ([], ctypes.c_int),
    "sgm_last_error": ([], ctypes.c_char_p),
    "sgm_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "sgm_plan_create": ([ctypes.POINTER(PlanDesc), _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "sgm_plan_destroy": ([_vp], ctypes.c_int),
    "sgm_plan_shapes": ([_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "sgm_forward": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "sgm_backward": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "sgm_backward_noalloc": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "sgm_plan_points": ([_vp, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "sgm_autotune_forget": ([], ctypes.c_int),
    "sgm_autotune_cache_path": ([ctypes.c_char_p, ctypes.c_int], ctypes.c_int),
    "sgm_project_derivative": ([_vp, _vp, ctypes.POINTER(ctypes.c_int), _vp, _vp, _vp], ctypes.c_int),
    "sgm_scalar_product": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "sgm_helmholtz_solve": ([_vp, ctypes.c_double, _vp, _vp, _vp], ctypes.c_int),
    "sgm_helmholtz_solve_physical": ([_vp, ctypes.c_double, _vp, _vp, _vp], ctypes.c_int),
    "sgm_biharmonic_solve": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "sgm_plan_timing": ([_vp, ctypes.c_int], ctypes.c_int),
    "sgm_plan_variants": ([_vp, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "sgm_gl_create": ([ctypes.POINTER(GLDesc), _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "sgm_gl_destroy": ([_vp], ctypes.c_int),
    "sgm_gl_offsets": ([_vp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "sgm_gl_count": ([_vp, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "sgm_gl_variant": ([_vp, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "sgm_fno_advance_checked": ([_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_uint64, _vp, _vp], ctypes.c_int),
    "sgm_gl_forward": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "sgm_gl_backward": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "sgm_gl_rhs": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "sgm_gl_step": ([_vp, _vp, ctypes.c_int, _vp], ctypes.c_int),
    "sgm_fno_create": ([ctypes.POINTER(FNODesc), ctypes.c_uint64, ctypes.POINTER(_vp)], ctypes.c_int),
    "sgm_fno_destroy": ([_vp], ctypes.c_int),
    "sgm_fno_num_params": ([_vp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "sgm_fno_set_params": ([_vp, _vp], ctypes.c_int),
    "sgm_fno_get_params": ([_vp, _vp], ctypes.c_int),
    "sgm_plan_solve_layout": ([_vp, _vp, _vp], ctypes.c_int),
    "sgm_plan_set_solve_rows": ([_vp, ctypes.c_int], ctypes.c_int),
    "sgm_fno_infer": ([_vp, _vp, _vp, ctypes.c_int, _vp], ctypes.c_int),
    "sgm_fno_set_ensemble": ([_vp, ctypes.c_int], ctypes.c_int),
    "sgm_fno_grads": ([_vp, _vp, _vp, ctypes.c_int, _vp, _vp, _vp], ctypes.c_int),
    "sgm_fno_train_step": ([_vp, _vp, _vp, ctypes.c_int, ctypes.c_float, _vp, _vp], ctypes.c_int),
    "sgm_fno_rel_l2": ([_vp, _vp, _vp, ctypes.c_int, _vp, _vp], ctypes.c_int),
    "sgm_fno_save": ([_vp, ctypes.c_char_p], ctypes.c_int),
    "sgm_fno_load": ([_vp, ctypes.c_char_p], ctypes.c_int),
    "sgm_fno_pack": ([_vp, _vp, ctypes.c_int64, _vp], ctypes.c_int),
    "sgm_fno_unpack": ([_vp, _vp, ctypes.c_int64, _vp], ctypes.c_int),
    "sgm_plan_pass_times": ([_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), ctypes.c_int],
                            ctypes.c_int),
}
NPASS = 8
SGM_TIMING_ONLY = 0x100
PASS_NAMES = ["last_fwd", "last_bwd", "mid_fwd", "mid_bwd", "cheb_fwd", "cheb_scalar", "cheb_bwd", "solve"]


def load():
    """Load libsgm.so (built by __graft_entry__.build() / paper_1708_03188_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SgmError(f"libsgm.so not found at {LIB_PATH}; build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status, what=""):
    if status != SGM_OK:
        lib = load()
        raise SgmError(f"{what}: {lib.sgm_status_string(status).decode()} ({lib.sgm_last_error().decode()})")
