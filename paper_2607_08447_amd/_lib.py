"""ctypes declarations of the C ABI in include/hkp.h (argument marshalling only).

The shared library is built in-tree by paper_2607_08447_amd/build.py.  There is
no fallback: if libhkp.so is missing or fails to load, importing this module
raises.
"""

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# HKP_LIB selects another build of the library (the sanitizer build in the
# CPU tests of the host-side argument checks)
LIB_PATH = os.environ.get("HKP_LIB") or os.path.join(_HERE, "libhkp.so")

HKP_OK = 0
HKP_W_NOT_CONVERGED = 1
HKP_E_ARG = -1
HKP_E_WORKSPACE = -2
HKP_E_NUMERICAL = -3
HKP_E_HIP = -4
HKP_E_UNSUPPORTED = -5
HKP_NB_MAX = 64
HKP_PREC_FP64 = 0
HKP_PREC_MIXED = 1
HKP_PRECOND_MULTIGRID = 0
HKP_PRECOND_JACOBI = 1
HKP_FLAG_X0 = 1
HKP_FLAG_GRAPH = 2
HKP_FLAG_NO_FP64_POLISH = 4
HKP_FLAG_NO_LOCK = 8
HKP_FLAG_X0_NEV = 16
HKP_FLAG_PSI_BLOCK = 32
HKP_FLAG_SPIN_FREE = 64
HKP_FLAG_CHEB_PRODUCT = 128
HKP_SP_PHI0 = 1
HKP_SP_EXACT_EIG = 2


class hkp_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h_nm", C.c_double)]


class hkp_material(C.Structure):
    _fields_ = [("gamma1", C.c_double), ("gamma2", C.c_double), ("gamma3", C.c_double),
                ("delta_so_eV", C.c_double), ("kappa", C.c_double), ("a_v_eV", C.c_double),
                ("b_eV", C.c_double), ("d_eV", C.c_double)]


class hkp_opts(C.Structure):
    _fields_ = [("nev", C.c_int32), ("nb", C.c_int32), ("degree", C.c_int32),
                ("max_iter", C.c_int32), ("tol_eV", C.c_double), ("precision", C.c_int32),
                ("flags", C.c_int32), ("seed", C.c_uint64)]


class hkp_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("n_converged", C.c_int32), ("n_hx_fp64", C.c_int64),
                ("n_hx_fp32", C.c_int64), ("fp64_switch_iter", C.c_int32), ("nb", C.c_int32),
                ("degree", C.c_int32), ("seconds", C.c_double), ("t_setup", C.c_double),
                ("t_filter", C.c_double), ("t_orth", C.c_double), ("t_rr", C.c_double),
                ("t_resid", C.c_double), ("lambda_max_bound", C.c_double),
                ("hx_bytes", C.c_double), ("n_stencil32", C.c_int64), ("n_stencil64", C.c_int64),
                ("t_stencil32", C.c_double), ("t_stencil64", C.c_double),
                ("bytes_stencil32", C.c_double), ("bytes_stencil64", C.c_double),
                ("n_stencil32x2", C.c_int64), ("t_stencil32x2", C.c_double),
                ("bytes_stencil32x2", C.c_double),
                ("n_graph_launches", C.c_int32), ("n_host_syncs", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class hkp_tune(C.Structure):
    _fields_ = [("tile_y", C.c_int32), ("vgroup", C.c_int32), ("dma", C.c_int32),
                ("two_step_tx", C.c_int32), ("two_step_ty", C.c_int32),
                ("reserved", C.c_int32), ("us_per_step", C.c_double), ("gbps", C.c_double),
                ("us_per_step_two", C.c_double)]


class hkp_pgrid(C.Structure):
    _fields_ = [("px", C.c_int32), ("py", C.c_int32), ("pz", C.c_int32), ("ox", C.c_int32),
                ("oy", C.c_int32), ("oz", C.c_int32)]


class hkp_sp_opts(C.Structure):
    _fields_ = [("n_holes", C.c_double), ("temperature_K", C.c_double), ("mixing", C.c_double),
                ("history", C.c_int32), ("max_iter", C.c_int32), ("tol_V", C.c_double),
                ("cg_tol", C.c_double), ("cg_max_iter", C.c_int32), ("flags", C.c_int32),
                ("anneal_K", C.c_double)]


class hkp_sp_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("delta_V", C.c_double),
                ("mu_eV", C.c_double), ("f_last", C.c_double), ("cg_iters", C.c_int64),
                ("schroedinger_iters", C.c_int32), ("solve_status", C.c_int32),
                ("poisson_status", C.c_int32), ("nb", C.c_int32), ("seconds", C.c_double),
                ("t_schroedinger", C.c_double), ("t_poisson", C.c_double),
                ("anneal_iters", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class hkp_ci_stats(C.Structure):
    _fields_ = [("cg_iters", C.c_int64), ("cg_relres", C.c_double),
                ("poisson_solves", C.c_int32), ("determinants", C.c_int32),
                ("t_poisson", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class hkp_gmatrix_result(C.Structure):
    _fields_ = [("g", C.c_double * 36), ("g_sym", C.c_double * 36), ("centre_nm", C.c_double * 12),
                ("kramers", C.c_double * 12), ("E_eV", C.c_double * 4), ("delta_eV", C.c_double),
                ("t_eV", C.c_double), ("d_nm", C.c_double)]


class hkp_st_opts(C.Structure):
    _fields_ = [("n_so", C.c_double * 3), ("lambda_so_nm", C.c_double), ("d_nm", C.c_double)]


class hkp_st_point(C.Structure):
    _fields_ = [("bbar_eV", C.c_double * 3), ("dbar_eV", C.c_double * 3), ("dEz_eV", C.c_double),
                ("E_eV", C.c_double * 5), ("Jtilde_eV", C.c_double * 9),
                ("J_perp_eV", C.c_double), ("J_par_eV", C.c_double)]


class hkp_iter_info(C.Structure):
    _fields_ = [("iter", C.c_int32), ("batch", C.c_int32), ("nb", C.c_int32), ("nev", C.c_int32),
                ("nconv", C.POINTER(C.c_int32)), ("fp64", C.POINTER(C.c_int32)),
                ("ritz_eV", C.POINTER(C.c_double)), ("resid_eV", C.POINTER(C.c_double))]


HKP_ITER_FN = C.CFUNCTYPE(C.c_int, C.POINTER(hkp_iter_info), C.c_void_p)

_P = C.c_void_p
_D = C.POINTER(C.c_double)

SIGNATURES = {
    "hkp_default_material": (None, [C.POINTER(hkp_material)]),
    "hkp_unit_constants": (None, [C.POINTER(C.c_double)]),
    "hkp_default_opts": (None, [C.POINTER(hkp_opts)]),
    "hkp_workspace_bytes": (C.c_size_t, [C.POINTER(hkp_grid), C.POINTER(hkp_opts), C.c_int32]),
    "hkp_block_size": (C.c_int32, [C.POINTER(hkp_grid), C.POINTER(hkp_opts)]),
    "hkp_solve": (C.c_int, [C.POINTER(hkp_grid), C.POINTER(hkp_material), C.POINTER(hkp_opts),
                            _P, _P, _D, _P, _P, _P, _P, _P, C.c_size_t, _P,
                            C.POINTER(hkp_stats)]),
    "hkp_solve_batch": (C.c_int, [C.POINTER(hkp_grid), C.POINTER(hkp_material),
                                  C.POINTER(hkp_opts), C.c_int32, _P, _P, _D, _P, _P, _P, _P,
                                  _P, C.c_size_t, _P, C.POINTER(hkp_stats)]),
    "hkp_apply_workspace_bytes": (C.c_size_t, [C.POINTER(hkp_grid), C.c_int32]),
    "hkp_filter_step": (C.c_int, [C.POINTER(hkp_grid), C.POINTER(hkp_material), _P, _P, _D,
                                  C.c_int32, _P, _P, _P, C.c_double, C.c_double, C.c_double,
                                  C.c_int32, _P, C.c_size_t, _P]),
    "hkp_filter_step2_workspace_bytes": (C.c_size_t, [C.POINTER(hkp_grid), C.c_int32]),
    "hkp_filter_step2": (C.c_int, [C.POINTER(hkp_grid), C.POINTER(hkp_material), _P, _P,
                                   C.POINTER(C.c_double), C.c_int32, _P, _P, _P, _P,
                                   C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), _P, C.c_size_t, _P,
                                   C.POINTER(C.c_int32)]),
    "hkp_apply": (C.c_int, [C.POINTER(hkp_grid), C.POINTER(hkp_material), _P, _P, _D, C.c_int32,
                            _P, _P, C.c_int32, _P, C.c_size_t, _P]),
    "hkp_gate_potential": (C.c_int, [C.c_int64, C.c_int32, _P, _P, _P, _P, _P]),
    "hkp_hf_grad_workspace_bytes": (C.c_size_t, [C.c_int32]),
    "hkp_hf_grad": (C.c_int, [C.c_int64, C.c_int32, _P, _P, C.c_int32, _P, _P, _P, C.c_size_t,
                              _P]),
    "hkp_hf_grad_noalloc": (C.c_int, [C.c_int64, C.c_int32, _P, _P, C.c_int32, _P, _P, _P]),
    "hkp_autotune": (C.c_int, [C.POINTER(hkp_grid), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                               _P, C.c_size_t, _P, C.POINTER(hkp_tune)]),
    "hkp_autotune_block": (C.c_int, [C.POINTER(hkp_grid), C.POINTER(hkp_material),
                                     C.POINTER(hkp_opts), _P, _P, _D, C.POINTER(C.c_int32),
                                     C.c_int32, _P, C.c_size_t, _P, C.POINTER(C.c_int32), _D]),
    "hkp_tuned_shape": (C.c_int, [C.POINTER(hkp_grid), C.c_int32, C.c_int32, C.c_int32,
                                  C.c_int32, C.POINTER(hkp_tune)]),
    "hkp_tune_cache_save": (C.c_int, [C.c_char_p]),
    "hkp_tune_cache_load": (C.c_int, [C.c_char_p]),
    "hkp_tune_cache_clear": (None, []),
    "hkp_soi_workspace_bytes": (C.c_size_t, [C.POINTER(hkp_grid), C.c_int32]),
    "hkp_soi_matrix": (C.c_int, [C.POINTER(hkp_grid), C.c_int32, _P, _P, C.c_double, _P, _P,
                                 C.c_size_t, _P]),
    "hkp_ci_workspace_bytes": (C.c_size_t, [C.POINTER(hkp_grid), C.c_int32,
                                            C.POINTER(hkp_pgrid)]),
    "hkp_ci_solve": (C.c_int, [C.POINTER(hkp_grid), C.c_int32, _P, _P, C.c_double,
                               C.POINTER(hkp_pgrid), _P, _P, C.c_double, C.c_int32, _P, _P, _P,
                               _P, _P, _P, C.c_size_t, _P, C.POINTER(hkp_ci_stats)]),
    "hkp_poisson_workspace_bytes": (C.c_size_t, [C.POINTER(hkp_pgrid)]),
    "hkp_poisson": (C.c_int, [C.POINTER(hkp_pgrid), C.c_double, _P, _P, _P, _P, _P, C.c_double,
                              C.c_int32, _P, C.c_size_t, _P, C.POINTER(C.c_int32), _D]),
    "hkp_occupancy": (C.c_int, [C.c_int32, _P, C.c_double, C.c_double, _P, _P, _P]),
    "hkp_hole_density": (C.c_int, [C.POINTER(hkp_grid), C.c_int32, _P, _P, _P, _P]),
    "hkp_sp_workspace_bytes": (C.c_size_t, [C.POINTER(hkp_grid), C.POINTER(hkp_opts),
                                            C.POINTER(hkp_pgrid), C.POINTER(hkp_sp_opts)]),
    "hkp_sp_solve": (C.c_int, [C.POINTER(hkp_grid), C.POINTER(hkp_material), C.POINTER(hkp_opts),
                               C.POINTER(hkp_pgrid), C.POINTER(hkp_sp_opts), _P, _P, _D, _P, _P,
                               _P, _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P,
                               C.POINTER(hkp_sp_stats)]),
    "hkp_gmatrix_workspace_bytes": (C.c_size_t, [C.POINTER(hkp_grid)]),
    "hkp_gmatrix": (C.c_int, [C.POINTER(hkp_grid), C.POINTER(hkp_material), _P, _P, _P, _P, _P,
                              C.c_size_t, _P]),
    "hkp_st_model": (C.c_int, [_P, _P, C.POINTER(hkp_st_opts), C.c_int32, _P, _P, _P, _P]),
    "hkp_poisson_preconditioner": (C.c_int, [C.c_int32]),
    "hkp_set_iter_callback": (None, [HKP_ITER_FN, C.c_void_p]),
    "hkp_last_error": (C.c_char_p, []),
    "hkp_version": (C.c_int, []),
}


def load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2607_08447_amd.build` "
            "(there is no CPU fallback)")
    # torch first: the library then binds to the HIP runtime torch has loaded
    # (one HIP/HSA runtime per process; a second copy would see no device)
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load()


class HkpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hkp error {code}: {msg}")
        self.code = code


def check(code):
    if code < 0:
        raise HkpError(code, lib.hkp_last_error().decode())
    return code
