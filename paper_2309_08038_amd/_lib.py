"""ctypes binding of librosar.so: the C structs, prototypes and status handling.

Argument marshalling only: every computation runs in the HIP kernels behind the C ABI
(include/rosar.h).  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librosar.so")

ROSAR_OK, ROSAR_ERR_INVALID_ARG, ROSAR_ERR_UNSUPPORTED, ROSAR_ERR_HIP, ROSAR_ERR_NO_MEMORY, ROSAR_ERR_WORKSPACE = range(6)
C64, C16_F16, C16_BF16 = 0, 1, 2
NEAREST, LINEAR = 0, 1

DTYPE_CODES = {"c64": C64, "f16": C16_F16, "bf16": C16_BF16}
INTERP_CODES = {"nearest": NEAREST, "linear": LINEAR}


class Geometry(C.Structure):
    _fields_ = [("n_pulses", C.c_int32), ("n_fast", C.c_int32), ("n_fft", C.c_int32), ("reserved", C.c_int32),
                ("radius_m", C.c_double), ("fc_hz", C.c_double), ("slope_hz_s", C.c_double),
                ("fs_hz", C.c_double), ("t_start_s", C.c_double), ("c_m_s", C.c_double),
                ("phi0_rad", C.c_double)]


class PolarGrid(C.Structure):
    _fields_ = [("n_range", C.c_int32), ("n_az", C.c_int32), ("r0_m", C.c_double), ("dr_m", C.c_double)]


class CartGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("x0_m", C.c_double), ("y0_m", C.c_double),
                ("dx_m", C.c_double), ("dy_m", C.c_double)]


class RcView(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("l_lo", C.c_int32), ("l_count", C.c_int32),
                ("halo", C.c_int32), ("ld", C.c_int64), ("scale", C.c_float), ("reserved", C.c_int32)]


class SparseSet(C.Structure):
    _fields_ = [("k", C.c_int32), ("window", C.c_int32), ("offsets", C.c_void_p), ("weights", C.c_void_p),
                ("w_dtype", C.c_int32), ("reserved", C.c_int32)]


class Tile(C.Structure):
    _fields_ = [("variant", C.c_int32), ("pixels_per_lane", C.c_int32), ("waves", C.c_int32),
                ("reserved", C.c_int32)]


class SasParams(C.Structure):
    _fields_ = [("iters", C.c_int32), ("max_newton", C.c_int32), ("th", C.c_double), ("phi_mw", C.c_double),
                ("d_angle", C.c_double), ("lam_b", C.c_double), ("eta", C.c_double), ("u_min", C.c_double),
                ("b_min", C.c_double), ("eps", C.c_double), ("mu", C.c_double), ("tau0", C.c_double),
                ("newton_tol", C.c_double), ("ls_alpha", C.c_double), ("ls_beta", C.c_double), ("ls_min", C.c_double)]


class RotationDesc(C.Structure):
    _fields_ = [("geom", Geometry), ("grid", PolarGrid), ("raw", C.c_void_p), ("window", C.c_void_p),
                ("y_t", C.c_void_p), ("l_lo", C.c_int32), ("l_count", C.c_int32), ("halo", C.c_int32),
                ("reserved", C.c_int32), ("ld", C.c_int64), ("set", SparseSet), ("image", C.c_void_p)]


# (name, restype, argtypes) for every symbol declared in include/rosar.h
_P = C.POINTER
PROTOTYPES = [
    ("rosar_version", C.c_char_p, []),
    ("rosar_status_str", C.c_char_p, [C.c_int]),
    ("rosar_last_error", C.c_char_p, []),
    ("rosar_range_compress", C.c_int, [_P(Geometry), C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                      C.c_int, C.c_float, C.c_void_p, C.c_int64, C.c_void_p]),
    ("rosar_sparse_filter", C.c_int, [_P(Geometry), _P(PolarGrid), _P(RcView), _P(SparseSet), C.c_void_p,
                                     C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    ("rosar_sparse_filter_tiled", C.c_int, [_P(Geometry), _P(PolarGrid), _P(RcView), _P(SparseSet), C.c_void_p,
                                           C.c_void_p, C.c_int, C.c_void_p, _P(Tile), C.c_void_p]),
    ("rosar_bp_full_workspace_size", C.c_int, [_P(Geometry), _P(C.c_size_t)]),
    ("rosar_bp_full", C.c_int, [_P(Geometry), _P(PolarGrid), _P(RcView), C.c_void_p, C.c_int, C.c_void_p,
                               C.c_void_p, C.c_size_t, C.c_void_p]),
    ("rosar_bp_full_noalloc", C.c_int, [_P(Geometry), _P(PolarGrid), _P(RcView), C.c_void_p, C.c_int, C.c_void_p,
                                       C.c_void_p]),
    ("rosar_sas_design_workspace_size", C.c_int, [_P(Geometry), _P(PolarGrid), _P(SasParams), _P(C.c_size_t),
                                                  _P(C.c_int32)]),
    ("rosar_sas_design", C.c_int, [_P(Geometry), _P(PolarGrid), _P(SasParams), C.c_void_p, C.c_int32, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("rosar_sparse_filter_backward_workspace_size", C.c_int, [_P(Geometry), _P(PolarGrid), _P(SparseSet),
                                                             _P(C.c_size_t)]),
    ("rosar_sparse_filter_backward", C.c_int, [_P(Geometry), _P(PolarGrid), _P(RcView), _P(SparseSet),
                                              C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("rosar_batch_plan_create", C.c_int, [_P(RotationDesc), C.c_int32, _P(Tile), _P(C.c_void_p)]),
    ("rosar_batch_run", C.c_int, [C.c_void_p, C.c_void_p]),
    ("rosar_batch_plan_info", C.c_int, [C.c_void_p, _P(C.c_int64), _P(C.c_int64), _P(C.c_int64)]),
    ("rosar_batch_plan_destroy", None, [C.c_void_p]),
    ("rosar_batch_autotune", C.c_int, [_P(RotationDesc), C.c_int32, C.c_int32, _P(Tile), _P(C.c_float),
                                      C.c_void_p]),
    ("rosar_autotune_sparse_filter", C.c_int, [_P(Geometry), _P(PolarGrid), _P(RcView), _P(SparseSet),
                                              C.c_void_p, C.c_int32, _P(Tile), _P(C.c_float), C.c_void_p]),
    ("rosar_sparse_plan_create", C.c_int, [_P(Geometry), _P(PolarGrid), _P(RcView), _P(SparseSet), C.c_int,
                                          _P(Tile), C.c_void_p, _P(C.c_void_p)]),
    ("rosar_sparse_plan_run", C.c_int, [C.c_void_p, _P(RcView), C.c_void_p, C.c_void_p]),
    ("rosar_sparse_plan_destroy", None, [C.c_void_p]),
    ("rosar_sparse_plan_workspace_size", C.c_int, [C.c_void_p, _P(C.c_size_t)]),
    ("rosar_sparse_plan_run_workspace", C.c_int, [C.c_void_p, _P(RcView), C.c_void_p, C.c_void_p, C.c_size_t,
                                                 C.c_void_p]),
    ("rosar_sparse_filter_cartesian", C.c_int, [_P(Geometry), _P(PolarGrid), _P(CartGrid), _P(RcView),
                                               _P(SparseSet), C.c_int, C.c_void_p, C.c_void_p]),
    ("rosar_bp_time_domain", C.c_int, [_P(Geometry), _P(PolarGrid), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                      C.c_int32, C.c_void_p, C.c_void_p]),
    ("rosar_bp_cartesian", C.c_int, [_P(Geometry), _P(CartGrid), _P(RcView), C.c_void_p, C.c_int, C.c_void_p,
                                     C.c_void_p]),
    ("rosar_sparse_filter_polar", C.c_int, [_P(Geometry), _P(PolarGrid), _P(RcView), _P(SparseSet), C.c_int,
                                            C.c_void_p, C.c_void_p]),
    ("rosar_beampattern", C.c_int, [_P(Geometry), _P(PolarGrid), _P(SparseSet), C.c_void_p, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p]),
    ("rosar_delta_r", C.c_int, [_P(Geometry), _P(PolarGrid), C.c_int32, C.c_void_p, C.c_int32, C.c_double,
                                C.c_void_p, C.c_void_p, C.c_void_p]),
    ("rosar_sas_time_domain", C.c_int, [_P(Geometry), _P(PolarGrid), C.c_void_p, C.c_void_p, _P(SparseSet),
                                       C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    ("rosar_sparse_filter_adjoint_band_workspace_size", C.c_int, [_P(Geometry), _P(PolarGrid), _P(RcView),
                                                                  _P(SparseSet), C.c_int, _P(C.c_size_t)]),
    ("rosar_sparse_filter_adjoint_band", C.c_int, [_P(Geometry), _P(PolarGrid), _P(RcView), _P(SparseSet), C.c_int,
                                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("rosar_autotune", C.c_int, [C.c_char_p]),
    ("rosar_autotune_lookup", C.c_int, [C.c_char_p, _P(Tile), _P(C.c_float), _P(C.c_int32)]),
    ("rosar_autotune_store", C.c_int, [C.c_char_p, _P(Tile), C.c_float]),
    ("rosar_sparse_plan_autotune", C.c_int, [_P(Geometry), _P(PolarGrid), _P(RcView), _P(SparseSet), C.c_int,
                                            C.c_void_p, C.c_int32, C.c_int32, _P(Tile), _P(C.c_float),
                                            C.c_void_p]),
]


PLAN_DIRECT, PLAN_FASTCONV = 1, 2


class RosarError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(message)


_lib = None


def lib():
    """The loaded librosar.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2309_08038_amd.build` "
                              "(or __graft_entry__.build()); there is no fallback implementation")
        h = C.CDLL(LIB_PATH)
        for name, res, args in PROTOTYPES:
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def check(status: int, what: str = ""):
    if status != ROSAR_OK:
        l = lib()
        name = l.rosar_status_str(status).decode()
        msg = l.rosar_last_error().decode()
        raise RosarError(status, f"{what}: {name}: {msg}" if what else f"{name}: {msg}")


def geometry(g) -> Geometry:
    """Geometry struct from any object with the rosar_geometry field names."""
    return Geometry(int(g.n_pulses), int(g.n_fast), int(g.n_fft), 0, float(g.radius_m), float(g.fc_hz),
                    float(g.slope_hz_s), float(g.fs_hz), float(g.t_start_s), float(g.c_m_s), float(g.phi0_rad))


def polar_grid(p) -> PolarGrid:
    return PolarGrid(int(p.n_range), int(p.n_az), float(p.r0_m), float(p.dr_m))
