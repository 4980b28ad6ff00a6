"""ctypes loader for libburn.so (argument marshalling only).

PyTorch is imported first so that libburn.so binds to the HIP runtime torch
already loaded (one runtime per process).  There is no fallback: if the
library is missing the import of the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (must precede the library load: shared HIP runtime)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libburn.so")

BN_SUCCESS, BN_EINVAL, BN_EHIP, BN_ENOMEM, BN_EUNSUPPORTED = 0, -1, -2, -3, -4
CELL_STATUS = {0: "OK", 1: "MAX_STEPS", 2: "STEP_UNDERFLOW", 3: "NONFINITE", 4: "BAD_INPUT"}
COUNTERS = ["n_steps", "n_rej_err", "n_newton_fail", "n_rhs", "n_jac", "n_lu", "n_solve", "order"]

# Every symbol include/burn.h declares.
EXPORTS = ["bn_network_create", "bn_network_destroy", "bn_network_n_species",
           "bn_network_n_reactions", "burn_batch", "burn_batch_ex",
           "burn_batch_multi_workspace_bytes", "burn_batch_multi_order_workspace_bytes",
           "burn_batch_multi", "burn_batch_multi_noalloc", "bn_network_autotune",
           "bn_network_set_launch", "bn_network_get_launch", "bn_network_autotune_persistent",
           "bn_network_set_persistent_launch", "bn_network_get_persistent_launch",
           "burn_batch_adjoint_workspace_bytes", "burn_batch_adjoint_states_bytes",
           "burn_batch_adjoint_forward",
           "burn_batch_adjoint_backward", "burn_batch_adjoint", "burn_batch_sdc",
           "bn_codegen_source", "bn_codegen_prebuild", "bn_network_generate",
           "bn_network_set_body", "bn_network_get_body", "bn_last_error", "bn_version"]
BODY_TABLE, BODY_GENERATED = 0, 1
MAX_ITEMS = 8


class NetworkDesc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("mass", C.POINTER(C.c_int32)), ("reactants", C.POINTER(C.c_int32)),
                ("products", C.POINTER(C.c_int32)), ("coef", C.POINTER(C.c_double)),
                ("q", C.POINTER(C.c_double)), ("c_v", C.c_double),
                ("screen", C.POINTER(C.c_double))]


def network_desc(spec):
    """(NetworkDesc, arrays it points into) for a NetworkSpec; keep the
    arrays alive while the descriptor is used."""
    import numpy as np
    arrays = [np.ascontiguousarray(spec.mass, dtype=np.int32),
              np.ascontiguousarray(spec.reactants, dtype=np.int32),
              np.ascontiguousarray(spec.products, dtype=np.int32),
              np.ascontiguousarray(spec.coef, dtype=np.float64),
              np.ascontiguousarray(spec.q, dtype=np.float64)]
    m, rs, ps, cf, q = arrays
    i32 = C.POINTER(C.c_int32)
    f64 = C.POINTER(C.c_double)
    scr = None
    if spec.screen is not None:
        scr = np.ascontiguousarray(spec.screen, dtype=np.float64)
        arrays.append(scr)
    desc = NetworkDesc(spec.n_species, spec.n_reactions, m.ctypes.data_as(i32),
                       rs.ctypes.data_as(i32), ps.ctypes.data_as(i32), cf.ctypes.data_as(f64),
                       q.ctypes.data_as(f64), spec.c_v,
                       scr.ctypes.data_as(f64) if scr is not None else None)
    return desc, arrays


class BurnOpts(C.Structure):
    _fields_ = [("max_steps", C.c_int32), ("lanes_per_cell", C.c_int32),
                ("block_waves", C.c_int32), ("order_cells", C.c_int32)]


class BatchItem(C.Structure):
    _fields_ = [("net", C.c_void_p), ("n_cells", C.c_int64), ("state", C.c_void_p),
                ("rho", C.c_void_p), ("T", C.c_void_p), ("log_mult", C.c_void_p),
                ("status", C.c_void_p), ("counters", C.c_void_p)]


class TuneResult(C.Structure):
    _fields_ = [("lanes_per_cell", C.c_int32), ("slots_per_lane", C.c_int32),
                ("block_waves", C.c_int32), ("status", C.c_int32), ("ms", C.c_double)]


class PersistentTuneResult(C.Structure):
    _fields_ = [("lanes_per_cell", C.c_int32), ("slots_per_lane", C.c_int32),
                ("waves_per_simd", C.c_int32), ("block_waves", C.c_int32),
                ("status", C.c_int32), ("ms", C.c_double)]


class BurnError(RuntimeError):
    pass


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise BurnError(f"{LIB_PATH} is not built (python -m paper_2312_02836_amd.build)")
    L = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.c_void_p, C.c_void_p
    L.bn_network_create.argtypes = [C.POINTER(NetworkDesc), C.POINTER(C.c_void_p)]
    L.bn_network_create.restype = C.c_int
    L.bn_network_destroy.argtypes = [vp]
    L.bn_network_destroy.restype = None
    L.bn_network_n_species.argtypes = [vp]
    L.bn_network_n_reactions.argtypes = [vp]
    L.burn_batch.argtypes = [vp, C.c_int64, dp, dp, dp, C.c_double, C.c_double, C.c_double, dp,
                             ip, ip, vp]
    L.burn_batch.restype = C.c_int
    L.burn_batch_ex.argtypes = [vp, C.c_int64, dp, dp, dp, C.c_double, C.c_double, C.c_double,
                                dp, ip, ip, C.POINTER(BurnOpts), vp]
    L.burn_batch_ex.restype = C.c_int
    L.burn_batch_multi_workspace_bytes.argtypes = [C.c_int32]
    L.burn_batch_multi_workspace_bytes.restype = C.c_size_t
    L.burn_batch_multi_order_workspace_bytes.argtypes = [C.c_int32, C.POINTER(BatchItem)]
    L.burn_batch_multi_order_workspace_bytes.restype = C.c_size_t
    L.burn_batch_multi.argtypes = [C.c_int32, C.POINTER(BatchItem), C.c_double, C.c_double,
                                   C.c_double, C.POINTER(BurnOpts), vp, C.c_size_t, vp]
    L.burn_batch_multi.restype = C.c_int
    L.burn_batch_multi_noalloc.argtypes = [C.c_int32, C.POINTER(BatchItem), C.c_double,
                                           C.c_double, C.c_double, C.POINTER(BurnOpts), vp]
    L.burn_batch_multi_noalloc.restype = C.c_int
    L.bn_network_autotune.argtypes = [vp, C.c_int64, dp, dp, dp, C.c_double, C.c_double,
                                      C.c_double, dp, C.c_int32, C.POINTER(TuneResult),
                                      C.c_int32, C.POINTER(C.c_int32), vp]
    L.bn_network_autotune.restype = C.c_int
    L.bn_network_autotune_persistent.argtypes = [vp, C.c_int64, dp, dp, dp, C.c_double,
                                                 C.c_double, C.c_double, dp, C.c_int32,
                                                 C.POINTER(PersistentTuneResult), C.c_int32,
                                                 C.POINTER(C.c_int32), vp]
    L.bn_network_autotune_persistent.restype = C.c_int
    L.bn_network_set_persistent_launch.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32,
                                                   C.c_int32, C.c_double]
    L.bn_network_set_persistent_launch.restype = C.c_int
    L.bn_network_get_persistent_launch.argtypes = [vp, C.POINTER(C.c_int32),
                                                   C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                                   C.POINTER(C.c_int32)]
    L.bn_network_get_persistent_launch.restype = C.c_int
    L.bn_network_set_launch.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
    L.bn_network_set_launch.restype = C.c_int
    L.bn_network_get_launch.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int32)]
    L.bn_network_get_launch.restype = C.c_int
    L.burn_batch_adjoint_workspace_bytes.argtypes = [vp, C.c_int64, C.c_int32]
    L.burn_batch_adjoint_workspace_bytes.restype = C.c_size_t
    L.burn_batch_adjoint_states_bytes.argtypes = [vp, C.c_int64]
    L.burn_batch_adjoint_states_bytes.restype = C.c_size_t
    L.burn_batch_adjoint_forward.argtypes = [vp, C.c_int64, dp, dp, dp, C.c_double, C.c_double,
                                             C.c_double, dp, C.c_int32, dp, dp, dp, ip, ip, ip,
                                             vp, C.c_size_t, vp]
    L.burn_batch_adjoint_forward.restype = C.c_int
    L.burn_batch_adjoint_backward.argtypes = [vp, C.c_int64, dp, dp, dp, C.c_double, C.c_double,
                                              C.c_double, dp, C.c_int32, dp, dp, dp, ip, vp,
                                              C.c_size_t, vp]
    L.burn_batch_adjoint_backward.restype = C.c_int
    L.burn_batch_adjoint.argtypes = [vp, C.c_int64, dp, dp, dp, C.c_double, C.c_double,
                                     C.c_double, dp, C.c_int32, dp, dp, dp, dp, dp, dp, ip, ip,
                                     ip, vp, C.c_size_t, vp]
    L.burn_batch_adjoint.restype = C.c_int
    L.burn_batch_sdc.argtypes = [vp, C.c_int64, dp, dp, dp, C.c_double, C.c_double, C.c_double,
                                 dp, dp, ip, ip, C.POINTER(BurnOpts), vp]
    L.burn_batch_sdc.restype = C.c_int
    L.bn_codegen_source.argtypes = [C.POINTER(NetworkDesc), C.c_int32, C.c_char_p, C.c_size_t,
                                    C.POINTER(C.c_size_t)]
    L.bn_codegen_source.restype = C.c_int
    L.bn_codegen_prebuild.argtypes = [C.POINTER(NetworkDesc), C.c_int32, C.c_char_p]
    L.bn_codegen_prebuild.restype = C.c_int
    L.bn_network_generate.argtypes = [vp, C.c_int32, C.c_char_p]
    L.bn_network_generate.restype = C.c_int
    L.bn_network_set_body.argtypes = [vp, C.c_int32]
    L.bn_network_set_body.restype = C.c_int
    L.bn_network_get_body.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.bn_network_get_body.restype = C.c_int
    L.bn_last_error.restype = C.c_char_p
    L.bn_version.restype = C.c_char_p
    _lib = L
    return L


def check(rc: int, what: str) -> None:
    if rc != BN_SUCCESS:
        msg = lib().bn_last_error().decode()
        raise BurnError(f"{what} failed ({rc}): {msg}")
