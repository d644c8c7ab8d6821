"""ctypes binding of libfspb.so (the C ABI in include/fspb.h).

Argument marshalling only: every step of the dose computation runs in the
library's HIP kernels.  Importing this module fails loudly when the library
has not been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

PKG = Path(__file__).resolve().parent
LIB_PATH = Path(os.environ.get("FSPB_LIBRARY", PKG / "libfspb.so"))

FSPB_OK = 0
FSPB_E_ARG = -1
FSPB_E_HIP = -2
FSPB_E_NOMEM = -3
FSPB_E_STATE = -4
FSPB_E_UNSUPPORTED = -5
FSPB_SCHEDULE_THROUGHPUT = 0
FSPB_SCHEDULE_LATENCY = 1


class fspb_ct(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_float), ("dy", C.c_float), ("dz", C.c_float),
                ("ox", C.c_float), ("oy", C.c_float), ("oz", C.c_float),
                ("density", C.c_void_p)]


class fspb_beam(C.Structure):
    _fields_ = [("gantry", C.c_float), ("couch", C.c_float), ("iso", C.c_float * 3),
                ("sad", C.c_float), ("nbx", C.c_int), ("nby", C.c_int),
                ("wx", C.c_float), ("wy", C.c_float), ("cx", C.c_float), ("cy", C.c_float)]


class fspb_table1d(C.Structure):
    _fields_ = [("start", C.c_float), ("step", C.c_float), ("n", C.c_int),
                ("v", C.POINTER(C.c_float))]


class fspb_tables(C.Structure):
    _fields_ = [("A", fspb_table1d), ("n_theta", C.c_int), ("theta_step", C.c_float)] + [
        (n, fspb_table1d) for n in ("u1x", "u1y", "u2x", "u2y", "w1", "w2",
                                    "fu1", "fu2", "fw1", "fw2", "b1", "b2")]


class fspb_options(C.Structure):
    _fields_ = [("roi_radius", C.c_float), ("rho_surface", C.c_float),
                ("smooth_sigma", C.c_float), ("rho_min", C.c_float), ("rho_max", C.c_float),
                ("sample_step", C.c_float), ("dc_enabled", C.c_int), ("flags", C.c_int),
                ("tile_shape", C.c_int), ("tile_waves", C.c_int), ("schedule", C.c_int)]


class fspb_info(C.Structure):
    _fields_ = [("n_beams", C.c_int), ("n_beamlets", C.c_int), ("nx", C.c_int),
                ("ny", C.c_int), ("nz", C.c_int), ("n_vox", C.c_longlong),
                ("k_stride", C.c_int), ("k_max", C.c_int), ("n_hit", C.c_int),
                ("n_entry_ambiguous", C.c_int), ("smooth_radius", C.c_int * 3),
                ("sample_step", C.c_float), ("dc_enabled", C.c_int),
                ("device_bytes", C.c_longlong), ("drift_tables", C.c_int),
                ("drift_ratio", C.c_float)]


class fspb_beamlet_info(C.Structure):
    _fields_ = [("hit", C.c_int), ("k_entry", C.c_int), ("n_samples", C.c_int), ("K", C.c_int),
                ("s_in", C.c_double), ("s_entry", C.c_double), ("theta", C.c_double),
                ("src", C.c_double * 3), ("dir", C.c_double * 3), ("ex", C.c_double * 3),
                ("ey", C.c_double * 3), ("entry_margin", C.c_double),
                ("pair_t", C.c_float * 4), ("pair_x", C.c_float * 4), ("pair_y", C.c_float * 4)]


class fspb_tune_result(C.Structure):
    _fields_ = [("shape", C.c_int), ("dims", C.c_int * 3), ("waves_per_block", C.c_int),
                ("ms", C.c_float), ("per_beam", C.c_int)]


class fspb_adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class fspb_surrogate_guard(C.Structure):
    _fields_ = [("rho_lo", C.c_float), ("rho_hi", C.c_float), ("het_max", C.c_float),
                ("band_lo", C.c_float * 6), ("band_hi", C.c_float * 6)]


class fspb_gamma_params(C.Structure):
    _fields_ = [("dist", C.c_float), ("dose_frac", C.c_float), ("gamma_cap", C.c_float),
                ("dose_max", C.c_float), ("iso_frac", C.c_float)]


class fspb_gamma_stats(C.Structure):
    _fields_ = [("gamma_max", C.c_double), ("gamma_avg_iso", C.c_double),
                ("pass_rate_iso", C.c_double), ("dose_max", C.c_double), ("n_iso", C.c_longlong)]


FSPB_FLAG_SIDDON = 1
FSPB_MLP_IN, FSPB_MLP_IN_PAD, FSPB_MLP_HIDDEN, FSPB_MLP_OUT = 202, 224, 64, 6
FSPB_MLP_PARAMS = 17542
FSPB_MLP_MAX_ROWS = 1 << 22

# name -> (restype, argtypes); the list of every symbol include/fspb.h declares
SIGNATURES = {
    "fspb_create_geometry": (C.c_int, [C.POINTER(fspb_ct), C.c_int, C.POINTER(fspb_beam),
                                       C.POINTER(fspb_tables), C.POINTER(fspb_options),
                                       C.c_void_p, C.POINTER(C.c_void_p)]),
    "fspb_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fspb_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fspb_beamlet_pair_counts": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fspb_set_adjoint_slab": (C.c_int, [C.c_void_p, C.c_int]),
    "fspb_get_adjoint_slab": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "fspb_autotune_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                        C.POINTER(C.c_int), C.POINTER(C.c_float), C.c_int,
                                        C.POINTER(C.c_int)]),
    "fspb_count_pairs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.POINTER(C.c_ulonglong), C.c_void_p]),
    "fspb_count_pairs_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fspb_set_dc": (C.c_int, [C.c_void_p, C.c_int]),
    "fspb_geometry_info": (C.c_int, [C.c_void_p, C.POINTER(fspb_info)]),
    "fspb_drift_tables": (C.c_int, [C.POINTER(fspb_tables), C.POINTER(C.c_float)]),
    "fspb_smoothed_density": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fspb_beamlet": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(fspb_beamlet_info),
                               C.POINTER(C.c_float), C.POINTER(C.c_float),
                               C.POINTER(C.c_float), C.c_int]),
    "fspb_update_density": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fspb_wait_ready": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fspb_tile_shapes": (C.c_int, [C.POINTER(C.c_int), C.c_int]),
    "fspb_set_schedule": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "fspb_get_schedule": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "fspb_set_tile": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p]),
    "fspb_get_tile": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "fspb_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                C.POINTER(fspb_tune_result), C.c_int, C.POINTER(C.c_int)]),
    "fspb_batch_create": (C.c_int, [C.c_int, C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int,
                                    C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "fspb_batch_forward": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.c_void_p]),
    "fspb_batch_capture": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_void_p), C.c_void_p]),
    "fspb_batch_replay": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fspb_batch_latencies": (C.c_int, [C.c_void_p, C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.c_void_p]),
    "fspb_batch_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_longlong)]),
    "fspb_batch_destroy": (None, [C.c_void_p]),
    "fspb_mlp_create": (C.c_int, [C.POINTER(C.c_float), C.POINTER(C.c_void_p)]),
    "fspb_mlp_set_scaling": (C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "fspb_mlp_set_guard": (C.c_int, [C.c_void_p, C.POINTER(fspb_surrogate_guard)]),
    "fspb_mlp_loss_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_longlong,
                                     C.c_void_p, C.c_void_p, C.c_void_p]),
    "fspb_mlp_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_longlong,
                                      C.POINTER(fspb_adam), C.c_void_p, C.c_void_p]),
    "fspb_mlp_predict": (C.c_int, [C.c_void_p, C.c_void_p, C.c_longlong, C.c_void_p,
                                   C.c_void_p]),
    "fspb_mlp_get_state": (C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                     C.POINTER(C.c_float), C.POINTER(C.c_longlong)]),
    "fspb_mlp_set_state": (C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                     C.POINTER(C.c_float), C.c_longlong]),
    "fspb_mlp_destroy": (None, [C.c_void_p]),
    "fspb_surrogate_samples": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_longlong,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fspb_surrogate_infer": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p]),
    "fspb_forward_surrogate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p]),
    "fspb_gamma": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_float,
                             C.c_float, C.c_float, C.POINTER(fspb_gamma_params), C.c_void_p,
                             C.POINTER(fspb_gamma_stats), C.c_void_p]),
    "fspb_destroy": (None, [C.c_void_p]),
    "fspb_release_cached_memory": (C.c_int, []),
    "fspb_error_string": (C.c_char_p, [C.c_int]),
    "fspb_last_error": (C.c_char_p, []),
    "fspb_set_log_level": (C.c_int, [C.c_int]),
}

_lib = None


def load() -> C.CDLL:
    """Loads libfspb.so; raises if it is missing (build it with
    ``python -m paper_1103_1164_amd.build``)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} not found: build the HIP library first "
                              "(python -m paper_1103_1164_amd.build)")
        L = C.CDLL(str(LIB_PATH))
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class FspbError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = load()
        msg = L.fspb_last_error().decode() or L.fspb_error_string(code).decode()
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


def check(code: int, where: str) -> None:
    if code != FSPB_OK:
        raise FspbError(code, where)
