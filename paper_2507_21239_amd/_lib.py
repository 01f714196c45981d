"""ctypes view of the C ABI in include/mcd.h (libmcd.so).

Argument marshalling only: every step of the method runs in the HIP
kernels of libmcd.so.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcd.so")

MCD_OK, MCD_EINVAL, MCD_ENOMEM, MCD_EHIP, MCD_ESTATE, MCD_EDEVICE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "MCD_OK", -1: "MCD_EINVAL", -2: "MCD_ENOMEM", -3: "MCD_EHIP",
                -4: "MCD_ESTATE", -5: "MCD_EDEVICE"}
KERNELS = {"physical": 0, "constant": 1, "linear": 2}
FLAG_BITS = {
    "brownian": 1 << 0, "turb": 1 << 1, "radial": 1 << 2, "azimuthal": 1 << 3,
    "settling": 1 << 4, "tr_drift": 1 << 8, "tr_settle": 1 << 9, "tr_mix_r": 1 << 10,
    "tr_mix_z": 1 << 11, "coag": 1 << 12,
}
PRECISIONS = {"fp64": 0, "mixed": 1}
SCHEDULES = {"plain": 0, "batched": 1}
GAS_FIELDS = 6
GEOM_FIELDS = 5

# every function declared in include/mcd.h
EXPORTS = ("mcd_workspace_size", "mcd_init", "mcd_bin", "mcd_rates", "mcd_row_sums", "mcd_step", "mcd_tune", "mcd_set_schedule",
           "mcd_set_gas_grid", "mcd_sigma_hist", "mcd_snapshot_bytes", "mcd_snapshot", "mcd_snapshot_wait",
           "mcd_get_stats", "mcd_get_cells", "mcd_set_event_log", "mcd_philox", "mcd_last_error",
           "mcd_free", "mcd_collide_noalloc")


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "sigma_g0", "T0", "p", "q", "alpha", "v_frag", "erosion_ratio", "a_mono", "rho_s",
        "mu", "m_star", "r_ref", "dm_max", "erosion_chi", "r_in", "r_col", "k0")] + [
        ("kernel", C.c_int32), ("n_r", C.c_int32), ("n_z", C.c_int32), ("column", C.c_int32),
        ("flags", C.c_uint32), ("n_comp", C.c_int32), ("seed", C.c_uint64),
        ("precision", C.c_int32), ("schedule", C.c_int32), ("frag_mode", C.c_int32),
        ("max_cells", C.c_int32), ("frag_width", C.c_double)]


FRAG_MODES = {"sharp": 0, "ramp": 1, "maxwell": 2}
SNAP_FIELDS = {"r": 1, "z": 2, "m": 4, "active": 8, "comp": 16}


class Particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("r", C.c_void_p), ("z", C.c_void_p), ("m", C.c_void_p),
                ("M", C.c_void_p), ("active", C.c_void_p), ("comp", C.c_void_p)]


class Cells(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("max_cell", C.c_int32), ("cell_start", C.c_void_p),
                ("order", C.c_void_p), ("gas", C.c_void_p)]


class TuneResult(C.Structure):
    _fields_ = [("small_max", C.c_int32), ("grid_per_cu", C.c_int32), ("trials", C.c_int32),
                ("pad", C.c_int32), ("ms_best", C.c_double), ("ms_default", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("events", C.c_int64), ("outcomes", C.c_int64 * 4), ("steps", C.c_int64),
                ("n_active", C.c_int64), ("t_sim", C.c_double), ("device_flags", C.c_uint32),
                ("n_cells", C.c_int32), ("max_cell", C.c_int32), ("pad", C.c_int32)]


_lib = None


def load() -> C.CDLL:
    """Load libmcd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2507_21239_amd/build.py "
                           "(or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
    sig = {
        "mcd_workspace_size": (i32, [C.POINTER(Params), i64, C.POINTER(C.c_size_t)]),
        "mcd_init": (i32, [C.POINTER(Params), C.POINTER(Particles), vp, vp, C.c_size_t,
                           C.POINTER(vp)]),
        "mcd_bin": (i32, [vp, C.POINTER(Cells)]),
        "mcd_rates": (i32, [vp, i32, vp, i64, vp]),
        "mcd_row_sums": (i32, [vp, vp]),
        "mcd_step": (i32, [vp, C.c_double, i64, i32]),
        "mcd_tune": (i32, [vp, C.c_double, i64, C.POINTER(TuneResult)]),
        "mcd_set_schedule": (i32, [vp, i32, i32]),
        "mcd_sigma_hist": (i32, [vp, vp, i32, vp, i32, vp, vp]),
        "mcd_set_gas_grid": (i32, [vp, vp, i32, vp, i32, vp, vp, vp]),
        "mcd_snapshot_bytes": (i32, [vp, u32, C.POINTER(C.c_size_t)]),
        "mcd_snapshot": (i32, [vp, u32, vp, C.c_size_t, C.POINTER(i64)]),
        "mcd_snapshot_wait": (i32, [vp, i64]),
        "mcd_get_stats": (i32, [vp, C.POINTER(Stats)]),
        "mcd_get_cells": (i32, [vp, vp, vp, vp, vp]),
        "mcd_set_event_log": (i32, [vp, vp, i64]),
        "mcd_philox": (i32, [vp, u32, u32, vp, i64, vp]),
        "mcd_last_error": (C.c_char_p, [vp]),
        "mcd_collide_noalloc": (i32, [C.POINTER(Params), C.POINTER(Particles), C.POINTER(Cells),
                                      C.c_double, i64, u32, vp, vp]),
        "mcd_free": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def make_params(d: dict, precision: str = "mixed", schedule: str = "batched",
                max_cells: int = 0) -> Params:
    p = Params()
    for name, _ in Params._fields_:
        if name == "kernel":
            p.kernel = KERNELS[d["kernel"]] if isinstance(d["kernel"], str) else int(d["kernel"])
        elif name == "flags":
            fl = d["flags"]
            p.flags = fl if isinstance(fl, int) else sum(FLAG_BITS[f] for f in fl)
        elif name == "precision":
            p.precision = PRECISIONS[precision]
        elif name == "schedule":
            p.schedule = SCHEDULES[schedule]
        elif name == "frag_mode":
            fm = d.get("frag_mode", "sharp")
            p.frag_mode = FRAG_MODES[fm] if isinstance(fm, str) else int(fm)
        elif name == "frag_width":
            p.frag_width = d.get("frag_width", 0.0)
        elif name == "max_cells":
            p.max_cells = int(max_cells)
        else:
            setattr(p, name, d[name])
    return p
