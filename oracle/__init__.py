"""ctypes wrapper of the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg.  The GPU library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

KERNELS = {"physical": 0, "constant": 1, "linear": 2}
FLAG_BITS = {
    "brownian": 1 << 0, "turb": 1 << 1, "radial": 1 << 2, "azimuthal": 1 << 3,
    "settling": 1 << 4, "tr_drift": 1 << 8, "tr_settle": 1 << 9, "tr_mix_r": 1 << 10,
    "tr_mix_z": 1 << 11, "coag": 1 << 12,
}
OUTCOMES = ("stick", "erode", "eroded_small", "frag")
GAS_FIELDS = 6


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "sigma_g0", "T0", "p", "q", "alpha", "v_frag", "erosion_ratio", "a_mono", "rho_s",
        "mu", "m_star", "r_ref", "dm_max", "erosion_chi", "r_in", "r_col", "k0")] + [
        ("kernel", C.c_int32), ("n_r", C.c_int32), ("n_z", C.c_int32), ("column", C.c_int32),
        ("flags", C.c_uint32), ("n_comp", C.c_int32), ("seed", C.c_uint64),
        ("frag_mode", C.c_int32), ("pad_", C.c_int32), ("frag_width", C.c_double),
        ("grid", C.c_void_p)]


class GasGrid(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("n_z", C.c_int32)] + [
        (n, C.POINTER(C.c_double)) for n in ("lr", "zn", "lrho", "lT", "lA", "lS")]


class LocalGas(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("rho_g", "T", "alpha", "cs", "Omega", "H", "slopeP", "corr")]


def grid_build(gas_grid: dict):
    """The oracle's gridded gas from node values: dict of r_nodes [n_r],
    z_nodes [n_z], rho, T, alpha [n_r, n_z].  Returns (GasGrid, arrays kept
    alive by the caller)."""
    rn = np.ascontiguousarray(gas_grid["r_nodes"], dtype=np.float64)
    zn = np.ascontiguousarray(gas_grid["z_nodes"], dtype=np.float64)
    nr, nz = len(rn), len(zn)
    rho, T, A = (np.ascontiguousarray(gas_grid[k], dtype=np.float64).reshape(nr, nz)
                 for k in ("rho", "T", "alpha"))
    out = dict(lr=np.zeros(nr), zn=np.zeros(nz), lrho=np.zeros((nr, nz)), lT=np.zeros((nr, nz)),
               lA=np.zeros((nr, nz)), lS=np.zeros(nr))
    lib().orc_grid_fill(nr, nz, _ptr(rn, C.c_double), _ptr(zn, C.c_double), _ptr(rho, C.c_double),
                        _ptr(T, C.c_double), _ptr(A, C.c_double),
                        *[_ptr(out[k], C.c_double) for k in ("lr", "zn", "lrho", "lT", "lA", "lS")])
    g = GasGrid(nr, nz, *[_ptr(out[k], C.c_double) for k in ("lr", "zn", "lrho", "lT", "lA", "lS")])
    return g, out


FRAG_MODES = {"sharp": 0, "ramp": 1, "maxwell": 2}


class Gas(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "V", "rho_g", "T", "alpha", "r_c", "zeta", "cs", "Omega", "H", "z_c", "eta_vK",
        "v_th", "lambda_", "nu", "Re", "St_eta", "Vg2")]


class Particle(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("m", "M", "a", "t_s", "St", "v_r", "v_phi", "v_z", "n")]


class CellStats(C.Structure):
    _fields_ = [("events", C.c_int64), ("outcomes", C.c_int64 * 4), ("t_end", C.c_double),
                ("drift", C.c_double)]


EVENT_DTYPE = np.dtype([("i", np.int32), ("j", np.int32), ("outcome", np.int32), ("pad", np.int32)])
STATS_DTYPE = np.dtype([("events", np.int64), ("outcomes", np.int64, (4,)), ("t_end", np.float64),
                        ("drift", np.float64)])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        u8p = C.POINTER(C.c_uint8)
        fp = C.POINTER(C.c_float)
        vp = C.c_void_p
        P = C.POINTER(Params)
        G = C.POINTER(Gas)
        Q = C.POINTER(Particle)
        sig = {
            "orc_philox4x32_10": (None, [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]),
            "orc_u01": (C.c_double, [C.c_uint32, C.c_uint32]),
            "orc_gas_derive": (None, [P, dp, G]),
            "orc_disk_local": (None, [P, C.c_double, C.c_double, dp, dp, dp, dp, dp, dp]),
            "orc_particle_props": (None, [P, G, C.c_double, C.c_double, Q]),
            "orc_dv2_turb": (C.c_double, [G, C.c_double, C.c_double]),
            "orc_rel_velocity": (C.c_double, [P, G, Q, Q]),
            "orc_pair_kernel": (C.c_double, [P, G, Q, Q]),
            "orc_rate": (C.c_double, [P, G, Q, Q]),
            "orc_frag_draw": (C.c_double, [C.c_double, C.c_double, C.c_double]),
            "orc_select": (C.c_int32, [dp, C.c_int32, C.c_double]),
            "orc_outcome": (C.c_int32, [P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                        dp]),
            "orc_frag_probability": (C.c_double, [P, C.c_double]),
            "orc_cell_rates": (None, [P, dp, C.c_int32, ip, dp, dp, dp, dp]),
            "orc_bin": (C.c_int64, [P, C.c_int64, dp, dp, u8p, ip, ip, dp, dp]),
            "orc_collide_cell": (C.c_int64, [P, dp, C.c_int32, C.c_uint32, C.c_int32, ip, dp, dp, fp,
                                             C.c_int64, C.c_double, C.c_int64, vp, C.c_int64, vp]),
            "orc_transport": (None, [P, C.c_int64, dp, dp, dp, u8p, C.c_uint32, C.c_double]),
            "orc_collide_all": (None, [P, C.c_int32, ip, ip, dp, C.c_uint32, dp, dp, fp, C.c_int64,
                                       C.c_double, C.c_int64, vp, C.c_int64, vp, C.c_int32]),
            "orc_grid_fill": (None, [C.c_int32, C.c_int32] + [dp] * 11),
            "orc_local_gas_at": (None, [P, C.c_double, C.c_double, vp]),
            "orc_sigma_hist": (C.c_int64, [C.c_int64, dp, dp, dp, u8p, dp, C.c_int32, dp, C.c_int32,
                                           C.c_int32, dp, C.POINTER(C.c_uint32)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def make_params(d: dict) -> Params:
    p = Params()
    for name, _ in Params._fields_:
        if name == "kernel":
            p.kernel = KERNELS[d["kernel"]] if isinstance(d["kernel"], str) else int(d["kernel"])
        elif name == "flags":
            fl = d["flags"]
            p.flags = sum(FLAG_BITS[f] for f in fl) if not isinstance(fl, int) else fl
        elif name == "frag_mode":
            fm = d.get("frag_mode", 0)
            p.frag_mode = FRAG_MODES[fm] if isinstance(fm, str) else int(fm)
        elif name == "frag_width":
            p.frag_width = d.get("frag_width", 0.0)
        elif name == "pad_":
            pass
        elif name == "grid":
            if d.get("gas_grid") is not None:
                g, keep = grid_build(d["gas_grid"])
                p._grid = (g, keep)          # alive as long as the Params object
                p.grid = C.cast(C.pointer(g), C.c_void_p)
            else:
                p.grid = None
        else:
            setattr(p, name, d[name])
    return p


def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def u01(lo: int, hi: int) -> float:
    return lib().orc_u01(lo, hi)


def gas_derive(params: dict, prim) -> Gas:
    g = Gas()
    pr = np.ascontiguousarray(prim, dtype=np.float64)
    lib().orc_gas_derive(C.byref(make_params(params)), _ptr(pr, C.c_double), C.byref(g))
    return g


def disk_local(params: dict, r: float, z: float) -> dict:
    out = [C.c_double() for _ in range(6)]
    lib().orc_disk_local(C.byref(make_params(params)), r, z, *[C.byref(o) for o in out])
    return dict(zip(("Sigma_g", "T", "cs", "Omega", "H", "rho_g"), [o.value for o in out]))


def particle(params: dict, gas: Gas, m: float, M: float) -> Particle:
    o = Particle()
    lib().orc_particle_props(C.byref(make_params(params)), C.byref(gas), m, M, C.byref(o))
    return o


def dv2_turb(gas: Gas, St_a: float, St_b: float) -> float:
    return lib().orc_dv2_turb(C.byref(gas), St_a, St_b)


def rel_velocity(params: dict, gas: Gas, pi: Particle, pj: Particle) -> float:
    return lib().orc_rel_velocity(C.byref(make_params(params)), C.byref(gas), C.byref(pi), C.byref(pj))


def pair_kernel(params: dict, gas: Gas, pi: Particle, pj: Particle) -> float:
    return lib().orc_pair_kernel(C.byref(make_params(params)), C.byref(gas), C.byref(pi), C.byref(pj))


def rate(params: dict, gas: Gas, pi: Particle, pj: Particle) -> float:
    return lib().orc_rate(C.byref(make_params(params)), C.byref(gas), C.byref(pi), C.byref(pj))


def frag_draw(lo: float, hi: float, u: float) -> float:
    return lib().orc_frag_draw(lo, hi, u)


def select(v, target: float) -> int:
    a = np.ascontiguousarray(v, dtype=np.float64)
    return int(lib().orc_select(_ptr(a, C.c_double), len(a), target))


def outcome(params: dict, dv: float, mi: float, mj: float, u: float,
            uf: float = 0.5) -> tuple[str, float]:
    """uf: the uniform of the fragmentation decision (unused when sharp)."""
    mn = C.c_double()
    code = lib().orc_outcome(C.byref(make_params(params)), dv, mi, mj, u, uf, C.byref(mn))
    return OUTCOMES[code], mn.value


def frag_probability(params: dict, dv: float) -> float:
    return lib().orc_frag_probability(C.byref(make_params(params)), dv)


def cell_rates(params: dict, prim, members, m, M) -> tuple[np.ndarray, np.ndarray]:
    members = np.ascontiguousarray(members, dtype=np.int32)
    n = len(members)
    m = np.ascontiguousarray(m, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    pr = np.ascontiguousarray(prim, dtype=np.float64)
    R = np.zeros((n, n))
    rs = np.zeros(n)
    lib().orc_cell_rates(C.byref(make_params(params)), _ptr(pr, C.c_double), n,
                         _ptr(members, C.c_int32), _ptr(m, C.c_double), _ptr(M, C.c_double),
                         _ptr(R, C.c_double), _ptr(rs, C.c_double))
    return R, rs


def bin_particles(params: dict, r, z, active) -> dict:
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    active = np.ascontiguousarray(active, dtype=np.uint8)
    N = len(r)
    nc = int(params["n_r"]) * int(params["n_z"])
    cell_start = np.zeros(nc + 1, dtype=np.int32)
    order = np.zeros(max(N, 1), dtype=np.int32)
    geom = np.zeros((nc, 5))
    gas = np.zeros((nc, GAS_FIELDS))
    na = lib().orc_bin(C.byref(make_params(params)), N, _ptr(r, C.c_double), _ptr(z, C.c_double),
                       _ptr(active, C.c_uint8), _ptr(cell_start, C.c_int32), _ptr(order, C.c_int32),
                       _ptr(geom, C.c_double), _ptr(gas, C.c_double))
    return dict(cell_start=cell_start, order=order[:na].copy(), geom=geom, gas=gas, n_active=int(na))


def collide_all(params: dict, cells: dict, step: int, part: dict, dt: float, max_events: int,
                log_per_cell: int = 0, threads: int = 0) -> dict:
    """Collide every cell once (in place on part['m'] and part['comp'])."""
    cs = np.ascontiguousarray(cells["cell_start"], dtype=np.int32)
    order = np.ascontiguousarray(cells["order"], dtype=np.int32)
    gas = np.ascontiguousarray(cells["gas"], dtype=np.float64)
    nc = len(cs) - 1
    m = part["m"]
    M = part["M"]
    assert m.dtype == np.float64 and m.flags.c_contiguous
    N = len(m)
    comp = part.get("comp")
    comp_p = _ptr(comp, C.c_float) if comp is not None else None
    stats = np.zeros(nc, dtype=STATS_DTYPE)
    log = np.zeros(nc * log_per_cell, dtype=EVENT_DTYPE) if log_per_cell > 0 else None
    lib().orc_collide_all(C.byref(make_params(params)), nc, _ptr(cs, C.c_int32), _ptr(order, C.c_int32),
                          _ptr(gas, C.c_double), step, _ptr(m, C.c_double),
                          _ptr(np.ascontiguousarray(M), C.c_double), comp_p, N, dt, max_events,
                          log.ctypes.data if log is not None else None, log_per_cell,
                          stats.ctypes.data, threads)
    out = dict(stats=stats)
    if log is not None:
        out["log"] = log.reshape(nc, log_per_cell)
    return out


def transport(params: dict, part: dict, step: int, dt: float) -> None:
    r, z, m, act = part["r"], part["z"], part["m"], part["active"]
    for a in (r, z, m):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    assert act.dtype == np.uint8
    lib().orc_transport(C.byref(make_params(params)), len(r), _ptr(r, C.c_double), _ptr(z, C.c_double),
                        _ptr(m, C.c_double), _ptr(act, C.c_uint8), step, dt)


def local_gas(params: dict, r: float, z: float) -> dict:
    o = LocalGas()
    prm = make_params(params)
    lib().orc_local_gas_at(C.byref(prm), r, z, C.byref(o))
    return {n: getattr(o, n) for n, _ in LocalGas._fields_}


def sigma_hist(part: dict, r_edges, m_edges, column: bool = False) -> tuple:
    """sigma_d(m, r) of the active particles: (sigma [n_rb, n_mb] in g/cm^2 per
    mass bin, count [n_rb, n_mb], particles counted)."""
    r = np.ascontiguousarray(part["r"], dtype=np.float64)
    m = np.ascontiguousarray(part["m"], dtype=np.float64)
    M = np.ascontiguousarray(part["M"], dtype=np.float64)
    act = np.ascontiguousarray(part["active"], dtype=np.uint8)
    re = np.ascontiguousarray(r_edges, dtype=np.float64)
    me = np.ascontiguousarray(m_edges, dtype=np.float64)
    nr, nm = len(re) - 1, len(me) - 1
    sigma = np.zeros((nr, nm))
    count = np.zeros((nr, nm), dtype=np.uint32)
    n = lib().orc_sigma_hist(len(r), _ptr(r, C.c_double), _ptr(m, C.c_double), _ptr(M, C.c_double),
                             _ptr(act, C.c_uint8), _ptr(re, C.c_double), nr, _ptr(me, C.c_double), nm,
                             1 if column else 0, _ptr(sigma, C.c_double), _ptr(count, C.c_uint32))
    return sigma, count, int(n)


def transport_on(params: dict) -> bool:
    return any(f in params["flags"] for f in ("tr_drift", "tr_settle", "tr_mix_r", "tr_mix_z"))


def step(params: dict, part: dict, step_index: int, dt: float, max_events: int = 0,
         cells: dict | None = None, log_per_cell: int = 0, threads: int = 0) -> dict:
    """One global step: bin (unless explicit cells are given) -> collide every
    cell -> transport.  Updates `part` in place; returns cells, stats, log."""
    if cells is None:
        cells = bin_particles(params, part["r"], part["z"], part["active"])
    out = dict(cells=cells)
    if "coag" in params["flags"]:
        out.update(collide_all(params, cells, step_index, part, dt, max_events, log_per_cell, threads))
    if transport_on(params):
        transport(params, part, step_index, dt)
    return out
