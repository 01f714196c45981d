"""Thin Python front end of libmcd.so: torch tensors hold device memory and
give the HIP stream; every call goes straight through the C ABI."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib

_STREAM = None


class MCDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _stream_handle(stream) -> int | None:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return t


class Simulation:
    """One context of the collision step over caller-owned particle tensors.

    particles: dict of device tensors r, z, m, M (float64 [N]), active
    (uint8 [N]) and optionally comp (float32 [n_comp, N]).  The library's
    device workspace is a torch tensor of this object (mcd_workspace_size
    bytes), sized for explicit grids of up to max_cells cells (default N).
    """

    def __init__(self, params: dict, particles: dict, precision: str = "mixed",
                 schedule: str = "batched", stream=None, max_cells: int | None = None):
        self.lib = _lib.load()
        self.params = dict(params)
        self.t = {k: _dev(particles[k], torch.float64, k) for k in ("r", "z", "m", "M")}
        self.t["active"] = _dev(particles["active"], torch.uint8, "active")
        comp = particles.get("comp")
        if comp is not None:
            self.t["comp"] = _dev(comp, torch.float32, "comp")
        self.N = self.t["m"].numel()
        # explicit grids of up to max_cells cells (default: one per particle)
        if max_cells is None:
            max_cells = min(self.N, 1 << 24)
        self._p = _lib.make_params(params, precision, schedule, max_cells)
        self._parts = _lib.Particles(
            self.N, self.t["r"].data_ptr(), self.t["z"].data_ptr(), self.t["m"].data_ptr(),
            self.t["M"].data_ptr(), self.t["active"].data_ptr(),
            self.t["comp"].data_ptr() if comp is not None else None)
        self.stream = stream
        nbytes = C.c_size_t()
        st = self.lib.mcd_workspace_size(C.byref(self._p), self.N, C.byref(nbytes))
        if st != 0:
            raise MCDError(st, "mcd_workspace_size rejected the parameters")
        # the library's device workspace: caller-owned torch memory
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.t["m"].device)
        ctx = C.c_void_p()
        st = self.lib.mcd_init(C.byref(self._p), C.byref(self._parts), _stream_handle(stream),
                               self.workspace.data_ptr(), nbytes.value, C.byref(ctx))
        if st != 0:
            raise MCDError(st, "mcd_init rejected the parameters or particles")
        self.ctx = ctx
        self._keep = []

    def _check(self, st: int, what: str) -> None:
        if st != 0:
            msg = self.lib.mcd_last_error(self.ctx)
            raise MCDError(st, f"{what}: {msg.decode() if msg else ''}")

    def bin(self, cells: dict | None = None, max_cell: int | None = None) -> None:
        """Adaptive binning (cells None), or the given explicit cells: device
        tensors cell_start, order, gas, kept alive here while the grid is in
        use.  max_cell: an upper bound on the cells' sizes (async planning),
        default cells.get("max_cell", 0) (the library measures, one sync)."""
        if cells is None:
            self._check(self.lib.mcd_bin(self.ctx, None), "mcd_bin")
            self._grid = None
            return
        cs = _dev(cells["cell_start"], torch.int32, "cell_start")
        order = _dev(cells["order"], torch.int32, "order")
        gas = _dev(cells["gas"], torch.float64, "gas")
        if max_cell is None:
            max_cell = int(cells.get("max_cell", 0))
        c = _lib.Cells(cs.numel() - 1, int(max_cell), cs.data_ptr(), order.data_ptr(),
                       gas.data_ptr())
        self._check(self.lib.mcd_bin(self.ctx, C.byref(c)), "mcd_bin")
        self._grid = (cs, order, gas)   # the library keeps views of these

    def step(self, dt: float, max_events: int = 0, n_steps: int = 1) -> None:
        self._check(self.lib.mcd_step(self.ctx, float(dt), int(max_events), int(n_steps)), "mcd_step")

    def tune(self, dt: float, max_events: int = 0) -> dict:
        """Autotune the batched schedule on the current cells (state kept)."""
        r = _lib.TuneResult()
        self._check(self.lib.mcd_tune(self.ctx, float(dt), int(max_events), C.byref(r)), "mcd_tune")
        return dict(small_max=r.small_max, grid_per_cu=r.grid_per_cu, trials=r.trials,
                    ms_best=r.ms_best, ms_default=r.ms_default)

    def set_schedule(self, small_max: int, grid_per_cu: int = 0) -> None:
        self._check(self.lib.mcd_set_schedule(self.ctx, int(small_max), int(grid_per_cu)),
                    "mcd_set_schedule")

    def set_gas_grid(self, grid: dict | None) -> None:
        """Gridded gas: dict of r_nodes [n_r], z_nodes [n_z], rho, T, alpha
        [n_r, n_z] (host arrays); None restores the power-law disk."""
        import numpy as np
        if grid is None:
            self._check(self.lib.mcd_set_gas_grid(self.ctx, None, 0, None, 0, None, None, None),
                        "mcd_set_gas_grid")
            return
        rn = np.ascontiguousarray(grid["r_nodes"], dtype=np.float64)
        zn = np.ascontiguousarray(grid["z_nodes"], dtype=np.float64)
        f = [np.ascontiguousarray(grid[k], dtype=np.float64).reshape(len(rn), len(zn))
             for k in ("rho", "T", "alpha")]
        self._check(self.lib.mcd_set_gas_grid(self.ctx, rn.ctypes.data, len(rn), zn.ctypes.data,
                                              len(zn), *[a.ctypes.data for a in f]),
                    "mcd_set_gas_grid")

    def sigma_hist(self, r_edges, m_edges) -> tuple[torch.Tensor, torch.Tensor]:
        """sigma_d(m, r) [n_rb, n_mb] (g/cm^2 per mass bin) and particle counts
        of the current particles over the given bin edges."""
        import numpy as np
        re = np.ascontiguousarray(r_edges, dtype=np.float64)
        me = np.ascontiguousarray(m_edges, dtype=np.float64)
        nr, nm = len(re) - 1, len(me) - 1
        dev = self.t["m"].device
        sigma = torch.empty((max(nr, 1), max(nm, 1)), dtype=torch.float64, device=dev)
        count = torch.empty((max(nr, 1), max(nm, 1)), dtype=torch.int32, device=dev)
        self._check(self.lib.mcd_sigma_hist(self.ctx, re.ctypes.data, nr, me.ctypes.data, nm,
                                            sigma.data_ptr(), count.data_ptr()), "mcd_sigma_hist")
        return sigma, count

    def snapshot(self, fields=("r", "z", "m", "active", "comp"), out: torch.Tensor | None = None):
        """Queue an asynchronous copy of the current particle state to pinned
        host memory (`out`, or a new pinned buffer); returns a Snapshot whose
        wait() gives numpy views of the fields."""
        fields = tuple(f for f in fields if f != "comp" or self.t.get("comp") is not None)
        bits = sum(_lib.SNAP_FIELDS[f] for f in fields)
        nbytes = C.c_size_t()
        self._check(self.lib.mcd_snapshot_bytes(self.ctx, bits, C.byref(nbytes)), "mcd_snapshot_bytes")
        if out is None:
            out = torch.empty(nbytes.value, dtype=torch.uint8, pin_memory=True)
        if out.device.type != "cpu" or out.numel() * out.element_size() < nbytes.value:
            raise ValueError("snapshot buffer must be host memory of at least %d bytes" % nbytes.value)
        ticket = C.c_int64()
        self._check(self.lib.mcd_snapshot(self.ctx, bits, out.data_ptr(), nbytes.value,
                                          C.byref(ticket)), "mcd_snapshot")
        return Snapshot(self, ticket.value, out, fields)

    def rates(self, cell: int, n: int) -> tuple[torch.Tensor, torch.Tensor]:
        out = torch.empty((max(n, 1), max(n, 1)), dtype=torch.float64, device=self.t["m"].device)
        rs = torch.empty(max(n, 1), dtype=torch.float64, device=self.t["m"].device)
        self._check(self.lib.mcd_rates(self.ctx, int(cell), out.data_ptr(), out.shape[1],
                                       rs.data_ptr()), "mcd_rates")
        return out[:n, :n], rs[:n]

    def row_sums(self, n_members: int) -> torch.Tensor:
        """Starting row sums of every cell as the collision launch builds
        them (indexed like the grid's order)."""
        out = torch.full((max(n_members, 1),), float("nan"), dtype=torch.float64,
                         device=self.t["m"].device)
        self._check(self.lib.mcd_row_sums(self.ctx, out.data_ptr()), "mcd_row_sums")
        return out[:n_members]

    def stats(self, check: bool = True) -> dict:
        s = _lib.Stats()
        st = self.lib.mcd_get_stats(self.ctx, C.byref(s))
        if check:
            self._check(st, "mcd_get_stats")
        return dict(events=s.events, outcomes=list(s.outcomes), steps=s.steps,
                    n_active=s.n_active, t_sim=s.t_sim, device_flags=s.device_flags,
                    n_cells=s.n_cells, max_cell=s.max_cell, status=st)

    def cells(self) -> dict:
        s = self.stats(check=False)
        nc = s["n_cells"]
        dev = self.t["m"].device
        cs = torch.empty(nc + 1, dtype=torch.int32, device=dev)
        self._check(self.lib.mcd_get_cells(self.ctx, cs.data_ptr(), None, None, None), "mcd_get_cells")
        na = int(cs[-1].item())
        order = torch.empty(max(na, 1), dtype=torch.int32, device=dev)
        geom = torch.empty((nc, _lib.GEOM_FIELDS), dtype=torch.float64, device=dev)
        gas = torch.empty((nc, _lib.GAS_FIELDS), dtype=torch.float64, device=dev)
        self._check(self.lib.mcd_get_cells(self.ctx, cs.data_ptr(), order.data_ptr(),
                                           geom.data_ptr(), gas.data_ptr()), "mcd_get_cells")
        return dict(cell_start=cs, order=order[:na], geom=geom, gas=gas)

    def set_event_log(self, buf: torch.Tensor | None, per_cell: int = 0) -> None:
        if buf is None:
            self._check(self.lib.mcd_set_event_log(self.ctx, None, 0), "mcd_set_event_log")
            return
        _dev(buf, torch.int32, "event log")
        self._keep.append(buf)
        self._check(self.lib.mcd_set_event_log(self.ctx, buf.data_ptr(), int(per_cell)),
                    "mcd_set_event_log")

    def close(self) -> None:
        if getattr(self, "ctx", None):
            self.lib.mcd_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Snapshot:
    """A queued particle snapshot (see Simulation.snapshot)."""

    def __init__(self, sim: Simulation, ticket: int, buf: torch.Tensor, fields: tuple):
        self.sim, self.ticket, self.buf, self.fields = sim, ticket, buf, fields

    def wait(self) -> dict:
        import numpy as np
        self.sim._check(self.sim.lib.mcd_snapshot_wait(self.sim.ctx, self.ticket), "mcd_snapshot_wait")
        raw = self.buf.numpy().view(np.uint8)
        n = self.sim.N
        nc = int(self.sim.params.get("n_comp", 0)) if "comp" in self.fields else 0
        sizes = dict(r=(np.float64, n), z=(np.float64, n), m=(np.float64, n),
                     active=(np.uint8, n), comp=(np.float32, nc * n))
        out, off = {}, 0
        for f in ("r", "z", "m", "active", "comp"):
            if f not in self.fields:
                continue
            dt, cnt = sizes[f]
            nb = np.dtype(dt).itemsize * cnt
            a = raw[off:off + nb].view(dt)
            out[f] = a.reshape(nc, n) if f == "comp" else a
            off += (nb + 15) // 16 * 16
        return out


def collide_noalloc(params: dict, particles: dict, cells: dict, dt: float, max_events: int,
                    step: int = 0, precision: str = "mixed", schedule: str = "batched",
                    max_cell: int | None = None, counts: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    """One collision step over explicit cells through mcd_collide_noalloc
    (no context, no workspace, no device allocation in the library); m and
    comp change in place.  Returns the device int64 counts [events,
    outcomes x4, flags] (`counts`, or a new tensor)."""
    lib = _lib.load()
    t = {k: _dev(particles[k], torch.float64, k) for k in ("m", "M")}
    comp = particles.get("comp")
    if comp is not None:
        _dev(comp, torch.float32, "comp")
    parts = _lib.Particles(t["m"].numel(), 0, 0, t["m"].data_ptr(), t["M"].data_ptr(), 0,
                           comp.data_ptr() if comp is not None else None)
    cs = _dev(cells["cell_start"], torch.int32, "cell_start")
    order = _dev(cells["order"], torch.int32, "order")
    gas = _dev(cells["gas"], torch.float64, "gas")
    if max_cell is None:
        max_cell = int(cells.get("max_cell", 0))
    c = _lib.Cells(cs.numel() - 1, int(max_cell), cs.data_ptr(), order.data_ptr(), gas.data_ptr())
    p = _lib.make_params(params, precision, schedule)
    if counts is None:
        counts = torch.zeros(6, dtype=torch.int64, device=t["m"].device)
    _dev(counts, torch.int64, "counts")
    st = lib.mcd_collide_noalloc(C.byref(p), C.byref(parts), C.byref(c), float(dt), int(max_events),
                                 int(step) & 0xFFFFFFFF, _stream_handle(stream), counts.data_ptr())
    if st != 0:
        msg = lib.mcd_last_error(None)
        raise MCDError(st, f"mcd_collide_noalloc: {msg.decode() if msg else ''}")
    return counts


def philox(ctr: torch.Tensor, key: int, stream=None) -> torch.Tensor:
    """Philox4x32-10 words on the device; ctr: int32 tensor [n, 4] (bit patterns)."""
    lib = _lib.load()
    ctr = _dev(ctr, torch.int32, "ctr")
    out = torch.empty_like(ctr)
    st = lib.mcd_philox(ctr.data_ptr(), key & 0xFFFFFFFF, (key >> 32) & 0xFFFFFFFF,
                        out.data_ptr(), ctr.shape[0], _stream_handle(stream))
    if st != 0:
        raise MCDError(st, "mcd_philox")
    return out


def to_device(part: dict, device="cuda") -> dict:
    """Copy a host particle dict (numpy arrays) to device tensors."""
    out = {}
    for k in ("r", "z", "m", "M"):
        out[k] = torch.as_tensor(part[k], dtype=torch.float64).to(device).contiguous()
    out["active"] = torch.as_tensor(part["active"], dtype=torch.uint8).to(device).contiguous()
    if part.get("comp") is not None:
        out["comp"] = torch.as_tensor(part["comp"], dtype=torch.float32).to(device).contiguous()
    return out


def cells_to_device(cells: dict, device="cuda") -> dict:
    return dict(
        cell_start=torch.as_tensor(cells["cell_start"], dtype=torch.int32).to(device).contiguous(),
        order=torch.as_tensor(cells["order"], dtype=torch.int32).to(device).contiguous(),
        gas=torch.as_tensor(cells["gas"], dtype=torch.float64).to(device).contiguous())
