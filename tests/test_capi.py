"""The C-ABI library without a GPU: it loads, exports every function that
include/mcd.h declares, its ctypes mirrors have the header's layout, the
workspace size follows the layout it documents, and argument validation
(parameters, particles, the caller's workspace) rejects bad input before any
device call."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2507_21239_amd import _lib
from paper_2507_21239_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcd.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = _lib.load()
    declared = _declared_functions()
    assert set(declared) == set(_lib.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (mcd_[a-z_]+)\b", out))
    assert set(declared) <= exported


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "layout.c"
    structs = {"mcd_params": _lib.Params, "mcd_particles": _lib.Particles,
               "mcd_cells": _lib.Cells, "mcd_stats": _lib.Stats,
               "mcd_tune_result": _lib.TuneResult}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mcd.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


FAKE = 0x1000   # never dereferenced: validation fails first


def _init(params, n=10, ws=FAKE, ws_bytes=1 << 40):
    lib = _lib.load()
    p = _lib.make_params(params)
    parts = _lib.Particles(n, FAKE, FAKE, FAKE, FAKE, FAKE, None)
    ctx = C.c_void_p()
    return lib.mcd_init(C.byref(p), C.byref(parts), None, ws, ws_bytes, C.byref(ctx)), ctx


def _ws_size(params, n, precision="mixed", max_cells=0):
    lib = _lib.load()
    p = _lib.make_params(params, precision, "batched", max_cells)
    b = C.c_size_t()
    st = lib.mcd_workspace_size(C.byref(p), n, C.byref(b))
    return st, b.value


def test_workspace_size_follows_its_layout():
    P = W.benchmark_params(n_r=50, n_z=2)     # zones of 2000 and 4000 particles
    st, b1 = _ws_size(P, 100_000)
    assert st == _lib.MCD_OK
    st, b2 = _ws_size(P, 200_000)
    # per particle: grid order 4, binning 2 x (4 + 4) + 1 + 4, tuning backup 8 (+ 256-byte
    # rounding and the radix histogram): about 34 bytes more per particle
    assert 30 * 100_000 < b2 - b1 < 40 * 100_000, b2 - b1
    # composition fractions add their tuning backup, 4 bytes per fraction and particle
    _, b3 = _ws_size(W.benchmark_params(n_r=50, n_z=2, n_comp=8), 100_000)
    assert abs((b3 - b1) - 32 * 100_000) <= 512
    # explicit grids of more cells size the two cell lists (8 bytes per cell)
    _, b4 = _ws_size(P, 100_000, max_cells=1_000_100)
    assert abs((b4 - b1) - 8 * 1_000_000) <= 1024
    # zones above 8192 particles need the global radix path's 20 bytes per particle
    _, b5 = _ws_size(W.benchmark_params(n_r=2, n_z=50), 100_000)
    _, b6 = _ws_size(W.benchmark_params(n_r=20, n_z=5), 100_000)
    assert abs((b5 - b6) - 20 * 100_000) <= 4096
    for bad in (0, -5, 1 << 31):
        assert _ws_size(P, bad)[0] == _lib.MCD_EINVAL
    assert _ws_size(W.benchmark_params(n_r=0), 100)[0] == _lib.MCD_EINVAL
    assert _ws_size(P, 100, max_cells=-1)[0] == _lib.MCD_EINVAL


def test_init_rejects_a_missing_or_small_workspace():
    P = W.benchmark_params(n_r=2, n_z=2)
    st, need = _ws_size(P, 10)
    assert st == _lib.MCD_OK
    assert _init(P, ws=None, ws_bytes=need)[0] == _lib.MCD_EINVAL
    st, ctx = _init(P, ws_bytes=need - 1)
    assert st == _lib.MCD_EINVAL and not ctx.value


@pytest.mark.parametrize("bad", [
    dict(T0=float("nan")), dict(sigma_g0=-1.0), dict(v_frag=0.0), dict(dm_max=1.5),
    dict(erosion_ratio=0.5), dict(kernel=7), dict(n_r=0), dict(n_comp=9), dict(flags=1 << 20),
    dict(alpha=-1e-3), dict(column=1, r_col=0.0),
])
def test_init_rejects_bad_params(bad):
    st, ctx = _init(W.benchmark_params(**bad))
    assert st == _lib.MCD_EINVAL
    assert not ctx.value


def test_init_rejects_bad_particles():
    lib = _lib.load()
    p = _lib.make_params(W.benchmark_params())
    ctx = C.c_void_p()
    ws = (FAKE, 1 << 40)
    parts = _lib.Particles(0, 1, 1, 1, 1, 1, None)
    assert lib.mcd_init(C.byref(p), C.byref(parts), None, *ws, C.byref(ctx)) == _lib.MCD_EINVAL
    parts = _lib.Particles(10, 1, None, 1, 1, 1, None)
    assert lib.mcd_init(C.byref(p), C.byref(parts), None, *ws, C.byref(ctx)) == _lib.MCD_EINVAL
    p = _lib.make_params(W.benchmark_params(n_comp=8))
    parts = _lib.Particles(10, 1, 1, 1, 1, 1, None)
    assert lib.mcd_init(C.byref(p), C.byref(parts), None, *ws, C.byref(ctx)) == _lib.MCD_EINVAL
    assert lib.mcd_init(None, C.byref(parts), None, *ws, C.byref(ctx)) == _lib.MCD_EINVAL


def test_null_context_calls_are_rejected():
    lib = _lib.load()
    assert lib.mcd_bin(None, None) == _lib.MCD_EINVAL
    assert lib.mcd_step(None, 1.0, 0, 1) == _lib.MCD_EINVAL
    assert lib.mcd_rates(None, 0, None, 0, None) == _lib.MCD_EINVAL
    assert lib.mcd_row_sums(None, None) == _lib.MCD_EINVAL
    assert lib.mcd_workspace_size(None, 10, None) == _lib.MCD_EINVAL
    assert lib.mcd_get_stats(None, None) == _lib.MCD_EINVAL
    assert lib.mcd_last_error(None) == b"null context"
    assert lib.mcd_philox(None, 0, 0, None, -1, None) == _lib.MCD_EINVAL
    assert lib.mcd_tune(None, 1.0, 0, None) == _lib.MCD_EINVAL
    assert lib.mcd_set_schedule(None, 256, 0) == _lib.MCD_EINVAL
    lib.mcd_free(None)
