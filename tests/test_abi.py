"""CPU-side checks of the C ABI: the built library loads, exports every function that
include/cmcg.h declares, and rejects invalid problems in host validation (no GPU touched:
these return before any HIP call)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cmcg.h")
LIB = os.path.join(ROOT, "paper_1903_12522_amd", "libcmcg.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cmcg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libcmcg.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "cmcg_create" in names and "cmcg_solve" in names and "cmcg_destroy" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_1903_12522_amd import cmcg
    assert set(cmcg.EXPORTED) == set(_declared())


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's field names, offsets and size: a C
    program compiled against include/cmcg.h prints sizeof and offsetof for each ctypes field."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    from paper_1903_12522_amd import cmcg
    pairs = [("cmcg_shot", cmcg._Shot), ("cmcg_problem", cmcg._Problem),
             ("cmcg_options", cmcg._Options), ("cmcg_report", cmcg._Report),
             ("cmcg_info", cmcg._Info), ("cmcg_server_options", cmcg._ServerOptions)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "cmcg.h"', "int main(void) {"]
    for cname, cls in pairs:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            *key, val = line.split()
            got[tuple(key)] = int(val)
    for cname, cls in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert got[(cname, field)] == getattr(cls, field).offset, (cname, field)


def _problem(cm, **kw):
    p = cm._Problem()
    p.dim, p.formulation = kw.get("dim", 2), kw.get("formulation", 1)
    for k, v in enumerate(kw.get("n", (16, 16, 1))):
        p.n[k] = v
    p.omega = kw.get("omega", 2 * math.pi)
    p.c_const = kw.get("c_const", 1.0)
    p.courant = kw.get("courant", 0.5)
    for k in range(6):
        p.face_bc[k] = kw.get("bc", 0)
    if kw.get("gD"):
        data = np.ones(17 * 17)
        _KEEP.append(data)
        p.gD_re = data.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if kw.get("f"):
        p.f_re = _array(16 * 16)
    shots = kw.get("shots")
    if shots is not None:
        # (harmonic, Dirichlet data?) per shot, each with a source
        table = (cm._Shot * max(1, len(shots)))()
        for k, (m, gd) in enumerate(shots):
            table[k].harmonic = m
            table[k].f_re = _array(16 * 16)
            if gd:
                table[k].gD_re = _array(17 * 17)
        _KEEP.append(table)
        p.n_shots = kw.get("n_shots", len(shots))
        if not kw.get("null_shots"):
            p.shots = ctypes.cast(table, ctypes.POINTER(cm._Shot))
    return p


def _array(n):
    data = np.ones(n)
    _KEEP.append(data)
    return data.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


_KEEP = []


def _create(cm, p, **ok):
    o = cm._Options()
    o.precision = ok.get("precision", 0)
    o.tol = ok.get("tol", 1e-6)
    o.max_iter = ok.get("max_iter", 10)
    o.riesz_mode = ok.get("riesz_mode", 0)
    o.runup_periods = ok.get("runup_periods", 0)
    o.output = ok.get("output", 0)
    h = cm._H()
    st = cm._lib.cmcg_create(ctypes.byref(p), ctypes.byref(o), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("kw,opt,expect", [
    (dict(courant=0.72), {}, -2),                       # sigma sqrt(2) >= 1: unstable leapfrog
    (dict(dim=3, formulation=2, n=(8, 8, 8), courant=0.58), {}, -2),
    (dict(omega=0.0), {}, -1),
    (dict(omega=float("nan")), {}, -1),
    (dict(c_const=-1.0), {}, -1),
    (dict(n=(1, 16, 1)), {}, -1),
    (dict(bc=7), {}, -1),
    (dict(), dict(precision=5), -1),
    (dict(), dict(max_iter=0), -1),
    (dict(dim=3, formulation=1, n=(8, 8, 8)), {}, -6),   # first-order 3D is not provided
    (dict(), dict(riesz_mode=7), -1),
    (dict(), dict(runup_periods=-1), -1),
    (dict(gD=True), {}, -1),                            # Dirichlet data needs a sound-soft mask
    (dict(bc=1), dict(runup_periods=2), -6),            # run-up of a closed undamped box
    # multi-frequency sources (N = 32 steps per base period here)
    (dict(shots=[(1, 0), (1, 0)]), {}, -1),             # repeated harmonic
    (dict(shots=[(0, 0)]), {}, -1),                     # harmonic below 1
    (dict(shots=[(1, 0), (16, 0)]), {}, -1),            # 2 m >= N: filters not separable
    (dict(shots=[(1, 0)] * 9, n_shots=9), {}, -1),      # more than CMCG_MAX_SHOTS
    (dict(shots=[(1, 0), (2, 0)], f=True), {}, -1),     # data both in the problem and the shots
    (dict(shots=[(1, 0), (2, 1)]), {}, -1),             # Dirichlet data without a mask
    (dict(shots=[(1, 0)], null_shots=True), {}, -1),    # n_shots without the array
    (dict(shots=[(1, 0)], n_shots=-1), {}, -1),
    # output modes
    (dict(), dict(output=5), -1),
    (dict(shots=[(1, 0), (2, 0)]), dict(output=1), -1),   # Step 6 reads one frequency
    (dict(dim=3, formulation=2, n=(8, 8, 8), bc=1), dict(output=1), -6),   # pure Neumann: eta
])
def test_invalid_inputs_rejected_before_device(kw, opt, expect):
    from paper_1903_12522_amd import cmcg as cm
    st, h = _create(cm, _problem(cm, **kw), **opt)
    assert st == expect
    assert not h.value
    assert cm._lib.cmcg_last_error().decode() != ""


def test_valid_shots_pass_host_validation():
    """Distinct harmonics below N / 2 pass validation (then the device is needed)."""
    from paper_1903_12522_amd import cmcg as cm
    st, h = _create(cm, _problem(cm, shots=[(1, 0), (3, 0), (15, 0)]))
    assert st in (0, -4)
    if h.value:
        cm._lib.cmcg_destroy(h)


def test_first_order_dirichlet_cells_pass_host_validation():
    """Dirichlet data on the first-order grid needs a sound-soft (cell) mask; with one it passes
    validation (then the device is needed)."""
    from paper_1903_12522_amd import cmcg as cm
    p = _problem(cm)
    mask = np.zeros(16 * 16, np.uint8)
    mask[100:104] = 1
    _KEEP.append(mask)
    p.sound_soft = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    p.gD_re = _array(16 * 16)
    st, h = _create(cm, p)
    assert st in (0, -4)
    if h.value:
        cm._lib.cmcg_destroy(h)


def test_nan_wave_speed_rejected():
    from paper_1903_12522_amd import cmcg as cm
    p = _problem(cm)
    c = np.ones(16 * 16)
    c[37] = np.nan
    p.c = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    st, h = _create(cm, p)
    assert st == -1 and not h.value


def test_status_strings():
    from paper_1903_12522_amd import cmcg as cm
    for s in (0, 1, -1, -2, -3, -4, -5, -6):
        assert cm.status_string(s)
    cm._lib.cmcg_destroy(None)      # NULL-safe
