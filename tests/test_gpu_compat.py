"""GPU parity of the compatibility corrections and the Step 6 outputs against the FP64 oracle:
the pure-Neumann filter correction (eq. cc_neumann_eta), the nodal Step 6 read-off with the
constant removed by eq. CC, and the first-order eq. mix_solution, each on states that carry
the mode it must ignore."""
import math

import numpy as np
import pytest

import cmcg_inputs as ci
from cmcg_inputs import Problem
from oracle.f1 import F1
from oracle.f2 import F2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    from paper_1903_12522_amd import cmcg
    return cmcg


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _face_data(n, rng, faces):
    g = []
    for axis in range(3):
        others = [a for a in range(3) if a != axis]
        fs = tuple(n[a] + 1 for a in reversed(others))
        g += [np.zeros(fs, complex), np.zeros(fs, complex)]
    for f in faces:
        g[f] = rng.standard_normal(g[f].shape) + 1j * rng.standard_normal(g[f].shape)
    return g


def _box(bc, seed, n=(70, 12, 9)):
    """Ragged box (two 64-node x tiles), variable c, a complex source block, random data on
    two faces."""
    rng = np.random.default_rng(seed)
    shp = tuple(m + 1 for m in reversed(n))
    c = 1.0 + rng.uniform(size=shp)
    f = np.zeros(shp, complex)
    f[3:6, 4:8, 20:30] = rng.standard_normal((3, 4, 10)) + 1j * rng.standard_normal((3, 4, 10))
    return Problem(dim=3, formulation=2, n=n, omega=2 * math.pi * 1.1, c=c, f=f,
                   gS=_face_data(n, rng, (1, 4)), face_bc=bc, courant=0.5, name="box")


def test_pure_neumann_filter_correction(cm):
    prob = _box((1,) * 6, 51)
    o = F2(prob)
    U, z = o.direct()
    ze = z + np.concatenate([np.zeros(o.nn), np.full(o.nn, 0.29)])
    with cm.Solver(prob, "fp64") as s:
        Ug = s.filter(ze)
        Uz = s.filter(z)
        with pytest.raises(cm.CMCGError):
            s.step6(z)
    assert _rel(Ug, o.filter(ze)) < 1e-12
    assert _rel(Ug, U) < 1e-11
    assert _rel(Uz, U) < 1e-11


def test_step6_removes_the_constant(cm):
    prob = _box((0, 1, 0, 0, 1, 0), 52)
    o = F2(prob)
    U, z = o.direct()
    zl = z + np.concatenate([np.full(o.nn, 0.47), np.zeros(o.nn)])
    with cm.Solver(prob, "fp64") as s:
        for x in (z, zl):
            Ug = s.step6(x)
            assert _rel(Ug, o.step6_discrete(x)) < 1e-12
            assert _rel(Ug, U) < 1e-11


def test_step6_solve_matches_oracle(cm):
    prob = _box((0, 1, 0, 0, 1, 0), 53)
    o = F2(prob)
    U, _ = o.direct()
    zo, _, it = o.solve(tol=1e-10, max_iter=5000)
    with cm.Solver(prob, "fp64", tol=1e-10, max_iter=5000, riesz_tol=1e-13, output="step6") as s:
        Ug, rep = s.solve()
    assert rep["converged"] and abs(rep["iterations"] - it) <= 1
    assert _rel(Ug, o.step6_discrete(zo)) < 1e-9
    assert _rel(Ug, U) < 1e-7


def test_step6_with_dirichlet_data(cm):
    p = ci.sound_soft_sphere_3d(n=12, freq=1.0, radius=0.2)
    rng = np.random.default_rng(6)
    p.gD = rng.standard_normal(p.sound_soft.shape) + 1j * rng.standard_normal(p.sound_soft.shape)
    o = F2(p)
    U, z = o.direct()
    with cm.Solver(p, "fp64") as s:
        Ug = s.step6(z)
    assert _rel(Ug, U) < 1e-11


def _f1_problem():
    rng = np.random.default_rng(54)
    nx, ny = 70, 37
    c = 1.0 + rng.uniform(size=(ny, nx))
    f = np.zeros((ny, nx), complex)
    f[10:14, 20:25] = rng.standard_normal((4, 5)) + 1j * rng.standard_normal((4, 5))
    gS = [rng.standard_normal(ny) + 1j * rng.standard_normal(ny), np.zeros(ny, complex),
          rng.standard_normal(nx), np.zeros(nx, complex)]
    return Problem(dim=2, formulation=1, n=(nx, ny), omega=2 * math.pi * 2.5, c=c, f=f, gS=gS,
                   face_bc=(0, 1, 1, 0), courant=0.5, name="f1_step6")


def test_first_order_step6(cm):
    prob = _f1_problem()
    o = F1(prob)
    U, z = o.direct()
    rng = np.random.default_rng(9)
    psi = np.zeros((o.ny + 1, o.nx + 1))
    psi[1:-1, 1:-1] = rng.standard_normal((o.ny - 1, o.nx - 1))
    Px = (psi[1:, 1:-1] - psi[:-1, 1:-1]) / o.h
    Py = -(psi[1:-1, 1:] - psi[1:-1, :-1]) / o.h
    zd = z + o.pack(Px, Py, np.zeros((o.ny, o.nx)))
    zr = rng.standard_normal(o.size)
    with cm.Solver(prob, "fp64") as s:
        Ur = s.step6(zr)
        Ud = s.step6(zd)
    assert _rel(Ur, o.step6_output(zr)) < 1e-13
    assert _rel(Ud, U) < 1e-12


def test_first_order_step6_solve(cm):
    """The first-order read-off differentiates the state (G v_0, D P_0, over sin(theta)), so it
    magnifies the CG iterate's error: here the oracle's own Step 6 output is ~7e-6 from the
    direct solution at tol 1e-10 while its filter output is ~4e-11.  GPU and oracle iterates
    differ only by rounding; the outputs are compared against a small fraction of that
    sensitivity (the state-level read-off is checked to 1e-13 above)."""
    prob = _f1_problem()
    o = F1(prob)
    U, _ = o.direct()
    zo, _, it = o.solve(tol=1e-10, max_iter=5000)
    So = o.step6_output(zo)
    err_o = _rel(So, U)
    with cm.Solver(prob, "fp64", tol=1e-10, max_iter=5000, output="step6") as s:
        Ug, rep = s.solve()
    assert rep["converged"] and abs(rep["iterations"] - it) <= 1
    assert _rel(Ug, So) < 0.05 * err_o
    assert _rel(Ug, U) < 1.1 * err_o


def test_step6_refuses_shots(cm):
    p = ci.supershot_2d(n=24, base_freq=1.0, harmonics=(1, 2), seed=2)
    with cm.Solver(p, "fp64") as s:
        with pytest.raises(cm.CMCGError):
            s.step6(np.zeros(s.info["state_len"]))
