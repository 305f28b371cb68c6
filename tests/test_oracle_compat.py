"""The oracle's compatibility corrections (Sec. 2.2) and Step 6 outputs.

* Pure-Neumann box: the mode eta (u growing linearly, v constant) is invisible to J and shifts
  the filter sums by exactly 2 eta dt / (e^{i w dt} - 1) (the closed form of sum n q^n over a
  period); the filter's compatibility correction (eq. cc_neumann_eta, discrete) removes it.
* Absorbing box without sound-soft nodes: the constant lam in u (Thm 1) is a periodic mode; the
  Step 6 output read off the discrete periodic state, corrected by the compatibility condition
  (eq. CC, discrete), is the time-discrete solution with or without that shift.
* First-order scheme: divergence-free flux fields are fixed points of the period (the
  non-uniqueness of Thm 2), and the time-discrete eq. mix_solution recovers u from the initial
  state alone, blind to them."""
import math

import numpy as np
import pytest

import cmcg_inputs as ci
from cmcg_inputs import Problem
from oracle.f1 import F1
from oracle.f2 import F2


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _neumann_box():
    """3D pure-Neumann box, variable c, complex source and Neumann data on two faces."""
    n = (7, 6, 5)
    rng = np.random.default_rng(41)
    shp = tuple(m + 1 for m in reversed(n))
    c = 1.0 + 0.5 * rng.uniform(size=shp)
    f = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    g = []
    for axis in range(3):
        others = [a for a in range(3) if a != axis]
        fs = tuple(n[a] + 1 for a in reversed(others))
        g += [np.zeros(fs, complex), np.zeros(fs, complex)]
    g[1] = rng.standard_normal(g[1].shape) + 1j * rng.standard_normal(g[1].shape)
    g[4] = rng.standard_normal(g[4].shape)
    return Problem(dim=3, formulation=2, n=n, omega=2 * math.pi * 0.9, c=c, f=f, gS=g,
                   face_bc=(1,) * 6, courant=0.5, name="neumann_box")


def _raw_filter(o, z):
    U = [np.zeros(o.shape, complex)]
    o.period(z, True, U_acc=U)
    return 2.0 * U[0] / o.N


@pytest.mark.parametrize("which", ["channel", "box"])
def test_eta_mode_shift_and_its_correction(which):
    prob = ci.channel_bounded_neumann_f2((16, 2), math.pi / 4) if which == "channel" \
        else _neumann_box()
    o = F2(prob)
    assert o.pure_neumann()
    U, z = o.direct()
    eta = 0.37
    ze = z + np.concatenate([np.zeros(o.nn), np.full(o.nn, eta)])
    # the mode is invisible to J: the misfit of the shifted state stays zero
    assert o.functional(ze) <= 1e-20 * o.functional(np.zeros(o.size))
    # raw filter sums: shifted by the closed-form constant
    q = np.exp(1j * o.omega * o.dt)
    shift = 2.0 * eta * o.dt / (q - 1.0)
    raw = _raw_filter(o, ze)
    assert np.max(np.abs(raw - U - shift)) < 1e-10 * max(1.0, np.max(np.abs(U)))
    # the corrected filter returns the time-discrete solution, with and without the mode
    assert _rel(o.filter(ze), U) < 1e-11
    assert _rel(o.filter(z), U) < 1e-11


def _absorbing_box():
    n = (6, 7, 5)
    rng = np.random.default_rng(43)
    shp = tuple(m + 1 for m in reversed(n))
    c = 1.0 + rng.uniform(size=shp)
    f = np.zeros(shp, complex)
    f[2:4, 3:5, 2:4] = rng.standard_normal((2, 2, 2)) + 1j
    g = ci.plane_wave_face_data(n, 1.0 / n[0], 2 * math.pi * 1.1, (1.0, 0.3, -0.2))
    return Problem(dim=3, formulation=2, n=n, omega=2 * math.pi * 1.1, c=c, f=f, gS=g,
                   face_bc=(0, 1, 0, 0, 1, 0), courant=0.5, name="absorbing_box")


def test_lambda_mode_is_periodic_and_step6_removes_it():
    o = F2(_absorbing_box())
    U, z = o.direct()
    lam = 0.61
    zl = z + np.concatenate([np.full(o.nn, lam), np.zeros(o.nn)])
    # a constant displacement is a periodic solution of the damped scheme
    d = np.concatenate([np.full(o.nn, lam), np.zeros(o.nn)])
    assert np.max(np.abs(o.period(d, False) - d)) < 1e-13
    assert _rel(o.step6_discrete(z), U) < 1e-11
    assert _rel(o.step6_discrete(zl), U) < 1e-11
    # without the correction the Step 6 read-off carries the shift
    wh = math.sin(o.omega * o.dt) / o.dt
    raw = zl[: o.nn] + 1j * zl[o.nn:] / wh
    assert np.allclose(raw.reshape(o.shape) - U, lam, atol=1e-10)
    # the filter ignores the shift
    assert _rel(o.filter(zl), U) < 1e-11


def test_step6_from_cmcg_iterate():
    """CG from rest on a box without sound-soft nodes (its Riesz map keeps zero-sum
    iterates): the corrected Step 6 output and the filter give the same solution."""
    o = F2(_absorbing_box())
    U, _ = o.direct()
    z, hist, it = o.solve(tol=1e-11, max_iter=5000)
    assert _rel(o.step6_discrete(z), U) < 1e-8
    assert _rel(o.filter(z), U) < 1e-8


def test_step6_with_dirichlet_data():
    p = ci.sound_soft_sphere_3d(n=10, freq=1.0, radius=0.2)
    rng = np.random.default_rng(5)
    p.gD = rng.standard_normal(p.sound_soft.shape) + 1j * rng.standard_normal(p.sound_soft.shape)
    o = F2(p)
    U, z = o.direct()
    assert _rel(o.step6_discrete(z), U) < 1e-11
    with pytest.raises(ValueError):
        F2(ci.channel_bounded_neumann_f2((8, 2), 1.0)).step6_discrete(z[:2])


def _f1_problem():
    rng = np.random.default_rng(44)
    nx, ny = 13, 9
    c = 1.0 + rng.uniform(size=(ny, nx))
    f = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    gS = [rng.standard_normal(ny) + 1j * rng.standard_normal(ny), np.zeros(ny, complex),
          rng.standard_normal(nx), np.zeros(nx, complex)]
    return Problem(dim=2, formulation=1, n=(nx, ny), omega=2 * math.pi * 1.3, c=c, f=f, gS=gS,
                   face_bc=(0, 1, 1, 0), courant=0.5, name="f1_compat")


def _divergence_free(o, seed):
    """Discrete curl of a stream function on the interior grid corners (zero on the boundary):
    interior-face fluxes with zero divergence in every cell."""
    rng = np.random.default_rng(seed)
    psi = np.zeros((o.ny + 1, o.nx + 1))
    psi[1:-1, 1:-1] = rng.standard_normal((o.ny - 1, o.nx - 1))
    Px = (psi[1:, 1:-1] - psi[:-1, 1:-1]) / o.h          # (ny, nx-1)
    Py = -(psi[1:-1, 1:] - psi[1:-1, :-1]) / o.h         # (ny-1, nx)
    return Px, Py


def test_first_order_divergence_free_fields_are_fixed_points():
    o = F1(_f1_problem())
    Px, Py = _divergence_free(o, 7)
    assert np.max(np.abs(o.div(Px, Py))) < 1e-12 * np.max(np.abs(Px))
    d = o.pack(Px, Py, np.zeros((o.ny, o.nx)))
    assert np.max(np.abs(o.period(d, False) - d)) < 1e-12 * np.max(np.abs(d))


def test_first_order_step6_output():
    o = F1(_f1_problem())
    U, z = o.direct()
    assert _rel(o.step6_output(z), U) < 1e-12
    Px, Py = _divergence_free(o, 8)
    zd = z + o.pack(Px, Py, np.zeros((o.ny, o.nx)))
    assert _rel(o.step6_output(zd), U) < 1e-12
    assert _rel(o.filter(zd), U) < 1e-11
    zc, _, _ = o.solve(tol=1e-11, max_iter=5000)
    assert _rel(o.step6_output(zc), U) < 1e-8
