"""The oracle's first-order Dirichlet data (eq. mixWE_DBC) on sound-soft cells: v is held at
Re(-i omega gD e^{-i omega t}) on masked cells, which carry no unknown.

Pins: the 1D closed form u = exp(i k x) with its Dirichlet value imposed at the first cell
centre; exact energy conservation of the masked scheme without absorption; the transposed
period against a brute-force dense transpose; CMCG and the Step 6 read-off against the direct
solve with Dirichlet rows; the filter returning gD on the mask; a multi-frequency source with
Dirichlet data per component."""
import math

import numpy as np
import pytest

import cmcg_inputs as ci
from cmcg_inputs import Problem, Shot
from oracle.f1 import F1


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _channel(nx, ny, k):
    """u = exp(i k x): the first column of cells is Dirichlet with u = exp(i k h / 2), x = 1
    absorbing without data, Neumann walls."""
    mask = np.zeros((ny, nx), np.uint8)
    mask[:, 0] = 1
    gD = np.zeros((ny, nx), complex)
    gD[:, 0] = np.exp(1j * k * 0.5 / nx)
    return Problem(dim=2, formulation=1, n=(nx, ny), omega=k, c_const=1.0, sound_soft=mask,
                   gD=gD, face_bc=(1, 0, 1, 1), courant=0.5, name="f1_dirichlet_channel")


def test_dirichlet_channel_converges_to_the_closed_form():
    k = 6 * math.pi
    errs = []
    for nx in (64, 128, 256):
        o = F1(_channel(nx, 4, k))
        U, _ = o.direct()
        x = (np.arange(nx) + 0.5) / nx
        errs.append(np.max(np.abs(U - np.exp(1j * k * x)[None, :])))
        # the Dirichlet column returns its data exactly
        assert np.max(np.abs(U[:, 0] - np.exp(1j * k * 0.5 / nx))) < 1e-12
    assert errs[0] < 0.2
    for a, b in zip(errs, errs[1:]):
        assert 1.85 < a / b < 2.15     # first order: the absorbing closure at x = 1


def _box_with_obstacle(bc=(1, 1, 1, 1), n=(14, 11), seed=3):
    rng = np.random.default_rng(seed)
    nx, ny = n
    c = 1.0 + rng.uniform(size=(ny, nx))
    mask = np.zeros((ny, nx), np.uint8)
    mask[4:7, 5:9] = 1
    mask[2, 1] = 1
    f = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    gD = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))) * mask
    return Problem(dim=2, formulation=1, n=n, omega=2 * math.pi * 1.7, c=c, f=f, gD=gD,
                   sound_soft=mask, face_bc=bc, courant=0.5, name="f1_obstacle_box")


def test_energy_conserved_with_dirichlet_cells():
    o = F1(_box_with_obstacle())
    rng = np.random.default_rng(4)
    Px = rng.standard_normal(o.shapes[0])
    Py = rng.standard_normal(o.shapes[1])
    v = o.free * rng.standard_normal(o.shapes[2])
    E0 = o.energy(Px, Py, v)
    for n in range(200):
        Px, Py, v = o.step(Px, Py, v, n, False)
        assert np.all(v[o.free < 0.5] == 0.0)
    assert abs(o.energy(Px, Py, v) - E0) < 1e-12 * E0


def test_transpose_with_dirichlet_cells_brute_force():
    o = F1(_box_with_obstacle(bc=(0, 1, 0, 1), n=(7, 6)))
    steps = 3
    E = np.stack([o.period(e, False, steps=steps) for e in np.eye(o.size)], axis=1)
    ET = np.stack([o.period_T(e, steps=steps) for e in np.eye(o.size)], axis=1)
    assert np.max(np.abs(ET - E.T)) < 1e-13 * np.max(np.abs(E))
    # masked velocities are neither read nor written
    vmask = np.concatenate([np.ones(o.sizes[0] + o.sizes[1]), o.free.ravel()]) < 0.5
    assert np.all(E[vmask, :] == 0.0) and np.all(E[:, vmask] == 0.0)


def test_cmcg_filter_and_step6_with_dirichlet_cells():
    o = F1(_box_with_obstacle(bc=(0, 1, 0, 0)))
    U, z = o.direct()
    mask = o.free < 0.5
    gD = o.comps[0][3]
    assert np.max(np.abs(U[mask] - gD[mask])) < 1e-12
    assert o.functional(z) <= 1e-24 * o.functional(np.zeros(o.size))
    assert _rel(o.filter(z), U) < 1e-11
    assert _rel(o.step6_output(z), U) < 1e-11
    zc, hist, it = o.solve(tol=1e-11, max_iter=5000)
    Uc = o.filter(zc)
    assert _rel(Uc, U) < 1e-8
    assert np.max(np.abs(Uc[mask] - gD[mask])) < 1e-10


def test_sound_soft_square_scattering():
    """Total-field scattering by a sound-soft square and by a square cavity: CMCG reaches the
    direct solution, which vanishes on the obstacle."""
    for cav in (False, True):
        o = F1(ci.sound_soft_square_2d(n=40, freq=2.0, side=0.4, cavity=cav))
        U, _ = o.direct()
        z, _, _ = o.solve(tol=1e-9, max_iter=8000)
        Uc = o.filter(z)
        assert _rel(Uc, U) < 1e-6
        assert np.max(np.abs(Uc[o.free < 0.5])) < 1e-9


def test_supershot_with_dirichlet_cells():
    prob = _box_with_obstacle(bc=(0, 1, 0, 0))
    rng = np.random.default_rng(8)
    mask = prob.sound_soft
    prob.shots = [Shot(1, f=prob.f, gD=prob.gD),
                  Shot(3, f=None, gD=(rng.standard_normal(mask.shape) + 1j) * mask)]
    prob.f = prob.gD = None
    o = F1(prob, N=60)
    U, z = o.direct()
    assert o.functional(z) <= 1e-24 * o.functional(np.zeros(o.size))
    Uf = o.filter(z)
    for k in range(2):
        assert _rel(Uf[k], U[k]) < 1e-10
        assert np.max(np.abs(Uf[k][mask > 0] - prob.shots[k].gD[mask > 0])) < 1e-10
