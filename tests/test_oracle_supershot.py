"""The oracle on multi-frequency ("super-shot") sources (Concluding remarks): a source that
superposes harmonics m omega of one base frequency has the common period T = 2 pi / omega, and
one CMCG solve followed by one filter per harmonic returns every component's Helmholtz solution.

Pins: (1) the sum of the components' periodic states (each from its own direct solve) is
periodic for the summed source; (2) each component's solution equals that of an independently
built single-frequency problem at frequency m omega with N / m steps per period (the same dt);
(3) the filters are orthogonal: a component without data filters to zero; (4) CMCG from rest
reaches every component's direct solution."""
import copy
import math

import numpy as np
import pytest

import cmcg_inputs as ci
from cmcg_inputs import Problem, Shot
from oracle.f1 import F1
from oracle.f2 import F2


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _f1_problem(harmonics=(1, 2, 3), zero_last=False):
    p = ci.supershot_2d(n=24, base_freq=1.0, harmonics=harmonics, seed=3)
    # a boundary-data component too, on the -x face of the first harmonic
    rng = np.random.default_rng(8)
    p.shots[0].gS = [rng.standard_normal(24) + 1j * rng.standard_normal(24),
                     np.zeros(24, complex), np.zeros(24, complex), np.zeros(24, complex)]
    if zero_last:
        p.shots[-1].f = None
    return p


def _f2_problem(harmonics=(1, 2, 3), with_gD=True):
    p = ci.supershot_sphere_3d(n=10, base_freq=1.0, harmonics=harmonics, radius=0.2, seed=4)
    if with_gD:
        rng = np.random.default_rng(9)
        for s in p.shots:
            s.gD = rng.standard_normal(p.sound_soft.shape) + 1j * rng.standard_normal(
                p.sound_soft.shape)
    return p


def _single(prob, k):
    """The single-frequency problem of component k: frequency m omega, that shot's data."""
    s = prob.shots[k]
    q = copy.copy(prob)
    q.shots = None
    q.omega = s.harmonic * prob.omega
    q.f, q.gS, q.gD = s.f, s.gS, s.gD
    return q


N1 = 96          # steps per base period, divisible by every harmonic used
N2 = 24


def test_superposed_state_is_periodic():
    for o in (F1(_f1_problem(), N=N1), F2(_f2_problem(), N=N2)):
        U, z = o.direct()
        assert U.shape[0] == 3
        assert o.functional(z) <= 1e-24 * o.functional(np.zeros(o.size))


@pytest.mark.parametrize("which", ["f1", "f2"])
def test_each_harmonic_is_its_own_problem(which):
    prob = _f1_problem() if which == "f1" else _f2_problem()
    cls, N = (F1, N1) if which == "f1" else (F2, N2)
    o = cls(prob, N=N)
    U, z = o.direct()
    Uf = o.filter(z)
    for k, s in enumerate(prob.shots):
        m = s.harmonic
        single = cls(_single(prob, k), N=N // m)
        assert abs(single.dt - o.dt) <= 1e-15 * o.dt
        Us, zs = single.direct()
        assert _rel(U[k], Us) < 1e-11, (which, m)
        assert _rel(Uf[k], Us) < 1e-10, (which, m)
        # the single-frequency problem's own filter of its own periodic state agrees as well
        assert _rel(single.filter(zs), Us) < 1e-10


def test_filters_are_orthogonal():
    """Without data on the last component, its filter of the periodic state vanishes while
    the other components are unchanged; the same holds for the second-order scheme."""
    o = F1(_f1_problem(zero_last=True), N=N1)
    U, z = o.direct()
    Uf = o.filter(z)
    scale = np.max(np.abs(Uf[0]))
    assert np.max(np.abs(Uf[2])) <= 1e-12 * scale
    assert np.max(np.abs(U[2])) == 0.0
    p2 = _f2_problem(with_gD=False)
    p2.shots[1].gS = None
    o2 = F2(p2, N=N2)
    U2, z2 = o2.direct()
    Uf2 = o2.filter(z2)
    assert np.max(np.abs(Uf2[1])) <= 1e-12 * np.max(np.abs(Uf2[0]))


@pytest.mark.parametrize("which", ["f1", "f2"])
def test_cmcg_extracts_every_harmonic(which):
    prob = _f1_problem() if which == "f1" else _f2_problem()
    o = F1(prob, N=N1) if which == "f1" else F2(prob, N=N2)
    Ud, _ = o.direct()
    z, hist, it = o.solve(tol=1e-10, max_iter=5000)
    assert hist[-1] <= 1e-10
    U = o.filter(z)
    for k in range(len(prob.shots)):
        assert _rel(U[k], Ud[k]) < 1e-7, (which, k)
    if which == "f2":
        # Dirichlet data of every component reproduced on the sound-soft nodes
        mask = prob.sound_soft.astype(bool)
        for k, s in enumerate(prob.shots):
            assert np.max(np.abs(U[k][mask] - s.gD[mask])) < 1e-12


def test_single_shot_list_is_the_plain_problem():
    """A problem given as one shot at harmonic 1 is the plain problem."""
    base = ci.single_source_2d(n=20, omega=2 * math.pi * 1.5, width=0.1)
    alt = copy.copy(base)
    alt.shots = [Shot(1, f=base.f)]
    alt.f = None
    a, b = F1(base), F1(alt)
    Ua, za = a.direct()
    Ub, zb = b.direct()
    assert np.array_equal(Ua, Ub) and np.array_equal(za, zb)
    assert np.array_equal(a.filter(za), b.filter(zb))
