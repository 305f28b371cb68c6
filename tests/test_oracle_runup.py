"""The oracle's run-up (Sec. 4.2.3) and do-nothing long-time solve (Sec. 4.2.2): Mur's
transient, convergence of the forced scheme from rest to the periodic state, the periodicity
misfit, and CMCG started from a run-up state."""
import math

import numpy as np
import pytest

import cmcg_inputs as ci
from oracle import cmcg as oc
from oracle.f1 import F1
from oracle.f2 import F2


def test_transient_switch_on():
    """theta_tr rises from 0 to 1, monotonically, with zero slope at t_tr and 1 after it."""
    t_tr = 3.7
    ts = np.linspace(0.0, t_tr, 2001)
    th = np.array([oc.transient(t, t_tr) for t in ts])
    assert th[0] == 0.0 and abs(th[-1] - 1.0) < 1e-15
    assert np.all(np.diff(th) >= 0.0)
    eps = 1e-6
    slope_end = (oc.transient(t_tr, t_tr) - oc.transient(t_tr - eps, t_tr)) / eps
    assert abs(slope_end) < 1e-5
    # initial slope: d/dt[(2 - sin s) sin s] = 2 cos s (1 - sin s) ds/dt -> pi / t_tr at 0
    slope0 = oc.transient(eps, t_tr) / eps
    assert abs(slope0 - math.pi / t_tr) < 1e-4
    assert oc.transient(2 * t_tr, t_tr) == 1.0


@pytest.fixture(scope="module")
def f1_small():
    o = F1(ci.single_source_2d(n=24, omega=2 * math.pi * 2, width=0.08))
    U, z = o.direct()
    return o, U, z


@pytest.fixture(scope="module")
def f2_small():
    o = F2(ci.sound_soft_sphere_3d(n=8, freq=1.0, radius=0.2))
    U, z = o.direct()
    return o, U, z


def test_periodic_state_has_no_misfit(f1_small, f2_small):
    for o, _, z in (f1_small, f2_small):
        assert o.functional(z) <= 1e-24 * o.functional(np.zeros(o.size))


def test_do_nothing_converges_to_the_periodic_state(f1_small):
    """With absorbing sides the forced scheme started from rest tends to the discrete periodic
    state: state error and misfit fall geometrically with the number of periods."""
    o, _, zs = f1_small
    errs, mis = [], []
    for L in (4, 8, 16, 32):
        z = o.runup(L, ramp=False)
        errs.append(np.linalg.norm(z - zs) / np.linalg.norm(zs))
        mis.append(o.functional(z))
    assert errs[-1] < 1e-4
    for a, b in zip(errs, errs[1:]):
        assert b < 0.5 * a
    for a, b in zip(mis, mis[1:]):
        assert b < 0.1 * a


def test_ramped_runup_reaches_a_smaller_transient(f1_small, f2_small):
    """Mur's switch-on leaves less of the start-up transient than switching on at once
    (second-order case at 4 periods, first-order at 32)."""
    for (o, _, _), L in ((f1_small, 32), (f2_small, 4)):
        assert o.functional(o.runup(L, ramp=True)) < o.functional(o.runup(L, ramp=False))


@pytest.mark.parametrize("which", ["f1", "f2"])
def test_cmcg_from_runup_same_solution_fewer_periods(which, f1_small, f2_small):
    """CMCG started from a run-up state, stopped at the accuracy of a start from rest, gives
    the same filtered solution and needs fewer periods in total (2 per iteration plus the
    run-up's)."""
    o, Ud, _ = f1_small if which == "f1" else f2_small
    z0, _, it0 = o.solve(tol=1e-8, max_iter=3000)
    z8, _, it8 = o.solve(tol=1e-8, max_iter=3000, runup_periods=8)
    for z in (z0, z8):
        assert np.linalg.norm(o.filter(z) - Ud) <= 1e-7 * np.linalg.norm(Ud)
    assert 2 * it8 + 8 < 2 * it0
