"""GPU parity for general boundary data (eq. HE): Dirichlet data on sound-soft nodes (nodal
formulation) and Neumann data on Neumann faces (both formulations), against the FP64 oracle."""
import dataclasses
import math

import numpy as np
import pytest

import cmcg_inputs as ci
from oracle.f1 import F1
from oracle.f2 import F2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    from paper_1903_12522_amd import cmcg
    return cmcg


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _sphere_with_data(n=12):
    base = ci.sound_soft_sphere_3d(n=n, freq=1.2, radius=0.2)
    rng = np.random.default_rng(8)
    shp = base.sound_soft.shape
    return dataclasses.replace(base, gD=rng.standard_normal(shp) + 1j * rng.standard_normal(shp))


def test_dirichlet_data_periods_match_oracle(cm):
    prob = _sphere_with_data()
    o = F2(prob)
    rng = np.random.default_rng(9)
    z = rng.standard_normal(o.size) * np.concatenate([o.free.ravel()] * 2)
    with cm.Solver(prob, "fp64") as s:
        assert _rel(s.apply(cm.OP_FORCED, z), o.period(z, True)) < 1e-13
        assert _rel(s.apply(cm.OP_FORWARD, z), o.period(z, False)) < 1e-13
        assert _rel(s.filter(z), o.filter(z)) < 1e-13


def test_dirichlet_data_cmcg_matches_oracle(cm):
    prob = _sphere_with_data()
    o = F2(prob)
    Ud, _ = o.direct()
    with cm.Solver(prob, "fp64", tol=1e-11, max_iter=3000, riesz_tol=1e-13) as s:
        U, rep = s.solve()
    assert rep["converged"]
    assert _rel(U, Ud) < 1e-9
    m = prob.sound_soft.astype(bool)
    assert np.max(np.abs(U[m] - prob.gD[m])) < 1e-11 * np.max(np.abs(prob.gD))


def test_paper_example_with_dirichlet_data_as_3d_channel(cm):
    """u = exp(i k x), k = 6 pi, u(0) = 1 on the plane x = 0 (Sec. 4.1)."""
    nx, k = 64, 6 * math.pi
    prob = ci.channel_dirichlet_f2((nx, 2, 2), k, 1.0)
    Ud, _ = F2(prob).direct()
    with cm.Solver(prob, "fp64", tol=1e-11, max_iter=5000, riesz_tol=1e-13) as s:
        U, rep = s.solve()
    assert rep["converged"]
    assert _rel(U, Ud) < 1e-8
    x = np.arange(nx + 1) / nx
    assert np.max(np.abs(U - np.exp(1j * k * x))) < 0.06


@pytest.mark.parametrize("formulation", [1, 2])
def test_neumann_data_channel_matches_oracle(cm, formulation):
    k = 2 * math.pi * 1.5
    n = (48, 4) if formulation == 1 else (32, 2, 2)
    prob = ci.channel_neumann_data(formulation, n, k)
    o = F1(prob) if formulation == 1 else F2(prob)
    Ud, _ = o.direct()
    kw = {} if formulation == 1 else {"riesz_tol": 1e-13}
    with cm.Solver(prob, "fp64", tol=1e-11, max_iter=5000, **kw) as s:
        U, rep = s.solve()
    assert rep["converged"]
    assert _rel(U, Ud) < 1e-8
