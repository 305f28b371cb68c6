"""General boundary data in the oracle (eq. HE with f, gS, gN, gD): inhomogeneous Neumann data
on both formulations and inhomogeneous Dirichlet data on the nodal one, against closed forms."""
import math

import numpy as np
import pytest

import cmcg_inputs as ci
from oracle.f1 import F1
from oracle.f2 import F2


@pytest.mark.parametrize("formulation", [1, 2])
def test_neumann_data_channel(formulation):
    """u = exp(i k x) with gN = -i k on the Neumann face x = 0 and an absorbing face at x = 1:
    first-order convergence on the staggered grid (cell-centred closure), second order on the
    nodal grid; CMCG equals the direct solve."""
    k = 2 * math.pi * 1.5
    errs = []
    for nx in (32, 64, 128):
        n = (nx, 4) if formulation == 1 else (nx, 2)
        prob = ci.channel_neumann_data(formulation, n, k)
        s = F1(prob) if formulation == 1 else F2(prob)
        U, _ = s.direct()
        x = (np.arange(nx) + 0.5) / nx if formulation == 1 else np.arange(nx + 1) / nx
        errs.append(np.max(np.abs(U - np.exp(1j * k * x)[None, :])))
        if nx == 32:
            z, _, _ = s.solve(tol=1e-12, max_iter=5000)
            assert np.linalg.norm(s.filter(z) - U) <= 1e-9 * np.linalg.norm(U)
    lo, hi = (1.85, 2.3) if formulation == 1 else (3.7, 4.4)
    for a, b in zip(errs, errs[1:]):
        assert lo < a / b < hi


def test_dirichlet_data_reciprocity_of_the_state():
    """Dirichlet data enters only the forced period: the homogeneous period and its transpose
    are those of the homogeneous-Dirichlet problem, and the state stays zero on the Dirichlet
    nodes."""
    base = ci.sound_soft_sphere_3d(n=8, freq=1.0, radius=0.2)
    rng = np.random.default_rng(3)
    gD = (rng.standard_normal(base.sound_soft.shape) + 1j * rng.standard_normal(base.sound_soft.shape))
    import dataclasses
    withdata = dataclasses.replace(base, gD=gD)
    a, b = F2(base), F2(withdata)
    z = rng.standard_normal(a.size) * np.concatenate([a.free.ravel()] * 2)
    assert np.array_equal(a.period(z, False), b.period(z, False))
    phi = b.period(z, True)
    assert np.all(phi[: b.nn][b.free.ravel() < 0.5] == 0) and np.all(phi[b.nn:][b.free.ravel() < 0.5] == 0)
    U, _ = b.direct()
    assert np.allclose(U[base.sound_soft.astype(bool)], gD[base.sound_soft.astype(bool)], atol=0, rtol=0)
    zc, _, _ = b.solve(tol=1e-12, max_iter=3000)
    assert np.linalg.norm(b.filter(zc) - U) <= 1e-9 * np.linalg.norm(U)
