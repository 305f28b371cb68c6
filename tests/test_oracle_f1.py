"""Pins for the first-order (F1) oracle against facts fixed by the paper and by mathematics,
not by the oracle itself: closed-form leapfrog dispersion, the CFL limit, exact discrete
energy conservation and the damped energy identity, brute-force dense transposes, the direct
sparse solve of the time-discretised Helmholtz system (the paper's Sec. 4.1 check in fully
discrete form), CG monotonicity, the filter of eq. TH_FILTERED_MIXED_SOLUTION on an exact
discrete harmonic and under the divergence-free null space of Thm. 2, the square's symmetry,
reciprocity, and the paper's 1D solution u = exp(i k x) (Sec. 4.1) in channel form."""
import math

import numpy as np
import pytest

import cmcg_inputs as ci
from cmcg_inputs import Problem
from oracle.f1 import F1, window


def _rng(seed=0):
    return np.random.default_rng(seed)


def _neumann_box(nx, ny, c, omega=2 * math.pi, N=None, courant=0.5):
    p = Problem(dim=2, formulation=1, n=(nx, ny), omega=omega, c=c, face_bc=(1, 1, 1, 1),
                courant=courant)
    return F1(p, N=N)


def test_dispersion_closed_form():
    """A cosine mode in a Neumann box with p = 0 evolves as cos(n w_d dt) times the mode,
    sin^2(w_d dt / 2) = (c dt / h)^2 (sin^2(pi p / 2nx) + sin^2(pi q / 2ny))."""
    nx, ny, pm, qm, c = 12, 10, 3, 2, 1.3
    s = _neumann_box(nx, ny, np.full((ny, nx), c), omega=2 * math.pi * 1.7)
    i = np.arange(nx)
    j = np.arange(ny)
    mode = np.outer(np.cos(math.pi * qm * (j + 0.5) / ny), np.cos(math.pi * pm * (i + 0.5) / nx))
    lam = (c * s.dt / s.h) ** 2 * (math.sin(math.pi * pm / (2 * nx)) ** 2
                                   + math.sin(math.pi * qm / (2 * ny)) ** 2)
    wd_dt = 2 * math.asin(math.sqrt(lam))
    Px, Py, v = np.zeros((ny, nx - 1)), np.zeros((ny - 1, nx)), mode.copy()
    for n in range(1, 60):
        Px, Py, v = s.step(Px, Py, v, n, forced=False)
        assert np.max(np.abs(v - math.cos(n * wd_dt) * mode)) < 1e-12


@pytest.mark.parametrize("cdt_h,stable", [(0.70, True), (0.72, False)])
def test_cfl_limit(cdt_h, stable):
    """The staggered scheme is stable iff c dt / h <= 1/sqrt(2): just below the highest mode
    stays bounded, just above it grows."""
    n = 12
    s = _neumann_box(n, n, np.ones((n, n)))
    s.dt = cdt_h * s.h
    s.gamma = np.zeros((n, n))
    i = np.arange(n)
    top = np.cos(math.pi * (n - 1) * (i + 0.5) / n)
    v = np.outer(top, top)
    Px, Py = np.zeros((n, n - 1)), np.zeros((n - 1, n))
    amp = []
    for _ in range(400):
        Px, Py, v = s.step(Px, Py, v, 0, forced=False)
        amp.append(np.abs(v).max())
    assert (max(amp) < 2.0) == stable


def test_energy_conserved_without_absorption():
    nx, ny = 14, 11
    rng = _rng(1)
    s = _neumann_box(nx, ny, 1.0 + rng.uniform(size=(ny, nx)))
    Px, Py, v = rng.standard_normal((ny, nx - 1)), rng.standard_normal((ny - 1, nx)), \
        rng.standard_normal((ny, nx))
    E0 = s.energy(Px, Py, v)
    for _ in range(100):
        z = s.period(s.pack(Px, Py, v), forced=False)
        Px, Py, v = s.unpack(z)
    assert abs(s.energy(Px, Py, v) - E0) / E0 < 1e-12


def test_damped_energy_identity():
    """E^{n+1} - E^n = - sum_cells dt h m / (4 c) (v^{n+1} + v^n)^2."""
    rng = _rng(2)
    p = Problem(dim=2, formulation=1, n=(9, 7), omega=5.0, c=1 + rng.uniform(size=(7, 9)),
                face_bc=(0, 0, 0, 1))
    s = F1(p)
    Px, Py, v = rng.standard_normal((7, 8)), rng.standard_normal((6, 9)), rng.standard_normal((7, 9))
    for n in range(30):
        E0 = s.energy(Px, Py, v)
        Px2, Py2, v2 = s.step(Px, Py, v, n, forced=False)
        dE = s.energy(Px2, Py2, v2) - E0
        loss = np.sum(s.dt * s.h * s.m / (4 * s.c) * (v2 + v) ** 2)
        assert abs(dE + loss) <= 1e-13 * E0
        Px, Py, v = Px2, Py2, v2


def test_transpose_is_dense_brute_force_transpose():
    rng = _rng(3)
    p = Problem(dim=2, formulation=1, n=(6, 5), omega=7.0, c=1 + rng.uniform(size=(5, 6)),
                face_bc=(0, 1, 0, 0))
    s = F1(p)
    E = np.column_stack([s.period(e, False) for e in np.eye(s.size)])
    for _ in range(3):
        y = rng.standard_normal(s.size)
        ref = E.T @ y
        assert np.max(np.abs(s.period_T(y) - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_adjoint_identity():
    """<E z, y> = <z, E^T y> to 1e-13 on a larger grid."""
    rng = _rng(4)
    prob = ci.random_medium_2d(n=32, freq=3.0, n_src=2, seed=5)
    s = F1(prob)
    z, y = rng.standard_normal(s.size), rng.standard_normal(s.size)
    lhs = s.period(z, False) @ y
    rhs = z @ s.period_T(y)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(s.period(z, False)) * np.linalg.norm(y)


@pytest.fixture(scope="module")
def small_random():
    prob = ci.random_medium_2d(n=16, freq=2.0, n_src=2, seed=11, width=0.08)
    s = F1(prob)
    rec = []
    z, hist, it = s.solve(tol=1e-13, max_iter=4000, record=rec)
    return prob, s, z, hist, it, rec


def test_cmcg_matches_direct_solve(small_random):
    """CMCG converges to the solution of the time-discretised Helmholtz system
    (Sec. 4.1, fully discrete)."""
    _, s, z, hist, it, _ = small_random
    U = s.filter(z)
    Ud, _ = s.direct()
    assert np.linalg.norm(U - Ud) / np.linalg.norm(Ud) < 1e-9
    assert hist[-1] <= 1e-13


def test_direct_state_is_periodic(small_random):
    _, s, _, _, _, _ = small_random
    _, zd = s.direct()
    assert np.linalg.norm(s.period(zd, True) - zd) <= 1e-12 * np.linalg.norm(zd)


def test_cg_monotone(small_random):
    """J(z_l) and ||z_l - z*||_{M_E} are non-increasing along PCG (Hestenes-Stiefel)."""
    _, s, z, _, _, rec = small_random
    J = [s.functional(x) for x in rec[:80]]
    assert all(J[k + 1] <= J[k] * (1 + 1e-10) + 1e-300 for k in range(len(J) - 1))
    w = s.weights()
    err = [math.sqrt(np.sum(w * (x - z) ** 2)) for x in rec[:80]]
    assert all(err[k + 1] <= err[k] * (1 + 1e-9) for k in range(len(err) - 1))


def test_filter_exact_on_discrete_harmonic(small_random):
    _, s, _, _, _, _ = small_random
    Ud, zd = s.direct()
    assert np.linalg.norm(s.filter(zd) - Ud) <= 1e-12 * np.linalg.norm(Ud)


def _curl(s, psi):
    """Discrete curl of a vertex potential vanishing on the boundary: divergence free."""
    nx, ny, h = s.nx, s.ny, s.h
    full = np.zeros((ny + 1, nx + 1))
    full[1:-1, 1:-1] = psi
    Px = (full[1:, 1:-1] - full[:-1, 1:-1]) / h           # (ny, nx-1)
    Py = -(full[1:-1, 1:] - full[1:-1, :-1]) / h          # (ny-1, nx)
    return Px, Py


def test_filter_invariant_under_divergence_free_flux(small_random):
    """Thm. 2: p_0 is determined only up to a divergence-free field; the filtered output is
    not affected by it."""
    _, s, z, _, _, _ = small_random
    psi = _rng(6).standard_normal((s.ny - 1, s.nx - 1))
    Px, Py = _curl(s, psi)
    assert np.max(np.abs(s.div(Px, Py))) < 1e-10
    dz = s.pack(Px, Py, np.zeros((s.ny, s.nx)))
    assert np.linalg.norm(s.period(dz, False) - dz) <= 1e-12 * np.linalg.norm(dz)
    U1, U2 = s.filter(z), s.filter(z + dz)
    assert np.linalg.norm(U1 - U2) <= 1e-12 * np.linalg.norm(U1)


def test_periodic_null_space_dimension():
    """ker(E - I) is exactly the (nx-1)(ny-1)-dimensional divergence-free flux space."""
    p = Problem(dim=2, formulation=1, n=(5, 4), omega=6.0, c=1.0 + 0.3 * _rng(7).uniform(size=(4, 5)),
                face_bc=(0, 0, 0, 0))
    s = F1(p)
    E = np.column_stack([s.period(e, False) for e in np.eye(s.size)])
    sv = np.linalg.svd(E - np.eye(s.size), compute_uv=False)
    assert int(np.sum(sv < 1e-10 * sv.max())) == (5 - 1) * (4 - 1)


def test_channel_plane_wave_converges():
    """Channel form of u = exp(i k x) (Sec. 4.1).  With cell-centred v the absorbing condition
    is imposed with the centre value h/2 inside the boundary, which is a first-order closure:
    the error halves with h (ratios measured 1.93, 1.94, 1.98, 1.99 for n = 16 .. 256) and is
    not a time-step effect (eight times smaller dt changes it by under 1%)."""
    errs = []
    k = 2 * math.pi * 1.5
    for n in (32, 64):
        prob = ci.channel_plane_wave_f1(n, 4, k)
        s = F1(prob)
        U, _ = s.direct()
        z, _, _ = s.solve(tol=1e-12, max_iter=5000)
        Uc = s.filter(z)
        assert np.linalg.norm(Uc - U) / np.linalg.norm(U) < 1e-8
        x = (np.arange(n) + 0.5) / n
        exact = np.exp(1j * k * x)[None, :]
        errs.append(np.max(np.abs(Uc - exact)))
    assert errs[0] < 0.15
    assert 1.85 < errs[0] / errs[1] < 2.15


def test_square_symmetry():
    """Constant c, centred source, all sides absorbing: u has the square's 8 symmetries."""
    prob = ci.single_source_2d(n=20, omega=2 * math.pi * 2, width=0.1)
    s = F1(prob)
    z, _, _ = s.solve(tol=1e-12, max_iter=5000)
    U = s.filter(z)
    for V in (U.T, U[::-1, :], U[:, ::-1], U[::-1, ::-1], U.T[::-1, :]):
        assert np.max(np.abs(U - V)) <= 1e-9 * np.max(np.abs(U))


def test_reciprocity():
    """The time-discretised Helmholtz operator is complex symmetric once the face unknowns are
    eliminated: the response at b to a unit source at a equals the response at a to one at b."""
    rng = _rng(8)
    nx = ny = 12
    c = 1 + rng.uniform(size=(ny, nx))
    a, b = (2, 3), (9, 7)
    out = []
    for src, rec in ((a, b), (b, a)):
        f = np.zeros((ny, nx), complex)
        f[src] = 1.0
        p = Problem(dim=2, formulation=1, n=(nx, ny), omega=2 * math.pi * 1.2, c=c, f=f,
                    face_bc=(0, 0, 0, 0))
        s = F1(p)
        z, _, _ = s.solve(tol=1e-13, max_iter=5000)
        out.append(s.filter(z)[rec])
    assert abs(out[0] - out[1]) <= 1e-9 * abs(out[0])


def test_window_reproduces_full_grid_away_from_cuts():
    """Sampled checks at full size use sub-windows: after K steps a cell only feels cells
    within K + 2, so a window with margin K + 2 reproduces the full-grid values."""
    prob = ci.random_medium_2d(n=48, freq=4.0, n_src=3, seed=3)
    full = F1(prob)
    K = 9
    rng = _rng(9)
    z = rng.standard_normal(full.size)
    zf = full.unpack(full.period(z, True, steps=K))
    Pxf, Pyf, vf = full.unpack(z)
    for (ci0, cj0) in ((0, 0), (20, 30), (47, 5)):
        m = K + 2
        i0, i1 = max(0, ci0 - m), min(48, ci0 + m + 1)
        j0, j1 = max(0, cj0 - m), min(48, cj0 + m + 1)
        sub = F1(window(prob, i0, i1, j0, j1), N=full.N)
        zs = sub.pack(Pxf[j0:j1, i0:i1 - 1], Pyf[j0:j1 - 1, i0:i1], vf[j0:j1, i0:i1])
        Pxs, Pys, vs = sub.unpack(sub.period(zs, True, steps=K))
        assert abs(vs[cj0 - j0, ci0 - i0] - zf[2][cj0, ci0]) < 1e-13 * (1 + abs(zf[2][cj0, ci0]))


@pytest.mark.slow
def test_single_source_128_end_to_end():
    """The 128^2, 4-wavelength, sigma = 0.5 configuration: N = 64, dt = 1/256, converges to
    1e-8 and agrees with the direct solve to the accuracy the tolerance allows."""
    s = F1(ci.single_source_2d())
    assert s.N == 64 and abs(s.dt - 1.0 / 256) < 1e-15
    z, hist, it = s.solve(tol=1e-8, max_iter=2000)
    assert hist[-1] <= 1e-8 and it < 1000
    U = s.filter(z)
    Ud, _ = s.direct()
    assert np.linalg.norm(U - Ud) / np.linalg.norm(Ud) < 1e-7
