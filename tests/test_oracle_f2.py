"""Pins for the second-order (F2) oracle: closed-form leapfrog dispersion (including the start
and end maps), exact energy conservation with and without sound-soft nodes, the damped energy
identity, the 7-point interior stencil, brute-force dense transposes, the direct sparse solve of
the time-discretised Helmholtz system, the Riesz map as an exact elliptic inverse (eq.
CMCG_PRECONDITIONIER), CG monotonicity, the filter of eq. fundamental-frequency-solution on an
exact discrete harmonic and under the constant shift lambda of Thm. 1, and the paper's 1D
solutions exp(i k x) (Sec. 4.1) and 2 i sin(k x) (Dirichlet at 0, Sec. 4.1) in channel form."""
import math

import numpy as np
import pytest

import cmcg_inputs as ci
from cmcg_inputs import Problem
from oracle.f2 import F2


def _rng(seed=0):
    return np.random.default_rng(seed)


def _box(n, c=None, bc=None, mask=None, f=None, omega=2 * math.pi, N=None):
    dim = len(n)
    return F2(Problem(dim=dim, formulation=2, n=tuple(n), omega=omega, c=c, f=f,
                      sound_soft=mask, face_bc=tuple(bc if bc is not None else [1] * 2 * dim)), N=N)


@pytest.mark.parametrize("n,modes", [((10, 8), (3, 2)), ((6, 5, 4), (2, 1, 3))])
def test_dispersion_closed_form(n, modes):
    """A cosine mode in a Neumann box started at rest evolves as cos(n w_d dt) times the mode,
    sin^2(w_d dt/2) = (c dt/h)^2 sum_k sin^2(pi p_k / 2 n_k); the end map returns
    v^N = -sin(N w_d dt) sin(w_d dt) / dt times the mode."""
    c = 1.4
    s = _box(n, c=np.full(tuple(m + 1 for m in reversed(n)), c), omega=2 * math.pi * 2.3)
    axes = [np.cos(math.pi * p * np.arange(m + 1) / m) for m, p in zip(n, modes)]
    mode = axes[0]
    for a in axes[1:]:
        mode = np.multiply.outer(a, mode)
    lam = (c * s.dt / s.h) ** 2 * sum(math.sin(math.pi * p / (2 * m)) ** 2 for m, p in zip(n, modes))
    th = 2 * math.asin(math.sqrt(lam))
    z = np.concatenate([mode.ravel(), np.zeros(mode.size)])
    U = np.zeros(mode.shape, complex)
    out = s.period(z, False, U_acc=[U])
    ref_U = sum(math.cos(k * th) * np.exp(1j * s.omega * k * s.dt) for k in range(s.N))
    assert np.max(np.abs(U - ref_U * mode)) < 1e-11
    assert np.max(np.abs(out[: s.nn] - math.cos(s.N * th) * mode.ravel())) < 1e-12
    vN = -math.sin(s.N * th) * math.sin(th) / s.dt
    assert np.max(np.abs(out[s.nn:] - vN * mode.ravel())) < 1e-10 * (1 + abs(vN))


def test_interior_seven_point_stencil():
    s = _box((6, 6, 6))
    e = np.zeros(s.shape)
    e[3, 2, 4] = 1.0
    Se = s.S(e)
    h = s.h
    assert abs(Se[3, 2, 4] - 6 * h) < 1e-15
    for idx in ((2, 2, 4), (4, 2, 4), (3, 1, 4), (3, 3, 4), (3, 2, 3), (3, 2, 5)):
        assert abs(Se[idx] + h) < 1e-15
    assert abs(np.sum(np.abs(Se)) - 12 * h) < 1e-14
    # the edge-flux apply and the assembled matrix are two writings of the same S
    x = _rng(1).standard_normal(s.nn)
    assert np.max(np.abs(s.stiffness_matrix() @ x - s.S(x.reshape(s.shape)).ravel())) < 1e-12


@pytest.mark.parametrize("masked", [False, True])
def test_energy_conserved_without_absorption(masked):
    rng = _rng(2)
    n = (7, 6, 5)
    shape = tuple(m + 1 for m in reversed(n))
    mask = None
    if masked:
        mask = np.zeros(shape, np.uint8)
        mask[2:4, 3:5, 3] = 1
    s = _box(n, c=1 + rng.uniform(size=shape), mask=mask)
    R = s.free
    u_prev = R * rng.standard_normal(shape)
    u = R * rng.standard_normal(shape)
    E0 = s.energy(u, u_prev)
    for _ in range(300):
        u_next = R * (2 * u - u_prev - s.dt ** 2 * s.S(u) / s.M)
        u_prev, u = u, u_next
    assert abs(s.energy(u, u_prev) - E0) < 1e-11 * abs(E0)


def test_damped_energy_identity():
    """E^{n+1/2} - E^{n-1/2} = -dt w^T B w with w = (u^{n+1} - u^{n-1}) / (2 dt), driven by the
    period map itself (start map, steps, end map)."""
    rng = _rng(3)
    n = (6, 5, 4)
    shape = tuple(m + 1 for m in reversed(n))
    s = _box(n, c=1 + rng.uniform(size=shape), bc=[0, 1, 0, 0, 1, 0], omega=2 * math.pi * 1.5)
    R, beta, dt = s.free, s.beta, s.dt
    um = rng.standard_normal(shape)
    u = rng.standard_normal(shape)
    for _ in range(40):
        up = (2 * u - (1 - beta) * um - dt ** 2 * s.S(u) / s.M) / (1 + beta)
        w = (up - um) / (2 * dt)
        dE = s.energy(up, u) - s.energy(u, um)
        assert abs(dE + dt * np.sum(w * s.B * w)) < 1e-12 * s.energy(u, um)
        um, u = u, up


@pytest.mark.parametrize("n", [(5, 4), (3, 3, 2)])
def test_transpose_is_dense_brute_force_transpose(n):
    rng = _rng(4)
    dim = len(n)
    shape = tuple(m + 1 for m in reversed(n))
    mask = np.zeros(shape, np.uint8)
    mask.flat[3] = 1
    s = _box(n, c=1 + rng.uniform(size=shape), bc=[0, 1, 0, 0, 1, 0][: 2 * dim], mask=mask,
             omega=2 * math.pi * 1.3)
    E = np.column_stack([s.period(e, False) for e in np.eye(s.size)])
    for _ in range(3):
        y = rng.standard_normal(s.size)
        ref = E.T @ y
        assert np.max(np.abs(s.period_T(y) - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_adjoint_identity_3d():
    prob = ci.inclusions_3d(n=16, freq=2.0, n_incl=6, seed=3, width=0.1)
    s = F2(prob)
    rng = _rng(5)
    z, y = rng.standard_normal(s.size), rng.standard_normal(s.size)
    Ez = s.period(z, False)
    assert abs(Ez @ y - z @ s.period_T(y)) <= 1e-13 * np.linalg.norm(Ez) * np.linalg.norm(y)


@pytest.fixture(scope="module")
def inclusions_small():
    prob = ci.inclusions_3d(n=8, freq=1.5, n_incl=5, seed=9, width=0.15, r_range=(0.1, 0.3))
    s = F2(prob)
    rec = []
    z, hist, it = s.solve(tol=1e-12, max_iter=3000, record=rec)
    return s, z, hist, it, rec


def test_cmcg_matches_direct_solve_pure_neumann_riesz(inclusions_small):
    s, z, hist, it, _ = inclusions_small
    Ud, zd = s.direct()
    assert np.linalg.norm(s.filter(z) - Ud) / np.linalg.norm(Ud) < 1e-9


def test_lambda_shift_invisible_to_filter(inclusions_small):
    """Thm. 1 with no sound-soft part: (1, 0) is periodic, and the filter removes it."""
    s, z, _, _, _ = inclusions_small
    one = np.concatenate([np.ones(s.nn), np.zeros(s.nn)])
    assert np.max(np.abs(s.period(one, False) - one)) < 1e-12
    lam = 3.7 * np.max(np.abs(z))
    U1, U2 = s.filter(z), s.filter(z + lam * one)
    # rounding of the shifted trajectory scales with lam, not with U
    assert np.linalg.norm(U1 - U2) <= 1e-13 * s.N * lam * math.sqrt(s.nn)
    assert np.linalg.norm(U1 - U2) <= 1e-9 * np.linalg.norm(U1)


def test_cg_monotone(inclusions_small):
    s, z, _, _, rec = inclusions_small
    J = [s.functional(x) for x in rec[:60]]
    assert all(J[k + 1] <= J[k] * (1 + 1e-10) for k in range(len(J) - 1))


def test_filter_exact_on_discrete_harmonic(inclusions_small):
    s, _, _, _, _ = inclusions_small
    Ud, zd = s.direct()
    assert np.linalg.norm(s.period(zd, True) - zd) <= 1e-12 * np.linalg.norm(zd)
    assert np.linalg.norm(s.filter(zd) - Ud) <= 1e-12 * np.linalg.norm(Ud)


def test_step6_output_differs_by_discrete_frequency(inclusions_small):
    """The paper's Step 6 output v_0 + (i/omega) v_1 equals Re U + i (wh/omega) Im U on the
    discrete periodic state (wh = sin(omega dt)/dt), i.e. it differs from the filter by the
    factor wh/omega on the imaginary part."""
    s, _, _, _, _ = inclusions_small
    Ud, zd = s.direct()
    wh = math.sin(s.omega * s.dt) / s.dt
    ref = Ud.real + 1j * (wh / s.omega) * Ud.imag
    assert np.max(np.abs(s.step6_output(zd) - ref)) < 1e-12 * np.max(np.abs(Ud))


def test_riesz_is_elliptic_inverse():
    rng = _rng(6)
    n = (6, 5, 4)
    shape = tuple(m + 1 for m in reversed(n))
    # pure Neumann: S x = r for zero-sum r, x zero-sum
    s = _box(n, c=1 + rng.uniform(size=shape), bc=[0] * 6)
    r = rng.standard_normal(s.nn)
    r -= r.mean()
    x = s.riesz(np.concatenate([r, np.zeros(s.nn)]))[: s.nn]
    assert np.max(np.abs(s.S(x.reshape(shape)).ravel() - r)) < 1e-10 * np.max(np.abs(r))
    assert abs(x.sum()) < 1e-10 * np.max(np.abs(x)) * s.nn
    # with sound-soft nodes: S x = r on free nodes, x = 0 on D
    mask = np.zeros(shape, np.uint8)
    mask[1:3, 2, 2:4] = 1
    s = _box(n, c=1 + rng.uniform(size=shape), mask=mask)
    r = rng.standard_normal(s.nn) * s.free.ravel()
    x = s.riesz(np.concatenate([r, np.zeros(s.nn)]))[: s.nn]
    assert np.max(np.abs(x[mask.ravel() == 1])) == 0
    res = (s.free * s.S(x.reshape(shape))).ravel() - r
    assert np.max(np.abs(res)) < 1e-10 * np.max(np.abs(r))


@pytest.mark.parametrize("dirichlet", [False, True])
def test_channel_closed_forms_second_order(dirichlet):
    """exp(i k x) (absorbing data at both ends) and 2 i sin(k x) (sound-soft plane x = 0,
    absorbing at x = 1): nodal errors fall as h^2 in space and time."""
    k = 2 * math.pi * 1.5
    errs = []
    for nx in (16, 32):
        prob = ci.channel_plane_wave_f2((nx, 2), k, dirichlet_at_zero=dirichlet)
        s = F2(prob)
        z, hist, _ = s.solve(tol=1e-12, max_iter=4000)
        U = s.filter(z)
        Ud, _ = s.direct()
        assert np.linalg.norm(U - Ud) <= 1e-8 * np.linalg.norm(Ud)
        x = np.arange(nx + 1) / nx
        exact = 2j * np.sin(k * x) if dirichlet else np.exp(1j * k * x)
        errs.append(np.max(np.abs(U - exact[None, :])))
    assert errs[0] < 0.3
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_sound_soft_sphere_small():
    """Scattering by a voxelised sound-soft ball with plane-wave data on the outer faces:
    CMCG equals the direct solve and the field vanishes on the obstacle."""
    prob = ci.sound_soft_sphere_3d(n=8, freq=1.0, radius=0.2)
    s = F2(prob)
    z, _, _ = s.solve(tol=1e-12, max_iter=3000)
    U = s.filter(z)
    Ud, _ = s.direct()
    assert np.linalg.norm(U - Ud) / np.linalg.norm(Ud) < 1e-9
    assert np.max(np.abs(U[prob.sound_soft.astype(bool)])) == 0.0


def test_sound_soft_cavity_small():
    """A nonconvex obstacle (a box-shaped shell open on one face): CMCG still equals the direct
    solve of the time-discrete system, and the field vanishes on the obstacle."""
    prob = ci.sound_soft_cavity_3d(n=16, freq=1.0)
    s = F2(prob)
    assert 0 < int(prob.sound_soft.sum()) < s.nn
    z, _, _ = s.solve(tol=1e-12, max_iter=4000)
    U = s.filter(z)
    Ud, _ = s.direct()
    assert np.linalg.norm(U - Ud) / np.linalg.norm(Ud) < 1e-9
    assert np.max(np.abs(U[prob.sound_soft.astype(bool)])) == 0.0


def test_window_reproduces_full_grid_away_from_cuts():
    """Sampled checks at full size use node windows: a period of K steps is K + 1 sweeps, so a
    window reaching K + 2 nodes past a sample (cut sides Neumann) reproduces the full grid's
    forward, forced and transposed periods there.  The box has random c, a sound-soft ball,
    a source, random data on every face and mixed face types, so a wrongly sliced field, face
    or mask changes a sampled value."""
    from oracle.f2 import window
    n = (26, 22, 24)
    prob = ci.sound_soft_sphere_3d(n=24, freq=1.5, radius=0.2)
    rng = np.random.default_rng(17)
    shape = tuple(m + 1 for m in reversed(n))
    prob.n = n
    prob.spacing = 1.0 / 24
    prob.c = 1.0 + rng.uniform(size=shape)
    prob.sound_soft = ci.sphere_mask(n, prob.spacing, (0.55, 0.45, 0.5), 0.2)
    prob.f = np.zeros(shape, complex)
    prob.f[3:9, 12:18, 2:7] = rng.standard_normal((6, 6, 5)) + 1j
    gS = []
    for a in range(3):
        others = [b for b in range(3) if b != a]
        fshape = tuple(n[b] + 1 for b in reversed(others))
        gS += [rng.standard_normal(fshape) + 1j * rng.standard_normal(fshape) for _ in range(2)]
    prob.gS = gS
    prob.face_bc = (0, 1, 0, 0, 1, 0)
    K = 5
    full = F2(prob, N=K)
    z = rng.standard_normal(full.size) * np.concatenate([full.free.ravel()] * 2)
    outs = {"fwd": full.period(z, False), "forced": full.period(z, True),
            "adj": full.period_T(z)}
    zu = z[: full.nn].reshape(full.shape)
    zv = z[full.nn:].reshape(full.shape)
    # samples (x, y, z): corners, faces, next to the ball, interior
    ball = (int(round(0.55 * 24 + 0.2 * 24)) + 1, int(round(0.45 * 24)), 12)
    samples = [(0, 0, 0), (26, 22, 24), (26, 0, 11), (0, 11, 24), ball, (8, 15, 5)]
    m = K + 2
    for s in samples:
        lo = [max(0, s[a] - m) for a in range(3)]
        hi = [min(n[a], s[a] + m) for a in range(3)]
        sub = F2(window(prob, lo, hi), N=K)
        assert sub.dt == full.dt
        sl = tuple(slice(lo[a], hi[a] + 1) for a in (2, 1, 0))
        zs = np.concatenate([zu[sl].ravel(), zv[sl].ravel()])
        subs = {"fwd": sub.period(zs, False), "forced": sub.period(zs, True),
                "adj": sub.period_T(zs)}
        li = (s[2] - lo[2], s[1] - lo[1], s[0] - lo[0])
        gi = (s[2], s[1], s[0])
        for key in outs:
            for part in range(2):
                a = outs[key][part * full.nn:(part + 1) * full.nn].reshape(full.shape)[gi]
                b = subs[key][part * sub.nn:(part + 1) * sub.nn].reshape(sub.shape)[li]
                assert abs(a - b) <= 1e-13 * (1 + abs(a)), (key, part, s, a, b)
