"""GPU parity for the second-order (F2, nodal 3D) path against the FP64 CPU oracle: periods, the
literal transpose, the Riesz map, the filter and full CMCG solves, element by element."""
import math

import numpy as np
import pytest

import cmcg_inputs as ci
from cmcg_inputs import Problem
from oracle.f2 import F2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    from paper_1903_12522_amd import cmcg
    return cmcg


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _mixed3d(n=(13, 11, 9), seed=3, masked=True):
    """Ragged box (rows of 14 nodes, several x tiles only at larger sizes), random c, a
    sound-soft block, complex source, boundary data on absorbing faces, one Neumann face pair."""
    rng = np.random.default_rng(seed)
    shape = tuple(m + 1 for m in reversed(n))
    c = 1.0 + rng.uniform(size=shape)
    f = np.zeros(shape, complex)
    f[2:5, 3:6, 4:8] = rng.standard_normal((3, 3, 4)) + 1j * rng.standard_normal((3, 3, 4))
    mask = None
    if masked:
        mask = np.zeros(shape, np.uint8)
        mask[4:6, 5:8, 6:9] = 1
    bc = (0, 0, 1, 0, 0, 1)
    gS = []
    for axis in range(3):
        others = [a for a in range(3) if a != axis]
        fshape = tuple(n[a] + 1 for a in reversed(others))
        for side in range(2):
            gS.append(rng.standard_normal(fshape) + 1j * rng.standard_normal(fshape))
    return Problem(dim=3, formulation=2, n=n, omega=2 * math.pi * 1.7, c=c, f=f, gS=gS,
                   sound_soft=mask, face_bc=bc, courant=0.5, name="mixed3d")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_temporal_blocking_is_bitwise(cm, prec):
    """Blocked launches (K = 2, 3, 4 homogeneous steps) give the same forward and backward
    periods bit for bit as one step per launch: every real node sees the same operands in the
    same order (a halo, LDS or barrier mistake would not).  71 x 31 x 41 nodes: two x tiles,
    several y tiles, two z chunks, a sound-soft block, absorbing and Neumann faces."""
    prob = _mixed3d(n=(70, 30, 40), seed=8)
    o = F2(prob)
    rng = np.random.default_rng(9)
    z = rng.standard_normal(o.size) * np.concatenate([o.free.ravel()] * 2)
    outs = []
    for k in (1, 2, 3, 4):
        with cm.Solver(prob, prec, steps_per_launch=k) as s:
            assert s.info["steps_per_launch"] == k
            outs.append((s.apply(cm.OP_FORWARD, z), s.apply(cm.OP_ADJOINT, z)))
    with cm.Solver(prob, prec) as s:
        # the nodal defaults: 4 steps per launch in FP32 (3 rows per wavefront), 3 in FP64 (2)
        assert s.info["steps_per_launch"] == (4 if prec == "fp32" else 3)
        assert (s.info["block_rows"], s.info["block_waves"]) == ((3 if prec == "fp32" else 2), 16)
    for k, (a, b) in zip((2, 3, 4), outs[1:]):
        assert np.array_equal(a, outs[0][0]), (k, np.max(np.abs(a - outs[0][0])))
        assert np.array_equal(b, outs[0][1]), (k, np.max(np.abs(b - outs[0][1])))
    if prec == "fp64":
        assert _rel(outs[2][0], o.period(z, False)) < 1e-13
        assert _rel(outs[2][1], o.period_T(z)) < 1e-13


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_blocked_tile_height_is_bitwise(cm, prec, monkeypatch):
    """Tiles of one row per wavefront (64 x 16) and of two (64 x 32, CMCG_F2_RPW=2; in FP32 also
    three and four, 64 x 48 and 64 x 64) give the same periods bit for bit on a ragged box with a
    sound-soft block and mixed faces, where tile edges fall at different rows."""
    prob = _mixed3d(n=(70, 45, 40), seed=12)
    o = F2(prob)
    z = np.random.default_rng(13).standard_normal(o.size) * np.concatenate([o.free.ravel()] * 2)
    outs = []
    for rpw in ("1", "2", "3", "4") if prec == "fp32" else ("1", "2"):
        monkeypatch.setenv("CMCG_F2_RPW", rpw)
        with cm.Solver(prob, prec, steps_per_launch=3) as s:
            outs.append((s.apply(cm.OP_FORWARD, z), s.apply(cm.OP_ADJOINT, z)))
    for out in outs[1:]:
        assert np.array_equal(outs[0][0], out[0])
        assert np.array_equal(outs[0][1], out[1])


@pytest.mark.parametrize("prec,rpw,chunk", [("fp64", None, None), ("fp32", None, None),
                                            ("fp64", "2", "32"), ("fp32", "2", "32"),
                                            ("fp32", "3", "32"), ("fp32", "4", "32"),
                                            ("fp32", "3", "16")])
def test_blocking_bitwise_around_a_sound_soft_ball(cm, prec, rpw, chunk, monkeypatch):
    """129^3 nodes, a sound-soft ball in the middle: interior tiles whose columns cross the
    ball's bounding box but whose plane chunk lies above or below it take the unmasked inner
    path, the others the masked one, and tiles whose chunk is clear of the z faces too the
    z-interior path (with chunks of 16 or 32 planes); blocked periods (K = 2, 3, 4) equal one
    step per launch bit for bit, in the default tile shape and in tiles of 2, 3 and 4 rows per
    wavefront, and the ball's nodes stay zero."""
    import torch
    if rpw:
        monkeypatch.setenv("CMCG_F2_RPW", rpw)
        monkeypatch.setenv("CMCG_F2_CHUNK", chunk)
    prob = ci.sound_soft_sphere_3d(n=128, freq=6.0, radius=0.15)
    mask = torch.as_tensor(np.concatenate([prob.sound_soft.ravel()] * 2) != 0).cuda()
    with cm.Solver(prob, prec, steps_per_launch=1) as s:
        n = s.info["state_len"]
        g = torch.Generator(device="cuda").manual_seed(15)
        z = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
        z[mask] = 0.0
        ref = (s.apply(cm.OP_FORWARD, z), s.apply(cm.OP_ADJOINT, z))
    assert torch.all(ref[0][mask] == 0) and torch.all(ref[1][mask] == 0)
    for k in (2, 3, 4):
        with cm.Solver(prob, prec, steps_per_launch=k) as s:
            out = (s.apply(cm.OP_FORWARD, z), s.apply(cm.OP_ADJOINT, z))
        for a, b in zip(out, ref):
            assert torch.equal(a, b), (k, (a - b).abs().max().item())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_blocking_bitwise_on_a_wide_box_without_mask(cm, prec):
    """201 x 151 x 81 nodes, absorbing and Neumann faces, random c, no sound-soft node: four x
    tiles and several y tiles, so the blocked launch takes every unmasked tile path (interior
    and z-interior tiles, tiles on a y face only, tiles on an x face); blocked periods (K = 2, 3,
    4) equal one step per launch bit for bit."""
    import torch
    prob = _mixed3d(n=(200, 150, 80), seed=21, masked=False)
    with cm.Solver(prob, prec, steps_per_launch=1) as s:
        n = s.info["state_len"]
        g = torch.Generator(device="cuda").manual_seed(22)
        z = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
        ref = (s.apply(cm.OP_FORWARD, z), s.apply(cm.OP_ADJOINT, z))
    for k in (2, 3, 4):
        with cm.Solver(prob, prec, steps_per_launch=k) as s:
            out = (s.apply(cm.OP_FORWARD, z), s.apply(cm.OP_ADJOINT, z))
        for a, b in zip(out, ref):
            assert torch.equal(a, b), (k, (a - b).abs().max().item())


def test_report_counts_compulsory_traffic(cm):
    """cmcg_report.dram_bytes of a nodal solve: blocked interior steps (5 words per 3 steps)
    and single-step start, end, metric and scaling sweeps, all in FP64: between the blocked rate
    and a few single-step passes (4 words) per node-step."""
    prob = ci.inclusions_3d(n=32, freq=1.5, n_incl=4, seed=9, width=0.12, r_range=(0.1, 0.25))
    with cm.Solver(prob, "fp64", tol=1e-6, max_iter=2000) as s:
        _, rep = s.solve()
    per = rep["dram_bytes"] / rep["grid_updates"]
    assert 5 * 8 / 3 <= per < 3 * 32, per


@pytest.mark.parametrize("masked", [True, False])
def test_periods_match_oracle_fp64(cm, masked):
    prob = _mixed3d(masked=masked)
    o = F2(prob)
    rng = np.random.default_rng(5)
    z = rng.standard_normal(o.size)
    z[: o.nn] *= o.free.ravel()
    z[o.nn:] *= o.free.ravel()
    with cm.Solver(prob, "fp64") as s:
        assert s.info["steps_per_period"] == o.N
        assert _rel(s.apply(cm.OP_FORWARD, z), o.period(z, False)) < 1e-13
        assert _rel(s.apply(cm.OP_FORCED, z), o.period(z, True)) < 1e-13
        assert _rel(s.apply(cm.OP_ADJOINT, z), o.period_T(z)) < 1e-13
        y = rng.standard_normal(o.size) * np.concatenate([o.free.ravel()] * 2)
        if not masked:
            y[: o.nn] -= y[: o.nn].mean()
        else:
            pass
        assert _rel(s.apply(cm.OP_RIESZ, y), o.riesz(y)) < 1e-8


def test_riesz_solve_at_its_iteration_cap_is_reported(cm):
    """A Riesz PCG solve that stops at riesz_max_iter above riesz_tol is not passed off as
    exact: cmcg_apply(OP_RIESZ) returns CMCG_ENOTCONV, the solve counts it in the report and
    returns CMCG_ENOTCONV; with the default cap nothing is flagged."""
    prob = ci.inclusions_3d(n=16, freq=1.5, n_incl=4, seed=9, width=0.12, r_range=(0.1, 0.25))
    o = F2(prob)
    y = np.random.default_rng(3).standard_normal(o.size)
    y[: o.nn] -= y[: o.nn].mean()
    with cm.Solver(prob, "fp64", tol=1e-6, max_iter=50, riesz_mode="solve", riesz_tol=1e-12,
                   riesz_max_iter=1) as s:
        s.apply(cm.OP_RIESZ, y)
        assert s.last_status == cm.ENOTCONV
        _, rep = s.solve()
        assert rep["riesz_unconverged"] > 0 and not rep["converged"]
    with cm.Solver(prob, "fp64", tol=1e-6, max_iter=2000, riesz_mode="solve") as s:
        s.apply(cm.OP_RIESZ, y)
        assert s.last_status == cm.OK
        _, rep = s.solve()
        assert rep["riesz_unconverged"] == 0 and rep["converged"]


def test_periods_fp32_within_rounding(cm):
    prob = _mixed3d(n=(70, 9, 8), seed=4)
    o = F2(prob)
    z = np.random.default_rng(6).standard_normal(o.size)
    z *= np.concatenate([o.free.ravel()] * 2)
    with cm.Solver(prob, "fp32") as s:
        assert _rel(s.apply(cm.OP_FORWARD, z), o.period(z, False)) < 5e-5
        assert _rel(s.apply(cm.OP_ADJOINT, z), o.period_T(z)) < 5e-5


def test_filter_matches_oracle(cm):
    prob = _mixed3d(seed=7)
    o = F2(prob)
    z = np.random.default_rng(8).standard_normal(o.size) * np.concatenate([o.free.ravel()] * 2)
    with cm.Solver(prob, "fp64") as s:
        assert _rel(s.filter(z), o.filter(z)) < 1e-13


def test_adjoint_identity_on_gpu(cm):
    prob = ci.inclusions_3d(n=32, freq=3.0, n_incl=8, seed=3, width=0.06)
    o = F2(prob)
    rng = np.random.default_rng(9)
    z, y = rng.standard_normal(o.size), rng.standard_normal(o.size)
    with cm.Solver(prob, "fp64") as s:
        Ez = s.apply(cm.OP_FORWARD, z)
        ETy = s.apply(cm.OP_ADJOINT, y)
    assert abs(Ez @ y - z @ ETy) <= 1e-13 * np.linalg.norm(Ez) * np.linalg.norm(y)


@pytest.mark.parametrize("kind", ["inclusions", "sphere"])
def test_cmcg_fp64_matches_oracle(cm, kind):
    if kind == "inclusions":
        prob = ci.inclusions_3d(n=12, freq=1.5, n_incl=6, seed=9, width=0.12, r_range=(0.1, 0.25))
    else:
        prob = ci.sound_soft_sphere_3d(n=12, freq=1.2, radius=0.2)
    o = F2(prob)
    zo, hist, it = o.solve(tol=1e-11, max_iter=3000)
    Uo = o.filter(zo)
    with cm.Solver(prob, "fp64", tol=1e-11, max_iter=3000, riesz_tol=1e-13) as s:
        U, rep = s.solve()
    assert rep["converged"]
    assert abs(rep["iterations"] - it) <= 2
    assert _rel(U, Uo) < 1e-9
    Ud, _ = o.direct()
    assert _rel(U, Ud) < 1e-8


def test_cg_iterates_track_oracle(cm):
    prob = ci.inclusions_3d(n=10, freq=1.5, n_incl=4, seed=2, width=0.15, r_range=(0.1, 0.3))
    o = F2(prob)
    rec = []
    o.solve(tol=0.0, max_iter=5, record=rec)
    with cm.Solver(prob, "fp64", tol=0.0, max_iter=5, riesz_tol=1e-13) as s:
        s.begin()
        for l in range(1, 6):
            s.iterate(1)
            zg = s.state(0)
            # the constant shift (lambda) is not fixed by CG: compare modulo constants in u
            du = zg[: o.nn] - rec[l][: o.nn]
            du -= du.mean()
            assert np.linalg.norm(du) <= 1e-9 * np.linalg.norm(rec[l][: o.nn])
            assert _rel(zg[o.nn:], rec[l][o.nn:]) < 1e-9


def test_fp32_mixed_matches_fp64(cm):
    prob = ci.inclusions_3d(n=32, freq=3.0, n_incl=10, seed=4, width=0.05)
    with cm.Solver(prob, "fp64", tol=1e-6, max_iter=2000) as s:
        U64, r64 = s.solve()
    with cm.Solver(prob, "fp32", tol=1e-6, max_iter=2000) as s:
        U32, r32 = s.solve()
    assert r64["converged"] and r32["converged"]
    assert _rel(U32, U64) < 1e-4
    assert r32["iterations"] <= 1.2 * r64["iterations"] + 5


@pytest.mark.parametrize("riesz", ["solve", "vcycle"])
@pytest.mark.parametrize("n,freq,width", [(32, 3.0, 0.05), (128, 8.0, 0.02)])
def test_fp32_mixed_storage_tracks_fp64(cm, n, freq, width, riesz):
    """FP32-mixed CG stores its residuals and the iterate's correction since the last reliable
    update in FP32 (FP64 arithmetic; the FP64 iterate is brought up to date at every refresh):
    the solution stays within 1e-4 of the FP64 solve's, in as many iterations within 5%."""
    prob = ci.inclusions_3d(n=n, freq=freq, n_incl=10, seed=4, width=width)
    with cm.Solver(prob, "fp64", tol=1e-6, max_iter=4000, riesz_mode=riesz) as s:
        U64, r64 = s.solve()
    with cm.Solver(prob, "fp32", tol=1e-6, max_iter=4000, riesz_mode=riesz) as s:
        U32, r32 = s.solve()
    assert r64["converged"] and r32["converged"]
    assert _rel(U32, U64) < 1e-4
    assert abs(r32["iterations"] - r64["iterations"]) <= 0.05 * r64["iterations"] + 1, \
        (r32["iterations"], r64["iterations"])


def test_sound_soft_field_vanishes_on_obstacle(cm):
    prob = ci.sound_soft_sphere_3d(n=24, freq=2.0, radius=0.2)
    with cm.Solver(prob, "fp64", tol=1e-8, max_iter=2000) as s:
        U, rep = s.solve()
    assert rep["converged"]
    assert np.max(np.abs(U[prob.sound_soft.astype(bool)])) == 0.0


@pytest.mark.parametrize("example", ["convergence_rates", "bounded_domain_filter"])
def test_paper_1d_examples_as_3d_channels(cm, example):
    """The paper's worked examples of Sec. 3.4 (u = -exp(i k x), k = 5 pi / 4, Dirichlet at 0,
    lifted to homogeneous data) and Sec. 3.5 (u = 16 x^2 (x - 1)^2, all faces Neumann, k = pi / 4)
    as 3D channels: the FP64 GPU solve equals the oracle's and the closed form to the
    discretisation error."""
    nx = 32
    if example == "convergence_rates":
        k = 5 * math.pi / 4
        prob = ci.channel_plane_wave_f2((nx, 2, 2), k, dirichlet_at_zero=True)
    else:
        k = math.pi / 4
        prob = ci.channel_bounded_neumann_f2((nx, 2, 2), k)
    o = F2(prob)
    Ud, _ = o.direct()
    with cm.Solver(prob, "fp64", tol=1e-11, max_iter=5000, riesz_tol=1e-13) as s:
        U, rep = s.solve()
    assert rep["converged"]
    assert _rel(U, Ud) < 1e-8
    x = np.arange(nx + 1) / nx
    if example == "convergence_rates":
        uh = -U - np.exp(-1j * k * x)
        assert np.max(np.abs(uh + np.exp(1j * k * x))) < 0.01
    else:
        assert np.max(np.abs(U - 16 * x ** 2 * (x - 1) ** 2)) < 0.07


@pytest.mark.parametrize("masked", [True, False])
def test_vcycle_riesz_is_symmetric_positive(cm, masked):
    """The fixed V-cycle that stands in for S^{-1} is a symmetric positive operator (on zero-sum
    vectors when S is singular) and spectrally close to S^{-1}: CG with it minimises the same J."""
    prob = _mixed3d(n=(16, 12, 8), seed=11, masked=masked)
    o = F2(prob)
    rng = np.random.default_rng(12)
    fr = np.concatenate([o.free.ravel()] * 2)
    x = rng.standard_normal(o.size) * fr
    y = rng.standard_normal(o.size) * fr
    u = slice(0, o.nn)
    if not masked:
        x[u] -= x[u].mean()
        y[u] -= y[u].mean()
    with cm.Solver(prob, "fp64", riesz_mode="vcycle") as s:
        Px = s.apply(cm.OP_RIESZ, x)
        Py = s.apply(cm.OP_RIESZ, y)
    assert abs(Px[u] @ y[u] - x[u] @ Py[u]) <= 1e-12 * np.linalg.norm(Px[u]) * np.linalg.norm(y[u])
    assert Px[u] @ x[u] > 0 and Py[u] @ y[u] > 0
    Ex = o.riesz(x)[u]
    assert 0.2 < (Px[u] @ x[u]) / (Ex @ x[u]) < 5.0
    # the velocity block is the exact M^{-1} in both modes
    assert _rel(Px[o.nn:], o.riesz(x)[o.nn:]) < 1e-13


@pytest.mark.parametrize("masked", [True, False])
def test_multigrid_plane_march_matches_row_kernels_bitwise(cm, masked, monkeypatch):
    """The multigrid's stencil sweeps (Jacobi, residual, S x) run as a march through chunks of
    planes; CMCG_MG_ROWS=1 runs them in the row kernels instead, and CMCG_MG_CHUNK fixes the
    chunk length.  Every form does each node's arithmetic on the same operands in the same
    order, so the V-cycle and the PCG Riesz solve give the same bits.  The grid has several
    64-wide x tiles, a ragged 4-row tail and four levels; chunks of 32 and 5 planes leave ragged
    last chunks (the automatic choice is one plane at this size)."""
    prob = _mixed3d(n=(96, 40, 72), seed=13, masked=masked)
    o = F2(prob)
    rng = np.random.default_rng(14)
    x = rng.standard_normal(o.size) * np.concatenate([o.free.ravel()] * 2)
    if not masked:
        x[: o.nn] -= x[: o.nn].mean()
    forms = [("0", None), ("0", "32"), ("0", "5"), ("1", None)]
    for mode in ("vcycle", "solve"):
        out = []
        for rows, chunk in forms:
            monkeypatch.setenv("CMCG_MG_ROWS", rows)
            if chunk is None:
                monkeypatch.delenv("CMCG_MG_CHUNK", raising=False)
            else:
                monkeypatch.setenv("CMCG_MG_CHUNK", chunk)
            with cm.Solver(prob, "fp64", riesz_mode=mode) as s:
                out.append(s.apply(cm.OP_RIESZ, x))
        monkeypatch.delenv("CMCG_MG_ROWS", raising=False)
        monkeypatch.delenv("CMCG_MG_CHUNK", raising=False)
        for f, a in zip(forms[1:], out[1:]):
            assert np.array_equal(a, out[0]), (mode, f, np.max(np.abs(a - out[0])))


@pytest.mark.parametrize("masked", [True, False])
def test_fp32_vcycle_is_the_fp64_vcycle_to_rounding(cm, masked):
    """FP32-mixed solves apply the fixed V-cycle with FP32 storage and arithmetic: it equals
    the FP64 V-cycle to FP32 rounding, and stays symmetric (to that rounding) and positive."""
    prob = _mixed3d(n=(96, 40, 72), seed=16, masked=masked)
    o = F2(prob)
    rng = np.random.default_rng(17)
    fr = np.concatenate([o.free.ravel()] * 2)
    x = rng.standard_normal(o.size) * fr
    y = rng.standard_normal(o.size) * fr
    u = slice(0, o.nn)
    if not masked:
        x[u] -= x[u].mean()
        y[u] -= y[u].mean()
    with cm.Solver(prob, "fp64", riesz_mode="vcycle") as s:
        P64x = s.apply(cm.OP_RIESZ, x)
    with cm.Solver(prob, "fp32", riesz_mode="vcycle") as s:
        Px = s.apply(cm.OP_RIESZ, x)
        Py = s.apply(cm.OP_RIESZ, y)
    assert _rel(Px[u], P64x[u]) < 1e-5
    assert abs(Px[u] @ y[u] - x[u] @ Py[u]) <= 1e-5 * np.linalg.norm(Px[u]) * np.linalg.norm(y[u])
    assert Px[u] @ x[u] > 0 and Py[u] @ y[u] > 0


@pytest.mark.parametrize("kind", ["inclusions", "sphere"])
def test_vcycle_riesz_reaches_the_same_solution(cm, kind):
    if kind == "inclusions":
        prob = ci.inclusions_3d(n=16, freq=1.5, n_incl=6, seed=9, width=0.12, r_range=(0.1, 0.25))
    else:
        prob = ci.sound_soft_sphere_3d(n=16, freq=1.2, radius=0.2)
    o = F2(prob)
    Ud, _ = o.direct()
    with cm.Solver(prob, "fp64", tol=1e-11, max_iter=4000, riesz_mode="vcycle") as s:
        U, rep = s.solve()
    assert rep["converged"]
    assert _rel(U, Ud) < 1e-8


# Full size (512^3 inclusions): the blocked launch configuration the benchmark times, checked by
# properties that hold at any size (the oracle's dependency cone of N = 123 steps spans the box)
@pytest.fixture(scope="module")
def c3():
    return ci.inclusions_3d()


def test_full_size_blocked_period_is_bitwise(cm, c3):
    """512^3, FP32: forward and backward homogeneous periods with 4 steps per launch (the
    default) and with 3 equal one step per launch bit for bit."""
    import torch
    outs = []
    for k in (1, 4, 3):
        with cm.Solver(c3, "fp32", steps_per_launch=k) as s:
            n = s.info["state_len"]
            g = torch.Generator(device="cuda").manual_seed(11)
            z = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
            outs.append((s.apply(cm.OP_FORWARD, z), s.apply(cm.OP_ADJOINT, z)))
            del z
            torch.cuda.synchronize()
    for out in outs[1:]:
        assert torch.equal(outs[0][0], out[0])
        assert torch.equal(outs[0][1], out[1])


def test_full_size_adjoint_identity_fp64(cm, c3):
    """512^3, FP64, default blocking: <E z, y> = <z, E^T y> for random device vectors z, y (the
    backward period is the literal transpose of the forward one), to rounding relative to
    |E z| |y|.  The inputs are written by torch on the caller's stream just before the calls."""
    import torch
    with cm.Solver(c3, "fp64") as s:
        n = s.info["state_len"]
        g = torch.Generator(device="cuda").manual_seed(12)
        z = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
        y = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
        Ez = s.apply(cm.OP_FORWARD, z)
        ETy = s.apply(cm.OP_ADJOINT, y)
        lhs, rhs = torch.dot(Ez, y).item(), torch.dot(z, ETy).item()
        bound = 1e-13 * (torch.linalg.vector_norm(Ez) * torch.linalg.vector_norm(y)).item()
    assert abs(lhs - rhs) <= bound, (lhs, rhs, bound)


def test_device_inputs_are_ordered_after_the_callers_stream(cm):
    """A device input that torch writes on the caller's (default) stream right before the call
    is complete when the library reads it: the binding runs each handle on its own stream and
    makes it wait for the caller's.  (Reading it early made periods differ run to run on a
    prefix of planes.)"""
    import torch
    prob = ci.inclusions_3d(n=256, freq=12.5)
    with cm.Solver(prob, "fp64") as s:
        n = s.info["state_len"]
        outs = []
        for _ in range(2):
            g = torch.Generator(device="cuda").manual_seed(13)
            z = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
            outs.append(s.apply(cm.OP_FORWARD, z))
            del z
    assert torch.equal(outs[0], outs[1])
