"""GPU parity for the first-order (F1) path: the HIP kernels behind the C ABI against the FP64
CPU oracle, element by element on the same seeded inputs."""
import math

import numpy as np
import pytest

import cmcg_inputs as ci
from cmcg_inputs import Problem
from oracle.f1 import F1, window

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    from paper_1903_12522_amd import cmcg
    return cmcg


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _mixed_problem(nx=70, ny=37, seed=3):
    """Ragged grid (several 64-wide tiles and a tail), random c, complex source, boundary data
    on two absorbing faces, one Neumann face."""
    rng = np.random.default_rng(seed)
    c = 1.0 + rng.uniform(size=(ny, nx))
    f = np.zeros((ny, nx), complex)
    f[5:9, 10:14] = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    gS = [rng.standard_normal(ny) + 1j * rng.standard_normal(ny), np.zeros(ny, complex),
          rng.standard_normal(nx) + 1j * rng.standard_normal(nx), np.zeros(nx, complex)]
    return Problem(dim=2, formulation=1, n=(nx, ny), omega=2 * math.pi * 2.5, c=c, f=f, gS=gS,
                   face_bc=(0, 0, 0, 1), courant=0.5, name="mixed")


@pytest.mark.parametrize("kblock", [1, 2, 3, 4, 6, 7, 8])
def test_periods_match_oracle_fp64(cm, kblock):
    prob = _mixed_problem()
    o = F1(prob)
    with cm.Solver(prob, "fp64", steps_per_launch=kblock) as s:
        assert s.info["steps_per_period"] == o.N
        rng = np.random.default_rng(10 + kblock)
        z = rng.standard_normal(o.size)
        assert _rel(s.apply(cm.OP_FORWARD, z), o.period(z, False)) < 1e-13
        assert _rel(s.apply(cm.OP_FORCED, z), o.period(z, True)) < 1e-13
        w = o.weights()
        ref = o.period_T(w * z) / w          # M_E^{-1} E^T M_E z
        assert _rel(s.apply(cm.OP_ADJOINT, z), ref) < 1e-13
        # partial runs (K steps) and the Riesz map M_E^{-1}
        assert _rel(s.apply(cm.OP_FORCED, z, steps=5), o.period(z, True, steps=5)) < 1e-13
        assert _rel(s.apply(cm.OP_RIESZ, z), z / w) < 1e-14


def test_periods_fp32_mixed_within_rounding(cm):
    prob = _mixed_problem(nx=130, ny=66, seed=4)
    o = F1(prob)
    with cm.Solver(prob, "fp32") as s:
        z = np.random.default_rng(1).standard_normal(o.size)
        assert _rel(s.apply(cm.OP_FORWARD, z), o.period(z, False)) < 2e-5
        w = o.weights()
        assert _rel(s.apply(cm.OP_ADJOINT, z), o.period_T(w * z) / w) < 2e-5


def test_temporal_blocking_is_bitwise_single_step(cm):
    """Every cell sees the same operands in the same order whatever the number of steps a launch
    fuses, so blocked and single-step periods agree bit for bit (a halo or LDS race would not)."""
    prob = _mixed_problem(nx=200, ny=90, seed=5)
    z = np.random.default_rng(2).standard_normal(F1(prob).size)
    outs = []
    for k in (1, 2, 3, 4, 5, 6, 7, 8):
        with cm.Solver(prob, "fp64", steps_per_launch=k) as s:
            outs.append((s.apply(cm.OP_FORCED, z), s.apply(cm.OP_ADJOINT, z)))
    for k, (a, b) in zip((2, 3, 4, 5, 6, 7, 8), outs[1:]):
        assert np.array_equal(a, outs[0][0]), (k, np.max(np.abs(a - outs[0][0])))
        assert np.array_equal(b, outs[0][1]), (k, np.max(np.abs(b - outs[0][1])))


def test_temporal_blocking_is_bitwise_fp32(cm):
    """FP32 periods: interior strips run the two-column fast variant and edge strips the
    one-column general body over sub-strips; strip and band boundaries move with the number of
    fused steps, so bitwise agreement across K checks the variants against each other."""
    prob = _mixed_problem(nx=420, ny=130, seed=6)
    z = np.random.default_rng(3).standard_normal(F1(prob).size)
    outs = []
    for k in (1, 2, 3, 4, 5, 6, 7, 8):
        with cm.Solver(prob, "fp32", steps_per_launch=k) as s:
            assert s.info["steps_per_launch"] == k
            outs.append((s.apply(cm.OP_FORWARD, z), s.apply(cm.OP_ADJOINT, z)))
    for prec in ("fp32", "fp64"):
        with cm.Solver(prob, prec) as s:
            assert s.info["steps_per_launch"] == 7   # the library default in both precisions
    for k, (a, b) in zip((2, 3, 4, 5, 6, 7, 8), outs[1:]):
        assert np.array_equal(a, outs[0][0]), (k, np.max(np.abs(a - outs[0][0])))
        assert np.array_equal(b, outs[0][1]), (k, np.max(np.abs(b - outs[0][1])))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fast_variants_match_general_body_bitwise(cm, prec, monkeypatch):
    """Interior tiles of the first launch of a period (opening half kick), of its last launch
    (output less a subtrahend, as in each CG iteration's E d - d), of the launches between, and
    of every launch of a forced period run register-streamed fast variants; CMCG_F1_GENERAL=1
    sends every tile through the general body instead.  Both must give the same bits for the
    periods and for CG iterates (whose initial gradient is a forced period less its input)."""
    prob = _mixed_problem(nx=420, ny=260, seed=8)
    z = np.random.default_rng(4).standard_normal(F1(prob).size)

    def run(k):
        with cm.Solver(prob, prec, tol=0.0, max_iter=50, steps_per_launch=k) as s:
            out = [s.apply(cm.OP_FORWARD, z), s.apply(cm.OP_ADJOINT, z),
                   s.apply(cm.OP_FORWARD, z, steps=k), s.apply(cm.OP_FORCED, z)]
            s.begin()
            s.iterate(3)
            out.append(s.state(0))
        return out

    for k in (1, 3, 7, 8):
        monkeypatch.delenv("CMCG_F1_GENERAL", raising=False)
        fast = run(k)
        monkeypatch.setenv("CMCG_F1_GENERAL", "1")
        gen = run(k)
        monkeypatch.delenv("CMCG_F1_GENERAL")
        for n, (a, b) in enumerate(zip(fast, gen)):
            assert np.array_equal(a, b), (k, n, np.max(np.abs(a - b)))


def test_adjoint_identity_on_gpu(cm):
    """<E z, y>_E = <z, E* y>_E to 1e-13 through the GPU alone."""
    prob = ci.random_medium_2d(n=96, freq=4.0, n_src=3, seed=7)
    o = F1(prob)
    w = o.weights()
    rng = np.random.default_rng(3)
    z, y = rng.standard_normal(o.size), rng.standard_normal(o.size)
    with cm.Solver(prob, "fp64") as s:
        Ez = s.apply(cm.OP_FORWARD, z)
        Esy = s.apply(cm.OP_ADJOINT, y)
    lhs, rhs = np.sum(w * Ez * y), np.sum(w * z * Esy)
    assert abs(lhs - rhs) <= 1e-13 * math.sqrt(np.sum(w * Ez ** 2) * np.sum(w * y ** 2))


def test_filter_matches_oracle(cm):
    prob = _mixed_problem(nx=66, ny=40, seed=6)
    o = F1(prob)
    z = np.random.default_rng(4).standard_normal(o.size)
    with cm.Solver(prob, "fp64") as s:
        assert _rel(s.filter(z), o.filter(z)) < 1e-13


def test_cmcg_fp64_matches_oracle_small(cm):
    prob = ci.random_medium_2d(n=32, freq=2.0, n_src=2, seed=11, width=0.06)
    o = F1(prob)
    zo, hist, it = o.solve(tol=1e-12, max_iter=3000)
    Uo = o.filter(zo)
    with cm.Solver(prob, "fp64", tol=1e-12, max_iter=3000) as s:
        U, rep = s.solve()
    assert rep["converged"]
    assert abs(rep["iterations"] - it) <= 2
    assert _rel(U, Uo) < 1e-9
    Ud, _ = o.direct()
    assert _rel(U, Ud) < 1e-9


@pytest.fixture(scope="module")
def c1_oracle():
    prob = ci.single_source_2d()
    o = F1(prob)
    z, hist, it = o.solve(tol=1e-8, max_iter=2000)
    return prob, o, o.filter(z), hist, it


def test_single_source_128_fp64(cm, c1_oracle):
    """128^2, omega = 8 pi, tol 1e-8, FP64.  Parity: after the oracle's own number of CG
    iterations the GPU result equals the oracle's to 1e-9.  Stopping at tol, the GPU needs the
    same number of iterations (+-1) and lands as close to the direct solve as the oracle does."""
    prob, o, Uo, hist, it = c1_oracle
    with cm.Solver(prob, "fp64", tol=0.0, max_iter=it) as s:
        U, rep = s.solve()
    assert rep["iterations"] == it and rep["steps_per_period"] == 64
    assert _rel(U, Uo) < 1e-9
    with cm.Solver(prob, "fp64", tol=1e-8, max_iter=2000) as s:
        U, rep = s.solve()
    assert rep["converged"] and abs(rep["iterations"] - it) <= 1
    Ud, _ = o.direct()
    assert _rel(U, Ud) < 2 * _rel(Uo, Ud) + 1e-9


def test_single_source_128_fp32_mixed(cm, c1_oracle):
    prob, o, Uo, hist, it = c1_oracle
    with cm.Solver(prob, "fp32", tol=1e-6, max_iter=2000) as s:
        U, rep = s.solve()
    assert rep["converged"]
    assert _rel(U, Uo) < 1e-4


def test_cg_iterates_track_oracle(cm):
    """After each of the first iterations the GPU iterate z_l equals the oracle's."""
    prob = ci.random_medium_2d(n=40, freq=2.5, n_src=2, seed=13, width=0.05)
    o = F1(prob)
    rec = []
    o.solve(tol=0.0, max_iter=6, record=rec)
    with cm.Solver(prob, "fp64", tol=0.0, max_iter=6) as s:
        s.begin()
        for l in range(1, 7):
            s.iterate(1)
            assert _rel(s.state(0), rec[l]) < 1e-11


def test_solve_is_deterministic(cm):
    prob = ci.random_medium_2d(n=64, freq=3.0, n_src=2, seed=17)
    with cm.Solver(prob, "fp32", tol=1e-5, max_iter=300) as s:
        U1, r1 = s.solve()
        U2, r2 = s.solve()
    assert np.array_equal(U1, U2) and r1["iterations"] == r2["iterations"]


def test_report_counts_compulsory_traffic(cm):
    """cmcg_report.dram_bytes: each blocked launch moves its 7 FP64 words per cell once for
    K = 7 steps (56 / 7 B per grid update), plus the subtrahend, the sources and the filter's
    accumulators on the few launches that read them, so the total stays well under one pass per
    step."""
    prob = ci.random_medium_2d(n=256, freq=8.0, n_src=2, seed=19)
    with cm.Solver(prob, "fp64", tol=1e-6, max_iter=500) as s:
        _, rep = s.solve()
    per = rep["dram_bytes"] / rep["grid_updates"]
    assert 56 / 7 <= per < 56 / 3, per


def test_notconv_returns_last_iterate(cm):
    prob = ci.single_source_2d(n=32, omega=2 * math.pi * 2)
    with cm.Solver(prob, "fp64", tol=1e-12, max_iter=1) as s:
        U, rep = s.solve()
    assert not rep["converged"] and rep["iterations"] == 1 and np.all(np.isfinite(U))


# ------------------------------------------------------------------------------------------
# Full size (4096^2, random medium, 8 sources): sampled parity of one period
# ------------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c2():
    return ci.random_medium_2d()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_full_size_period_sampled(cm, c2, prec, tol):
    """One forced period on the full 4096^2 grid, in the launch configuration the benchmark
    uses, checked at sampled cells (corners, edges, sources, interior) against the oracle run on
    windows of radius N + 2 around each sample (exact: the dependency cone of N steps)."""
    prob = c2
    n = prob.n[0]
    o_full_N = int(math.ceil((2 * math.pi / prob.omega) * prob.c_max() / (0.5 / n)))
    with cm.Solver(prob, prec) as s:
        N = s.info["steps_per_period"]
        assert N == o_full_N == 164
        rng = np.random.default_rng(21)
        ny = nx = n
        sizes = [ny * (nx - 1), (ny - 1) * nx, ny * nx]
        z = rng.standard_normal(sum(sizes)) * 1e-2
        out = s.apply(cm.OP_FORCED, z)
    Px = z[: sizes[0]].reshape(ny, nx - 1)
    Py = z[sizes[0]: sizes[0] + sizes[1]].reshape(ny - 1, nx)
    v = z[sizes[0] + sizes[1]:].reshape(ny, nx)
    vo = out[sizes[0] + sizes[1]:].reshape(ny, nx)
    Pxo = out[: sizes[0]].reshape(ny, nx - 1)
    samples = [(0, 0), (nx - 1, ny - 1), (0, ny // 2), (nx // 2, 0), (2047, 2048), (1000, 3100)]
    m = N + 2
    for (ci0, cj0) in samples:
        i0, i1 = max(0, ci0 - m), min(nx, ci0 + m + 1)
        j0, j1 = max(0, cj0 - m), min(ny, cj0 + m + 1)
        sub = F1(window(prob, i0, i1, j0, j1), N=N)
        zs = sub.pack(Px[j0:j1, i0:i1 - 1], Py[j0:j1 - 1, i0:i1], v[j0:j1, i0:i1])
        Pxs, Pys, vs = sub.unpack(sub.period(zs, True))
        scale = np.max(np.abs(vs)) + 1e-300
        assert abs(vo[cj0, ci0] - vs[cj0 - j0, ci0 - i0]) <= tol * scale
        if ci0 < nx - 1:
            sp = np.max(np.abs(Pxs)) + 1e-300
            assert abs(Pxo[cj0, ci0] - Pxs[cj0 - j0, ci0 - i0]) <= tol * sp


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_full_size_homogeneous_periods_sampled(cm, c2, prec, tol):
    """The homogeneous forward period E z and the backward period E* z = M_E^{-1} E^T M_E z on the
    full 4096^2 grid, in the default launch configuration (K = 7, 32-row bands: every launch
    between a period's first and last, forward or backward, runs the forward middle instance),
    checked at sampled cells against the oracle on windows of radius N + 2 around each sample.
    The samples include corners, edges, band and strip boundaries and the interior."""
    prob = c2
    n = prob.n[0]
    ny = nx = n
    sizes = [ny * (nx - 1), (ny - 1) * nx, ny * nx]
    with cm.Solver(prob, prec) as s:
        N = s.info["steps_per_period"]
        assert N == 164 and s.info["steps_per_launch"] == 7
        z = np.random.default_rng(23).standard_normal(sum(sizes))
        outf = s.apply(cm.OP_FORWARD, z)
        outa = s.apply(cm.OP_ADJOINT, z)

    def fields(x):
        return (x[: sizes[0]].reshape(ny, nx - 1),
                x[sizes[0]: sizes[0] + sizes[1]].reshape(ny - 1, nx),
                x[sizes[0] + sizes[1]:].reshape(ny, nx))

    Px, Py, v = fields(z)
    samples = [(0, 0), (nx - 1, ny - 1), (nx - 1, 0), (0, ny // 2 + 13), (nx // 2, 0),
               (2047, 2048), (48 * 40, 32 * 50 + 31), (48 * 61 - 1, 32 * 77), (1000, 3100)]
    m = N + 2
    for (ci0, cj0) in samples:
        i0, i1 = max(0, ci0 - m), min(nx, ci0 + m + 1)
        j0, j1 = max(0, cj0 - m), min(ny, cj0 + m + 1)
        sub = F1(window(prob, i0, i1, j0, j1), N=N)
        zs = sub.pack(Px[j0:j1, i0:i1 - 1], Py[j0:j1 - 1, i0:i1], v[j0:j1, i0:i1])
        w = sub.weights()
        refs = {"forward": (outf, sub.period(zs, False)),
                "backward": (outa, sub.period_T(w * zs) / w)}
        for name, (full, ref) in refs.items():
            Pxo, Pyo, vo = fields(full)
            Pxs, Pys, vs = sub.unpack(ref)
            li, lj = ci0 - i0, cj0 - j0
            sv = np.max(np.abs(vs)) + 1e-300
            assert abs(vo[cj0, ci0] - vs[lj, li]) <= tol * sv, (name, ci0, cj0)
            if ci0 < nx - 1:
                sp = np.max(np.abs(Pxs)) + 1e-300
                assert abs(Pxo[cj0, ci0] - Pxs[lj, li]) <= tol * sp, (name, ci0, cj0)
            if cj0 < ny - 1:
                sp = np.max(np.abs(Pys)) + 1e-300
                assert abs(Pyo[cj0, ci0] - Pys[lj, li]) <= tol * sp, (name, ci0, cj0)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2 * 164 * 6e-8)])
def test_full_size_adjoint_identity(cm, c2, prec, tol):
    """4096^2 in the default launch configuration (K = 7, the benchmark's): <E z, y>_E =
    <z, E* y>_E for random device vectors, relative to
    |E z|_E |y|_E.  The energy weights are read back from the library's own Riesz map
    (M_E^{-1} applied to ones).  FP64 holds to rounding; FP32 periods round each of N = 164 steps
    at eps_32, hence the bound 2 N eps_32 there."""
    import torch
    with cm.Solver(c2, prec) as s:
        n = s.info["state_len"]
        g = torch.Generator(device="cuda").manual_seed(22)
        z = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
        y = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
        w = 1.0 / s.apply(cm.OP_RIESZ, torch.ones(n, dtype=torch.float64, device="cuda"))
        Ez = s.apply(cm.OP_FORWARD, z)
        Esy = s.apply(cm.OP_ADJOINT, y)
        lhs, rhs = torch.dot(w * Ez, y).item(), torch.dot(w * z, Esy).item()
        scale = math.sqrt(torch.dot(w * Ez, Ez).item() * torch.dot(w * y, y).item())
    assert abs(lhs - rhs) <= tol * scale, (lhs, rhs, scale)


def test_fp32_mixed_reliable_updates_match_fp64(cm):
    """FP32 periods alone stall above 1e-6 on a heterogeneous medium; with FP64 residual
    refreshes the FP32-mixed solve converges in about the FP64 iteration count and lands within
    1e-4 (relative L2) of the FP64 solution."""
    prob = ci.random_medium_2d(n=512, freq=12.5, n_src=4, seed=99)
    with cm.Solver(prob, "fp64", tol=1e-6, max_iter=3000) as s:
        U64, r64 = s.solve()
    with cm.Solver(prob, "fp32", tol=1e-6, max_iter=3000) as s:
        U32, r32 = s.solve()
    assert r64["converged"] and r32["converged"]
    assert r32["fp64_refreshes"] >= 1
    assert r32["iterations"] <= 1.15 * r64["iterations"] + 5
    assert _rel(U32, U64) < 1e-4
