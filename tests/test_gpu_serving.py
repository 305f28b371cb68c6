"""GPU tests of the continuous-batching server: each result is the same alone and in a mix of
concurrently resident solves (bit for bit: a solve's arithmetic does not depend on its batch),
served results equal the single-solve path, admission respects the HBM budget, and a served
FP64 solve matches the CPU oracle."""
import math

import numpy as np
import pytest

import cmcg_inputs as ci
from oracle.f1 import F1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    from paper_1903_12522_amd import cmcg
    return cmcg


def _req(n, W, seed, pos=(0.45, 0.55)):
    return ci.request_problem(n, W, pos, seed)


def _serve(cm, probs, precision="fp32", tol=1e-5, stagger=0, budget=8 << 30, slots=16):
    """Submit `probs` (one every `stagger` steps) and step until all are done."""
    out = {}
    with cm.Server(budget, max_slots=slots) as srv:
        ids = []
        k = 0
        steps = 0
        while len(out) < len(probs):
            if k < len(probs) and steps % max(1, stagger) == 0:
                ids.append(srv.submit(probs[k], precision=precision, tol=tol, max_iter=2000))
                k += 1
            srv.step()
            used, act, q = srv.stats()
            assert used <= budget
            steps += 1
            for j, rid in enumerate(ids):
                if j in out:
                    continue
                state, U, rep, st = srv.poll(rid)
                assert state != cm.REQ_FAILED
                if state == cm.REQ_DONE:
                    out[j] = (U, rep, st)
            assert steps < 200000
    return [out[j] for j in range(len(probs))]


def test_served_equals_single_solve(cm):
    prob = _req(96, 5.0, 7)
    (U, rep, st), = _serve(cm, [prob], precision="fp32", tol=1e-5)
    with cm.Solver(prob, "fp32", tol=1e-5, max_iter=2000) as s:
        Us, reps = s.solve()
    assert st == 0 and rep["iterations"] == reps["iterations"]
    assert np.array_equal(U, Us)


def test_alone_and_in_mix_identical(cm):
    probs = [_req(64, 4.0, 1), _req(128, 7.5, 2, pos=(0.4, 0.6)), _req(96, 12.0, 3),
             _req(80, 6.0, 4, pos=(0.55, 0.35))]
    alone = [_serve(cm, [p])[0] for p in probs]
    mixed = _serve(cm, probs, stagger=3)
    for (Ua, ra, sa), (Um, rm, sm) in zip(alone, mixed):
        assert sa == 0 and sm == 0
        assert ra["iterations"] == rm["iterations"]
        assert np.array_equal(Ua, Um)


def test_admission_respects_budget(cm):
    """Budget for one of the two solves at a time: the second waits in the queue until the first
    has finished and released its memory."""
    big, small = _req(256, 6.0, 5), _req(128, 6.0, 6)
    sizes = []
    for p in (big, small):
        with cm.Solver(p, "fp32") as s:
            sizes.append(s.info["device_bytes"])
    budget = max(sizes) + min(sizes) // 2
    with cm.Server(budget, max_slots=8) as srv:
        ids = [srv.submit(big, "fp32", 1e-5, 2000), srv.submit(small, "fp32", 1e-5, 2000)]
        seen_queue = False
        done = set()
        for _ in range(200000):
            act, q = srv.step()
            used, act2, q2 = srv.stats()
            assert used <= budget and act <= 1
            seen_queue |= q > 0
            for rid in ids:
                if rid not in done and srv.poll(rid)[0] == cm.REQ_DONE:
                    done.add(rid)
            if len(done) == 2:
                break
        assert seen_queue and len(done) == 2
        assert srv.stats()[0] == 0


def test_request_too_large_is_rejected(cm):
    with cm.Server(1 << 20) as srv:
        with pytest.raises(cm.CMCGError):
            srv.submit(_req(256, 6.0, 5), "fp32", 1e-5, 100)


def test_served_fp64_matches_oracle(cm):
    prob = _req(48, 3.0, 9)
    o = F1(prob)
    z, hist, it = o.solve(tol=1e-10, max_iter=3000)
    Uo = o.filter(z)
    (U, rep, st), = _serve(cm, [prob], precision="fp64", tol=1e-10)
    assert st == 0 and abs(rep["iterations"] - it) <= 1
    assert np.linalg.norm(U - Uo) / np.linalg.norm(Uo) < 1e-8


def test_mini_workload_real_time(cm):
    """A scaled-down arrival replay: 12 seeded requests on small grids at 40/s, all served."""
    from paper_1903_12522_amd import serving
    reqs = ci.serving_requests(count=12, rate_hz=40.0, seed=5, sides=(64, 96, 128),
                               wavelengths=(4.0, 12.0))
    with cm.Server(8 << 30, max_slots=6) as srv:
        recs, summ = serving.run(srv, reqs, precision="fp32", tol=1e-5, max_iter=2000)
    assert summ["completed"] == 12 and summ["converged"] == 12
    assert summ["p99_latency_s"] >= summ["p50_latency_s"] > 0
    assert summ["peak_active"] >= 2


def test_served_solve_stops_at_max_iter_after_refresh(cm):
    """A refresh on the last allowed iteration ends the served solve there (not converged), as it
    ends the single solve: same iteration count, status and result bits."""
    prob = _req(64, 4.0, 11)
    max_iter = 6
    with cm.Solver(prob, "fp32", tol=1e-12, max_iter=max_iter, fp64_refresh=0.999) as s:
        Us, reps = s.solve()
    assert not reps["converged"] and reps["iterations"] == max_iter
    assert reps["fp64_refreshes"] >= max_iter - 1
    with cm.Server(8 << 30, max_slots=4) as srv:
        rid = srv.submit(prob, precision="fp32", tol=1e-12, max_iter=max_iter,
                         fp64_refresh=0.999)
        for _ in range(100000):
            srv.step()
            state, U, rep, st = srv.poll(rid)
            if state in (cm.REQ_DONE, cm.REQ_FAILED):
                break
        assert state == cm.REQ_DONE and st == cm.ENOTCONV
        assert rep["iterations"] == max_iter and rep["fp64_refreshes"] == reps["fp64_refreshes"]
        assert np.array_equal(U, Us)
        # the poll that reported DONE released the request
        assert srv.stats() == (0, 0, 0)


def test_one_tick_is_one_kernel_launch(cm):
    """Each server tick advances every resident solve through many rounds (period launches,
    reductions and CG decisions) inside one launch of the persistent serving kernel."""
    probs = [_req(64, 4.0, 21), _req(96, 6.0, 22, pos=(0.4, 0.6)), _req(80, 5.0, 23)]
    with cm.Server(8 << 30, max_slots=8) as srv:
        ids = [srv.submit(p, precision="fp32", tol=1e-5, max_iter=2000) for p in probs]
        done = {}
        for _ in range(10000):
            srv.step()
            for rid in ids:
                if rid in done:
                    continue
                state, U, rep, st = srv.poll(rid)
                if state == cm.REQ_DONE:
                    done[rid] = rep
            if len(done) == len(ids):
                break
        ticks, launches, rounds = srv.launches()
    assert len(done) == len(ids)
    assert ticks >= 1 and launches == ticks and rounds > ticks
    # a solve takes thousands of period launches; the ticks are far fewer
    iters = sum(r["iterations"] for r in done.values())
    assert ticks < iters


def test_barrier_that_gives_up_fails_the_tick(cm):
    """A grid barrier whose wait runs out (a spin limit of one poll, forced from the host)
    ends the serving kernel: the tick reports CMCG_EDEVICE and fails the resident solves;
    a server with the default limit then serves the same request normally."""
    prob = _req(64, 4.0, 31)
    with cm.Server(8 << 30, max_slots=4, barrier_spin_limit=1) as srv:
        rid = srv.submit(prob, precision="fp32", tol=1e-5, max_iter=2000)
        with pytest.raises(cm.CMCGError) as e:
            srv.step()
        assert e.value.status == cm.EDEVICE
        state, U, rep, st = srv.poll(rid)
        assert state == cm.REQ_FAILED and st == cm.EDEVICE
        assert srv.stats() == (0, 0, 0)
    (U, rep, st), = _serve(cm, [prob], precision="fp32", tol=1e-5)
    assert st == 0 and rep["iterations"] > 0
