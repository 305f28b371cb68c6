"""Benchmark of the CMCG hot path on one MI355X.

Workload: the 4096^2 first-order random-medium problem (c a seeded Gaussian random field in
[1, 2], omega = 2 pi 100, 8 seeded Gaussian sources, absorbing sides; N = 164 leapfrog steps per
period).  A timed *step* is one CMCG iteration in FP32-mixed precision: a homogeneous forward
period, the adjoint (backward) period, the energy inner products and the CG update, i.e.
2 N x 4096^2 grid-point updates.  `value` is grid-point updates per second (GLUP/s) over the
timed steps, inputs resident in HBM.

Also reported: time-to-solution at relative residual 1e-6 in FP32-mixed and FP64 (full solves
from z = 0 including the filter) on the 4096^2 problem and on the 512^3 second-order inclusions
problem (both precisions with the same Riesz map, one fixed V-cycle, so that their ratio is the
precision's alone), their ratios and the FP32-mixed errors against FP64; the roofline of each
workload's dominant kernel from the library's HIP events around that kernel's own launches;
and the CPU oracle timed on a bounded sample of the 4096^2 workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-tts] [--no-cpu] [--no-c3]
       python bench.py --c3-iters K   (K FP32-mixed CG iterations of the 512^3 problem only)
       python bench.py --calibrate-copy   (one 1 GiB device copy, for counter calibration)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "leapfrog GLUP/s + CMCG time-to-solution at rel. residual 1e-6, FP32-mixed vs FP64"


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def calibrate_copy():
    import torch
    n = 1 << 27                      # 2^27 doubles = 1 GiB
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": n * 8}))


def measured_traffic(kernel: str, workload: str = ""):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter record
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain-copy calibration; records are keyed
    "kernel @ workload", since one kernel instance serves several workloads), or None when the
    record was taken on another version of the kernel's source files."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        rec = json.load(open(rec_path))
    except (OSError, ValueError):
        return None
    e = rec.get("kernels", {}).get(f"{kernel} @ {workload}" if workload else kernel)
    if not e or "source" not in e:
        return None
    names = [e["source"]] if isinstance(e["source"], str) else list(e["source"])
    for name in names:
        src = os.path.join(ROOT, "paper_1903_12522_amd", "csrc", name)
        try:
            sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        except OSError:
            return None
        if rec.get("sources", {}).get(name) != sha:
            return None
    return int(e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"])


def roofline_entry(kernel: str, launch_s: float, alg_bytes: float, one_pass_bytes: float,
                   launches: int, workload: str = "", **extra):
    """The roofline of one kernel instance from its own average launch time.

    * achieved / frac: the scope's convention for the leapfrog sweep, single-step compulsory
      bytes per grid-point update times the updates of one launch (K steps of every point),
      divided by the launch time.  With temporal blocking one HBM pass serves K steps, so frac
      can exceed 1: it measures the sweep's rate, not the position under the HBM roof.
    * one_pass_bytes / frac_one_pass: the launch's own compulsory traffic (its inputs read once,
      its outputs written once) at the 8 TB/s peak, against its launch time: where the kernel
      sits under the roof.
    * traffic / measured_GBps / frac_measured: the HBM bytes the counters saw per launch
      (null once the kernel's source has changed since they were taken)."""
    traffic = measured_traffic(kernel, workload)
    achieved = alg_bytes / launch_s / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 3),
           "frac_convention": "single-step compulsory bytes x K steps per launch / launch time "
                              "(temporally blocked: can exceed 1)",
           "traffic": traffic,
           "kernel": kernel, "avg_launch_us": round(launch_s * 1e6, 2), "launches": launches,
           "algorithmic_bytes_per_launch": int(alg_bytes),
           "one_pass_bytes": int(one_pass_bytes),
           "one_pass_time_us": round(one_pass_bytes / (HBM_PEAK_GBS * 1e9) * 1e6, 2),
           "frac_one_pass": round(one_pass_bytes / launch_s / 1e9 / HBM_PEAK_GBS, 3)}
    if traffic is not None:
        out["measured_GBps"] = round(traffic / launch_s / 1e9, 1)
        out["frac_measured"] = round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 3)
    out.update(extra)
    return out


def single_source_tts():
    """Time to solution of the 128^2 single-source first-order problem (FP64, tol 1e-8)."""
    import torch
    import cmcg_inputs as ci
    from paper_1903_12522_amd import cmcg
    prob = ci.single_source_2d()
    with cmcg.Solver(prob, "fp64", tol=1e-8, max_iter=5000) as s:
        s.solve()                                   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rep = s.solve(device_output=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    return {"workload": "first-order 128x128, c=1, omega=8pi, tol 1e-8, FP64",
            "seconds": round(rep["seconds"], 4), "wall_seconds": round(wall, 4),
            "iterations": rep["iterations"], "steps_per_period": rep["steps_per_period"],
            "converged": rep["converged"]}


def nodal_3d(which: str, precision: str, max_iter: int, chunk: int = 10, keep=None,
             riesz_mode: str = "default", tol: float = 1e-6):
    """Time to solution of a 3D second-order workload: begin, iterations in chunks of `chunk`
    (a progress line per chunk), finish, timed on the host around device-synchronised calls;
    with the roofline of the blocked kernel from the library's events around its launches."""
    import torch
    import cmcg_inputs as ci
    from paper_1903_12522_amd import cmcg
    prob = ci.inclusions_3d() if which == "inclusions" else ci.sound_soft_sphere_3d()
    torch.cuda.empty_cache()
    with cmcg.Solver(prob, precision, tol=tol, max_iter=max_iter, riesz_mode=riesz_mode) as s:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.begin()
        conv, rep = False, None
        done = 0
        while not conv and done < max_iter:
            conv, rep = s.iterate(min(chunk, max_iter - done))
            done = rep["iterations"]
            log(f"{which} {precision}: iteration {done} rel {rep['rel_residual']:.3e} "
                f"({time.perf_counter() - t0:.1f} s)")
        u, rep = s.finish(device_output=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gb = s.info["device_bytes"] / 1e9
        kb = s.info["steps_per_launch"]
        rpw, wv = s.info["block_rows"], s.info["block_waves"]
        if keep is not None:
            keep[precision] = torch.complex(u[0], u[1]).clone()
        del u
    nodes = (prob.n[0] + 1) * (prob.n[1] + 1) * (prob.n[2] + 1)
    out = {"workload": f"second-order {which} {prob.n[0]}^3, {precision}", "nodes": nodes,
           "riesz_mode": riesz_mode,
           "seconds": round(wall, 3), "iterations": rep["iterations"], "converged": bool(conv),
           "rel_residual": rep["rel_residual"], "steps_per_period": rep["steps_per_period"],
           "seconds_fwd": round(rep["seconds_fwd"], 3), "seconds_adj": round(rep["seconds_adj"], 3),
           "seconds_riesz": round(rep["seconds_riesz"], 3),
           "seconds_other": round(rep["seconds_other"], 3),
           "riesz_iterations": rep["riesz_iterations"], "fp64_refreshes": rep["fp64_refreshes"],
           "glups_periods": round(rep["grid_updates"] / max(rep["seconds_fwd"] + rep["seconds_adj"], 1e-9) / 1e9, 1),
           "stencil_dram_GB": round(rep["dram_bytes"] / 1e9, 1),
           "device_GB": round(gb, 1)}
    nl = rep["bulk_launches_fwd"] + rep["bulk_launches_adj"]
    if nl > 0:
        t = (rep["seconds_bulk_fwd"] + rep["seconds_bulk_adj"]) / nl
        esz = 4 if precision == "fp32" else 8
        lam = prob.c is not None           # the per-node coefficient is read when c varies
        step_words = 4 if lam else 3       # one step: read u^n, u^(n-1) (, lambda), write u^(n+1)
        launch_words = 5 if lam else 4     # a blocked launch also writes u^(n+K-1)
        tname = "float" if precision == "fp32" else "double"
        # (the tile shape, rows per wavefront and wavefronts per workgroup, as the library reports)
        out["roofline"] = roofline_entry(
            f"f2_block_kernel<{tname}, {kb}, {rpw}, {wv}>", t, step_words * esz * nodes * kb,
            launch_words * esz * nodes, nl,
            workload="inclusions 512^3" if which == "inclusions" else "sphere 1024^3",
            fwd_avg_launch_us=round(rep["seconds_bulk_fwd"] / max(1, rep["bulk_launches_fwd"]) * 1e6, 2),
            adj_avg_launch_us=round(rep["seconds_bulk_adj"] / max(1, rep["bulk_launches_adj"]) * 1e6, 2))
    return out


def nodal_cpu_baseline(which: str, steps: int = 2):
    """The nodal oracle as it stands, on the full grid of a 3D workload: a forward and a
    transposed run of `steps` leapfrog steps (the oracle built with N = steps: the same step,
    start and end maps, a shorter period), timed on one host core and scaled to GLUP/s."""
    import numpy as np
    import cmcg_inputs as ci
    from oracle.f2 import F2
    # the sphere's 1024^3 grid would need about 200 GB of host memory in the oracle: its rate
    # per node-step is sampled on the same problem at 512^3
    prob = ci.inclusions_3d() if which == "inclusions" else ci.sound_soft_sphere_3d(n=512)
    log(f"timing the nodal oracle on {which} {prob.n[0]}^3 ({steps} + {steps} steps)")
    o = F2(prob, N=steps)
    z = np.random.default_rng(0).standard_normal(o.size)
    t0 = time.perf_counter()
    o.period(z, False)
    o.period_T(z)
    dt = time.perf_counter() - t0
    return {"value": round(2 * steps * o.nn / dt / 1e9, 4), "unit": "GLUP/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} forward + {steps} transposed leapfrog steps of the NumPy FP64 "
                      f"nodal oracle on a {prob.n[0]}^3 grid of this workload ({dt:.1f} s; "
                      f"NumPy element-wise kernels run on one thread)",
            "seconds": round(dt, 2)}


def serving_run(count: int):
    import cmcg_inputs as ci
    from paper_1903_12522_amd import cmcg, serving
    reqs = ci.serving_requests(count=count)
    with cmcg.Server(64 << 30, max_slots=32) as srv:
        recs, summ = serving.run(srv, reqs, precision="fp32", tol=1e-6, max_iter=2000,
                                 on_event=lambda m: log("serving: " + m))
    summ["workload"] = (f"{count} requests, Poisson 20/s, sides 256-2048, 4-64 wavelengths, "
                        "FP32-mixed, tol 1e-6, HBM budget 64 GiB, 32 slots")
    return summ


def runup_study(prob, runups=(0, 4, 16, 32), longtime=(16, 64, 256)):
    """Initial run-up and do-nothing long-time solve on a first-order workload.
    * FP32-mixed CMCG to 1e-6 after a ramped run-up of L periods: time, CG iterations and the
      total number of periods integrated (2 per CG iteration, 2 per FP64 refresh, L, and the
      reference gradient at rest when L > 0).
    * The do-nothing solve (source switched on at once) after L periods: relative periodicity
      misfit sqrt(J(z_L) / J(0)) and the error of its filtered output against the CMCG solution."""
    import numpy as np
    import torch
    from paper_1903_12522_amd import cmcg
    out = {"cmcg": [], "do_nothing": []}
    U_ref = None
    for L in runups:
        with cmcg.Solver(prob, "fp32", tol=1e-6, max_iter=20000, runup_periods=L) as s:
            s.solve(device_output=True)                 # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            U, rep = s.solve(device_output=True)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        periods = 2 * rep["iterations"] + 2 * rep["fp64_refreshes"] + L + (2 if L > 0 else 0) + 2
        out["cmcg"].append({"runup_periods": L, "seconds": round(wall, 3),
                            "iterations": rep["iterations"], "converged": rep["converged"],
                            "seconds_runup": round(rep["seconds_runup"], 3),
                            "total_periods": periods})
        log(f"run-up {L}: {wall:.2f} s, {rep['iterations']} iterations, {periods} periods")
        if U_ref is None:
            U_ref = torch.complex(U[0], U[1])
    with cmcg.Solver(prob, "fp64") as s:
        J0 = s.misfit(np.zeros(s.info["state_len"]))
        for L in longtime:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            z = s.runup(L, ramp=False)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            J = s.misfit(z)
            Uz = s.filter(z)
            err = float(np.linalg.norm(Uz - U_ref.cpu().numpy()) / torch.linalg.vector_norm(U_ref).item())
            out["do_nothing"].append({"periods": L, "seconds": round(wall, 3),
                                      "relative_misfit": float(np.sqrt(J / J0)),
                                      "filtered_rel_error_vs_cmcg": err})
            log(f"do-nothing {L} periods: misfit {np.sqrt(J / J0):.3e}, error {err:.3e}")
    return out


def obstacle_study(n: int = 128, freq: float = 6.0, longtime=(16, 64, 256, 1024)):
    """CMCG against the do-nothing long-time solve for a convex (ball) and a nonconvex (open
    box-shaped cavity) sound-soft obstacle under the same plane-wave data, second-order n^3.
    CMCG: FP32-mixed to 1e-6.  Do-nothing: FP64, relative misfit sqrt(J(z_L) / J(0)) and the
    filtered output's error against the CMCG solution after L periods."""
    import numpy as np
    import torch
    import cmcg_inputs as ci
    from paper_1903_12522_amd import cmcg
    out = {}
    for name, prob in (("ball", ci.sound_soft_sphere_3d(n=n, freq=freq, radius=0.2)),
                       ("cavity", ci.sound_soft_cavity_3d(n=n, freq=freq))):
        torch.cuda.empty_cache()
        with cmcg.Solver(prob, "fp32", tol=1e-6, max_iter=20000) as s:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            U, rep = s.solve(device_output=True)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            Uref = torch.complex(U[0], U[1]).cpu().numpy()
        res = {"workload": f"second-order {n}^3, sound-soft {name}, {freq} wavelengths",
               "cmcg": {"seconds": round(wall, 3), "iterations": rep["iterations"],
                        "converged": rep["converged"],
                        "periods": 2 * rep["iterations"] + 2 * rep["fp64_refreshes"] + 3},
               "do_nothing": []}
        log(f"{name}: CMCG {wall:.2f} s, {rep['iterations']} iterations")
        with cmcg.Solver(prob, "fp64") as s:
            J0 = s.misfit(np.zeros(s.info["state_len"]))
            for L in longtime:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                z = s.runup(L, ramp=False)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                J = s.misfit(z)
                err = float(np.linalg.norm(s.filter(z) - Uref) / np.linalg.norm(Uref))
                res["do_nothing"].append({"periods": L, "seconds": round(wall, 3),
                                          "relative_misfit": float(np.sqrt(J / J0)),
                                          "filtered_rel_error_vs_cmcg": err})
                log(f"{name}: do-nothing {L} periods: misfit {np.sqrt(J / J0):.3e}, error {err:.3e}")
        out[name] = res
    return out


def supershot_study(n: int = 2048, base_freq: float = 25.0, harmonics=(1, 2, 4)):
    """One CMCG solve of a multi-frequency source against separate single-frequency solves of
    its components (Concluding remarks), on the first-order n^2 random medium, FP32-mixed to
    1e-6.  The harmonics divide the base period's step count, so every separate problem has the
    super-shot's time step and both compute the same discrete solutions: their relative
    difference is the solvers' tolerance."""
    import copy
    import numpy as np
    import torch
    import cmcg_inputs as ci
    from paper_1903_12522_amd import cmcg

    def timed(prob):
        with cmcg.Solver(prob, "fp32", tol=1e-6, max_iter=20000) as s:
            N = s.info["steps_per_period"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            U, rep = s.solve()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        periods = 2 * rep["iterations"] + 2 * rep["fp64_refreshes"] + 3
        return U, {"seconds": round(wall, 3), "iterations": rep["iterations"],
                   "converged": rep["converged"], "steps_per_period": N,
                   "leapfrog_steps": periods * N}

    prob = ci.supershot_2d(n=n, base_freq=base_freq, harmonics=harmonics, seed=99)
    log(f"super-shot {n}^2, base {base_freq}, harmonics {harmonics}")
    U, sup = timed(prob)
    log(f"super-shot: {sup['seconds']} s, {sup['iterations']} iterations")
    separate = []
    for k, sh in enumerate(prob.shots):
        q = copy.copy(prob)
        q.shots = None
        q.omega = sh.harmonic * prob.omega
        q.f, q.gS = sh.f, sh.gS
        Uk, r = timed(q)
        r["harmonic"] = sh.harmonic
        r["rel_diff_vs_supershot"] = float(np.linalg.norm(U[k] - Uk) / np.linalg.norm(Uk))
        separate.append(r)
        log(f"harmonic {sh.harmonic}: {r['seconds']} s, {r['iterations']} iterations, "
            f"difference {r['rel_diff_vs_supershot']:.2e}")
    total = sum(r["seconds"] for r in separate)
    return {"workload": f"first-order random medium {n}x{n}, {len(harmonics)} Gaussian sources at "
                        f"harmonics {list(harmonics)} of {base_freq} (frequencies "
                        f"{[m * base_freq for m in harmonics]}), FP32-mixed, tol 1e-6",
            "supershot": sup, "separate": separate,
            "separate_total_seconds": round(total, 3),
            "separate_over_supershot": round(total / sup["seconds"], 3)}


def obstacle_study_2d(n: int = 400, freq: float = 10.0, side: float = 0.3,
                      longtime=(16, 64, 256, 1024)):
    """The same comparison in 2D on the first-order scheme with Dirichlet cells: a box ten
    wavelengths wide (c = 1, k = 2 pi freq, h = 1/n), plane wave at 135 degrees, a sound-soft
    square of the given side or a square cavity of that size open on its -x wall."""
    import numpy as np
    import torch
    import cmcg_inputs as ci
    from paper_1903_12522_amd import cmcg
    out = {}
    for name, cav in (("square", False), ("cavity", True)):
        prob = ci.sound_soft_square_2d(n=n, freq=freq, side=side, cavity=cav)
        with cmcg.Solver(prob, "fp32", tol=1e-6, max_iter=20000) as s:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            U, rep = s.solve()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        res = {"workload": f"first-order {n}^2, {freq:g} wavelengths across, sound-soft {name} "
                           f"of side {side}, plane wave at 135 degrees",
               "cmcg": {"seconds": round(wall, 3), "iterations": rep["iterations"],
                        "converged": rep["converged"],
                        "periods": 2 * rep["iterations"] + 2 * rep["fp64_refreshes"] + 3},
               "do_nothing": []}
        log(f"2D {name}: CMCG {wall:.2f} s, {rep['iterations']} iterations")
        with cmcg.Solver(prob, "fp64") as s:
            J0 = s.misfit(np.zeros(s.info["state_len"]))
            for L in longtime:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                z = s.runup(L, ramp=False)
                torch.cuda.synchronize()
                w = time.perf_counter() - t0
                J = s.misfit(z)
                err = float(np.linalg.norm(s.filter(z) - U) / np.linalg.norm(U))
                res["do_nothing"].append({"periods": L, "seconds": round(w, 3),
                                          "relative_misfit": float(np.sqrt(J / J0)),
                                          "filtered_rel_error_vs_cmcg": err})
                log(f"2D {name}: do-nothing {L} periods: misfit {np.sqrt(J / J0):.3e}, error {err:.3e}")
        out[name] = res
    return out


def cpu_baseline(prob, steps: int = 20):
    """The oracle as it stands, on the full grid: `steps` forward leapfrog steps plus `steps`
    transposed steps (the two halves of a CG iteration), timed on one host core."""
    from oracle.f1 import F1
    import numpy as np
    o = F1(prob)
    rng = np.random.default_rng(0)
    z = rng.standard_normal(o.size)
    t0 = time.perf_counter()
    o.period(z, False, steps=steps)
    o.period_T(z, steps=steps)
    dt = time.perf_counter() - t0
    cells = prob.n[0] * prob.n[1]
    return {"value": round(2 * steps * cells / dt / 1e9, 4), "unit": "GLUP/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} forward + {steps} transposed leapfrog steps of the NumPy FP64 oracle "
                      f"on the full {prob.n[0]}x{prob.n[1]} grid ({dt:.1f} s; NumPy element-wise "
                      f"kernels run on one thread)",
            "seconds": round(dt, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--steps-per-launch", type=int, default=0)
    ap.add_argument("--no-tts", action="store_true")
    ap.add_argument("--tts-runs", type=int, default=3,
                    help="timed solves per precision after one warm-up (the median is reported)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--fp64-step", action="store_true",
                    help="time FP64 CG iterations instead (the FP64 path's rate and roofline)")
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the 512^3 second-order inclusions solves (FP32-mixed and FP64)")
    ap.add_argument("--c3-iters", type=int, default=0,
                    help="only K FP32-mixed CG iterations of the 512^3 problem (for profiling)")
    ap.add_argument("--nodal", default="", help="comma list of inclusions,sphere: 3D solves")
    ap.add_argument("--nodal-max-iter", type=int, default=3000)
    ap.add_argument("--nodal-precisions", default="fp32", help="comma list of fp32,fp64")
    ap.add_argument("--nodal-cpu", action="store_true",
                    help="also time the nodal oracle on a bounded sample of each 3D workload")
    ap.add_argument("--serving", type=int, default=0, help="replay this many serving requests")
    ap.add_argument("--runup-study", action="store_true",
                    help="run-up and do-nothing long-time solve on the 4096^2 workload")
    ap.add_argument("--obstacle-study", action="store_true",
                    help="CMCG vs the do-nothing solve for a convex and a nonconvex obstacle")
    ap.add_argument("--supershot-study", action="store_true",
                    help="one multi-frequency CMCG solve vs separate single-frequency solves")
    args = ap.parse_args()

    if args.calibrate_copy:
        calibrate_copy()
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU slab decomposition is described, not implemented",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import cmcg_inputs as ci
    from paper_1903_12522_amd import cmcg

    torch.cuda.set_device(0)
    log("building the 4096^2 random-medium workload")
    prob = ci.random_medium_2d(n=args.n)
    cells = prob.n[0] * prob.n[1]
    spl = args.steps_per_launch

    # ---------------------------------------------------------------- timed CG iterations
    step_prec = "fp64" if args.fp64_step else "fp32"
    with cmcg.Solver(prob, step_prec, tol=0.0, max_iter=1 << 30, steps_per_launch=spl) as s:
        N = s.info["steps_per_period"]
        s.begin()
        log(f"N = {N} steps per period; {args.warmup} warm-up iterations")
        _, rep0 = s.iterate(args.warmup) if args.warmup > 0 else (None, None)
        if rep0 is None:
            _, rep0 = s.iterate(0)
        # the K timed iterations run in one cmcg_iterate call: the library's own iteration loop,
        # as in cmcg_solve
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.iterate(args.steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, rep1 = s.iterate(0)
        kb = s.info["steps_per_launch"]
        dev_bytes = s.info["device_bytes"]
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    # every leapfrog update done in the timed region (FP64 residual refreshes included)
    updates = rep1["grid_updates"] - rep0["grid_updates"]
    glups = updates / elapsed / 1e9
    log(f"{args.steps} iterations in {elapsed:.3f} s: {ms_per_step:.2f} ms/iteration, {glups:.1f} GLUP/s")

    # roofline of the dominant kernel: the launches between each period's first and last, in
    # both directions the forward middle instance, timed by the library's HIP events around them
    nl = (rep1["bulk_launches_fwd"] - rep0["bulk_launches_fwd"]
          + rep1["bulk_launches_adj"] - rep0["bulk_launches_adj"])
    tb = (rep1["seconds_bulk_fwd"] - rep0["seconds_bulk_fwd"]
          + rep1["seconds_bulk_adj"] - rep0["seconds_bulk_adj"])
    fwd_us = 1e6 * (rep1["seconds_bulk_fwd"] - rep0["seconds_bulk_fwd"]) / max(
        1, rep1["bulk_launches_fwd"] - rep0["bulk_launches_fwd"])
    adj_us = 1e6 * (rep1["seconds_bulk_adj"] - rep0["seconds_bulk_adj"]) / max(
        1, rep1["bulk_launches_adj"] - rep0["bulk_launches_adj"])
    # read Px, Py, v, kap; write Px, Py, v
    bytes_per_update = 56 if args.fp64_step else 28
    kname = f"f1_stream_kernel<{'double' if args.fp64_step else 'float'}, {kb}, false, false, 0>"
    roofline = roofline_entry(kname, tb / nl, bytes_per_update * cells * kb,
                              bytes_per_update * cells, nl, workload="random medium 4096^2",
                              fwd_avg_launch_us=round(fwd_us, 2), adj_avg_launch_us=round(adj_us, 2))

    out = {"metric": METRIC, "value": round(glups, 2), "unit": "GLUP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.fp64_step else "f32", "data": "synthetic",
           "config": {"workload": f"first-order random medium {prob.n[0]}x{prob.n[1]}, "
                                  f"omega=2pi*100, 8 sources, "
                                  f"{'FP64' if args.fp64_step else 'FP32-mixed'} CG iteration",
                      "cells": cells, "steps_per_period": N, "steps_per_launch": kb,
                      "grid_updates_per_step": 2 * N * cells, "device_bytes": dev_bytes},
           "roofline": roofline}

    # ---------------------------------------------------------------- time to solution
    if not args.no_tts:
        res = {}
        U = {}
        for prec in ("fp32", "fp64"):
            with cmcg.Solver(prob, prec, tol=1e-6, max_iter=5000, steps_per_launch=spl) as s:
                # one warm-up solve, then the median of --tts-runs solves on the same handle
                # (each from z = 0; creation excluded)
                s.solve(device_output=True)
                runs = []
                for _ in range(max(1, args.tts_runs)):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    u, rep = s.solve(device_output=True)
                    torch.cuda.synchronize()
                    runs.append((rep["seconds"], time.perf_counter() - t0, rep))
                U[prec] = torch.complex(u[0], u[1])
            runs.sort(key=lambda r: r[0])
            sec, wall, rep = runs[len(runs) // 2]
            res[prec] = {"seconds": round(sec, 3), "wall_seconds": round(wall, 3),
                         "runs": len(runs), "seconds_min": round(runs[0][0], 3),
                         "seconds_max": round(runs[-1][0], 3),
                         "iterations": rep["iterations"], "converged": rep["converged"],
                         "rel_residual": rep["rel_residual"],
                         "glups": round(rep["grid_updates"] / rep["seconds"] / 1e9, 2),
                         "stencil_dram_GB": round(rep["dram_bytes"] / 1e9, 1),
                         "stencil_dram_GB_per_s": round(rep["dram_bytes"] / rep["seconds"] / 1e9, 1)}
            log(f"TTS {prec}: median {sec:.3f} s of {len(runs)}, {rep['iterations']} iterations")
        err = float(torch.linalg.vector_norm(U["fp32"] - U["fp64"]) / torch.linalg.vector_norm(U["fp64"]))
        out["time_to_solution"] = {
            "tol": 1e-6, "fp32_mixed": res["fp32"], "fp64": res["fp64"],
            "fp64_over_fp32_mixed": round(res["fp64"]["seconds"] / res["fp32"]["seconds"], 3),
            "fp32_mixed_rel_l2_vs_fp64": err}
        del U

    out["single_source_128"] = single_source_tts()

    # ---------------------------------------------------------------- 512^3 second order
    if args.c3_iters > 0:
        out["c3_iterations"] = nodal_3d("inclusions", "fp32", args.c3_iters, tol=0.0)
    elif not args.no_c3 and not args.no_tts:
        # both precisions with the same Riesz map (one fixed V-cycle per iteration), so the
        # time ratio is the precision's alone; one solve each (about a minute apiece)
        kept = {}
        c3 = {p: nodal_3d("inclusions", p, 3000, keep=kept, riesz_mode="vcycle")
              for p in ("fp32", "fp64")}
        c3["fp64_over_fp32_mixed"] = round(c3["fp64"]["seconds"] / c3["fp32"]["seconds"], 3)
        c3["fp32_mixed_rel_l2_vs_fp64"] = float(
            torch.linalg.vector_norm(kept["fp32"] - kept["fp64"])
            / torch.linalg.vector_norm(kept["fp64"]))
        del kept
        out["time_to_solution_c3"] = c3
    for which in [w for w in args.nodal.split(",") if w]:
        kept = {}
        out[f"nodal_{which}"] = {p: nodal_3d(which, p, args.nodal_max_iter, keep=kept)
                                 for p in args.nodal_precisions.split(",") if p}
        if "fp32" in kept and "fp64" in kept:
            out[f"nodal_{which}"]["fp32_mixed_rel_l2_vs_fp64"] = float(
                torch.linalg.vector_norm(kept["fp32"] - kept["fp64"])
                / torch.linalg.vector_norm(kept["fp64"]))
        del kept
        if args.nodal_cpu:
            cb = nodal_cpu_baseline(which)
            runs = [r for r in out[f"nodal_{which}"].values() if r["converged"]]
            if runs:
                # the oracle's step rate carried over to each converged solve: two periods of
                # N steps per CG iteration (Riesz solves and vector work not counted)
                for r in runs:
                    r["cpu_extrapolated_seconds"] = round(
                        2 * r["steps_per_period"] * r["iterations"] * r["nodes"]
                        / (cb["value"] * 1e9), 0)
                cb["extrapolated_note"] = ("cpu_extrapolated_seconds in each solve: its CG "
                                           "iterations x 2 periods x N steps at the sampled "
                                           "oracle rate")
            out[f"nodal_{which}"]["cpu_baseline"] = cb
    if args.serving > 0:
        out["serving"] = serving_run(args.serving)
    if args.runup_study:
        out["runup_study"] = runup_study(prob)
    if args.obstacle_study:
        out["obstacle_study"] = obstacle_study()
        out["obstacle_study_2d"] = obstacle_study_2d()
    if args.supershot_study:
        out["supershot_study"] = supershot_study()

    # ---------------------------------------------------------------- CPU oracle baseline
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        cb = cpu_baseline(prob)
        tts = out.get("time_to_solution")
        if tts:
            # the oracle's step rate carried over to the FP64 solve's iterations: two periods of
            # N steps per CG iteration (vector work and the filter not counted)
            its = tts["fp64"]["iterations"]
            cb["extrapolated_tts_seconds"] = round(2 * N * its * cells / (cb["value"] * 1e9), 0)
            cb["extrapolated_tts_note"] = (f"extrapolated: {its} FP64 CG iterations x 2 periods "
                                           f"x {N} steps at the sampled oracle rate")
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
