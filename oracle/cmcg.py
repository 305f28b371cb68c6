"""The CMCG Algorithm (Sec. 2.3, Steps 1-6), for any discretised wave scheme.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

Discrete reading (discretise-then-optimise).  With the forced one-period map
Phi(z) = E z + s and the energy Gram matrix M_E, the functional of eq. cost_functional_J
(resp. eq. mix_cost_functional_J) is  J(z) = 1/2 (Phi(z) - z)^T M_E (Phi(z) - z).  Its
gradient (the dual object g of eq. J1_derivative_final / eq. mixJ_deriative_2) is

    ghat = (E^T - I) M_E (Phi(z) - z),

the backward (adjoint) wave solve being the literal transpose E^T, and the Riesz
representer of eq. CMCG_PRECONDITIONIER is g~ = P ghat.  The CG of Steps 2-5 then runs
with the primal residual r = g~ and the dual residual rhat = ghat, so that
rhat^T r = ||grad r_0||^2 + ||r_1 / c||^2 (the numerator of alpha in Step 5.3) and
qhat^T d = (grad g~_0, grad d_0) + (g~_1 / c^2, d_1) (its denominator).  The loop index
starts at 0 (Step 4 sets r^(0) while Step 5 counts from 1; both describe the same loop).
"""
from __future__ import annotations

import math
from typing import Callable, List, Optional

import numpy as np


def cmcg(phi: Callable[[np.ndarray], np.ndarray],
         E: Callable[[np.ndarray], np.ndarray],
         ET: Callable[[np.ndarray], np.ndarray],
         ME: Callable[[np.ndarray], np.ndarray],
         riesz: Callable[[np.ndarray], np.ndarray],
         size: int, tol: float, max_iter: int,
         z0: Optional[np.ndarray] = None,
         record: Optional[List[np.ndarray]] = None,
         delta_ref: Optional[float] = None):
    """Run CMCG from z0 (default 0, as in the paper's experiments) until the relative
    energy-norm residual sqrt(rhat^T r / delta_ref) <= tol (Step 5.8) or max_iter
    iterations; delta_ref defaults to the start's own rhat0^T r0.  (A start from a run-up
    state passes the value at z = 0, so that it stops at the accuracy a start from rest
    stops at.)  Returns (z, history, iterations) with history[l] the relative residual after
    iteration l.  If `record` is a list, every iterate z_l (including z_0) is appended."""
    z = np.zeros(size) if z0 is None else np.array(z0, dtype=np.float64)
    if record is not None:
        record.append(z.copy())
    # Step 2: forward (forced) and backward periods give the gradient at z.
    w = phi(z) - z
    rhat = ET(ME(w)) - ME(w)
    # Steps 3-4: Riesz representer, first direction.
    r = riesz(rhat)
    d = r.copy()
    delta = float(rhat @ r)
    delta0 = delta if delta_ref is None else float(delta_ref)
    history = [math.sqrt(delta / delta0) if delta0 > 0.0 else 0.0]
    if delta == 0.0 or history[0] <= tol:
        return z, history, 0
    it = 0
    for it in range(1, max_iter + 1):
        # Step 5.1: homogeneous forward period on d, then the backward period.
        w = E(d) - d
        qhat = ET(ME(w)) - ME(w)
        # Step 5.2: Riesz representer.
        q = riesz(qhat)
        # Step 5.3
        alpha = delta / float(qhat @ d)
        # Steps 5.4, 5.5 (primal and dual residual)
        z = z - alpha * d
        r = r - alpha * q
        rhat = rhat - alpha * qhat
        if record is not None:
            record.append(z.copy())
        delta_new = float(rhat @ r)
        rel = math.sqrt(max(delta_new, 0.0) / delta0)
        history.append(rel)
        # Step 5.8
        if rel <= tol:
            break
        # Steps 5.6, 5.7
        beta = delta_new / delta
        d = r + beta * d
        delta = delta_new
    return z, history, it


def gradient_delta(phi, ET, ME, riesz, size: int) -> float:
    """rhat^T r of the gradient at z = 0 (Steps 2-3 from rest)."""
    w = phi(np.zeros(size))
    rhat = ET(ME(w)) - ME(w)
    return float(rhat @ riesz(rhat))


def functional(phi, ME, z: np.ndarray) -> float:
    """J(z) = 1/2 (Phi(z) - z)^T M_E (Phi(z) - z)  (eq. cost_functional_J, discrete)."""
    w = phi(z) - z
    return 0.5 * float(w @ ME(w))


def transient(t: float, t_tr: float) -> float:
    """Mur's smooth switch-on of the time-harmonic source (Sec. 4.2.3, eq. transientfunction):
    theta(t) = (2 - sin(s)) sin(s) with s = (t / t_tr) pi / 2 while t <= t_tr, and 1 after.
    It rises from 0 to 1 with zero slope at t_tr."""
    if t >= t_tr:
        return 1.0
    s = 0.5 * math.pi * t / t_tr
    return (2.0 - math.sin(s)) * math.sin(s)


def runup(period_at: Callable[[np.ndarray, int], np.ndarray], size: int, periods: int) -> np.ndarray:
    """Time integration of the forced wave equation from rest over `periods` periods (the
    run-up of Sec. 4.2.3 or the do-nothing long-time solve of Sec. 4.2.2): period p maps the
    state at t = pT to the state at (p + 1)T, `period_at(z, p)`."""
    z = np.zeros(size)
    for p in range(periods):
        z = period_at(z, p)
    return z


def components(prob):
    """The time-harmonic components of a problem's data, as (m, f, gS, gD) with angular
    frequency m * omega.  A multi-frequency ("super-shot") problem superposes several
    harmonics of one base frequency omega (Concluding remarks): the forced wave equation then
    has the common period T = 2 pi / omega, and each component's Helmholtz solution is the
    filter of the one periodic solution at that component's frequency.  A problem without
    shots is the single component m = 1 carrying its own data."""
    shots = getattr(prob, "shots", None)
    if shots:
        return [(int(s.harmonic), s.f, s.gS, s.gD) for s in shots]
    return [(1, prob.f, prob.gS, prob.gD)]
