"""First-order formulation (Sec. 3.1, eq. mixWE): the oracle's staggered leapfrog scheme.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

Continuous system (eq. mixWE, 2D):  (1/c^2) v_t - div p = Re(f e^{-i w t}),
p_t = grad v,  p.n + v / c = Re(gS e^{-i w t}) on absorbing faces, p.n = 0 on Neumann faces.

Space (reading of the paper's mass-lumped FE on a structured grid): v and c live at
the centres of n_x x n_y square cells of side h; the flux p lives on interior faces
(Px on faces normal to x, Py on faces normal to y); boundary faces carry no unknown, their
flux is given by the boundary condition.  (G v) on a face is the difference across it
over h; the divergence D = -G^T on interior faces plus, on each absorbing boundary face
of a cell, (gS - v/c) / h.

Time (leapfrog, reading: kick-drift-kick with p half kicks, damping centred in time),
with t_{n+1/2} = (n + 1/2) dt and gamma = dt c m / (2 h), m = number of absorbing faces of
the cell:
    p+      = p^n + dt/2 G v^n
    (1+gamma) v^{n+1} = (1-gamma) v^n + dt c^2 [ D p+ + Re(f e^{-iwt}) + (1/h) sum_abs Re(gS e^{-iwt}) ]
    p^{n+1} = p+ + dt/2 G v^{n+1}
One period T = 2 pi / omega takes an integer number N = ceil(T c_max / (sigma h)) of
steps (the paper uses a step count that divides the period), dt = T / N.

Dirichlet data (eq. mixWE_DBC) lives on sound-soft cells (mask R = 0): their v is no unknown;
the homogeneous step multiplies v by R on input and in the velocity update, and a forced step
holds it at Re(-i w gD e^{-i w t}) at t_n (input) and t_{n+1} (output, ramped like the source).
The state is zero there.

Energy metric (eq. mix_cost_functional_J):  M_E = diag(h^2 on faces, h^2 / c^2 on cells).
Riesz map: M_E^{-1} (the control space is L^2, so no elliptic solve is needed, Sec. 3).
Output (eq. TH_FILTERED_MIXED_SOLUTION, discrete): V = (2/N) sum_{n<N} v^n e^{i w t_n},
u = i V / omega.

State vector layout (same packed order as the C ABI):  [Px (ny, nx-1), Py (ny-1, nx),
v (ny, nx)], each row-major with x fastest.
"""
from __future__ import annotations

import math
from typing import List, Optional, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import cmcg as _cmcg

ABSORBING = 0


class F1:
    """The discrete first-order scheme for one problem (2D)."""

    def __init__(self, prob, N: Optional[int] = None):
        assert prob.dim == 2 and prob.formulation == 1
        self.prob = prob
        self.nx, self.ny = int(prob.n[0]), int(prob.n[1])
        self.h = float(prob.h)
        self.c = prob.c_array().reshape(self.ny, self.nx)
        self.omega = float(prob.omega)
        self.T = 2.0 * math.pi / self.omega
        if N is None:
            N = int(math.ceil(self.T * float(self.c.max()) / (prob.courant * self.h)))
        self.N = N
        self.dt = self.T / N
        bc = list(prob.face_bc)[:4]
        self.bc = bc
        m = np.zeros((self.ny, self.nx))
        if bc[0] == ABSORBING:
            m[:, 0] += 1
        if bc[1] == ABSORBING:
            m[:, -1] += 1
        if bc[2] == ABSORBING:
            m[0, :] += 1
        if bc[3] == ABSORBING:
            m[-1, :] += 1
        self.m = m
        self.gamma = self.dt * self.c * m / (2.0 * self.h)
        # Dirichlet (sound-soft) cells: R = 0 there; v is held at the data, not an unknown
        self.free = (np.ones((self.ny, self.nx)) if prob.sound_soft is None
                     else 1.0 - np.asarray(prob.sound_soft, dtype=np.float64).reshape(self.ny, self.nx))
        # data of each time-harmonic component: (m, f, g, gD), angular frequency m * omega
        self.comps = []
        for m, f, gS, gD in _cmcg.components(prob):
            f = (np.zeros((self.ny, self.nx), complex) if f is None
                 else np.asarray(f, dtype=complex).reshape(self.ny, self.nx))
            if gS is None:
                g = [np.zeros(self.ny, complex), np.zeros(self.ny, complex),
                     np.zeros(self.nx, complex), np.zeros(self.nx, complex)]
            else:
                g = [np.asarray(a, dtype=complex).reshape(-1) for a in gS[:4]]
            gD = (None if gD is None or prob.sound_soft is None
                  else (1.0 - self.free) * np.asarray(gD, dtype=complex).reshape(self.ny, self.nx))
            self.comps.append((m, f, g, gD))
        self.shapes = [(self.ny, self.nx - 1), (self.ny - 1, self.nx), (self.ny, self.nx)]
        self.sizes = [a * b for a, b in self.shapes]
        self.size = sum(self.sizes)

    # ---------------------------------------------------------------- packing
    def unpack(self, z: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        a, b, _ = self.sizes
        return (z[:a].reshape(self.shapes[0]), z[a:a + b].reshape(self.shapes[1]),
                z[a + b:].reshape(self.shapes[2]))

    @staticmethod
    def pack(Px, Py, v) -> np.ndarray:
        return np.concatenate([Px.ravel(), Py.ravel(), v.ravel()])

    # ---------------------------------------------------------------- operators
    def grad(self, v):
        """G v on the interior faces."""
        h = self.h
        return (v[:, 1:] - v[:, :-1]) / h, (v[1:, :] - v[:-1, :]) / h

    def div(self, Px, Py):
        """D p over the interior faces of each cell (boundary fluxes are added by the
        caller from the boundary condition)."""
        h = self.h
        out = np.zeros((self.ny, self.nx))
        out[:, :-1] += Px / h       # right face of cell i is face i+1/2
        out[:, 1:] -= Px / h        # left face of cell i+1
        out[:-1, :] += Py / h
        out[1:, :] -= Py / h
        return out

    def grad_T(self, Px, Py):
        """Literal transpose of `grad` (a map from faces to cells)."""
        h = self.h
        out = np.zeros((self.ny, self.nx))
        out[:, 1:] += Px / h
        out[:, :-1] -= Px / h
        out[1:, :] += Py / h
        out[:-1, :] -= Py / h
        return out

    def div_T(self, v):
        """Literal transpose of `div` (a map from cells to faces)."""
        h = self.h
        return (v[:, :-1] - v[:, 1:]) / h, (v[:-1, :] - v[1:, :]) / h

    def source(self, t: float) -> np.ndarray:
        """Re(f e^{-iwt}) + (1/h) sum over the boundary faces of Re(g e^{-iwt}): the prescribed
        part of the outward flux p.n, gS on absorbing faces (p.n = gS - v/c) and gN on Neumann
        faces (p.n = gN); summed over the components, each at its own frequency m w."""
        h = self.h
        F = np.zeros((self.ny, self.nx))
        for m, f, g, _ in self.comps:
            e = np.exp(-1j * m * self.omega * t)
            F += (f * e).real
            F[:, 0] += (g[0] * e).real / h
            F[:, -1] += (g[1] * e).real / h
            F[0, :] += (g[2] * e).real / h
            F[-1, :] += (g[3] * e).real / h
        return F

    def dirichlet_v(self, t: float) -> np.ndarray:
        """v on the Dirichlet cells at time t (eq. mixWE_DBC): Re(-i m w gD e^{-i m w t}) summed
        over the components (zero elsewhere)."""
        out = np.zeros((self.ny, self.nx))
        for m, _, _, gD in self.comps:
            if gD is not None:
                w = m * self.omega
                out += (-1j * w * gD * np.exp(-1j * w * t)).real
        return out

    def has_dirichlet_data(self) -> bool:
        return any(c[3] is not None for c in self.comps)

    # ---------------------------------------------------------------- time stepping
    def step(self, Px, Py, v, n: int, forced: bool, ramp=None):
        """Step n (t_n -> t_{n+1}); the source is sampled at t_{n+1/2} and multiplied by
        ramp(t_{n+1/2}) when a ramp is given.  On Dirichlet cells v is the data at t_n (input,
        forced) or 0, and the data at t_{n+1} (ramped like the source) or 0 on output."""
        dt, c, gam, R = self.dt, self.c, self.gamma, self.free
        amp = (lambda t: 1.0) if ramp is None else ramp
        dirichlet = forced and self.has_dirichlet_data()
        v = R * v + ((1.0 - R) * amp(n * dt) * self.dirichlet_v(n * dt) if dirichlet else 0.0)
        gx, gy = self.grad(v)
        Px = Px + 0.5 * dt * gx
        Py = Py + 0.5 * dt * gy
        rhs = self.div(Px, Py)
        if forced:
            t = (n + 0.5) * dt
            rhs = rhs + amp(t) * self.source(t)
        v = R * ((1.0 - gam) * v + dt * c * c * rhs) / (1.0 + gam)
        if dirichlet:
            t1 = (n + 1) * dt
            v = v + (1.0 - R) * amp(t1) * self.dirichlet_v(t1)
        gx, gy = self.grad(v)
        Px = Px + 0.5 * dt * gx
        Py = Py + 0.5 * dt * gy
        return Px, Py, v

    def step_T(self, Px, Py, v):
        """Literal transpose of the homogeneous step: the transposes of its sub-maps (input
        mask, half kick, masked damped velocity update, half kick) applied in reverse order."""
        dt, c, gam, R = self.dt, self.c, self.gamma, self.free
        a = (1.0 - gam) / (1.0 + gam)
        b = dt * c * c / (1.0 + gam)
        # transpose of the second half kick  p <- p + dt/2 G v
        v = v + 0.5 * dt * self.grad_T(Px, Py)
        # transpose of  v <- R (a v + b D p)   (p unchanged)
        tx, ty = self.div_T(b * R * v)
        Px = Px + tx
        Py = Py + ty
        v = a * R * v
        # transpose of the first half kick, then of the input mask v <- R v
        v = v + 0.5 * dt * self.grad_T(Px, Py)
        return Px, Py, R * v

    def period(self, z: np.ndarray, forced: bool, t0_step: int = 0,
               steps: Optional[int] = None, ramp=None) -> np.ndarray:
        """Phi(z) (forced) or E z (homogeneous): N leapfrog steps from t = t0_step dt, the
        source optionally multiplied by ramp(t)."""
        Px, Py, v = self.unpack(z)
        for n in range(self.N if steps is None else steps):
            Px, Py, v = self.step(Px, Py, v, t0_step + n, forced, ramp)
        # the state is zero on the Dirichlet cells
        return self.pack(Px, Py, self.free * v)

    def runup(self, periods: int, ramp: bool) -> np.ndarray:
        """State at t = periods T of the forced scheme started from rest, with the source
        switched on by Mur's transient over the whole interval if `ramp` (Sec. 4.2.3), or at
        once (the do-nothing long-time solve of Sec. 4.2.2)."""
        t_tr = periods * self.T
        th = (lambda t: _cmcg.transient(t, t_tr)) if ramp else None
        return _cmcg.runup(lambda z, p: self.period(z, True, t0_step=p * self.N, ramp=th),
                           self.size, periods)

    def period_T(self, y: np.ndarray, steps: Optional[int] = None) -> np.ndarray:
        """E^T y: the transposed steps, last step first (all steps are equal here)."""
        Px, Py, v = self.unpack(y)
        for _ in range(self.N if steps is None else steps):
            Px, Py, v = self.step_T(Px, Py, v)
        return self.pack(Px, Py, v)

    # ---------------------------------------------------------------- metric, Riesz
    def weights(self) -> np.ndarray:
        """Diagonal of M_E (zero on the Dirichlet cells, which carry no unknown)."""
        h2 = self.h * self.h
        return np.concatenate([np.full(self.sizes[0], h2), np.full(self.sizes[1], h2),
                               (self.free * h2 / (self.c * self.c)).ravel()])

    def ME(self, w):
        return self.weights() * w

    def riesz(self, rhat):
        """M_E^{-1} on the unknowns (zero on the Dirichlet cells)."""
        w = self.weights()
        out = np.zeros_like(rhat)
        nz = w > 0
        out[nz] = rhat[nz] / w[nz]
        return out

    def energy(self, Px, Py, v) -> float:
        """Discrete energy conserved by the undamped scheme:
        1/2 h^2 |p|^2 - dt^2/8 h^2 |G v|^2 + 1/2 h^2 sum v^2 / c^2."""
        h2 = self.h * self.h
        gx, gy = self.grad(v)
        return (0.5 * h2 * (np.sum(Px * Px) + np.sum(Py * Py))
                - self.dt ** 2 / 8.0 * h2 * (np.sum(gx * gx) + np.sum(gy * gy))
                + 0.5 * h2 * np.sum(v * v / (self.c * self.c)))

    # ---------------------------------------------------------------- CMCG and output
    def solve(self, tol: float, max_iter: int = 10000, z0=None, record=None,
              runup_periods: int = 0):
        """CMCG from rest, or from the state of a ramped run-up of `runup_periods` periods
        (Sec. 4.2.3) with the stopping test measured against the residual at rest."""
        ref = None
        if runup_periods > 0:
            z0 = self.runup(runup_periods, True)
            ref = _cmcg.gradient_delta(lambda x: self.period(x, True), self.period_T, self.ME,
                                       self.riesz, self.size)
        z, hist, it = _cmcg.cmcg(lambda x: self.period(x, True),
                                 lambda x: self.period(x, False),
                                 self.period_T, self.ME, self.riesz,
                                 self.size, tol, max_iter, z0=z0, record=record, delta_ref=ref)
        return z, hist, it

    def filter(self, z: np.ndarray) -> np.ndarray:
        """u = i V / omega with V = (2/N) sum_{n<N} v^n e^{i w t_n} over one forced period
        from z (eq. TH_FILTERED_MIXED_SOLUTION with the rectangle rule).  With several
        components, one such sum per component at its frequency m w (u = i V / (m w)) over the
        same period; the result is then stacked, shape (components, ny, nx)."""
        Px, Py, v = self.unpack(z)
        # v^0 on the Dirichlet cells is the data at t = 0
        v = self.free * v + (1.0 - self.free) * self.dirichlet_v(0.0)
        V = [np.zeros((self.ny, self.nx), complex) for _ in self.comps]
        for n in range(self.N):
            for c, (m, _, _, _) in enumerate(self.comps):
                V[c] += v * np.exp(1j * m * self.omega * n * self.dt)
            Px, Py, v = self.step(Px, Py, v, n, True)
        U = [1j * (2.0 / self.N) * Vc / (c[0] * self.omega) for Vc, c in zip(V, self.comps)]
        return U[0] if len(U) == 1 else np.stack(U)

    def step6_output(self, z: np.ndarray) -> np.ndarray:
        """The solution read off the initial state alone (eq. mix_solution in time-discrete
        form, single component).  The frequency system's face rows give the flux amplitude
        Q = i dt G V / (2 sin(theta)); with Re V = v_0 and Re Q = P_0 / cos(theta) this gives
        Q = P_0 / cos(theta) + i dt G v_0 / (2 sin(theta)), and the cell rows then give
        V = dt c^2 (Fhat + D Q) / (-2 i sin(theta) + 2 gamma cos(theta)), u = i V / omega.
        Divergence-free flux fields (the non-uniqueness of Thm 2) drop out through D."""
        assert len(self.comps) == 1, "Step 6 output of a single-frequency problem"
        Px, Py, v = self.unpack(z)
        dt, h = self.dt, self.h
        th = 0.5 * self.omega * dt
        _, f, g, gD = self.comps[0]
        # Dirichlet cells: V = -i omega gD is data; its real part is v_0 there
        VD = np.zeros((self.ny, self.nx), complex) if gD is None else -1j * self.omega * gD
        v = self.free * v + (1.0 - self.free) * VD.real
        gx, gy = self.grad(v)
        Qx = Px / math.cos(th) + 1j * dt * gx / (2.0 * math.sin(th))
        Qy = Py / math.cos(th) + 1j * dt * gy / (2.0 * math.sin(th))
        DQ = np.zeros((self.ny, self.nx), complex)
        DQ[:, :-1] += Qx / h
        DQ[:, 1:] -= Qx / h
        DQ[:-1, :] += Qy / h
        DQ[1:, :] -= Qy / h
        Fhat = f.copy()
        Fhat[:, 0] += g[0] / h
        Fhat[:, -1] += g[1] / h
        Fhat[0, :] += g[2] / h
        Fhat[-1, :] += g[3] / h
        V = dt * self.c ** 2 * (Fhat + DQ) / (-2j * math.sin(th) + 2.0 * self.gamma * math.cos(th))
        V = self.free * V + (1.0 - self.free) * VD
        return 1j * V / self.omega

    def functional(self, z):
        return _cmcg.functional(lambda x: self.period(x, True), self.ME, z)

    # ---------------------------------------------------------------- direct solve
    def frequency_system(self, comp: int = 0):
        """Sparse time-discretised Helmholtz system for the amplitudes V (cells) and Q
        (faces, at half steps) of the discrete periodic solution
        v^n = Re(V e^{-iwt_n}), p^{n+1/2} = Re(Q e^{-iwt_{n+1/2}}), theta = w dt / 2:
            -2 i sin(theta) Q - dt G V = 0
            (-2 i sin(theta) + 2 gamma cos(theta)) V - dt c^2 D Q = dt c^2 Fhat,
        Fhat = f + (1/h) sum over the boundary faces of g (gS or gN), for component `comp`
        (w its frequency m omega, same dt)."""
        nx, ny, h, dt = self.nx, self.ny, self.h, self.dt
        m, f, g, gD = self.comps[comp]
        th = 0.5 * m * self.omega * dt

        def d1(m):
            return sp.diags([-np.ones(m - 1), np.ones(m - 1)], [0, 1], shape=(m - 1, m)) / h

        Gx = sp.kron(sp.identity(ny), d1(nx))
        Gy = sp.kron(d1(ny), sp.identity(nx))
        G = sp.vstack([Gx, Gy]).tocsr()
        D = -G.T
        nf = G.shape[0]
        c2 = (self.c * self.c).ravel()
        gam = self.gamma.ravel()
        A = sp.bmat([[-2j * math.sin(th) * sp.identity(nf), -dt * G],
                     [-dt * sp.diags(c2) @ D,
                      sp.diags(-2j * math.sin(th) + 2.0 * gam * math.cos(th))]]).tocsc()
        Fhat = f.copy()
        Fhat[:, 0] += g[0] / h
        Fhat[:, -1] += g[1] / h
        Fhat[0, :] += g[2] / h
        Fhat[-1, :] += g[3] / h
        rhs = np.concatenate([np.zeros(nf, complex), dt * c2 * Fhat.ravel()])
        dcells = np.flatnonzero(self.free.ravel() < 0.5)
        if dcells.size:
            # Dirichlet cells: V = -i m omega gD is known (eq. mixWE_DBC); identity rows
            rows = nf + dcells
            A = A.tolil()
            A[rows, :] = 0.0
            A[rows, rows] = 1.0
            A = A.tocsc()
            VD = np.zeros(nx * ny, complex) if gD is None else -1j * m * self.omega * gD.ravel()
            rhs[rows] = VD[dcells]
        return A, rhs, nf

    def direct(self):
        """Direct sparse solve of the frequency-domain system.  Returns (u, z_periodic):
        u = i V / omega and the periodic state (P^0, v^0) = (cos(theta) Re Q, Re V).  With
        several components, u is stacked per component (u = i V / (m omega) at theta =
        m omega dt / 2) and the periodic state is the sum of the components' states (the
        scheme is linear)."""
        U, z = [], np.zeros(self.size)
        for c, (m, _, _, _) in enumerate(self.comps):
            A, rhs, nf = self.frequency_system(c)
            x = spla.spsolve(A, rhs)
            Q, V = x[:nf], x[nf:]
            th = 0.5 * m * self.omega * self.dt
            z = z + np.concatenate([math.cos(th) * Q.real, self.free.ravel() * V.real])
            U.append((1j * V / (m * self.omega)).reshape(self.ny, self.nx))
        return (U[0] if len(U) == 1 else np.stack(U)), z


def window(prob, i0: int, i1: int, j0: int, j1: int):
    """Sub-problem on cells [i0, i1) x [j0, j1) of `prob`, for sampled checks: sides that
    lie on the original boundary keep its condition and data, cut sides become Neumann.
    After K steps, values more than K + 2 cells away from a cut side equal those of the
    full problem (each step couples a cell only to its face neighbours)."""
    import copy
    sub = copy.copy(prob)
    nx, ny = prob.n[0], prob.n[1]
    sub.n = (i1 - i0, j1 - j0)
    sub.spacing = prob.h
    c = prob.c_array().reshape(ny, nx)
    sub.c = c[j0:j1, i0:i1].copy()
    sub.f = None if prob.f is None else np.asarray(prob.f).reshape(ny, nx)[j0:j1, i0:i1].copy()
    bc = list(prob.face_bc)[:4]
    g = prob.gS
    newbc = [bc[0] if i0 == 0 else 1, bc[1] if i1 == nx else 1,
             bc[2] if j0 == 0 else 1, bc[3] if j1 == ny else 1]
    sub.face_bc = tuple(newbc)
    if g is not None:
        sub.gS = [np.asarray(g[0])[j0:j1], np.asarray(g[1])[j0:j1],
                  np.asarray(g[2])[i0:i1], np.asarray(g[3])[i0:i1]]
    return sub
