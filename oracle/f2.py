"""Second-order formulation (Sec. 2, eq. WE): the oracle's nodal leapfrog scheme.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

Continuous system (eq. WE):  (1/c^2) y_tt - lap y = Re(f e^{-iwt}),
dy/dn + (1/c) y_t = Re(gS e^{-iwt}) on absorbing faces, dy/dn = Re(gN e^{-iwt}) on Neumann
faces, y = Re(gD e^{-iwt}) on the sound-soft (Dirichlet) set D (eq. WE_DBC).

Space (reading of the paper's mass-lumped P1 FE on a structured grid): nodes x_I = I h,
I in {0..n}^d.  Lumped mass w_I = h^d prod_k (1/2 if I_k is 0 or n_k), M = diag(w / c^2).
Stiffness (S u)_I = sum over the axis edges e = (I, J) of a_e (u_I - u_J), with
a_e = h^{d-2} prod over the other axes k' of (1/2 if the edge lies in a boundary plane
x_k' = 0 or 1).  Absorbing faces add the boundary mass B_I = (1/c_I) sum over absorbing
faces containing I of the lumped face weight h^{d-1} prod (1/2 on the face's own edges).
Load F^n = w Re(f e^{-iwt_n}) + sum over faces (face weight) Re(g e^{-iwt_n}), g = gS or gN.
Dirichlet nodes are not unknowns: forced periods hold them at Re(gD e^{-iwt_n}) (their state
entries stay zero), homogeneous ones at zero.

Time (leapfrog, damping centred), t_n = n dt:
    (M + dt/2 B) u^{n+1} = 2 M u^n - (M - dt/2 B) u^{n-1} - dt^2 (S u^n - F^n),  u = 0 on D
    start  u^1 = u^0 + dt (1 - beta) v^0 - dt^2/2 M^{-1} (S u^0 - F^0)   (ghost u^{-1} = u^1 - 2 dt v^0)
    end    v^N = (u^{N+1} - u^{N-1}) / (2 dt),  Phi(u^0, v^0) = (u^N, v^N)
with beta = dt B / (2 M).

Energy metric (eq. cost_functional_J):  M_E = blockdiag(S, M) on the free nodes.
Riesz map (eq. CMCG_PRECONDITIONIER): blockdiag(S^{-1}, M^{-1}); when D is empty S is
singular (constants) and its pseudo-inverse on zero-sum vectors is used.
Output (eq. fundamental-frequency-solution, discrete): U = (2/N) sum_{n<N} u^n e^{i w t_n}.

Arrays: node fields of shape (nz+1, ny+1, nx+1) (3D) or (ny+1, nx+1) (2D), x fastest.
State vector: [u (all nodes), v (all nodes)], sound-soft entries zero.
"""
from __future__ import annotations

import math
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import cmcg as _cmcg

ABSORBING = 0


def _half(m: int) -> np.ndarray:
    """1/2 at both ends of an axis of m+1 nodes, 1 inside."""
    a = np.ones(m + 1)
    a[0] = a[-1] = 0.5
    return a


class F2:
    """The discrete second-order scheme for one problem (2D or 3D)."""

    def __init__(self, prob, N: Optional[int] = None):
        assert prob.formulation == 2 and prob.dim in (2, 3)
        self.prob = prob
        self.d = d = prob.dim
        self.n = [int(m) for m in prob.n[:d]]          # x, y[, z]
        self.h = h = float(prob.h)
        self.shape = tuple(m + 1 for m in reversed(self.n))
        self.c = prob.c_array().reshape(self.shape)
        self.omega = float(prob.omega)
        self.T = 2.0 * math.pi / self.omega
        if N is None:
            N = int(math.ceil(self.T * float(self.c.max()) / (prob.courant * h)))
        assert N >= 2
        self.N = N
        self.dt = self.T / N
        self.bc = list(prob.face_bc)[: 2 * d]
        self.free = (np.ones(self.shape) if prob.sound_soft is None
                     else 1.0 - np.asarray(prob.sound_soft, dtype=np.float64).reshape(self.shape))
        # per-axis half factors broadcast to the node array (axis k -> numpy axis d-1-k)
        self.halfs = []
        for k in range(d):
            sh = [1] * d
            sh[d - 1 - k] = self.n[k] + 1
            self.halfs.append(_half(self.n[k]).reshape(sh))
        w = np.full(self.shape, h ** d)
        for k in range(d):
            w = w * self.halfs[k]
        self.w = w
        self.M = w / (self.c * self.c)
        # boundary mass and face weights
        B = np.zeros(self.shape)
        self.face_w = []
        for k in range(d):
            fw = np.full(self.shape, h ** (d - 1))
            for kk in range(d):
                if kk != k:
                    fw = fw * self.halfs[kk]
            for side in (0, 1):
                sel = [slice(None)] * d
                sel[d - 1 - k] = 0 if side == 0 else self.n[k]
                self.face_w.append((tuple(sel), fw[tuple(sel)]))
                if self.bc[2 * k + side] == ABSORBING:
                    B[tuple(sel)] += fw[tuple(sel)] / self.c[tuple(sel)]
        self.B = B
        self.beta = 0.5 * self.dt * B / self.M
        # data of each time-harmonic component: (m, f, g, gD), angular frequency m * omega;
        # gD is kept on the sound-soft nodes only
        self.comps = []
        for m, f, gS, gD in _cmcg.components(prob):
            f = (np.zeros(self.shape, complex) if f is None
                 else np.asarray(f, dtype=complex).reshape(self.shape))
            g = None if gS is None else [np.asarray(a, dtype=complex) for a in gS]
            gD = (None if gD is None or prob.sound_soft is None
                  else (1.0 - self.free) * np.asarray(gD, dtype=complex).reshape(self.shape))
            self.comps.append((m, f, g, gD))
        self.has_gD = any(c[3] is not None for c in self.comps)
        self.nn = int(np.prod(self.shape))
        self.size = 2 * self.nn
        self._S_lu = None

    # ---------------------------------------------------------------- operators
    def S(self, u: np.ndarray) -> np.ndarray:
        """Stiffness apply, summed edge by edge."""
        d, h = self.d, self.h
        out = np.zeros(self.shape)
        for k in range(d):
            ax = d - 1 - k
            a = np.full([1] * d, h ** (d - 2))
            for kk in range(d):
                if kk != k:
                    a = a * self.halfs[kk]
            lo = [slice(None)] * d
            hi = [slice(None)] * d
            lo[ax] = slice(0, -1)
            hi[ax] = slice(1, None)
            lo, hi = tuple(lo), tuple(hi)
            ae = np.broadcast_to(a, self.shape)[lo]
            flux = ae * (u[hi] - u[lo])
            out[lo] -= flux
            out[hi] += flux
        return out

    def load(self, t: float) -> np.ndarray:
        """Lumped load at time t: w Re(f e^{-i m w t}) plus the face weight times
        Re(g e^{-i m w t}) on the boundary nodes, summed over the components."""
        F = np.zeros(self.shape)
        for m, f, g, _ in self.comps:
            e = np.exp(-1j * m * self.omega * t)
            F += self.w * (f * e).real
            if g is not None:
                for idx, (sel, fw) in enumerate(self.face_w):
                    F[sel] += fw * (g[idx].reshape(fw.shape) * e).real
        return F

    def dirichlet_value(self, t: float) -> np.ndarray:
        """Re(gD e^{-i m w t}) on the sound-soft nodes, summed over the components."""
        out = np.zeros(self.shape)
        for m, _, _, gD in self.comps:
            if gD is not None:
                out += (gD * np.exp(-1j * m * self.omega * t)).real
        return out

    # ---------------------------------------------------------------- time stepping
    def _accel(self, u, F):
        """dt^2 M^{-1} (S u - F) (F may be None)."""
        r = self.S(u)
        if F is not None:
            r = r - F
        return self.dt ** 2 * r / self.M

    def period(self, z: np.ndarray, forced: bool, U_acc: Optional[List[np.ndarray]] = None,
               t0: float = 0.0, ramp=None):
        """Phi(z) (forced) or E z (homogeneous) over [t0, t0 + T], the load at t_n = t0 + n dt
        optionally multiplied by ramp(t_n).  If U_acc is given (one array per component),
        u^n e^{i m w t_n} for n < N is accumulated into U_acc[c] (the filter sums, t0 = 0)."""
        dt, beta, R = self.dt, self.beta, self.free
        amp = (lambda t: 1.0) if ramp is None else ramp
        if not forced:
            F = lambda n: None
        else:
            F = lambda n: amp(t0 + n * dt) * self.load(t0 + n * dt)
        # values on the Dirichlet nodes at t_n (zero unless forced with data)
        if forced and self.has_gD:
            dirichlet = lambda n: amp(t0 + n * dt) * self.dirichlet_value(t0 + n * dt)
        else:
            dirichlet = lambda n: 0.0

        def accumulate(u, n):
            for c, (m, _, _, _) in enumerate(self.comps):
                U_acc[c] += u * np.exp(1j * m * self.omega * n * dt)
        u0 = R * z[: self.nn].reshape(self.shape) + dirichlet(0)
        v0 = R * z[self.nn:].reshape(self.shape)
        um = u0
        u = R * (u0 + dt * (1.0 - beta) * v0 - 0.5 * self._accel(u0, F(0))) + dirichlet(1)
        if U_acc is not None:
            accumulate(um, 0)
        for n in range(1, self.N + 1):
            if U_acc is not None and n < self.N:
                accumulate(u, n)
            up = R * ((2.0 * u - (1.0 - beta) * um - self._accel(u, F(n))) / (1.0 + beta)) \
                + dirichlet(n + 1)
            if n == self.N:
                vN = R * (up - um) / (2.0 * dt)
                return np.concatenate([(R * u).ravel(), vN.ravel()])
            um, u = u, up

    def runup(self, periods: int, ramp: bool) -> np.ndarray:
        """State (u, v) at t = periods T of the forced scheme started from rest, the load
        switched on by Mur's transient if `ramp` (Sec. 4.2.3), else at once (Sec. 4.2.2)."""
        t_tr = periods * self.T
        th = (lambda t: _cmcg.transient(t, t_tr)) if ramp else None
        return _cmcg.runup(lambda z, p: self.period(z, True, t0=p * self.T, ramp=th),
                           self.size, periods)

    def period_T(self, y: np.ndarray) -> np.ndarray:
        """E^T y, with E = (end map) (step map)^{N-1} (start map) on the states
        (u^0, v^0) -> (u^1, u^0) -> ... -> (u^N, u^{N-1}) -> (u^N, v^N); each transpose is
        written out from its map and they are applied in reverse order."""
        dt, beta, R = self.dt, self.beta, self.free
        x = R * y[: self.nn].reshape(self.shape)
        yv = R * y[self.nn:].reshape(self.shape)

        def KT(q):
            """Transpose of K a = (2 a - dt^2 M^{-1} S a) / (1 + beta), masked."""
            s = R * q / (1.0 + beta)
            return R * (2.0 * s - self.dt ** 2 * self.S(s / self.M))

        L = -(1.0 - beta) / (1.0 + beta)
        # end map (a, b) -> (a, (K a + L b - b) / (2 dt)):  transpose
        a = x + KT(yv) / (2.0 * dt)
        b = R * (L - 1.0) * yv / (2.0 * dt)
        # step map (a, b) -> (K a + L b, a):  transpose (x, y) -> (K^T x + y, L x)
        for _ in range(self.N - 1):
            a, b = KT(a) + b, R * L * a
        # start map (u0, v0) -> (A u0 + B v0, u0), A = I - dt^2/2 M^{-1} S, B = dt (1 - beta)
        u0 = R * (a - 0.5 * self.dt ** 2 * self.S(R * a / self.M)) + b
        v0 = R * dt * (1.0 - beta) * a
        return np.concatenate([u0.ravel(), v0.ravel()])

    # ---------------------------------------------------------------- metric, Riesz
    def ME(self, w: np.ndarray) -> np.ndarray:
        R = self.free
        u = R * w[: self.nn].reshape(self.shape)
        v = R * w[self.nn:].reshape(self.shape)
        return np.concatenate([(R * self.S(u)).ravel(), (R * self.M * v).ravel()])

    def stiffness_matrix(self) -> sp.csr_matrix:
        """S as a sparse matrix, built edge by edge (independent of `S`)."""
        d, h = self.d, self.h
        idx = np.arange(self.nn).reshape(self.shape)
        rows, cols, vals = [], [], []
        for k in range(d):
            ax = d - 1 - k
            a = np.full([1] * d, h ** (d - 2))
            for kk in range(d):
                if kk != k:
                    a = a * self.halfs[kk]
            lo = [slice(None)] * d
            hi = [slice(None)] * d
            lo[ax] = slice(0, -1)
            hi[ax] = slice(1, None)
            I = idx[tuple(lo)].ravel()
            J = idx[tuple(hi)].ravel()
            ae = np.broadcast_to(a, self.shape)[tuple(lo)].ravel()
            rows += [I, J, I, J]
            cols += [I, J, J, I]
            vals += [ae, ae, -ae, -ae]
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.nn, self.nn))

    def _riesz_factor(self):
        if self._S_lu is None:
            S = self.stiffness_matrix()
            free = np.flatnonzero(self.free.ravel() > 0.5)
            self._pure_neumann = bool(self.free.min() > 0.5)
            keep = free[1:] if self._pure_neumann else free
            self._keep = keep
            self._S_lu = spla.splu(S[keep][:, keep].tocsc())
        return self._S_lu

    def riesz(self, rhat: np.ndarray) -> np.ndarray:
        """blockdiag(S^{-1}, M^{-1}) on the free nodes; with no sound-soft node, S^+ on
        zero-sum vectors (solve with the first node pinned, then remove the mean)."""
        lu = self._riesz_factor()
        ru = rhat[: self.nn]
        xu = np.zeros(self.nn)
        xu[self._keep] = lu.solve(ru[self._keep])
        if self._pure_neumann:
            xu -= xu.mean()
        xv = (self.free * rhat[self.nn:].reshape(self.shape) / self.M).ravel()
        return np.concatenate([xu, xv])

    def energy(self, u_next: np.ndarray, u: np.ndarray) -> float:
        """E^{n+1/2} = 1/2 delta^T M delta + 1/2 (u^{n+1})^T S u^n, delta = (u^{n+1}-u^n)/dt."""
        dl = (u_next - u) / self.dt
        return 0.5 * float(np.sum(dl * self.M * dl)) + 0.5 * float(np.sum(u_next * self.S(u)))

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
        return _cmcg.cmcg(lambda x: self.period(x, True), lambda x: self.period(x, False),
                          self.period_T, self.ME, self.riesz, self.size, tol, max_iter,
                          z0=z0, record=record, delta_ref=ref)

    def filter(self, z: np.ndarray) -> np.ndarray:
        """U = (2/N) sum_{n<N} u^n e^{i w t_n} over one forced period from z.  With several
        components, one such sum per component at its frequency m w over the same period,
        stacked (shape (components,) + node shape).  On a pure-Neumann box the sums are then
        shifted by the constant that the compatibility condition fixes (`compatible`)."""
        U = [np.zeros(self.shape, complex) for _ in self.comps]
        self.period(z, True, U_acc=U)
        U = [2.0 * Uc / self.N for Uc in U]
        if self.pure_neumann():
            U = [self.compatible(Uc, c) for c, Uc in enumerate(U)]
        return U[0] if len(U) == 1 else np.stack(U)

    def pure_neumann(self) -> bool:
        """No absorbing face and no sound-soft node."""
        return all(b != ABSORBING for b in self.bc) and bool(self.free.min() > 0.5)

    def compatible(self, V: np.ndarray, comp: int = 0) -> np.ndarray:
        """V - lam with the constant lam for which V - lam satisfies the compatibility condition
        of the time-discrete system, 1^T [S - wt^2 M - i wh B] U = 1^T Fhat (eq. CC for the
        absorbing case, eq. cc_neumann / eq. cc_neumann_eta for the pure-Neumann case; the
        stiffness drops out because S 1 = 0).  With the frequency m omega of component
        `comp`:  lam = (1^T Fhat + wt^2 1^T M V + i wh 1^T B V) / (wt^2 1^T M + i wh 1^T B).
        Only meaningful without sound-soft nodes (then the constant is a free mode)."""
        m, f, g, _ = self.comps[comp]
        w, dt = m * self.omega, self.dt
        wt2 = (2.0 / dt * math.sin(0.5 * w * dt)) ** 2
        wh = math.sin(w * dt) / dt
        Fh = self.w * f
        if g is not None:
            for idx, (sel, fw) in enumerate(self.face_w):
                Fh[sel] += fw * g[idx].reshape(fw.shape)
        lam = (Fh.sum() + wt2 * np.sum(self.M * V) + 1j * wh * np.sum(self.B * V)) / \
            (wt2 * self.M.sum() + 1j * wh * self.B.sum())
        return V - lam

    def step6_output(self, z: np.ndarray) -> np.ndarray:
        """The paper's Step 6 output u = v_0 + (i / omega) v_1."""
        return (z[: self.nn] + 1j * z[self.nn:] / self.omega).reshape(self.shape)

    def step6_discrete(self, z: np.ndarray) -> np.ndarray:
        """Step 6 read off the time-discrete periodic state (single component): the periodic
        state of a time-harmonic U is (Re U, wh Im U) with wh = sin(w dt) / dt, so
        v = u_0 + i v_1 / wh; the Dirichlet data on the sound-soft nodes.  Without sound-soft
        nodes a minimiser may carry a constant shift lam in u_0 (Thm 1), removed by the
        compatibility condition (eq. CC, `compatible`).  A pure-Neumann box also admits the
        mode eta, which this output cannot see: use the filter there."""
        assert len(self.comps) == 1, "Step 6 output of a single-frequency problem"
        if self.pure_neumann():
            raise ValueError("pure Neumann: the Step 6 output is undetermined (eta)")
        wh = math.sin(self.omega * self.dt) / self.dt
        R = self.free
        V = R * (z[: self.nn].reshape(self.shape) + 1j * z[self.nn:].reshape(self.shape) / wh)
        gD = self.comps[0][3]
        if gD is not None:
            V = V + gD
        if self.free.min() > 0.5:
            V = self.compatible(V)
        return V

    def functional(self, z):
        return _cmcg.functional(lambda x: self.period(x, True), self.ME, z)

    # ---------------------------------------------------------------- direct solve
    def direct(self):
        """Direct sparse solve of [S - wt^2 M - i wh B] U = Fhat on the free nodes with
        wt = (2/dt) sin(w dt / 2), wh = sin(w dt) / dt, Fhat = w f + sum over faces (face
        weight) g, and U = gD on the Dirichlet nodes.  Returns (U, z_periodic) with
        z = (Re U, wh Im U) on the free nodes.  With several components: one solve per
        component at its frequency m omega (same dt), U stacked per component and z the sum
        of the components' periodic states (the scheme is linear)."""
        dt = self.dt
        S = self.stiffness_matrix()
        free = np.flatnonzero(self.free.ravel() > 0.5)
        R = self.free.ravel()
        Us, z = [], np.zeros(self.size)
        for m, f, g, gD in self.comps:
            w = m * self.omega
            wt2 = (2.0 / dt * math.sin(0.5 * w * dt)) ** 2
            wh = math.sin(w * dt) / dt
            A = (S - wt2 * sp.diags(self.M.ravel()) - 1j * wh * sp.diags(self.B.ravel())).tocsr()
            Fh = self.w * f
            if g is not None:
                for idx, (sel, fw) in enumerate(self.face_w):
                    Fh[sel] += fw * g[idx].reshape(fw.shape)
            U = np.zeros(self.nn, complex)
            rhs = Fh.ravel()[free]
            if gD is not None:
                # Dirichlet values are known: move their couplings to the right-hand side
                dnodes = np.flatnonzero(self.free.ravel() < 0.5)
                gd = gD.ravel()[dnodes]
                rhs = rhs - A[free][:, dnodes] @ gd
                U[dnodes] = gd
            U[free] = spla.spsolve(A[free][:, free].tocsc(), rhs)
            z = z + np.concatenate([R * U.real, R * wh * U.imag])
            Us.append(U.reshape(self.shape))
        return (Us[0] if len(Us) == 1 else np.stack(Us)), z


def window(prob, lo, hi):
    """Sub-problem on the nodes lo[a] <= I_a <= hi[a] (axis a = x, y[, z]) of `prob`, for sampled
    checks of large grids: sides that lie on the original boundary keep its condition and data,
    cut sides become Neumann with zero data.  A period of N steps is N + 1 stencil sweeps (the
    start map and N recurrence steps), each coupling a node only to its axis neighbours, and only
    the nodes on a cut plane carry a changed stencil (half weights); so values at nodes more
    than N + 2 from every cut plane equal those of the full problem."""
    import copy
    d = prob.dim
    n = [int(m) for m in prob.n[:d]]
    lo, hi = [int(a) for a in lo[:d]], [int(a) for a in hi[:d]]
    shape = tuple(m + 1 for m in reversed(n))
    nodes = tuple(slice(lo[a], hi[a] + 1) for a in reversed(range(d)))   # numpy order

    def cut_field(x):
        return None if x is None else np.asarray(x).reshape(shape)[nodes].copy()

    keep = []
    for a in range(d):
        keep += [lo[a] == 0, hi[a] == n[a]]

    def cut_faces(g):
        if g is None:
            return None
        out = []
        for a in range(d):
            others = [b for b in range(d) if b != a]
            fshape = tuple(n[b] + 1 for b in reversed(others))
            sel = tuple(slice(lo[b], hi[b] + 1) for b in reversed(others))
            for side in range(2):
                arr = np.asarray(g[2 * a + side], dtype=complex).reshape(fshape)[sel]
                out.append(arr.copy() if keep[2 * a + side] else np.zeros_like(arr))
        return out

    sub = copy.copy(prob)
    sub.n = tuple(hi[a] - lo[a] for a in range(d))
    sub.spacing = prob.h
    if prob.c is not None:
        sub.c = cut_field(prob.c)
    sub.f = cut_field(prob.f)
    sub.gS = cut_faces(prob.gS)
    sub.sound_soft = cut_field(prob.sound_soft)
    sub.gD = cut_field(prob.gD)
    bc = list(prob.face_bc)[: 2 * d]
    sub.face_bc = tuple(bc[k] if keep[k] else 1 for k in range(2 * d)) + tuple(prob.face_bc)[2 * d:]
    if prob.shots:
        sub.shots = [copy.copy(s) for s in prob.shots]
        for s0, s in zip(prob.shots, sub.shots):
            s.f, s.gS, s.gD = cut_field(s0.f), cut_faces(s0.gS), cut_field(s0.gD)
    return sub
