"""Seeded synthetic inputs for the controllability (CMCG) Helmholtz solver.

This module only *describes problems*: grids, wave-speed fields, source
amplitudes, boundary data, obstacle masks and request arrival times.  It holds
none of the solver's arithmetic (no time stepping, no energy products, no CG),
so that the CPU oracle and the GPU path can both take their inputs from it
without sharing any of the method.

Layouts (shared vocabulary with the C ABI in ``include/cmcg.h``):

* First-order formulation (F1, 2D): cell-centred arrays of shape ``(ny, nx)``,
  x fastest; cell ``(j, i)`` has centre ``((i+1/2) h, (j+1/2) h)``.
* Second-order formulation (F2): node arrays of shape ``(nz+1, ny+1, nx+1)``
  (3D) or ``(ny+1, nx+1)`` (2D), node ``I`` at ``I h``.
* Boundary data ``gS``: one complex array per box face, in the order
  ``-x, +x, -y, +y[, -z, +z]``.  F1: one value per boundary cell face (length
  ``ny`` for the x faces, ``nx`` for the y faces).  F2: the nodes of that face
  in array order of the two remaining axes (slower axis first).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

ABSORBING = 0
NEUMANN = 1


@dataclasses.dataclass
class Shot:
    """One time-harmonic component of a multi-frequency ("super-shot") source: data f, gS/gN
    and gD as in `Problem`, oscillating at `harmonic` times the problem's base frequency."""

    harmonic: int
    f: Optional[np.ndarray] = None
    gS: Optional[List[np.ndarray]] = None
    gD: Optional[np.ndarray] = None


@dataclasses.dataclass
class Problem:
    """Helmholtz problem  -lap u - k^2 u = f,  du/dn - i k u = gS on absorbing faces,
    du/dn = gN on Neumann faces, u = gD on sound-soft nodes (eq. HE), posed on the box
    [0, n_x h] x [0, n_y h] (x [0, n_z h]) with h = 1 / n_x.  The per-face data `gS` holds gS on
    absorbing faces and gN on Neumann faces."""

    dim: int
    formulation: int                      # 1 = first-order staggered, 2 = second-order nodal
    n: Sequence[int]                      # cells per axis (x, y[, z])
    omega: float
    c: Optional[np.ndarray] = None        # wave speed on the F1 cells / F2 nodes; None -> c_const
    c_const: float = 1.0
    f: Optional[np.ndarray] = None        # complex source amplitude, same layout as c
    gS: Optional[List[np.ndarray]] = None  # complex boundary data per face (gS or gN)
    sound_soft: Optional[np.ndarray] = None  # uint8 mask, 1 = Dirichlet node (F2) or cell (F1)
    gD: Optional[np.ndarray] = None       # complex Dirichlet data u = gD there (layout of c), or 0
    face_bc: Sequence[int] = (ABSORBING,) * 6
    courant: float = 0.5
    name: str = ""
    spacing: Optional[float] = None       # grid spacing; None -> 1 / n_x (unit-width box)
    # multi-frequency source: the sum of these components, omega being their base frequency
    # (then f, gS and gD above stay None); None -> the single component (1, f, gS, gD)
    shots: Optional[List[Shot]] = None

    @property
    def h(self) -> float:
        return self.spacing if self.spacing is not None else 1.0 / self.n[0]

    def field_shape(self):
        if self.formulation == 1:
            return tuple(reversed(self.n[: self.dim]))
        return tuple(m + 1 for m in reversed(self.n[: self.dim]))

    def c_array(self) -> np.ndarray:
        if self.c is not None:
            return np.asarray(self.c, dtype=np.float64)
        return np.full(self.field_shape(), float(self.c_const))

    def c_max(self) -> float:
        return float(np.max(self.c)) if self.c is not None else float(self.c_const)


# --------------------------------------------------------------------------------------
# Random fields and sources
# --------------------------------------------------------------------------------------
def gaussian_random_field(shape, h: float, corr_len: float, seed: int,
                          lo: float = 1.0, hi: float = 2.0) -> np.ndarray:
    """Stationary Gaussian field with covariance exp(-r^2 / (2 l^2)), made by filtering
    PCG64 white noise in Fourier space with the square root of that covariance's
    spectral density, exp(-|k|^2 l^2 / 4), then mapped affinely so min -> lo, max -> hi."""
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.standard_normal(shape)
    k2 = np.zeros(shape)
    for ax, m in enumerate(shape):
        kk = 2.0 * np.pi * np.fft.fftfreq(m, d=h)
        sh = [1] * len(shape)
        sh[ax] = m
        k2 = k2 + (kk ** 2).reshape(sh)
    field = np.fft.ifftn(np.fft.fftn(noise) * np.exp(-k2 * corr_len ** 2 / 4.0)).real
    del k2, noise
    fmin, fmax = field.min(), field.max()
    return lo + (hi - lo) * (field - fmin) / (fmax - fmin)


def cell_centres_2d(nx: int, ny: int, h: float):
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    return np.meshgrid(x, y, indexing="xy")       # each (ny, nx)


def gaussian_bumps_2d(nx, ny, h, centres, width) -> np.ndarray:
    """Sum of exp(-|x - x_k|^2 / w^2) at cell centres, evaluated per bump on the box
    where it exceeds 1e-300 relative (outside that box it underflows to 0 anyway)."""
    out = np.zeros((ny, nx))
    xs = (np.arange(nx) + 0.5) * h
    ys = (np.arange(ny) + 0.5) * h
    rad = width * math.sqrt(700.0)
    for (cx, cy) in centres:
        i0, i1 = np.searchsorted(xs, [cx - rad, cx + rad])
        j0, j1 = np.searchsorted(ys, [cy - rad, cy + rad])
        X, Y = np.meshgrid(xs[i0:i1], ys[j0:j1], indexing="xy")
        out[j0:j1, i0:i1] += np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / width ** 2)
    return out


# --------------------------------------------------------------------------------------
# The five workloads (and small variants of them for tests)
# --------------------------------------------------------------------------------------
def single_source_2d(n: int = 128, omega: float = 8 * math.pi, width: float = 0.05,
                     c: float = 1.0) -> Problem:
    """2D unit square, n x n cells, first-order system, constant c, one Gaussian source
    exp(-|x-(1/2,1/2)|^2/w^2) at the centre, absorbing on all four sides, sigma = 0.5.
    With n = 128, omega = 8 pi, w = 0.05 this is the 128^2 four-wavelength case."""
    h = 1.0 / n
    f = gaussian_bumps_2d(n, n, h, [(0.5, 0.5)], width).astype(np.complex128)
    return Problem(dim=2, formulation=1, n=(n, n), omega=omega, c=None, c_const=c, f=f,
                   face_bc=(ABSORBING,) * 4, courant=0.5, name=f"f1_single_{n}")


def random_medium_2d(n: int = 4096, freq: float = 100.0, n_src: int = 8, seed: int = 1234,
                     width: Optional[float] = None, corr_len: float = 0.05) -> Problem:
    """2D unit square, n x n cells, first-order system, c a seeded Gaussian random field
    (correlation length 0.05) mapped to [1, 2], omega = 2 pi freq, n_src Gaussian sources at
    seeded positions in [0.1, 0.9]^2, absorbing on all sides.  The source width defaults
    to a quarter of the shortest wavelength (1 / (4 freq) at c_min = 1)."""
    h = 1.0 / n
    c = gaussian_random_field((n, n), h, corr_len, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    centres = rng.uniform(0.1, 0.9, size=(n_src, 2))
    w = width if width is not None else 1.0 / (4.0 * freq)
    f = gaussian_bumps_2d(n, n, h, [tuple(p) for p in centres], w).astype(np.complex128)
    return Problem(dim=2, formulation=1, n=(n, n), omega=2 * math.pi * freq, c=c, f=f,
                   face_bc=(ABSORBING,) * 4, courant=0.5, name=f"f1_random_{n}")


def supershot_2d(n: int = 256, base_freq: float = 4.0, harmonics=(1, 2, 3), seed: int = 99,
                 corr_len: float = 0.05, c=None) -> Problem:
    """Multi-frequency source on the first-order 2D random medium: c a seeded Gaussian random
    field in [1, 2] (or the given array), base frequency omega = 2 pi base_freq, and for each
    harmonic m one Gaussian source of width 1 / (4 m base_freq) at a seeded position in
    [0.2, 0.8]^2 with a seeded complex amplitude of modulus 1, absorbing on all sides.  The
    period T = 1 / base_freq is common to all components."""
    h = 1.0 / n
    if c is None:
        c = gaussian_random_field((n, n), h, corr_len, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    shots = []
    for m in harmonics:
        pos = rng.uniform(0.2, 0.8, size=2)
        phase = np.exp(2j * math.pi * rng.uniform())
        f = phase * gaussian_bumps_2d(n, n, h, [tuple(pos)], 1.0 / (4.0 * m * base_freq))
        shots.append(Shot(int(m), f=f.astype(np.complex128)))
    return Problem(dim=2, formulation=1, n=(n, n), omega=2 * math.pi * base_freq, c=c,
                   face_bc=(ABSORBING,) * 4, courant=0.5, shots=shots,
                   name=f"f1_supershot_{n}_{'_'.join(str(m) for m in harmonics)}")


def plane_wave_face_data_f1(nx: int, ny: int, h: float, k: float, direction) -> List[np.ndarray]:
    """First-order boundary data gS = (d/dn - i k) u_in for the incident wave u_in = exp(i k
    d.x), i.e. i k (d.n - 1) u_in at the boundary-face midpoints (faces -x, +x, -y, +y)."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    yc = (np.arange(ny) + 0.5) * h
    xc = (np.arange(nx) + 0.5) * h
    L, H = nx * h, ny * h
    out = []
    for normal, (x, y) in (((-1, 0), (np.zeros(ny), yc)), ((1, 0), (np.full(ny, L), yc)),
                           ((0, -1), (xc, np.zeros(nx))), ((0, 1), (xc, np.full(nx, H)))):
        uin = np.exp(1j * k * (d[0] * x + d[1] * y))
        out.append(1j * k * (d[0] * normal[0] + d[1] * normal[1] - 1.0) * uin)
    return out


def sound_soft_square_2d(n: int = 256, freq: float = 10.0, side: float = 0.2,
                         direction=(-1.0, 1.0), cavity: bool = False,
                         wall: Optional[float] = None, aperture: float = 0.06) -> Problem:
    """2D unit square, n x n cells, first-order system, c = 1, total-field scattering of the
    plane wave exp(i k d.x) (k = 2 pi freq; the default direction is the angle 135 degrees) by
    a sound-soft obstacle at the centre: the cells whose centres lie in a square of the given
    side (convex), or, if `cavity`, in the walls of a square shell (wall thickness
    max(2h, side / 10)) open by `aperture` in the middle of its -x wall (nonconvex).  Dirichlet
    data 0 (total field), absorbing outer faces carry gS = (d/dn - i k) u_in."""
    h = 1.0 / n
    k = 2 * math.pi * freq
    xc = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    lo, hi = 0.5 - side / 2, 0.5 + side / 2
    inside = (X >= lo) & (X <= hi) & (Y >= lo) & (Y <= hi)
    if cavity:
        w = wall if wall is not None else max(2 * h, side / 10)
        hollow = (X > lo + w) & (X < hi - w) & (Y > lo + w) & (Y < hi - w)
        opening = (X < lo + w) & (np.abs(Y - 0.5) < aperture / 2)
        inside = inside & ~hollow & ~opening
    mask = inside.astype(np.uint8)
    gS = plane_wave_face_data_f1(n, n, h, k, direction)
    return Problem(dim=2, formulation=1, n=(n, n), omega=k, c=None, c_const=1.0, f=None, gS=gS,
                   sound_soft=mask, face_bc=(ABSORBING,) * 4, courant=0.5,
                   name=f"f1_sound_soft_{'cavity' if cavity else 'square'}_{n}")


def channel_plane_wave_f1(nx: int, ny: int, k: float) -> Problem:
    """Channel version of the paper's 1D test u = exp(i k x): c = 1, omega = k, f = 0,
    absorbing at x = 0 with data gS = -2 i k, absorbing at x = 1 with gS = 0, Neumann
    walls at y = 0 and y = ny h, so the exact Helmholtz solution is exp(i k x)."""
    gS = [np.full(ny, -2j * k), np.zeros(ny, complex), np.zeros(nx, complex),
          np.zeros(nx, complex)]
    return Problem(dim=2, formulation=1, n=(nx, ny), omega=k, c=None, c_const=1.0, f=None,
                   gS=gS, face_bc=(ABSORBING, ABSORBING, NEUMANN, NEUMANN), courant=0.5,
                   name=f"f1_channel_{nx}x{ny}")


def node_coords(n: Sequence[int], h: float):
    """Node coordinate grids for the F2 layout (slowest axis first)."""
    axes = [np.arange(m + 1) * h for m in reversed(n)]
    grids = np.meshgrid(*axes, indexing="ij")
    return list(reversed(grids))                  # x, y[, z], each of field shape


def inclusions_3d(n: int = 512, freq: float = 25.0, n_incl: int = 64, seed: int = 2024,
                  width: float = 0.01, r_range=(0.02, 0.08), c_range=(1.5, 3.0)) -> Problem:
    """3D unit cube, n^3 cells, second-order nodal system, c = 1 with n_incl seeded spheres
    (centres uniform in the cube, radii and speeds uniform in the given ranges; where spheres
    overlap the larger speed wins), a point-like Gaussian source of width w at the centre,
    absorbing on all six faces."""
    h = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(0.0, 1.0, size=(n_incl, 3))
    radii = rng.uniform(r_range[0], r_range[1], size=n_incl)
    speeds = rng.uniform(c_range[0], c_range[1], size=n_incl)
    c = np.ones((n + 1,) * 3, dtype=np.float64)
    ax = np.arange(n + 1) * h
    for (cx, cy, cz), r, cs in zip(centres, radii, speeds):
        lo = [max(0, int(math.floor((q - r) / h))) for q in (cx, cy, cz)]
        hi = [min(n, int(math.ceil((q + r) / h))) for q in (cx, cy, cz)]
        Z, Y, X = np.meshgrid(ax[lo[2]:hi[2] + 1], ax[lo[1]:hi[1] + 1], ax[lo[0]:hi[0] + 1],
                              indexing="ij")
        inside = (X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2 <= r * r
        sub = c[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
        sub[inside] = np.maximum(sub[inside], cs)
    f = np.zeros((n + 1,) * 3, dtype=np.complex128)
    rad = width * math.sqrt(700.0)
    lo = max(0, int(math.floor((0.5 - rad) / h)))
    hi = min(n, int(math.ceil((0.5 + rad) / h)))
    Z, Y, X = np.meshgrid(ax[lo:hi + 1], ax[lo:hi + 1], ax[lo:hi + 1], indexing="ij")
    f[lo:hi + 1, lo:hi + 1, lo:hi + 1] = np.exp(
        -((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2) / width ** 2)
    return Problem(dim=3, formulation=2, n=(n, n, n), omega=2 * math.pi * freq, c=c, f=f,
                   face_bc=(ABSORBING,) * 6, courant=0.5, name=f"f2_inclusions_{n}")


def plane_wave_face_data(n: Sequence[int], h: float, k: float, direction) -> List[np.ndarray]:
    """gS = (d/dn - i k) u_in on each box face for the incident wave u_in = exp(i k d.x),
    i.e. i k (d.n - 1) u_in at the face nodes (F2 node layout per face)."""
    dim = len(n)
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    out = []
    for axis in range(dim):
        for side in (0, 1):
            normal = np.zeros(dim)
            normal[axis] = -1.0 if side == 0 else 1.0
            others = [a for a in range(dim) if a != axis]
            coords = [np.arange(n[a] + 1) * h for a in others]
            grids = np.meshgrid(*reversed(coords), indexing="ij")   # slower axis first
            grids = list(reversed(grids))                          # in order of `others`
            phase = d[axis] * (0.0 if side == 0 else n[axis] * h)
            for a, g in zip(others, grids):
                phase = phase + d[a] * g
            uin = np.exp(1j * k * phase) * np.ones(grids[0].shape if grids else ())
            out.append(1j * k * (float(d @ normal) - 1.0) * uin)
    return out


def sphere_mask(n: Sequence[int], h: float, centre, radius) -> np.ndarray:
    """uint8 node mask of the voxelised ball |x - centre| <= radius."""
    coords = node_coords(n, h)
    r2 = sum((g - q) ** 2 for g, q in zip(coords, centre))
    return (r2 <= radius * radius).astype(np.uint8)


def sound_soft_sphere_3d(n: int = 1024, freq: float = 100.0, radius: float = 0.15,
                         direction=(1.0, 1.0, 1.0)) -> Problem:
    """3D unit cube, n^3 cells, second-order nodal system, c = 1, total-field scattering of
    the plane wave exp(i k d.x), d = direction / |direction|, by a sound-soft ball of the
    given radius at the centre (homogeneous Dirichlet on its voxelised nodes); absorbing
    outer faces carry gS = (d/dn - i k) u_in."""
    h = 1.0 / n
    k = 2 * math.pi * freq
    gS = plane_wave_face_data((n, n, n), h, k, direction)
    mask = sphere_mask((n, n, n), h, (0.5, 0.5, 0.5), radius)
    return Problem(dim=3, formulation=2, n=(n, n, n), omega=k, c=None, c_const=1.0, f=None,
                   gS=gS, sound_soft=mask, face_bc=(ABSORBING,) * 6, courant=0.5,
                   name=f"f2_sphere_{n}")


def supershot_sphere_3d(n: int = 128, base_freq: float = 2.0, harmonics=(1, 2, 3),
                        radius: float = 0.15, seed: int = 5) -> Problem:
    """Multi-frequency scattering by the sound-soft ball of `sound_soft_sphere_3d`: base
    frequency omega = 2 pi base_freq, and for each harmonic m an incident plane wave
    exp(i m omega d_m.x) with a seeded direction d_m, entering through the absorbing faces as
    gS = (d/dn - i k_m) u_in (c = 1)."""
    h = 1.0 / n
    k0 = 2 * math.pi * base_freq
    rng = np.random.Generator(np.random.PCG64(seed))
    shots = []
    for m in harmonics:
        d = rng.standard_normal(3)
        shots.append(Shot(int(m), gS=plane_wave_face_data((n, n, n), h, m * k0, tuple(d))))
    mask = sphere_mask((n, n, n), h, (0.5, 0.5, 0.5), radius)
    return Problem(dim=3, formulation=2, n=(n, n, n), omega=k0, c=None, c_const=1.0,
                   sound_soft=mask, face_bc=(ABSORBING,) * 6, courant=0.5, shots=shots,
                   name=f"f2_supershot_sphere_{n}")


def cavity_mask(n: Sequence[int], h: float, lo: float = 0.3, hi: float = 0.7,
                wall: Optional[float] = None, aperture: Optional[float] = 0.08) -> np.ndarray:
    """uint8 node mask of a box-shaped shell [lo, hi]^3 of wall thickness `wall` (default two
    cells or 0.02, whichever is larger) with a square opening of half-width `aperture` in the
    middle of its +x face (None: the whole face open): a nonconvex obstacle whose interior
    traps waves."""
    wall = max(2.0 * h, 0.02) if wall is None else wall
    x, y, z = node_coords(n, h)
    inside_outer = (x >= lo) & (x <= hi) & (y >= lo) & (y <= hi) & (z >= lo) & (z <= hi)
    inside_inner = ((x > lo + wall) & (x < hi - wall) & (y > lo + wall) & (y < hi - wall)
                    & (z > lo + wall) & (z < hi - wall))
    mid = 0.5 * (lo + hi)
    a = (hi - lo) if aperture is None else aperture
    opening = (x >= hi - wall) & (np.abs(y - mid) < a) & (np.abs(z - mid) < a)
    return (inside_outer & ~inside_inner & ~opening).astype(np.uint8)


def sound_soft_cavity_3d(n: int = 128, freq: float = 6.0, direction=(-1.0, -1.0, -1.0)) -> Problem:
    """3D unit cube, n^3 cells, second-order nodal system, c = 1, total-field scattering of the
    plane wave exp(i k d.x), d = direction / |direction| (arriving from the open side), by a
    sound-soft box-shaped cavity [0.3, 0.7]^3 with a square opening (half-width 0.08) in its +x
    face; absorbing outer faces carry gS = (d/dn - i k) u_in.  Stands in for the nonconvex
    cavity of the paper's scattering tests.""" 
    h = 1.0 / n
    k = 2 * math.pi * freq
    gS = plane_wave_face_data((n, n, n), h, k, direction)
    mask = cavity_mask((n, n, n), h)
    return Problem(dim=3, formulation=2, n=(n, n, n), omega=k, c=None, c_const=1.0, f=None,
                   gS=gS, sound_soft=mask, face_bc=(ABSORBING,) * 6, courant=0.5,
                   name=f"f2_cavity_{n}")


def channel_plane_wave_f2(n: Sequence[int], k: float, dirichlet_at_zero: bool = False) -> Problem:
    """Channel versions of the paper's 1D closed forms on the F2 nodal grid (c = 1, f = 0,
    lateral faces Neumann so the solution does not vary across the channel):
    * dirichlet_at_zero False: u = exp(i k x), absorbing at x = 0 with gS = -2 i k and at
      x = L with gS = 0;
    * dirichlet_at_zero True: u = 2 i sin(k x), sound-soft nodes on the plane x = 0 and
      absorbing at x = L with gS = 2 i k exp(-i k L)... precisely (d/dn - i k) u at x = L,
      which is 2 i k cos(k L) + 2 k sin(k L) = 2 i k exp(-i k L)."""
    dim = len(n)
    h = 1.0 / n[0]
    L = n[0] * h
    shp = tuple(m + 1 for m in reversed(n))
    face_shapes = []
    for axis in range(dim):
        others = [a for a in range(dim) if a != axis]
        face_shapes.append(tuple(n[a] + 1 for a in reversed(others)))
    gS = []
    for axis in range(dim):
        for side in (0, 1):
            gS.append(np.zeros(face_shapes[axis], dtype=np.complex128))
    bc = [NEUMANN] * (2 * dim)
    bc[1] = ABSORBING
    mask = None
    if dirichlet_at_zero:
        gS[1][...] = 2j * k * np.exp(-1j * k * L)
        mask = np.zeros(shp, dtype=np.uint8)
        mask[..., 0] = 1
    else:
        bc[0] = ABSORBING
        gS[0][...] = -2j * k
    return Problem(dim=dim, formulation=2, n=tuple(n), omega=k, c=None, c_const=1.0, f=None,
                   gS=gS, sound_soft=mask, face_bc=tuple(bc), courant=0.5,
                   name="f2_channel" + ("_dirichlet" if dirichlet_at_zero else ""))


def channel_dirichlet_f2(n: Sequence[int], k: float, u0: complex) -> Problem:
    """Channel with Dirichlet data: the nodes of the plane x = 0 are Dirichlet nodes with
    u = u0, the face x = L is absorbing with no data, the lateral faces are Neumann; c = 1,
    omega = k, f = 0.  The exact Helmholtz solution is u0 exp(i k x)."""
    dim = len(n)
    shp = tuple(m + 1 for m in reversed(n))
    face_shapes = []
    for axis in range(dim):
        others = [a for a in range(dim) if a != axis]
        face_shapes.append(tuple(n[a] + 1 for a in reversed(others)))
    gS = [np.zeros(face_shapes[a // 2], dtype=np.complex128) for a in range(2 * dim)]
    bc = [NEUMANN] * (2 * dim)
    bc[1] = ABSORBING
    mask = np.zeros(shp, dtype=np.uint8)
    mask[..., 0] = 1
    gD = np.zeros(shp, dtype=np.complex128)
    gD[..., 0] = u0
    return Problem(dim=dim, formulation=2, n=tuple(n), omega=k, c=None, c_const=1.0, f=None,
                   gS=gS, sound_soft=mask, gD=gD, face_bc=tuple(bc), courant=0.5,
                   name="f2_channel_dirichlet_data")


def channel_neumann_data(formulation: int, n: Sequence[int], k: float) -> Problem:
    """Channel with Neumann data: u = exp(i k x) has outward derivative -u'(0) = -i k on the
    face x = 0, which is a Neumann face carrying gN = -i k; the face x = L is absorbing with no
    data, the lateral faces are Neumann with no data; c = 1, omega = k, f = 0."""
    dim = len(n)
    if formulation == 1:
        nx, ny = n
        g = [np.full(ny, -1j * k), np.zeros(ny, complex), np.zeros(nx, complex),
             np.zeros(nx, complex)]
    else:
        g = []
        for axis in range(dim):
            others = [a for a in range(dim) if a != axis]
            fshape = tuple(n[a] + 1 for a in reversed(others))
            g += [np.zeros(fshape, dtype=np.complex128), np.zeros(fshape, dtype=np.complex128)]
        g[0][...] = -1j * k
    bc = [NEUMANN] * (2 * dim)
    bc[1] = ABSORBING
    return Problem(dim=dim, formulation=formulation, n=tuple(n), omega=k, c=None, c_const=1.0,
                   f=None, gS=g, face_bc=tuple(bc), courant=0.5,
                   name=f"f{formulation}_channel_neumann_data")


def channel_bounded_neumann_f2(n: Sequence[int], k: float) -> Problem:
    """Channel version of the bounded-domain example u(x) = 16 x^2 (x - 1)^2 on the F2 nodal
    grid: c = 1, omega = k, every face Neumann (no absorption, no sound-soft nodes), real source
    f = -u'' - k^2 u = -16 (12 x^2 - 12 x + 2) - 16 k^2 x^2 (x - 1)^2 sampled at the nodes."""
    dim = len(n)
    h = 1.0 / n[0]
    shp = tuple(m + 1 for m in reversed(n))
    x = np.broadcast_to(np.arange(n[0] + 1) * h, shp)
    f = -16.0 * (12 * x * x - 12 * x + 2) - 16.0 * k * k * x * x * (x - 1) ** 2
    return Problem(dim=dim, formulation=2, n=tuple(n), omega=k, c=None, c_const=1.0,
                   f=f.astype(np.complex128), gS=None, sound_soft=None,
                   face_bc=(NEUMANN,) * (2 * dim), courant=0.5, name="f2_bounded_neumann")


@dataclasses.dataclass
class Request:
    arrival_s: float
    problem: Problem
    seed: int


def serving_requests(count: int = 256, rate_hz: float = 20.0, seed: int = 77,
                     sides=(256, 512, 1024, 2048), wavelengths=(4.0, 64.0),
                     build_fields: bool = True) -> List[Request]:
    """Seeded serving workload: Poisson arrivals at rate_hz, each a 2D first-order solve on
    an n x n grid with n uniform over `sides`, W wavelengths (at c = 1) log-uniform over
    `wavelengths`, omega = 2 pi W, a Gaussian random field c in [1, 2] and one Gaussian
    source of width 1 / (4 W) at a seeded position in [0.3, 0.7]^2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(count):
        n = int(sides[rng.integers(len(sides))])
        W = float(math.exp(rng.uniform(math.log(wavelengths[0]), math.log(wavelengths[1]))))
        pos = rng.uniform(0.3, 0.7, size=2)
        s = int(rng.integers(1 << 30))
        if build_fields:
            prob = request_problem(n, W, pos, s)
        else:
            prob = Problem(dim=2, formulation=1, n=(n, n), omega=2 * math.pi * W,
                           name=f"req{r}")
        out.append(Request(float(arrivals[r]), prob, s))
    return out


def request_problem(n: int, W: float, pos, seed: int) -> Problem:
    h = 1.0 / n
    c = gaussian_random_field((n, n), h, 0.05, seed)
    f = gaussian_bumps_2d(n, n, h, [tuple(pos)], 1.0 / (4.0 * W)).astype(np.complex128)
    return Problem(dim=2, formulation=1, n=(n, n), omega=2 * math.pi * W, c=c, f=f,
                   face_bc=(ABSORBING,) * 4, courant=0.5, name=f"req_{n}_{W:.2f}")


def random_state(shape_list, seed: int) -> List[np.ndarray]:
    """Seeded standard-normal arrays of the given shapes (test vectors for period and
    adjoint checks)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.standard_normal(s) for s in shape_list]
