// Second-order (nodal, 3D) leapfrog on gfx950: start map, steps and end map of one period, the
// literal transpose of each (the backward period), the energy metric, and the CG vector kernels.
//
// Scheme (Sec. 2, eq. WE; mass-lumped nodal discretisation of a structured box, leapfrog with an
// integer number of steps per period).  Nodes I in {0..n}^3, eta_I = prod over axes of (1/2 if I
// is on that axis' boundary), lumped mass M = h^3 eta / c^2, stiffness S = diag(h eta) L where L
// is the 7-point operator 6 u_I - sum of the six neighbours with mirrored neighbours across the
// box faces (u_{-1} = u_1, u_{n+1} = u_{n-1}).  Hence
//     dt^2 M^{-1} S u = lambda L u,          dt^2 S M^{-1} s = eta L(lambda s / eta),
// lambda = (c dt / h)^2.  Absorbing faces add beta = sqrt(lambda) m (m = number of absorbing faces
// at the node), the load enters as F = dt^2 c^2 Re(G e^{-i w t}), G = f + (2/h) sum_abs gS, and
// sound-soft nodes are held at zero (R = 1 - mask).
// Forced periods of a problem with Dirichlet data hold the sound-soft nodes at Re(gD e^{-iwt})
// (the start map reads the data at its input time on those nodes, every forced sweep writes it
// at its output time there); the period's output state stays zero on them.
//   start:  u^1 = R(u^0 + dt (1-beta) v^0 - (lambda L u^0 - F^0)/2)
//   step:   u^{n+1} = R(2 u^n - (1-beta) u^{n-1} - lambda L u^n + F^n) / (1+beta)
//   end:    v^N = (u^{N+1} - u^{N-1}) / (2 dt),  Phi(u^0, v^0) = (u^N, v^N)
// The transposed period runs the same three-level recurrence backward on a = adjoint state:
//   a_{m+1} = K^T a_m + Lb a_{m-1},  K^T a = R(2 s - eta L(lambda s / eta)),  s = R a / (1+beta),
//   Lb = -(1-beta)/(1+beta)
// with the transposed end map as its start and the transposed start map as its end.
//
// The backward period is run in the scaled variable g = psi a, psi = lambda R / ((1+beta) eta).
// Because eta L = S / h is symmetric, psi K^T a = K g, and the recurrence becomes
//   g_{m+1} = K g_m + Lb g_{m-1},   K g = R (2 g - lambda L g) / (1 + beta),
// the forward homogeneous step itself; the transposed end map enters g (g_y = psi y_v stencilled
// plainly) and the transposed start map leaves it (a = (1 + beta) eta g / lambda, stencilling
// (1 + beta) g = lambda R a / eta).  Only the first and last sweeps carry per-node transforms.
//
// Kernel design: one thread per (i, j) column marches through a run of planes k, keeping the
// planes k-1, k, k+1 of the stencilled field in registers.  The x neighbours come from the
// adjacent lanes through DPP shifts (the two end lanes of a wavefront load theirs), the y
// neighbours from the rows that the neighbouring wavefronts load anyway (L1/L2 hits), so HBM sees
// each field once per sweep.  Interior nodes (no absorbing face, beta = 0) take a division-free
// update.
#include <algorithm>
#include <cstdlib>

#include "f2_internal.h"
#include "dpp.h"

namespace cmcg {
namespace {

__device__ __forceinline__ int mirror(int i, int n) { return i < 0 ? 1 : (i > n ? n - 1 : i); }

__device__ __forceinline__ double eta_of(const F2Geom &g, int i, int j, int k) {
  double e = 1.0;
  if (i == 0 || i == g.nx) e *= 0.5;
  if (j == 0 || j == g.ny) e *= 0.5;
  if (k == 0 || k == g.nz) e *= 0.5;
  return e;
}

__device__ __forceinline__ int abs_faces(const F2Geom &g, int i, int j, int k) {
  return (i == 0 ? g.abs_face[0] : 0) + (i == g.nx ? g.abs_face[1] : 0) +
         (j == 0 ? g.abs_face[2] : 0) + (j == g.ny ? g.abs_face[3] : 0) +
         (k == 0 ? g.abs_face[4] : 0) + (k == g.nz ? g.abs_face[5] : 0);
}

__device__ __forceinline__ bool masked(const F2Geom &g, int i, int j, int k) {
  if (!g.mask) return false;
  if (i < g.mlo[0] || i > g.mhi[0] || j < g.mlo[1] || j > g.mhi[1] || k < g.mlo[2] || k > g.mhi[2])
    return false;
  return g.mask[g.idx(i, j, k)] != 0;
}

template <typename T>
__device__ __forceinline__ T lam_at(const F2Geom &g, const T *lam, size_t o) {
  return lam ? lam[o] : (T)g.lam_const;
}

// The absorbing-face coefficient beta = m sqrt(lambda) and a step's division by 1 + beta.  FP64
// takes the correctly rounded square root and quotient; FP32 (the FP32-mixed stencils) the
// hardware's approximations (v_sqrt_f32, v_rcp_f32, about one ulp each), a few instructions
// where the correctly rounded forms take about 25 on every wavefront that holds a face node.
// Every kernel that takes a leapfrog step uses these, so blocked and single-step launches
// still agree bit for bit.
__device__ __forceinline__ float face_beta(int m, float l) {
  return (float)m * __builtin_amdgcn_sqrtf(l);
}
__device__ __forceinline__ double face_beta(int m, double l) { return (double)m * sqrt(l); }
__device__ __forceinline__ float face_div(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}
__device__ __forceinline__ double face_div(double a, double b) { return a / b; }

// Dirichlet data value at device index o (dc, ds: cos/sin weights of the time)
template <typename T>
__device__ __forceinline__ T dirichlet_at(const F2Args<T> &p, size_t o, double dc, double ds) {
  double v = p.dre[o] * dc;
  if (p.dim) v = fma(p.dim[o], ds, v);
  return (T)v;
}

// value of the stencilled field at a node, per sweep, from the stored value a there
template <typename T, int MODE>
__device__ __forceinline__ T sfix(const F2Geom &g, const T *lam, int i, int j, int k, T a) {
  if (MODE == kF2Metric) return masked(g, i, j, k) ? T(0) : a;
  if (MODE == kF2AdjEnd) {
    // (1 + beta) g  (g vanishes on sound-soft nodes)
    const int m = abs_faces(g, i, j, k);
    if (m == 0) return a;
    return (T(1) + face_beta(m, lam_at(g, lam, g.idx(i, j, k)))) * a;
  }
  return a;
}
template <typename T, int MODE>
__device__ __forceinline__ T sval(const F2Geom &g, const T *f, const T *lam, int i, int j, int k) {
  return sfix<T, MODE>(g, lam, i, j, k, f[g.idx(i, j, k)]);
}

// Output of one node of one sweep, given the stencilled centre value zc, the 7-point operator
// lap of the stencilled field, the node's second input aux, lambda and the source value F.
template <typename T, int MODE>
__device__ __forceinline__ void node_update(const F2Geom &g, const F2Args<T> &p, size_t o, int i,
                                            int j, int k, T zc, T lap, T aux, T l, T F) {
  const T dt = (T)g.dt;
  const bool R = !masked(g, i, j, k);
  const int m = abs_faces(g, i, j, k);
  const T beta = m ? face_beta(m, l) : T(0);
  if (MODE == kF2FwdStart) {
    // u^1 = R(u^0 + dt (1-beta) v^0 - (lambda L u^0 - F^0) / 2)
    if (p.ure) {
      p.ure[o] += (double)zc * p.wcos;
      p.uim[o] += (double)zc * p.wsin;
    }
    const T hold = p.dre ? dirichlet_at(p, o, p.dcos1, p.dsin1) : T(0);
    p.out[o] = R ? zc + dt * (T(1) - beta) * aux - T(0.5) * (l * lap - F) : hold;
  } else if (MODE == kF2FwdStep) {
    if (p.ure) {
      p.ure[o] += (double)zc * p.wcos;
      p.uim[o] += (double)zc * p.wsin;
    }
    T un;
    if (m == 0) un = fma(-l, lap, T(2) * zc - aux) + F;
    else un = face_div(T(2) * zc - (T(1) - beta) * aux - (l * lap - F), T(1) + beta);
    const T hold = (!R && p.dre) ? dirichlet_at(p, o, p.dcos1, p.dsin1) : T(0);
    p.out[o] = R ? un : hold;
  } else if (MODE == kF2FwdEnd) {
    // out = (u^N, (u^{N+1} - u^{N-1}) / (2 dt)) - sub
    T up;
    if (m == 0) up = fma(-l, lap, T(2) * zc - aux) + F;
    else up = face_div(T(2) * zc - (T(1) - beta) * aux - (l * lap - F), T(1) + beta);
    T ou = zc, ov = (up - aux) / (T(2) * dt);
    if (p.sub) {
      ou -= p.sub[o];
      ov -= p.sub[o + g.fs];
    }
    p.out[o] = R ? ou : T(0);                // the state is zero on Dirichlet nodes
    p.out[o + g.fs] = R ? ov : T(0);
  } else if (MODE == kF2Metric) {
    // y = M_E w = (S w_u, M w_v) on the free nodes
    const T eta = (T)eta_of(g, i, j, k);
    const T h = (T)g.h;
    const T c2 = l * (T)(g.h * g.h / (g.dt * g.dt));
    p.out[o] = R ? h * eta * lap : T(0);
    p.out[o + g.fs] = (R && c2 > T(0)) ? h * h * h * eta / c2 * aux : T(0);
  } else if (MODE == kF2AdjInit) {
    // st = g_y = psi y_v, aux = y_u:  g_0 = psi y_u + K g_y / (2 dt),
    //                                 psi b_0 = (Lb - 1) g_y / (2 dt) = -g_y / ((1+beta) dt)
    const T eta = (T)eta_of(g, i, j, k);
    const T psi = R ? l / ((T(1) + beta) * eta) : T(0);
    const T Kg = R ? face_div(T(2) * zc - l * lap, T(1) + beta) : T(0);
    p.out[o] = psi * aux + Kg / (T(2) * dt);
    p.out2[o] = R ? -zc / ((T(1) + beta) * dt) : T(0);
  } else if (MODE == kF2AdjStepFirst) {
    // g_1 = K g_0 + psi b_0
    T gn;
    if (m == 0) gn = fma(-l, lap, T(2) * zc);
    else gn = face_div(T(2) * zc - l * lap, T(1) + beta);
    p.out[o] = R ? gn + aux : T(0);
  } else if (MODE == kF2AdjEnd) {
    // st = g_M (stencilled as (1+beta) g), aux = g_{M-1}; a = (1+beta) eta g / lambda:
    //   u_0 = R(a - eta L((1+beta) g) / 2) + Lb a_{M-1},  Lb a_{M-1} = -(1-beta) eta g_{M-1} / lambda
    //   v_0 = R dt (1-beta) a
    const T eta = (T)eta_of(g, i, j, k);
    const T a = eta * zc / l;
    T ou = R ? a - T(0.5) * eta * lap - (T(1) - beta) * eta * aux / l : T(0);
    T ov = R ? dt * (T(1) - beta) * a : T(0);
    if (p.sub) {
      ou -= p.sub[o];
      ov -= p.sub[o + g.fs];
    }
    p.out[o] = ou;
    p.out[o + g.fs] = ov;
  }
}

// The loads one plane's update needs (raw values of the plainly stencilled sweeps).
template <typename T>
struct PlaneLoads {
  T zp, xe, ym, yp, aux, lam, fr, fi;
};

template <typename T, int MODE>
__device__ __forceinline__ void plane_loads(const F2Geom &g, const F2Args<T> &p, int ic, int xend,
                                            int j, int jm, int jp, int k, PlaneLoads<T> &q) {
  q.zp = p.st[g.idx(ic, j, mirror(k + 1, g.nz))];
  q.xe = p.st[g.idx(xend, j, k)];
  q.ym = p.st[g.idx(ic, jm, k)];
  q.yp = p.st[g.idx(ic, jp, k)];
  const size_t o = g.idx(ic, j, k);
  q.aux = p.aux[o];
  q.lam = lam_at(g, p.lam, o);
  q.fr = q.fi = T(0);
  if (MODE == kF2FwdStart || MODE == kF2FwdStep || MODE == kF2FwdEnd) {
    if (p.forced) {
      q.fr = p.fre[o];
      if (p.fim) q.fi = p.fim[o];
    }
  }
}

// The grid is (x tiles of 64 nodes, y tiles of 4 rows, z chunks); each wavefront owns one row.
// Lanes past the last node shadow it so that every lane takes part in the DPP shifts; they
// never store.  The two end lanes of a wavefront load their outer x neighbour in the same load
// instruction in which the other lanes reload their own node (a cache hit).  The sweeps issue
// the loads of plane k+1 before computing plane k (register double buffering), which doubles
// the bytes each wavefront keeps in flight; the metric and the transposed start map stencil a
// transform of the stored values (sfix), applied to each loaded value.  Only the start map of a
// forced period or one with Dirichlet data (whose stencil reads the data on sound-soft nodes)
// loads plane by plane.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void f2_march_kernel(F2Geom g, F2Args<T> p) {
  const bool prefetch = MODE != kF2FwdStart || (!p.forced && p.dre == nullptr);
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 64 + lane;
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (j > g.ny) return;                      // a whole wavefront
  const bool live = i <= g.nx;
  const int ic = live ? i : g.nx;
  const bool last = ic == g.nx;              // right neighbour is the mirrored left one
  const int iml = mirror(ic - 1, g.nx), ipl = mirror(ic + 1, g.nx);
  const int xend = lane == 0 ? iml : (lane == 63 ? ipl : ic);
  const int jm = mirror(j - 1, g.ny), jp = mirror(j + 1, g.ny);
  const int k0 = blockIdx.z * g.kchunk;
  const int k1 = min(k0 + g.kchunk, g.nz + 1);
  T zm = sval<T, MODE>(g, p.st, p.lam, ic, j, mirror(k0 - 1, g.nz));
  T zc = sval<T, MODE>(g, p.st, p.lam, ic, j, k0);
  if (prefetch) {
    PlaneLoads<T> nxt;
    plane_loads<T, MODE>(g, p, ic, xend, j, jm, jp, k0, nxt);
    for (int k = k0; k < k1; ++k) {
      PlaneLoads<T> q = nxt;
      if (k + 1 < k1) plane_loads<T, MODE>(g, p, ic, xend, j, jm, jp, k + 1, nxt);
      if (MODE == kF2Metric || MODE == kF2AdjEnd) {
        q.zp = sfix<T, MODE>(g, p.lam, ic, j, mirror(k + 1, g.nz), q.zp);
        q.xe = sfix<T, MODE>(g, p.lam, xend, j, k, q.xe);
        q.ym = sfix<T, MODE>(g, p.lam, ic, jm, k, q.ym);
        q.yp = sfix<T, MODE>(g, p.lam, ic, jp, k, q.yp);
      }
      T xl = lane_from_left(zc);
      T xr = lane_from_right(zc);
      if (lane == 0) xl = q.xe;
      if (lane == 63) xr = q.xe;
      if (last) xr = xl;
      const T lap = T(6) * zc - (zm + q.zp + xl + xr + q.ym + q.yp);
      if (live) {
        const T F = fma(q.fi, (T)p.fsin, q.fr * (T)p.fcos);
        node_update<T, MODE>(g, p, g.idx(ic, j, k), ic, j, k, zc, lap, q.aux, q.lam, F);
      }
      zm = zc;
      zc = q.zp;
    }
  } else {
    // the start map of a forced period with Dirichlet data reads the data (at the period's
    // start) where the input state holds zero
    const bool din = MODE == kF2FwdStart && p.dre != nullptr;
    auto val = [&](int a, int b, int c) -> T {
      if (din && masked(g, a, b, c)) return dirichlet_at(p, g.idx(a, b, c), p.dcos0, p.dsin0);
      return sval<T, MODE>(g, p.st, p.lam, a, b, c);
    };
    if (din) {
      zm = val(ic, j, mirror(k0 - 1, g.nz));
      zc = val(ic, j, k0);
    }
    for (int k = k0; k < k1; ++k) {
      const T zp = val(ic, j, mirror(k + 1, g.nz));
      const T xe = val(xend, j, k);
      T xl = lane_from_left(zc);
      T xr = lane_from_right(zc);
      if (lane == 0) xl = xe;
      if (lane == 63) xr = xe;
      if (last) xr = xl;
      const T ym = val(ic, jm, k);
      const T yp = val(ic, jp, k);
      const T lap = T(6) * zc - (zm + zp + xl + xr + ym + yp);
      if (live) {
        const size_t o = g.idx(ic, j, k);
        T F = T(0);
        if (MODE == kF2FwdStart && p.forced) {
          F = p.fre[o] * (T)p.fcos;
          if (p.fim) F = fma(p.fim[o], (T)p.fsin, F);
        }
        node_update<T, MODE>(g, p, o, ic, j, k, zc, lap, p.aux[o], lam_at(g, p.lam, o), F);
      }
      zm = zc;
      zc = zp;
    }
  }
}

// Temporal blocking of the homogeneous step u^{n+1} = R (2 u^n - (1-beta) u^{n-1} - lambda L u^n)
// / (1 + beta) (every step of a forward period but its start and end, and every interior step of
// the backward period in the scaled variable).  A workgroup of WV wavefronts owns a (64 x TY)
// column tile, TY = WV RPW (each wavefront RPW consecutive rows, one column per lane), and
// marches a chunk of planes; the K steps of a launch are K pipeline levels: at plane
// iteration p, level 0 loads plane p of u^n and u^{n-1}, and level s computes plane p - s of
// u^{n+s} from level s-1's planes p-s-1 .. p-s+1 (a register window), level s-2's plane p-s (the
// older state) and the neighbours: x through lane shifts, y from the wavefront's own other row
// or, across wavefronts, through a double-buffered LDS plane per level (one barrier per plane
// iteration).  Each level loses one lane, one row and one plane of validity at the tile's edges,
// so the tile writes its inner (64 - 2K) x (TY - 2K) columns and the chunk's planes, preceded by
// K lead-in planes; it writes u^{n+K} and u^{n+K-1}.  Taller tiles re-read fewer halo rows
// (64 x 32 tiles write 58 x 26 columns at K = 3, against 58 x 10 of 64 x 16).  On the box faces a
// real node takes its mirrored neighbour from the true node, as the single-step kernel does, so
// every real node sees the same operands in the same order: blocked and single-step periods
// agree bit for bit.  Halo lanes, rows and planes outside the box read clamped addresses and are
// never stored.
constexpr int kBlockWaves = 16;   // wavefronts per workgroup unless the shape says otherwise
constexpr int kBlockChunk = 32;

// Launch shape of the blocked sweep: planes per workgroup and whether workgroups are dealt to the
// 8 XCDs in contiguous runs (so that neighbouring tiles, whose halos overlap, share an L2).
struct F2BlockShape {
  int chunk = kBlockChunk;
  int xcd = 0;
};

// Default tile shapes, from sweeps on a 513^3 grid with a per-node lambda and a 1025^3 ball with a
// constant lambda (us per step of the blocked launch, 16 wavefronts unless noted):
//   FP32, K x rows per wavefront    3 x 2    3 x 2 (12 waves)    3 x 3    4 x 2    4 x 3    4 x 4
//   513^3, 32-plane chunks            293          294             305      273      260      503
//   1025^3, 64-plane chunks          1584           --            1753     1428     1345     2051
//   FP64, 513^3, 32-plane chunks: 3 x 1 525-563, 3 x 2 472, 4 x 1 573
// A 16-wave workgroup holds its CU alone once its instance needs more than 64 VGPRs, so up to
// 128 VGPRs taller tiles cost no occupancy and re-read fewer halo rows (64 x 48 tiles write
// 56 x 40 columns at K = 4).  The deepest blocking pays in FP32, where a step of the interior
// path is about ten vector instructions; FP64 does best at K = 3 with two rows (the solver picks
// K per precision).  The 4-row tile spills heavily.
template <typename T>
constexpr int default_rpw() { return sizeof(T) == 4 ? 3 : 2; }
// Planes per workgroup: 64 when the grid still has at least 8 workgroups per CU that way
// (1025^3 ball, FP32: 1345 against 1545 us per step with 32), 32 otherwise (513^3: 260 against
// 267 with 64, whose 9 chunks leave 4.6 workgroups per CU).
inline int default_chunk(long tiles_xy, int nz, int cus) {
  return tiles_xy * ((nz + 1 + 63) / 64) >= 8L * cus ? 64 : kBlockChunk;
}

// Tile (bx, by, bz) of workgroup blockIdx: in launch order, or XCD-aware (consecutive workgroup
// ids go round-robin over the XCDs; the remap gives each XCD a contiguous run of tiles).
__device__ __forceinline__ void block_tile(int xcd, int &bx, int &by, int &bz) {
  const int gx = gridDim.x, gy = gridDim.y, nb = gx * gy * gridDim.z;
  int b = (blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
  if (xcd && nb % 8 == 0) b = (b % 8) * (nb / 8) + b / 8;
  bx = b % gx;
  by = (b / gx) % gy;
  bz = b / (gx * gy);
}

// Raw buffer access of one plane: the resource's base is the plane's first node and its size the
// plane's bytes (under 2^31 for every grid the library accepts), the lane's column offset is a
// VGPR computed once, so a plane's loads and stores cost no per-lane address arithmetic.  A lane
// offset of 2^31, or a resource of size 0, is out of range: the hardware drops such a store, so
// halo lanes and planes outside the chunk store without branching.
constexpr int kPlaneRsrcWord3 = 0x00020000;   // gfx9 resource word 3: raw (unswizzled) access
constexpr unsigned kPlaneDrop = 0x80000000u;
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const T *base, const F2Geom &g,
                                                             int k, bool live) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(base + (size_t)k * g.plane), (short)0,
                                           live ? (int)(g.plane * sizeof(T)) : 0,
                                           kPlaneRsrcWord3);
}
__device__ __forceinline__ void plane_ld(float &x, __amdgpu_buffer_rsrc_t r, unsigned vo) {
  x = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, 0, 0));
}
__device__ __forceinline__ void plane_ld(double &x, __amdgpu_buffer_rsrc_t r, unsigned vo) {
  x = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, 0, 0));
}
typedef int f2_i32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void plane_st(float x, __amdgpu_buffer_rsrc_t r, unsigned vo) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(x), r, (int)vo, 0, 0);
}
__device__ __forceinline__ void plane_st(double x, __amdgpu_buffer_rsrc_t r, unsigned vo) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(f2_i32x2, x), r, (int)vo, 0, 0);
}

// lambda in the blocked tile: read per node if the array is present (kLamAny), or known to be
// present (kLamArray) or absent (kLamConst, the constant (c dt / h)^2)
enum { kLamAny = 0, kLamArray = 1, kLamConst = 2 };

// EDGE: which of the per-node boundary treatments the tile needs.  kEdgeX: its columns (halo
// included) meet an x box face (per-lane mirror substitution, absorption, clamped columns);
// kEdgeY: its rows meet a y face (row-uniform mirror and absorption, clamped rows); kEdgeM: it
// may hold sound-soft nodes (the mask).  A tile with none (EDGE = 0) keeps only the z face
// planes' mirror and absorption, which are plane-uniform.  ZIN: no plane the chunk computes is a
// z face plane either, so those drop out too.
enum { kEdgeX = 1, kEdgeY = 2, kEdgeM = 4 };
template <typename T, int K, int RPW, int WV, int EDGE, bool ZIN, int LAM>
__device__ __forceinline__ void f2_block_tile(const F2Geom &g, const T *cur, const T *prev,
                                              const T *lam, T *out_k, T *out_km1,
                                              T (&lds)[K][2][WV * RPW][64], int bx, int by,
                                              int bz, int chunk) {
  constexpr int TY = WV * RPW, OW = 64 - 2 * K, OH = TY - 2 * K;
  constexpr bool EX = EDGE & kEdgeX, EY = EDGE & kEdgeY, EM = EDGE & kEdgeM;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = bx * OW - K + lane;
  const int k0 = bz * chunk, k1 = min(k0 + chunk, g.nz + 1);
  const int ic = EX ? min(max(i, 0), g.nx) : i;
  // per row t of this wavefront: tile row R = RPW w + t, box row j
  int jr[RPW], jcr[RPW], mxy[RPW];
  unsigned vo[RPW], vs[RPW];   // byte offset of the column in a plane; for stores, or the drop

#pragma unroll
  for (int t = 0; t < RPW; ++t) {
    const int R = RPW * w + t;
    const int j = by * OH - K + R;
    jr[t] = j;
    jcr[t] = EY ? min(max(j, 0), g.ny) : j;
    vo[t] = (unsigned)(((size_t)jcr[t] * g.px + ic) * sizeof(T));
    const bool store = lane >= K && lane < 64 - K && R >= K && R < TY - K && i <= g.nx && j <= g.ny;
    vs[t] = store ? vo[t] : kPlaneDrop;
    // absorbing faces at this column from the x faces (per lane) and the y faces (per row)
    mxy[t] = (EX ? (ic == 0 ? g.abs_face[0] : 0) + (ic == g.nx ? g.abs_face[1] : 0) : 0) +
             (EY ? (jcr[t] == 0 ? g.abs_face[2] : 0) + (jcr[t] == g.ny ? g.abs_face[3] : 0) : 0);
  }
  // the rows just outside this wavefront's rows (clamped to the tile), read from LDS
  const int Rlo = RPW * w > 0 ? RPW * w - 1 : 0;
  const int Rhi = RPW * w + RPW < TY ? RPW * w + RPW : TY - 1;
  T W[RPW][K][3];             // level s: its values at the three latest planes
  T Ld[RPW][K + 1], Rd[RPW][K + 1];   // lambda and R at planes p, p-1, ..., p-K
  T b1[RPW];                  // u^{n-1} at plane p-1 (the older state of level 1)
#pragma unroll
  for (int t = 0; t < RPW; ++t) {
    b1[t] = T(0);
#pragma unroll
    for (int s = 0; s < K; ++s) W[t][s][0] = W[t][s][1] = W[t][s][2] = T(0);
#pragma unroll
    for (int d = 0; d <= K; ++d) Ld[t][d] = Rd[t][d] = T(1);
  }
  // The loads of plane p + 1 are issued before plane p is computed, into the other of two
  // register sets (the loop is unrolled by two so that the sets trade roles without copies),
  // and the barrier waits for LDS only: the loads stay in flight across it.  (Loads two planes
  // ahead, with three register sets, measured slower.)
  struct Plane {
    T a[RPW], b[RPW], l[RPW], r[RPW];
  };
  auto load_plane = [&](int p, Plane &x) {
    const int pc = min(max(p, 0), g.nz);
    const auto rc = plane_rsrc(cur, g, pc, true), rp = plane_rsrc(prev, g, pc, true);
#pragma unroll
    for (int t = 0; t < RPW; ++t) {
      plane_ld(x.a[t], rc, vo[t]);
      plane_ld(x.b[t], rp, vo[t]);
      if (LAM == kLamArray || (LAM == kLamAny && lam))
        plane_ld(x.l[t], plane_rsrc(lam, g, pc, true), vo[t]);
      else
        x.l[t] = (T)g.lam_const;
      x.r[t] = EM ? (masked(g, ic, jcr[t], pc) ? T(0) : T(1)) : T(1);
    }
  };
  auto plane_iteration = [&](int p, const Plane &x) {
#pragma unroll
    for (int t = 0; t < RPW; ++t) {
#pragma unroll
      for (int d = K; d > 0; --d) {
        Ld[t][d] = Ld[t][d - 1];
        if (EM) Rd[t][d] = Rd[t][d - 1];
      }
      Ld[t][0] = x.l[t];
      if (EM) Rd[t][0] = x.r[t];
      W[t][0][0] = W[t][0][1];
      W[t][0][1] = W[t][0][2];
      W[t][0][2] = x.a[t];
      lds[0][p & 1][RPW * w + t][lane] = x.a[t];
    }
#pragma unroll
    for (int s = 1; s <= K; ++s) {
      const int q = p - s;
      // the wavefront's neighbour rows of level s-1 at plane q (written one iteration ago)
      const T yl = lds[s - 1][(p - 1) & 1][Rlo][lane];
      const T yh = lds[s - 1][(p - 1) & 1][Rhi][lane];
      T un[RPW];
#pragma unroll
      for (int t = 0; t < RPW; ++t) {
        T zm = W[t][s - 1][0];
        const T zc = W[t][s - 1][1];
        T zp = W[t][s - 1][2];
        T xl = lane_from_left(zc), xr = lane_from_right(zc);
        // (at the tile's first and last rows Rlo and Rhi are the wavefront's own rows, whose
        // LDS values are zc itself)
        T ym = t > 0 ? W[t - 1][s - 1][1] : yl;
        T yp = t < RPW - 1 ? W[t + 1][s - 1][1] : yh;
        if (EX) {
          if (i == 0) xl = xr;
          if (i == g.nx) xr = xl;
        }
        if (EY) {
          if (jr[t] == 0) ym = yp;
          if (jr[t] == g.ny) yp = ym;
        }
        if (!ZIN) {
          if (q == 0) zm = zp;
          if (q == g.nz) zp = zm;
        }
        const T lap = T(6) * zc - (zm + zp + xl + xr + ym + yp);
        const T l = Ld[t][s];
        const T aux = s == 1 ? b1[t] : W[t][s >= 2 ? s - 2 : 0][0];
        const int m =
            mxy[t] + (ZIN ? 0 : (q == 0 ? g.abs_face[4] : 0) + (q == g.nz ? g.abs_face[5] : 0));
        if (m == 0) {
          un[t] = fma(-l, lap, T(2) * zc - aux);
        } else {
          const T beta = face_beta(m, l);
          un[t] = face_div(T(2) * zc - (T(1) - beta) * aux - l * lap, T(1) + beta);
        }
        if (EM) un[t] = Rd[t][s] != T(0) ? un[t] : T(0);
      }
#pragma unroll
      for (int t = 0; t < RPW; ++t) {
        if (s < K) {
          W[t][s][0] = W[t][s][1];
          W[t][s][1] = W[t][s][2];
          W[t][s][2] = un[t];
          lds[s][p & 1][RPW * w + t][lane] = un[t];
        }
      }
      if (s >= K - 1) {
        const auto ro = plane_rsrc(s == K ? out_k : out_km1, g, min(max(q, 0), g.nz),
                                   q >= k0 && q < k1);
#pragma unroll
        for (int t = 0; t < RPW; ++t) plane_st(un[t], ro, vs[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < RPW; ++t) b1[t] = x.b[t];
    // LDS-only barrier: this plane's LDS writes are visible to the next iteration's reads,
    // and the next iteration's writes (the other parity) follow this iteration's reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  };
  const int pend = k1 + K - 1;
  Plane x0, x1;
  load_plane(k0 - K, x0);
  // (the loads past the last plane read clamped planes and are not used: unconditional loads
  // need no copies of the register set they replace)
  if constexpr (ZIN) {
    // Unrolled by 12, a multiple of every window's period (3 planes per level, K + 1 of lambda,
    // 2 load sets), so that the windows' shifts are register renames rather than moves.
    Plane xs[2] = {x0, x1};
    int p = k0 - K;
    for (; p + 11 <= pend; p += 12) {
#pragma unroll
      for (int u = 0; u < 12; ++u) {
        load_plane(p + u + 1, xs[(u + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        plane_iteration(p + u, xs[u & 1]);
      }
    }
#pragma unroll
    for (int u = 0; u < 11; ++u) {
      if (p + u > pend) break;
      load_plane(p + u + 1, xs[(u + 1) & 1]);
      __builtin_amdgcn_sched_barrier(0);
      plane_iteration(p + u, xs[u & 1]);
    }
    return;
  }
  for (int p = k0 - K; p <= pend; p += 2) {
    load_plane(p + 1, x1);
    __builtin_amdgcn_sched_barrier(0);   // issue the loads before this plane's work
    plane_iteration(p, x0);
    if (p + 1 > pend) break;
    load_plane(p + 2, x0);
    __builtin_amdgcn_sched_barrier(0);
    plane_iteration(p + 1, x1);
  }
}

// waves per SIMD a workgroup shape is compiled for (1: the compiler's choice); 12-wave
// workgroups are held to 6 waves per SIMD, two workgroups per CU
template <int WV>
struct F2BlockOccupancy {
  static constexpr int value = WV == 12 ? 6 : 1;
};

template <typename T, int K, int RPW, int WV>
__global__ __launch_bounds__(64 * WV)
__attribute__((amdgpu_waves_per_eu(F2BlockOccupancy<WV>::value))) void f2_block_kernel(
    F2Geom g, const T *cur, const T *prev, const T *lam, T *out_k, T *out_km1,
    F2BlockShape shape) {
  constexpr int TY = WV * RPW, OW = 64 - 2 * K, OH = TY - 2 * K;
  __shared__ T lds[K][2][TY][64];
  int bx, by, bz;
  block_tile(shape.xcd, bx, by, bz);
  const int i0 = bx * OW - K, j0 = by * OH - K;
  const int i1 = i0 + 63, j1 = j0 + TY - 1;
  const bool fx = i0 < 1 || i1 > g.nx - 1, fy = j0 < 1 || j1 > g.ny - 1;
  // the tile reads planes k0 - K .. k1 + K - 1 of its chunk: it meets a sound-soft node only if
  // that slab meets the mask's bounding box too
  const int k0 = bz * shape.chunk, k1 = min(k0 + shape.chunk, g.nz + 1);
  const bool mask = g.mask && i1 >= g.mlo[0] && i0 <= g.mhi[0] && j1 >= g.mlo[1] &&
                    j0 <= g.mhi[1] && k1 + K - 1 >= g.mlo[2] && k0 - K <= g.mhi[2];
  // level s computes planes p - s for p = k0 - K .. k1 + K - 1: planes k0 - 2K .. k1 + K - 2
  const bool zin = k0 - 2 * K >= 1 && k1 + K - 2 <= g.nz - 1;
#define CMCG_F2_TILE(E, Z, L)                                                                  \
  f2_block_tile<T, K, RPW, WV, E, Z, L>(g, cur, prev, lam, out_k, out_km1, lds, bx, by, bz,     \
                                        shape.chunk)
  if (!fx && !fy && !mask && zin && lam) CMCG_F2_TILE(0, true, kLamArray);
  else if (!fx && !fy && !mask && zin) CMCG_F2_TILE(0, true, kLamConst);
  else if (!fx && !fy && !mask) CMCG_F2_TILE(0, false, kLamAny);
  else if (!fx && !mask) CMCG_F2_TILE(kEdgeY, false, kLamAny);
  else if (!mask) CMCG_F2_TILE(kEdgeX | kEdgeY, false, kLamAny);
  else CMCG_F2_TILE(kEdgeX | kEdgeY | kEdgeM, false, kLamAny);
#undef CMCG_F2_TILE
}

// out = psi in, psi = lambda R / ((1 + beta) eta)
template <typename T>
__global__ void f2_psi_scale_kernel(F2Geom g, const T *in, const T *lam, T *out) {
  F2_ROWS(g)
  if (masked(g, i, j, k)) {
    out[o] = T(0);
    continue;
  }
  const T l = lam_at(g, lam, o);
  const int m = abs_faces(g, i, j, k);
  if (m == 0 && i > 0 && i < g.nx && j > 0 && j < g.ny && k > 0 && k < g.nz) {
    out[o] = l * in[o];
  } else {
    const T beta = m ? face_beta(m, l) : T(0);
    out[o] = l * in[o] / ((T(1) + beta) * (T)eta_of(g, i, j, k));
  }
  F2_ROWS_END
}

// ---------------------------------------------------------------------------------------
// vector kernels (plain dot products: dual x primal)
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ __forceinline__ double block_sum(double x) {
  __shared__ double part[kRedThreads / 64];
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) part[wv] = x;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kRedThreads / 64; ++k) t += part[k];
  __syncthreads();
  return t;
}

// Each thread sums its grid-stride elements in index order; the loads of four consecutive
// elements of its sequence are issued together, and their products added in that order.
template <typename TA, typename TB>
__global__ __launch_bounds__(kRedThreads) void dot_kernel(const TA *a, const TB *b, size_t n,
                                                          double *partials) {
  double acc = 0.0;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; k + 3 * stride < n; k += 4 * stride) {
    TA x[4];
    TB y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = a[k + u * stride];
      y[u] = b[k + u * stride];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += (double)x[u] * (double)y[u];
  }
  for (; k < n; k += stride) acc += (double)a[k] * (double)b[k];
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// M^{-1} on the velocity block, per node: c^2 / (h^3 eta) on free nodes, 0 on sound-soft nodes
template <typename T>
__device__ __forceinline__ double minv_at(const F2Geom &g, const T *lam, size_t o, int i, int j,
                                          int k) {
  if (masked(g, i, j, k)) return 0.0;
  const double l = lam ? (double)lam[o] : g.lam_const;
  return l * (g.h * g.h / (g.dt * g.dt)) / (g.h * g.h * g.h * eta_of(g, i, j, k));
}

// Steps 5.4-5.5 with primal and dual residuals (the velocity block of the primal residual is
// r_v = M^{-1} rh_v and is not stored):  z -= alpha d, r_u -= alpha q_u, rh -= alpha qh;
// partial delta' = <rh, r> = rh_u . r_u + rh_v . M^{-1} rh_v.  The arithmetic is FP64; TR is the
// residuals' storage type, and TZ the iterate's: FP64 z, or (FP32-mixed) the FP32 correction
// dz accumulated since the iterate was last brought up to date (z -= alpha d becomes
// dz -= alpha d, and z += dz, dz = 0 at every reliable update).
template <typename T, typename TQ, typename TR, typename TZ>
__global__ __launch_bounds__(kRedThreads) void f2_cg_update_kernel(F2Geom g, TZ *z, TR *ru,
                                                                   TR *rh, const T *d,
                                                                   const TQ *qu, const T *qh,
                                                                   const T *lam, const double *sc,
                                                                   double *partials) {
  const double alpha = sc[kAlpha];
  const size_t fs = g.fs;
  double acc = 0.0;
  F2_ROWS(g)
  z[o] = (TZ)((double)z[o] - alpha * (double)d[o]);
  z[o + fs] = (TZ)((double)z[o + fs] - alpha * (double)d[o + fs]);
  const TR rn = (TR)((double)ru[o] - alpha * (double)qu[o]);
  ru[o] = rn;
  const TR rhu = (TR)((double)rh[o] - alpha * (double)qh[o]);
  const TR rhv = (TR)((double)rh[o + fs] - alpha * (double)qh[o + fs]);
  rh[o] = rhu;
  rh[o + fs] = rhv;
  acc += (double)rhu * (double)rn + (double)rhv * (double)rhv * minv_at(g, lam, o, i, j, k);
  F2_ROWS_END
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// delta = <rh, r> with r_v = M^{-1} rh_v; with `rus`, `rhs` non-null the residuals (FP64) are
// also stored there in their storage type
template <typename T, typename TR>
__global__ __launch_bounds__(kRedThreads) void f2_delta_kernel(F2Geom g, const double *ru,
                                                               const double *rh, const T *lam,
                                                               TR *rus, TR *rhs,
                                                               double *partials) {
  const size_t fs = g.fs;
  double acc = 0.0;
  F2_ROWS(g)
  acc += rh[o] * ru[o] + rh[o + fs] * rh[o + fs] * minv_at(g, lam, o, i, j, k);
  if (rus) {
    rus[o] = (TR)ru[o];
    rhs[o] = (TR)rh[o];
    rhs[o + fs] = (TR)rh[o + fs];
  }
  F2_ROWS_END
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// Step 5.7: d = r + beta d  (d_u = r_u + beta d_u, d_v = M^{-1} rh_v + beta d_v); beta from sc,
// or 0 when `first` (d = r)
template <typename T, typename TR>
__global__ void f2_direction_kernel(F2Geom g, T *d, const TR *ru, const TR *rh, const T *lam,
                                    const double *sc, int first) {
  const size_t fs = g.fs;
  const double beta = first ? 0.0 : sc[kBeta];
  F2_ROWS(g)
  d[o] = (T)((double)ru[o] + beta * (double)d[o]);
  d[o + fs] = (T)(minv_at(g, lam, o, i, j, k) * (double)rh[o + fs] + beta * (double)d[o + fs]);
  F2_ROWS_END
}

// out = z + dz (two fields), the iterate with its FP32 correction; `clear`: dz = 0 (out == z
// brings the iterate up to date in place)
__global__ void f2_iterate_kernel(F2Geom g, const double *z, float *dz, double *out, int clear) {
  const size_t fs = g.fs;
  F2_ROWS(g)
  const double a = z[o] + (double)dz[o], b = z[o + fs] + (double)dz[o + fs];
  out[o] = a;
  out[o + fs] = b;
  if (clear) {
    dz[o] = 0.0f;
    dz[o + fs] = 0.0f;
  }
  F2_ROWS_END
}

// out = in (two fields: u, and the velocity block through M^{-1}), widened to FP64
template <typename TR, typename T>
__global__ void f2_primal_kernel(F2Geom g, const TR *ru, const TR *rh, const T *lam, double *out) {
  const size_t fs = g.fs;
  F2_ROWS(g)
  out[o] = (double)ru[o];
  out[o + fs] = minv_at(g, lam, o, i, j, k) * (double)rh[o + fs];
  F2_ROWS_END
}

// Node sums of the compatibility condition 1^T [S - wt^2 M - i wh B] U = 1^T Fhat (S 1 = 0):
// the lumped mass M = h eta dt^2 / lambda, the absorbing boundary mass B = 2 h eta dt m /
// sqrt(lambda) (m absorbing faces at the node), the load Fhat = h eta F / lambda (F the device
// load field dt^2 c^2 G), and M a, B a for a = sa ar + i sb ai.  One partial per block of each
// of the kCompatSums sums, stored sum-major.
__global__ __launch_bounds__(kRedThreads) void f2_compat_kernel(F2Geom g, const double *lam,
                                                                const double *Fre,
                                                                const double *Fim,
                                                                const double *ar, double sa,
                                                                const double *ai, double sb,
                                                                double *partials) {
  double acc[kCompatSums] = {};
  F2_ROWS(g)
  const double l = lam ? lam[o] : g.lam_const;
  const double he = g.h * eta_of(g, i, j, k);
  const int m = abs_faces(g, i, j, k);
  const double M = he * g.dt * g.dt / l;
  const double B = m ? 2.0 * he * g.dt * m / sqrt(l) : 0.0;
  const double a = sa * ar[o], b = ai ? sb * ai[o] : 0.0;
  acc[0] += M;
  acc[1] += B;
  acc[2] += Fre ? he * Fre[o] / l : 0.0;
  acc[3] += Fim ? he * Fim[o] / l : 0.0;
  acc[4] += M * a;
  acc[5] += M * b;
  acc[6] += B * a;
  acc[7] += B * b;
  F2_ROWS_END
#pragma unroll
  for (int q = 0; q < kCompatSums; ++q) {
    const double t = block_sum(acc[q]);
    if (threadIdx.x == 0) partials[(size_t)q * gridDim.x + blockIdx.x] = t;
  }
}

// q_v = M^{-1} qh_v on the free nodes (the velocity block of the Riesz map)
template <typename T>
__global__ void f2_mass_inverse_kernel(F2Geom g, const T *qh_v, double *q_v, const T *lam) {
  F2_ROWS(g)
  q_v[o] = (double)qh_v[o] * minv_at(g, lam, o, i, j, k);
  F2_ROWS_END
}

template <typename T>
__global__ void f2_setup_kernel(F2Geom g, const double *c, double c_const, const double *fre,
                                const double *fim, const double *gre, const double *gim,
                                T *lam, T *Fre, T *Fim) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  F2_ROWS(g)
  const size_t u = ((size_t)k * (ny + 1) + j) * (nx + 1) + i;   // packed user index
  const double cv = c ? c[u] : c_const;
  const double l = (cv * g.dt / g.h) * (cv * g.dt / g.h);
  if (lam) lam[o] = (T)l;
  if (Fre) {
    double ar = fre ? fre[u] : 0.0, ai = fim ? fim[u] : 0.0;
    if (gre || gim) {
      // faces -x, +x, -y, +y, -z, +z; nodes in order of the remaining axes, slower first
      const size_t sx = (size_t)(nz + 1) * (ny + 1), sy = (size_t)(nz + 1) * (nx + 1);
      const size_t off[6] = {0, sx, 2 * sx, 2 * sx + sy, 2 * sx + 2 * sy,
                             2 * sx + 2 * sy + (size_t)(ny + 1) * (nx + 1)};
      const bool on[6] = {i == 0, i == nx, j == 0, j == ny, k == 0, k == nz};
      const size_t along[6] = {(size_t)k * (ny + 1) + j, (size_t)k * (ny + 1) + j,
                               (size_t)k * (nx + 1) + i, (size_t)k * (nx + 1) + i,
                               (size_t)j * (nx + 1) + i, (size_t)j * (nx + 1) + i};
      for (int f = 0; f < 6; ++f) {
        if (!on[f]) continue;
        if (gre) ar += 2.0 / g.h * gre[off[f] + along[f]];
        if (gim) ai += 2.0 / g.h * gim[off[f] + along[f]];
      }
    }
    const double s = g.dt * g.dt * cv * cv;
    Fre[o] = (T)(s * ar);
    if (Fim) Fim[o] = (T)(s * ai);
  }
  F2_ROWS_END
}

// packed user node array (FP64) <-> device layout (T); sound-soft entries enter as 0
template <typename T>
__global__ void f2_unpack_kernel(F2Geom g, const double *packed, T *dev, int nfields) {
  const size_t nn = (size_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
  F2_ROWS(g)
  const size_t u = ((size_t)k * (g.ny + 1) + j) * (g.nx + 1) + i;
  const bool m = masked(g, i, j, k);
  for (int f = 0; f < nfields; ++f) dev[o + f * g.fs] = m ? T(0) : (T)packed[f * nn + u];
  F2_ROWS_END
}

template <typename T>
__global__ void f2_pack_kernel(F2Geom g, const T *dev, double *packed, int nfields) {
  const size_t nn = (size_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
  F2_ROWS(g)
  const size_t u = ((size_t)k * (g.ny + 1) + j) * (g.nx + 1) + i;
  for (int f = 0; f < nfields; ++f) packed[f * nn + u] = (double)dev[o + f * g.fs];
  F2_ROWS_END
}

// blocks for a row loop: four rows per 256-thread block
inline int rows_grid(const F2Geom &g) {
  const long rows = (long)(g.ny + 1) * (g.nz + 1);
  const long b = (rows + 3) / 4;
  return (int)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

template <typename T>
hipError_t f2_march(int mode, const F2Geom &g, const F2Args<T> &p, hipStream_t s) {
  dim3 grid((g.nx + 1 + 63) / 64, (g.ny + 1 + 3) / 4, (g.nz + 1 + g.kchunk - 1) / g.kchunk);
  dim3 block(256);
  switch (mode) {
#define CASE(M) \
  case M: hipLaunchKernelGGL((f2_march_kernel<T, M>), grid, block, 0, s, g, p); break;
    CASE(kF2FwdStart)
    CASE(kF2FwdStep)
    CASE(kF2FwdEnd)
    CASE(kF2Metric)
    CASE(kF2AdjInit)
    CASE(kF2AdjStepFirst)
    CASE(kF2AdjEnd)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Tile shape of the blocked launches: rows per wavefront and wavefronts per workgroup.
// CMCG_F2_RPW and CMCG_F2_WAVES (environment, read per call) override them for sweeps and tests:
// rows 1 or 2 (FP32 also 3 or 4), and 12 wavefronts instead of 16 with two rows.
template <typename T>
void f2_block_shape(int *rpw, int *wv) {
  const char *re = std::getenv("CMCG_F2_RPW");
  const char *we = std::getenv("CMCG_F2_WAVES");
  const int want = re ? std::atoi(re) : 0;
  const int rmax = sizeof(T) == 4 ? 4 : 2;
  *rpw = (want >= 1 && want <= rmax) ? want : default_rpw<T>();
  *wv = (*rpw == 2 && we && std::atoi(we) == 12) ? 12 : kBlockWaves;
}

template <typename T>
hipError_t f2_march_block(const F2Geom &g, const T *cur, const T *prev, const T *lam, T *out_k,
                          T *out_km1, int K, hipStream_t s) {
  // CMCG_F2_CHUNK and CMCG_F2_XCD (environment, read per launch) override the launch shape for
  // sweeps and tests (chunk 0: the tile shape's default)
  F2BlockShape env_shape;
  env_shape.chunk = 0;
  if (const char *e = std::getenv("CMCG_F2_CHUNK")) env_shape.chunk = std::max(1, std::atoi(e));
  if (const char *e = std::getenv("CMCG_F2_XCD")) env_shape.xcd = std::atoi(e);
  int rpw = 0, wv = 0;
  f2_block_shape<T>(&rpw, &wv);
  dim3 block(64 * wv);
  F2BlockShape shape = env_shape;
  auto tiles = [&](int k, int ax) {
    const int n = ax == 0 ? g.nx : g.ny, w = (ax == 0 ? 64 : wv * rpw) - 2 * k;
    return (n + 1 + w - 1) / w;
  };
  if (shape.chunk == 0) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return hipErrorInvalidDevice;
    shape.chunk = default_chunk((long)tiles(K, 0) * tiles(K, 1), g.nz, cus);
  }
  auto grid = [&](int k) {
    return dim3(tiles(k, 0), tiles(k, 1), (g.nz + 1 + shape.chunk - 1) / shape.chunk);
  };
#define CMCG_F2_BLOCK(KK, RR, WW)                                                              \
  hipLaunchKernelGGL((f2_block_kernel<T, KK, RR, WW>), grid(KK), block, 0, s, g, cur, prev,    \
                     lam, out_k, out_km1, shape)
  if constexpr (sizeof(T) == 4) {
    switch ((K * 8 + rpw) * 32 + wv) {
      case (2 * 8 + 3) * 32 + 16: CMCG_F2_BLOCK(2, 3, 16); return hipGetLastError();
      case (3 * 8 + 3) * 32 + 16: CMCG_F2_BLOCK(3, 3, 16); return hipGetLastError();
      case (4 * 8 + 3) * 32 + 16: CMCG_F2_BLOCK(4, 3, 16); return hipGetLastError();
      case (2 * 8 + 4) * 32 + 16: CMCG_F2_BLOCK(2, 4, 16); return hipGetLastError();
      case (3 * 8 + 4) * 32 + 16: CMCG_F2_BLOCK(3, 4, 16); return hipGetLastError();
      case (4 * 8 + 4) * 32 + 16: CMCG_F2_BLOCK(4, 4, 16); return hipGetLastError();
      default: break;
    }
  }
  switch ((K * 8 + rpw) * 32 + wv) {
    case (2 * 8 + 1) * 32 + 16: CMCG_F2_BLOCK(2, 1, 16); break;
    case (3 * 8 + 1) * 32 + 16: CMCG_F2_BLOCK(3, 1, 16); break;
    case (4 * 8 + 1) * 32 + 16: CMCG_F2_BLOCK(4, 1, 16); break;
    case (2 * 8 + 2) * 32 + 16: CMCG_F2_BLOCK(2, 2, 16); break;
    case (3 * 8 + 2) * 32 + 16: CMCG_F2_BLOCK(3, 2, 16); break;
    case (4 * 8 + 2) * 32 + 16: CMCG_F2_BLOCK(4, 2, 16); break;
    case (2 * 8 + 2) * 32 + 12: CMCG_F2_BLOCK(2, 2, 12); break;
    case (3 * 8 + 2) * 32 + 12: CMCG_F2_BLOCK(3, 2, 12); break;
    case (4 * 8 + 2) * 32 + 12: CMCG_F2_BLOCK(4, 2, 12); break;
    default: return hipErrorInvalidValue;
  }
#undef CMCG_F2_BLOCK
  return hipGetLastError();
}

template <typename T>
hipError_t f2_psi_scale(const F2Geom &g, const T *in, const T *lam, T *out, hipStream_t s) {
  hipLaunchKernelGGL((f2_psi_scale_kernel<T>), dim3(rows_grid(g)), dim3(256), 0, s, g, in, lam, out);
  return hipGetLastError();
}

template <typename TA, typename TB>
hipError_t dot_plain(const TA *a, const TB *b, size_t n, double *partials, hipStream_t s) {
  hipLaunchKernelGGL((dot_kernel<TA, TB>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b, n,
                     partials);
  return hipGetLastError();
}

template <typename T, typename TQ, typename TR, typename TZ>
hipError_t f2_cg_update(const F2Geom &g, TZ *z, TR *ru, TR *rh, const T *d, const TQ *qu,
                        const T *qh, const T *lam, const double *sc, double *partials,
                        hipStream_t s) {
  hipLaunchKernelGGL((f2_cg_update_kernel<T, TQ, TR, TZ>), dim3(kRedBlocks), dim3(kRedThreads), 0,
                     s, g, z, ru, rh, d, qu, qh, lam, sc, partials);
  return hipGetLastError();
}

template <typename T, typename TR>
hipError_t f2_delta(const F2Geom &g, const double *ru, const double *rh, const T *lam, TR *rus,
                    TR *rhs, double *partials, hipStream_t s) {
  hipLaunchKernelGGL((f2_delta_kernel<T, TR>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, g, ru,
                     rh, lam, rus, rhs, partials);
  return hipGetLastError();
}

template <typename T, typename TR>
hipError_t f2_direction(const F2Geom &g, T *d, const TR *ru, const TR *rh, const T *lam,
                        const double *sc, int first, hipStream_t s) {
  hipLaunchKernelGGL((f2_direction_kernel<T, TR>), dim3(rows_grid(g)), dim3(256), 0, s, g, d, ru,
                     rh, lam, sc, first);
  return hipGetLastError();
}

hipError_t f2_iterate(const F2Geom &g, const double *z, float *dz, double *out, int clear,
                      hipStream_t s) {
  hipLaunchKernelGGL(f2_iterate_kernel, dim3(rows_grid(g)), dim3(256), 0, s, g, z, dz, out, clear);
  return hipGetLastError();
}

template <typename TR, typename T>
hipError_t f2_primal(const F2Geom &g, const TR *ru, const TR *rh, const T *lam, double *out,
                     hipStream_t s) {
  hipLaunchKernelGGL((f2_primal_kernel<TR, T>), dim3(rows_grid(g)), dim3(256), 0, s, g, ru, rh,
                     lam, out);
  return hipGetLastError();
}

template <typename T>
hipError_t f2_mass_inverse(const F2Geom &g, const T *qh_v, double *q_v, const T *lam,
                           hipStream_t s) {
  hipLaunchKernelGGL((f2_mass_inverse_kernel<T>), dim3(rows_grid(g)), dim3(256), 0, s, g, qh_v,
                     q_v, lam);
  return hipGetLastError();
}

hipError_t f2_compat_sums(const F2Geom &g, const double *lam, const double *Fre, const double *Fim,
                          const double *ar, double sa, const double *ai, double sb,
                          double *partials, hipStream_t s) {
  hipLaunchKernelGGL(f2_compat_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, s, g, lam, Fre, Fim,
                     ar, sa, ai, sb, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t f2_setup(const F2Geom &g, const double *c, double c_const, const double *fre,
                    const double *fim, const double *gre, const double *gim, T *lam, T *Fre, T *Fim,
                    hipStream_t s) {
  hipLaunchKernelGGL((f2_setup_kernel<T>), dim3(rows_grid(g)), dim3(256), 0, s, g, c, c_const, fre,
                     fim, gre, gim, lam, Fre, Fim);
  return hipGetLastError();
}

template <typename T>
hipError_t f2_unpack(const F2Geom &g, const double *packed, T *dev, int nfields, hipStream_t s) {
  hipLaunchKernelGGL((f2_unpack_kernel<T>), dim3(rows_grid(g)), dim3(256), 0, s, g, packed, dev,
                     nfields);
  return hipGetLastError();
}

template <typename T>
hipError_t f2_pack(const F2Geom &g, const T *dev, double *packed, int nfields, hipStream_t s) {
  hipLaunchKernelGGL((f2_pack_kernel<T>), dim3(rows_grid(g)), dim3(256), 0, s, g, dev, packed,
                     nfields);
  return hipGetLastError();
}

#define INST(T)                                                                                   \
  template hipError_t f2_march<T>(int, const F2Geom &, const F2Args<T> &, hipStream_t);          \
  template hipError_t f2_psi_scale<T>(const F2Geom &, const T *, const T *, T *, hipStream_t);   \
  template hipError_t f2_march_block<T>(const F2Geom &, const T *, const T *, const T *, T *,    \
                                        T *, int, hipStream_t);                                  \
  template void f2_block_shape<T>(int *, int *);                                                 \
  template hipError_t f2_mass_inverse<T>(const F2Geom &, const T *, double *, const T *,         \
                                         hipStream_t);                                            \
  template hipError_t f2_setup<T>(const F2Geom &, const double *, double, const double *,        \
                                  const double *, const double *, const double *, T *, T *, T *, \
                                  hipStream_t);                                                   \
  template hipError_t f2_unpack<T>(const F2Geom &, const double *, T *, int, hipStream_t);       \
  template hipError_t f2_pack<T>(const F2Geom &, const T *, double *, int, hipStream_t);
INST(float)
INST(double)
// CG vector passes: FP64 solves (FP64 everything), FP32-mixed solves (FP32 d, q, residuals and
// iterate correction; q_u in FP64 from a PCG Riesz solve or FP32 from a V-cycle)
template hipError_t f2_cg_update<double, double, double, double>(
    const F2Geom &, double *, double *, double *, const double *, const double *, const double *,
    const double *, const double *, double *, hipStream_t);
template hipError_t f2_cg_update<float, double, float, float>(
    const F2Geom &, float *, float *, float *, const float *, const double *, const float *,
    const float *, const double *, double *, hipStream_t);
template hipError_t f2_cg_update<float, float, float, float>(
    const F2Geom &, float *, float *, float *, const float *, const float *, const float *,
    const float *, const double *, double *, hipStream_t);
template hipError_t f2_delta<double, double>(const F2Geom &, const double *, const double *,
                                             const double *, double *, double *, double *,
                                             hipStream_t);
template hipError_t f2_delta<double, float>(const F2Geom &, const double *, const double *,
                                            const double *, float *, float *, double *,
                                            hipStream_t);
template hipError_t f2_direction<double, double>(const F2Geom &, double *, const double *,
                                                 const double *, const double *, const double *,
                                                 int, hipStream_t);
template hipError_t f2_direction<float, float>(const F2Geom &, float *, const float *,
                                               const float *, const float *, const double *, int,
                                               hipStream_t);
template hipError_t f2_primal<double, double>(const F2Geom &, const double *, const double *,
                                              const double *, double *, hipStream_t);
template hipError_t f2_primal<float, double>(const F2Geom &, const float *, const float *,
                                             const double *, double *, hipStream_t);
#undef INST
template hipError_t dot_plain<double, double>(const double *, const double *, size_t, double *, hipStream_t);
template hipError_t dot_plain<float, float>(const float *, const float *, size_t, double *, hipStream_t);
template hipError_t dot_plain<double, float>(const double *, const float *, size_t, double *, hipStream_t);
template hipError_t dot_plain<float, double>(const float *, const double *, size_t, double *, hipStream_t);

}  // namespace cmcg
