// First-order (staggered, 2D) solver runtime: memory plan, period loops, and the CG driver of the
// CMCG Algorithm (Sec. 2.3, Steps 1-6, with the first-order gradient of eq. mixJ_deriative_2).
//
// Precision policy.  FP64 mode: every period in FP64.  FP32-mixed mode: the CG iterations' forward
// and backward periods run in FP32 (state, coefficients and stencil arithmetic), while the iterate
// z, the residual r, every inner product and every CG scalar stay FP64.  Because one period is a
// long product of step matrices, an FP32 period has a rounding floor of about 1e-6 |d| that is not
// small against (E - I) d for nearly periodic directions; CG on the FP32 operator alone stalls far
// above 1e-6.  The mixed mode therefore uses reliable updates (residual replacement): whenever the
// recursive residual has fallen by the refresh factor since the last refresh (and before declaring
// convergence), the true gradient at the FP64 iterate is recomputed with one FP64 forward and one
// FP64 backward period and replaces r; the search direction is kept.  The initial gradient and the
// output filter period are FP64 as well.
#include <cstring>
#include <deque>
#include <map>
#include <tuple>
#include <type_traits>

#include "f1_device.h"
#include "solver.h"

namespace cmcg {
namespace {

constexpr double kPi = 3.14159265358979323846;

// kap = dt c^2 / h per cell and h Fhat, Fhat = f + (1/h) sum_abs gS the forcing amplitude of every
// cell (the boundary data enters the velocity equation through the boundary flux p.n = gS - v/c).
template <typename T>
__global__ void f1_setup_kernel(F1Geom g, const double *c, double c_const, const double *fre,
                                const double *fim, const double *gre, const double *gim, T *cc,
                                T *Fre, T *Fim, size_t fs) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const int nx = g.nx, ny = g.ny;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < fs; o += stride) {
    const int j = (int)(o / g.pitch), i = (int)(o % g.pitch);
    if (i >= nx) {
      cc[o] = T(1);
      Fre[o] = T(0);
      if (Fim) Fim[o] = T(0);
      continue;
    }
    const size_t k = (size_t)j * nx + i;
    const double cv = c ? c[k] : c_const;
    cc[o] = (T)(g.dt * cv * cv / g.h);        // kap = dt c^2 / h
    double ar = fre ? fre[k] : 0.0, ai = fim ? fim[k] : 0.0;
    const double ih = 1.0 / g.h;
    if (gre || gim) {
      // faces: -x (ny values), +x (ny), -y (nx), +y (nx)
      const size_t off[4] = {0, (size_t)ny, (size_t)2 * ny, (size_t)2 * ny + nx};
      const bool on[4] = {i == 0, i == nx - 1, j == 0, j == ny - 1};
      const int along[4] = {j, j, i, i};
      for (int f = 0; f < 4; ++f) {
        if (!on[f]) continue;
        if (gre) ar += gre[off[f] + along[f]] * ih;
        if (gim) ai += gim[off[f] + along[f]] * ih;
      }
    }
    Fre[o] = (T)(g.h * ar);                   // h Fhat
    if (Fim) Fim[o] = (T)(g.h * ai);
  }
}

// u = i V / omega with V = (2/N) (Ure + i Uim)  (eq. TH_FILTERED_MIXED_SOLUTION, discrete)
__global__ void f1_output_kernel(const double *ure, const double *uim, double scale, double *out_re,
                                 double *out_im, size_t fs) {
  f1_output_block(ure, uim, scale, out_re, out_im, fs, blockIdx.x, gridDim.x);
}

// Weights (c, s)_j of the components at one time: amp (cos, sin)(m_j omega t), amp the ramp.
struct ShotWeights {
  int nshots = 0;
  double c[CMCG_MAX_SHOTS] = {}, s[CMCG_MAX_SHOTS] = {};
};

// Source field of one step of a multi-frequency forced period: sum_j (Fre_j c_j + Fim_j s_j) at
// the step's source time (h Fhat summed over the components), which the streaming kernel then
// reads with weight 1 as it reads a single component's field; and, with Dirichlet data, v on the
// Dirichlet cells summed over the components at the step's input time (DA, weights w0) and
// output time (DB, weights w1).
template <typename T>
__global__ void f1_combine_kernel(const T *Fre, const T *Fim, ShotWeights w, T *out,
                                  const double *Dre, const double *Dim, ShotWeights w0,
                                  ShotWeights w1, double *DA, double *DB, size_t fs) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < fs; o += stride) {
    double a = 0.0;
#pragma unroll
    for (int j = 0; j < CMCG_MAX_SHOTS; ++j) {
      if (j >= w.nshots) break;
      a = fma((double)Fre[j * fs + o], w.c[j], a);
      if (Fim) a = fma((double)Fim[j * fs + o], w.s[j], a);
    }
    out[o] = (T)a;
    if (Dre) {
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int j = 0; j < CMCG_MAX_SHOTS; ++j) {
        if (j >= w.nshots) break;
        const double dr = Dre[j * fs + o], di = Dim ? Dim[j * fs + o] : 0.0;
        a0 = fma(dr, w0.c[j], fma(di, w0.s[j], a0));
        a1 = fma(dr, w1.c[j], fma(di, w1.s[j], a1));
      }
      DA[o] = a0;
      DB[o] = a1;
    }
  }
}

// Filter sums of a multi-frequency problem at one step: (Ure_j, Uim_j) += v (cos, sin)(m_j w t_n);
// on the Dirichlet cells v is the data at t_n (DA)
__global__ void f1_accumulate_kernel(const double *v, const uint8_t *mask, const double *DA,
                                     ShotWeights w, double *ure, double *uim, size_t fs) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < fs; o += stride) {
    const double x = (mask && mask[o]) ? (DA ? DA[o] : 0.0) : v[o];
#pragma unroll
    for (int j = 0; j < CMCG_MAX_SHOTS; ++j) {
      if (j >= w.nshots) break;
      ure[j * fs + o] += x * w.c[j];
      uim[j * fs + o] += x * w.s[j];
    }
  }
}

// The solution read off a state (eq. mix_solution, time-discrete): per cell, the flux amplitudes
// on its interior faces Q = P_0 / cos(theta) + i (dt/h) (difference of v_0 across the face) /
// (2 sin(theta)), then V = kap (h Fhat + sum of signed face Q) / (-2 i sin(theta) +
// 2 gamma cos(theta)) and u = i V / omega into (ure, uim) (device layout).  kap = dt c^2 / h.
// Dirichlet cells (mask): V = dre + i dim is data (the amplitude -i omega gD of v), its real
// part stands for v_0 there.
__device__ __forceinline__ double f1_v0(const double *v, const uint8_t *mask, const double *dre,
                                        size_t o) {
  if (mask && mask[o]) return dre ? dre[o] : 0.0;
  return v[o];
}

__global__ void f1_step6_kernel(F1Geom g, const double *z, const double *cc, const double *Fre,
                                const double *Fim, const double *dre, const double *dim,
                                double theta, double omega, double *ure, double *uim, size_t fs) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const int nx = g.nx, ny = g.ny;
  const size_t pitch = (size_t)g.pitch;
  const double dth = g.dt / g.h, ic = 1.0 / cos(theta), is2 = 0.5 / sin(theta);
  const double *px = z, *py = z + fs, *v = z + 2 * fs;
  const uint8_t *mask = g.mask;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < fs; o += stride) {
    const int j = (int)(o / pitch), i = (int)(o % pitch);
    if (i >= nx) continue;
    if (mask && mask[o]) {
      const double Vr = dre ? dre[o] : 0.0, Vi = dim ? dim[o] : 0.0;
      ure[o] = -Vi / omega;
      uim[o] = Vr / omega;
      continue;
    }
    const double vc = v[o];
    double sr = 0.0, si = 0.0;           // sum over the faces of the outward flux amplitude
    if (i <= nx - 2) { sr += px[o] * ic;          si += dth * (f1_v0(v, mask, dre, o + 1) - vc) * is2; }
    if (i >= 1)      { sr -= px[o - 1] * ic;      si -= dth * (vc - f1_v0(v, mask, dre, o - 1)) * is2; }
    if (j <= ny - 2) { sr += py[o] * ic;          si += dth * (f1_v0(v, mask, dre, o + pitch) - vc) * is2; }
    if (j >= 1)      { sr -= py[o - pitch] * ic;  si -= dth * (vc - f1_v0(v, mask, dre, o - pitch)) * is2; }
    const double kap = cc[o];
    const double nr = kap * (Fre[o] + sr), ni = kap * ((Fim ? Fim[o] : 0.0) + si);
    const int m = (i == 0 ? g.abs_face[0] : 0) + (i == nx - 1 ? g.abs_face[1] : 0) +
                  (j == 0 ? g.abs_face[2] : 0) + (j == ny - 1 ? g.abs_face[3] : 0);
    const double gam = 0.5 * m * sqrt(kap * dth);
    const double dr = 2.0 * gam * cos(theta), di = -2.0 * sin(theta);
    const double den = dr * dr + di * di;
    const double Vr = (nr * dr + ni * di) / den, Vi = (ni * dr - nr * di) / den;
    ure[o] = -Vi / omega;
    uim[o] = Vr / omega;
  }
}

// Riesz map of the first-order formulation, M_E^{-1} y (the control space is L^2): faces 1/h^2,
// cells c^2 / h^2 = kap / (h dt)
template <typename T>
__global__ void f1_riesz_kernel(F1Geom g, T *y, const T *cc, size_t fs) {
  const double ih2 = 1.0 / (g.h * g.h), ihdt = 1.0 / (g.h * g.dt);
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < fs; o += stride) {
    y[o] = (T)((double)y[o] * ih2);
    y[o + fs] = (T)((double)y[o + fs] * ih2);
    y[o + 2 * fs] = (T)((double)y[o + 2 * fs] * ihdt * (double)cc[o]);
  }
}

// One precision's working set: two ping-pong states, the period output w and the backward
// output q, the coefficient field, the forcing fields (one pair per source component) and, with
// several components, the summed source field of one step.
struct F1Set {
  int prec = CMCG_FP64;
  void *S0 = nullptr, *S1 = nullptr, *W = nullptr, *Q = nullptr;
  void *cc = nullptr, *Fre = nullptr, *Fim = nullptr, *Fk = nullptr;
};

template <typename T>
T *tp(void *p) { return static_cast<T *>(p); }
template <typename T>
const T *tpc(const void *p) { return static_cast<const T *>(p); }

class F1Solver final : public Solver {
 public:
  F1Geom g{};
  size_t fs = 0, vecN = 0;
  SolverConfig cfg;
  hipStream_t s = nullptr;
  DeviceArena arena;
  PhaseEvents ev;
  BulkTimer bulk;
  int bulk_dir = -1;     // >= 0: time the bulk launches of the next periods in this direction
  F1Set lo, hi;          // lo: precision of the CG periods; hi: FP64 (the same set in FP64 mode)
  bool mixed = false;
  void *D = nullptr;     // search direction, lo precision
  double *Z = nullptr, *R = nullptr, *Ure = nullptr, *Uim = nullptr;   // filter sums: nshots fields
  uint8_t *mask = nullptr;     // Dirichlet cells (device layout), or null
  // Dirichlet data of v, one field pair per component: v = Dre cos(m w t) + Dim sin(m w t),
  // Dre = m w Im(gD), Dim = -m w Re(gD) (the real part of -i m w gD e^{-i m w t}); or null
  double *Dre = nullptr, *Dim = nullptr;
  double *DA = nullptr, *DB = nullptr;   // several components: v on the Dirichlet cells of a step
  double *partials = nullptr, *scalars = nullptr, *h_scalars = nullptr;
  bool started = false;
  bool multi = false;    // several source components: per-step source fields, separate filter sums
  int iter = 0, refreshes = 0, last_refresh = 0, runup_done = 0;
  double rel = 1.0, delta_at_refresh = 0.0;
  double t_fwd = 0, t_adj = 0, t_other = 0, t_total = 0, t_runup = 0, updates = 0;
  double dram = 0;   // compulsory HBM bytes of the stencil launches since cmcg_begin
  // source ramp of forced periods: absolute start time of the period and switch-on length
  // (t_tr = 0: no ramp)
  double t_offset = 0.0, t_tr = 0.0;

  // fixed-buffer mode: device memory from a caller's buffer, scalars in host memory of the
  // object, no events
  bool fixed = false;
  double h_scalars_local[kNumScalars] = {};

  ~F1Solver() override {
    if (s) (void)hipStreamSynchronize(s);
    if (h_scalars && !fixed) (void)hipHostFree(h_scalars);
  }

  size_t device_bytes() const override { return arena.bytes(); }

  // ------------------------------------------------------------------ create
  cmcg_status create(const cmcg_problem *P) {
    const int nx = (int)P->n[0], ny = (int)P->n[1];
    s = cfg.stream;
    g.nx = nx;
    g.ny = ny;
    g.pitch = (nx + 63) / 64 * 64;
    g.h = cfg.h;
    g.dt = cfg.dt;
    for (int f = 0; f < 4; ++f) g.abs_face[f] = P->face_bc[f] == CMCG_ABSORBING ? 1 : 0;
    fs = (size_t)ny * g.pitch;
    vecN = 3 * fs;
    mixed = cfg.prec == CMCG_FP32_MIXED;
    const std::vector<cmcg_shot> shots = shots_of(P);
    const int J = (int)shots.size();
    multi = J > 1;
    if (fixed) {
      h_scalars = h_scalars_local;
    } else {
      CMCG_TRY(ev.init(10));
      CMCG_TRY(bulk.init());
      CMCG_HIP(hipHostMalloc((void **)&h_scalars, kNumScalars * sizeof(double)));
    }
    std::fill(h_scalars, h_scalars + kNumScalars, 0.0);
    bool has_im = false;
    for (const cmcg_shot &sh : shots) has_im = has_im || sh.f_im || sh.gS_im;
    CMCG_TRY(alloc_set(hi, CMCG_FP64, has_im, J));
    if (mixed) {
      CMCG_TRY(alloc_set(lo, CMCG_FP32_MIXED, has_im, J));
    } else {
      lo = hi;
    }
    CMCG_TRY(arena.alloc(vecN * (mixed ? sizeof(float) : sizeof(double)), &D, s));
    CMCG_TRY(arena.alloc_n(vecN, &Z, s));
    CMCG_TRY(arena.alloc_n(vecN, &R, s));
    CMCG_TRY(arena.alloc_n(J * fs, &Ure, s));
    CMCG_TRY(arena.alloc_n(J * fs, &Uim, s));
    CMCG_TRY(arena.alloc_n(kRedBlocks, &partials, s));
    CMCG_TRY(arena.alloc_n(kNumScalars, &scalars, s));
    // host inputs -> temporary device copies -> setup kernels for each set and component
    const size_t ncell = (size_t)nx * ny, nface = 2 * (size_t)ny + 2 * (size_t)nx;
    if (P->sound_soft) CMCG_TRY(setup_dirichlet(P, shots));
    for (int j = 0; j < J; ++j) {
      // the inputs' device copies (in fixed-buffer mode carved from the same buffer, where they
      // stay until the solver goes)
      DeviceArena tmp_own;
      DeviceArena &tmp = fixed ? arena : tmp_own;
      const double *src[5] = {P->c, shots[j].f_re, shots[j].f_im, shots[j].gS_re, shots[j].gS_im};
      const size_t len[5] = {ncell, ncell, ncell, nface, nface};
      double *dev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
      for (int k = 0; k < 5; ++k) {
        if (!src[k]) continue;
        CMCG_TRY(tmp.alloc_n(len[k], &dev[k], s));
        CMCG_HIP(hipMemcpyAsync(dev[k], src[k], len[k] * sizeof(double), hipMemcpyHostToDevice, s));
      }
      const size_t off = (size_t)j * fs;
      hipLaunchKernelGGL((f1_setup_kernel<double>), dim3(grid_for(fs)), dim3(256), 0, s, g, dev[0],
                         P->c_const, dev[1], dev[2], dev[3], dev[4], tp<double>(hi.cc),
                         tp<double>(hi.Fre) + off, hi.Fim ? tp<double>(hi.Fim) + off : nullptr, fs);
      CMCG_HIP(hipGetLastError());
      if (mixed) {
        hipLaunchKernelGGL((f1_setup_kernel<float>), dim3(grid_for(fs)), dim3(256), 0, s, g,
                           dev[0], P->c_const, dev[1], dev[2], dev[3], dev[4], tp<float>(lo.cc),
                           tp<float>(lo.Fre) + off, lo.Fim ? tp<float>(lo.Fim) + off : nullptr, fs);
        CMCG_HIP(hipGetLastError());
      }
      CMCG_HIP(hipStreamSynchronize(s));
    }
    return CMCG_OK;
  }

  // Dirichlet cells: the mask in the device layout and its box, and the data fields of v
  cmcg_status setup_dirichlet(const cmcg_problem *P, const std::vector<cmcg_shot> &shots) {
    const int nx = g.nx, ny = g.ny, J = (int)shots.size();
    int lo[2] = {1 << 30, 1 << 30}, hi2[2] = {-1, -1};
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        if (P->sound_soft[(size_t)j * nx + i]) {
          lo[0] = std::min(lo[0], i), hi2[0] = std::max(hi2[0], i);
          lo[1] = std::min(lo[1], j), hi2[1] = std::max(hi2[1], j);
        }
    if (hi2[0] < 0) return CMCG_OK;          // an empty mask
    CMCG_TRY(arena.alloc_n(fs, &mask, s));
    CMCG_HIP(hipMemcpy2DAsync(mask, g.pitch, P->sound_soft, nx, nx, ny, hipMemcpyHostToDevice, s));
    g.mask = mask;
    for (int a = 0; a < 2; ++a) {
      g.mlo[a] = lo[a];
      g.mhi[a] = hi2[a];
    }
    bool has_d = false;
    for (const cmcg_shot &sh : shots) has_d = has_d || sh.gD_re || sh.gD_im;
    if (has_d) {
      std::vector<double> hre((size_t)J * fs, 0.0), him((size_t)J * fs, 0.0);
      for (int c = 0; c < J; ++c) {
        const double w = cfg.omega_of(c);
        for (int j = 0; j < ny; ++j)
          for (int i = 0; i < nx; ++i) {
            const size_t u = (size_t)j * nx + i, o = (size_t)c * fs + (size_t)j * g.pitch + i;
            if (!P->sound_soft[u]) continue;
            const double gr = shots[c].gD_re ? shots[c].gD_re[u] : 0.0;
            const double gi = shots[c].gD_im ? shots[c].gD_im[u] : 0.0;
            hre[o] = w * gi;
            him[o] = -w * gr;
          }
      }
      CMCG_TRY(arena.alloc_n((size_t)J * fs, &Dre, s));
      CMCG_TRY(arena.alloc_n((size_t)J * fs, &Dim, s));
      CMCG_HIP(hipMemcpyAsync(Dre, hre.data(), hre.size() * sizeof(double), hipMemcpyHostToDevice, s));
      CMCG_HIP(hipMemcpyAsync(Dim, him.data(), him.size() * sizeof(double), hipMemcpyHostToDevice, s));
      if (J > 1) {
        CMCG_TRY(arena.alloc_n(fs, &DA, s));
        CMCG_TRY(arena.alloc_n(fs, &DB, s));
      }
      CMCG_HIP(hipStreamSynchronize(s));
    }
    return CMCG_OK;
  }

  cmcg_status alloc_set(F1Set &b, int prec, bool has_im, int J) {
    const size_t esz = prec == CMCG_FP64 ? sizeof(double) : sizeof(float);
    b.prec = prec;
    CMCG_TRY(arena.alloc(vecN * esz, &b.S0, s));
    CMCG_TRY(arena.alloc(vecN * esz, &b.S1, s));
    CMCG_TRY(arena.alloc(vecN * esz, &b.W, s));
    CMCG_TRY(arena.alloc(vecN * esz, &b.Q, s));
    CMCG_TRY(arena.alloc(fs * esz, &b.cc, s));
    CMCG_TRY(arena.alloc(J * fs * esz, &b.Fre, s));
    if (has_im) CMCG_TRY(arena.alloc(J * fs * esz, &b.Fim, s));
    if (J > 1) CMCG_TRY(arena.alloc(fs * esz, &b.Fk, s));
    return CMCG_OK;
  }

  // ------------------------------------------------------------------ periods
  // Parameters of the launch that advances a period from step n0 (all earlier launches of the
  // period had exactly K steps; the state ping-pongs between S0 and S1; the first launch reads
  // `in`, the last writes `out` - `sub`).  Returns the number of steps of this launch.
  template <typename T>
  int build_launch(const F1Set &b, bool forced, const T *in, T *out, const T *sub, int steps,
                   int n0, int K, bool filter, F1Ptrs<T> *pp, F1Launch *LL) const {
    T *S[2] = {tp<T>(b.S0), tp<T>(b.S1)};
    // a period of `steps` steps runs in launches of K steps; the remainder, if any, opens it, so
    // that the last launch (which also reads the subtrahend) advances a full K steps
    const int first_ns = (steps % K) ? steps % K : std::min(K, steps);
    const int ns = (n0 == 0) ? first_ns : std::min(K, steps - n0);
    const int l = (n0 == 0) ? 0 : 1 + (n0 - first_ns) / K;   // launch index (buffer ping-pong)
    const bool lastl = (n0 + ns == steps);
    F1Launch L{};
    L.nsteps = ns;
    L.first = (n0 == 0);
    L.last = lastl;
    L.forced = forced ? 1 : 0;
    // several components: forced launches take one step each and read the field that
    // `combine` writes for it (weight 1); the filter sums run in `f1_accumulate_kernel`
    L.accumulate = (filter && !multi) ? 1 : 0;
    const double w0 = cfg.omega_of(0);
    for (int k = 0; k < ns; ++k) {
      const double t = (n0 + k + 0.5) * cfg.dt;      // source at t_{n+1/2}
      const double amp = transient(t_offset + t, t_tr);
      L.cs[k] = multi ? 1.0 : amp * std::cos(w0 * t);
      L.sn[k] = multi ? 0.0 : amp * std::sin(w0 * t);
    }
    L.fcos = std::cos(w0 * n0 * cfg.dt);              // filter weight at t_n
    L.fsin = std::sin(w0 * n0 * cfg.dt);
    // Dirichlet cells: the data at the launch's input time t_n0 (k = 0) and at each level's
    // output time t_{n0+k}; several components read DB (output) and DA (input) with weights
    // (1, 0) and (0, 1)
    for (int k = 0; k <= ns; ++k) {
      const double t = (n0 + k) * cfg.dt, amp = transient(t_offset + t, t_tr);
      L.dc[k] = multi ? (k == 0 ? 0.0 : 1.0) : amp * std::cos(w0 * t);
      L.ds[k] = multi ? (k == 0 ? 1.0 : 0.0) : amp * std::sin(w0 * t);
    }
    F1Ptrs<T> p{};
    p.in = (l == 0) ? in : S[(l - 1) & 1];
    p.out = lastl ? out : S[l & 1];
    p.sub = lastl ? sub : nullptr;
    p.cc = tp<T>(b.cc);
    p.fre = multi ? tp<T>(b.Fk) : tp<T>(b.Fre);
    p.fim = multi ? nullptr : tp<T>(b.Fim);
    p.ure = Ure;
    p.uim = Uim;
    p.fs = fs;
    if (forced && Dre) {
      p.dre = multi ? DB : Dre;
      p.dim = multi ? DA : Dim;
    }
    *pp = p;
    *LL = L;
    return ns;
  }

  // Compulsory HBM bytes of one launch: the input state (3 fields) and kap read, the output
  // state (3 fields) written, plus the subtrahend, the source fields and the filter's FP64
  // accumulators (read and written) when the launch uses them
  template <typename T>
  double launch_bytes(const F1Ptrs<T> &p, const F1Launch &L) const {
    const double words = 7.0 + (p.sub ? 3.0 : 0.0) + (L.forced ? (p.fim ? 2.0 : 1.0) : 0.0);
    return (words * sizeof(T) + (L.accumulate ? 32.0 : 0.0)) * g.nx * g.ny;
  }

  // Weights of the components' Dirichlet data at t_n (ramped)
  ShotWeights dirichlet_weights(int n) const {
    ShotWeights w;
    w.nshots = cfg.nshots;
    const double t = n * cfg.dt, amp = transient(t_offset + t, t_tr);
    for (int j = 0; j < cfg.nshots; ++j) {
      w.c[j] = amp * std::cos(cfg.omega_of(j) * t);
      w.s[j] = amp * std::sin(cfg.omega_of(j) * t);
    }
    return w;
  }

  // Weights of the components at step n: the source at t_{n+1/2} (ramped) if `source`, else
  // the filter weight at t_n.
  ShotWeights shot_weights(int n, bool source) const {
    ShotWeights w;
    w.nshots = cfg.nshots;
    const double t = source ? (n + 0.5) * cfg.dt : n * cfg.dt;
    const double amp = source ? transient(t_offset + t, t_tr) : 1.0;
    for (int j = 0; j < cfg.nshots; ++j) {
      w.c[j] = amp * std::cos(cfg.omega_of(j) * t);
      w.s[j] = amp * std::sin(cfg.omega_of(j) * t);
    }
    return w;
  }

  // u = i V / (m omega) with V = (2/N) (Ure + i Uim) for each component, staged in `stage` (two
  // fields) and copied to the caller's n_fields output fields
  cmcg_status output_fields(double *stage, double *u_re, double *u_im) {
    double *ore = stage, *oim = stage + fs;
    const size_t row = (size_t)g.nx * sizeof(double), pitchb = (size_t)g.pitch * sizeof(double);
    const size_t flen = (size_t)g.nx * g.ny;
    for (int j = 0; j < cfg.nshots; ++j) {
      hipLaunchKernelGGL(f1_output_kernel, dim3(grid_for(fs)), dim3(256), 0, s, Ure + j * fs,
                         Uim + j * fs, 2.0 / (cfg.N * cfg.omega_of(j)), ore, oim, fs);
      CMCG_HIP(hipGetLastError());
      if (u_re)
        CMCG_HIP(hipMemcpy2DAsync(u_re + j * flen, row, ore, pitchb, row, g.ny, hipMemcpyDefault, s));
      if (u_im)
        CMCG_HIP(hipMemcpy2DAsync(u_im + j * flen, row, oim, pitchb, row, g.ny, hipMemcpyDefault, s));
    }
    return CMCG_OK;
  }

  template <typename T>
  cmcg_status period_t(const F1Set &b, bool adjoint, bool forced, const T *in, T *out, const T *sub,
                       int steps, bool filter) {
    // the filter accumulates every step's state, and a multi-frequency source is summed per
    // step: such periods take one step per launch
    const int K = (filter || (multi && forced)) ? 1 : cfg.kblock;
    if (multi && filter && !std::is_same<T, double>::value)
      return set_error("the filter period runs in FP64"), CMCG_EINVAL;
    long long mids = 0;
    for (int n0 = 0; n0 < steps;) {
      F1Ptrs<T> p;
      F1Launch L;
      const int ns = build_launch<T>(b, forced, in, out, sub, steps, n0, K, filter, &p, &L);
      dram += launch_bytes<T>(p, L);
      // the bulk of a period: its launches between the first and the last, all of K steps
      const bool mid = bulk_dir >= 0 && !L.first && !L.last;
      if (mid && mids == 0) CMCG_TRY(bulk.begin(bulk_dir, s));
      if (multi && forced) {
        hipLaunchKernelGGL((f1_combine_kernel<T>), dim3(grid_for(fs)), dim3(256), 0, s,
                           tpc<T>(b.Fre), tpc<T>(b.Fim), shot_weights(n0, true), tp<T>(b.Fk),
                           Dre, Dim, dirichlet_weights(n0), dirichlet_weights(n0 + 1), DA, DB,
                           fs);
        CMCG_HIP(hipGetLastError());
      }
      if (multi && filter) {
        // v^n of the launch's input state (the data on the Dirichlet cells)
        hipLaunchKernelGGL(f1_accumulate_kernel, dim3(grid_for(fs)), dim3(256), 0, s,
                           reinterpret_cast<const double *>(p.in) + 2 * fs, mask, DA,
                           shot_weights(n0, false), Ure, Uim, fs);
        CMCG_HIP(hipGetLastError());
      }
      CMCG_HIP(adjoint ? f1_adjoint_launch<T>(g, p, L, K, s) : f1_forward_launch<T>(g, p, L, K, s));
      if (mid) {
        ++mids;
        if (steps - (n0 + ns) <= K) CMCG_TRY(bulk.end(bulk_dir, mids, s));   // next is the last
      }
      n0 += ns;
    }
    updates += (double)steps * g.nx * g.ny;
    return CMCG_OK;
  }

  cmcg_status period(const F1Set &b, bool adjoint, bool forced, const void *in, void *out,
                     const void *sub, int steps, bool filter) {
    if (b.prec == CMCG_FP64)
      return period_t<double>(b, adjoint, forced, tpc<double>(in), tp<double>(out),
                              tpc<double>(sub), steps, filter);
    return period_t<float>(b, adjoint, forced, tpc<float>(in), tp<float>(out), tpc<float>(sub),
                           steps, filter);
  }

  cmcg_status dot_to(const F1Set &b, const void *x, const void *y, int mode) {
    // <x, y>_E with x, y in the precision of set b
    if (b.prec == CMCG_FP64)
      CMCG_HIP(f1_dot<double, double>(g, tpc<double>(x), tpc<double>(y), b.cc, 1, fs, partials, s));
    else
      CMCG_HIP(f1_dot<float, float>(g, tpc<float>(x), tpc<float>(y), b.cc, 0, fs, partials, s));
    CMCG_HIP(finalize(partials, kRedBlocks, scalars, mode, 0, s));
    return CMCG_OK;
  }

  cmcg_status read_scalars() {
    CMCG_HIP(hipMemcpyAsync(h_scalars, scalars, kNumScalars * sizeof(double),
                            hipMemcpyDeviceToHost, s));
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  // r = E*(Phi(z) - z) - (Phi(z) - z) at the FP64 iterate, with FP64 periods (Steps 2-3)
  cmcg_status true_gradient(int mode) {
    CMCG_TRY(period(hi, false, true, Z, hi.W, Z, cfg.N, false));
    CMCG_TRY(period(hi, true, false, hi.W, hi.Q, hi.W, cfg.N, false));
    CMCG_HIP(hipMemcpyAsync(R, hi.Q, vecN * sizeof(double), hipMemcpyDeviceToDevice, s));
    CMCG_HIP(f1_dot<double, double>(g, R, R, hi.cc, 1, fs, partials, s));
    CMCG_HIP(finalize(partials, kRedBlocks, scalars, mode, 0, s));
    return CMCG_OK;
  }

  // ------------------------------------------------------------------ CG driver
  // The forced scheme from rest over `periods` periods (FP64), the source ramped by Mur's
  // transient over the whole interval if `ramp`; the final state goes to `state` (FP64 device
  // layout).  Uses hi.W and hi.Q as the two state buffers.
  cmcg_status run_forced_periods(int periods, bool ramp, double *state) {
    double *a = tp<double>(hi.Q), *b = tp<double>(hi.W);
    CMCG_HIP(hipMemsetAsync(a, 0, vecN * sizeof(double), s));
    t_tr = ramp ? periods * cfg.T : 0.0;
    for (int p = 0; p < periods; ++p) {
      t_offset = p * cfg.T;
      const cmcg_status st = period(hi, false, true, a, b, nullptr, cfg.N, false);
      if (st != CMCG_OK) {
        t_offset = t_tr = 0.0;
        return st;
      }
      std::swap(a, b);
    }
    t_offset = t_tr = 0.0;
    CMCG_HIP(hipMemcpyAsync(state, a, vecN * sizeof(double), hipMemcpyDeviceToDevice, s));
    return CMCG_OK;
  }

  cmcg_status begin() override {
    if (fixed) return set_error("a fixed-buffer solver serves stage calls only"), CMCG_EUNSUPPORTED;
    t_fwd = t_adj = t_other = t_total = t_runup = 0.0;
    updates = 0;
    dram = 0;
    bulk.reset();
    iter = refreshes = last_refresh = runup_done = 0;
    CMCG_HIP(hipEventRecord(ev[0], s));
    // Steps 1-4: z = 0, gradient, r = d = gradient (the Riesz map M_E^{-1} is built into E*)
    CMCG_HIP(hipMemsetAsync(Z, 0, vecN * sizeof(double), s));
    CMCG_TRY(true_gradient(kFinStart));
    if (cfg.runup > 0) {
      // start from the run-up state; delta0 stays the residual at rest (stopping reference)
      CMCG_HIP(hipEventRecord(ev[8], s));
      CMCG_TRY(run_forced_periods(cfg.runup, true, Z));
      CMCG_HIP(hipEventRecord(ev[9], s));
      CMCG_HIP(hipMemcpyAsync(scalars + kTmp, scalars + kDelta, sizeof(double),
                              hipMemcpyDeviceToDevice, s));
      CMCG_TRY(true_gradient(kFinRefresh));
      runup_done = cfg.runup;
    }
    if (mixed) CMCG_HIP(convert<float, double>(tp<float>(D), R, vecN, s));
    else CMCG_HIP(hipMemcpyAsync(D, R, vecN * sizeof(double), hipMemcpyDeviceToDevice, s));
    CMCG_HIP(hipEventRecord(ev[1], s));
    CMCG_TRY(read_scalars());
    t_other += PhaseEvents::seconds(ev[0], ev[1]);
    if (runup_done) {
      t_runup = PhaseEvents::seconds(ev[8], ev[9]);
      t_other -= t_runup;
    }
    rel = h_scalars[kRel];
    delta_at_refresh = h_scalars[kDelta];
    started = true;
    if (h_scalars[kBreak] != 0.0) return set_error("non-finite initial gradient"), CMCG_EBREAKDOWN;
    return CMCG_OK;
  }

  cmcg_status iterate(int iters, int *converged) override {
    if (!started) return set_error("cmcg_begin first"), CMCG_EINVAL;
    *converged = (rel <= cfg.tol || h_scalars[kDelta0] == 0.0) ? 1 : 0;
    for (int it = 0; it < iters && !*converged; ++it) {
      CMCG_HIP(hipEventRecord(ev[2], s));
      // Step 5.1: w = E d - d (forward), q = E* w - w (backward)
      bulk_dir = 0;
      cmcg_status st = period(lo, false, false, D, lo.W, D, cfg.N, false);
      CMCG_HIP(hipEventRecord(ev[3], s));
      bulk_dir = 1;
      if (st == CMCG_OK) st = period(lo, true, false, lo.W, lo.Q, lo.W, cfg.N, false);
      bulk_dir = -1;
      CMCG_TRY(st);
      CMCG_HIP(hipEventRecord(ev[4], s));
      // Step 5.3: alpha = delta / <q, d>_E
      CMCG_TRY(dot_to(lo, lo.Q, D, kFinAlpha));
      // Steps 5.4-5.5 and delta' = <r, r>_E; beta = delta' / delta
      if (mixed)
        CMCG_HIP(f1_cg_update<float>(g, Z, R, tpc<float>(D), tpc<float>(lo.Q), lo.cc, fs, scalars,
                                     partials, s));
      else
        CMCG_HIP(f1_cg_update<double>(g, Z, R, tpc<double>(D), tpc<double>(lo.Q), lo.cc, fs,
                                      scalars, partials, s));
      CMCG_HIP(finalize(partials, kRedBlocks, scalars, kFinBeta, 0, s));
      CMCG_HIP(hipEventRecord(ev[5], s));
      CMCG_TRY(read_scalars());
      bulk.collect();
      t_fwd += PhaseEvents::seconds(ev[2], ev[3]);
      t_adj += PhaseEvents::seconds(ev[3], ev[4]);
      t_other += PhaseEvents::seconds(ev[4], ev[5]);
      ++iter;
      if (h_scalars[kBreak] != 0.0)
        return set_error("CG breakdown: <qhat, d> <= 0 or non-finite scalar"), CMCG_EBREAKDOWN;
      rel = h_scalars[kRel];
      if (mixed && cfg.refresh > 0.0 &&
          (rel <= cfg.tol || h_scalars[kDelta] <= cfg.refresh * cfg.refresh * delta_at_refresh)) {
        // reliable update: replace the recursive residual by the true FP64 gradient
        CMCG_HIP(hipEventRecord(ev[6], s));
        CMCG_TRY(true_gradient(kFinRefresh));
        CMCG_HIP(hipEventRecord(ev[7], s));
        CMCG_TRY(read_scalars());
        t_other += PhaseEvents::seconds(ev[6], ev[7]);
        rel = h_scalars[kRel];
        delta_at_refresh = h_scalars[kDelta];
        ++refreshes;
        last_refresh = iter;
      }
      // Step 5.8
      if (rel <= cfg.tol) {
        *converged = 1;
        break;
      }
      // Step 5.7: d = r + beta d
      if (mixed) CMCG_HIP(direction_update<float>(tp<float>(D), R, scalars, vecN, s));
      else CMCG_HIP(direction_update<double>(tp<double>(D), R, scalars, vecN, s));
    }
    return CMCG_OK;
  }

  cmcg_status filter_from_hi(const double *z, double *u_re, double *u_im) {
    CMCG_HIP(hipMemsetAsync(Ure, 0, cfg.nshots * fs * sizeof(double), s));
    CMCG_HIP(hipMemsetAsync(Uim, 0, cfg.nshots * fs * sizeof(double), s));
    CMCG_TRY(period(hi, false, true, z, hi.Q, nullptr, cfg.N, true));
    CMCG_HIP(hipEventRecord(ev[6], s));
    CMCG_TRY(output_fields(tp<double>(hi.W), u_re, u_im));
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  cmcg_status finish(double *u_re, double *u_im) override {
    if (!started) return set_error("cmcg_begin first"), CMCG_EINVAL;
    if (cfg.output == CMCG_OUTPUT_STEP6) {
      CMCG_TRY(step6_from(Z, u_re, u_im));
      CMCG_HIP(hipEventRecord(ev[6], s));
      return CMCG_OK;
    }
    // Step 6 through the fundamental-frequency filter: one forced FP64 period from z
    return filter_from_hi(Z, u_re, u_im);
  }

  // u from a device-layout FP64 state (eq. mix_solution), staged in hi.S1
  cmcg_status step6_from(const double *zdev, double *u_re, double *u_im) {
    if (cfg.nshots > 1)
      return set_error("the Step 6 output reads one frequency off the state: no shots"),
             CMCG_EINVAL;
    double *ore = tp<double>(hi.S1), *oim = tp<double>(hi.S1) + fs;
    hipLaunchKernelGGL(f1_step6_kernel, dim3(grid_for(fs)), dim3(256), 0, s, g, zdev,
                       tpc<double>(hi.cc), tpc<double>(hi.Fre), tpc<double>(hi.Fim), Dre, Dim,
                       0.5 * cfg.omega_of(0) * cfg.dt, cfg.omega_of(0), ore, oim, fs);
    CMCG_HIP(hipGetLastError());
    const size_t row = (size_t)g.nx * sizeof(double), pitchb = (size_t)g.pitch * sizeof(double);
    if (u_re) CMCG_HIP(hipMemcpy2DAsync(u_re, row, ore, pitchb, row, g.ny, hipMemcpyDefault, s));
    if (u_im) CMCG_HIP(hipMemcpy2DAsync(u_im, row, oim, pitchb, row, g.ny, hipMemcpyDefault, s));
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  cmcg_status step6(const double *z, double *u_re, double *u_im) override {
    CMCG_HIP(f1_unpack<double>(g, z, tp<double>(hi.W), fs, s));
    return step6_from(tp<double>(hi.W), u_re, u_im);
  }

  cmcg_status solve(double *u_re, double *u_im) override {
    CMCG_TRY(begin());
    int conv = 0;
    CMCG_TRY(iterate(cfg.max_iter, &conv));
    CMCG_HIP(hipEventRecord(ev[7], s));
    CMCG_TRY(finish(u_re, u_im));
    t_other += PhaseEvents::seconds(ev[7], ev[6]);
    t_total = PhaseEvents::seconds(ev[0], ev[6]);
    return conv ? CMCG_OK : CMCG_ENOTCONV;
  }

  // ------------------------------------------------------------------ stage calls
  cmcg_status apply(int op, int steps, const double *in, double *out) override {
    const int ns = steps > 0 ? steps : cfg.N;
    void *W = lo.W, *Q = lo.Q;
    if (lo.prec == CMCG_FP64) CMCG_HIP(f1_unpack<double>(g, in, tp<double>(W), fs, s));
    else CMCG_HIP(f1_unpack<float>(g, in, tp<float>(W), fs, s));
    if (op == CMCG_OP_FORWARD || op == CMCG_OP_FORCED) {
      CMCG_TRY(period(lo, false, op == CMCG_OP_FORCED, W, Q, nullptr, ns, false));
    } else if (op == CMCG_OP_ADJOINT) {
      CMCG_TRY(period(lo, true, false, W, Q, nullptr, ns, false));
    } else {
      if (lo.prec == CMCG_FP64)
        hipLaunchKernelGGL((f1_riesz_kernel<double>), dim3(grid_for(fs)), dim3(256), 0, s, g,
                           tp<double>(W), tp<double>(lo.cc), fs);
      else
        hipLaunchKernelGGL((f1_riesz_kernel<float>), dim3(grid_for(fs)), dim3(256), 0, s, g,
                           tp<float>(W), tp<float>(lo.cc), fs);
      CMCG_HIP(hipGetLastError());
      Q = W;
    }
    if (lo.prec == CMCG_FP64) CMCG_HIP(f1_pack<double>(g, tp<double>(Q), out, fs, s));
    else CMCG_HIP(f1_pack<float>(g, tp<float>(Q), out, fs, s));
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  cmcg_status filter(const double *z, double *u_re, double *u_im) override {
    // the period reads its input only in its first launch and never writes hi.W
    CMCG_HIP(f1_unpack<double>(g, z, tp<double>(hi.W), fs, s));
    CMCG_HIP(hipMemsetAsync(Ure, 0, cfg.nshots * fs * sizeof(double), s));
    CMCG_HIP(hipMemsetAsync(Uim, 0, cfg.nshots * fs * sizeof(double), s));
    CMCG_TRY(period(hi, false, true, hi.W, hi.Q, nullptr, cfg.N, true));
    CMCG_TRY(output_fields(tp<double>(hi.S1), u_re, u_im));
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  cmcg_status get_state(int which, double *out) override {
    if (which == 0) CMCG_HIP(f1_pack<double>(g, Z, out, fs, s));
    else if (which == 1) CMCG_HIP(f1_pack<double>(g, R, out, fs, s));
    else if (mixed) CMCG_HIP(f1_pack<float>(g, tp<float>(D), out, fs, s));
    else CMCG_HIP(f1_pack<double>(g, tp<double>(D), out, fs, s));
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  cmcg_status runup(int periods, int ramp, double *z_out) override {
    CMCG_TRY(run_forced_periods(periods, ramp != 0, tp<double>(hi.W)));
    CMCG_HIP(f1_pack<double>(g, tp<double>(hi.W), z_out, fs, s));
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  cmcg_status misfit(const double *z, double *J) override {
    // w = Phi(z) - z with one FP64 forced period; J = <w, w>_E / 2
    double *a = tp<double>(hi.Q), *w = tp<double>(hi.W);
    CMCG_HIP(f1_unpack<double>(g, z, a, fs, s));
    CMCG_TRY(period(hi, false, true, a, w, a, cfg.N, false));
    CMCG_HIP(f1_dot<double, double>(g, w, w, hi.cc, 1, fs, partials, s));
    CMCG_HIP(finalize(partials, kRedBlocks, scalars, kFinStore, kMisfit, s));
    CMCG_TRY(read_scalars());
    *J = 0.5 * h_scalars[kMisfit];
    return CMCG_OK;
  }

  void report(cmcg_report *r) const override {
    r->iterations = iter;
    r->steps_per_period = cfg.N;
    r->dt = cfg.dt;
    r->rel_residual = rel;
    r->seconds = t_total;
    r->seconds_fwd = t_fwd;
    r->seconds_adj = t_adj;
    r->seconds_riesz = 0.0;
    r->seconds_other = t_other;
    r->grid_updates = updates;
    r->dram_bytes = dram;
    r->riesz_iterations = 0;
    r->riesz_unconverged = 0;
    r->seconds_bulk_fwd = bulk.seconds[0];
    r->seconds_bulk_adj = bulk.seconds[1];
    r->bulk_launches_fwd = bulk.launches[0];
    r->bulk_launches_adj = bulk.launches[1];
    r->fp64_refreshes = refreshes;
    r->runup_periods = runup_done;
    r->seconds_runup = t_runup;
  }

  void info(cmcg_info *i) const override {
    const int64_t nx = g.nx, ny = g.ny;
    i->steps_per_period = cfg.N;
    i->dt = cfg.dt;
    i->T = cfg.T;
    i->h = cfg.h;
    i->state_len = ny * (nx - 1) + (ny - 1) * nx + nx * ny;
    i->field_len = nx * ny;
    i->device_bytes = (int64_t)arena.bytes();
    i->n_fields = cfg.nshots;
    i->steps_per_launch = cfg.kblock;
  }
};

}  // namespace

cmcg_status make_f1_solver(const cmcg_problem *P, const SolverConfig &cfg, Solver **out) {
  *out = nullptr;
  F1Solver *S = new F1Solver();
  S->cfg = cfg;
  cmcg_status st = S->create(P);
  if (st != CMCG_OK) {
    delete S;
    return st;
  }
  *out = S;
  return CMCG_OK;
}

cmcg_status make_f1_solver_in(const cmcg_problem *P, const SolverConfig &cfg, void *base,
                              size_t cap, Solver **out) {
  *out = nullptr;
  F1Solver *S = new F1Solver();
  S->cfg = cfg;
  S->fixed = true;
  S->arena.use_buffer(base, cap);
  cmcg_status st = S->create(P);
  if (st != CMCG_OK) {
    delete S;
    return st;
  }
  *out = S;
  return CMCG_OK;
}


// =========================================================================================
// Continuous-batching server for first-order solves.
//
// Requests are admitted in arrival order while the sum of their device footprints stays within
// the HBM budget and the slot cap; each admitted solve keeps its whole CG state resident in its
// own buffers.  One server tick is ONE launch of the persistent serving kernel (f1_serve.hip):
// it advances every running solve through rounds of its CG algorithm, one operation per solve
// per round (a period launch, a vector pass, a reduction, a decision), the decisions taken on
// the device from each solve's own scalars, until a work budget is spent or every solve has
// finished.  The host then copies out finished results and admits queued requests.  A solve's
// arithmetic does not depend on what else is resident: the kernel runs the standalone path's
// tiles and vector passes on its buffers, with the same launch parameters.
// =========================================================================================
namespace {

size_t f1_footprint(int nx, int ny, int prec, bool has_im, int N) {
  const size_t pitch = (size_t)(nx + 63) / 64 * 64, fs = (size_t)ny * pitch, vecN = 3 * fs;
  auto r8 = [](size_t b) { return b == 0 ? 8 : b; };
  size_t total = 0;
  auto set = [&](size_t esz) {
    total += 4 * r8(vecN * esz) + 2 * r8(fs * esz) + (has_im ? r8(fs * esz) : 0);
  };
  set(8);
  if (prec == CMCG_FP32_MIXED) set(4);
  total += r8(vecN * (prec == CMCG_FP32_MIXED ? 4 : 8));
  total += 2 * r8(vecN * 8) + 2 * r8(fs * 8);
  total += r8(kRedBlocks * 8) + r8(kNumScalars * 8);
  total += r8((size_t)N * 4 * 8);    // the launch-parameter table of the serving kernel
  return total;
}

struct ServeRequest {
  int64_t id = 0;
  int state = 0;                 // 0 queued, 1 running, 2 done, -1 failed
  cmcg_problem P{};
  cmcg_options O{};
  std::vector<double> c, fre, fim, gre, gim;
  size_t footprint = 0;
  F1Solver *S = nullptr;
  DeviceArena extra;             // the serving kernel's launch-parameter table
  ServeSlot slot{};
  serve::State st{};
  cmcg_status status = CMCG_OK;
  std::vector<double> ure, uim;
  cmcg_report rep{};
};

// Steps per launch of a served period: one of the serving kernel's launch sizes, at most the
// requested K (FP32 7, 4, 2, 1; FP64 4, 2, 1).  Results do not depend on it.
int served_K(int k, bool fp64) {
  int K = k > 0 ? k : 7;
  if (fp64 && K > 4) K = 4;
  return K >= 7 ? 7 : K >= 4 ? 4 : K >= 2 ? 2 : 1;
}

class F1Server final : public Server {
 public:
  int64_t budget = 0;
  int max_slots = 16, kblock = 0, device = 0;
  unsigned long long spin_limit = 1ull << 24;
  hipStream_t s = nullptr;
  std::map<int64_t, ServeRequest *> reqs;
  std::deque<int64_t> queue;
  std::vector<int64_t> active;
  size_t used = 0;
  int64_t next_id = 1;
  int64_t ticks = 0, launches = 0, rounds = 0;
  int grid = 0;
  // device slot table, states and control block of the serving kernel, their pinned staging
  // buffers, and the host-settable abort flag the kernel's waits watch
  ServeSlot *d_slots = nullptr, *h_slots = nullptr;
  serve::State *d_states = nullptr, *h_states = nullptr;
  ServeControl *d_ctl = nullptr, *h_ctl = nullptr;
  int *h_abort = nullptr;
  // per tick: rounds and grid-point updates of the last launch
  static constexpr int kMaxRounds = 1 << 16;
  static constexpr double kTickUpdates = 1.0e10;

  ~F1Server() override {
    if (s) (void)hipStreamSynchronize(s);
    for (auto &kv : reqs) {
      delete kv.second->S;
      delete kv.second;
    }
    if (d_slots) (void)hipFree(d_slots);
    if (d_states) (void)hipFree(d_states);
    if (d_ctl) (void)hipFree(d_ctl);
    if (h_slots) (void)hipHostFree(h_slots);
    if (h_states) (void)hipHostFree(h_states);
    if (h_ctl) (void)hipHostFree(h_ctl);
    if (h_abort) (void)hipHostFree(h_abort);
  }

  cmcg_status init() {
    CMCG_HIP(hipSetDevice(device));
    CMCG_HIP(hipMalloc((void **)&d_slots, kServeMaxSlots * sizeof(ServeSlot)));
    CMCG_HIP(hipMalloc((void **)&d_states, kServeMaxSlots * sizeof(serve::State)));
    CMCG_HIP(hipMalloc((void **)&d_ctl, sizeof(ServeControl)));
    CMCG_HIP(hipHostMalloc((void **)&h_slots, kServeMaxSlots * sizeof(ServeSlot)));
    CMCG_HIP(hipHostMalloc((void **)&h_states, kServeMaxSlots * sizeof(serve::State)));
    CMCG_HIP(hipHostMalloc((void **)&h_ctl, sizeof(ServeControl)));
    CMCG_HIP(hipHostMalloc((void **)&h_abort, sizeof(int)));
    *h_abort = 0;
    CMCG_HIP(f1_serve_grid(&grid));
    if (max_slots > kServeMaxSlots) max_slots = kServeMaxSlots;
    return CMCG_OK;
  }

  cmcg_status submit(const cmcg_problem *P, const cmcg_options *O, int64_t *id) override {
    if (!P || !O || !id) return set_error("null argument"), CMCG_EINVAL;
    CMCG_TRY(validate_problem(P, O));
    if (P->formulation != 1 || P->dim != 2)
      return set_error("the server batches first-order 2D solves"), CMCG_EUNSUPPORTED;
    if (O->runup_periods > 0)
      return set_error("the server starts every solve from rest (runup_periods must be 0)"),
             CMCG_EUNSUPPORTED;
    if (P->n_shots > 0)
      return set_error("the server takes single-frequency sources (n_shots must be 0)"),
             CMCG_EUNSUPPORTED;
    if (O->output != CMCG_OUTPUT_FILTER)
      return set_error("served solves return the filter output"), CMCG_EUNSUPPORTED;
    if (P->sound_soft)
      return set_error("served solves have no Dirichlet cells"), CMCG_EUNSUPPORTED;
    SolverConfig cfg;
    CMCG_TRY(make_config(P, O, s, &cfg));
    auto *R = new ServeRequest();
    R->id = next_id++;
    R->P = *P;
    R->O = *O;
    const size_t ncell = (size_t)P->n[0] * P->n[1], nface = 2 * (size_t)(P->n[0] + P->n[1]);
    auto keep = [](const double *src, size_t n, std::vector<double> &dst) -> const double * {
      if (!src) return nullptr;
      dst.assign(src, src + n);
      return dst.data();
    };
    R->P.c = keep(P->c, ncell, R->c);
    R->P.f_re = keep(P->f_re, ncell, R->fre);
    R->P.f_im = keep(P->f_im, ncell, R->fim);
    R->P.gS_re = keep(P->gS_re, nface, R->gre);
    R->P.gS_im = keep(P->gS_im, nface, R->gim);
    R->P.sound_soft = nullptr;
    R->O.hip_stream = nullptr;
    R->O.steps_per_launch = O->steps_per_launch > 0 ? O->steps_per_launch : kblock;
    R->footprint = f1_footprint((int)P->n[0], (int)P->n[1], O->precision,
                                P->f_im != nullptr || P->gS_im != nullptr, cfg.N);
    if ((int64_t)R->footprint > budget) {
      delete R;
      return set_error("request larger than the server's HBM budget"), CMCG_ENOMEM;
    }
    reqs[R->id] = R;
    queue.push_back(R->id);
    *id = R->id;
    return CMCG_OK;
  }

  // The serving kernel's view of an admitted solve, and its start state (Step 1: z = 0)
  cmcg_status make_slot(ServeRequest *R) {
    F1Solver *S = R->S;
    const SolverConfig &cfg = S->cfg;
    ServeSlot &sl = R->slot;
    sl = ServeSlot{};
    sl.g = S->g;
    sl.fs = S->fs;
    sl.vecN = S->vecN;
    int nbx, nby, band;
    f1_launch_shape(S->g.nx, S->g.ny, 1, &nbx, &nby, &band);
    sl.band = band;
    sl.N = cfg.N;
    sl.mixed = S->mixed ? 1 : 0;
    sl.K_lo = served_K(cfg.kblock, !S->mixed);
    sl.K_hi = served_K(cfg.kblock, true);
    sl.max_iter = cfg.max_iter;
    sl.tol = cfg.tol;
    sl.refresh = cfg.refresh;
    sl.out_scale = 2.0 / (cfg.N * cfg.omega_of(0));
    sl.lo_S0 = S->lo.S0;
    sl.lo_S1 = S->lo.S1;
    sl.lo_W = S->lo.W;
    sl.lo_Q = S->lo.Q;
    sl.lo_cc = S->lo.cc;
    sl.lo_Fre = S->lo.Fre;
    sl.lo_Fim = S->lo.Fim;
    sl.hi_S0 = tp<double>(S->hi.S0);
    sl.hi_S1 = tp<double>(S->hi.S1);
    sl.hi_W = tp<double>(S->hi.W);
    sl.hi_Q = tp<double>(S->hi.Q);
    sl.hi_cc = tp<double>(S->hi.cc);
    sl.hi_Fre = tp<double>(S->hi.Fre);
    sl.hi_Fim = tp<double>(S->hi.Fim);
    sl.D = S->D;
    sl.Z = S->Z;
    sl.R = S->R;
    sl.Ure = S->Ure;
    sl.Uim = S->Uim;
    sl.partials = S->partials;
    sl.scalars = S->scalars;
    // the launch parameters the standalone period loop computes (no source ramp): the source
    // weights at t_{n+1/2} and the filter weights at t_n
    const int N = cfg.N;
    const double w0 = cfg.omega_of(0);
    std::vector<double> tab((size_t)4 * N);
    for (int n = 0; n < N; ++n) {
      const double t = (n + 0.5) * cfg.dt;
      tab[4 * n] = std::cos(w0 * t);
      tab[4 * n + 1] = std::sin(w0 * t);
      tab[4 * n + 2] = std::cos(w0 * n * cfg.dt);
      tab[4 * n + 3] = std::sin(w0 * n * cfg.dt);
    }
    double *dtab = nullptr;
    CMCG_TRY(R->extra.alloc_n(tab.size(), &dtab, s));
    CMCG_HIP(hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s));
    CMCG_HIP(hipStreamSynchronize(s));
    sl.tab = dtab;
    R->st = serve::State{};
    R->st.active = 1;
    R->st.phase = serve::kGradFwd;
    R->st.grad_mode = serve::kModeStart;
    return CMCG_OK;
  }

  cmcg_status admit() {
    while (!queue.empty()) {
      ServeRequest *R = reqs[queue.front()];
      if ((int)active.size() >= max_slots || (int64_t)(used + R->footprint) > budget) break;
      queue.pop_front();
      SolverConfig cfg;
      cmcg_status st = make_config(&R->P, &R->O, s, &cfg);
      Solver *base = nullptr;
      if (st == CMCG_OK) st = make_f1_solver(&R->P, cfg, &base);
      if (st != CMCG_OK) {
        R->state = -1;
        R->status = st;
        continue;
      }
      R->S = static_cast<F1Solver *>(base);
      R->state = 1;
      F1Solver *S = R->S;
      CMCG_HIP(hipMemsetAsync(S->Z, 0, S->vecN * sizeof(double), s));
      st = make_slot(R);
      if (st != CMCG_OK) {
        fail(R, st);
        continue;
      }
      used += S->arena.bytes() + R->extra.bytes();
      active.push_back(R->id);
    }
    return CMCG_OK;
  }

  // result of a finished solve: the output field (in the FP64 W buffer) and the report
  cmcg_status complete(ServeRequest *R) {
    F1Solver *S = R->S;
    const serve::State &st = R->st;
    const double *ore = tp<double>(S->hi.W), *oim = tp<double>(S->hi.W) + S->fs;
    const size_t nxy = (size_t)S->g.nx * S->g.ny;
    R->ure.resize(nxy);
    R->uim.resize(nxy);
    const size_t row = (size_t)S->g.nx * sizeof(double), pitchb = (size_t)S->g.pitch * sizeof(double);
    CMCG_HIP(hipMemcpy2DAsync(R->ure.data(), row, ore, pitchb, row, S->g.ny, hipMemcpyDeviceToHost, s));
    CMCG_HIP(hipMemcpy2DAsync(R->uim.data(), row, oim, pitchb, row, S->g.ny, hipMemcpyDeviceToHost, s));
    CMCG_TRY(S->read_scalars());
    S->iter = st.iter;
    S->refreshes = st.refreshes;
    S->updates = st.updates;
    S->dram = st.dram;
    S->rel = S->h_scalars[kRel];
    S->report(&R->rep);
    R->status = st.converged ? CMCG_OK : CMCG_ENOTCONV;
    R->state = 2;
    release(R);
    return CMCG_OK;
  }

  cmcg_status fail(ServeRequest *R, cmcg_status st) {
    R->status = st;
    R->state = -1;
    release(R);
    return CMCG_OK;
  }

  void release(ServeRequest *R) {
    if (!R->S) return;
    (void)hipStreamSynchronize(s);
    used -= R->S->arena.bytes() + R->extra.bytes();
    delete R->S;
    R->S = nullptr;
    R->extra.release();
    active.erase(std::remove(active.begin(), active.end(), R->id), active.end());
  }

  cmcg_status step(int *n_active, int *n_queued) override {
    CMCG_HIP(hipSetDevice(device));
    CMCG_TRY(admit());
    std::vector<ServeRequest *> run;
    for (int64_t id : active) {
      ServeRequest *R = reqs[id];
      if (R->S && R->st.active == 1) run.push_back(R);
    }
    cmcg_status result = CMCG_OK;
    if (!run.empty()) {
      const int n = (int)run.size();
      for (int k = 0; k < n; ++k) {
        h_slots[k] = run[k]->slot;
        h_states[k] = run[k]->st;
      }
      *h_ctl = ServeControl{};
      CMCG_HIP(hipMemcpyAsync(d_slots, h_slots, n * sizeof(ServeSlot), hipMemcpyHostToDevice, s));
      CMCG_HIP(hipMemcpyAsync(d_states, h_states, n * sizeof(serve::State), hipMemcpyHostToDevice, s));
      CMCG_HIP(hipMemcpyAsync(d_ctl, h_ctl, sizeof(ServeControl), hipMemcpyHostToDevice, s));
      CMCG_HIP(f1_serve_launch(d_slots, d_states, n, d_ctl, h_abort, kMaxRounds, kTickUpdates,
                               spin_limit, grid, s));
      ++launches;
      ++ticks;
      CMCG_HIP(hipMemcpyAsync(h_states, d_states, n * sizeof(serve::State), hipMemcpyDeviceToHost, s));
      CMCG_HIP(hipMemcpyAsync(h_ctl, d_ctl, sizeof(ServeControl), hipMemcpyDeviceToHost, s));
      CMCG_HIP(hipStreamSynchronize(s));
      rounds += h_ctl->rounds;
      if (h_ctl->failed) {
        // a barrier wait gave up: the solves' states are not consistent any more
        set_error("serving kernel: a grid barrier wait gave up (spin limit or abort)");
        for (ServeRequest *R : run) fail(R, CMCG_EDEVICE);
        result = CMCG_EDEVICE;
      } else {
        for (int k = 0; k < n; ++k) {
          ServeRequest *R = run[k];
          R->st = h_states[k];
          if (R->st.active == 2) CMCG_TRY(complete(R));
          else if (R->st.active == 3) fail(R, static_cast<cmcg_status>(R->st.status));
        }
      }
    }
    if (n_active) *n_active = (int)run.size();
    if (n_queued) *n_queued = (int)queue.size();
    return result;
  }

  cmcg_status poll(int64_t id, int *state, double *u_re, double *u_im, cmcg_report *rep) override {
    auto it = reqs.find(id);
    if (it == reqs.end()) return set_error("unknown request id"), CMCG_EINVAL;
    ServeRequest *R = it->second;
    *state = R->state;
    if (R->state != 2 && R->state != -1) return CMCG_OK;
    // a finished request is handed over once: its result, copied inputs and id are released
    if (R->state == 2) {
      if (u_re) std::memcpy(u_re, R->ure.data(), R->ure.size() * sizeof(double));
      if (u_im) std::memcpy(u_im, R->uim.data(), R->uim.size() * sizeof(double));
      if (rep) *rep = R->rep;
    }
    const cmcg_status st = R->status;
    delete R->S;
    delete R;
    reqs.erase(it);
    return st;
  }

  void stats(int64_t *used_bytes, int *n_active, int *n_queued) const override {
    *used_bytes = (int64_t)used;
    *n_active = (int)active.size();
    *n_queued = (int)queue.size();
  }

  void counters(int64_t *n_ticks, int64_t *n_launches, int64_t *n_rounds) const override {
    *n_ticks = ticks;
    *n_launches = launches;
    *n_rounds = rounds;
  }
};

}  // namespace

cmcg_status make_f1_server(const cmcg_server_options *o, hipStream_t s, Server **out) {
  *out = nullptr;
  auto *S = new F1Server();
  S->budget = o->hbm_budget_bytes;
  S->max_slots = o->max_slots > 0 ? o->max_slots : 16;
  S->kblock = o->steps_per_launch > 0 ? o->steps_per_launch : 0;   // 0: per-solve default
  S->device = o->device;
  if (o->barrier_spin_limit > 0) S->spin_limit = (unsigned long long)o->barrier_spin_limit;
  S->s = s;
  cmcg_status st = S->init();
  if (st != CMCG_OK) {
    delete S;
    return st;
  }
  *out = S;
  return CMCG_OK;
}

}  // namespace cmcg
