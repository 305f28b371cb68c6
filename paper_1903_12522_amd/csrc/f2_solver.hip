// Second-order (nodal, 3D) solver runtime: memory plan, the forward / backward period sequences,
// the energy metric, the Riesz map, and the CG driver of the CMCG Algorithm (Sec. 2.3, Steps 1-6).
//
// One CG iteration (Step 5):  w = E d - d;  y = M_E w;  qh = E^T y - y  (the literal transpose
// of the discrete period, discretise-then-optimise);  q = P qh with P = blockdiag(S^{-1}, M^{-1})
// (Riesz representer, eq. CMCG_PRECONDITIONIER; with no sound-soft node S^{-1} acts on zero-sum
// vectors);  alpha = delta / <qh, d>;  z -= alpha d, r -= alpha q, rh -= alpha qh;
// delta' = <rh, r>;  beta = delta' / delta;  d = r + beta d.  r_v = M^{-1} rh_v is not stored.
// Precision policy as in the first-order solver: FP32-mixed runs the CG periods in FP32 and
// refreshes the true gradient with FP64 periods (reliable updates); z, residuals, the Riesz solve
// and every reduction are FP64.
#include <type_traits>

#include "f2_internal.h"
#include "solver.h"

namespace cmcg {
namespace {

template <typename T>
T *tp(void *p) { return static_cast<T *>(p); }
template <typename T>
const T *tpc(const void *p) { return static_cast<const T *>(p); }

__global__ void mask_unpack_kernel(F2Geom g, const uint8_t *packed, uint8_t *dev) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < g.fs; o += stride) {
    const int i = (int)(o % g.px);
    const int j = (int)((o / g.px) % (g.ny + 1));
    const int k = (int)(o / g.plane);
    dev[o] = (i <= g.nx) ? packed[((size_t)k * (g.ny + 1) + j) * (g.nx + 1) + i] : 0;
  }
}

// Dirichlet data of the sound-soft nodes: packed user node array -> device layout (zero on the
// other nodes)
__global__ void dirichlet_unpack_kernel(F2Geom g, const double *packed, double *dev) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < g.fs; o += stride) {
    const int i = (int)(o % g.px);
    const int j = (int)((o / g.px) % (g.ny + 1));
    const int k = (int)(o / g.plane);
    double v = 0.0;
    if (i <= g.nx && g.mask[o]) v = packed[((size_t)k * (g.ny + 1) + j) * (g.nx + 1) + i];
    dev[o] = v;
  }
}

// filter output u = (2/N) (Ure + i Uim), copied into a contiguous node array
__global__ void f2_output_kernel(F2Geom g, const double *ure, const double *uim, double scale,
                                 double *ore, double *oim) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < g.fs; o += stride) {
    const int i = (int)(o % g.px);
    if (i > g.nx) continue;
    const int j = (int)((o / g.px) % (g.ny + 1));
    const int k = (int)(o / g.plane);
    const size_t u = ((size_t)k * (g.ny + 1) + j) * (g.nx + 1) + i;
    ore[u] = scale * ure[o];
    oim[u] = scale * uim[o];
  }
}

// Homogeneous steps fused per launch by default (temporal blocking; 1 = one step per launch):
// 4 in FP32 and 3 in FP64, the depths at which each precision's blocked launch does a step
// fastest (with its default tile shape).
constexpr int kF2DefaultBlock32 = 4, kF2DefaultBlock64 = 3;

// Weights of the source components at one time: (c, s)_j = amp (cos, sin)(m_j omega t).
struct ShotPhase {
  double c[CMCG_MAX_SHOTS] = {}, s[CMCG_MAX_SHOTS] = {};
};

// Per-step fields of a multi-frequency forced sweep: the load sum_j (Fre_j c_j + Fim_j s_j) at
// the sweep's source time into Fc (if Fre), and the Dirichlet values sum_j Re(gD_j e^{-i m_j w t})
// at its output time into D1 and, for the start map, at its input time into D0 (if Dre).
template <typename T>
__global__ void f2_combine_kernel(size_t fs, int nshots, const T *Fre, const T *Fim, ShotPhase wf,
                                  T *Fc, const double *Dre, const double *Dim, ShotPhase w1,
                                  double *D1, ShotPhase w0, double *D0) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < fs; o += stride) {
    if (Fc) {
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < CMCG_MAX_SHOTS; ++j) {
        if (j >= nshots) break;
        a = fma((double)Fre[j * fs + o], wf.c[j], a);
        if (Fim) a = fma((double)Fim[j * fs + o], wf.s[j], a);
      }
      Fc[o] = (T)a;
    }
    if (Dre) {
      double a1 = 0.0, a0 = 0.0;
#pragma unroll
      for (int j = 0; j < CMCG_MAX_SHOTS; ++j) {
        if (j >= nshots) break;
        const double dr = Dre[j * fs + o], di = Dim ? Dim[j * fs + o] : 0.0;
        a1 = fma(dr, w1.c[j], fma(di, w1.s[j], a1));
        a0 = fma(dr, w0.c[j], fma(di, w0.s[j], a0));
      }
      D1[o] = a1;
      if (D0) D0[o] = a0;
    }
  }
}

// Filter sums of a multi-frequency problem at step n: (Ure_j, Uim_j) += u^n (cos, sin)(m_j w t_n).
// At n = 0 the state u^0 is the input's free-node values plus the Dirichlet values d0 (zero
// without data) on the sound-soft nodes; later states hold both already.
__global__ void f2_accumulate_kernel(F2Geom g, int nshots, const double *u, int first,
                                     const double *d0, ShotPhase w, double *ure, double *uim) {
  F2_ROWS(g)
  double x = u[o];
  if (first && g.mask && g.mask[o]) x = d0 ? d0[o] : 0.0;
#pragma unroll
  for (int jj = 0; jj < CMCG_MAX_SHOTS; ++jj) {
    if (jj >= nshots) break;
    ure[jj * g.fs + o] += x * w.c[jj];
    uim[jj * g.fs + o] += x * w.s[jj];
  }
  F2_ROWS_END
}

// Step 6 read off a device-layout state z into contiguous node arrays: u = u_0 + i v_1 / wh on
// the free nodes, the Dirichlet data (or 0) on the sound-soft nodes
__global__ void f2_step6_kernel(F2Geom g, const double *z, double inv_wh, const double *dre,
                                const double *dim, double *ore, double *oim) {
  F2_ROWS(g)
  const size_t u = ((size_t)k * (g.ny + 1) + j) * (g.nx + 1) + i;
  if (g.mask && g.mask[o]) {
    ore[u] = dre ? dre[o] : 0.0;
    oim[u] = dim ? dim[o] : 0.0;
  } else {
    ore[u] = z[o];
    oim[u] = z[g.fs + o] * inv_wh;
  }
  F2_ROWS_END
}

// (re, im) -= (a, b) over n contiguous values
__global__ void shift_kernel(double *re, double *im, size_t n, double a, double b) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    re[k] -= a;
    im[k] -= b;
  }
}

int gridn(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

// blocks for a node-row loop: four rows per 256-thread block
int rows_grid_of(const F2Geom &g) {
  const long rows = (long)(g.ny + 1) * (g.nz + 1);
  const long b = (rows + 3) / 4;
  return (int)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

struct F2Set {
  int prec = CMCG_FP64;
  void *A = nullptr, *B = nullptr, *C = nullptr;   // three-level state buffers (one field each)
  void *D = nullptr;                               // fourth one for blocked launches, or null
  void *W = nullptr, *Y = nullptr;                 // two-field: period output / metric output
  void *lam = nullptr;
  void *Fre = nullptr, *Fim = nullptr;             // load amplitudes, one field per component
  void *Fc = nullptr;                              // several components: the load of one sweep
  int kstep = 1;                                   // homogeneous steps per blocked launch
};

class F2Solver final : public Solver {
 public:
  F2Geom g;
  SolverConfig cfg;
  hipStream_t s = nullptr;
  DeviceArena arena;
  PhaseEvents ev;
  BulkTimer bulk;
  int bulk_dir = -1;   // >= 0: time the full-depth blocked launches in this direction
  F2Set lo, hi;
  bool mixed = false;
  uint8_t *mask = nullptr;
  void *D = nullptr;                 // direction (lo, two fields)
  double *Z = nullptr;               // iterate (two fields)
  float *DZ = nullptr;               // FP32-mixed: the iterate's FP32 correction since the last
                                     // reliable update (the iterate is Z + DZ)
  void *RU = nullptr;                // primal residual, u block (FP64; FP32 in FP32-mixed mode)
  void *RH = nullptr;                // dual residual (two fields, like RU)
  double *QU = nullptr;              // Riesz output, u block
  double *Ure = nullptr, *Uim = nullptr;   // filter sums, one field per component
  double *Dre = nullptr, *Dim = nullptr;   // Dirichlet data on the sound-soft nodes (one field per
                                           // component), or null
  bool multi = false;                      // several source components
  double *DA = nullptr, *DB = nullptr;     // several components: Dirichlet values of one sweep
  bool pure_neumann = false;               // no absorbing face and no sound-soft node
  double *cpart = nullptr, *h_cpart = nullptr;   // compatibility sums: device partials, host copy
  double *partials = nullptr, *scalars = nullptr, *h_scalars = nullptr;
  RieszMGT<double> mg;     // FP64 hierarchy: the PCG solve, and FP64 solves' V-cycle
  RieszMGT<float> mg32;    // FP32 hierarchy: the V-cycle of FP32-mixed solves
  bool mg_f32 = false;
  bool started = false;
  int iter = 0, refreshes = 0;
  long long riesz_iters = 0;
  int riesz_unconverged = 0;   // Riesz PCG solves that stopped at riesz_max_iter above riesz_tol
  double rel = 1.0, delta_at_refresh = 0.0;
  double riesz_tol = 1e-10;
  int riesz_max = 500;
  double t_fwd = 0, t_adj = 0, t_riesz = 0, t_other = 0, t_total = 0, t_runup = 0, updates = 0;
  double dram = 0;   // compulsory HBM bytes of the stencil launches since cmcg_begin
  int runup_done = 0;
  // source ramp of forced periods: absolute start time of the period and switch-on length
  // (t_tr = 0: no ramp)
  double t_offset = 0.0, t_tr = 0.0;

  ~F2Solver() override {
    if (s) (void)hipStreamSynchronize(s);
    if (h_scalars) (void)hipHostFree(h_scalars);
    if (h_cpart) (void)hipHostFree(h_cpart);
  }
  size_t device_bytes() const override { return arena.bytes(); }

  cmcg_status alloc_set(F2Set &b, int prec, bool var_c, bool forced, bool has_im, int J,
                        bool blocked) {
    const size_t esz = prec == CMCG_FP64 ? sizeof(double) : sizeof(float);
    b.prec = prec;
    CMCG_TRY(arena.alloc(g.fs * esz, &b.A, s));
    CMCG_TRY(arena.alloc(g.fs * esz, &b.B, s));
    CMCG_TRY(arena.alloc(g.fs * esz, &b.C, s));
    if (blocked) CMCG_TRY(arena.alloc(g.fs * esz, &b.D, s));
    CMCG_TRY(arena.alloc(2 * g.fs * esz, &b.W, s));
    CMCG_TRY(arena.alloc(2 * g.fs * esz, &b.Y, s));
    if (var_c) CMCG_TRY(arena.alloc(g.fs * esz, &b.lam, s));
    if (forced) CMCG_TRY(arena.alloc(J * g.fs * esz, &b.Fre, s));
    if (forced && has_im) CMCG_TRY(arena.alloc(J * g.fs * esz, &b.Fim, s));
    if (forced && J > 1) CMCG_TRY(arena.alloc(g.fs * esz, &b.Fc, s));
    return CMCG_OK;
  }

  cmcg_status create(const cmcg_problem *P) {
    s = cfg.stream;
    g.nx = (int)P->n[0];
    g.ny = (int)P->n[1];
    g.nz = (int)P->n[2];
    g.px = (g.nx + 1 + 63) / 64 * 64;
    g.plane = (size_t)g.px * (g.ny + 1);
    g.fs = g.plane * (g.nz + 1);
    g.h = cfg.h;
    g.dt = cfg.dt;
    for (int f = 0; f < 6; ++f) g.abs_face[f] = P->face_bc[f] == CMCG_ABSORBING ? 1 : 0;
    g.lam_const = (P->c_const * cfg.dt / cfg.h) * (P->c_const * cfg.dt / cfg.h);
    g.kchunk = 16;
    mixed = cfg.prec == CMCG_FP32_MIXED;
    riesz_tol = cfg.riesz_tol > 0 ? cfg.riesz_tol : 1e-10;
    riesz_max = cfg.riesz_max_iter > 0 ? cfg.riesz_max_iter : 500;
    CMCG_TRY(ev.init(12));
    CMCG_TRY(bulk.init());
    CMCG_HIP(hipHostMalloc((void **)&h_scalars, kNumScalars * sizeof(double)));
    std::fill(h_scalars, h_scalars + kNumScalars, 0.0);
    const size_t nn = (size_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    // sound-soft mask and its bounding box
    if (P->sound_soft) {
      // bounding box of the sound-soft nodes (kernels skip the mask outside it)
      int lo3[3] = {1 << 30, 1 << 30, 1 << 30}, hi3[3] = {-1, -1, -1};
      for (int k = 0; k <= g.nz; ++k)
        for (int j = 0; j <= g.ny; ++j) {
          const uint8_t *row = P->sound_soft + ((size_t)k * (g.ny + 1) + j) * (g.nx + 1);
          for (int i = 0; i <= g.nx; ++i)
            if (row[i]) {
              lo3[0] = std::min(lo3[0], i), hi3[0] = std::max(hi3[0], i);
              lo3[1] = std::min(lo3[1], j), hi3[1] = std::max(hi3[1], j);
              lo3[2] = std::min(lo3[2], k), hi3[2] = std::max(hi3[2], k);
            }
        }
      if (hi3[0] >= 0) {
        DeviceArena tmp;
        uint8_t *dm = nullptr;
        CMCG_TRY(tmp.alloc_n(nn, &dm, s));
        CMCG_HIP(hipMemcpyAsync(dm, P->sound_soft, nn, hipMemcpyHostToDevice, s));
        CMCG_TRY(arena.alloc_n(g.fs, &mask, s));
        hipLaunchKernelGGL(mask_unpack_kernel, dim3(gridn(g.fs)), dim3(256), 0, s, g, dm, mask);
        CMCG_HIP(hipGetLastError());
        CMCG_HIP(hipStreamSynchronize(s));
        g.mask = mask;
        for (int a = 0; a < 3; ++a) {
          g.mlo[a] = lo3[a];
          g.mhi[a] = hi3[a];
        }
      }
    }
    const std::vector<cmcg_shot> shots = shots_of(P);
    const int J = (int)shots.size();
    multi = J > 1;
    const bool var_c = P->c != nullptr;
    bool forced = false, has_im = false, has_d = false, has_dim = false;
    for (const cmcg_shot &sh : shots) {
      forced = forced || sh.f_re || sh.f_im || sh.gS_re || sh.gS_im;
      has_im = has_im || sh.f_im || sh.gS_im;
      has_d = has_d || sh.gD_re || sh.gD_im;
      has_dim = has_dim || sh.gD_im;
    }
    // temporal blocking of the homogeneous steps: K steps per launch (1 = off); each set gets
    // the fourth state buffer it needs (in FP32-mixed mode the FP64 set's backward periods, in
    // the refreshes, then run blocked too)
    const int kreq = cfg.steps_request > 0 ? std::min(cfg.steps_request, 4) : 0;
    hi.kstep = kreq ? kreq : kF2DefaultBlock64;
    lo.kstep = kreq ? kreq : kF2DefaultBlock32;
    // (a blocked launch addresses each plane through a buffer resource of the plane's bytes,
    // which must stay below 2^31 in FP64; larger planes step one step per launch)
    if (g.plane * sizeof(double) > 0x7fffffffull) hi.kstep = lo.kstep = 1;
    CMCG_TRY(alloc_set(hi, CMCG_FP64, var_c, forced, has_im, J, hi.kstep > 1));
    if (mixed) CMCG_TRY(alloc_set(lo, CMCG_FP32_MIXED, var_c, forced, has_im, J, lo.kstep > 1));
    else lo = hi;
    CMCG_TRY(arena.alloc(2 * g.fs * (mixed ? sizeof(float) : sizeof(double)), &D, s));
    CMCG_TRY(arena.alloc_n(2 * g.fs, &Z, s));
    if (mixed) CMCG_TRY(arena.alloc_n(2 * g.fs, &DZ, s));
    const size_t rsz = mixed ? sizeof(float) : sizeof(double);
    CMCG_TRY(arena.alloc(g.fs * rsz, &RU, s));
    CMCG_TRY(arena.alloc(2 * g.fs * rsz, &RH, s));
    CMCG_TRY(arena.alloc_n(g.fs, &QU, s));
    CMCG_TRY(arena.alloc_n(J * g.fs, &Ure, s));
    CMCG_TRY(arena.alloc_n(J * g.fs, &Uim, s));
    CMCG_TRY(arena.alloc_n(kRedBlocks, &partials, s));
    CMCG_TRY(arena.alloc_n(kNumScalars, &scalars, s));
    // coefficients and load, component by component (lambda is rewritten with equal values)
    for (int jj = 0; jj < J; ++jj) {
      const size_t sx = (size_t)(g.nz + 1) * (g.ny + 1), sy = (size_t)(g.nz + 1) * (g.nx + 1),
                   sz = (size_t)(g.ny + 1) * (g.nx + 1);
      const size_t nface = 2 * (sx + sy + sz);
      DeviceArena tmp;
      const double *src[5] = {P->c, shots[jj].f_re, shots[jj].f_im, shots[jj].gS_re,
                              shots[jj].gS_im};
      const size_t len[5] = {nn, nn, nn, nface, nface};
      double *dev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
      for (int k = 0; k < 5; ++k) {
        if (!src[k]) continue;
        CMCG_TRY(tmp.alloc_n(len[k], &dev[k], s));
        CMCG_HIP(hipMemcpyAsync(dev[k], src[k], len[k] * sizeof(double), hipMemcpyHostToDevice, s));
      }
      const size_t off = (size_t)jj * g.fs;
      CMCG_HIP(f2_setup<double>(g, dev[0], P->c_const, dev[1], dev[2], dev[3], dev[4],
                                tp<double>(hi.lam), hi.Fre ? tp<double>(hi.Fre) + off : nullptr,
                                hi.Fim ? tp<double>(hi.Fim) + off : nullptr, s));
      if (mixed)
        CMCG_HIP(f2_setup<float>(g, dev[0], P->c_const, dev[1], dev[2], dev[3], dev[4],
                                 tp<float>(lo.lam), lo.Fre ? tp<float>(lo.Fre) + off : nullptr,
                                 lo.Fim ? tp<float>(lo.Fim) + off : nullptr, s));
      CMCG_HIP(hipStreamSynchronize(s));
    }
    // Dirichlet data (only where there are sound-soft nodes), one field per component; a zero
    // real part is kept when only imaginary parts are given so that the kernels' reads are valid
    if (g.mask && has_d) {
      CMCG_TRY(arena.alloc_n(J * g.fs, &Dre, s));
      if (has_dim) CMCG_TRY(arena.alloc_n(J * g.fs, &Dim, s));
      for (int jj = 0; jj < J; ++jj) {
        DeviceArena tmp;
        const double *src[2] = {shots[jj].gD_re, shots[jj].gD_im};
        double *dst[2] = {Dre + jj * g.fs, Dim ? Dim + jj * g.fs : nullptr};
        for (int k = 0; k < 2; ++k) {
          if (!src[k]) continue;
          double *dpk = nullptr;
          CMCG_TRY(tmp.alloc_n(nn, &dpk, s));
          CMCG_HIP(hipMemcpyAsync(dpk, src[k], nn * sizeof(double), hipMemcpyHostToDevice, s));
          hipLaunchKernelGGL(dirichlet_unpack_kernel, dim3(gridn(g.fs)), dim3(256), 0, s, g, dpk,
                             dst[k]);
          CMCG_HIP(hipGetLastError());
        }
        CMCG_HIP(hipStreamSynchronize(s));
      }
      if (multi) {
        CMCG_TRY(arena.alloc_n(g.fs, &DA, s));
        CMCG_TRY(arena.alloc_n(g.fs, &DB, s));
      }
    }
    bool absorbing = false;
    for (int f = 0; f < 6; ++f) absorbing = absorbing || g.abs_face[f];
    pure_neumann = !absorbing && !g.mask;
    if (!g.mask) {
      // the constant is a free mode: compatibility sums for the outputs
      CMCG_TRY(arena.alloc_n((size_t)kCompatSums * kRedBlocks, &cpart, s));
      CMCG_HIP(hipHostMalloc((void **)&h_cpart, (size_t)kCompatSums * kRedBlocks * sizeof(double)));
    }
    // the Riesz map of an FP32-mixed solve in V-cycle mode is one FP32 V-cycle, in the CG
    // iterations and the FP64 refreshes alike (the same fixed operator throughout)
    mg_f32 = mixed && cfg.riesz_mode == CMCG_RIESZ_VCYCLE;
    if (mg_f32) CMCG_TRY(mg32.build(g, arena, s));
    else CMCG_TRY(mg.build(g, arena, s));
    return CMCG_OK;
  }

  // The constant lam that makes a - lam satisfy the compatibility condition of component j's
  // time-discrete system, 1^T [S - wt^2 M - i wh B] (a - lam) = 1^T Fhat (eq. CC and eq.
  // cc_neumann_eta; S 1 = 0), a = sa ar + i sb ai in the device layout:
  //   lam = (sum Fhat + wt^2 sum M a + i wh sum B a) / (wt^2 sum M + i wh sum B).
  // The sums are fixed-order block reductions, added on the host in block order.
  cmcg_status compat_constant(int j, const double *ar, double sa, const double *ai, double sb,
                              double *lre, double *lim) {
    const double *Fr = hi.Fre ? tpc<double>(hi.Fre) + (size_t)j * g.fs : nullptr;
    const double *Fi = hi.Fim ? tpc<double>(hi.Fim) + (size_t)j * g.fs : nullptr;
    CMCG_HIP(f2_compat_sums(g, tpc<double>(hi.lam), Fr, Fi, ar, sa, ai, sb, cpart, s));
    CMCG_HIP(hipMemcpyAsync(h_cpart, cpart, (size_t)kCompatSums * kRedBlocks * sizeof(double),
                            hipMemcpyDeviceToHost, s));
    CMCG_HIP(hipStreamSynchronize(s));
    double S[kCompatSums] = {};
    for (int q = 0; q < kCompatSums; ++q)
      for (int b = 0; b < kRedBlocks; ++b) S[q] += h_cpart[(size_t)q * kRedBlocks + b];
    const double w = cfg.omega_of(j), dt = cfg.dt;
    const double wt2 = std::pow(2.0 / dt * std::sin(0.5 * w * dt), 2), wh = std::sin(w * dt) / dt;
    // numerator n = Fhat + wt2 M a + i wh B a; denominator d = wt2 M + i wh B
    const double nr = S[2] + wt2 * S[4] - wh * S[7], ni = S[3] + wt2 * S[5] + wh * S[6];
    const double dr = wt2 * S[0], di = wh * S[1];
    const double den = dr * dr + di * di;
    if (!(den > 0.0)) return set_error("compatibility condition: zero mass"), CMCG_EBREAKDOWN;
    *lre = (nr * dr + ni * di) / den;
    *lim = (ni * dr - nr * di) / den;
    return CMCG_OK;
  }

  // ------------------------------------------------------------------ periods
  // `count` homogeneous steps from (cur, prev) = (u^n, u^{n-1}); on return they point to
  // u^{n+count} and u^{n+count-1}.  With the set's fourth buffer, b.kstep steps per blocked launch
  // (then the remainder one at a time); outputs always go to buffers that are not inputs.
  // Compulsory HBM bytes of one sweep: each array its arguments name read (or written) once,
  // the subtrahend as two fields, the filter's FP64 accumulators read and written
  template <typename T>
  double sweep_bytes(const F2Args<T> &p) const {
    const double nn = (double)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    const int w = (p.st ? 1 : 0) + (p.aux ? 1 : 0) + (p.sub ? 2 : 0) + (p.lam ? 1 : 0) +
                  (p.forced && p.fre ? 1 : 0) + (p.forced && p.fim ? 1 : 0) + (p.out ? 1 : 0) +
                  (p.out2 ? 1 : 0);
    return nn * (w * (double)sizeof(T) + (p.ure ? 32.0 : 0.0));
  }
  // a blocked launch reads u^n, u^{n-1} (and lambda) and writes u^{n+K}, u^{n+K-1}; the scaling
  // into the adjoint variable reads a field (and lambda) and writes one
  template <typename T>
  double fields_bytes(int fields, const T *lam) const {
    return (double)(g.nx + 1) * (g.ny + 1) * (g.nz + 1) * sizeof(T) * (fields + (lam ? 1 : 0));
  }

  template <typename T>
  cmcg_status homogeneous_steps(const F2Set &b, const T *&cur, const T *&prev, int count,
                                F2Args<T> p) {
    T *pool[4] = {tp<T>(b.A), tp<T>(b.B), tp<T>(b.C), tp<T>(b.D)};
    const int npool = b.D ? 4 : 3;
    auto pick = [&](const T *x, const T *y, const T *z) -> T * {
      for (int k = 0; k < npool; ++k)
        if (pool[k] != x && pool[k] != y && pool[k] != z) return pool[k];
      return nullptr;
    };
    long long full = 0;   // blocked launches of full depth so far (the bulk of the period)
    while (count > 0) {
      const int kstep = b.kstep;
      const int K = (b.D && kstep > 1 && count >= 2) ? std::min(kstep, count) : 1;
      if (K >= 2) {
        T *ok = pick(cur, prev, nullptr);
        T *okm1 = pick(cur, prev, ok);
        if (!ok || !okm1) return set_error("blocked march: no free buffer"), CMCG_EDEVICE;
        dram += fields_bytes<T>(4, tpc<T>(b.lam));
        const bool timed = bulk_dir >= 0 && K == kstep;
        if (timed && full == 0) CMCG_TRY(bulk.begin(bulk_dir, s));
        CMCG_HIP(f2_march_block<T>(g, cur, prev, tpc<T>(b.lam), ok, okm1, K, s));
        if (timed) {
          ++full;
          if (count - K < kstep) CMCG_TRY(bulk.end(bulk_dir, full, s));   // the last full one
        }
        cur = ok;
        prev = okm1;
      } else {
        T *o = pick(cur, prev, nullptr);
        if (!o) return set_error("march: no free buffer"), CMCG_EDEVICE;
        p.st = cur;
        p.aux = prev;
        p.out = o;
        dram += sweep_bytes<T>(p);
        CMCG_HIP(f2_march<T>(kF2FwdStep, g, p, s));
        prev = cur;
        cur = o;
      }
      count -= K;
    }
    return CMCG_OK;
  }

  // Component weights (cos, sin)(m_j omega t_n) at step time t_n = n dt, times the source ramp
  // if `ramped`
  ShotPhase shot_phase(int n, bool ramped) const {
    ShotPhase w;
    const double t = n * cfg.dt, amp = ramped ? transient(t_offset + t, t_tr) : 1.0;
    for (int j = 0; j < cfg.nshots; ++j) {
      w.c[j] = amp * std::cos(cfg.omega_of(j) * t);
      w.s[j] = amp * std::sin(cfg.omega_of(j) * t);
    }
    return w;
  }

  // Several components: the load of the sweep whose source time is t_nf (into b.Fc) and the
  // Dirichlet values at t_nd (into DB) and, if start, at t_0 (into DA).
  template <typename T>
  cmcg_status combine(const F2Set &b, bool load, bool dir, int nf, int nd, bool start) {
    if (!load && !dir) return CMCG_OK;
    hipLaunchKernelGGL((f2_combine_kernel<T>), dim3(gridn(g.fs)), dim3(256), 0, s, g.fs,
                       cfg.nshots, tpc<T>(b.Fre), tpc<T>(b.Fim), shot_phase(nf, true),
                       load ? tp<T>(b.Fc) : nullptr, dir ? Dre : nullptr, Dim,
                       shot_phase(nd, true), DB, shot_phase(0, true), start ? DA : nullptr);
    CMCG_HIP(hipGetLastError());
    return CMCG_OK;
  }

  // Several components: filter sums of u^n (FP64 state)
  cmcg_status accumulate(const double *u, int n) {
    hipLaunchKernelGGL(f2_accumulate_kernel, dim3(rows_grid_of(g)), dim3(256), 0, s, g, cfg.nshots,
                       u, n == 0 ? 1 : 0, n == 0 ? DA : nullptr, shot_phase(n, false), Ure, Uim);
    CMCG_HIP(hipGetLastError());
    return CMCG_OK;
  }

  // One component: its load enters the sweeps with the weights (cos, sin)(m omega t) of the
  // sweep's time, and the filter sum runs inside the sweeps.  Several components: before each
  // sweep, `combine` writes that sweep's summed load (read with weights (1, 0)) and Dirichlet
  // values (DB at the output time, DA at the start map's input time, read through the data
  // pointers with weights (1, 0) and (0, 1)), and `accumulate` adds u^n to every filter sum.
  template <typename T>
  cmcg_status fwd_t(const F2Set &b, bool forced, const T *zin, T *out, const T *sub, bool filter) {
    const int N = cfg.N;
    const double w0 = cfg.omega_of(0);
    const bool load = forced && b.Fre, dir = forced && Dre;
    if (multi && filter && !std::is_same<T, double>::value)
      return set_error("the filter period runs in FP64"), CMCG_EINVAL;
    F2Args<T> p;
    p.lam = tpc<T>(b.lam);
    p.fre = multi ? tpc<T>(b.Fc) : tpc<T>(b.Fre);
    p.fim = multi ? nullptr : tpc<T>(b.Fim);
    p.forced = load ? 1 : 0;
    if (filter && !multi) {
      p.ure = Ure;
      p.uim = Uim;
    }
    if (dir) {
      p.dre = multi ? DB : Dre;
      p.dim = multi ? DA : Dim;
    }
    // weights of Re(g e^{-i m w t}) at the step time t_n = n dt of this period (ramped)
    auto phase = [&](int n, double *c, double *sn) {
      const double t = n * cfg.dt, amp = transient(t_offset + t, t_tr);
      *c = multi ? 1.0 : amp * std::cos(w0 * t);
      *sn = multi ? 0.0 : amp * std::sin(w0 * t);
    };
    T *buf[3] = {tp<T>(b.A), tp<T>(b.B), tp<T>(b.C)};
    // start map: u^1 from (u^0, v^0)
    p.st = zin;
    p.aux = zin + g.fs;
    p.out = buf[0];
    p.fcos = multi ? 1.0 : transient(t_offset, t_tr);
    p.fsin = 0.0;
    p.wcos = 1.0;
    p.wsin = 0.0;
    if (multi) {
      p.dcos0 = 0.0;
      p.dsin0 = 1.0;
    } else {
      phase(0, &p.dcos0, &p.dsin0);
    }
    phase(1, &p.dcos1, &p.dsin1);
    if (multi) {
      CMCG_TRY(combine<T>(b, load, dir, 0, 1, true));
      if (filter) CMCG_TRY(accumulate(reinterpret_cast<const double *>(zin), 0));
    }
    dram += sweep_bytes<T>(p);
    CMCG_HIP(f2_march<T>(kF2FwdStart, g, p, s));
    const T *prev = zin;
    int cur = 0;
    const T *curp = buf[0];
    if (!load && !dir && !filter) {
      // homogeneous steps 1 .. N-1, temporally blocked
      CMCG_TRY(homogeneous_steps<T>(b, curp, prev, N - 1, p));
    }
    for (int n = 1; n < N && (load || dir || filter); ++n) {
      const double t = n * cfg.dt;
      const double amp = transient(t_offset + t, t_tr);
      p.wcos = std::cos(w0 * t);
      p.wsin = std::sin(w0 * t);
      p.fcos = multi ? 1.0 : amp * p.wcos;
      p.fsin = multi ? 0.0 : amp * p.wsin;
      phase(n + 1, &p.dcos1, &p.dsin1);
      const int nxt = (cur + 1) % 3;
      p.st = buf[cur];
      p.aux = prev;
      p.out = buf[nxt];
      if (multi) {
        CMCG_TRY(combine<T>(b, load, dir, n, n + 1, false));
        if (filter) CMCG_TRY(accumulate(reinterpret_cast<const double *>(buf[cur]), n));
      }
      dram += sweep_bytes<T>(p);
      CMCG_HIP(f2_march<T>(kF2FwdStep, g, p, s));
      prev = buf[cur];
      cur = nxt;
      curp = buf[cur];
    }
    // end map: (u^N, v^N) with v^N = (u^{N+1} - u^{N-1}) / (2 dt)
    p.ure = p.uim = nullptr;
    const double ampN = transient(t_offset + N * cfg.dt, t_tr);
    p.fcos = multi ? 1.0 : ampN * std::cos(w0 * N * cfg.dt);
    p.fsin = multi ? 0.0 : ampN * std::sin(w0 * N * cfg.dt);
    p.st = curp;
    p.aux = prev;
    p.out = out;
    p.sub = sub;
    if (multi) CMCG_TRY(combine<T>(b, load, false, N, N, false));
    dram += sweep_bytes<T>(p);
    CMCG_HIP(f2_march<T>(kF2FwdEnd, g, p, s));
    updates += (double)(N + 1) * (g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    return CMCG_OK;
  }

  template <typename T>
  cmcg_status metric_t(const F2Set &b, const T *w, T *y) {
    F2Args<T> p;
    p.lam = tpc<T>(b.lam);
    p.st = w;
    p.aux = w + g.fs;
    p.out = y;
    dram += sweep_bytes<T>(p);
    CMCG_HIP(f2_march<T>(kF2Metric, g, p, s));
    return CMCG_OK;
  }

  // out = E^T y (- sub), run in the scaled adjoint variable g = psi a (psi = lambda R /
  // ((1 + beta) eta)), in which every interior transposed step is the homogeneous forward step
  template <typename T>
  cmcg_status adj_t(const F2Set &b, const T *y, T *out, const T *sub) {
    const int N = cfg.N;
    F2Args<T> p;
    p.lam = tpc<T>(b.lam);
    T *buf[3] = {tp<T>(b.A), tp<T>(b.B), tp<T>(b.C)};
    // g_y = psi y_v (C)
    dram += fields_bytes<T>(2, p.lam);
    CMCG_HIP(f2_psi_scale<T>(g, y + g.fs, p.lam, buf[2], s));
    // transposed end map: g_0 (A), psi b_0 (B)
    p.st = buf[2];
    p.aux = y;
    p.out = buf[0];
    p.out2 = buf[1];
    dram += sweep_bytes<T>(p);
    CMCG_HIP(f2_march<T>(kF2AdjInit, g, p, s));
    p.out2 = nullptr;
    // first transposed step: g_1 = K g_0 + psi b_0 -> C
    p.st = buf[0];
    p.aux = buf[1];
    p.out = buf[2];
    dram += sweep_bytes<T>(p);
    CMCG_HIP(f2_march<T>(kF2AdjStepFirst, g, p, s));
    // interior transposed steps 1 .. N-2: forward homogeneous steps in g (temporally blocked)
    const T *curp = buf[2], *prevp = buf[0];
    CMCG_TRY(homogeneous_steps<T>(b, curp, prevp, N - 2, p));
    // transposed start map, back to the adjoint state
    p.st = curp;
    p.aux = prevp;
    p.out = out;
    p.sub = sub;
    dram += sweep_bytes<T>(p);
    CMCG_HIP(f2_march<T>(kF2AdjEnd, g, p, s));
    updates += (double)(N + 1) * (g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    return CMCG_OK;
  }

  cmcg_status fwd(const F2Set &b, bool forced, const void *zin, void *out, const void *sub,
                  bool filter) {
    if (b.prec == CMCG_FP64)
      return fwd_t<double>(b, forced, tpc<double>(zin), tp<double>(out), tpc<double>(sub), filter);
    return fwd_t<float>(b, forced, tpc<float>(zin), tp<float>(out), tpc<float>(sub), filter);
  }
  cmcg_status metric(const F2Set &b, const void *w, void *y) {
    if (b.prec == CMCG_FP64) return metric_t<double>(b, tpc<double>(w), tp<double>(y));
    return metric_t<float>(b, tpc<float>(w), tp<float>(y));
  }
  cmcg_status adj(const F2Set &b, const void *y, void *out, const void *sub) {
    if (b.prec == CMCG_FP64) return adj_t<double>(b, tpc<double>(y), tp<double>(out), tpc<double>(sub));
    return adj_t<float>(b, tpc<float>(y), tp<float>(out), tpc<float>(sub));
  }

  // qh = (E^T - I) M_E (E z - z [+ s])  into set b's W (the metric output Y is the subtrahend)
  cmcg_status gradient_dual(const F2Set &b, bool forced, const void *zin) {
    CMCG_TRY(fwd(b, forced, zin, b.W, zin, false));
    CMCG_TRY(metric(b, b.W, b.Y));
    CMCG_TRY(adj(b, b.Y, b.W, b.Y));
    return CMCG_OK;
  }

  // FP32-mixed V-cycle: q_u left in the FP32 hierarchy's buffer (*out), read directly by the CG
  // update (FP32 to FP64 is exact, so this equals converting it first)
  cmcg_status riesz_u_f32(const void *qh_u, const float **out) {
    CMCG_HIP(hipEventRecord(ev[8], s));
    CMCG_TRY(mg32.apply_vcycle_native(qh_u, 1, out));
    CMCG_HIP(hipEventRecord(ev[9], s));
    CMCG_HIP(hipEventSynchronize(ev[9]));
    t_riesz += PhaseEvents::seconds(ev[8], ev[9]);
    riesz_iters += 1;
    return CMCG_OK;
  }

  cmcg_status riesz_u(const void *qh_u, int is_float, double *out) {
    int it = 0;
    CMCG_HIP(hipEventRecord(ev[8], s));
    if (cfg.riesz_mode == CMCG_RIESZ_VCYCLE) {
      CMCG_TRY(mg_f32 ? mg32.apply_vcycle(qh_u, is_float, out)
                      : mg.apply_vcycle(qh_u, is_float, out));
      it = 1;
    } else {
      const cmcg_status st = mg.solve(qh_u, is_float, out, riesz_tol, riesz_max, &it);
      if (st < 0) return st;
      if (st == CMCG_ENOTCONV) ++riesz_unconverged;
    }
    CMCG_HIP(hipEventRecord(ev[9], s));
    CMCG_HIP(hipEventSynchronize(ev[9]));
    t_riesz += PhaseEvents::seconds(ev[8], ev[9]);
    riesz_iters += it;
    return CMCG_OK;
  }

  cmcg_status read_scalars() {
    CMCG_HIP(hipMemcpyAsync(h_scalars, scalars, kNumScalars * sizeof(double),
                            hipMemcpyDeviceToHost, s));
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  // true gradient at the FP64 iterate: RH = qh (dual), RU = S^{-1} qh_u; delta via `mode`.
  // FP32-mixed: the iterate is first brought up to date (Z += DZ, DZ = 0: the reliable update),
  // delta is formed from the FP64 residuals, which are then stored in FP32.
  cmcg_status true_gradient(int mode) {
    if (mixed) CMCG_HIP(f2_iterate(g, Z, DZ, Z, 1, s));
    CMCG_TRY(gradient_dual(hi, true, Z));
    if (mixed) {
      CMCG_TRY(riesz_u(hi.W, 0, QU));
      CMCG_HIP((f2_delta<double, float>(g, QU, tpc<double>(hi.W), tpc<double>(hi.lam),
                                        tp<float>(RU), tp<float>(RH), partials, s)));
    } else {
      CMCG_HIP(hipMemcpyAsync(RH, hi.W, 2 * g.fs * sizeof(double), hipMemcpyDeviceToDevice, s));
      CMCG_TRY(riesz_u(RH, 0, tp<double>(RU)));
      CMCG_HIP((f2_delta<double, double>(g, tpc<double>(RU), tpc<double>(RH),
                                         tpc<double>(hi.lam), nullptr, nullptr, partials, s)));
    }
    CMCG_HIP(finalize(partials, kRedBlocks, scalars, mode, 0, s));
    return CMCG_OK;
  }

  cmcg_status direction(int first) {
    if (mixed)
      CMCG_HIP((f2_direction<float, float>(g, tp<float>(D), tpc<float>(RU), tpc<float>(RH),
                                           tpc<float>(lo.lam), scalars, first, s)));
    else
      CMCG_HIP((f2_direction<double, double>(g, tp<double>(D), tpc<double>(RU), tpc<double>(RH),
                                             tpc<double>(lo.lam), scalars, first, s)));
    return CMCG_OK;
  }

  // The current iterate as an FP64 device field: Z, or (FP32-mixed) Z + DZ staged in `stage`
  // (the state itself is left as it is, so that reading it changes no later rounding)
  cmcg_status current_iterate(double *stage, const double **z) {
    *z = Z;
    if (!mixed) return CMCG_OK;
    CMCG_HIP(f2_iterate(g, Z, DZ, stage, 0, s));
    *z = stage;
    return CMCG_OK;
  }

  // ------------------------------------------------------------------ CG driver
  // The forced scheme from rest over `periods` periods (FP64), the load ramped by Mur's
  // transient over the whole interval if `ramp`; the final state (u, v) goes to `state` (two
  // FP64 fields).  Uses hi.Y and hi.W as the two state buffers.
  cmcg_status run_forced_periods(int periods, bool ramp, double *state) {
    double *a = tp<double>(hi.Y), *b = tp<double>(hi.W);
    CMCG_HIP(hipMemsetAsync(a, 0, 2 * g.fs * sizeof(double), s));
    t_tr = ramp ? periods * cfg.T : 0.0;
    for (int p = 0; p < periods; ++p) {
      t_offset = p * cfg.T;
      const cmcg_status st = fwd(hi, true, a, b, nullptr, false);
      if (st != CMCG_OK) {
        t_offset = t_tr = 0.0;
        return st;
      }
      std::swap(a, b);
    }
    t_offset = t_tr = 0.0;
    CMCG_HIP(hipMemcpyAsync(state, a, 2 * g.fs * sizeof(double), hipMemcpyDeviceToDevice, s));
    return CMCG_OK;
  }

  cmcg_status begin() override {
    t_fwd = t_adj = t_riesz = t_other = t_total = t_runup = 0.0;
    updates = 0;
    dram = 0;
    iter = refreshes = runup_done = 0;
    riesz_iters = 0;
    riesz_unconverged = 0;
    bulk.reset();
    CMCG_HIP(hipEventRecord(ev[0], s));
    CMCG_HIP(hipMemsetAsync(Z, 0, 2 * g.fs * sizeof(double), s));
    if (mixed) CMCG_HIP(hipMemsetAsync(DZ, 0, 2 * g.fs * sizeof(float), s));
    CMCG_TRY(true_gradient(kFinStart));
    if (cfg.runup > 0) {
      // start from the run-up state; delta0 stays the residual at rest (stopping reference)
      CMCG_HIP(hipEventRecord(ev[10], s));
      CMCG_TRY(run_forced_periods(cfg.runup, true, Z));
      CMCG_HIP(hipEventRecord(ev[11], s));
      CMCG_HIP(hipMemcpyAsync(scalars + kTmp, scalars + kDelta, sizeof(double),
                              hipMemcpyDeviceToDevice, s));
      CMCG_TRY(true_gradient(kFinRefresh));
      runup_done = cfg.runup;
    }
    CMCG_TRY(direction(1));
    CMCG_HIP(hipEventRecord(ev[1], s));
    CMCG_TRY(read_scalars());
    t_other += PhaseEvents::seconds(ev[0], ev[1]);
    if (runup_done) {
      t_runup = PhaseEvents::seconds(ev[10], ev[11]);
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
      // Step 5.1: w = E d - d, y = M_E w, qh = E^T y - y
      bulk_dir = 0;
      cmcg_status st = fwd(lo, false, D, lo.W, D, false);
      if (st == CMCG_OK) st = metric(lo, lo.W, lo.Y);
      CMCG_HIP(hipEventRecord(ev[3], s));
      bulk_dir = 1;
      if (st == CMCG_OK) st = adj(lo, lo.Y, lo.W, lo.Y);
      bulk_dir = -1;
      CMCG_TRY(st);
      CMCG_HIP(hipEventRecord(ev[4], s));
      // Step 5.2: q_u = S^{-1} qh_u (q_v = M^{-1} qh_v is applied on the fly)
      const float *qu32 = nullptr;
      if (mg_f32) CMCG_TRY(riesz_u_f32(lo.W, &qu32));
      else CMCG_TRY(riesz_u(lo.W, mixed ? 1 : 0, QU));
      CMCG_HIP(hipEventRecord(ev[5], s));
      // Steps 5.3-5.6
      if (mixed) {
        CMCG_HIP(dot_plain<float, float>(tpc<float>(lo.W), tpc<float>(D), 2 * g.fs, partials, s));
        CMCG_HIP(finalize(partials, kRedBlocks, scalars, kFinAlpha, 0, s));
        if (qu32)
          CMCG_HIP((f2_cg_update<float, float, float, float>(
              g, DZ, tp<float>(RU), tp<float>(RH), tpc<float>(D), qu32, tpc<float>(lo.W),
              tpc<float>(lo.lam), scalars, partials, s)));
        else
          CMCG_HIP((f2_cg_update<float, double, float, float>(
              g, DZ, tp<float>(RU), tp<float>(RH), tpc<float>(D), QU, tpc<float>(lo.W),
              tpc<float>(lo.lam), scalars, partials, s)));
      } else {
        CMCG_HIP(dot_plain<double, double>(tpc<double>(lo.W), tpc<double>(D), 2 * g.fs, partials, s));
        CMCG_HIP(finalize(partials, kRedBlocks, scalars, kFinAlpha, 0, s));
        CMCG_HIP((f2_cg_update<double, double, double, double>(
            g, Z, tp<double>(RU), tp<double>(RH), tpc<double>(D), QU, tpc<double>(lo.W),
            tpc<double>(lo.lam), scalars, partials, s)));
      }
      CMCG_HIP(finalize(partials, kRedBlocks, scalars, kFinBeta, 0, s));
      CMCG_HIP(hipEventRecord(ev[6], s));
      CMCG_TRY(read_scalars());
      bulk.collect();
      t_fwd += PhaseEvents::seconds(ev[2], ev[3]);
      t_adj += PhaseEvents::seconds(ev[3], ev[4]);
      t_other += PhaseEvents::seconds(ev[5], ev[6]);
      ++iter;
      if (h_scalars[kBreak] != 0.0)
        return set_error("CG breakdown: <qhat, d> <= 0 or non-finite scalar"), CMCG_EBREAKDOWN;
      rel = h_scalars[kRel];
      if (mixed && cfg.refresh > 0.0 &&
          (rel <= cfg.tol || h_scalars[kDelta] <= cfg.refresh * cfg.refresh * delta_at_refresh)) {
        CMCG_HIP(hipEventRecord(ev[6], s));
        CMCG_TRY(true_gradient(kFinRefresh));
        CMCG_HIP(hipEventRecord(ev[7], s));
        CMCG_TRY(read_scalars());
        t_other += PhaseEvents::seconds(ev[6], ev[7]);
        rel = h_scalars[kRel];
        delta_at_refresh = h_scalars[kDelta];
        ++refreshes;
      }
      if (rel <= cfg.tol) {
        *converged = 1;
        break;
      }
      CMCG_TRY(direction(0));
    }
    return CMCG_OK;
  }

  // U = (2/N) (Ure + i Uim) per component, staged in `stage` (two fields of fs >= nn values) as
  // contiguous node arrays and copied to the caller's n_fields output fields
  cmcg_status output_fields(double *stage, double *u_re, double *u_im) {
    double *ore = stage, *oim = stage + g.fs;
    const size_t nn = (size_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    for (int j = 0; j < cfg.nshots; ++j) {
      hipLaunchKernelGGL(f2_output_kernel, dim3(gridn(g.fs)), dim3(256), 0, s, g, Ure + j * g.fs,
                         Uim + j * g.fs, 2.0 / cfg.N, ore, oim);
      CMCG_HIP(hipGetLastError());
      if (pure_neumann) {
        // the mode eta of a closed box shifts the filter sums by a constant, which the
        // compatibility condition fixes (eq. cc_neumann_eta)
        double lr = 0.0, li = 0.0;
        CMCG_TRY(compat_constant(j, Ure + j * g.fs, 2.0 / cfg.N, Uim + j * g.fs, 2.0 / cfg.N, &lr,
                                 &li));
        hipLaunchKernelGGL(shift_kernel, dim3(gridn(nn)), dim3(256), 0, s, ore, oim, nn, lr, li);
        CMCG_HIP(hipGetLastError());
      }
      if (u_re) CMCG_HIP(hipMemcpyAsync(u_re + j * nn, ore, nn * sizeof(double), hipMemcpyDefault, s));
      if (u_im) CMCG_HIP(hipMemcpyAsync(u_im + j * nn, oim, nn * sizeof(double), hipMemcpyDefault, s));
    }
    return CMCG_OK;
  }

  cmcg_status output(const double *z, double *u_re, double *u_im, bool record) {
    CMCG_HIP(hipMemsetAsync(Ure, 0, cfg.nshots * g.fs * sizeof(double), s));
    CMCG_HIP(hipMemsetAsync(Uim, 0, cfg.nshots * g.fs * sizeof(double), s));
    CMCG_TRY(fwd(hi, true, z, hi.W, nullptr, true));
    if (record) CMCG_HIP(hipEventRecord(ev[7], s));
    CMCG_TRY(output_fields(tp<double>(hi.Y), u_re, u_im));
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  cmcg_status finish(double *u_re, double *u_im) override {
    if (!started) return set_error("cmcg_begin first"), CMCG_EINVAL;
    const double *z = Z;
    if (cfg.output == CMCG_OUTPUT_STEP6) {
      // (step6_from stages its output in hi.Y)
      CMCG_TRY(current_iterate(tp<double>(hi.W), &z));
      CMCG_TRY(step6_from(z, u_re, u_im));
      CMCG_HIP(hipEventRecord(ev[7], s));
      return CMCG_OK;
    }
    // (the forced period reads its input from hi.Y and writes hi.W)
    CMCG_TRY(current_iterate(tp<double>(hi.Y), &z));
    return output(z, u_re, u_im, true);
  }

  // Step 6 read off a device-layout FP64 state (u_0 + i v_1 / wh, Dirichlet data on the
  // sound-soft nodes), the constant shift removed by the compatibility condition when there is
  // no sound-soft node (eq. CC); staged in hi.Y
  cmcg_status step6_from(const double *zdev, double *u_re, double *u_im) {
    if (cfg.nshots > 1)
      return set_error("the Step 6 output reads one frequency off the state: no shots"),
             CMCG_EINVAL;
    if (pure_neumann)
      return set_error("pure-Neumann box: the Step 6 output misses the mode eta; use the filter"),
             CMCG_EUNSUPPORTED;
    const double wh = std::sin(cfg.omega_of(0) * cfg.dt) / cfg.dt;
    double *ore = tp<double>(hi.Y), *oim = tp<double>(hi.Y) + g.fs;
    hipLaunchKernelGGL(f2_step6_kernel, dim3(rows_grid_of(g)), dim3(256), 0, s, g, zdev, 1.0 / wh,
                       Dre, Dim, ore, oim);
    CMCG_HIP(hipGetLastError());
    const size_t nn = (size_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    if (!g.mask) {
      double lr = 0.0, li = 0.0;
      CMCG_TRY(compat_constant(0, zdev, 1.0, zdev + g.fs, 1.0 / wh, &lr, &li));
      hipLaunchKernelGGL(shift_kernel, dim3(gridn(nn)), dim3(256), 0, s, ore, oim, nn, lr, li);
      CMCG_HIP(hipGetLastError());
    }
    if (u_re) CMCG_HIP(hipMemcpyAsync(u_re, ore, nn * sizeof(double), hipMemcpyDefault, s));
    if (u_im) CMCG_HIP(hipMemcpyAsync(u_im, oim, nn * sizeof(double), hipMemcpyDefault, s));
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  cmcg_status step6(const double *z, double *u_re, double *u_im) override {
    CMCG_HIP(f2_unpack<double>(g, z, tp<double>(hi.W), 2, s));
    return step6_from(tp<double>(hi.W), u_re, u_im);
  }

  cmcg_status solve(double *u_re, double *u_im) override {
    CMCG_TRY(begin());
    int conv = 0;
    CMCG_TRY(iterate(cfg.max_iter, &conv));
    CMCG_HIP(hipEventRecord(ev[6], s));
    CMCG_TRY(finish(u_re, u_im));
    t_other += PhaseEvents::seconds(ev[6], ev[7]);
    t_total = PhaseEvents::seconds(ev[0], ev[7]);
    // an inexact Riesz map changes the operator CG works with: not a converged solve
    return (conv && riesz_unconverged == 0) ? CMCG_OK : CMCG_ENOTCONV;
  }

  // ------------------------------------------------------------------ stage calls
  cmcg_status apply(int op, int steps, const double *in, double *out) override {
    if (steps != 0) return set_error("second-order periods take steps = 0"), CMCG_EINVAL;
    // stage the packed input into set lo's Y, run, pack lo's W
    if (lo.prec == CMCG_FP64) CMCG_HIP(f2_unpack<double>(g, in, tp<double>(lo.Y), 2, s));
    else CMCG_HIP(f2_unpack<float>(g, in, tp<float>(lo.Y), 2, s));
    if (op == CMCG_OP_FORWARD || op == CMCG_OP_FORCED) {
      CMCG_TRY(fwd(lo, op == CMCG_OP_FORCED, lo.Y, lo.W, nullptr, false));
    } else if (op == CMCG_OP_ADJOINT) {
      // the literal transpose E^T (not weighted by M_E: M_E is singular without sound-soft nodes)
      CMCG_TRY(adj(lo, lo.Y, lo.W, nullptr));
    } else {
      // P y = (S^{-1} y_u, M^{-1} y_v), FP64
      CMCG_HIP(f2_unpack<double>(g, in, tp<double>(hi.Y), 2, s));
      const int unconv0 = riesz_unconverged;
      CMCG_TRY(riesz_u(hi.Y, 0, QU));
      CMCG_HIP(f2_mass_inverse<double>(g, tp<double>(hi.Y) + g.fs, tp<double>(hi.W) + g.fs,
                                       tpc<double>(hi.lam), s));
      CMCG_HIP(hipMemcpyAsync(hi.W, QU, g.fs * sizeof(double), hipMemcpyDeviceToDevice, s));
      CMCG_HIP(f2_pack<double>(g, tp<double>(hi.W), out, 2, s));
      CMCG_HIP(hipStreamSynchronize(s));
      return riesz_unconverged > unconv0 ? CMCG_ENOTCONV : CMCG_OK;
    }
    if (lo.prec == CMCG_FP64) CMCG_HIP(f2_pack<double>(g, tp<double>(lo.W), out, 2, s));
    else CMCG_HIP(f2_pack<float>(g, tp<float>(lo.W), out, 2, s));
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  cmcg_status filter(const double *z, double *u_re, double *u_im) override {
    // stage z in hi.W (the forced period writes only A/B/C and its output, here hi.Y is free)
    CMCG_HIP(f2_unpack<double>(g, z, tp<double>(hi.W), 2, s));
    CMCG_HIP(hipMemsetAsync(Ure, 0, cfg.nshots * g.fs * sizeof(double), s));
    CMCG_HIP(hipMemsetAsync(Uim, 0, cfg.nshots * g.fs * sizeof(double), s));
    CMCG_TRY(fwd(hi, true, hi.W, hi.Y, nullptr, true));
    CMCG_TRY(output_fields(tp<double>(hi.W), u_re, u_im));
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  cmcg_status get_state(int which, double *out) override {
    if (which == 0) {
      const double *z = Z;
      CMCG_TRY(current_iterate(tp<double>(hi.W), &z));
      CMCG_HIP(f2_pack<double>(g, z, out, 2, s));
    } else if (which == 1) {
      // primal residual (r_u, M^{-1} rh_v)
      if (mixed)
        CMCG_HIP((f2_primal<float, double>(g, tpc<float>(RU), tpc<float>(RH),
                                           tpc<double>(hi.lam), tp<double>(hi.W), s)));
      else
        CMCG_HIP((f2_primal<double, double>(g, tpc<double>(RU), tpc<double>(RH),
                                            tpc<double>(hi.lam), tp<double>(hi.W), s)));
      CMCG_HIP(f2_pack<double>(g, tp<double>(hi.W), out, 2, s));
    } else if (mixed) {
      CMCG_HIP(f2_pack<float>(g, tp<float>(D), out, 2, s));
    } else {
      CMCG_HIP(f2_pack<double>(g, tp<double>(D), out, 2, s));
    }
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  cmcg_status runup(int periods, int ramp, double *z_out) override {
    CMCG_TRY(run_forced_periods(periods, ramp != 0, tp<double>(hi.W)));
    CMCG_HIP(f2_pack<double>(g, tp<double>(hi.W), z_out, 2, s));
    CMCG_HIP(hipStreamSynchronize(s));
    return CMCG_OK;
  }

  cmcg_status misfit(const double *z, double *J) override {
    // w = Phi(z) - z with one FP64 forced period, y = M_E w, J = w . y / 2
    double *a = tp<double>(hi.Y), *w = tp<double>(hi.W);
    CMCG_HIP(f2_unpack<double>(g, z, a, 2, s));
    CMCG_TRY(fwd(hi, true, a, w, a, false));
    CMCG_TRY(metric(hi, w, a));
    CMCG_HIP(dot_plain<double, double>(w, a, 2 * g.fs, partials, s));
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
    r->seconds_riesz = t_riesz;
    r->seconds_other = t_other;
    r->grid_updates = updates;
    r->dram_bytes = dram;
    r->riesz_iterations = riesz_iters;
    r->riesz_unconverged = riesz_unconverged;
    r->seconds_bulk_fwd = bulk.seconds[0];
    r->seconds_bulk_adj = bulk.seconds[1];
    r->bulk_launches_fwd = bulk.launches[0];
    r->bulk_launches_adj = bulk.launches[1];
    r->fp64_refreshes = refreshes;
    r->runup_periods = runup_done;
    r->seconds_runup = t_runup;
  }

  void info(cmcg_info *i) const override {
    const int64_t nn = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    i->steps_per_period = cfg.N;
    i->dt = cfg.dt;
    i->T = cfg.T;
    i->h = cfg.h;
    i->state_len = 2 * nn;
    i->field_len = nn;
    i->device_bytes = (int64_t)arena.bytes();
    i->n_fields = cfg.nshots;
    // the set that runs the CG iterations' periods
    i->steps_per_launch = lo.kstep;
    if (lo.kstep > 1) {
      if (mixed) f2_block_shape<float>(&i->block_rows, &i->block_waves);
      else f2_block_shape<double>(&i->block_rows, &i->block_waves);
    }
  }
};

}  // namespace

cmcg_status make_f2_solver(const cmcg_problem *P, const SolverConfig &cfg, Solver **out) {
  *out = nullptr;
  if (P->n[2] < 2) return set_error("second-order solver needs n[2] >= 2"), CMCG_EINVAL;
  F2Solver *S = new F2Solver();
  S->cfg = cfg;
  cmcg_status st = S->create(P);
  if (st != CMCG_OK) {
    delete S;
    return st;
  }
  *out = S;
  return CMCG_OK;
}

}  // namespace cmcg
