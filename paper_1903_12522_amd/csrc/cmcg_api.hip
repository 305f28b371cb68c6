// C ABI and solver runtime: validation, memory plan, period loops, the CG driver of the CMCG
// Algorithm (Sec. 2.3, Steps 1-6) and the output filter.  All arithmetic of the method runs in
// the HIP kernels; the host only sequences launches and reads back the stop-test scalar.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>

#include "cmcg_internal.h"
#include "f2_runtime.h"

namespace cmcg {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

namespace {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------------------
// Setup kernels (run once in cmcg_create)
// ---------------------------------------------------------------------------------------
// c^2 per cell and the forcing amplitude Fhat = f + (1/h) sum_abs gS of every cell (the
// boundary data enters the velocity equation through the boundary flux p.n = gS - v/c).
template <typename T>
__global__ void f1_setup_kernel(F1Geom g, const double *c, double c_const, const double *fre,
                                const double *fim, const double *gre, const double *gim,
                                T *cc, T *Fre, T *Fim, size_t fs) {
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
    cc[o] = (T)(cv * cv);
    double ar = fre ? fre[k] : 0.0, ai = fim ? fim[k] : 0.0;
    const double ih = 1.0 / g.h;
    // faces: -x (ny values), +x (ny), -y (nx), +y (nx)
    if (gre || gim) {
      const size_t off[4] = {0, (size_t)ny, (size_t)2 * ny, (size_t)2 * ny + nx};
      const bool on[4] = {i == 0, i == nx - 1, j == 0, j == ny - 1};
      const int along[4] = {j, j, i, i};
      for (int f = 0; f < 4; ++f) {
        if (!on[f] || !g.abs_face[f]) continue;
        if (gre) ar += gre[off[f] + along[f]] * ih;
        if (gim) ai += gim[off[f] + along[f]] * ih;
      }
    }
    Fre[o] = (T)ar;
    if (Fim) Fim[o] = (T)ai;
  }
}

// u = i V / omega with V = (2/N) (Ure + i Uim)  (eq. TH_FILTERED_MIXED_SOLUTION, discrete)
__global__ void f1_output_kernel(F1Geom g, const double *ure, const double *uim, double scale,
                                 double *out_re, double *out_im, size_t fs) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < fs; o += stride) {
    out_re[o] = -scale * uim[o];
    out_im[o] = scale * ure[o];
  }
}

// F1 Riesz map M_E^{-1} y on the device layout
template <typename T>
__global__ void f1_riesz_kernel(F1Geom g, T *y, const T *cc, size_t fs) {
  const double ih2 = 1.0 / (g.h * g.h);
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < fs; o += stride) {
    y[o] = (T)((double)y[o] * ih2);
    y[o + fs] = (T)((double)y[o + fs] * ih2);
    y[o + 2 * fs] = (T)((double)y[o + 2 * fs] * ih2 * (double)cc[o]);
  }
}

int grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)std::max<size_t>(1, std::min<size_t>(b, 8192));
}

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

}  // namespace
}  // namespace cmcg

using namespace cmcg;

struct cmcg_handle {
  // problem
  int dim = 0, form = 0, prec = 0;
  int64_t n[3] = {0, 0, 0};
  double h = 0, omega = 0, T = 0, dt = 0;
  int N = 0;
  int bc[6] = {0, 0, 0, 0, 0, 0};
  double tol = 1e-6;
  int max_iter = 1000;
  int kblock = 4;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t device_bytes = 0;
  std::vector<void *> allocs;
  // F1 state
  F1Geom g1{};
  size_t fs = 0;       // field stride
  size_t vecN = 0;     // 3 * fs
  size_t esz = 8;      // element size of T
  void *S0 = nullptr, *S1 = nullptr, *W = nullptr, *Q = nullptr, *D = nullptr;
  double *Z = nullptr, *R = nullptr;
  void *cc = nullptr, *Fre = nullptr, *Fim = nullptr;
  double *Ure = nullptr, *Uim = nullptr;
  double *partials = nullptr, *scalars = nullptr, *h_scalars = nullptr;
  // F2 state
  F2Solver *f2 = nullptr;
  // iteration state
  bool started = false;
  int iter = 0;
  double rel = 1.0;
  hipEvent_t ev[8] = {};
  double t_fwd = 0, t_adj = 0, t_riesz = 0, t_other = 0, t_total = 0;
  double updates = 0;
};

namespace {

cmcg_status dev_alloc(cmcg_handle *H, size_t bytes, void **p) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    set_error(std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
    (void)hipGetLastError();
    return CMCG_ENOMEM;
  }
  H->allocs.push_back(*p);
  H->device_bytes += bytes;
  CMCG_HIP(hipMemsetAsync(*p, 0, bytes, H->stream));
  return CMCG_OK;
}

template <typename T>
T *tp(void *p) { return static_cast<T *>(p); }

// ---------------------------------------------------------------------------------------
// F1 period loops
// ---------------------------------------------------------------------------------------
template <typename T>
cmcg_status f1_period(cmcg_handle *H, bool adjoint, bool forced, const T *in, T *out,
                      const T *sub, int steps, bool filter) {
  const int K = filter ? 1 : H->kblock;
  int n0 = 0, l = 0;
  T *S[2] = {tp<T>(H->S0), tp<T>(H->S1)};
  while (n0 < steps) {
    const int ns = std::min(K, steps - n0);
    const bool lastl = (n0 + ns == steps);
    F1Launch L{};
    L.nsteps = ns;
    L.first = (n0 == 0);
    L.last = lastl;
    L.forced = forced ? 1 : 0;
    L.accumulate = filter ? 1 : 0;
    for (int s = 0; s < ns; ++s) {
      const double t = (n0 + s + 0.5) * H->dt;
      L.cs[s] = std::cos(H->omega * t);
      L.sn[s] = std::sin(H->omega * t);
    }
    L.fcos = std::cos(H->omega * n0 * H->dt);
    L.fsin = std::sin(H->omega * n0 * H->dt);
    F1Ptrs<T> p{};
    p.in = (l == 0) ? in : S[(l - 1) & 1];
    p.out = lastl ? out : S[l & 1];
    p.sub = lastl ? sub : nullptr;
    p.cc = tp<T>(H->cc);
    p.fre = tp<T>(H->Fre);
    p.fim = tp<T>(H->Fim);
    p.ure = H->Ure;
    p.uim = H->Uim;
    p.fs = H->fs;
    hipError_t e = adjoint ? f1_adjoint_launch<T>(H->g1, p, L, K, H->stream)
                           : f1_forward_launch<T>(H->g1, p, L, K, H->stream);
    CMCG_HIP(e);
    n0 += ns;
    ++l;
  }
  H->updates += (double)steps * H->g1.nx * H->g1.ny;
  return CMCG_OK;
}

double elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
  return ms * 1e-3;
}

template <typename T>
cmcg_status f1_begin(cmcg_handle *H) {
  hipStream_t s = H->stream;
  T *W = tp<T>(H->W), *Q = tp<T>(H->Q), *D = tp<T>(H->D);
  const size_t vb = H->vecN * sizeof(T);
  H->updates = 0;
  CMCG_HIP(hipEventRecord(H->ev[0], s));
  // Step 2: forced period from z = 0 gives w = Phi(0) - 0; backward period gives the gradient.
  CMCG_HIP(hipMemsetAsync(Q, 0, vb, s));
  CMCG_TRY(f1_period<T>(H, false, true, Q, W, nullptr, H->N, false));
  CMCG_TRY(f1_period<T>(H, true, false, W, Q, W, H->N, false));
  // Steps 3-4: r = d = gradient (Riesz map of F1 is M_E^{-1}, already applied by E*).
  CMCG_HIP(hipMemsetAsync(H->Z, 0, H->vecN * sizeof(double), s));
  CMCG_HIP(convert<double, T>(H->R, Q, H->vecN, s));
  CMCG_HIP(hipMemcpyAsync(D, Q, vb, hipMemcpyDeviceToDevice, s));
  CMCG_HIP(f1_dot<double, double>(H->g1, H->R, H->R, H->cc, H->prec == CMCG_FP64, H->fs,
                                  H->partials, s));
  CMCG_HIP(finalize(H->partials, kRedBlocks, H->scalars, kFinStart, 0, s));
  CMCG_HIP(hipMemcpyAsync(H->h_scalars, H->scalars, kNumScalars * sizeof(double),
                          hipMemcpyDeviceToHost, s));
  CMCG_HIP(hipEventRecord(H->ev[1], s));
  CMCG_HIP(hipStreamSynchronize(s));
  H->t_other += elapsed(H->ev[0], H->ev[1]);
  H->iter = 0;
  H->rel = 1.0;
  H->started = true;
  if (H->h_scalars[kBreak] != 0.0) {
    set_error("non-finite initial gradient");
    return CMCG_EBREAKDOWN;
  }
  return CMCG_OK;
}

template <typename T>
cmcg_status f1_iterate(cmcg_handle *H, int iters, int *converged) {
  hipStream_t s = H->stream;
  T *W = tp<T>(H->W), *Q = tp<T>(H->Q), *D = tp<T>(H->D);
  *converged = (H->rel <= H->tol || H->h_scalars[kDelta0] == 0.0) ? 1 : 0;
  for (int it = 0; it < iters && !*converged; ++it) {
    CMCG_HIP(hipEventRecord(H->ev[2], s));
    // Step 5.1: forward period on d (w = E d - d), backward period (q = E* w - w).
    CMCG_TRY(f1_period<T>(H, false, false, D, W, D, H->N, false));
    CMCG_HIP(hipEventRecord(H->ev[3], s));
    CMCG_TRY(f1_period<T>(H, true, false, W, Q, W, H->N, false));
    CMCG_HIP(hipEventRecord(H->ev[4], s));
    // Step 5.3: alpha = delta / <q, d>_E
    CMCG_HIP(f1_dot<T, T>(H->g1, Q, D, H->cc, H->prec == CMCG_FP64, H->fs, H->partials, s));
    CMCG_HIP(finalize(H->partials, kRedBlocks, H->scalars, kFinAlpha, 0, s));
    // Steps 5.4-5.5 and the new <r, r>_E; Step 5.6 beta; Step 5.7 d = r + beta d
    CMCG_HIP(f1_cg_update<T>(H->g1, H->Z, H->R, D, Q, H->cc, H->fs, H->scalars, H->partials, s));
    CMCG_HIP(finalize(H->partials, kRedBlocks, H->scalars, kFinBeta, 0, s));
    CMCG_HIP(direction_update<T>(D, H->R, H->scalars, H->vecN, s));
    CMCG_HIP(hipMemcpyAsync(H->h_scalars, H->scalars, kNumScalars * sizeof(double),
                            hipMemcpyDeviceToHost, s));
    CMCG_HIP(hipEventRecord(H->ev[5], s));
    CMCG_HIP(hipStreamSynchronize(s));
    H->t_fwd += elapsed(H->ev[2], H->ev[3]);
    H->t_adj += elapsed(H->ev[3], H->ev[4]);
    H->t_other += elapsed(H->ev[4], H->ev[5]);
    H->iter += 1;
    if (H->h_scalars[kBreak] != 0.0) {
      set_error("CG breakdown: <qhat, d> <= 0 or non-finite scalar");
      return CMCG_EBREAKDOWN;
    }
    H->rel = H->h_scalars[kRel];
    // Step 5.8
    if (H->rel <= H->tol) *converged = 1;
  }
  return CMCG_OK;
}

template <typename T>
cmcg_status f1_filter_from(cmcg_handle *H, const T *z, double *u_re, double *u_im) {
  hipStream_t s = H->stream;
  const size_t fb = H->fs * sizeof(double);
  CMCG_HIP(hipMemsetAsync(H->Ure, 0, fb, s));
  CMCG_HIP(hipMemsetAsync(H->Uim, 0, fb, s));
  CMCG_TRY(f1_period<T>(H, false, true, z, tp<T>(H->Q), nullptr, H->N, true));
  // scale in place into the (now free) FP64 residual buffer, then copy rows out
  double *ore = H->R, *oim = H->R + H->fs;
  const double scale = 2.0 / (H->N * H->omega);
  hipLaunchKernelGGL(f1_output_kernel, dim3(grid_for(H->fs)), dim3(256), 0, s, H->g1, H->Ure,
                     H->Uim, scale, ore, oim, H->fs);
  CMCG_HIP(hipGetLastError());
  CMCG_HIP(hipEventRecord(H->ev[6], s));
  const size_t row = (size_t)H->g1.nx * sizeof(double);
  const size_t pitchb = (size_t)H->g1.pitch * sizeof(double);
  if (u_re)
    CMCG_HIP(hipMemcpy2DAsync(u_re, row, ore, pitchb, row, H->g1.ny, hipMemcpyDefault, s));
  if (u_im)
    CMCG_HIP(hipMemcpy2DAsync(u_im, row, oim, pitchb, row, H->g1.ny, hipMemcpyDefault, s));
  CMCG_HIP(hipStreamSynchronize(s));
  return CMCG_OK;
}

template <typename T>
cmcg_status f1_finish(cmcg_handle *H, double *u_re, double *u_im) {
  // Step 6 via the filter: one forced period from z (rounded to the field precision)
  CMCG_HIP(convert<T, double>(tp<T>(H->W), H->Z, H->vecN, H->stream));
  cmcg_status st = f1_filter_from<T>(H, tp<T>(H->W), u_re, u_im);
  // the residual buffer held the output; the solve is over, so it is not needed any more
  H->started = false;
  return st;
}

template <typename T>
cmcg_status f1_apply(cmcg_handle *H, int op, int steps, const double *in, double *out) {
  hipStream_t s = H->stream;
  T *W = tp<T>(H->W), *Q = tp<T>(H->Q);
  CMCG_HIP(f1_unpack<T>(H->g1, in, W, H->fs, s));
  const int ns = steps > 0 ? steps : H->N;
  if (op == CMCG_OP_FORWARD || op == CMCG_OP_FORCED) {
    CMCG_TRY(f1_period<T>(H, false, op == CMCG_OP_FORCED, W, Q, nullptr, ns, false));
  } else if (op == CMCG_OP_ADJOINT) {
    CMCG_TRY(f1_period<T>(H, true, false, W, Q, nullptr, ns, false));
  } else {
    hipLaunchKernelGGL((f1_riesz_kernel<T>), dim3(grid_for(H->fs)), dim3(256), 0, s, H->g1, W,
                       tp<T>(H->cc), H->fs);
    CMCG_HIP(hipGetLastError());
    Q = W;
  }
  CMCG_HIP(f1_pack<T>(H->g1, Q, out, H->fs, s));
  CMCG_HIP(hipStreamSynchronize(s));
  return CMCG_OK;
}

// ---------------------------------------------------------------------------------------
// create
// ---------------------------------------------------------------------------------------
cmcg_status validate(const cmcg_problem *P, const cmcg_options *O) {
  if (!P || !O) return set_error("null problem or options"), CMCG_EINVAL;
  if (P->dim != 2 && P->dim != 3) return set_error("dim must be 2 or 3"), CMCG_EINVAL;
  if (P->formulation != 1 && P->formulation != 2)
    return set_error("formulation must be 1 or 2"), CMCG_EINVAL;
  for (int k = 0; k < P->dim; ++k)
    if (P->n[k] < 2 || P->n[k] > (1 << 20)) return set_error("n out of range"), CMCG_EINVAL;
  if (!(P->omega > 0.0) || !std::isfinite(P->omega)) return set_error("omega must be > 0"), CMCG_EINVAL;
  if (!P->c && (!(P->c_const > 0.0) || !std::isfinite(P->c_const)))
    return set_error("c_const must be > 0"), CMCG_EINVAL;
  for (int k = 0; k < 2 * P->dim; ++k)
    if (P->face_bc[k] != CMCG_ABSORBING && P->face_bc[k] != CMCG_NEUMANN)
      return set_error("face_bc must be 0 or 1"), CMCG_EINVAL;
  const double sigma = P->courant == 0.0 ? 0.5 : P->courant;
  if (!(sigma > 0.0)) return set_error("courant must be > 0"), CMCG_EINVAL;
  if (sigma * std::sqrt((double)P->dim) >= 1.0)
    return set_error("courant * sqrt(dim) >= 1: leapfrog unstable"), CMCG_ECFL;
  if (O->precision != CMCG_FP64 && O->precision != CMCG_FP32_MIXED)
    return set_error("precision must be 0 or 1"), CMCG_EINVAL;
  if (!(O->tol >= 0.0) || O->max_iter <= 0) return set_error("tol >= 0 and max_iter > 0 required"), CMCG_EINVAL;
  if (!((P->dim == 2 && P->formulation == 1) || (P->dim == 3 && P->formulation == 2)))
    return set_error("supported: dim 2 with formulation 1, dim 3 with formulation 2"),
           CMCG_EUNSUPPORTED;
  return CMCG_OK;
}

template <typename T>
cmcg_status f1_create(cmcg_handle *H, const cmcg_problem *P) {
  const int nx = (int)P->n[0], ny = (int)P->n[1];
  hipStream_t s = H->stream;
  F1Geom &g = H->g1;
  g.nx = nx;
  g.ny = ny;
  g.pitch = (nx + 63) / 64 * 64;
  g.h = H->h;
  g.dt = H->dt;
  for (int f = 0; f < 4; ++f) g.abs_face[f] = P->face_bc[f] == CMCG_ABSORBING ? 1 : 0;
  H->fs = (size_t)ny * g.pitch;
  H->vecN = 3 * H->fs;
  H->esz = sizeof(T);
  const size_t vb = H->vecN * sizeof(T), fb = H->fs * sizeof(T);
  CMCG_TRY(dev_alloc(H, vb, &H->S0));
  CMCG_TRY(dev_alloc(H, vb, &H->S1));
  CMCG_TRY(dev_alloc(H, vb, &H->W));
  CMCG_TRY(dev_alloc(H, vb, &H->Q));
  CMCG_TRY(dev_alloc(H, vb, &H->D));
  CMCG_TRY(dev_alloc(H, H->vecN * sizeof(double), (void **)&H->Z));
  CMCG_TRY(dev_alloc(H, H->vecN * sizeof(double), (void **)&H->R));
  CMCG_TRY(dev_alloc(H, fb, &H->cc));
  CMCG_TRY(dev_alloc(H, fb, &H->Fre));
  if (P->f_im || P->gS_im) CMCG_TRY(dev_alloc(H, fb, &H->Fim));
  CMCG_TRY(dev_alloc(H, H->fs * sizeof(double), (void **)&H->Ure));
  CMCG_TRY(dev_alloc(H, H->fs * sizeof(double), (void **)&H->Uim));
  // host inputs -> temporary device copies -> setup kernel
  const size_t ncell = (size_t)nx * ny, nface = 2 * (size_t)ny + 2 * (size_t)nx;
  std::vector<void *> tmp;
  auto upload = [&](const double *src, size_t n, double **dst) -> cmcg_status {
    *dst = nullptr;
    if (!src) return CMCG_OK;
    void *p = nullptr;
    CMCG_HIP(hipMalloc(&p, n * sizeof(double)));
    tmp.push_back(p);
    CMCG_HIP(hipMemcpyAsync(p, src, n * sizeof(double), hipMemcpyHostToDevice, s));
    *dst = static_cast<double *>(p);
    return CMCG_OK;
  };
  double *dc, *dfr, *dfi, *dgr, *dgi;
  cmcg_status st = CMCG_OK;
  if ((st = upload(P->c, ncell, &dc)) == CMCG_OK && (st = upload(P->f_re, ncell, &dfr)) == CMCG_OK &&
      (st = upload(P->f_im, ncell, &dfi)) == CMCG_OK && (st = upload(P->gS_re, nface, &dgr)) == CMCG_OK &&
      (st = upload(P->gS_im, nface, &dgi)) == CMCG_OK) {
    hipLaunchKernelGGL((f1_setup_kernel<T>), dim3(grid_for(H->fs)), dim3(256), 0, s, g, dc,
                       P->c_const, dfr, dfi, dgr, dgi, tp<T>(H->cc), tp<T>(H->Fre), tp<T>(H->Fim),
                       H->fs);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      set_error(std::string("f1 setup: ") + hipGetErrorString(e));
      st = CMCG_EDEVICE;
    }
  }
  hipStreamSynchronize(s);
  for (void *p : tmp) hipFree(p);
  return st;
}

}  // namespace

// =========================================================================================
// extern "C" API
// =========================================================================================
extern "C" {

const char *cmcg_status_string(cmcg_status s) {
  switch (s) {
    case CMCG_OK: return "ok";
    case CMCG_ENOTCONV: return "not converged (max_iter reached)";
    case CMCG_EINVAL: return "invalid argument";
    case CMCG_ECFL: return "CFL condition violated";
    case CMCG_ENOMEM: return "out of device memory";
    case CMCG_EDEVICE: return "HIP device error";
    case CMCG_EBREAKDOWN: return "CG breakdown";
    case CMCG_EUNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

const char *cmcg_last_error(void) { return g_last_error.c_str(); }

void cmcg_destroy(cmcg_handle *H) {
  if (!H) return;
  hipSetDevice(H->device);
  if (H->stream) hipStreamSynchronize(H->stream);
  if (H->f2) {
    f2_destroy(H->f2);
    H->f2 = nullptr;
  }
  for (void *p : H->allocs) hipFree(p);
  if (H->h_scalars) hipHostFree(H->h_scalars);
  for (auto &e : H->ev)
    if (e) hipEventDestroy(e);
  if (H->own_stream && H->stream) hipStreamDestroy(H->stream);
  delete H;
}

cmcg_status cmcg_create(const cmcg_problem *P, const cmcg_options *O, cmcg_handle **out) {
  if (!out) return set_error("out is NULL"), CMCG_EINVAL;
  *out = nullptr;
  g_last_error.clear();
  CMCG_TRY(validate(P, O));
  const int dim = P->dim;
  // wave speed checks (host-side validation of the input only)
  const int64_t nnodes = P->formulation == 1 ? P->n[0] * P->n[1]
                                             : (P->n[0] + 1) * (P->n[1] + 1) * (dim == 3 ? P->n[2] + 1 : 1);
  double cmax = P->c_const;
  if (P->c) {
    cmax = 0.0;
    for (int64_t k = 0; k < nnodes; ++k) {
      const double c = P->c[k];
      if (!(c > 0.0) || !std::isfinite(c)) return set_error("c must be finite and > 0"), CMCG_EINVAL;
      cmax = std::max(cmax, c);
    }
  }
  int ndev = 0;
  const hipError_t de = hipGetDeviceCount(&ndev);
  if (de != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return set_error(std::string("no HIP device: hipGetDeviceCount -> ") + hipGetErrorString(de) +
                     ", count " + std::to_string(ndev)),
           CMCG_EDEVICE;
  }
  if (O->device < 0 || O->device >= ndev) return set_error("device ordinal out of range"), CMCG_EINVAL;
  std::unique_ptr<cmcg_handle> H(new cmcg_handle());
  H->dim = dim;
  H->form = P->formulation;
  H->prec = O->precision;
  for (int k = 0; k < 3; ++k) H->n[k] = P->n[k];
  for (int k = 0; k < 6; ++k) H->bc[k] = P->face_bc[k];
  H->h = 1.0 / (double)P->n[0];
  H->omega = P->omega;
  H->T = 2.0 * kPi / P->omega;
  const double sigma = P->courant == 0.0 ? 0.5 : P->courant;
  H->N = (int)std::ceil(H->T * cmax / (sigma * H->h));
  if (H->N < 3) H->N = 3;
  H->dt = H->T / H->N;
  H->tol = O->tol;
  H->max_iter = O->max_iter;
  H->device = O->device;
  int kb = O->steps_per_launch > 0 ? O->steps_per_launch : 4;
  if (kb < 1 || kb > kMaxBlockSteps) return set_error("steps_per_launch must be in 1..8"), CMCG_EINVAL;
  H->kblock = kb;
  CMCG_HIP(hipSetDevice(H->device));
  if (O->hip_stream) {
    H->stream = static_cast<hipStream_t>(O->hip_stream);
  } else {
    CMCG_HIP(hipStreamCreateWithFlags(&H->stream, hipStreamNonBlocking));
    H->own_stream = true;
  }
  for (auto &e : H->ev) CMCG_HIP(hipEventCreate(&e));
  CMCG_HIP(hipHostMalloc((void **)&H->h_scalars, kNumScalars * sizeof(double)));
  std::memset(H->h_scalars, 0, kNumScalars * sizeof(double));
  cmcg_status st;
  if (H->form == 1) {
    CMCG_TRY(dev_alloc(H.get(), kRedBlocks * sizeof(double), (void **)&H->partials));
    CMCG_TRY(dev_alloc(H.get(), kNumScalars * sizeof(double), (void **)&H->scalars));
    st = H->prec == CMCG_FP64 ? f1_create<double>(H.get(), P) : f1_create<float>(H.get(), P);
  } else {
    F2Params fp{};
    fp.n[0] = (int)P->n[0];
    fp.n[1] = (int)P->n[1];
    fp.n[2] = (int)P->n[2];
    fp.h = H->h;
    fp.dt = H->dt;
    fp.omega = H->omega;
    fp.N = H->N;
    fp.prec = H->prec;
    fp.kblock = H->kblock;
    for (int k = 0; k < 6; ++k) fp.abs_face[k] = P->face_bc[k] == CMCG_ABSORBING ? 1 : 0;
    fp.tol = H->tol;
    fp.max_iter = H->max_iter;
    fp.riesz_tol = O->riesz_tol > 0 ? O->riesz_tol : 0.0;
    fp.riesz_max_iter = O->riesz_max_iter > 0 ? O->riesz_max_iter : 0;
    st = f2_create(&H->f2, fp, P, H->stream);
    if (st == CMCG_OK) H->device_bytes += f2_device_bytes(H->f2);
  }
  if (st != CMCG_OK) {
    cmcg_destroy(H.release());
    return st;
  }
  *out = H.release();
  return CMCG_OK;
}

cmcg_status cmcg_get_info(const cmcg_handle *H, cmcg_info *info) {
  if (!H || !info) return set_error("null argument"), CMCG_EINVAL;
  info->steps_per_period = H->N;
  info->dt = H->dt;
  info->T = H->T;
  info->h = H->h;
  if (H->form == 1) {
    const int64_t nx = H->n[0], ny = H->n[1];
    info->state_len = ny * (nx - 1) + (ny - 1) * nx + nx * ny;
    info->field_len = nx * ny;
  } else {
    const int64_t nn = (H->n[0] + 1) * (H->n[1] + 1) * (H->n[2] + 1);
    info->state_len = 2 * nn;
    info->field_len = nn;
  }
  info->device_bytes = (int64_t)H->device_bytes;
  return CMCG_OK;
}

static void fill_report(cmcg_handle *H, cmcg_report *rep) {
  if (!rep) return;
  if (H->form == 2) {
    f2_report(H->f2, rep);
    return;
  }
  rep->iterations = H->iter;
  rep->steps_per_period = H->N;
  rep->dt = H->dt;
  rep->rel_residual = H->rel;
  rep->seconds = H->t_total;
  rep->seconds_fwd = H->t_fwd;
  rep->seconds_adj = H->t_adj;
  rep->seconds_riesz = H->t_riesz;
  rep->seconds_other = H->t_other;
  rep->grid_updates = H->updates;
  rep->riesz_iterations = 0;
}

cmcg_status cmcg_begin(cmcg_handle *H) {
  if (!H) return set_error("null handle"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  if (H->form == 2) return f2_begin(H->f2);
  H->t_fwd = H->t_adj = H->t_riesz = H->t_other = H->t_total = 0.0;
  return H->prec == CMCG_FP64 ? f1_begin<double>(H) : f1_begin<float>(H);
}

cmcg_status cmcg_iterate(cmcg_handle *H, int32_t iters, int32_t *converged, cmcg_report *rep) {
  if (!H || iters < 0) return set_error("bad argument"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  int conv = 0;
  cmcg_status st;
  if (H->form == 2) {
    st = f2_iterate(H->f2, iters, &conv);
  } else {
    if (!H->started) return set_error("cmcg_begin first"), CMCG_EINVAL;
    st = H->prec == CMCG_FP64 ? f1_iterate<double>(H, iters, &conv) : f1_iterate<float>(H, iters, &conv);
  }
  if (converged) *converged = conv;
  fill_report(H, rep);
  return st;
}

cmcg_status cmcg_finish(cmcg_handle *H, double *u_re, double *u_im, cmcg_report *rep) {
  if (!H) return set_error("null handle"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  cmcg_status st;
  if (H->form == 2) {
    st = f2_finish(H->f2, u_re, u_im);
  } else {
    if (!H->started) return set_error("cmcg_begin first"), CMCG_EINVAL;
    st = H->prec == CMCG_FP64 ? f1_finish<double>(H, u_re, u_im) : f1_finish<float>(H, u_re, u_im);
  }
  fill_report(H, rep);
  return st;
}

cmcg_status cmcg_solve(cmcg_handle *H, double *u_re, double *u_im, cmcg_report *rep) {
  if (!H) return set_error("null handle"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  if (H->form == 2) {
    cmcg_status st = f2_solve(H->f2, u_re, u_im);
    fill_report(H, rep);
    return st;
  }
  const auto t0 = std::chrono::steady_clock::now();
  CMCG_TRY(cmcg_begin(H));
  int conv = 0;
  CMCG_TRY(H->prec == CMCG_FP64 ? f1_iterate<double>(H, H->max_iter, &conv)
                                : f1_iterate<float>(H, H->max_iter, &conv));
  CMCG_HIP(hipEventRecord(H->ev[7], H->stream));
  cmcg_status st = H->prec == CMCG_FP64 ? f1_finish<double>(H, u_re, u_im) : f1_finish<float>(H, u_re, u_im);
  if (st < 0) return st;
  H->t_other += elapsed(H->ev[7], H->ev[6]);
  H->t_total = elapsed(H->ev[0], H->ev[6]);
  (void)t0;
  fill_report(H, rep);
  return conv ? CMCG_OK : CMCG_ENOTCONV;
}

cmcg_status cmcg_apply(cmcg_handle *H, int32_t op, int32_t steps, const double *in, double *out) {
  if (!H || !in || !out || op < 0 || op > 3 || steps < 0) return set_error("bad argument"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  if (H->form == 2) {
    if (steps != 0) return set_error("F2: steps must be 0"), CMCG_EINVAL;
    return f2_apply(H->f2, op, in, out);
  }
  return H->prec == CMCG_FP64 ? f1_apply<double>(H, op, steps, in, out)
                              : f1_apply<float>(H, op, steps, in, out);
}

cmcg_status cmcg_filter(cmcg_handle *H, const double *z, double *u_re, double *u_im) {
  if (!H || !z) return set_error("bad argument"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  if (H->form == 2) return f2_filter(H->f2, z, u_re, u_im);
  if (H->prec == CMCG_FP64) {
    CMCG_HIP(f1_unpack<double>(H->g1, z, tp<double>(H->W), H->fs, H->stream));
    return f1_filter_from<double>(H, tp<double>(H->W), u_re, u_im);
  }
  CMCG_HIP(f1_unpack<float>(H->g1, z, tp<float>(H->W), H->fs, H->stream));
  return f1_filter_from<float>(H, tp<float>(H->W), u_re, u_im);
}

cmcg_status cmcg_get_state(cmcg_handle *H, int32_t which, double *out) {
  if (!H || !out || which < 0 || which > 2) return set_error("bad argument"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  if (H->form == 2) return f2_get_state(H->f2, which, out);
  hipStream_t s = H->stream;
  if (which == 0) CMCG_HIP(f1_pack<double>(H->g1, H->Z, out, H->fs, s));
  else if (which == 1) CMCG_HIP(f1_pack<double>(H->g1, H->R, out, H->fs, s));
  else if (H->prec == CMCG_FP64) CMCG_HIP(f1_pack<double>(H->g1, tp<double>(H->D), out, H->fs, s));
  else CMCG_HIP(f1_pack<float>(H->g1, tp<float>(H->D), out, H->fs, s));
  CMCG_HIP(hipStreamSynchronize(s));
  return CMCG_OK;
}

}  // extern "C"
