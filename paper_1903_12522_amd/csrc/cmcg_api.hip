// C ABI: argument validation, the period-count rule (an integer number N of leapfrog steps per
// period, dt = T / N), and dispatch to the formulation's solver.  No arithmetic of the method
// happens here; it all runs in the HIP kernels of the solvers.
#include <cstring>
#include <memory>

#include "solver.h"

namespace cmcg {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

namespace {

constexpr double kPi = 3.14159265358979323846;

}  // namespace

cmcg_status validate_problem(const cmcg_problem *P, const cmcg_options *O) {
  if (!P || !O) return set_error("null problem or options"), CMCG_EINVAL;
  if (P->dim != 2 && P->dim != 3) return set_error("dim must be 2 or 3"), CMCG_EINVAL;
  if (P->formulation != 1 && P->formulation != 2)
    return set_error("formulation must be 1 or 2"), CMCG_EINVAL;
  for (int k = 0; k < P->dim; ++k)
    if (P->n[k] < 2 || P->n[k] > (1 << 20)) return set_error("n out of range"), CMCG_EINVAL;
  if (!(P->omega > 0.0) || !std::isfinite(P->omega))
    return set_error("omega must be finite and > 0"), CMCG_EINVAL;
  if (!P->c && (!(P->c_const > 0.0) || !std::isfinite(P->c_const)))
    return set_error("c_const must be finite and > 0"), CMCG_EINVAL;
  for (int k = 0; k < 2 * P->dim; ++k)
    if (P->face_bc[k] != CMCG_ABSORBING && P->face_bc[k] != CMCG_NEUMANN)
      return set_error("face_bc entries must be 0 (absorbing) or 1 (Neumann)"), CMCG_EINVAL;
  const double sigma = P->courant == 0.0 ? 0.5 : P->courant;
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return set_error("courant must be > 0"), CMCG_EINVAL;
  if (sigma * std::sqrt((double)P->dim) >= 1.0)
    return set_error("courant * sqrt(dim) >= 1: leapfrog would be unstable"), CMCG_ECFL;
  if (O->precision != CMCG_FP64 && O->precision != CMCG_FP32_MIXED)
    return set_error("precision must be CMCG_FP64 or CMCG_FP32_MIXED"), CMCG_EINVAL;
  if (!(O->tol >= 0.0) || O->max_iter <= 0)
    return set_error("tol >= 0 and max_iter > 0 required"), CMCG_EINVAL;
  if (O->riesz_mode != CMCG_RIESZ_DEFAULT && O->riesz_mode != CMCG_RIESZ_SOLVE &&
      O->riesz_mode != CMCG_RIESZ_VCYCLE)
    return set_error("riesz_mode must be CMCG_RIESZ_DEFAULT, _SOLVE or _VCYCLE"), CMCG_EINVAL;
  if (O->runup_periods < 0 || O->runup_periods > 1000000)
    return set_error("runup_periods must be in [0, 1e6]"), CMCG_EINVAL;
  if (O->steps_per_launch < 0 || O->steps_per_launch > kMaxBlockSteps)
    return set_error("steps_per_launch must be in 0..8"), CMCG_EINVAL;
  if (!((P->dim == 2 && P->formulation == 1) || (P->dim == 3 && P->formulation == 2)))
    return set_error("supported: dim 2 with formulation 1, dim 3 with formulation 2"),
           CMCG_EUNSUPPORTED;
  if (P->n_shots < 0 || P->n_shots > CMCG_MAX_SHOTS)
    return set_error("n_shots must be in 0..CMCG_MAX_SHOTS"), CMCG_EINVAL;
  if (P->n_shots > 0) {
    if (!P->shots) return set_error("n_shots > 0 needs the shots array"), CMCG_EINVAL;
    if (P->f_re || P->f_im || P->gS_re || P->gS_im || P->gD_re || P->gD_im)
      return set_error("with shots, the source and boundary data go in the shots"), CMCG_EINVAL;
    for (int j = 0; j < P->n_shots; ++j) {
      if (P->shots[j].harmonic < 1) return set_error("shot harmonics must be >= 1"), CMCG_EINVAL;
      for (int k = 0; k < j; ++k)
        if (P->shots[k].harmonic == P->shots[j].harmonic)
          return set_error("shot harmonics must be distinct"), CMCG_EINVAL;
    }
  }
  for (const cmcg_shot &sh : shots_of(P))
    if ((sh.gD_re || sh.gD_im) && !P->sound_soft)
      return set_error("Dirichlet data needs a sound-soft mask"), CMCG_EINVAL;
  if (O->output != CMCG_OUTPUT_FILTER && O->output != CMCG_OUTPUT_STEP6)
    return set_error("output must be CMCG_OUTPUT_FILTER or CMCG_OUTPUT_STEP6"), CMCG_EINVAL;
  if (O->output == CMCG_OUTPUT_STEP6) {
    if (P->n_shots > 0)
      return set_error("the Step 6 output reads one frequency off the state: no shots"),
             CMCG_EINVAL;
    if (P->formulation == 2 && !P->sound_soft) {
      bool absorbing = false;
      for (int f = 0; f < 2 * P->dim; ++f) absorbing = absorbing || P->face_bc[f] == CMCG_ABSORBING;
      if (!absorbing)
        return set_error("pure-Neumann box: the Step 6 output misses the mode eta; use the filter"),
               CMCG_EUNSUPPORTED;
    }
  }
  if (O->runup_periods > 0) {
    // a closed box without absorption or Dirichlet nodes drifts linearly under a source with
    // non-zero mean (the eta mode of Sec. 2.2), which the run-up start would carry into CG
    bool damped = P->sound_soft != nullptr;
    for (int f = 0; f < 2 * P->dim; ++f) damped = damped || P->face_bc[f] == CMCG_ABSORBING;
    if (!damped)
      return set_error("the run-up needs an absorbing face or Dirichlet nodes"), CMCG_EUNSUPPORTED;
  }
  return CMCG_OK;
}

cmcg_status make_config(const cmcg_problem *P, const cmcg_options *O, hipStream_t stream,
                        SolverConfig *cfg) {
  CMCG_TRY(validate_problem(P, O));
  const int64_t npts = P->formulation == 1
                           ? P->n[0] * P->n[1]
                           : (P->n[0] + 1) * (P->n[1] + 1) * (P->dim == 3 ? P->n[2] + 1 : 1);
  double cmax = P->c_const;
  if (P->c) {
    cmax = 0.0;
    for (int64_t k = 0; k < npts; ++k) {
      const double c = P->c[k];
      if (!(c > 0.0) || !std::isfinite(c)) return set_error("c must be finite and > 0"), CMCG_EINVAL;
      cmax = std::max(cmax, c);
    }
  }
  cfg->prec = O->precision;
  cfg->tol = O->tol;
  cfg->max_iter = O->max_iter;
  // default temporal blocking depth: the fastest measured on a 4096^2 first-order CG iteration
  // in both precisions (FP64 at K = 8 loses a wave per SIMD in the backward sweep)
  cfg->kblock = O->steps_per_launch > 0 ? O->steps_per_launch : 7;
  cfg->steps_request = O->steps_per_launch;
  cfg->refresh = O->fp64_refresh == 0.0 ? 0.1 : O->fp64_refresh;
  cfg->riesz_tol = O->riesz_tol;
  cfg->riesz_max_iter = O->riesz_max_iter;
  cfg->runup = O->runup_periods;
  cfg->output = O->output;
  cfg->riesz_mode = O->riesz_mode != CMCG_RIESZ_DEFAULT
                        ? O->riesz_mode
                        : (O->precision == CMCG_FP64 ? CMCG_RIESZ_SOLVE : CMCG_RIESZ_VCYCLE);
  cfg->stream = stream;
  cfg->h = 1.0 / (double)P->n[0];
  cfg->omega = P->omega;
  cfg->T = 2.0 * kPi / P->omega;
  const double sigma = P->courant == 0.0 ? 0.5 : P->courant;
  // integer number of leapfrog steps per period, c_max dt / h <= sigma
  cfg->N = std::max(3, (int)std::ceil(cfg->T * cmax / (sigma * cfg->h)));
  cfg->dt = cfg->T / cfg->N;
  const std::vector<cmcg_shot> shots = shots_of(P);
  cfg->nshots = (int)shots.size();
  for (int j = 0; j < cfg->nshots; ++j) {
    cfg->harmonic[j] = shots[j].harmonic;
    // the filters of distinct harmonics m < N / 2 are orthogonal over the N steps of a period
    if (2 * (int64_t)shots[j].harmonic >= cfg->N)
      return set_error("shot harmonic m needs more than 2 m leapfrog steps per base period (N = " +
                       std::to_string(cfg->N) + ")"),
             CMCG_EINVAL;
  }
  return CMCG_OK;
}

}  // namespace cmcg

using namespace cmcg;

struct cmcg_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Solver *solver = nullptr;
  int started = 0;
};

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
  (void)hipSetDevice(H->device);
  if (H->stream) (void)hipStreamSynchronize(H->stream);
  delete H->solver;
  if (H->own_stream && H->stream) (void)hipStreamDestroy(H->stream);
  delete H;
}

cmcg_status cmcg_create(const cmcg_problem *P, const cmcg_options *O, cmcg_handle **out) {
  if (!out) return set_error("out is NULL"), CMCG_EINVAL;
  *out = nullptr;
  g_last_error.clear();
  SolverConfig cfg;
  CMCG_TRY(make_config(P, O, nullptr, &cfg));
  int ndev = 0;
  const hipError_t de = hipGetDeviceCount(&ndev);
  if (de != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return set_error(std::string("no HIP device: ") + hipGetErrorString(de)), CMCG_EDEVICE;
  }
  if (O->device < 0 || O->device >= ndev) return set_error("device ordinal out of range"), CMCG_EINVAL;
  std::unique_ptr<cmcg_handle> H(new cmcg_handle());
  H->device = O->device;
  CMCG_HIP(hipSetDevice(H->device));
  if (O->hip_stream) {
    H->stream = static_cast<hipStream_t>(O->hip_stream);
  } else {
    CMCG_HIP(hipStreamCreateWithFlags(&H->stream, hipStreamNonBlocking));
    H->own_stream = true;
  }
  cfg.stream = H->stream;
  Solver *S = nullptr;
  cmcg_status st = P->formulation == 1 ? make_f1_solver(P, cfg, &S) : make_f2_solver(P, cfg, &S);
  if (st != CMCG_OK) {
    cmcg_destroy(H.release());
    return st;
  }
  H->solver = S;
  *out = H.release();
  return CMCG_OK;
}

cmcg_status cmcg_get_info(const cmcg_handle *H, cmcg_info *info) {
  if (!H || !info) return set_error("null argument"), CMCG_EINVAL;
  *info = cmcg_info{};
  H->solver->info(info);
  return CMCG_OK;
}

cmcg_status cmcg_begin(cmcg_handle *H) {
  if (!H) return set_error("null handle"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  cmcg_status st = H->solver->begin();
  H->started = st == CMCG_OK;
  return st;
}

cmcg_status cmcg_iterate(cmcg_handle *H, int32_t iters, int32_t *converged, cmcg_report *rep) {
  if (!H || iters < 0) return set_error("bad argument"), CMCG_EINVAL;
  if (!H->started) return set_error("cmcg_begin first"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  int conv = 0;
  cmcg_status st = H->solver->iterate(iters, &conv);
  if (converged) *converged = conv;
  if (rep) H->solver->report(rep);
  return st;
}

cmcg_status cmcg_finish(cmcg_handle *H, double *u_re, double *u_im, cmcg_report *rep) {
  if (!H) return set_error("null handle"), CMCG_EINVAL;
  if (!H->started) return set_error("cmcg_begin first"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  cmcg_status st = H->solver->finish(u_re, u_im);
  if (rep) H->solver->report(rep);
  return st;
}

cmcg_status cmcg_solve(cmcg_handle *H, double *u_re, double *u_im, cmcg_report *rep) {
  if (!H) return set_error("null handle"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  cmcg_status st = H->solver->solve(u_re, u_im);
  H->started = st >= 0;
  if (rep) H->solver->report(rep);
  return st;
}

cmcg_status cmcg_apply(cmcg_handle *H, int32_t op, int32_t steps, const double *in, double *out) {
  if (!H || !in || !out || op < 0 || op > 3 || steps < 0)
    return set_error("bad argument"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  return H->solver->apply(op, steps, in, out);
}

cmcg_status cmcg_filter(cmcg_handle *H, const double *z, double *u_re, double *u_im) {
  if (!H || !z) return set_error("bad argument"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  return H->solver->filter(z, u_re, u_im);
}

cmcg_status cmcg_step6(cmcg_handle *H, const double *z, double *u_re, double *u_im) {
  if (!H || !z) return set_error("bad argument"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  return H->solver->step6(z, u_re, u_im);
}

cmcg_status cmcg_get_state(cmcg_handle *H, int32_t which, double *out) {
  if (!H || !out || which < 0 || which > 2) return set_error("bad argument"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  return H->solver->get_state(which, out);
}

cmcg_status cmcg_runup(cmcg_handle *H, int32_t periods, int32_t ramp, double *z_out) {
  if (!H || !z_out || periods < 1 || periods > 1000000)
    return set_error("cmcg_runup: handle, z_out and periods in [1, 1e6] required"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  return H->solver->runup(periods, ramp, z_out);
}

cmcg_status cmcg_misfit(cmcg_handle *H, const double *z, double *J) {
  if (!H || !z || !J) return set_error("cmcg_misfit: null argument"), CMCG_EINVAL;
  CMCG_HIP(hipSetDevice(H->device));
  return H->solver->misfit(z, J);
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// continuous-batching server
// ---------------------------------------------------------------------------------------
struct cmcg_server {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Server *impl = nullptr;
};

extern "C" {

void cmcg_server_destroy(cmcg_server *S) {
  if (!S) return;
  (void)hipSetDevice(S->device);
  delete S->impl;
  if (S->own_stream && S->stream) (void)hipStreamDestroy(S->stream);
  delete S;
}

cmcg_status cmcg_server_create(const cmcg_server_options *o, cmcg_server **out) {
  if (!o || !out) return set_error("null argument"), CMCG_EINVAL;
  *out = nullptr;
  if (o->hbm_budget_bytes <= 0 || o->max_slots < 0 || o->max_slots > kServeMaxSlots ||
      o->steps_per_launch < 0 || o->steps_per_launch > kMaxBlockSteps ||
      o->barrier_spin_limit < 0)
    return set_error("bad server options"), CMCG_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return set_error("no HIP device"), CMCG_EDEVICE;
  }
  if (o->device < 0 || o->device >= ndev) return set_error("device ordinal out of range"), CMCG_EINVAL;
  std::unique_ptr<cmcg_server> S(new cmcg_server());
  S->device = o->device;
  CMCG_HIP(hipSetDevice(S->device));
  if (o->hip_stream) {
    S->stream = static_cast<hipStream_t>(o->hip_stream);
  } else {
    CMCG_HIP(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
    S->own_stream = true;
  }
  cmcg_status st = make_f1_server(o, S->stream, &S->impl);
  if (st != CMCG_OK) {
    cmcg_server_destroy(S.release());
    return st;
  }
  *out = S.release();
  return CMCG_OK;
}

cmcg_status cmcg_server_submit(cmcg_server *S, const cmcg_problem *p, const cmcg_options *o,
                               int64_t *id) {
  if (!S) return set_error("null server"), CMCG_EINVAL;
  return S->impl->submit(p, o, id);
}

cmcg_status cmcg_server_step(cmcg_server *S, int32_t *active, int32_t *queued) {
  if (!S) return set_error("null server"), CMCG_EINVAL;
  int a = 0, q = 0;
  cmcg_status st = S->impl->step(&a, &q);
  if (active) *active = a;
  if (queued) *queued = q;
  return st;
}

cmcg_status cmcg_server_poll(cmcg_server *S, int64_t id, int32_t *state, double *u_re,
                             double *u_im, cmcg_report *rep) {
  if (!S || !state) return set_error("null argument"), CMCG_EINVAL;
  int st = 0;
  cmcg_status r = S->impl->poll(id, &st, u_re, u_im, rep);
  *state = st;
  return r;
}

cmcg_status cmcg_server_stats(const cmcg_server *S, int64_t *used_bytes, int32_t *active,
                              int32_t *queued) {
  if (!S || !used_bytes || !active || !queued) return set_error("null argument"), CMCG_EINVAL;
  int a = 0, q = 0;
  S->impl->stats(used_bytes, &a, &q);
  *active = a;
  *queued = q;
  return CMCG_OK;
}

cmcg_status cmcg_server_launches(const cmcg_server *S, int64_t *ticks, int64_t *launches,
                                 int64_t *rounds) {
  if (!S || !ticks || !launches || !rounds) return set_error("null argument"), CMCG_EINVAL;
  S->impl->counters(ticks, launches, rounds);
  return CMCG_OK;
}

}  // extern "C"
