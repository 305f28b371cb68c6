// Formulation-independent solver interface behind the C ABI, and small runtime utilities.
#pragma once

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "cmcg_internal.h"

namespace cmcg {

// Options resolved from cmcg_options / cmcg_problem at create time.
struct SolverConfig {
  int prec = CMCG_FP64;
  double tol = 1e-6;
  int max_iter = 1000;
  int kblock = 4;          // leapfrog steps per launch
  int steps_request = 0;   // cmcg_options.steps_per_launch as given (0: library default)
  double refresh = 0.1;    // FP32-mixed: FP64 residual refresh factor (<= 0: never)
  double riesz_tol = 0.0;
  int riesz_max_iter = 0;
  int riesz_mode = CMCG_RIESZ_SOLVE;   // resolved: CMCG_RIESZ_SOLVE or CMCG_RIESZ_VCYCLE
  int runup = 0;           // initial run-up periods before the CG iteration
  int output = CMCG_OUTPUT_FILTER;   // how the minimiser becomes u
  hipStream_t stream = nullptr;
  double h = 0, omega = 0, T = 0, dt = 0;
  int N = 0;
  // time-harmonic components of the source: harmonic[j] * omega is component j's frequency
  int nshots = 1;
  int harmonic[CMCG_MAX_SHOTS] = {1};
  double omega_of(int j) const { return harmonic[j] * omega; }
};

// The components of a problem's source: its shots, or its own data as the single component at
// the base frequency.
inline std::vector<cmcg_shot> shots_of(const cmcg_problem *P) {
  if (P->n_shots > 0) return std::vector<cmcg_shot>(P->shots, P->shots + P->n_shots);
  cmcg_shot s{1, P->f_re, P->f_im, P->gS_re, P->gS_im, P->gD_re, P->gD_im};
  return {s};
}

// Device allocations owned by one solver (freed in the destructor).  In fixed-buffer mode
// (use_buffer) the allocations are carved from a device buffer the caller owns: nothing is
// allocated or freed, a request beyond the buffer fails with CMCG_ENOMEM, and every piece is
// cleared by a fill kernel rather than a memset.
class DeviceArena {
 public:
  ~DeviceArena() { release(); }
  void use_buffer(void *base, size_t cap) {
    base_ = static_cast<char *>(base);
    cap_ = cap;
    off_ = 0;
  }
  cmcg_status alloc(size_t bytes, void **p, hipStream_t s) {
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    if (base_) {
      const size_t off = (off_ + 255) / 256 * 256;
      if (off > cap_ || bytes > cap_ - off) {
        set_error("the problem needs more device memory than the fixed " +
                  std::to_string(cap_ >> 20) + " MiB buffer holds (a further " +
                  std::to_string(bytes) + " B at offset " + std::to_string(off) + ")");
        return CMCG_ENOMEM;
      }
      *p = base_ + off;
      off_ = off + bytes;
      bytes_ += bytes;
      CMCG_HIP(zero_device(*p, bytes, s));
      return CMCG_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error("hipMalloc(" + std::to_string(bytes) + " B): " + hipGetErrorString(e));
      return CMCG_ENOMEM;
    }
    ptrs_.push_back(*p);
    bytes_ += bytes;
    CMCG_HIP(hipMemsetAsync(*p, 0, bytes, s));
    return CMCG_OK;
  }
  template <typename T>
  cmcg_status alloc_n(size_t n, T **p, hipStream_t s) {
    return alloc(n * sizeof(T), reinterpret_cast<void **>(p), s);
  }
  void release() {
    for (void *p : ptrs_) (void)hipFree(p);
    ptrs_.clear();
    bytes_ = 0;
    off_ = 0;
  }
  size_t bytes() const { return bytes_; }
  bool fixed() const { return base_ != nullptr; }

 private:
  std::vector<void *> ptrs_;
  size_t bytes_ = 0;
  char *base_ = nullptr;   // fixed-buffer mode
  size_t cap_ = 0, off_ = 0;
};

// Phase timer: pairs of HIP events recorded on the solver's stream.
class PhaseEvents {
 public:
  ~PhaseEvents() {
    for (auto e : ev_)
      if (e) (void)hipEventDestroy(e);
  }
  cmcg_status init(int n) {
    ev_.assign(n, nullptr);
    for (auto &e : ev_) CMCG_HIP(hipEventCreate(&e));
    return CMCG_OK;
  }
  hipEvent_t operator[](int k) const { return ev_[k]; }
  static double seconds(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
      (void)hipGetLastError();
      return 0.0;
    }
    return 1e-3 * ms;
  }

 private:
  std::vector<hipEvent_t> ev_;
};

// Device time of the bulk launches of the CG iterations' periods, per direction (0 forward,
// 1 backward): one event before the first and one after the last of a period's consecutive run
// of them, read once the stream has synchronised.  The bulk launches run one kernel instance
// (first order: the launches between a period's first and last; second order: the blocked
// launches of full depth), so their mean is that instance's own launch time.
class BulkTimer {
 public:
  ~BulkTimer() {
    for (auto &d : ev_)
      for (auto &e : d)
        if (e) (void)hipEventDestroy(e);
  }
  cmcg_status init() {
    for (auto &d : ev_)
      for (auto &e : d) CMCG_HIP(hipEventCreate(&e));
    return CMCG_OK;
  }
  void reset() {
    for (int d = 0; d < 2; ++d) {
      seconds[d] = 0.0;
      launches[d] = 0;
      pending_[d] = 0;
    }
  }
  cmcg_status begin(int dir, hipStream_t s) {
    CMCG_HIP(hipEventRecord(ev_[dir][0], s));
    return CMCG_OK;
  }
  cmcg_status end(int dir, long long n, hipStream_t s) {
    CMCG_HIP(hipEventRecord(ev_[dir][1], s));
    pending_[dir] = n;
    return CMCG_OK;
  }
  // after the stream has synchronised
  void collect() {
    for (int d = 0; d < 2; ++d) {
      if (!pending_[d]) continue;
      seconds[d] += PhaseEvents::seconds(ev_[d][0], ev_[d][1]);
      launches[d] += pending_[d];
      pending_[d] = 0;
    }
  }
  double seconds[2] = {0.0, 0.0};
  long long launches[2] = {0, 0};

 private:
  hipEvent_t ev_[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  long long pending_[2] = {0, 0};
};

class Solver {
 public:
  virtual ~Solver() {}
  virtual cmcg_status begin() = 0;
  virtual cmcg_status iterate(int iters, int *converged) = 0;
  virtual cmcg_status finish(double *u_re, double *u_im) = 0;
  // begin + iterate(max_iter) + finish, timed end to end on the device
  virtual cmcg_status solve(double *u_re, double *u_im) = 0;
  virtual cmcg_status apply(int op, int steps, const double *in, double *out) = 0;
  virtual cmcg_status filter(const double *z, double *u_re, double *u_im) = 0;
  // the solution read off a packed state without time stepping (Step 6, time-discrete)
  virtual cmcg_status step6(const double *z, double *u_re, double *u_im) = 0;
  virtual cmcg_status get_state(int which, double *out) = 0;
  virtual cmcg_status runup(int periods, int ramp, double *z_out) = 0;
  virtual cmcg_status misfit(const double *z, double *J) = 0;
  virtual void report(cmcg_report *r) const = 0;
  virtual void info(cmcg_info *i) const = 0;
  virtual size_t device_bytes() const = 0;
};

// Validates a problem and its options (host-side checks only) and resolves the solver
// configuration: T = 2 pi / omega, N = ceil(T c_max / (courant h)) (>= 3), dt = T / N.
cmcg_status validate_problem(const cmcg_problem *P, const cmcg_options *O);
cmcg_status make_config(const cmcg_problem *P, const cmcg_options *O, hipStream_t stream,
                        SolverConfig *cfg);

cmcg_status make_f1_solver(const cmcg_problem *P, const SolverConfig &cfg, Solver **out);
// A first-order solver whose device memory is carved from [base, base + cap) (allocates
// nothing: no device, pinned-host or event allocation; see DeviceArena::use_buffer).  Its
// stage calls work as the ordinary solver's; the phase timers are not kept.
cmcg_status make_f1_solver_in(const cmcg_problem *P, const SolverConfig &cfg, void *base,
                              size_t cap, Solver **out);
cmcg_status make_f2_solver(const cmcg_problem *P, const SolverConfig &cfg, Solver **out);

// Continuous-batching request server (first-order solves).
class Server {
 public:
  virtual ~Server() {}
  virtual cmcg_status submit(const cmcg_problem *P, const cmcg_options *O, int64_t *id) = 0;
  virtual cmcg_status step(int *n_active, int *n_queued) = 0;
  virtual cmcg_status poll(int64_t id, int *state, double *u_re, double *u_im,
                           cmcg_report *rep) = 0;
  virtual void stats(int64_t *used_bytes, int *n_active, int *n_queued) const = 0;
  virtual void counters(int64_t *n_ticks, int64_t *n_launches, int64_t *n_rounds) const = 0;
};
cmcg_status make_f1_server(const cmcg_server_options *o, hipStream_t s, Server **out);

// Mur's switch-on of the time-harmonic source (Sec. 4.2.3, eq. transientfunction):
// (2 - sin s) sin s with s = (t / t_tr) pi / 2 for t < t_tr, 1 afterwards.
inline double transient(double t, double t_tr) {
  if (!(t_tr > 0.0) || t >= t_tr) return 1.0;
  const double s = 0.5 * 3.14159265358979323846 * t / t_tr;
  return (2.0 - std::sin(s)) * std::sin(s);
}

inline int grid_for(size_t n, int threads = 256) {
  size_t b = (n + threads - 1) / threads;
  return (int)std::max<size_t>(1, std::min<size_t>(b, 8192));
}

}  // namespace cmcg
