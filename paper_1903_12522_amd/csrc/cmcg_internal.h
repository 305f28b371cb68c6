// Internal declarations shared by the HIP translation units of libcmcg.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/cmcg.h"
#include "serve_plan.h"

namespace cmcg {

void set_error(const std::string &msg);

#define CMCG_HIP(...)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (__VA_ARGS__);                                                          \
    if (e_ != hipSuccess) {                                                                 \
      ::cmcg::set_error(std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_));         \
      return e_ == hipErrorOutOfMemory ? CMCG_ENOMEM : CMCG_EDEVICE;                        \
    }                                                                                       \
  } while (0)

#define CMCG_TRY(...)                   \
  do {                                  \
    cmcg_status s_ = (__VA_ARGS__);     \
    if (s_ < 0) return s_;              \
  } while (0)

// ---------------------------------------------------------------------------------------
// Reductions: every CG scalar is a fixed-order FP64 sum: each block writes one partial,
// then one block sums the partials in index order.  Same grid -> same bits.
// ---------------------------------------------------------------------------------------
constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

// Device scalar slots (FP64) used by the CG driver.
enum Scalar : int {
  kDelta = 0,     // current <rhat, r>
  kDelta0 = 1,    // initial <rhat, r>
  kQd = 2,        // <qhat, d>
  kAlpha = 3,
  kBeta = 4,
  kRel = 5,       // sqrt(delta / delta0)
  kBreak = 6,     // 1 if breakdown
  kTmp = 7,
  kRz = 8,        // Riesz PCG scalars from here on
  kMisfit = 20,   // 2 J(z) of cmcg_misfit
  kNumScalars = 24
};

// Finalize modes of the one-block reduction.
enum FinalMode : int {
  kFinStart = 0,   // delta0 = delta = sum; rel = 1
  kFinAlpha = 1,   // qd = sum; alpha = delta / qd; breakdown if qd <= 0 or non-finite
  kFinBeta = 2,    // beta = sum / delta; delta = sum; rel = sqrt(sum / delta0)
  kFinStore = 3,   // scalars[slot] = sum
  kFinRefresh = 4  // true residual replaced the recursive one: beta = sum / delta_before, delta = sum
};

// Clears `bytes` of device memory with a fill kernel on stream s.
hipError_t zero_device(void *p, size_t bytes, hipStream_t s);

// Launches a one-block kernel that sums `n` partials in order and applies `mode`.
hipError_t finalize(const double *partials, int n, double *scalars, int mode, int slot,
                    hipStream_t s);

// ---------------------------------------------------------------------------------------
// First-order (staggered, 2D) device layout: three fields Px, Py, v, each ny rows of `pitch`
// values (x fastest).  Px[j][i] is the face between cells i and i+1 (valid for i <= nx-2),
// Py[j][i] the face between rows j and j+1 (valid for j <= ny-2); the invalid entries and
// the padding columns i >= nx hold 0 in every vector.
// ---------------------------------------------------------------------------------------
struct F1Geom {
  int nx, ny, pitch;
  double h, dt;
  int abs_face[4];     // 1 if the -x, +x, -y, +y face is absorbing
  // Dirichlet (sound-soft) cells, 1 per masked cell in the device layout, or null; the box of
  // the masked cells: columns mlo[0]..mhi[0], rows mlo[1]..mhi[1]
  const uint8_t *mask;
  int mlo[2], mhi[2];
};

constexpr int kMaxBlockSteps = 8;

struct F1Launch {
  int nsteps;          // leapfrog steps in this launch (<= template KMAX)
  int first;           // opening half-step of the period before the first step
  int last;            // the last step of the period ends with a half-step
  int forced;          // add the source term
  int accumulate;      // filter: add v^n (fc, fs) to (Ure, Uim) before stepping (KMAX = 1)
  int general;         // run every tile through the general body (a bitwise check of the fast one)
  double cs[kMaxBlockSteps], sn[kMaxBlockSteps];   // cos/sin(omega t) at each step's source time
  double fcos, fsin;   // filter weights cos/sin(omega t_n)
  // Dirichlet cells of a forced period: v = dre dc[k] + dim ds[k] at the launch's input time
  // (k = 0) and at the output time of level k (k >= 1)
  double dc[kMaxBlockSteps + 1], ds[kMaxBlockSteps + 1];
};

template <typename T>
struct F1Ptrs {
  const T *in;         // input state (3 fields, field stride fs)
  T *out;              // output state
  const T *sub;        // epilogue: out = result - sub (nullptr: out = result)
  const T *cc;         // c^2 per cell
  const T *fre, *fim;  // forcing amplitude per cell (fim may be nullptr)
  double *ure, *uim;   // filter accumulators (cell field, FP64)
  size_t fs;           // field stride in elements (ny * pitch)
  const double *dre, *dim;   // Dirichlet data of v on the masked cells (dim may be null)
};

// Launch geometry of the streaming kernel for an nx x ny grid at K steps per launch.
void f1_launch_shape(int nx, int ny, int K, int *nbx, int *nby, int *band);
template <typename T>
hipError_t f1_forward_launch(const F1Geom &g, const F1Ptrs<T> &p, const F1Launch &L, int kmax,
                             hipStream_t s);
template <typename T>
hipError_t f1_adjoint_launch(const F1Geom &g, const F1Ptrs<T> &p, const F1Launch &L, int kmax,
                             hipStream_t s);

// CG vector kernels over the F1 layout (3 fields; v weighted by 1 / c^2).
template <typename TA, typename TB>
hipError_t f1_dot(const F1Geom &g, const TA *a, const TB *b, const void *cc, int cc_is_double,
                  size_t fs, double *partials, hipStream_t s);
template <typename T>
hipError_t f1_cg_update(const F1Geom &g, double *z, double *r, const T *d, const T *q,
                        const void *cc, size_t fs, const double *scalars, double *partials,
                        hipStream_t s);

// ---------------------------------------------------------------------------------------
// Persistent serving kernel (continuous batching of first-order solves): one launch per
// server tick runs rounds of every resident solve's CG operations (serve_plan.h), a grid
// barrier between rounds; decisions are taken on the device.
// ---------------------------------------------------------------------------------------
constexpr int kServeMaxSlots = 64;

// One resident solve: geometry, constants and buffers (written by the host at admission).
// lo: the CG periods' precision (FP32 in FP32-mixed mode); hi: FP64.  In FP64 mode they are
// the same buffers.
struct ServeSlot {
  F1Geom g;
  size_t fs, vecN;
  int band;            // rows per band of the streaming tiles
  int N, K_lo, K_hi, mixed, max_iter;
  double tol, refresh;
  double out_scale;    // 2 / (N omega)
  void *lo_S0, *lo_S1, *lo_W, *lo_Q, *lo_cc, *lo_Fre, *lo_Fim;
  double *hi_S0, *hi_S1, *hi_W, *hi_Q, *hi_cc, *hi_Fre, *hi_Fim;
  void *D;
  double *Z, *R, *Ure, *Uim, *partials, *scalars;
  const double *tab;   // per step n < N: cos and sin of omega t_{n+1/2}, then of omega t_n
};

// Device control block of the serving kernel.
struct ServeControl {
  unsigned count;        // grid barrier: arrivals of the current round ...
  unsigned pad0[31];
  unsigned gen;          // ... and its generation, polled on a cache line of its own
  unsigned pad1[31];
  int failed;            // a barrier wait gave up (spin limit or the host's abort flag)
  int rounds;            // rounds the last launch ran
  double work;           // grid-point updates the last launch did
};

// Generic flat-array helpers.
template <typename TD, typename TS>
hipError_t convert(TD *dst, const TS *src, size_t n, hipStream_t s);
template <typename T>
hipError_t direction_update(T *d, const double *r, const double *scalars, size_t n, hipStream_t s);

// The serving kernel: its co-resident grid on the current device, and one tick.
hipError_t f1_serve_grid(int *blocks);
hipError_t f1_serve_launch(const ServeSlot *slots, serve::State *states, int nslots,
                           ServeControl *ctl, const int *abort_flag, int max_rounds,
                           double work_budget, unsigned long long spin_limit, int blocks,
                           hipStream_t s);

// Pack / unpack between the packed user vector (FP64) and the device layout (T).
template <typename T>
hipError_t f1_unpack(const F1Geom &g, const double *packed, T *dev, size_t fs, hipStream_t s);
template <typename T>
hipError_t f1_pack(const F1Geom &g, const T *dev, double *packed, size_t fs, hipStream_t s);

}  // namespace cmcg
