// Internal declarations shared by the HIP translation units of libcmcg.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/cmcg.h"

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

// One solve's share of a batched (multi-solve) launch.
template <typename T>
struct F1SlotLaunch {
  F1Geom g;
  F1Ptrs<T> p;
  F1Launch L;
  int band, nbx, block0, nblocks;
};

// Launch geometry of the streaming kernel for an nx x ny grid at K steps per launch.
void f1_launch_shape(int nx, int ny, int K, int *nbx, int *nby, int *band);
// Fast-variant set of a launch's kernel instance: 0 the launches between a period's first and
// last (forward and backward alike: a backward middle launch is a forward homogeneous launch in
// the backward period's variables), 1 those two, 3 every launch of a forced (forward) period.
int f1_fast_set(const F1Launch &L, bool has_sub, bool adjoint);
template <typename T>
hipError_t f1_multi_launch(int K, bool adjoint, int set, const F1SlotLaunch<T> *slots, int nslots,
                           int blocks, hipStream_t s);

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

// Generic flat-array helpers.
template <typename TD, typename TS>
hipError_t convert(TD *dst, const TS *src, size_t n, hipStream_t s);
template <typename T>
hipError_t direction_update(T *d, const double *r, const double *scalars, size_t n, hipStream_t s);

// Pack / unpack between the packed user vector (FP64) and the device layout (T).
template <typename T>
hipError_t f1_unpack(const F1Geom &g, const double *packed, T *dev, size_t fs, hipStream_t s);
template <typename T>
hipError_t f1_pack(const F1Geom &g, const T *dev, double *packed, size_t fs, hipStream_t s);

}  // namespace cmcg
