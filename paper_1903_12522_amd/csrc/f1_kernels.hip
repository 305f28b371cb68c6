// First-order (velocity / flux) staggered leapfrog on gfx950: the forward period map, its exact
// transpose in the energy inner product (the backward / adjoint period), and the CG vector
// kernels over the staggered layout.
//
// Scheme (Sec. 3.1, eq. mixWE, on a structured grid; leapfrog with an integer number of steps
// per period): v at cell centres, flux p on interior faces, G = face difference / h,
// D = -G^T, gamma = dt c m / (2h) with m the number of absorbing faces of the cell.
//   forward step:  p+ = p + dt/2 G v;  (1+gamma) v' = (1-gamma) v + dt c^2 (D p+ + F);
//                  p' = p+ + dt/2 G v'
// Consecutive half kicks of p merge, so one period is: an opening half kick of p, then N
// fused [velocity update, p kick] steps, the last kick being a half kick.
// The backward period applies E* = M_E^{-1} E^T M_E (M_E = diag(h^2 on faces, h^2/c^2 on cells),
// eq. mix_cost_functional_J): per step the transposes of the three sub-maps in reverse order,
//   v <- v - dt/2 c^2 D p;   p <- p - dt G (v / (1+gamma)),  v <- a v;   v <- v - dt/2 c^2 D p
// with a = (1-gamma)/(1+gamma); its half kicks of v merge the same way.  In the variables
// Q = -p, u = v / (1+gamma) a merged backward step reads
//   Q <- Q + dt G u;   (1+gamma) u' = (1-gamma) u + dt c^2 D Q,
// the forward's [velocity update, kick] pair shifted by half a step.  So a backward period is a
// prologue (the opening half kick of v, the change of variables and the first Q kick), N - 1
// forward homogeneous steps on (Q, u), and an epilogue (the closing half update straight back to
// v = (1-gamma) u + dt/2 c^2 D Q, p = -Q).  Only the first and last launches of a backward period
// differ from forward launches; the ones between run the forward kernel instance itself.
//
// Kernel design (register streaming with temporal blocking).  Each 64-lane wavefront owns a
// strip of 64 consecutive columns (one column per lane, so every row access is one coalesced
// 256/512-byte segment) and marches upward through a band of rows.  The K leapfrog steps of a
// launch are K pipeline levels held in registers: at row iteration j, level k advances row
// j - k from level k-1, so one HBM read and one HBM write of the state serve K steps.  Left and
// right neighbours come from the adjacent lanes (cross-lane shuffles), the row below from the
// previous iteration's registers; each level narrows the valid lanes by one on each side, so a
// wave writes 64 - 2(K+1) columns, and each band starts K+2 rows early to fill the pipeline.
// There is no LDS and no barrier.  The period's opening half kick is folded into level 0.
#include <cstdlib>

#include "f1_device.h"

// The file is compiled twice so that the two precisions' stream-kernel instances build in
// parallel: CMCG_F1_PART 1 holds the FP32 instances and everything else, 2 the FP64 instances.
#ifndef CMCG_F1_PART
#define CMCG_F1_PART 0
#endif
#define CMCG_F1_FP32 (CMCG_F1_PART != 2)
#define CMCG_F1_FP64 (CMCG_F1_PART != 1)

namespace cmcg {
namespace {

template <typename T, int K, bool ADJ, bool MASK, int SET>
__global__ __launch_bounds__(kThreads) void f1_stream_kernel(F1Geom g, F1Ptrs<T> p, F1Launch L,
                                                             int band) {
  int bx, by;
  tile_of_block(bx, by);
  f1_stream_tile<T, K, ADJ, MASK, SET>(g, p, L, band, bx, by);
}

// Rows per band.  Besides its band, each wavefront loads 2K + 3 rows to fill its pipeline, so
// taller bands waste fewer loads and shorter ones give more wavefronts to hide latency with.  On
// n x n grids from 128^2 to 4096^2 (FP32 with K = 7, FP64 with K = 8) the fastest height was
// ny / 128 rounded down to a power of two: one row at 128^2, 32 rows at 4096^2.
// CMCG_F1_BAND (environment, read once) overrides the band height for launch-shape sweeps.
inline int band_rows(int nx, int ny, int K) {
  (void)nx;
  (void)K;
  static const int forced = [] {
    const char *e = std::getenv("CMCG_F1_BAND");
    return e ? std::atoi(e) : 0;
  }();
  if (forced > 0) return forced;
  int band = 1;
  while (band < 256 && ny / (2 * band) >= 128) band *= 2;
  return band;
}

template <typename T, int K, bool ADJ>
hipError_t launch_one(const F1Geom &g, const F1Ptrs<T> &p, const F1Launch &L, hipStream_t s) {
  constexpr int OW = 64 - 2 * (K + 1);
  const int strips = (g.nx + OW - 1) / OW;
  const int band = band_rows(g.nx, g.ny, K);
  dim3 grid((strips + 3) / 4, (g.ny + band - 1) / band);
  // CMCG_F1_GENERAL=1 (environment) runs every tile through the general body, so that tests can
  // compare the fast variants with it bit for bit
  const char *gen = std::getenv("CMCG_F1_GENERAL");
  F1Launch Lx = L;
  Lx.general = (gen && gen[0] == '1') ? 1 : 0;
  // A backward launch between its period's first and last is a forward homogeneous launch in
  // the variables (Q, u) = (-p, v / (1 + gamma)), so it runs the forward middle instance.
  const bool ends = ADJ ? (L.first || L.last) : (L.first || p.sub);
#define CMCG_F1_LAUNCH(DIR, MASK, SET)                                                         \
  hipLaunchKernelGGL((f1_stream_kernel<T, K, DIR, MASK, SET>), grid, dim3(kThreads), 0, s, g, p, \
                     Lx, band)
  if (!ADJ && (L.forced || L.accumulate)) {
    // forced (forward) periods: every launch of the period runs the instance with the source
    // (and the filter sums, which only forced periods take)
    if (g.mask) CMCG_F1_LAUNCH(false, true, kFastForced);
    else CMCG_F1_LAUNCH(false, false, kFastForced);
  } else if (ends) {
    if (g.mask) CMCG_F1_LAUNCH(ADJ, true, kFastEnds);
    else CMCG_F1_LAUNCH(ADJ, false, kFastEnds);
  } else {
    if (g.mask) CMCG_F1_LAUNCH(false, true, kFastMiddle);
    else CMCG_F1_LAUNCH(false, false, kFastMiddle);
  }
#undef CMCG_F1_LAUNCH
  return hipGetLastError();
}

template <typename T, bool ADJ>
hipError_t launch_dispatch(const F1Geom &g, const F1Ptrs<T> &p, const F1Launch &L, int kmax,
                           hipStream_t s) {
  (void)kmax;
  switch (L.nsteps) {
    case 1: return launch_one<T, 1, ADJ>(g, p, L, s);
    case 2: return launch_one<T, 2, ADJ>(g, p, L, s);
    case 3: return launch_one<T, 3, ADJ>(g, p, L, s);
    case 4: return launch_one<T, 4, ADJ>(g, p, L, s);
    case 5: return launch_one<T, 5, ADJ>(g, p, L, s);
    case 6: return launch_one<T, 6, ADJ>(g, p, L, s);
    case 7: return launch_one<T, 7, ADJ>(g, p, L, s);
    case 8: return launch_one<T, 8, ADJ>(g, p, L, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------------------
// ---------------------------------------------------------------------------------------
// CG vector kernels
// ---------------------------------------------------------------------------------------
template <typename TA, typename TB, typename TC>
__global__ __launch_bounds__(kRedThreads) void f1_dot_kernel(F1Geom g, const TA *a, const TB *b,
                                                             const TC *cc, size_t fs,
                                                             double *partials) {
  f1_dot_block<TA, TB, TC>(g, a, b, cc, fs, partials, blockIdx.x, gridDim.x);
}

template <typename T, typename TC>
__global__ __launch_bounds__(kRedThreads) void f1_cg_update_kernel(F1Geom g, double *z, double *r,
                                                                   const T *d, const T *q,
                                                                   const TC *cc, size_t fs,
                                                                   const double *scalars,
                                                                   double *partials) {
  f1_cg_update_block<T, TC>(g, z, r, d, q, cc, fs, scalars, partials, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kRedThreads) void finalize_kernel(const double *partials, int n,
                                                               double *sc, int mode, int slot) {
  finalize_block(partials, n, sc, mode, slot);
}

template <typename TD, typename TS>
__global__ void convert_kernel(TD *dst, const TS *src, size_t n) {
  convert_block<TD, TS>(dst, src, n, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void direction_kernel(T *d, const double *r, const double *sc, size_t n) {
  direction_block<T>(d, r, sc, n, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void f1_unpack_kernel(F1Geom g, const double *packed, T *dev, size_t fs) {
  const int nx = g.nx, ny = g.ny;
  const size_t offPy = (size_t)ny * (nx - 1), offV = offPy + (size_t)(ny - 1) * nx;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < fs; o += stride) {
    const int j = (int)(o / g.pitch), i = (int)(o % g.pitch);
    T px = 0, py = 0, v = 0;
    if (i < nx) {
      if (i < nx - 1) px = (T)packed[(size_t)j * (nx - 1) + i];
      if (j < ny - 1) py = (T)packed[offPy + (size_t)j * nx + i];
      v = (T)packed[offV + (size_t)j * nx + i];
    }
    dev[o] = px;
    dev[o + fs] = py;
    dev[o + 2 * fs] = v;
  }
}

template <typename T>
__global__ void f1_pack_kernel(F1Geom g, const T *dev, double *packed, size_t fs) {
  const int nx = g.nx, ny = g.ny;
  const size_t offPy = (size_t)ny * (nx - 1), offV = offPy + (size_t)(ny - 1) * nx;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < fs; o += stride) {
    const int j = (int)(o / g.pitch), i = (int)(o % g.pitch);
    if (i >= nx) continue;
    if (i < nx - 1) packed[(size_t)j * (nx - 1) + i] = (double)dev[o];
    if (j < ny - 1) packed[offPy + (size_t)j * nx + i] = (double)dev[o + fs];
    packed[offV + (size_t)j * nx + i] = (double)dev[o + 2 * fs];
  }
}

inline int grid_for(size_t n, int threads = 256) {
  size_t b = (n + threads - 1) / threads;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

#if CMCG_F1_FP32
hipError_t finalize(const double *partials, int n, double *scalars, int mode, int slot,
                    hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, n, scalars,
                     mode, slot);
  return hipGetLastError();
}

#endif

template <typename T>
hipError_t f1_forward_launch(const F1Geom &g, const F1Ptrs<T> &p, const F1Launch &L, int kmax,
                             hipStream_t s) {
  return launch_dispatch<T, false>(g, p, L, kmax, s);
}
template <typename T>
hipError_t f1_adjoint_launch(const F1Geom &g, const F1Ptrs<T> &p, const F1Launch &L, int kmax,
                             hipStream_t s) {
  return launch_dispatch<T, true>(g, p, L, kmax, s);
}

#if CMCG_F1_FP32
void f1_launch_shape(int nx, int ny, int K, int *nbx, int *nby, int *band) {
  const int ow = 64 - 2 * (K + 1);
  const int strips = (nx + ow - 1) / ow;
  *band = band_rows(nx, ny, K);
  *nbx = (strips + 3) / 4;
  *nby = (ny + *band - 1) / *band;
}

#endif

template <typename TA, typename TB>
hipError_t f1_dot(const F1Geom &g, const TA *a, const TB *b, const void *cc, int cc_is_double,
                  size_t fs, double *partials, hipStream_t s) {
  if (cc_is_double)
    hipLaunchKernelGGL((f1_dot_kernel<TA, TB, double>), dim3(kRedBlocks), dim3(kRedThreads), 0, s,
                       g, a, b, static_cast<const double *>(cc), fs, partials);
  else
    hipLaunchKernelGGL((f1_dot_kernel<TA, TB, float>), dim3(kRedBlocks), dim3(kRedThreads), 0, s,
                       g, a, b, static_cast<const float *>(cc), fs, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t f1_cg_update(const F1Geom &g, double *z, double *r, const T *d, const T *q,
                        const void *cc, size_t fs, const double *scalars, double *partials,
                        hipStream_t s) {
  hipLaunchKernelGGL((f1_cg_update_kernel<T, T>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, g, z,
                     r, d, q, static_cast<const T *>(cc), fs, scalars, partials);
  return hipGetLastError();
}

template <typename TD, typename TS>
hipError_t convert(TD *dst, const TS *src, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((convert_kernel<TD, TS>), dim3(grid_for(n)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

template <typename T>
hipError_t direction_update(T *d, const double *r, const double *scalars, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((direction_kernel<T>), dim3(grid_for(n)), dim3(256), 0, s, d, r, scalars, n);
  return hipGetLastError();
}

template <typename T>
hipError_t f1_unpack(const F1Geom &g, const double *packed, T *dev, size_t fs, hipStream_t s) {
  hipLaunchKernelGGL((f1_unpack_kernel<T>), dim3(grid_for(fs)), dim3(256), 0, s, g, packed, dev, fs);
  return hipGetLastError();
}
template <typename T>
hipError_t f1_pack(const F1Geom &g, const T *dev, double *packed, size_t fs, hipStream_t s) {
  hipLaunchKernelGGL((f1_pack_kernel<T>), dim3(grid_for(fs)), dim3(256), 0, s, g, dev, packed, fs);
  return hipGetLastError();
}

// explicit instantiations
#if CMCG_F1_FP32
template hipError_t f1_forward_launch<float>(const F1Geom &, const F1Ptrs<float> &, const F1Launch &, int, hipStream_t);
template hipError_t f1_adjoint_launch<float>(const F1Geom &, const F1Ptrs<float> &, const F1Launch &, int, hipStream_t);
template hipError_t f1_dot<float, float>(const F1Geom &, const float *, const float *, const void *, int, size_t, double *, hipStream_t);
template hipError_t f1_dot<double, double>(const F1Geom &, const double *, const double *, const void *, int, size_t, double *, hipStream_t);
template hipError_t f1_dot<double, float>(const F1Geom &, const double *, const float *, const void *, int, size_t, double *, hipStream_t);
template hipError_t f1_cg_update<float>(const F1Geom &, double *, double *, const float *, const float *, const void *, size_t, const double *, double *, hipStream_t);
template hipError_t f1_cg_update<double>(const F1Geom &, double *, double *, const double *, const double *, const void *, size_t, const double *, double *, hipStream_t);
template hipError_t convert<float, double>(float *, const double *, size_t, hipStream_t);
template hipError_t convert<double, float>(double *, const float *, size_t, hipStream_t);
template hipError_t convert<double, double>(double *, const double *, size_t, hipStream_t);
template hipError_t convert<float, float>(float *, const float *, size_t, hipStream_t);
template hipError_t direction_update<float>(float *, const double *, const double *, size_t, hipStream_t);
template hipError_t direction_update<double>(double *, const double *, const double *, size_t, hipStream_t);
template hipError_t f1_unpack<float>(const F1Geom &, const double *, float *, size_t, hipStream_t);
template hipError_t f1_unpack<double>(const F1Geom &, const double *, double *, size_t, hipStream_t);
template hipError_t f1_pack<float>(const F1Geom &, const float *, double *, size_t, hipStream_t);
template hipError_t f1_pack<double>(const F1Geom &, const double *, double *, size_t, hipStream_t);
#endif
#if CMCG_F1_FP64
template hipError_t f1_forward_launch<double>(const F1Geom &, const F1Ptrs<double> &, const F1Launch &, int, hipStream_t);
template hipError_t f1_adjoint_launch<double>(const F1Geom &, const F1Ptrs<double> &, const F1Launch &, int, hipStream_t);
#endif

}  // namespace cmcg
