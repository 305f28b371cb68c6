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
// with a = (1-gamma)/(1+gamma); its half kicks of v merge the same way.
//
// Kernel design: a block owns a 64 x TY output tile and stages the tile plus a halo of
// KMAX+1 cells of every field in LDS; it runs up to KMAX leapfrog steps there (temporal
// blocking: one HBM read and one write of the state per KMAX steps) and writes back only the
// tile, whose values are exact because each step widens the dependency cone by one cell.
// Rows are read and written with 64 consecutive lanes on consecutive x (coalesced).
#include "cmcg_internal.h"

namespace cmcg {
namespace {

constexpr int kTX = 64;
constexpr int kThreads = 256;

__device__ __forceinline__ int absorbing_faces(const F1Geom &g, int i, int j) {
  return (i == 0 ? g.abs_face[0] : 0) + (i == g.nx - 1 ? g.abs_face[1] : 0) +
         (j == 0 ? g.abs_face[2] : 0) + (j == g.ny - 1 ? g.abs_face[3] : 0);
}

// XCD-aware tile order: hardware dispatches consecutive workgroups round-robin over the 8
// XCDs; remap so that each XCD walks a contiguous band of tiles (neighbouring tiles share halo
// rows in that XCD's L2).
__device__ __forceinline__ void tile_of_block(int &bx, int &by) {
  const int nbx = gridDim.x, nby = gridDim.y;
  const int nb = nbx * nby;
  const int b = blockIdx.y * nbx + blockIdx.x;
  int t = b;
  if (nb % 8 == 0) t = (b % 8) * (nb / 8) + b / 8;
  bx = t % nbx;
  by = t / nbx;
}

template <typename T, int KMAX, int TY>
__global__ __launch_bounds__(kThreads) void f1_forward_kernel(F1Geom g, F1Ptrs<T> p, F1Launch L) {
  constexpr int H = KMAX + 1;
  constexpr int LX = kTX + 2 * H;
  constexpr int LY = TY + 2 * H;
  __shared__ T sPx[LY][LX];
  __shared__ T sPy[LY][LX];
  __shared__ T sv[LY][LX];
  __shared__ T scc[LY][LX];
  int bx, by;
  tile_of_block(bx, by);
  const int i0 = bx * kTX - H;
  const int j0 = by * TY - H;
  const int tid = threadIdx.x;
  const T dt = (T)g.dt;
  const T inv_h = (T)(1.0 / g.h);
  const T half_inv_h = (T)(0.5 / g.h);
  const size_t fs = p.fs;

  for (int idx = tid; idx < LX * LY; idx += kThreads) {
    const int ly = idx / LX, lx = idx - (idx / LX) * LX;
    const int i = i0 + lx, j = j0 + ly;
    const bool in = (i >= 0) && (i < g.nx) && (j >= 0) && (j < g.ny);
    const size_t o = (size_t)j * g.pitch + i;
    sPx[ly][lx] = in ? p.in[o] : T(0);
    sPy[ly][lx] = in ? p.in[o + fs] : T(0);
    sv[ly][lx] = in ? p.in[o + 2 * fs] : T(0);
    scc[ly][lx] = in ? p.cc[o] : T(0);
  }
  __syncthreads();

  if (L.accumulate) {
    // filter sum: (Ure, Uim) += v^n (cos, sin)(omega t_n) on the tile
    for (int idx = tid; idx < kTX * TY; idx += kThreads) {
      const int ly = H + idx / kTX, lx = H + idx % kTX;
      const int i = i0 + lx, j = j0 + ly;
      if (i < g.nx && j < g.ny) {
        const size_t o = (size_t)j * g.pitch + i;
        const double v = (double)sv[ly][lx];
        p.ure[o] += v * L.fcos;
        p.uim[o] += v * L.fsin;
      }
    }
  }

  if (L.first) {
    // opening half kick  p <- p + dt/2 G v
    const T k = T(0.5) * dt;
    for (int idx = tid; idx < LX * LY; idx += kThreads) {
      const int ly = idx / LX, lx = idx - (idx / LX) * LX;
      const int i = i0 + lx, j = j0 + ly;
      if (i < 0 || j < 0 || j >= g.ny || i >= g.nx) continue;
      if (i <= g.nx - 2 && lx <= LX - 2) sPx[ly][lx] += k * ((sv[ly][lx + 1] - sv[ly][lx]) * inv_h);
      if (j <= g.ny - 2 && ly <= LY - 2) sPy[ly][lx] += k * ((sv[ly + 1][lx] - sv[ly][lx]) * inv_h);
    }
    __syncthreads();
  }

  for (int s = 0; s < L.nsteps; ++s) {
    const T cs = (T)L.cs[s], sn = (T)L.sn[s];
    // velocity update  (1+gamma) v' = (1-gamma) v + dt c^2 (D p + F)
    for (int idx = tid; idx < LX * LY; idx += kThreads) {
      const int ly = idx / LX, lx = idx - (idx / LX) * LX;
      const int i = i0 + lx, j = j0 + ly;
      if (lx < 1 || ly < 1 || i < 0 || j < 0 || i >= g.nx || j >= g.ny) continue;
      T div = (sPx[ly][lx] - sPx[ly][lx - 1] + sPy[ly][lx] - sPy[ly - 1][lx]) * inv_h;
      if (L.forced) {
        const size_t o = (size_t)j * g.pitch + i;
        div += p.fre[o] * cs;
        if (p.fim) div += p.fim[o] * sn;
      }
      const T c2 = scc[ly][lx];
      const int m = absorbing_faces(g, i, j);
      T v = sv[ly][lx];
      if (m == 0) {
        v = v + dt * c2 * div;
      } else {
        const T gam = dt * (T)m * sqrt(c2) * half_inv_h;
        v = ((T(1) - gam) * v + dt * c2 * div) / (T(1) + gam);
      }
      sv[ly][lx] = v;
    }
    __syncthreads();
    // flux kick  p <- p + kick G v'
    const T k = (L.last && s == L.nsteps - 1) ? T(0.5) * dt : dt;
    for (int idx = tid; idx < LX * LY; idx += kThreads) {
      const int ly = idx / LX, lx = idx - (idx / LX) * LX;
      const int i = i0 + lx, j = j0 + ly;
      if (i < 0 || j < 0 || j >= g.ny || i >= g.nx) continue;
      if (i <= g.nx - 2 && lx <= LX - 2) sPx[ly][lx] += k * ((sv[ly][lx + 1] - sv[ly][lx]) * inv_h);
      if (j <= g.ny - 2 && ly <= LY - 2) sPy[ly][lx] += k * ((sv[ly + 1][lx] - sv[ly][lx]) * inv_h);
    }
    __syncthreads();
  }

  for (int idx = tid; idx < kTX * TY; idx += kThreads) {
    const int ly = H + idx / kTX, lx = H + idx % kTX;
    const int i = i0 + lx, j = j0 + ly;
    if (i >= g.nx || j >= g.ny) continue;
    const size_t o = (size_t)j * g.pitch + i;
    T a = sPx[ly][lx], b = sPy[ly][lx], c = sv[ly][lx];
    if (p.sub) {
      a -= p.sub[o];
      b -= p.sub[o + fs];
      c -= p.sub[o + 2 * fs];
    }
    p.out[o] = a;
    p.out[o + fs] = b;
    p.out[o + 2 * fs] = c;
  }
}

template <typename T, int KMAX, int TY>
__global__ __launch_bounds__(kThreads) void f1_adjoint_kernel(F1Geom g, F1Ptrs<T> p, F1Launch L) {
  constexpr int H = KMAX + 1;
  constexpr int LX = kTX + 2 * H;
  constexpr int LY = TY + 2 * H;
  __shared__ T sPx[LY][LX];
  __shared__ T sPy[LY][LX];
  __shared__ T sv[LY][LX];
  __shared__ T scc[LY][LX];
  int bx, by;
  tile_of_block(bx, by);
  const int i0 = bx * kTX - H;
  const int j0 = by * TY - H;
  const int tid = threadIdx.x;
  const T dt = (T)g.dt;
  const T inv_h = (T)(1.0 / g.h);
  const T half_inv_h = (T)(0.5 / g.h);
  const size_t fs = p.fs;

  for (int idx = tid; idx < LX * LY; idx += kThreads) {
    const int ly = idx / LX, lx = idx - (idx / LX) * LX;
    const int i = i0 + lx, j = j0 + ly;
    const bool in = (i >= 0) && (i < g.nx) && (j >= 0) && (j < g.ny);
    const size_t o = (size_t)j * g.pitch + i;
    sPx[ly][lx] = in ? p.in[o] : T(0);
    sPy[ly][lx] = in ? p.in[o + fs] : T(0);
    sv[ly][lx] = in ? p.in[o + 2 * fs] : T(0);
    scc[ly][lx] = in ? p.cc[o] : T(0);
  }
  __syncthreads();

  if (L.first) {
    // opening half kick  v <- v - dt/2 c^2 D p
    const T k = T(0.5) * dt;
    for (int idx = tid; idx < LX * LY; idx += kThreads) {
      const int ly = idx / LX, lx = idx - (idx / LX) * LX;
      const int i = i0 + lx, j = j0 + ly;
      if (lx < 1 || ly < 1 || i < 0 || j < 0 || i >= g.nx || j >= g.ny) continue;
      const T div = (sPx[ly][lx] - sPx[ly][lx - 1] + sPy[ly][lx] - sPy[ly - 1][lx]) * inv_h;
      sv[ly][lx] -= k * scc[ly][lx] * div;
    }
    __syncthreads();
  }

  for (int s = 0; s < L.nsteps; ++s) {
    // flux update  p <- p - dt G (v / (1+gamma))
    for (int idx = tid; idx < LX * LY; idx += kThreads) {
      const int ly = idx / LX, lx = idx - (idx / LX) * LX;
      const int i = i0 + lx, j = j0 + ly;
      if (i < 0 || j < 0 || j >= g.ny || i >= g.nx) continue;
      const int m0 = absorbing_faces(g, i, j);
      const T w0 = m0 ? sv[ly][lx] / (T(1) + dt * (T)m0 * sqrt(scc[ly][lx]) * half_inv_h) : sv[ly][lx];
      if (i <= g.nx - 2 && lx <= LX - 2) {
        const int m1 = absorbing_faces(g, i + 1, j);
        const T w1 = m1 ? sv[ly][lx + 1] / (T(1) + dt * (T)m1 * sqrt(scc[ly][lx + 1]) * half_inv_h)
                        : sv[ly][lx + 1];
        sPx[ly][lx] -= dt * ((w1 - w0) * inv_h);
      }
      if (j <= g.ny - 2 && ly <= LY - 2) {
        const int m1 = absorbing_faces(g, i, j + 1);
        const T w1 = m1 ? sv[ly + 1][lx] / (T(1) + dt * (T)m1 * sqrt(scc[ly + 1][lx]) * half_inv_h)
                        : sv[ly + 1][lx];
        sPy[ly][lx] -= dt * ((w1 - w0) * inv_h);
      }
    }
    __syncthreads();
    // velocity update  v <- a v - kick c^2 D p
    const T k = (L.last && s == L.nsteps - 1) ? T(0.5) * dt : dt;
    for (int idx = tid; idx < LX * LY; idx += kThreads) {
      const int ly = idx / LX, lx = idx - (idx / LX) * LX;
      const int i = i0 + lx, j = j0 + ly;
      if (lx < 1 || ly < 1 || i < 0 || j < 0 || i >= g.nx || j >= g.ny) continue;
      const T div = (sPx[ly][lx] - sPx[ly][lx - 1] + sPy[ly][lx] - sPy[ly - 1][lx]) * inv_h;
      const T c2 = scc[ly][lx];
      const int m = absorbing_faces(g, i, j);
      T v = sv[ly][lx];
      if (m) {
        const T gam = dt * (T)m * sqrt(c2) * half_inv_h;
        v = (T(1) - gam) / (T(1) + gam) * v;
      }
      sv[ly][lx] = v - k * c2 * div;
    }
    __syncthreads();
  }

  for (int idx = tid; idx < kTX * TY; idx += kThreads) {
    const int ly = H + idx / kTX, lx = H + idx % kTX;
    const int i = i0 + lx, j = j0 + ly;
    if (i >= g.nx || j >= g.ny) continue;
    const size_t o = (size_t)j * g.pitch + i;
    T a = sPx[ly][lx], b = sPy[ly][lx], c = sv[ly][lx];
    if (p.sub) {
      a -= p.sub[o];
      b -= p.sub[o + fs];
      c -= p.sub[o + 2 * fs];
    }
    p.out[o] = a;
    p.out[o + fs] = b;
    p.out[o + 2 * fs] = c;
  }
}

template <typename T, int KMAX, int TY, bool ADJ>
hipError_t launch_one(const F1Geom &g, const F1Ptrs<T> &p, const F1Launch &L, hipStream_t s) {
  dim3 grid((g.nx + kTX - 1) / kTX, (g.ny + TY - 1) / TY);
  if (ADJ)
    hipLaunchKernelGGL((f1_adjoint_kernel<T, KMAX, TY>), grid, dim3(kThreads), 0, s, g, p, L);
  else
    hipLaunchKernelGGL((f1_forward_kernel<T, KMAX, TY>), grid, dim3(kThreads), 0, s, g, p, L);
  return hipGetLastError();
}

template <typename T, bool ADJ>
hipError_t launch_dispatch(const F1Geom &g, const F1Ptrs<T> &p, const F1Launch &L, int kmax,
                           hipStream_t s) {
  switch (kmax) {
    case 1: return launch_one<T, 1, 16, ADJ>(g, p, L, s);
    case 2: return launch_one<T, 2, 16, ADJ>(g, p, L, s);
    case 4: return launch_one<T, 4, 32, ADJ>(g, p, L, s);
    case 8: return launch_one<T, 8, 32, ADJ>(g, p, L, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------------------
// CG vector kernels
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Block sum in a fixed order; result valid in thread 0.
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

template <typename TC>
__device__ __forceinline__ double load_d(const void *p, size_t o) {
  return (double)static_cast<const TC *>(p)[o];
}

template <typename TA, typename TB, typename TC>
__global__ __launch_bounds__(kRedThreads) void f1_dot_kernel(F1Geom g, const TA *a, const TB *b,
                                                             const TC *cc, size_t fs,
                                                             double *partials) {
  // <a, b>_E = h^2 (sum over faces a b + sum over cells a b / c^2)
  double acc_p = 0.0, acc_v = 0.0;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < fs; o += stride) {
    acc_p += (double)a[o] * (double)b[o] + (double)a[o + fs] * (double)b[o + fs];
    acc_v += (double)a[o + 2 * fs] * (double)b[o + 2 * fs] / (double)cc[o];
  }
  const double h2 = g.h * g.h;
  const double t = block_sum(h2 * acc_p + h2 * acc_v);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <typename T, typename TC>
__global__ __launch_bounds__(kRedThreads) void f1_cg_update_kernel(F1Geom g, double *z, double *r,
                                                                   const T *d, const T *q,
                                                                   const TC *cc, size_t fs,
                                                                   const double *scalars,
                                                                   double *partials) {
  // Steps 5.4-5.5: z -= alpha d, r -= alpha q; partial <r, r>_E of the new residual
  const double alpha = scalars[kAlpha];
  double acc_p = 0.0, acc_v = 0.0;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < fs; o += stride) {
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const size_t k = o + f * fs;
      z[k] -= alpha * (double)d[k];
      const double rn = r[k] - alpha * (double)q[k];
      r[k] = rn;
      if (f < 2) acc_p += rn * rn;
      else acc_v += rn * rn / (double)cc[o];
    }
  }
  const double h2 = g.h * g.h;
  const double t = block_sum(h2 * acc_p + h2 * acc_v);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(kRedThreads) void finalize_kernel(const double *partials, int n,
                                                               double *sc, int mode, int slot) {
  double x = 0.0;
  for (int k = threadIdx.x; k < n; k += kRedThreads) x += partials[k];
  const double sum = block_sum(x);
  if (threadIdx.x != 0) return;
  switch (mode) {
    case kFinStart:
      sc[kDelta] = sum;
      sc[kDelta0] = sum;
      sc[kRel] = 1.0;
      sc[kBreak] = (sum >= 0.0 && isfinite(sum)) ? 0.0 : 1.0;
      break;
    case kFinAlpha:
      sc[kQd] = sum;
      if (!(sum > 0.0) || !isfinite(sum)) {
        sc[kBreak] = 1.0;
        sc[kAlpha] = 0.0;
      } else {
        sc[kAlpha] = sc[kDelta] / sum;
      }
      break;
    case kFinBeta: {
      const double d = sc[kDelta];
      sc[kBeta] = d > 0.0 ? sum / d : 0.0;
      sc[kDelta] = sum;
      sc[kRel] = sc[kDelta0] > 0.0 ? sqrt(fmax(sum, 0.0) / sc[kDelta0]) : 0.0;
      if (!isfinite(sum)) sc[kBreak] = 1.0;
      break;
    }
    default:
      sc[slot] = sum;
  }
}

template <typename TD, typename TS>
__global__ void convert_kernel(TD *dst, const TS *src, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
    dst[k] = (TD)src[k];
}

template <typename T>
__global__ void direction_kernel(T *d, const double *r, const double *sc, size_t n) {
  // Step 5.7: d = r + beta d
  const double beta = sc[kBeta];
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
    d[k] = (T)(r[k] + beta * (double)d[k]);
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

hipError_t finalize(const double *partials, int n, double *scalars, int mode, int slot,
                    hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, n, scalars,
                     mode, slot);
  return hipGetLastError();
}

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
template hipError_t f1_forward_launch<float>(const F1Geom &, const F1Ptrs<float> &, const F1Launch &, int, hipStream_t);
template hipError_t f1_forward_launch<double>(const F1Geom &, const F1Ptrs<double> &, const F1Launch &, int, hipStream_t);
template hipError_t f1_adjoint_launch<float>(const F1Geom &, const F1Ptrs<float> &, const F1Launch &, int, hipStream_t);
template hipError_t f1_adjoint_launch<double>(const F1Geom &, const F1Ptrs<double> &, const F1Launch &, int, hipStream_t);
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

}  // namespace cmcg
