// Riesz representer of eq. CMCG_PRECONDITIONIER on the device: the elliptic solve S x = b with the
// mass-lumped nodal stiffness S = diag(h eta) L (L: 7-point operator with mirrored neighbours at
// the box faces), homogeneous Dirichlet on sound-soft nodes.  Conjugate gradients in FP64,
// preconditioned by a symmetric geometric multigrid V-cycle:
//   * levels: cells halved per axis while every axis stays even and >= 2 cells; the coarse
//     operator is the same discretisation with spacing 2h; a coarse node is sound-soft when the
//     fine node at its position is;
//   * smoother: damped Jacobi (the diagonal of S is 6 h eta), the same number of sweeps before and
//     after the coarse correction, so the cycle is a symmetric operator;
//   * transfers: trilinear prolongation P and restriction P^T, both restricted to free nodes;
//   * coarsest level: a fixed number of Jacobi sweeps from zero (a fixed symmetric polynomial).
// With no sound-soft node S is singular (constant vectors); right-hand side, preconditioned
// residuals and the solution are kept zero-sum (plain sum over nodes).
// The hierarchy is a template over its storage and arithmetic type: FP64 for the PCG solve and
// FP64 solves, FP32 for the single fixed V-cycle that FP32-mixed solves use in place of S^{-1}
// (the reductions of the zero-sum projection accumulate in FP64 either way).
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "f2_internal.h"
#include "solver.h"

namespace cmcg {
namespace {

__device__ __forceinline__ int mir(int i, int n) { return i < 0 ? 1 : (i > n ? n - 1 : i); }

__device__ __forceinline__ double eta3(const F2Geom &g, int i, int j, int k) {
  double e = 1.0;
  if (i == 0 || i == g.nx) e *= 0.5;
  if (j == 0 || j == g.ny) e *= 0.5;
  if (k == 0 || k == g.nz) e *= 0.5;
  return e;
}

__device__ __forceinline__ bool msk(const F2Geom &g, int i, int j, int k) {
  if (!g.mask) return false;
  if (i < g.mlo[0] || i > g.mhi[0] || j < g.mlo[1] || j > g.mhi[1] || k < g.mlo[2] || k > g.mhi[2])
    return false;
  return g.mask[g.idx(i, j, k)] != 0;
}

template <typename T>
__device__ __forceinline__ T lap7(const F2Geom &g, const T *x, int i, int j, int k) {
  const T c = x[g.idx(i, j, k)];
  return T(6) * c - (x[g.idx(mir(i - 1, g.nx), j, k)] + x[g.idx(mir(i + 1, g.nx), j, k)] +
                    x[g.idx(i, mir(j - 1, g.ny), k)] + x[g.idx(i, mir(j + 1, g.ny), k)] +
                    x[g.idx(i, j, mir(k - 1, g.nz))] + x[g.idx(i, j, mir(k + 1, g.nz))]);
}

// y = R S x
template <typename T>
__global__ void s_apply_kernel(F2Geom g, const T *x, T *y) {
  F2_ROWS(g)
  y[o] = msk(g, i, j, k) ? T(0) : (T)(g.h * eta3(g, i, j, k)) * lap7(g, x, i, j, k);
  F2_ROWS_END
}

// r = R (b - S x)
template <typename T>
__global__ void residual_kernel(F2Geom g, const T *x, const T *b, T *r) {
  F2_ROWS(g)
  r[o] = msk(g, i, j, k) ? T(0) : b[o] - (T)(g.h * eta3(g, i, j, k)) * lap7(g, x, i, j, k);
  F2_ROWS_END
}

// damped Jacobi: xo = R (x + omega (b - S x) / (6 h eta))
template <typename T>
__global__ void jacobi_kernel(F2Geom g, const T *x, const T *b, T *xo, double omega,
                              int from_zero) {
  const T om = (T)omega;
  F2_ROWS(g)
  if (msk(g, i, j, k)) {
    xo[o] = T(0);
    continue;
  }
  const T he = (T)(g.h * eta3(g, i, j, k));
  if (from_zero) {
    xo[o] = om * b[o] / (T(6) * he);
  } else {
    xo[o] = x[o] + om * (b[o] - he * lap7(g, x, i, j, k)) / (T(6) * he);
  }
  F2_ROWS_END
}

// The same three stencil sweeps (Jacobi from a previous iterate, residual, y = R S x) as a
// march through the planes: wavefront w of a block owns row j = 4 by + w, its lanes the columns
// i = 64 bx + lane, and it walks the planes of chunk bz keeping x of its own column at k-1, k and
// k+1 in registers.  Each node's operands and the order of their arithmetic are those of the row
// kernels above, so the results are the same bit for bit; what changes is where the operands come
// from.  In the row kernels the rows of planes k - 1 and k + 1 are loaded by workgroups on other
// dies, so each plane of x crosses the memory system about three times.  Here those values are
// already in registers, and the x and y neighbours are rows that this and the neighbouring
// wavefronts load at the same plane.  Workgroups are ordered chunk-major and dealt to the eight
// dies in contiguous ranges, so vertically adjacent rows share an L2.  A chunk spans `chunk`
// planes (32 on large levels, fewer where that would leave the launch short of workgroups).
enum MGSweep : int { kMGJacobi = 0, kMGResidual = 1, kMGApply = 2 };
constexpr int kMGChunk = 32;

template <typename T, int MODE>
__global__ __launch_bounds__(256) void mg_march_kernel(F2Geom g, const T *x, const T *b, T *out,
                                                       double omega, int nbx, int nby,
                                                       int chunk) {
  const T om = (T)omega;
  const int nb = (int)gridDim.x;
  int t = (int)blockIdx.x;
  if (nb % 8 == 0) t = (t % 8) * (nb / 8) + t / 8;
  const int bx = t % nbx, by = (t / nbx) % nby, bz = t / (nbx * nby);
  const int i = bx * 64 + (int)(threadIdx.x & 63), j = by * 4 + (int)(threadIdx.x >> 6);
  if (i > g.nx || j > g.ny) return;          // no barriers below
  const int k0 = bz * chunk, k1 = min(k0 + chunk, g.nz + 1);
  const size_t col = (size_t)j * g.px + i;
  const size_t oim = (size_t)j * g.px + mir(i - 1, g.nx), oip = (size_t)j * g.px + mir(i + 1, g.nx);
  const size_t ojm = (size_t)mir(j - 1, g.ny) * g.px + i, ojp = (size_t)mir(j + 1, g.ny) * g.px + i;
  // operands of plane k held in registers; those of plane k + 1 are loaded while plane k is
  // computed (the plane after the last one is read at its mirror index, inside the field)
  T xm = x[(size_t)mir(k0 - 1, g.nz) * g.plane + col];
  T xc = x[(size_t)k0 * g.plane + col];
  T xp = x[(size_t)mir(k0 + 1, g.nz) * g.plane + col];
  size_t pk = (size_t)k0 * g.plane;
  T nim = x[pk + oim], nip = x[pk + oip], njm = x[pk + ojm], njp = x[pk + ojp];
  T bk = MODE == kMGApply ? T(0) : b[pk + col];
  for (int k = k0; k < k1; ++k) {
    const size_t pn = (size_t)mir(k + 1, g.nz) * g.plane;
    const T xpp = x[(size_t)mir(k + 2 > g.nz ? g.nz + 1 : k + 2, g.nz) * g.plane + col];
    const T nim1 = x[pn + oim], nip1 = x[pn + oip], njm1 = x[pn + ojm], njp1 = x[pn + ojp];
    const T bk1 = MODE == kMGApply ? T(0) : b[pn + col];
    const size_t o = pk + col;
    T res = T(0);
    if (!msk(g, i, j, k)) {
      const T he = (T)(g.h * eta3(g, i, j, k));
      const T lap = T(6) * xc - (nim + nip + njm + njp + xm + xp);
      if (MODE == kMGJacobi) res = xc + om * (bk - he * lap) / (T(6) * he);
      else if (MODE == kMGResidual) res = bk - he * lap;
      else res = he * lap;
    }
    out[o] = res;
    xm = xc;
    xc = xp;
    xp = xpp;
    nim = nim1;
    nip = nip1;
    njm = njm1;
    njp = njp1;
    bk = bk1;
    pk = (size_t)(k + 1) * g.plane;
  }
}

// bc = R_c P^T rf  (full weighting over the 27 fine neighbours of the coarse node's position).
// All 27 loads are issued before the sum (neighbours outside the fine box read a clamped node);
// the terms are then added in the fixed (k, j, i) order, each only where its neighbour exists,
// so the sum is the plain loop's, operation for operation.
template <typename T>
__global__ void restrict_kernel(F2Geom gf, F2Geom gc, const T *rf, T *bc) {
  F2_ROWS(gc)
  const bool m = msk(gc, i, j, k);
  T x[3][3][3];
#pragma unroll
  for (int dk = -1; dk <= 1; ++dk) {
    const int fk = min(max(2 * k + dk, 0), gf.nz);
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      const int fj = min(max(2 * j + dj, 0), gf.ny);
      const size_t row = gf.idx(0, fj, fk);
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const int fi = min(max(2 * i + di, 0), gf.nx);
        x[dk + 1][dj + 1][di + 1] = rf[row + fi];
      }
    }
  }
  T acc = T(0);
#pragma unroll
  for (int dk = -1; dk <= 1; ++dk) {
    const int fk = 2 * k + dk;
    const bool vk = fk >= 0 && fk <= gf.nz;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      const int fj = 2 * j + dj;
      const bool vj = vk && fj >= 0 && fj <= gf.ny;
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const int fi = 2 * i + di;
        const bool v = vj && fi >= 0 && fi <= gf.nx;
        const T w = (T)((di ? 0.5 : 1.0) * (dj ? 0.5 : 1.0) * (dk ? 0.5 : 1.0));
        const T t = acc + w * x[dk + 1][dj + 1][di + 1];
        acc = v ? t : acc;
      }
    }
  }
  bc[o] = m ? T(0) : acc;
  F2_ROWS_END
}

// xf += R_f P xc  (trilinear interpolation).  The up to 8 coarse neighbours (ci0, ci1) x (cj0,
// cj1) x (ck0, ck1), equal pairs where a fine index is even, are all loaded before the sum;
// the terms are then added in the fixed (k, j, i) order, the second of an equal pair skipped,
// so the sum is the plain loop's, operation for operation.
template <typename T>
__global__ void prolong_add_kernel(F2Geom gf, F2Geom gc, const T *xc, T *xf) {
  F2_ROWS(gf)
  const bool m = msk(gf, i, j, k);
  const int ci[2] = {i >> 1, (i + 1) >> 1};
  const int cj[2] = {j >> 1, (j + 1) >> 1};
  const int ck[2] = {k >> 1, (k + 1) >> 1};
  const bool oi = i & 1, oj = j & 1, ok = k & 1;
  const T wi = oi ? T(0.5) : T(1), wj = oj ? T(0.5) : T(1), wk = ok ? T(0.5) : T(1);
  T x[2][2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const size_t row = gc.idx(0, cj[b], ck[c]);
#pragma unroll
      for (int a = 0; a < 2; ++a) x[c][b][a] = xc[row + ci[a]];
    }
  const T f = xf[o];
  T acc = T(0);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const bool v = (c == 0 || ok) && (b == 0 || oj) && (a == 0 || oi);
        const T t = acc + wi * wj * wk * x[c][b][a];
        acc = v ? t : acc;
      }
  xf[o] = m ? T(0) : f + acc;
  F2_ROWS_END
}

// coarse mask: node I sound-soft iff the fine node 2I is
__global__ void coarse_mask_kernel(F2Geom gf, F2Geom gc, const uint8_t *mf, uint8_t *mc) {
  F2_ROWS(gc)
  mc[o] = mf[gf.idx(2 * i, 2 * j, 2 * k)];
  F2_ROWS_END
}

__device__ __forceinline__ double wsum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// per-block partial sums of v over the real nodes (fixed order)
template <typename T>
__global__ __launch_bounds__(kRedThreads) void sum_kernel(F2Geom g, const T *v, double *partials) {
  __shared__ double part[kRedThreads / 64];
  double acc = 0.0;
  F2_ROWS(g)
  acc += (double)v[o];
  F2_ROWS_END
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kRedThreads / 64; ++w) t += part[w];
    partials[blockIdx.x] = t;
  }
}

// v -= s[slot] / count on the real nodes (mean removal)
template <typename T>
__global__ void sub_mean_kernel(F2Geom g, T *v, const double *sc, int slot, double count) {
  const T m = (T)(sc[slot] / count);
  F2_ROWS(g)
  v[o] -= m;
  F2_ROWS_END
}

__global__ void axpy2_kernel(double *x, double *r, const double *p, const double *q, double alpha,
                             size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    x[k] += alpha * p[k];
    r[k] -= alpha * q[k];
  }
}

__global__ void xpay_kernel(double *p, const double *z, double beta, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
    p[k] = z[k] + beta * p[k];
}

// blocks for a row loop: four rows per 256-thread block
int rows_grid(const F2Geom &g) {
  const long rows = (long)(g.ny + 1) * (g.nz + 1);
  const long b = (rows + 3) / 4;
  return (int)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

int gridn(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

// One stencil sweep of a level: the plane march, or the row kernels when `rows` is set.  The
// march's chunk length is halved from 32 planes until the launch has 8192 workgroups (one plane
// at 129^3 nodes, 32 from 513^3 up); `chunk_req` > 0 fixes it instead.
template <typename T>
hipError_t mg_sweep(int mode, bool rows, int chunk_req, const F2Geom &g, const T *x, const T *b,
                    T *out, double omega, hipStream_t s) {
  if (rows) {
    if (mode == kMGJacobi)
      hipLaunchKernelGGL(jacobi_kernel<T>, dim3(rows_grid(g)), dim3(256), 0, s, g, x, b, out, omega,
                         0);
    else if (mode == kMGResidual)
      hipLaunchKernelGGL(residual_kernel<T>, dim3(rows_grid(g)), dim3(256), 0, s, g, x, b, out);
    else
      hipLaunchKernelGGL(s_apply_kernel<T>, dim3(rows_grid(g)), dim3(256), 0, s, g, x, out);
    return hipGetLastError();
  }
  const int nbx = (g.nx + 1 + 63) / 64, nby = (g.ny + 1 + 3) / 4;
  int chunk = kMGChunk;
  if (chunk_req > 0) chunk = std::min(chunk_req, g.nz + 1);
  else
    while (chunk > 1 && (long)nbx * nby * ((g.nz + chunk) / chunk) < 8192) chunk /= 2;
  const int nbz = (g.nz + chunk) / chunk;
  const dim3 grid((unsigned)(nbx * nby * nbz));
  if (mode == kMGJacobi)
    hipLaunchKernelGGL((mg_march_kernel<T, kMGJacobi>), grid, dim3(256), 0, s, g, x, b, out, omega, nbx,
                       nby, chunk);
  else if (mode == kMGResidual)
    hipLaunchKernelGGL((mg_march_kernel<T, kMGResidual>), grid, dim3(256), 0, s, g, x, b, out, omega, nbx,
                       nby, chunk);
  else
    hipLaunchKernelGGL((mg_march_kernel<T, kMGApply>), grid, dim3(256), 0, s, g, x, b, out, omega, nbx,
                       nby, chunk);
  return hipGetLastError();
}

}  // namespace

template <typename T>
RieszMGT<T>::~RieszMGT() {
  if (h_scal_) (void)hipHostFree(h_scal_);
}

template <typename T>
cmcg_status RieszMGT<T>::build(const F2Geom &fine, DeviceArena &arena, hipStream_t s) {
  s_ = s;
  lv_.clear();
  neumann_ = fine.mask == nullptr;
  MGLevelT<T> L0;
  L0.g = fine;
  lv_.push_back(L0);
  while (true) {
    const F2Geom &g = lv_.back().g;
    if (lv_.size() >= 12 || g.nx % 2 || g.ny % 2 || g.nz % 2 || g.nx < 4 || g.ny < 4 || g.nz < 4)
      break;
    MGLevelT<T> L;
    L.g = g;
    L.g.nx = g.nx / 2;
    L.g.ny = g.ny / 2;
    L.g.nz = g.nz / 2;
    L.g.px = (L.g.nx + 1 + 63) / 64 * 64;
    L.g.plane = (size_t)L.g.px * (L.g.ny + 1);
    L.g.fs = L.g.plane * (L.g.nz + 1);
    L.g.h = 2.0 * g.h;
    for (int a = 0; a < 3; ++a) {
      L.g.mlo[a] = g.mlo[a] / 2;
      L.g.mhi[a] = (g.mhi[a] + 1) / 2;
    }
    L.g.mask = nullptr;
    lv_.push_back(L);
  }
  for (size_t l = 0; l < lv_.size(); ++l) {
    MGLevelT<T> &L = lv_[l];
    if (l > 0) {
      CMCG_TRY(arena.alloc_n(L.g.fs, &L.x, s));
      CMCG_TRY(arena.alloc_n(L.g.fs, &L.b, s));
    }
    if (l > 0) CMCG_TRY(arena.alloc_n(L.g.fs, &L.r, s));
    CMCG_TRY(arena.alloc_n(L.g.fs, &L.t, s));
    if (l > 0 && fine.mask) {
      CMCG_TRY(arena.alloc_n(L.g.fs, &L.maskbuf, s));
      hipLaunchKernelGGL(coarse_mask_kernel, dim3(rows_grid(L.g)), dim3(256), 0, s, lv_[l - 1].g,
                         L.g, lv_[l - 1].g.mask, L.maskbuf);
      CMCG_HIP(hipGetLastError());
      L.g.mask = L.maskbuf;
    }
    L.nfree = (size_t)(L.g.nx + 1) * (L.g.ny + 1) * (L.g.nz + 1);
  }
  const size_t n = fine.fs;
  CMCG_TRY(arena.alloc_n(n, &pr_, s));
  if (std::is_same<T, double>::value) {
    // the PCG vectors; S p is consumed before each V-cycle, so its buffer serves as the
    // fine residual
    CMCG_TRY(arena.alloc_n(n, &pz_, s));
    CMCG_TRY(arena.alloc_n(n, &pp_, s));
    CMCG_TRY(arena.alloc_n(n, &pq_, s));
    lv_[0].r = pq_;
  } else {
    // V-cycle only: its own fine residual and the FP32 result before the FP64 output
    CMCG_TRY(arena.alloc_n(n, &lv_[0].r, s));
    CMCG_TRY(arena.alloc_n(n, &xo_, s));
  }
  CMCG_TRY(arena.alloc_n(kRedBlocks, &partials_, s));
  CMCG_TRY(arena.alloc_n(kNumScalars, &scal_, s));
  if (!h_scal_) CMCG_HIP(hipHostMalloc((void **)&h_scal_, kNumScalars * sizeof(double)));
  CMCG_HIP(hipStreamSynchronize(s));
  return CMCG_OK;
}

template <typename T>
cmcg_status RieszMGT<T>::dot(const double *a, const double *b, size_t n, double *out) {
  CMCG_HIP(dot_plain<double, double>(a, b, n, partials_, s_));
  CMCG_HIP(finalize(partials_, kRedBlocks, scal_, kFinStore, 0, s_));
  CMCG_HIP(hipMemcpyAsync(h_scal_, scal_, sizeof(double), hipMemcpyDeviceToHost, s_));
  CMCG_HIP(hipStreamSynchronize(s_));
  *out = h_scal_[0];
  return CMCG_OK;
}

template <typename T>
cmcg_status RieszMGT<T>::project(T *v, int l) {
  // v <- v - (sum v) / count over the real nodes (pure Neumann only)
  const F2Geom &g = lv_[l].g;
  hipLaunchKernelGGL(sum_kernel<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, s_, g, v, partials_);
  CMCG_HIP(hipGetLastError());
  CMCG_HIP(finalize(partials_, kRedBlocks, scal_, kFinStore, 1, s_));
  hipLaunchKernelGGL(sub_mean_kernel<T>, dim3(rows_grid(g)), dim3(256), 0, s_, g, v, scal_, 1,
                     (double)lv_[l].nfree);
  CMCG_HIP(hipGetLastError());
  return CMCG_OK;
}

template <typename T>
cmcg_status RieszMGT<T>::smooth(int l, int sweeps) {
  // `sweeps` damped Jacobi sweeps from x = 0, ping-pong between x and t, result left in x
  MGLevelT<T> &L = lv_[l];
  T *cur = L.x, *other = L.t;
  for (int k = 0; k < sweeps; ++k) {
    if (k == 0) {
      hipLaunchKernelGGL(jacobi_kernel<T>, dim3(rows_grid(L.g)), dim3(256), 0, s_, L.g, cur, L.b,
                         other, omega_, 1);
      CMCG_HIP(hipGetLastError());
    } else {
      CMCG_HIP(mg_sweep<T>(kMGJacobi, rows_, chunk_, L.g, cur, L.b, other, omega_, s_));
    }
    std::swap(cur, other);
  }
  if (cur != L.x)
    CMCG_HIP(hipMemcpyAsync(L.x, cur, L.g.fs * sizeof(T), hipMemcpyDeviceToDevice, s_));
  return CMCG_OK;
}

template <typename T>
cmcg_status RieszMGT<T>::vcycle_level(int l) {
  MGLevelT<T> &L = lv_[l];
  const int last = (int)lv_.size() - 1;
  if (l == last) {
    CMCG_TRY(smooth(l, coarse_sweeps_));
    return CMCG_OK;
  }
  CMCG_TRY(smooth(l, pre_));
  CMCG_HIP(mg_sweep<T>(kMGResidual, rows_, chunk_, L.g, L.x, L.b, L.r, 0.0, s_));
  MGLevelT<T> &C = lv_[l + 1];
  hipLaunchKernelGGL(restrict_kernel<T>, dim3(rows_grid(C.g)), dim3(256), 0, s_, L.g, C.g, L.r, C.b);
  CMCG_HIP(hipGetLastError());
  CMCG_TRY(vcycle_level(l + 1));
  hipLaunchKernelGGL(prolong_add_kernel<T>, dim3(rows_grid(L.g)), dim3(256), 0, s_, L.g, C.g, C.x, L.x);
  CMCG_HIP(hipGetLastError());
  // post-smoothing continues from the corrected x: x <- x + omega D^{-1}(b - S x), `post` times
  T *cur = L.x, *other = L.t;
  for (int k = 0; k < post_; ++k) {
    CMCG_HIP(mg_sweep<T>(kMGJacobi, rows_, chunk_, L.g, cur, L.b, other, omega_, s_));
    std::swap(cur, other);
  }
  if (cur != L.x)
    CMCG_HIP(hipMemcpyAsync(L.x, cur, L.g.fs * sizeof(T), hipMemcpyDeviceToDevice, s_));
  return CMCG_OK;
}

// CMCG_MG_ROWS=1 (environment) runs the stencil sweeps in the row kernels and CMCG_MG_CHUNK=<n>
// fixes the march's chunk length, so that tests can compare the forms bit for bit
template <typename T>
void RieszMGT<T>::read_sweep_env() {
  const char *e = std::getenv("CMCG_MG_ROWS");
  rows_ = e && e[0] == '1';
  const char *c = std::getenv("CMCG_MG_CHUNK");
  chunk_ = c ? std::atoi(c) : 0;
}

template <typename T>
cmcg_status RieszMGT<T>::vcycle(const T *b, T *x) {
  read_sweep_env();
  MGLevelT<T> &L = lv_[0];
  L.b = const_cast<T *>(b);
  L.x = x;
  CMCG_TRY(vcycle_level(0));
  if (neumann_) CMCG_TRY(project(x, 0));
  return CMCG_OK;
}

template <typename T>
cmcg_status RieszMGT<T>::apply_vcycle(const void *b, int b_is_float, double *x) {
  const size_t n = lv_[0].g.fs;
  if (b_is_float)
    CMCG_HIP(convert<T, float>(pr_, static_cast<const float *>(b), n, s_));
  else
    CMCG_HIP(convert<T, double>(pr_, static_cast<const double *>(b), n, s_));
  if (neumann_) CMCG_TRY(project(pr_, 0));
  if constexpr (std::is_same<T, double>::value) {
    return vcycle(pr_, x);
  } else {
    CMCG_TRY(vcycle(pr_, xo_));
    CMCG_HIP(convert<double, float>(x, xo_, n, s_));
    return CMCG_OK;
  }
}

template <typename T>
cmcg_status RieszMGT<T>::apply_vcycle_native(const void *b, int b_is_float, const T **x) {
  // the result buffer: FP32, the V-cycle's own; FP64, the PCG vector z (used by solve only)
  T *dst = std::is_same<T, float>::value ? xo_ : pz_;
  const size_t n = lv_[0].g.fs;
  if (b_is_float)
    CMCG_HIP(convert<T, float>(pr_, static_cast<const float *>(b), n, s_));
  else
    CMCG_HIP(convert<T, double>(pr_, static_cast<const double *>(b), n, s_));
  if (neumann_) CMCG_TRY(project(pr_, 0));
  CMCG_TRY(vcycle(pr_, dst));
  *x = dst;
  return CMCG_OK;
}

template <typename T>
cmcg_status RieszMGT<T>::solve(const void *b, int b_is_float, double *x, double tol, int max_iter,
                               int *iters) {
  static_assert(std::is_same<T, double>::value, "the PCG solve runs in FP64");
  const F2Geom &g = lv_[0].g;
  const size_t n = g.fs;
  *iters = 0;
  read_sweep_env();
  CMCG_HIP(hipMemsetAsync(x, 0, n * sizeof(double), s_));
  if (b_is_float)
    CMCG_HIP(convert<double, float>(pr_, static_cast<const float *>(b), n, s_));
  else
    CMCG_HIP(hipMemcpyAsync(pr_, b, n * sizeof(double), hipMemcpyDeviceToDevice, s_));
  if (neumann_) CMCG_TRY(project(pr_, 0));
  double bb = 0.0;
  CMCG_TRY(dot(pr_, pr_, n, &bb));
  if (bb == 0.0) return CMCG_OK;
  CMCG_TRY(vcycle(pr_, pz_));
  CMCG_HIP(hipMemcpyAsync(pp_, pz_, n * sizeof(double), hipMemcpyDeviceToDevice, s_));
  double rz = 0.0;
  CMCG_TRY(dot(pr_, pz_, n, &rz));
  bool met = false;
  for (int it = 1; it <= max_iter; ++it) {
    CMCG_HIP(mg_sweep<T>(kMGApply, rows_, chunk_, g, pp_, nullptr, pq_, 0.0, s_));
    double pq = 0.0;
    CMCG_TRY(dot(pp_, pq_, n, &pq));
    if (!(pq > 0.0)) return set_error("Riesz PCG breakdown"), CMCG_EBREAKDOWN;
    const double alpha = rz / pq;
    hipLaunchKernelGGL(axpy2_kernel, dim3(gridn(n)), dim3(256), 0, s_, x, pr_, pp_, pq_, alpha, n);
    CMCG_HIP(hipGetLastError());
    *iters = it;
    double rr = 0.0;
    CMCG_TRY(dot(pr_, pr_, n, &rr));
    if (rr <= tol * tol * bb) {
      met = true;
      break;
    }
    CMCG_TRY(vcycle(pr_, pz_));
    double rz2 = 0.0;
    CMCG_TRY(dot(pr_, pz_, n, &rz2));
    hipLaunchKernelGGL(xpay_kernel, dim3(gridn(n)), dim3(256), 0, s_, pp_, pz_, rz2 / rz, n);
    CMCG_HIP(hipGetLastError());
    rz = rz2;
  }
  if (neumann_) CMCG_TRY(project(x, 0));
  return met ? CMCG_OK : CMCG_ENOTCONV;
}

template class RieszMGT<double>;
// the FP32 hierarchy serves the V-cycle only
template RieszMGT<float>::~RieszMGT();
template cmcg_status RieszMGT<float>::build(const F2Geom &, DeviceArena &, hipStream_t);
template cmcg_status RieszMGT<float>::apply_vcycle(const void *, int, double *);
template cmcg_status RieszMGT<float>::apply_vcycle_native(const void *, int, const float **);

}  // namespace cmcg
