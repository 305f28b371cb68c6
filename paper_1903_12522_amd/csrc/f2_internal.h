// Second-order (nodal, 3D) device layout, kernel launchers and the Riesz (elliptic) solver.
#pragma once

#include "cmcg_internal.h"

namespace cmcg {

// Node fields: (nz+1) planes of (ny+1) rows of `px` values (x fastest, rows padded to 64).
struct F2Geom {
  int nx = 0, ny = 0, nz = 0;        // cells per axis (nodes are n+1)
  int px = 0;                        // row pitch in elements
  size_t plane = 0, fs = 0;          // plane stride, field stride
  double h = 0, dt = 0;
  int abs_face[6] = {0, 0, 0, 0, 0, 0};
  double lam_const = 0;              // (c dt / h)^2 when c is constant (lam array absent)
  const uint8_t *mask = nullptr;     // sound-soft nodes (device layout), or null
  int mlo[3] = {0, 0, 0}, mhi[3] = {-1, -1, -1};   // bounding box of the sound-soft nodes
  int kchunk = 16;                   // planes per thread column
  __host__ __device__ size_t idx(int i, int j, int k) const {
    return (size_t)k * plane + (size_t)j * px + i;
  }
};

// Node loop over the real nodes of a field: one wavefront per (j, k) row, lanes over i; rows are
// dealt to the wavefronts of the grid in a fixed order (reductions stay deterministic).  Padding
// columns i > nx are never visited.  Close with F2_ROWS_END.
#define F2_ROWS(g)                                                                          \
  const int lane_ = threadIdx.x & 63;                                                       \
  const int wpb_ = blockDim.x >> 6;                                                         \
  const int nrows_ = ((g).ny + 1) * ((g).nz + 1);                                           \
  for (int r_ = blockIdx.x * wpb_ + (threadIdx.x >> 6); r_ < nrows_; r_ += gridDim.x * wpb_) { \
    const int j = r_ % ((g).ny + 1), k = r_ / ((g).ny + 1);                                 \
    const size_t row_ = (size_t)r_ * (g).px;                                                \
    for (int i = lane_; i <= (g).nx; i += 64) {                                             \
      const size_t o = row_ + i;
#define F2_ROWS_END \
  }                 \
  }

// Sweeps of the period kernel.  The backward period runs in the scaled adjoint variable
// g = psi a, psi = lambda R / ((1 + beta) eta): in it the transposed step is the forward step,
// so only its first sweep (transposed end map) and last sweep (transposed start map) differ.
enum F2Mode : int {
  kF2FwdStart = 0,      // start map u^1 from (u^0, v^0)
  kF2FwdStep = 1,       // u^{n+1} from (u^n, u^{n-1}); also every interior backward step
  kF2FwdEnd = 2,        // end map (u^N, v^N) - sub
  kF2Metric = 3,        // y = M_E w
  kF2AdjInit = 4,       // transposed end map in g: g_0 and psi b_0 from (g_y = psi y_v, y_u)
  kF2AdjStepFirst = 5,  // g_1 = K g_0 + psi b_0
  kF2AdjEnd = 6         // transposed start map from (g_M, g_{M-1}) back to (u_0, v_0) - sub
};

template <typename T>
struct F2Args {
  const T *st = nullptr;     // stencilled field
  const T *aux = nullptr;    // second input (v^0, u^{n-1}, w_v, y_u, b_0 or a_{m-1})
  const T *sub = nullptr;    // epilogue subtrahend (two fields) or null
  const T *lam = nullptr;    // (c dt / h)^2 per node, or null (constant)
  const T *fre = nullptr, *fim = nullptr;   // dt^2 c^2 G per node
  T *out = nullptr, *out2 = nullptr;
  double *ure = nullptr, *uim = nullptr;    // filter accumulators
  int forced = 0;
  double fcos = 1, fsin = 0;                // source phase cos/sin(omega t_n)
  double wcos = 1, wsin = 0;                // filter weight cos/sin(omega t_n)
  // Dirichlet data Re(gD e^{-i w t}) on the sound-soft nodes of a forced period (null: zero):
  // the value at time t is dre * dcos + dim * dsin with dcos, dsin = cos, sin(w t) (times the
  // source ramp).  *0: the sweep's input time (start map), *1: its output time.
  const double *dre = nullptr, *dim = nullptr;
  double dcos0 = 0, dsin0 = 0, dcos1 = 0, dsin1 = 0;
};

template <typename T>
hipError_t f2_march(int mode, const F2Geom &g, const F2Args<T> &p, hipStream_t s);
// rows per wavefront and wavefronts per workgroup of the blocked launches in precision T
template <typename T>
void f2_block_shape(int *rpw, int *wv);
// K (2..4) homogeneous steps in one launch, temporally blocked: from u^n (cur) and u^{n-1}
// (prev) to u^{n+K} (out_k) and u^{n+K-1} (out_km1); the outputs may alias neither input
template <typename T>
hipError_t f2_march_block(const F2Geom &g, const T *cur, const T *prev, const T *lam, T *out_k,
                          T *out_km1, int K, hipStream_t s);
// out = psi in, psi = lambda R / ((1 + beta) eta) (entry into the scaled adjoint variable)
template <typename T>
hipError_t f2_psi_scale(const F2Geom &g, const T *in, const T *lam, T *out, hipStream_t s);
template <typename TA, typename TB>
hipError_t dot_plain(const TA *a, const TB *b, size_t n, double *partials, hipStream_t s);
// Steps 5.4-5.5 (FP64 arithmetic): z -= alpha d, r_u -= alpha q_u, rh -= alpha qh, partials of
// delta.  qu: the primal Riesz update q_u in FP64, or (FP32-mixed V-cycle) the FP32 V-cycle
// result; TR: residual storage; TZ: the iterate (FP64), or its FP32 correction dz (FP32-mixed)
template <typename T, typename TQ, typename TR, typename TZ>
hipError_t f2_cg_update(const F2Geom &g, TZ *z, TR *ru, TR *rh, const T *d, const TQ *qu,
                        const T *qh, const T *lam, const double *sc, double *partials,
                        hipStream_t s);
// partials of delta = <rh, r> from FP64 residuals; rus, rhs (may be null): their stored copies
template <typename T, typename TR>
hipError_t f2_delta(const F2Geom &g, const double *ru, const double *rh, const T *lam, TR *rus,
                    TR *rhs, double *partials, hipStream_t s);
template <typename T, typename TR>
hipError_t f2_direction(const F2Geom &g, T *d, const TR *ru, const TR *rh, const T *lam,
                        const double *sc, int first, hipStream_t s);
// out = z + dz (two fields); `clear`: dz = 0 (with out == z: z += dz, dz = 0)
hipError_t f2_iterate(const F2Geom &g, const double *z, float *dz, double *out, int clear,
                      hipStream_t s);
// out = (r_u, M^{-1} rh_v) in FP64 (the primal residual)
template <typename TR, typename T>
hipError_t f2_primal(const F2Geom &g, const TR *ru, const TR *rh, const T *lam, double *out,
                     hipStream_t s);
template <typename T>
hipError_t f2_mass_inverse(const F2Geom &g, const T *qh_v, double *q_v, const T *lam, hipStream_t s);
// Partial sums (kCompatSums x kRedBlocks, sum-major) of the compatibility condition: sum M,
// sum B, sum Fhat (re, im), sum M a (re, im), sum B a (re, im) with a = sa ar + i sb ai
// (ai may be null); FP64 fields of the device layout.
constexpr int kCompatSums = 8;
hipError_t f2_compat_sums(const F2Geom &g, const double *lam, const double *Fre, const double *Fim,
                          const double *ar, double sa, const double *ai, double sb,
                          double *partials, hipStream_t s);
template <typename T>
hipError_t f2_setup(const F2Geom &g, const double *c, double c_const, const double *fre,
                    const double *fim, const double *gre, const double *gim, T *lam, T *Fre, T *Fim,
                    hipStream_t s);
template <typename T>
hipError_t f2_unpack(const F2Geom &g, const double *packed, T *dev, int nfields, hipStream_t s);
template <typename T>
hipError_t f2_pack(const F2Geom &g, const T *dev, double *packed, int nfields, hipStream_t s);

// ---------------------------------------------------------------------------------------
// Riesz map of eq. CMCG_PRECONDITIONIER: solve S x = b on the free nodes (S = diag(h eta) L,
// the mass-lumped stiffness), by conjugate gradients preconditioned with one geometric multigrid
// V-cycle (damped Jacobi smoothing, trilinear prolongation, its transpose as restriction,
// rediscretised coarse operators, sound-soft mask injected to coarse nodes).  With no sound-soft
// node S is singular (constants): right-hand side and iterates are kept zero-sum.
// ---------------------------------------------------------------------------------------
template <typename T>
struct MGLevelT {
  F2Geom g;                         // geometry (mask pointer into `maskbuf`)
  T *x = nullptr, *b = nullptr, *r = nullptr, *t = nullptr;
  uint8_t *maskbuf = nullptr;
  size_t nfree = 0;                 // number of free (non-sound-soft) real nodes
};

class DeviceArena;

// T: the storage and arithmetic type of the hierarchy.  FP64 serves the PCG solve and FP64
// solves; FP32 serves the fixed V-cycle of FP32-mixed solves (apply_vcycle only).
template <typename T>
class RieszMGT {
 public:
  ~RieszMGT();
  cmcg_status build(const F2Geom &fine, DeviceArena &arena, hipStream_t s);
  // x = S^{-1} b (x: FP64 fine-level field; b: fine-level field in FP64, or FP32 if b_is_float;
  // x may not alias b).  *iters receives the number of PCG iterations.  FP64 hierarchy only.
  // Returns CMCG_ENOTCONV when max_iter iterations did not reach the relative tolerance (x is
  // then the last iterate).
  cmcg_status solve(const void *b, int b_is_float, double *x, double tol, int max_iter, int *iters);
  // x = Pi B Pi b for an FP64 or FP32 right-hand side (Pi: zero-sum projection when S is
  // singular): the fixed symmetric V-cycle used in place of S^{-1}; x is FP64
  cmcg_status apply_vcycle(const void *b, int b_is_float, double *x);
  // the same V-cycle, its result left in the hierarchy's own type: *x points at a buffer of
  // the hierarchy, valid until its next call
  cmcg_status apply_vcycle_native(const void *b, int b_is_float, const T **x);
  bool pure_neumann() const { return neumann_; }

 private:
  // x = B b: one V-cycle on the fine level (b is not modified)
  cmcg_status vcycle(const T *b, T *x);
  cmcg_status vcycle_level(int l);
  cmcg_status smooth(int l, int sweeps);
  cmcg_status project(T *v, int l);
  cmcg_status dot(const double *a, const double *b, size_t n, double *out);
  std::vector<MGLevelT<T>> lv_;
  T *pr_ = nullptr;                 // the fine right-hand side (converted or copied)
  T *pz_ = nullptr, *pp_ = nullptr, *pq_ = nullptr;   // fine PCG vectors (FP64 only)
  T *xo_ = nullptr;                 // FP32: the V-cycle's result before its FP64 output
  double *partials_ = nullptr, *scal_ = nullptr, *h_scal_ = nullptr;
  hipStream_t s_ = nullptr;
  bool neumann_ = false;
  bool rows_ = false;               // stencil sweeps in the row kernels instead of the plane march
  int chunk_ = 0;                   // planes per march chunk (0: chosen per level)
  void read_sweep_env();
  int pre_ = 2, post_ = 2, coarse_sweeps_ = 64;
  double omega_ = 0.8;
};

}  // namespace cmcg
