// First-order device code shared by the standalone kernels (f1_kernels.hip) and the persistent
// serving kernel (f1_serve.hip): the streaming tile of a period launch and the CG vector passes.
// See f1_kernels.hip for the scheme and the kernel design.
#pragma once

#include <type_traits>

#include "cmcg_internal.h"
#include "dpp.h"

namespace cmcg {
namespace {

constexpr int kThreads = 256;   // 4 wavefronts per workgroup, each an independent strip

// XCD-aware workgroup order: consecutive workgroup ids are dispatched round-robin over the 8
// XCDs; remap so each XCD walks a contiguous band of (column group, row band) tiles, whose
// overlapping halo rows and columns then meet in that XCD's L2 (without the remap the FP32
// middle launch on a 4096^2 grid takes 189 instead of 178 us).
__device__ __forceinline__ void tile_of_block(int &bx, int &by) {
  const int nbx = gridDim.x, nby = gridDim.y;
  const int nb = nbx * nby;
  const int b = blockIdx.y * nbx + blockIdx.x;
  int t = b;
  if (nb % 8 == 0) t = (b % 8) * (nb / 8) + b / 8;
  bx = t % nbx;
  by = t / nbx;
}

// The coefficient field holds kap = dt c^2 / h per cell and the forcing field h Fhat, so that
//   dt c^2 (D p + F) = kap (dsum + h F),   dsum = (Px - Px_left) + (Py - Py_below),
//   p-kick  kick G v = (kick / h) (v_right - v),   gamma = m sqrt(kap dt / h) / 2.
// EDGE = false is the compile-time fast path of wavefronts whose 64 columns are all interior
// (1 <= i <= nx-2): no column masks and no absorbing faces except on the first and last row,
// which are wave-uniform branches.
// MASK = true handles Dirichlet (sound-soft) cells, R = 0: their v carries no unknown.  Forward:
// a forced period holds v there at the data (at the input time when the period starts, at each
// level's output time after its update), a homogeneous one at 0.  Backward (the transposed
// step): v enters the velocity update as R v.  The period's last launch stores v = 0 there.
template <typename T>
__device__ __forceinline__ T f1_dirichlet(const F1Ptrs<T> &p, size_t o, double dc, double ds) {
  double v = p.dre[o] * dc;
  if (p.dim) v = fma(p.dim[o], ds, v);
  return (T)v;
}

// Number of absorbing faces of cell (i, r): mx counts the x faces of column i.
__device__ __forceinline__ int f1_abs_faces(const F1Geom &g, int mx, int r) {
  return mx + (r == 0 ? g.abs_face[2] : 0) + (r == g.ny - 1 ? g.abs_face[3] : 0);
}

// MID: the launch is one between a period's first and last (no opening kick, no subtrahend, no
// source, no filter sums): those paths are compiled out, which keeps the register count of the
// instance these launches run at that of its fast variant.
template <typename T, int K, bool ADJ, bool EDGE, bool MASK, bool MID = false>
__device__ __forceinline__ void f1_stream_body(const F1Geom &g, const F1Ptrs<T> &p,
                                               const F1Launch &L, const int i, const int lane,
                                               const int s0, const int s1) {
  constexpr int H = K + 1;
  const int nx = g.nx, ny = g.ny;
  const size_t pitch = (size_t)g.pitch, fs = p.fs;
  const T dth = (T)(g.dt / g.h);                // dt / h
  const T hdth = T(0.5) * dth;
  const bool colIn = EDGE ? ((i >= 0) && (i < nx)) : true;
  const bool pxCol = EDGE ? ((i >= 0) && (i <= nx - 2)) : true;
  const int mx = EDGE ? ((i == 0 ? g.abs_face[0] : 0) + (i == nx - 1 ? g.abs_face[1] : 0)) : 0;
  const bool laneOut = colIn && lane >= H && lane < 64 - H;

  // per-level emissions of the previous (p) and current (c) row iteration:
  // level k emits v^k(r), Px^k(r) and Py^k(r-1) with r = j - k; CC is kap of row r.
  T Vp[K + 1], PXp[K + 1], PYp[K + 1], CCp[K + 1];
  T Vc[K + 1], PXc[K + 1], PYc[K + 1], CCc[K + 1];
  T HOLD0 = T(0);   // level 0: raw Py of the current row
  T RMp[K + 1], RMc[K + 1];   // MASK: R of the emitted row (1 free, 0 Dirichlet)
  const bool dirichlet = MASK && !ADJ && !MID && L.forced && p.dre != nullptr;
#pragma unroll
  for (int k = 0; k <= K; ++k) {
    Vp[k] = PXp[k] = PYp[k] = CCp[k] = T(0);
    Vc[k] = PXc[k] = PYc[k] = CCc[k] = T(0);
    RMp[k] = RMc[k] = T(1);
  }
  const int jstart = s0 - K - 2, jend = s1 + K;
  if (colIn && jstart - 1 >= 0 && jstart - 1 < ny) HOLD0 = p.in[(size_t)(jstart - 1) * pitch + i + fs];

  for (int j = jstart; j <= jend; ++j) {
    // ---- level 0: load row j
    const bool rowIn = (j >= 0) && (j < ny);
    const bool in0 = rowIn && colIn;
    const size_t o0 = (size_t)(rowIn ? j : 0) * pitch + (colIn ? i : 0);
    T v0 = T(0), px0 = T(0), py0 = T(0), c0 = T(0);
    if (in0) {
      v0 = p.in[o0 + 2 * fs];
      px0 = p.in[o0];
      py0 = p.in[o0 + fs];
      c0 = p.cc[o0];
    }
    T rm0 = T(1);
    if (MASK) {
      if (in0 && g.mask[o0]) rm0 = T(0);
      // a forward period starts from a state that is zero on the Dirichlet cells
      if (!ADJ && !MID && L.first && rm0 == T(0))
        v0 = dirichlet ? f1_dirichlet(p, o0, L.dc[0], L.ds[0]) : T(0);
    }
    if (!MID && L.accumulate && laneOut && j >= s0 && j < s1) {
      const double vv = (double)v0;
      p.ure[o0] += vv * L.fcos;
      p.uim[o0] += vv * L.fsin;
    }
    T pyprev = HOLD0;   // raw Py(j-1)
    HOLD0 = py0;
    if (!MID && L.first) {
      if (!ADJ) {
        // opening half kick  p <- p + dt/2 G v  (Px of row j, Py of row j-1)
        const T vr = lane_from_right(v0);
        if (in0 && pxCol) px0 = fma(hdth, vr - v0, px0);
        if (colIn && j - 1 >= 0 && j - 1 <= ny - 2) pyprev = fma(hdth, v0 - Vp[0], pyprev);
      } else {
        // backward prologue: the opening half kick v <- v - dt/2 c^2 D p (row j), then the
        // change of variables Q = -p, u = R v / (1 + gamma), then the first kick
        // Q <- Q + dt G u (Px of row j, Py of row j-1)
        const T pl = lane_from_left(px0);
        if (in0) v0 = fma(T(-0.5) * c0, (px0 - pl) + (py0 - pyprev), v0);
        if (EDGE || j == 0 || j == ny - 1) {
          const int m = in0 ? f1_abs_faces(g, mx, j) : 0;
          if (m) v0 = v0 / (T(1) + T(0.5) * (T)m * sqrt(c0 * dth));
        }
        if (MASK && rm0 == T(0)) v0 = T(0);
        const T vr = lane_from_right(v0);
        if (in0 && pxCol) px0 = fma(dth, vr - v0, -px0);
        if (colIn && j - 1 >= 0 && j - 1 <= ny - 2) pyprev = fma(dth, v0 - Vp[0], -pyprev);
      }
    }
    Vc[0] = v0;
    PXc[0] = px0;
    PYc[0] = pyprev;
    CCc[0] = c0;
    RMc[0] = rm0;

    // ---- levels 1..K: [velocity update, flux kick] (forward: v and p; backward: u and Q)
#pragma unroll
    for (int k = 1; k <= K; ++k) {
      const int r = j - k;
      const bool rIn = (r >= 0) && (r < ny);
      const bool cin = rIn && colIn;
      const bool lastk = L.last && k == K;
      const T v = Vp[k - 1], px = PXp[k - 1], pyr = PYc[k - 1], pyrm1 = PYp[k - 1];
      const T kap = CCp[k - 1];
      const T pl = lane_from_left(px);
      T dsum = (px - pl) + (pyr - pyrm1);
      if (!ADJ && !MID && L.forced && cin) {
        const size_t o = (size_t)r * pitch + i;
        dsum = fma(p.fre[o], (T)L.cs[k - 1], dsum);
        if (p.fim) dsum = fma(p.fim[o], (T)L.sn[k - 1], dsum);
      }
      const bool rowB = (r == 0) || (r == ny - 1);
      if (ADJ && lastk) {
        // backward epilogue: the closing half update back in the original variables,
        // v = (1 - gamma) u + dt/2 c^2 D Q, p = -Q
        T vn = T(0);
        const T hk = T(0.5) * kap;
        if (!EDGE && !rowB) {
          if (rIn) vn = fma(hk, dsum, v);
        } else if (cin) {
          const int m = f1_abs_faces(g, mx, r);
          if (m == 0) vn = fma(hk, dsum, v);
          else vn = fma(hk, dsum, (T(1) - T(0.5) * (T)m * sqrt(kap * dth)) * v);
        }
        const bool pyv = colIn && (r - 1 >= 0) && (r - 1 <= ny - 2);
        Vc[k] = vn;
        PXc[k] = (cin && pxCol) ? -px : px;
        PYc[k] = pyv ? -pyrm1 : pyrm1;
        CCc[k] = kap;
        RMc[k] = RMp[k - 1];
        continue;
      }
      const T kick_h = (!ADJ && lastk) ? hdth : dth;
      T vn = T(0);
      if (!EDGE && !rowB) {
        if (rIn) vn = fma(kap, dsum, v);
      } else if (cin) {
        const int m = f1_abs_faces(g, mx, r);
        if (m == 0) {
          vn = fma(kap, dsum, v);
        } else {
          const T gam = T(0.5) * (T)m * sqrt(kap * dth);
          vn = fma(kap, dsum, (T(1) - gam) * v) / (T(1) + gam);
        }
      }
      if (MASK && cin && RMp[k - 1] == T(0))
        vn = dirichlet ? f1_dirichlet(p, (size_t)r * pitch + i, L.dc[k], L.ds[k]) : T(0);
      const T vr = lane_from_right(vn);
      const T pxn = (cin && pxCol) ? fma(kick_h, vr - vn, px) : px;
      const bool pyv = colIn && (r - 1 >= 0) && (r - 1 <= ny - 2);
      const T pyn = pyv ? fma(kick_h, vn - Vp[k], pyrm1) : pyrm1;
      Vc[k] = vn;
      PXc[k] = pxn;
      PYc[k] = pyn;
      CCc[k] = kap;
      RMc[k] = RMp[k - 1];
    }

    // ---- write level K: v, Px of row j-K and Py of row j-K-1
    if (laneOut) {
      const int ro = j - K;
      if (ro >= s0 && ro < s1) {
        const size_t o = (size_t)ro * pitch + i;
        T a = PXc[K], c = Vc[K];
        if (MASK && L.last && RMc[K] == T(0)) c = T(0);   // the state is zero there
        if (!MID && p.sub) {
          a -= p.sub[o];
          c -= p.sub[o + 2 * fs];
        }
        p.out[o] = a;
        p.out[o + 2 * fs] = c;
      }
      if (ro - 1 >= s0 && ro - 1 < s1) {
        const size_t o = (size_t)(ro - 1) * pitch + i;
        T b = PYc[K];
        if (!MID && p.sub) b -= p.sub[o + fs];
        p.out[o + fs] = b;
      }
    }
#pragma unroll
    for (int k = 0; k <= K; ++k) {
      Vp[k] = Vc[k];
      PXp[k] = PXc[k];
      PYp[k] = PYc[k];
      CCp[k] = CCc[k];
      RMp[k] = RMc[k];
    }
  }
}

// Raw buffer access for the fast variant: one resource per array (wave-uniform base and byte
// size), the lane's column offset in a VGPR and the row/field offset in an SGPR, so a row costs
// no per-lane address arithmetic.  Every resource is below 2^31 bytes and every scalar offset
// below 2^31, so a lane offset of 2^31 is out of range whatever is added to it: the hardware's
// range check drops such a lane's store (and returns 0 for its load).  Halo lanes and rows
// outside the band store with that offset instead of branching around the store, so every row
// iteration issues the same memory operations and the compiler can wait for exactly the loads it
// needs rather than for everything outstanding.
constexpr int kBufWord3 = 0x00020000;      // gfx9 resource word 3: raw (unswizzled) access
constexpr unsigned kBufDrop = 0x80000000u;
constexpr unsigned long long kBufMax = 0x7fffffffull;
typedef int i32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kBufWord3);
}
__device__ __forceinline__ void buf_ld(float &x, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  x = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ void buf_ld(double &x, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  x = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
}
// The state a launch writes is read again only by the next launch, after every tile has streamed
// through L2, so the stores are non-temporal (cache-policy bit nt) and do not evict the rows
// that neighbouring tiles are about to re-read: 172.7 against 177.8 us per FP32 middle launch on
// a 4096^2 grid.
constexpr int kStorePolicy = 2;
__device__ __forceinline__ void buf_st(float x, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(x), r, (int)vo, (int)so, kStorePolicy);
}
__device__ __forceinline__ void buf_st(double x, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(i32x2, x), r, (int)vo, (int)so,
                                        kStorePolicy);
}

// a * b + c in one rounding, as fma(a, b, c), always in the three-address VOP3 form.  The
// compiler otherwise selects the two-address v_fmac (result register = addend register); in the
// row loop, whose previous and current register sets trade roles, that tie forces a copy before
// almost every FMA.  The FP32 middle instance's loop goes from 168 vector instructions per two
// rows (53 of them moves) to 132 (17), and the launch on a 4096^2 grid from 163.4 to 160.0 us.
// Arithmetic only: no memory is touched.  A translation unit that defines CMCG_FMA_TIED before
// including this header gets plain fma instead: the persistent serving kernel, held to 128
// VGPRs, spills 71 registers with the untied form against 34.
#ifdef CMCG_FMA_TIED
template <typename T>
__device__ __forceinline__ T fma3(T a, T b, T c) {
  return fma(a, b, c);
}
#else
__device__ __forceinline__ float fma3(float a, float b, float c) {
  float r;
  asm("v_fma_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ double fma3(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
#endif

// Resources and offsets of one fast-variant wavefront.
struct FastIO {
  __amdgpu_buffer_rsrc_t in, cc, out, sub, fre, fim;
  unsigned vo;        // this lane's column offset (bytes)
  unsigned vo_st;     // column offset for stores: vo, or out of range for a halo lane
  unsigned pitchb, fsb;
};

// Column offsets of the rows that row iteration j stores: Px and v of row j - K (A) and Py of
// row j - K - 1 (B), or out of range outside the band.
template <int K>
__device__ __forceinline__ void fast_store_rows(const FastIO &io, int j, int s0, int s1,
                                                unsigned &voA, unsigned &soA, unsigned &voB,
                                                unsigned &soB) {
  const int ro = j - K;
  voA = (ro >= s0 && ro < s1) ? io.vo_st : kBufDrop;
  voB = (ro - 1 >= s0 && ro - 1 < s1) ? io.vo_st : kBufDrop;
  soA = (unsigned)ro * io.pitchb;
  soB = (unsigned)(ro - 1) * io.pitchb;
}

// One row iteration of the fast variant: level 0 takes row j (v, Px, kap and the Py face above
// the row; the face below is held from the previous iteration), level k advances row j - k from
// level k-1 using the previous iteration's emissions (*p arrays) and writes this iteration's
// (*c arrays); row j - K leaves the pipeline.
// FIRST: the period's opening at level 0 (forward: the half kick p += dt/2 G v; backward: the
// prologue, half kick v -= dt/2 c^2 D p, Q = -p, Q += dt G v).  Backward launches end their
// period with the epilogue at level K when L.last (v = u + dt/2 c^2 D Q, p = -Q).  SUB: the
// stored values less the subtrahend (sub_a: Px, sub_c: v of row j - K; sub_b: Py of row
// j - K - 1), loaded one row ahead with the inputs.
// FORCED (forward): level k adds the source of its row j - k at the step's time, read from the
// forcing fields (rows that the previous levels read too, so mostly cache hits); `has_fim` is
// wave-uniform.
template <typename T, int K, bool ADJ, bool FIRST, bool SUB, bool FORCED>
__device__ __forceinline__ void f1_fast_row(const FastIO &io, const F1Launch &L, const int j,
                                            const int s0, const int s1, const T dth, const T hdth,
                                            const bool has_fim,
                                            T in_v, T in_px, const T in_py, const T in_cc,
                                            const T sub_a, const T sub_b, const T sub_c,
                                            const T (&Vp)[K + 1],
                                            const T (&PXp)[K + 1], const T (&PYp)[K + 1],
                                            const T (&CCp)[K + 1], T (&Vc)[K + 1],
                                            T (&PXc)[K + 1], T (&PYc)[K + 1], T (&CCc)[K + 1],
                                            T &HOLD0) {
  T pyprev = HOLD0;        // Py(j-1)
  if (FIRST) {
    if (!ADJ) {
      const T vr = lane_from_right(in_v);
      in_px = fma(hdth, vr - in_v, in_px);
      pyprev = fma(hdth, in_v - Vp[0], pyprev);
    } else {
      const T pl = lane_from_left(in_px);
      in_v = fma(T(-0.5) * in_cc, (in_px - pl) + (in_py - pyprev), in_v);
      const T vr = lane_from_right(in_v);
      in_px = fma(dth, vr - in_v, -in_px);
      pyprev = fma(dth, in_v - Vp[0], -pyprev);
    }
  }
  Vc[0] = in_v;
  PXc[0] = in_px;
  PYc[0] = pyprev;
  HOLD0 = in_py;
  CCc[0] = in_cc;
#pragma unroll
  for (int k = 1; k <= K; ++k) {
    const bool lastk = L.last && k == K;
    const T v = Vp[k - 1], px = PXp[k - 1], pyr = PYc[k - 1], pyrm1 = PYp[k - 1];
    const T kap = CCp[k - 1];
    const T pl = lane_from_left(px);
    T dsum = (px - pl) + (pyr - pyrm1);
    if (!ADJ && FORCED) {
      const unsigned so = (unsigned)(j - k) * io.pitchb;
      T fr;
      buf_ld(fr, io.fre, io.vo, so);
      dsum = fma(fr, (T)L.cs[k - 1], dsum);
      if (has_fim) {
        T fi;
        buf_ld(fi, io.fim, io.vo, so);
        dsum = fma(fi, (T)L.sn[k - 1], dsum);
      }
    }
    if (ADJ && lastk) {
      Vc[k] = fma(T(0.5) * kap, dsum, v);
      PXc[k] = -px;
      PYc[k] = -pyrm1;
      CCc[k] = kap;
      continue;
    }
    const T kick_h = (!ADJ && lastk) ? hdth : dth;
    const T vn = fma3(kap, dsum, v);
    const T vr = lane_from_right(vn);
    Vc[k] = vn;
    PXc[k] = fma3(kick_h, vr - vn, px);
    PYc[k] = fma3(kick_h, vn - Vp[k], pyrm1);
    CCc[k] = kap;
  }
  // row ro = j - K: Px and v; row ro - 1: Py (its upper face is complete only now)
  unsigned voA, soA, voB, soB;
  fast_store_rows<K>(io, j, s0, s1, voA, soA, voB, soB);
  T a = PXc[K], b = PYc[K], c = Vc[K];
  if (SUB) {
    a -= sub_a;
    b -= sub_b;
    c -= sub_c;
  }
  buf_st(a, io.out, voA, soA);
  buf_st(c, io.out, voA, soA + 2 * io.fsb);
  buf_st(b, io.out, voB, soB + io.fsb);
}

// Fast variant of the body for wavefronts whose 64 columns are interior (1 <= i <= nx-2), whose
// rows (with its pipeline margin) are interior, and a launch with no source and no filter, on
// arrays below 2^31 bytes.  FIRST (the period's first launch) and SUB (its last, out = result -
// sub) are compile-time variants.  No masks and no branches remain in the row loop; the
// arithmetic per cell is identical to the general body's, so results do not depend on which
// variant ran.  The row loop is unrolled by two with the previous/current register sets trading
// roles (no register copies), and each row's loads are issued one row ahead of their use.
template <typename T, int K, bool ADJ, bool FIRST, bool SUB, bool FORCED>
__device__ __forceinline__ void f1_stream_fast(const F1Geom &g, const F1Ptrs<T> &p,
                                               const F1Launch &L, const int i, const int lane,
                                               const int s0, const int s1) {
  constexpr int H = K + 1;
  const T dth = (T)(g.dt / g.h);
  const T hdth = T(0.5) * dth;
  FastIO io;
  io.fsb = (unsigned)(p.fs * sizeof(T));
  io.pitchb = (unsigned)((size_t)g.pitch * sizeof(T));
  io.in = buf_rsrc(p.in, 3 * io.fsb);
  io.cc = buf_rsrc(p.cc, io.fsb);
  io.out = buf_rsrc(p.out, 3 * io.fsb);
  io.sub = buf_rsrc(SUB ? p.sub : p.in, 3 * io.fsb);
  io.fre = buf_rsrc(FORCED ? p.fre : p.cc, io.fsb);
  io.fim = buf_rsrc(FORCED && p.fim ? p.fim : p.cc, io.fsb);
  const bool has_fim = FORCED && p.fim != nullptr;
  io.vo = (unsigned)i * (unsigned)sizeof(T);
  io.vo_st = (lane >= H && lane < 64 - H) ? io.vo : kBufDrop;
  T Va[K + 1], PXa[K + 1], PYa[K + 1], CCa[K + 1];
  T Vb[K + 1], PXb[K + 1], PYb[K + 1], CCb[K + 1];
  T HOLD0 = T(0);
#pragma unroll
  for (int k = 0; k <= K; ++k) {
    Va[k] = PXa[k] = PYa[k] = CCa[k] = T(0);
    Vb[k] = PXb[k] = PYb[k] = CCb[k] = T(0);
  }
  const int jstart = s0 - K - 2, jend = s1 + K;
  buf_ld(HOLD0, io.in, io.vo, (unsigned)(jstart - 1) * io.pitchb + io.fsb);
  // level-0 inputs of a row iteration (and the subtrahend of the rows it stores), loaded one
  // iteration ahead of their use
  struct RowIn {
    T v, px, py, cc, sa, sb, sc;
  };
  auto load_row = [&](int r, RowIn &x) {
    x.sa = x.sb = x.sc = T(0);
    if (SUB) {
      unsigned voA, soA, voB, soB;
      fast_store_rows<K>(io, r, s0, s1, voA, soA, voB, soB);
      buf_ld(x.sa, io.sub, voA, soA);
      buf_ld(x.sc, io.sub, voA, soA + 2 * io.fsb);
      buf_ld(x.sb, io.sub, voB, soB + io.fsb);
    }
    const unsigned so = (unsigned)r * io.pitchb;
    buf_ld(x.v, io.in, io.vo, so + 2 * io.fsb);
    buf_ld(x.px, io.in, io.vo, so);
    buf_ld(x.py, io.in, io.vo, so + io.fsb);
    buf_ld(x.cc, io.cc, io.vo, so);
  };
  // Schedules, chosen by measurement on a 4096^2 grid: the FP32 forward sweep is fastest with
  // the next row's loads issued unconditionally (row jend + 1 <= ny - 1 is in range) and held
  // ahead of the row's arithmetic by a scheduling barrier; the backward sweep, and FP64 (whose
  // register count that barrier raises past an occupancy step), with the compiler's schedule.
  constexpr bool pinned = !ADJ && sizeof(T) == 4;
  RowIn A;
  load_row(jstart, A);
  int j = jstart;
  for (; j + 1 <= jend; j += 2) {
    const RowIn x0 = A;
    load_row(j + 1, A);
    if (pinned) __builtin_amdgcn_sched_barrier(0);
    f1_fast_row<T, K, ADJ, FIRST, SUB, FORCED>(io, L, j, s0, s1, dth, hdth, has_fim, x0.v, x0.px,
                                               x0.py, x0.cc, x0.sa, x0.sb, x0.sc, Va, PXa, PYa,
                                               CCa, Vb, PXb, PYb, CCb, HOLD0);
    const RowIn x1 = A;
    if (pinned || j + 2 <= jend) load_row(j + 2, A);
    if (pinned) __builtin_amdgcn_sched_barrier(0);
    f1_fast_row<T, K, ADJ, FIRST, SUB, FORCED>(io, L, j + 1, s0, s1, dth, hdth, has_fim, x1.v,
                                               x1.px, x1.py, x1.cc, x1.sa, x1.sb, x1.sc, Vb, PXb,
                                               PYb, CCb, Va, PXa, PYa, CCa, HOLD0);
  }
  if (j <= jend)
    f1_fast_row<T, K, ADJ, FIRST, SUB, FORCED>(io, L, j, s0, s1, dth, hdth, has_fim, A.v, A.px,
                                               A.py, A.cc, A.sa, A.sb, A.sc, Va, PXa, PYa, CCa, Vb,
                                               PXb, PYb, CCb, HOLD0);
}

// Which fast variants a kernel instance holds.  The first and last launches of a period, and
// the launches of a forced period, run their own instances, so that the register allocation of
// the instance every other launch runs is not raised by variants it never takes.
enum F1FastSet { kFastMiddle = 0, kFastEnds = 1, kFastForced = 3 };

// Tile (bx, by) of a launch: wavefront w of the workgroup owns column strip 4 bx + w of the
// band of rows by.  Interior wavefronts (all 64 columns in 1..nx-2) of interior bands take the
// fast variant.
template <typename T, int K, bool ADJ, bool MASK, int SET>
__device__ __forceinline__ void f1_stream_tile(const F1Geom &g, const F1Ptrs<T> &p,
                                               const F1Launch &L, int band, int bx, int by) {
  constexpr int H = K + 1;             // lanes lost on each side: K levels + the opening kick
  constexpr int OW = 64 - 2 * H;       // columns written per wavefront
  const int lane = threadIdx.x & 63;
  const int strip = bx * (kThreads / 64) + (threadIdx.x >> 6);
  if (strip * OW >= g.nx) return;      // wave-uniform
  const int i0 = strip * OW - H;
  const int s0 = by * band;
  const int s1 = min(s0 + band, g.ny);
  const bool inner_cols = i0 >= 1 && i0 + 63 <= g.nx - 2;
  const bool inner_rows = s0 >= 2 * K + 3 && s1 + K <= g.ny - 2;
  const bool small = 3ull * p.fs * sizeof(T) <= kBufMax;
  constexpr bool MID = SET == kFastMiddle;
  if (MASK) {
    // wavefronts whose columns and pipeline rows (s0 - K - 3 .. s1 + K) meet the box of the
    // Dirichlet cells take the masked body; the others never touch a masked cell
    const bool meets = i0 + 63 >= g.mlo[0] && i0 <= g.mhi[0] && s1 + K >= g.mlo[1] &&
                       s0 - K - 3 <= g.mhi[1];
    if (meets) {
      if (inner_cols)
        f1_stream_body<T, K, ADJ, false, true, MID>(g, p, L, i0 + lane, lane, s0, s1);
      else
        f1_stream_body<T, K, ADJ, true, true, MID>(g, p, L, i0 + lane, lane, s0, s1);
      return;
    }
  }
  const bool fast = inner_cols && inner_rows && small && !L.accumulate && !L.general &&
                    !(L.first && p.sub) && (!L.forced || (SET == kFastForced && !ADJ));
  const bool ends = L.first || p.sub;
  if (SET == kFastForced) {
    if (fast && L.first)
      f1_stream_fast<T, K, ADJ, true, false, true>(g, p, L, i0 + lane, lane, s0, s1);
    else if (fast && p.sub)
      f1_stream_fast<T, K, ADJ, false, true, true>(g, p, L, i0 + lane, lane, s0, s1);
    else if (fast)
      f1_stream_fast<T, K, ADJ, false, false, true>(g, p, L, i0 + lane, lane, s0, s1);
    else if (inner_cols)
      f1_stream_body<T, K, ADJ, false, false>(g, p, L, i0 + lane, lane, s0, s1);
    else
      f1_stream_body<T, K, ADJ, true, false>(g, p, L, i0 + lane, lane, s0, s1);
    return;
  }
  if (SET != kFastMiddle && fast && L.first)
    f1_stream_fast<T, K, ADJ, true, false, false>(g, p, L, i0 + lane, lane, s0, s1);
  else if (SET != kFastMiddle && fast && p.sub)
    f1_stream_fast<T, K, ADJ, false, true, false>(g, p, L, i0 + lane, lane, s0, s1);
  else if (SET != kFastEnds && fast && !ends)
    f1_stream_fast<T, K, ADJ, false, false, false>(g, p, L, i0 + lane, lane, s0, s1);
  else if (inner_cols)
    f1_stream_body<T, K, ADJ, false, false, MID>(g, p, L, i0 + lane, lane, s0, s1);
  else
    f1_stream_body<T, K, ADJ, true, false, MID>(g, p, L, i0 + lane, lane, s0, s1);
}

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

// The CG vector passes as the work of block vb of a grid of nvb blocks of kRedThreads threads,
// so that a standalone kernel (vb = blockIdx.x) and a persistent one (vb a work item) do the
// same arithmetic in the same order.

// partial of <a, b>_E = h^2 (sum over faces a b + sum over cells a b / c^2); the cell weight
// h^2 / c^2 = h dt / kap
template <typename TA, typename TB, typename TC>
__device__ __forceinline__ void f1_dot_block(const F1Geom &g, const TA *a, const TB *b,
                                             const TC *cc, size_t fs, double *partials, int vb,
                                             int nvb) {
  double acc_p = 0.0, acc_v = 0.0;
  const size_t stride = (size_t)nvb * kRedThreads;
  for (size_t o = (size_t)vb * kRedThreads + threadIdx.x; o < fs; o += stride) {
    acc_p += (double)a[o] * (double)b[o] + (double)a[o + fs] * (double)b[o + fs];
    acc_v += (double)a[o + 2 * fs] * (double)b[o + 2 * fs] / (double)cc[o];
  }
  const double t = block_sum(g.h * g.h * acc_p + g.h * g.dt * acc_v);
  if (threadIdx.x == 0) partials[vb] = t;
}

// Steps 5.4-5.5: z -= alpha d, r -= alpha q; partial <r, r>_E of the new residual
template <typename T, typename TC>
__device__ __forceinline__ void f1_cg_update_block(const F1Geom &g, double *z, double *r,
                                                   const T *d, const T *q, const TC *cc,
                                                   size_t fs, const double *scalars,
                                                   double *partials, int vb, int nvb) {
  const double alpha = scalars[kAlpha];
  double acc_p = 0.0, acc_v = 0.0;
  const size_t stride = (size_t)nvb * kRedThreads;
  for (size_t o = (size_t)vb * kRedThreads + threadIdx.x; o < fs; o += stride) {
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
  const double t = block_sum(g.h * g.h * acc_p + g.h * g.dt * acc_v);
  if (threadIdx.x == 0) partials[vb] = t;
}

// one block: sum the n partials in index order and apply `mode` to the scalars
__device__ __forceinline__ void finalize_block(const double *partials, int n, double *sc, int mode,
                                               int slot) {
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
      sc[kTmp] = d;
      sc[kBeta] = d > 0.0 ? sum / d : 0.0;
      sc[kDelta] = sum;
      sc[kRel] = sc[kDelta0] > 0.0 ? sqrt(fmax(sum, 0.0) / sc[kDelta0]) : 0.0;
      if (!isfinite(sum)) sc[kBreak] = 1.0;
      break;
    }
    case kFinRefresh: {
      // the recursive residual was replaced by the true one: beta and delta from it
      const double d = sc[kTmp];
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
__device__ __forceinline__ void convert_block(TD *dst, const TS *src, size_t n, int vb, int nvb) {
  const size_t stride = (size_t)nvb * 256;
  for (size_t k = (size_t)vb * 256 + threadIdx.x; k < n; k += stride) dst[k] = (TD)src[k];
}

// Step 5.7: d = r + beta d
template <typename T>
__device__ __forceinline__ void direction_block(T *d, const double *r, const double *sc, size_t n,
                                                int vb, int nvb) {
  const double beta = sc[kBeta];
  const size_t stride = (size_t)nvb * 256;
  for (size_t k = (size_t)vb * 256 + threadIdx.x; k < n; k += stride)
    d[k] = (T)(r[k] + beta * (double)d[k]);
}

// u = i V / omega with V = (2/N) (Ure + i Uim)  (eq. TH_FILTERED_MIXED_SOLUTION, discrete)
__device__ __forceinline__ void f1_output_block(const double *ure, const double *uim,
                                                double scale, double *out_re, double *out_im,
                                                size_t fs, int vb, int nvb) {
  const size_t stride = (size_t)nvb * 256;
  for (size_t o = (size_t)vb * 256 + threadIdx.x; o < fs; o += stride) {
    out_re[o] = -scale * uim[o];
    out_im[o] = scale * ure[o];
  }
}

}  // namespace
}  // namespace cmcg
