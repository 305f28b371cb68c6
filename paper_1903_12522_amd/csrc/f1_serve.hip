// The persistent serving kernel: one launch per server tick advances every resident first-order
// solve through rounds of its CG algorithm.  A round runs one operation of each running solve
// (serve_plan.h): a launch of a period (the streaming tiles of K leapfrog steps), a CG vector
// pass (in the virtual blocks of the standalone kernel, so that every sum is formed in the same
// order), a reduction, or a decision taken from the solve's scalars; a grid barrier separates
// rounds.  Every workgroup holds the solves' states in LDS and plans each round itself, from the
// same states and the same scalars, so the plans agree without being exchanged; workgroup 0
// writes the states back when the tick ends.  The items of a round (the tiles and blocks of all
// solves' operations) are dealt to the workgroups round-robin.
//
// The grid is the co-resident one (a cooperative launch).  Every barrier wait is bounded: a
// workgroup gives up after `spin_limit` polls, or when the host sets the abort flag (pinned
// host memory) or another workgroup has given up; the kernel then ends at that barrier and the
// tick reports the failure.
// (the two-address FMA form: the untied one raises this kernel's spills at its 128-VGPR cap)
#define CMCG_FMA_TIED
#include "f1_device.h"

namespace cmcg {
namespace {

using namespace serve;

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Grid barrier with a bounded wait.  The generation is read before arriving, so it cannot move
// on before this workgroup has arrived.  Arrivals release this workgroup's writes; the last one
// acquires them all, resets the count and releases the next generation; the others poll the
// generation with relaxed loads (no cache maintenance per poll) and acquire once it moved.
// Returns false (in every thread) if this workgroup gave up.
__device__ bool grid_sync(ServeControl *ctl, const int *abort_flag,
                          unsigned long long spin_limit) {
  __shared__ int ok_s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned g0 = __hip_atomic_load(&ctl->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived =
        __hip_atomic_fetch_add(&ctl->count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (arrived == gridDim.x) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(&ctl->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&ctl->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      // (the abort flag lives in host memory: it is read every 4096 polls only, so that the
      // waiting workgroups do not all cross PCIe on every poll)
      unsigned long long spins = 0;
      while (__hip_atomic_load(&ctl->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
        ++spins;
        if (spins > spin_limit ||
            __hip_atomic_load(&ctl->failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
            ((spins & 4095) == 0 &&
             __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0)) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (!ok) __hip_atomic_store(&ctl->failed, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ok_s = ok;
  }
  __syncthreads();
  return ok_s != 0;
}

__device__ __forceinline__ Params params_of(const ServeSlot &sl) {
  Params P;
  P.N = sl.N;
  P.K_lo = sl.K_lo;
  P.K_hi = sl.K_hi;
  P.mixed = sl.mixed;
  P.max_iter = sl.max_iter;
  P.tol = sl.tol;
  P.refresh = sl.refresh;
  return P;
}

__device__ __forceinline__ double load_scalar(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// virtual blocks of an element-wise pass over n values (the standalone kernels' grid)
__device__ __forceinline__ int vblocks(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

// tiles of a launch of ns steps: strips of 64 - 2 (ns + 1) columns, four per workgroup
__device__ __forceinline__ void launch_tiles(const F1Geom &g, int ns, int band, int *nbx,
                                             int *nby) {
  const int ow = 64 - 2 * (ns + 1);
  const int strips = (g.nx + ow - 1) / ow;
  *nbx = (strips + 3) / 4;
  *nby = (g.ny + band - 1) / band;
}

// Tile kinds: 0 a launch between a period's first and last (forward or backward: the same
// forward instance), 1 a forward period's first or last, 2 a backward period's first or last,
// 3 a forced (FP64) period's launch.
template <typename T, int NS>
__device__ __forceinline__ void tile_k(int kind, const F1Geom &g, const F1Ptrs<T> &p,
                                       const F1Launch &L, int band, int bx, int by) {
  if (kind == 0) f1_stream_tile<T, NS, false, false, kFastMiddle>(g, p, L, band, bx, by);
  else if (kind == 1) f1_stream_tile<T, NS, false, false, kFastEnds>(g, p, L, band, bx, by);
  else if (kind == 2) f1_stream_tile<T, NS, true, false, kFastEnds>(g, p, L, band, bx, by);
  else if constexpr (sizeof(T) == 8)
    f1_stream_tile<T, NS, false, false, kFastForced>(g, p, L, band, bx, by);
}

// The launch sizes a served period uses: FP32 7, 4, 2, 1 steps, FP64 4, 2, 1.
template <typename T>
__device__ __forceinline__ void tile(int ns, int kind, const F1Geom &g, const F1Ptrs<T> &p,
                                     const F1Launch &L, int band, int bx, int by) {
  switch (ns) {
    case 1: tile_k<T, 1>(kind, g, p, L, band, bx, by); break;
    case 2: tile_k<T, 2>(kind, g, p, L, band, bx, by); break;
    case 4: tile_k<T, 4>(kind, g, p, L, band, bx, by); break;
    case 7:
      if constexpr (sizeof(T) == 4) tile_k<T, 7>(kind, g, p, L, band, bx, by);
      break;
    default: break;
  }
}

// One tile of this round's launch of a period (the buffers and launch parameters the
// standalone period loop gives the same launch).
template <typename T>
__device__ __forceinline__ void period_item(const ServeSlot &sl, int phase, int n0, int launch,
                                            int ns, int item) {
  const bool hiset = phase == kGradFwd || phase == kGradAdj || phase == kFilter;
  T *S0 = static_cast<T *>(hiset ? (void *)sl.hi_S0 : sl.lo_S0);
  T *S1 = static_cast<T *>(hiset ? (void *)sl.hi_S1 : sl.lo_S1);
  const T *in = nullptr, *sub = nullptr;
  T *out = nullptr;
  switch (phase) {
    case kGradFwd: in = (const T *)sl.Z; out = (T *)sl.hi_W; sub = (const T *)sl.Z; break;
    case kGradAdj: in = (const T *)sl.hi_W; out = (T *)sl.hi_Q; sub = (const T *)sl.hi_W; break;
    case kFwd: in = (const T *)sl.D; out = (T *)sl.lo_W; sub = (const T *)sl.D; break;
    case kAdj: in = (const T *)sl.lo_W; out = (T *)sl.lo_Q; sub = (const T *)sl.lo_W; break;
    default: in = (const T *)sl.Z; out = (T *)sl.hi_Q; sub = nullptr; break;   // the filter
  }
  const bool last = n0 + ns == sl.N;
  F1Ptrs<T> p{};
  p.in = launch == 0 ? in : ((launch - 1) & 1 ? S1 : S0);
  p.out = last ? out : (launch & 1 ? S1 : S0);
  p.sub = last ? sub : nullptr;
  p.cc = static_cast<const T *>(hiset ? (const void *)sl.hi_cc : sl.lo_cc);
  p.fre = static_cast<const T *>(hiset ? (const void *)sl.hi_Fre : sl.lo_Fre);
  p.fim = static_cast<const T *>(hiset ? (const void *)sl.hi_Fim : sl.lo_Fim);
  p.ure = sl.Ure;
  p.uim = sl.Uim;
  p.fs = sl.fs;
  F1Launch L{};
  L.nsteps = ns;
  L.first = n0 == 0;
  L.last = last;
  L.forced = (phase == kGradFwd || phase == kFilter) ? 1 : 0;
  L.accumulate = phase == kFilter ? 1 : 0;
  // (every entry filled, those past the launch's steps from a clamped step, so that the
  // array is indexed by constants only)
#pragma unroll
  for (int k = 0; k < kMaxBlockSteps; ++k) {
    const int n = min(n0 + k, sl.N - 1);
    L.cs[k] = sl.tab[4 * n];
    L.sn[k] = sl.tab[4 * n + 1];
  }
  L.fcos = sl.tab[4 * n0 + 2];
  L.fsin = sl.tab[4 * n0 + 3];
  const bool adj = phase == kGradAdj || phase == kAdj;
  const int kind = L.forced ? 3 : adj ? ((L.first || L.last) ? 2 : 0) : ((L.first || p.sub) ? 1 : 0);
  int nbx, nby;
  launch_tiles(sl.g, ns, sl.band, &nbx, &nby);
  tile<T>(ns, kind, sl.g, p, L, sl.band, item % nbx, item / nbx);
}

// One item of a solve's operation this round.
__device__ __forceinline__ void run_item(const ServeSlot &sl, int op, int phase, int n0,
                                         int launch, int ns, int mode, int item) {
  const int nvb = vblocks(sl.vecN), nvf = vblocks(sl.fs);
  switch (op) {
    case kOpPeriod:
      if (sl.mixed && (phase == kFwd || phase == kAdj))
        period_item<float>(sl, phase, n0, launch, ns, item);
      else
        period_item<double>(sl, phase, n0, launch, ns, item);
      break;
    case kOpCopy:   // r <- the backward period's output
      convert_block<double, double>(sl.R, sl.hi_Q, sl.vecN, item, nvb);
      break;
    case kOpDotGrad:
      f1_dot_block<double, double, double>(sl.g, sl.R, sl.R, sl.hi_cc, sl.fs, sl.partials, item,
                                           kRedBlocks);
      break;
    case kOpFinalize:
      finalize_block(sl.partials, kRedBlocks, sl.scalars, mode, 0);
      break;
    case kOpConvert:
      if (sl.mixed) convert_block<float, double>((float *)sl.D, sl.R, sl.vecN, item, nvb);
      else convert_block<double, double>((double *)sl.D, sl.R, sl.vecN, item, nvb);
      break;
    case kOpDotIt:
      if (sl.mixed)
        f1_dot_block<float, float, float>(sl.g, (const float *)sl.lo_Q, (const float *)sl.D,
                                          (const float *)sl.lo_cc, sl.fs, sl.partials, item,
                                          kRedBlocks);
      else
        f1_dot_block<double, double, double>(sl.g, (const double *)sl.lo_Q, (const double *)sl.D,
                                             (const double *)sl.lo_cc, sl.fs, sl.partials, item,
                                             kRedBlocks);
      break;
    case kOpUpdate:
      if (sl.mixed)
        f1_cg_update_block<float, float>(sl.g, sl.Z, sl.R, (const float *)sl.D,
                                         (const float *)sl.lo_Q, (const float *)sl.lo_cc, sl.fs,
                                         sl.scalars, sl.partials, item, kRedBlocks);
      else
        f1_cg_update_block<double, double>(sl.g, sl.Z, sl.R, (const double *)sl.D,
                                           (const double *)sl.lo_Q, (const double *)sl.lo_cc,
                                           sl.fs, sl.scalars, sl.partials, item, kRedBlocks);
      break;
    case kOpDirection:
      if (sl.mixed) direction_block<float>((float *)sl.D, sl.R, sl.scalars, sl.vecN, item, nvb);
      else direction_block<double>((double *)sl.D, sl.R, sl.scalars, sl.vecN, item, nvb);
      break;
    case kOpZero: {   // the filter sums
      const size_t stride = (size_t)nvf * 256;
      for (size_t o = (size_t)item * 256 + threadIdx.x; o < sl.fs; o += stride) {
        sl.Ure[o] = 0.0;
        sl.Uim[o] = 0.0;
      }
      break;
    }
    case kOpOutput:
      f1_output_block(sl.Ure, sl.Uim, sl.out_scale, sl.hi_W, sl.hi_W + sl.fs, sl.fs, item, nvf);
      break;
    default: break;
  }
}

// Occupancy.  Holding every tile variant, the kernel would take 161 VGPRs (3 waves per SIMD, the
// FP64 variants set the count); capped at 128 it runs 4 waves per SIMD and spills about 100
// bytes per lane in the variants that need more.  Measured on 8 resident 1024^2 FP32-mixed solves:
// 185 GLUP/s capped against 154 uncapped.  (The compiler rejects caps of 5 and 6 waves.)
#ifndef CMCG_SERVE_WAVES
#define CMCG_SERVE_WAVES 4
#endif

__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(CMCG_SERVE_WAVES, CMCG_SERVE_WAVES))) void f1_serve_kernel(const ServeSlot *__restrict__ slots,
                                                       State *states, int nslots,
                                                       ServeControl *ctl, const int *abort_flag,
                                                       int max_rounds, double budget,
                                                       unsigned long long spin_limit) {
  __shared__ State st[kServeMaxSlots];
  __shared__ int first[kServeMaxSlots + 1], cnt[kServeMaxSlots];
  __shared__ int opk[kServeMaxSlots], nsk[kServeMaxSlots], modek[kServeMaxSlots];
  __shared__ double rwk[kServeMaxSlots];
  __shared__ int stop;
  __shared__ double round_work;
  for (int i = threadIdx.x; i < nslots; i += blockDim.x) st[i] = states[i];
  __syncthreads();
  double work = 0.0;
  int rounds = 0;
  for (;;) {
    // plan the round: thread s takes solve s (the same in every workgroup)
    if (threadIdx.x < nslots) {
      const int s = threadIdx.x;
      int op = kOpNone, n = 0, ns = 0, mode = 0;
      double rw = 0.0;
      State &S = st[s];
      if (S.active == 1) {
        const ServeSlot &sl = slots[s];
        const Params P = params_of(sl);
        if (S.phase == kGradDecide || S.phase == kItDecide) {
          Scalars sc;
          sc.delta = load_scalar(sl.scalars + kDelta);
          sc.delta0 = load_scalar(sl.scalars + kDelta0);
          sc.rel = load_scalar(sl.scalars + kRel);
          sc.brk = load_scalar(sl.scalars + kBreak);
          decide(P, S, sc);
        }
        if (S.active == 1) {
          op = op_of(S.phase);
          if (op == kOpPeriod) {
            ns = launch_steps(P.N, period_K(P, S.phase), S.n0);
            int nbx, nby;
            launch_tiles(sl.g, ns, sl.band, &nbx, &nby);
            n = nbx * nby;
            rw = (double)ns * sl.g.nx * sl.g.ny;
          } else if (op == kOpFinalize) {
            n = 1;
            mode = finalize_mode(S);
          } else if (op == kOpDotGrad || op == kOpDotIt || op == kOpUpdate) {
            n = kRedBlocks;
          } else if (op == kOpZero || op == kOpOutput) {
            n = vblocks(sl.fs);
          } else {
            n = vblocks(sl.vecN);
          }
        }
      }
      opk[s] = op;
      nsk[s] = ns;
      modek[s] = mode;
      cnt[s] = n;
      rwk[s] = rw;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int total = 0;
      double rw = 0.0;
      for (int s = 0; s < nslots; ++s) {
        first[s] = total;
        total += cnt[s];
        rw += rwk[s];
      }
      first[nslots] = total;
      stop = (total == 0 || rounds >= max_rounds || work >= budget) ? 1 : 0;
      round_work = rw;
    }
    __syncthreads();
    if (stop) break;
    // this workgroup's items
    const int total = uniform(first[nslots]);
    for (int it = blockIdx.x; it < total; it += gridDim.x) {
      int s = 0;
      while (first[s + 1] <= it) ++s;
      s = uniform(s);
      const State &S = st[s];
      run_item(slots[s], uniform(opk[s]), uniform(S.phase), uniform(S.n0), uniform(S.launch),
               uniform(nsk[s]), uniform(modek[s]), uniform(it - first[s]));
    }
    __syncthreads();
    // advance past this round's operations (thread s, solve s)
    if (threadIdx.x < nslots && opk[threadIdx.x] != kOpNone) {
      const int s = threadIdx.x;
      const ServeSlot &sl = slots[s];
      State &S = st[s];
      if (opk[s] == kOpPeriod) {
        const double cells = (double)sl.g.nx * sl.g.ny;
        const bool single = sl.mixed && (S.phase == kFwd || S.phase == kAdj);
        const double esz = single ? 4.0 : 8.0;
        const bool last = S.n0 + nsk[s] == sl.N;
        const bool sub = last && S.phase != kFilter;
        const bool forced = S.phase == kGradFwd || S.phase == kFilter;
        S.updates += nsk[s] * cells;
        S.dram += ((7.0 + (sub ? 3.0 : 0.0) + (forced ? 2.0 : 0.0)) * esz +
                   (S.phase == kFilter ? 32.0 : 0.0)) * cells;
      }
      advance(params_of(sl), S, nsk[s]);
    }
    work += round_work;
    ++rounds;
    if (!grid_sync(ctl, abort_flag, spin_limit)) break;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < nslots; i += blockDim.x) states[i] = st[i];
    if (threadIdx.x == 0) {
      ctl->rounds = rounds;
      ctl->work = work;
    }
  }
}

}  // namespace

hipError_t f1_serve_grid(int *blocks) {
  int dev = 0, per_cu = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f1_serve_kernel, 256, 0);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  *blocks = per_cu * cus;
  return *blocks > 0 ? hipSuccess : hipErrorInvalidConfiguration;
}

hipError_t f1_serve_launch(const ServeSlot *slots, State *states, int nslots, ServeControl *ctl,
                           const int *abort_flag, int max_rounds, double work_budget,
                           unsigned long long spin_limit, int blocks, hipStream_t s) {
  if (nslots < 1 || nslots > kServeMaxSlots) return hipErrorInvalidValue;
  void *args[] = {(void *)&slots, (void *)&states, (void *)&nslots, (void *)&ctl,
                  (void *)&abort_flag, (void *)&max_rounds, (void *)&work_budget,
                  (void *)&spin_limit};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(f1_serve_kernel), dim3(blocks),
                                    dim3(256), args, 0, s);
}

}  // namespace cmcg
