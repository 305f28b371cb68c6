// Round planner of the persistent serving kernel: the CG algorithm of each resident first-order
// solve (Sec. 2.3 Steps 1-6, with the reliable FP64 refreshes of the FP32-mixed mode) as a
// state machine that advances by one operation per round.  A round runs one operation of every
// running solve (a period launch of K leapfrog steps, a CG vector pass, a reduction or a
// decision); a grid barrier separates rounds.  The planner is plain C++ used by the kernel (on
// the device, identically in every workgroup) and by a CPU model of the rounds in the tests.
#pragma once

#if defined(__HIPCC__)
#define CMCG_HD __host__ __device__
#else
#define CMCG_HD
#endif

namespace cmcg {
namespace serve {

// Phases of a solve.  Period phases run launches of a period; the others run one vector pass.
enum Phase : int {
  kGradFwd = 0,    // FP64 forced period Phi(z) - z            (true gradient, Steps 2-3)
  kGradAdj,        // FP64 backward period, less its input
  kGradCopy,       // r = the backward output
  kGradDot,        // partials of <r, r>_E
  kGradFin,        // delta (start: delta0) from the partials
  kGradDecide,     // converged, or on to the iteration
  kInitD,          // d = r (rounded to the CG periods' precision)
  kFwd,            // E d - d                                  (Step 5.1)
  kAdj,            // E* w - w
  kItDot,          // partials of <q, d>_E                      (Step 5.3)
  kItFinA,         // alpha
  kItUpd,          // z -= alpha d, r -= alpha q, partials of <r, r>_E   (Steps 5.4-5.5)
  kItFinB,         // beta, delta, rel                          (Step 5.6)
  kItDecide,       // refresh, stop (Step 5.8) or the next direction
  kDir,            // d = r + beta d                            (Step 5.7)
  kFiltZero,       // the filter sums start at zero
  kFilter,         // FP64 forced period from z, one step per launch, accumulating the sums
  kOutput,         // u = i V / omega                           (Step 6 by the filter)
  kDone,
  kFailed
};

enum Op : int {
  kOpNone = 0,
  kOpPeriod,       // one launch of a period: ns steps from step n0
  kOpCopy,         // r <- hi Q
  kOpDotGrad,      // FP64 <r, r>_E partials
  kOpFinalize,     // one block: partials -> scalars (mode)
  kOpConvert,      // d <- r
  kOpDotIt,        // <q, d>_E partials in the CG periods' precision
  kOpUpdate,       // CG update with partials
  kOpDirection,    // d <- r + beta d
  kOpZero,         // filter sums <- 0
  kOpOutput        // output field from the sums
};

// The dynamic state of one resident solve.
struct State {
  int active;          // 1 running, 2 done (output field ready), 3 failed, 0 empty
  int phase;
  int n0;              // steps of the current period done
  int launch;          // launches of the current period done (buffer ping-pong)
  int iter, refreshes;
  int grad_mode;       // finalize mode of the true gradient: start or refresh
  int converged;
  int status;          // 0, or the failure status
  double delta_at_refresh;
  double updates;      // grid-point updates done
  double dram;         // compulsory HBM bytes of its stencil launches
};

// Constants of one solve that the planner needs.
struct Params {
  int N;               // steps per period
  int K_lo, K_hi;      // steps per launch of the CG periods and of the FP64 periods
  int mixed;           // FP32-mixed (CG periods in FP32, FP64 refreshes)
  int max_iter;
  double tol, refresh;
};

// The scalars a decision reads (a copy of the solve's device scalars after a finalize).
struct Scalars {
  double delta, delta0, rel, brk;
};

// Finalize modes (the values of the library's FinalMode).
constexpr int kModeStart = 0, kModeAlpha = 1, kModeBeta = 2, kModeRefresh = 4;

// Steps of the next launch of a period of N steps at K steps per launch, n0 steps done: the
// remainder N mod K first, as descending powers of two, then launches of K.  Launch counts
// and step counts of every launch are then one of K, 4, 2, 1.
CMCG_HD inline int launch_steps(int N, int K, int n0) {
  const int r = N % K;
  if (n0 < r) {
    int p = 1;
    while (2 * p <= r - n0) p *= 2;
    return p;
  }
  return K;
}

CMCG_HD inline bool is_period(int phase) {
  return phase == kGradFwd || phase == kGradAdj || phase == kFwd || phase == kAdj ||
         phase == kFilter;
}

// Steps per launch of the period of `phase`.
CMCG_HD inline int period_K(const Params &P, int phase) {
  if (phase == kFilter) return 1;
  if (phase == kGradFwd || phase == kGradAdj) return P.K_hi;
  return P.K_lo;
}

// The operation of this round (after any decision the phase called for).  `sc` holds the
// solve's scalars as the last finalize left them.
CMCG_HD inline int decide(const Params &P, State &S, const Scalars &sc) {
  if (S.phase == kGradDecide) {
    if (sc.brk != 0.0) {
      S.phase = kFailed;
      S.active = 3;
      S.status = -5;   // CMCG_EBREAKDOWN
      return S.phase;
    }
    S.delta_at_refresh = sc.delta;
    if (S.grad_mode == kModeStart) {
      // Step 4: d = r; a start already at the tolerance (or a zero gradient) is converged
      if (sc.rel <= P.tol || sc.delta0 == 0.0) {
        S.converged = 1;
        S.phase = kFiltZero;
      } else {
        S.phase = kInitD;
      }
    } else {
      ++S.refreshes;
      if (sc.rel <= P.tol) {
        S.converged = 1;
        S.phase = kFiltZero;
      } else if (S.iter >= P.max_iter) {
        S.phase = kFiltZero;
      } else {
        S.phase = kDir;
      }
    }
  } else if (S.phase == kItDecide) {
    ++S.iter;
    if (sc.brk != 0.0) {
      S.phase = kFailed;
      S.active = 3;
      S.status = -5;
      return S.phase;
    }
    if (P.mixed && P.refresh > 0.0 &&
        (sc.rel <= P.tol || sc.delta <= P.refresh * P.refresh * S.delta_at_refresh)) {
      // reliable update: the true gradient at the FP64 iterate replaces the residual
      S.grad_mode = kModeRefresh;
      S.phase = kGradFwd;
    } else if (sc.rel <= P.tol) {
      S.converged = 1;
      S.phase = kFiltZero;
    } else if (S.iter >= P.max_iter) {
      S.phase = kFiltZero;
    } else {
      S.phase = kDir;
    }
  }
  return S.phase;
}

// The phase that follows a completed one-round phase or a completed period.
CMCG_HD inline int next_phase(int phase) {
  switch (phase) {
    case kGradFwd: return kGradAdj;
    case kGradAdj: return kGradCopy;
    case kGradCopy: return kGradDot;
    case kGradDot: return kGradFin;
    case kGradFin: return kGradDecide;
    case kInitD: return kFwd;
    case kFwd: return kAdj;
    case kAdj: return kItDot;
    case kItDot: return kItFinA;
    case kItFinA: return kItUpd;
    case kItUpd: return kItFinB;
    case kItFinB: return kItDecide;
    case kDir: return kFwd;
    case kFiltZero: return kFilter;
    case kFilter: return kOutput;
    case kOutput: return kDone;
    default: return phase;
  }
}

CMCG_HD inline int op_of(int phase) {
  switch (phase) {
    case kGradFwd: case kGradAdj: case kFwd: case kAdj: case kFilter: return kOpPeriod;
    case kGradCopy: return kOpCopy;
    case kGradDot: return kOpDotGrad;
    case kGradFin: case kItFinA: case kItFinB: return kOpFinalize;
    case kInitD: return kOpConvert;
    case kItDot: return kOpDotIt;
    case kItUpd: return kOpUpdate;
    case kDir: return kOpDirection;
    case kFiltZero: return kOpZero;
    case kOutput: return kOpOutput;
    default: return kOpNone;
  }
}

CMCG_HD inline int finalize_mode(const State &S) {
  if (S.phase == kGradFin) return S.grad_mode;
  return S.phase == kItFinA ? kModeAlpha : kModeBeta;
}

// Advance past this round's operation (ns: the steps of its launch, for a period).
CMCG_HD inline void advance(const Params &P, State &S, int ns) {
  if (is_period(S.phase)) {
    S.n0 += ns;
    ++S.launch;
    if (S.n0 < P.N) return;
    S.n0 = 0;
    S.launch = 0;
  }
  S.phase = next_phase(S.phase);
  if (S.phase == kDone) S.active = 2;
}

}  // namespace serve
}  // namespace cmcg
