// CPU model of the persistent serving kernel's round logic (serve_plan.h) and of its bounded
// grid barrier.  Prints "ok" lines; any failed check aborts with a message.
//
// plan: a solve is driven round by round with scripted scalars; the periods' launches must
// cover each period's N steps exactly (remainder first, in powers of two, then K), carry the
// opening flag on the first launch and the closing one on the last, alternate the two work
// buffers, and the CG phases must follow the single-solve order (gradient, iterations, FP64
// refreshes in FP32-mixed mode, the stop at max_iter after a refresh, the filter).
// barrier: T threads run R rounds through a generation barrier with the kernel's algorithm;
// no thread may start round r + 1 before every thread finished round r; with a spin limit of
// one poll every thread must leave (the give-up path).
#include <atomic>
#include <chrono>
#include <cmath>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "../../paper_1903_12522_amd/csrc/serve_plan.h"

using namespace cmcg::serve;

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      std::exit(1);                                                     \
    }                                                                   \
  } while (0)

// One period: the launches the planner issues from phase `ph`.
static void check_period(const Params &P, State &S, int ph) {
  CHECK(S.phase == ph && S.n0 == 0 && S.launch == 0);
  const int K = period_K(P, ph);
  int steps = 0, launches = 0;
  while (S.phase == ph) {
    const int ns = launch_steps(P.N, K, S.n0);
    CHECK(ns == K || (ns < K && (ns & (ns - 1)) == 0));      // K or a power of two below it
    CHECK(S.launch == launches);                              // buffer ping-pong index
    const bool first = S.n0 == 0, last = S.n0 + ns == P.N;
    CHECK(first == (launches == 0));
    if (ns < K) CHECK(S.n0 < P.N % K);                        // the remainder comes first
    steps += ns;
    ++launches;
    advance(P, S, ns);
    if (last) CHECK(S.phase != ph || P.N == 0);
  }
  CHECK(steps == P.N);
}

static int run_solve(const Params &P, const std::vector<double> &rels, int *refreshes,
                     bool *converged) {
  State S{};
  S.active = 1;
  S.phase = kGradFwd;
  S.grad_mode = kModeStart;
  double delta0 = 1.0, delta = 1.0;
  size_t k = 0;
  int guard = 0;
  while (S.active == 1 && ++guard < 1000000) {
    if (S.phase == kGradDecide || S.phase == kItDecide) {
      Scalars sc{delta, delta0, delta <= 0 ? 0 : 1.0, 0.0};
      sc.rel = std::sqrt(delta / delta0);
      decide(P, S, sc);
      continue;
    }
    const int op = op_of(S.phase);
    CHECK(op != kOpNone);
    if (op == kOpPeriod) {
      check_period(P, S, S.phase);
      continue;
    }
    if (op == kOpFinalize) {
      const int mode = finalize_mode(S);
      if (S.phase == kGradFin) {
        CHECK(mode == S.grad_mode);
        if (mode == kModeStart) delta = delta0 = 1.0;
        else {
          // the true gradient at the current iterate: the last recursive residual
          const double r = rels.at(std::min(k > 0 ? k - 1 : 0, rels.size() - 1));
          delta = r * r;
        }
      } else if (S.phase == kItFinA) {
        CHECK(mode == kModeAlpha);
      } else {
        CHECK(mode == kModeBeta);
        const double r = rels.at(std::min(k++, rels.size() - 1));
        delta = r * r;
      }
    }
    advance(P, S, 0);
  }
  CHECK(S.active == 2);
  *refreshes = S.refreshes;
  *converged = S.converged != 0;
  return S.iter;
}

static void model_plan() {
  // launch splits: every (N, K) covers N exactly
  for (int K : {1, 2, 4, 7})
    for (int N = 3; N < 300; ++N) {
      Params P{N, K, 4, 1, 10, 1e-6, 0.1};
      State S{};
      S.active = 1;
      S.phase = kFwd;
      check_period(P, S, kFwd);
    }
  // FP64: residual falls by 0.5 per iteration, no refreshes, converges at 2^-20 < 1e-6
  {
    std::vector<double> rels;
    for (int i = 1; i <= 40; ++i) rels.push_back(std::pow(0.5, i));
    Params P{164, 4, 4, 0, 1000, 1e-6, 0.1};
    int refr = 0;
    bool conv = false;
    const int it = run_solve(P, rels, &refr, &conv);
    CHECK(conv && it == 20 && refr == 0);
  }
  // FP32-mixed: a refresh whenever delta fell by 100 (refresh 0.1), i.e. every 4 iterations,
  // the last one confirming convergence at iteration 20
  {
    std::vector<double> rels;
    for (int i = 1; i <= 40; ++i) rels.push_back(std::pow(0.5, i));
    Params P{164, 7, 4, 1, 1000, 1e-6, 0.1};
    int refr = 0;
    bool conv = false;
    const int it = run_solve(P, rels, &refr, &conv);
    CHECK(conv && it == 20 && refr == 5);
  }
  // FP32-mixed with a refresh on every iteration and max_iter 6: stops at 6, not converged
  {
    std::vector<double> rels;
    for (int i = 1; i <= 40; ++i) rels.push_back(0.9 * std::pow(0.99, i));
    Params P{30, 7, 4, 1, 6, 1e-12, 0.9999};
    int refr = 0;
    bool conv = false;
    const int it = run_solve(P, rels, &refr, &conv);
    CHECK(!conv && it == 6 && refr == 6);
  }
  std::printf("ok plan\n");
}

// The kernel's barrier: read the generation, arrive; the last arrival resets the count and
// advances the generation; the others poll the generation with a bounded wait.
struct Ctl {
  std::atomic<unsigned> count{0}, gen{0};
  std::atomic<int> failed{0};
};

static bool grid_sync(Ctl &c, unsigned nblocks, unsigned long long spin_limit) {
  const unsigned g0 = c.gen.load(std::memory_order_relaxed);
  const unsigned arrived = c.count.fetch_add(1, std::memory_order_release) + 1;
  if (arrived == nblocks) {
    std::atomic_thread_fence(std::memory_order_acquire);
    c.count.store(0, std::memory_order_relaxed);
    c.gen.fetch_add(1, std::memory_order_release);
    return true;
  }
  unsigned long long spins = 0;
  while (c.gen.load(std::memory_order_relaxed) == g0) {
    if (++spins > spin_limit || c.failed.load(std::memory_order_relaxed)) {
      c.failed.store(1, std::memory_order_relaxed);
      return false;
    }
    std::this_thread::yield();
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return true;
}

static void model_barrier() {
  const int T = 16, R = 2000;
  Ctl c;
  std::vector<std::atomic<int>> done(R);
  for (auto &d : done) d.store(0);
  std::vector<std::thread> th;
  std::atomic<int> bad{0};
  for (int t = 0; t < T; ++t)
    th.emplace_back([&, t] {
      for (int r = 0; r < R; ++r) {
        if (r > 0 && done[r - 1].load() != T) bad.fetch_add(1);   // a round started early
        done[r].fetch_add(1);
        if (!grid_sync(c, T, 1ull << 40)) {
          bad.fetch_add(1000);
          return;
        }
      }
      (void)t;
    });
  for (auto &x : th) x.join();
  CHECK(bad.load() == 0 && c.count.load() == 0 && c.gen.load() == (unsigned)R);
  // give-up path: a spin limit of one poll; every thread must leave
  Ctl c2;
  std::atomic<int> left{0};
  std::vector<std::thread> th2;
  for (int t = 0; t < T; ++t)
    th2.emplace_back([&, t] {
      for (int r = 0; r < R; ++r) {
        if (t == 0 && r == 5) std::this_thread::sleep_for(std::chrono::milliseconds(20));
        if (!grid_sync(c2, T, 1)) break;
      }
      left.fetch_add(1);
    });
  for (auto &x : th2) x.join();
  CHECK(left.load() == T && c2.failed.load() == 1);
  std::printf("ok barrier\n");
}

int main() {
  model_plan();
  model_barrier();
  return 0;
}
