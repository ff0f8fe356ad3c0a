// CPU test of the launch plans of the pair kernels and of the workspace
// layout (plan.h): every size the library accepts up to 2^18 landmarks, every
// precision mode and kind of step.  No GPU involved; built with the address
// and undefined-behaviour sanitizers by the test-suite.
#include "plan.h"

#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(c, n)                                                                  \
  do {                                                                               \
    if (!(c)) {                                                                      \
      std::printf("FAIL n=%d line %d: %s\n", (int)(n), __LINE__, #c);                \
      std::exit(1);                                                                  \
    }                                                                                \
  } while (0)

namespace {

bool width_ok(int w) { return w == 1 || w == 2 || w == 4 || w == 8 || w == 12 || w == 16; }

// The decomposition the kernels assume: S chunks of `chunk` j cover [0, n)
// with none empty; the waves' ranges cover every chunk; grids fit int.
void check_plan(const lddmm::Plan& p, int n) {
  CHECK(p.n == n && p.nb == (n + 63) / 64, n);
  CHECK(p.S >= 1 && width_ok(p.W) && width_ok(p.Wa), n);
  CHECK((long long)p.S * p.chunk >= n && (long long)(p.S - 1) * p.chunk < n, n);
  CHECK((long long)p.W * p.wchunk >= p.chunk && (long long)p.Wa * p.wchunk_a >= p.chunk, n);
  CHECK(p.wchunk >= 1 && p.wchunk_a >= 1, n);
  CHECK((long long)p.nb * p.S < (1LL << 31), n);
  // at least 16 pairs per wave before widening; widened plans keep >= 4
  CHECK(p.wchunk >= 4 || n < 64 || p.W <= 8, n);
  // the 8 x 2 plans of small N are never widened
  if (p.S == 2 && p.chunk <= 240) CHECK(p.W <= 8 && p.Wa <= 8, n);
}

void check_layout(const lddmm_params& prm, const lddmm::Plan& p) {
  const lddmm::Layout L = lddmm::make_layout(prm, p);
  const size_t offs[] = {L.st, L.ad, L.hp0, L.hq0, L.xc, L.cen, L.h0p, L.out3, L.traj,
                         L.arec, L.ckpt, L.partial, L.hpT, L.hqT, L.hTp, L.stT, L.recT,
                         L.rk_acc, L.rk_lam, L.total};
  for (size_t k = 0; k + 1 < sizeof offs / sizeof offs[0]; ++k) {
    CHECK(offs[k] % 256 == 0, prm.n);
    CHECK(offs[k] <= offs[k + 1], prm.n);   // in order, so no two buffers overlap
  }
  const size_t n = (size_t)prm.n, rb = lddmm::rec_bytes(prm.precision);
  CHECK(L.ad - L.st >= 48 * n && L.arec - L.traj >= (size_t)L.slots * n * rb, prm.n);
  if (p.S > 1) CHECK(L.hpT - L.partial >= (size_t)p.S * 9 * n * lddmm::acc_bytes(prm.precision), prm.n);
}

}  // namespace

int main() {
  std::vector<int> sizes;
  for (int n = 1; n <= 70000; ++n) sizes.push_back(n);
  for (int n = 70001; n <= (1 << 18); n += 997) sizes.push_back(n);
  sizes.push_back(1 << 18);
  long checked = 0;
  for (int n : sizes)
    for (int mode = 0; mode <= 2; ++mode)
      for (int rk = 0; rk <= 1; ++rk) {
        lddmm::Plan p = lddmm::make_plan(n, 16384);
        lddmm::widen_plan(p, mode, rk != 0);
        check_plan(p, n);
        if (n % 61 == 0 || n < 300) {
          lddmm_params prm{};
          prm.n = n; prm.T = 7; prm.sigma = 1.0; prm.lambda = 1.0; prm.precision = mode;
          prm.ckpt_every = (n % 3 == 0) ? 3 : 0; prm.energy = n % 2; prm.integrator = rk;
          check_layout(prm, p);
        }
        ++checked;
      }
  std::printf("plans ok (%ld checked)\n", checked);
  return 0;
}
