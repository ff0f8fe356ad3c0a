// A C-ABI consumer: one loss+gradient evaluation and a short solve through
// liblddmm, with device memory from the HIP runtime, checked against the
// FP64 CPU oracle (test infrastructure, linked here only to check).
// Exit status 0 when every check passes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lddmm.h"

extern "C" int oracle_shoot_grad(int n, int T, double sigma, double lambda, const double* q0,
                                 const double* p0, const double* x, double* loss, double* grad,
                                 double* q1, double* terms, int compensated);

namespace {

// Seeded inputs: a 64-bit linear congruential generator mapped to [-1, 1).
struct Lcg {
  unsigned long long s;
  double next() {
    s = s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(s >> 11) / 4503599627370496.0 * 2.0 - 1.0;
  }
};

bool ok(hipError_t e, const char* what) {
  if (e != hipSuccess) std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
  return e == hipSuccess;
}

double rel(const std::vector<double>& a, const std::vector<double>& b) {
  double num = 0, den = 0;
  for (size_t k = 0; k < a.size(); ++k) {
    num += (a[k] - b[k]) * (a[k] - b[k]);
    den += b[k] * b[k];
  }
  return std::sqrt(num / den);
}

}  // namespace

int main() {
  const int n = 777, T = 8;
  const double sigma = 1.5, lambda = 1.0;
  const size_t bytes = 3 * (size_t)n * sizeof(double);
  Lcg rng{2024};
  std::vector<double> q0(3 * n), p0(3 * n), x(3 * n);
  for (int k = 0; k < 3 * n; ++k) {
    q0[k] = 3.0 * rng.next();
    p0[k] = 0.3 * rng.next();
    x[k] = q0[k] + 0.5 * rng.next();
  }
  double *dq0, *dp0, *dx, *dgrad, *dout3;
  if (!ok(hipMalloc(&dq0, bytes), "hipMalloc") || !ok(hipMalloc(&dp0, bytes), "hipMalloc") ||
      !ok(hipMalloc(&dx, bytes), "hipMalloc") || !ok(hipMalloc(&dgrad, bytes), "hipMalloc") ||
      !ok(hipMalloc(&dout3, 3 * sizeof(double)), "hipMalloc"))
    return 2;
  hipMemcpy(dq0, q0.data(), bytes, hipMemcpyHostToDevice);
  hipMemcpy(dp0, p0.data(), bytes, hipMemcpyHostToDevice);
  hipMemcpy(dx, x.data(), bytes, hipMemcpyHostToDevice);

  lddmm_ctx* ctx = nullptr;
  if (lddmm_ctx_create(0, 0, &ctx) != LDDMM_OK) {
    std::fprintf(stderr, "ctx: %s\n", lddmm_last_error(nullptr));
    return 2;
  }
  lddmm_params prm{};
  prm.n = n;
  prm.T = T;
  prm.sigma = sigma;
  prm.lambda = lambda;
  prm.precision = LDDMM_FP64;
  int failures = 0;

  // one evaluation against the oracle
  if (lddmm_shoot_grad(ctx, &prm, dq0, dp0, dx, dout3, dgrad, nullptr, nullptr) != LDDMM_OK) {
    std::fprintf(stderr, "shoot_grad: %s\n", lddmm_last_error(ctx));
    return 2;
  }
  std::vector<double> grad(3 * n), og(3 * n), oq1(3 * n);
  double out3[3], oloss = 0, terms[2];
  if (!ok(hipDeviceSynchronize(), "sync")) return 2;
  hipMemcpy(grad.data(), dgrad, bytes, hipMemcpyDeviceToHost);
  hipMemcpy(out3, dout3, sizeof out3, hipMemcpyDeviceToHost);
  oracle_shoot_grad(n, T, sigma, lambda, q0.data(), p0.data(), x.data(), &oloss, og.data(),
                    oq1.data(), terms, 0);
  const double eg = rel(grad, og), el = std::fabs(out3[0] - oloss) / std::fabs(oloss);
  std::printf("shoot_grad fp64: loss rel err %.2e, grad rel err %.2e\n", el, eg);
  failures += !(eg < 1e-12 && el < 1e-12);

  // a short solve from p0 = 0: status, and the loss decreases
  lddmm_solve_opts opts;
  lddmm_solve_opts_default(LDDMM_FP64, &opts);
  opts.max_iter = 25;
  lddmm_solve_result res{};
  const lddmm_status st = lddmm_solve(ctx, &prm, &opts, dq0, dx, dp0, &res, nullptr, nullptr);
  double l0 = 0;
  for (int k = 0; k < 3 * n; ++k) l0 += lambda * (q0[k] - x[k]) * (q0[k] - x[k]);
  std::printf("solve fp64: status %d, %d iterations, %d evaluations, loss %.6g (start %.6g)\n",
              (int)st, res.iters, res.fevals, res.loss, l0);
  failures += !((st == LDDMM_OK || st == LDDMM_ENOTCONV) && res.loss < l0 && res.iters > 0);

  // a rejected call leaves the context usable
  lddmm_params bad = prm;
  bad.sigma = -1.0;
  failures += lddmm_shoot_grad(ctx, &bad, dq0, dp0, dx, dout3, dgrad, nullptr, nullptr) !=
              LDDMM_EINVAL;
  failures += lddmm_ctx_check(ctx, nullptr) != LDDMM_OK;

  lddmm_ctx_destroy(ctx);
  hipFree(dq0);
  hipFree(dp0);
  hipFree(dx);
  hipFree(dgrad);
  hipFree(dout3);
  std::printf("%s\n", failures ? "FAILED" : "ok");
  return failures ? 1 : 0;
}
