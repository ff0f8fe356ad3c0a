// Internal interface of the on-device L-BFGS (lbfgs.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lddmm {

constexpr int kMaxHistory = 16;

enum SolveStatus : int { kConverged = 0, kNotConverged = 1, kNonFinite = -4 };

struct LbfgsOpts {
  int max_iter, m, max_fev;
  double gtol, ftol_rel, c1, c2;
};

// Device-resident optimiser state (one per problem).
struct LbfgsState {
  double f, gnorm, d0, a;                  // accepted loss, |g|, g.d, current trial step
  double a_prev, f_prev, dp_prev;          // previous bracketing trial
  double a_lo, f_lo, dp_lo, a_hi, f_hi, dp_hi;
  double rho[kMaxHistory], alpha[kMaxHistory];
  int phase, fev, bi;                      // search phase, evaluations in it, bracket step
  int iters, fevals, status, done;
  int used, newest;                        // curvature pairs held, newest slot
};

// Device buffers of one problem: vectors of m3 = 3N doubles.
struct LbfgsBufs {
  int m3;
  double *x, *g, *d, *xt, *gt;             // iterate, gradient, direction, trial point and its gradient
  double *S, *Y;                           // [m][m3] curvature pairs
  const double* ft;                        // {L, H0, mismatch} at the trial point (device)
  double* trace;                           // optional [max_iter+1][2] (loss, |g|) per accepted step
  const double* q1t;                       // optional: q(1) at the trial point, [m3]
  double* q1a;                             // with q1t: q(1) at the accepted point
  double* out3a;                           // with q1t: {L, H0, mismatch} at the accepted point
};

// One job of a batched optimiser step.
struct LbfgsJob {
  int active;
  LbfgsBufs B;
  LbfgsState* state;
  LbfgsOpts o;
};

struct LbfgsResult {
  double loss, H0, mismatch, grad_norm, avg_dist, max_dist;
  int32_t iters, fevals, status, done;
};

hipError_t launch_lbfgs_init(const LbfgsBufs& B, LbfgsState* state, int init, const double* q0,
                             const double* x, const double* p_in, int T, hipStream_t s);
hipError_t launch_lbfgs_step(const LbfgsBufs& B, LbfgsState* state, const LbfgsOpts& o,
                             hipStream_t s);
// One workgroup per slot; inactive slots return at once.
hipError_t launch_lbfgs_step_batch(const LbfgsJob* jobs, int max_slots, hipStream_t s);
// done[k] = the optimiser of slot k has finished (0 for empty slots).
hipError_t launch_gather_done(const LbfgsJob* jobs, int max_slots, int* done, hipStream_t s);
hipError_t launch_lbfgs_result(int n, const double* q1, const double* x, const double* out3,
                               const LbfgsState* state, LbfgsResult* res, hipStream_t s);

}  // namespace lddmm
