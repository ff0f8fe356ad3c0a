// On-device FP64 L-BFGS over the initial momentum p0 (paper Sec. 2.1 and
// Alg. 1, steps (e)-(f): line-search evaluations and quasi-Newton updates
// repeated until convergence or an iteration cap).
//
// The paper runs VNL's L-BFGS on the host and pays one host/device round
// trip per evaluation.  Here the optimiser lives on the GPU: after every
// loss+gradient evaluation one workgroup advances a line-search state
// machine and, on acceptance, updates the curvature history and computes the
// next direction by the two-loop recursion.  The host only launches
// evaluations and polls a done flag; there is no synchronisation inside an
// iteration.
//
// Algorithm (Nocedal & Wright, Numerical Optimization, Algs. 3.5, 3.6, 7.4):
//  * direction d = -H g by the two-loop recursion over the m newest pairs
//    (s, y), scaled by gamma = s.y / y.y of the newest pair; steepest descent
//    (and a cleared history) when d is not a descent direction;
//  * first trial step 1/|d| with an empty history, else 1;
//  * strong-Wolfe search, c1 = 1e-4, c2 = 0.9: steps double until the
//    bracket closes, then a zoom with the safeguarded cubic minimiser
//    (midpoint when the cubic is unusable), at most max_fev evaluations;
//  * a pair is stored only when s.y > 0 and s.y > 1e-16 y.y;
//  * stop: |g| <= gtol max(1, |x|) (converged), relative decrease below
//    ftol_rel (converged), max_iter accepted steps, or a failed line search
//    (not converged; x stays the last accepted point).
// Every dot product is a fixed-order tree over one workgroup, so the state
// machine takes the same decisions on every run.
#include "lbfgs_internal.h"

#include <cmath>

namespace lddmm {

namespace {

constexpr int kThreads = 1024;

enum Phase : int { kInit = 0, kBracket = 1, kZoom = 2 };

// Block-wide sums of per-thread partials in a fixed order: a butterfly within
// each wave (lane 0's total is used), then the waves' totals in wave order.
// Two barriers per call.
__device__ __forceinline__ double block_sum(double s, double* red) {
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < kThreads / 64; ++w) r += red[w];
  __syncthreads();   // red is reused by the next reduction
  return r;
}

// Two sums in one pass of barriers; each is summed exactly as block_sum would.
__device__ __forceinline__ void block_sum2(double s, double t, double* red, double* rs,
                                           double* rt) {
  constexpr int NW = kThreads / 64;
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    t += __shfl_xor(t, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = s;
    red[NW + (threadIdx.x >> 6)] = t;
  }
  __syncthreads();
  double a = red[0], b = red[NW];
  for (int w = 1; w < NW; ++w) {
    a += red[w];
    b += red[NW + w];
  }
  __syncthreads();
  *rs = a;
  *rt = b;
}

// Each thread owns elements k = threadIdx.x + j kThreads of every vector and
// sums its products in increasing k, so fusing passes below changes no bit.
// A pass visits the thread's elements in that order, kBatch at a time: the
// loads of a batch (NV source vectors) are all issued before the first of its
// elements is used.  One workgroup serves a whole problem, so a pass that waited
// for each element's loads in turn would take one memory latency per element.
// Only the thread's own elements are read and written, so reading a batch ahead
// of the batch's stores changes nothing.
constexpr int kBatch = 8;

template <int NV, typename F>
__device__ __forceinline__ void own_elems(int m, const double* const (&src)[NV], F&& f) {
  for (int k0 = threadIdx.x; k0 < m; k0 += kBatch * kThreads) {
    double v[kBatch][NV];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int k = k0 + u * kThreads;
#pragma unroll
      for (int c = 0; c < NV; ++c) v[u][c] = k < m ? src[c][k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int k = k0 + u * kThreads;
      if (k < m) f(k, v[u]);
    }
  }
}

__device__ __forceinline__ double block_dot(const double* __restrict__ a,
                                            const double* __restrict__ b, int m, double* red) {
  double s = 0.0;
  const double* src[2] = {a, b};
  own_elems<2>(m, src, [&](int, const double* v) { s += v[0] * v[1]; });
  return block_sum(s, red);
}

// x_t = x + a d without FMA contraction (the same rounding as x + a*d on a host)
__device__ __forceinline__ void trial_point(const LbfgsBufs& B, double a) {
  const double* src[2] = {B.x, B.d};
  own_elems<2>(B.m3, src,
               [&](int k, const double* v) { B.xt[k] = __dadd_rn(v[0], __dmul_rn(a, v[1])); });
}

// Safeguarded cubic step between (a0,f0,d0) and (a1,f1,d1).
__device__ double cubic_step(double a0, double f0, double d0, double a1, double f1, double d1) {
  const double lo = a0 < a1 ? a0 : a1, hi = a0 < a1 ? a1 : a0, w = hi - lo;
  const double mid = 0.5 * (a0 + a1);
  const double t1 = d0 + d1 - 3.0 * (f0 - f1) / (a0 - a1);
  const double disc = t1 * t1 - d0 * d1;
  if (!(disc >= 0.0)) return mid;
  double t2 = sqrt(disc);
  if (a1 < a0) t2 = -t2;
  const double den = d1 - d0 + 2.0 * t2;
  const double a = a1 - (a1 - a0) * ((d1 + t2 - t1) / den);
  if (!isfinite(a) || a < lo + 0.1 * w || a > hi - 0.1 * w) return mid;
  return a;
}

// Keep q(1) and {L, H0, mismatch} of the point just accepted, so a finished
// job reports them without another evaluation.
__device__ __forceinline__ void snapshot(const LbfgsBufs& B) {
  if (!B.q1t) return;
  const double* src[1] = {B.q1t};
  own_elems<1>(B.m3, src, [&](int k, const double* v) { B.q1a[k] = v[0]; });
  if (threadIdx.x < 3) B.out3a[threadIdx.x] = B.ft[threadIdx.x];
}

// New search direction from g and the history; sets d0, the first trial step
// and x_t.  Called by every thread; st is the workgroup's shared copy of the
// state, read by all threads and written by thread 0 only, between barriers.
__device__ void new_direction(const LbfgsBufs& B, const LbfgsOpts& o, LbfgsState& st,
                              double* red) {
  // Two-loop recursion (Nocedal & Wright, Alg. 7.4).  Every thread updates
  // only its own elements of d, so each update is fused with the inner
  // product the next step needs: one vector pass per history entry instead of
  // two, the same arithmetic in the same order.
  const int m3 = B.m3, M = o.m;
  const int used = st.used, newest = st.newest;
  const auto slot = [&](int h) { return (newest - h + M) % M; };   // h = 0: newest
  const auto Sv = [&](int h) { return B.S + (size_t)slot(h) * m3; };
  const auto Yv = [&](int h) { return B.Y + (size_t)slot(h) * m3; };
  double gd, dd = 0.0;
  if (used == 0) {                               // steepest descent: d = -g
    double a = 0.0, b = 0.0;
    const double* src[1] = {B.g};
    own_elems<1>(m3, src, [&](int k, const double* g) {
      const double v = -g[0];
      B.d[k] = v;
      a += g[0] * v;
      b += v * v;
    });
    block_sum2(a, b, red, &gd, &dd);
  } else {
    double sy, yy;                               // H0 scaling from the newest pair
    {
      const double* Sn = Sv(0);
      const double* Yn = Yv(0);
      double a = 0.0, b = 0.0;
      const double* src[2] = {Sn, Yn};
      own_elems<2>(m3, src, [&](int, const double* v) {
        a += v[0] * v[1];
        b += v[1] * v[1];
      });
      block_sum2(a, b, red, &sy, &yy);
    }
    const double gamma = sy / yy;
    double acc = 0.0;                            // d = g, and S_0 . d
    {
      const double* src[2] = {B.g, Sv(0)};
      own_elems<2>(m3, src, [&](int k, const double* v) {
        B.d[k] = v[0];
        acc += v[1] * v[0];
      });
    }
    for (int h = 0; h < used; ++h) {             // newest to oldest
      const double al = st.rho[slot(h)] * block_sum(acc, red);
      if (threadIdx.x == 0) st.alpha[slot(h)] = al;
      const double* Ys = Yv(h);
      const bool last = h + 1 == used;
      const double* Nx = last ? Yv(used - 1) : Sv(h + 1);   // the next inner product's vector
      acc = 0.0;
      const double* src[3] = {B.d, Ys, Nx};
      own_elems<3>(m3, src, [&](int k, const double* w) {
        double v = w[0] - al * w[1];
        if (last) v *= gamma;
        B.d[k] = v;
        acc += w[2] * v;
      });
    }
    for (int h = used - 1; h >= 0; --h) {         // oldest to newest
      const double beta = st.rho[slot(h)] * block_sum(acc, red);
      const double al = st.alpha[slot(h)];
      const double* Ss = Sv(h);
      const bool last = h == 0;
      const double* Nx = last ? B.g : Yv(h - 1);
      acc = 0.0;
      const double* src[3] = {B.d, Ss, Nx};
      own_elems<3>(m3, src, [&](int k, const double* w) {
        double v = w[0] + (al - beta) * w[1];
        if (last) v = -v;                        // the direction is -H g
        B.d[k] = v;
        acc += w[2] * v;
      });
    }
    gd = block_sum(acc, red);
  }
  const bool restart = !(gd < 0.0);             // not a descent direction: restart
  if (restart) {
    double a = 0.0, b = 0.0;
    const double* src[1] = {B.g};
    own_elems<1>(m3, src, [&](int k, const double* g) {
      const double v = -g[0];
      B.d[k] = v;
      a += g[0] * v;
      b += v * v;
    });
    block_sum2(a, b, red, &gd, &dd);
  }
  const double a0 = (restart || used == 0) ? 1.0 / sqrt(dd) : 1.0;
  if (threadIdx.x == 0) {
    if (restart) { st.used = 0; st.newest = -1; }
    st.d0 = gd;
    st.a = a0;
    st.phase = kBracket;
    st.fev = 0;
    st.bi = 1;
    st.a_prev = 0.0;
    st.f_prev = st.f;
    st.dp_prev = gd;
  }
  trial_point(B, a0);
  __syncthreads();
}

// Accepted step: curvature pair, move to x_t, convergence tests, next direction.
__device__ void accept(const LbfgsBufs& B, const LbfgsOpts& o, LbfgsState& st, double ft,
                       double* red) {
  const int m3 = B.m3, M = o.m;
  const int slot = (st.newest + 1) % M;
  const double f_old = st.f;
  double* Ss = B.S + (size_t)slot * m3;
  double* Ys = B.Y + (size_t)slot * m3;
  double a = 0.0, b = 0.0, gg = 0.0, xx = 0.0;
  const double* src[4] = {B.xt, B.x, B.gt, B.g};
  own_elems<4>(m3, src, [&](int k, const double* v) {   // new pair; x, g move to x_t, g_t
    const double sv = v[0] - v[1];
    const double yv = v[2] - v[3];
    Ss[k] = sv;
    Ys[k] = yv;
    a += sv * yv;
    b += yv * yv;
    const double xv = v[0], gv = v[2];
    B.x[k] = xv;
    B.g[k] = gv;
    gg += gv * gv;
    xx += xv * xv;
  });
  snapshot(B);
  double sy, yy, gsq, xsq;
  block_sum2(a, b, red, &sy, &yy);
  block_sum2(gg, xx, red, &gsq, &xsq);
  const double gnorm = sqrt(gsq);
  const double xnorm = sqrt(xsq);
  if (threadIdx.x == 0) {
    if (sy > 1e-16 * yy && sy > 0.0) {
      st.rho[slot] = 1.0 / sy;
      st.newest = slot;
      if (st.used < M) ++st.used;
    }
    st.f = ft;
    st.iters += 1;
    st.gnorm = gnorm;
    if (B.trace && st.iters <= o.max_iter) {
      B.trace[2 * st.iters] = st.f;
      B.trace[2 * st.iters + 1] = st.gnorm;
    }
    if (gnorm <= o.gtol * fmax(1.0, xnorm)) {
      st.done = 1; st.status = kConverged;
    } else if (o.ftol_rel > 0.0 &&
               f_old - ft <= o.ftol_rel * fmax(fmax(fabs(f_old), fabs(ft)), 1.0)) {
      st.done = 1; st.status = kConverged;
    } else if (st.iters >= o.max_iter) {
      st.done = 1; st.status = kNotConverged;
    }
  }
  __syncthreads();
  if (!st.done) new_direction(B, o, st, red);
}

}  // namespace

__global__ __launch_bounds__(kThreads) void k_lbfgs_init(LbfgsBufs B, LbfgsState* state,
                                                         int init, const double* __restrict__ q0,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ p_in,
                                                         double inv_T) {
  for (int k = threadIdx.x; k < B.m3; k += kThreads) {
    double v = 0.0;
    if (init == 1) v = (x[k] - q0[k]) * inv_T;
    else if (init == 2) v = p_in[k];
    B.x[k] = v;
    B.xt[k] = v;
  }
  if (threadIdx.x == 0) {
    LbfgsState s{};
    s.phase = kInit;
    s.newest = -1;
    s.status = kNotConverged;
    *state = s;
  }
}

// Consumes the evaluation at x_t (loss *B.ft, gradient B.gt) and prepares the
// next trial point, or sets done.  st and action live in LDS.
__device__ void step_body(const LbfgsBufs& B, LbfgsState* state, const LbfgsOpts& o,
                          double* red, LbfgsState& st, int& action) {
  // action: 0 accept, 1 new trial at st.a, 2 failed search
  if (threadIdx.x == 0) st = *state;
  __syncthreads();
  if (st.done) return;
  const double ft = *B.ft;
  const int m3 = B.m3;
  if (threadIdx.x == 0) st.fevals += 1;

  if (st.phase == kInit) {
    const double* src[1] = {B.gt};
    own_elems<1>(m3, src, [&](int k, const double* v) { B.g[k] = v[0]; });
    snapshot(B);
    __syncthreads();
    const double gg = block_dot(B.g, B.g, m3, red);
    const double xx = block_dot(B.x, B.x, m3, red);
    if (threadIdx.x == 0) {
      st.f = ft;
      st.gnorm = sqrt(gg);
      if (B.trace) { B.trace[0] = st.f; B.trace[1] = st.gnorm; }
      if (!isfinite(st.f) || !isfinite(st.gnorm)) { st.done = 1; st.status = kNonFinite; }
      else if (st.gnorm <= o.gtol * fmax(1.0, sqrt(xx))) { st.done = 1; st.status = kConverged; }
      else if (o.max_iter <= 0) { st.done = 1; st.status = kNotConverged; }
    }
    __syncthreads();
    if (!st.done) new_direction(B, o, st, red);
  } else {
    const double da = block_dot(B.gt, B.d, m3, red);
    if (threadIdx.x == 0) {
      const double a = st.a, f = st.f, d0 = st.d0;
      st.fev += 1;
      bool to_zoom = false;
      action = 1;
      if (st.phase == kBracket) {
        if (!isfinite(ft) || !isfinite(da) || ft > f + o.c1 * a * d0 ||
            (st.bi > 1 && ft >= st.f_prev)) {
          st.a_lo = st.a_prev; st.f_lo = st.f_prev; st.dp_lo = st.dp_prev;
          st.a_hi = a; st.f_hi = ft; st.dp_hi = da;
          to_zoom = true;
        } else if (fabs(da) <= -o.c2 * d0) {
          action = 0;
        } else if (da >= 0.0) {
          st.a_lo = a; st.f_lo = ft; st.dp_lo = da;
          st.a_hi = st.a_prev; st.f_hi = st.f_prev; st.dp_hi = st.dp_prev;
          to_zoom = true;
        } else {
          st.a_prev = a; st.f_prev = ft; st.dp_prev = da;
          st.a = 2.0 * a;
          st.bi += 1;
          if (st.fev >= o.max_fev) action = 2;
        }
      } else {   // zoom: the trial was a_j = st.a
        if (!isfinite(ft) || !isfinite(da) || ft > f + o.c1 * a * d0 || ft >= st.f_lo) {
          st.a_hi = a; st.f_hi = ft; st.dp_hi = da;
        } else if (fabs(da) <= -o.c2 * d0) {
          action = 0;
        } else {
          if (da * (st.a_hi - st.a_lo) >= 0.0) {
            st.a_hi = st.a_lo; st.f_hi = st.f_lo; st.dp_hi = st.dp_lo;
          }
          st.a_lo = a; st.f_lo = ft; st.dp_lo = da;
        }
        if (action == 1) to_zoom = true;
      }
      if (to_zoom) {
        st.phase = kZoom;
        if (st.fev >= o.max_fev ||
            fabs(st.a_hi - st.a_lo) <= 1e-14 * fabs(st.a_lo) + 1e-300) {
          action = 2;
        } else {
          st.a = (isfinite(st.f_hi) && isfinite(st.dp_hi))
                     ? cubic_step(st.a_lo, st.f_lo, st.dp_lo, st.a_hi, st.f_hi, st.dp_hi)
                     : 0.5 * (st.a_lo + st.a_hi);
        }
      }
      if (action == 2) { st.done = 1; st.status = kNotConverged; }
    }
    __syncthreads();
    if (action == 0) accept(B, o, st, ft, red);
    else if (action == 1) trial_point(B, st.a);
  }
  __syncthreads();
  if (threadIdx.x == 0) *state = st;
}

__global__ __launch_bounds__(kThreads) void k_lbfgs_step(LbfgsBufs B, LbfgsState* state,
                                                         LbfgsOpts o) {
  __shared__ double red[kThreads];
  __shared__ LbfgsState st;
  __shared__ int action;
  step_body(B, state, o, red, st, action);
}

__global__ __launch_bounds__(kThreads) void k_lbfgs_step_batch(const LbfgsJob* __restrict__ J) {
  __shared__ double red[kThreads];
  __shared__ LbfgsState st;
  __shared__ int action;
  const LbfgsJob& j = J[blockIdx.x];
  if (!j.active) return;
  step_body(j.B, j.state, j.o, red, st, action);
}

__global__ void k_gather_done(const LbfgsJob* __restrict__ J, int max_slots, int* __restrict__ done) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < max_slots) done[k] = J[k].active ? J[k].state->done : 0;
}

// Result of a finished solve: AverageDist / MaxDist of q(1) against x
// (Sec. 3.1) from the final evaluation, and the solver's counters.
__global__ __launch_bounds__(kThreads) void k_lbfgs_result(int n, const double* __restrict__ q1,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ out3,
                                                           const LbfgsState* __restrict__ state,
                                                           LbfgsResult* __restrict__ res) {
  __shared__ double red[kThreads];
  __shared__ double redm[kThreads];
  double s = 0.0, mx = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const double dx = q1[3 * i] - x[3 * i], dy = q1[3 * i + 1] - x[3 * i + 1],
                 dz = q1[3 * i + 2] - x[3 * i + 2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    s += r;
    mx = fmax(mx, r);
  }
  red[threadIdx.x] = s;
  redm[threadIdx.x] = mx;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[threadIdx.x] += red[threadIdx.x + off];
      redm[threadIdx.x] = fmax(redm[threadIdx.x], redm[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    res->loss = out3[0];
    res->H0 = out3[1];
    res->mismatch = out3[2];
    res->grad_norm = state->gnorm;
    res->avg_dist = red[0] / n;
    res->max_dist = redm[0];
    res->iters = state->iters;
    res->fevals = state->fevals;
    res->status = state->status;
    res->done = state->done;
  }
}

hipError_t launch_lbfgs_init(const LbfgsBufs& B, LbfgsState* state, int init, const double* q0,
                             const double* x, const double* p_in, int T, hipStream_t s) {
  k_lbfgs_init<<<1, kThreads, 0, s>>>(B, state, init, q0, x, p_in, 1.0 / T);
  return hipGetLastError();
}

hipError_t launch_lbfgs_step(const LbfgsBufs& B, LbfgsState* state, const LbfgsOpts& o,
                             hipStream_t s) {
  k_lbfgs_step<<<1, kThreads, 0, s>>>(B, state, o);
  return hipGetLastError();
}

hipError_t launch_lbfgs_step_batch(const LbfgsJob* jobs, int max_slots, hipStream_t s) {
  k_lbfgs_step_batch<<<max_slots, kThreads, 0, s>>>(jobs);
  return hipGetLastError();
}

hipError_t launch_gather_done(const LbfgsJob* jobs, int max_slots, int* done, hipStream_t s) {
  k_gather_done<<<(max_slots + 255) / 256, 256, 0, s>>>(jobs, max_slots, done);
  return hipGetLastError();
}

hipError_t launch_lbfgs_result(int n, const double* q1, const double* x, const double* out3,
                               const LbfgsState* state, LbfgsResult* res, hipStream_t s) {
  k_lbfgs_result<<<1, kThreads, 0, s>>>(n, q1, x, out3, state, res);
  return hipGetLastError();
}

}  // namespace lddmm
