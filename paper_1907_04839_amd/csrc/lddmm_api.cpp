// C ABI of liblddmm: validation, context and workspace, and the host-side
// order of kernel launches for one forward pass, the loss, and one adjoint
// pass (Alg. 1, ComputeGradient), optionally with checkpoint recompute.
#include "lddmm.h"
#include "lbfgs_internal.h"
#include "shoot_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace lddmm;

namespace {

// Event pairs bracketing pair-kernel launches (benchmark timing).
struct Timer {
  struct Rec { hipEvent_t ev[2]; int kind; };
  bool on = false;
  std::vector<Rec> pending, spare;
  double ms[3] = {0.0, 0.0, 0.0};       // kind 0: forward, 1: adjoint, 2: point flow
  int64_t count[3] = {0, 0, 0};

  // Events for the next launch of `kind`, or null when timing is off.
  hipEvent_t* take(int kind) {
    if (!on) return nullptr;
    Rec r{};
    if (!spare.empty()) {
      r = spare.back();
      spare.pop_back();
    } else if (hipEventCreate(&r.ev[0]) != hipSuccess || hipEventCreate(&r.ev[1]) != hipSuccess) {
      return nullptr;
    }
    r.kind = kind;
    pending.push_back(r);
    return pending.back().ev;
  }

  hipError_t collect() {
    for (Rec& r : pending) {
      hipError_t e = hipEventSynchronize(r.ev[1]);
      if (e != hipSuccess) return e;
      float t = 0.0f;
      e = hipEventElapsedTime(&t, r.ev[0], r.ev[1]);
      if (e != hipSuccess) return e;
      ms[r.kind] += t;
      count[r.kind] += 1;
      spare.push_back(r);
    }
    pending.clear();
    return hipSuccess;
  }

  void destroy() {
    for (auto* v : {&pending, &spare})
      for (Rec& r : *v) { (void)hipEventDestroy(r.ev[0]); (void)hipEventDestroy(r.ev[1]); }
    pending.clear();
    spare.clear();
  }
};

}  // namespace

struct lddmm_ctx {
  int device = 0;
  size_t budget = 0;         // cap on ws_bytes + sws_bytes (0: none)
  void* ws = nullptr;        // workspace
  size_t ws_bytes = 0;
  int* flag = nullptr;       // device non-finite flag
  Timer timer;
  void* sws = nullptr;       // solver workspace
  size_t sws_bytes = 0;
  int* host_done = nullptr;  // pinned: two done flags of the solver poll
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  void* scratch = nullptr;   // the device's fixed scratch (lddmm_shoot_grad_noalloc)
  std::string err;
};

namespace {

thread_local std::string g_err;   // errors that have no context

// Size limits.  Landmark arrays are indexed with 32-bit ints in the kernels
// (6 n fits), point arrays of the flow with 64-bit offsets; T + 1 trajectory
// slots must not overflow either.
constexpr int kMaxLandmarks = 1 << 26;
constexpr int kMaxSteps = 1 << 20;
constexpr int kMaxPoints = 1 << 30;

// Waves the pair kernels aim to have in a launch (256 CUs x 4 SIMDs x 16,
// queued as resources free up); LDDMM_TARGET_WAVES overrides it for tuning.
int target_waves() {
  static const int v = [] {
    const char* e = std::getenv("LDDMM_TARGET_WAVES");
    const int t = e ? std::atoi(e) : 0;
    return t > 0 ? t : 16384;
  }();
  return v;
}

// Tuning runs that set the plan through the environment get that plan as is.
bool plan_overridden() {
  static const bool v = std::getenv("LDDMM_TARGET_WAVES") || std::getenv("LDDMM_MAX_WG_WAVES");
  return v;
}

lddmm_status fail(lddmm_ctx* ctx, lddmm_status st, const char* fmt, ...)
    __attribute__((format(printf, 3, 4)));

lddmm_status fail(lddmm_ctx* ctx, lddmm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  (ctx ? ctx->err : g_err) = buf;
  return st;
}

lddmm_status hip_fail(lddmm_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, LDDMM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr, what)                       \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

lddmm_status check_params(lddmm_ctx* ctx, const lddmm_params* p) {
  if (!p) return fail(ctx, LDDMM_EINVAL, "params is NULL");
  if (p->n < 1) return fail(ctx, LDDMM_EINVAL, "n must be >= 1 (got %d)", p->n);
  if (p->n > kMaxLandmarks) return fail(ctx, LDDMM_EINVAL, "n too large (%d)", p->n);
  if (p->T < 1 || p->T > kMaxSteps)
    return fail(ctx, LDDMM_EINVAL, "T must be in 1..%d (got %d)", kMaxSteps, p->T);
  if (!(p->sigma > 0.0) || !std::isfinite(p->sigma))
    return fail(ctx, LDDMM_EINVAL, "sigma must be finite and > 0");
  if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda))
    return fail(ctx, LDDMM_EINVAL, "lambda must be finite and >= 0");
  if (p->precision < LDDMM_FP32 || p->precision > LDDMM_FP64)
    return fail(ctx, LDDMM_EINVAL, "unknown precision %d", p->precision);
  if (p->ckpt_every < 0) return fail(ctx, LDDMM_EINVAL, "ckpt_every must be >= 0");
  if (p->energy != LDDMM_ENERGY_INITIAL && p->energy != LDDMM_ENERGY_FINAL)
    return fail(ctx, LDDMM_EINVAL, "unknown energy term %d", p->energy);
  if (p->dim != 0 && p->dim != 2 && p->dim != 3)
    return fail(ctx, LDDMM_EINVAL, "dim must be 2 or 3 (got %d)", p->dim);
  if (p->integrator != LDDMM_EULER && p->integrator != LDDMM_RK4)
    return fail(ctx, LDDMM_EINVAL, "unknown integrator %d", p->integrator);
  return LDDMM_OK;
}

template <typename T>
T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }

lddmm_status ensure_ws(lddmm_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return LDDMM_OK;
  if (ctx->budget && (bytes > ctx->budget || ctx->sws_bytes > ctx->budget - bytes))
    return fail(ctx, LDDMM_ENOMEM,
                "workspace of %zu bytes (+ %zu of solver workspace) exceeds the context's "
                "budget of %zu bytes", bytes, ctx->sws_bytes, ctx->budget);
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (ctx->ws) {
    HIP_TRY(ctx, hipDeviceSynchronize(), "hipDeviceSynchronize");
    HIP_TRY(ctx, hipFree(ctx->ws), "hipFree");
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  // headroom for slightly larger problems, unless a budget is set
  const size_t want = ctx->budget ? a256(bytes) : a256(bytes + bytes / 4);
  if (hipMalloc(&ctx->ws, want) != hipSuccess) {
    ctx->ws = nullptr;
    (void)hipGetLastError();
    return fail(ctx, LDDMM_ENOMEM, "hipMalloc of %zu bytes failed", want);
  }
  ctx->ws_bytes = want;
  return LDDMM_OK;
}

// Everything one pass over a problem needs, resolved to device addresses.
struct Job {
  lddmm_params p;
  Plan plan;
  Scales sc;
  Layout L;
  void* ws;
  double *st, *ad, *hp0, *hq0, *xc, *cen, *h0p, *out3, *ckpt;
  double *hpT, *hqT, *hTp, *stT, *rk_acc, *rk_lam;
  void* recT;
  char *traj, *arec;
  void* partial;
  size_t rb;
  int dim;   // 2 (planar) or 3
  int spt;   // records per step: 1 (Euler) or 4 (Runge-Kutta stage states)

  // Record of stage s (0-based) of step t; (t, 0) is the state at step t.
  void* rec(int t, int s = 0) const {
    const int r = spt * t + s;
    const int k = L.nseg > 0 ? r % L.slots : r;
    return traj + (size_t)k * p.n * rb;
  }
  void* arec_buf(int k) const { return arec + (size_t)k * p.n * rb; }
  double* ckpt_state(int seg) const { return ckpt + (size_t)seg * 6 * p.n; }
};

// The launch plan of a problem (the workspace layout depends on its S).
Plan plan_for(const lddmm_params& p) {
  Plan plan = make_plan(p.n, target_waves());
  if (!plan_overridden()) widen_plan(plan, p.precision, p.integrator == LDDMM_RK4);
  return plan;
}

Job make_job(const lddmm_params& p, void* ws) {
  Job j{};
  j.p = p;
  j.plan = plan_for(p);
  j.sc = make_scales(p.sigma, p.T);
  j.L = make_layout(p, j.plan);
  j.ws = ws;
  j.st = at<double>(ws, j.L.st);
  j.ad = at<double>(ws, j.L.ad);
  j.hp0 = at<double>(ws, j.L.hp0);
  j.hq0 = at<double>(ws, j.L.hq0);
  j.xc = at<double>(ws, j.L.xc);
  j.cen = at<double>(ws, j.L.cen);
  j.h0p = at<double>(ws, j.L.h0p);
  j.out3 = at<double>(ws, j.L.out3);
  j.ckpt = at<double>(ws, j.L.ckpt);
  j.traj = at<char>(ws, j.L.traj);
  j.arec = at<char>(ws, j.L.arec);
  j.partial = at<void>(ws, j.L.partial);
  j.hpT = at<double>(ws, j.L.hpT);
  j.hqT = at<double>(ws, j.L.hqT);
  j.hTp = at<double>(ws, j.L.hTp);
  j.stT = at<double>(ws, j.L.stT);
  j.recT = at<void>(ws, j.L.recT);
  j.rk_acc = at<double>(ws, j.L.rk_acc);
  j.rk_lam = at<double>(ws, j.L.rk_lam);
  j.spt = p.integrator == LDDMM_RK4 ? 4 : 1;
  j.rb = rec_bytes(p.precision);
  j.dim = p.dim == 2 ? 2 : 3;
  return j;
}

// Forward steps t in [t0, t1): one launch per Euler step, four per Runge-Kutta
// step (its stages).  first: capture Hp(q0,p0) and H0 at t == 0.
hipError_t run_forward(const Job& j, int t0, int t1, bool first, bool store_ckpt, hipStream_t s,
                       Timer* tm, bool want_hq0 = false) {
  const int mode = j.p.precision;
  const int stages = j.spt;
  for (int t = t0; t < t1; ++t) {
    for (int st = 0; st < stages; ++st) {
      const bool last = st == stages - 1;   // this launch writes the state of step t + 1
      FwdArgs a{};
      a.n = j.p.n; a.nb = j.plan.nb; a.S = j.plan.S; a.chunk = j.plan.chunk;
      a.wchunk = j.plan.wchunk;
      a.dim = j.dim;
      a.rk = stages == 4 ? st + 1 : 0;
      a.rk_acc = j.rk_acc;
      a.sc = j.sc;
      a.rec_t = j.rec(t, st);
      a.rec_t1 = last ? j.rec(t + 1) : j.rec(t, st + 1);
      a.st = j.st;
      const bool t0_field = first && t == 0 && st == 0;   // the field at (q0, p0)
      a.hp0 = t0_field ? j.hp0 : nullptr;
      a.hq0 = t0_field && want_hq0 ? j.hq0 : nullptr;
      a.h0_part = t0_field ? j.h0p : nullptr;
      const int s_every = j.p.ckpt_every;
      a.ckpt = (last && store_ckpt && j.L.nseg > 0 && (t + 1) % s_every == 0 && t + 1 < j.p.T)
                   ? j.ckpt_state((t + 1) / s_every) : nullptr;
      a.partial = j.partial;
      hipError_t e = launch_fwd_step(mode, j.plan, a, s, tm->take(0));
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// Adjoint steps t = t1-1 down to t0 (Runge-Kutta: stages 4 down to 1 each);
// *cur is the adjoint record buffer in use.
hipError_t run_adjoint(const Job& j, int t0, int t1, int* cur, double* grad, hipStream_t s,
                       Timer* tm, double* grad_q0 = nullptr) {
  const int mode = j.p.precision;
  const int stages = j.spt;
  for (int t = t1 - 1; t >= t0; --t) {
    for (int st = stages - 1; st >= 0; --st) {
      AdjArgs a{};
      a.n = j.p.n; a.nb = j.plan.nb; a.S = j.plan.S; a.chunk = j.plan.chunk;
      a.wchunk = j.plan.wchunk_a;
      a.dim = j.dim;
      a.rk = stages == 4 ? st + 1 : 0;
      a.rk_lam = j.rk_lam;
      a.sc = j.sc;
      a.rec_t = j.rec(t, st);
      a.arec = j.arec_buf(*cur);
      a.arec_next = j.arec_buf(*cur ^ 1);
      a.ad = j.ad;
      const bool fin = j.p.energy == LDDMM_ENERGY_FINAL;   // then dL/dp0 = b(0), dL/dq0 = a(0)
      const bool end = t == 0 && st == 0;                   // the adjoint at t = 0 is complete
      a.hp0 = fin ? nullptr : j.hp0;
      a.grad = end ? grad : nullptr;
      a.hq0 = fin ? nullptr : j.hq0;
      a.grad_q0 = end ? grad_q0 : nullptr;
      a.partial = j.partial;
      hipError_t e = launch_adj_step(mode, j.plan, a, s, tm->take(1));
      if (e != hipSuccess) return e;
      *cur ^= 1;
    }
  }
  return hipSuccess;
}

// extra: bytes the caller needs past the job's buffers, at ws + L.total.
lddmm_status begin(lddmm_ctx* ctx, const lddmm_params* params, Job* job, size_t extra = 0) {
  if (!ctx) return fail(nullptr, LDDMM_EINVAL, "ctx is NULL");
  lddmm_status st = check_params(ctx, params);
  if (st != LDDMM_OK) return st;
  const Layout L = make_layout(*params, plan_for(*params));
  st = ensure_ws(ctx, L.total + a256(extra));
  if (st != LDDMM_OK) return st;
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  *job = make_job(*params, ctx->ws);
  return LDDMM_OK;
}

// One loss+gradient evaluation (Alg. 1 ComputeGradient) of a prepared job.
// tm: the per-kernel timer (the context's, or one that stays off).
lddmm_status run_grad(lddmm_ctx* ctx, const Job& j, const double* q0, const double* p0,
                      const double* target, double* out3, double* grad, double* q1,
                      hipStream_t s, double* grad_q0 = nullptr, double* grad_x = nullptr,
                      Timer* tm = nullptr) {
  if (!tm) tm = &ctx->timer;
  const lddmm_params* params = &j.p;
  const int n = params->n, T = params->T, mode = params->precision;
  HIP_TRY(ctx, launch_centroid(q0, n, j.cen, s), "centroid");
  HIP_TRY(ctx, launch_stage(mode, n, q0, p0, target, j.cen, j.sc.k, j.st, j.xc, j.rec(0), s),
          "stage");
  if (j.L.nseg > 0)
    HIP_TRY(ctx, hipMemcpyAsync(j.ckpt_state(0), j.st, 6 * (size_t)n * 8, hipMemcpyDeviceToDevice, s),
            "checkpoint 0");
  HIP_TRY(ctx, run_forward(j, 0, T, true, true, s, tm, grad_q0 != nullptr), "forward step");
  const bool fin = params->energy == LDDMM_ENERGY_FINAL;
  if (fin) {
    // Energy at t = 1 (the loss as Alg. 1 evaluates it after the forward loop): the
    // forward sums at the final state, taken by one more forward launch on a scratch
    // copy of the state, so the trajectory and the state stay as they are.
    HIP_TRY(ctx, hipMemcpyAsync(j.stT, j.st, 6 * (size_t)n * 8, hipMemcpyDeviceToDevice, s),
            "final state copy");
    FwdArgs a{};
    a.n = n; a.nb = j.plan.nb; a.S = j.plan.S; a.chunk = j.plan.chunk; a.wchunk = j.plan.wchunk;
    a.dim = j.dim;
    a.sc = j.sc;
    a.rec_t = j.rec(T);
    a.rec_t1 = j.recT;
    a.st = j.stT;
    a.hp0 = j.hpT;
    a.hq0 = j.hqT;
    a.h0_part = j.hTp;
    a.partial = j.partial;
    HIP_TRY(ctx, launch_fwd_step(mode, j.plan, a, s, tm->take(0)), "final energy");
  }
  const double rscale = j.spt == 4 ? j.sc.dt / 6.0 : 1.0;   // first stage adjoint: dt/6 lambda
  HIP_TRY(ctx, launch_loss(mode, n, j.plan.nb, params->lambda, j.sc.bscale, rscale, j.st, j.xc,
                           j.cen, fin ? j.hTp : j.h0p, j.ad, j.arec_buf(0), out3, q1, nullptr,
                           ctx->flag, grad_x, fin ? j.hqT : nullptr, fin ? j.hpT : nullptr, s),
          "loss");
  int cur = 0;
  if (j.L.nseg == 0) {
    HIP_TRY(ctx, run_adjoint(j, 0, T, &cur, grad, s, tm, grad_q0), "adjoint step");
  } else {
    const int every = params->ckpt_every;
    for (int seg = j.L.nseg - 1; seg >= 0; --seg) {
      const int t0 = seg * every, t1 = std::min(T, t0 + every);
      if (seg != j.L.nseg - 1) {   // the last segment is still in the ring of slots
        HIP_TRY(ctx, launch_restore(mode, n, j.ckpt_state(seg), j.sc.k, j.st, j.rec(t0), s),
                "restore");
        HIP_TRY(ctx, run_forward(j, t0, t1, false, false, s, tm), "recompute step");
      }
      HIP_TRY(ctx, run_adjoint(j, t0, t1, &cur, grad, s, tm, grad_q0), "adjoint step");
    }
  }
  return LDDMM_OK;
}

}  // namespace

extern "C" {

const char* lddmm_version(void) { return "0.1.0"; }

const char* lddmm_status_string(lddmm_status s) {
  switch (s) {
    case LDDMM_OK: return "ok";
    case LDDMM_ENOTCONV: return "not converged (result written)";
    case LDDMM_EINVAL: return "invalid argument";
    case LDDMM_ENOMEM: return "out of device memory";
    case LDDMM_EDEVICE: return "HIP runtime error";
    case LDDMM_ENONFINITE: return "non-finite value";
    case LDDMM_EBUSY: return "busy";
  }
  return "unknown status";
}

const char* lddmm_last_error(lddmm_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

lddmm_status lddmm_ctx_create(int device, size_t hbm_budget_bytes, lddmm_ctx** out) {
  if (!out) return fail(nullptr, LDDMM_EINVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
  if (device < 0 || device >= count)
    return fail(nullptr, LDDMM_EINVAL, "device %d out of range (%d devices)", device, count);
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
  lddmm_ctx* c = new (std::nothrow) lddmm_ctx;
  if (!c) return fail(nullptr, LDDMM_ENOMEM, "host allocation failed");
  c->device = device;
  c->budget = hbm_budget_bytes;
  e = hipMalloc(&c->flag, 256);
  if (e == hipSuccess) e = hipMemset(c->flag, 0, 256);
  if (e == hipSuccess) e = hipHostMalloc(&c->host_done, 2 * sizeof(int), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->poll_ev[0], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->poll_ev[1], hipEventDisableTiming);
  if (e == hipSuccess) e = scratch_address(device, &c->scratch);
  if (e != hipSuccess) {
    lddmm_ctx_destroy(c);
    return hip_fail(nullptr, e, "context allocation");
  }
  *out = c;
  return LDDMM_OK;
}

lddmm_status lddmm_ctx_destroy(lddmm_ctx* ctx) {
  if (!ctx) return LDDMM_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->flag) (void)hipFree(ctx->flag);
  if (ctx->sws) (void)hipFree(ctx->sws);
  if (ctx->host_done) (void)hipHostFree(ctx->host_done);
  for (hipEvent_t& e : ctx->poll_ev)
    if (e) (void)hipEventDestroy(e);
  ctx->timer.destroy();
  delete ctx;
  return LDDMM_OK;
}

lddmm_status lddmm_workspace_size(const lddmm_params* params, size_t* bytes) {
  lddmm_status st = check_params(nullptr, params);
  if (st != LDDMM_OK) return st;
  if (!bytes) return fail(nullptr, LDDMM_EINVAL, "bytes is NULL");
  *bytes = make_layout(*params, plan_for(*params)).total;
  return LDDMM_OK;
}

lddmm_status lddmm_shoot_forward(lddmm_ctx* ctx, const lddmm_params* params, const double* q0,
                                 const double* p0, double* q1, double* p1, double* H0,
                                 void* stream) {
  if (ctx && (!q0 || !p0)) return fail(ctx, LDDMM_EINVAL, "q0 and p0 must not be NULL");
  Job j;
  lddmm_status st = begin(ctx, params, &j);
  if (st != LDDMM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = params->n;
  HIP_TRY(ctx, launch_centroid(q0, n, j.cen, s), "centroid");
  HIP_TRY(ctx, launch_stage(params->precision, n, q0, p0, nullptr, j.cen, j.sc.k, j.st, j.xc,
                            j.rec(0), s), "stage");
  HIP_TRY(ctx, run_forward(j, 0, params->T, true, false, s, &ctx->timer), "forward step");
  HIP_TRY(ctx, launch_forward_out(n, j.plan.nb, j.st, j.cen, j.h0p, H0, q1, p1, s), "forward out");
  return LDDMM_OK;
}

lddmm_status lddmm_shoot_grad(lddmm_ctx* ctx, const lddmm_params* params, const double* q0,
                              const double* p0, const double* target, double* out3,
                              double* grad, double* q1, void* stream) {
  if (ctx && (!q0 || !p0 || !target || !out3 || !grad))
    return fail(ctx, LDDMM_EINVAL, "q0, p0, target, out3 and grad must not be NULL");
  Job j;
  lddmm_status st = begin(ctx, params, &j);
  if (st != LDDMM_OK) return st;
  return run_grad(ctx, j, q0, p0, target, out3, grad, q1, static_cast<hipStream_t>(stream));
}

lddmm_status lddmm_shoot_grad_noalloc(lddmm_ctx* ctx, const lddmm_params* params,
                                      const double* q0, const double* p0, const double* target,
                                      double* out3, double* grad, double* q1, void* stream) {
  if (!ctx) return fail(nullptr, LDDMM_EINVAL, "ctx is NULL");
  if (!q0 || !p0 || !target || !out3 || !grad)
    return fail(ctx, LDDMM_EINVAL, "q0, p0, target, out3 and grad must not be NULL");
  lddmm_status st = check_params(ctx, params);
  if (st != LDDMM_OK) return st;
  const Layout L = make_layout(*params, plan_for(*params));
  if (L.total > kScratchBytes)
    return fail(ctx, LDDMM_ENOMEM,
                "workspace of %zu bytes exceeds the fixed scratch of %zu bytes of "
                "lddmm_shoot_grad_noalloc (use lddmm_shoot_grad, or checkpoints)",
                L.total, kScratchBytes);
  if (!ctx->scratch) return fail(ctx, LDDMM_EDEVICE, "no scratch address for the device");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  const Job j = make_job(*params, ctx->scratch);
  Timer off;   // timing stays off: no events are created on this path
  return run_grad(ctx, j, q0, p0, target, out3, grad, q1, static_cast<hipStream_t>(stream),
                  nullptr, nullptr, &off);
}

lddmm_status lddmm_shoot_grad_all(lddmm_ctx* ctx, const lddmm_params* params, const double* q0,
                                  const double* p0, const double* target, double* out3,
                                  double* grad_p0, double* grad_q0, double* grad_x, double* q1,
                                  void* stream) {
  if (ctx && (!q0 || !p0 || !target || !out3 || !grad_p0))
    return fail(ctx, LDDMM_EINVAL, "q0, p0, target, out3 and grad_p0 must not be NULL");
  Job j;
  lddmm_status st = begin(ctx, params, &j);
  if (st != LDDMM_OK) return st;
  return run_grad(ctx, j, q0, p0, target, out3, grad_p0, q1, static_cast<hipStream_t>(stream),
                  grad_q0, grad_x);
}

namespace {

FlowArgs flow_args(const Job& j, int m, int W) {
  FlowArgs a{};
  a.n = j.p.n;
  a.m = m;
  a.slots = j.L.slots;
  a.spt = j.spt;
  a.wchunk = (j.p.n + W - 1) / W;
  a.dim = j.dim;
  a.k = j.sc.k;
  a.dt = j.sc.dt;
  a.traj = j.traj;
  a.cen = j.cen;
  return a;
}

}  // namespace

lddmm_status lddmm_velocity(lddmm_ctx* ctx, const lddmm_params* params, const double* q,
                            const double* p, int32_t m, const double* x, double* v,
                            void* stream) {
  if (m < 0 || m > kMaxPoints)
    return fail(ctx, LDDMM_EINVAL, "m must be in 0..%d (got %d)", kMaxPoints, m);
  if (ctx && params && (!q || !p || (m > 0 && (!x || !v))))
    return fail(ctx, LDDMM_EINVAL, "q and p must not be NULL, x and v non-NULL if m > 0");
  if (!params) return fail(ctx, LDDMM_EINVAL, "params is NULL");
  lddmm_params one = *params;   // one state: no trajectory beyond slot 0
  one.T = 1;
  one.ckpt_every = 0;
  one.integrator = LDDMM_EULER;   // no steps are taken
  Job j;
  lddmm_status st = begin(ctx, &one, &j);
  if (st != LDDMM_OK) return st;
  if (m == 0) return LDDMM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = one.n;
  HIP_TRY(ctx, launch_centroid(q, n, j.cen, s), "centroid");
  HIP_TRY(ctx, launch_stage(one.precision, n, q, p, nullptr, j.cen, j.sc.k, j.st, j.xc, j.rec(0), s),
          "stage");
  const int W = flow_waves(n);
  FlowArgs a = flow_args(j, m, W);
  a.t0 = 0;
  a.t1 = 1;
  a.x_in = x;
  a.v_out = v;
  HIP_TRY(ctx, launch_flow(one.precision, W, a, s, ctx->timer.take(2)), "velocity");
  return LDDMM_OK;
}

lddmm_status lddmm_flow(lddmm_ctx* ctx, const lddmm_params* params, const double* q0,
                        const double* p0, int32_t m, const double* x0, double* x1, double* q1,
                        double* p1, void* stream) {
  if (m < 0 || m > kMaxPoints)
    return fail(ctx, LDDMM_EINVAL, "m must be in 0..%d (got %d)", kMaxPoints, m);
  if (ctx && params && (!q0 || !p0 || (m > 0 && (!x0 || !x1))))
    return fail(ctx, LDDMM_EINVAL, "q0 and p0 must not be NULL, x0 and x1 non-NULL if m > 0");
  if (!params) return fail(ctx, LDDMM_EINVAL, "params is NULL");
  const bool seg = params->ckpt_every > 0 && params->ckpt_every < params->T;
  Job j;
  lddmm_status st = begin(ctx, params, &j, seg ? 3 * (size_t)(m > 0 ? m : 0) * 8 : 0);
  if (st != LDDMM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = params->n, T = params->T;
  HIP_TRY(ctx, launch_centroid(q0, n, j.cen, s), "centroid");
  HIP_TRY(ctx, launch_stage(params->precision, n, q0, p0, nullptr, j.cen, j.sc.k, j.st, j.xc,
                            j.rec(0), s), "stage");
  const int W = flow_waves(n);
  double* xs = at<double>(ctx->ws, j.L.total);
  // Segments of the landmark forward pass, each followed by the points' steps
  // over the same records (one segment when the whole trajectory is kept).
  const int every = seg ? params->ckpt_every : T;
  for (int t0 = 0; t0 < T; t0 += every) {
    const int t1 = t0 + every < T ? t0 + every : T;
    HIP_TRY(ctx, run_forward(j, t0, t1, t0 == 0, false, s, &ctx->timer), "forward step");
    if (m == 0) continue;
    FlowArgs a = flow_args(j, m, W);
    a.t0 = t0;
    a.t1 = t1;
    a.x_in = t0 == 0 ? x0 : nullptr;
    a.x_out = t1 == T ? x1 : nullptr;
    a.xs = xs;
    HIP_TRY(ctx, launch_flow(params->precision, W, a, s, ctx->timer.take(2)), "point flow");
  }
  if (q1 || p1)
    HIP_TRY(ctx, launch_forward_out(n, j.plan.nb, j.st, j.cen, j.h0p, nullptr, q1, p1, s),
            "forward out");
  return LDDMM_OK;
}

lddmm_status lddmm_solve_opts_default(int32_t precision, lddmm_solve_opts* o) {
  if (!o) return fail(nullptr, LDDMM_EINVAL, "opts is NULL");
  if (precision < LDDMM_FP32 || precision > LDDMM_FP64)
    return fail(nullptr, LDDMM_EINVAL, "unknown precision %d", precision);
  o->max_iter = 100;
  o->m = 5;
  o->max_fev = 20;
  o->gtol = precision == LDDMM_FP64 ? 1e-8 : 1e-6;
  o->ftol_rel = 0.0;
  o->c1 = 1e-4;
  o->c2 = 0.9;
  o->init = 0;
  return LDDMM_OK;
}

lddmm_status lddmm_solve(lddmm_ctx* ctx, const lddmm_params* params, const lddmm_solve_opts* opts,
                         const double* q0, const double* target, double* p0_inout,
                         lddmm_solve_result* result, double* trace, void* stream) {
  if (ctx && (!opts || !q0 || !target || !p0_inout))
    return fail(ctx, LDDMM_EINVAL, "opts, q0, target and p0_inout must not be NULL");
  if (ctx) {
    if (opts->max_iter < 0) return fail(ctx, LDDMM_EINVAL, "max_iter must be >= 0");
    if (opts->m < 1 || opts->m > kMaxHistory)
      return fail(ctx, LDDMM_EINVAL, "m must be in 1..%d", kMaxHistory);
    if (opts->max_fev < 1) return fail(ctx, LDDMM_EINVAL, "max_fev must be >= 1");
    if (!(opts->c1 > 0.0 && opts->c1 < opts->c2 && opts->c2 < 1.0))
      return fail(ctx, LDDMM_EINVAL, "need 0 < c1 < c2 < 1");
    if (!(opts->gtol >= 0.0) || !(opts->ftol_rel >= 0.0))
      return fail(ctx, LDDMM_EINVAL, "gtol and ftol_rel must be >= 0");
    if (opts->init < 0 || opts->init > 2) return fail(ctx, LDDMM_EINVAL, "init must be 0, 1 or 2");
  }
  Job j;
  lddmm_status st = begin(ctx, params, &j);
  if (st != LDDMM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = params->n;
  const size_t m3 = 3 * (size_t)n;

  // solver workspace: x g d xt gt, S Y, q1, out3, state, result, trace
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += a256(bytes); return o; };
  const size_t o_vec = take(5 * m3 * 8), o_hist = take(2 * (size_t)opts->m * m3 * 8);
  const size_t o_q1 = take(m3 * 8), o_out3 = take(4 * 8), o_state = take(sizeof(LbfgsState));
  const size_t o_res = take(sizeof(LbfgsResult));
  const size_t o_trace = take(2 * ((size_t)opts->max_iter + 1) * 8);
  if (off > ctx->sws_bytes) {
    if (ctx->budget && (off > ctx->budget || ctx->ws_bytes > ctx->budget - off))
      return fail(ctx, LDDMM_ENOMEM,
                  "solver workspace of %zu bytes (+ %zu of workspace) exceeds the context's "
                  "budget of %zu bytes", off, ctx->ws_bytes, ctx->budget);
    HIP_TRY(ctx, hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (ctx->sws) HIP_TRY(ctx, hipFree(ctx->sws), "hipFree");
    ctx->sws = nullptr;
    ctx->sws_bytes = 0;
    if (hipMalloc(&ctx->sws, off) != hipSuccess) {
      ctx->sws = nullptr;
      (void)hipGetLastError();
      return fail(ctx, LDDMM_ENOMEM, "hipMalloc of %zu bytes (solver) failed", off);
    }
    ctx->sws_bytes = off;
  }
  LbfgsBufs B{};
  B.m3 = (int)m3;
  double* vec = at<double>(ctx->sws, o_vec);
  B.x = vec; B.g = vec + m3; B.d = vec + 2 * m3; B.xt = vec + 3 * m3; B.gt = vec + 4 * m3;
  B.S = at<double>(ctx->sws, o_hist);
  B.Y = B.S + (size_t)opts->m * m3;
  double* q1 = at<double>(ctx->sws, o_q1);
  double* out3 = at<double>(ctx->sws, o_out3);
  B.ft = out3;
  B.trace = at<double>(ctx->sws, o_trace);
  LbfgsState* state = at<LbfgsState>(ctx->sws, o_state);
  LbfgsResult* dres = at<LbfgsResult>(ctx->sws, o_res);
  LbfgsOpts o{opts->max_iter, opts->m, opts->max_fev, opts->gtol, opts->ftol_rel, opts->c1, opts->c2};

  HIP_TRY(ctx, launch_lbfgs_init(B, state, opts->init, q0, target, p0_inout, params->T, s),
          "solver init");
  // Evaluation c and the optimiser step that consumes it are enqueued before
  // the host waits on evaluation c-1, so the device never idles on the poll;
  // at most one evaluation after convergence is wasted (its step is a no-op).
  const long cap = 1 + (long)opts->max_iter * opts->max_fev;
  for (long c = 0;; ++c) {
    st = run_grad(ctx, j, q0, B.xt, target, out3, B.gt, nullptr, s);
    if (st != LDDMM_OK) return st;
    HIP_TRY(ctx, launch_lbfgs_step(B, state, o, s), "solver step");
    HIP_TRY(ctx, hipMemcpyAsync(&ctx->host_done[c & 1], &state->done, sizeof(int),
                                hipMemcpyDeviceToHost, s), "poll copy");
    HIP_TRY(ctx, hipEventRecord(ctx->poll_ev[c & 1], s), "poll event");
    if (c >= 1) {
      HIP_TRY(ctx, hipEventSynchronize(ctx->poll_ev[(c - 1) & 1]), "poll wait");
      if (ctx->host_done[(c - 1) & 1]) break;
    }
    if (c + 1 >= cap) break;
  }
  // final evaluation at the accepted iterate, for the reported loss terms and q(1)
  st = run_grad(ctx, j, q0, B.x, target, out3, B.gt, q1, s);
  if (st != LDDMM_OK) return st;
  HIP_TRY(ctx, launch_lbfgs_result(n, q1, target, out3, state, dres, s), "solver result");
  HIP_TRY(ctx, hipMemcpyAsync(p0_inout, B.x, m3 * 8, hipMemcpyDeviceToDevice, s), "p0 copy");
  LbfgsResult hr{};
  HIP_TRY(ctx, hipMemcpyAsync(&hr, dres, sizeof hr, hipMemcpyDeviceToHost, s), "result copy");
  if (trace)
    HIP_TRY(ctx, hipMemcpyAsync(trace, B.trace, 2 * ((size_t)opts->max_iter + 1) * 8,
                                hipMemcpyDeviceToHost, s), "trace copy");
  HIP_TRY(ctx, hipStreamSynchronize(s), "hipStreamSynchronize");
  const lddmm_status rs = hr.status == kConverged ? LDDMM_OK
                          : hr.status == kNonFinite ? LDDMM_ENONFINITE : LDDMM_ENOTCONV;
  if (result) {
    result->loss = hr.loss;
    result->H0 = hr.H0;
    result->mismatch = hr.mismatch;
    result->grad_norm = hr.grad_norm;
    result->avg_dist = hr.avg_dist;
    result->max_dist = hr.max_dist;
    result->iters = hr.iters;
    result->fevals = hr.fevals;
    result->status = rs;
  }
  if (!hr.done) return fail(ctx, LDDMM_ENOTCONV, "evaluation cap reached");
  if (rs == LDDMM_ENONFINITE) return fail(ctx, rs, "non-finite loss or gradient");
  return rs;
}

lddmm_status lddmm_ctx_set_timing(lddmm_ctx* ctx, int enable) {
  if (!ctx) return fail(nullptr, LDDMM_EINVAL, "ctx is NULL");
  ctx->timer.on = enable != 0;
  return LDDMM_OK;
}

lddmm_status lddmm_ctx_timing(lddmm_ctx* ctx, lddmm_timing* out, int reset) {
  if (!ctx || !out) return fail(ctx, LDDMM_EINVAL, "ctx and out must not be NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  HIP_TRY(ctx, ctx->timer.collect(), "timing events");
  out->fwd_ms = ctx->timer.ms[0];
  out->adj_ms = ctx->timer.ms[1];
  out->fwd_launches = ctx->timer.count[0];
  out->adj_launches = ctx->timer.count[1];
  out->flow_ms = ctx->timer.ms[2];
  out->flow_launches = ctx->timer.count[2];
  if (reset)
    for (int k = 0; k < 3; ++k) {
      ctx->timer.ms[k] = 0.0;
      ctx->timer.count[k] = 0;
    }
  return LDDMM_OK;
}

lddmm_status lddmm_ctx_check(lddmm_ctx* ctx, void* stream) {
  if (!ctx) return fail(nullptr, LDDMM_EINVAL, "ctx is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  HIP_TRY(ctx, hipStreamSynchronize(static_cast<hipStream_t>(stream)), "hipStreamSynchronize");
  int f = 0;
  HIP_TRY(ctx, hipMemcpy(&f, ctx->flag, sizeof f, hipMemcpyDeviceToHost), "flag read");
  if (f) {
    HIP_TRY(ctx, hipMemset(ctx->flag, 0, sizeof f), "flag clear");
    return fail(ctx, LDDMM_ENONFINITE, "a non-finite loss was produced");
  }
  return LDDMM_OK;
}

}  // extern "C"
