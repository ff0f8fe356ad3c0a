// C ABI of liblddmm: validation, context and workspace, and the host-side
// order of kernel launches for one forward pass, the loss, and one adjoint
// pass (Alg. 1, ComputeGradient), optionally with checkpoint recompute.
#include "lddmm.h"
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
  struct Rec { hipEvent_t ev[2]; int kind; };   // kind 0: forward, 1: adjoint
  bool on = false;
  std::vector<Rec> pending, spare;
  double ms[2] = {0.0, 0.0};
  int64_t count[2] = {0, 0};

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
  void* ws = nullptr;        // workspace
  size_t ws_bytes = 0;
  int* flag = nullptr;       // device non-finite flag
  Timer timer;
  std::string err;
};

namespace {

thread_local std::string g_err;   // errors that have no context

// Waves the pair kernels aim to keep in flight (256 CUs x 4 SIMDs x 4);
// LDDMM_TARGET_WAVES overrides it for tuning.
int target_waves() {
  static const int v = [] {
    const char* e = std::getenv("LDDMM_TARGET_WAVES");
    const int t = e ? std::atoi(e) : 0;
    return t > 0 ? t : 4096;
  }();
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
  if (p->n > (1 << 26)) return fail(ctx, LDDMM_EINVAL, "n too large (%d)", p->n);
  if (p->T < 1) return fail(ctx, LDDMM_EINVAL, "T must be >= 1 (got %d)", p->T);
  if (!(p->sigma > 0.0) || !std::isfinite(p->sigma))
    return fail(ctx, LDDMM_EINVAL, "sigma must be finite and > 0");
  if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda))
    return fail(ctx, LDDMM_EINVAL, "lambda must be finite and >= 0");
  if (p->precision < LDDMM_FP32 || p->precision > LDDMM_FP64)
    return fail(ctx, LDDMM_EINVAL, "unknown precision %d", p->precision);
  if (p->ckpt_every < 0) return fail(ctx, LDDMM_EINVAL, "ckpt_every must be >= 0");
  return LDDMM_OK;
}

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

// Byte offsets of the workspace buffers of one problem.
struct Layout {
  size_t st, ad, hp0, xc, cen, h0p, out3, traj, arec, ckpt, partial, total;
  int slots;   // trajectory slots
  int nseg;    // checkpoint segments (0 = full trajectory)
};

Layout make_layout(const lddmm_params& p, const Plan& plan) {
  Layout L{};
  const size_t n = (size_t)p.n, rb = rec_bytes(p.precision), ab = acc_bytes(p.precision);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += a256(bytes); return o; };
  L.st = take(6 * n * 8);
  L.ad = take(6 * n * 8);
  L.hp0 = take(3 * n * 8);
  L.xc = take(3 * n * 8);
  L.cen = take(4 * 8);
  L.h0p = take((size_t)plan.nb * 8);
  L.out3 = take(4 * 8);
  const int s = p.ckpt_every;
  const bool ck = s > 0 && s < p.T;
  L.slots = ck ? s + 1 : p.T + 1;
  L.nseg = ck ? (p.T + s - 1) / s : 0;
  L.traj = take((size_t)L.slots * n * rb);
  L.arec = take(2 * n * rb);
  L.ckpt = take((size_t)L.nseg * 6 * n * 8);
  L.partial = take(plan.S > 1 ? (size_t)plan.S * 9 * n * ab : 0);
  L.total = off;
  return L;
}

template <typename T>
T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }

lddmm_status ensure_ws(lddmm_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return LDDMM_OK;
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (ctx->ws) {
    HIP_TRY(ctx, hipDeviceSynchronize(), "hipDeviceSynchronize");
    HIP_TRY(ctx, hipFree(ctx->ws), "hipFree");
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  const size_t want = a256(bytes + bytes / 4);   // headroom for slightly larger problems
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
  double *st, *ad, *hp0, *xc, *cen, *h0p, *out3, *ckpt;
  char *traj, *arec;
  void* partial;
  size_t rb;

  void* slot(int t) const {
    const int k = L.nseg > 0 ? t % L.slots : t;
    return traj + (size_t)k * p.n * rb;
  }
  void* arec_buf(int k) const { return arec + (size_t)k * p.n * rb; }
  double* ckpt_state(int seg) const { return ckpt + (size_t)seg * 6 * p.n; }
};

Job make_job(const lddmm_params& p, void* ws) {
  Job j{};
  j.p = p;
  j.plan = make_plan(p.n, target_waves());
  j.sc = make_scales(p.sigma, p.T);
  j.L = make_layout(p, j.plan);
  j.ws = ws;
  j.st = at<double>(ws, j.L.st);
  j.ad = at<double>(ws, j.L.ad);
  j.hp0 = at<double>(ws, j.L.hp0);
  j.xc = at<double>(ws, j.L.xc);
  j.cen = at<double>(ws, j.L.cen);
  j.h0p = at<double>(ws, j.L.h0p);
  j.out3 = at<double>(ws, j.L.out3);
  j.ckpt = at<double>(ws, j.L.ckpt);
  j.traj = at<char>(ws, j.L.traj);
  j.arec = at<char>(ws, j.L.arec);
  j.partial = at<void>(ws, j.L.partial);
  j.rb = rec_bytes(p.precision);
  return j;
}

// Forward Euler steps t in [t0, t1).  first: capture Hp(q0,p0) and H0 at t == 0.
hipError_t run_forward(const Job& j, int t0, int t1, bool first, bool store_ckpt, hipStream_t s,
                       Timer* tm) {
  const int mode = j.p.precision;
  for (int t = t0; t < t1; ++t) {
    FwdArgs a{};
    a.n = j.p.n; a.nb = j.plan.nb; a.S = j.plan.S; a.chunk = j.plan.chunk; a.wchunk = j.plan.wchunk;
    a.sc = j.sc;
    a.rec_t = j.slot(t);
    a.rec_t1 = j.slot(t + 1);
    a.st = j.st;
    a.hp0 = (first && t == 0) ? j.hp0 : nullptr;
    a.h0_part = (first && t == 0) ? j.h0p : nullptr;
    const int s_every = j.p.ckpt_every;
    a.ckpt = (store_ckpt && j.L.nseg > 0 && (t + 1) % s_every == 0 && t + 1 < j.p.T)
                 ? j.ckpt_state((t + 1) / s_every) : nullptr;
    a.partial = j.partial;
    hipError_t e = launch_fwd_step(mode, j.plan, a, s, tm->take(0));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Adjoint steps t = t1-1 down to t0; *cur is the adjoint record buffer in use.
hipError_t run_adjoint(const Job& j, int t0, int t1, int* cur, double* grad, hipStream_t s,
                       Timer* tm) {
  const int mode = j.p.precision;
  for (int t = t1 - 1; t >= t0; --t) {
    AdjArgs a{};
    a.n = j.p.n; a.nb = j.plan.nb; a.S = j.plan.S; a.chunk = j.plan.chunk; a.wchunk = j.plan.wchunk;
    a.sc = j.sc;
    a.rec_t = j.slot(t);
    a.arec = j.arec_buf(*cur);
    a.arec_next = j.arec_buf(*cur ^ 1);
    a.ad = j.ad;
    a.hp0 = j.hp0;
    a.grad = t == 0 ? grad : nullptr;
    a.partial = j.partial;
    hipError_t e = launch_adj_step(mode, j.plan, a, s, tm->take(1));
    if (e != hipSuccess) return e;
    *cur ^= 1;
  }
  return hipSuccess;
}

lddmm_status begin(lddmm_ctx* ctx, const lddmm_params* params, Job* job) {
  if (!ctx) return fail(nullptr, LDDMM_EINVAL, "ctx is NULL");
  lddmm_status st = check_params(ctx, params);
  if (st != LDDMM_OK) return st;
  const Plan plan = make_plan(params->n, target_waves());
  const Layout L = make_layout(*params, plan);
  st = ensure_ws(ctx, L.total);
  if (st != LDDMM_OK) return st;
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  *job = make_job(*params, ctx->ws);
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

lddmm_status lddmm_ctx_create(int device, lddmm_ctx** out) {
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
  e = hipMalloc(&c->flag, 256);
  if (e == hipSuccess) e = hipMemset(c->flag, 0, 256);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(nullptr, e, "flag allocation");
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
  ctx->timer.destroy();
  delete ctx;
  return LDDMM_OK;
}

lddmm_status lddmm_workspace_size(const lddmm_params* params, size_t* bytes) {
  lddmm_status st = check_params(nullptr, params);
  if (st != LDDMM_OK) return st;
  if (!bytes) return fail(nullptr, LDDMM_EINVAL, "bytes is NULL");
  *bytes = make_layout(*params, make_plan(params->n, target_waves())).total;
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
                            j.slot(0), s), "stage");
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
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = params->n, T = params->T, mode = params->precision;
  HIP_TRY(ctx, launch_centroid(q0, n, j.cen, s), "centroid");
  HIP_TRY(ctx, launch_stage(mode, n, q0, p0, target, j.cen, j.sc.k, j.st, j.xc, j.slot(0), s),
          "stage");
  if (j.L.nseg > 0)
    HIP_TRY(ctx, hipMemcpyAsync(j.ckpt_state(0), j.st, 6 * (size_t)n * 8, hipMemcpyDeviceToDevice, s),
            "checkpoint 0");
  HIP_TRY(ctx, run_forward(j, 0, T, true, true, s, &ctx->timer), "forward step");
  HIP_TRY(ctx, launch_loss(mode, n, j.plan.nb, params->lambda, j.sc.bscale, j.st, j.xc, j.cen,
                           j.h0p, j.ad, j.arec_buf(0), out3, q1, nullptr, ctx->flag, s),
          "loss");
  int cur = 0;
  if (j.L.nseg == 0) {
    HIP_TRY(ctx, run_adjoint(j, 0, T, &cur, grad, s, &ctx->timer), "adjoint step");
  } else {
    const int every = params->ckpt_every;
    for (int seg = j.L.nseg - 1; seg >= 0; --seg) {
      const int t0 = seg * every, t1 = std::min(T, t0 + every);
      if (seg != j.L.nseg - 1) {   // the last segment is still in the ring of slots
        HIP_TRY(ctx, launch_restore(mode, n, j.ckpt_state(seg), j.sc.k, j.st, j.slot(t0), s),
                "restore");
        HIP_TRY(ctx, run_forward(j, t0, t1, false, false, s, &ctx->timer), "recompute step");
      }
      HIP_TRY(ctx, run_adjoint(j, t0, t1, &cur, grad, s, &ctx->timer), "adjoint step");
    }
  }
  return LDDMM_OK;
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
  if (reset) {
    ctx->timer.ms[0] = ctx->timer.ms[1] = 0.0;
    ctx->timer.count[0] = ctx->timer.count[1] = 0;
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
