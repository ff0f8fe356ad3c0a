// Continuous-batching registration server (lddmm_server_*).
//
// Registrations (Alg. 1 solves of uneven size) arrive over time.  A worker
// thread admits them, first come first served, whenever a slot is free and
// the job's device footprint fits a preallocated HBM arena; every running
// job keeps its trajectory, adjoint state and L-BFGS state on the device.
// The worker then advances ALL running jobs by one loss+gradient evaluation
// and one optimiser step per round, as one replay of a captured hipGraph:
// batched stage, T forward pair-sum launches, batched loss, T adjoint
// launches, batched L-BFGS step.  Each pair-sum launch covers every
// (job, 64-landmark i-block) item of its kind (once planar jobs have come,
// each step has a launch for the 3D items and one for the planar items,
// which leave the z terms out), so small jobs share the chip instead of
// leaving it idle.  Jobs join at the next round after admission and leave
// when their optimiser finishes; finished jobs are skipped on the device, so
// nothing is wasted while the host notices.
//
// Everything is ordered on one HIP stream: a job's memory can be handed to a
// new job as soon as its result copies are enqueued.  The host learns about
// finished jobs one round late (it waits on round r-1 only after round r is
// queued), so the device never idles on the poll.
#include "arena.h"
#include "lbfgs_internal.h"
#include "lddmm.h"
#include "shoot_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace lddmm;

namespace {

using Clock = std::chrono::steady_clock;

enum JobState { kQueued, kRunning, kFinalizing, kDone, kFailed };

struct ServerJob {
  int64_t id = 0;
  lddmm_params p{};
  lddmm_solve_opts o{};
  std::vector<double> q0, x, p0in, p0out;
  const double* x_dev = nullptr;   // the target in the job's device block
  size_t footprint = 0, off = Arena::npos;
  int slot = -1;
  int64_t first_round = 0;         // first batched round that includes the job
  JobState state = kQueued;
  double t_submit = 0, t_admit = 0, t_done = 0;
  lddmm_solve_result res{};
};

// Byte layout of one job inside its arena block.
struct JobLayout {
  size_t q0, x, cen, st, ad, hp0, xc, h0p, out3, traj, arec, q1, vec, hist, state, out3a, q1a;
  size_t rk_acc, rk_lam;
  size_t total;
};

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

// spt: point records per step, 1 for Euler steps, 4 for Runge-Kutta stages.
JobLayout job_layout(int n, int T, int precision, int m, int spt) {
  JobLayout L{};
  const size_t N = (size_t)n, m3 = 3 * N, rb = rec_bytes(precision), nb = (N + 63) / 64;
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += a256(b); return o; };
  L.q0 = take(m3 * 8);
  L.x = take(m3 * 8);
  L.cen = take(4 * 8);
  L.st = take(6 * N * 8);
  L.ad = take(6 * N * 8);
  L.hp0 = take(m3 * 8);
  L.xc = take(m3 * 8);
  L.h0p = take(nb * 8);
  L.out3 = take(4 * 8);
  L.traj = take(((size_t)spt * T + 1) * N * rb);
  L.arec = take(2 * N * rb);
  L.q1 = take(m3 * 8);
  L.vec = take(5 * m3 * 8);
  L.hist = take(2 * (size_t)m * m3 * 8);
  L.state = take(sizeof(LbfgsState));
  L.out3a = take(4 * 8);
  L.q1a = take(m3 * 8);
  L.rk_acc = take(spt == 4 ? 6 * N * 8 : 0);
  L.rk_lam = take(spt == 4 ? 6 * N * 8 : 0);
  L.total = off;
  return L;
}

template <typename T>
T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }

}  // namespace

struct lddmm_server {
  lddmm_server_config cfg{};
  int capacity = 0;                 // pair-kernel workgroups per launch (max items)
  Clock::time_point t0;

  void* arena_base = nullptr;
  Arena arena;
  hipStream_t stream = nullptr;
  int* flag = nullptr;

  // device tables read by the graph, and their pinned staging (two sets)
  BatchJob* d_jobs = nullptr;
  LbfgsJob* d_ljobs = nullptr;
  int2* d_items = nullptr;
  int* d_nitems = nullptr;
  int* d_done = nullptr;
  BatchJob* h_jobs[2] = {nullptr, nullptr};
  LbfgsJob* h_ljobs[2] = {nullptr, nullptr};
  int2* h_items[2] = {nullptr, nullptr};
  int* h_nitems[2] = {nullptr, nullptr};
  int* h_done[2] = {nullptr, nullptr};
  hipEvent_t round_ev[2] = {nullptr, nullptr};

  // per-slot result staging
  LbfgsResult* d_fin = nullptr;
  LbfgsResult* h_fin = nullptr;
  double* h_fin_p0 = nullptr;
  std::vector<hipEvent_t> fin_ev;

  // host view of the slots
  std::vector<BatchJob> tab;
  std::vector<LbfgsJob> ltab;
  std::vector<ServerJob*> slot_job;   // running or finalizing job of each slot
  bool tables_dirty = true;

  hipGraphExec_t graph = nullptr;
  // Pair-kernel instances the graph launches per step: bit 0 for 3D jobs, bit 1
  // for planar jobs.  dims_seen grows as jobs of each kind are admitted; the
  // graph is captured again when it has grown (at most twice per server).
  int graph_dims = 0, dims_seen = 0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<ServerJob*> queue;
  std::unordered_map<int64_t, ServerJob*> jobs;
  int64_t next_id = 1;
  bool stop = false;
  bool failed = false;
  std::string err;
  std::thread worker;

  int64_t n_running = 0, n_completed = 0, rounds = 0, job_evals = 0;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

thread_local std::string g_serr;

lddmm_status sfail(lddmm_server* s, lddmm_status st, const std::string& msg) {
  if (s) {
    std::lock_guard<std::mutex> g(s->mu);
    s->err = msg;
  } else {
    g_serr = msg;
  }
  return st;
}

bool check_opts(const lddmm_solve_opts& o) {
  return o.max_iter >= 0 && o.m >= 1 && o.m <= kMaxHistory && o.max_fev >= 1 && o.c1 > 0.0 &&
         o.c1 < o.c2 && o.c2 < 1.0 && o.gtol >= 0.0 && o.ftol_rel >= 0.0 && o.init >= 0 &&
         o.init <= 2;
}

// Worker-side HIP error: the server stops accepting work and every pending
// job is reported as a device error.
void worker_fail(lddmm_server* s, hipError_t e, const char* what) {
  std::lock_guard<std::mutex> g(s->mu);
  s->failed = true;
  s->err = std::string(what) + ": " + hipGetErrorString(e);
  for (auto& kv : s->jobs) {
    ServerJob* j = kv.second;
    if (j->state != kDone) {
      j->state = kFailed;
      j->res.status = LDDMM_EDEVICE;
    }
  }
  s->cv_done.notify_all();
}

#define W_TRY(s, expr, what)                               \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) { worker_fail(s, e_, what); return false; } \
  } while (0)

// The same in a function that returns nothing.
#define W_TRY_V(s, expr, what)                             \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) { worker_fail(s, e_, what); return; } \
  } while (0)

// Puts a queued job into slot k: copies its inputs, centres them, and
// initialises its optimiser (all enqueued on the server stream).
bool admit(lddmm_server* s, ServerJob* j, int k) {
  const int n = j->p.n, T = s->cfg.T, mode = s->cfg.precision;
  const int spt = s->cfg.integrator == LDDMM_RK4 ? 4 : 1;
  const JobLayout L = job_layout(n, T, mode, j->o.m, spt);
  void* base = static_cast<char*>(s->arena_base) + j->off;
  const size_t m3 = 3 * (size_t)n;
  double* q0 = at<double>(base, L.q0);
  double* x = at<double>(base, L.x);
  double* vec = at<double>(base, L.vec);
  const Scales sc = make_scales(j->p.sigma, T);

  BatchJob b{};
  b.active = 1;
  b.n = n;
  b.nb = (n + 63) / 64;
  b.lambda = j->p.lambda;
  b.sc = sc;
  b.q0 = q0;
  b.cen = at<double>(base, L.cen);
  b.st = at<double>(base, L.st);
  b.ad = at<double>(base, L.ad);
  b.hp0 = at<double>(base, L.hp0);
  b.xc = at<double>(base, L.xc);
  b.h0p = at<double>(base, L.h0p);
  b.out3 = at<double>(base, L.out3);
  b.traj = at<void>(base, L.traj);
  b.arec = at<void>(base, L.arec);
  b.q1 = at<double>(base, L.q1);
  b.flag = s->flag;
  b.spt = spt;
  b.rk_acc = at<double>(base, L.rk_acc);
  b.rk_lam = at<double>(base, L.rk_lam);

  LbfgsJob lj{};
  lj.active = 1;
  LbfgsBufs& B = lj.B;
  B.m3 = (int)m3;
  B.x = vec; B.g = vec + m3; B.d = vec + 2 * m3; B.xt = vec + 3 * m3; B.gt = vec + 4 * m3;
  B.S = at<double>(base, L.hist);
  B.Y = B.S + (size_t)j->o.m * m3;
  B.ft = b.out3;
  B.trace = nullptr;
  B.q1t = b.q1;
  B.q1a = at<double>(base, L.q1a);
  B.out3a = at<double>(base, L.out3a);
  lj.state = at<LbfgsState>(base, L.state);
  lj.o = LbfgsOpts{j->o.max_iter, j->o.m, j->o.max_fev, j->o.gtol, j->o.ftol_rel, j->o.c1, j->o.c2};
  b.p0 = B.xt;
  b.grad = B.gt;
  b.done = &lj.state->done;

  hipStream_t st = s->stream;
  W_TRY(s, hipMemcpyAsync(q0, j->q0.data(), m3 * 8, hipMemcpyHostToDevice, st), "input copy");
  W_TRY(s, hipMemcpyAsync(x, j->x.data(), m3 * 8, hipMemcpyHostToDevice, st), "input copy");
  double* p_in = nullptr;
  if (j->o.init == 2) {
    p_in = B.gt;   // scratch until the first evaluation writes it
    W_TRY(s, hipMemcpyAsync(p_in, j->p0in.data(), m3 * 8, hipMemcpyHostToDevice, st), "p0 copy");
  }
  W_TRY(s, launch_centroid(q0, n, b.cen, st), "centroid");
  // centred target (the state and record it also writes are rewritten every round)
  W_TRY(s, launch_stage(mode, n, q0, q0, x, b.cen, sc.k, b.st, b.xc, b.traj, st), "stage");
  W_TRY(s, launch_lbfgs_init(B, lj.state, j->o.init, q0, x, p_in, T, st), "solver init");
  s->tab[k] = b;
  s->ltab[k] = lj;
  s->slot_job[k] = j;
  j->slot = k;
  j->x_dev = x;
  s->tables_dirty = true;
  return true;
}

bool upload_tables(lddmm_server* s, int parity) {
  const int M = s->cfg.max_slots;
  // items of 3D jobs first, then those of planar jobs (each group has its own
  // pair-kernel launch); within a group the largest jobs first, so their
  // i-blocks are dispatched first
  int ni = 0;
  for (int dim : {3, 2}) {
    std::vector<int> order;
    for (int k = 0; k < M; ++k)
      if (s->tab[k].active && (s->slot_job[k]->p.dim == 2 ? 2 : 3) == dim) order.push_back(k);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return s->tab[a].n > s->tab[b].n; });
    const int first = ni;
    for (int k : order)
      for (int ib = 0; ib < s->tab[k].nb; ++ib) s->h_items[parity][ni++] = make_int2(k, ib);
    s->h_nitems[parity][dim == 3 ? 0 : 1] = ni - first;
    if (ni > first) s->dims_seen |= dim == 3 ? 1 : 2;
  }
  std::memcpy(s->h_jobs[parity], s->tab.data(), sizeof(BatchJob) * M);
  std::memcpy(s->h_ljobs[parity], s->ltab.data(), sizeof(LbfgsJob) * M);
  hipStream_t st = s->stream;
  W_TRY(s, hipMemcpyAsync(s->d_jobs, s->h_jobs[parity], sizeof(BatchJob) * M,
                          hipMemcpyHostToDevice, st), "table copy");
  W_TRY(s, hipMemcpyAsync(s->d_ljobs, s->h_ljobs[parity], sizeof(LbfgsJob) * M,
                          hipMemcpyHostToDevice, st), "table copy");
  if (ni > 0)
    W_TRY(s, hipMemcpyAsync(s->d_items, s->h_items[parity], sizeof(int2) * ni,
                            hipMemcpyHostToDevice, st), "table copy");
  W_TRY(s, hipMemcpyAsync(s->d_nitems, s->h_nitems[parity], 2 * sizeof(int),
                          hipMemcpyHostToDevice, st), "table copy");
  s->tables_dirty = false;
  return true;
}

// One round as a graph: every running job does one evaluation and one step.
bool build_graph(lddmm_server* s) {
  const int mode = s->cfg.precision, T = s->cfg.T, M = s->cfg.max_slots;
  hipStream_t st = s->stream;
  W_TRY(s, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "capture");
  // stages: 0 (one Euler launch per step) or the Runge-Kutta stages 1..4
  const bool rk = s->cfg.integrator == LDDMM_RK4;
  const int s0 = rk ? 1 : 0, s1 = rk ? 4 : 0;
  const int dims = s->dims_seen;
  hipError_t e = launch_stage_batch(mode, s->d_jobs, M, s->cfg.max_n, st);
  for (int t = 0; t < T && e == hipSuccess; ++t)
    for (int k = s0; k <= s1 && e == hipSuccess; ++k)
      for (int d : {3, 2})
        if (e == hipSuccess && (dims & (d == 3 ? 1 : 2)))
          e = launch_fwd_batch(mode, d, s->d_jobs, s->d_items, s->d_nitems, s->capacity, t, k,
                               st);
  if (e == hipSuccess) e = launch_loss_batch(mode, s->d_jobs, M, st);
  for (int t = T - 1; t >= 0 && e == hipSuccess; --t)
    for (int k = s1; k >= s0 && e == hipSuccess; --k)
      for (int d : {3, 2})
        if (e == hipSuccess && (dims & (d == 3 ? 1 : 2)))
          e = launch_adj_batch(mode, d, s->d_jobs, s->d_items, s->d_nitems, s->capacity, t, k,
                               T, st);
  if (e == hipSuccess) e = launch_lbfgs_step_batch(s->d_ljobs, M, st);
  if (e == hipSuccess) e = launch_gather_done(s->d_ljobs, M, s->d_done, st);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(st, &g);
  if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); worker_fail(s, e, "graph capture"); return false; }
  if (e2 != hipSuccess) { worker_fail(s, e2, "graph capture"); return false; }
  e = hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) { worker_fail(s, e, "graph instantiate"); return false; }
  s->graph_dims = dims;
  return true;
}

// Enqueue the result copies of a finished job and release its memory.
bool finalize(lddmm_server* s, int k) {
  ServerJob* j = s->slot_job[k];
  const LbfgsJob& lj = s->ltab[k];
  const int n = j->p.n;
  hipStream_t st = s->stream;
  W_TRY(s, launch_lbfgs_result(n, lj.B.q1a, j->x_dev, lj.B.out3a, lj.state, s->d_fin + k, st),
        "result");
  W_TRY(s, hipMemcpyAsync(s->h_fin_p0 + (size_t)k * 3 * s->cfg.max_n, lj.B.x, 3 * (size_t)n * 8,
                          hipMemcpyDeviceToHost, st), "result copy");
  W_TRY(s, hipMemcpyAsync(s->h_fin + k, s->d_fin + k, sizeof(LbfgsResult), hipMemcpyDeviceToHost,
                          st), "result copy");
  W_TRY(s, hipEventRecord(s->fin_ev[k], st), "result event");
  std::lock_guard<std::mutex> g(s->mu);
  j->state = kFinalizing;
  s->tab[k].active = 0;
  s->ltab[k].active = 0;
  s->tables_dirty = true;
  // later users of this memory are ordered after the copies on the stream
  s->arena.release(j->off);
  j->off = Arena::npos;
  --s->n_running;
  return true;
}

// Jobs whose result copies have landed become visible to poll().
void collect(lddmm_server* s, bool block) {
  for (int k = 0; k < s->cfg.max_slots; ++k) {
    ServerJob* j = s->slot_job[k];
    if (!j || j->state != kFinalizing) continue;
    hipError_t q = block ? hipEventSynchronize(s->fin_ev[k]) : hipEventQuery(s->fin_ev[k]);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) { worker_fail(s, q, "result event"); return; }
    const LbfgsResult& r = s->h_fin[k];
    std::lock_guard<std::mutex> g(s->mu);
    j->p0out.assign(s->h_fin_p0 + (size_t)k * 3 * s->cfg.max_n,
                    s->h_fin_p0 + (size_t)k * 3 * s->cfg.max_n + 3 * (size_t)j->p.n);
    j->res.loss = r.loss;
    j->res.H0 = r.H0;
    j->res.mismatch = r.mismatch;
    j->res.grad_norm = r.grad_norm;
    j->res.avg_dist = r.avg_dist;
    j->res.max_dist = r.max_dist;
    j->res.iters = r.iters;
    j->res.fevals = r.fevals;
    j->res.status = r.status == kConverged ? LDDMM_OK
                    : r.status == kNonFinite ? LDDMM_ENONFINITE : LDDMM_ENOTCONV;
    j->t_done = s->now();
    j->state = kDone;
    s->slot_job[k] = nullptr;
    ++s->n_completed;
    s->cv_done.notify_all();
  }
}

void worker_main(lddmm_server* s) {
  if (hipSetDevice(s->cfg.device) != hipSuccess) {
    worker_fail(s, hipErrorInvalidDevice, "device");
    return;
  }
  const int M = s->cfg.max_slots;
  int64_t r = 0;          // rounds launched
  bool pending = false;   // the done flags of round r-1 are not read yet
  for (;;) {
    // ---- admission: first come, first served; the head waits until it fits
    std::vector<std::pair<ServerJob*, int>> admitted;
    {
      std::unique_lock<std::mutex> g(s->mu);
      if (s->stop || s->failed) break;
      while (!s->queue.empty()) {
        int k = -1;
        for (int c = 0; c < M; ++c)
          if (!s->slot_job[c]) { k = c; break; }
        if (k < 0) break;
        ServerJob* j = s->queue.front();
        const size_t off = s->arena.alloc(j->footprint);
        if (off == Arena::npos) break;
        s->queue.pop_front();
        j->off = off;
        j->state = kRunning;
        j->t_admit = s->now();
        j->first_round = r;
        s->slot_job[k] = j;   // reserved; filled in by admit()
        ++s->n_running;
        admitted.emplace_back(j, k);
      }
      bool busy = s->n_running > 0 || pending;
      for (int k = 0; k < M && !busy; ++k) busy = s->slot_job[k] != nullptr;
      if (!busy) {
        s->cv_work.wait_for(g, std::chrono::milliseconds(20));
        continue;
      }
    }
    for (auto& jk : admitted)
      if (!admit(s, jk.first, jk.second)) return;

    // ---- one round for every running job
    bool launched = false;
    if (s->n_running > 0) {
      const int par = (int)(r & 1);
      if (s->tables_dirty && !upload_tables(s, par)) return;
      if (s->graph && s->graph_dims != s->dims_seen) {
        // a job of a new kind: capture a graph that also launches its pair kernels
        // (the old one may still run: wait for it before destroying it)
        W_TRY_V(s, hipStreamSynchronize(s->stream), "graph rebuild");
        (void)hipGraphExecDestroy(s->graph);
        s->graph = nullptr;
      }
      if (!s->graph && !build_graph(s)) return;
      hipError_t e = hipGraphLaunch(s->graph, s->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(s->h_done[par], s->d_done, sizeof(int) * M, hipMemcpyDeviceToHost,
                           s->stream);
      if (e == hipSuccess) e = hipEventRecord(s->round_ev[par], s->stream);
      if (e != hipSuccess) { worker_fail(s, e, "round"); return; }
      std::lock_guard<std::mutex> g(s->mu);
      ++s->rounds;
      s->job_evals += s->n_running;
      launched = true;
    }
    // ---- finished jobs of the previous round (the next one is already queued)
    if (pending) {
      const int pp = (int)((r - 1) & 1);
      const hipError_t e = hipEventSynchronize(s->round_ev[pp]);
      if (e != hipSuccess) { worker_fail(s, e, "round wait"); return; }
      for (int k = 0; k < M; ++k) {
        // a flag of round r-1 belongs to the slot's job only if it was in that round
        ServerJob* j = s->slot_job[k];
        if (j && j->state == kRunning && j->first_round <= r - 1 && s->h_done[pp][k] &&
            !finalize(s, k))
          return;
      }
    }
    pending = launched;
    if (launched) ++r;
    collect(s, !launched);
  }
  (void)hipStreamSynchronize(s->stream);
}

}  // namespace

extern "C" {

lddmm_status lddmm_server_job_footprint(const lddmm_server_config* cfg, int32_t n, int32_t m,
                                        size_t* bytes) {
  if (!cfg || !bytes || n < 1 || n > (1 << 26) || m < 1 || m > kMaxHistory || cfg->T < 1 ||
      cfg->T > (1 << 20) ||
      cfg->precision < LDDMM_FP32 || cfg->precision > LDDMM_FP64 ||
      (cfg->integrator != LDDMM_EULER && cfg->integrator != LDDMM_RK4))
    return sfail(nullptr, LDDMM_EINVAL, "invalid footprint query");
  *bytes = job_layout(n, cfg->T, cfg->precision, m, cfg->integrator == LDDMM_RK4 ? 4 : 1).total;
  return LDDMM_OK;
}

lddmm_status lddmm_server_create(const lddmm_server_config* cfg, lddmm_server** out) {
  if (!cfg || !out) return sfail(nullptr, LDDMM_EINVAL, "cfg and out must not be NULL");
  *out = nullptr;
  if (cfg->max_slots < 1 || cfg->max_slots > 1024 || cfg->max_n < 1 || cfg->max_n > (1 << 20) ||
      cfg->T < 1 || cfg->T > (1 << 20) || cfg->precision < LDDMM_FP32 ||
      cfg->precision > LDDMM_FP64 ||
      (cfg->integrator != LDDMM_EULER && cfg->integrator != LDDMM_RK4) ||
      cfg->hbm_budget_bytes < 4096)
    return sfail(nullptr, LDDMM_EINVAL, "invalid server configuration");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || cfg->device < 0 || cfg->device >= count)
    return sfail(nullptr, LDDMM_EINVAL, "invalid device");
  if (hipSetDevice(cfg->device) != hipSuccess) return sfail(nullptr, LDDMM_EDEVICE, "hipSetDevice");
  lddmm_server* s = new (std::nothrow) lddmm_server;
  if (!s) return sfail(nullptr, LDDMM_ENOMEM, "host allocation");
  s->cfg = *cfg;
  s->t0 = Clock::now();
  const int M = cfg->max_slots;
  s->capacity = M * ((cfg->max_n + 63) / 64);
  s->tab.assign(M, BatchJob{});
  s->ltab.assign(M, LbfgsJob{});
  s->slot_job.assign(M, nullptr);
  s->fin_ev.assign(M, nullptr);
  hipError_t e = hipMalloc(&s->arena_base, cfg->hbm_budget_bytes);
  if (e == hipSuccess) s->arena.reset(cfg->hbm_budget_bytes);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&s->flag, 256);
  if (e == hipSuccess) e = hipMemset(s->flag, 0, 256);
  if (e == hipSuccess) e = hipMalloc(&s->d_jobs, sizeof(BatchJob) * M);
  if (e == hipSuccess) e = hipMalloc(&s->d_ljobs, sizeof(LbfgsJob) * M);
  if (e == hipSuccess) e = hipMalloc(&s->d_items, sizeof(int2) * s->capacity);
  if (e == hipSuccess) e = hipMalloc(&s->d_nitems, sizeof(int) * 64);
  if (e == hipSuccess) e = hipMalloc(&s->d_done, sizeof(int) * M);
  if (e == hipSuccess) e = hipMalloc(&s->d_fin, sizeof(LbfgsResult) * M);
  for (int p = 0; p < 2 && e == hipSuccess; ++p) {
    e = hipHostMalloc(&s->h_jobs[p], sizeof(BatchJob) * M, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&s->h_ljobs[p], sizeof(LbfgsJob) * M, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&s->h_items[p], sizeof(int2) * s->capacity, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&s->h_nitems[p], 64, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&s->h_done[p], sizeof(int) * M, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->round_ev[p], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipHostMalloc(&s->h_fin, sizeof(LbfgsResult) * M, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc(&s->h_fin_p0, sizeof(double) * 3 * (size_t)cfg->max_n * M, hipHostMallocDefault);
  for (int k = 0; k < M && e == hipSuccess; ++k)
    e = hipEventCreateWithFlags(&s->fin_ev[k], hipEventDisableTiming);
  if (e == hipSuccess) {
    // empty tables until the first admission
    e = hipMemsetAsync(s->d_jobs, 0, sizeof(BatchJob) * M, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_ljobs, 0, sizeof(LbfgsJob) * M, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_nitems, 0, 2 * sizeof(int), s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  }
  if (e != hipSuccess) {
    const std::string m = std::string("server allocation: ") + hipGetErrorString(e);
    lddmm_server_destroy(s);
    return sfail(nullptr, e == hipErrorOutOfMemory ? LDDMM_ENOMEM : LDDMM_EDEVICE, m);
  }
  try {
    s->worker = std::thread(worker_main, s);
  } catch (...) {
    lddmm_server_destroy(s);
    return sfail(nullptr, LDDMM_ENOMEM, "worker thread");
  }
  *out = s;
  return LDDMM_OK;
}

lddmm_status lddmm_server_submit(lddmm_server* s, const lddmm_params* p,
                                 const lddmm_solve_opts* o, const double* q0,
                                 const double* target, const double* p0, int64_t* job_id) {
  if (!s || !p || !o || !q0 || !target || !job_id)
    return sfail(s, LDDMM_EINVAL, "NULL argument");
  if (p->n < 1 || p->n > s->cfg.max_n)
    return sfail(s, LDDMM_EINVAL, "n must be in 1..max_n");
  if (p->T != s->cfg.T || p->precision != s->cfg.precision)
    return sfail(s, LDDMM_EINVAL, "T and precision must match the server's");
  if (p->energy != LDDMM_ENERGY_INITIAL)
    return sfail(s, LDDMM_EINVAL, "the server takes the energy term at t = 0 only");
  if (p->dim != 0 && p->dim != 2 && p->dim != 3)
    return sfail(s, LDDMM_EINVAL, "dim must be 2 or 3");
  if (p->integrator != s->cfg.integrator)
    return sfail(s, LDDMM_EINVAL, "the integrator must match the server's");
  if (!(p->sigma > 0.0) || !(p->lambda >= 0.0) || !std::isfinite(p->sigma) ||
      !std::isfinite(p->lambda))
    return sfail(s, LDDMM_EINVAL, "sigma must be > 0 and lambda >= 0");
  if (!check_opts(*o)) return sfail(s, LDDMM_EINVAL, "invalid solver options");
  if (o->init == 2 && !p0) return sfail(s, LDDMM_EINVAL, "init 2 needs p0");
  ServerJob* j = new (std::nothrow) ServerJob;
  if (!j) return sfail(s, LDDMM_ENOMEM, "host allocation");
  const size_t m3 = 3 * (size_t)p->n;
  j->p = *p;
  j->o = *o;
  j->q0.assign(q0, q0 + m3);
  j->x.assign(target, target + m3);
  if (o->init == 2) j->p0in.assign(p0, p0 + m3);
  j->footprint =
      job_layout(p->n, p->T, p->precision, o->m, p->integrator == LDDMM_RK4 ? 4 : 1).total;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->failed) { delete j; return LDDMM_EDEVICE; }
  if (Arena::round_up(j->footprint) > s->arena.size()) {
    delete j;
    s->err = "job footprint exceeds the server's HBM budget";
    return LDDMM_ENOMEM;
  }
  j->id = s->next_id++;
  j->t_submit = s->now();
  s->jobs[j->id] = j;
  s->queue.push_back(j);
  *job_id = j->id;
  s->cv_work.notify_one();
  return LDDMM_OK;
}

lddmm_status lddmm_server_poll(lddmm_server* s, int64_t job_id, double* p0_out,
                               lddmm_solve_result* result, lddmm_job_times* times) {
  if (!s) return sfail(nullptr, LDDMM_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) { s->err = "unknown job id"; return LDDMM_EINVAL; }
  ServerJob* j = it->second;
  if (j->state == kFailed) return LDDMM_EDEVICE;
  if (j->state != kDone) return LDDMM_EBUSY;
  if (p0_out) std::memcpy(p0_out, j->p0out.data(), j->p0out.size() * sizeof(double));
  if (result) *result = j->res;
  if (times) {
    times->submit_s = j->t_submit;
    times->admit_s = j->t_admit;
    times->done_s = j->t_done;
  }
  const lddmm_status st = (lddmm_status)j->res.status;
  s->jobs.erase(it);
  delete j;
  return st;
}

lddmm_status lddmm_server_wait(lddmm_server* s, int64_t job_id, double timeout_s) {
  if (!s) return sfail(nullptr, LDDMM_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> g(s->mu);
  auto ready = [&] {
    auto it = s->jobs.find(job_id);
    return it == s->jobs.end() || it->second->state == kDone || it->second->state == kFailed;
  };
  if (timeout_s < 0) s->cv_done.wait(g, ready);
  else if (!s->cv_done.wait_for(g, std::chrono::duration<double>(timeout_s), ready))
    return LDDMM_EBUSY;
  if (s->jobs.find(job_id) == s->jobs.end()) return LDDMM_EINVAL;
  return LDDMM_OK;
}

lddmm_status lddmm_server_stats_get(lddmm_server* s, lddmm_server_stats* out) {
  if (!s || !out) return sfail(s, LDDMM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  out->queued = (int64_t)s->queue.size();
  out->running = s->n_running;
  out->completed = s->n_completed;
  out->rounds = s->rounds;
  out->job_evaluations = s->job_evals;
  out->hbm_used_bytes = s->arena.used_bytes();
  out->hbm_budget_bytes = s->arena.size();
  return LDDMM_OK;
}

const char* lddmm_server_last_error(lddmm_server* s) {
  if (!s) return g_serr.c_str();
  std::lock_guard<std::mutex> g(s->mu);
  thread_local std::string copy;
  copy = s->err;
  return copy.c_str();
}

lddmm_status lddmm_server_destroy(lddmm_server* s) {
  if (!s) return LDDMM_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->cfg.device);
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->graph) (void)hipGraphExecDestroy(s->graph);
  for (auto& kv : s->jobs) delete kv.second;
  s->jobs.clear();
  for (int p = 0; p < 2; ++p) {
    if (s->h_jobs[p]) (void)hipHostFree(s->h_jobs[p]);
    if (s->h_ljobs[p]) (void)hipHostFree(s->h_ljobs[p]);
    if (s->h_items[p]) (void)hipHostFree(s->h_items[p]);
    if (s->h_nitems[p]) (void)hipHostFree(s->h_nitems[p]);
    if (s->h_done[p]) (void)hipHostFree(s->h_done[p]);
    if (s->round_ev[p]) (void)hipEventDestroy(s->round_ev[p]);
  }
  for (hipEvent_t e : s->fin_ev)
    if (e) (void)hipEventDestroy(e);
  if (s->h_fin) (void)hipHostFree(s->h_fin);
  if (s->h_fin_p0) (void)hipHostFree(s->h_fin_p0);
  for (void* p : {(void*)s->d_jobs, (void*)s->d_ljobs, (void*)s->d_items, (void*)s->d_nitems,
                  (void*)s->d_done, (void*)s->d_fin, (void*)s->flag, s->arena_base})
    if (p) (void)hipFree(p);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return LDDMM_OK;
}

}  // extern "C"
