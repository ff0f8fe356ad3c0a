// HIP kernels for landmark geodesic shooting on gfx950 (CDNA4).
//
// The hot path is the all-pairs Gaussian-kernel sums of one explicit Euler
// step of the Hamiltonian flow (eq. 2 with H = 1/2 <p, K(q) p>, eq. 1) and of
// its exact discrete adjoint, which together give dL/dp0 for the loss of
// eq. 3.  The paper streams pair terms through on-chip memory instead of
// materialising the N x N kernel matrix (Sec. 2.5); this file keeps that idea
// and re-plans it for wave64 hardware:
//
//  * Lane l of a wave owns landmark i = 64 ib + l and keeps its data and its
//    running sums in VGPRs.  The j landmarks are wave-uniform, so their
//    records arrive through scalar loads into SGPRs and every VALU
//    instruction of the pair term reads at most one SGPR operand; there is no
//    LDS traffic and no barrier inside the j loop.
//  * Coordinates are stored pre-scaled by k = sqrt(log2(e) / (2 sigma^2)), so
//    g_ij = exp2(-|k q_i - k q_j|^2) is one v_exp_f32 with a negate modifier.
//    A forward pair costs 16 VALU + 1 exp, an adjoint pair 37 VALU + 1 exp.
//  * The j range is split over the W waves of a workgroup and, when one
//    workgroup per i-block would not fill the chip, over S workgroups.
//    Partials are combined in a fixed order (waves through LDS, workgroups
//    through a [S][C][N] buffer): no float atomics, so results are
//    bit-reproducible and depend only on N, never on what else is running.
//  * Precision modes: FP32 with one running FP32 sum per wave ("naive");
//    FP32 with per-64-pair FP32 tile sums folded into FP64 ("compensated");
//    or everything in FP64.  The live state (q, p, a, b), the Euler updates,
//    the Hamiltonian and the loss are FP64 in every mode.
#include "shoot_internal.h"

#include <cstdlib>
#include <type_traits>

namespace lddmm {

namespace {

constexpr int kTile = 64;               // pairs per FP32 tile in compensated mode
constexpr int kLossThreads = 1024;

// Point record: (k q, 0, p, 0) for the trajectory, (a, 0, b_hat, 0) for the
// adjoint.  Eight scalars so that one record is one 32-byte (FP32) or
// 64-byte (FP64) scalar load.
template <typename R>
struct alignas(8 * sizeof(R)) Rec {
  R x, y, z, u, px, py, pz, w;
};

// Pointers that arrive through a descriptor in memory carry no address
// space; the pair loops read records through a global (address space 1)
// pointer so that wave-uniform loads can become scalar loads.
template <typename T>
using GlobalPtr = const __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ GlobalPtr<T> global_ptr(const T* p) {
  return (GlobalPtr<T>)p;
}

template <typename R, bool COMP>
struct AccOf { using type = double; };

template <typename R>
struct Rec;

// Record j as one 8-wide vector load (an address-space-qualified struct
// cannot be copied as a whole): a wave-uniform j gives one s_load_dwordx8
// (FP32) or s_load_dwordx16 (FP64) that the compiler issues ahead of use.
template <typename R>
using Vec8 = R __attribute__((ext_vector_type(8)));

template <typename R>
__device__ __forceinline__ Rec<R> load_rec(GlobalPtr<Rec<R>> p, int j) {
  const Vec8<R> v = *reinterpret_cast<GlobalPtr<Vec8<R>>>(p + j);
  Rec<R> r;
  r.x = v[0]; r.y = v[1]; r.z = v[2]; r.u = v[3];
  r.px = v[4]; r.py = v[5]; r.pz = v[6]; r.w = v[7];
  return r;
}
template <>
struct AccOf<float, false> { using type = float; };

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double ex2(double x) { return exp2(x); }

template <typename R>
__device__ __forceinline__ Rec<R> make_rec(double x, double y, double z, double a, double b,
                                           double c) {
  Rec<R> r;
  r.x = (R)x; r.y = (R)y; r.z = (R)z; r.u = (R)0;
  r.px = (R)a; r.py = (R)b; r.pz = (R)c; r.w = (R)0;
  return r;
}

// ---------------------------------------------------------------------------
// forward pair sums over j in [j0, j1) for the lane's landmark i:
//   h[0..2] += sum_j g_ij p_j                      (Hp)
//   h[3..5] += sum_j g_ij (p_i . p_j) (kq_i - kq_j)  (Hq up to the factor -c/k)
// D = 2 is the planar specialisation: the z terms are left out (every z is 0
// there), which leaves 11 VALU + 1 exp per pair.  On planar data the two
// forms give bitwise the same sums: each z term the 3D loop adds is an exact 0.
// ---------------------------------------------------------------------------
template <typename R, int D>
__device__ __forceinline__ void fwd_range(const Rec<R>* __restrict__ Xp, const Rec<R>& ri, int j0,
                                          int j1, R h[6]) {
  const GlobalPtr<Rec<R>> X = global_ptr(Xp);
  R hp0 = h[0], hp1 = h[1], hp2 = h[2], hq0 = h[3], hq1 = h[4], hq2 = h[5];
#pragma unroll 4
  for (int j = j0; j < j1; ++j) {
    const Rec<R> rj = load_rec<R>(X, j);
    const R dx = ri.x - rj.x, dy = ri.y - rj.y;
    R r2 = dx * dx;
    r2 = fma(dy, dy, r2);
    R dz = (R)0;
    if constexpr (D == 3) {
      dz = ri.z - rj.z;
      r2 = fma(dz, dz, r2);
    }
    const R g = ex2(-r2);
    hp0 = fma(g, rj.px, hp0);
    hp1 = fma(g, rj.py, hp1);
    if constexpr (D == 3) hp2 = fma(g, rj.pz, hp2);
    R s = ri.px * rj.px;
    s = fma(ri.py, rj.py, s);
    if constexpr (D == 3) s = fma(ri.pz, rj.pz, s);
    const R gs = g * s;
    hq0 = fma(gs, dx, hq0);
    hq1 = fma(gs, dy, hq1);
    if constexpr (D == 3) hq2 = fma(gs, dz, hq2);
  }
  h[0] = hp0; h[1] = hp1; h[2] = hp2; h[3] = hq0; h[4] = hq1; h[5] = hq2;
}

// ---------------------------------------------------------------------------
// adjoint pair sums over j in [j0, j1).  With D = kq_i - kq_j, db = b^_i - b^_j
// (b^ = kappa k b), e = D.db, s = p_i.p_j, pi = a_i.p_j + p_i.a_j:
//   h[0..2] += sum_j g s db                (A1)
//   h[3..5] += sum_j g (pi + s e) D        (A2)
//   h[6..8] += sum_j g (a_j + e p_j)       (B)
// and A = (c/k)(A1/kappa - A2).
// ---------------------------------------------------------------------------
template <typename R, int D>
__device__ __forceinline__ void adj_range(const Rec<R>* __restrict__ Xp,
                                          const Rec<R>* __restrict__ Yp, const Rec<R>& ri,
                                          const Rec<R>& yi, int j0, int j1, R h[9]) {
  const GlobalPtr<Rec<R>> X = global_ptr(Xp);
  const GlobalPtr<Rec<R>> Y = global_ptr(Yp);
  R a10 = h[0], a11 = h[1], a12 = h[2], a20 = h[3], a21 = h[4], a22 = h[5];
  R b0 = h[6], b1 = h[7], b2 = h[8];
  constexpr bool Z = D == 3;   // planar (D = 2): the z terms are all 0 and left out
#pragma unroll 2
  for (int j = j0; j < j1; ++j) {
    const Rec<R> rj = load_rec<R>(X, j);
    const Rec<R> yj = load_rec<R>(Y, j);
    const R dx = ri.x - rj.x, dy = ri.y - rj.y;
    const R dz = Z ? ri.z - rj.z : (R)0;
    R r2 = dx * dx;
    r2 = fma(dy, dy, r2);
    if constexpr (Z) r2 = fma(dz, dz, r2);
    const R g = ex2(-r2);
    const R ex = yi.px - yj.px, ey = yi.py - yj.py;
    const R ez = Z ? yi.pz - yj.pz : (R)0;
    R e = dx * ex;
    e = fma(dy, ey, e);
    if constexpr (Z) e = fma(dz, ez, e);
    R s = ri.px * rj.px;
    s = fma(ri.py, rj.py, s);
    if constexpr (Z) s = fma(ri.pz, rj.pz, s);
    R pi = yi.x * rj.px;
    pi = fma(yi.y, rj.py, pi);
    if constexpr (Z) pi = fma(yi.z, rj.pz, pi);
    pi = fma(ri.px, yj.x, pi);
    pi = fma(ri.py, yj.y, pi);
    if constexpr (Z) pi = fma(ri.pz, yj.z, pi);
    const R gs = g * s;
    const R v = g * fma(s, e, pi);
    a10 = fma(gs, ex, a10);
    a11 = fma(gs, ey, a11);
    if constexpr (Z) a12 = fma(gs, ez, a12);
    a20 = fma(v, dx, a20);
    a21 = fma(v, dy, a21);
    if constexpr (Z) a22 = fma(v, dz, a22);
    const R ge = g * e;
    b0 = fma(g, yj.x, b0);
    b1 = fma(g, yj.y, b1);
    if constexpr (Z) b2 = fma(g, yj.z, b2);
    b0 = fma(ge, rj.px, b0);
    b1 = fma(ge, rj.py, b1);
    if constexpr (Z) b2 = fma(ge, rj.pz, b2);
  }
  h[0] = a10; h[1] = a11; h[2] = a12; h[3] = a20; h[4] = a21; h[5] = a22;
  h[6] = b0; h[7] = b1; h[8] = b2;
}

// One wave's share of the j range, in the precision of the mode.
template <typename R, bool COMP, int NC, typename F>
__device__ __forceinline__ void wave_sums(int j0, int j1, typename AccOf<R, COMP>::type o[NC],
                                          F&& range) {
  if constexpr (std::is_same<R, float>::value && COMP) {
    for (int c = 0; c < NC; ++c) o[c] = 0.0;
    for (int t0 = j0; t0 < j1; t0 += kTile) {
      float h[NC];
      for (int c = 0; c < NC; ++c) h[c] = 0.0f;
      range(t0, min(j1, t0 + kTile), h);
      for (int c = 0; c < NC; ++c) o[c] += (double)h[c];
    }
  } else {
    R h[NC];
    for (int c = 0; c < NC; ++c) h[c] = (R)0;
    range(j0, j1, h);
    for (int c = 0; c < NC; ++c) o[c] = h[c];
  }
}

// Combine the W waves' sums of a workgroup in wave order; afterwards red[c*64+l]
// holds the workgroup's sum of component c for lane l.
template <typename Acc, int NC, int W>
__device__ __forceinline__ void block_combine(Acc* red, const Acc o[NC], int w, int lane) {
  for (int c = 0; c < NC; ++c) red[(w * NC + c) * 64 + lane] = o[c];
  __syncthreads();
  for (int idx = threadIdx.x; idx < NC * 64; idx += 64 * W) {
    Acc sum = red[idx];
    for (int v = 1; v < W; ++v) sum += red[v * NC * 64 + idx];
    red[idx] = sum;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// per-landmark Euler updates (FP64), shared by the fused and the split path
// ---------------------------------------------------------------------------
// FP64 state of one landmark, loaded before the sums it is combined with so
// that its memory latency overlaps them.
struct FwdState { double q[3], p[3]; };
struct AdjState { double a[3], b[3], hp0[3], hq0[3]; };

__device__ __forceinline__ FwdState load_fwd_state(const FwdArgs& A, int i) {
  FwdState v;
  const int ic = min(i, A.n - 1);
  for (int c = 0; c < 3; ++c) { v.q[c] = A.st[c * A.n + ic]; v.p[c] = A.st[(3 + c) * A.n + ic]; }
  return v;
}

__device__ __forceinline__ AdjState load_adj_state(const AdjArgs& A, int i) {
  AdjState v;
  const int ic = min(i, A.n - 1);
  for (int c = 0; c < 3; ++c) {
    v.a[c] = A.ad[c * A.n + ic];
    v.b[c] = A.ad[(3 + c) * A.n + ic];
    v.hp0[c] = (A.grad && A.hp0) ? A.hp0[c * A.n + ic] : 0.0;
    v.hq0[c] = (A.grad_q0 && A.hq0) ? A.hq0[c * A.n + ic] : 0.0;
  }
  return v;
}

template <typename R>
__device__ __forceinline__ void fwd_finish(const FwdArgs& A, int ib, int lane, FwdState v,
                                           const double hp[3], const double hqs[3]) {
  const int n = A.n;
  const int i = ib * 64 + lane;
  double h0 = 0.0;
  if (i < n) {
    if (A.hp0) {
      for (int c = 0; c < 3; ++c) A.hp0[c * n + i] = hp[c];
      h0 = v.p[0] * hp[0] + v.p[1] * hp[1] + v.p[2] * hp[2];
    }
    for (int c = 0; c < 3; ++c) {
      const double hq = A.sc.hq * hqs[c];
      if (A.hq0) A.hq0[c * n + i] = hq;
      v.q[c] = v.q[c] + A.sc.dt * hp[c];
      v.p[c] = v.p[c] - A.sc.dt * hq;
    }
    for (int c = 0; c < 3; ++c) { A.st[c * n + i] = v.q[c]; A.st[(3 + c) * n + i] = v.p[c]; }
    if (A.ckpt)
      for (int c = 0; c < 3; ++c) { A.ckpt[c * n + i] = v.q[c]; A.ckpt[(3 + c) * n + i] = v.p[c]; }
    const double k = A.sc.k;
    static_cast<Rec<R>*>(A.rec_t1)[i] =
        make_rec<R>(k * v.q[0], k * v.q[1], k * v.q[2], v.p[0], v.p[1], v.p[2]);
  }
  if (A.h0_part) {          // whole wave takes part: fixed butterfly order
    for (int off = 32; off > 0; off >>= 1) h0 += __shfl_xor(h0, off, 64);
    if (lane == 0) A.h0_part[ib] = h0;
  }
}

template <typename R>
__device__ __forceinline__ void adj_finish(const AdjArgs& A, int ib, int lane, AdjState v,
                                           const double s[9]) {
  const int n = A.n;
  const int i = ib * 64 + lane;
  if (i >= n) return;
  const double inv_kappa = 1.0 / A.sc.kappa;
  for (int c = 0; c < 3; ++c) {
    const double Ac = A.sc.adj_a * (s[c] * inv_kappa - s[3 + c]);
    v.a[c] = v.a[c] + A.sc.dt * Ac;
    v.b[c] = v.b[c] + A.sc.dt * s[6 + c];
  }
  for (int c = 0; c < 3; ++c) { A.ad[c * n + i] = v.a[c]; A.ad[(3 + c) * n + i] = v.b[c]; }
  const double bs = A.sc.bscale;
  static_cast<Rec<R>*>(A.arec_next)[i] =
      make_rec<R>(v.a[0], v.a[1], v.a[2], bs * v.b[0], bs * v.b[1], bs * v.b[2]);
  if (A.grad)
    for (int c = 0; c < 3; ++c) A.grad[3 * i + c] = v.b[c] + v.hp0[c];
  if (A.grad_q0)
    for (int c = 0; c < 3; ++c) A.grad_q0[3 * i + c] = v.a[c] + v.hq0[c];
}

// ---------------------------------------------------------------------------
// pair kernels
// ---------------------------------------------------------------------------
// One workgroup's share of a pair-sum step: i-block ib (64 landmarks, one
// per lane) against j-chunk s, split over the W waves.  With S == 1 the sums
// are final and wave 0 applies the Euler update; otherwise the workgroup
// writes its partial for the combine kernel.  red: W*C*64 accumulators of LDS.
template <typename R, bool COMP, int W, int D>
__device__ __forceinline__ void fwd_block(const FwdArgs& A, int ib, int s,
                                          typename AccOf<R, COMP>::type* red) {
  using Acc = typename AccOf<R, COMP>::type;
  constexpr int NC = 6;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const Rec<R>* __restrict__ X = static_cast<const Rec<R>*>(A.rec_t);
  const Rec<R> ri = X[min(ib * 64 + lane, A.n - 1)];
  const int jb = s * A.chunk;
  const int je = min(A.n, jb + A.chunk);
  const int j0 = min(je, jb + w * A.wchunk);
  const int j1 = min(je, j0 + A.wchunk);
  FwdState v{};
  if (A.S == 1 && w == 0) v = load_fwd_state(A, ib * 64 + lane);
  Acc o[NC];
  wave_sums<R, COMP, NC>(j0, j1, o,
                         [&](int a, int b, auto* h) { fwd_range<R, D>(X, ri, a, b, h); });
  block_combine<Acc, NC, W>(red, o, w, lane);
  if (A.S == 1) {
    if (w == 0) {
      double h[NC];
      for (int c = 0; c < NC; ++c) h[c] = red[c * 64 + lane];
      fwd_finish<R>(A, ib, lane, v, h, h + 3);
    }
  } else {
    Acc* P = static_cast<Acc*>(A.partial);
    for (int idx = threadIdx.x; idx < NC * 64; idx += 64 * W) {
      const int c = idx >> 6, i = ib * 64 + (idx & 63);
      if (i < A.n) P[((size_t)s * NC + c) * A.n + i] = red[idx];
    }
  }
}

template <typename R, bool COMP, int W, int D>
__device__ __forceinline__ void adj_block(const AdjArgs& A, int ib, int s,
                                          typename AccOf<R, COMP>::type* red) {
  using Acc = typename AccOf<R, COMP>::type;
  constexpr int NC = 9;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const Rec<R>* __restrict__ X = static_cast<const Rec<R>*>(A.rec_t);
  const Rec<R>* __restrict__ Y = static_cast<const Rec<R>*>(A.arec);
  const int ic = min(ib * 64 + lane, A.n - 1);
  const Rec<R> ri = X[ic];
  const Rec<R> yi = Y[ic];
  const int jb = s * A.chunk;
  const int je = min(A.n, jb + A.chunk);
  const int j0 = min(je, jb + w * A.wchunk);
  const int j1 = min(je, j0 + A.wchunk);
  AdjState v{};
  if (A.S == 1 && w == 0) v = load_adj_state(A, ib * 64 + lane);
  Acc o[NC];
  wave_sums<R, COMP, NC>(j0, j1, o,
                         [&](int a, int b, auto* h) { adj_range<R, D>(X, Y, ri, yi, a, b, h); });
  block_combine<Acc, NC, W>(red, o, w, lane);
  if (A.S == 1) {
    if (w == 0) {
      double h[NC];
      for (int c = 0; c < NC; ++c) h[c] = red[c * 64 + lane];
      adj_finish<R>(A, ib, lane, v, h);
    }
  } else {
    Acc* P = static_cast<Acc*>(A.partial);
    for (int idx = threadIdx.x; idx < NC * 64; idx += 64 * W) {
      const int c = idx >> 6, i = ib * 64 + (idx & 63);
      if (i < A.n) P[((size_t)s * NC + c) * A.n + i] = red[idx];
    }
  }
}

template <typename R, bool COMP, int W, int D>
__global__ __launch_bounds__(64 * W) void k_fwd(FwdArgs A) {
  __shared__ typename AccOf<R, COMP>::type red[W * 6 * 64];
  fwd_block<R, COMP, W, D>(A, blockIdx.x / A.S, blockIdx.x % A.S, red);
}

template <typename R, bool COMP, int W, int D>
__global__ __launch_bounds__(64 * W) void k_adj(AdjArgs A) {
  __shared__ typename AccOf<R, COMP>::type red[W * 9 * 64];
  adj_block<R, COMP, W, D>(A, blockIdx.x / A.S, blockIdx.x % A.S, red);
}

// ---------------------------------------------------------------------------
// flow of arbitrary points (eq. 4)
// ---------------------------------------------------------------------------
// v += sum_j g(x, q_j) p_j over landmarks j in [j0, j1) for the lane's point
// (pre-scaled coordinates xs = k x): 9 VALU + 1 exp per pair.
template <typename R, int D>
__device__ __forceinline__ void vel_range(const Rec<R>* __restrict__ Xp, R x0, R x1, R x2,
                                          int j0, int j1, R h[3]) {
  const GlobalPtr<Rec<R>> X = global_ptr(Xp);
  R v0 = h[0], v1 = h[1], v2 = h[2];
#pragma unroll 4
  for (int j = j0; j < j1; ++j) {
    const Rec<R> rj = load_rec<R>(X, j);
    const R dx = x0 - rj.x, dy = x1 - rj.y;
    R r2 = dx * dx;
    r2 = fma(dy, dy, r2);
    if constexpr (D == 3) {
      const R dz = x2 - rj.z;
      r2 = fma(dz, dz, r2);
    }
    const R g = ex2(-r2);
    v0 = fma(g, rj.px, v0);
    v1 = fma(g, rj.py, v1);
    if constexpr (D == 3) v2 = fma(g, rj.pz, v2);
  }
  h[0] = v0; h[1] = v1; h[2] = v2;
}

// One workgroup: 64 points (one per lane) through all steps [t0, t1).  Every
// wave keeps the same FP64 copy of its lanes' points; wave w sums landmarks
// [w wchunk, (w+1) wchunk) and the W sums are combined in wave order, so the
// result depends on n and W only.
template <typename R, bool COMP, int W, int D>
__global__ __launch_bounds__(64 * W) void k_flow(FlowArgs A) {
  using Acc = typename AccOf<R, COMP>::type;
  __shared__ Acc red[W > 1 ? W * 3 * 64 : 1];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int i = blockIdx.x * 64 + lane;
  const int ic = min(i, A.m - 1);
  double x[3];
  for (int c = 0; c < 3; ++c)
    x[c] = A.x_in ? A.x_in[3 * ic + c] - A.cen[c] : A.xs[(size_t)c * A.m + ic];
  const int j0 = min(A.n, w * A.wchunk);
  const int j1 = min(A.n, j0 + A.wchunk);
  double v[3] = {0.0, 0.0, 0.0};
  for (int t = A.t0; t < A.t1; ++t) {
    const Rec<R>* X = static_cast<const Rec<R>*>(A.traj) + (size_t)(t % A.slots) * A.n;
    const R s0 = (R)(A.k * x[0]), s1 = (R)(A.k * x[1]), s2 = (R)(A.k * x[2]);
    Acc o[3];
    wave_sums<R, COMP, 3>(j0, j1, o,
                          [&](int a, int b, auto* h) { vel_range<R, D>(X, s0, s1, s2, a, b, h); });
    if constexpr (W > 1) {
      block_combine<Acc, 3, W>(red, o, w, lane);
      for (int c = 0; c < 3; ++c) v[c] = red[c * 64 + lane];
      __syncthreads();   // red is rewritten by the next step
    } else {
      for (int c = 0; c < 3; ++c) v[c] = o[c];
    }
    if (A.v_out) break;
    for (int c = 0; c < 3; ++c) x[c] = x[c] + A.dt * v[c];
  }
  if (w != 0 || i >= A.m) return;
  if (A.v_out) {
    for (int c = 0; c < 3; ++c) A.v_out[3 * i + c] = v[c];
  } else if (A.x_out) {
    for (int c = 0; c < 3; ++c) A.x_out[3 * i + c] = x[c] + A.cen[c];
  } else {
    for (int c = 0; c < 3; ++c) A.xs[(size_t)c * A.m + i] = x[c];
  }
}

// Launch KERNEL<targs..., W, D> with W waves per workgroup (1, 2, 4, 8 or 16)
// for planar (D = 2) or 3D (D = 3) problems; other W: invalid value.
#define LDDMM_LAUNCH_WD(W, D, grid, s, args, KERNEL, ...)                     \
  switch ((D) == 2 ? (W) : -(W)) {                                            \
    case 1: KERNEL<__VA_ARGS__, 1, 2><<<grid, 64, 0, s>>>(args); break;       \
    case 2: KERNEL<__VA_ARGS__, 2, 2><<<grid, 128, 0, s>>>(args); break;      \
    case 4: KERNEL<__VA_ARGS__, 4, 2><<<grid, 256, 0, s>>>(args); break;      \
    case 8: KERNEL<__VA_ARGS__, 8, 2><<<grid, 512, 0, s>>>(args); break;      \
    case 16: KERNEL<__VA_ARGS__, 16, 2><<<grid, 1024, 0, s>>>(args); break;   \
    case -1: KERNEL<__VA_ARGS__, 1, 3><<<grid, 64, 0, s>>>(args); break;      \
    case -2: KERNEL<__VA_ARGS__, 2, 3><<<grid, 128, 0, s>>>(args); break;     \
    case -4: KERNEL<__VA_ARGS__, 4, 3><<<grid, 256, 0, s>>>(args); break;     \
    case -8: KERNEL<__VA_ARGS__, 8, 3><<<grid, 512, 0, s>>>(args); break;     \
    case -16: KERNEL<__VA_ARGS__, 16, 3><<<grid, 1024, 0, s>>>(args); break;  \
    default: return hipErrorInvalidValue;                                     \
  }

template <typename R, bool COMP>
hipError_t flow_dispatch(int W, const FlowArgs& a, hipStream_t s, hipEvent_t* ev) {
  const dim3 grid((unsigned)((a.m + 63) / 64));
  if (ev) (void)hipEventRecord(ev[0], s);
  LDDMM_LAUNCH_WD(W, a.dim, grid, s, a, k_flow, R, COMP)
  if (ev) (void)hipEventRecord(ev[1], s);
  return hipGetLastError();
}

// Split path (S > 1): combine the S workgroup partials in chunk order, then
// update.  A separate launch: combining through memory inside the pair
// kernel needs agent-scope release/acquire per workgroup, whose L2
// write-back and invalidate cost more than this launch.  The partials were
// written by workgroups on other XCDs, so every load is a memory round
// trip: with the chunk count SC known at compile time all of them are in
// flight at once (SC = 0: any S, loaded chunk by chunk).
template <typename Acc, int NC, int SC>
__device__ __forceinline__ void gather_partials(const Acc* __restrict__ P, int n, int S, int ic,
                                                double h[NC]) {
  if constexpr (SC > 0) {
    Acc v[SC][NC];
#pragma unroll
    for (int s = 0; s < SC; ++s)
#pragma unroll
      for (int c = 0; c < NC; ++c) v[s][c] = P[((size_t)s * NC + c) * n + ic];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      Acc sum = v[0][c];
#pragma unroll
      for (int s = 1; s < SC; ++s) sum += v[s][c];
      h[c] = sum;
    }
  } else {
    Acc sum[NC];
    for (int c = 0; c < NC; ++c) sum[c] = P[(size_t)c * n + ic];
    for (int s = 1; s < S; ++s)
      for (int c = 0; c < NC; ++c) sum[c] += P[((size_t)s * NC + c) * n + ic];
    for (int c = 0; c < NC; ++c) h[c] = sum[c];
  }
}

// One wave per i-block and latency-bound: let the scheduler spend registers
// on loads in flight rather than on occupancy.
#define LDDMM_LATENCY_BOUND __attribute__((amdgpu_waves_per_eu(1, 2)))

template <typename R, bool COMP, int SC>
__global__ __launch_bounds__(64) LDDMM_LATENCY_BOUND void k_fwd_update(FwdArgs A) {
  using Acc = typename AccOf<R, COMP>::type;
  const int ib = blockIdx.x, lane = threadIdx.x;
  const FwdState v = load_fwd_state(A, ib * 64 + lane);
  double h[6];
  gather_partials<Acc, 6, SC>(static_cast<const Acc*>(A.partial), A.n, A.S,
                              min(ib * 64 + lane, A.n - 1), h);
  fwd_finish<R>(A, ib, lane, v, h, h + 3);
}

template <typename R, bool COMP, int SC>
__global__ __launch_bounds__(64) LDDMM_LATENCY_BOUND void k_adj_update(AdjArgs A) {
  using Acc = typename AccOf<R, COMP>::type;
  const int ib = blockIdx.x, lane = threadIdx.x;
  const AdjState v = load_adj_state(A, ib * 64 + lane);
  double h[9];
  gather_partials<Acc, 9, SC>(static_cast<const Acc*>(A.partial), A.n, A.S,
                              min(ib * 64 + lane, A.n - 1), h);
  adj_finish<R>(A, ib, lane, v, h);
}

// ---------------------------------------------------------------------------
// O(N) kernels: centroid, staging, checkpoint restore, loss, outputs
// ---------------------------------------------------------------------------

// Fixed-order block tree sum over kLossThreads values (result in red[0]).
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = kLossThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kLossThreads) void k_centroid(const double* __restrict__ q0, int n,
                                                           double* __restrict__ cen) {
  __shared__ double red[kLossThreads];
  for (int c = 0; c < 3; ++c) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kLossThreads) s += q0[3 * i + c];
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) cen[c] = t / n;
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_stage(int n, const double* __restrict__ q0,
                                               const double* __restrict__ p0,
                                               const double* __restrict__ x,
                                               const double* __restrict__ cen, double k,
                                               double* __restrict__ st, double* __restrict__ xc,
                                               Rec<R>* __restrict__ rec0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double q[3], p[3];
  for (int c = 0; c < 3; ++c) {
    q[c] = q0[3 * i + c] - cen[c];
    p[c] = p0[3 * i + c];
    st[c * n + i] = q[c];
    st[(3 + c) * n + i] = p[c];
    if (x) xc[c * n + i] = x[3 * i + c] - cen[c];
  }
  rec0[i] = make_rec<R>(k * q[0], k * q[1], k * q[2], p[0], p[1], p[2]);
}

template <typename R>
__global__ __launch_bounds__(256) void k_restore(int n, const double* __restrict__ ck, double k,
                                                 double* __restrict__ st, Rec<R>* __restrict__ rec) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v[6];
  for (int c = 0; c < 6; ++c) { v[c] = ck[c * n + i]; st[c * n + i] = v[c]; }
  rec[i] = make_rec<R>(k * v[0], k * v[1], k * v[2], v[3], v[4], v[5]);
}

__device__ __forceinline__ double sum_h0(const double* __restrict__ h0_part, int nb, double* red) {
  double h = 0.0;
  for (int b = threadIdx.x; b < nb; b += kLossThreads) h += h0_part[b];
  return 0.5 * block_sum(h, red);
}

template <typename R>
__device__ __forceinline__ void loss_body(int n, int nb, double lambda, const double* __restrict__ st,
                                          const double* __restrict__ xc,
                                          const double* __restrict__ cen,
                                          const double* __restrict__ h0_part,
                                          double* __restrict__ ad, Rec<R>* __restrict__ arec0,
                                          double* __restrict__ out3, double* __restrict__ q1,
                                          double* __restrict__ p1, int* __restrict__ flag,
                                          double* __restrict__ grad_x,
                                          const double* __restrict__ hqT,
                                          const double* __restrict__ hpT, double bscale,
                                          double* red) {
  double mis = 0.0;
  for (int i = threadIdx.x; i < n; i += kLossThreads) {
    double a[3], b[3];
    for (int c = 0; c < 3; ++c) {
      const double q = st[c * n + i];
      const double r = q - xc[c * n + i];
      mis += r * r;
      a[c] = 2.0 * lambda * r;           // dL/dq(1) of the mismatch
      b[c] = 0.0;                        // dL/dp(1)
      if (grad_x) grad_x[3 * i + c] = -a[c];
      if (hqT) {                         // energy term H(q(1), p(1))
        a[c] += hqT[c * n + i];
        b[c] = hpT[c * n + i];
      }
      ad[c * n + i] = a[c];
      ad[(3 + c) * n + i] = b[c];
      if (q1) q1[3 * i + c] = q + cen[c];
      if (p1) p1[3 * i + c] = st[(3 + c) * n + i];
    }
    arec0[i] = make_rec<R>(a[0], a[1], a[2], bscale * b[0], bscale * b[1], bscale * b[2]);
  }
  const double m = block_sum(mis, red);
  const double H0 = sum_h0(h0_part, nb, red);
  if (threadIdx.x == 0) {
    const double L = H0 + lambda * m;
    out3[0] = L;
    out3[1] = H0;
    out3[2] = m;
    if (!isfinite(L)) atomicOr(flag, 1);
  }
}

template <typename R>
__global__ __launch_bounds__(kLossThreads) void k_loss(
    int n, int nb, double lambda, const double* __restrict__ st, const double* __restrict__ xc,
    const double* __restrict__ cen, const double* __restrict__ h0_part, double* __restrict__ ad,
    Rec<R>* __restrict__ arec0, double* __restrict__ out3, double* __restrict__ q1,
    double* __restrict__ p1, int* __restrict__ flag, double* __restrict__ grad_x,
    const double* __restrict__ hqT, const double* __restrict__ hpT, double bscale) {
  __shared__ double red[kLossThreads];
  loss_body<R>(n, nb, lambda, st, xc, cen, h0_part, ad, arec0, out3, q1, p1, flag, grad_x, hqT,
               hpT, bscale, red);
}

__global__ __launch_bounds__(kLossThreads) void k_forward_out(
    int n, int nb, const double* __restrict__ st, const double* __restrict__ cen,
    const double* __restrict__ h0_part, double* __restrict__ H0, double* __restrict__ q1,
    double* __restrict__ p1) {
  __shared__ double red[kLossThreads];
  for (int i = threadIdx.x; i < n; i += kLossThreads)
    for (int c = 0; c < 3; ++c) {
      if (q1) q1[3 * i + c] = st[c * n + i] + cen[c];
      if (p1) p1[3 * i + c] = st[(3 + c) * n + i];
    }
  const double h = sum_h0(h0_part, nb, red);
  if (threadIdx.x == 0 && H0) *H0 = h;
}

// ---------------------------------------------------------------------------
// batched kernels: several registrations per launch
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool job_live(const BatchJob& b) { return b.active && *b.done == 0; }

template <typename R>
__global__ __launch_bounds__(256) void k_stage_batch(const BatchJob* __restrict__ J) {
  const BatchJob& b = J[blockIdx.y];
  if (!job_live(b)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  const int n = b.n;
  double q[3], p[3];
  for (int c = 0; c < 3; ++c) {
    q[c] = b.q0[3 * i + c] - b.cen[c];
    p[c] = b.p0[3 * i + c];
    b.st[c * n + i] = q[c];
    b.st[(3 + c) * n + i] = p[c];
  }
  const double k = b.sc.k;
  static_cast<Rec<R>*>(b.traj)[i] = make_rec<R>(k * q[0], k * q[1], k * q[2], p[0], p[1], p[2]);
}

template <typename R>
__device__ __forceinline__ FwdArgs batch_fwd_args(const BatchJob& b, int t) {
  FwdArgs A{};
  A.n = b.n; A.nb = b.nb; A.S = 1; A.chunk = b.n; A.wchunk = (b.n + kBatchWaves - 1) / kBatchWaves;
  A.dim = 3;
  A.sc = b.sc;
  A.rec_t = static_cast<const Rec<R>*>(b.traj) + (size_t)t * b.n;
  A.rec_t1 = static_cast<Rec<R>*>(b.traj) + (size_t)(t + 1) * b.n;
  A.st = b.st;
  A.hp0 = t == 0 ? b.hp0 : nullptr;
  A.h0_part = t == 0 ? b.h0p : nullptr;
  return A;
}

template <typename R, bool COMP>
__global__ __launch_bounds__(64 * kBatchWaves) void k_fwd_batch(const BatchJob* __restrict__ J,
                                                                const int2* __restrict__ items,
                                                                const int* __restrict__ nitems,
                                                                int t) {
  __shared__ typename AccOf<R, COMP>::type red[kBatchWaves * 6 * 64];
  if ((int)blockIdx.x >= *nitems) return;
  const int2 it = items[blockIdx.x];
  const BatchJob& b = J[it.x];
  if (!job_live(b)) return;
  fwd_block<R, COMP, kBatchWaves, 3>(batch_fwd_args<R>(b, t), it.y, 0, red);
}

template <typename R, bool COMP>
__global__ __launch_bounds__(64 * kBatchWaves) void k_adj_batch(const BatchJob* __restrict__ J,
                                                                const int2* __restrict__ items,
                                                                const int* __restrict__ nitems,
                                                                int t, int T) {
  __shared__ typename AccOf<R, COMP>::type red[kBatchWaves * 9 * 64];
  if ((int)blockIdx.x >= *nitems) return;
  const int2 it = items[blockIdx.x];
  const BatchJob& b = J[it.x];
  if (!job_live(b)) return;
  AdjArgs A{};
  A.n = b.n; A.nb = b.nb; A.S = 1; A.chunk = b.n; A.wchunk = (b.n + kBatchWaves - 1) / kBatchWaves;
  A.dim = 3;
  A.sc = b.sc;
  const int cur = (T - 1 - t) & 1;   // the loss kernel fills adjoint buffer 0 for t = T-1
  A.rec_t = static_cast<const Rec<R>*>(b.traj) + (size_t)t * b.n;
  A.arec = static_cast<const Rec<R>*>(b.arec) + (size_t)cur * b.n;
  A.arec_next = static_cast<Rec<R>*>(b.arec) + (size_t)(cur ^ 1) * b.n;
  A.ad = b.ad;
  A.hp0 = b.hp0;
  A.grad = t == 0 ? b.grad : nullptr;
  adj_block<R, COMP, kBatchWaves, 3>(A, it.y, 0, red);
}

template <typename R>
__global__ __launch_bounds__(kLossThreads) void k_loss_batch(const BatchJob* __restrict__ J) {
  __shared__ double red[kLossThreads];
  const BatchJob& b = J[blockIdx.x];
  if (!job_live(b)) return;
  loss_body<R>(b.n, b.nb, b.lambda, b.st, b.xc, b.cen, b.h0p, b.ad, static_cast<Rec<R>*>(b.arec),
               b.out3, b.q1, nullptr, b.flag, nullptr, nullptr, nullptr, 0.0, red);
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
template <typename R, bool COMP>
hipError_t fwd_dispatch(const Plan& p, const FwdArgs& a, hipStream_t s, hipEvent_t* ev) {
  const dim3 grid(p.nb * p.S);
  if (ev) (void)hipEventRecord(ev[0], s);
  LDDMM_LAUNCH_WD(p.W, a.dim, grid, s, a, k_fwd, R, COMP)
  if (ev) (void)hipEventRecord(ev[1], s);
  switch (p.S) {
    case 1: break;
    case 2: k_fwd_update<R, COMP, 2><<<p.nb, 64, 0, s>>>(a); break;
    case 3: k_fwd_update<R, COMP, 3><<<p.nb, 64, 0, s>>>(a); break;
    case 4: k_fwd_update<R, COMP, 4><<<p.nb, 64, 0, s>>>(a); break;
    case 8: k_fwd_update<R, COMP, 8><<<p.nb, 64, 0, s>>>(a); break;
    case 16: k_fwd_update<R, COMP, 16><<<p.nb, 64, 0, s>>>(a); break;
    default: k_fwd_update<R, COMP, 0><<<p.nb, 64, 0, s>>>(a); break;
  }
  return hipGetLastError();
}

template <typename R, bool COMP>
hipError_t adj_dispatch(const Plan& p, const AdjArgs& a, hipStream_t s, hipEvent_t* ev) {
  const dim3 grid(p.nb * p.S);
  if (ev) (void)hipEventRecord(ev[0], s);
  LDDMM_LAUNCH_WD(p.W, a.dim, grid, s, a, k_adj, R, COMP)
  if (ev) (void)hipEventRecord(ev[1], s);
  switch (p.S) {
    case 1: break;
    case 2: k_adj_update<R, COMP, 2><<<p.nb, 64, 0, s>>>(a); break;
    case 3: k_adj_update<R, COMP, 3><<<p.nb, 64, 0, s>>>(a); break;
    case 4: k_adj_update<R, COMP, 4><<<p.nb, 64, 0, s>>>(a); break;
    case 8: k_adj_update<R, COMP, 8><<<p.nb, 64, 0, s>>>(a); break;
    case 16: k_adj_update<R, COMP, 16><<<p.nb, 64, 0, s>>>(a); break;
    default: k_adj_update<R, COMP, 0><<<p.nb, 64, 0, s>>>(a); break;
  }
  return hipGetLastError();
}

inline unsigned blocks256(int n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
Plan make_plan(int n, int target_waves) {
  Plan p{};
  p.n = n;
  p.nb = (n + 63) / 64;
  // Waves per i-block: enough to give the chip ~target_waves waves, at most
  // 64 and at least 16 pairs per wave.  Workgroups of at most 8 waves:
  // measured on N = 4096, 16384 and 65536, 8-wave workgroups with up to 4x
  // more waves beat 16-wave ones by 3 %, 22 % and 17 % (shorter LDS combine
  // and barriers, two workgroups per CU interleaving their phases); 64 waves
  // per i-block was the best split at N = 4096 and 16384.
  int per_i = (target_waves + p.nb - 1) / p.nb;
  if (per_i > 64) per_i = 64;
  const int max_per_i = n / 16 > 1 ? n / 16 : 1;
  if (per_i > max_per_i) per_i = max_per_i;
  if (per_i < 1) per_i = 1;
  static const int max_w = [] {
    const char* e = std::getenv("LDDMM_MAX_WG_WAVES");
    const int v = e ? std::atoi(e) : 0;
    return (v == 1 || v == 2 || v == 4 || v == 8 || v == 16) ? v : 8;
  }();
  int W = 1;
  while (W * 2 <= per_i && W * 2 <= max_w) W *= 2;
  p.W = W;
  int S = (per_i + W - 1) / W;
  // the combine kernel keeps all S loads in flight for S in {2, 3, 4, 8, 16}
  if (S > 4 && S < 8) S = 4;
  else if (S > 8 && S < 16) S = 8;
  p.S = S < 1 ? 1 : S;
  p.chunk = (n + p.S - 1) / p.S;
  p.wchunk = (p.chunk + W - 1) / W;
  return p;
}

Scales make_scales(double sigma, int T) {
  Scales s{};
  const double log2e = 1.4426950408889634;
  const double c = 1.0 / (sigma * sigma);
  s.k = std::sqrt(log2e / (2.0 * sigma * sigma));
  s.hq = -c / s.k;
  s.adj_a = c / s.k;
  s.kappa = c / (s.k * s.k);
  s.bscale = s.kappa * s.k;
  s.dt = 1.0 / T;
  return s;
}

size_t rec_bytes(int mode) { return mode == kFP64 ? sizeof(Rec<double>) : sizeof(Rec<float>); }
size_t acc_bytes(int mode) { return mode == kFP32 ? sizeof(float) : sizeof(double); }

hipError_t launch_centroid(const double* q0, int n, double* cen, hipStream_t s) {
  k_centroid<<<1, kLossThreads, 0, s>>>(q0, n, cen);
  return hipGetLastError();
}

hipError_t launch_stage(int mode, int n, const double* q0, const double* p0, const double* x,
                        const double* cen, double k, double* st, double* xc, void* rec0,
                        hipStream_t s) {
  if (mode == kFP64)
    k_stage<double><<<blocks256(n), 256, 0, s>>>(n, q0, p0, x, cen, k, st, xc,
                                                 static_cast<Rec<double>*>(rec0));
  else
    k_stage<float><<<blocks256(n), 256, 0, s>>>(n, q0, p0, x, cen, k, st, xc,
                                                static_cast<Rec<float>*>(rec0));
  return hipGetLastError();
}

hipError_t launch_restore(int mode, int n, const double* ckpt, double k, double* st, void* rec,
                          hipStream_t s) {
  if (mode == kFP64)
    k_restore<double><<<blocks256(n), 256, 0, s>>>(n, ckpt, k, st, static_cast<Rec<double>*>(rec));
  else
    k_restore<float><<<blocks256(n), 256, 0, s>>>(n, ckpt, k, st, static_cast<Rec<float>*>(rec));
  return hipGetLastError();
}

hipError_t launch_fwd_step(int mode, const Plan& p, const FwdArgs& a, hipStream_t s,
                           hipEvent_t* ev) {
  switch (mode) {
    case kFP32: return fwd_dispatch<float, false>(p, a, s, ev);
    case kFP32Comp: return fwd_dispatch<float, true>(p, a, s, ev);
    case kFP64: return fwd_dispatch<double, false>(p, a, s, ev);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adj_step(int mode, const Plan& p, const AdjArgs& a, hipStream_t s,
                           hipEvent_t* ev) {
  switch (mode) {
    case kFP32: return adj_dispatch<float, false>(p, a, s, ev);
    case kFP32Comp: return adj_dispatch<float, true>(p, a, s, ev);
    case kFP64: return adj_dispatch<double, false>(p, a, s, ev);
  }
  return hipErrorInvalidValue;
}

int flow_waves(int n) {
  static const int forced = [] {
    const char* e = std::getenv("LDDMM_FLOW_WAVES");
    return e ? std::atoi(e) : 0;
  }();
  if (forced == 1 || forced == 2 || forced == 4 || forced == 8 || forced == 16) return forced;
  // at least 1024 landmarks per wave and step: measured best at N = 4096
  // (W = 4 runs the 64^3-grid flow 1.2x faster than W = 1 and 1.4x faster
  // than W = 16, whose per-step combine no longer pays)
  int W = 1;
  while (W < 16 && (W * 2) * 1024 <= n) W *= 2;
  return W;
}

hipError_t launch_flow(int mode, int W, const FlowArgs& a, hipStream_t s, hipEvent_t* ev) {
  if (a.m <= 0 || a.n <= 0 || a.t1 <= a.t0 || a.slots <= 0) return hipErrorInvalidValue;
  if (a.v_out && a.t1 != a.t0 + 1) return hipErrorInvalidValue;
  switch (mode) {
    case kFP32: return flow_dispatch<float, false>(W, a, s, ev);
    case kFP32Comp: return flow_dispatch<float, true>(W, a, s, ev);
    case kFP64: return flow_dispatch<double, false>(W, a, s, ev);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_loss(int mode, int n, int nb, double lambda, double bscale, const double* st,
                       const double* xc, const double* cen, const double* h0_part, double* ad,
                       void* arec0, double* out3, double* q1, double* p1, int* flag,
                       double* grad_x, const double* hqT, const double* hpT, hipStream_t s) {
  if (mode == kFP64)
    k_loss<double><<<1, kLossThreads, 0, s>>>(n, nb, lambda, st, xc, cen, h0_part, ad,
                                              static_cast<Rec<double>*>(arec0), out3, q1, p1, flag,
                                              grad_x, hqT, hpT, bscale);
  else
    k_loss<float><<<1, kLossThreads, 0, s>>>(n, nb, lambda, st, xc, cen, h0_part, ad,
                                             static_cast<Rec<float>*>(arec0), out3, q1, p1, flag,
                                             grad_x, hqT, hpT, bscale);
  return hipGetLastError();
}

hipError_t launch_forward_out(int n, int nb, const double* st, const double* cen,
                              const double* h0_part, double* H0, double* q1, double* p1,
                              hipStream_t s) {
  k_forward_out<<<1, kLossThreads, 0, s>>>(n, nb, st, cen, h0_part, H0, q1, p1);
  return hipGetLastError();
}

hipError_t launch_stage_batch(int mode, const BatchJob* jobs, int max_slots, int max_n,
                              hipStream_t s) {
  const dim3 grid((max_n + 255) / 256, max_slots);
  if (mode == kFP64) k_stage_batch<double><<<grid, 256, 0, s>>>(jobs);
  else k_stage_batch<float><<<grid, 256, 0, s>>>(jobs);
  return hipGetLastError();
}

hipError_t launch_fwd_batch(int mode, const BatchJob* jobs, const int2* items, const int* nitems,
                            int capacity, int t, hipStream_t s) {
  const int threads = 64 * kBatchWaves;
  switch (mode) {
    case kFP32: k_fwd_batch<float, false><<<capacity, threads, 0, s>>>(jobs, items, nitems, t); break;
    case kFP32Comp: k_fwd_batch<float, true><<<capacity, threads, 0, s>>>(jobs, items, nitems, t); break;
    case kFP64: k_fwd_batch<double, false><<<capacity, threads, 0, s>>>(jobs, items, nitems, t); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adj_batch(int mode, const BatchJob* jobs, const int2* items, const int* nitems,
                            int capacity, int t, int T, hipStream_t s) {
  const int threads = 64 * kBatchWaves;
  switch (mode) {
    case kFP32: k_adj_batch<float, false><<<capacity, threads, 0, s>>>(jobs, items, nitems, t, T); break;
    case kFP32Comp: k_adj_batch<float, true><<<capacity, threads, 0, s>>>(jobs, items, nitems, t, T); break;
    case kFP64: k_adj_batch<double, false><<<capacity, threads, 0, s>>>(jobs, items, nitems, t, T); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_loss_batch(int mode, const BatchJob* jobs, int max_slots, hipStream_t s) {
  if (mode == kFP64) k_loss_batch<double><<<max_slots, kLossThreads, 0, s>>>(jobs);
  else k_loss_batch<float><<<max_slots, kLossThreads, 0, s>>>(jobs);
  return hipGetLastError();
}

}  // namespace lddmm
