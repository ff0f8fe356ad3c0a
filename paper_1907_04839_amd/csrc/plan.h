// Host-side planning shared by the C-ABI layer and the kernels' launchers:
// the work decomposition of the pair sums, the scale factors, and the byte
// layout of a problem's workspace.  Plain C++ (no HIP), so the host tests
// build it with the sanitizers.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdlib>

#include "lddmm.h"

namespace lddmm {

// Precision of the pair sums (the FP64 state, loss and optimiser are FP64 in
// every mode).
enum Mode : int { kFP32 = 0, kFP32Comp = 1, kFP64 = 2 };

// Work decomposition of one N x N pair sum.  Landmark i is owned by lane
// (i mod 64) of a wave of i-block ib = i / 64; the j range is split into S
// chunks (one workgroup each) and, inside a workgroup, over W waves.
// Partial sums of different chunks are combined in chunk order.
struct Plan {
  int n;        // landmarks
  int nb;       // i-blocks of 64
  int S;        // j-chunks (workgroups) per i-block
  int W;        // waves per workgroup of the forward pair kernel
  int chunk;    // j per workgroup
  int wchunk;   // j per wave of the forward pair kernel
  int Wa;       // waves per workgroup of the adjoint pair kernel
  int wchunk_a; // j per wave of the adjoint pair kernel
};

// Coordinates enter the pair kernels pre-scaled by k = sqrt(log2(e) / (2 sigma^2)),
// so that the kernel value is exp2(-|k q_i - k q_j|^2).
struct Scales {
  double k;         // coordinate pre-scale
  double hq;        // Hq = hq * sum g s (kq_i - kq_j)           = -(c / k)
  double adj_a;     // A  = adj_a * (A1 / kappa - A2)            =  c / k
  double kappa;     // 2 ln 2 = c / k^2 (independent of sigma)
  double bscale;    // adjoint record stores b_hat = bscale * b = kappa k b
  double dt;
};

inline Plan make_plan(int n, int target_waves) {
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
  p.Wa = W;
  p.wchunk_a = p.wchunk;
  return p;
}

// Wider workgroups for the 8 x 8 plans (N from about 900 to 16384), where a
// launch has 2 or fewer workgroups per CU: with 12 (or 16) waves each, two
// resident workgroups fill more of a CU's wave slots than two of 8, and each
// wave's j range is shorter.  The best width depends on the registers of the
// kernel instance and was measured per precision and kind of step (ms per
// loss+gradient evaluation, widths forward/adjoint vs 8/8): FP32-compensated
// 12/12 (N = 4096: 1.308 vs 1.348; 1847: 0.661 vs 0.676; 16384 with T = 100:
// 31.7 vs 32.5; planar 4096: 1.100 vs 1.125), FP32 16/16 (4096: 1.229 vs
// 1.303), FP64 12/8 (4096: 2.375 vs 2.416; planar: 2.048 vs 2.106).  Other
// widths were slower: 10 and 14 leave the four SIMDs unevenly loaded, 16
// fits one FP32-compensated adjoint workgroup per CU, 12 one FP64 adjoint.
// Runge-Kutta stage kernels hold more registers and keep 8/8 where
// workgroups share CUs (12/12: 1.494 vs 1.382 ms in FP32-compensated, 3.06
// vs 2.43 in FP64).  The 8 x 2 plans of N from about 65000 to 116000 (eight
// workgroups per CU in turn; the 8 x 2 plans of N = 144-271 stay 8/8) gain too
// in FP32 modes, where two 12-wave workgroups divide the turns evenly:
// N = 65536 FP32-compensated 12/12 238.4 vs 242.3 ms, FP32 16/16 233.2 vs
// 240.6; FP64 12/8 585 vs 583 (kept at 8/8).  The 8 x 4 and 8 x 3 plans
// (N from 272 to 911, and from about 16400 to 65000) take 12/12 in both
// FP32 modes: FP32-compensated N = 600 0.58 vs 0.647 ms, 800 0.637 vs 0.722,
// 32768 (T = 10) 12.05 vs 12.23, 50000 (T = 4) 12.12 vs 12.29; FP32 N = 800
// 0.618 vs 0.706, 32768 11.82 vs 12.12, 50000 11.89 vs 12.19 (16/16 was
// erratic at N = 600 and slower in the FP32-compensated adjoint at 32768).
// FP64 gains from width only while a launch has at most one workgroup per CU
// (no workgroups compete for a CU's registers): 12/12 at N = 350 0.764 vs
// 0.886 ms, N = 800 0.955 vs 1.124 and N = 1847 (232 workgroups) 0.925 vs
// 0.946, and 16/16 better still (0.726, 0.894, 0.919), but at N = 32768 and
// 50000 12/12 was 10-23 % slower and 12/8 equal to 8/8.  Runge-Kutta stage
// kernels likewise gain where a launch has at most one workgroup per CU
// (T = 10): FP32-compensated 12/12 N = 800 0.662 vs 0.800 ms, FP64 16/16
// N = 350 0.757 vs 0.971 and N = 800 0.917 vs 1.207; FP32 stages were not
// measured and keep 8/8.  The sum order within a workgroup follows the
// width, so results change at rounding level.
// The workgroup widths measured fastest for the pair kernels of a precision
// mode and kind of step (rk: Runge-Kutta stages), applied to the plans of 8
// waves and 8, 4, 3 or 2 j-chunks; other plans are left as they are.
inline void widen_plan(Plan& p, int mode, bool rk) {
  constexpr int kCUs = 256;   // MI355X
  if (p.W != 8) return;
  if (p.S != 8 && p.S != 4 && p.S != 3 && p.S != 2) return;
  // make_plan also gives 8 x 2 plans at N = 144-271, where 12 or 16 waves
  // would leave fewer than 8 (or no) j per wave: the 8 x 2 widths were
  // measured at N = 65536 only, so they apply where every wave keeps >= 16 j.
  if (p.S == 2 && (p.chunk + 15) / 16 < 16) return;
  const bool one_per_cu = p.nb * p.S <= kCUs;
  int wf = 8, wa = 8;
  if (rk) {
    // Runge-Kutta stages, only where no workgroups compete for a CU
    if (!one_per_cu) return;
    if (mode == kFP32Comp) { wf = 12; wa = 12; }
    else if (mode == kFP64) { wf = 16; wa = 16; }
    else return;
  } else if (mode == kFP32Comp) {
    wf = 12; wa = 12;
  } else if (mode == kFP32) {
    wf = wa = (p.S == 8 || p.S == 2) ? 16 : 12;
  } else if (mode == kFP64) {
    if (one_per_cu) { wf = 16; wa = 16; }
    else if (p.S == 8) { wf = 12; wa = 8; }
  }
  p.W = wf;
  p.wchunk = (p.chunk + wf - 1) / wf;
  p.Wa = wa;
  p.wchunk_a = (p.chunk + wa - 1) / wa;
}

inline Scales make_scales(double sigma, int T) {
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

// Size in bytes of one point record ((k q, 0, p, 0) or (a, 0, b_hat, 0): eight
// values) and of one partial-sum element.
inline size_t rec_bytes(int mode) { return mode == kFP64 ? 64 : 32; }
inline size_t acc_bytes(int mode) { return mode == kFP32 ? sizeof(float) : sizeof(double); }


inline size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

// Byte offsets of the workspace buffers of one problem.
struct Layout {
  size_t st, ad, hp0, hq0, xc, cen, h0p, out3, traj, arec, ckpt, partial;
  size_t hpT, hqT, hTp, stT, recT;   // energy at t = 1 only (else empty)
  size_t rk_acc, rk_lam;             // Runge-Kutta steps only (else empty)
  size_t total;
  int slots;   // trajectory slots (records: 1 per Euler step, 4 per Runge-Kutta step)
  int nseg;    // checkpoint segments (0 = full trajectory)
};

inline Layout make_layout(const lddmm_params& p, const Plan& plan) {
  Layout L{};
  const size_t n = (size_t)p.n, rb = rec_bytes(p.precision), ab = acc_bytes(p.precision);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += a256(bytes); return o; };
  L.st = take(6 * n * 8);
  L.ad = take(6 * n * 8);
  L.hp0 = take(3 * n * 8);
  L.hq0 = take(3 * n * 8);
  L.xc = take(3 * n * 8);
  L.cen = take(4 * 8);
  L.h0p = take((size_t)plan.nb * 8);
  L.out3 = take(4 * 8);
  const int s = p.ckpt_every;
  const bool ck = s > 0 && s < p.T;
  const int spt = p.integrator == LDDMM_RK4 ? 4 : 1;   // records per step
  L.slots = spt * (ck ? s : p.T) + 1;
  L.nseg = ck ? (p.T + s - 1) / s : 0;
  L.traj = take((size_t)L.slots * n * rb);
  L.arec = take(2 * n * rb);
  L.ckpt = take((size_t)L.nseg * 6 * n * 8);
  L.partial = take(plan.S > 1 ? (size_t)plan.S * 9 * n * ab : 0);
  const bool fin = p.energy == LDDMM_ENERGY_FINAL;
  L.hpT = take(fin ? 3 * n * 8 : 0);
  L.hqT = take(fin ? 3 * n * 8 : 0);
  L.hTp = take(fin ? (size_t)plan.nb * 8 : 0);
  L.stT = take(fin ? 6 * n * 8 : 0);
  L.recT = take(fin ? n * rb : 0);
  L.rk_acc = take(spt == 4 ? 6 * n * 8 : 0);
  L.rk_lam = take(spt == 4 ? 6 * n * 8 : 0);
  L.total = off;
  return L;
}

}  // namespace lddmm
