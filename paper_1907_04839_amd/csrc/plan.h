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

// Wider workgroups for the plans of 8 waves and 8, 4, 3 or 2 j-chunks.  The
// best width depends on the kernel instance's registers and LDS and on how
// many workgroups share a CU.  Measured per precision mode and kind of step
// (ms per loss+gradient evaluation; widths forward/adjoint 12/12, 8/8, 16/16;
// Euler unless marked):
//   FP32-compensated: N = 4096 1.298, 1.351, 1.451; 16384 (T = 4) 1.298,
//     1.322, 1.585; 65536 (T = 3) 14.38, 14.78, 17.35; 800 (T = 10) 0.167,
//     0.187, 0.163; Runge-Kutta N = 4096 (T = 10) 1.317, 1.378, 1.469
//     -> 12/12 everywhere.  Its 16-wave workgroups, like the FP64 ones, hold
//     72 KiB of LDS for the wave combine and were slow wherever workgroups
//     share a CU.
//   FP32 (16/16 first): N = 4096 1.213, 1.241, 1.296; 32768 (T = 2) 2.384,
//     2.438, 2.446; 65536 13.93, 14.17, 14.33; 800 0.156, 0.162, 0.183
//     -> 16/16; Runge-Kutta N = 4096 1.288, 1.269, 1.320; 800 (T = 3) 0.192,
//     0.199, 0.227 -> 12/12, or 16/16 where a launch has at most one
//     workgroup per CU.
//   FP64: N = 4096 2.314, 2.415, 2.694; 16384 2.845, 2.913, 3.310; 65536
//     33.58, 34.43, 41.39; with at most one workgroup per CU (16/16 first)
//     N = 800 0.245, 0.261, 0.312 and 1847 0.938, 0.952, 0.994 -> 16/16 there,
//     else 12/12; Runge-Kutta N = 4096 8/8 2.356 against 2.573 (12/12) ->
//     unwidened unless at most one workgroup per CU (16/16: N = 800 0.286
//     against 0.350 at 8/8).
// Widths 10 and 14 leave the four SIMDs unevenly loaded (measured slower).
// The sum order within a workgroup follows the width, so results change at
// rounding level.
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
    if (mode == kFP32Comp) { wf = wa = 12; }
    else if (mode == kFP32) { wf = wa = one_per_cu ? 16 : 12; }
    else if (mode == kFP64) {
      if (!one_per_cu) return;   // 12 or 16 waves measured slower there
      wf = wa = 16;
    }
  } else if (mode == kFP32Comp) {
    wf = wa = 12;
  } else if (mode == kFP32) {
    wf = wa = 16;
  } else if (mode == kFP64) {
    wf = wa = one_per_cu ? 16 : 12;
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
