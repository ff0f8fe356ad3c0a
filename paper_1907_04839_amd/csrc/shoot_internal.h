// Internal interface between the C-ABI layer (lddmm_api.cpp) and the HIP
// kernels (shoot_kernels.hip).  Not installed; callers use include/lddmm.h.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "plan.h"

namespace lddmm {

// Arguments of one forward Euler step, or of one stage of a classical
// Runge-Kutta step (pair sums + update).
struct FwdArgs {
  int n, nb, S, chunk, wchunk;
  int dim;              // 3, or 2 for planar problems (z terms left out)
  int rk;               // 0: Euler step.  1..4: Runge-Kutta stage rk, whose pair
                        // sums are taken at the stage state in rec_t; stages
                        // 1-3 write the next stage state's record to rec_t1,
                        // stage 4 the new state (st, rec_t1)
  double* rk_acc;       // [6][n] k1 + 2 k2 + 2 k3, built over stages 1-3
  Scales sc;
  const void* rec_t;    // point records at step t (k q, p)
  void* rec_t1;         // point records at step t+1 (written)
  double* st;           // FP64 state [6][n]: q (3 rows) then p (3 rows), centred
  double* hp0;          // [3][n]: Hp(q0,p0) (written at t == 0, else null)
  double* hq0;          // [3][n]: Hq(q0,p0) (optional, with hp0)
  double* h0_part;      // [nb]: per i-block sum p0.Hp0 (t == 0, else null)
  double* ckpt;         // [6][n]: copy of the new state (null unless a checkpoint)
  void* partial;        // [S][6][n] partial sums when S > 1
};

// Arguments of one backward (adjoint) Euler step, or of one stage of the
// adjoint of a Runge-Kutta step.
struct AdjArgs {
  int n, nb, S, chunk, wchunk;
  int dim;              // 3, or 2 for planar problems
  int rk;               // 0: Euler step.  1..4: stage rk of the Runge-Kutta
                        // adjoint (taken from 4 down to 1): the pair sums give
                        // w = J(Y_rk)^T u for the stage state in rec_t and the
                        // stage adjoint u in arec; ad keeps lambda' (the adjoint
                        // after the step) until stage 1 writes the new one
  double* rk_lam;       // [6][n] lambda' + the w of the stages taken so far
  Scales sc;
  const void* rec_t;    // point records at step t (k q, p)
  const void* arec;     // adjoint records (a, b_hat) entering the step
  void* arec_next;      // adjoint records leaving the step (written)
  double* ad;           // FP64 adjoint state [6][n]: a (3 rows) then b (3 rows)
  const double* hp0;    // [3][n] Hp(q0,p0), added to the gradient (null: nothing added)
  double* grad;         // [n][3] gradient, written at t == 0 (else null)
  const double* hq0;    // [3][n] Hq(q0,p0), with grad_q0
  double* grad_q0;      // [n][3] dL/dq0 = a(0) + Hq(q0,p0), at t == 0 (optional)
  void* partial;        // [S][9][n] partial sums when S > 1
};

// Size of the fixed device scratch of lddmm_shoot_grad_noalloc, and its device
// address on `device` (looked up on the first call for that device, with the
// device current; the same address afterwards).
constexpr size_t kScratchBytes = size_t(64) << 20;
hipError_t scratch_address(int device, void** out);

hipError_t launch_centroid(const double* q0, int n, double* cen, hipStream_t s);
hipError_t launch_stage(int mode, int n, const double* q0, const double* p0, const double* x,
                        const double* cen, double k, double* st, double* xc, void* rec0,
                        hipStream_t s);
hipError_t launch_restore(int mode, int n, const double* ckpt, double k, double* st, void* rec,
                          hipStream_t s);
// ev (optional): two events recorded on s around the pair kernel alone.
hipError_t launch_fwd_step(int mode, const Plan& p, const FwdArgs& a, hipStream_t s,
                           hipEvent_t* ev = nullptr);
hipError_t launch_adj_step(int mode, const Plan& p, const AdjArgs& a, hipStream_t s,
                           hipEvent_t* ev = nullptr);
// Points carried by the landmark motion (eq. 4): over steps [t0, t1) of a
// stored trajectory, x <- x + dt v(x, t) with v(x, t) = sum_l g(|q_l(t) - x|)
// p_l(t).  One lane owns one point for all the steps; the landmarks are split
// over the W waves of a workgroup and combined in wave order every step.
struct FlowArgs {
  int n, m;             // landmarks, points
  int t0, t1;           // steps
  int slots;            // trajectory slots: record r is slot r % slots
  int spt;              // records per step: 1 (Euler), 4 (Runge-Kutta stage states;
                        // record spt t + s is stage s + 1 of step t)
  int wchunk;           // landmarks per wave
  int dim;              // 3, or 2 for planar problems
  double k, dt;
  const void* traj;     // landmark records (k q, p), slot-major
  const double* cen;    // landmark centroid; point coordinates are centred on it
  const double* x_in;   // [m][3] uncentred points (first segment), else read xs
  double* xs;           // [3][m] centred FP64 point state between segments
  double* x_out;        // [m][3] uncentred points after t1 (last segment), else write xs
  double* v_out;        // [m][3]: write v(x, t0) and take no step (t1 == t0 + 1)
};

// Waves per workgroup of the flow kernel for n landmarks (1, 2, 4, 8 or 16;
// LDDMM_FLOW_WAVES overrides it).  It depends on n only, so a point's result
// does not depend on how many other points are carried with it.
int flow_waves(int n);
hipError_t launch_flow(int mode, int W, const FlowArgs& a, hipStream_t s,
                       hipEvent_t* ev = nullptr);

// Loss and terminal adjoint: L = E + lambda |q(1) - x|^2, a = 2 lambda (q(1) - x), b = 0,
// with the energy term E summed from h0_part.  With hqT/hpT ([3][n], the forward sums at the
// final state) E is H(q(1), p(1)) and the terminal adjoint gains a += HqT, b = HpT.
// out3 = {loss, E, mismatch}; q1/p1 (optional) receive the final state, uncentred, [n][3].
// grad_x (optional): dL/dx = -2 lambda (q(1) - x), [n][3].
// arec0 receives the record of rscale (a, b) for the first adjoint launch
// (1 for Euler steps, dt / 6 for the last stage of a Runge-Kutta step).
hipError_t launch_loss(int mode, int n, int nb, double lambda, double bscale, double rscale,
                       const double* st, const double* xc, const double* cen,
                       const double* h0_part, double* ad, void* arec0, double* out3, double* q1,
                       double* p1, int* flag, double* grad_x, const double* hqT,
                       const double* hpT, hipStream_t s);
// Forward-only epilogue: writes H0 (device scalar) and the final state.
hipError_t launch_forward_out(int n, int nb, const double* st, const double* cen,
                              const double* h0_part, double* H0, double* q1, double* p1,
                              hipStream_t s);

// One registration of a batched launch, as the batched kernels see it.  All
// jobs of a batch share T, the precision and the kind of step; planar and 3D
// jobs have pair kernels of their own.  The decomposition of every job
// is one workgroup of batch_waves waves per 64-landmark i-block and no j split, so a
// job's results do not depend on which other jobs share the launch.
struct BatchJob {
  int active;               // the slot holds a job
  int n, nb;
  double lambda;
  Scales sc;
  const double* q0;         // [n][3] template
  const double* p0;         // [n][3] momentum to evaluate (the optimiser's trial point)
  const int* done;          // the job's optimiser has finished: skip it
  double *cen, *st, *ad, *hp0, *xc, *h0p, *out3;
  void *traj, *arec;        // (spt T + 1) point records, two adjoint record buffers
  double* q1;               // [n][3] q(1) of the latest evaluation
  double* grad;             // [n][3] gradient of the latest evaluation
  int* flag;                // non-finite flag
  int spt;                  // records per step: 1 (Euler), 4 (Runge-Kutta stages)
  double *rk_acc, *rk_lam;  // [6][n] each, Runge-Kutta steps only
};

// Waves per workgroup of the batched pair kernels.  On the 48-job serving
// stream (FP32-compensated, Euler steps) 12-wave workgroups gave 15.7 solves/s
// against 14.9 for 8-wave and 13.8 for 16-wave ones: two 12-wave workgroups
// fill the 24 wave slots per CU that the adjoint's registers leave.  FP32,
// FP64 and Runge-Kutta stage instances keep 8 (their registers differ; 12 was
// measured only in the FP32-compensated Euler case).
constexpr int batch_waves(bool compensated, bool rk) { return compensated && !rk ? 12 : 8; }

// Launch shapes of a batch of at most max_slots jobs with n <= max_n:
// stage (max_n/256, max_slots), pair kernels `capacity` workgroups (one per
// (job, i-block) item), loss max_slots.  items holds nitems[0] items of 3D
// jobs followed by nitems[1] items of planar jobs; the pair launch for dim 3
// (or 2) takes its group, and its workgroups beyond the group's count exit.
hipError_t launch_stage_batch(int mode, const BatchJob* jobs, int max_slots, int max_n,
                              hipStream_t s);
// stage: 0 for an Euler step, else the Runge-Kutta stage (1..4) of step t;
// every job of the batch takes steps of the same kind.
hipError_t launch_fwd_batch(int mode, int dim, const BatchJob* jobs, const int2* items,
                            const int* nitems, int capacity, int t, int stage, hipStream_t s);
hipError_t launch_loss_batch(int mode, const BatchJob* jobs, int max_slots, hipStream_t s);
hipError_t launch_adj_batch(int mode, int dim, const BatchJob* jobs, const int2* items,
                            const int* nitems, int capacity, int t, int stage, int T,
                            hipStream_t s);

}  // namespace lddmm
