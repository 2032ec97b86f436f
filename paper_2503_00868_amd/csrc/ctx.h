// Host-side context of the fluidsim library and the launchers the runtime
// calls.  Every launcher only enqueues work on ctx->stream.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fluidsim.h"

namespace fs {

// Device scalar slots (double) and flag slots (int) used by the solvers.
enum ScalarSlot {
  S_BB = 0,    // |b|^2
  S_RZ,        // r.z of the current iterate
  S_RZ_PREV,   // r.z of the previous iterate
  S_DQ,        // d.Ad
  S_BETA,      // direction update coefficient
  S_RR,        // true residual |b - Ax|^2 at the last check
  S_ZQ,        // z.q (flexible CG)
  S_DR,        // d.r (flexible CG)
  S_DOT0,      // general-purpose reduction results
  S_DOT1,
  S_DOT2,
  S_ALPHA_PREV,  // alpha of the previous iteration (two-step iterate update)
  S_NET_SUMSQ,   // learned preconditioner: |r|^2 of its input
  S_NET_RMS,     //   rms of r over liquid cells
  S_NET_RZ,      //   training: r.z, r.e, z.Az (contiguous)
  S_NET_RE,
  S_NET_ZAZ,
  S_ALPHA_Q0,    // alphas of the first three iterations of a four-step iterate update
  S_ALPHA_Q1,
  S_ALPHA_Q2,
  S_ADV_DT,      // backward: sum over steps of <lam, d advect / d dt> (departure-point motion)
  S_LSUM0,       //   sums over steps of the adjoint at the body force, per component
  S_LSUM1,       //   (active faces): dJ/dg_c = dt * S_LSUMc
  S_LSUM2,
  S_GUESS0,      // scaled warm start: x.b, x.Ax (and two unused)
  S_GUESS1,
  S_GUESS2,
  S_GUESS3,
  S_COUNT = 32
};
// F_DONE: 0 running, 1 converged, 2 breakdown, 3 (flexible and viscosity CG)
// the recursive residual met the tolerance inside a block of iterations: the
// block's remaining iterations are skipped, the flexible CG's iterate update
// and the FP64 check still run, and the check turns 3 into 1, or into 0 with
// a restart (beta = 0: F_RESTART for the flexible CG's beta).
enum FlagSlot { F_DONE = 0, F_ITERS, F_ITERS_AT_DONE, F_BAD, F_RESTART, F_COUNT = 16 };

struct F3 {
  float* c[3];
};
struct CF3 {
  const float* c[3];
};

// Kinds of preconditioner application inside the Poisson CG.
enum PrecKind { PK_JACOBI = 0, PK_ZARRAY = 1 };

// What the one-block finalize kernel does with the summed partials
// ([...] lists the partial sums per block it expects).
enum FinMode : int {
  FIN_PCG_INIT = 0,  // [bb, rz]      -> BB, RR, RZ, RZ_PREV, BETA = 0; flags reset
  FIN_DQ,            // [dq]          -> DQ; iteration counted; breakdown if dq <= 0
  FIN_RZ_UPD,        // [rz]          -> RZ_PREV = RZ, RZ, BETA = rz / RZ_PREV
  FIN_RZ_FIRST,      // [rz]          -> RZ, RZ_PREV, BETA = 0
  FIN_CHECK,         // [rr, rz]      -> RR; (jacobi) RZ, BETA, else NET_SUMSQ = |r|^2; done at tol
  FIN_FCG_DQDR,      // [dq, dr]      -> DQ, DR; iteration counted; breakdown
  FIN_FCG_BETA,      // [zq]          -> BETA = -zq / DQ
  FIN_DCG_INIT,      // [bb, rz, rr]  -> BB, RZ, RZ_PREV, RR, BETA = 0; done at tol
  FIN_SLOT,          // [v]           -> scal[slot] = (acc ? scal[slot] : 0) + scale * v
  FIN_SLOTS4,        // [v0..v3]      -> scal[slot + q] = (acc ? scal[slot + q] : 0) + scale * vq
  FIN_FCG_RR,        // [rr]          -> NET_SUMSQ; at tol (phase = slot < 3): F_DONE = 3, later alphas 0
  FIN_DCG_UPD,       // [rz, rr]      -> as FIN_RZ_UPD; F_DONE = 3 when rr meets tol
};

}  // namespace fs

struct UNetState;
struct Profiler;

struct sim_ctx {
  sim_desc desc;
  sim_params params;
  int params_set = 0;
  int n = 0;
  hipStream_t stream = nullptr;
  int64_t C = 0;  // cells
  int64_t F = 0;  // faces per component
  int64_t n_active = 0;
  int64_t n_liquid = 0;

  // per-mask tables
  uint8_t* cell = nullptr;   // C
  uint8_t* cdiag = nullptr;  // C: Poisson diagonal (0 off liquid)
  uint8_t* fcode = nullptr;  // 3F: face codes, stacked u|v|w

  // Poisson solver vectors (cells)
  double* x = nullptr;
  float* r = nullptr;
  float* z = nullptr;
  float* dA = nullptr;
  float* dB = nullptr;
  float* dC = nullptr;      // Jacobi-PCG: four rotating direction buffers dA..dD
  float* dD = nullptr;
  float* q = nullptr;
  float* b = nullptr;
  float* rprev = nullptr;   // flexible CG
  float* precon = nullptr;  // MIC(0) factor
  float* mq = nullptr;      // MIC(0) forward-sweep result
  double* pc_acc = nullptr; // recurrent conv solver: weight-gradient sums (28)
  // warm starts: the last three pressures of the rollout's forward steps (xw
  // newest, xw2, xw3) and how many are known; the previous adjoint pressure
  double* xw = nullptr;
  double* xw2 = nullptr;
  double* xw3 = nullptr;
  int warm_n = 0;
  double* xwa = nullptr;

  // face-domain buffers, each 3F stacked
  float* tmp = nullptr;  // advection output / diffusion right-hand side
  double* fx = nullptr;  // FP64 iterate of the viscosity solve
  float* fr = nullptr;
  float* fdA = nullptr;
  float* fdB = nullptr;
  float* fq = nullptr;
  float* lam = nullptr;   // adjoint state
  float* lam2 = nullptr;  // adjoint scratch

  // reductions
  double* partials = nullptr;
  double* scal = nullptr;
  int* flags = nullptr;
  int* work = nullptr;  // SIM_KERN_COUNT counters: launches that did work (timing hooks)

  // rollout recording
  float* ckpt = nullptr;  // (ckpt_slots) x 3F
  double* ckpt_x = nullptr;   // warm start: (ckpt_slots) x C pressures xw at the checkpoints
  double* ckpt_x2 = nullptr;  // and xw2
  double* ckpt_x3 = nullptr;  // and xw3
  std::vector<int> ckpt_warm;  // and warm_n
  double* xhist = nullptr;   // store_pressures: max_steps x C pressures of the recorded steps
  float* vhist = nullptr;    // store_pressures: max_steps x 3F implicit viscosity outputs
  int ckpt_slots = 0;
  float* seg = nullptr;  // (2 * checkpoint_every) x 3F: state and diffusion operand per step
  int rec_steps = 0;
  int recorded = 0;

  // learned preconditioner
  UNetState* net = nullptr;
  void* net_ws = nullptr;
  size_t net_ws_bytes = 0;

  // launch shapes
  int grid_cells = 0;  // blocks for cell-domain kernels
  int grid_faces = 0;  // blocks per component for face-domain kernels

  // host readback
  double* h_scal = nullptr;  // pinned: S_COUNT doubles + F_COUNT ints
  Profiler* prof = nullptr;  // kernel timing (sim_profile_*), off by default
  std::string err;
};

namespace fs {

// Kernel timing: HIP events around the main kernel of each kind, recorded
// on ctx->stream when profiling is enabled (no-op otherwise).
void prof_mark(sim_ctx* c, int kind, bool begin);

// ---- launchers (k_*.hip) ----
void launch_finalize(sim_ctx* c, int nblocks, int nv, int mode, double tol2, int jacobi, int slot,
                     double scale, int acc);
void launch_setup_tables(sim_ctx* c);
void launch_mic0_setup(sim_ctx* c);
void launch_mic0_apply(sim_ctx* c, const float* r, float* z, const int* flags);

void launch_advect(sim_ctx* c, CF3 in, F3 out, float dth, const float force[3]);
void launch_diffuse_explicit(sim_ctx* c, CF3 in, F3 out, float alpha);
void launch_divergence(sim_ctx* c, CF3 in, float* b);
void launch_pressure_update(sim_ctx* c, const double* x, F3 u);
void launch_mask_scale(sim_ctx* c, CF3 in, F3 out, float s);
void launch_copy_faces(sim_ctx* c, CF3 in, F3 out);

// Poisson CG pieces
void launch_pcg_init(sim_ctx* c, int prec);
void launch_pcg_dir_spmv(sim_ctx* c, int prec, const float* d_in, float* d_out);
void launch_pcg_update(sim_ctx* c, int prec, const float* d);
// Jacobi only: odd iterations update r; even ones also x += a_prev d_prev + a d
void launch_pcg_update2(sim_ctx* c, const float* d, const float* d_prev, bool with_x);
// Jacobi-PCG with the FP64 iterate updated every fourth iteration: phase =
// iteration % 4; dirs[0..3] are the directions of iterations phase-3..phase
// of the current group (only dirs[3] is read before phase 3).
void launch_pcg_update4(sim_ctx* c, const float* const dirs[4], int phase);
// the same four-step iterate update for the flexible CG (alpha = d.r / d.q)
// also reduces |r|^2 into S_NET_SUMSQ (the learned preconditioner's input scale)
// check_follows: the FP64 check runs next (phase 3 then updates x alone)
void launch_fcg_update4(sim_ctx* c, const float* const dirs[4], int phase, double tol,
                        bool check_follows);
void launch_pcg_rz(sim_ctx* c);  // r.z with z from an explicit preconditioner, and beta
void launch_pcg_rz_first(sim_ctx* c, int first);
void launch_pcg_check(sim_ctx* c, int prec, double tol);
void launch_poisson_apply(sim_ctx* c, const float* x, float* y);
void launch_jacobi_apply(sim_ctx* c, const float* r, float* z);
// out = x over the cells; skipped when flags (nullable) has the done flag raised
void launch_x_to_double(sim_ctx* c, const double* x, double* out, const int* flags = nullptr);
// Polynomial extrapolation of the sequence ..., o, b, a (a newest) one step
// ahead, into o: order 2 (linear) o = 2 a - b; order 3 (quadratic)
// o = 3 a - 3 b + o.
void launch_x_extrapolate(sim_ctx* c, const double* a, const double* b, double* o, int order);
void launch_guess_scale(sim_ctx* c, double* x);
// out = (float)(xref - x) over the cells (FP64 difference)
void launch_err_snapshot(sim_ctx* c, const double* xref, float* out);

// flexible CG pieces (learned preconditioner)
void launch_fcg_init(sim_ctx* c);
void launch_fcg_dir_spmv(sim_ctx* c, const float* d_in, float* d_out);
void launch_fcg_update(sim_ctx* c, const float* d);
void launch_fcg_beta(sim_ctx* c);
void launch_fcg_beta_first(sim_ctx* c, int first);
void launch_fcg_check(sim_ctx* c, double tol);
// beta from z.q block partials that the network's output layer reduced
void launch_fcg_beta_partials(sim_ctx* c, int nblocks);

// implicit viscosity CG pieces (face domain, FP64 iterate ctx->fx, rhs ctx->tmp)
void launch_dcg_init(sim_ctx* c, float alpha);
void launch_dcg_dir_spmv(sim_ctx* c, float alpha, const float* d_in, float* d_out);
void launch_dcg_update(sim_ctx* c, float alpha, const float* d, double tol);
void launch_dcg_check(sim_ctx* c, float alpha, double tol);
void launch_dcg_finish(sim_ctx* c, F3 out);

// adjoint and loss
// Adds (d advect / d u)^T lam to g (scatter = true; g is not touched when
// false) and accumulates into scal[S_ADV_DT] the sum over active faces of
// lam * d advect / d dt, and into scal[S_LSUM0 + c] the sum of lam over the
// active c-faces (accumulate = 0 first clears the four slots).
void launch_advect_adjoint(sim_ctx* c, CF3 u, CF3 lam, F3 g, float dth, bool scatter,
                           int accumulate);
// The paper's upwind convection surrogate of the advection adjoint: g =
// lam - dt sum_c Lam_c D_i V_c on active faces (0 elsewhere), v the
// convected field (upwind.hip).
void launch_convection_grad_upwind(sim_ctx* c, CF3 v, CF3 lam, F3 g);
void launch_zero_faces(sim_ctx* c, F3 out);
// scal[slot] = (accumulate ? scal[slot] : 0) + scale * <a, L y>
void launch_dot_lap(sim_ctx* c, CF3 a, CF3 y, int slot, double scale, int accumulate);
void launch_dot_faces(sim_ctx* c, CF3 a, CF3 b, int slot, int masked);
void launch_loss_mse(sim_ctx* c, CF3 u, CF3 t, F3 g, int slot);
void launch_axpy_faces(sim_ctx* c, CF3 a, F3 y, float alpha);

}  // namespace fs
