// Host runtime and C ABI of fluidsim: argument validation, workspace
// carving, the conjugate-gradient drivers, the step and rollout loop, and
// the checkpointed reverse pass.  Device work is enqueued on the caller's
// stream; the only device-to-host traffic is the solver's control block
// (scalars and flags) once per convergence check.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "ctx.h"
#include "net.h"

using namespace fs;

struct Profiler {
  static constexpr int kPairs = 1 << 15;
  bool on = false;
  std::vector<hipEvent_t> ev;  // 2 per timed launch
  std::vector<int> kind;
  int used = 0;   // events recorded
  int open = -1;  // index of an unmatched begin event
  double ms[SIM_KERN_COUNT] = {};
  int64_t launches[SIM_KERN_COUNT] = {};
};

// Folds the recorded event pairs into the per-kind totals and frees the
// events for reuse (waits for the last recorded event).
static hipError_t prof_drain(Profiler* p) {
  int pairs = p->used / 2;
  if (pairs == 0) return hipSuccess;
  hipError_t e = hipEventSynchronize(p->ev[2 * pairs - 1]);
  if (e != hipSuccess) return e;
  for (int q = 0; q < pairs; ++q) {
    float t = 0.f;
    e = hipEventElapsedTime(&t, p->ev[2 * q], p->ev[2 * q + 1]);
    if (e != hipSuccess) return e;
    p->ms[p->kind[q]] += t;
    p->launches[p->kind[q]] += 1;
  }
  p->used = 0;
  return hipSuccess;
}

void fs::prof_mark(sim_ctx* c, int kind, bool begin) {
  Profiler* p = c->prof;
  if (!p || !p->on) return;
  if (begin) {
    if (p->used + 2 > (int)p->ev.size() && prof_drain(p) != hipSuccess) return;
    if (hipEventRecord(p->ev[p->used], c->stream) != hipSuccess) return;
    p->kind[p->used / 2] = kind;
    p->open = p->used++;
  } else {
    if (p->open < 0) return;
    if (hipEventRecord(p->ev[p->used], c->stream) != hipSuccess) return;
    p->used++;
    p->open = -1;
  }
}

namespace {

constexpr size_t kAlign = 256;
constexpr int kCtrlBytes = S_COUNT * sizeof(double) + F_COUNT * sizeof(int);

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Carver {
  char* base;  // nullptr: only count
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    size_t o = off;
    off = align_up(off + count * sizeof(T));
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

int grid_for(int64_t elems) {
  int64_t g = (elems + kBlock * 4 - 1) / (kBlock * 4);
  g = (g + 7) / 8 * 8;
  if (g < 8) g = 8;
  if (g > kMaxGrid) g = kMaxGrid;
  return (int)g;
}

bool recording_enabled(const sim_desc& d) { return d.max_steps > 0; }

// Lays out every buffer of a context; with c == nullptr only sizes.
size_t carve(const sim_desc& d, char* base, sim_ctx* c) {
  Carver cv{base};
  const int n = d.n;
  const int64_t C = cells(n), F = face_count(n), F3n = 3 * F;
  sim_ctx dummy;
  sim_ctx* t = c ? c : &dummy;
  t->cell = cv.take<uint8_t>(C);
  t->cdiag = cv.take<uint8_t>(C);
  t->fcode = cv.take<uint8_t>(F3n);
  t->x = cv.take<double>(C);
  t->r = cv.take<float>(C);
  t->z = cv.take<float>(C);
  t->dA = cv.take<float>(C);
  t->dB = cv.take<float>(C);
  const bool four = d.precond == SIM_PRECOND_JACOBI || d.precond == SIM_PRECOND_LEARNED;
  t->dC = four ? cv.take<float>(C) : nullptr;
  t->dD = four ? cv.take<float>(C) : nullptr;
  t->q = cv.take<float>(C);
  t->b = cv.take<float>(C);
  const bool mic = d.precond == SIM_PRECOND_MIC0;
  t->precon = mic ? cv.take<float>(C) : nullptr;
  t->mq = mic ? cv.take<float>(C) : nullptr;
  t->rprev = d.precond == SIM_PRECOND_LEARNED ? cv.take<float>(C) : nullptr;
  t->xw = d.warm_start ? cv.take<double>(C) : nullptr;
  t->xw2 = d.warm_start ? cv.take<double>(C) : nullptr;
  t->xw3 = d.warm_start ? cv.take<double>(C) : nullptr;
  t->xwa = d.warm_start ? cv.take<double>(C) : nullptr;
  t->tmp = cv.take<float>(F3n);
  t->fx = cv.take<double>(F3n);
  t->fr = cv.take<float>(F3n);
  t->fdA = cv.take<float>(F3n);
  t->fdB = cv.take<float>(F3n);
  t->fq = cv.take<float>(F3n);
  t->lam = cv.take<float>(F3n);
  t->lam2 = cv.take<float>(F3n);
  t->partials = cv.take<double>((size_t)kPartialDoubles);
  t->pc_acc = cv.take<double>(32);
  // control block: scalars then flags, copied to the host in one transfer
  char* ctrl = cv.take<char>(kCtrlBytes);
  t->scal = reinterpret_cast<double*>(ctrl);
  t->flags = ctrl ? reinterpret_cast<int*>(ctrl + S_COUNT * sizeof(double)) : nullptr;
  t->work = cv.take<int>(SIM_KERN_COUNT);
  if (recording_enabled(d)) {
    t->ckpt_slots = (d.max_steps + d.checkpoint_every - 1) / d.checkpoint_every;
    t->ckpt = cv.take<float>((size_t)t->ckpt_slots * F3n);
    t->ckpt_x = d.warm_start ? cv.take<double>((size_t)t->ckpt_slots * C) : nullptr;
    t->ckpt_x2 = d.warm_start ? cv.take<double>((size_t)t->ckpt_slots * C) : nullptr;
    t->ckpt_x3 = d.warm_start ? cv.take<double>((size_t)t->ckpt_slots * C) : nullptr;
    t->xhist = d.store_pressures ? cv.take<double>((size_t)d.max_steps * C) : nullptr;
    t->vhist = d.store_pressures && d.diffusion != SIM_DIFFUSION_EXPLICIT
                   ? cv.take<float>((size_t)d.max_steps * F3n)
                   : nullptr;
    t->seg = cv.take<float>((size_t)2 * d.checkpoint_every * F3n);
  } else {
    t->ckpt_slots = 0;
    t->ckpt = nullptr;
    t->ckpt_x = nullptr;
    t->ckpt_x2 = nullptr;
    t->ckpt_x3 = nullptr;
    t->xhist = nullptr;
    t->vhist = nullptr;
    t->seg = nullptr;
  }
  if (d.precond == SIM_PRECOND_LEARNED) {
    size_t nb = net_workspace_bytes(n);
    t->net_ws = cv.take<char>(nb);
    t->net_ws_bytes = nb;
  } else {
    t->net_ws = nullptr;
    t->net_ws_bytes = 0;
  }
  return cv.off;
}

const char* validate_desc(const sim_desc* d) {
  if (!d) return "desc is NULL";
  if (d->n < 4 || d->n > 1024) return "n must be in [4, 1024]";
  if (d->precond < SIM_PRECOND_JACOBI || d->precond > SIM_PRECOND_LEARNED)
    return "precond must be JACOBI, MIC0 or LEARNED";
  if (d->precond == SIM_PRECOND_LEARNED && d->n % 4 != 0)
    return "the learned preconditioner needs n divisible by 4";
  if (d->diffusion < SIM_DIFFUSION_AUTO || d->diffusion > SIM_DIFFUSION_IMPLICIT)
    return "diffusion must be AUTO, EXPLICIT or IMPLICIT";
  if (d->max_iter < 1) return "max_iter must be >= 1";
  if (d->check_every < 1 || d->check_every > 1024) return "check_every must be in [1, 1024]";
  if (d->checkpoint_every < 1) return "checkpoint_every must be >= 1";
  if (d->max_steps < 0) return "max_steps must be >= 0";
  if (d->precond == SIM_PRECOND_LEARNED && d->learned_max_iter < 1)
    return "learned_max_iter must be >= 1";
  if (!(d->tol > 0.0 && d->tol < 1.0)) return "tol must be in (0, 1)";
  if (!(d->diff_tol > 0.0 && d->diff_tol < 1.0)) return "diff_tol must be in (0, 1)";
  if (d->warm_start != 0 && d->warm_start != 1) return "warm_start must be 0 or 1";
  if (d->store_pressures != 0 && d->store_pressures != 1) return "store_pressures must be 0 or 1";
  if (d->store_pressures && d->max_steps == 0) return "store_pressures needs max_steps > 0";
  if (d->convection_grad != SIM_CONVGRAD_EXACT && d->convection_grad != SIM_CONVGRAD_UPWIND)
    return "convection_grad must be EXACT or UPWIND";
  return nullptr;
}

// Host check of the cell types: values in {0,1,2}, and every 6-connected
// liquid region shares a face with an air cell (else the Poisson matrix of
// that region is singular: pure Neumann).
int check_mask(int n, const uint8_t* cell, std::string& err, int64_t& n_liquid) {
  const int64_t C = cells(n);
  n_liquid = 0;
  for (int64_t q = 0; q < C; ++q) {
    if (cell[q] > 2) {
      err = "cell types must be 0 (air), 1 (liquid) or 2 (solid)";
      return SIM_ERR_INVALID_ARG;
    }
    n_liquid += cell[q] == 1;
  }
  std::vector<uint8_t> seen(C, 0);
  std::vector<int64_t> stack;
  for (int64_t s0 = 0; s0 < C; ++s0) {
    if (cell[s0] != 1 || seen[s0]) continue;
    bool touches_air = false;
    stack.clear();
    stack.push_back(s0);
    seen[s0] = 1;
    while (!stack.empty()) {
      int64_t q = stack.back();
      stack.pop_back();
      int i = (int)(q % n), j = (int)((q / n) % n), k = (int)(q / ((int64_t)n * n));
      const int nb[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
      for (auto& o : nb) {
        int ii = i + o[0], jj = j + o[1], kk = k + o[2];
        if (ii < 0 || jj < 0 || kk < 0 || ii >= n || jj >= n || kk >= n) continue;
        int64_t m = ii + (int64_t)n * (jj + (int64_t)n * kk);
        if (cell[m] == 0) touches_air = true;
        if (cell[m] == 1 && !seen[m]) {
          seen[m] = 1;
          stack.push_back(m);
        }
      }
    }
    if (!touches_air) {
      err = "a liquid region touches no air cell (singular pressure system)";
      return SIM_ERR_SINGULAR_MASK;
    }
  }
  return SIM_OK;
}

// Active faces of the mask (for the loss normalisation).
int64_t count_active(int n, const uint8_t* cell) {
  auto ct = [&](int i, int j, int k) -> int {
    if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n) return 2;
    return cell[i + (int64_t)n * (j + (int64_t)n * k)];
  };
  int64_t cnt = 0;
  for (int comp = 0; comp < 3; ++comp) {
    Dims d = face_dims(n, comp);
    for (int k = 0; k < d.nz; ++k)
      for (int j = 0; j < d.ny; ++j)
        for (int i = 0; i < d.nx; ++i) {
          int a = ct(i - (comp == 0), j - (comp == 1), k - (comp == 2)), b = ct(i, j, k);
          if (a == 2 || b == 2) continue;
          cnt += (a == 1 || b == 1);
        }
  }
  return cnt;
}

#define HIPCHK(expr)                                                            \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      c->err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
      return SIM_ERR_HIP;                                                       \
    }                                                                           \
  } while (0)

int launch_status(sim_ctx* c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    c->err = std::string("kernel launch: ") + hipGetErrorString(e);
    return SIM_ERR_HIP;
  }
  return SIM_OK;
}

F3 f3(float* u, float* v, float* w) { return F3{{u, v, w}}; }
CF3 cf3(const float* u, const float* v, const float* w) { return CF3{{u, v, w}}; }
F3 stacked(sim_ctx* c, float* base) { return F3{{base, base + c->F, base + 2 * c->F}}; }
CF3 cstacked(sim_ctx* c, const float* base) {
  return CF3{{base, base + c->F, base + 2 * c->F}};
}

struct HostCtrl {
  double s[S_COUNT];
  int f[F_COUNT];
};

HostCtrl* host_slot(sim_ctx* c, int slot) { return reinterpret_cast<HostCtrl*>(c->h_scal) + slot; }

// The iteration driver shared by every CG variant.  `block` enqueues one
// block of m iterations followed by the FP64 check.  Blocks are enqueued one
// ahead of the host's read of the previous block's control block, so the
// GPU does not wait for the host between blocks; kernels of blocks enqueued
// after convergence return at once (they test the done flag).
struct LoopResult {
  int status;  // SIM_OK, SIM_ERR_NOT_CONVERGED or breakdown (2 in flags)
  int done;
  int iters;
  double rr, bb;
  bool stalled;  // stopped early: the residual fell too slowly (see run_blocks)
};

// min_rate (0: off): stop early when, between two consecutive checks, the
// true residual norm fell by less than a factor min_rate per iteration
// (the block already enqueued still runs).
template <typename Block>
int run_blocks(sim_ctx* c, int m, int max_iter, Block block, LoopResult& res,
               double min_rate = 0.0) {
  hipEvent_t ev[2];
  HIPCHK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  auto cleanup = [&]() {
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
  };
  int enq = 0, blk = 0;
  double rr_prev = -1.0;
  int it_prev = 0;
  res.stalled = false;
  for (;;) {
    int todo = std::min(m, max_iter - enq);
    block(todo);
    enq += todo;
    int rc = launch_status(c);
    if (rc) {
      cleanup();
      return rc;
    }
    HIPCHK(hipMemcpyAsync(host_slot(c, blk & 1), c->scal, kCtrlBytes, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipEventRecord(ev[blk & 1], c->stream));
    if (blk >= 1) {
      HIPCHK(hipEventSynchronize(ev[(blk - 1) & 1]));
      const HostCtrl* hp = host_slot(c, (blk - 1) & 1);
      if (hp->f[F_DONE]) break;
      if (min_rate > 0.0) {
        const double rr = hp->s[S_RR];
        const int it = hp->f[F_ITERS];
        if (rr_prev > 0.0 && it > it_prev &&
            std::pow(rr / rr_prev, 0.5 / (double)(it - it_prev)) > min_rate) {
          res.stalled = true;
          break;
        }
        rr_prev = rr;
        it_prev = it;
      }
    }
    if (enq >= max_iter) break;
    ++blk;
  }
  // the newest block's copy reflects the final state: blocks enqueued after
  // the done flag was raised change nothing
  HIPCHK(hipEventSynchronize(ev[blk & 1]));
  HostCtrl* hc = host_slot(c, blk & 1);
  cleanup();
  res.done = hc->f[F_DONE];
  res.iters = hc->f[F_DONE] == 1 ? hc->f[F_ITERS_AT_DONE] : hc->f[F_ITERS];
  res.rr = hc->s[S_RR];
  res.bb = hc->s[S_BB];
  res.status = res.done == 1 ? SIM_OK : SIM_ERR_NOT_CONVERGED;
  return SIM_OK;
}

double relres_of(const LoopResult& r) { return r.bb > 0 ? std::sqrt(r.rr / r.bb) : 0.0; }

// Starting iterate of a solve.
enum Start { START_ZERO, START_GUESS, START_CURRENT };

// x = x0 (FP64 copy) after the zero-start setup, then r = b - A x through the
// FP64 check with the solve's tolerance: a guess that already meets it ends
// the solve with no iteration.  With b = 0 the setup has already raised the
// done flag and x stays 0.
void start_from_guess(sim_ctx* c, int prec_kind, const double* x0) {
  launch_x_to_double(c, x0, c->x, c->flags);
  launch_pcg_check(c, prec_kind, c->desc.tol);
}

// PCG on the Poisson matrix with rhs c->b, result in c->x.  Jacobi is fused
// into the CG kernels; MIC(0) is applied between them.  The iterate starts at
// 0, at x0 (START_GUESS), or at the current c->x (START_CURRENT, a restart
// that keeps the scale ||b|| of the interrupted solve).
int pcg_solve(sim_ctx* c, int prec_kind, int start, const double* x0, sim_stats* st) {
  const int pk = prec_kind;
  if (start == START_CURRENT) {
    // restart from the current x: r = b - A x, fresh direction
    launch_pcg_check(c, pk, 0.0);
    HIPCHK(hipMemsetAsync(c->dA, 0, sizeof(float) * c->C, c->stream));
  } else {
    launch_pcg_init(c, pk);
    if (start == START_GUESS) start_from_guess(c, pk, x0);
  }
  if (pk == PK_ZARRAY) {
    launch_mic0_apply(c, c->r, c->z, c->flags);
    launch_pcg_rz_first(c, 1);
  }
  float* din = c->dA;
  float* dout = c->dB;
  const double tol = c->desc.tol;
  // Jacobi: the FP64 iterate is updated every fourth iteration (four
  // directions at once, from four rotating buffers; the initial direction
  // buffer dA is zero), so blocks hold a multiple of 4 iterations and every
  // check sees an up-to-date x.
  const bool four_step = pk == PK_JACOBI && c->dC && c->dD;
  const int group = four_step ? 4 : (pk == PK_JACOBI ? 2 : 1);
  const int m = (c->desc.check_every + group - 1) / group * group;
  const int max_it = (c->desc.max_iter + group - 1) / group * group;
  float* const dbuf[4] = {c->dA, c->dB, c->dC, c->dD};
  int it = 0;  // iterations enqueued in this solve
  auto block = [&](int todo) {
    for (int t = 0; t < todo; ++t, ++it) {
      if (four_step) {
        // iteration k reads dbuf[k % 4] (the previous direction) and writes dbuf[(k + 1) % 4]
        const int ph = it & 3;
        launch_pcg_dir_spmv(c, pk, dbuf[ph], dbuf[(ph + 1) & 3]);
        const float* dirs[4] = {dbuf[(ph + 2) & 3], dbuf[(ph + 3) & 3], dbuf[ph],
                                dbuf[(ph + 1) & 3]};
        launch_pcg_update4(c, dirs, ph);
        if (t == todo - 1) launch_pcg_check(c, pk, tol);
        continue;
      }
      launch_pcg_dir_spmv(c, pk, din, dout);
      if (pk == PK_JACOBI)
        launch_pcg_update2(c, dout, din, (t & 1) != 0);
      else
        launch_pcg_update(c, pk, dout);
      if (t == todo - 1) launch_pcg_check(c, pk, tol);
      if (pk == PK_ZARRAY) {
        launch_mic0_apply(c, c->r, c->z, c->flags);
        launch_pcg_rz(c);
      }
      std::swap(din, dout);
    }
  };
  LoopResult lr{};
  int rc = run_blocks(c, m, max_it, block, lr);
  if (rc) return rc;
  if (st) {
    st->iters += lr.iters;
    st->rel_residual = relres_of(lr);
  }
  if (lr.done == 2) {
    c->err = "PCG breakdown (non-positive curvature or NaN)";
    return SIM_ERR_NOT_CONVERGED;
  }
  if (lr.status != SIM_OK) c->err = "pressure solve did not reach tol within max_iter";
  return lr.status;
}

// Below this residual reduction per iteration the network does not pay for
// itself: one application costs about 20 Jacobi-PCG iterations, so even a
// factor 0.9 per iteration is slower than Jacobi-PCG on large grids.
constexpr double kFcgMinRate = 0.9;

// Flexible CG with the learned preconditioner.  On breakdown, after
// learned_max_iter iterations, or when the residual stalls (kFcgMinRate),
// it restarts Jacobi-PCG from the current x.
int fcg_solve(sim_ctx* c, const double* x0, sim_stats* st) {
  launch_fcg_init(c);
  if (x0) start_from_guess(c, PK_ZARRAY, x0);
  int rc = net_apply(c, c->r, c->z, c->flags);
  if (rc) return rc;
  launch_fcg_beta_first(c, 1);
  // the FP64 iterate is updated every fourth iteration from four rotating
  // direction buffers (as in Jacobi-PCG), so blocks hold multiples of 4
  const double tol = c->desc.tol;
  int inner_rc = SIM_OK;
  float* const dbuf[4] = {c->dA, c->dB, c->dC, c->dD};
  const int zq_blocks = net_conv_out_blocks(c->n);
  const bool zq_fused = zq_blocks <= kPartialDoubles;
  int it = 0;
  auto block = [&](int todo) {
    for (int t = 0; t < todo; ++t, ++it) {
      const int ph = it & 3;
      launch_fcg_dir_spmv(c, dbuf[ph], dbuf[(ph + 1) & 3]);
      const float* dirs[4] = {dbuf[(ph + 2) & 3], dbuf[(ph + 3) & 3], dbuf[ph], dbuf[(ph + 1) & 3]};
      // the update ends the block early when the recursive residual meets the
      // tolerance; the FP64 check runs at block ends only, where x is up to date
      launch_fcg_update4(c, dirs, ph, tol, t == todo - 1);
      if (t == todo - 1) launch_fcg_check(c, tol);
      // |r|^2 for the network: reduced by the update, or by the check when it
      // has just replaced r by the true residual; z.q for beta: reduced by
      // the network's output layer (when its block partials fit)
      int r2 = net_apply(c, c->r, c->z, c->flags, true, zq_fused ? c->q : nullptr);
      if (r2) inner_rc = r2;
      if (zq_fused)
        launch_fcg_beta_partials(c, zq_blocks);
      else
        launch_fcg_beta(c);
    }
  };
  const int m = (c->desc.check_every + 3) / 4 * 4;
  const int max_it = (std::min(c->desc.learned_max_iter, c->desc.max_iter) + 3) / 4 * 4;
  LoopResult lr{};
  rc = run_blocks(c, m, max_it, block, lr, kFcgMinRate);
  if (rc) return rc;
  if (inner_rc) return inner_rc;
  if (st) {
    st->iters += lr.iters;
    st->rel_residual = relres_of(lr);
  }
  if (lr.done == 1) return SIM_OK;
  // fallback: Jacobi-PCG from the current iterate, judged by the same FP64
  // check (on this chip it beats MIC(0)-PCG, whose hyperplane sweeps are
  // latency-bound, from 64^3 up)
  if (st) st->fallback_used = 1;
  HIPCHK(hipMemsetAsync(c->flags, 0, sizeof(int) * F_COUNT, c->stream));
  rc = pcg_solve(c, PK_JACOBI, START_CURRENT, nullptr, st);
  if (rc == SIM_OK) return SIM_OK_FALLBACK;
  return rc;
}

// x0 (nullable): starting iterate.
// A learned context without weights solves with Jacobi-PCG.
int poisson_solve(sim_ctx* c, const double* x0, sim_stats* st) {
  if (c->desc.precond == SIM_PRECOND_LEARNED && net_ready(c)) return fcg_solve(c, x0, st);
  return pcg_solve(c, c->desc.precond == SIM_PRECOND_MIC0 ? PK_ZARRAY : PK_JACOBI,
                   x0 ? START_GUESS : START_ZERO, x0, st);
}

bool diffusion_explicit(sim_ctx* c) {
  if (c->desc.diffusion == SIM_DIFFUSION_EXPLICIT) return true;
  if (c->desc.diffusion == SIM_DIFFUSION_IMPLICIT) return false;
  const double lam = c->params.nu * c->params.dt * (double)c->n * (double)c->n;
  return lam <= 1.0 / 12.0;
}

float diffusion_alpha(sim_ctx* c) {
  return (float)(c->params.nu * c->params.dt * (double)c->n * (double)c->n);
}

// Solve (I - alpha L) x = c->tmp on the active faces (initial guess: the
// right-hand side) and round the FP64 solution into out.
int diffuse_implicit(sim_ctx* c, F3 out, sim_stats* st) {
  const float alpha = diffusion_alpha(c);
  launch_dcg_init(c, alpha);
  float* din = c->fdA;
  float* dout = c->fdB;
  const double tol = c->desc.diff_tol;
  auto block = [&](int todo) {
    for (int t = 0; t < todo; ++t) {
      launch_dcg_dir_spmv(c, alpha, din, dout);
      launch_dcg_update(c, alpha, dout, tol);  // may end the block early
      if (t == todo - 1) launch_dcg_check(c, alpha, tol);
      std::swap(din, dout);
    }
  };
  LoopResult lr{};
  int rc = run_blocks(c, c->desc.check_every, c->desc.max_iter, block, lr);
  if (rc) return rc;
  launch_dcg_finish(c, out);
  if (st) {
    st->diff_iters += lr.iters;
    st->diff_rel_residual = relres_of(lr);
  }
  if (lr.status != SIM_OK) c->err = "viscosity solve did not reach diff_tol within max_iter";
  int ls = launch_status(c);
  return ls ? ls : lr.status;
}

// Viscosity sub-step: out = D(c->tmp).
int diffuse_into(sim_ctx* c, F3 out, sim_stats* st) {
  if (diffusion_explicit(c)) {
    launch_diffuse_explicit(c, cstacked(c, c->tmp), out, diffusion_alpha(c));
    return launch_status(c);
  }
  return diffuse_implicit(c, out, st);
}

// Pressure projection of (u, v, w) in place; non-active faces (the adjoint
// state can carry values there) count as zero in the divergence and are
// zeroed by the pressure update.  warm (nullable): the solve starts from it
// and the new pressure is stored back into it.
// scale_warm: the start is first rescaled to the multiple of it closest to
// the new solution in the A-norm (the adjoint solves, whose right-hand sides
// change in size from step to step).
int project_inplace(sim_ctx* c, F3 u, sim_stats* st, double* warm = nullptr,
                    bool scale_warm = false) {
  CF3 cu = cf3(u.c[0], u.c[1], u.c[2]);
  launch_divergence(c, cu, c->b);
  if (warm && scale_warm) launch_guess_scale(c, warm);
  int rc = poisson_solve(c, warm, st);
  if (rc != SIM_OK && rc != SIM_OK_FALLBACK) return rc;
  if (warm) launch_x_to_double(c, c->x, warm);
  launch_pressure_update(c, c->x, u);
  int lr = launch_status(c);
  return lr ? lr : rc;
}

void advect_force(sim_ctx* c, CF3 in, F3 out) {
  const float dth = (float)(c->params.dt * c->n);
  const float force[3] = {(float)(c->params.dt * c->params.gravity[0]),
                          (float)(c->params.dt * c->params.gravity[1]),
                          (float)(c->params.dt * c->params.gravity[2])};
  launch_advect(c, in, out, dth, force);
}

// Warm-started projection of a rollout's forward step: the solve starts from
// the quadratic extrapolation 3 x1 - 3 x2 + x3 of the last three steps'
// pressures (x1 newest; the linear 2 x1 - x2 with two known, x1 with fewer;
// x1 is zero at the rollout's start), and its pressure becomes x1.  The guess
// is formed in x3's storage, the solve stores into it, and the pointers
// rotate.  (Measured at 256^3 over the benchmark rollout, flexible-CG
// iterations per forward solve: 30.8 from x1, 25.3 linear, 24.3 quadratic;
// weights 0.7 and 1.3 on the linear difference instead of 1 gave 27.6 and
// 26.7.  The adjoint solves, whose right-hand sides change less smoothly
// from step to step, ran more iterations from a linear extrapolation and
// keep the previous pressure.)
int project_warm(sim_ctx* c, F3 u, sim_stats* st) {
  if (!c->xw || !c->xw2 || !c->xw3) return project_inplace(c, u, st, c->xw);
  double* guess = c->xw3;
  if (c->warm_n >= 3)
    launch_x_extrapolate(c, c->xw, c->xw2, guess, 3);
  else if (c->warm_n == 2)
    launch_x_extrapolate(c, c->xw, c->xw2, guess, 2);
  else
    launch_x_to_double(c, c->xw, guess);
  const int rc = project_inplace(c, u, st, guess);
  c->xw3 = c->xw2;
  c->xw2 = c->xw;
  c->xw = guess;
  if (c->warm_n < 3) ++c->warm_n;
  return rc;
}

// One step in place: advect (+force) -> viscosity -> projection.
// rec_step >= 0: a recorded step whose implicit viscosity output is kept in
// the history (store_pressures).
int step_once(sim_ctx* c, F3 u, sim_stats* st, int rec_step = -1) {
  advect_force(c, cf3(u.c[0], u.c[1], u.c[2]), stacked(c, c->tmp));
  int rc = diffuse_into(c, u, st);
  if (rc) return rc;
  if (rec_step >= 0 && c->vhist && !diffusion_explicit(c))
    launch_copy_faces(c, cf3(u.c[0], u.c[1], u.c[2]),
                      stacked(c, c->vhist + (int64_t)rec_step * 3 * c->F));
  return project_warm(c, u, st);
}

int combine(int a, int b) {
  if (a < 0) return a;
  if (b < 0) return b;
  return a > b ? a : b;
}

bool check_ctx(sim_ctx* c) { return c != nullptr; }

}  // namespace

// =================================================================== ABI

extern "C" {

int sim_workspace_size(const sim_desc* desc, size_t* bytes) {
  if (!bytes || validate_desc(desc)) return SIM_ERR_INVALID_ARG;
  *bytes = carve(*desc, nullptr, nullptr);
  return SIM_OK;
}

int sim_create(const sim_desc* desc, const uint8_t* h_cell_type, void* d_workspace,
               size_t workspace_bytes, void* hip_stream, sim_ctx** out) {
  if (!out) return SIM_ERR_INVALID_ARG;
  *out = nullptr;
  if (validate_desc(desc) || !h_cell_type || !d_workspace) return SIM_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign != 0) return SIM_ERR_INVALID_ARG;
  const size_t need = carve(*desc, nullptr, nullptr);
  if (workspace_bytes < need) return SIM_ERR_WORKSPACE_TOO_SMALL;
  std::string err;
  int64_t n_liquid = 0;
  int mrc = check_mask(desc->n, h_cell_type, err, n_liquid);
  if (mrc) return mrc;

  sim_ctx* c = new (std::nothrow) sim_ctx();
  if (!c) return SIM_ERR_INVALID_ARG;
  c->desc = *desc;
  c->n = desc->n;
  c->C = cells(c->n);
  c->F = face_count(c->n);
  c->n_liquid = n_liquid;
  c->n_active = count_active(c->n, h_cell_type);
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  carve(*desc, reinterpret_cast<char*>(d_workspace), c);
  c->ckpt_warm.assign((size_t)c->ckpt_slots, 0);
  c->grid_cells = grid_for(c->C);
  c->grid_faces = grid_for(c->F);
  auto fail = [&](int code) {
    if (c->h_scal) (void)hipHostFree(c->h_scal);
    delete c;
    return code;
  };
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_scal), 2 * kCtrlBytes, 0) != hipSuccess)
    return fail(SIM_ERR_HIP);
  if (hipMemcpyAsync(c->cell, h_cell_type, c->C, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return fail(SIM_ERR_HIP);
  if (hipMemsetAsync(c->scal, 0, kCtrlBytes, c->stream) != hipSuccess) return fail(SIM_ERR_HIP);
  if (hipMemsetAsync(c->work, 0, sizeof(int) * SIM_KERN_COUNT, c->stream) != hipSuccess)
    return fail(SIM_ERR_HIP);
  for (double* wbuf : {c->xw, c->xw2, c->xw3, c->xwa})
    if (wbuf && hipMemsetAsync(wbuf, 0, sizeof(double) * c->C, c->stream) != hipSuccess)
      return fail(SIM_ERR_HIP);
  launch_setup_tables(c);
  if (c->precon) {
    if (hipMemsetAsync(c->precon, 0, sizeof(float) * c->C, c->stream) != hipSuccess)
      return fail(SIM_ERR_HIP);
    launch_mic0_setup(c);
  }
  if (desc->precond == SIM_PRECOND_LEARNED && net_init(c, h_cell_type) != SIM_OK) return fail(SIM_ERR_HIP);
  if (hipGetLastError() != hipSuccess) return fail(SIM_ERR_HIP);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(SIM_ERR_HIP);
  *out = c;
  return SIM_OK;
}

int sim_profile_enable(sim_ctx* c, int32_t on) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (on && !c->prof) {
    Profiler* p = new (std::nothrow) Profiler();
    if (!p) return SIM_ERR_INVALID_ARG;
    p->ev.resize(2 * Profiler::kPairs);
    p->kind.resize(Profiler::kPairs);
    for (auto& e : p->ev) {
      if (hipEventCreate(&e) != hipSuccess) {
        c->err = "hipEventCreate failed";
        return SIM_ERR_HIP;
      }
    }
    c->prof = p;
  }
  if (c->prof) {
    c->prof->on = on != 0;
    c->prof->used = 0;
    c->prof->open = -1;
    for (int k = 0; k < SIM_KERN_COUNT; ++k) c->prof->ms[k] = 0.0, c->prof->launches[k] = 0;
    HIPCHK(hipMemsetAsync(c->work, 0, sizeof(int) * SIM_KERN_COUNT, c->stream));
  }
  return SIM_OK;
}

int sim_profile_read(sim_ctx* c, double* h_ms, int64_t* h_launches) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!h_ms || !h_launches) {
    c->err = "NULL output";
    return SIM_ERR_INVALID_ARG;
  }
  Profiler* p = c->prof;
  for (int k = 0; k < SIM_KERN_COUNT; ++k) h_ms[k] = 0.0, h_launches[k] = 0;
  if (!p) return SIM_OK;
  HIPCHK(hipStreamSynchronize(c->stream));
  if (p->open >= 0) p->used = p->open;  // drop an unmatched begin
  HIPCHK(prof_drain(p));
  p->open = -1;
  // kinds whose kernels return at once once the solve has converged (the
  // launches of a block enqueued ahead): count the launches that did work
  int work[SIM_KERN_COUNT];
  HIPCHK(hipMemcpy(work, c->work, sizeof work, hipMemcpyDeviceToHost));
  HIPCHK(hipMemsetAsync(c->work, 0, sizeof work, c->stream));
  for (int k = 0; k < SIM_KERN_COUNT; ++k) {
    const bool skips = k == SIM_KERN_PCG_DIR_SPMV || k == SIM_KERN_PCG_UPDATE ||
                       k == SIM_KERN_PCG_CHECK || k == SIM_KERN_DCG_DIR_SPMV ||
                       k == SIM_KERN_DCG_UPDATE || k == SIM_KERN_NET;
    h_ms[k] = p->ms[k];
    h_launches[k] = skips ? std::min<int64_t>(work[k], p->launches[k]) : p->launches[k];
    p->ms[k] = 0.0;
    p->launches[k] = 0;
  }
  return SIM_OK;
}

int sim_destroy(sim_ctx* c) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (c->prof) {
    for (auto& e : c->prof->ev) (void)hipEventDestroy(e);
    delete c->prof;
  }
  net_destroy(c);
  if (c->h_scal) (void)hipHostFree(c->h_scal);
  delete c;
  return SIM_OK;
}

const char* sim_last_error(const sim_ctx* c) {
  if (!c) return "NULL context";
  return c->err.c_str();
}

int sim_set_params(sim_ctx* c, const sim_params* p) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!p) {
    c->err = "params is NULL";
    return SIM_ERR_INVALID_ARG;
  }
  if (!(p->nu > 0.0 && std::isfinite(p->nu))) {
    c->err = "nu must be > 0";
    return SIM_ERR_INVALID_ARG;
  }
  if (!(p->s > 0.0 && std::isfinite(p->s))) {
    c->err = "s must be > 0";
    return SIM_ERR_INVALID_ARG;
  }
  if (!(p->dt > 0.0 && std::isfinite(p->dt))) {
    c->err = "dt must be > 0";
    return SIM_ERR_INVALID_ARG;
  }
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->gravity[a])) {
      c->err = "gravity must be finite";
      return SIM_ERR_INVALID_ARG;
    }
  c->params = *p;
  c->params_set = 1;
  // a recorded rollout belongs to the parameters it ran with
  c->recorded = 0;
  return SIM_OK;
}

int sim_init_state(sim_ctx* c, const float* gu, const float* gv, const float* gw, float* u, float* v,
                   float* w) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!gu || !gv || !gw || !u || !v || !w) {
    c->err = "NULL field pointer";
    return SIM_ERR_INVALID_ARG;
  }
  if (!c->params_set) {
    c->err = "sim_set_params has not been called";
    return SIM_ERR_STATE;
  }
  launch_mask_scale(c, cf3(gu, gv, gw), f3(u, v, w), (float)c->params.s);
  if (c->xw) HIPCHK(hipMemsetAsync(c->xw, 0, sizeof(double) * c->C, c->stream));
  c->warm_n = 0;
  return launch_status(c);
}

int sim_step(sim_ctx* c, float* u, float* v, float* w, int32_t nsteps, int32_t record,
             sim_stats* stats) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!u || !v || !w || nsteps < 0) {
    c->err = "NULL field pointer or negative nsteps";
    return SIM_ERR_INVALID_ARG;
  }
  if (!c->params_set) {
    c->err = "sim_set_params has not been called";
    return SIM_ERR_STATE;
  }
  if (record && (!recording_enabled(c->desc) || nsteps > c->desc.max_steps)) {
    c->err = "record needs max_steps > 0 and nsteps <= max_steps";
    return SIM_ERR_INVALID_ARG;
  }
  if (record) {
    c->recorded = 0;
    c->rec_steps = nsteps;
  }
  F3 U = f3(u, v, w);
  const int K = c->desc.checkpoint_every;
  const int64_t F3n = 3 * c->F;
  int worst = SIM_OK;
  for (int s = 0; s < nsteps; ++s) {
    if (record && s % K == 0) {
      launch_copy_faces(c, cf3(u, v, w), stacked(c, c->ckpt + (int64_t)(s / K) * F3n));
      if (c->ckpt_x) {
        launch_x_to_double(c, c->xw, c->ckpt_x + (int64_t)(s / K) * c->C);
        launch_x_to_double(c, c->xw2, c->ckpt_x2 + (int64_t)(s / K) * c->C);
        launch_x_to_double(c, c->xw3, c->ckpt_x3 + (int64_t)(s / K) * c->C);
        c->ckpt_warm[s / K] = c->warm_n;
      }
    }
    sim_stats st{};
    int rc = step_once(c, U, &st, record ? s : -1);
    st.status = rc;
    if (stats) stats[s] = st;
    worst = combine(worst, rc);
    if (rc < 0) return rc;
    if (record && c->xhist) launch_x_to_double(c, c->x, c->xhist + (int64_t)s * c->C);
  }
  if (record) c->recorded = 1;
  HIPCHK(hipStreamSynchronize(c->stream));
  return worst;
}

int sim_project(sim_ctx* c, float* u, float* v, float* w, double* p_out, sim_stats* stats) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!u || !v || !w) {
    c->err = "NULL field pointer";
    return SIM_ERR_INVALID_ARG;
  }
  sim_stats st{};
  int rc = project_inplace(c, f3(u, v, w), &st);
  if (rc >= 0 && p_out) launch_x_to_double(c, c->x, p_out);
  st.status = rc;
  if (stats) *stats = st;
  HIPCHK(hipStreamSynchronize(c->stream));
  return rc;
}

int sim_loss_mse(sim_ctx* c, const float* u, const float* v, const float* w, const float* tu,
                 const float* tv, const float* tw, double* h_loss, float* gu, float* gv,
                 float* gw) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!u || !v || !w || !tu || !tv || !tw || !h_loss) {
    c->err = "NULL pointer";
    return SIM_ERR_INVALID_ARG;
  }
  if ((gu || gv || gw) && !(gu && gv && gw)) {
    c->err = "gradient pointers must be all set or all NULL";
    return SIM_ERR_INVALID_ARG;
  }
  launch_loss_mse(c, cf3(u, v, w), cf3(tu, tv, tw), f3(gu, gv, gw), S_DOT0);
  int rc = launch_status(c);
  if (rc) return rc;
  double val = 0.0;
  HIPCHK(hipMemcpyAsync(&val, c->scal + S_DOT0, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *h_loss = c->n_active > 0 ? val / (double)c->n_active : 0.0;
  return SIM_OK;
}

// Reverse pass over the recorded rollout, one checkpoint segment at a time:
// restore the segment's first state, recompute its steps while storing each
// state and its viscosity operand, then walk the steps backwards:
//   lam1 = P lam                        (projection is a symmetric projector)
//   explicit: dJ/dnu += dt <lam1, L a>,   lam2 = (I + nu dt L) lam1
//   implicit: mu = (I - nu dt L)^-1 lam1, dJ/dnu += dt <mu, L u**>, lam2 = mu
//   lam = (d advect / d u)^T lam2, or the paper's upwind surrogate of it
//   dJ/dg_c += dt sum_{active c-faces} lam2;  dJ/ddt += <lam2, d advect / d dt>
//                                                     + g . (those sums)
// and at the end dJ/ddt += (nu / dt) dJ/dnu (the viscous factor is nu dt).
int sim_backward(sim_ctx* c, const float* gu, const float* gv, const float* gw, const float* ugu,
                 const float* ugv, const float* ugw, float* g0u, float* g0v, float* g0w,
                 double* h_grad, sim_stats* stats) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!gu || !gv || !gw || !g0u || !g0v || !g0w || !h_grad) {
    c->err = "NULL pointer";
    return SIM_ERR_INVALID_ARG;
  }
  const bool have_ugen = ugu || ugv || ugw;
  if (have_ugen && !(ugu && ugv && ugw)) {
    c->err = "ugen pointers must be all set or all NULL";
    return SIM_ERR_INVALID_ARG;
  }
  if (!c->recorded || !c->params_set) {
    c->err = "no recorded rollout (call sim_step with record = 1 first)";
    return SIM_ERR_STATE;
  }
  const int T = c->rec_steps;
  const int K = c->desc.checkpoint_every;
  const int64_t F3n = 3 * c->F;
  const bool explicit_d = diffusion_explicit(c);
  const float alpha = diffusion_alpha(c);
  F3 lam = stacked(c, c->lam);
  F3 lam2 = stacked(c, c->lam2);
  sim_stats st{};
  int worst = SIM_OK;
  const bool upwind = c->desc.convection_grad == SIM_CONVGRAD_UPWIND;
  launch_copy_faces(c, cf3(gu, gv, gw), lam);
  HIPCHK(hipMemsetAsync(c->scal + S_DOT1, 0, sizeof(double), c->stream));
  HIPCHK(hipMemsetAsync(c->scal + S_ADV_DT, 0, 4 * sizeof(double), c->stream));
  if (c->xwa) HIPCHK(hipMemsetAsync(c->xwa, 0, sizeof(double) * c->C, c->stream));
  for (int s0 = ((T - 1) / K) * K; T > 0 && s0 >= 0; s0 -= K) {
    const int s1 = std::min(s0 + K, T);
    // recompute the segment
    float* state0 = c->seg;  // slot q: state of step s0+q; slot K+q: viscosity operand
    launch_copy_faces(c, cstacked(c, c->ckpt + (int64_t)(s0 / K) * F3n), stacked(c, state0));
    // the recompute repeats the forward solves from the same starting iterates
    if (c->ckpt_x) {
      launch_x_to_double(c, c->ckpt_x + (int64_t)(s0 / K) * c->C, c->xw);
      launch_x_to_double(c, c->ckpt_x2 + (int64_t)(s0 / K) * c->C, c->xw2);
      launch_x_to_double(c, c->ckpt_x3 + (int64_t)(s0 / K) * c->C, c->xw3);
      c->warm_n = c->ckpt_warm[s0 / K];
    }
    // with the history, the implicit viscosity outputs are the forward's own
    // (copied: no advection, no viscosity solve)
    const bool have_visc = c->vhist && !explicit_d;
    for (int s = s0; s < s1; ++s) {
      const int q = s - s0;
      F3 us = stacked(c, c->seg + (int64_t)q * F3n);
      F3 op = stacked(c, c->seg + (int64_t)(K + q) * F3n);
      const float* vs = have_visc ? c->vhist + (int64_t)s * F3n : nullptr;
      if (!have_visc) advect_force(c, cf3(us.c[0], us.c[1], us.c[2]), stacked(c, c->tmp));
      if (s + 1 < s1) {
        F3 nxt = stacked(c, c->seg + (int64_t)(q + 1) * F3n);
        if (have_visc) {
          launch_copy_faces(c, cstacked(c, vs), nxt);
        } else {
          int rc = diffuse_into(c, nxt, nullptr);
          if (rc) return rc;
        }
        if (explicit_d)
          launch_copy_faces(c, cstacked(c, c->tmp), op);
        else
          launch_copy_faces(c, cf3(nxt.c[0], nxt.c[1], nxt.c[2]), op);
        // the forward's own pressure (stored) or its warm start
        const int rc = c->xhist ? project_inplace(c, nxt, nullptr, c->xhist + (int64_t)s * c->C)
                                : project_warm(c, nxt, nullptr);
        worst = combine(worst, rc);
        if (rc < 0) return rc;
      } else {
        if (explicit_d) {
          launch_copy_faces(c, cstacked(c, c->tmp), op);
        } else if (have_visc) {
          launch_copy_faces(c, cstacked(c, vs), op);
        } else {
          int rc = diffuse_into(c, op, nullptr);
          if (rc) return rc;
        }
      }
    }
    // reverse through the segment
    for (int s = s1 - 1; s >= s0; --s) {
      const int q = s - s0;
      F3 us = stacked(c, c->seg + (int64_t)q * F3n);
      F3 op = stacked(c, c->seg + (int64_t)(K + q) * F3n);
      // the learned preconditioner's adjoint solves start from the previous
      // adjoint pressure rescaled; Jacobi-PCG ran more iterations from it
      int rc = project_inplace(c, lam, &st, c->xwa, c->desc.precond == SIM_PRECOND_LEARNED);
      worst = combine(worst, rc);
      if (rc < 0) return rc;
      if (explicit_d) {
        launch_dot_lap(c, cstacked(c, c->lam), cf3(op.c[0], op.c[1], op.c[2]), S_DOT1,
                       c->params.dt, 1);
        launch_copy_faces(c, cstacked(c, c->lam), stacked(c, c->tmp));
        launch_diffuse_explicit(c, cstacked(c, c->tmp), lam2, alpha);
      } else {
        launch_copy_faces(c, cstacked(c, c->lam), stacked(c, c->tmp));
        rc = diffuse_implicit(c, lam2, &st);
        if (rc) return rc;
        launch_dot_lap(c, cstacked(c, c->lam2), cf3(op.c[0], op.c[1], op.c[2]), S_DOT1,
                       c->params.dt, 1);
      }
      const float dth = (float)(c->params.dt * c->n);
      if (upwind) {
        launch_convection_grad_upwind(c, cf3(us.c[0], us.c[1], us.c[2]), cstacked(c, c->lam2), lam);
        launch_advect_adjoint(c, cf3(us.c[0], us.c[1], us.c[2]), cstacked(c, c->lam2), lam, dth,
                              false, 1);
      } else {
        launch_zero_faces(c, lam);
        launch_advect_adjoint(c, cf3(us.c[0], us.c[1], us.c[2]), cstacked(c, c->lam2), lam, dth,
                              true, 1);
      }
      rc = launch_status(c);
      if (rc) return rc;
    }
  }
  // initial state: u0 = s * mask(ugen)
  launch_mask_scale(c, cstacked(c, c->lam), lam, 1.0f);
  if (have_ugen) {
    launch_dot_faces(c, cstacked(c, c->lam), cf3(ugu, ugv, ugw), S_DOT2, 1);
    launch_mask_scale(c, cstacked(c, c->lam), f3(g0u, g0v, g0w), (float)c->params.s);
  } else {
    HIPCHK(hipMemsetAsync(c->scal + S_DOT2, 0, sizeof(double), c->stream));
    launch_copy_faces(c, cstacked(c, c->lam), f3(g0u, g0v, g0w));
  }
  int rc = launch_status(c);
  if (rc) return rc;
  double host[S_LSUM2 + 1];
  HIPCHK(hipMemcpyAsync(host, c->scal, sizeof host, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const double dt = c->params.dt, dnu = host[S_DOT1];
  h_grad[0] = dnu;
  h_grad[1] = host[S_DOT2];
  h_grad[2] = host[S_ADV_DT] + (c->params.nu / dt) * dnu;
  for (int a = 0; a < 3; ++a) {
    h_grad[2] += c->params.gravity[a] * host[S_LSUM0 + a];
    h_grad[3 + a] = dt * host[S_LSUM0 + a];
  }
  st.status = worst;
  if (stats) *stats = st;
  return worst;
}

int sim_harvest_pairs(sim_ctx* c, const float* u, const float* v, const float* w,
                      const int32_t* iters, int32_t count, int32_t mode, double tol, float* r_out,
                      float* e_out, sim_stats* stats) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!u || !v || !w || !iters || count < 1 || !r_out || !e_out || !(tol > 0.0 && tol < 1.0) ||
      (mode != 0 && mode != 1)) {
    c->err = "invalid harvest arguments";
    return SIM_ERR_INVALID_ARG;
  }
  for (int j = 0; j < count; ++j)
    if (iters[j] < 0 || (mode == 0 && iters[j] % 2) || (j && iters[j] <= iters[j - 1])) {
      c->err = "harvest iterations must be strictly increasing (and even for Jacobi-PCG)";
      return SIM_ERR_INVALID_ARG;
    }
  if (mode == 1 && !net_ready(c)) {
    c->err = "learned preconditioner has no weights";
    return SIM_ERR_STATE;
  }
  // 1. reference solution x* (Jacobi-PCG to tol), kept in FP64 in the
  //    viscosity solver's FP64 buffer (3F >= C doubles, unused here)
  launch_divergence(c, cf3(u, v, w), c->b);
  double* xref = c->fx;
  const double tol_keep = c->desc.tol;
  c->desc.tol = tol;
  float* din = c->dA;
  float* dout = c->dB;
  auto block = [&](int todo) {
    for (int t = 0; t < todo; ++t) {
      launch_pcg_dir_spmv(c, PK_JACOBI, din, dout);
      launch_pcg_update2(c, dout, din, (t & 1) != 0);
      if (t == todo - 1) launch_pcg_check(c, PK_JACOBI, tol);
      std::swap(din, dout);
    }
  };
  launch_pcg_init(c, PK_JACOBI);
  LoopResult lr{};
  const int m = (c->desc.check_every + 1) / 2 * 2;
  const int max_it = (c->desc.max_iter + 1) / 2 * 2;
  int rc = run_blocks(c, m, max_it, block, lr);
  c->desc.tol = tol_keep;
  if (rc) return rc;
  if (lr.status != SIM_OK) {
    c->err = "harvest reference solve did not reach tol within max_iter";
    return lr.status;
  }
  launch_x_to_double(c, c->x, xref);

  // 2. the iterates: r_k = b - A x_k (FP64 check, tolerance 0) and
  //    e_k = x* - x_k formed in FP64
  auto snap = [&](int j) -> int {
    launch_pcg_check(c, mode == 0 ? PK_JACOBI : PK_ZARRAY, 0.0);
    HIPCHK(hipMemcpyAsync(r_out + (int64_t)j * c->C, c->r, sizeof(float) * c->C,
                          hipMemcpyDeviceToDevice, c->stream));
    launch_err_snapshot(c, xref, e_out + (int64_t)j * c->C);
    return SIM_OK;
  };
  din = c->dA;
  dout = c->dB;
  int done_it = 0;
  bool fcg_broke = false;
  if (mode == 0) {
    launch_pcg_init(c, PK_JACOBI);
    for (int j = 0; j < count; ++j) {
      for (int t = 0; done_it < iters[j]; ++t, ++done_it) {
        launch_pcg_dir_spmv(c, PK_JACOBI, din, dout);
        launch_pcg_update2(c, dout, din, (t & 1) != 0);
        std::swap(din, dout);
      }
      if (snap(j)) return SIM_ERR_HIP;
    }
  } else {
    launch_fcg_init(c);
    int j = 0;
    if (iters[0] == 0 && snap(j++)) return SIM_ERR_HIP;
    rc = net_apply(c, c->r, c->z, c->flags);
    if (rc) return rc;
    launch_fcg_beta_first(c, 1);
    while (j < count) {
      launch_fcg_dir_spmv(c, din, dout);
      launch_fcg_update(c, dout);
      ++done_it;
      if (done_it == iters[j] && snap(j++)) return SIM_ERR_HIP;
      rc = net_apply(c, c->r, c->z, c->flags);
      if (rc) return rc;
      launch_fcg_beta(c);
      std::swap(din, dout);
    }
  }
  // did the flexible CG break down (later pairs would not be its iterates)?
  int fl[F_COUNT];
  HIPCHK(hipMemcpyAsync(fl, c->flags, sizeof fl, hipMemcpyDeviceToHost, c->stream));
  rc = launch_status(c);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  fcg_broke = mode == 1 && fl[F_DONE] == 2;
  if (stats) {
    stats->iters = lr.iters + done_it;
    stats->rel_residual = relres_of(lr);
    stats->fallback_used = fcg_broke ? 1 : 0;
    stats->status = SIM_OK;
  }
  return SIM_OK;
}

// ---------------------------------------------------------- single operators

int sim_op_advect(sim_ctx* c, const float* u, const float* v, const float* w, float* au, float* av,
                  float* aw) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!u || !v || !w || !au || !av || !aw || !c->params_set) {
    c->err = "NULL pointer or params not set";
    return SIM_ERR_INVALID_ARG;
  }
  advect_force(c, cf3(u, v, w), f3(au, av, aw));
  return launch_status(c);
}

int sim_op_diffuse(sim_ctx* c, const float* u, const float* v, const float* w, float* ou, float* ov,
                   float* ow, sim_stats* stats) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!u || !v || !w || !ou || !ov || !ow || !c->params_set) {
    c->err = "NULL pointer or params not set";
    return SIM_ERR_INVALID_ARG;
  }
  launch_copy_faces(c, cf3(u, v, w), stacked(c, c->tmp));
  sim_stats st{};
  int rc = diffuse_into(c, f3(ou, ov, ow), &st);
  st.status = rc;
  if (stats) *stats = st;
  return rc;
}

int sim_op_divergence(sim_ctx* c, const float* u, const float* v, const float* w, float* b) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!u || !v || !w || !b) {
    c->err = "NULL pointer";
    return SIM_ERR_INVALID_ARG;
  }
  launch_divergence(c, cf3(u, v, w), b);
  return launch_status(c);
}

int sim_op_poisson_apply(sim_ctx* c, const float* xin, float* y) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!xin || !y) {
    c->err = "NULL pointer";
    return SIM_ERR_INVALID_ARG;
  }
  launch_poisson_apply(c, xin, y);
  return launch_status(c);
}

int sim_op_precond_apply(sim_ctx* c, int32_t precond, const float* r, float* z) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!r || !z) {
    c->err = "NULL pointer";
    return SIM_ERR_INVALID_ARG;
  }
  if (precond == SIM_PRECOND_JACOBI) {
    launch_jacobi_apply(c, r, z);
  } else if (precond == SIM_PRECOND_MIC0) {
    if (!c->precon) {
      c->err = "context was created without the MIC(0) factor";
      return SIM_ERR_INVALID_ARG;
    }
    launch_mic0_apply(c, r, z, nullptr);
  } else if (precond == SIM_PRECOND_LEARNED) {
    if (!net_ready(c)) {
      c->err = "learned preconditioner has no weights";
      return SIM_ERR_STATE;
    }
    return net_apply(c, r, z, nullptr);
  } else {
    c->err = "unknown preconditioner";
    return SIM_ERR_INVALID_ARG;
  }
  return launch_status(c);
}

int sim_op_advect_adjoint(sim_ctx* c, const float* u, const float* v, const float* w,
                          const float* lu, const float* lv, const float* lw, float* g0,
                          float* g1, float* g2) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!u || !v || !w || !lu || !lv || !lw || !g0 || !g1 || !g2 || !c->params_set) {
    c->err = "NULL pointer or params not set";
    return SIM_ERR_INVALID_ARG;
  }
  launch_advect_adjoint(c, cf3(u, v, w), cf3(lu, lv, lw), f3(g0, g1, g2),
                        (float)(c->params.dt * c->n), true, 0);
  return launch_status(c);
}

}  // extern "C"
