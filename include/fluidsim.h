/*
 * fluidsim — MI355X (gfx950) library for the differentiable MAC-grid liquid
 * step of arXiv 2503.00868: semi-Lagrangian advection, viscosity and
 * pressure projection by preconditioned conjugate gradients, with the exact
 * discrete adjoint and a learned U-Net preconditioner inside flexible CG.
 *
 * Paper passages the operations follow (section numbers of the paper):
 *   - momentum equation with pressure, viscosity and gravity: Section 3.2.2,
 *     Eq. (v); operator splitting after Chorin: Section 3.2.2;
 *   - semi-Lagrangian back-tracing of the convection term: Section 3.4.1;
 *   - a learned convolutional solver for the pressure Poisson equation,
 *     fitted on pressure pairs taken before and after an implicit solve:
 *     Section 3.4.1 (PeRCNN, Fig. "percnn_str_fit");
 *   - differentiability with respect to the simulation parameters and the
 *     masked L2 velocity loss: Section 3.4.2, Eq. (optLoss); parameter
 *     normalisation by an exponential activation: Section 3.4.2.
 *
 * GRID.  Unit box, n cells per axis, h = 1/n.  All arrays are flat, x fastest:
 *   cell (i,j,k)            -> i + n*(j + n*k)                 n^3 entries
 *   u face (i,j,k), i <= n  -> i + (n+1)*(j + n*k)            (n+1)n^2 entries
 *   v face (i,j,k), j <= n  -> i + n*(j + (n+1)*k)            (n+1)n^2 entries
 *   w face (i,j,k), k <= n  -> i + n*(j + n*k)                (n+1)n^2 entries
 * Cell types (uint8): 0 air, 1 liquid, 2 solid; outside the box is solid.
 * A face is a WALL if a solid cell touches it, ACTIVE if otherwise a liquid
 * cell touches it, INACTIVE otherwise.  Every operation leaves zero on every
 * non-active face.  Velocities are float32 in m/s (box side 1 m).
 *
 * MEMORY.  Pointers named d_* are DEVICE pointers owned by the caller and
 * must stay valid for the duration of the call (and, for the workspace, for
 * the life of the context).  Pointers named h_* are host pointers.  The
 * library allocates no device memory: every buffer it needs lives in the
 * caller's workspace (size from sim_workspace_size).  The sim_ctx object is
 * host memory owned by the library and freed by sim_destroy.
 *
 * STREAMS.  All device work is enqueued on the stream given to sim_create.
 * Calls return after their work is complete on that stream (they read back
 * convergence scalars), except sim_init_state and sim_op_* which only enqueue.
 *
 * ERRORS.  Every entry point returns one of the SIM_* codes below and never
 * throws.  Arguments are validated on the host before any device work, so
 * an invalid call leaves device memory untouched.  sim_last_error returns a
 * message for the last failure on a context.
 */
#ifndef FLUIDSIM_H
#define FLUIDSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sim_ctx sim_ctx; /* opaque, host memory owned by the library */

enum {
    SIM_OK = 0,
    SIM_OK_FALLBACK = 1,           /* converged, but the learned solve fell back to Jacobi-PCG */
    SIM_ERR_INVALID_ARG = -1,
    SIM_ERR_WORKSPACE_TOO_SMALL = -2,
    SIM_ERR_HIP = -3,
    SIM_ERR_NOT_CONVERGED = -4,    /* fields hold the last iterate; stats are filled */
    SIM_ERR_SINGULAR_MASK = -5,    /* a liquid region touches no air: pure-Neumann system */
    SIM_ERR_STATE = -6             /* e.g. backward without a recorded rollout */
};

enum { SIM_PRECOND_JACOBI = 0, SIM_PRECOND_MIC0 = 1, SIM_PRECOND_LEARNED = 2 };
enum { SIM_DIFFUSION_AUTO = 0, SIM_DIFFUSION_EXPLICIT = 1, SIM_DIFFUSION_IMPLICIT = 2 };
/* Transpose of the advection's velocity dependence in sim_backward: the
 * exact discrete one, or the paper's upwind analytic surrogate of the
 * convection gradient (Section 3.4.1; sim_op_convection_grad_upwind). */
enum { SIM_CONVGRAD_EXACT = 0, SIM_CONVGRAD_UPWIND = 1 };

/* Static configuration, fixed for the life of a context. */
typedef struct {
    int32_t n;                 /* cells per axis, 4 <= n <= 1024; n % 4 == 0 for LEARNED */
    int32_t precond;           /* SIM_PRECOND_* for the pressure solve */
    int32_t diffusion;         /* SIM_DIFFUSION_*; AUTO = explicit iff nu*dt*n^2 <= 1/12 */
    int32_t max_iter;          /* per solve, >= 1 (Jacobi and learned: rounded up to a
                                  multiple of 4) */
    int32_t check_every;       /* FP64 true-residual check period m, 1..1024 (Jacobi and
                                  learned: rounded up to a multiple of 4; they update the FP64
                                  iterate every 4 iterations) */
    int32_t checkpoint_every;  /* K: rollout checkpoint spacing for sim_backward, >= 1 */
    int32_t max_steps;         /* longest recordable rollout (0 = no recording) */
    int32_t learned_max_iter;  /* flexible-CG iterations before the Jacobi-PCG restart (it also
                                  restarts on breakdown, or when the residual falls by less
                                  than a factor 0.9 per iteration between two checks) */
    double tol;                /* relative L2 true residual of the pressure solve, (0, 1) */
    double diff_tol;           /* same for the implicit viscosity solve, (0, 1) */
    int32_t warm_start;        /* 1: each pressure solve of a rollout starts from the quadratic
                                  extrapolation 3 p[s-1] - 3 p[s-2] + p[s-3] of the previous
                                  steps' pressures (the linear 2 p[s-1] - p[s-2] at the third
                                  step, p[s-1] at the second, 0 at the first), each adjoint
                                  solve of sim_backward from the previous
                                  adjoint solve's (with SIM_PRECOND_LEARNED scaled by
                                  x.b / x.Ax, its multiple closest to the new solution
                                  in the A-norm); the
                                  stopping test, relative to the
                                  right-hand side, is unchanged; 0: every solve starts at 0 */
    int32_t store_pressures;   /* 1 (needs max_steps > 0): a recorded rollout also keeps each
                                  step's FP64 pressure (max_steps x n^3 doubles of workspace)
                                  and, unless diffusion is EXPLICIT, its implicit viscosity
                                  output (max_steps x 3 x (n+1) n^2 floats).  sim_backward's
                                  recompute then starts every projection from the stored
                                  pressure (the solve stops at its first check with no
                                  iteration) and takes the viscosity output as stored */
    int32_t convection_grad;   /* SIM_CONVGRAD_*: what sim_backward takes for the transpose of
                                  the advection's dependence on the velocity (the derivatives
                                  in dt and gravity are the exact ones in both modes) */
} sim_desc;

/* Dynamic parameters (sim_set_params).  Density is 1: the solver works with
 * the scaled pressure p*dt/rho, which does not depend on rho. */
typedef struct {
    double nu;                 /* kinematic viscosity, > 0 */
    double s;                  /* initial-velocity scale used by sim_init_state, > 0 */
    double dt;                 /* time step, > 0 */
    double gravity[3];         /* body acceleration, m/s^2, e.g. {0, -9.8, 0} */
} sim_params;

/* Per-solve statistics (host struct filled by the library). */
typedef struct {
    int32_t status;            /* SIM_* code of this step or solve */
    int32_t iters;             /* pressure (F)CG iterations, including any fallback */
    int32_t diff_iters;        /* implicit viscosity CG iterations (0 if explicit) */
    int32_t fallback_used;     /* 1 if the learned solve restarted with Jacobi-PCG */
    double rel_residual;       /* final FP64 true relative residual of the pressure */
    double diff_rel_residual;  /* same for the viscosity solve */
} sim_stats;

/* Bytes of device workspace a context with this description needs.
 * Host only.  Returns SIM_ERR_INVALID_ARG on a bad description. */
int sim_workspace_size(const sim_desc* desc, size_t* bytes);

/* Validate desc and the cell types (host copy h_cell_type, n^3 bytes, values
 * 0/1/2; every connected liquid region must share a face with an air cell,
 * else SIM_ERR_SINGULAR_MASK), carve the workspace (d_workspace, >= the
 * size above, 256-byte aligned), upload the mask and build the per-mask
 * tables (face codes, Poisson diagonal, MIC(0) factor).  hip_stream is a
 * hipStream_t (NULL = default stream). */
int sim_create(const sim_desc* desc, const uint8_t* h_cell_type, void* d_workspace,
               size_t workspace_bytes, void* hip_stream, sim_ctx** out);

/* Set nu, s, dt and gravity; host only, checks ranges.  Required before
 * sim_step / sim_init_state / sim_backward.  Forgets any recorded rollout
 * (it ran with the previous parameters): sim_backward then returns
 * SIM_ERR_STATE until sim_step records again. */
int sim_set_params(sim_ctx* ctx, const sim_params* params);

/* u0 = s * ugen on active faces, 0 elsewhere (the fitted initial velocity
 * scale of the rollout).  Enqueue only. */
int sim_init_state(sim_ctx* ctx, const float* d_ugen_u, const float* d_ugen_v,
                   const float* d_ugen_w, float* d_u, float* d_v, float* d_w);

/* Advance (d_u, d_v, d_w) in place by nsteps steps, each: advection (+ gravity),
 * viscosity (explicit or implicit), pressure projection.  With record != 0
 * the entry state is recorded as the start of a rollout (checkpoints every
 * checkpoint_every steps) so sim_backward can differentiate it; nsteps must
 * then be <= max_steps.  h_stats (nullable) receives nsteps entries. */
int sim_step(sim_ctx* ctx, float* d_u, float* d_v, float* d_w, int32_t nsteps, int32_t record,
             sim_stats* h_stats);

/* Pressure projection alone, in place.  d_p_out (nullable) receives the
 * scaled pressure p*dt/rho per cell as float64 (zero off liquid). */
int sim_project(sim_ctx* ctx, float* d_u, float* d_v, float* d_w, double* d_p_out,
                sim_stats* h_stats);

/* Reverse-mode gradient of the last recorded rollout (Section 3.4.2: the
 * gradients of the loss with respect to the simulation parameters).  In:
 * dJ/du_T (d_gu, d_gv, d_gw).  Out: (d_gu0, d_gv0, d_gw0) = dJ/du0 on active
 * faces, or dJ/dugen = s * dJ/du0 when d_ugen_* are given (the same ugen that
 * sim_init_state used).  h_grad (host, 6 doubles): [0] dJ/dnu, [1] dJ/ds (0
 * when ugen is NULL), [2] dJ/ddt (the back-trace distance, the body-force
 * increment dt*g and the viscous factor nu*dt; the scaled pressure does not
 * depend on dt), [3..5] dJ/dgravity.  The transpose of the advection is the
 * one desc.convection_grad selects.  h_stats (nullable) receives one entry
 * with the summed iterations.  SIM_ERR_STATE without a recorded rollout (or
 * after sim_set_params). */
int sim_backward(sim_ctx* ctx, const float* d_gu, const float* d_gv, const float* d_gw,
                 const float* d_ugen_u, const float* d_ugen_v, const float* d_ugen_w,
                 float* d_gu0, float* d_gv0, float* d_gw0, double* h_grad, sim_stats* h_stats);

/* MSE over active faces between (u,v,w) and a target (the L2 term of
 * Eq. (optLoss)): h_loss receives J; (d_gu, d_gv, d_gw) (nullable) receive
 * dJ/du. */
int sim_loss_mse(sim_ctx* ctx, const float* d_u, const float* d_v, const float* d_w,
                 const float* d_tu, const float* d_tv, const float* d_tw, double* h_loss,
                 float* d_gu, float* d_gv, float* d_gw);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * loss and gradient as sim_loss_mse without a context or workspace.  The
 * active faces come from the cell types d_cell (n^3 bytes, as sim_create's,
 * on the device); J goes to the device double *d_loss (nothing is copied to
 * the host, nothing synchronises); (d_gu, d_gv, d_gw) (all or none) receive
 * dJ/du.  The block partial sums live in one fixed array of 49,408 bytes per
 * device inside the library (looked up on the first call on each device and
 * kept until the process ends); the call allocates nothing.  Calls that
 * overlap on one device race on that array.  Enqueued on hip_stream (NULL =
 * default stream).  SIM_ERR_INVALID_ARG, before any device work, for n
 * outside [4, 1024] (the largest grid the library takes), a NULL input, a
 * partial gradient set or a gradient output aliasing another argument;
 * SIM_ERR_HIP if the array's address cannot be found or a launch fails. */
int sim_loss_mse_noalloc(int32_t n, const uint8_t* d_cell, const float* d_u, const float* d_v,
                         const float* d_w, const float* d_tu, const float* d_tv,
                         const float* d_tw, double* d_loss, float* d_gu, float* d_gv,
                         float* d_gw, void* hip_stream);

/* The paper's masked cosine + L2 velocity loss (Section 3.4.2,
 * Eq. (optLoss)) between the simulated field (d_u, d_v, d_w) and a reference
 * (d_tu, d_tv, d_tw), both MAC face arrays of the context's grid.  Per cell,
 * with a and b the two velocities at the cell centre (component c the mean
 * of the cell's two c-faces):
 *   l = alpha (1 - a.b / sqrt((|a|^2 + eps^2)(|b|^2 + eps^2))) + beta |a - b|^2
 * weighted by the cell's class from the context's cell types:
 * h_weights[0] for air (empty) cells, h_weights[1] for liquid cells with no
 * air neighbour among the six (occupied), h_weights[2] for liquid cells with
 * one (surface); solid cells and the outside of the box weigh 0.
 * h_loss receives J = sum w l / sum w (0 when sum w = 0).  (d_gu, d_gv, d_gw)
 * (all or none) receive dJ/d(d_u, d_v, d_w) on every face: half of dJ/da of
 * each cell the face separates.  Uses the context's partial-sum buffers and
 * three of its solver buffers (free outside a solve); synchronises the
 * stream.  SIM_ERR_INVALID_ARG for NULL inputs, a partial gradient set, a
 * gradient output aliasing an input, non-finite alpha or beta, eps < 0 or
 * not finite, or a negative / non-finite weight. */
int sim_loss_cos_l2(sim_ctx* ctx, const float* d_u, const float* d_v, const float* d_w,
                    const float* d_tu, const float* d_tv, const float* d_tw, double alpha,
                    double beta, double eps, const double* h_weights, double* h_loss,
                    float* d_gu, float* d_gv, float* d_gw);

/* ---- learned preconditioner (Section 3.4.1 analogue) ---------------------
 * A 3-level 3-D U-Net (16/32/64 channels, 3x3x3 bias-free convolutions,
 * ReLU, 2x average pooling, nearest upsampling with skip concatenation, one
 * 16->1 output convolution) maps (r / rms(r), liquid mask) to a correction;
 * z = mask * rms(r) * out.  Weights are one float32 blob in the order and
 * shapes sim_net_param_count documents; the library keeps bf16 copies. */
int sim_net_param_count(int64_t* count);
int sim_net_set_weights(sim_ctx* ctx, const float* d_weights, int64_t count);
int sim_net_forward(sim_ctx* ctx, const float* d_r, float* d_z);

/* Tile skipping of the network's inference pass (default on).  The network
 * is bias-free and its input vanishes off liquid, so each activation is zero
 * beyond a fixed distance of the liquid; and z is masked to liquid, so the
 * late decoder layers matter only near it (c10's output within 1 cell, c9's
 * within 2, and so on; the counts are in the implementation).  At creation
 * the library marks, per layer, the 16 x 16 tiles of each plane that come
 * within the smaller of the two distances; with skipping on, the inference
 * kernels neither compute nor store the other tiles.  z is bitwise that of
 * the dense pass (on = 0); the switch exists to check exactly that.  d_r
 * passed to sim_net_forward (or met in the solver) is read on liquid cells
 * only.  Returns SIM_ERR_STATE for a context without the learned
 * preconditioner. */
int sim_net_set_tile_skip(sim_ctx* ctx, int32_t on);

/* Loss and weight gradient of the U-Net with its current weights on a batch
 * of (r, e) pairs, e = A^-1 r (cell arrays, batch-major, zero off liquid):
 * loss = mean over the batch of 1 - (r.z)^2 / ((r.e)(z.Az)), the squared sine
 * of the A-norm angle between z = net(r) and the true error e.  d_grad
 * receives dloss/dweights (float32 blob, sim_net_param_count entries) with
 * the bf16 rounding of weights and activations treated as the identity. */
int sim_net_grad(sim_ctx* ctx, const float* d_r, const float* d_e, int32_t batch, float* d_grad,
                 double* h_loss);

/* Training pairs for the network, taken from the projection the way the
 * paper fits its learned solver on pressure before and after an implicit
 * solve (Section 3.4.1).  For the projection of (u, v, w) (not modified),
 * iterate A x = b and at each requested iteration k (strictly increasing,
 * h_iters[count]; even for mode 0) record the true residual
 * r_k = b - A x_k and the error e_k = x* - x_k into d_r_out[j], d_e_out[j]
 * (count x n^3 float32 each).  x* comes first, from a Jacobi-PCG solve to
 * tol kept in FP64, and e_k is formed in FP64 before rounding (late
 * iterates differ from x* by less than FP32 resolves in x).
 * mode 0: the iterates of Jacobi-PCG itself; mode 1: the iterates of the
 * flexible CG with the current network (its own residuals, for on-policy
 * training; needs weights).  h_stats->fallback_used = 1 reports that the
 * flexible CG broke down, so pairs from later iterations are not its iterates. */
int sim_harvest_pairs(sim_ctx* ctx, const float* d_u, const float* d_v, const float* d_w,
                      const int32_t* h_iters, int32_t count, int32_t mode, double tol,
                      float* d_r_out, float* d_e_out, sim_stats* h_stats);

/* One Adam step (beta 0.9/0.999, eps 1e-8) of the U-Net on a batch of pairs
 * (as sim_net_grad).  d_master: float32 weights (updated in place, then used
 * by the preconditioner), d_adam: 2*count float32 moments (zero before the
 * first step), step: 1-based Adam step.  h_loss receives the batch loss
 * before the update. */
int sim_net_train_step(sim_ctx* ctx, const float* d_r, const float* d_e, int32_t batch,
                       float* d_master, float* d_adam, int32_t step, float lr, double* h_loss);

/* ---- single operators, for parity tests and custom drivers (enqueue only) --
 * Each acts on the context's mask; outputs get zero on non-active faces /
 * non-liquid cells.  b is the Poisson right-hand side -h * (net outflow). */
int sim_op_advect(sim_ctx* ctx, const float* d_u, const float* d_v, const float* d_w,
                  float* d_au, float* d_av, float* d_aw);
int sim_op_diffuse(sim_ctx* ctx, const float* d_u, const float* d_v, const float* d_w,
                   float* d_ou, float* d_ov, float* d_ow, sim_stats* h_stats);
int sim_op_divergence(sim_ctx* ctx, const float* d_u, const float* d_v, const float* d_w,
                      float* d_b);
int sim_op_poisson_apply(sim_ctx* ctx, const float* d_x, float* d_y);
int sim_op_precond_apply(sim_ctx* ctx, int32_t precond, const float* d_r, float* d_z);
int sim_op_advect_adjoint(sim_ctx* ctx, const float* d_u, const float* d_v, const float* d_w,
                          const float* d_lu, const float* d_lv, const float* d_lw, float* d_gu,
                          float* d_gv, float* d_gw);
/* The paper's upwind analytic convection gradient (Section 3.4.1), a
 * surrogate for the advection adjoint above: for the convected field
 * (d_u, d_v, d_w) and lam = dJ/d(convected field) (d_lu, d_lv, d_lw),
 * d_g_i = lam_i - dt sum_c Lam_c D_i V_c on active faces (0 elsewhere), with
 * V_c, Lam_c the components at the face's position (four-face means across
 * components) and D_i the first-order upwind difference along the face's
 * axis against the sign of v_i.  dt from sim_set_params.  Outputs must not
 * alias inputs. */
int sim_op_convection_grad_upwind(sim_ctx* ctx, const float* d_u, const float* d_v,
                                  const float* d_w, const float* d_lu, const float* d_lv,
                                  const float* d_lw, float* d_gu, float* d_gv, float* d_gw);

/* ---- recurrent convolutional pressure solver (Section 3.4.1) -----------
 * The paper solves the pressure Poisson equation inside its optimisation
 * with a PeRCNN-style recurrent convolution whose kernel is fitted on
 * pressure pairs from an implicit solve.  One layer here is
 *   p_{k+1}(c) = L(c) s(c) ( sum_t W_t p_k(c + t) + w_b b(c) ),
 * t over the 27 offsets of a 3x3x3 stencil (tap (dx+1) + 3 (dy+1) + 9 (dz+1)),
 * p_k = 0 outside the box, L the liquid mask of the context and s = 6 / n_c
 * (n_c the Poisson diagonal of c, the number of its non-solid faces); b is a
 * right-hand side as the projection forms it.  W = 1/6 on the six face taps
 * with w_b = 1/6 is one Jacobi sweep of the projection's Poisson system.
 * h_w: host array of 28 floats, W_0 .. W_26 then w_b.  Cell arrays are n^3
 * float32 on the device, [z][y][x].  Work is enqueued on the context's
 * stream and uses two of its cell buffers, so it must not overlap another
 * call on the same context.  Outputs must not alias inputs. */

/* K >= 0 layers from d_p0.  d_out (nullable) receives p_K; d_hist (nullable,
 * (K+1) n^3 floats) receives p_0 .. p_K for sim_percnn_backward.  At least
 * one of the two must be given.  Returns SIM_ERR_INVALID_ARG for NULL inputs,
 * K < 0 or aliasing outputs. */
int sim_percnn_forward(sim_ctx* ctx, const float* h_w, int32_t K, const float* d_p0,
                       const float* d_b, float* d_out, float* d_hist);

/* Reverse pass of sim_percnn_forward for a loss L with dL/dp_K = d_g, given
 * the states d_hist it recorded (same h_w, K, d_b).  d_gp0 (nullable)
 * receives dL/dp_0, d_gb (nullable) dL/db; h_grad_w (host, 28 doubles)
 * receives dL/dW_0 .. dL/dW_26 and dL/dw_b.  Synchronises the stream. */
int sim_percnn_backward(sim_ctx* ctx, const float* h_w, int32_t K, const float* d_b,
                        const float* d_hist, const float* d_g, float* d_gp0, float* d_gb,
                        double* h_grad_w);

/* One Adam step (beta 0.9 / 0.999, eps 1e-12) of the kernel fit of the
 * recurrent solver: the paper fits the solver's convolution on pressure
 * fields taken before and after an implicit solve (Section 3.4.1).  For each
 * of npairs pairs (stacked npairs x n^3 float32 device arrays: starting
 * pressure d_p0, the solve's pressure d_target, right-hand side d_b), K >= 1
 * layers run from p0 with their states kept in d_hist ((K+1) n^3 floats,
 * overwritten), the loss sum over liquid cells of (p_K - target)^2 and its
 * seed gradient 2 (p_K - target) are formed on the device, and the reverse
 * pass gives dL/dW.  Then the 28 weights h_w (host doubles, W_0 .. W_26,
 * w_b; in/out) take one Adam step of size lr on the mean gradient over the
 * pairs, with the moments h_adam (host, 56 doubles: m then v; zero before
 * step 1; in/out) and the 1-based step.  h_loss (nullable) receives the mean
 * loss over the pairs before the update.  Uses the context's solver buffers
 * (q, two direction buffers) and partial sums; synchronises the stream.
 * SIM_ERR_INVALID_ARG for a NULL pointer, step < 1, K < 1, npairs < 1,
 * lr not > 0, a non-finite weight, or d_hist overlapping a pair array. */
int sim_percnn_fit_step(sim_ctx* ctx, double* h_w, double* h_adam, int32_t step, double lr,
                        int32_t K, int32_t npairs, const float* d_p0, const float* d_target,
                        const float* d_b, float* d_hist, double* h_loss);

/* ---- constrained divergence projection (Section 3.3, Eq. (divProj)) ----
 * In place on (d_u, d_v, d_w) (face arrays as sim_step's): the fields are
 * first masked to the active faces (the variables), then `iters` iterations
 * of the constraint projection run over the liquid cells' constraints
 * C_i = (div v)_i: lambda_i = -C_i / (sum_k |dC_i/dv_k|^2 + eps), every face
 * moved by the multipliers of its two cells at once.  With eps = 0 one
 * iteration is one Jacobi sweep of the projection's pressure system applied
 * as a pressure update; the iterations converge to sim_project's field.
 * h_rel_div (nullable) receives |b(v_K)| / |b(v_0)| (L2 of the projection's
 * right-hand side after and before; synchronises the stream).  Uses the
 * context's pressure and right-hand-side buffers.  SIM_ERR_INVALID_ARG for
 * NULL fields, iters < 0 or eps < 0 / not finite. */
int sim_constrained_project(sim_ctx* ctx, float* d_u, float* d_v, float* d_w, int32_t iters,
                            double eps, double* h_rel_div);

/* ---- screen-space constrained projection (Section 3.3, Eq. (div2DV)) ----
 * The 2-D screen velocity of the reconstructed surface must have the
 * divergence the divergence-free 3-D motion implies:
 *   div v = s,  s = -(u dvz/du + v dvz/dv + 2 vz) / z,
 * with (u, v) screen coordinates normalised to [-1, 1] at pixel centres
 * (spacings du = 2/W, dv = 2/H), vz the out-of-plane velocity and z the depth
 * per pixel (the derivatives second-order central, one-sided at the border).
 * The velocity is staggered on pixel edges: d_a (the u component) on the
 * H x (W+1) vertical edges, a[j*(W+1) + i] the edge left of pixel (j, i);
 * d_b on the (H+1) x W horizontal edges, b[j*W + i] the edge below pixel
 * (j, i).  d_mask (H x W bytes, nonzero = the region where detection failed
 * and the velocity was interpolated): an edge is free when one of its two
 * pixels is in the region and both lie in the image; every other edge keeps
 * its value.  The free edges of (d_a, d_b) lose, in place, the gradient of the
 * potential p that is 0 off the region and solves A p = s - div v on it (A
 * the masked 5-point Laplacian over the free edges): the least change that
 * meets the constraint on the region.  Every connected part of the region
 * must border a pixel outside it, or the system is singular.
 * The solve runs Jacobi-PCG in FP64 to the relative residual tol (0 < tol < 1),
 * at most max_iter iterations, in the caller's workspace (256-byte aligned,
 * sim_screen_workspace_size bytes: seven FP64 pixel vectors and 33 KB).  All
 * pointers are device pointers except h_*; work is enqueued on hip_stream and
 * the call returns when it is done.  h_iters and h_rel_residual (nullable)
 * receive the iterations and the true relative residual |A p - rhs| / |rhs|.
 * SIM_ERR_INVALID_ARG (before any device work) for H or W outside [3, 16384],
 * a NULL pointer, tol outside (0, 1), max_iter < 1 or a misaligned workspace;
 * SIM_ERR_WORKSPACE_TOO_SMALL; SIM_ERR_NOT_CONVERGED (the update of the last
 * iterate is still applied) when tol was not reached or the solve broke down. */
int sim_screen_workspace_size(int32_t H, int32_t W, size_t* bytes);
int sim_screen_project(int32_t H, int32_t W, float* d_a, float* d_b, const float* d_vz,
                       const float* d_z, const uint8_t* d_mask, double tol, int32_t max_iter,
                       void* d_workspace, size_t workspace_bytes, void* hip_stream,
                       int32_t* h_iters, double* h_rel_residual);

/* ---- the paper's APIC transfers (Section 3.2.2, Eq. (particle_map)) -----
 * On the MAC grid each velocity component lives on its own lattice, the
 * centres of its faces (component 0's node (i, j, k) at h (i, j + 1/2,
 * k + 1/2), and likewise), with quadratic B-spline weights (a product over
 * the three axes); nodes outside a lattice are skipped (weight 0 for
 * particles at least one cell inside the box).  Particles are device arrays
 * of structures in the unit box: positions d_x (P x 3: x y z), velocities
 * d_vp (P x 3), affine matrices d_C (P x 9, row a the affine part of
 * component a), masses d_m (P).  P in [0, 2^31).  Both calls are
 * asynchronous on the context's stream. */

/* Particles to grid: (d_u, d_v, d_w) receive, per face node,
 * sum_p w m_p (v_pa + C_p[a] . (x_i - x_p)) / sum_p w m_p (0 where no mass
 * arrived) and (d_mu, d_mv, d_mw) the weighted masses sum_p w m_p.  The six
 * grid outputs are overwritten and must be distinct.  The summation order of
 * the FP32 atomic scatter is not fixed.  SIM_ERR_INVALID_ARG for P out of
 * range or a NULL pointer (the particle pointers may be NULL when P = 0). */
int sim_apic_p2g(sim_ctx* ctx, int64_t P, const float* d_x, const float* d_vp, const float* d_C,
                 const float* d_m, float* d_u, float* d_v, float* d_w, float* d_mu, float* d_mv,
                 float* d_mw);

/* Grid to particles and the particle move: for the grid field (d_u, d_v,
 * d_w) (the field after the grid step), d_vp receives v_pa = sum_i w v_ai,
 * d_C row a receives 4/h^2 sum_i w v_ai (x_i - x_p), and d_x is moved by
 * dt times the new velocity (in place).  SIM_ERR_INVALID_ARG for P out of
 * range, a NULL pointer or a non-finite dt. */
int sim_apic_g2p(sim_ctx* ctx, int64_t P, const float* d_u, const float* d_v, const float* d_w,
                 double dt, float* d_x, float* d_vp, float* d_C);

/* ---- kernel timing for benchmarks -------------------------------------
 * When enabled, HIP events on the context's stream bracket every launch of
 * the kernels below (the finalize reductions are not included); durations
 * accumulate per kind until read.  sim_profile_read synchronises the
 * stream, writes SIM_KERN_COUNT totals in milliseconds and launch counts,
 * and resets them.  For the CG kinds and the network, whose kernels return
 * at once when the solve has already converged (the library enqueues a
 * block of iterations ahead of its convergence test), the count is of the
 * launches that did work; the time includes the others.  Every 1<<15 timed launches the library waits for the
 * stream once to fold the recorded events into the totals. */
enum {
    SIM_KERN_PCG_DIR_SPMV = 0,  /* d = M^-1 r + beta d ; q = A d ; d.q            */
    SIM_KERN_PCG_UPDATE,        /* x += alpha d ; r -= alpha q ; r.M^-1 r          */
    SIM_KERN_PCG_CHECK,         /* FP64 true residual and residual replacement     */
    SIM_KERN_ADVECT,            /* semi-Lagrangian advection + body force          */
    SIM_KERN_DIFFUSE_EXPLICIT,  /* explicit viscosity step                          */
    SIM_KERN_DCG_DIR_SPMV,      /* implicit viscosity CG: direction + SpMV          */
    SIM_KERN_DCG_UPDATE,        /* implicit viscosity CG: update                    */
    SIM_KERN_MIC0,              /* one MIC(0) apply (all hyperplane launches)        */
    SIM_KERN_NET,               /* one U-Net preconditioner apply                   */
    SIM_KERN_ADVECT_ADJOINT,    /* advection adjoint scatter                        */
    SIM_KERN_PERCNN,            /* one recurrent conv solver layer                  */
    SIM_KERN_PERCNN_ADJ,        /* one reverse layer of the recurrent conv solver   */
    SIM_KERN_COUNT
};
int sim_profile_enable(sim_ctx* ctx, int32_t on);
int sim_profile_read(sim_ctx* ctx, double* h_ms, int64_t* h_launches);

int sim_destroy(sim_ctx* ctx);
const char* sim_last_error(const sim_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
