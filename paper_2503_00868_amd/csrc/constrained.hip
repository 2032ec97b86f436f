// Constrained divergence projection (Section 3.3, Eq. (divProj)): per
// liquid cell i the constraint C_i = (div v)_i over its active faces; each
// iteration sets lambda_i = -C_i / (sum_k |dC_i/dv_k|^2 + eps) for every
// constraint at once and moves each face by its two cells' multipliers.
// With b = -h (signed outflow) the projection's right-hand side and n_c the
// number of active faces of i (the Poisson diagonal), sum_k |dC_i/dv_k|^2 =
// n_c / h^2 and C_i = -b_i / h^2, so lambda_i = b_i / (n_c + eps h^2), and the
// face update v_f += (lambda_low - lambda_high) / h is the projection's
// pressure update with p = lambda.  One iteration is therefore the
// divergence kernel, the multiplier kernel below and the pressure-update
// kernel of the projection.
#include <cmath>

#include "common.h"
#include "ctx.h"
#include "net.h"

namespace fs {

// lambda (FP64, as the pressure update reads it) = b / (n_c + eps h^2) on
// liquid cells, 0 elsewhere
__global__ void __launch_bounds__(kBlock)
    k_cp_lambda(int64_t C, const float* __restrict__ b, const uint8_t* __restrict__ cdiag,
                double eps_h2, double* __restrict__ lam) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < C; i += (int64_t)gridDim.x * kBlock) {
    const uint8_t d = cdiag[i];
    lam[i] = d ? (double)b[i] / ((double)d + eps_h2) : 0.0;
  }
}


}  // namespace fs

using namespace fs;

extern "C" int sim_constrained_project(sim_ctx* c, float* u, float* v, float* w, int32_t iters,
                                       double eps, double* h_rel_div) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!u || !v || !w || iters < 0 || !(eps >= 0.0) || !std::isfinite(eps)) {
    c->err = "sim_constrained_project: NULL field, iters < 0 or eps not a finite value >= 0";
    return SIM_ERR_INVALID_ARG;
  }
  const F3 U{{u, v, w}};
  const CF3 cu{{u, v, w}};
  // the variables are the active faces: the others hold 0
  launch_mask_scale(c, cu, U, 1.0f);
  auto div_norm2 = [&](double* out) -> int {
    launch_divergence(c, cu, c->b);
    launch_dot_cells_slot(c, c->b, c->b, S_DOT1, nullptr);
    if (hipMemcpyAsync(out, c->scal + S_DOT1, sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return SIM_ERR_HIP;
    return SIM_OK;
  };
  double bb0 = 0.0;
  if (h_rel_div && div_norm2(&bb0)) return SIM_ERR_HIP;
  const double eps_h2 = eps / ((double)c->n * c->n);
  for (int it = 0; it < iters; ++it) {
    launch_divergence(c, cu, c->b);
    hipLaunchKernelGGL(k_cp_lambda, dim3(c->grid_cells), dim3(kBlock), 0, c->stream, c->C, c->b,
                       c->cdiag, eps_h2, c->x);
    launch_pressure_update(c, c->x, U);
  }
  if (h_rel_div) {
    double bb = 0.0;
    if (div_norm2(&bb)) return SIM_ERR_HIP;
    *h_rel_div = bb0 > 0.0 ? std::sqrt(bb / bb0) : 0.0;
  }
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_ERR_HIP;
}
