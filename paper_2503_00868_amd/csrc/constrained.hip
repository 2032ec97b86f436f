// Constrained divergence projection (Section 3.3, Eq. (divProj)): per
// liquid cell i the constraint C_i = (div v)_i over its active faces; each
// iteration sets lambda_i = -C_i / (sum_k |dC_i/dv_k|^2 + eps) for every
// constraint at once and moves each face by its two cells' multipliers.
// With b = -h (signed outflow) the projection's right-hand side and n_c the
// number of active faces of i (the Poisson diagonal), sum_k |dC_i/dv_k|^2 =
// n_c / h^2 and C_i = -b_i / h^2, so lambda_i = b_i / (n_c + eps h^2), and the
// face update v_f += (lambda_low - lambda_high) / h is the projection's
// pressure update with p = lambda.  One iteration is therefore the kernel
// below (the projection's divergence and the multiplier in one pass) and
// the projection's pressure-update kernel.
#include <cmath>

#include "common.h"
#include "ctx.h"
#include "net.h"

namespace fs {

// lambda (FP64, as the pressure update reads it) = b / (n_c + eps h^2) on
// liquid cells, 0 elsewhere, with b = -h (signed outflow) formed as the
// projection's divergence kernel forms it (FP32, same order)
__global__ void __launch_bounds__(kBlock)
    k_cp_lambda(int n, const uint8_t* __restrict__ cdiag, CF3 in, double eps_h2,
                double* __restrict__ lam) {
  const int64_t nn = (int64_t)n * n, C = nn * n;
  const float h = 1.0f / (float)n;
  for (int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x; idx < C;
       idx += (int64_t)gridDim.x * kBlock) {
    const uint8_t d = cdiag[idx];
    double out = 0.0;
    if (d) {
      const int i = (int)(idx % n), j = (int)((idx / n) % n), k = (int)(idx / nn);
      const int64_t iu = i + (int64_t)(n + 1) * (j + (int64_t)n * k);
      const int64_t iv = i + (int64_t)n * (j + (int64_t)(n + 1) * k);
      const float flux = (in.c[0][iu + 1] - in.c[0][iu]) + (in.c[1][iv + n] - in.c[1][iv]) +
                         (in.c[2][idx + nn] - in.c[2][idx]);
      const float b = -h * flux;
      out = (double)b / ((double)d + eps_h2);
    }
    lam[idx] = out;
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
    hipLaunchKernelGGL(k_cp_lambda, dim3(c->grid_cells), dim3(kBlock), 0, c->stream, c->n,
                       c->cdiag, cu, eps_h2, c->x);
    launch_pressure_update(c, c->x, U);
  }
  if (h_rel_div) {
    double bb = 0.0;
    if (div_norm2(&bb)) return SIM_ERR_HIP;
    *h_rel_div = bb0 > 0.0 ? std::sqrt(bb / bb0) : 0.0;
  }
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_ERR_HIP;
}
