// Scaled warm start of a projection solve: the previous solution x is
// replaced by gamma x with gamma = x.b / x.Ax, the multiple of x closest to
// the solution in the A-norm (a one-dimensional Galerkin step; A is the
// pressure Poisson matrix of Section 3.2.2, b the current right-hand side).
#include "common.h"
#include "ctx.h"

namespace fs {

// partials [x.b, x.Ax, 0, 0] over liquid cells; x is zero off the liquid
// cells, as every solve leaves it, so neighbours are summed unmasked as in
// the FP64 residual check
__global__ void __launch_bounds__(kBlock)
    k_guess_dots(int n, const uint8_t* __restrict__ cdiag, const float* __restrict__ b,
                 const double* __restrict__ x, double* partials) {
  const int64_t C = cells(n), sz = (int64_t)n * n;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t idx = (int64_t)lb * kBlock + threadIdx.x; idx < C; idx += (int64_t)gridDim.x * kBlock) {
    const uint8_t dg = cdiag[idx];
    if (!dg) continue;
    const int i = (int)(idx % n), j = (int)((idx / n) % n), k = (int)(idx / sz);
    double s = 0.0;
    if (i > 0) s += x[idx - 1];
    if (i + 1 < n) s += x[idx + 1];
    if (j > 0) s += x[idx - n];
    if (j + 1 < n) s += x[idx + n];
    if (k > 0) s += x[idx - sz];
    if (k + 1 < n) s += x[idx + sz];
    const double xc = x[idx];
    v[0] += xc * (double)b[idx];
    v[1] += xc * ((double)dg * xc - s);
  }
  store_partials<4>(v, partials, lb);
}

__global__ void __launch_bounds__(kBlock)
    k_guess_scale(int64_t C, double* __restrict__ x, const double* __restrict__ scal) {
  const double xax = scal[S_GUESS0 + 1];
  if (!(xax > 0.0)) return;  // x = 0: nothing to scale
  const double gamma = scal[S_GUESS0] / xax;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < C; i += (int64_t)gridDim.x * kBlock)
    x[i] *= gamma;
}

void launch_guess_scale(sim_ctx* c, double* x) {
  hipLaunchKernelGGL(k_guess_dots, dim3(c->grid_cells), dim3(kBlock), 0, c->stream, c->n, c->cdiag,
                     c->b, x, c->partials);
  launch_finalize(c, c->grid_cells, 4, FIN_SLOTS4, 0.0, 0, S_GUESS0, 1.0, 0);
  hipLaunchKernelGGL(k_guess_scale, dim3(1024), dim3(kBlock), 0, c->stream, c->C, x, c->scal);
}

}  // namespace fs
