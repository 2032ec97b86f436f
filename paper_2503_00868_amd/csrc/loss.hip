// The paper's masked cosine + L2 velocity loss (Section 3.4.2, Eq. (optLoss))
// on the MAC grid: per cell, with a and b the simulated and reference
// velocities at the cell centre (each component the mean of its two faces),
//
//   l = alpha (1 - a.b / sqrt((|a|^2 + eps^2)(|b|^2 + eps^2))) + beta |a - b|^2,
//
// weighted by the cell's class (empty: air; surface: liquid with an air
// neighbour; occupied: other liquid; solid cells weigh 0), and
// J = sum w l / sum w.  Three launches: per cell the weighted term, the
// weight and the weighted dJ/da (before the 1/sum w), with block partial
// sums; one block folds the partials; per face half the gradients of the
// two cells it separates, times 1/sum w read on the device.
#include <cmath>

#include "common.h"
#include "ctx.h"

namespace fs {

struct LossCoef {
  float alpha, beta, eps2;
  float w[3];  // empty, occupied, surface
};

// cells: fewer than 2^31 for n <= 1024, so 32-bit indexes suffice
__global__ void __launch_bounds__(kBlock)
    k_loss_cells(int n, const uint8_t* __restrict__ cell, CF3 s, CF3 r, LossCoef cf, float* __restrict__ ga0,
                 float* __restrict__ ga1, float* __restrict__ ga2, double* __restrict__ partials) {
  const unsigned un = n, nn = un * un, C = nn * un;
  double acc[2] = {0.0, 0.0};
  for (unsigned idx = blockIdx.x * kBlock + threadIdx.x; idx < C; idx += gridDim.x * kBlock) {
    const unsigned row = idx / un, k = row / un;
    const unsigned i = idx - row * un, j = row - k * un;
    const uint8_t t = cell[idx];
    float wgt = 0.f;
    if (t == AIR) {
      wgt = cf.w[0];
    } else if (t == LIQUID) {
      const bool air = (i > 0 && cell[idx - 1] == AIR) || (i + 1 < un && cell[idx + 1] == AIR) ||
                       (j > 0 && cell[idx - un] == AIR) || (j + 1 < un && cell[idx + un] == AIR) ||
                       (k > 0 && cell[idx - nn] == AIR) || (k + 1 < un && cell[idx + nn] == AIR);
      wgt = air ? cf.w[2] : cf.w[1];
    }
    float g[3] = {0.f, 0.f, 0.f};
    if (wgt != 0.f) {
      // faces of cell (i, j, k): x-faces i, i+1 of row (j, k) with n+1 per row;
      // y-faces j, j+1 of plane k with n+1 rows; z-faces k, k+1
      const unsigned iu = i + (un + 1) * row;
      const unsigned iv = i + un * (j + (un + 1) * k);
      const float a[3] = {0.5f * (s.c[0][iu] + s.c[0][iu + 1]), 0.5f * (s.c[1][iv] + s.c[1][iv + un]),
                          0.5f * (s.c[2][idx] + s.c[2][idx + nn])};
      const float b[3] = {0.5f * (r.c[0][iu] + r.c[0][iu + 1]), 0.5f * (r.c[1][iv] + r.c[1][iv + un]),
                          0.5f * (r.c[2][idx] + r.c[2][idx + nn])};
      const float aa = a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + cf.eps2;
      const float bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2] + cf.eps2;
      const float ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
      const float AB = sqrtf(aa * bb);
      const float cosv = AB > 0.f ? ab / AB : 0.f;
      const float d[3] = {a[0] - b[0], a[1] - b[1], a[2] - b[2]};
      const float l = cf.alpha * (1.f - cosv) + cf.beta * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      acc[0] += (double)wgt * (double)l;
      acc[1] += (double)wgt;
      // d cos / da = b / AB - (a.b / (|a|^2 + eps^2)) a / AB
      const float inv = AB > 0.f ? 1.f / AB : 0.f;
      const float ca = AB > 0.f ? ab / aa : 0.f;
#pragma unroll
      for (int q = 0; q < 3; ++q)
        g[q] = wgt * (-cf.alpha * (b[q] - ca * a[q]) * inv + 2.f * cf.beta * d[q]);
    }
    if (ga0) {
      ga0[idx] = g[0];
      ga1[idx] = g[1];
      ga2[idx] = g[2];
    }
  }
  store_partials<2>(acc, partials, blockIdx.x);
}

// one block: the two sums over the per-block partials -> scal[S_DOT0], scal[S_DOT1]
__global__ void __launch_bounds__(kBlock)
    k_loss_fold(const double* __restrict__ partials, int nblocks, double* __restrict__ scal) {
  double v[2] = {0.0, 0.0};
  for (int blk = threadIdx.x; blk < nblocks; blk += kBlock) {
    v[0] += partials[2 * blk];
    v[1] += partials[2 * blk + 1];
  }
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    scal[S_DOT0] = v[0];
    scal[S_DOT1] = v[1];
  }
}

// the I-faces: half of each adjacent cell's dJ/da_I, times 1 / sum w
template <int I>
__device__ inline void loss_faces(int n, const float* __restrict__ ga, float invw, float* __restrict__ g) {
  const unsigned un = n, nx = un + (I == 0), ny = un + (I == 1);
  const unsigned count = nx * ny * (un + (I == 2));
  for (unsigned idx = blockIdx.x * kBlock + threadIdx.x; idx < count; idx += gridDim.x * kBlock) {
    const unsigned row = idx / nx, z = row / ny;
    const unsigned x = idx - row * nx, y = row - z * ny;
    const unsigned q = I == 0 ? x : (I == 1 ? y : z);  // the face's index along its axis
    const unsigned stride = I == 0 ? 1u : (I == 1 ? un : un * un);
    const unsigned cidx = x + un * (y + un * z);  // the cell after the face (when q < n)
    float s = 0.f;
    if (q > 0) s += ga[cidx - stride];
    if (q < un) s += ga[cidx];
    g[idx] = 0.5f * invw * s;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_loss_face_grad(int n, const float* __restrict__ ga0, const float* __restrict__ ga1,
                     const float* __restrict__ ga2, const double* __restrict__ scal, float* __restrict__ g0,
                     float* __restrict__ g1, float* __restrict__ g2) {
  const double W = scal[S_DOT1];
  const float invw = W > 0.0 ? (float)(1.0 / W) : 0.f;
  if (blockIdx.y == 0)
    loss_faces<0>(n, ga0, invw, g0);
  else if (blockIdx.y == 1)
    loss_faces<1>(n, ga1, invw, g1);
  else
    loss_faces<2>(n, ga2, invw, g2);
}

}  // namespace fs

using namespace fs;

extern "C" int sim_loss_cos_l2(sim_ctx* c, const float* u, const float* v, const float* w, const float* tu,
                               const float* tv, const float* tw, double alpha, double beta, double eps,
                               const double* h_weights, double* h_loss, float* gu, float* gv, float* gw) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!u || !v || !w || !tu || !tv || !tw || !h_weights || !h_loss) {
    c->err = "sim_loss_cos_l2: NULL pointer";
    return SIM_ERR_INVALID_ARG;
  }
  if ((gu || gv || gw) && !(gu && gv && gw)) {
    c->err = "sim_loss_cos_l2: gradient pointers must be all set or all NULL";
    return SIM_ERR_INVALID_ARG;
  }
  if (!std::isfinite(alpha) || !std::isfinite(beta) || !(eps >= 0.0) || !std::isfinite(eps)) {
    c->err = "sim_loss_cos_l2: alpha and beta must be finite, eps finite and >= 0";
    return SIM_ERR_INVALID_ARG;
  }
  for (int q = 0; q < 3; ++q)
    if (!(h_weights[q] >= 0.0) || !std::isfinite(h_weights[q])) {
      c->err = "sim_loss_cos_l2: class weights must be finite and >= 0";
      return SIM_ERR_INVALID_ARG;
    }
  if (gu) {
    const float* outs[3] = {gu, gv, gw};
    const float* ins[6] = {u, v, w, tu, tv, tw};
    for (const float* o : outs)
      for (const float* p : ins)
        if (o == p) {
          c->err = "sim_loss_cos_l2: a gradient output aliases an input";
          return SIM_ERR_INVALID_ARG;
        }
  }
  LossCoef cf;
  cf.alpha = (float)alpha;
  cf.beta = (float)beta;
  cf.eps2 = (float)(eps * eps);
  for (int q = 0; q < 3; ++q) cf.w[q] = (float)h_weights[q];
  // the per-cell weighted dJ/da lives in three solver buffers (free outside a solve)
  float* ga[3] = {gu ? c->dA : nullptr, gu ? c->dB : nullptr, gu ? c->q : nullptr};
  const int blocks = c->grid_cells;  // 2 partials per block, within the partials buffer
  hipLaunchKernelGGL(k_loss_cells, dim3(blocks), dim3(kBlock), 0, c->stream, c->n, c->cell,
                     CF3{{u, v, w}}, CF3{{tu, tv, tw}}, cf, ga[0], ga[1], ga[2], c->partials);
  hipLaunchKernelGGL(k_loss_fold, dim3(1), dim3(kBlock), 0, c->stream, c->partials, blocks, c->scal);
  if (gu)
    hipLaunchKernelGGL(k_loss_face_grad, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->n, ga[0],
                       ga[1], ga[2], c->scal, gu, gv, gw);
  if (hipGetLastError() != hipSuccess) return SIM_ERR_HIP;
  double sums[2] = {0.0, 0.0};
  if (hipMemcpyAsync(sums, c->scal + S_DOT0, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
          hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return SIM_ERR_HIP;
  *h_loss = sums[1] > 0.0 ? sums[0] / sums[1] : 0.0;
  return SIM_OK;
}
