// The paper's screen-space constrained projection (Section 3.3,
// Eq. (div2DV)): the 2-D screen velocity must have the divergence that the
// divergence-free 3-D surface motion implies, div v = s with
// s = -(u dvz/du + v dvz/dv + 2 vz) / z.  Where optical flow failed (a pixel
// region), the interpolated velocity is projected onto that constraint by a
// potential that is zero off the region.
//
// Reading used here: screen coordinates normalised to [-1, 1] at pixel
// centres (spacings du = 2/W, dv = 2/H); the velocity staggered on pixel
// edges (a, the u component, on the H x (W + 1) vertical edges; b on the
// (H + 1) x W horizontal ones); second-order central differences of vz, one
// sided (second order) at the image border; an edge is free when one of its
// two pixels is in the region and both lie in the image; the potential p
// solves A p = s - div v on the region (A the masked 5-point Laplacian over
// the free edges) and the free edges lose the gradient of p.
//
// The solve is Jacobi-preconditioned CG in FP64 (the system is 2-D and
// small next to the 3-D step), matrix-free from the mask: directions are zero
// off the region, so a region pixel's row is diag * d - sum of its in-image
// neighbours' d / h^2.  alpha and beta are formed on the device; the host
// reads the done flag every kCheck iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <utility>

#include "../../include/fluidsim.h"
#include "common.h"

namespace fs {
namespace {

constexpr int kS2MaxGrid = 2048;
constexpr int kCheck = 16;
enum { S2_BB = 0, S2_RZ, S2_DQ, S2_ALPHA, S2_BETA, S2_RR, S2_TRUE, S2_SCAL = 8 };
enum { S2F_DONE = 0, S2F_ITERS, S2F_COUNT = 4 };

struct S2 {
  int H, W;
  double du, dv;
};

__device__ inline double s2_target(const S2& g, const float* __restrict__ vz,
                                   const float* __restrict__ z, int j, int i) {
  const int W = g.W, H = g.H;
  const int64_t p = (int64_t)j * W + i;
  double gu, gv;
  if (i == 0)
    gu = (-3.0 * vz[p] + 4.0 * vz[p + 1] - vz[p + 2]) / (2.0 * g.du);
  else if (i == W - 1)
    gu = (3.0 * vz[p] - 4.0 * vz[p - 1] + vz[p - 2]) / (2.0 * g.du);
  else
    gu = ((double)vz[p + 1] - (double)vz[p - 1]) / (2.0 * g.du);
  if (j == 0)
    gv = (-3.0 * vz[p] + 4.0 * vz[p + W] - vz[p + 2 * W]) / (2.0 * g.dv);
  else if (j == H - 1)
    gv = (3.0 * vz[p] - 4.0 * vz[p - W] + vz[p - 2 * W]) / (2.0 * g.dv);
  else
    gv = ((double)vz[p + W] - (double)vz[p - W]) / (2.0 * g.dv);
  const double u = -1.0 + (2.0 * i + 1.0) / W, v = -1.0 + (2.0 * j + 1.0) / H;
  return -(u * gu + v * gv + 2.0 * (double)vz[p]) / (double)z[p];
}

// diagonal of a region pixel's row: one 1/h^2 per in-image edge
__device__ inline double s2_diag(const S2& g, int j, int i) {
  const double iu = 1.0 / (g.du * g.du), iv = 1.0 / (g.dv * g.dv);
  return iu * ((i > 0) + (i < g.W - 1)) + iv * ((j > 0) + (j < g.H - 1));
}

// Per pixel: the right-hand side s - div v on the region (kept in rhs and as
// the first residual), x = 0, z = r / diag, d = 0; partials [|rhs|^2, r.z].
__global__ void __launch_bounds__(kBlock)
    k_s2_setup(S2 g, const float* __restrict__ a, const float* __restrict__ b,
               const float* __restrict__ vz, const float* __restrict__ z,
               const uint8_t* __restrict__ mask, double* __restrict__ rhs, double* __restrict__ x,
               double* __restrict__ r, double* __restrict__ zz, double* __restrict__ d,
               double* partials) {
  const int64_t N = (int64_t)g.H * g.W;
  double v[2] = {0.0, 0.0};
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < N; p += (int64_t)gridDim.x * kBlock) {
    const int j = (int)(p / g.W), i = (int)(p - (int64_t)j * g.W);
    double rv = 0.0, zv = 0.0;
    if (mask[p]) {
      const int64_t ea = (int64_t)j * (g.W + 1) + i, eb = p;
      const double div = ((double)a[ea + 1] - (double)a[ea]) / g.du +
                         ((double)b[eb + g.W] - (double)b[eb]) / g.dv;
      rv = s2_target(g, vz, z, j, i) - div;
      zv = rv / s2_diag(g, j, i);
    }
    rhs[p] = rv;
    r[p] = rv;
    zz[p] = zv;
    x[p] = 0.0;
    d[p] = 0.0;
    v[0] += rv * rv;
    v[1] += rv * zv;
  }
  store_partials<2>(v, partials, blockIdx.x);
}

__device__ inline double s2_dir(const uint8_t* __restrict__ mask, const double* __restrict__ zz,
                                const double* __restrict__ d_in, double beta, int64_t p) {
  return mask[p] ? zz[p] + beta * d_in[p] : 0.0;
}

// d_out = z + beta d_in at every pixel (0 off the region), q = A d_out, and
// the partial d.q.  Returns at once when the solve is done.
__global__ void __launch_bounds__(kBlock)
    k_s2_dir_spmv(S2 g, const uint8_t* __restrict__ mask, const double* __restrict__ zz,
                  const double* __restrict__ d_in, double* __restrict__ d_out,
                  double* __restrict__ q, const double* __restrict__ scal,
                  const int* __restrict__ flags, double* partials) {
  if (flags[S2F_DONE]) return;
  const int64_t N = (int64_t)g.H * g.W;
  const double beta = scal[S2_BETA];
  const double iu = 1.0 / (g.du * g.du), iv = 1.0 / (g.dv * g.dv);
  double v[1] = {0.0};
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < N; p += (int64_t)gridDim.x * kBlock) {
    const int j = (int)(p / g.W), i = (int)(p - (int64_t)j * g.W);
    const double dc = s2_dir(mask, zz, d_in, beta, p);
    double qv = 0.0;
    if (mask[p]) {
      double nb_u = 0.0, nb_v = 0.0;
      if (i > 0) nb_u += s2_dir(mask, zz, d_in, beta, p - 1);
      if (i < g.W - 1) nb_u += s2_dir(mask, zz, d_in, beta, p + 1);
      if (j > 0) nb_v += s2_dir(mask, zz, d_in, beta, p - g.W);
      if (j < g.H - 1) nb_v += s2_dir(mask, zz, d_in, beta, p + g.W);
      qv = s2_diag(g, j, i) * dc - iu * nb_u - iv * nb_v;
    }
    d_out[p] = dc;
    q[p] = qv;
    v[0] += dc * qv;
  }
  store_partials<1>(v, partials, blockIdx.x);
}

// x += alpha d, r -= alpha q, z = r / diag; partials [r.z, |r|^2]
__global__ void __launch_bounds__(kBlock)
    k_s2_update(S2 g, const uint8_t* __restrict__ mask, const double* __restrict__ d,
                const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r,
                double* __restrict__ zz, const double* __restrict__ scal,
                const int* __restrict__ flags, double* partials) {
  if (flags[S2F_DONE]) return;
  const int64_t N = (int64_t)g.H * g.W;
  const double alpha = scal[S2_ALPHA];
  double v[2] = {0.0, 0.0};
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < N; p += (int64_t)gridDim.x * kBlock) {
    if (!mask[p]) continue;
    const int j = (int)(p / g.W), i = (int)(p - (int64_t)j * g.W);
    x[p] += alpha * d[p];
    const double rv = r[p] - alpha * q[p];
    const double zv = rv / s2_diag(g, j, i);
    r[p] = rv;
    zz[p] = zv;
    v[0] += rv * zv;
    v[1] += rv * rv;
  }
  store_partials<2>(v, partials, blockIdx.x);
}

enum S2Fin { S2_FIN_INIT = 0, S2_FIN_DQ, S2_FIN_UPD, S2_FIN_TRUE };

__global__ void __launch_bounds__(kBlock)
    k_s2_finalize(const double* __restrict__ partials, int nblocks, int nv, int mode,
                  double* __restrict__ scal, int* __restrict__ flags, double tol2) {
  if ((mode == S2_FIN_DQ || mode == S2_FIN_UPD) && flags[S2F_DONE]) return;
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kBlock)
    for (int t = 0; t < nv; ++t) v[t] += partials[(int64_t)b * nv + t];
  block_sum<2>(v);
  if (threadIdx.x != 0) return;
  switch (mode) {
    case S2_FIN_INIT:
      scal[S2_BB] = v[0];
      scal[S2_RR] = v[0];
      scal[S2_RZ] = v[1];
      scal[S2_BETA] = 0.0;
      flags[S2F_DONE] = v[0] == 0.0 ? 1 : 0;
      flags[S2F_ITERS] = 0;
      break;
    case S2_FIN_DQ:
      scal[S2_DQ] = v[0];
      scal[S2_ALPHA] = scal[S2_RZ] / v[0];
      flags[S2F_ITERS] += 1;
      if (!(v[0] > 0.0)) flags[S2F_DONE] = 2;  // breakdown (a singular or indefinite system)
      break;
    case S2_FIN_UPD:
      scal[S2_BETA] = v[0] / scal[S2_RZ];
      scal[S2_RZ] = v[0];
      scal[S2_RR] = v[1];
      if (v[1] <= tol2 * scal[S2_BB]) flags[S2F_DONE] = 1;
      else if (!(v[1] == v[1])) flags[S2F_DONE] = 2;
      break;
    case S2_FIN_TRUE:
      scal[S2_TRUE] = v[0];
      break;
  }
}

// the true residual |rhs - A x|^2 (partials [value])
__global__ void __launch_bounds__(kBlock)
    k_s2_true_residual(S2 g, const uint8_t* __restrict__ mask, const double* __restrict__ rhs,
                       const double* __restrict__ x, double* partials) {
  const int64_t N = (int64_t)g.H * g.W;
  const double iu = 1.0 / (g.du * g.du), iv = 1.0 / (g.dv * g.dv);
  double v[1] = {0.0};
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < N; p += (int64_t)gridDim.x * kBlock) {
    if (!mask[p]) continue;
    const int j = (int)(p / g.W), i = (int)(p - (int64_t)j * g.W);
    double nb_u = 0.0, nb_v = 0.0;
    if (i > 0 && mask[p - 1]) nb_u += x[p - 1];
    if (i < g.W - 1 && mask[p + 1]) nb_u += x[p + 1];
    if (j > 0 && mask[p - g.W]) nb_v += x[p - g.W];
    if (j < g.H - 1 && mask[p + g.W]) nb_v += x[p + g.W];
    const double res = rhs[p] - (s2_diag(g, j, i) * x[p] - iu * nb_u - iv * nb_v);
    v[0] += res * res;
  }
  store_partials<1>(v, partials, blockIdx.x);
}

// every free edge loses the gradient of p (p = 0 off the region): a-edges
// (j, i) for 1 <= i <= W - 1, then b-edges (j, i) for 1 <= j <= H - 1
__global__ void __launch_bounds__(kBlock)
    k_s2_apply(S2 g, const uint8_t* __restrict__ mask, const double* __restrict__ x,
               float* __restrict__ a, float* __restrict__ b) {
  const int64_t NA = (int64_t)g.H * (g.W + 1), NB = (int64_t)(g.H + 1) * g.W;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < NA + NB;
       e += (int64_t)gridDim.x * kBlock) {
    if (e < NA) {
      const int j = (int)(e / (g.W + 1)), i = (int)(e - (int64_t)j * (g.W + 1));
      if (i == 0 || i == g.W) continue;
      const int64_t lo = (int64_t)j * g.W + i - 1, hi = lo + 1;
      if (!(mask[lo] | mask[hi])) continue;
      const double plo = mask[lo] ? x[lo] : 0.0, phi = mask[hi] ? x[hi] : 0.0;
      a[e] = (float)((double)a[e] - (phi - plo) / g.du);
    } else {
      const int64_t f = e - NA;
      const int j = (int)(f / g.W), i = (int)(f - (int64_t)j * g.W);
      if (j == 0 || j == g.H) continue;
      const int64_t lo = (int64_t)(j - 1) * g.W + i, hi = lo + g.W;
      if (!(mask[lo] | mask[hi])) continue;
      const double plo = mask[lo] ? x[lo] : 0.0, phi = mask[hi] ? x[hi] : 0.0;
      b[f] = (float)((double)b[f] - (phi - plo) / g.dv);
    }
  }
}

size_t s2_align(size_t v) { return (v + 255) / 256 * 256; }

// workspace: rhs, x, r, z, dA, dB, q (FP64 pixel vectors), partials, scalars, flags
size_t s2_bytes(int H, int W, size_t offs[10]) {
  const size_t N = (size_t)H * W;
  size_t o = 0;
  for (int t = 0; t < 7; ++t) {
    offs[t] = o;
    o = s2_align(o + N * sizeof(double));
  }
  offs[7] = o;
  o = s2_align(o + (size_t)kS2MaxGrid * 2 * sizeof(double));
  offs[8] = o;
  o = s2_align(o + S2_SCAL * sizeof(double));
  offs[9] = o;
  o = s2_align(o + S2F_COUNT * sizeof(int));
  return o;
}

int s2_grid(int64_t items) {
  int64_t g = (items + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g > kS2MaxGrid ? kS2MaxGrid : g));
}

}  // namespace
}  // namespace fs

using namespace fs;

extern "C" int sim_screen_workspace_size(int32_t H, int32_t W, size_t* bytes) {
  if (!bytes || H < 3 || W < 3 || H > 16384 || W > 16384) return SIM_ERR_INVALID_ARG;
  size_t offs[10];
  *bytes = s2_bytes(H, W, offs);
  return SIM_OK;
}

extern "C" int sim_screen_project(int32_t H, int32_t W, float* d_a, float* d_b, const float* d_vz,
                                  const float* d_z, const uint8_t* d_mask, double tol,
                                  int32_t max_iter, void* d_workspace, size_t workspace_bytes,
                                  void* hip_stream, int32_t* h_iters, double* h_rel_residual) {
  if (H < 3 || W < 3 || H > 16384 || W > 16384) return SIM_ERR_INVALID_ARG;
  if (!d_a || !d_b || !d_vz || !d_z || !d_mask || !d_workspace) return SIM_ERR_INVALID_ARG;
  if (!(tol > 0.0 && tol < 1.0) || max_iter < 1) return SIM_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0) return SIM_ERR_INVALID_ARG;
  size_t offs[10];
  if (workspace_bytes < s2_bytes(H, W, offs)) return SIM_ERR_WORKSPACE_TOO_SMALL;
  char* base = static_cast<char*>(d_workspace);
  double* vec[7];
  for (int t = 0; t < 7; ++t) vec[t] = reinterpret_cast<double*>(base + offs[t]);
  double *rhs = vec[0], *x = vec[1], *r = vec[2], *zz = vec[3], *dA = vec[4], *dB = vec[5],
         *q = vec[6];
  double* partials = reinterpret_cast<double*>(base + offs[7]);
  double* scal = reinterpret_cast<double*>(base + offs[8]);
  int* flags = reinterpret_cast<int*>(base + offs[9]);
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const S2 g{H, W, 2.0 / W, 2.0 / H};
  const int64_t N = (int64_t)H * W;
  const int nb = s2_grid(N);
  const double tol2 = tol * tol;

  hipLaunchKernelGGL(k_s2_setup, dim3(nb), dim3(kBlock), 0, st, g, d_a, d_b, d_vz, d_z, d_mask, rhs,
                     x, r, zz, dA, partials);
  hipLaunchKernelGGL(k_s2_finalize, dim3(1), dim3(kBlock), 0, st, partials, nb, 2, (int)S2_FIN_INIT,
                     scal, flags, tol2);
  int it = 0, fl[S2F_COUNT] = {0, 0, 0, 0};
  double* din = dA;
  double* dout = dB;
  while (it < max_iter) {
    const int todo = std::min(kCheck, max_iter - it);
    for (int t = 0; t < todo; ++t) {
      hipLaunchKernelGGL(k_s2_dir_spmv, dim3(nb), dim3(kBlock), 0, st, g, d_mask, zz, din, dout, q,
                         scal, flags, partials);
      hipLaunchKernelGGL(k_s2_finalize, dim3(1), dim3(kBlock), 0, st, partials, nb, 1,
                         (int)S2_FIN_DQ, scal, flags, tol2);
      hipLaunchKernelGGL(k_s2_update, dim3(nb), dim3(kBlock), 0, st, g, d_mask, dout, q, x, r, zz,
                         scal, flags, partials);
      hipLaunchKernelGGL(k_s2_finalize, dim3(1), dim3(kBlock), 0, st, partials, nb, 2,
                         (int)S2_FIN_UPD, scal, flags, tol2);
      std::swap(din, dout);
    }
    it += todo;
    if (hipGetLastError() != hipSuccess) return SIM_ERR_HIP;
    if (hipMemcpyAsync(fl, flags, sizeof fl, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return SIM_ERR_HIP;
    if (fl[S2F_DONE]) break;
  }
  hipLaunchKernelGGL(k_s2_true_residual, dim3(nb), dim3(kBlock), 0, st, g, d_mask, rhs, x, partials);
  hipLaunchKernelGGL(k_s2_finalize, dim3(1), dim3(kBlock), 0, st, partials, nb, 1,
                     (int)S2_FIN_TRUE, scal, flags, tol2);
  hipLaunchKernelGGL(k_s2_apply, dim3(s2_grid((int64_t)H * (W + 1) + (int64_t)(H + 1) * W)),
                     dim3(kBlock), 0, st, g, d_mask, x, d_a, d_b);
  double sc[S2_SCAL];
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(sc, scal, sizeof sc, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(fl, flags, sizeof fl, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SIM_ERR_HIP;
  if (h_iters) *h_iters = fl[S2F_ITERS];
  const double rel = sc[S2_BB] > 0.0 ? std::sqrt(sc[S2_TRUE] / sc[S2_BB]) : 0.0;
  if (h_rel_residual) *h_rel_residual = rel;
  if (fl[S2F_DONE] == 2) return SIM_ERR_NOT_CONVERGED;
  return rel <= tol * 1.01 || fl[S2F_DONE] == 1 ? SIM_OK : SIM_ERR_NOT_CONVERGED;
}
