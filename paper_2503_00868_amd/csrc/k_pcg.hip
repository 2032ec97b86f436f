// Conjugate-gradient kernels.
//
// Pressure (cell domain): the Poisson matrix A is matrix-free from the
// per-cell diagonal byte (number of non-wall faces of a liquid cell, zero
// off liquid); off-diagonals are -1 between liquid neighbours.  Every vector
// is zero off liquid, so a neighbour read needs no mask.  The iterate x is
// FP64; r, z, d, q are FP32; every dot product is accumulated in FP64.
// The scalars alpha and beta never leave the device: the last block of each
// reduction computes them (deterministic order) for the next kernel.
//
// One iteration of Jacobi PCG is two kernels:
//   dir_spmv : d' = M^-1 r + beta d ; q = A d' ; partial d'.q
//   update   : alpha = rz / dq ; x += alpha d' ; r -= alpha q ; partial r.M^-1 r
// With an explicit preconditioner (MIC(0), learned) z is an array computed
// between update and the next dir_spmv, and a separate kernel reduces r.z.
// Every m iterations `check` recomputes r = b - A x from the FP64 x (FP64
// residual replacement), reduces |r|^2 and raises the done flag at tol.
// Every kernel returns at once when the done flag is set, so the host can
// enqueue the next block of iterations before it has read the flag.
#include "common.h"
#include "ctx.h"

namespace fs {

struct Chunk2 {
  int64_t begin, end;
};

__device__ inline Chunk2 chunk_of(int64_t total, int nblocks, int lb) {
  int64_t per = (total + nblocks - 1) / nblocks;
  per = (per + kBlock - 1) / kBlock * kBlock;
  int64_t b = per * lb;
  int64_t e = b + per < total ? b + per : total;
  return Chunk2{b, e};
}

__constant__ float c_inv_count[8] = {0.f, 1.f, 0.5f, 1.f / 3.f, 0.25f, 0.2f, 1.f / 6.f, 0.f};

// (A v)_c for liquid c, in the precision of T.
template <typename T, typename V>
__device__ inline T poisson_row(const V* __restrict__ v, int64_t idx, uint8_t dg, const Walker& w,
                                int n) {
  const int64_t sy = n, sz = (int64_t)n * n;
  T s = (T)dg * (T)v[idx];
  if (w.i > 0) s -= (T)v[idx - 1];
  if (w.i < n - 1) s -= (T)v[idx + 1];
  if (w.j > 0) s -= (T)v[idx - sy];
  if (w.j < n - 1) s -= (T)v[idx + sy];
  if (w.k > 0) s -= (T)v[idx - sz];
  if (w.k < n - 1) s -= (T)v[idx + sz];
  return s;
}

// ---------------------------------------------------------------- Poisson

template <int PREC>
__global__ void __launch_bounds__(kBlock)
    k_pcg_init(int n, const uint8_t* __restrict__ cdiag, const float* __restrict__ b,
               double* __restrict__ x, float* __restrict__ r, float* __restrict__ d0,
               double* partials, unsigned* counter, double* scal, int* flags) {
  const int64_t C = cells(n);
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(C, gridDim.x, lb);
  double v[2] = {0.0, 0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    const float bv = b[idx];
    x[idx] = 0.0;
    r[idx] = bv;
    d0[idx] = 0.f;
    v[0] += (double)bv * bv;
    if (PREC == PK_JACOBI) v[1] += (double)bv * bv * c_inv_count[cdiag[idx]];
  }
  double tot[2];
  if (finish_sums<2>(v, partials, counter, gridDim.x, lb, tot) && threadIdx.x == 0) {
    scal[S_BB] = tot[0];
    scal[S_RR] = tot[0];
    scal[S_RZ] = tot[1];
    scal[S_RZ_PREV] = tot[1];
    scal[S_BETA] = 0.0;
    flags[F_DONE] = tot[0] == 0.0 ? 1 : 0;
    flags[F_ITERS] = 0;
    flags[F_ITERS_AT_DONE] = 0;
  }
}

template <int PREC>
__global__ void __launch_bounds__(kBlock)
    k_pcg_dir_spmv(int n, const uint8_t* __restrict__ cdiag, const float* __restrict__ r,
                   const float* __restrict__ z, const float* __restrict__ d_in,
                   float* __restrict__ d_out, float* __restrict__ q, double* partials,
                   unsigned* counter, double* scal, int* flags) {
  if (flags[F_DONE]) return;
  const int64_t C = cells(n);
  const float beta = (float)scal[S_BETA];
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(C, gridDim.x, lb);
  const int64_t sy = n, sz = (int64_t)n * n;
  auto dir = [&](int64_t m) -> float {
    const float zm = PREC == PK_JACOBI ? r[m] * c_inv_count[cdiag[m]] : z[m];
    return zm + beta * d_in[m];
  };
  Walker w;
  w.init(Dims{n, n, n}, ch.begin + threadIdx.x, kBlock);
  double v[1] = {0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock, w.next()) {
    const uint8_t dg = cdiag[idx];
    if (!dg) {
      d_out[idx] = 0.f;
      q[idx] = 0.f;
      continue;
    }
    const float dc = dir(idx);
    float s = 0.f;
    if (w.i > 0) s += dir(idx - 1);
    if (w.i < n - 1) s += dir(idx + 1);
    if (w.j > 0) s += dir(idx - sy);
    if (w.j < n - 1) s += dir(idx + sy);
    if (w.k > 0) s += dir(idx - sz);
    if (w.k < n - 1) s += dir(idx + sz);
    const float qc = (float)dg * dc - s;
    d_out[idx] = dc;
    q[idx] = qc;
    v[0] += (double)dc * (double)qc;
  }
  double tot[1];
  if (finish_sums<1>(v, partials, counter, gridDim.x, lb, tot) && threadIdx.x == 0) {
    scal[S_DQ] = tot[0];
    if (!(tot[0] > 0.0)) flags[F_DONE] = 2;  // breakdown (NaN or non-positive curvature)
  }
}

template <int PREC>
__global__ void __launch_bounds__(kBlock)
    k_pcg_update(int n, const uint8_t* __restrict__ cdiag, double* __restrict__ x,
                 float* __restrict__ r, const float* __restrict__ d, const float* __restrict__ q,
                 double* partials, unsigned* counter, double* scal, int* flags) {
  if (flags[F_DONE]) return;
  const int64_t C = cells(n);
  const double alpha = scal[S_RZ] / scal[S_DQ];
  const float alpha_f = (float)alpha;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(C, gridDim.x, lb);
  double v[1] = {0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    const uint8_t dg = cdiag[idx];
    if (!dg) continue;
    x[idx] += alpha * (double)d[idx];
    const float rn = r[idx] - alpha_f * q[idx];
    r[idx] = rn;
    if (PREC == PK_JACOBI) v[0] += (double)rn * (double)rn * c_inv_count[dg];
  }
  if (PREC != PK_JACOBI && blockIdx.x == 0 && threadIdx.x == 0) flags[F_ITERS] += 1;
  if (PREC == PK_JACOBI) {
    double tot[1];
    if (finish_sums<1>(v, partials, counter, gridDim.x, lb, tot) && threadIdx.x == 0) {
      const double rz_old = scal[S_RZ];
      scal[S_RZ_PREV] = rz_old;
      scal[S_RZ] = tot[0];
      scal[S_BETA] = tot[0] / rz_old;
      flags[F_ITERS] += 1;
    }
  }
}

// r.z for an explicit preconditioner output z; beta = rz_new / rz_old
// (first = 1: start of a solve, beta = 0 and no iteration counted).
__global__ void __launch_bounds__(kBlock)
    k_pcg_rz(int n, const float* __restrict__ r, const float* __restrict__ z, int first,
             double* partials, unsigned* counter, double* scal, int* flags) {
  if (flags[F_DONE]) return;
  const int64_t C = cells(n);
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(C, gridDim.x, lb);
  double v[1] = {0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock)
    v[0] += (double)r[idx] * (double)z[idx];
  double tot[1];
  if (finish_sums<1>(v, partials, counter, gridDim.x, lb, tot) && threadIdx.x == 0) {
    if (first) {
      scal[S_RZ] = tot[0];
      scal[S_RZ_PREV] = tot[0];
      scal[S_BETA] = 0.0;
    } else {
      const double rz_old = scal[S_RZ];
      scal[S_RZ_PREV] = rz_old;
      scal[S_RZ] = tot[0];
      scal[S_BETA] = tot[0] / rz_old;
    }
    if (!(tot[0] > 0.0) && !(tot[0] == 0.0 && scal[S_BB] == 0.0)) flags[F_DONE] = 2;
  }
}

// True residual in FP64 from the FP64 iterate; replaces r.  For Jacobi also
// recomputes r.M^-1 r and beta from the replaced residual.
template <int PREC>
__global__ void __launch_bounds__(kBlock)
    k_pcg_check(int n, const uint8_t* __restrict__ cdiag, const float* __restrict__ b,
                const double* __restrict__ x, float* __restrict__ r, double tol2,
                double* partials, unsigned* counter, double* scal, int* flags) {
  if (flags[F_DONE]) return;
  const int64_t C = cells(n);
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(C, gridDim.x, lb);
  Walker w;
  w.init(Dims{n, n, n}, ch.begin + threadIdx.x, kBlock);
  double v[2] = {0.0, 0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock, w.next()) {
    const uint8_t dg = cdiag[idx];
    if (!dg) continue;
    const double rc = (double)b[idx] - poisson_row<double>(x, idx, dg, w, n);
    const float rf = (float)rc;
    r[idx] = rf;
    v[0] += rc * rc;
    if (PREC == PK_JACOBI) v[1] += (double)rf * (double)rf * c_inv_count[dg];
  }
  double tot[2];
  if (finish_sums<2>(v, partials, counter, gridDim.x, lb, tot) && threadIdx.x == 0) {
    scal[S_RR] = tot[0];
    if (PREC == PK_JACOBI) {
      scal[S_RZ] = tot[1];
      scal[S_BETA] = scal[S_RZ_PREV] > 0.0 ? tot[1] / scal[S_RZ_PREV] : 0.0;
    }
    if (tot[0] <= tol2 * scal[S_BB]) {
      flags[F_DONE] = 1;
      flags[F_ITERS_AT_DONE] = flags[F_ITERS];
    }
  }
}

__global__ void __launch_bounds__(kBlock)
    k_poisson_apply(int n, const uint8_t* __restrict__ cdiag, const float* __restrict__ xin,
                    float* __restrict__ y) {
  const int64_t C = cells(n);
  const Chunk2 ch = chunk_of(C, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  Walker w;
  w.init(Dims{n, n, n}, ch.begin + threadIdx.x, kBlock);
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock, w.next()) {
    const uint8_t dg = cdiag[idx];
    y[idx] = dg ? poisson_row<float>(xin, idx, dg, w, n) : 0.f;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_jacobi_apply(int n, const uint8_t* __restrict__ cdiag, const float* __restrict__ r,
                   float* __restrict__ z) {
  const int64_t C = cells(n);
  const Chunk2 ch = chunk_of(C, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock)
    z[idx] = r[idx] * c_inv_count[cdiag[idx]];
}

__global__ void __launch_bounds__(kBlock)
    k_copy_double(int64_t C, const double* __restrict__ a, double* __restrict__ o) {
  for (int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x; idx < C;
       idx += (int64_t)gridDim.x * kBlock)
    o[idx] = a[idx];
}

void launch_pcg_init(sim_ctx* c, int prec) {
  if (prec == PK_JACOBI)
    hipLaunchKernelGGL(k_pcg_init<PK_JACOBI>, dim3(c->grid_cells), dim3(kBlock), 0, c->stream,
                       c->n, c->cdiag, c->b, c->x, c->r, c->dA, c->partials, c->counter, c->scal,
                       c->flags);
  else
    hipLaunchKernelGGL(k_pcg_init<PK_ZARRAY>, dim3(c->grid_cells), dim3(kBlock), 0, c->stream,
                       c->n, c->cdiag, c->b, c->x, c->r, c->dA, c->partials, c->counter, c->scal,
                       c->flags);
}

void launch_pcg_dir_spmv(sim_ctx* c, int prec, const float* d_in, float* d_out) {
  if (prec == PK_JACOBI)
    hipLaunchKernelGGL(k_pcg_dir_spmv<PK_JACOBI>, dim3(c->grid_cells), dim3(kBlock), 0, c->stream,
                       c->n, c->cdiag, c->r, c->z, d_in, d_out, c->q, c->partials, c->counter,
                       c->scal, c->flags);
  else
    hipLaunchKernelGGL(k_pcg_dir_spmv<PK_ZARRAY>, dim3(c->grid_cells), dim3(kBlock), 0, c->stream,
                       c->n, c->cdiag, c->r, c->z, d_in, d_out, c->q, c->partials, c->counter,
                       c->scal, c->flags);
}

void launch_pcg_update(sim_ctx* c, int prec, const float* d) {
  if (prec == PK_JACOBI)
    hipLaunchKernelGGL(k_pcg_update<PK_JACOBI>, dim3(c->grid_cells), dim3(kBlock), 0, c->stream,
                       c->n, c->cdiag, c->x, c->r, d, c->q, c->partials, c->counter, c->scal,
                       c->flags);
  else
    hipLaunchKernelGGL(k_pcg_update<PK_ZARRAY>, dim3(c->grid_cells), dim3(kBlock), 0, c->stream,
                       c->n, c->cdiag, c->x, c->r, d, c->q, c->partials, c->counter, c->scal,
                       c->flags);
}

void launch_pcg_rz_first(sim_ctx* c, int first) {
  hipLaunchKernelGGL(k_pcg_rz, dim3(c->grid_cells), dim3(kBlock), 0, c->stream, c->n, c->r, c->z,
                     first, c->partials, c->counter, c->scal, c->flags);
}

void launch_pcg_rz(sim_ctx* c) { launch_pcg_rz_first(c, 0); }

void launch_pcg_check(sim_ctx* c, int prec, double tol) {
  if (prec == PK_JACOBI)
    hipLaunchKernelGGL(k_pcg_check<PK_JACOBI>, dim3(c->grid_cells), dim3(kBlock), 0, c->stream,
                       c->n, c->cdiag, c->b, c->x, c->r, tol * tol, c->partials, c->counter,
                       c->scal, c->flags);
  else
    hipLaunchKernelGGL(k_pcg_check<PK_ZARRAY>, dim3(c->grid_cells), dim3(kBlock), 0, c->stream,
                       c->n, c->cdiag, c->b, c->x, c->r, tol * tol, c->partials, c->counter,
                       c->scal, c->flags);
}

void launch_poisson_apply(sim_ctx* c, const float* xin, float* y) {
  hipLaunchKernelGGL(k_poisson_apply, dim3(c->grid_cells), dim3(kBlock), 0, c->stream, c->n,
                     c->cdiag, xin, y);
}

void launch_jacobi_apply(sim_ctx* c, const float* r, float* z) {
  hipLaunchKernelGGL(k_jacobi_apply, dim3(c->grid_cells), dim3(kBlock), 0, c->stream, c->n,
                     c->cdiag, r, z);
}

void launch_x_to_double(sim_ctx* c, const double* xin, double* out) {
  hipLaunchKernelGGL(k_copy_double, dim3(1024), dim3(kBlock), 0, c->stream, c->C, xin, out);
}

// ---------------------------------------------------------- flexible CG
// Notay's flexible CG with one stored direction:
//   alpha = d.r / d.q ; x += alpha d ; r -= alpha q ; z = B(r) ;
//   beta = -(z.q) / (d.q) ; d = z + beta d.

__global__ void __launch_bounds__(kBlock)
    k_fcg_dir_spmv(int n, const uint8_t* __restrict__ cdiag, const float* __restrict__ r,
                   const float* __restrict__ z, const float* __restrict__ d_in,
                   float* __restrict__ d_out, float* __restrict__ q, double* partials,
                   unsigned* counter, double* scal, int* flags) {
  if (flags[F_DONE]) return;
  const int64_t C = cells(n);
  const float beta = (float)scal[S_BETA];
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(C, gridDim.x, lb);
  const int64_t sy = n, sz = (int64_t)n * n;
  auto dir = [&](int64_t m) -> float { return z[m] + beta * d_in[m]; };
  Walker w;
  w.init(Dims{n, n, n}, ch.begin + threadIdx.x, kBlock);
  double v[2] = {0.0, 0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock, w.next()) {
    const uint8_t dg = cdiag[idx];
    if (!dg) {
      d_out[idx] = 0.f;
      q[idx] = 0.f;
      continue;
    }
    const float dc = dir(idx);
    float s = 0.f;
    if (w.i > 0) s += dir(idx - 1);
    if (w.i < n - 1) s += dir(idx + 1);
    if (w.j > 0) s += dir(idx - sy);
    if (w.j < n - 1) s += dir(idx + sy);
    if (w.k > 0) s += dir(idx - sz);
    if (w.k < n - 1) s += dir(idx + sz);
    const float qc = (float)dg * dc - s;
    d_out[idx] = dc;
    q[idx] = qc;
    v[0] += (double)dc * (double)qc;
    v[1] += (double)dc * (double)r[idx];
  }
  double tot[2];
  if (finish_sums<2>(v, partials, counter, gridDim.x, lb, tot) && threadIdx.x == 0) {
    scal[S_DQ] = tot[0];
    scal[S_DR] = tot[1];
    if (!(tot[0] > 0.0) || !(tot[1] > 0.0)) flags[F_DONE] = 2;  // not a descent direction
  }
}

__global__ void __launch_bounds__(kBlock)
    k_fcg_update(int n, const uint8_t* __restrict__ cdiag, double* __restrict__ x,
                 float* __restrict__ r, const float* __restrict__ d, const float* __restrict__ q,
                 double* scal, int* flags) {
  if (flags[F_DONE]) return;
  const int64_t C = cells(n);
  const double alpha = scal[S_DR] / scal[S_DQ];
  const float alpha_f = (float)alpha;
  const Chunk2 ch = chunk_of(C, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    if (!cdiag[idx]) continue;
    x[idx] += alpha * (double)d[idx];
    r[idx] -= alpha_f * q[idx];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) flags[F_ITERS] += 1;
}

// beta = -(z.q)/(d.q); first = 1 at the start of a solve (beta = 0).
__global__ void __launch_bounds__(kBlock)
    k_fcg_beta(int n, const float* __restrict__ z, const float* __restrict__ q, int first,
               double* partials, unsigned* counter, double* scal, int* flags) {
  if (flags[F_DONE]) return;
  const int64_t C = cells(n);
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(C, gridDim.x, lb);
  double v[1] = {0.0};
  if (!first)
    for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock)
      v[0] += (double)z[idx] * (double)q[idx];
  double tot[1];
  if (finish_sums<1>(v, partials, counter, gridDim.x, lb, tot) && threadIdx.x == 0) {
    if (first) {
      scal[S_BETA] = 0.0;
    } else {
      scal[S_BETA] = -tot[0] / scal[S_DQ];
    }
    if (!(scal[S_BETA] == scal[S_BETA])) flags[F_DONE] = 2;
  }
}

void launch_fcg_init(sim_ctx* c) { launch_pcg_init(c, PK_ZARRAY); }

void launch_fcg_dir_spmv(sim_ctx* c, const float* d_in, float* d_out) {
  hipLaunchKernelGGL(k_fcg_dir_spmv, dim3(c->grid_cells), dim3(kBlock), 0, c->stream, c->n,
                     c->cdiag, c->r, c->z, d_in, d_out, c->q, c->partials, c->counter, c->scal,
                     c->flags);
}

void launch_fcg_update(sim_ctx* c, const float* d) {
  hipLaunchKernelGGL(k_fcg_update, dim3(c->grid_cells), dim3(kBlock), 0, c->stream, c->n, c->cdiag,
                     c->x, c->r, d, c->q, c->scal, c->flags);
}

void launch_fcg_beta_first(sim_ctx* c, int first) {
  hipLaunchKernelGGL(k_fcg_beta, dim3(c->grid_cells), dim3(kBlock), 0, c->stream, c->n, c->z, c->q,
                     first, c->partials, c->counter, c->scal, c->flags);
}

void launch_fcg_beta(sim_ctx* c) { launch_fcg_beta_first(c, 0); }

void launch_fcg_check(sim_ctx* c, double tol) { launch_pcg_check(c, PK_ZARRAY, tol); }

// ------------------------------------------------- implicit viscosity CG
// Solves (I - alpha L) x = b on the active faces of all three components at
// once (one CG on the stacked vector), Jacobi-preconditioned with
// diag = 1 + alpha * (number of Laplacian neighbours).  As for the pressure,
// the iterate is FP64 with FP64 residual replacement: with alpha = nu dt/h^2
// up to ~55 at 256^3 the rounding of an FP32 iterate alone would leave a
// relative residual of |M| * 2^-24 ~ 4e-5.  r, d, q are FP32, dots FP64.
// b is ctx->tmp; the FP64 iterate is ctx->fx; the result is rounded into
// the output fields at the end.

__device__ inline float mrow_diag_inv(uint8_t code, float alpha) {
  return (code & FC_ACTIVE) ? 1.f / (1.f + alpha * (float)__popc(code & 63u)) : 0.f;
}

template <typename T, typename V>
__device__ inline T mrow(const V* __restrict__ f, int64_t idx, uint8_t code, int64_t sy, int64_t sz,
                         T alpha) {
  const T v = (T)f[idx];
  T acc = 0;
  if (code & 1) acc += (T)f[idx - 1] - v;
  if (code & 2) acc += (T)f[idx + 1] - v;
  if (code & 4) acc += (T)f[idx - sy] - v;
  if (code & 8) acc += (T)f[idx + sy] - v;
  if (code & 16) acc += (T)f[idx - sz] - v;
  if (code & 32) acc += (T)f[idx + sz] - v;
  return v - alpha * acc;
}

// x = b (initial guess), r = b - M b, d0 = 0
__global__ void __launch_bounds__(kBlock)
    k_dcg_init(int n, const uint8_t* __restrict__ fcode, float alpha, const float* __restrict__ b,
               double* __restrict__ x, float* __restrict__ r, float* __restrict__ d0, int64_t F,
               double* partials, unsigned* counter, double* scal, int* flags, double tol2) {
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  const int64_t sy = d.nx, sz = (int64_t)d.nx * d.ny;
  const uint8_t* __restrict__ code = fcode + comp * F;
  const float* __restrict__ bc = b + comp * F;
  double* __restrict__ xc = x + comp * F;
  float* __restrict__ rc = r + comp * F;
  float* __restrict__ dc = d0 + comp * F;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(F, gridDim.x, lb);
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    const uint8_t cd = code[idx];
    dc[idx] = 0.f;
    if (!(cd & FC_ACTIVE)) {
      rc[idx] = 0.f;
      xc[idx] = 0.0;
      continue;
    }
    xc[idx] = (double)bc[idx];
    const double rv = (double)bc[idx] - mrow<double>(bc, idx, cd, sy, sz, (double)alpha);
    const float rf = (float)rv;
    rc[idx] = rf;
    v[0] += (double)bc[idx] * bc[idx];
    v[1] += (double)rf * rf * mrow_diag_inv(cd, alpha);
    v[2] += rv * rv;
  }
  double tot[3];
  if (finish_sums<3>(v, partials, counter, gridDim.x * gridDim.y, comp * gridDim.x + lb, tot) &&
      threadIdx.x == 0) {
    scal[S_BB] = tot[0];
    scal[S_RZ] = tot[1];
    scal[S_RZ_PREV] = tot[1];
    scal[S_RR] = tot[2];
    scal[S_BETA] = 0.0;
    flags[F_DONE] = tot[2] <= tol2 * tot[0] ? 1 : 0;
    flags[F_ITERS] = 0;
    flags[F_ITERS_AT_DONE] = 0;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_dcg_dir_spmv(int n, const uint8_t* __restrict__ fcode, float alpha,
                   const float* __restrict__ r, const float* __restrict__ d_in,
                   float* __restrict__ d_out, float* __restrict__ q, int64_t F, double* partials,
                   unsigned* counter, double* scal, int* flags) {
  if (flags[F_DONE]) return;
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  const int64_t sy = d.nx, sz = (int64_t)d.nx * d.ny;
  const float beta = (float)scal[S_BETA];
  const uint8_t* __restrict__ code = fcode + comp * F;
  const float* __restrict__ rc = r + comp * F;
  const float* __restrict__ di = d_in + comp * F;
  float* __restrict__ dout = d_out + comp * F;
  float* __restrict__ qc = q + comp * F;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(F, gridDim.x, lb);
  auto dir = [&](int64_t m) -> float { return rc[m] * mrow_diag_inv(code[m], alpha) + beta * di[m]; };
  double v[1] = {0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    const uint8_t cd = code[idx];
    if (!(cd & FC_ACTIVE)) {
      dout[idx] = 0.f;
      qc[idx] = 0.f;
      continue;
    }
    const float dcur = dir(idx);
    float acc = 0.f;
    if (cd & 1) acc += dir(idx - 1) - dcur;
    if (cd & 2) acc += dir(idx + 1) - dcur;
    if (cd & 4) acc += dir(idx - sy) - dcur;
    if (cd & 8) acc += dir(idx + sy) - dcur;
    if (cd & 16) acc += dir(idx - sz) - dcur;
    if (cd & 32) acc += dir(idx + sz) - dcur;
    const float qv = dcur - alpha * acc;
    dout[idx] = dcur;
    qc[idx] = qv;
    v[0] += (double)dcur * (double)qv;
  }
  double tot[1];
  if (finish_sums<1>(v, partials, counter, gridDim.x * gridDim.y, comp * gridDim.x + lb, tot) &&
      threadIdx.x == 0) {
    scal[S_DQ] = tot[0];
    if (!(tot[0] > 0.0)) flags[F_DONE] = 2;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_dcg_update(const uint8_t* __restrict__ fcode, float alpha, double* __restrict__ x,
                 float* __restrict__ r, const float* __restrict__ d, const float* __restrict__ q,
                 int64_t F, double* partials, unsigned* counter, double* scal, int* flags) {
  if (flags[F_DONE]) return;
  const int comp = blockIdx.y;
  const double a = scal[S_RZ] / scal[S_DQ];
  const float af = (float)a;
  const uint8_t* __restrict__ code = fcode + comp * F;
  double* __restrict__ xc = x + comp * F;
  float* __restrict__ rc = r + comp * F;
  const float* __restrict__ dc = d + comp * F;
  const float* __restrict__ qc = q + comp * F;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(F, gridDim.x, lb);
  double v[1] = {0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    const uint8_t cd = code[idx];
    if (!(cd & FC_ACTIVE)) continue;
    xc[idx] += a * (double)dc[idx];
    const float rn = rc[idx] - af * qc[idx];
    rc[idx] = rn;
    v[0] += (double)rn * (double)rn * mrow_diag_inv(cd, alpha);
  }
  double tot[1];
  if (finish_sums<1>(v, partials, counter, gridDim.x * gridDim.y, comp * gridDim.x + lb, tot) &&
      threadIdx.x == 0) {
    const double rz_old = scal[S_RZ];
    scal[S_RZ_PREV] = rz_old;
    scal[S_RZ] = tot[0];
    scal[S_BETA] = tot[0] / rz_old;
    flags[F_ITERS] += 1;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_dcg_check(int n, const uint8_t* __restrict__ fcode, float alpha, const float* __restrict__ b,
                const double* __restrict__ x, float* __restrict__ r, int64_t F, double tol2,
                double* partials, unsigned* counter, double* scal, int* flags) {
  if (flags[F_DONE]) return;
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  const int64_t sy = d.nx, sz = (int64_t)d.nx * d.ny;
  const uint8_t* __restrict__ code = fcode + comp * F;
  const float* __restrict__ bc = b + comp * F;
  const double* __restrict__ xc = x + comp * F;
  float* __restrict__ rc = r + comp * F;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(F, gridDim.x, lb);
  double v[2] = {0.0, 0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    const uint8_t cd = code[idx];
    if (!(cd & FC_ACTIVE)) continue;
    const double rv = (double)bc[idx] - mrow<double>(xc, idx, cd, sy, sz, (double)alpha);
    const float rf = (float)rv;
    rc[idx] = rf;
    v[0] += rv * rv;
    v[1] += (double)rf * rf * mrow_diag_inv(cd, alpha);
  }
  double tot[2];
  if (finish_sums<2>(v, partials, counter, gridDim.x * gridDim.y, comp * gridDim.x + lb, tot) &&
      threadIdx.x == 0) {
    scal[S_RR] = tot[0];
    scal[S_RZ] = tot[1];
    scal[S_BETA] = scal[S_RZ_PREV] > 0.0 ? tot[1] / scal[S_RZ_PREV] : 0.0;
    if (tot[0] <= tol2 * scal[S_BB]) {
      flags[F_DONE] = 1;
      flags[F_ITERS_AT_DONE] = flags[F_ITERS];
    }
  }
}

// out = (float) x on active faces, 0 elsewhere
__global__ void __launch_bounds__(kBlock)
    k_dcg_finish(const uint8_t* __restrict__ fcode, const double* __restrict__ x, F3 out,
                 int64_t F) {
  const int comp = blockIdx.y;
  const uint8_t* __restrict__ code = fcode + comp * F;
  const double* __restrict__ xc = x + comp * F;
  const Chunk2 ch = chunk_of(F, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock)
    out.c[comp][idx] = (code[idx] & FC_ACTIVE) ? (float)xc[idx] : 0.f;
}

void launch_dcg_init(sim_ctx* c, float alpha) {
  hipLaunchKernelGGL(k_dcg_init, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->n,
                     c->fcode, alpha, c->tmp, c->fx, c->fr, c->fdA, c->F, c->partials, c->counter,
                     c->scal, c->flags, c->desc.diff_tol * c->desc.diff_tol);
}

void launch_dcg_dir_spmv(sim_ctx* c, float alpha, const float* d_in, float* d_out) {
  hipLaunchKernelGGL(k_dcg_dir_spmv, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->n,
                     c->fcode, alpha, c->fr, d_in, d_out, c->fq, c->F, c->partials, c->counter,
                     c->scal, c->flags);
}

void launch_dcg_update(sim_ctx* c, float alpha, const float* d) {
  hipLaunchKernelGGL(k_dcg_update, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->fcode,
                     alpha, c->fx, c->fr, d, c->fq, c->F, c->partials, c->counter, c->scal,
                     c->flags);
}

void launch_dcg_check(sim_ctx* c, float alpha, double tol) {
  hipLaunchKernelGGL(k_dcg_check, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->n,
                     c->fcode, alpha, c->tmp, c->fx, c->fr, c->F, tol * tol, c->partials,
                     c->counter, c->scal, c->flags);
}

void launch_dcg_finish(sim_ctx* c, F3 out) {
  hipLaunchKernelGGL(k_dcg_finish, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->fcode,
                     c->fx, out, c->F);
}

}  // namespace fs
