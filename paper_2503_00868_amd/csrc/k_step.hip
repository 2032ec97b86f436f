// Kernels of one liquid step outside the linear solvers: the per-mask tables,
// semi-Lagrangian advection with the body force, the explicit viscosity
// sub-step, the Poisson right-hand side and the pressure-gradient update.
//
// Paper: momentum equation with gravity, viscosity and pressure (Section
// 3.2.2, Eq. (v)), split into sub-steps (Section 3.2.2); semi-Lagrangian
// back-tracing of the convection term (Section 3.4.1).
//
// All face-domain kernels run on a (blocks, 3) grid: blockIdx.y is the
// velocity component and each block owns one contiguous run of that
// component's faces (XCD-contiguous block order).  They are HBM-bound
// streaming/stencil kernels; neighbour reuse comes from L1/L2.
#include "common.h"
#include "ctx.h"

namespace fs {

struct Chunk {
  int64_t begin, end;
};

__device__ inline Chunk block_chunk(int64_t total, int nblocks, int lb) {
  int64_t per = (total + nblocks - 1) / nblocks;
  per = (per + kBlock - 1) / kBlock * kBlock;
  int64_t b = per * lb;
  int64_t e = b + per < total ? b + per : total;
  return Chunk{b, e};
}

__device__ inline uint8_t cell_at(const uint8_t* cell, int n, int i, int j, int k) {
  if ((unsigned)i >= (unsigned)n || (unsigned)j >= (unsigned)n || (unsigned)k >= (unsigned)n)
    return SOLID;
  return cell[i + (int64_t)n * (j + (int64_t)n * k)];
}

enum { CLS_INACTIVE = 0, CLS_ACTIVE = 1, CLS_WALL = 2 };

__device__ inline int face_class(const uint8_t* cell, int n, int comp, int i, int j, int k) {
  Dims d = face_dims(n, comp);
  if (i < 0 || j < 0 || k < 0 || i >= d.nx || j >= d.ny || k >= d.nz) return CLS_WALL;
  uint8_t a = cell_at(cell, n, i - (comp == 0), j - (comp == 1), k - (comp == 2));
  uint8_t b = cell_at(cell, n, i, j, k);
  if (a == SOLID || b == SOLID) return CLS_WALL;
  if (a == LIQUID || b == LIQUID) return CLS_ACTIVE;
  return CLS_INACTIVE;
}

// ---------------------------------------------------------------- tables

__global__ void __launch_bounds__(kBlock) k_face_codes(int n, const uint8_t* __restrict__ cell,
                                                       uint8_t* __restrict__ fcode, int64_t F) {
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  const Chunk ch = block_chunk(F, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  Walker w;
  w.init(d, ch.begin + threadIdx.x, kBlock);
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock, w.next()) {
    uint8_t code = 0;
    if (face_class(cell, n, comp, w.i, w.j, w.k) == CLS_ACTIVE) {
      code = FC_ACTIVE;
      for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s) {
          int o = s ? 1 : -1;
          int cls = face_class(cell, n, comp, w.i + (a == 0) * o, w.j + (a == 1) * o,
                               w.k + (a == 2) * o);
          if (cls == CLS_ACTIVE || (cls == CLS_WALL && a == comp)) code |= (uint8_t)(1u << (2 * a + s));
        }
    }
    fcode[comp * F + idx] = code;
  }
}

__global__ void __launch_bounds__(kBlock) k_cell_diag(int n, const uint8_t* __restrict__ cell,
                                                      uint8_t* __restrict__ cdiag) {
  const int64_t C = cells(n);
  const Chunk ch = block_chunk(C, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  Walker w;
  w.init(Dims{n, n, n}, ch.begin + threadIdx.x, kBlock);
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock, w.next()) {
    uint8_t v = 0;
    if (cell[idx] == LIQUID) {
      int cnt = 0;
      cnt += cell_at(cell, n, w.i - 1, w.j, w.k) != SOLID;
      cnt += cell_at(cell, n, w.i + 1, w.j, w.k) != SOLID;
      cnt += cell_at(cell, n, w.i, w.j - 1, w.k) != SOLID;
      cnt += cell_at(cell, n, w.i, w.j + 1, w.k) != SOLID;
      cnt += cell_at(cell, n, w.i, w.j, w.k - 1) != SOLID;
      cnt += cell_at(cell, n, w.i, w.j, w.k + 1) != SOLID;
      v = (uint8_t)cnt;
    }
    cdiag[idx] = v;
  }
}

void launch_setup_tables(sim_ctx* c) {
  hipLaunchKernelGGL(k_face_codes, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->n,
                     c->cell, c->fcode, c->F);
  hipLaunchKernelGGL(k_cell_diag, dim3(c->grid_cells), dim3(kBlock), 0, c->stream, c->n, c->cell,
                     c->cdiag);
}

// -------------------------------------------------------------- sampling

// Lower node and fraction along one axis of a node lattice with cnt nodes,
// for the position base + rho (base an integer node index, rho a small
// offset).  Clamped to the lattice: below the first node -> (0, 0), past the
// last -> (cnt-2, 1).  floor() breaks ties at exact nodes.
__device__ inline void lattice_axis(int base, float rho, int cnt, int& i0, float& fr) {
  float fl = floorf(rho);
  int ii = base + (int)fl;
  float f = rho - fl;
  if (ii < 0) {
    ii = 0;
    f = 0.f;
  } else if (ii > cnt - 2) {
    ii = cnt - 2;
    f = 1.f;
  }
  i0 = ii;
  fr = f;
}

// Trilinear sample of a component array with dims d at node-lattice
// position (i + rx, j + ry, k + rz).
__device__ inline float sample3(const float* __restrict__ f, Dims d, int i, int j, int k, float rx,
                                float ry, float rz) {
  int i0, j0, k0;
  float fx, fy, fz;
  lattice_axis(i, rx, d.nx, i0, fx);
  lattice_axis(j, ry, d.ny, j0, fy);
  lattice_axis(k, rz, d.nz, k0, fz);
  const int64_t sy = d.nx, sz = (int64_t)d.nx * d.ny;
  const float* p = f + i0 + sy * j0 + sz * k0;
  float c00 = p[0] + fx * (p[1] - p[0]);
  float c10 = p[sy] + fx * (p[sy + 1] - p[sy]);
  float c01 = p[sz] + fx * (p[sz + 1] - p[sz]);
  float c11 = p[sz + sy] + fx * (p[sz + sy + 1] - p[sz + sy]);
  float c0 = c00 + fy * (c10 - c00);
  float c1 = c01 + fy * (c11 - c01);
  return c0 + fz * (c1 - c0);
}

// Offset, in lattice units of component a, of a face of component c from
// the node with the same (i,j,k): +1/2 along a, -1/2 along c, 0 otherwise.
__device__ inline float cross_offset(int axis, int c, int a) {
  if (axis == a) return 0.5f;
  if (axis == c) return -0.5f;
  return 0.f;
}

// ------------------------------------------------------------- advection

// Semi-Lagrangian advection plus body force (Section 3.4.1; Section 3.2.2).
// Every active face samples the velocity at its own position, steps back by
// dt along it and takes the trilinear sample of its own component there;
// force[c] = dt * g_c is then added.  Non-active faces get zero.
__global__ void __launch_bounds__(kBlock)
    k_advect(int n, const uint8_t* __restrict__ fcode, CF3 in, F3 out, float dth, float f0,
             float f1, float f2, int64_t F) {
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  const Dims d0 = face_dims(n, 0), d1 = face_dims(n, 1), d2 = face_dims(n, 2);
  const float force = comp == 0 ? f0 : (comp == 1 ? f1 : f2);
  const float* __restrict__ src = in.c[comp];
  float* __restrict__ dst = out.c[comp];
  const uint8_t* __restrict__ code = fcode + comp * F;
  const Chunk ch = block_chunk(F, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  Walker w;
  w.init(d, ch.begin + threadIdx.x, kBlock);
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock, w.next()) {
    if (!(code[idx] & FC_ACTIVE)) {
      dst[idx] = 0.f;
      continue;
    }
    float U[3];
    U[comp] = src[idx];
    if (comp != 0)
      U[0] = sample3(in.c[0], d0, w.i, w.j, w.k, cross_offset(0, comp, 0), cross_offset(1, comp, 0),
                     cross_offset(2, comp, 0));
    if (comp != 1)
      U[1] = sample3(in.c[1], d1, w.i, w.j, w.k, cross_offset(0, comp, 1), cross_offset(1, comp, 1),
                     cross_offset(2, comp, 1));
    if (comp != 2)
      U[2] = sample3(in.c[2], d2, w.i, w.j, w.k, cross_offset(0, comp, 2), cross_offset(1, comp, 2),
                     cross_offset(2, comp, 2));
    float val = sample3(src, d, w.i, w.j, w.k, -dth * U[0], -dth * U[1], -dth * U[2]);
    dst[idx] = val + force;
  }
}

void launch_advect(sim_ctx* c, CF3 in, F3 out, float dth, const float force[3]) {
  prof_mark(c, SIM_KERN_ADVECT, true);
  hipLaunchKernelGGL(k_advect, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->n, c->fcode,
                     in, out, dth, force[0], force[1], force[2], c->F);
  prof_mark(c, SIM_KERN_ADVECT, false);
}

// --------------------------------------------------------------- viscosity

// Componentwise 7-point Laplacian on active faces (face codes select the
// neighbours that enter: active faces, and walls along the face's own axis
// whose stored value is zero).  out = in + alpha * sum (in_nbr - in), with
// alpha = nu * dt / h^2.
__device__ inline float lap_sum(const float* __restrict__ f, int64_t idx, uint8_t code, int64_t sy,
                                int64_t sz) {
  const float v = f[idx];
  float acc = 0.f;
  if (code & 1) acc += f[idx - 1] - v;
  if (code & 2) acc += f[idx + 1] - v;
  if (code & 4) acc += f[idx - sy] - v;
  if (code & 8) acc += f[idx + sy] - v;
  if (code & 16) acc += f[idx - sz] - v;
  if (code & 32) acc += f[idx + sz] - v;
  return acc;
}

__global__ void __launch_bounds__(kBlock)
    k_diffuse_explicit(int n, const uint8_t* __restrict__ fcode, CF3 in, F3 out, float alpha,
                       int64_t F) {
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  const int64_t sy = d.nx, sz = (int64_t)d.nx * d.ny;
  const float* __restrict__ src = in.c[comp];
  float* __restrict__ dst = out.c[comp];
  const uint8_t* __restrict__ code = fcode + comp * F;
  const Chunk ch = block_chunk(F, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    const uint8_t cd = code[idx];
    dst[idx] = (cd & FC_ACTIVE) ? src[idx] + alpha * lap_sum(src, idx, cd, sy, sz) : 0.f;
  }
}

void launch_diffuse_explicit(sim_ctx* c, CF3 in, F3 out, float alpha) {
  prof_mark(c, SIM_KERN_DIFFUSE_EXPLICIT, true);
  hipLaunchKernelGGL(k_diffuse_explicit, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->n,
                     c->fcode, in, out, alpha, c->F);
  prof_mark(c, SIM_KERN_DIFFUSE_EXPLICIT, false);
}

// --------------------------------------------------- Poisson right-hand side

// b_c = -h * (net outward flux of liquid cell c); zero off liquid.
__global__ void __launch_bounds__(kBlock)
    k_divergence(int n, const uint8_t* __restrict__ cdiag, const uint8_t* __restrict__ fcode,
                 int64_t F, CF3 in, float* __restrict__ b) {
  const int64_t C = cells(n);
  // non-active faces (solid walls, air-air) count as zero, whatever they hold
  auto face = [&](int comp, int64_t i) -> float {
    return (fcode[comp * F + i] & FC_ACTIVE) ? in.c[comp][i] : 0.f;
  };
  const float h = 1.0f / (float)n;
  const Chunk ch = block_chunk(C, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  Walker w;
  w.init(Dims{n, n, n}, ch.begin + threadIdx.x, kBlock);
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock, w.next()) {
    float out = 0.f;
    if (cdiag[idx]) {
      const int64_t iu = w.i + (int64_t)(n + 1) * (w.j + (int64_t)n * w.k);
      const int64_t iv = w.i + (int64_t)n * (w.j + (int64_t)(n + 1) * w.k);
      const int64_t iw = idx;
      float flux = (face(0, iu + 1) - face(0, iu)) + (face(1, iv + n) - face(1, iv)) +
                   (face(2, iw + (int64_t)n * n) - face(2, iw));
      out = -h * flux;
    }
    b[idx] = out;
  }
}

void launch_divergence(sim_ctx* c, CF3 in, float* b) {
  hipLaunchKernelGGL(k_divergence, dim3(c->grid_cells), dim3(kBlock), 0, c->stream, c->n, c->cdiag,
                     c->fcode, c->F, in, b);
}

// -------------------------------------------------- pressure-gradient update

// u_f -= (p_plus - p_minus) / h on active faces (p is zero off liquid, so
// air neighbours read zero); every other face is set to zero.  The
// difference is taken in FP64 from the FP64 pressure iterate.
__global__ void __launch_bounds__(kBlock)
    k_pressure_update(int n, const uint8_t* __restrict__ fcode, const double* __restrict__ x, F3 u,
                      int64_t F) {
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  float* __restrict__ f = u.c[comp];
  const uint8_t* __restrict__ code = fcode + comp * F;
  const int64_t cstep = comp == 0 ? 1 : (comp == 1 ? (int64_t)n : (int64_t)n * n);
  const Chunk ch = block_chunk(F, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  Walker w;
  w.init(d, ch.begin + threadIdx.x, kBlock);
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock, w.next()) {
    if (!(code[idx] & FC_ACTIVE)) {
      f[idx] = 0.f;
      continue;
    }
    const int64_t plus = w.i + (int64_t)n * (w.j + (int64_t)n * w.k);
    const double grad = (x[plus] - x[plus - cstep]) * (double)n;
    f[idx] = (float)((double)f[idx] - grad);
  }
}

void launch_pressure_update(sim_ctx* c, const double* x, F3 u) {
  hipLaunchKernelGGL(k_pressure_update, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->n,
                     c->fcode, x, u, c->F);
}

// ----------------------------------------------------------- face utilities

__global__ void __launch_bounds__(kBlock)
    k_mask_scale(const uint8_t* __restrict__ fcode, CF3 in, F3 out, float s, int64_t F) {
  const int comp = blockIdx.y;
  const uint8_t* __restrict__ code = fcode + comp * F;
  const Chunk ch = block_chunk(F, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock)
    out.c[comp][idx] = (code[idx] & FC_ACTIVE) ? s * in.c[comp][idx] : 0.f;
}

void launch_mask_scale(sim_ctx* c, CF3 in, F3 out, float s) {
  hipLaunchKernelGGL(k_mask_scale, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->fcode,
                     in, out, s, c->F);
}

__global__ void __launch_bounds__(kBlock) k_copy_faces(CF3 in, F3 out, int64_t F) {
  const int comp = blockIdx.y;
  const Chunk ch = block_chunk(F, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock)
    out.c[comp][idx] = in.c[comp][idx];
}

void launch_copy_faces(sim_ctx* c, CF3 in, F3 out) {
  hipLaunchKernelGGL(k_copy_faces, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, in, out,
                     c->F);
}

__global__ void __launch_bounds__(kBlock) k_zero_faces(F3 out, int64_t F) {
  const int comp = blockIdx.y;
  const Chunk ch = block_chunk(F, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) out.c[comp][idx] = 0.f;
}

void launch_zero_faces(sim_ctx* c, F3 out) {
  hipLaunchKernelGGL(k_zero_faces, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, out, c->F);
}

__global__ void __launch_bounds__(kBlock) k_axpy_faces(CF3 a, F3 y, float alpha, int64_t F) {
  const int comp = blockIdx.y;
  const Chunk ch = block_chunk(F, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock)
    y.c[comp][idx] += alpha * a.c[comp][idx];
}

void launch_axpy_faces(sim_ctx* c, CF3 a, F3 y, float alpha) {
  hipLaunchKernelGGL(k_axpy_faces, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, a, y, alpha,
                     c->F);
}

// ------------------------------------------------------- face reductions

// scal[slot] = sum over faces of a*b (active faces only when masked).
__global__ void __launch_bounds__(kBlock)
    k_dot_faces(const uint8_t* __restrict__ fcode, CF3 a, CF3 b, int masked, int64_t F,
                double* partials) {
  const int comp = blockIdx.y;
  const uint8_t* __restrict__ code = fcode + comp * F;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk ch = block_chunk(F, gridDim.x, lb);
  double v[1] = {0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock)
    if (!masked || (code[idx] & FC_ACTIVE)) v[0] += (double)a.c[comp][idx] * (double)b.c[comp][idx];
  store_partials<1>(v, partials, comp * gridDim.x + lb);
}

void launch_dot_faces(sim_ctx* c, CF3 a, CF3 b, int slot, int masked) {
  hipLaunchKernelGGL(k_dot_faces, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->fcode, a,
                     b, masked, c->F, c->partials);
  launch_finalize(c, 3 * c->grid_faces, 1, FIN_SLOT, 0.0, 0, slot, 1.0, 0);
}

// scal[slot] = (accumulate ? scal[slot] : 0) + scale * <a, L y>, with L the
// viscous Laplacian including 1/h^2.
__global__ void __launch_bounds__(kBlock)
    k_dot_lap(int n, const uint8_t* __restrict__ fcode, CF3 a, CF3 y, int64_t F, double* partials) {
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  const int64_t sy = d.nx, sz = (int64_t)d.nx * d.ny;
  const uint8_t* __restrict__ code = fcode + comp * F;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk ch = block_chunk(F, gridDim.x, lb);
  const double inv_h2 = (double)n * (double)n;
  double v[1] = {0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    const uint8_t cd = code[idx];
    if (cd & FC_ACTIVE) v[0] += (double)a.c[comp][idx] * (double)lap_sum(y.c[comp], idx, cd, sy, sz);
  }
  v[0] *= inv_h2;
  store_partials<1>(v, partials, comp * gridDim.x + lb);
}

void launch_dot_lap(sim_ctx* c, CF3 a, CF3 y, int slot, double scale, int accumulate) {
  hipLaunchKernelGGL(k_dot_lap, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->n, c->fcode,
                     a, y, c->F, c->partials);
  launch_finalize(c, 3 * c->grid_faces, 1, FIN_SLOT, 0.0, 0, slot, scale, accumulate);
}

// MSE over active faces: scal[slot] = sum (u - t)^2 (the caller divides by
// the active-face count); g (nullable components) = 2 (u - t) / count.
__global__ void __launch_bounds__(kBlock)
    k_loss_mse(const uint8_t* __restrict__ fcode, CF3 u, CF3 t, F3 g, float inv_count, int64_t F,
               double* partials) {
  const int comp = blockIdx.y;
  const uint8_t* __restrict__ code = fcode + comp * F;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk ch = block_chunk(F, gridDim.x, lb);
  float* __restrict__ gc = g.c[comp];
  double v[1] = {0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    float diff = 0.f;
    if (code[idx] & FC_ACTIVE) diff = u.c[comp][idx] - t.c[comp][idx];
    v[0] += (double)diff * (double)diff;
    if (gc) gc[idx] = 2.f * diff * inv_count;
  }
  store_partials<1>(v, partials, comp * gridDim.x + lb);
}

void launch_loss_mse(sim_ctx* c, CF3 u, CF3 t, F3 g, int slot) {
  float inv = c->n_active > 0 ? 1.0f / (float)c->n_active : 0.f;
  hipLaunchKernelGGL(k_loss_mse, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->fcode, u, t,
                     g, inv, c->F, c->partials);
  launch_finalize(c, 3 * c->grid_faces, 1, FIN_SLOT, 0.0, 0, slot, 1.0, 0);
}

// ------------------------------------------------------- advection adjoint

// Adds (d advect / d u)^T lam to g.  The sampled value depends on the field
// through the trilinear weights at the departure point, and on the
// departure point through the face velocity, itself a trilinear sample of
// the three components at the face.  Both parts are scattered with FP32
// atomics.  The body force is a constant and drops out.
//
// Consecutive lanes hold consecutive faces of a row, and their 2x2x2
// targets usually sit side by side along x: when the next lane's base node
// is this lane's base node + 1 in x (same y and z), this lane's +x column of
// four targets is the next lane's own column, so the next lane adds the four
// values into its atomics and this lane issues none for that column.  Both
// lanes test the same shuffled integers, so they agree; a lane with nothing
// to scatter passes an impossible base (on = false).  Every lane of the wave
// must call this together.
__device__ inline void scatter3_merged(float* __restrict__ g, Dims d, int i, int j, int k,
                                       float rx, float ry, float rz, float s, bool on) {
  int i0, j0, k0;
  float fx, fy, fz;
  lattice_axis(i, rx, d.nx, i0, fx);
  lattice_axis(j, ry, d.ny, j0, fy);
  lattice_axis(k, rz, d.nz, k0, fz);
  const int key_i = on ? i0 : -1000;
  const int key_jk = j0 | (k0 << 16);
  const float wx[2] = {1.f - fx, fx}, wy[2] = {1.f - fy, fy}, wz[2] = {1.f - fz, fz};
  float v[2][2][2];  // [z][y][x]
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) v[c][b][a] = on ? s * wx[a] * wy[b] * wz[c] : 0.f;
  const int lane = threadIdx.x & 63;
  const int prev_i = __shfl_up(key_i, 1);
  const int prev_jk = __shfl_up(key_jk, 1);
  const int next_i = __shfl_down(key_i, 1);
  const int next_jk = __shfl_down(key_jk, 1);
  float pv[2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b) pv[c][b] = __shfl_up(v[c][b][1], 1);
  const bool take = lane > 0 && on && prev_i + 1 == key_i && prev_jk == key_jk;
  const bool give = lane < 63 && on && key_i + 1 == next_i && key_jk == next_jk;
  if (!on) return;
  const int64_t sy = d.nx, sz = (int64_t)d.nx * d.ny;
  float* p = g + i0 + sy * j0 + sz * k0;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const float w0 = take ? v[c][b][0] + pv[c][b] : v[c][b][0];
      if (w0 != 0.f) atomicAdd(p + sy * b + sz * c, w0);
      if (!give && v[c][b][1] != 0.f) atomicAdd(p + 1 + sy * b + sz * c, v[c][b][1]);
    }
}

// Gradient of the trilinear sample with respect to the position (lattice
// units); zero along axes where the position was clamped.
__device__ inline void sample3_grad(const float* __restrict__ f, Dims d, int i, int j, int k,
                                    float rx, float ry, float rz, float g[3]) {
  int i0, j0, k0;
  float fx, fy, fz;
  lattice_axis(i, rx, d.nx, i0, fx);
  lattice_axis(j, ry, d.ny, j0, fy);
  lattice_axis(k, rz, d.nz, k0, fz);
  // clamped axes: the unclamped position lies outside [0, cnt-1]
  const float tx = (float)i + rx, ty = (float)j + ry, tz = (float)k + rz;
  const bool cx = tx < 0.f || tx > (float)(d.nx - 1);
  const bool cy = ty < 0.f || ty > (float)(d.ny - 1);
  const bool cz = tz < 0.f || tz > (float)(d.nz - 1);
  const int64_t sy = d.nx, sz = (int64_t)d.nx * d.ny;
  const float* p = f + i0 + sy * j0 + sz * k0;
  float c[2][2][2];
#pragma unroll
  for (int zz = 0; zz < 2; ++zz)
#pragma unroll
    for (int yy = 0; yy < 2; ++yy)
#pragma unroll
      for (int xx = 0; xx < 2; ++xx) c[zz][yy][xx] = p[xx + sy * yy + sz * zz];
  const float wx[2] = {1.f - fx, fx}, wy[2] = {1.f - fy, fy}, wz[2] = {1.f - fz, fz};
  float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
  for (int zz = 0; zz < 2; ++zz)
#pragma unroll
    for (int yy = 0; yy < 2; ++yy) gx += wy[yy] * wz[zz] * (c[zz][yy][1] - c[zz][yy][0]);
#pragma unroll
  for (int zz = 0; zz < 2; ++zz)
#pragma unroll
    for (int xx = 0; xx < 2; ++xx) gy += wx[xx] * wz[zz] * (c[zz][1][xx] - c[zz][0][xx]);
#pragma unroll
  for (int yy = 0; yy < 2; ++yy)
#pragma unroll
    for (int xx = 0; xx < 2; ++xx) gz += wx[xx] * wy[yy] * (c[1][yy][xx] - c[0][yy][xx]);
  g[0] = cx ? 0.f : gx;
  g[1] = cy ? 0.f : gy;
  g[2] = cz ? 0.f : gz;
}

// One thread per face.  With SCATTER the transpose above is scattered into
// g; in both forms the thread adds, in FP64, lam times the derivative of its
// advected value with respect to dt (the departure point moves by -U per
// unit dt: -n grad I . U in lattice units) and lam itself (the body force
// dt * g_c is added to every active face), for the block partials
// [dt term, lam sum of component 0, 1, 2].
template <bool SCATTER>
__global__ void __launch_bounds__(kBlock)
    k_advect_adjoint(int n, const uint8_t* __restrict__ fcode, CF3 u, CF3 lam, F3 g, float dth,
                     int64_t F, double* partials) {
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  const Dims dd[3] = {face_dims(n, 0), face_dims(n, 1), face_dims(n, 2)};
  const uint8_t* __restrict__ code = fcode + comp * F;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk ch = block_chunk(F, gridDim.x, lb);
  const float fn = (float)n;
  double acc_dt = 0.0, acc_l = 0.0;
  Walker w;
  w.init(d, ch.begin + threadIdx.x, kBlock);
  // the trip count is the same for the whole wave (lanes past the chunk's
  // end take part with nothing to scatter), so the merged scatters' shuffles
  // see every lane
  const int lane = threadIdx.x & 63;
  for (int64_t base = ch.begin + threadIdx.x - lane; base < ch.end; base += kBlock, w.next()) {
    const int64_t idx = base + lane;
    bool on = idx < ch.end && (code[idx] & FC_ACTIVE);
    const float l = on ? lam.c[comp][idx] : 0.f;
    on = on && l != 0.f;
    float U[3] = {0.f, 0.f, 0.f};
    float off[3][3];
    float grad[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) off[a][ax] = a == comp ? 0.f : cross_offset(ax, comp, a);
    if (on) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
        U[a] = a == comp ? u.c[comp][idx]
                         : sample3(u.c[a], dd[a], w.i, w.j, w.k, off[a][0], off[a][1], off[a][2]);
    }
    const float rx = -dth * U[0], ry = -dth * U[1], rz = -dth * U[2];
    if (on) {
      sample3_grad(u.c[comp], d, w.i, w.j, w.k, rx, ry, rz, grad);
      acc_l += (double)l;
      acc_dt -= (double)l * (double)(fn * (grad[0] * U[0] + grad[1] * U[1] + grad[2] * U[2]));
    }
    if (SCATTER) {
      scatter3_merged(g.c[comp], d, w.i, w.j, w.k, rx, ry, rz, l, on);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float s = l * (-dth) * grad[a];
        if (a == comp) {
          // zero offset: the face itself
          if (on && s != 0.f) atomicAdd(g.c[comp] + idx, s);
        } else {
          scatter3_merged(g.c[a], dd[a], w.i, w.j, w.k, off[a][0], off[a][1], off[a][2], s,
                          on && s != 0.f);
        }
      }
    }
  }
  double v[4] = {acc_dt, comp == 0 ? acc_l : 0.0, comp == 1 ? acc_l : 0.0, comp == 2 ? acc_l : 0.0};
  store_partials<4>(v, partials, comp * gridDim.x + lb);
}

void launch_advect_adjoint(sim_ctx* c, CF3 u, CF3 lam, F3 g, float dth, bool scatter,
                           int accumulate) {
  prof_mark(c, SIM_KERN_ADVECT_ADJOINT, true);
  if (scatter)
    hipLaunchKernelGGL(k_advect_adjoint<true>, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream,
                       c->n, c->fcode, u, lam, g, dth, c->F, c->partials);
  else
    hipLaunchKernelGGL(k_advect_adjoint<false>, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream,
                       c->n, c->fcode, u, lam, g, dth, c->F, c->partials);
  prof_mark(c, SIM_KERN_ADVECT_ADJOINT, false);
  launch_finalize(c, 3 * c->grid_faces, 4, FIN_SLOTS4, 0.0, 0, S_ADV_DT, 1.0, accumulate);
}

}  // namespace fs
