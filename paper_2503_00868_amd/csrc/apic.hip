// The paper's affine particle-in-cell transfers (Section 3.2.2,
// Eq. (particle_map) and the transfer back) on the MAC grid: each velocity
// component on its own lattice (the centres of its faces), quadratic
// B-spline weights, row a of C_p the affine part of component a, nodes
// outside a lattice skipped.
//
// Particles to grid: per component, each particle's weighted mass and
// weighted momentum (v_pa + C_p[a] . (x_i - x_p)) go to its 27 nodes; a
// thread sums a run of particles per cell in registers first and adds the
// sums with FP32 global atomics; a face pass divides momentum by mass (0
// where no mass arrived).  Grid to particles: one thread per
// particle gathers the 27 nodes per component, forms v_p and
// C_p[a] = 4/h^2 sum w v_i (x_i - x_p), and moves x_p by dt v_p.
//
// Particles are arrays of structures: x (P x 3, x y z), v (P x 3),
// C (P x 9, row-major by component), m (P).
#include <cmath>

#include "common.h"
#include "ctx.h"

namespace fs {

// quadratic B-spline weights of the three nodes from `base` along one axis;
// X in lattice units.  The base is clamped so any input, NaN included, gives
// a defined integer; nodes outside a lattice are skipped by the callers.
__device__ inline void ap_axis(float X, int& base, float w[3], float r[3]) {
  const float fb = fminf(fmaxf(floorf(X - 0.5f), -4.f), 4100.f);
  base = (int)fb;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const float t = X - (fb + (float)q);  // x_p - x_i in cells
    const float a = fabsf(t);
    w[q] = a < 0.5f ? 0.75f - a * a : (a < 1.5f ? 0.5f * (1.5f - a) * (1.5f - a) : 0.f);
    r[q] = -t;  // x_i - x_p in cells
  }
}

struct ApStencil {
  int b[3];
  float w[3][3], r[3][3];  // [axis][node]
};

// the stencil of component A's lattice around position (x, y, z) (unit box)
template <int A>
__device__ inline ApStencil ap_stencil(int n, float x, float y, float z) {
  const float fn = (float)n;
  ApStencil s;
  ap_axis(x * fn - (A == 0 ? 0.f : 0.5f), s.b[0], s.w[0], s.r[0]);
  ap_axis(y * fn - (A == 1 ? 0.f : 0.5f), s.b[1], s.w[1], s.r[1]);
  ap_axis(z * fn - (A == 2 ? 0.f : 0.5f), s.b[2], s.w[2], s.r[2]);
  return s;
}

// Particles to grid, one thread per run of kApRun consecutive particles.
// For each component the thread accumulates its particles' weighted mass and
// momentum in registers over the node window of the current particle's
// cell, and adds the window to the grid with FP32 atomics only when the cell
// changes (and at the end of the run).  With particles ordered by cell (the
// usual layout) a run of eight particles of one cell issues 72 atomics per
// component instead of 8 x 54, and neighbouring lanes, which hold
// neighbouring cells, share few nodes.  Any order gives the same sums.
//
// Window of component A around cell (ci, cj, ck): along A's own axis nodes
// c-1 .. c+2 (the base floor(X - 1/2) of a particle in the cell is c-1 or c),
// along the other two axes nodes c-1 .. c+1 (the lattice is offset by half
// a cell there, so the base is always c-1): 4 x 3 x 3 = 36 nodes.
constexpr int kApRun = 8;

template <int A>
struct ApWin {
  static constexpr int EX = A == 0 ? 4 : 3, EY = A == 1 ? 4 : 3, EZ = A == 2 ? 4 : 3;
  float m[36], p[36];
  int ci, cj, ck;
};

// per axis: weights and offsets (in cells) of the window's nodes for one
// particle at lattice coordinate X whose cell starts at node lo (the window's
// first node); own: the axis has 4 window nodes (the base is lo or lo + 1)
__device__ inline void ap_axis_win(float X, int lo, bool own, float w[4], float r[4]) {
  const int base = (int)floorf(X - 0.5f);
  const int sh = base - lo;  // 0, or 1 along the own axis
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float t = X - (float)(lo + q);  // x_p - x_i in cells
    const float a = fabsf(t);
    float wq = a < 0.5f ? 0.75f - a * a : (a < 1.5f ? 0.5f * (1.5f - a) * (1.5f - a) : 0.f);
    // only the three nodes from the particle's base take part
    const bool in = q >= sh && q < sh + 3 && (own || q < 3);
    w[q] = in ? wq : 0.f;
    r[q] = -t;
  }
}

template <int A>
__device__ inline void ap_flush(int n, ApWin<A>& W, float* __restrict__ mom, float* __restrict__ mass) {
  const int nx = n + (A == 0), ny = n + (A == 1), nz = n + (A == 2);
#pragma unroll
  for (int c = 0; c < ApWin<A>::EZ; ++c) {
    const int iz = W.ck - 1 + c;
#pragma unroll
    for (int b = 0; b < ApWin<A>::EY; ++b) {
      const int iy = W.cj - 1 + b;
#pragma unroll
      for (int a = 0; a < ApWin<A>::EX; ++a) {
        const int ix = W.ci - 1 + a;
        const int q = a + ApWin<A>::EX * (b + ApWin<A>::EY * c);
        const float wm = W.m[q];
        if (wm != 0.f && (unsigned)ix < (unsigned)nx && (unsigned)iy < (unsigned)ny &&
            (unsigned)iz < (unsigned)nz) {
          const int64_t idx = ix + (int64_t)nx * (iy + (int64_t)ny * iz);
          atomicAdd(mom + idx, W.p[q]);
          atomicAdd(mass + idx, wm);
        }
        W.m[q] = 0.f;
        W.p[q] = 0.f;
      }
    }
  }
}

template <int A>
__device__ inline void ap_run(int n, int64_t p0, int64_t p1, const float* __restrict__ xp,
                              const float* __restrict__ vp, const float* __restrict__ Cp,
                              const float* __restrict__ mp, float* __restrict__ mom,
                              float* __restrict__ mass) {
  const float fn = (float)n, h = 1.f / fn;
  ApWin<A> W;
#pragma unroll
  for (int q = 0; q < 36; ++q) W.m[q] = W.p[q] = 0.f;
  W.ci = W.cj = W.ck = INT32_MIN;
  for (int64_t p = p0; p < p1; ++p) {
    // positions in cells, clamped so that any input (NaN included) gives a
    // bounded cell; nodes outside the lattice are skipped by the flush
    float P[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) P[d] = fminf(fmaxf(xp[3 * p + d] * fn, -4.f), fn + 4.f);
    const int ci = (int)floorf(P[0]), cj = (int)floorf(P[1]), ck = (int)floorf(P[2]);
    if (ci != W.ci || cj != W.cj || ck != W.ck) {
      if (W.ci != INT32_MIN) ap_flush<A>(n, W, mom, mass);
      W.ci = ci;
      W.cj = cj;
      W.ck = ck;
    }
    float wx[4], rx[4], wy[4], ry[4], wz[4], rz[4];
    ap_axis_win(P[0] - (A == 0 ? 0.f : 0.5f), ci - 1, A == 0, wx, rx);
    ap_axis_win(P[1] - (A == 1 ? 0.f : 0.5f), cj - 1, A == 1, wy, ry);
    ap_axis_win(P[2] - (A == 2 ? 0.f : 0.5f), ck - 1, A == 2, wz, rz);
    const float m = mp[p], va = vp[3 * p + A];
    const float c0 = Cp[9 * p + 3 * A] * h, c1 = Cp[9 * p + 3 * A + 1] * h, c2 = Cp[9 * p + 3 * A + 2] * h;
#pragma unroll
    for (int c = 0; c < ApWin<A>::EZ; ++c)
#pragma unroll
      for (int b = 0; b < ApWin<A>::EY; ++b) {
        const float wyz = m * wy[b] * wz[c];
        const float vyz = va + c1 * ry[b] + c2 * rz[c];
#pragma unroll
        for (int a = 0; a < ApWin<A>::EX; ++a) {
          const int q = a + ApWin<A>::EX * (b + ApWin<A>::EY * c);
          const float wm = wyz * wx[a];
          W.m[q] += wm;
          W.p[q] += wm * (vyz + c0 * rx[a]);
        }
      }
  }
  if (W.ci != INT32_MIN) ap_flush<A>(n, W, mom, mass);
}

__global__ void __launch_bounds__(kBlock)
    k_apic_p2g(int n, int64_t P, const float* __restrict__ xp, const float* __restrict__ vp,
               const float* __restrict__ Cp, const float* __restrict__ mp, F3 mom, F3 mass) {
  const int64_t runs = (P + kApRun - 1) / kApRun;
  for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < runs; t += (int64_t)gridDim.x * kBlock) {
    const int64_t p0 = t * kApRun, p1 = p0 + kApRun < P ? p0 + kApRun : P;
    ap_run<0>(n, p0, p1, xp, vp, Cp, mp, mom.c[0], mass.c[0]);
    ap_run<1>(n, p0, p1, xp, vp, Cp, mp, mom.c[1], mass.c[1]);
    ap_run<2>(n, p0, p1, xp, vp, Cp, mp, mom.c[2], mass.c[2]);
  }
}

// fills both accumulators of every face with 0 (a kernel, so that the call
// can sit in a captured graph)
__global__ void __launch_bounds__(kBlock) k_apic_zero(int64_t F, F3 a, F3 b) {
  const int comp = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < F; i += (int64_t)gridDim.x * kBlock) {
    a.c[comp][i] = 0.f;
    b.c[comp][i] = 0.f;
  }
}

// v = momentum / mass where mass > 0, else 0 (in place over the momentum)
__global__ void __launch_bounds__(kBlock) k_apic_normalize(int64_t F, F3 mom, CF3 mass) {
  const int comp = blockIdx.y;
  float* __restrict__ v = mom.c[comp];
  const float* __restrict__ m = mass.c[comp];
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < F; i += (int64_t)gridDim.x * kBlock) {
    const float mi = m[i];
    v[i] = mi > 0.f ? v[i] / mi : 0.f;
  }
}

template <int A>
__device__ inline void ap_gather(int n, const float* __restrict__ g, float x, float y, float z, float& v,
                                 float c[3]) {
  const int nx = n + (A == 0), ny = n + (A == 1), nz = n + (A == 2);
  const ApStencil s = ap_stencil<A>(n, x, y, z);
  float sv = 0.f, s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int iz = s.b[2] + k;
    if ((unsigned)iz >= (unsigned)nz) continue;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int iy = s.b[1] + j;
      if ((unsigned)iy >= (unsigned)ny) continue;
      const float wyz = s.w[1][j] * s.w[2][k];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int ix = s.b[0] + i;
        if ((unsigned)ix >= (unsigned)nx) continue;
        const float wv = wyz * s.w[0][i] * g[ix + (int64_t)nx * (iy + (int64_t)ny * iz)];
        sv += wv;
        s0 += wv * s.r[0][i];
        s1 += wv * s.r[1][j];
        s2 += wv * s.r[2][k];
      }
    }
  }
  // 4 / h^2 times sum w v (x_i - x_p), with x_i - x_p = r h
  const float f = 4.f * (float)n;
  v = sv;
  c[0] = f * s0;
  c[1] = f * s1;
  c[2] = f * s2;
}

__global__ void __launch_bounds__(kBlock)
    k_apic_g2p(int n, int64_t P, CF3 grid, float dt, float* __restrict__ xp, float* __restrict__ vp,
               float* __restrict__ Cp) {
  for (int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x; p < P; p += (int64_t)gridDim.x * kBlock) {
    const float x = xp[3 * p], y = xp[3 * p + 1], z = xp[3 * p + 2];
    float v[3], c[3][3];
    ap_gather<0>(n, grid.c[0], x, y, z, v[0], c[0]);
    ap_gather<1>(n, grid.c[1], x, y, z, v[1], c[1]);
    ap_gather<2>(n, grid.c[2], x, y, z, v[2], c[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      vp[3 * p + a] = v[a];
#pragma unroll
      for (int j = 0; j < 3; ++j) Cp[9 * p + 3 * a + j] = c[a][j];
    }
    xp[3 * p] = x + dt * v[0];
    xp[3 * p + 1] = y + dt * v[1];
    xp[3 * p + 2] = z + dt * v[2];
  }
}

int ap_blocks(int64_t P) {
  const int64_t g = (P + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g > 8 * kMaxGrid ? 8 * kMaxGrid : g));
}

}  // namespace fs

using namespace fs;

extern "C" int sim_apic_p2g(sim_ctx* c, int64_t P, const float* xp, const float* vp, const float* Cp,
                            const float* mp, float* u, float* v, float* w, float* mu, float* mv, float* mw) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (P < 0 || P > INT32_MAX || (P > 0 && (!xp || !vp || !Cp || !mp)) || !u || !v || !w || !mu || !mv ||
      !mw) {
    c->err = "sim_apic_p2g: P out of [0, 2^31), or a NULL pointer";
    return SIM_ERR_INVALID_ARG;
  }
  const float* outs[6] = {u, v, w, mu, mv, mw};
  for (int a = 0; a < 6; ++a)
    for (int b = a + 1; b < 6; ++b)
      if (outs[a] == outs[b]) {
        c->err = "sim_apic_p2g: the six grid outputs must be distinct";
        return SIM_ERR_INVALID_ARG;
      }
  const F3 mom{{u, v, w}}, mass{{mu, mv, mw}};
  hipLaunchKernelGGL(k_apic_zero, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->F, mom, mass);
  if (P > 0)
    hipLaunchKernelGGL(k_apic_p2g, dim3(ap_blocks(P)), dim3(kBlock), 0, c->stream, c->n, P, xp, vp, Cp, mp,
                       mom, mass);
  hipLaunchKernelGGL(k_apic_normalize, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->F, mom,
                     CF3{{mu, mv, mw}});
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_ERR_HIP;
}

extern "C" int sim_apic_g2p(sim_ctx* c, int64_t P, const float* u, const float* v, const float* w, double dt,
                            float* xp, float* vp, float* Cp) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (P < 0 || P > INT32_MAX || !u || !v || !w || (P > 0 && (!xp || !vp || !Cp)) || !std::isfinite(dt)) {
    c->err = "sim_apic_g2p: P out of [0, 2^31), a NULL pointer or a non-finite dt";
    return SIM_ERR_INVALID_ARG;
  }
  if (P > 0)
    hipLaunchKernelGGL(k_apic_g2p, dim3(ap_blocks(P)), dim3(kBlock), 0, c->stream, c->n, P,
                       CF3{{u, v, w}}, (float)dt, xp, vp, Cp);
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_ERR_HIP;
}
