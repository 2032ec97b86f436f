// The paper's upwind analytic convection gradient (Section 3.4.1), the
// surrogate it uses in place of differentiating the semi-Lagrangian
// back-trace: for the convected field v and lam = dJ/dv,
//
//   dJ/dv'_i (f) = [f active] ( lam_i(f) - dt sum_c Lam_c(f) D_i V_c(f) )
//
// on every face f of component i.  V_c, Lam_c: v_c, lam_c at the position of
// f (the value itself for c = i, else the mean of the four c-faces around
// it, zero outside the box).  D_i: the first-order upwind difference along
// axis i against the sign of v_i(f), divided by h.  One thread per face;
// the gathers hit the cache lines of the neighbouring faces (this is an
// operator of the backward pass, not of the hot loop).
#include "common.h"
#include "ctx.h"

namespace fs {

struct UpFaces {
  const float* a[3];
};

// face (x, y, z) of component C (zero outside its array); a component holds
// fewer than 2^31 faces for n <= 1024, so 32-bit indexes suffice
template <int C>
__device__ inline float up_face(const UpFaces& f, int n, int x, int y, int z) {
  const int nx = n + (C == 0), ny = n + (C == 1), nz = n + (C == 2);
  if ((unsigned)x >= (unsigned)nx || (unsigned)y >= (unsigned)ny || (unsigned)z >= (unsigned)nz)
    return 0.f;
  return f.a[C][x + nx * (y + ny * z)];
}

// component C at the position of the I-face (x, y, z)
template <int C, int I>
__device__ inline float up_at(const UpFaces& f, int n, int x, int y, int z) {
  if constexpr (C == I) {
    return up_face<C>(f, n, x, y, z);
  } else {
    const int nx = n + (I == 0), ny = n + (I == 1), nz = n + (I == 2);
    if ((unsigned)x >= (unsigned)nx || (unsigned)y >= (unsigned)ny || (unsigned)z >= (unsigned)nz)
      return 0.f;
    float s = 0.f;
#pragma unroll
    for (int da = -1; da <= 0; ++da)
#pragma unroll
      for (int dc = 0; dc <= 1; ++dc) {
        int q[3] = {x, y, z};
        q[I] += da;  // the cells on either side along the face's axis
        q[C] += dc;  // the two C-faces of the cell along axis C
        if ((unsigned)q[I] >= (unsigned)n) continue;
        s += up_face<C>(f, n, q[0], q[1], q[2]);
      }
    return 0.25f * s;
  }
}

// sum_c Lam_c(f) D_I V_c(f) for the I-face (x, y, z), nb its upwind neighbour
template <int C, int I>
__device__ inline float up_term(const UpFaces& v, const UpFaces& lam, int n, int x, int y, int z,
                                const int (&nb)[3], float v0, float sgn) {
  const float vc = C == I ? v0 : up_at<C, I>(v, n, x, y, z);
  const float d = sgn * (vc - up_at<C, I>(v, n, nb[0], nb[1], nb[2]));
  return up_at<C, I>(lam, n, x, y, z) * d;
}

template <int I>
__device__ inline void upwind_faces(int n, const uint8_t* __restrict__ code, const UpFaces& v,
                                    const UpFaces& lam, float dt_over_h, float* __restrict__ g) {
  const unsigned nx = n + (I == 0), ny = n + (I == 1);
  const unsigned count = nx * ny * (unsigned)(n + (I == 2));
  for (unsigned idx = blockIdx.x * kBlock + threadIdx.x; idx < count; idx += gridDim.x * kBlock) {
    if (!(code[idx] & FC_ACTIVE)) {
      g[idx] = 0.f;
      continue;
    }
    const unsigned row = idx / nx, zu = row / ny;
    const int x = (int)(idx - row * nx), y = (int)(row - zu * ny), z = (int)zu;
    const float v0 = v.a[I][idx];
    // the upwind neighbour: one face back along axis I when v_I > 0, else one
    // forward; D_I V_c = sgn (V_c(f) - V_c(neighbour)) / h
    const float sgn = v0 > 0.f ? 1.f : -1.f;
    int nb[3] = {x, y, z};
    nb[I] -= v0 > 0.f ? 1 : -1;
    const float acc = up_term<0, I>(v, lam, n, x, y, z, nb, v0, sgn) +
                      up_term<1, I>(v, lam, n, x, y, z, nb, v0, sgn) +
                      up_term<2, I>(v, lam, n, x, y, z, nb, v0, sgn);
    g[idx] = lam.a[I][idx] - dt_over_h * acc;
  }
}

// grid (blocks, 3): blockIdx.y is the face component, uniform per block
__global__ void __launch_bounds__(kBlock)
    k_convection_grad_upwind(int n, int64_t F, const uint8_t* __restrict__ fcode, UpFaces v,
                             UpFaces lam, float dt_over_h, float* __restrict__ g0,
                             float* __restrict__ g1, float* __restrict__ g2) {
  if (blockIdx.y == 0)
    upwind_faces<0>(n, fcode, v, lam, dt_over_h, g0);
  else if (blockIdx.y == 1)
    upwind_faces<1>(n, fcode + F, v, lam, dt_over_h, g1);
  else
    upwind_faces<2>(n, fcode + 2 * F, v, lam, dt_over_h, g2);
}

void launch_convection_grad_upwind(sim_ctx* c, CF3 v, CF3 lam, F3 g) {
  UpFaces fv{{v.c[0], v.c[1], v.c[2]}}, fl{{lam.c[0], lam.c[1], lam.c[2]}};
  hipLaunchKernelGGL(k_convection_grad_upwind, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream,
                     c->n, c->F, c->fcode, fv, fl, (float)(c->params.dt * c->n), g.c[0], g.c[1],
                     g.c[2]);
}

}  // namespace fs

using namespace fs;

extern "C" int sim_op_convection_grad_upwind(sim_ctx* c, const float* u, const float* v,
                                             const float* w, const float* lu, const float* lv,
                                             const float* lw, float* g0, float* g1, float* g2) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!u || !v || !w || !lu || !lv || !lw || !g0 || !g1 || !g2 || !c->params_set) {
    c->err = "NULL pointer or params not set";
    return SIM_ERR_INVALID_ARG;
  }
  const float* outs[3] = {g0, g1, g2};
  const float* ins[6] = {u, v, w, lu, lv, lw};
  for (const float* o : outs)
    for (const float* p : ins)
      if (o == p) {
        c->err = "sim_op_convection_grad_upwind: an output aliases an input";
        return SIM_ERR_INVALID_ARG;
      }
  launch_convection_grad_upwind(c, CF3{{u, v, w}}, CF3{{lu, lv, lw}}, F3{{g0, g1, g2}});
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_ERR_HIP;
}
