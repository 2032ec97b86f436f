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

// face (x, y, z) of component c (zero outside its array)
__device__ inline float up_face(const UpFaces& f, int n, int c, int x, int y, int z) {
  const int nx = n + (c == 0), ny = n + (c == 1), nz = n + (c == 2);
  if ((unsigned)x >= (unsigned)nx || (unsigned)y >= (unsigned)ny || (unsigned)z >= (unsigned)nz)
    return 0.f;
  return f.a[c][x + (int64_t)nx * (y + (int64_t)ny * z)];
}

// component c at the position of the i-face (x, y, z)
__device__ inline float up_at(const UpFaces& f, int n, int c, int i, int x, int y, int z) {
  if (c == i) return up_face(f, n, c, x, y, z);
  const int nx = n + (i == 0), ny = n + (i == 1), nz = n + (i == 2);
  if ((unsigned)x >= (unsigned)nx || (unsigned)y >= (unsigned)ny || (unsigned)z >= (unsigned)nz)
    return 0.f;
  float s = 0.f;
#pragma unroll
  for (int da = -1; da <= 0; ++da)
#pragma unroll
    for (int dc = 0; dc <= 1; ++dc) {
      int q[3] = {x, y, z};
      q[i] += da;  // the cells on either side along the face's axis
      q[c] += dc;  // the two c-faces of the cell along axis c
      if ((unsigned)q[i] >= (unsigned)n) continue;
      s += up_face(f, n, c, q[0], q[1], q[2]);
    }
  return 0.25f * s;
}

__global__ void __launch_bounds__(kBlock)
    k_convection_grad_upwind(int n, int64_t F, const uint8_t* __restrict__ fcode, UpFaces v,
                             UpFaces lam, float dt_over_h, float* __restrict__ g0,
                             float* __restrict__ g1, float* __restrict__ g2) {
  const int i = blockIdx.y;  // face component
  float* g = i == 0 ? g0 : (i == 1 ? g1 : g2);
  const int nx = n + (i == 0), ny = n + (i == 1);
  const int64_t count = (int64_t)nx * ny * (n + (i == 2));
  const uint8_t* code = fcode + i * F;
  for (int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x; idx < count;
       idx += (int64_t)gridDim.x * kBlock) {
    if (!(code[idx] & FC_ACTIVE)) {
      g[idx] = 0.f;
      continue;
    }
    const int x = (int)(idx % nx), y = (int)((idx / nx) % ny), z = (int)(idx / ((int64_t)nx * ny));
    const bool pos = v.a[i][idx] > 0.f;
    int lo[3] = {x, y, z}, hi[3] = {x, y, z};
    lo[i] -= 1;
    hi[i] += 1;
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float v0 = up_at(v, n, c, i, x, y, z);
      const float d = pos ? v0 - up_at(v, n, c, i, lo[0], lo[1], lo[2])
                          : up_at(v, n, c, i, hi[0], hi[1], hi[2]) - v0;
      acc += up_at(lam, n, c, i, x, y, z) * d;
    }
    g[idx] = lam.a[i][idx] - dt_over_h * acc;
  }
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
  UpFaces fv{{u, v, w}}, fl{{lu, lv, lw}};
  hipLaunchKernelGGL(k_convection_grad_upwind, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream,
                     c->n, c->F, c->fcode, fv, fl, (float)(c->params.dt * c->n), g0, g1, g2);
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_ERR_HIP;
}
