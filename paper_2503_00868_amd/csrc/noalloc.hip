// sim_loss_mse_noalloc: the MSE loss over active faces (as sim_loss_mse)
// for callers that cannot allocate device memory (code under HIP graph
// capture, serving loops, harnesses that forbid allocation).  It needs no
// context and no workspace: the face classes come from the cell types on the
// fly, and the block partial sums live in one file-scope device array of a
// fixed size.  Every call on a device shares that device's array, so calls
// that overlap on one device race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "common.h"
#include "ctx.h"

namespace fs {
namespace {

constexpr int kNaBlocks = 1024;                    // blocks per face component, at most
constexpr int kNaPartials = 3 * kNaBlocks * 2;     // [block][sum of squares, active count]
constexpr int kNaResult = kNaPartials;             // then: 1 / active count (as a float value)
constexpr int kNaScratchDoubles = kNaPartials + 32;
constexpr int kNaMaxDevices = 64;

}  // namespace

// The only device memory the entry point uses beyond its arguments
// (kNaScratchDoubles doubles, 49,408 bytes per device).  In host code this
// name is a host-side stand-in: kernels get its device address from
// hipGetSymbolAddress, kept per device below.
static __device__ __align__(256) double scratch[kNaScratchDoubles];

namespace {

__device__ inline uint8_t na_cell(const uint8_t* __restrict__ cell, int n, int i, int j, int k) {
  if ((unsigned)i >= (unsigned)n || (unsigned)j >= (unsigned)n || (unsigned)k >= (unsigned)n)
    return SOLID;
  return cell[i + (int64_t)n * (j + (int64_t)n * k)];
}

// a face is active when no solid cell (or the outside of the box) touches
// it and a liquid cell does
__device__ inline bool na_active(const uint8_t* __restrict__ cell, int n, int comp, int i, int j,
                                 int k) {
  const uint8_t a = na_cell(cell, n, i - (comp == 0), j - (comp == 1), k - (comp == 2));
  const uint8_t b = na_cell(cell, n, i, j, k);
  if (a == SOLID || b == SOLID) return false;
  return a == LIQUID || b == LIQUID;
}

__device__ inline void na_coords(int64_t idx, Dims d, int& i, int& j, int& k) {
  const int64_t row = idx / d.nx;
  i = (int)(idx - row * d.nx);
  j = (int)(row % d.ny);
  k = (int)(row / d.ny);
}

// grid (nb, 3): per block, the sum of (u - t)^2 and the number of active
// faces of its component
__global__ void __launch_bounds__(kBlock)
    k_na_mse_sum(int n, const uint8_t* __restrict__ cell, CF3 u, CF3 t, double* __restrict__ part) {
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  const int64_t F = face_count(n);
  double v[2] = {0.0, 0.0};
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < F;
       idx += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    na_coords(idx, d, i, j, k);
    if (na_active(cell, n, comp, i, j, k)) {
      const float diff = u.c[comp][idx] - t.c[comp][idx];
      v[0] += (double)diff * (double)diff;
      v[1] += 1.0;
    }
  }
  store_partials<2>(v, part, comp * gridDim.x + blockIdx.x);
}

// one block: J = sum / count into *loss, 1 / count (float) into res
__global__ void __launch_bounds__(kBlock)
    k_na_mse_final(const double* __restrict__ part, int nparts, double* __restrict__ loss,
                   double* __restrict__ res) {
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nparts; b += kBlock) {
    v[0] += part[2 * b];
    v[1] += part[2 * b + 1];
  }
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    const double cnt = v[1];
    *loss = cnt > 0.0 ? v[0] / cnt : 0.0;
    res[0] = cnt > 0.0 ? (double)(1.0f / (float)cnt) : 0.0;
  }
}

// g = 2 (u - t) / count on active faces, 0 elsewhere
__global__ void __launch_bounds__(kBlock)
    k_na_mse_grad(int n, const uint8_t* __restrict__ cell, CF3 u, CF3 t, F3 g,
                  const double* __restrict__ res) {
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  const int64_t F = face_count(n);
  const float inv = (float)res[0];
  float* __restrict__ gc = g.c[comp];
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < F;
       idx += (int64_t)gridDim.x * kBlock) {
    int i, j, k;
    na_coords(idx, d, i, j, k);
    float diff = 0.f;
    if (na_active(cell, n, comp, i, j, k)) diff = u.c[comp][idx] - t.c[comp][idx];
    gc[idx] = 2.f * diff * inv;
  }
}

std::mutex g_na_mu;
double* g_na_ptr[kNaMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array).
int na_scratch(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNaMaxDevices) return SIM_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_na_mu);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SIM_ERR_HIP;
    g_na_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_na_ptr[dev];
  return SIM_OK;
}

}  // namespace
}  // namespace fs

using namespace fs;

extern "C" int sim_loss_mse_noalloc(int32_t n, const uint8_t* d_cell, const float* d_u,
                                    const float* d_v, const float* d_w, const float* d_tu,
                                    const float* d_tv, const float* d_tw, double* d_loss,
                                    float* d_gu, float* d_gv, float* d_gw, void* hip_stream) {
  if (n < 4 || n > 1024) return SIM_ERR_INVALID_ARG;
  if (!d_cell || !d_u || !d_v || !d_w || !d_tu || !d_tv || !d_tw || !d_loss)
    return SIM_ERR_INVALID_ARG;
  const bool any_g = d_gu || d_gv || d_gw;
  if (any_g && !(d_gu && d_gv && d_gw)) return SIM_ERR_INVALID_ARG;
  if (any_g) {
    const void* outs[3] = {d_gu, d_gv, d_gw};
    const void* ins[7] = {d_u, d_v, d_w, d_tu, d_tv, d_tw, d_loss};
    for (int a = 0; a < 3; ++a) {
      for (int b = a + 1; b < 3; ++b)
        if (outs[a] == outs[b]) return SIM_ERR_INVALID_ARG;
      for (const void* p : ins)
        if (outs[a] == p) return SIM_ERR_INVALID_ARG;
    }
  }
  double* sc = nullptr;
  int rc = na_scratch(&sc);
  if (rc) return rc;
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  const int64_t F = face_count(n);
  int64_t nb = (F + kBlock - 1) / kBlock;
  nb = nb < 1 ? 1 : (nb > kNaBlocks ? kNaBlocks : nb);
  const CF3 u{{d_u, d_v, d_w}}, t{{d_tu, d_tv, d_tw}};
  hipLaunchKernelGGL(k_na_mse_sum, dim3((unsigned)nb, 3), dim3(kBlock), 0, stream, n, d_cell, u, t,
                     sc);
  hipLaunchKernelGGL(k_na_mse_final, dim3(1), dim3(kBlock), 0, stream, sc, (int)(3 * nb), d_loss,
                     sc + kNaResult);
  if (any_g)
    hipLaunchKernelGGL(k_na_mse_grad, dim3((unsigned)nb, 3), dim3(kBlock), 0, stream, n, d_cell, u,
                       t, F3{{d_gu, d_gv, d_gw}}, sc + kNaResult);
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_ERR_HIP;
}
