// Recurrent convolutional pressure solver (Section 3.4.1, PeRCNN-style): K
// layers
//
//   p_{k+1}(c) = L(c) s(c) ( sum_t W_t p_k(c + t) + w_b b(c) )
//
// over the 27 offsets t of a 3x3x3 stencil (tap (dx+1) + 3 (dy+1) + 9 (dz+1)),
// p_k = 0 outside the box.  The boundary-condition latent is the liquid mask L
// and s = 6 / n_c, n_c the Poisson diagonal (the context's cdiag, 0 off
// liquid); b is the velocity latent (the projection's right-hand side).  With
// W = 1/6 on the six face taps and w_b = 1/6 a layer is one Jacobi sweep.
//
// One layer is a memory-bound 27-point stencil (27 FMAs per cell against
// 13 bytes: p and b in, the diagonal code in, p out).  A block owns a 64 x 16
// tile of the xy-plane and marches through a run of z-planes: each plane of
// p (with a one-cell halo) is staged in a 4-slot LDS ring, so every value is
// read from memory once per block (plus the halo), and the loads of plane
// z+2 are in flight while plane z is computed.  Thread (tx, tg) owns column
// x0 + tx, rows y0 + 4 tg .. y0 + 4 tg + 3, and reads their 6 x 3 x 3
// neighbourhood from LDS once for the 4 outputs.
//
// The reverse pass of a layer (u = L s g_{k+1}):
//   g_k(c) = sum_t W_t u(c - t),  dL/db += w_b u,
//   dL/dW_t += sum_c u(c) p_k(c + t),  dL/dw_b += sum_c u(c) b(c);
// one kernel forms u on the fly from g_{k+1} and the diagonal, stages u and
// p_k in two rings, and writes g_k, gb and 28 per-block partial sums.
#include <cmath>

#include "common.h"
#include "ctx.h"

namespace fs {

constexpr int PC_TX = 64, PC_TY = 16;
constexpr int PC_RW = PC_TX + 2, PC_RH = PC_TY + 2;
constexpr int PC_PLANE = PC_RW * PC_RH;                       // 1188 staged values
constexpr int PC_ITEMS = (PC_PLANE + kBlock - 1) / kBlock;    // per thread
constexpr int PC_NW = 28;                                      // 27 taps, w_b
constexpr int PC_MAX_BLOCKS = kPartialDoubles / PC_NW;        // reverse-pass partials

struct PcWeights {
  float w[PC_NW];
};

// 6 / n_c for a diagonal code n_c in 0 .. 6 (0 off liquid), by selects: a
// table indexed per lane would be a memory load waited for at once
__device__ inline float six_over(uint32_t nc) {
  float s = 0.f;
  s = nc == 1u ? 6.f : s;
  s = nc == 2u ? 3.f : s;
  s = nc == 3u ? 2.f : s;
  s = nc == 4u ? 1.5f : s;
  s = nc == 5u ? 1.2f : s;
  s = nc == 6u ? 1.f : s;
  return s;
}

struct PcShape {
  int zc, blocks;
};

// 64 x 16 tiles; z-runs sized for about `target` blocks (at least 4 planes)
static PcShape pc_shape(int n, int target) {
  const int tiles = ((n + PC_TX - 1) / PC_TX) * ((n + PC_TY - 1) / PC_TY);
  int chunks = target / tiles;
  if (chunks < 1) chunks = 1;
  if (chunks > (n + 3) / 4) chunks = (n + 3) / 4;
  const int zc = (n + chunks - 1) / chunks;
  return PcShape{zc, tiles * ((n + zc - 1) / zc)};
}

struct PcTile {
  int x0, y0, z0, z1, tx, tg;
};

__device__ inline PcTile pc_tile(int n, int zc) {
  const int tiles_x = (n + PC_TX - 1) / PC_TX, tiles_y = (n + PC_TY - 1) / PC_TY;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int tile = lb % (tiles_x * tiles_y), chunk = lb / (tiles_x * tiles_y);
  PcTile t;
  t.x0 = (tile % tiles_x) * PC_TX;
  t.y0 = (tile / tiles_x) * PC_TY;
  t.z0 = chunk * zc;
  t.z1 = min(t.z0 + zc, n);
  t.tx = threadIdx.x % PC_TX;
  t.tg = threadIdx.x / PC_TX;
  return t;
}

// Staging of one plane of a cell array (with the one-cell xy halo) through
// registers: item k of the thread is staged value threadIdx.x + k kBlock;
// its in-plane offset is fixed for the block (0, a valid address, outside
// the box).  Loads go out raw; the mask is applied when the plane is stored,
// one plane later, so no wave waits for its loads at the load.
template <typename T>
struct PlaneStage {
  int off[PC_ITEMS];
  bool ok[PC_ITEMS];
  T raw[PC_ITEMS];
  bool on;

  __device__ void init(int n, int x0, int y0) {
#pragma unroll
    for (int k = 0; k < PC_ITEMS; ++k) {
      const int hv = threadIdx.x + k * kBlock;
      const int gx = x0 - 1 + hv % PC_RW, gy = y0 - 1 + hv / PC_RW;
      ok[k] = hv < PC_PLANE && (unsigned)gx < (unsigned)n && (unsigned)gy < (unsigned)n;
      off[k] = ok[k] ? gx + n * gy : 0;
    }
  }
  __device__ void load(const T* __restrict__ a, int n, int zi) {
    on = (unsigned)zi < (unsigned)n;
    if (!on) {
#pragma unroll
      for (int k = 0; k < PC_ITEMS; ++k) raw[k] = T(0);
      return;
    }
    const T* pl = a + (int64_t)zi * n * n;
#pragma unroll
    for (int k = 0; k < PC_ITEMS; ++k) raw[k] = pl[off[k]];
  }
  __device__ bool valid(int k) const { return on && ok[k]; }
};

// ------------------------------------------------------------- forward

__global__ void __launch_bounds__(kBlock)
    k_percnn_layer(int n, int zc, PcWeights W, const float* __restrict__ p,
                   const float* __restrict__ b, const uint8_t* __restrict__ cdiag,
                   float* __restrict__ out) {
  __shared__ float ring[4][PC_RH][PC_RW];
  const PcTile t = pc_tile(n, zc);
  if (t.z0 >= n) return;
  const int64_t nn = (int64_t)n * n;
  const int x = t.x0 + t.tx;
  PlaneStage<float> st;
  st.init(n, t.x0, t.y0);
  auto store = [&](int zi) {
    float* s = &ring[(zi + 4) & 3][0][0];
#pragma unroll
    for (int k = 0; k < PC_ITEMS; ++k) {
      const int hv = threadIdx.x + k * kBlock;
      if (hv < PC_PLANE) s[hv] = st.valid(k) ? st.raw[k] : 0.f;
    }
  };
  // b and the diagonal codes of the thread's 4 cells of a plane, loaded raw
  // (a clamped address for cells outside); outputs outside are not stored
  auto centre = [&](int zi, float (&bo)[4], uint8_t (&go)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int y = t.y0 + 4 * t.tg + j;
      const bool ok = x < n && y < n && zi < t.z1;
      const int64_t v = ok ? x + (int64_t)n * y + nn * zi : 0;
      bo[j] = b[v];
      go[j] = cdiag[v];
    }
  };
  st.load(p, n, t.z0 - 1);
  store(t.z0 - 1);
  st.load(p, n, t.z0);
  store(t.z0);
  st.load(p, n, t.z0 + 1);
  float bc[4];
  uint8_t gc[4];
  centre(t.z0, bc, gc);
  for (int z = t.z0; z < t.z1; ++z) {
    store(z + 1);
    __syncthreads();
    float bn[4];
    uint8_t gn[4];
    centre(z + 1, bn, gn);
    if (z + 2 <= t.z1) st.load(p, n, z + 2);
    float acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = W.w[27] * bc[j];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
      const float(*s)[PC_RW] = ring[(z + 3 + dz) & 3];
#pragma unroll
      for (int rr = 0; rr < 6; ++rr) {
        const float v0 = s[4 * t.tg + rr][t.tx], v1 = s[4 * t.tg + rr][t.tx + 1],
                    v2 = s[4 * t.tg + rr][t.tx + 2];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int dy = rr - j;  // 0, 1, 2 for offsets -1, 0, +1
          if (dy < 0 || dy > 2) continue;
          const int tb = 9 * dz + 3 * dy;
          acc[j] += W.w[tb] * v0 + W.w[tb + 1] * v1 + W.w[tb + 2] * v2;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int y = t.y0 + 4 * t.tg + j;
      if (x < n && y < n) out[x + (int64_t)n * y + nn * z] = six_over(gc[j]) * acc[j];
      bc[j] = bn[j];
      gc[j] = gn[j];
    }
  }
}

// ------------------------------------------------------------- reverse

// Wf: the weights with the taps reversed (Wf_t = W_{26-t}: offset -t), so
// that g_k(c) = sum_t Wf_t u(c + t); wb = w_b.  GB: gb accumulates dL/db
// (a template flag, so that its loads are unconditional and issued a plane
// ahead).
template <bool GB>
__global__ void __launch_bounds__(kBlock)
    k_percnn_layer_adj(int n, int zc, PcWeights Wf, const float* __restrict__ g,
                       const uint8_t* __restrict__ cdiag, const float* __restrict__ p,
                       const float* __restrict__ b, float* __restrict__ gout,
                       float* __restrict__ gb, double* __restrict__ partials) {
  __shared__ float uring[4][PC_RH][PC_RW];
  __shared__ float pring[4][PC_RH][PC_RW];
  const PcTile t = pc_tile(n, zc);
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  float dw[PC_NW];
#pragma unroll
  for (int q = 0; q < PC_NW; ++q) dw[q] = 0.f;
  if (t.z0 < n) {
    const int64_t nn = (int64_t)n * n;
    const int x = t.x0 + t.tx;
    PlaneStage<float> sg, sp;
    PlaneStage<uint8_t> sd;
    sg.init(n, t.x0, t.y0);
    sp.init(n, t.x0, t.y0);
    sd.init(n, t.x0, t.y0);
    auto load = [&](int zi) {
      sg.load(g, n, zi);
      sd.load(cdiag, n, zi);
      sp.load(p, n, zi);
    };
    auto store = [&](int zi) {
      float* su = &uring[(zi + 4) & 3][0][0];
      float* sq = &pring[(zi + 4) & 3][0][0];
#pragma unroll
      for (int k = 0; k < PC_ITEMS; ++k) {
        const int hv = threadIdx.x + k * kBlock;
        if (hv < PC_PLANE) {
          su[hv] = sg.valid(k) ? six_over(sd.raw[k]) * sg.raw[k] : 0.f;
          sq[hv] = sp.valid(k) ? sp.raw[k] : 0.f;
        }
      }
    };
    // b and (when accumulated) gb of the thread's 4 cells of a plane, loaded
    // raw one plane ahead (clamped address outside; those are not stored)
    auto centre_b = [&](int zi, float (&bo)[4], float (&go)[4]) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int y = t.y0 + 4 * t.tg + j;
        const bool ok = x < n && y < n && zi < t.z1;
        const int64_t v = ok ? x + (int64_t)n * y + nn * zi : 0;
        bo[j] = b[v];
        go[j] = GB ? gb[v] : 0.f;
      }
    };
    load(t.z0 - 1);
    store(t.z0 - 1);
    load(t.z0);
    store(t.z0);
    load(t.z0 + 1);
    float bc[4], gbc[4];
    centre_b(t.z0, bc, gbc);
    for (int z = t.z0; z < t.z1; ++z) {
      store(z + 1);
      __syncthreads();
      // the centre values go out first: a wait for them (in the epilogue)
      // then does not wait for the plane loads behind them
      float bn[4], gbn[4];
      centre_b(z + 1, bn, gbn);
      if (z + 2 <= t.z1) load(z + 2);
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
      float uc[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) uc[j] = uring[z & 3][4 * t.tg + j + 1][t.tx + 1];
#pragma unroll
      for (int dz = 0; dz < 3; ++dz) {
        const float(*su)[PC_RW] = uring[(z + 3 + dz) & 3];
        const float(*sq)[PC_RW] = pring[(z + 3 + dz) & 3];
#pragma unroll
        for (int rr = 0; rr < 6; ++rr) {
          const float u0 = su[4 * t.tg + rr][t.tx], u1 = su[4 * t.tg + rr][t.tx + 1],
                      u2 = su[4 * t.tg + rr][t.tx + 2];
          const float p0 = sq[4 * t.tg + rr][t.tx], p1 = sq[4 * t.tg + rr][t.tx + 1],
                      p2 = sq[4 * t.tg + rr][t.tx + 2];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int dy = rr - j;
            if (dy < 0 || dy > 2) continue;
            const int tb = 9 * dz + 3 * dy;
            acc[j] += Wf.w[tb] * u0 + Wf.w[tb + 1] * u1 + Wf.w[tb + 2] * u2;
            dw[tb] += uc[j] * p0;
            dw[tb + 1] += uc[j] * p1;
            dw[tb + 2] += uc[j] * p2;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int y = t.y0 + 4 * t.tg + j;
        dw[27] += uc[j] * bc[j];
        if (x < n && y < n) {
          const int64_t v = x + (int64_t)n * y + nn * z;
          gout[v] = acc[j];
          if (GB) gb[v] = gbc[j] + Wf.w[27] * uc[j];
        }
        bc[j] = bn[j];
        gbc[j] = gbn[j];
      }
    }
  }
  // block sums of the 28 weight-gradient terms (every thread takes part)
  __shared__ double red[kBlock / 64][PC_NW];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < PC_NW; ++q) {
    double v = dw[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[wv][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < PC_NW) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
    partials[(int64_t)lb * PC_NW + threadIdx.x] = s;
  }
}

// acc[q] += sum over blocks of partials[blk * 28 + q]; block q sums term q
__global__ void __launch_bounds__(kBlock)
    k_percnn_fold(const double* __restrict__ partials, int nblocks, double* __restrict__ acc) {
  __shared__ double red[kBlock / 64];
  const int q = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double v = 0.0;
  for (int blk = threadIdx.x; blk < nblocks; blk += kBlock) v += partials[(int64_t)blk * PC_NW + q];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) red[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += red[w];
    acc[q] += s;
  }
}

__global__ void __launch_bounds__(kBlock) k_percnn_zero(double* __restrict__ acc, float* __restrict__ gb,
                                                        int64_t count) {
  if (blockIdx.x == 0 && threadIdx.x < PC_NW) acc[threadIdx.x] = 0.0;
  if (gb)
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock)
      gb[i] = 0.f;
}

// The fit's loss and its seed gradient for one pair: over liquid cells
// (Poisson diagonal non-zero) e = p_K - target, g = 2 e, and the block
// partial of sum e^2; zero elsewhere.
__global__ void __launch_bounds__(kBlock)
    k_percnn_fit_seed(int64_t C, const uint8_t* __restrict__ cdiag, const float* __restrict__ pK,
                      const float* __restrict__ target, float* __restrict__ g,
                      double* __restrict__ partials) {
  double v[1] = {0.0};
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < C; i += (int64_t)gridDim.x * kBlock) {
    const float e = cdiag[i] ? pK[i] - target[i] : 0.f;
    g[i] = 2.f * e;
    v[0] += (double)e * (double)e;
  }
  store_partials<1>(v, partials, blockIdx.x);
}

}  // namespace fs

using namespace fs;

extern "C" {

int sim_percnn_forward(sim_ctx* c, const float* h_w, int32_t K, const float* p0, const float* b,
                       float* out, float* hist) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!h_w || !p0 || !b || (!out && !hist) || K < 0) {
    c->err = "sim_percnn_forward: NULL pointer or K < 0";
    return SIM_ERR_INVALID_ARG;
  }
  const int64_t C = c->C;
  if (out && (out == p0 || out == b)) {
    c->err = "sim_percnn_forward: out aliases an input";
    return SIM_ERR_INVALID_ARG;
  }
  if (hist && (hist == p0 || hist == b || (out && out >= hist && out < hist + (K + 1) * C))) {
    c->err = "sim_percnn_forward: hist aliases an input or the output";
    return SIM_ERR_INVALID_ARG;
  }
  PcWeights W;
  for (int q = 0; q < PC_NW; ++q) W.w[q] = h_w[q];
  const PcShape sh = pc_shape(c->n, 1024);
  auto layer = [&](const float* src, float* dst) {
    prof_mark(c, SIM_KERN_PERCNN, true);
    hipLaunchKernelGGL(k_percnn_layer, dim3(sh.blocks), dim3(kBlock), 0, c->stream, c->n, sh.zc, W,
                       src, b, c->cdiag, dst);
    prof_mark(c, SIM_KERN_PERCNN, false);
  };
  if (hist) {
    if (hipMemcpyAsync(hist, p0, sizeof(float) * C, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
      return SIM_ERR_HIP;
    for (int k = 0; k < K; ++k) layer(hist + k * C, hist + (k + 1) * C);
  } else {
    const float* src = p0;
    for (int k = 0; k < K; ++k) {
      float* dst = k == K - 1 ? out : ((k & 1) ? c->dB : c->dA);
      layer(src, dst);
      src = dst;
    }
  }
  if (out && (hist || K == 0)) {
    const float* last = hist ? hist + K * C : p0;
    if (hipMemcpyAsync(out, last, sizeof(float) * C, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
      return SIM_ERR_HIP;
  }
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_ERR_HIP;
}

int sim_percnn_backward(sim_ctx* c, const float* h_w, int32_t K, const float* b, const float* hist,
                        const float* g, float* gp0, float* gb, double* h_grad_w) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!h_w || !b || !hist || !g || !h_grad_w || K < 0) {
    c->err = "sim_percnn_backward: NULL pointer or K < 0";
    return SIM_ERR_INVALID_ARG;
  }
  const int64_t C = c->C;
  if ((gp0 && (gp0 == g || gp0 == b || (gp0 >= hist && gp0 < hist + (K + 1) * C))) ||
      (gb && (gb == g || gb == b || gb == gp0 || (gb >= hist && gb < hist + (K + 1) * C)))) {
    c->err = "sim_percnn_backward: an output aliases an input";
    return SIM_ERR_INVALID_ARG;
  }
  PcWeights Wf;
  for (int q = 0; q < 27; ++q) Wf.w[q] = h_w[26 - q];
  Wf.w[27] = h_w[27];
  const PcShape sh = pc_shape(c->n, 768);
  if (sh.blocks > PC_MAX_BLOCKS) {
    c->err = "sim_percnn_backward: grid too large for the partial sums";
    return SIM_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_percnn_zero, dim3(gb ? 1024 : 1), dim3(kBlock), 0, c->stream, c->pc_acc, gb, C);
  const float* src = g;
  for (int k = K - 1; k >= 0; --k) {
    float* dst = (k == 0 && gp0) ? gp0 : (((K - 1 - k) & 1) ? c->dB : c->dA);
    prof_mark(c, SIM_KERN_PERCNN_ADJ, true);
    if (gb)
      hipLaunchKernelGGL(k_percnn_layer_adj<true>, dim3(sh.blocks), dim3(kBlock), 0, c->stream, c->n,
                         sh.zc, Wf, src, c->cdiag, hist + k * C, b, dst, gb, c->partials);
    else
      hipLaunchKernelGGL(k_percnn_layer_adj<false>, dim3(sh.blocks), dim3(kBlock), 0, c->stream, c->n,
                         sh.zc, Wf, src, c->cdiag, hist + k * C, b, dst, gb, c->partials);
    prof_mark(c, SIM_KERN_PERCNN_ADJ, false);
    hipLaunchKernelGGL(k_percnn_fold, dim3(PC_NW), dim3(kBlock), 0, c->stream, c->partials, sh.blocks,
                       c->pc_acc);
    src = dst;
  }
  if (K == 0 && gp0 &&
      hipMemcpyAsync(gp0, g, sizeof(float) * C, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return SIM_ERR_HIP;
  // dL/dW in the caller's tap order: dL/dW_t = sum_c u(c) p(c + t), which the
  // kernel accumulates per tap t of the forward stencil
  double acc[PC_NW];
  if (hipMemcpyAsync(acc, c->pc_acc, sizeof acc, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return SIM_ERR_HIP;
  for (int q = 0; q < PC_NW; ++q) h_grad_w[q] = acc[q];
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_ERR_HIP;
}

// One Adam step of the kernel fit: for every pair, K layers from its p0 with
// the states kept in d_hist, the loss and seed gradient on the device, and
// the reverse pass for dL/dW; then the Adam update of the 28 weights here on
// the host (beta 0.9 / 0.999, eps 1e-12).
int sim_percnn_fit_step(sim_ctx* c, double* h_w, double* h_adam, int32_t step, double lr, int32_t K,
                        int32_t npairs, const float* p0, const float* target, const float* b,
                        float* hist, double* h_loss) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!h_w || !h_adam || !p0 || !target || !b || !hist || step < 1 || K < 1 || npairs < 1 ||
      !(lr > 0.0 && std::isfinite(lr))) {
    c->err = "sim_percnn_fit_step: NULL pointer, step < 1, K < 1, npairs < 1 or lr not > 0";
    return SIM_ERR_INVALID_ARG;
  }
  const int64_t C = c->C;
  const float* ins[3] = {p0, target, b};
  for (const float* q : ins)
    if (q + (int64_t)npairs * C > hist && q < hist + (int64_t)(K + 1) * C) {
      c->err = "sim_percnn_fit_step: hist overlaps a pair array";
      return SIM_ERR_INVALID_ARG;
    }
  float wf[PC_NW];
  for (int q = 0; q < PC_NW; ++q) {
    if (!std::isfinite(h_w[q])) {
      c->err = "sim_percnn_fit_step: non-finite weight";
      return SIM_ERR_INVALID_ARG;
    }
    wf[q] = (float)h_w[q];
  }
  double grad[PC_NW] = {}, loss = 0.0;
  float* g = c->q;  // the seed gradient (a solver buffer, free outside a solve)
  const int nb = 1024;
  for (int pr = 0; pr < npairs; ++pr) {
    const int64_t off = (int64_t)pr * C;
    int rc = sim_percnn_forward(c, wf, K, p0 + off, b + off, nullptr, hist);
    if (rc) return rc;
    hipLaunchKernelGGL(k_percnn_fit_seed, dim3(nb), dim3(kBlock), 0, c->stream, C, c->cdiag,
                       hist + (int64_t)K * C, target + off, g, c->partials);
    launch_finalize(c, nb, 1, FIN_SLOT, 0.0, 0, S_DOT0, 1.0, 0);
    double gw[PC_NW];
    rc = sim_percnn_backward(c, wf, K, b + off, hist, g, nullptr, nullptr, gw);
    if (rc) return rc;
    double l = 0.0;
    if (hipMemcpyAsync(&l, c->scal + S_DOT0, sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return SIM_ERR_HIP;
    loss += l;
    for (int q = 0; q < PC_NW; ++q) grad[q] += gw[q];
  }
  const double inv = 1.0 / npairs;
  const double c1 = 1.0 - std::pow(0.9, step), c2 = 1.0 - std::pow(0.999, step);
  for (int q = 0; q < PC_NW; ++q) {
    const double gq = grad[q] * inv;
    double& m = h_adam[q];
    double& v = h_adam[PC_NW + q];
    m = 0.9 * m + 0.1 * gq;
    v = 0.999 * v + 0.001 * gq * gq;
    h_w[q] -= lr * (m / c1) / (std::sqrt(v / c2) + 1e-12);
  }
  if (h_loss) *h_loss = loss * inv;
  return SIM_OK;
}

}  // extern "C"
