// Kernels of the learned preconditioner (3-level 3-D U-Net) and its training.
//
// The paper replaces the pressure solve by a convolutional network fitted on
// pressure pairs from an implicit solve (Section 3.4.1).  Here the network is
// a preconditioner inside flexible CG.  Activations are bf16, channels-last
// ([z][y][x][C], C a multiple of 8); weights bf16; accumulation fp32.
//
// Convolution = implicit GEMM on the 16x16x32 bf16 MFMA of gfx950:
//   M = 16 output voxels along x, N = 16 output channels, K = 32 =
//   (2 taps x 16 channels) or (4 taps x 8 channels).
// A block computes a 16 x 4 x 4 voxel tile for all output channels; the
// input halo tile (18 x 6 x 6 voxels, one 16- or 8-channel chunk at a time)
// is staged in LDS, weights stream from L2.  MFMA lane layout (checked on the
// device): A[row = lane%16][k = 8(lane/16)+i], B[k = 8(lane/16)+i][col =
// lane%16], D[row = 4(lane/16)+i][col = lane%16].
//
// The input of a convolution can be the concatenation of a nearest-upsampled
// coarse tensor and a same-level skip tensor; the halo loader reads both, so
// neither the upsampled tensor nor the concatenation is ever stored.
// Backward: the data gradient is the same kernel with transposed, tap-flipped
// weights; the weight gradient is an LDS-tiled fp32 kernel.
#include "common.h"
#include "ctx.h"
#include "net.h"

namespace fs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TX = 16, TY = 4, TZ = 4;
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HV = HX * HY * HZ;  // 648 halo voxels
constexpr int TAPS = 28;  // 27 taps padded with a zero tap

__device__ inline bool inside(int x, int y, int z, int n) {
  return (unsigned)x < (unsigned)n && (unsigned)y < (unsigned)n && (unsigned)z < (unsigned)n;
}

__device__ inline int64_t vox(int x, int y, int z, int n) {
  return x + (int64_t)n * (y + (int64_t)n * z);
}

struct TileXYZ {
  int x0, y0, z0;
};

__device__ inline TileXYZ tile_of(int n, int b) {
  const int tx = (n + TX - 1) / TX, ty = (n + TY - 1) / TY;
  TileXYZ t;
  t.x0 = (b % tx) * TX;
  t.y0 = ((b / tx) % ty) * TY;
  t.z0 = (b / (tx * ty)) * TZ;
  return t;
}

int conv_tiles(int n) { return ((n + TX - 1) / TX) * ((n + TY - 1) / TY) * ((n + TZ - 1) / TZ); }

// Channels [c0, c0+CK) of the (possibly concatenated) input over the halo of
// a tile, as [HV][CK] bf16, zero outside the volume: load() issues all of a
// thread's loads (from valid clamped addresses), store() writes them to LDS,
// so the staging waits for one load latency, not one per item.
template <int CK>
struct HaloRegs {
  static constexpr int PV = CK / 8;  // 16-byte vectors per voxel
  static constexpr int NV = HV * PV;
  static constexpr int NI = (NV + kBlock - 1) / kBlock;
  uint4 raw[NI];
  bool ok[NI];

  __device__ inline void load(const NetSrc& s, int n, TileXYZ t, int c0) {
    const int nc = n / 2;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int vi = threadIdx.x + k * kBlock;
      const int hv = vi / PV, part = vi - hv * PV;
      const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
      const int gx = t.x0 - 1 + hx, gy = t.y0 - 1 + hy, gz = t.z0 - 1 + hz;
      ok[k] = vi < NV && inside(gx, gy, gz, n);
      const int c = c0 + part * 8;
      const __bf16* src = s.a;
      if (ok[k]) {
        if (c < s.ca) {
          const int64_t v = s.up ? vox(gx >> 1, gy >> 1, gz >> 1, nc) : vox(gx, gy, gz, n);
          src = s.a + v * s.ca + c;
        } else {
          src = s.b + vox(gx, gy, gz, n) * s.cb + (c - s.ca);
        }
      }
      raw[k] = *reinterpret_cast<const uint4*>(src);
    }
  }
  __device__ inline void store(__bf16* __restrict__ lds) const {
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int vi = threadIdx.x + k * kBlock;
      if (vi < NV)
        *reinterpret_cast<uint4*>(lds + vi * 8) = ok[k] ? raw[k] : make_uint4(0u, 0u, 0u, 0u);
    }
  }
};

template <int CK>
__device__ inline void load_halo(__bf16* __restrict__ lds, const NetSrc& s, int n, TileXYZ t,
                                 int c0) {
  HaloRegs<CK> h;
  h.load(s, n, t, c0);
  h.store(lds);
}

// ------------------------------------------------------------ convolution

template <int CIN, int COUT, int CK, int EPI>
__global__ void __launch_bounds__(kBlock)
    k_conv(int n, NetSrc src, const __bf16* __restrict__ w, NetOut out,
           const int* __restrict__ flags) {
  if (flags && flags[F_DONE]) return;
  static_assert(CIN % CK == 0 && COUT % 16 == 0, "channel counts");
  constexpr int NT = COUT / 16;
  constexpr int STEPS = CK == 16 ? 14 : 7;
  constexpr int HALO_E = HV * CK;
  constexpr int OUT_E = TX * TY * TZ * COUT;
  // 64-output-channel layers (the coarsest level) stage each chunk's weights
  // in LDS as [tap][half][c_out][8]: the 16 lanes of a fragment read
  // consecutive 16-byte words, and no step waits on an L2 load
  constexpr bool WL = CK == 16 && COUT == 64;
  constexpr int WL_E = WL ? TAPS * 2 * COUT * 8 : 8;
  // the epilogue's output tile overlays the halo and the weights, so that
  // the 64-channel layers (78 KB) fit two blocks per CU
  constexpr int SM_E = HALO_E + WL_E > OUT_E ? HALO_E + WL_E : OUT_E;
  __shared__ __attribute__((aligned(16))) __bf16 smem[SM_E];
  __bf16* const lds = smem;
  __bf16* const wl = smem + HALO_E;
  const TileXYZ t = tile_of(n, blockIdx.x);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, col = lane & 15;
  f32x4 acc[4][NT];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  // a chunk's halo and (WL) weight words: all of a thread's loads are issued
  // before its first store
  constexpr int NW = TAPS * 2 * COUT;
  constexpr int NWI = WL ? (NW + kBlock - 1) / kBlock : 1;
#pragma unroll 1
  for (int c0 = 0; c0 < CIN; c0 += CK) {
    __syncthreads();
    HaloRegs<CK> hr;
    uint4 wr[NWI];
    hr.load(src, n, t, c0);
    if (WL) {
#pragma unroll
      for (int k = 0; k < NWI; ++k) {
        const int q = threadIdx.x + k * kBlock;
        const int qq = q < NW ? q : 0;
        const int co = qq % COUT, half = (qq / COUT) & 1, tap = qq / (2 * COUT);
        wr[k] = *reinterpret_cast<const uint4*>(w + ((int64_t)co * TAPS + tap) * CIN + c0 + half * 8);
      }
    }
    hr.store(lds);
    if (WL) {
#pragma unroll
      for (int k = 0; k < NWI; ++k) {
        const int q = threadIdx.x + k * kBlock;
        if (q < NW) *reinterpret_cast<uint4*>(wl + (int64_t)q * 8) = wr[k];
      }
    }
    __syncthreads();
#pragma unroll 2
    for (int s = 0; s < STEPS; ++s) {
      const int tap = CK == 16 ? 2 * s + (g >> 1) : 4 * s + g;
      const int coff = CK == 16 ? (g & 1) * 8 : 0;
      const int tp = tap < 27 ? tap : 26;  // tap 27 has zero weights
      const int dx = tp % 3, dy = (tp / 3) % 3, dz = tp / 9;
      bf16x8 bfr[NT];
#pragma unroll
      for (int b = 0; b < NT; ++b)
        bfr[b] = WL ? *reinterpret_cast<const bf16x8*>(wl + ((tap * 2 + (g & 1)) * COUT + b * 16 + col) * 8)
                    : *reinterpret_cast<const bf16x8*>(
                          w + ((int64_t)(b * 16 + col) * TAPS + tap) * CIN + c0 + coff);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int hv = (col + dx) + HX * ((a + dy) + HY * (wv + dz));
        const bf16x8 afr = *reinterpret_cast<const bf16x8*>(lds + hv * CK + coff);
#pragma unroll
        for (int b = 0; b < NT; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[b], acc[a][b], 0, 0, 0);
      }
    }
  }

  if (EPI == NET_EPI_OUT) {
    // channel 0 only: z = mask * rms * o (fp32); lanes with col 0 hold it
    if (col == 0) {
      const double rms = *out.rms;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int x = t.x0 + g * 4 + i, y = t.y0 + a, z = t.z0 + wv;
          if (!inside(x, y, z, n)) continue;
          const int64_t v = vox(x, y, z, n);
          out.f32[v] = out.mask[v] ? (float)(rms * (double)acc[a][0][i]) : 0.f;
        }
    }
    return;
  }
  // other epilogues: stage the tile in LDS as [voxel][COUT] bf16, copy out coalesced
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int lv = (g * 4 + i) + TX * (a + TY * wv);
        float v = acc[a][b][i];
        if (EPI == NET_EPI_RELU) v = v > 0.f ? v : 0.f;
        lds[lv * COUT + b * 16 + col] = (__bf16)v;
      }
  __syncthreads();
  constexpr int PV = COUT / 8;
  for (int vi = threadIdx.x; vi < TX * TY * TZ * PV; vi += kBlock) {
    const int lv = vi / PV, part = vi - lv * PV;
    const int x = t.x0 + lv % TX, y = t.y0 + (lv / TX) % TY, z = t.z0 + lv / (TX * TY);
    if (!inside(x, y, z, n)) continue;
    const int64_t v = vox(x, y, z, n);
    uint4 val = *reinterpret_cast<const uint4*>(lds + lv * COUT + part * 8);
    if (EPI == NET_EPI_MASKGRAD) {
      // gradient through the ReLU whose output (post-activation) is out.relu_of
      const uint4 pm = *reinterpret_cast<const uint4*>(out.relu_of + v * COUT + part * 8);
      const uint32_t* pw = reinterpret_cast<const uint32_t*>(&pm);
      uint32_t* vw = reinterpret_cast<uint32_t*>(&val);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // bf16 > 0: sign bit clear and not +0
        const uint32_t lo = pw[q] & 0xffffu, hi = pw[q] >> 16;
        const uint32_t keep_lo = (lo != 0u && !(lo & 0x8000u)) ? 0xffffu : 0u;
        const uint32_t keep_hi = (hi != 0u && !(hi & 0x8000u)) ? 0xffff0000u : 0u;
        vw[q] &= (keep_lo | keep_hi);
      }
    }
    *reinterpret_cast<uint4*>(out.bf + v * COUT + part * 8) = val;
  }
}

// ------------------------------------------------------------ weight grad
// dW[co][ci][tap] += sum over voxels of G[v][co] * X[v + off(tap)][ci], for
// one 16-channel block of c_out and one CK-channel chunk of c_in per block;
// each thread owns one (co, ci) pair (two threads per pair when CK = 8) and
// 27 fp32 accumulators; the block walks `tiles` voxel tiles, then adds to dW
// with fp32 atomics.
template <int CK>
__global__ void __launch_bounds__(kBlock)
    k_wgrad(int n, NetSrc src, int cin_real, const __bf16* __restrict__ G, int g_stride,
            int cout_real, float* __restrict__ dW, int tiles_per_block, int ntiles) {
  __shared__ float xs[HV * CK];
  __shared__ float gs[TX * TY * TZ * 16];
  constexpr int PAIRS = 16 * CK;
  constexpr int SPLIT = kBlock / PAIRS;  // threads per pair (1 or 2)
  const int pair = threadIdx.x % PAIRS, sub = threadIdx.x / PAIRS;
  const int co_l = pair / CK, ci_l = pair % CK;
  const int c0 = blockIdx.y * CK;
  const int co0 = blockIdx.z * 16;
  float acc[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) acc[q] = 0.f;
  __shared__ __attribute__((aligned(16))) __bf16 stage[HV * CK];
  for (int tt = 0; tt < tiles_per_block; ++tt) {
    const int tb = blockIdx.x * tiles_per_block + tt;
    if (tb >= ntiles) break;
    const TileXYZ t = tile_of(n, tb);
    __syncthreads();
    load_halo<CK>(stage, src, n, t, c0);
    for (int vi = threadIdx.x; vi < TX * TY * TZ * 16; vi += kBlock) {
      const int lv = vi / 16, c = vi % 16;
      const int x = t.x0 + lv % TX, y = t.y0 + (lv / TX) % TY, z = t.z0 + lv / (TX * TY);
      float gv = 0.f;
      if (inside(x, y, z, n) && co0 + c < cout_real) gv = (float)G[vox(x, y, z, n) * g_stride + co0 + c];
      gs[vi] = gv;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < HV * CK; q += kBlock) xs[q] = (float)stage[q];
    __syncthreads();
    for (int lv = sub; lv < TX * TY * TZ; lv += SPLIT) {
      const float gv = gs[lv * 16 + co_l];
      const int x = lv % TX, y = (lv / TX) % TY, z = lv / (TX * TY);
      const int base = x + HX * (y + HY * z);
#pragma unroll
      for (int q = 0; q < 27; ++q) {
        const int off = (q % 3) + HX * (((q / 3) % 3) + HY * (q / 9));
        acc[q] += gv * xs[(base + off) * CK + ci_l];
      }
    }
  }
  const int co = co0 + co_l, ci = c0 + ci_l;
  if (co < cout_real && ci < cin_real) {
    float* dst = dW + ((int64_t)co * cin_real + ci) * 27;
#pragma unroll
    for (int q = 0; q < 27; ++q)
      if (acc[q] != 0.f) atomicAdd(dst + q, acc[q]);
  }
}

// --------------------------------------------------------------- helpers

// 2x2x2 average pool of a bf16 tensor with C channels: level n -> n/2.
__global__ void __launch_bounds__(kBlock)
    k_pool(int n, int C, const __bf16* __restrict__ in, __bf16* __restrict__ out,
           const int* __restrict__ flags) {
  if (flags && flags[F_DONE]) return;
  const int nc = n / 2;
  const int64_t total = (int64_t)nc * nc * nc * C;
  for (int64_t q = blockIdx.x * (int64_t)kBlock + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlock) {
    const int c = (int)(q % C);
    const int64_t v = q / C;
    const int x = (int)(v % nc), y = (int)((v / nc) % nc), z = (int)(v / ((int64_t)nc * nc));
    float s = 0.f;
#pragma unroll
    for (int d = 0; d < 8; ++d)
      s += (float)in[vox(2 * x + (d & 1), 2 * y + ((d >> 1) & 1), 2 * z + (d >> 2), n) * C + c];
    out[q] = (__bf16)(0.125f * s);
  }
}

// Input of the network: channel 0 = r / rms(r), channel 1 = liquid mask,
// channels 2..7 = 0.  rms = sqrt(sum r^2 / n_liquid) from scal[slot].
__global__ void __launch_bounds__(kBlock)
    k_net_input(int n, const float* __restrict__ r, const uint8_t* __restrict__ cdiag,
                const double* __restrict__ sumsq, double n_liquid, double* __restrict__ rms_out,
                __bf16* __restrict__ x0, const int* __restrict__ flags) {
  if (flags && flags[F_DONE]) return;
  const double rms = n_liquid > 0.0 ? sqrt(*sumsq / n_liquid) : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *rms_out = rms;
  const float inv = rms > 0.0 ? (float)(1.0 / rms) : 0.f;
  const int64_t C = cells(n);
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < C;
       v += (int64_t)gridDim.x * kBlock) {
    __bf16 o[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = (__bf16)0.f;
    o[0] = (__bf16)(r[v] * inv);
    o[1] = (__bf16)(cdiag[v] ? 1.f : 0.f);
    *reinterpret_cast<uint4*>(x0 + v * 8) = *reinterpret_cast<const uint4*>(o);
  }
}

// Gradient of the A-norm loss with respect to the network output o, written
// as the 8-channel bf16 gradient of the output convolution (channel 0):
//   L = 1 - (r.z)^2 / ((r.e)(z.Az)),  z = mask rms o
//   dL/dz = c1 r + c2 Az,  c1 = -2 rz/(re zAz),  c2 = 2 rz^2/(re zAz^2).
__global__ void __launch_bounds__(kBlock)
    k_loss_grad(int n, const float* __restrict__ r, const float* __restrict__ Az,
                const uint8_t* __restrict__ cdiag, const double* __restrict__ dots /*rz re zAz*/,
                const double* __restrict__ rms, __bf16* __restrict__ g11) {
  const double rz = dots[0], re = dots[1], zAz = dots[2];
  const double c1 = -2.0 * rz / (re * zAz), c2 = 2.0 * rz * rz / (re * zAz * zAz);
  const double s = *rms;
  const int64_t C = cells(n);
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < C;
       v += (int64_t)gridDim.x * kBlock) {
    __bf16 o[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = (__bf16)0.f;
    if (cdiag[v]) o[0] = (__bf16)(s * (c1 * (double)r[v] + c2 * (double)Az[v]));
    *reinterpret_cast<uint4*>(g11 + v * 8) = *reinterpret_cast<const uint4*>(o);
  }
}

// Backward of "cat(up(coarse), skip)" for the coarse part: the gradient of
// the coarse tensor is the sum over its 8 children of the first Cc channels
// of the concatenated gradient T (stride Ct), times the ReLU mask of the
// coarse post-activation P.
__global__ void __launch_bounds__(kBlock)
    k_upsum_mask(int n_fine, int Cc, int Ct, const __bf16* __restrict__ T,
                 const __bf16* __restrict__ P, __bf16* __restrict__ out) {
  const int nc = n_fine / 2;
  const int64_t total = (int64_t)nc * nc * nc * Cc;
  for (int64_t q = blockIdx.x * (int64_t)kBlock + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlock) {
    const int c = (int)(q % Cc);
    const int64_t v = q / Cc;
    const int x = (int)(v % nc), y = (int)((v / nc) % nc), z = (int)(v / ((int64_t)nc * nc));
    float s = 0.f;
#pragma unroll
    for (int d = 0; d < 8; ++d)
      s += (float)T[vox(2 * x + (d & 1), 2 * y + ((d >> 1) & 1), 2 * z + (d >> 2), n_fine) * Ct + c];
    out[q] = (float)P[q] > 0.f ? (__bf16)s : (__bf16)0.f;
  }
}

// Gradient of a skip tensor E (fine level, C channels) that feeds both the
// concatenation (channels [off, off+C) of T) and an average pool whose
// gradient is gp (coarse level): (T_skip + gp[parent] / 8) * (E > 0).
__global__ void __launch_bounds__(kBlock)
    k_skip_grad(int n, int C, const __bf16* __restrict__ T, int Ct, int off,
                const __bf16* __restrict__ gp, const __bf16* __restrict__ E,
                __bf16* __restrict__ out) {
  const int nc = n / 2;
  const int64_t total = cells(n) * C;
  for (int64_t q = blockIdx.x * (int64_t)kBlock + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlock) {
    const int c = (int)(q % C);
    const int64_t v = q / C;
    const int x = (int)(v % n), y = (int)((v / n) % n), z = (int)(v / ((int64_t)n * n));
    const float s = (float)T[v * Ct + off + c] + 0.125f * (float)gp[vox(x >> 1, y >> 1, z >> 1, nc) * C + c];
    out[q] = (float)E[q] > 0.f ? (__bf16)s : (__bf16)0.f;
  }
}

// Master fp32 weights (PyTorch layout [co][ci][27]) -> bf16 forward layout
// [co_pad][28][ci_pad] and transposed, tap-flipped data-gradient layout
// [ci][28][co_pad8] for one convolution.
__global__ void __launch_bounds__(kBlock)
    k_pack_weights(const float* __restrict__ W, int cin, int cout, int cin_p, int cout_p,
                   int cout_pd, __bf16* __restrict__ wf, __bf16* __restrict__ wd) {
  const int64_t nf = (int64_t)cout_p * TAPS * cin_p;
  const int64_t nd = wd ? (int64_t)cin * TAPS * cout_pd : 0;
  for (int64_t q = blockIdx.x * (int64_t)kBlock + threadIdx.x; q < nf + nd;
       q += (int64_t)gridDim.x * kBlock) {
    if (q < nf) {
      const int ci = (int)(q % cin_p), tap = (int)((q / cin_p) % TAPS), co = (int)(q / (cin_p * TAPS));
      const float v = (co < cout && ci < cin && tap < 27) ? W[((int64_t)co * cin + ci) * 27 + tap] : 0.f;
      wf[q] = (__bf16)v;
    } else {
      const int64_t p = q - nf;
      const int co = (int)(p % cout_pd), tap = (int)((p / cout_pd) % TAPS), ci = (int)(p / (cout_pd * TAPS));
      const float v = (co < cout && tap < 27) ? W[((int64_t)co * cin + ci) * 27 + (26 - tap)] : 0.f;
      wd[p] = (__bf16)v;
    }
  }
}

// Adam on the fp32 master weights with the batch-mean gradient dW / batch.
__global__ void __launch_bounds__(kBlock)
    k_adam(int64_t count, float* __restrict__ W, float* __restrict__ m, float* __restrict__ v,
           const float* __restrict__ dW, float inv_batch, float lr, float b1, float b2, float eps,
           float bc1, float bc2) {
  for (int64_t q = blockIdx.x * (int64_t)kBlock + threadIdx.x; q < count;
       q += (int64_t)gridDim.x * kBlock) {
    const float gq = dW[q] * inv_batch;
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    W[q] -= lr * (mq / bc1) / (sqrtf(vq / bc2) + eps);
  }
}

__global__ void __launch_bounds__(kBlock)
    k_scale_copy(const float* __restrict__ a, float* __restrict__ o, int64_t count, float s) {
  for (int64_t q = blockIdx.x * (int64_t)kBlock + threadIdx.x; q < count;
       q += (int64_t)gridDim.x * kBlock)
    o[q] = s * a[q];
}

// --------------------------------------------------------------- launchers

template <int CIN, int COUT, int CK, int EPI>
static void conv_launch(sim_ctx* c, int n, NetSrc src, const __bf16* w, NetOut out,
                        const int* flags) {
  hipLaunchKernelGGL((k_conv<CIN, COUT, CK, EPI>), dim3(conv_tiles(n)), dim3(kBlock), 0, c->stream,
                     n, src, w, out, flags);
}

// Dispatch on the channel configuration of the U-Net's convolutions (forward
// and data-gradient); returns false for an unknown configuration.
bool net_conv(sim_ctx* c, int n, int cin, int cout, int epi, NetSrc src, const __bf16* w,
              NetOut out, const int* flags) {
  if (net_conv_zm(c, n, cin, cout, epi, src, w, out, flags)) return true;
  // only the z-marching kernels add partial sums or pool
  if (epi == NET_EPI_RELU_ADD || epi == NET_EPI_RELU_POOL) return false;
#define FS_CONV(CI, CO, CK)                                                   \
  if (cin == CI && cout == CO) {                                              \
    if (epi == NET_EPI_RELU) conv_launch<CI, CO, CK, NET_EPI_RELU>(c, n, src, w, out, flags);        \
    else if (epi == NET_EPI_RAW) conv_launch<CI, CO, CK, NET_EPI_RAW>(c, n, src, w, out, flags);     \
    else if (epi == NET_EPI_MASKGRAD) conv_launch<CI, CO, CK, NET_EPI_MASKGRAD>(c, n, src, w, out, flags); \
    else conv_launch<CI, CO, CK, NET_EPI_OUT>(c, n, src, w, out, flags);     \
    return true;                                                              \
  }
  // forward
  FS_CONV(8, 16, 8)
  FS_CONV(16, 16, 16)
  FS_CONV(16, 32, 16)
  FS_CONV(32, 32, 16)
  FS_CONV(32, 64, 16)
  FS_CONV(64, 64, 16)
  FS_CONV(96, 32, 16)
  FS_CONV(48, 16, 16)
  // data gradient (c_in and c_out swapped)
  FS_CONV(32, 96, 16)
  FS_CONV(16, 48, 16)
  FS_CONV(64, 32, 16)
  FS_CONV(32, 16, 16)
#undef FS_CONV
  return false;
}

void net_wgrad(sim_ctx* c, int n, NetSrc src, int cin_real, int cin_pad, const __bf16* G,
               int g_stride, int cout_real, float* dW) {
  const int ntiles = conv_tiles(n);
  const int tpb = ntiles >= 4096 ? 8 : (ntiles >= 512 ? 4 : 1);
  const int bx = (ntiles + tpb - 1) / tpb;
  const int co_blocks = (cout_real + 15) / 16;
  if (cin_pad % 16 == 0) {
    hipLaunchKernelGGL(k_wgrad<16>, dim3(bx, cin_pad / 16, co_blocks), dim3(kBlock), 0, c->stream,
                       n, src, cin_real, G, g_stride, cout_real, dW, tpb, ntiles);
  } else {
    hipLaunchKernelGGL(k_wgrad<8>, dim3(bx, cin_pad / 8, co_blocks), dim3(kBlock), 0, c->stream, n,
                       src, cin_real, G, g_stride, cout_real, dW, tpb, ntiles);
  }
}

static int grid_for_elems(int64_t e) {
  int64_t g = (e + kBlock - 1) / kBlock;
  return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

void net_pool(sim_ctx* c, int n, int C, const __bf16* in, __bf16* out, const int* flags) {
  const int64_t e = (int64_t)(n / 2) * (n / 2) * (n / 2) * C;
  hipLaunchKernelGGL(k_pool, dim3(grid_for_elems(e)), dim3(kBlock), 0, c->stream, n, C, in, out,
                     flags);
}

void net_input(sim_ctx* c, const float* r, const double* sumsq, double* rms_out, __bf16* x0,
               const int* flags) {
  hipLaunchKernelGGL(k_net_input, dim3(grid_for_elems(c->C)), dim3(kBlock), 0, c->stream, c->n, r,
                     c->cdiag, sumsq, (double)c->n_liquid, rms_out, x0, flags);
}

void net_loss_grad(sim_ctx* c, const float* r, const float* Az, const double* dots,
                   const double* rms, __bf16* g11) {
  hipLaunchKernelGGL(k_loss_grad, dim3(grid_for_elems(c->C)), dim3(kBlock), 0, c->stream, c->n, r,
                     Az, c->cdiag, dots, rms, g11);
}

void net_upsum_mask(sim_ctx* c, int n_fine, int Cc, int Ct, const __bf16* T, const __bf16* P,
                    __bf16* out) {
  const int64_t e = (int64_t)(n_fine / 2) * (n_fine / 2) * (n_fine / 2) * Cc;
  hipLaunchKernelGGL(k_upsum_mask, dim3(grid_for_elems(e)), dim3(kBlock), 0, c->stream, n_fine, Cc,
                     Ct, T, P, out);
}

void net_skip_grad(sim_ctx* c, int n, int C, const __bf16* T, int Ct, int off, const __bf16* gp,
                   const __bf16* E, __bf16* out) {
  hipLaunchKernelGGL(k_skip_grad, dim3(grid_for_elems(cells(n) * C)), dim3(kBlock), 0, c->stream, n,
                     C, T, Ct, off, gp, E, out);
}

void net_pack_weights(sim_ctx* c, const float* W, int cin, int cout, int cin_p, int cout_p,
                      int cout_pd, __bf16* wf, __bf16* wd) {
  const int64_t e = (int64_t)cout_p * TAPS * cin_p + (wd ? (int64_t)cin * TAPS * cout_pd : 0);
  hipLaunchKernelGGL(k_pack_weights, dim3(grid_for_elems(e)), dim3(kBlock), 0, c->stream, W, cin,
                     cout, cin_p, cout_p, cout_pd, wf, wd);
}

void launch_scale_copy(sim_ctx* c, const float* a, float* out, int64_t count, float s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(grid_for_elems(count)), dim3(kBlock), 0, c->stream, a, out,
                     count, s);
}

void net_adam(sim_ctx* c, int64_t count, float* W, float* m, float* v, const float* dW,
              float inv_batch, float lr, int step) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_for_elems(count)), dim3(kBlock), 0, c->stream, count, W, m,
                     v, dW, inv_batch, lr, b1, b2, eps, bc1, bc2);
}

}  // namespace fs
