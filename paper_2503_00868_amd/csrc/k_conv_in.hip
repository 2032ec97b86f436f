// First convolution of the learned preconditioner fused with its input:
// x0 = (r / rms(r), liquid mask) -> c1 (2 -> 16 channels, 3x3x3), ReLU.
//
// With two input channels a K = 32 MFMA step holds 16 taps x 2 channels, so
// the 27 taps take 2 steps per output row (instead of 15 steps of 2 taps x 16
// zero-padded channels).  Lane (g, col) of the input operand carries voxel
// col and k = 8g + 2j + ch, i.e. tap 16s + 4g + j, channel ch: it gathers 4
// taps of the (r, mask) pair, 4 bytes each, from an LDS ring of three input
// planes (z-marching as in k_conv_zm.hip).  The weights are the MFMA's A
// operand and the input its B operand, so the result is [output channel]
// [voxel] and each lane stores 4 channels of one voxel straight from its
// registers.  r and the mask are read directly from the solver's arrays, so
// the 2-channel input tensor is never stored.
#include "block_or.h"
#include "common.h"
#include "ctx.h"
#include "net.h"

namespace fs {

typedef __bf16 bf16x8i __attribute__((ext_vector_type(8)));
typedef float f32x4i __attribute__((ext_vector_type(4)));

constexpr int IT = 16;          // output tile edge in x and y
constexpr int IR = IT + 2;      // ring plane edge with halo
constexpr int IRV = IR * IR;    // 324 voxels per ring plane
constexpr int IMAXC = 128;      // planes per block at most

struct InGrid {
  int zc, blocks;
};

static InGrid in_grid(int n) {
  const int tiles = ((n + IT - 1) / IT) * ((n + IT - 1) / IT);
  // shorter z-runs on large grids, as in k_conv_zm
  const int target = tiles >= 256 ? 4096 : 1024;
  int chunks = (target + tiles - 1) / tiles;
  if (chunks > n) chunks = n;
  int zc = (n + chunks - 1) / chunks;
  if (zc < 2) zc = 2;
  if (zc > IMAXC) zc = IMAXC;
  return InGrid{zc, tiles * ((n + zc - 1) / zc)};
}

// w: packed c1 weights [16][28][8] (forward layout, channels 0 = r, 1 = mask).
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
    k_conv_in(int n, int zc, const float* __restrict__ r, const uint8_t* __restrict__ cdiag,
              const double* __restrict__ sumsq, double n_liquid, double* __restrict__ rms_out,
              const __bf16* __restrict__ w, __bf16* __restrict__ out, const int* __restrict__ flags,
              const uint8_t* __restrict__ act, int* __restrict__ work) {
  if (flags && flags[F_DONE]) return;
  count_work(work);
  __shared__ uint32_t ring[4][IRV];  // (r / rms, mask) as two bf16; four slots as in k_conv_zm
  __shared__ __attribute__((aligned(16))) int votes[4][4];  // per ring slot
  const double rms = n_liquid > 0.0 ? sqrt(*sumsq / n_liquid) : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *rms_out = rms;
  const float inv = rms > 0.0 ? (float)(1.0 / rms) : 0.f;

  const int tpr = (n + IT - 1) / IT;
  const int tiles = tpr * tpr;
  int tile, chunk;
  net_block_of(blockIdx.x, gridDim.x, tpr, tile, chunk);
  const int x0 = (tile % tpr) * IT, y0 = (tile / tpr) * IT;
  const int z0 = chunk * zc;
  const int z1 = min(z0 + zc, n);
  if (z0 >= n) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, col = lane & 15;
  // tile-plane activity (block-uniform) of planes z0-1 .. z1+1, as in
  // k_conv_zm
  __shared__ uint8_t live_s[IMAXC + 3];
  if (act) {
    int any = 0;
    for (int t = threadIdx.x; t < z1 - z0 + 3; t += kBlock) {
      const int zi = z0 - 1 + t;
      live_s[t] = (unsigned)zi < (unsigned)n ? act[(int64_t)zi * tiles + tile] : 0;
      any |= t >= 1 && t <= z1 - z0 && live_s[t];
    }
    if (!__syncthreads_or(any)) return;  // no live output plane
  }
  auto live = [&](int zi) -> bool { return !act || live_s[zi - z0 + 1] != 0; };

  // weight fragments: step s, output channel col, k = 8g + i -> tap
  // 16s + 4g + i/2, channel i % 2
  bf16x8i bw[2];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int tap = 16 * s + 4 * g + (i >> 1);
      bw[s][i] = tap < 27 ? w[((int64_t)col * 28 + tap) * 8 + (i & 1)] : (__bf16)0.f;
    }

  // halo plane loads: 324 voxels, two per thread at most.  The raw values
  // stay in registers while the MFMAs of the current plane run; they are
  // converted only when stored into the ring.
  constexpr int PFI = (IRV + kBlock - 1) / kBlock;
  struct Raw {
    float r[PFI];
    uint8_t m[PFI];
    bool ok[PFI];
  };
  Raw ra, rb;  // two planes in flight
  auto load_plane = [&](int zi, Raw& o) {
    const bool on = live(zi);
#pragma unroll
    for (int k = 0; k < PFI; ++k) {
      const int hv = threadIdx.x + k * kBlock;
      const int gx = x0 - 1 + hv % IR, gy = y0 - 1 + hv / IR;
      const bool ok = on && hv < IRV && (unsigned)gx < (unsigned)n && (unsigned)gy < (unsigned)n &&
                      (unsigned)zi < (unsigned)n;
      // clamped address: always a valid load, the value is dropped when !ok
      const int64_t v = ok ? (int64_t)gx + (int64_t)n * (gy + (int64_t)n * zi) : 0;
      o.r[k] = r[v];
      o.m[k] = cdiag[v];
      o.ok[k] = ok;
    }
  };
  auto store_plane = [&](int zi, const Raw& o) -> int {
    uint32_t any = 0u;
#pragma unroll
    for (int k = 0; k < PFI; ++k) {
      const int hv = threadIdx.x + k * kBlock;
      if (hv < IRV) {
        __bf16 pair[2];
        // r is read on liquid cells only
        pair[0] = (__bf16)(o.ok[k] && o.m[k] ? o.r[k] * inv : 0.f);
        pair[1] = (__bf16)(o.ok[k] && o.m[k] ? 1.f : 0.f);
        const uint32_t bits = *reinterpret_cast<const uint32_t*>(pair);
        ring[(zi + 4) & 3][hv] = bits;
        any |= bits;
      }
    }
    return any != 0u;
  };

  // all-zero neighbourhoods (air far from liquid) skip the MFMAs, as in
  // k_conv_zm
  load_plane(z0 - 1, ra);
  int nz_m = barrier_or(store_plane(z0 - 1, ra), votes[(z0 + 3) & 3]);
  load_plane(z0, ra);
  int nz_0 = barrier_or(store_plane(z0, ra), votes[z0 & 3]);
  load_plane(z0 + 1, ra);
  if (z0 + 2 <= z1) load_plane(z0 + 2, rb);

  // one output plane: plane z+1 (held in cur) goes to the ring, and cur
  // takes the loads of plane z+3, which stay in flight for two planes
  // (the per-plane work of this layer is too small to hide one load
  // latency)
  auto plane_step = [&](int z, Raw& cur) {
    const int nz_p = barrier_or(store_plane(z + 1, cur), votes[(z + 1) & 3]);
    if (z + 3 <= z1) load_plane(z + 3, cur);
    const bool work = (nz_m | nz_0 | nz_p) != 0;
    nz_m = nz_0;
    nz_0 = nz_p;
    if (!live(z)) return;  // zero output plane: nothing to store

    f32x4i acc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) acc[a] = f32x4i{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < (work ? 2 : 0); ++s) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        bf16x8i af;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int tap = 16 * s + 4 * g + j;
          uint32_t pv = 0u;
          if (tap < 27) {
            const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;
            pv = ring[(z + 3 + dz) & 3][(4 * wv + a + dy) * IR + col + dx];
          }
          const __bf16* pp = reinterpret_cast<const __bf16*>(&pv);
          af[2 * j] = pp[0];
          af[2 * j + 1] = pp[1];
        }
        // weights as A, input as B: D = [output channel][voxel]
        acc[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[s], af, acc[a], 0, 0, 0);
      }
    }

    // ReLU, bf16: lane (g, col) holds channels 4g .. 4g+3 of voxel x0 + col
    // in row y0 + 4 wv + a and stores them as one 8-byte word (a wave's
    // store of one row is 512 contiguous bytes)
    const int x = x0 + col;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int y = y0 + 4 * wv + a;
      if (x >= n || y >= n) continue;
      __bf16 h[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) h[i] = (__bf16)(acc[a][i] > 0.f ? acc[a][i] : 0.f);
      const int64_t v = (int64_t)x + (int64_t)n * (y + (int64_t)n * z);
      *reinterpret_cast<uint2*>(out + v * 16 + 4 * g) = *reinterpret_cast<const uint2*>(h);
    }
  };
  for (int z = z0; z < z1; z += 2) {
    plane_step(z, ra);
    if (z + 1 < z1) plane_step(z + 1, rb);
  }
}

void net_conv_in(sim_ctx* c, const float* r, const double* sumsq, double* rms_out,
                 const __bf16* w, __bf16* out, const int* flags, const uint8_t* act,
                 int* work) {
  const InGrid g = in_grid(c->n);
  hipLaunchKernelGGL(k_conv_in, dim3(g.blocks), dim3(kBlock), 0, c->stream, c->n, g.zc, r,
                     c->cdiag, sumsq, (double)c->n_liquid, rms_out, w, out, flags, act, work);
}

}  // namespace fs
