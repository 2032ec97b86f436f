// Output convolution of the learned preconditioner (c11, 16 -> 1 channels,
// 3x3x3) fused with the output map z = mask * rms * o.
//
// With one output channel the MFMA would waste 15 of its 16 columns, so this
// layer runs on the vector ALU: v_dot2 multiplies two bf16 channels and adds
// them to an fp32 sum, and its weight operand sits in scalar registers (the
// weights are the same for every lane).  A block owns a 16 x 16 tile of the
// xy-plane, one thread per column, and marches through its z-run one input
// plane at a time: plane p (with a one-voxel halo, 16 channels) is staged in
// LDS, and each thread adds its 3 x 3 neighbourhood of p to the three output
// planes it touches (p + 1, p, p - 1 through the kernel's z-slices 0, 1, 2).
// After plane p, output plane p - 1 is complete and is stored.  Every input
// voxel is read from memory once per block (plus the xy halo), the output is
// written once.
#include "block_or.h"
#include "common.h"
#include "ctx.h"
#include "net.h"

namespace fs {

typedef __bf16 bf16x2o __attribute__((ext_vector_type(2)));

constexpr int OT = 16;         // tile edge in x and y (one thread per column)
constexpr int OR = OT + 2;     // staged plane edge with halo
constexpr int ORV = OR * OR;   // 324 voxels per staged plane
constexpr int OITEMS = 2 * ORV;                       // 16-byte items per plane
constexpr int OPF = (OITEMS + kBlock - 1) / kBlock;   // items per thread
constexpr int OMAXC = 128;     // planes per block at most

struct OutGrid {
  int zc, blocks;
};

static OutGrid out_grid(int n) {
  const int tiles = ((n + OT - 1) / OT) * ((n + OT - 1) / OT);
  const int target = tiles >= 256 ? 4096 : 1024;
  int chunks = (target + tiles - 1) / tiles;
  if (chunks > n) chunks = n;
  int zc = (n + chunks - 1) / chunks;
  if (zc > OMAXC) zc = OMAXC;
  return OutGrid{zc, tiles * ((n + zc - 1) / zc)};
}

// D: c10's output [voxel][16] bf16.  w: the packed layer weights in the
// forward layout [16][28][16] bf16 (only output channel 0 is real), read as
// bf16 pairs: w2[tap * 8 + j] holds input channels 2j, 2j + 1 of tap
// dx + 3 dy + 9 dz.  act_in, act (nullable, both or neither): activity maps
// of D and of z.  qdot (nullable): the block also reduces z . qdot over its
// voxels into partials[blockIdx.x] (FP64), the flexible CG's z.q for beta,
// which then needs no pass of its own over z and q.
__global__ void __launch_bounds__(kBlock)
    k_conv_out(int n, int zc, const __bf16* __restrict__ D, const uint32_t* __restrict__ w2,
               float* __restrict__ z, const uint8_t* __restrict__ mask,
               const double* __restrict__ rms_p, const int* __restrict__ flags,
               const uint8_t* __restrict__ act_in, const uint8_t* __restrict__ act,
               const float* __restrict__ qdot, double* __restrict__ partials) {
  if (flags && flags[F_DONE]) return;
  // two staged planes, each as two 8-channel halves [half][voxel] (16 B per
  // voxel and half: the 16 lanes of a row read consecutive words)
  __shared__ uint4 ring[2][2][ORV];
  __shared__ __attribute__((aligned(16))) int votes[2][4];  // per ring slot
  __shared__ uint8_t live_s[OMAXC + 3], live_in_s[OMAXC + 3];

  const int tpr = (n + OT - 1) / OT;
  const int tiles = tpr * tpr;
  int tile, chunk;
  net_block_of(blockIdx.x, gridDim.x, tpr, tile, chunk);
  const int x0 = (tile % tpr) * OT, y0 = (tile / tpr) * OT;
  const int z0 = chunk * zc;
  const int z1 = min(z0 + zc, n);
  if (z0 >= n) {
    if (qdot && threadIdx.x == 0) partials[blockIdx.x] = 0.0;
    return;
  }
  const int tx = threadIdx.x & (OT - 1), ty = threadIdx.x / OT;
  const int x = x0 + tx, y = y0 + ty;
  const bool own = x < n && y < n;
  const int64_t nn = (int64_t)n * n;

  // tile-plane activity of planes z0-1 .. z1 (block-uniform): output planes
  // marked 0 in act store zeros, input planes marked 0 in act_in read as zero
  if (act)
    for (int t = threadIdx.x; t < z1 - z0 + 3; t += kBlock) {
      const int zi = z0 - 1 + t;
      const bool in = (unsigned)zi < (unsigned)n;
      live_s[t] = in ? act[(int64_t)zi * tiles + tile] : 0;
      live_in_s[t] = in ? act_in[(int64_t)zi * tiles + tile] : 0;
    }
  __syncthreads();
  auto live = [&](int zi) -> bool { return !act || live_s[zi - z0 + 1] != 0; };
  auto live_in = [&](int zi) -> bool { return !act || live_in_s[zi - z0 + 1] != 0; };

  // load items: it = threadIdx.x + k * kBlock is half (it & 1) of halo voxel
  // it >> 1; its byte offset within a plane of D is fixed for the block
  uint32_t ioff[OPF];
  bool iok[OPF];
#pragma unroll
  for (int k = 0; k < OPF; ++k) {
    const int it = threadIdx.x + k * kBlock;
    const int hv = it >> 1, h = it & 1;
    const int gx = x0 - 1 + hv % OR, gy = y0 - 1 + hv / OR;
    iok[k] = it < OITEMS && (unsigned)gx < (unsigned)n && (unsigned)gy < (unsigned)n;
    ioff[k] = iok[k] ? (uint32_t)((((int64_t)gx + (int64_t)n * gy) * 16 + h * 8) * 2) : 0u;
  }
  // the raw loads stay unmasked in registers while the current plane is
  // computed; items outside the grid (loaded from a valid clamped address)
  // and planes that read as zero are masked only when stored into the ring
  uint4 pf[OPF];
  bool pf_on = false;  // block-uniform
  auto load_plane = [&](int zi) {
    pf_on = live_in(zi) && (unsigned)zi < (unsigned)n;
    if (!pf_on) return;
    const char* pl = reinterpret_cast<const char*>(D) + zi * nn * 32;
#pragma unroll
    for (int k = 0; k < OPF; ++k) pf[k] = *reinterpret_cast<const uint4*>(pl + ioff[k]);
  };
  // returns whether this thread's part of the plane holds a non-zero bit
  auto store_plane = [&](int slot) -> int {
    const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
    uint32_t any = 0u;
#pragma unroll
    for (int k = 0; k < OPF; ++k) {
      const int it = threadIdx.x + k * kBlock;
      if (it < OITEMS) {
        const uint4 v = pf_on && iok[k] ? pf[k] : zero;
        ring[slot][it & 1][it >> 1] = v;
        any |= v.x | v.y | v.z | v.w;
      }
    }
    return any != 0u;
  };

  const float rms = (float)*rms_p;
  // sums of the output planes p - 1, p and p + 1 for the input plane p
  float s_lo = 0.f, s_mid = 0.f, s_hi = 0.f;
  double zq = 0.0;
  load_plane(z0 - 1);
  for (int p = z0 - 1; p <= z1; ++p) {
    const int slot = p & 1;
    // the slot was last read for plane p - 2, before the previous barrier
    const int nz = barrier_or(store_plane(slot), votes[slot]);
    // the output plane p - 1 is complete after this plane; its mask byte is
    // loaded (from a clamped address) ahead of the next plane's loads, so
    // that waiting for it does not wait for them
    const int o = p - 1;
    const bool out_here = o >= z0 && own;
    const bool want_m = out_here && live(o);
    const uint8_t m_raw = mask[want_m ? (int64_t)x + (int64_t)n * y + nn * o : 0];
    if (p + 1 <= z1) load_plane(p + 1);
    if (nz) {
      float c0 = 0.f, c1 = 0.f, c2 = 0.f;  // z-slices 0, 1, 2
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const int v = (ty + dy) * OR + tx + dx;
          const uint4 lo = ring[slot][0][v], hi = ring[slot][1][v];
          const uint32_t a[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
          const int t0 = dx + 3 * dy;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const bf16x2o av = __builtin_bit_cast(bf16x2o, a[j]);
            c0 = __builtin_amdgcn_fdot2_f32_bf16(av, __builtin_bit_cast(bf16x2o, w2[t0 * 8 + j]), c0, false);
            c1 = __builtin_amdgcn_fdot2_f32_bf16(av, __builtin_bit_cast(bf16x2o, w2[(t0 + 9) * 8 + j]), c1, false);
            c2 = __builtin_amdgcn_fdot2_f32_bf16(av, __builtin_bit_cast(bf16x2o, w2[(t0 + 18) * 8 + j]), c2, false);
          }
        }
      // input plane p is slice 0 of output p + 1, slice 1 of p, slice 2 of p - 1
      s_hi += c0;
      s_mid += c1;
      s_lo += c2;
    }
    if (out_here) {
      const int64_t idx = (int64_t)x + (int64_t)n * y + nn * o;
      const float zv = want_m && m_raw ? rms * s_lo : 0.f;
      z[idx] = zv;
      if (qdot && zv != 0.f) zq += (double)zv * (double)qdot[idx];
    }
    s_lo = s_mid;
    s_mid = s_hi;
    s_hi = 0.f;
  }
  if (qdot) {
    double v[1] = {zq};
    store_partials<1>(v, partials, blockIdx.x);
  }
}

int net_conv_out_blocks(int n) { return out_grid(n).blocks; }

void net_conv_out(sim_ctx* c, int n, const __bf16* D, const __bf16* w, float* z, const double* rms,
                  const int* flags, const uint8_t* act_in, const uint8_t* act, const float* qdot) {
  const OutGrid g = out_grid(n);
  hipLaunchKernelGGL(k_conv_out, dim3(g.blocks), dim3(kBlock), 0, c->stream, n, g.zc, D,
                     reinterpret_cast<const uint32_t*>(w), z, c->cdiag, rms, flags, act_in, act,
                     qdot, c->partials);
}

}  // namespace fs
