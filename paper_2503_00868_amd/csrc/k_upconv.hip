// Upsampled half of the U-Net's concatenating convolutions (decoder layers
// c7 and c9), evaluated on the coarse grid.
//
// The decoder convolves cat(up(coarse), skip) with a 3x3x3 kernel, where up
// is the nearest x2 upsampling.  For a fine voxel x = 2X + p (p its parity
// along one axis) a fine tap d in {-1, 0, 1} reads coarse voxel
// floor((p + d) / 2) + X: parity 0 sees offsets {-1, 0, 0}, parity 1
// {0, 0, +1}.  So per parity class (px, py, pz) the upsampled part is a
// 2x2x2 convolution of the coarse tensor, whose weights are sums of the
// fine taps that land on the same coarse voxel.  Evaluating it that way
// takes 8 instead of 27 taps per output (and reads the coarse tensor, not
// an 8x larger upsampled copy); the z-marching kernel then adds these fp16
// partial sums to its skip-channel convolution before the ReLU.
//
// MFMA mapping (16x16x32 bf16): M = 16 coarse voxels along X, N = 16 output
// channels, K = 32 coarse channels of one coarse tap offset.  A wave owns 4
// coarse rows and issues 8 parities x 8 taps x 4 rows MFMAs per K-step and
// 64 coarse voxels.
#include "common.h"
#include "ctx.h"
#include "net.h"

namespace fs {

typedef __bf16 bf16x8u __attribute__((ext_vector_type(8)));
typedef float f32x4u __attribute__((ext_vector_type(4)));

constexpr int UX = 16;   // coarse voxels per wave row (MFMA M)
constexpr int UR = 4;    // coarse rows per wave
constexpr int UY = 16;   // coarse rows per block (4 waves)
constexpr int UMAXZ = 128;  // coarse planes per block at most
// Launch sizes (measured at 256^3): the 64-channel layer stages 128 KB of
// weights per output group, so its blocks take runs of 4 coarse planes.
constexpr int UP_TARGET32 = 512;  // blocks for the 32-channel layer
constexpr int UP_TARGET64 = 256;  // blocks for the 64-channel layer
constexpr int UP_SB = 8;  // 16-byte weight words per thread and staging batch

// Coarse offset of fine tap d (-1, 0, 1) for parity q (0, 1).
__host__ __device__ constexpr int up_off(int q, int d) { return (q + d + 2) / 2 - 1; }

struct UpGrid {
  int zr, blocks;
};

// target: blocks to aim for.  A block stages its weights (8 x 8 x CC x 16
// bf16 per output group) once for its whole run, so wide layers, whose
// staging fills most of the LDS, take fewer blocks with longer runs.
static UpGrid up_grid(int nc, int target) {
  const int tiles = ((nc + UX - 1) / UX) * ((nc + UY - 1) / UY);
  int runs = (target + tiles - 1) / tiles;
  if (runs > nc) runs = nc;
  int zr = (nc + runs - 1) / runs;
  if (zr > UMAXZ) zr = UMAXZ;
  return UpGrid{zr, tiles * ((nc + zr - 1) / zr)};
}

// A block owns a 16 x 16 coarse tile and a run of zr coarse planes.  For each
// 16-channel output group the group's per-parity weights are staged in LDS
// once (8 x 8 x CC x 16 bf16), then every plane of the run is computed: per
// (ox, oz, K-step) a wave loads the 6 coarse rows its 4 output rows need and
// reuses them for the three oy offsets and every parity class using them.
template <int CC, int COUT>
__global__ void __launch_bounds__(kBlock)
    k_upconv(int n, int zr, const __bf16* __restrict__ coarse, const __bf16* __restrict__ weff,
             _Float16* __restrict__ out, const int* __restrict__ flags,
             const uint8_t* __restrict__ act) {
  if (flags && flags[F_DONE]) return;
  static_assert(CC % 32 == 0 && COUT % 16 == 0, "channel counts");
  constexpr int KS = CC / 32;
  constexpr int NT = COUT / 16;
  constexpr int WL = 8 * 8 * 16 * CC;  // bf16 of one output group's weights
  __shared__ __attribute__((aligned(16))) __bf16 wl[WL];
  __shared__ __attribute__((aligned(16))) _Float16 stage[4][UR * 2 * UX * 16];
  const int nc = n / 2;
  const int tx = (nc + UX - 1) / UX, ty = (nc + UY - 1) / UY;
  int tile, run;
  if (tx == ty) {
    net_block_of(blockIdx.x, gridDim.x, tx, tile, run);
  } else {
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    tile = lb % (tx * ty);
    run = lb / (tx * ty);
  }
  const int X0 = (tile % tx) * UX, Y0 = (tile / tx) * UY;
  const int Z0 = run * zr, Z1 = min(Z0 + zr, nc);
  if (Z0 >= nc) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, col = lane & 15;
  const int Yw = Y0 + UR * wv;
  // coarse tile-plane activity of the run, read once; a run with no live
  // plane ends here
  __shared__ uint8_t live_s[UMAXZ];
  if (act) {
    int any = 0;
    for (int t = threadIdx.x; t < Z1 - Z0; t += kBlock) {
      live_s[t] = act[(int64_t)(Z0 + t) * (tx * ty) + tile];
      any |= live_s[t];
    }
    if (!__syncthreads_or(any)) return;
  }

#pragma unroll 1
  for (int t = 0; t < NT; ++t) {
    __syncthreads();  // the previous group's weights are no longer read
    // LDS layout [p*8 + tap][c / 8][col][8]: the 16 lanes of one weight
    // fragment read consecutive 16-byte words (no bank conflicts)
    // (batches of UP_SB words per thread: all loads of a batch are issued
    // before its first store)
    static_assert((WL / 8) % (kBlock * UP_SB) == 0, "staging batches");
#pragma unroll 1
    for (int q0 = 0; q0 < WL / 8; q0 += kBlock * UP_SB) {
      uint4 tmp[UP_SB];
#pragma unroll
      for (int j = 0; j < UP_SB; ++j) {
        const int q = q0 + threadIdx.x + j * kBlock;
        const int cl = q % 16, kc = (q / 16) % (CC / 8), pt = q / (16 * (CC / 8));
        tmp[j] = *reinterpret_cast<const uint4*>(weff + ((int64_t)pt * COUT + t * 16 + cl) * CC + kc * 8);
      }
#pragma unroll
      for (int j = 0; j < UP_SB; ++j)
        *reinterpret_cast<uint4*>(wl + (int64_t)(q0 + threadIdx.x + j * kBlock) * 8) = tmp[j];
    }
    __syncthreads();

#pragma unroll 1
    for (int Z = Z0; Z < Z1; ++Z) {
      // coarse tile-plane known to be zero (with its halo): its fine outputs
      // are zero and stay as cleared (block-uniform)
      if (act && !live_s[Z - Z0]) continue;
      f32x4u acc[8][UR];
#pragma unroll
      for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int r = 0; r < UR; ++r) acc[p][r] = f32x4u{0.f, 0.f, 0.f, 0.f};

      // The (oz, ox, K-step) steps in order; each loads rows Yw-1 .. Yw+4 of
      // coarse plane Z+oz, shifted by ox.  The loads of step s+1 are issued
      // before the MFMAs of step s, and out-of-volume rows (loaded from a
      // clamped, valid address) are zeroed only when their step runs, so
      // that no wave waits for a load right after issuing it.
      constexpr int NSTEP = 9 * KS;
      auto load_step = [&](int s, uint4 (&raw)[UR + 2], uint32_t& okm) {
        const int oz = s / (3 * KS) - 1, ox = (s / KS) % 3 - 1, ks = s % KS;
        const int cx = X0 + col + ox, cz = Z + oz;
        const bool xz_ok = (unsigned)cx < (unsigned)nc && (unsigned)cz < (unsigned)nc;
        okm = 0u;
#pragma unroll
        for (int rr = 0; rr < UR + 2; ++rr) {
          const int cy = Yw + rr - 1;
          const bool ok = xz_ok && (unsigned)cy < (unsigned)nc;
          const int64_t v = ok ? (int64_t)cx + (int64_t)nc * (cy + (int64_t)nc * cz) : 0;
          raw[rr] = *reinterpret_cast<const uint4*>(coarse + v * CC + ks * 32 + 8 * g);
          okm |= ok ? 1u << rr : 0u;
        }
      };
      uint4 ra[UR + 2], rb[UR + 2];
      uint32_t oka, okb;
      load_step(0, ra, oka);
#pragma unroll
      for (int s = 0; s < NSTEP; ++s) {
        const int oz = s / (3 * KS) - 1, ox = (s / KS) % 3 - 1, ks = s % KS;
        uint4(&cur)[UR + 2] = (s & 1) ? rb : ra;
        const uint32_t okc = (s & 1) ? okb : oka;
        if (s + 1 < NSTEP) {
          if (s & 1)
            load_step(s + 1, ra, oka);
          else
            load_step(s + 1, rb, okb);
        }
        bf16x8u f[UR + 2];
#pragma unroll
        for (int rr = 0; rr < UR + 2; ++rr) {
          const uint4 val = (okc >> rr) & 1u ? cur[rr] : make_uint4(0u, 0u, 0u, 0u);
          f[rr] = *reinterpret_cast<const bf16x8u*>(&val);
        }
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
          for (int pz = 0; pz < 2; ++pz) {
            if (oz == (pz ? -1 : 1)) continue;  // parity 0 never reads +1, parity 1 never -1
#pragma unroll
            for (int py = 0; py < 2; ++py) {
              if (oy == (py ? -1 : 1)) continue;
#pragma unroll
              for (int px = 0; px < 2; ++px) {
                if (ox == (px ? -1 : 1)) continue;
                const int p = px + 2 * py + 4 * pz;
                const int tap =
                    (ox + (px ? 0 : 1)) + 2 * (oy + (py ? 0 : 1)) + 4 * (oz + (pz ? 0 : 1));
                const bf16x8u bw = *reinterpret_cast<const bf16x8u*>(
                    wl + (((p * 8 + tap) * (CC / 8) + ks * 4 + g) * 16 + col) * 8);
#pragma unroll
                for (int r = 0; r < UR; ++r)
                  acc[p][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[r + oy + 1], bw,
                                                                      acc[p][r], 0, 0, 0);
              }
            }
          }
      }

      // epilogue: one fine (y-parity, z-parity) slab at a time through LDS,
      // as UR rows of 2*UX fine voxels x 16 channels
#pragma unroll
      for (int pz = 0; pz < 2; ++pz)
#pragma unroll
        for (int py = 0; py < 2; ++py) {
          _Float16* st = stage[wv];
#pragma unroll
          for (int px = 0; px < 2; ++px)
#pragma unroll
            for (int r = 0; r < UR; ++r)
#pragma unroll
              for (int i = 0; i < 4; ++i)
                st[(r * 2 * UX + 2 * (4 * g + i) + px) * 16 + col] =
                    (_Float16)acc[px + 2 * py + 4 * pz][r][i];
          wave_sync();  // per-wave staging
          const int fz = 2 * Z + pz;
#pragma unroll
          for (int k = 0; k < (UR * 2 * UX * 2) / 64; ++k) {
            const int it = lane + 64 * k;  // (row, fx, half)
            const int half = it & 1, fx = (it >> 1) % (2 * UX), r = (it >> 1) / (2 * UX);
            const int gx = 2 * X0 + fx, gy = 2 * (Yw + r) + py;
            if (gx < n && gy < n) {
              const uint4 v = *reinterpret_cast<const uint4*>(st + (r * 2 * UX + fx) * 16 + half * 8);
              *reinterpret_cast<uint4*>(out + ((int64_t)gx + (int64_t)n * (gy + (int64_t)n * fz)) * COUT +
                                        t * 16 + half * 8) = v;
            }
          }
          wave_sync();
        }
    }
  }
}

// ------------------------------------------------- one parity class per wave
// The same upsampled half as k_upconv, for the fine level n (a multiple of
// 16) with 64 coarse channels and 32 outputs, organised like the coarse half
// of k_conv_cat: a block of 8 waves owns a 16 x 16 fine tile (8 x 8 coarse
// voxels) and a run of coarse planes Z, and computes the fine planes 2Z and
// 2Z + 1 of each.  Wave w takes parity class (px, py, pz) = bits 0, 1, 2 of
// w and keeps that class's summed weights (8 taps x 2 K-steps x 2 output
// groups = 32 fragments) in registers for the whole run.  The coarse planes,
// 10 x 10 with the halo and 64 channels, pass through a four-slot LDS ring
// (one barrier per plane: plane Z + 1 is stored while Z - 3 is no longer
// read).  The weights are the MFMA's A operand and the coarse voxels its B
// operand, so the result is [output channel][voxel] and each lane stores 4
// channels of one voxel (8 bytes of fp16) straight from its registers.  M
// block b (as in k_conv_cat) holds coarse rows b and b + 4 of the tile, so
// five B fragments per (tz, tx, K-step) feed sixteen MFMAs.
constexpr int UC_BLOCK = 512;
constexpr int UC_KT = 10;                  // ring plane edge (8 + halo)
constexpr int UC_KRV = UC_KT * UC_KT;      // 100 coarse voxels per ring plane
constexpr int UC_CC = 64, UC_COUT = 32;
constexpr int UC_SLOT = UC_KRV * UC_CC;    // bf16 per ring slot
constexpr int UC_ITEMS = UC_KRV * (UC_CC / 8);  // uint4 items per coarse plane
constexpr int UC_PF = (UC_ITEMS + UC_BLOCK - 1) / UC_BLOCK;
constexpr int UC_TARGET = 256;             // blocks to aim for (one per CU: 128 -> 65 us at
                                           // 256^3 against 512 blocks, 73 us)
constexpr int UC_MAXZ = 64;                // coarse planes per block at most

__global__ void __launch_bounds__(UC_BLOCK)
    k_upconv_cls(int n, int zr, const __bf16* __restrict__ coarse, const __bf16* __restrict__ weff,
                 _Float16* __restrict__ out, const int* __restrict__ flags,
                 const uint8_t* __restrict__ act) {
  if (flags && flags[F_DONE]) return;
  constexpr int KS = UC_CC / 32, NG = UC_COUT / 16;
  __shared__ __attribute__((aligned(16))) __bf16 ring[4 * UC_SLOT];
  __shared__ uint8_t live_s[2 * UC_MAXZ];
  const int nc = n >> 1, tpr = n / 16;
  int tile, run;
  net_block_of(blockIdx.x, gridDim.x, tpr, tile, run);
  const int X0 = (tile % tpr) * 8, Y0 = (tile / tpr) * 8;  // coarse tile origin
  const int Z0 = run * zr, Z1 = min(Z0 + zr, nc);
  if (Z0 >= nc) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, col = lane & 15;
  const int px = wave & 1, py = (wave >> 1) & 1, pz = wave >> 2;
  // fine tile-plane activity of the run's output planes (planes marked 0
  // are not read by the layer that adds these sums: not computed)
  if (act) {
    int any = 0;
    for (int t = threadIdx.x; t < 2 * (Z1 - Z0); t += UC_BLOCK) {
      live_s[t] = act[(int64_t)(2 * Z0 + t) * (tpr * tpr) + tile];
      any |= live_s[t];
    }
    if (!__syncthreads_or(any)) return;
  }

  // the class's weight fragments (A operand): lane (g, col) holds output
  // channel 16 grp + col, coarse channels 32 ks + 8 g .. + 7 of tap t
  const int p = px + 2 * py + 4 * pz;
  bf16x8u wr[NG][KS][8];
#pragma unroll
  for (int grp = 0; grp < NG; ++grp)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int t = 0; t < 8; ++t)
        wr[grp][ks][t] = *reinterpret_cast<const bf16x8u*>(
            weff + ((int64_t)(p * 8 + t) * UC_COUT + grp * 16 + col) * UC_CC + ks * 32 + 8 * g);

  // coarse plane loads: item it = 8 v + part (v a ring voxel, part 8 of the
  // 64 channels); ring layout [part][voxel][8]
  uint32_t koff[UC_PF];
  bool kok[UC_PF];
#pragma unroll
  for (int k = 0; k < UC_PF; ++k) {
    const int it = threadIdx.x + k * UC_BLOCK;
    const int cv = it >> 3, part = it & 7;
    const int cx = X0 - 1 + cv % UC_KT, cy = Y0 - 1 + cv / UC_KT;
    kok[k] = it < UC_ITEMS && (unsigned)cx < (unsigned)nc && (unsigned)cy < (unsigned)nc;
    koff[k] = kok[k] ? (uint32_t)(((int64_t)cx + (int64_t)nc * cy) * UC_CC + part * 8) : 0u;
  }
  const int64_t cplane = (int64_t)nc * nc * UC_CC;
  uint4 kpf[UC_PF];
  bool kpf_on = false;
  auto load_coarse = [&](int K) {
    kpf_on = (unsigned)K < (unsigned)nc;
    const __bf16* pc = coarse + (int64_t)(kpf_on ? K : 0) * cplane;
#pragma unroll
    for (int k = 0; k < UC_PF; ++k) kpf[k] = *reinterpret_cast<const uint4*>(pc + koff[k]);
  };
  auto store_coarse = [&](int K) {
    __bf16* slot = ring + ((K + 4) & 3) * UC_SLOT;
#pragma unroll
    for (int k = 0; k < UC_PF; ++k) {
      const int it = threadIdx.x + k * UC_BLOCK;
      if (it < UC_ITEMS) {
        const bool on = kpf_on && kok[k];
        uint4 v = kpf[k];
        // component selects (a select of whole vectors went through scratch)
        v.x = on ? v.x : 0u;
        v.y = on ? v.y : 0u;
        v.z = on ? v.z : 0u;
        v.w = on ? v.w : 0u;
        *reinterpret_cast<uint4*>(slot + ((it & 7) * UC_KRV + (it >> 3)) * 8) = v;
      }
    }
  };

  // prologue: planes Z0 - 1 and Z0 in the ring, Z0 + 1 in flight
  load_coarse(Z0 - 1);
  store_coarse(Z0 - 1);
  load_coarse(Z0);
  store_coarse(Z0);
  load_coarse(Z0 + 1);

#pragma unroll 1
  for (int Z = Z0; Z < Z1; ++Z) {
    // slot of Z + 1 last held Z - 3, read before the previous barrier
    store_coarse(Z + 1);
    __syncthreads();
    if (Z + 2 <= Z1) load_coarse(Z + 2);
    const int fz = 2 * Z + pz;
    if (act && !live_s[fz - 2 * Z0]) continue;  // wave-uniform

    f32x4u acc[NG][4];
#pragma unroll
    for (int grp = 0; grp < NG; ++grp)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[grp][b] = f32x4u{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tz = 0; tz < 2; ++tz) {
      // coarse plane offset tz - (pz ? 0 : 1)
      const __bf16* sl = ring + ((Z + tz - 1 + pz + 4) & 3) * UC_SLOT;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const __bf16* sp = sl + (ks * 4 + g) * UC_KRV * 8;
#pragma unroll
        for (int tx = 0; tx < 2; ++tx) {
          // ring column of coarse x offset tx - (px ? 0 : 1), row of row
          // offset e - (py ? 0 : 1), both with the halo's +1
          const int cx = (col & 7) + tx + px;
          bf16x8u B[5];
#pragma unroll
          for (int e = 0; e < 5; ++e) {
            const int cy = e + 4 * (col >> 3) + py;
            B[e] = *reinterpret_cast<const bf16x8u*>(sp + (cy * UC_KT + cx) * 8);
          }
#pragma unroll
          for (int ty = 0; ty < 2; ++ty)
#pragma unroll
            for (int grp = 0; grp < NG; ++grp)
#pragma unroll
              for (int b = 0; b < 4; ++b)
                acc[grp][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    wr[grp][ks][tx + 2 * ty + 4 * tz], B[b + ty], acc[grp][b], 0, 0, 0);
        }
      }
    }
    // lane (g, col): channels 16 grp + 4 g .. + 3 of coarse voxel (col % 8,
    // b + 4 (col / 8)) of the tile, i.e. fine voxel (2 x + px, 2 y + py, fz)
    const int fx = 2 * (X0 + (col & 7)) + px;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int fy = 2 * (Y0 + b + 4 * (col >> 3)) + py;
      if (fx >= n || fy >= n) continue;
      _Float16* o = out + ((int64_t)fx + (int64_t)n * (fy + (int64_t)n * fz)) * UC_COUT + 4 * g;
#pragma unroll
      for (int grp = 0; grp < NG; ++grp) {
        _Float16 h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) h[i] = (_Float16)acc[grp][b][i];
        *reinterpret_cast<uint2*>(o + grp * 16) = *reinterpret_cast<const uint2*>(h);
      }
    }
  }
}

// weff[p][tap][co][c] = sum of W[co][c][fine tap] over the fine taps of
// parity class p that read coarse offset tap; wskip = the skip channels in
// the forward layout [cout_p][28][cin - cc] (tap 27 and co >= cout zero).
__global__ void __launch_bounds__(kBlock)
    k_pack_split(const float* __restrict__ W, int cin, int cout, int cc, int cout_p,
                 __bf16* __restrict__ weff, __bf16* __restrict__ wskip) {
  const int cs = cin - cc;
  const int64_t ne = (int64_t)8 * 8 * cout * cc;
  const int64_t ns = (int64_t)cout_p * 28 * cs;
  for (int64_t q = blockIdx.x * (int64_t)kBlock + threadIdx.x; q < ne + ns;
       q += (int64_t)gridDim.x * kBlock) {
    if (q < ne) {
      const int c = (int)(q % cc);
      const int co = (int)((q / cc) % cout);
      const int tap = (int)((q / ((int64_t)cc * cout)) % 8);
      const int p = (int)(q / ((int64_t)cc * cout * 8));
      const int px = p & 1, py = (p >> 1) & 1, pz = p >> 2;
      const int tx = tap & 1, ty = (tap >> 1) & 1, tz = tap >> 2;
      float s = 0.f;
      for (int dz = -1; dz <= 1; ++dz) {
        if (up_off(pz, dz) != tz - (pz ? 0 : 1)) continue;
        for (int dy = -1; dy <= 1; ++dy) {
          if (up_off(py, dy) != ty - (py ? 0 : 1)) continue;
          for (int dx = -1; dx <= 1; ++dx) {
            if (up_off(px, dx) != tx - (px ? 0 : 1)) continue;
            s += W[((int64_t)co * cin + c) * 27 + (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)];
          }
        }
      }
      weff[q] = (__bf16)s;
    } else {
      const int64_t k = q - ne;
      const int ci = (int)(k % cs), tap = (int)((k / cs) % 28), co = (int)(k / ((int64_t)cs * 28));
      const float v = (co < cout && tap < 27) ? W[((int64_t)co * cin + cc + ci) * 27 + tap] : 0.f;
      wskip[k] = (__bf16)v;
    }
  }
}

bool net_upconv_cls(sim_ctx* c, int n, int cc, int cout, const __bf16* coarse, const __bf16* weff,
                    _Float16* out, const int* flags, const uint8_t* act) {
  if (cc != UC_CC || cout != UC_COUT || n % 16 != 0) return false;
  const int nc = n / 2, tiles = (n / 16) * (n / 16);
  int runs = (UC_TARGET + tiles - 1) / tiles;
  if (runs > nc) runs = nc;
  int zr = (nc + runs - 1) / runs;
  if (zr > UC_MAXZ) zr = UC_MAXZ;
  const int blocks = tiles * ((nc + zr - 1) / zr);
  hipLaunchKernelGGL(k_upconv_cls, dim3(blocks), dim3(UC_BLOCK), 0, c->stream, n, zr, coarse, weff,
                     out, flags, act);
  return true;
}

bool net_upconv(sim_ctx* c, int n, int cc, int cout, const __bf16* coarse, const __bf16* weff,
                _Float16* out, const int* flags, const uint8_t* act) {
  const UpGrid ug = up_grid(n / 2, cc == 64 ? UP_TARGET64 : UP_TARGET32);
  if (cc == 32 && cout == 16) {
    hipLaunchKernelGGL((k_upconv<32, 16>), dim3(ug.blocks), dim3(kBlock), 0, c->stream, n, ug.zr,
                       coarse, weff, out, flags, act);
    return true;
  }
  if (cc == 64 && cout == 32) {
    hipLaunchKernelGGL((k_upconv<64, 32>), dim3(ug.blocks), dim3(kBlock), 0, c->stream, n, ug.zr,
                       coarse, weff, out, flags, act);
    return true;
  }
  return false;
}

void net_pack_split(sim_ctx* c, const float* W, int cin, int cout, int cc, int cout_p,
                    __bf16* weff, __bf16* wskip) {
  const int64_t e = (int64_t)8 * 8 * cout * cc + (int64_t)cout_p * 28 * (cin - cc);
  const int64_t gb = (e + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_pack_split, dim3((unsigned)(gb < 4096 ? gb : 4096)), dim3(kBlock), 0,
                     c->stream, W, cin, cout, cc, cout_p, weff, wskip);
}

}  // namespace fs
