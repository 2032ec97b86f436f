// Convolutions of the learned preconditioner's two finer levels (and their
// data gradients in training): a z-marching implicit GEMM on the 16x16x32
// bf16 MFMA of gfx950.
//
// A block owns a 16 x 16 tile of the xy-plane and walks a run of z-planes.
// The three input planes z-1, z, z+1 (with a one-voxel xy halo, 18 x 18
// voxels, all input channels) sit in an LDS ring; while the MFMAs work on
// plane z, the global loads of plane z+2 are already in flight, and they land
// in the ring slot that plane z-1 frees.  Each input voxel is thus read from
// memory about once per layer (1.27x for the xy halo), instead of once per
// overlapping 3-D tile.  A ring slot stores its plane as 8-channel
// sub-planes [part][voxel][8]: the lanes that read one fragment row then
// take consecutive 16-byte words, free of LDS bank conflicts.
//
// MFMA mapping (lane layout checked on the device): M = 16 output voxels
// along x, N = 16 output channels, K = 32 (the layers with 32 or more
// channels swap the operands, see k_conv_zm's epilogue; the A and B register
// layouts are the same, so only the output layout changes).  A K-step pairs
// two taps of one
// 16-channel chunk: lanes 0-31 carry tap T0, lanes 32-63 tap T1.  The 27
// taps form 15 steps per chunk:
//   steps 0-8    (dx, dy) = (s % 3, s / 3), T0 = dz 0, T1 = dz 1
//   steps 9-11   dy = s - 9,  T0 = (0, dy, 2), T1 = (1, dy, 2)
//   steps 12-14  dy = s - 12, T0 = (2, dy, 2), T1 = the zero tap
// Within a step group the A fragment depends only on halo row a + dy, so a
// wave (4 output rows) loads 6 fragments and issues 12 MFMAs per group.
// Weight fragments stay in registers for the whole block.
#include "block_or.h"
#include "common.h"
#include "ctx.h"
#include "net.h"

namespace fs {

typedef __bf16 bf16x8z __attribute__((ext_vector_type(8)));
typedef float f32x4z __attribute__((ext_vector_type(4)));

constexpr int ZT = 16;              // output tile edge in x and y
constexpr int ZR = ZT + 2;          // ring plane edge with halo
constexpr int ZRV = ZR * ZR;        // 324 voxels per ring plane
constexpr int ZSTEPS = 15;          // K-steps per 16-channel chunk
constexpr int ZTAPS = 28;           // packed taps per weight row (27 + zero)
constexpr int ZMAXC = 128;          // planes per block at most
// bf16 between the 8-channel parts of a ring plane.  A 16-byte LDS read
// whose 16-lane groups each read 256 contiguous bytes runs without bank
// conflicts on gfx950 only when the groups' start addresses differ by
// multiples of 256 B (measured: any other offset costs a two-way conflict),
// and a fragment read's lane groups differ by the part stride: the plane's
// 324 voxels (5184 B) padded to 5376 B.  The 16-channel kernels keep the
// tight stride: the padding's 1.5 KB would cost c10 its third block per CU.
// (The offsets are written as voxels times 8, the form the tight stride's
// register allocation was tuned in: c10 stays at 168 VGPRs, three waves per
// SIMD.)
constexpr int ZPS_PAD = ZRV * 8 + 96;
constexpr int ZPS_TIGHT = ZRV * 8;
template <int NCH>
constexpr int zm_ps() { return NCH >= 2 ? ZPS_PAD : ZPS_TIGHT; }

__device__ inline int zm_tap0(int s) {
  if (s < 9) return (s % 3) + 3 * (s / 3);              // dz 0
  if (s < 12) return 0 + 3 * (s - 9) + 18;              // (0, dy, 2)
  return 2 + 3 * (s - 12) + 18;                         // (2, dy, 2)
}
__device__ inline int zm_tap1(int s) {
  if (s < 9) return (s % 3) + 3 * (s / 3) + 9;          // dz 1
  if (s < 12) return 1 + 3 * (s - 9) + 18;              // (1, dy, 2)
  return 27;                                            // zero tap
}

// The 15 steps of a chunk in 5 groups whose A fragments share one halo
// column: groups k = 0-2 are dx = k with taps dz 0 | dz 1 (planes z-1 | z),
// group 3 is dz 2 with (dx 0 | dx 1), group 4 dz 2 with (dx 2 | zero).  Step
// of group k at row offset dy:
__device__ inline int zm_group_step(int k, int dy) {
  return k < 3 ? k + 3 * dy : 9 + 3 * (k - 3) + dy;
}

// The 6 halo rows (4 output rows + 2) of group gi = 5 q + k for this lane:
// 8 channels (half g & 1 of chunk q) at column col + the group's x offset,
// from the ring slots of planes z-1 (sm), z (s0) and z+1 (sp).
template <int PS>
__device__ inline void zm_load_group(int gi, const __bf16* sm, const __bf16* s0, const __bf16* sp,
                                     int wv, int g, int col, bf16x8z (&f)[6]) {
  const int q = gi / 5, k = gi % 5;
  const __bf16* base = k < 3 ? (g < 2 ? sm : s0) : sp;
  const int xo = k < 3 ? k : (k == 3 ? (g < 2 ? 0 : 1) : 2);
  base += (int64_t)(2 * q + (g & 1)) * (PS / 8) * 8;
#pragma unroll
  for (int r = 0; r < 6; ++r)
    f[r] = *reinterpret_cast<const bf16x8z*>(base + ((4 * wv + r) * ZR + col + xo) * 8);
}

struct ZmGrid {
  int tx, ty, zc, nchunks, blocks;
};

static ZmGrid zm_grid(int n) {
  ZmGrid g;
  g.tx = (n + ZT - 1) / ZT;
  g.ty = g.tx;
  const int tiles = g.tx * g.ty;
  // large levels take shorter z-runs: blocks whose tiles are mostly zero
  // (skipped) then balance against the busy ones
  const int target = tiles >= 256 ? 4096 : 1024;
  int chunks = (target + tiles - 1) / tiles;
  if (chunks > n) chunks = n;
  g.zc = (n + chunks - 1) / chunks;
  g.zc += g.zc & 1;  // even: a block owns whole plane pairs (fused 2x2x2 pooling)
  if (g.zc > ZMAXC) g.zc = ZMAXC;
  g.nchunks = (n + g.zc - 1) / g.zc;
  g.blocks = tiles * g.nchunks;
  return g;
}

// Layers with two 16-channel output groups and two input chunks (32 -> 32)
// split their output groups over two sets of four waves: 512 threads per
// block, wave w takes rows 4 (w % 4) .. + 3 for output group w / 4 and holds
// only that group's weight fragments, so that two waves fit per SIMD (both
// groups in one wave need 60 fragments and leave one wave per SIMD).  (The
// 16 -> 32 layer, with 30 fragments, measured slower split.)
template <int CIN, int COUT, int EPI>
__host__ __device__ constexpr bool zm_split() {
  return CIN == 32 && COUT == 32 &&
         (EPI == NET_EPI_RELU || EPI == NET_EPI_RAW || EPI == NET_EPI_MASKGRAD);
}
template <int CIN, int COUT, int EPI>
__host__ __device__ constexpr int zm_block() { return zm_split<CIN, COUT, EPI>() ? 2 * kBlock : kBlock; }

// CIN: channels held per ring voxel (multiple of 16; the source may have
// fewer, the rest is zero).  WS: channel stride of the packed weights.
// COUT: output channels (16 or 48).
template <int CIN, int WS, int COUT, int EPI>
__global__ void __launch_bounds__((zm_block<CIN, COUT, EPI>()))
    k_conv_zm(int n, int zc, NetSrc src, const __bf16* __restrict__ w, NetOut out,
              const int* __restrict__ flags) {
  if (flags && flags[F_DONE]) return;
  static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channel counts");
  static_assert(EPI != NET_EPI_RELU_ADD && EPI != NET_EPI_RELU_POOL, "k_conv_zm_pa");
  constexpr int NCH = CIN / 16;          // 16-channel chunks
  constexpr int NT = COUT / 16;          // 16-channel output groups
  constexpr int P8 = CIN / 8;            // 8-channel parts per voxel
  constexpr int ITEMS = ZRV * P8;        // uint4 items per ring plane
  constexpr bool SPLIT = zm_split<CIN, COUT, EPI>();
  constexpr int BLOCK = zm_block<CIN, COUT, EPI>();
  constexpr int NTW = SPLIT ? 1 : NT;    // output groups per wave
  constexpr int PF = (ITEMS + BLOCK - 1) / BLOCK;
  constexpr int PS = zm_ps<NCH>();    // bf16 per 8-channel part
  constexpr int SLOT = NCH * 2 * PS;   // bf16 per ring slot
  // four slots: the store of plane z+1 (slot (z+1) % 4, last read by the
  // compute of plane z-2) needs no barrier of its own
  __shared__ __attribute__((aligned(16))) __bf16 ring[4 * SLOT];
  __shared__ __attribute__((aligned(16))) int votes[4][8];  // per ring slot
  // Epilogue: layers with 32 or more channels on either side take the
  // weights as the MFMA's A operand (D = [output channel][voxel]) and store
  // straight from registers; 16 -> 16 layers take the input as A (D =
  // [voxel][output channel]) and store through an LDS stage, which measured
  // faster for them.
  constexpr bool DIRECT = NT > 1 || NCH > 1;
  constexpr int STAGE_BYTES = DIRECT ? 16 : 4 * 4 * ZT * COUT * 2;
  __shared__ __attribute__((aligned(16))) char stage_raw[STAGE_BYTES];
  __bf16* stage = reinterpret_cast<__bf16*>(stage_raw);

  const int tiles = ((n + ZT - 1) / ZT) * ((n + ZT - 1) / ZT);
  const int tpr = (n + ZT - 1) / ZT;
  int tile, chunk;
  net_block_of(blockIdx.x, gridDim.x, tpr, tile, chunk);
  const int x0 = (tile % tpr) * ZT, y0 = (tile / tpr) * ZT;
  const int z0 = chunk * zc;
  const int z1 = min(z0 + zc, n);
  if (z0 >= n) return;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wv = wave & 3, g = lane >> 4,
            col = lane & 15;
  const int tg = SPLIT ? wave >> 2 : 0;  // this wave's first output group
  // block-wide OR with one barrier (barrier_or, or its 8-wave form)
  auto bvote = [&](int v, int* slot) -> int {
    if constexpr (!SPLIT) {
      return barrier_or(v, slot);
    } else {
      const bool any = __ballot(v != 0) != 0ull;
      if (lane == 0) slot[wave] = any;
      __syncthreads();
      const int4 a = *reinterpret_cast<const int4*>(slot);
      const int4 b = *reinterpret_cast<const int4*>(slot + 4);
      return a.x | a.y | a.z | a.w | b.x | b.y | b.z | b.w;
    }
  };
  const int nc = n >> 1;

  // tile-plane activity (block-uniform): an output plane marked 0 in
  // out.act is neither computed nor stored, an input plane marked 0 in
  // src.act (else out.act) is read as zero.  The flags of planes z0-1 ..
  // z1+1 are read once, so that no plane's loads wait on a flag; a block
  // with no live output plane ends here (the output layer still stores its
  // zeros).
  __shared__ uint8_t live_s[ZMAXC + 3], live_in_s[ZMAXC + 3];
  if (out.act) {
    const uint8_t* act_in = src.act ? src.act : out.act;
    int any = 0;
    for (int t = threadIdx.x; t < z1 - z0 + 3; t += BLOCK) {
      const int zi = z0 - 1 + t;
      const bool in = (unsigned)zi < (unsigned)n;
      live_s[t] = in ? out.act[(int64_t)zi * tiles + tile] : 0;
      live_in_s[t] = in ? act_in[(int64_t)zi * tiles + tile] : 0;
      any |= t >= 1 && t <= z1 - z0 && live_s[t];
    }
    if (!__syncthreads_or(any) && EPI != NET_EPI_OUT) return;
  }
  auto live = [&](int zi) -> bool { return !out.act || live_s[zi - z0 + 1] != 0; };
  auto live_in = [&](int zi) -> bool { return !out.act || live_in_s[zi - z0 + 1] != 0; };

  // weight fragments: bw[q][s][t] for chunk q, step s, output group tg + t
  bf16x8z bw[NCH][ZSTEPS][NTW];
#pragma unroll
  for (int q = 0; q < NCH; ++q)
#pragma unroll
    for (int s = 0; s < ZSTEPS; ++s) {
      const int tap = g < 2 ? zm_tap0(s) : zm_tap1(s);
      const int ci = q * 16 + (g & 1) * 8;
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        bf16x8z v;
        if (ci < WS) {
          v = *reinterpret_cast<const bf16x8z*>(w + ((int64_t)((tg + t) * 16 + col) * ZTAPS + tap) * WS + ci);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = (__bf16)0.f;
        }
        bw[q][s][t] = v;
      }
    }

  // Load items of this thread: item it = threadIdx.x + k * BLOCK holds 8
  // channels (part p) of halo voxel hv.  Its byte offset within one plane of
  // its source is fixed for the block; only the (uniform) plane offset moves
  // with z.  src: 0 none (outside the volume or channel padding), 1 a, 2 b.
  uint32_t ioff[PF];
  uint8_t isrc[PF];
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const int it = threadIdx.x + k * BLOCK;
    const int hv = it / P8, p = it - hv * P8;
    const int gx = x0 - 1 + hv % ZR, gy = y0 - 1 + hv / ZR;
    const int c = p * 8;
    ioff[k] = 0u;
    isrc[k] = 0;
    if (it < ITEMS && (unsigned)gx < (unsigned)n && (unsigned)gy < (unsigned)n) {
      if (c < src.ca) {
        const int64_t v = src.up ? (int64_t)(gx >> 1) + (int64_t)nc * (gy >> 1) : (int64_t)gx + (int64_t)n * gy;
        ioff[k] = (uint32_t)((v * src.ca + c) * 2);
        isrc[k] = 1;
      } else if (c < src.ca + src.cb) {
        ioff[k] = (uint32_t)((((int64_t)gx + (int64_t)n * gy) * src.cb + (c - src.ca)) * 2);
        isrc[k] = 2;
      }
    }
  }
  const int64_t plane_a = (int64_t)(src.up ? nc : n) * (src.up ? nc : n) * src.ca * 2;
  const int64_t plane_b = (int64_t)n * n * src.cb * 2;

  // global -> registers for input plane zi.  The raw loads stay unmasked
  // while the MFMAs of the current plane run: items with no source (outside
  // the volume, channel padding; loaded from a valid clamped offset) and
  // planes known to be zero are masked only when stored into the ring.  A
  // select right after the load would make the wave wait for it there.
  uint4 pf[PF];
  auto load_plane = [&](int zi) {
    if (!live_in(zi) || (unsigned)zi >= (unsigned)n) {
#pragma unroll
      for (int k = 0; k < PF; ++k) pf[k] = make_uint4(0u, 0u, 0u, 0u);
      return;
    }
    const char* pa = reinterpret_cast<const char*>(src.a) + (int64_t)(src.up ? zi >> 1 : zi) * plane_a;
    if (!src.b) {
#pragma unroll
      for (int k = 0; k < PF; ++k) pf[k] = *reinterpret_cast<const uint4*>(pa + ioff[k]);
    } else {
      const char* pb = reinterpret_cast<const char*>(src.b) + (int64_t)zi * plane_b;
#pragma unroll
      for (int k = 0; k < PF; ++k)
        pf[k] = *reinterpret_cast<const uint4*>((isrc[k] == 2 ? pb : pa) + ioff[k]);
    }
  };
  // stores the prefetched plane; returns whether this thread's part of it
  // holds any non-zero bit
  auto store_plane = [&](int zi) -> int {
    const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
    __bf16* slot = ring + ((zi + 4) & 3) * SLOT;
    uint32_t any = 0u;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int it = threadIdx.x + k * BLOCK;
      if (it < ITEMS) {
        const int hv = it / P8, p = it - hv * P8;
        const uint4 v = isrc[k] ? pf[k] : zero;
        *reinterpret_cast<uint4*>(slot + (p * (PS / 8) + hv) * 8) = v;
        any |= v.x | v.y | v.z | v.w;
      }
    }
    return any != 0u;
  };

  // Output mapping (the MFMA takes the weights as A and the input as B, so
  // D is [output channel][voxel]): lane (g, col) holds channels 4g .. 4g+3
  // of output group t for voxel x0 + col of row y0 + 4 wv + a, and stores
  // them as one 8-byte word; a wave's store of one row is 512 contiguous
  // bytes.  No staging through LDS.
  const int ox = x0 + col;
  const bool ox_ok = ox < n;
  // staged epilogue: lane l owns voxel (x0 + l % 16, row l / 16) of its
  // wave's rows for the output layer's mask and store
  const int oy = y0 + 4 * wv + (lane >> 4);
  const bool own = ox < n && oy < n;
  const int64_t nn = (int64_t)n * n;
  const float rms_f = EPI == NET_EPI_OUT ? (float)*out.rms : 0.f;
  auto vox = [&](int a, int z) -> int64_t { return (int64_t)ox + (int64_t)n * (y0 + 4 * wv + a) + nn * z; };
  auto row_ok = [&](int a) -> bool { return ox_ok && y0 + 4 * wv + a < n; };
  auto pack4 = [](float f0, float f1, float f2, float f3) -> uint2 {
    __bf16 h[4] = {(__bf16)f0, (__bf16)f1, (__bf16)f2, (__bf16)f3};
    return *reinterpret_cast<const uint2*>(h);
  };

  // A bias-free network maps an all-zero input neighbourhood to zero, so the
  // MFMAs of a plane are skipped when planes z-1, z, z+1 of the tile (with
  // halo) are all zero; the flags come with the barrier after each store.
  load_plane(z0 - 1);
  int nz_m = bvote(store_plane(z0 - 1), votes[(z0 + 3) & 3]);
  load_plane(z0);
  int nz_0 = bvote(store_plane(z0), votes[z0 & 3]);
  load_plane(z0 + 1);

  // one output plane: the prefetched plane z+1 goes to the ring, plane z+2
  // is loaded while the MFMAs of plane z run
  auto plane_step = [&](int z) {
    const int nz_p = bvote(store_plane(z + 1), votes[(z + 1) & 3]);
    if (z + 2 <= z1) load_plane(z + 2);
    const bool work = (nz_m | nz_0 | nz_p) != 0;
    nz_m = nz_0;
    nz_0 = nz_p;

    // an output plane known to be zero is neither computed nor stored; the
    // output layer stores zeros
    if (!live(z)) {
      if (EPI == NET_EPI_OUT && DIRECT && g == 0) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
          if (row_ok(a)) out.f32[vox(a, z)] = 0.f;
      }
      if (EPI == NET_EPI_OUT && !DIRECT && own) out.f32[(int64_t)ox + (int64_t)n * oy + nn * z] = 0.f;
      return;
    }

    // issued before the MFMAs, consumed in the epilogue
    uint8_t mk[4] = {0, 0, 0, 0};
    uint8_t own_mask = 0;
    if (EPI == NET_EPI_OUT && DIRECT && g == 0) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (row_ok(a)) mk[a] = out.mask[vox(a, z)];
    }
    if (EPI == NET_EPI_OUT && !DIRECT && own)
      own_mask = out.mask[(int64_t)ox + (int64_t)n * oy + nn * z];

    f32x4z acc[4][NTW];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int t = 0; t < NTW; ++t) acc[a][t] = f32x4z{0.f, 0.f, 0.f, 0.f};

    const __bf16* sm = ring + ((z + 3) & 3) * SLOT;  // plane z-1 (dz = 0)
    const __bf16* s0 = ring + (z & 3) * SLOT;        // plane z   (dz = 1)
    const __bf16* sp = ring + ((z + 1) & 3) * SLOT;  // plane z+1 (dz = 2)
    if (work) {
      // the 5 step groups of each chunk in turn, the fragments of group gi + 1
      // read from LDS before the MFMAs of group gi are issued
      bf16x8z fa[6], fb[6];
      zm_load_group<PS>(0, sm, s0, sp, wv, g, col, fa);
      __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
#pragma unroll
      for (int gi = 0; gi < 5 * NCH; ++gi) {
        bf16x8z(&f)[6] = (gi & 1) ? fb : fa;
        if (gi + 1 < 5 * NCH) zm_load_group<PS>(gi + 1, sm, s0, sp, wv, g, col, (gi & 1) ? fa : fb);
        const int q = gi / 5, k = gi % 5;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const int st = zm_group_step(k, dy);
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int t = 0; t < NTW; ++t)
              acc[a][t] = DIRECT ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[q][st][t], f[a + dy],
                                                                           acc[a][t], 0, 0, 0)
                                 : __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[a + dy], bw[q][st][t],
                                                                           acc[a][t], 0, 0, 0);
        }
        // keep that order in the schedule: the next group's 6 LDS reads, then
        // this group's MFMAs
        if (gi + 1 < 5 * NCH) __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 12 * NTW, 0);
      }
    }

    if constexpr (DIRECT) {
      if (EPI == NET_EPI_OUT) {
        // channel 0 is row 0 of D: lanes g = 0, element 0
        if (g == 0) {
#pragma unroll
          for (int a = 0; a < 4; ++a)
            if (row_ok(a)) out.f32[vox(a, z)] = mk[a] ? rms_f * acc[a][0][0] : 0.f;
        }
        return;
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const bool ok = row_ok(a);
        const int64_t v = vox(a, z);
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
          const int64_t e = v * COUT + (tg + t) * 16 + 4 * g;  // element of channel 4g
          float f[4] = {acc[a][t][0], acc[a][t][1], acc[a][t][2], acc[a][t][3]};
          if (EPI == NET_EPI_RELU) {
#pragma unroll
            for (int i = 0; i < 4; ++i) f[i] = f[i] > 0.f ? f[i] : 0.f;
          }
          uint2 o = pack4(f[0], f[1], f[2], f[3]);
          if (EPI == NET_EPI_MASKGRAD) {
            // the gradient passes where the post-activation is positive
            uint2 pm = make_uint2(0u, 0u);
            if (ok) pm = *reinterpret_cast<const uint2*>(out.relu_of + e);
            const uint32_t* pw = reinterpret_cast<const uint32_t*>(&pm);
            uint32_t* ow = reinterpret_cast<uint32_t*>(&o);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              const uint32_t lo = pw[j] & 0xffffu, hi = pw[j] >> 16;
              const uint32_t keep_lo = (lo != 0u && !(lo & 0x8000u)) ? 0xffffu : 0u;
              const uint32_t keep_hi = (hi != 0u && !(hi & 0x8000u)) ? 0xffff0000u : 0u;
              ow[j] &= (keep_lo | keep_hi);
            }
          }
          if (ok) *reinterpret_cast<uint2*>(out.bf + e) = o;
        }
      }
    } else {
      // epilogue: rows y0 + 4 wv + a, voxels x0 + 4 g + i, channel t*16 + col
      if (EPI == NET_EPI_OUT) {
        // channel 0 (lanes with col 0) through LDS: lane l then stores voxel
        // (row l / 16, x l % 16) of the wave's rows, coalesced
        float* so = reinterpret_cast<float*>(stage) + wv * 64;
        if (col == 0) {
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) so[a * 16 + 4 * g + i] = acc[a][0][i];
        }
        wave_sync();  // per-wave staging
        if (own)
          out.f32[(int64_t)ox + (int64_t)n * (oy + (int64_t)n * z)] =
              own_mask ? rms_f * so[lane] : 0.f;
        return;
      }
      __bf16* st = stage + wv * (4 * ZT * COUT);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float v = acc[a][t][i];
            if (EPI == NET_EPI_RELU) v = v > 0.f ? v : 0.f;
            st[((a * ZT) + 4 * g + i) * COUT + t * 16 + col] = (__bf16)v;
          }
      wave_sync();  // per-wave staging
      constexpr int PV = COUT / 8;
#pragma unroll
      for (int k = 0; k < (4 * ZT * PV + 63) / 64; ++k) {
        const int it = lane + 64 * k;
        if (it >= 4 * ZT * PV) break;
        const int lv = it / PV, part = it - lv * PV;
        const int a = lv / ZT, xl = lv % ZT;
        const int x = x0 + xl, y = y0 + 4 * wv + a;
        if (x >= n || y >= n) continue;
        const int64_t v = (int64_t)x + (int64_t)n * (y + (int64_t)n * z);
        uint4 val = *reinterpret_cast<const uint4*>(st + lv * COUT + part * 8);
        if (EPI == NET_EPI_MASKGRAD) {
          const uint4 pm = *reinterpret_cast<const uint4*>(out.relu_of + v * COUT + part * 8);
          const uint32_t* pw = reinterpret_cast<const uint32_t*>(&pm);
          uint32_t* vw = reinterpret_cast<uint32_t*>(&val);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint32_t lo = pw[e] & 0xffffu, hi = pw[e] >> 16;
            const uint32_t keep_lo = (lo != 0u && !(lo & 0x8000u)) ? 0xffffu : 0u;
            const uint32_t keep_hi = (hi != 0u && !(hi & 0x8000u)) ? 0xffff0000u : 0u;
            vw[e] &= (keep_lo | keep_hi);
          }
        }
        *reinterpret_cast<uint4*>(out.bf + v * COUT + part * 8) = val;
      }
    }
  };
  for (int z = z0; z < z1; ++z) plane_step(z);
}

// Variant for the layers with the add and pool epilogues: the plane loads
// do their address arithmetic per item and plane, and the epilogue stages
// through LDS.  The same source compiled into the kernel below (whose
// streamlined loads suit the other epilogues) measured 10-35% slower for
// these two epilogues, so they keep this form.
// CIN: channels held per ring voxel (multiple of 16; the source may have
// fewer, the rest is zero).  WS: channel stride of the packed weights.
// COUT: output channels (16 or 48).
// The 16 -> 16 pool layer runs at three waves per SIMD (its LDS allows three
// blocks per CU; the register limit costs a few spilled values): 296 -> 267 us
// for c2 at 256^3.  The add layer does not fit that limit.
// The 32 -> 32 layers with these epilogues split their output groups over
// two sets of four waves as k_conv_zm does (the two waves of a row group meet
// at a block barrier before the epilogue reads both halves of the stage).
template <int CIN, int COUT, int EPI>
__host__ __device__ constexpr bool zm_pa_split() {
  return CIN == 32 && COUT == 32 && (EPI == NET_EPI_RELU_POOL || EPI == NET_EPI_RELU_ADD);
}
template <int CIN, int COUT, int EPI>
__host__ __device__ constexpr int zm_pa_block() { return zm_pa_split<CIN, COUT, EPI>() ? 2 * kBlock : kBlock; }
template <int CIN, int COUT, int EPI>
constexpr int zm_pa_min_waves() {
  return CIN == 16 && COUT == 16 && EPI == NET_EPI_RELU_POOL ? 3 : (zm_pa_split<CIN, COUT, EPI>() ? 2 : 1);
}

template <int CIN, int WS, int COUT, int EPI>
__global__ void __launch_bounds__((zm_pa_block<CIN, COUT, EPI>()))
    __attribute__((amdgpu_waves_per_eu(zm_pa_min_waves<CIN, COUT, EPI>())))
    k_conv_zm_pa(int n, int zc, NetSrc src, const __bf16* __restrict__ w, NetOut out,
              const int* __restrict__ flags) {
  if (flags && flags[F_DONE]) return;
  static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channel counts");
  constexpr int NCH = CIN / 16;          // 16-channel chunks
  constexpr int NT = COUT / 16;          // 16-channel output groups
  constexpr int P8 = CIN / 8;            // 8-channel parts per voxel
  constexpr int ITEMS = ZRV * P8;        // uint4 items per ring plane
  constexpr bool SPLIT = zm_pa_split<CIN, COUT, EPI>();
  constexpr int BLOCK = zm_pa_block<CIN, COUT, EPI>();
  constexpr int NTW = SPLIT ? 1 : NT;    // output groups per wave
  constexpr int PF = (ITEMS + BLOCK - 1) / BLOCK;
  constexpr int PS = zm_ps<NCH>();    // bf16 per 8-channel part
  constexpr int SLOT = NCH * 2 * PS;   // bf16 per ring slot
  // four slots: the store of plane z+1 (slot (z+1) % 4, last read by the
  // compute of plane z-2) needs no barrier of its own
  __shared__ __attribute__((aligned(16))) __bf16 ring[4 * SLOT];
  __shared__ __attribute__((aligned(16))) int votes[4][8];  // per ring slot
  constexpr int STAGE_BYTES = 4 * 4 * ZT * COUT * (EPI == NET_EPI_RELU_ADD ? 4 : 2);
  __shared__ __attribute__((aligned(16))) char stage_raw[STAGE_BYTES];
  __bf16* stage = reinterpret_cast<__bf16*>(stage_raw);

  const int tiles = ((n + ZT - 1) / ZT) * ((n + ZT - 1) / ZT);
  const int tpr = (n + ZT - 1) / ZT;
  int tile, chunk;
  net_block_of(blockIdx.x, gridDim.x, tpr, tile, chunk);
  const int x0 = (tile % tpr) * ZT, y0 = (tile / tpr) * ZT;
  const int z0 = chunk * zc;
  const int z1 = min(z0 + zc, n);
  if (z0 >= n) return;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wv = wave & 3, g = lane >> 4,
            col = lane & 15;
  const int tg = SPLIT ? wave >> 2 : 0;  // this wave's first output group
  auto bvote = [&](int v, int* slot) -> int {
    if constexpr (!SPLIT) {
      return barrier_or(v, slot);
    } else {
      const bool any = __ballot(v != 0) != 0ull;
      if (lane == 0) slot[wave] = any;
      __syncthreads();
      const int4 a = *reinterpret_cast<const int4*>(slot);
      const int4 b = *reinterpret_cast<const int4*>(slot + 4);
      return a.x | a.y | a.z | a.w | b.x | b.y | b.z | b.w;
    }
  };
  const int nc = n >> 1;

  // tile-plane activity (block-uniform): an output plane marked 0 in
  // out.act is neither computed nor stored, an input plane marked 0 in
  // src.act (else out.act) is read as zero.  The flags of planes z0-1 ..
  // z1+1 are read once, so that no plane's loads wait on a flag; a block
  // with no live output plane ends here (the output layer still stores its
  // zeros).
  __shared__ uint8_t live_s[ZMAXC + 3], live_in_s[ZMAXC + 3];
  if (out.act) {
    const uint8_t* act_in = src.act ? src.act : out.act;
    int any = 0;
    for (int t = threadIdx.x; t < z1 - z0 + 3; t += BLOCK) {
      const int zi = z0 - 1 + t;
      const bool in = (unsigned)zi < (unsigned)n;
      live_s[t] = in ? out.act[(int64_t)zi * tiles + tile] : 0;
      live_in_s[t] = in ? act_in[(int64_t)zi * tiles + tile] : 0;
      any |= t >= 1 && t <= z1 - z0 && live_s[t];
    }
    if (!__syncthreads_or(any) && EPI != NET_EPI_OUT) return;
  }
  auto live = [&](int zi) -> bool { return !out.act || live_s[zi - z0 + 1] != 0; };
  auto live_in = [&](int zi) -> bool { return !out.act || live_in_s[zi - z0 + 1] != 0; };

  // weight fragments: bw[q][s][t] for chunk q, step s, output group t
  bf16x8z bw[NCH][ZSTEPS][NTW];
#pragma unroll
  for (int q = 0; q < NCH; ++q)
#pragma unroll
    for (int s = 0; s < ZSTEPS; ++s) {
      const int tap = g < 2 ? zm_tap0(s) : zm_tap1(s);
      const int ci = q * 16 + (g & 1) * 8;
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        bf16x8z v;
        if (ci < WS) {
          v = *reinterpret_cast<const bf16x8z*>(w + ((int64_t)((tg + t) * 16 + col) * ZTAPS + tap) * WS + ci);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = (__bf16)0.f;
        }
        bw[q][s][t] = v;
      }
    }

  // plane loads as in k_conv_zm: per-item offsets fixed for the block, raw
  // loads from valid clamped offsets, masked when stored into the ring
  uint32_t ioff[PF];
  uint8_t isrc[PF];
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const int it = threadIdx.x + k * BLOCK;
    const int hv = it / P8, p = it - hv * P8;
    const int gx = x0 - 1 + hv % ZR, gy = y0 - 1 + hv / ZR;
    const int c = p * 8;
    ioff[k] = 0u;
    isrc[k] = 0;
    if (it < ITEMS && (unsigned)gx < (unsigned)n && (unsigned)gy < (unsigned)n) {
      if (c < src.ca) {
        const int64_t v = src.up ? (int64_t)(gx >> 1) + (int64_t)nc * (gy >> 1) : (int64_t)gx + (int64_t)n * gy;
        ioff[k] = (uint32_t)((v * src.ca + c) * 2);
        isrc[k] = 1;
      } else if (c < src.ca + src.cb) {
        ioff[k] = (uint32_t)((((int64_t)gx + (int64_t)n * gy) * src.cb + (c - src.ca)) * 2);
        isrc[k] = 2;
      }
    }
  }
  const int64_t plane_a = (int64_t)(src.up ? nc : n) * (src.up ? nc : n) * src.ca * 2;
  const int64_t plane_b = (int64_t)n * n * src.cb * 2;
  uint4 pf[PF];
  auto load_plane = [&](int zi) {
    if (!live_in(zi) || (unsigned)zi >= (unsigned)n) {
#pragma unroll
      for (int k = 0; k < PF; ++k) pf[k] = make_uint4(0u, 0u, 0u, 0u);
      return;
    }
    const char* pa = reinterpret_cast<const char*>(src.a) + (int64_t)(src.up ? zi >> 1 : zi) * plane_a;
    if (!src.b) {
#pragma unroll
      for (int k = 0; k < PF; ++k) pf[k] = *reinterpret_cast<const uint4*>(pa + ioff[k]);
    } else {
      const char* pb = reinterpret_cast<const char*>(src.b) + (int64_t)zi * plane_b;
#pragma unroll
      for (int k = 0; k < PF; ++k)
        pf[k] = *reinterpret_cast<const uint4*>((isrc[k] == 2 ? pb : pa) + ioff[k]);
    }
  };
  // stores the prefetched plane; returns whether this thread's part of it
  // holds any non-zero bit
  auto store_plane = [&](int zi) -> int {
    const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
    __bf16* slot = ring + ((zi + 4) & 3) * SLOT;
    uint32_t any = 0u;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int it = threadIdx.x + k * BLOCK;
      if (it < ITEMS) {
        const int hv = it / P8, p = it - hv * P8;
        const uint4 v = isrc[k] ? pf[k] : zero;
        *reinterpret_cast<uint4*>(slot + (p * (PS / 8) + hv) * 8) = v;
        any |= v.x | v.y | v.z | v.w;
      }
    }
    return any != 0u;
  };

  // output layer: rms once per block; each lane owns one voxel of its wave's
  // 4 x 16 output rows for the mask and the store
  const float rms_f = EPI == NET_EPI_OUT ? (float)*out.rms : 0.f;
  const int oy = y0 + 4 * wv + (lane >> 4), ox = x0 + (lane & 15);
  const bool own = ox < n && oy < n;

  // A bias-free network maps an all-zero input neighbourhood to zero, so the
  // MFMAs of a plane are skipped when planes z-1, z, z+1 of the tile (with
  // halo) are all zero; the flags come with the barrier after each store.
  load_plane(z0 - 1);
  int nz_m = bvote(store_plane(z0 - 1), votes[(z0 + 3) & 3]);
  load_plane(z0);
  int nz_0 = bvote(store_plane(z0), votes[z0 & 3]);
  load_plane(z0 + 1);
  float pacc[8];  // RELU_POOL: sums of the even plane of a z pair
#pragma unroll
  for (int e = 0; e < 8; ++e) pacc[e] = 0.f;

  // one output plane: the prefetched plane z+1 goes to the ring, plane z+2
  // is loaded while the MFMAs of plane z run
  auto plane_step = [&](int z) {
    const int nz_p = bvote(store_plane(z + 1), votes[(z + 1) & 3]);
    if (z + 2 <= z1) load_plane(z + 2);
    const bool work = (nz_m | nz_0 | nz_p) != 0;
    nz_m = nz_0;
    nz_0 = nz_p;

    // an output plane known to be zero is neither computed nor stored (a
    // pooled pair is live if either plane is); the output layer stores zeros
    if (!live(z) && !(EPI == NET_EPI_RELU_POOL && live(z ^ 1))) {
      if (EPI == NET_EPI_OUT && own) out.f32[(int64_t)ox + (int64_t)n * (oy + (int64_t)n * z)] = 0.f;
      return;
    }

    // issued before the MFMAs, consumed in the epilogue
    uint8_t own_mask = 0;
    if (EPI == NET_EPI_OUT && own)
      own_mask = out.mask[(int64_t)ox + (int64_t)n * (oy + (int64_t)n * z)];
    // RELU_ADD: the fp16 partial sums of this plane's epilogue items (item
    // it = lane + 64 k: voxel it / PV8 of the wave's rows, 8 channels part
    // it % PV8), from a clamped address where the item is outside
    constexpr int PV8 = COUT / 8;
    constexpr int ADD_K = EPI == NET_EPI_RELU_ADD ? (4 * ZT * PV8 + 63) / 64 : 1;
    // items per wave: a split pair shares its row group's items
    constexpr bool ADD_SPLIT = SPLIT && EPI == NET_EPI_RELU_ADD;
    constexpr int ADD_KW = ADD_SPLIT ? ADD_K / 2 : ADD_K;
    static_assert(!ADD_SPLIT || ADD_K % 2 == 0, "split add items");
    uint4 hadd[ADD_KW];
    if (EPI == NET_EPI_RELU_ADD) {
#pragma unroll
      for (int k = 0; k < ADD_KW; ++k) {
        const int it = lane + 64 * ((ADD_SPLIT ? tg : 0) * ADD_KW + k);
        const int lv = it / PV8, part = it - lv * PV8;
        const int x = x0 + lv % ZT, y = y0 + 4 * wv + lv / ZT;
        const bool ok = it < 4 * ZT * PV8 && x < n && y < n;
        const int64_t v = ok ? (int64_t)x + (int64_t)n * (y + (int64_t)n * z) : 0;
        hadd[k] = *reinterpret_cast<const uint4*>(out.add + v * COUT + part * 8);
      }
    }

    f32x4z acc[4][NTW];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int t = 0; t < NTW; ++t) acc[a][t] = f32x4z{0.f, 0.f, 0.f, 0.f};

    const __bf16* sm = ring + ((z + 3) & 3) * SLOT;  // plane z-1 (dz = 0)
    const __bf16* s0 = ring + (z & 3) * SLOT;        // plane z   (dz = 1)
    const __bf16* sp = ring + ((z + 1) & 3) * SLOT;  // plane z+1 (dz = 2)
    if (work) {
      // as in k_conv_zm: group gi + 1's fragments are read before group gi's MFMAs
      bf16x8z fa[6], fb[6];
      zm_load_group<PS>(0, sm, s0, sp, wv, g, col, fa);
      // (not for the 16-channel pool layer: at its three waves per SIMD the
      // deeper pipeline spills, and the compiler's own order measured faster)
      if (!(NCH == 1 && EPI == NET_EPI_RELU_POOL)) __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
#pragma unroll
      for (int gi = 0; gi < 5 * NCH; ++gi) {
        bf16x8z(&f)[6] = (gi & 1) ? fb : fa;
        if (gi + 1 < 5 * NCH) zm_load_group<PS>(gi + 1, sm, s0, sp, wv, g, col, (gi & 1) ? fa : fb);
        const int q = gi / 5, k = gi % 5;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const int st = zm_group_step(k, dy);
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int t = 0; t < NTW; ++t)
              acc[a][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f[a + dy], bw[q][st][t], acc[a][t],
                                                                  0, 0, 0);
        }
        if (!(NCH == 1 && EPI == NET_EPI_RELU_POOL)) {
          if (gi + 1 < 5 * NCH) __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 12 * NTW, 0);
        }
      }
    }

    // epilogue: rows y0 + 4 wv + a, voxels x0 + 4 g + i, channel t*16 + col
    if (EPI == NET_EPI_OUT) {
      // channel 0 (lanes with col 0) through LDS: lane l then stores voxel
      // (row l / 16, x l % 16) of the wave's rows, coalesced
      float* so = reinterpret_cast<float*>(stage) + wv * 64;
      if (col == 0) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int i = 0; i < 4; ++i) so[a * 16 + 4 * g + i] = acc[a][0][i];
      }
      wave_sync();  // per-wave staging
      if (own)
        out.f32[(int64_t)ox + (int64_t)n * (oy + (int64_t)n * z)] =
            own_mask ? rms_f * so[lane] : 0.f;
      return;
    }
    if (EPI == NET_EPI_RELU_ADD) {
      // raw fp32 sums through LDS; each store adds the fp16 partial sums of
      // the upsampled channels, then applies the ReLU
      float* sf = reinterpret_cast<float*>(stage_raw) + wv * (4 * ZT * COUT);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int t = 0; t < NTW; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            sf[((a * ZT) + 4 * g + i) * COUT + (tg + t) * 16 + col] = acc[a][t][i];
      if constexpr (SPLIT)
        __syncthreads();  // both output groups of the row group staged
      else
        wave_sync();  // per-wave staging
#pragma unroll
      for (int k = 0; k < ADD_KW; ++k) {
        const int it = lane + 64 * ((ADD_SPLIT ? tg : 0) * ADD_KW + k);
        if (it >= 4 * ZT * PV8) break;
        const int lv = it / PV8, part = it - lv * PV8;
        const int a = lv / ZT, xl = lv % ZT;
        const int x = x0 + xl, y = y0 + 4 * wv + a;
        if (x >= n || y >= n) continue;
        const int64_t v = (int64_t)x + (int64_t)n * (y + (int64_t)n * z);
        const _Float16* hp = reinterpret_cast<const _Float16*>(&hadd[k]);
        const float* s8 = sf + lv * COUT + part * 8;
        __bf16 o8[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float sum = s8[e] + (float)hp[e];
          o8[e] = (__bf16)(sum > 0.f ? sum : 0.f);
        }
        *reinterpret_cast<uint4*>(out.bf + v * COUT + part * 8) = *reinterpret_cast<const uint4*>(o8);
      }
      return;
    }
    __bf16* st = stage + wv * (4 * ZT * COUT);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int t = 0; t < NTW; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float v = acc[a][t][i];
          if (EPI == NET_EPI_RELU || EPI == NET_EPI_RELU_POOL) v = v > 0.f ? v : 0.f;
          st[((a * ZT) + 4 * g + i) * COUT + (tg + t) * 16 + col] = (__bf16)v;
        }
    if constexpr (SPLIT)
      __syncthreads();  // both output groups of the row group staged
    else
      wave_sync();  // per-wave staging
    if (EPI == NET_EPI_RELU_POOL) {
      // 2x2 in xy from the staged rows of this plane; the z pair (z even,
      // z + 1) accumulates in pacc, the odd plane stores the average
      constexpr int PP = COUT / 8;
      // a split pair shares the parts: wave tg takes parts tg * PPW .. + PPW - 1
      constexpr int PPW = SPLIT ? PP / 2 : PP;
      if (lane < 2 * 8 * PPW) {
        const int part = tg * PPW + lane % PPW, cxy = lane / PPW, cx = cxy % 8, cy = cxy / 8;
        float s8[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) s8[e] = 0.f;
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const uint4 pv = *reinterpret_cast<const uint4*>(
                st + ((2 * cy + dy) * ZT + 2 * cx + dx) * COUT + part * 8);
            const __bf16* pb = reinterpret_cast<const __bf16*>(&pv);
#pragma unroll
            for (int e = 0; e < 8; ++e) s8[e] += (float)pb[e];
          }
        if ((z & 1) == 0) {
#pragma unroll
          for (int e = 0; e < 8; ++e) pacc[e] = s8[e];
        } else {
          const int nh = n >> 1;
          const int px = (x0 >> 1) + cx, py = ((y0 + 4 * wv) >> 1) + cy;
          if (px < nh && py < nh) {
            __bf16 o8[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) o8[e] = (__bf16)(0.125f * (pacc[e] + s8[e]));
            *reinterpret_cast<uint4*>(out.pool + ((int64_t)px + (int64_t)nh * (py + (int64_t)nh * (z >> 1))) * COUT + part * 8) =
                *reinterpret_cast<const uint4*>(o8);
          }
        }
      }
    }
    constexpr int PV = COUT / 8;
    constexpr int SK = (4 * ZT * PV + 63) / 64;  // store items per lane of a row group
    constexpr int SKW = SPLIT ? SK / 2 : SK;     // a split pair shares them
    static_assert(!SPLIT || SK % 2 == 0, "split store items");
#pragma unroll
    for (int k = 0; k < SKW; ++k) {
      const int it = lane + 64 * (tg * SKW + k);
      if (it >= 4 * ZT * PV) break;
      const int lv = it / PV, part = it - lv * PV;
      const int a = lv / ZT, xl = lv % ZT;
      const int x = x0 + xl, y = y0 + 4 * wv + a;
      if (x >= n || y >= n) continue;
      const int64_t v = (int64_t)x + (int64_t)n * (y + (int64_t)n * z);
      uint4 val = *reinterpret_cast<const uint4*>(st + lv * COUT + part * 8);
      if (EPI == NET_EPI_MASKGRAD) {
        const uint4 pm = *reinterpret_cast<const uint4*>(out.relu_of + v * COUT + part * 8);
        const uint32_t* pw = reinterpret_cast<const uint32_t*>(&pm);
        uint32_t* vw = reinterpret_cast<uint32_t*>(&val);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t lo = pw[e] & 0xffffu, hi = pw[e] >> 16;
          const uint32_t keep_lo = (lo != 0u && !(lo & 0x8000u)) ? 0xffffu : 0u;
          const uint32_t keep_hi = (hi != 0u && !(hi & 0x8000u)) ? 0xffff0000u : 0u;
          vw[e] &= (keep_lo | keep_hi);
        }
      }
      *reinterpret_cast<uint4*>(out.bf + v * COUT + part * 8) = val;
    }
  };
  for (int z = z0; z < z1; ++z) plane_step(z);
}

// Decoder layer c9 in one pass: ReLU(conv3(cat(up(D2), E1))) at the fine
// level, with the upsampled half evaluated on the coarse grid as in k_upconv
// (per parity class a 2x2x2 convolution of the 32-channel coarse tensor with
// summed weights) and the skip half as in k_conv_zm_pa, inside one z-march:
// the two halves meet in LDS instead of through an FP16 partial-sum tensor
// written and read back (two passes over 32 B per fine voxel).
//
// A block has 8 waves: waves 0-3 compute the skip half of rows 4 j .. 4 j + 3
// (j = wave % 4) as k_conv_zm_pa does, waves 4-7 the coarse half of the tile
// plane, each into an FP32 stage; after a second barrier every thread adds
// the two stages for 8 channels of one voxel and stores.
//
// Coarse half, per fine plane z (parity pz, coarse plane Z = z / 2): coarse
// wave w takes one parity class, y parity cP = (w / 2) % 2 and x parity
// cpx = w % 2, over the whole 16 x 16 tile (8 x 8 voxels); its 16 summed
// weight fragments (8 taps x 2 z parities, the B operand) stay in registers,
// in the registers that hold a skip wave's weights.  M block b (0..3) holds
// coarse rows b and b + 4 of the tile, so for the two y taps the input
// fragment of (b, ty = 1) is that of (b + 1, ty = 0): per (tz, tx) five A
// fragments from LDS feed eight MFMAs, and no weight is read from LDS.  The
// coarse planes Z-1 .. Z+1 (10 x 10 voxels with the halo, 32 channels) sit
// in a three-slot ring; coarse plane K is stored at fine step 2K - 1 and
// last read at 2K + 2.
constexpr int CAT_BLOCK = 512;

// 16-byte chunk of channels 4 q .. 4 q + 3 of stage voxel x: the coarse
// waves' stores (voxels two apart in x) would put four lanes on the same
// banks without the swizzle, two with it
__device__ inline int cat_chunk(int q, int x) { return q ^ ((x >> 1) & 3); }
constexpr int CAT_KT = ZT / 2 + 2;          // coarse ring plane edge with halo
constexpr int CAT_KRV = CAT_KT * CAT_KT;    // 100 coarse voxels per ring plane
constexpr int CAT_KSLOT = CAT_KRV * 32;     // bf16 per coarse ring slot
constexpr int CAT_KITEMS = CAT_KRV * 4;     // uint4 items per coarse plane
constexpr int CAT_KPF = (CAT_KITEMS + CAT_BLOCK - 1) / CAT_BLOCK;

__global__ void __launch_bounds__(CAT_BLOCK)
    k_conv_cat(int n, int zc, const __bf16* __restrict__ coarse, const __bf16* __restrict__ skip,
               const __bf16* __restrict__ weff, const __bf16* __restrict__ wskip,
               __bf16* __restrict__ out, const int* __restrict__ flags,
               const uint8_t* __restrict__ act) {
  if (flags && flags[F_DONE]) return;
  constexpr int P8 = 2;                  // 8-channel parts per skip voxel
  constexpr int ITEMS = ZRV * P8;
  constexpr int PF = (ITEMS + CAT_BLOCK - 1) / CAT_BLOCK;
  constexpr int PS = ZPS_PAD;  // c9 runs one block per CU either way
  constexpr int SLOT = 2 * PS;
  __shared__ __attribute__((aligned(16))) __bf16 ring[4 * SLOT];
  __shared__ __attribute__((aligned(16))) __bf16 kring[3 * CAT_KSLOT];
  // the coarse half's partial sums of the last two planes, [voxel y*16+x][16],
  // and the skip half's last K-step group, which the coarse waves compute
  __shared__ __attribute__((aligned(16))) float stage[2][ZT * ZT * 16];
  __shared__ __attribute__((aligned(16))) float stage2[2][ZT * ZT * 16];
  __shared__ __attribute__((aligned(16))) int votes[4][8];
  __shared__ uint8_t live_s[ZMAXC + 3];

  const int tiles = ((n + ZT - 1) / ZT) * ((n + ZT - 1) / ZT);
  const int tpr = (n + ZT - 1) / ZT;
  int tile, chunk;
  net_block_of(blockIdx.x, gridDim.x, tpr, tile, chunk);
  const int x0 = (tile % tpr) * ZT, y0 = (tile / tpr) * ZT;
  const int z0 = chunk * zc;
  const int z1 = min(z0 + zc, n);
  if (z0 >= n) return;
  const int nc = n >> 1, X0 = x0 >> 1, Y0 = y0 >> 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, col = lane & 15;
  const int wv = wave & 3;             // row group of this wave
  const bool coarse_role = wave >= 4;  // block-uniform per wave

  // output tile-plane activity (as in k_conv_zm: planes marked 0 are neither
  // computed nor stored, input planes marked 0 read as zero)
  if (act) {
    int any = 0;
    for (int t = threadIdx.x; t < z1 - z0 + 3; t += CAT_BLOCK) {
      const int zi = z0 - 1 + t;
      live_s[t] = (unsigned)zi < (unsigned)n ? act[(int64_t)zi * tiles + tile] : 0;
      any |= t >= 1 && t <= z1 - z0 && live_s[t];
    }
    if (!__syncthreads_or(any)) return;
  }
  auto live = [&](int zi) -> bool { return !act || live_s[zi - z0 + 1] != 0; };
  // block-wide OR with one barrier (as barrier_or, for 8 waves)
  auto vote = [&](int v, int* slot) -> int {
    const bool any = __ballot(v != 0) != 0ull;
    if (lane == 0) slot[wave] = any;
    __syncthreads();
    const int4 a = *reinterpret_cast<const int4*>(slot);
    const int4 b = *reinterpret_cast<const int4*>(slot + 4);
    return a.x | a.y | a.z | a.w | b.x | b.y | b.z | b.w;
  };

  // weight fragments (B operand) in registers, one array for both roles so
  // that they share registers: a skip wave's ZSTEPS steps (as in
  // k_conv_zm_pa); a coarse wave's 16 summed fragments (tap, z parity) of its
  // parity class (y parity cP, x parity cpx)
  const int cP = (wave >> 1) & 1, cpx = wave & 1;
  constexpr int NWR = 16;
  static_assert(ZSTEPS <= NWR, "skip steps");
  bf16x8z wr[NWR];
#pragma unroll
  for (int j = 0; j < NWR; ++j) {
    const int st = j < ZSTEPS ? j : 0;
    const int stap = g < 2 ? zm_tap0(st) : zm_tap1(st);
    const int p = cpx + 2 * cP + 4 * (j >> 3);
    const __bf16* src = coarse_role ? weff + (((int64_t)(p * 8 + (j & 7)) * 16 + col) * 32 + 8 * g)
                                    : wskip + ((int64_t)col * ZTAPS + stap) * 16 + (g & 1) * 8;
    wr[j] = *reinterpret_cast<const bf16x8z*>(src);
  }
  // the skip half's last group (steps 12-14: dz 2 with dx 2 | the zero tap)
  // runs on the coarse waves, which have 32 MFMAs per plane against the
  // skip waves' 60: 48 and 44 after the move
  constexpr int CAT_SKIP_GROUPS = 4;
  bf16x8z wg4[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int st = zm_group_step(4, i);
    const int stap = g < 2 ? zm_tap0(st) : zm_tap1(st);
    wg4[i] = coarse_role ? *reinterpret_cast<const bf16x8z*>(wskip + ((int64_t)col * ZTAPS + stap) * 16 + (g & 1) * 8)
                         : wr[0];
  }

  // skip plane loads: per-item offsets fixed for the block
  uint32_t ioff[PF];
  bool iok[PF];
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const int it = threadIdx.x + k * CAT_BLOCK;
    const int hv = it / P8, p = it - hv * P8;
    const int gx = x0 - 1 + hv % ZR, gy = y0 - 1 + hv / ZR;
    iok[k] = it < ITEMS && (unsigned)gx < (unsigned)n && (unsigned)gy < (unsigned)n;
    ioff[k] = iok[k] ? (uint32_t)((((int64_t)gx + (int64_t)n * gy) * 16 + p * 8) * 2) : 0u;
  }
  const int64_t splane = (int64_t)n * n * 16 * 2;
  uint4 pf[PF];
  auto load_plane = [&](int zi) {
    if (!live(zi) || (unsigned)zi >= (unsigned)n) {
#pragma unroll
      for (int k = 0; k < PF; ++k) pf[k] = make_uint4(0u, 0u, 0u, 0u);
      return;
    }
    const char* pa = reinterpret_cast<const char*>(skip) + (int64_t)zi * splane;
#pragma unroll
    for (int k = 0; k < PF; ++k) pf[k] = *reinterpret_cast<const uint4*>(pa + ioff[k]);
  };
  auto store_plane = [&](int zi) -> int {
    __bf16* slot = ring + ((zi + 4) & 3) * SLOT;
    uint32_t any = 0u;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int it = threadIdx.x + k * CAT_BLOCK;
      if (it < ITEMS) {
        const int hv = it / P8, p = it - hv * P8;
        // component selects (a select of whole vectors went through scratch)
        uint4 v = pf[k];
        v.x = iok[k] ? v.x : 0u;
        v.y = iok[k] ? v.y : 0u;
        v.z = iok[k] ? v.z : 0u;
        v.w = iok[k] ? v.w : 0u;
        *reinterpret_cast<uint4*>(slot + (p * (PS / 8) + hv) * 8) = v;
        any |= v.x | v.y | v.z | v.w;
      }
    }
    return any != 0u;
  };

  // coarse plane loads: item it = 4 v + part (v a halo voxel of the 10 x 10
  // coarse plane, part 8 of its 32 channels)
  uint32_t koff[CAT_KPF];
  bool kok[CAT_KPF];
#pragma unroll
  for (int k = 0; k < CAT_KPF; ++k) {
    const int it = threadIdx.x + k * CAT_BLOCK;
    const int cv = it >> 2, part = it & 3;
    const int cx = X0 - 1 + cv % CAT_KT, cy = Y0 - 1 + cv / CAT_KT;
    kok[k] = it < CAT_KITEMS && (unsigned)cx < (unsigned)nc && (unsigned)cy < (unsigned)nc;
    koff[k] = kok[k] ? (uint32_t)((((int64_t)cx + (int64_t)nc * cy) * 32 + part * 8) * 2) : 0u;
  }
  const int64_t cplane = (int64_t)nc * nc * 32 * 2;
  uint4 kpf[CAT_KPF];
  bool kpf_on = false;
  auto load_coarse = [&](int K) {
    kpf_on = (unsigned)K < (unsigned)nc;
    const char* pc = reinterpret_cast<const char*>(coarse) + (int64_t)(kpf_on ? K : 0) * cplane;
#pragma unroll
    for (int k = 0; k < CAT_KPF; ++k) kpf[k] = *reinterpret_cast<const uint4*>(pc + koff[k]);
  };
  auto kslot = [](int K) -> int { return ((K % 3) + 3) % 3; };
  auto store_coarse = [&](int K) {
    __bf16* slot = kring + kslot(K) * CAT_KSLOT;
#pragma unroll
    for (int k = 0; k < CAT_KPF; ++k) {
      const int it = threadIdx.x + k * CAT_BLOCK;
      if (it < CAT_KITEMS) {
        const int cv = it >> 2, part = it & 3;
        const bool on = kpf_on && kok[k];
        uint4 v = kpf[k];
        v.x = on ? v.x : 0u;
        v.y = on ? v.y : 0u;
        v.z = on ? v.z : 0u;
        v.w = on ? v.w : 0u;
        *reinterpret_cast<uint4*>(slot + (part * CAT_KRV + cv) * 8) = v;
      }
    }
  };

  // prologue: skip planes z0-1, z0 and coarse planes Z0-1, Z0 to LDS, skip
  // plane z0+1 and coarse plane Z0+1 in flight
  const int Z0 = z0 >> 1;
  load_coarse(Z0 - 1);
  store_coarse(Z0 - 1);
  load_coarse(Z0);
  store_coarse(Z0);
  load_plane(z0 - 1);
  int nz_m = vote(store_plane(z0 - 1), votes[(z0 + 3) & 3]);
  load_plane(z0);
  int nz_0 = vote(store_plane(z0), votes[z0 & 3]);
  load_plane(z0 + 1);
  load_coarse(Z0 + 1);

  // Skip waves lag one plane: at plane z (after its barrier) they finish
  // plane z - 1 from their accumulators and the coarse partial sums that the
  // coarse waves staged during plane z - 1, then compute plane z's skip half;
  // the stage is double-buffered by plane parity, so one barrier per plane
  // orders both.  Both halves use the weights as the MFMA's A operand: lane
  // (g, col) holds output channels 4 g .. 4 g + 3 of voxel col of its M block.
  f32x4z acc[4];
  int zprev = -1;  // skip waves: plane whose accumulators are pending
  auto finish = [&]() {
    // plane zprev, rows 4 wv + a, x = col: skip + coarse, ReLU, 4 bf16
    const float* st = stage[zprev & 1];
    const float* st2 = stage2[zprev & 1];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int y = 4 * wv + a;
      const int so = (y * ZT + col) * 16 + 4 * cat_chunk(g, col);
      const float4 c4 = *reinterpret_cast<const float4*>(st + so);
      const float4 s4 = *reinterpret_cast<const float4*>(st2 + so);
      const float v[4] = {acc[a][0] + (c4.x + s4.x), acc[a][1] + (c4.y + s4.y), acc[a][2] + (c4.z + s4.z),
                          acc[a][3] + (c4.w + s4.w)};
      __bf16 h[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) h[i] = (__bf16)(v[i] > 0.f ? v[i] : 0.f);
      *reinterpret_cast<uint2*>(out + ((int64_t)(x0 + col) + (int64_t)n * (y0 + y + (int64_t)n * zprev)) * 16 +
                                4 * g) = *reinterpret_cast<const uint2*>(h);
    }
    zprev = -1;
  };
  auto plane_step = [&](int z) {
    // coarse plane (z + 1) / 2 is first read at odd z
    if (z & 1) store_coarse((z + 1) >> 1);
    const int nz_p = vote(store_plane(z + 1), votes[(z + 1) & 3]);
    if (z + 2 <= z1) load_plane(z + 2);
    if ((z & 1) && z + 2 < z1) load_coarse((z + 3) >> 1);
    const bool work = (nz_m | nz_0 | nz_p) != 0;
    nz_m = nz_0;
    nz_0 = nz_p;
    if (!coarse_role && zprev >= 0) finish();
    if (!live(z)) return;

    if (!coarse_role) {
      // skip half (as k_conv_zm_pa, operands swapped)
#pragma unroll
      for (int a = 0; a < 4; ++a) acc[a] = f32x4z{0.f, 0.f, 0.f, 0.f};
      const __bf16* sm = ring + ((z + 3) & 3) * SLOT;
      const __bf16* s0 = ring + (z & 3) * SLOT;
      const __bf16* sp = ring + ((z + 1) & 3) * SLOT;
      if (work) {
        bf16x8z fa[6], fb[6];
        zm_load_group<PS>(0, sm, s0, sp, wv, g, col, fa);
#pragma unroll
        for (int gi = 0; gi < CAT_SKIP_GROUPS; ++gi) {
          bf16x8z(&f)[6] = (gi & 1) ? fb : fa;
          if (gi + 1 < CAT_SKIP_GROUPS) zm_load_group<PS>(gi + 1, sm, s0, sp, wv, g, col, (gi & 1) ? fa : fb);
#pragma unroll
          for (int dy = 0; dy < 3; ++dy) {
            const int st = zm_group_step(gi, dy);
#pragma unroll
            for (int a = 0; a < 4; ++a)
              acc[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[st], f[a + dy], acc[a], 0, 0, 0);
          }
        }
      }
      zprev = z;
    } else {
      // coarse half: the wave's parity class (cP, cpx) over the whole tile
      // plane; M block b holds coarse rows b and b + 4 of the tile (voxel
      // col: coarse row b + 4 (col >> 3), coarse x col & 7), so that the
      // input fragment of (b, ty = 1) is that of (b + 1, ty = 0): five
      // fragments per (tz, tx) feed eight MFMAs
      f32x4z kacc[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) kacc[b] = f32x4z{0.f, 0.f, 0.f, 0.f};
      const int Zc = z >> 1;
#pragma unroll
      for (int pz = 0; pz < 2; ++pz) {
        if (pz != (z & 1)) continue;  // block-uniform; keeps the weight index static
#pragma unroll
        for (int tz = 0; tz < 2; ++tz) {
          const int oz = tz - (pz ? 0 : 1);
          const __bf16* ks = kring + kslot(Zc + oz) * CAT_KSLOT + g * CAT_KRV * 8;
#pragma unroll
          for (int tx = 0; tx < 2; ++tx) {
            // ring column of coarse x offset tx - (cpx ? 0 : 1), row of row
            // offset e - (cP ? 0 : 1) (both with the halo's +1)
            const int cx = (col & 7) + tx + cpx;
            bf16x8z A[5];
#pragma unroll
            for (int e = 0; e < 5; ++e) {
              const int cy = e + 4 * (col >> 3) + cP;
              A[e] = *reinterpret_cast<const bf16x8z*>(ks + (cy * CAT_KT + cx) * 8);
            }
#pragma unroll
            for (int ty = 0; ty < 2; ++ty)
#pragma unroll
              for (int b = 0; b < 4; ++b)
                kacc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[pz * 8 + tx + 2 * ty + 4 * tz], A[b + ty],
                                                                  kacc[b], 0, 0, 0);
          }
        }
      }
      // to the stage of this plane: fine voxel (2 (col % 8) + cpx,
      // 2 (b + 4 (col / 8)) + cP), channels 4 g .. 4 g + 3
      float* st = stage[z & 1];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int y = 2 * (b + 4 * (col >> 3)) + cP, x = 2 * (col & 7) + cpx;
        *reinterpret_cast<float4*>(st + (y * ZT + x) * 16 + 4 * cat_chunk(g, x)) =
            make_float4(kacc[b][0], kacc[b][1], kacc[b][2], kacc[b][3]);
      }
      // the skip half's last group for the rows of skip wave wv (the same
      // operands and layout as there), to the second stage
      f32x4z sacc[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) sacc[a] = f32x4z{0.f, 0.f, 0.f, 0.f};
      if (work) {
        const __bf16* sm = ring + ((z + 3) & 3) * SLOT;
        const __bf16* s0 = ring + (z & 3) * SLOT;
        const __bf16* sp = ring + ((z + 1) & 3) * SLOT;
        bf16x8z f[6];
        zm_load_group<PS>(4, sm, s0, sp, wv, g, col, f);
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int a = 0; a < 4; ++a)
            sacc[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wg4[dy], f[a + dy], sacc[a], 0, 0, 0);
      }
      float* st2 = stage2[z & 1];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int y = 4 * wv + a;
        *reinterpret_cast<float4*>(st2 + (y * ZT + col) * 16 + 4 * cat_chunk(g, col)) =
            make_float4(sacc[a][0], sacc[a][1], sacc[a][2], sacc[a][3]);
      }
    }
  };
  for (int z = z0; z < z1; ++z) plane_step(z);
  // the last plane's coarse partial sums
  __syncthreads();
  if (!coarse_role && zprev >= 0) finish();
}

bool net_conv_cat(sim_ctx* c, int n, const __bf16* coarse, const __bf16* skip, const __bf16* weff,
                  const __bf16* wskip, __bf16* out, const int* flags, const uint8_t* act) {
  if (n % ZT != 0) return false;
  // (longer z-runs, to stage the weights less often, measured slower: the
  // busy tiles then load the CUs unevenly)
  const ZmGrid g = zm_grid(n);
  hipLaunchKernelGGL(k_conv_cat, dim3(g.blocks), dim3(CAT_BLOCK), 0, c->stream, n, g.zc, coarse, skip,
                     weff, wskip, out, flags, act);
  return true;
}

template <int CIN, int WS, int COUT, int EPI>
static void zm_launch(sim_ctx* c, int n, NetSrc src, const __bf16* w, NetOut out,
                      const int* flags) {
  const ZmGrid g = zm_grid(n);
  if constexpr (EPI == NET_EPI_RELU_ADD || EPI == NET_EPI_RELU_POOL)
    hipLaunchKernelGGL((k_conv_zm_pa<CIN, WS, COUT, EPI>), dim3(g.blocks), dim3(zm_pa_block<CIN, COUT, EPI>()), 0,
                       c->stream, n, g.zc, src, w, out, flags);
  else
    hipLaunchKernelGGL((k_conv_zm<CIN, WS, COUT, EPI>), dim3(g.blocks), dim3(zm_block<CIN, COUT, EPI>()), 0,
                       c->stream, n, g.zc, src, w, out, flags);
}

template <int CIN, int WS, int COUT>
static void zm_epi(sim_ctx* c, int n, int epi, NetSrc src, const __bf16* w, NetOut out,
                   const int* flags) {
  switch (epi) {
    case NET_EPI_RELU: zm_launch<CIN, WS, COUT, NET_EPI_RELU>(c, n, src, w, out, flags); break;
    case NET_EPI_RAW: zm_launch<CIN, WS, COUT, NET_EPI_RAW>(c, n, src, w, out, flags); break;
    case NET_EPI_MASKGRAD: zm_launch<CIN, WS, COUT, NET_EPI_MASKGRAD>(c, n, src, w, out, flags); break;
    case NET_EPI_RELU_ADD: zm_launch<CIN, WS, COUT, NET_EPI_RELU_ADD>(c, n, src, w, out, flags); break;
    case NET_EPI_RELU_POOL: zm_launch<CIN, WS, COUT, NET_EPI_RELU_POOL>(c, n, src, w, out, flags); break;
    default: zm_launch<CIN, WS, COUT, NET_EPI_OUT>(c, n, src, w, out, flags); break;
  }
}

bool net_conv_zm(sim_ctx* c, int n, int cin, int cout, int epi, NetSrc src, const __bf16* w,
                 NetOut out, const int* flags) {
  if (cin == 8 && cout == 16) {
    zm_epi<16, 8, 16>(c, n, epi, src, w, out, flags);
    return true;
  }
  if (cin == 16 && cout == 16) {
    zm_epi<16, 16, 16>(c, n, epi, src, w, out, flags);
    return true;
  }
  if (cin == 48 && cout == 16) {
    zm_epi<48, 48, 16>(c, n, epi, src, w, out, flags);
    return true;
  }
  if (cin == 16 && cout == 32) {
    zm_epi<16, 16, 32>(c, n, epi, src, w, out, flags);
    return true;
  }
  if (cin == 32 && cout == 32) {
    zm_epi<32, 32, 32>(c, n, epi, src, w, out, flags);
    return true;
  }
  if (cin == 16 && cout == 48) {
    zm_epi<16, 16, 48>(c, n, epi, src, w, out, flags);
    return true;
  }
  return false;
}

}  // namespace fs
