// Device-side helpers shared by the fluidsim kernels: grid layout, the
// XCD-aware block order and wave64/LDS reductions in FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fs {

constexpr int kBlock = 256;  // threads per block for streaming/stencil kernels
constexpr int kMaxGrid = 2048;  // blocks per cell-domain launch (and per face component)
// the block partial sums hold kMaxGrid * 3 * 4 doubles
constexpr int kPartialDoubles = kMaxGrid * 3 * 4;
constexpr int kWave = 64;

enum : uint8_t { AIR = 0, LIQUID = 1, SOLID = 2 };

// Face code bits (one byte per face, built once per mask):
//   bit a (0..5) -> the neighbour along -x,+x,-y,+y,-z,+z enters the viscous
//                   Laplacian (an active face, or a wall along the face's own
//                   axis, whose stored value is always zero);
//   bit 6        -> the face itself is active.
enum : uint8_t { FC_ACTIVE = 1u << 6 };

struct Dims {
  int nx, ny, nz;
};

__host__ __device__ inline Dims face_dims(int n, int comp) {
  return Dims{n + (comp == 0), n + (comp == 1), n + (comp == 2)};
}

__host__ __device__ inline int64_t face_count(int n) { return (int64_t)(n + 1) * n * n; }

__host__ __device__ inline int64_t cells(int n) { return (int64_t)n * n * n; }

// Walks a flat index of a 3-D array (x fastest) in fixed strides without a
// division per step.
struct Walker {
  int i, j, k;
  int ai, aj, ak;  // the stride decomposed along x, y, z
  Dims d;
  __device__ inline void init(Dims dd, int64_t start, int64_t stride) {
    d = dd;
    int64_t row = start / d.nx;
    i = (int)(start - row * d.nx);
    j = (int)(row % d.ny);
    k = (int)(row / d.ny);
    int64_t srow = stride / d.nx;
    ai = (int)(stride - srow * d.nx);
    aj = (int)(srow % d.ny);
    ak = (int)(srow / d.ny);
  }
  __device__ inline void next() {
    i += ai;
    int c = i >= d.nx;
    i -= c ? d.nx : 0;
    j += aj + c;
    c = j >= d.ny;
    j -= c ? d.ny : 0;
    k += ak + c;
  }
};

// Blocks are dispatched to the 8 XCDs round-robin by block id, and each XCD
// has its own L2.  Renumber so every XCD gets one contiguous run of logical
// blocks: stencil neighbours (the next row, the next plane) then sit in the
// same L2 as the block that needs them.
__device__ inline int xcd_logical_block(int b, int nblocks) {
  const int nx = 8;
  int q = nblocks / nx, r = nblocks % nx;
  int x = b % nx;
  int prefix = x * q + (x < r ? x : r);
  return prefix + b / nx;
}

// Block order of the network's z-marching kernels, whose grid is nch z-runs
// x (tpr x tpr) xy-tiles.  Only the tiles near liquid hold work, and the
// liquid of a volume is not spread evenly in z, so handing each XCD one
// contiguous range of z (xcd_logical_block) loads the XCDs unevenly (1.5x the
// mean on the 256^3 benchmark mask).  Instead XCD x = b % 8 takes the tile
// rows ty of run c with (c + ty) % 8 == x, each row whole (x-neighbouring
// tiles share their halo columns in that XCD's L2), in run order: every XCD
// gets rows of every z-range.  Needs tpr % 8 == 0 (else the contiguous order).
__device__ inline void net_block_of(int b, int nblocks, int tpr, int& tile, int& chunk) {
  const int tiles = tpr * tpr;
  if ((tpr & 7) == 0 && nblocks % tiles == 0) {
    const int x = b & 7, i = b >> 3;
    const int k = i / tpr, tx = i - k * tpr;  // k-th row of this XCD, tile tx in it
    const int m = tpr >> 3;                   // rows per run that fall to one XCD
    const int c = k / m, j = k - c * m;
    const int ty = ((x - c) & 7) + 8 * j;
    tile = ty * tpr + tx;
    chunk = c;
    return;
  }
  const int lb = xcd_logical_block(b, nblocks);
  tile = lb % tiles;
  chunk = lb / tiles;
}

// Orders LDS traffic between the lanes of one wave (a wave's LDS operations
// execute in order; this keeps the compiler from moving them across).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over a block of kBlock threads; result valid in thread 0.
template <int NV>
__device__ inline void block_sum(double (&v)[NV]) {
  __shared__ double lds[NV][kBlock / kWave];
#pragma unroll
  for (int q = 0; q < NV; ++q)
    for (int off = kWave / 2; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off, kWave);
  int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) lds[q][wid] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0.0;
      for (int w = 0; w < kBlock / kWave; ++w) s += lds[q][w];
      v[q] = s;
    }
  }
}

// Block-level partial sums are stored per block; a one-block finalize
// kernel (k_finalize) adds them in block order (deterministic for a given
// grid) and turns them into solver scalars.  A kernel boundary, not a
// device-scope fence per block, makes the partials visible: on this chip a
// release fence per block costs ~20 ns each, serialised.
// Counts a launch that did work (passed its done check) for the timing
// hooks: block (0, 0) adds one to *work (nullable).
__device__ inline void count_work(int* work) {
  if (work && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) atomicAdd(work, 1);
}

template <int NV>
__device__ inline void store_partials(double (&v)[NV], double* partials, int block_id) {
  block_sum<NV>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) partials[(int64_t)block_id * NV + q] = v[q];
  }
}

}  // namespace fs
