// Conjugate-gradient kernels.
//
// Pressure (cell domain): the Poisson matrix A is matrix-free from the
// per-cell diagonal byte (number of non-wall faces of a liquid cell, zero
// off liquid); off-diagonals are -1 between liquid neighbours.  Every vector
// is zero off liquid, so a neighbour read needs no mask.  The iterate x is
// FP64; r, z, d, q are FP32; every dot product is accumulated in FP64.
//
// One iteration of Jacobi PCG is two streaming kernels, each followed by a
// one-block finalize kernel that reduces the per-block partials and computes
// the CG scalar on the device:
//   dir_spmv : d' = M^-1 r + beta d ; q = A d' ; partial d'.q  -> alpha
//   update   : x += alpha d' ; r -= alpha q ; partial r.M^-1 r -> beta
// With an explicit preconditioner (MIC(0), learned) z is an array computed
// between update and the next dir_spmv, and a separate kernel reduces r.z.
// Every m iterations `check` recomputes r = b - A x from the FP64 x (FP64
// residual replacement), reduces |r|^2 and raises the done flag at tol.
// Every kernel returns at once when the done flag is set, so the host can
// enqueue the next block of iterations before it has read the flag.
//
// Cell-domain kernels take V = 4 consecutive x-cells per thread (float4,
// double2 and 32-bit mask loads) when n % 4 == 0, else V = 1.  The x
// neighbours of a thread's cells come from the adjacent lanes by wave
// shuffle; y and z neighbours are vector loads served mostly by L2.
#include "common.h"
#include "ctx.h"
#include "net.h"

namespace fs {

__constant__ float c_inv_count[8] = {0.f, 1.f, 0.5f, 1.f / 3.f, 0.25f, 0.2f, 1.f / 6.f, 0.f};

// ------------------------------------------------------------ vector I/O

template <int V>
__device__ inline void ldf(const float* __restrict__ p, float (&o)[V]) {
  if constexpr (V == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    o[0] = t.x, o[1] = t.y, o[2] = t.z, o[3] = t.w;
  } else {
    o[0] = *p;
  }
}

template <int V>
__device__ inline void stf(float* __restrict__ p, const float (&o)[V]) {
  if constexpr (V == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
  } else {
    *p = o[0];
  }
}

template <int V>
__device__ inline void ldd(const double* __restrict__ p, double (&o)[V]) {
  if constexpr (V == 4) {
    const double2 a = reinterpret_cast<const double2*>(p)[0];
    const double2 b = reinterpret_cast<const double2*>(p)[1];
    o[0] = a.x, o[1] = a.y, o[2] = b.x, o[3] = b.y;
  } else {
    o[0] = *p;
  }
}

template <int V>
__device__ inline void std_(double* __restrict__ p, const double (&o)[V]) {
  if constexpr (V == 4) {
    reinterpret_cast<double2*>(p)[0] = make_double2(o[0], o[1]);
    reinterpret_cast<double2*>(p)[1] = make_double2(o[2], o[3]);
  } else {
    *p = o[0];
  }
}

template <int V>
__device__ inline void ldg(const uint8_t* __restrict__ p, uint8_t (&o)[V]) {
  if constexpr (V == 4) {
    const uint32_t t = *reinterpret_cast<const uint32_t*>(p);
    o[0] = t & 255u, o[1] = (t >> 8) & 255u, o[2] = (t >> 16) & 255u, o[3] = t >> 24;
  } else {
    o[0] = *p;
  }
}

// Block-contiguous run of V-cell groups with a uniform trip count, so every
// lane takes part in every shuffle.
struct Run {
  int64_t begin, end;  // in groups
  int trips;
};

__device__ inline Run group_run(int64_t groups, int nblocks, int lb) {
  int64_t per = (groups + nblocks - 1) / nblocks;
  per = (per + kBlock - 1) / kBlock * kBlock;
  Run r;
  r.begin = per * lb;
  r.end = r.begin + per < groups ? r.begin + per : groups;
  r.trips = (int)(per / kBlock);
  return r;
}

// ------------------------------------------------------------ finalize

__global__ void __launch_bounds__(kBlock)
    k_finalize(const double* __restrict__ partials, int nblocks, int nv, int mode, double* scal,
               int* flags, double tol2, int jacobi, int slot, double scale, int acc) {
  const bool in_loop = mode == FIN_DQ || mode == FIN_RZ_UPD || mode == FIN_RZ_FIRST ||
                       mode == FIN_CHECK || mode == FIN_FCG_DQDR || mode == FIN_FCG_BETA ||
                       mode == FIN_FCG_RR || mode == FIN_DCG_UPD;
  // the check also runs after an early stop (F_DONE = 3), which it decides
  if (in_loop && flags[F_DONE] && !(mode == FIN_CHECK && flags[F_DONE] == 3)) return;
  // four blocks' partials per thread and pass, loaded before they are added
  // (a dependent load per block made the larger reductions latency-bound)
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b0 = threadIdx.x; b0 < nblocks; b0 += 4 * kBlock) {
    double t[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = b0 + u * kBlock;
#pragma unroll
      for (int q = 0; q < 4; ++q) t[u][q] = b < nblocks && q < nv ? partials[(int64_t)b * nv + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] += t[u][q];
  }
  block_sum<4>(v);
  if (threadIdx.x != 0) return;
  switch (mode) {
    case FIN_PCG_INIT:
      scal[S_BB] = v[0];
      scal[S_RR] = v[0];
      scal[S_RZ] = v[1];
      scal[S_RZ_PREV] = v[1];
      scal[S_BETA] = 0.0;
      flags[F_DONE] = v[0] == 0.0 ? 1 : 0;
      flags[F_ITERS] = 0;
      flags[F_ITERS_AT_DONE] = 0;
      flags[F_RESTART] = 0;
      break;
    case FIN_DQ:
      scal[S_DQ] = v[0];
      flags[F_ITERS] += 1;
      if (!(v[0] > 0.0)) flags[F_DONE] = 2;  // breakdown: NaN or non-positive curvature
      break;
    case FIN_RZ_UPD: {
      const double rz_old = scal[S_RZ];
      scal[S_RZ_PREV] = rz_old;
      scal[S_RZ] = v[0];
      scal[S_BETA] = v[0] / rz_old;
      if (!(v[0] >= 0.0)) flags[F_DONE] = 2;
      break;
    }
    case FIN_RZ_FIRST:
      scal[S_RZ] = v[0];
      scal[S_RZ_PREV] = v[0];
      scal[S_BETA] = 0.0;
      if (!(v[0] > 0.0)) flags[F_DONE] = 2;
      break;
    case FIN_CHECK:
      scal[S_RR] = v[0];
      if (jacobi) {
        scal[S_RZ] = v[1];
        scal[S_BETA] = scal[S_RZ_PREV] > 0.0 ? v[1] / scal[S_RZ_PREV] : 0.0;
      } else {
        scal[S_NET_SUMSQ] = v[1];  // |r|^2 of the replaced residual (the network's input scale)
      }
      if (v[0] <= tol2 * scal[S_BB]) {
        flags[F_DONE] = 1;
        flags[F_ITERS_AT_DONE] = flags[F_ITERS];
      } else if (!(v[0] == v[0])) {
        flags[F_DONE] = 2;
      } else if (flags[F_DONE] == 3) {
        // an early stop the true residual does not confirm: go on from the
        // updated iterate with a fresh direction (the skipped iterations
        // left the direction buffers behind)
        flags[F_DONE] = 0;
        if (jacobi)
          scal[S_BETA] = 0.0;
        else
          flags[F_RESTART] = 1;
      }
      break;
    case FIN_FCG_DQDR:
      // d.r may have either sign (the step alpha = d.r / d.q takes it); only
      // a direction with no positive curvature, or a NaN, is a breakdown
      scal[S_DQ] = v[0];
      scal[S_DR] = v[1];
      flags[F_ITERS] += 1;
      if (!(v[0] > 0.0) || !(v[1] == v[1])) flags[F_DONE] = 2;
      break;
    case FIN_FCG_BETA:
      scal[S_BETA] = flags[F_RESTART] ? 0.0 : -v[0] / scal[S_DQ];
      flags[F_RESTART] = 0;
      if (!(scal[S_BETA] == scal[S_BETA])) flags[F_DONE] = 2;
      break;
    case FIN_DCG_UPD: {
      const double rz_old = scal[S_RZ];
      scal[S_RZ_PREV] = rz_old;
      scal[S_RZ] = v[0];
      scal[S_BETA] = v[0] / rz_old;
      if (!(v[0] >= 0.0))
        flags[F_DONE] = 2;
      else if (v[1] <= tol2 * scal[S_BB])
        flags[F_DONE] = 3;  // the rest of the block is skipped; the check decides
      break;
    }
    case FIN_FCG_RR:
      // the recursive |r|^2 after the update of phase `slot` (0..2): at the
      // tolerance the block's later iterations are skipped and drop out of
      // the four-step iterate update (their alphas 0)
      scal[S_NET_SUMSQ] = v[0];
      if (v[0] <= tol2 * scal[S_BB]) {
        flags[F_DONE] = 3;
        for (int q = slot + 1; q < 3; ++q) scal[S_ALPHA_Q0 + q] = 0.0;
      }
      break;
    case FIN_DCG_INIT:
      scal[S_BB] = v[0];
      scal[S_RZ] = v[1];
      scal[S_RZ_PREV] = v[1];
      scal[S_RR] = v[2];
      scal[S_BETA] = 0.0;
      flags[F_DONE] = v[2] <= tol2 * v[0] ? 1 : 0;
      flags[F_ITERS] = 0;
      flags[F_ITERS_AT_DONE] = 0;
      break;
    case FIN_SLOT:
      scal[slot] = (acc ? scal[slot] : 0.0) + scale * v[0];
      break;
    case FIN_SLOTS4:
      for (int q = 0; q < 4; ++q) scal[slot + q] = (acc ? scal[slot + q] : 0.0) + scale * v[q];
      break;
  }
}

void launch_finalize(sim_ctx* c, int nblocks, int nv, int mode, double tol2, int jacobi, int slot,
                     double scale, int acc) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, c->stream, c->partials, nblocks, nv,
                     mode, c->scal, c->flags, tol2, jacobi, slot, scale, acc);
}

// ---------------------------------------------------------------- Poisson

template <int V>
__device__ inline void walk_init(Walker& w, int n, int64_t g0) {
  w.init(Dims{n / V, n, n}, g0, kBlock);
}

template <int V, int PREC>
__global__ void __launch_bounds__(kBlock)
    k_pcg_init(int n, const uint8_t* __restrict__ cdiag, const float* __restrict__ b,
               double* __restrict__ x, float* __restrict__ r, float* __restrict__ d0,
               double* partials) {
  const int64_t G = cells(n) / V;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Run run = group_run(G, gridDim.x, lb);
  double v[2] = {0.0, 0.0};
  for (int64_t g = run.begin + threadIdx.x; g < run.end; g += kBlock) {
    const int64_t idx = g * V;
    float bv[V], z[V];
    uint8_t dg[V];
    double xz[V];
    ldf<V>(b + idx, bv);
    ldg<V>(cdiag + idx, dg);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      z[e] = 0.f;
      xz[e] = 0.0;
      v[0] += (double)bv[e] * bv[e];
      if (PREC == PK_JACOBI) v[1] += (double)bv[e] * bv[e] * c_inv_count[dg[e]];
    }
    std_<V>(x + idx, xz);
    stf<V>(r + idx, bv);
    stf<V>(d0 + idx, z);
  }
  store_partials<2>(v, partials, lb);
}

// Direction at V cells: z + beta * d_in with z = r / diag (Jacobi) or z.
template <int V, int PREC>
__device__ inline void dir_at(const float* __restrict__ r, const float* __restrict__ z,
                              const uint8_t* __restrict__ cdiag, const float* __restrict__ d_in,
                              int64_t idx, float beta, float (&o)[V]) {
  float dv[V], zv[V];
  ldf<V>(d_in + idx, dv);
  if (PREC == PK_JACOBI) {
    float rv[V];
    uint8_t gv[V];
    ldf<V>(r + idx, rv);
    ldg<V>(cdiag + idx, gv);
#pragma unroll
    for (int e = 0; e < V; ++e) zv[e] = rv[e] * c_inv_count[gv[e]];
  } else {
    ldf<V>(z + idx, zv);
  }
#pragma unroll
  for (int e = 0; e < V; ++e) o[e] = beta != 0.f ? zv[e] + beta * dv[e] : zv[e];
}

// d' = z + beta d_in ; q = A d' ; partials d'.q (and d'.r for flexible CG).
template <int V, int PREC, bool FLEX>
__global__ void __launch_bounds__(kBlock)
    k_dir_spmv(int n, const uint8_t* __restrict__ cdiag, const float* __restrict__ r,
               const float* __restrict__ z, const float* __restrict__ d_in,
               float* __restrict__ d_out, float* __restrict__ q, const double* __restrict__ scal,
               const int* __restrict__ flags, double* partials, int* __restrict__ work) {
  if (flags[F_DONE]) return;
  count_work(work);
  const int64_t G = cells(n) / V;
  const float beta = (float)scal[S_BETA];
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Run run = group_run(G, gridDim.x, lb);
  const int64_t sy = n, sz = (int64_t)n * n;
  const int lane = threadIdx.x & (kWave - 1);
  Walker w;
  walk_init<V>(w, n, run.begin + threadIdx.x);
  double v[2] = {0.0, 0.0};
  for (int t = 0; t < run.trips; ++t, w.next()) {
    const int64_t g = run.begin + threadIdx.x + (int64_t)t * kBlock;
    const bool act = g < run.end;
    const int64_t idx = g * V;
    const int i = w.i * V;
    float dc[V];
    uint8_t dg[V];
#pragma unroll
    for (int e = 0; e < V; ++e) dc[e] = 0.f, dg[e] = 0;
    if (act) {
      dir_at<V, PREC>(r, z, cdiag, d_in, idx, beta, dc);
      ldg<V>(cdiag + idx, dg);
    }
    // x neighbours from the adjacent lanes (the previous/next group of the same row)
    float left = __shfl_up(dc[V - 1], 1, kWave);
    float right = __shfl_down(dc[0], 1, kWave);
    if (!act) continue;
    if (i > 0 && lane == 0) {
      float t1[1];
      dir_at<1, PREC>(r, z, cdiag, d_in, idx - 1, beta, t1);
      left = t1[0];
    }
    if (i + V < n && lane == kWave - 1) {
      float t1[1];
      dir_at<1, PREC>(r, z, cdiag, d_in, idx + V, beta, t1);
      right = t1[0];
    }
    float s[V];
#pragma unroll
    for (int e = 0; e < V; ++e) s[e] = 0.f;
    if (w.j > 0) {
      float t4[V];
      dir_at<V, PREC>(r, z, cdiag, d_in, idx - sy, beta, t4);
#pragma unroll
      for (int e = 0; e < V; ++e) s[e] += t4[e];
    }
    if (w.j < n - 1) {
      float t4[V];
      dir_at<V, PREC>(r, z, cdiag, d_in, idx + sy, beta, t4);
#pragma unroll
      for (int e = 0; e < V; ++e) s[e] += t4[e];
    }
    if (w.k > 0) {
      float t4[V];
      dir_at<V, PREC>(r, z, cdiag, d_in, idx - sz, beta, t4);
#pragma unroll
      for (int e = 0; e < V; ++e) s[e] += t4[e];
    }
    if (w.k < n - 1) {
      float t4[V];
      dir_at<V, PREC>(r, z, cdiag, d_in, idx + sz, beta, t4);
#pragma unroll
      for (int e = 0; e < V; ++e) s[e] += t4[e];
    }
    if (i > 0) s[0] += left;
    if (i + V < n) s[V - 1] += right;
#pragma unroll
    for (int e = 1; e < V; ++e) s[e] += dc[e - 1];
#pragma unroll
    for (int e = 0; e + 1 < V; ++e) s[e] += dc[e + 1];
    float qv[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      qv[e] = dg[e] ? (float)dg[e] * dc[e] - s[e] : 0.f;
      v[0] += (double)dc[e] * (double)qv[e];
    }
    if (FLEX) {
      float rv[V];
      ldf<V>(r + idx, rv);
#pragma unroll
      for (int e = 0; e < V; ++e) v[1] += (double)dc[e] * (double)rv[e];
    }
    stf<V>(d_out + idx, dc);
    stf<V>(q + idx, qv);
  }
  store_partials<2>(v, partials, lb);
}

// ------------------------------------------------- z-marching stencils
// The same d' = z + beta d ; q = A d' (and the FP64 check) organised so
// every cell's direction is formed exactly once: a block owns a tile of
// 64 (x) x 16 (y) cells and marches up a chunk of z planes.  Each thread
// holds one 4-cell group; the direction of planes z-1, z, z+1 stays in
// registers, the current plane (plus a one-cell halo) goes through LDS for
// the x and y neighbours.  Halo cells outside the box are written as zero,
// which is also their contribution (every vector is zero off liquid).
// Target launch sizes of the z-marching stencils (compile-time settings):
// fewer blocks mean longer z-runs and less halo re-reading, more blocks more
// latency hiding (measured at 256^3: the Jacobi direction + SpMV and the FP64
// check are fastest at 1024 blocks, the flexible direction + SpMV, which reads
// four arrays per plane, at 768, the viscosity stencil at 2048).
#ifndef FS_ZM_BLOCKS
#define FS_ZM_BLOCKS 1024
#endif
#ifndef FS_ZM_BLOCKS_FLEX
#define FS_ZM_BLOCKS_FLEX 768
#endif
#ifndef FS_DZ_BLOCKS
#define FS_DZ_BLOCKS 2048
#endif
constexpr int ZM_GX = 16;  // 4-cell groups per tile along x (64 cells)
constexpr int ZM_TY = 16;  // rows per tile (ZM_GX * ZM_TY = kBlock threads)
constexpr int ZM_W = 4 * ZM_GX + 2;

struct ZTile {
  int x0, y0, z0, z1, x, y, gx, ty;
  bool in_xy;
};

__device__ inline ZTile ztile(int n, int zc) {
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int tiles_x = (n + 4 * ZM_GX - 1) / (4 * ZM_GX);
  const int tiles_y = (n + ZM_TY - 1) / ZM_TY;
  ZTile t;
  const int txi = lb % tiles_x;
  const int rest = lb / tiles_x;
  t.x0 = txi * 4 * ZM_GX;
  t.y0 = (rest % tiles_y) * ZM_TY;
  t.z0 = (rest / tiles_y) * zc;
  t.z1 = t.z0 + zc < n ? t.z0 + zc : n;
  t.gx = threadIdx.x % ZM_GX;
  t.ty = threadIdx.x / ZM_GX;
  t.x = t.x0 + 4 * t.gx;
  t.y = t.y0 + t.ty;
  t.in_xy = t.x < n && t.y < n;
  return t;
}

// Raw inputs of the direction at one 4-cell group (z = r/diag for Jacobi,
// else the explicit z array).  A group of the tile's own output planes (own)
// also carries what its stencil row needs after the barrier: the diagonal
// codes and, for the flexible variant's second dot, r; the planes just below
// and above a z-run feed only the z neighbours and need the direction alone.
template <int PREC>
struct DirRaw {
  float a[4];  // r (Jacobi) or z
  float d[4];
  uint32_t g;
  float rr[4];  // r of a centre group in the flexible variant
};

template <int PREC, bool CENTER, bool FLEX>
__device__ inline void dir_raw_load(const float* __restrict__ r, const float* __restrict__ z,
                                    const uint8_t* __restrict__ cdiag,
                                    const float* __restrict__ d_in, int64_t idx, bool ok,
                                    bool own, DirRaw<PREC>& o) {
  if (ok) {
    ldf<4>((PREC == PK_JACOBI ? r : z) + idx, o.a);
    ldf<4>(d_in + idx, o.d);
    o.g = PREC == PK_JACOBI || (CENTER && own) ? *reinterpret_cast<const uint32_t*>(cdiag + idx)
                                                : 0u;
    if (CENTER && FLEX) {
      if (own) {
        ldf<4>(r + idx, o.rr);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) o.rr[e] = 0.f;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) o.a[e] = 0.f, o.d[e] = 0.f, o.rr[e] = 0.f;
    o.g = 0u;
  }
}

template <int PREC>
__device__ inline void dir_raw_eval(const DirRaw<PREC>& w, float beta, float (&o)[4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float zv =
        PREC == PK_JACOBI ? w.a[e] * c_inv_count[(w.g >> (8 * e)) & 255u] : w.a[e];
    // beta = 0 (first direction, restart): the previous direction is not read
    o[e] = beta != 0.f ? zv + beta * w.d[e] : zv;
  }
}

template <int PREC, bool FLEX>
__global__ void __launch_bounds__(kBlock)
    k_dir_spmv_zm(int n, int zc, const uint8_t* __restrict__ cdiag, const float* __restrict__ r,
                  const float* __restrict__ z, const float* __restrict__ d_in,
                  float* __restrict__ d_out, float* __restrict__ q, const double* __restrict__ scal,
                  const int* __restrict__ flags, double* partials, int* __restrict__ work) {
  if (flags[F_DONE]) return;
  count_work(work);
  // two plane slots: plane zz is written to slot zz & 1, so the slot written
  // for plane zz + 1 was last read for plane zz - 1, before this plane's
  // barrier, and one barrier per plane suffices
  __shared__ float sd2[2][ZM_TY + 2][ZM_W];
  const float beta = (float)scal[S_BETA];
  const ZTile t = ztile(n, zc);
  const int64_t sz = (int64_t)n * n;
  auto gidx = [&](int xx, int yy, int zz) -> int64_t { return xx + (int64_t)n * yy + sz * zz; };
  auto in_box = [&](int xx, int yy, int zz) {
    return xx >= 0 && xx < n && yy >= 0 && yy < n && zz >= 0 && zz < n;
  };
  // halo roles: a y-halo group (top or bottom row of the tile) and an x-halo cell
  const int hy = t.ty == 0 ? t.y0 - 1 : (t.ty == ZM_TY - 1 ? t.y0 + ZM_TY : -1);
  const int hrow = t.ty == 0 ? 0 : ZM_TY + 1;
  const int hx = t.gx == 0 ? t.x0 - 1 : (t.gx == ZM_GX - 1 ? t.x0 + 4 * ZM_GX : -1);
  const int hcol = t.gx == 0 ? 0 : ZM_W - 1;
  const bool has_hy = (t.ty == 0 || t.ty == ZM_TY - 1) && t.x < n;
  const bool has_hx = t.gx == 0 || t.gx == ZM_GX - 1;

  // planes z0 - 1 .. z1 are read, z0 .. z1 - 1 with their diagonal codes (and r)
  auto load_center = [&](int zz, DirRaw<PREC>& o) {
    dir_raw_load<PREC, true, FLEX>(r, z, cdiag, d_in, gidx(t.x, t.y, zz),
                                   t.in_xy && zz >= 0 && zz < n && zz <= t.z1,
                                   zz >= t.z0 && zz < t.z1, o);
  };
  auto load_hy = [&](int zz, DirRaw<PREC>& o) {
    dir_raw_load<PREC, false, false>(r, z, cdiag, d_in, gidx(t.x, hy, zz),
                                     has_hy && zz < t.z1 && in_box(t.x, hy, zz), false, o);
  };
  auto load_hx = [&](int zz, float& a, float& d, uint8_t& g) {
    if (has_hx && zz < t.z1 && in_box(hx, t.y, zz)) {
      const int64_t m = gidx(hx, t.y, zz);
      a = (PREC == PK_JACOBI ? r : z)[m];
      d = d_in[m];
      g = PREC == PK_JACOBI ? cdiag[m] : 0;
    } else {
      a = 0.f, d = 0.f, g = 0;
    }
  };

  // pipeline: centre raw data two planes ahead, halo raw data one plane ahead
  DirRaw<PREC> c1, c2, h1;
  float hxa, hxd;
  uint8_t hxg;
  float dm[4], dc[4], dp[4];
  // diagonal codes and (flexible) r of the current plane's group
  uint32_t gc;
  float rc[4];
  {
    DirRaw<PREC> c0;
    load_center(t.z0 - 1, c0);
    load_center(t.z0, c1);
    dir_raw_eval<PREC>(c0, beta, dm);
    dir_raw_eval<PREC>(c1, beta, dc);
    gc = c1.g;
#pragma unroll
    for (int e = 0; e < 4; ++e) rc[e] = c1.rr[e];
  }
  load_center(t.z0 + 1, c1);
  load_hy(t.z0, h1);
  load_hx(t.z0, hxa, hxd, hxg);
  double v[2] = {0.0, 0.0};
  for (int zz = t.z0; zz < t.z1; ++zz) {
    // halo values of plane zz from the data loaded one iteration ago
    float hyv[4];
    dir_raw_eval<PREC>(h1, beta, hyv);
    const float hxz = PREC == PK_JACOBI ? hxa * c_inv_count[hxg] : hxa;
    const float hxv = beta != 0.f ? hxz + beta * hxd : hxz;
    dir_raw_eval<PREC>(c1, beta, dp);
    // issue the next loads before the barrier
    load_center(zz + 2, c2);
    load_hy(zz + 1, h1);
    load_hx(zz + 1, hxa, hxd, hxg);
    float(&sd)[ZM_TY + 2][ZM_W] = sd2[zz & 1];
#pragma unroll
    for (int e = 0; e < 4; ++e) sd[t.ty + 1][1 + 4 * t.gx + e] = dc[e];
    if (has_hx) sd[t.ty + 1][hcol] = hxv;
    if (t.ty == 0 || t.ty == ZM_TY - 1) {
#pragma unroll
      for (int e = 0; e < 4; ++e) sd[hrow][1 + 4 * t.gx + e] = hyv[e];
    }
    __syncthreads();
    if (t.in_xy) {
      const int64_t idx = gidx(t.x, t.y, zz);
      const int c0 = 1 + 4 * t.gx;
      float qv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t dg = (gc >> (8 * e)) & 255u;
        const float s = sd[t.ty + 1][c0 + e - 1] + sd[t.ty + 1][c0 + e + 1] + sd[t.ty][c0 + e] +
                        sd[t.ty + 2][c0 + e] + dm[e] + dp[e];
        qv[e] = dg ? (float)dg * dc[e] - s : 0.f;
        v[0] += (double)dc[e] * (double)qv[e];
      }
      if (FLEX) {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[1] += (double)dc[e] * (double)rc[e];
      }
      stf<4>(d_out + idx, dc);
      stf<4>(q + idx, qv);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) dm[e] = dc[e], dc[e] = dp[e], rc[e] = c1.rr[e];
    gc = c1.g;
    c1 = c2;
  }
  store_partials<2>(v, partials, xcd_logical_block(blockIdx.x, gridDim.x));
}

// FP64 true residual r = b - A x with the same tiling (x in LDS as double).
template <int PREC>
__global__ void __launch_bounds__(kBlock)
    k_check_zm(int n, int zc, const uint8_t* __restrict__ cdiag, const float* __restrict__ b,
               const double* __restrict__ x, float* __restrict__ r, const int* __restrict__ flags,
               double* partials, int* __restrict__ work) {
  if (flags[F_DONE] == 1 || flags[F_DONE] == 2) return;  // runs after an early stop (3)
  count_work(work);
  // two plane slots, one barrier per plane (as in k_dir_spmv_zm)
  __shared__ double sx2[2][ZM_TY + 2][ZM_W];
  const ZTile t = ztile(n, zc);
  const int64_t sz = (int64_t)n * n;
  auto gidx = [&](int xx, int yy, int zz) -> int64_t { return xx + (int64_t)n * yy + sz * zz; };
  auto group_x = [&](int xx, int yy, int zz, double (&o)[4]) {
    if (xx >= 0 && xx < n && yy >= 0 && yy < n && zz >= 0 && zz < n)
      ldd<4>(x + gidx(xx, yy, zz), o);
    else
      o[0] = o[1] = o[2] = o[3] = 0.0;
  };
  auto cell_x = [&](int xx, int yy, int zz) -> double {
    if (xx < 0 || xx >= n || yy < 0 || yy >= n) return 0.0;
    return x[gidx(xx, yy, zz)];
  };
  // b and the diagonal codes of the thread's group, loaded one plane ahead
  auto group_bg = [&](int zz, float (&bo)[4], uint32_t& go) {
    if (t.in_xy && zz < t.z1) {
      const int64_t idx = gidx(t.x, t.y, zz);
      ldf<4>(b + idx, bo);
      go = *reinterpret_cast<const uint32_t*>(cdiag + idx);
    } else {
      bo[0] = bo[1] = bo[2] = bo[3] = 0.f;
      go = 0u;
    }
  };
  double xm[4], xc[4], xp[4];
  float bc[4], bn[4];
  uint32_t gc, gn;
  group_x(t.in_xy ? t.x : -1, t.y, t.z0 - 1, xm);
  group_x(t.in_xy ? t.x : -1, t.y, t.z0, xc);
  group_bg(t.z0, bc, gc);
  double v[2] = {0.0, 0.0};
  for (int zz = t.z0; zz < t.z1; ++zz) {
    group_x(t.in_xy ? t.x : -1, t.y, zz + 1, xp);
    group_bg(zz + 1, bn, gn);
    double(&sx)[ZM_TY + 2][ZM_W] = sx2[zz & 1];
#pragma unroll
    for (int e = 0; e < 4; ++e) sx[t.ty + 1][1 + 4 * t.gx + e] = xc[e];
    if (t.gx == 0) sx[t.ty + 1][0] = cell_x(t.x0 - 1, t.y, zz);
    if (t.gx == ZM_GX - 1) sx[t.ty + 1][ZM_W - 1] = cell_x(t.x0 + 4 * ZM_GX, t.y, zz);
    if (t.ty == 0) {
      double o[4];
      group_x(t.x < n ? t.x : -1, t.y0 - 1, zz, o);
#pragma unroll
      for (int e = 0; e < 4; ++e) sx[0][1 + 4 * t.gx + e] = o[e];
    }
    if (t.ty == ZM_TY - 1) {
      double o[4];
      group_x(t.x < n ? t.x : -1, t.y0 + ZM_TY, zz, o);
#pragma unroll
      for (int e = 0; e < 4; ++e) sx[ZM_TY + 1][1 + 4 * t.gx + e] = o[e];
    }
    __syncthreads();
    if (t.in_xy) {
      const int64_t idx = gidx(t.x, t.y, zz);
      float rf[4];
      const int c0 = 1 + 4 * t.gx;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t dg = (gc >> (8 * e)) & 255u;
        const double s = sx[t.ty + 1][c0 + e - 1] + sx[t.ty + 1][c0 + e + 1] + sx[t.ty][c0 + e] +
                         sx[t.ty + 2][c0 + e] + xm[e] + xp[e];
        const double rc = dg ? (double)bc[e] - ((double)dg * xc[e] - s) : 0.0;
        rf[e] = (float)rc;
        v[0] += rc * rc;
        v[1] += PREC == PK_JACOBI ? (double)rf[e] * (double)rf[e] * c_inv_count[dg]
                                  : (double)rf[e] * (double)rf[e];
      }
      stf<4>(r + idx, rf);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) xm[e] = xc[e], xc[e] = xp[e], bc[e] = bn[e];
    gc = gn;
  }
  store_partials<2>(v, partials, xcd_logical_block(blockIdx.x, gridDim.x));
}

// Launch shape of the z-marching kernels: tiles of 64 x 16 cells and a z
// chunk sized for about 4 blocks per CU (at most 4096 blocks in total).
struct ZmShape {
  int blocks, zc;
};

static ZmShape zm_shape(int n, int target = FS_ZM_BLOCKS) {
  const int tiles = ((n + 4 * ZM_GX - 1) / (4 * ZM_GX)) * ((n + ZM_TY - 1) / ZM_TY);
  int chunks = target / tiles;
  if (chunks < 1) chunks = 1;
  if (chunks > n / 4) chunks = n / 4 > 0 ? n / 4 : 1;
  int zc = (n + chunks - 1) / chunks;
  chunks = (n + zc - 1) / zc;
  return ZmShape{tiles * chunks, zc};
}

// Jacobi PCG update that touches the FP64 iterate only every second
// iteration: on odd iterations only r -= alpha q (alpha kept in S_ALPHA_PREV),
// on even iterations x += alpha_prev d_prev + alpha d, r -= alpha q.  Both
// directions are still in the ping-pong buffers, so this saves the 16 B/cell
// read-modify-write of x on half of the iterations.
template <int V, bool WITH_X>
__global__ void __launch_bounds__(kBlock)
    k_update2(int n, const uint8_t* __restrict__ cdiag, double* __restrict__ x,
              float* __restrict__ r, const float* __restrict__ d, const float* __restrict__ d_prev,
              const float* __restrict__ q, double* __restrict__ scal,
              const int* __restrict__ flags, double* partials, int* __restrict__ work) {
  if (flags[F_DONE]) return;
  count_work(work);
  const int64_t G = cells(n) / V;
  const double alpha = scal[S_RZ] / scal[S_DQ];
  const double alpha_prev = scal[S_ALPHA_PREV];
  const float alpha_f = (float)alpha;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Run run = group_run(G, gridDim.x, lb);
  double v[1] = {0.0};
  for (int64_t g = run.begin + threadIdx.x; g < run.end; g += kBlock) {
    const int64_t idx = g * V;
    float qv[V], rv[V];
    uint8_t dg[V];
    ldf<V>(q + idx, qv);
    ldf<V>(r + idx, rv);
    ldg<V>(cdiag + idx, dg);
    if (WITH_X) {
      double xv[V];
      float dv[V], pv[V];
      ldd<V>(x + idx, xv);
      ldf<V>(d + idx, dv);
      ldf<V>(d_prev + idx, pv);
#pragma unroll
      for (int e = 0; e < V; ++e) xv[e] += alpha_prev * (double)pv[e] + alpha * (double)dv[e];
      std_<V>(x + idx, xv);
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
      rv[e] -= alpha_f * qv[e];
      v[0] += (double)rv[e] * (double)rv[e] * c_inv_count[dg[e]];
    }
    stf<V>(r + idx, rv);
  }
  store_partials<1>(v, partials, lb);
  if (!WITH_X && blockIdx.x == 0 && threadIdx.x == 0) scal[S_ALPHA_PREV] = alpha;
}

// Four-step variant: r -= alpha q every iteration; the alphas of the first
// three iterations of a group of four are kept in scal, and on the fourth
// x += a0 d0 + a1 d1 + a2 d2 + a3 d3 in FP64 (one read-modify-write of x per
// four iterations).
// FLEX: the flexible CG's step alpha = d.r / d.q, and no r.z partials.
// KEEP_R false: the iterate update alone (an FP64 check that replaces r by
// the true residual follows at once), no r update and no reduction.
template <int V, bool WITH_X, bool FLEX, bool KEEP_R = true>
__global__ void __launch_bounds__(kBlock)
    k_update4(int n, const uint8_t* __restrict__ cdiag, double* __restrict__ x,
              float* __restrict__ r, const float* __restrict__ d0, const float* __restrict__ d1,
              const float* __restrict__ d2, const float* __restrict__ d3,
              const float* __restrict__ q, double* __restrict__ scal, int phase,
              const int* __restrict__ flags, double* partials, int* __restrict__ work) {
  // after an early stop of the flexible CG (F_DONE = 3) the block's iterate
  // update still runs, without a step of its own (alpha 0) and with the
  // skipped iterations' alphas zeroed
  const int done = flags[F_DONE];
  const bool early = FLEX && WITH_X && done == 3;
  if (done && !early) return;
  count_work(work);
  const int64_t G = cells(n) / V;
  const double alpha = early ? 0.0 : (FLEX ? scal[S_DR] : scal[S_RZ]) / scal[S_DQ];
  const float alpha_f = (float)alpha;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Run run = group_run(G, gridDim.x, lb);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (WITH_X) {
    a0 = scal[S_ALPHA_Q0];
    a1 = scal[S_ALPHA_Q1];
    a2 = scal[S_ALPHA_Q2];
  }
  static_assert(KEEP_R || WITH_X, "an update without r needs the iterate");
  double v[1] = {0.0};
  for (int64_t g = run.begin + threadIdx.x; g < run.end; g += kBlock) {
    const int64_t idx = g * V;
    float qv[V], rv[V];
    uint8_t dg[V];
    if (KEEP_R) {
      ldf<V>(q + idx, qv);
      ldf<V>(r + idx, rv);
      ldg<V>(cdiag + idx, dg);
    }
    if (WITH_X) {
      double xv[V];
      float e0[V], e1[V], e2[V], e3[V];
      ldd<V>(x + idx, xv);
      ldf<V>(d0 + idx, e0);
      ldf<V>(d1 + idx, e1);
      ldf<V>(d2 + idx, e2);
      ldf<V>(d3 + idx, e3);
      // a zero alpha leaves its direction unread (a skipped iteration's
      // buffer may hold anything)
#pragma unroll
      for (int e = 0; e < V; ++e)
        xv[e] += ((a0 != 0.0 ? a0 * (double)e0[e] : 0.0) + (a1 != 0.0 ? a1 * (double)e1[e] : 0.0)) +
                 ((a2 != 0.0 ? a2 * (double)e2[e] : 0.0) + (alpha != 0.0 ? alpha * (double)e3[e] : 0.0));
      std_<V>(x + idx, xv);
    }
    if (KEEP_R) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        rv[e] -= alpha_f * qv[e];
        // Jacobi: r.M^-1 r; flexible CG: |r|^2, the learned preconditioner's
        // input scale (it would otherwise read r once more for it)
        v[0] += FLEX ? (double)rv[e] * (double)rv[e] : (double)rv[e] * (double)rv[e] * c_inv_count[dg[e]];
      }
      stf<V>(r + idx, rv);
    }
  }
  if (KEEP_R) store_partials<1>(v, partials, lb);
  if (!WITH_X && blockIdx.x == 0 && threadIdx.x == 0) scal[S_ALPHA_Q0 + phase] = alpha;
}

// x += alpha d ; r -= alpha q ; (Jacobi) partial r.M^-1 r.
// alpha = RZ / DQ (PCG) or DR / DQ (flexible CG).
template <int V, int PREC, bool FLEX>
__global__ void __launch_bounds__(kBlock)
    k_update(int n, const uint8_t* __restrict__ cdiag, double* __restrict__ x,
             float* __restrict__ r, const float* __restrict__ d, const float* __restrict__ q,
             const double* __restrict__ scal, const int* __restrict__ flags, double* partials, int* __restrict__ work) {
  if (flags[F_DONE]) return;
  count_work(work);
  const int64_t G = cells(n) / V;
  const double alpha = (FLEX ? scal[S_DR] : scal[S_RZ]) / scal[S_DQ];
  const float alpha_f = (float)alpha;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Run run = group_run(G, gridDim.x, lb);
  double v[1] = {0.0};
  for (int64_t g = run.begin + threadIdx.x; g < run.end; g += kBlock) {
    const int64_t idx = g * V;
    double xv[V];
    float dv[V], qv[V], rv[V];
    uint8_t dg[V];
    ldd<V>(x + idx, xv);
    ldf<V>(d + idx, dv);
    ldf<V>(q + idx, qv);
    ldf<V>(r + idx, rv);
    if (PREC == PK_JACOBI) ldg<V>(cdiag + idx, dg);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      xv[e] += alpha * (double)dv[e];
      rv[e] -= alpha_f * qv[e];
      if (PREC == PK_JACOBI) v[0] += (double)rv[e] * (double)rv[e] * c_inv_count[dg[e]];
    }
    std_<V>(x + idx, xv);
    stf<V>(r + idx, rv);
  }
  if (PREC == PK_JACOBI) store_partials<1>(v, partials, lb);
}

// partial a.b over cells (r.z for an explicit preconditioner, z.q for the
// flexible-CG beta).
template <int V>
__global__ void __launch_bounds__(kBlock)
    k_dot_cells(int n, const float* __restrict__ a, const float* __restrict__ b,
                const int* __restrict__ flags, double* partials) {
  if (flags && flags[F_DONE]) return;
  const int64_t G = cells(n) / V;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Run run = group_run(G, gridDim.x, lb);
  double v[1] = {0.0};
  for (int64_t g = run.begin + threadIdx.x; g < run.end; g += kBlock) {
    float av[V], bv[V];
    ldf<V>(a + g * V, av);
    ldf<V>(b + g * V, bv);
#pragma unroll
    for (int e = 0; e < V; ++e) v[0] += (double)av[e] * (double)bv[e];
  }
  store_partials<1>(v, partials, lb);
}

// r = b - A x in FP64 from the FP64 iterate (residual replacement);
// partials |r|^2 and (Jacobi) r.M^-1 r.
template <int V, int PREC>
__global__ void __launch_bounds__(kBlock)
    k_check(int n, const uint8_t* __restrict__ cdiag, const float* __restrict__ b,
            const double* __restrict__ x, float* __restrict__ r, const int* __restrict__ flags,
            double* partials, int* __restrict__ work) {
  if (flags[F_DONE] == 1 || flags[F_DONE] == 2) return;  // runs after an early stop (3)
  count_work(work);
  const int64_t G = cells(n) / V;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Run run = group_run(G, gridDim.x, lb);
  const int64_t sy = n, sz = (int64_t)n * n;
  const int lane = threadIdx.x & (kWave - 1);
  Walker w;
  walk_init<V>(w, n, run.begin + threadIdx.x);
  double v[2] = {0.0, 0.0};
  for (int t = 0; t < run.trips; ++t, w.next()) {
    const int64_t g = run.begin + threadIdx.x + (int64_t)t * kBlock;
    const bool act = g < run.end;
    const int64_t idx = g * V;
    const int i = w.i * V;
    double xc[V];
#pragma unroll
    for (int e = 0; e < V; ++e) xc[e] = 0.0;
    if (act) ldd<V>(x + idx, xc);
    double left = __shfl_up(xc[V - 1], 1, kWave);
    double right = __shfl_down(xc[0], 1, kWave);
    if (!act) continue;
    if (i > 0 && lane == 0) left = x[idx - 1];
    if (i + V < n && lane == kWave - 1) right = x[idx + V];
    double s[V];
#pragma unroll
    for (int e = 0; e < V; ++e) s[e] = 0.0;
    auto add = [&](int64_t m) {
      double t4[V];
      ldd<V>(x + m, t4);
#pragma unroll
      for (int e = 0; e < V; ++e) s[e] += t4[e];
    };
    if (w.j > 0) add(idx - sy);
    if (w.j < n - 1) add(idx + sy);
    if (w.k > 0) add(idx - sz);
    if (w.k < n - 1) add(idx + sz);
    if (i > 0) s[0] += left;
    if (i + V < n) s[V - 1] += right;
#pragma unroll
    for (int e = 1; e < V; ++e) s[e] += xc[e - 1];
#pragma unroll
    for (int e = 0; e + 1 < V; ++e) s[e] += xc[e + 1];
    float bv[V], rf[V];
    uint8_t dg[V];
    ldf<V>(b + idx, bv);
    ldg<V>(cdiag + idx, dg);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const double rc = dg[e] ? (double)bv[e] - ((double)dg[e] * xc[e] - s[e]) : 0.0;
      rf[e] = (float)rc;
      v[0] += rc * rc;
      v[1] += PREC == PK_JACOBI ? (double)rf[e] * (double)rf[e] * c_inv_count[dg[e]]
                                : (double)rf[e] * (double)rf[e];
    }
    stf<V>(r + idx, rf);
  }
  store_partials<2>(v, partials, lb);
}

template <int V>
__global__ void __launch_bounds__(kBlock)
    k_poisson_apply(int n, const uint8_t* __restrict__ cdiag, const float* __restrict__ xin,
                    float* __restrict__ y) {
  const int64_t G = cells(n) / V;
  const Run run = group_run(G, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  const int64_t sy = n, sz = (int64_t)n * n;
  Walker w;
  walk_init<V>(w, n, run.begin + threadIdx.x);
  for (int64_t g = run.begin + threadIdx.x; g < run.end; g += kBlock, w.next()) {
    const int64_t idx = g * V;
    const int i = w.i * V;
    float xc[V], s[V], out[V];
    uint8_t dg[V];
    ldf<V>(xin + idx, xc);
    ldg<V>(cdiag + idx, dg);
#pragma unroll
    for (int e = 0; e < V; ++e) s[e] = 0.f;
    auto add = [&](int64_t m) {
      float t4[V];
      ldf<V>(xin + m, t4);
#pragma unroll
      for (int e = 0; e < V; ++e) s[e] += t4[e];
    };
    if (w.j > 0) add(idx - sy);
    if (w.j < n - 1) add(idx + sy);
    if (w.k > 0) add(idx - sz);
    if (w.k < n - 1) add(idx + sz);
    if (i > 0) s[0] += xin[idx - 1];
    if (i + V < n) s[V - 1] += xin[idx + V];
#pragma unroll
    for (int e = 1; e < V; ++e) s[e] += xc[e - 1];
#pragma unroll
    for (int e = 0; e + 1 < V; ++e) s[e] += xc[e + 1];
#pragma unroll
    for (int e = 0; e < V; ++e) out[e] = dg[e] ? (float)dg[e] * xc[e] - s[e] : 0.f;
    stf<V>(y + idx, out);
  }
}

__global__ void __launch_bounds__(kBlock)
    k_jacobi_apply(int n, const uint8_t* __restrict__ cdiag, const float* __restrict__ r,
                   float* __restrict__ z) {
  const int64_t C = cells(n);
  for (int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x; idx < C;
       idx += (int64_t)gridDim.x * kBlock)
    z[idx] = r[idx] * c_inv_count[cdiag[idx]];
}

// out = (float) x, or out = (float)(x - (double) out) when err != 0.
__global__ void __launch_bounds__(kBlock)
    k_err_snapshot(int64_t C, const double* __restrict__ xref, const double* __restrict__ x,
                   float* __restrict__ out) {
  for (int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x; idx < C;
       idx += (int64_t)gridDim.x * kBlock)
    out[idx] = (float)(xref[idx] - x[idx]);
}

void launch_err_snapshot(sim_ctx* c, const double* xref, float* out) {
  hipLaunchKernelGGL(k_err_snapshot, dim3(2048), dim3(kBlock), 0, c->stream, c->C, xref, c->x,
                     out);
}

__global__ void __launch_bounds__(kBlock)
    k_copy_double(int64_t C, const double* __restrict__ a, double* __restrict__ o,
                  const int* __restrict__ flags) {
  if (flags && flags[F_DONE]) return;
  for (int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x; idx < C;
       idx += (int64_t)gridDim.x * kBlock)
    o[idx] = a[idx];
}

__global__ void __launch_bounds__(kBlock)
    k_extrapolate_double(int64_t C, const double* __restrict__ a, const double* __restrict__ b,
                         double* __restrict__ o, int order) {
  for (int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x; idx < C;
       idx += (int64_t)gridDim.x * kBlock)
    o[idx] = order == 3 ? 3.0 * (a[idx] - b[idx]) + o[idx] : 2.0 * a[idx] - b[idx];
}

// ----------------------------------------------------------- launchers

// Launch kern<4, ...> when rows hold whole 4-cell groups, else kern<1, ...>;
// the kernel arguments come from the ARGS macro defined at the call site.
#define FS_CELL_LAUNCH(kern, ...)                                                       \
  do {                                                                                  \
    if (c->n % 4 == 0)                                                                  \
      hipLaunchKernelGGL((kern<4, ##__VA_ARGS__>), dim3(c->grid_cells), dim3(kBlock), 0, \
                         c->stream, ARGS);                                              \
    else                                                                                \
      hipLaunchKernelGGL((kern<1, ##__VA_ARGS__>), dim3(c->grid_cells), dim3(kBlock), 0, \
                         c->stream, ARGS);                                              \
  } while (0)

static double tol_sq(double t) { return t * t; }

void launch_pcg_init(sim_ctx* c, int prec) {
#define ARGS c->n, c->cdiag, c->b, c->x, c->r, c->dA, c->partials
  if (prec == PK_JACOBI)
    FS_CELL_LAUNCH(k_pcg_init, PK_JACOBI);
  else
    FS_CELL_LAUNCH(k_pcg_init, PK_ZARRAY);
#undef ARGS
  launch_finalize(c, c->grid_cells, 2, FIN_PCG_INIT, 0.0, prec == PK_JACOBI, 0, 0.0, 0);
}

template <bool FLEX>
static int dir_spmv_any(sim_ctx* c, int prec, const float* d_in, float* d_out) {
  if (c->n % 4 == 0) {
    const ZmShape zs = zm_shape(c->n, FLEX ? FS_ZM_BLOCKS_FLEX : FS_ZM_BLOCKS);
    if (prec == PK_JACOBI)
      hipLaunchKernelGGL((k_dir_spmv_zm<PK_JACOBI, FLEX>), dim3(zs.blocks), dim3(kBlock), 0,
                         c->stream, c->n, zs.zc, c->cdiag, c->r, c->z, d_in, d_out, c->q, c->scal,
                         c->flags, c->partials, c->work + SIM_KERN_PCG_DIR_SPMV);
    else
      hipLaunchKernelGGL((k_dir_spmv_zm<PK_ZARRAY, FLEX>), dim3(zs.blocks), dim3(kBlock), 0,
                         c->stream, c->n, zs.zc, c->cdiag, c->r, c->z, d_in, d_out, c->q, c->scal,
                         c->flags, c->partials, c->work + SIM_KERN_PCG_DIR_SPMV);
    return zs.blocks;
  }
#define ARGS c->n, c->cdiag, c->r, c->z, d_in, d_out, c->q, c->scal, c->flags, c->partials, \
             c->work + SIM_KERN_PCG_DIR_SPMV
  if (prec == PK_JACOBI)
    hipLaunchKernelGGL((k_dir_spmv<1, PK_JACOBI, FLEX>), dim3(c->grid_cells), dim3(kBlock), 0,
                       c->stream, ARGS);
  else
    hipLaunchKernelGGL((k_dir_spmv<1, PK_ZARRAY, FLEX>), dim3(c->grid_cells), dim3(kBlock), 0,
                       c->stream, ARGS);
#undef ARGS
  return c->grid_cells;
}

void launch_pcg_dir_spmv(sim_ctx* c, int prec, const float* d_in, float* d_out) {
  prof_mark(c, SIM_KERN_PCG_DIR_SPMV, true);
  const int nb = dir_spmv_any<false>(c, prec, d_in, d_out);
  prof_mark(c, SIM_KERN_PCG_DIR_SPMV, false);
  launch_finalize(c, nb, 2, FIN_DQ, 0.0, 0, 0, 0.0, 0);
}

void launch_pcg_update(sim_ctx* c, int prec, const float* d) {
#define ARGS c->n, c->cdiag, c->x, c->r, d, c->q, c->scal, c->flags, c->partials, \
             c->work + SIM_KERN_PCG_UPDATE
  prof_mark(c, SIM_KERN_PCG_UPDATE, true);
  if (prec == PK_JACOBI) {
    FS_CELL_LAUNCH(k_update, PK_JACOBI, false);
    prof_mark(c, SIM_KERN_PCG_UPDATE, false);
    launch_finalize(c, c->grid_cells, 1, FIN_RZ_UPD, 0.0, 1, 0, 0.0, 0);
  } else {
    FS_CELL_LAUNCH(k_update, PK_ZARRAY, false);
    prof_mark(c, SIM_KERN_PCG_UPDATE, false);
  }
#undef ARGS
}

void launch_pcg_update2(sim_ctx* c, const float* d, const float* d_prev, bool with_x) {
#define ARGS c->n, c->cdiag, c->x, c->r, d, d_prev, c->q, c->scal, c->flags, c->partials, \
             c->work + SIM_KERN_PCG_UPDATE
  prof_mark(c, SIM_KERN_PCG_UPDATE, true);
  if (with_x)
    FS_CELL_LAUNCH(k_update2, true);
  else
    FS_CELL_LAUNCH(k_update2, false);
  prof_mark(c, SIM_KERN_PCG_UPDATE, false);
#undef ARGS
  launch_finalize(c, c->grid_cells, 1, FIN_RZ_UPD, 0.0, 1, 0, 0.0, 0);
}

void launch_pcg_update4(sim_ctx* c, const float* const dirs[4], int phase) {
#define ARGS c->n, c->cdiag, c->x, c->r, dirs[0], dirs[1], dirs[2], dirs[3], c->q, c->scal, \
             phase, c->flags, c->partials, c->work + SIM_KERN_PCG_UPDATE
  prof_mark(c, SIM_KERN_PCG_UPDATE, true);
  if (phase == 3)
    FS_CELL_LAUNCH(k_update4, true, false);
  else
    FS_CELL_LAUNCH(k_update4, false, false);
  prof_mark(c, SIM_KERN_PCG_UPDATE, false);
  launch_finalize(c, c->grid_cells, 1, FIN_RZ_UPD, 0.0, 1, 0, 0.0, 0);
}

void launch_fcg_update4(sim_ctx* c, const float* const dirs[4], int phase, double tol,
                        bool check_follows) {
  prof_mark(c, SIM_KERN_PCG_UPDATE, true);
  // before the FP64 check (which recomputes r from x and reduces its |r|^2)
  // only the iterate is updated
  const bool x_only = phase == 3 && check_follows;
  if (x_only)
    FS_CELL_LAUNCH(k_update4, true, true, false);
  else if (phase == 3)
    FS_CELL_LAUNCH(k_update4, true, true);
  else
    FS_CELL_LAUNCH(k_update4, false, true);
  prof_mark(c, SIM_KERN_PCG_UPDATE, false);
#undef ARGS
  if (x_only) return;
  // |r|^2 of the updated residual, for the learned preconditioner's input;
  // inside a block it also ends the block early once it meets the tolerance
  // (the FP64 check at the block's end decides; a stop it refuses restarts
  // the directions.  Measured at 256^3: stopping at 0.8, 0.9, 0.97 and 1.0
  // times the tolerance gave 6955, 6904, 6883 and 6853 ms per bench step)
  if (phase < 3)
    launch_finalize(c, c->grid_cells, 1, FIN_FCG_RR, tol_sq(tol), 0, phase, 0.0, 0);
  else
    launch_finalize(c, c->grid_cells, 1, FIN_SLOT, 0.0, 0, S_NET_SUMSQ, 1.0, 0);
}

void launch_pcg_rz_first(sim_ctx* c, int first) {
#define ARGS c->n, c->r, c->z, c->flags, c->partials
  FS_CELL_LAUNCH(k_dot_cells);
#undef ARGS
  launch_finalize(c, c->grid_cells, 1, first ? FIN_RZ_FIRST : FIN_RZ_UPD, 0.0, 0, 0, 0.0, 0);
}

void launch_pcg_rz(sim_ctx* c) { launch_pcg_rz_first(c, 0); }

void launch_dot_cells_slot(sim_ctx* c, const float* a, const float* b, int slot,
                           const int* flags) {
#define ARGS c->n, a, b, flags, c->partials
  FS_CELL_LAUNCH(k_dot_cells);
#undef ARGS
  launch_finalize(c, c->grid_cells, 1, FIN_SLOT, 0.0, 0, slot, 1.0, 0);
}

void launch_pcg_check(sim_ctx* c, int prec, double tol) {
  prof_mark(c, SIM_KERN_PCG_CHECK, true);
  int nb = c->grid_cells;
  if (c->n % 4 == 0) {
    const ZmShape zs = zm_shape(c->n);
    nb = zs.blocks;
    if (prec == PK_JACOBI)
      hipLaunchKernelGGL((k_check_zm<PK_JACOBI>), dim3(zs.blocks), dim3(kBlock), 0, c->stream,
                         c->n, zs.zc, c->cdiag, c->b, c->x, c->r, c->flags, c->partials,
                         c->work + SIM_KERN_PCG_CHECK);
    else
      hipLaunchKernelGGL((k_check_zm<PK_ZARRAY>), dim3(zs.blocks), dim3(kBlock), 0, c->stream,
                         c->n, zs.zc, c->cdiag, c->b, c->x, c->r, c->flags, c->partials,
                         c->work + SIM_KERN_PCG_CHECK);
  } else {
#define ARGS c->n, c->cdiag, c->b, c->x, c->r, c->flags, c->partials, c->work + SIM_KERN_PCG_CHECK
    if (prec == PK_JACOBI)
      hipLaunchKernelGGL((k_check<1, PK_JACOBI>), dim3(c->grid_cells), dim3(kBlock), 0, c->stream,
                         ARGS);
    else
      hipLaunchKernelGGL((k_check<1, PK_ZARRAY>), dim3(c->grid_cells), dim3(kBlock), 0, c->stream,
                         ARGS);
#undef ARGS
  }
  prof_mark(c, SIM_KERN_PCG_CHECK, false);
  launch_finalize(c, nb, 2, FIN_CHECK, tol_sq(tol), prec == PK_JACOBI, 0, 0.0, 0);
}

void launch_poisson_apply(sim_ctx* c, const float* xin, float* y) {
#define ARGS c->n, c->cdiag, xin, y
  FS_CELL_LAUNCH(k_poisson_apply);
#undef ARGS
}

void launch_jacobi_apply(sim_ctx* c, const float* r, float* z) {
  hipLaunchKernelGGL(k_jacobi_apply, dim3(c->grid_cells), dim3(kBlock), 0, c->stream, c->n,
                     c->cdiag, r, z);
}

void launch_x_to_double(sim_ctx* c, const double* xin, double* out, const int* flags) {
  hipLaunchKernelGGL(k_copy_double, dim3(1024), dim3(kBlock), 0, c->stream, c->C, xin, out,
                     flags);
}

void launch_x_extrapolate(sim_ctx* c, const double* a, const double* b, double* o, int order) {
  hipLaunchKernelGGL(k_extrapolate_double, dim3(1024), dim3(kBlock), 0, c->stream, c->C, a, b, o,
                     order);
}

// ---------------------------------------------------------- flexible CG
// Notay's flexible CG with one stored direction:
//   alpha = d.r / d.q ; x += alpha d ; r -= alpha q ; z = B(r) ;
//   beta = -(z.q) / (d.q) ; d = z + beta d.

void launch_fcg_init(sim_ctx* c) {
#define ARGS c->n, c->cdiag, c->b, c->x, c->r, c->dA, c->partials
  FS_CELL_LAUNCH(k_pcg_init, PK_ZARRAY);
#undef ARGS
  launch_finalize(c, c->grid_cells, 2, FIN_PCG_INIT, 0.0, 0, 0, 0.0, 0);
}

void launch_fcg_dir_spmv(sim_ctx* c, const float* d_in, float* d_out) {
  prof_mark(c, SIM_KERN_PCG_DIR_SPMV, true);
  const int nb = dir_spmv_any<true>(c, PK_ZARRAY, d_in, d_out);
  prof_mark(c, SIM_KERN_PCG_DIR_SPMV, false);
  launch_finalize(c, nb, 2, FIN_FCG_DQDR, 0.0, 0, 0, 0.0, 0);
}

void launch_fcg_update(sim_ctx* c, const float* d) {
#define ARGS c->n, c->cdiag, c->x, c->r, d, c->q, c->scal, c->flags, c->partials, \
             c->work + SIM_KERN_PCG_UPDATE
  prof_mark(c, SIM_KERN_PCG_UPDATE, true);
  FS_CELL_LAUNCH(k_update, PK_ZARRAY, true);
  prof_mark(c, SIM_KERN_PCG_UPDATE, false);
#undef ARGS
}

void launch_fcg_beta_first(sim_ctx* c, int first) {
  if (first) {
    // beta = 0 for the first direction
    launch_finalize(c, 0, 1, FIN_SLOT, 0.0, 0, S_BETA, 0.0, 0);
    return;
  }
#define ARGS c->n, c->z, c->q, c->flags, c->partials
  FS_CELL_LAUNCH(k_dot_cells);
#undef ARGS
  launch_finalize(c, c->grid_cells, 1, FIN_FCG_BETA, 0.0, 0, 0, 0.0, 0);
}

void launch_fcg_beta(sim_ctx* c) { launch_fcg_beta_first(c, 0); }

void launch_fcg_beta_partials(sim_ctx* c, int nblocks) {
  launch_finalize(c, nblocks, 1, FIN_FCG_BETA, 0.0, 0, 0, 0.0, 0);
}

void launch_fcg_check(sim_ctx* c, double tol) { launch_pcg_check(c, PK_ZARRAY, tol); }

// ------------------------------------------------- implicit viscosity CG
// Solves (I - alpha L) x = b on the active faces of all three components at
// once (one CG on the stacked vector), Jacobi-preconditioned with
// diag = 1 + alpha * (number of Laplacian neighbours).  As for the pressure,
// the iterate is FP64 with FP64 residual replacement: with alpha = nu dt/h^2
// up to ~55 at 256^3 the rounding of an FP32 iterate alone would leave a
// relative residual of |M| * 2^-24 ~ 4e-5.  r, d, q are FP32, dots FP64.
// b is ctx->tmp; the FP64 iterate is ctx->fx; the result is rounded into
// the output fields at the end.

struct Chunk2 {
  int64_t begin, end;
};

__device__ inline Chunk2 chunk_of(int64_t total, int nblocks, int lb) {
  int64_t per = (total + nblocks - 1) / nblocks;
  per = (per + kBlock - 1) / kBlock * kBlock;
  int64_t b = per * lb;
  int64_t e = b + per < total ? b + per : total;
  return Chunk2{b, e};
}

__device__ inline float mrow_diag_inv(uint8_t code, float alpha) {
  return (code & FC_ACTIVE) ? 1.f / (1.f + alpha * (float)__popc(code & 63u)) : 0.f;
}

template <typename T, typename V>
__device__ inline T mrow(const V* __restrict__ f, int64_t idx, uint8_t code, int64_t sy, int64_t sz,
                         T alpha) {
  // all seven loads issued at once (an absent neighbour reads the face
  // itself), then the same additions in the same order as a branchy form
  const V f0 = f[idx];
  const V fm1 = f[code & 1 ? idx - 1 : idx], fp1 = f[code & 2 ? idx + 1 : idx];
  const V fmy = f[code & 4 ? idx - sy : idx], fpy = f[code & 8 ? idx + sy : idx];
  const V fmz = f[code & 16 ? idx - sz : idx], fpz = f[code & 32 ? idx + sz : idx];
  const T v = (T)f0;
  T acc = 0;
  acc = code & 1 ? acc + ((T)fm1 - v) : acc;
  acc = code & 2 ? acc + ((T)fp1 - v) : acc;
  acc = code & 4 ? acc + ((T)fmy - v) : acc;
  acc = code & 8 ? acc + ((T)fpy - v) : acc;
  acc = code & 16 ? acc + ((T)fmz - v) : acc;
  acc = code & 32 ? acc + ((T)fpz - v) : acc;
  return v - alpha * acc;
}

// x = b (initial guess), r = b - M b, d0 = 0
__global__ void __launch_bounds__(kBlock)
    k_dcg_init(int n, const uint8_t* __restrict__ fcode, float alpha, const float* __restrict__ b,
               double* __restrict__ x, float* __restrict__ r, float* __restrict__ d0, int64_t F,
               double* partials) {
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  const int64_t sy = d.nx, sz = (int64_t)d.nx * d.ny;
  const uint8_t* __restrict__ code = fcode + comp * F;
  const float* __restrict__ bc = b + comp * F;
  double* __restrict__ xc = x + comp * F;
  float* __restrict__ rc = r + comp * F;
  float* __restrict__ dc = d0 + comp * F;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(F, gridDim.x, lb);
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    const uint8_t cd = code[idx];
    dc[idx] = 0.f;
    if (!(cd & FC_ACTIVE)) {
      rc[idx] = 0.f;
      xc[idx] = 0.0;
      continue;
    }
    xc[idx] = (double)bc[idx];
    const double rv = (double)bc[idx] - mrow<double>(bc, idx, cd, sy, sz, (double)alpha);
    const float rf = (float)rv;
    rc[idx] = rf;
    v[0] += (double)bc[idx] * bc[idx];
    v[1] += (double)rf * rf * mrow_diag_inv(cd, alpha);
    v[2] += rv * rv;
  }
  store_partials<3>(v, partials, comp * gridDim.x + lb);
}

__global__ void __launch_bounds__(kBlock)
    k_dcg_dir_spmv(int n, const uint8_t* __restrict__ fcode, float alpha,
                   const float* __restrict__ r, const float* __restrict__ d_in,
                   float* __restrict__ d_out, float* __restrict__ q, int64_t F,
                   const double* __restrict__ scal, const int* __restrict__ flags,
                   double* partials, int* __restrict__ work) {
  if (flags[F_DONE]) return;
  count_work(work);
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  const int64_t sy = d.nx, sz = (int64_t)d.nx * d.ny;
  const float beta = (float)scal[S_BETA];
  const uint8_t* __restrict__ code = fcode + comp * F;
  const float* __restrict__ rc = r + comp * F;
  const float* __restrict__ di = d_in + comp * F;
  float* __restrict__ dout = d_out + comp * F;
  float* __restrict__ qc = q + comp * F;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(F, gridDim.x, lb);
  // beta = 0 (first direction, restart): the previous direction is not read
  auto dir = [&](int64_t m) -> float {
    const float zv = rc[m] * mrow_diag_inv(code[m], alpha);
    return beta != 0.f ? zv + beta * di[m] : zv;
  };
  double v[1] = {0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    const uint8_t cd = code[idx];
    if (!(cd & FC_ACTIVE)) {
      dout[idx] = 0.f;
      qc[idx] = 0.f;
      continue;
    }
    const float dcur = dir(idx);
    float acc = 0.f;
    if (cd & 1) acc += dir(idx - 1) - dcur;
    if (cd & 2) acc += dir(idx + 1) - dcur;
    if (cd & 4) acc += dir(idx - sy) - dcur;
    if (cd & 8) acc += dir(idx + sy) - dcur;
    if (cd & 16) acc += dir(idx - sz) - dcur;
    if (cd & 32) acc += dir(idx + sz) - dcur;
    const float qv = dcur - alpha * acc;
    dout[idx] = dcur;
    qc[idx] = qv;
    v[0] += (double)dcur * (double)qv;
  }
  store_partials<1>(v, partials, comp * gridDim.x + lb);
}

// The same step organised as a z-march (as k_dir_spmv_zm for the cells): a
// block owns a 64 x 16 tile of one face component's (x, y) plane and walks a
// run of z planes.  Each face's direction is formed once per plane; planes
// z-1, z, z+1 stay in registers for the z neighbours, plane z (with a
// one-face halo) goes through LDS for the x and y neighbours.  Thread (tx,
// tg) owns the faces of column x0 + tx in rows y0 + tg + 4k, k = 0..3.
constexpr int DZ_TX = 64, DZ_TY = 16, DZ_K = DZ_TY / (kBlock / DZ_TX);

struct DcgZmShape {
  int tiles_x, tiles, chunks, zc;
};

__host__ __device__ inline DcgZmShape dcg_zm_shape(int n) {
  // the largest face grid, (n + 1) x (n + 1) x (n + 1), bounds all three
  DcgZmShape s;
  s.tiles_x = (n + 1 + DZ_TX - 1) / DZ_TX;
  s.tiles = s.tiles_x * ((n + 1 + DZ_TY - 1) / DZ_TY);
  int chunks = (FS_DZ_BLOCKS + s.tiles - 1) / s.tiles;
  if (chunks > n + 1) chunks = n + 1;
  s.zc = (n + 1 + chunks - 1) / chunks;
  s.chunks = (n + 1 + s.zc - 1) / s.zc;
  return s;
}

__global__ void __launch_bounds__(kBlock)
    k_dcg_dir_spmv_zm(int n, const uint8_t* __restrict__ fcode, float alpha,
                      const float* __restrict__ r, const float* __restrict__ d_in,
                      float* __restrict__ d_out, float* __restrict__ q, int64_t F,
                      const double* __restrict__ scal, const int* __restrict__ flags,
                      double* partials, int* __restrict__ work) {
  if (flags[F_DONE]) return;
  count_work(work);
  // two plane slots, one barrier per plane (as in k_dir_spmv_zm)
  __shared__ float sd2[2][DZ_TY + 2][DZ_TX + 2];
  const int comp = blockIdx.y;
  const Dims dm3 = face_dims(n, comp);
  const int64_t sy = dm3.nx, sz = (int64_t)dm3.nx * dm3.ny;
  const float beta = (float)scal[S_BETA];
  const uint8_t* __restrict__ code = fcode + comp * F;
  const float* __restrict__ rc = r + comp * F;
  const float* __restrict__ di = d_in + comp * F;
  float* __restrict__ dout = d_out + comp * F;
  float* __restrict__ qc = q + comp * F;
  const DcgZmShape sh = dcg_zm_shape(n);
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int tile = lb % sh.tiles, chunk = lb / sh.tiles;
  const int x0 = (tile % sh.tiles_x) * DZ_TX, y0 = (tile / sh.tiles_x) * DZ_TY;
  const int z0 = chunk * sh.zc;
  const int z1 = min(z0 + sh.zc, dm3.nz);
  double v[1] = {0.0};
  if (x0 < dm3.nx && y0 < dm3.ny && z0 < dm3.nz) {
    const int tx = threadIdx.x % DZ_TX, tg = threadIdx.x / DZ_TX;
    const int x = x0 + tx;
    auto in_grid = [&](int xx, int yy, int zz) {
      return xx >= 0 && xx < dm3.nx && yy >= 0 && yy < dm3.ny && zz >= 0 && zz < dm3.nz;
    };
    // beta = 0 (first direction, restart): the previous direction is not read
    auto dir_of = [&](float rv, float dv, uint8_t cd) {
      const float zv = rv * mrow_diag_inv(cd, alpha);
      return beta != 0.f ? zv + beta * dv : zv;
    };
    // raw (r, d, code) of this thread's faces of one plane, and of its halo face
    struct Raw {
      float r[DZ_K], d[DZ_K];
      uint8_t c[DZ_K];
    };
    // planes z0 - 1 .. z1 (the one above the run feeds only the z neighbours)
    auto load_own = [&](int zz, Raw& o) {
#pragma unroll
      for (int k = 0; k < DZ_K; ++k) {
        const int y = y0 + tg + 4 * k;
        if (zz <= z1 && in_grid(x, y, zz)) {
          const int64_t m = x + sy * y + sz * zz;
          o.r[k] = rc[m];
          o.d[k] = di[m];
          o.c[k] = code[m];
        } else {
          o.r[k] = 0.f, o.d[k] = 0.f, o.c[k] = 0;
        }
      }
    };
    // halo face h (threads 0..159): x-halo for h < 32, y-halo otherwise
    const int h = threadIdx.x;
    int hx = -1, hy = -1, hrow = 0, hcol = 0;
    if (h < 2 * DZ_TY) {
      hrow = 1 + (h % DZ_TY);
      hcol = h < DZ_TY ? 0 : DZ_TX + 1;
      hx = h < DZ_TY ? x0 - 1 : x0 + DZ_TX;
      hy = y0 + h % DZ_TY;
    } else if (h < 2 * DZ_TY + 2 * DZ_TX) {
      const int j = h - 2 * DZ_TY;
      hcol = 1 + (j % DZ_TX);
      hrow = j < DZ_TX ? 0 : DZ_TY + 1;
      hx = x0 + j % DZ_TX;
      hy = j < DZ_TX ? y0 - 1 : y0 + DZ_TY;
    }
    float hr = 0.f, hd = 0.f;
    uint8_t hc = 0;
    auto load_halo = [&](int zz) {
      if (hx != -1 && zz < z1 && in_grid(hx, hy, zz)) {
        const int64_t m = hx + sy * hy + sz * zz;
        hr = rc[m], hd = di[m], hc = code[m];
      } else {
        hr = 0.f, hd = 0.f, hc = 0;
      }
    };

    float dmv[DZ_K], dcv[DZ_K], dpv[DZ_K];
    uint8_t cc[DZ_K];
    Raw c1, c2;
    {
      Raw c0;
      load_own(z0 - 1, c0);
      load_own(z0, c1);
#pragma unroll
      for (int k = 0; k < DZ_K; ++k) {
        dmv[k] = dir_of(c0.r[k], c0.d[k], c0.c[k]);
        dcv[k] = dir_of(c1.r[k], c1.d[k], c1.c[k]);
        cc[k] = c1.c[k];
      }
    }
    load_own(z0 + 1, c1);
    load_halo(z0);
    for (int zz = z0; zz < z1; ++zz) {
      const float hv = dir_of(hr, hd, hc);
      uint8_t cn[DZ_K];
#pragma unroll
      for (int k = 0; k < DZ_K; ++k) {
        dpv[k] = dir_of(c1.r[k], c1.d[k], c1.c[k]);
        cn[k] = c1.c[k];
      }
      // next loads before the barrier
      load_own(zz + 2, c2);
      load_halo(zz + 1);
      float(&sd)[DZ_TY + 2][DZ_TX + 2] = sd2[zz & 1];
#pragma unroll
      for (int k = 0; k < DZ_K; ++k) sd[1 + tg + 4 * k][1 + tx] = dcv[k];
      if (hx != -1) sd[hrow][hcol] = hv;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < DZ_K; ++k) {
        const int y = y0 + tg + 4 * k;
        if (x < dm3.nx && y < dm3.ny) {
          const int row = 1 + tg + 4 * k, col = 1 + tx;
          const uint8_t cd = cc[k];
          const float dcur = dcv[k];
          float acc = 0.f;
          if (cd & 1) acc += sd[row][col - 1] - dcur;
          if (cd & 2) acc += sd[row][col + 1] - dcur;
          if (cd & 4) acc += sd[row - 1][col] - dcur;
          if (cd & 8) acc += sd[row + 1][col] - dcur;
          if (cd & 16) acc += dmv[k] - dcur;
          if (cd & 32) acc += dpv[k] - dcur;
          const bool act = (cd & FC_ACTIVE) != 0;
          const float qv = act ? dcur - alpha * acc : 0.f;
          const float dv = act ? dcur : 0.f;
          const int64_t m = x + sy * y + sz * zz;
          dout[m] = dv;
          qc[m] = qv;
          v[0] += (double)dv * (double)qv;
        }
      }
#pragma unroll
      for (int k = 0; k < DZ_K; ++k) dmv[k] = dcv[k], dcv[k] = dpv[k], cc[k] = cn[k];
      c1 = c2;
    }
  }
  store_partials<1>(v, partials, comp * gridDim.x + lb);
}

__global__ void __launch_bounds__(kBlock)
    k_dcg_update(const uint8_t* __restrict__ fcode, float alpha, double* __restrict__ x,
                 float* __restrict__ r, const float* __restrict__ d, const float* __restrict__ q,
                 int64_t F, const double* __restrict__ scal, const int* __restrict__ flags,
                 double* partials, int* __restrict__ work) {
  if (flags[F_DONE]) return;
  count_work(work);
  const int comp = blockIdx.y;
  const double a = scal[S_RZ] / scal[S_DQ];
  const float af = (float)a;
  const uint8_t* __restrict__ code = fcode + comp * F;
  double* __restrict__ xc = x + comp * F;
  float* __restrict__ rc = r + comp * F;
  const float* __restrict__ dc = d + comp * F;
  const float* __restrict__ qc = q + comp * F;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(F, gridDim.x, lb);
  // [r.M^-1 r, |r|^2 for the early stop]
  double v[2] = {0.0, 0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    const uint8_t cd = code[idx];
    if (!(cd & FC_ACTIVE)) continue;
    xc[idx] += a * (double)dc[idx];
    const float rn = rc[idx] - af * qc[idx];
    rc[idx] = rn;
    v[0] += (double)rn * (double)rn * mrow_diag_inv(cd, alpha);
    v[1] += (double)rn * (double)rn;
  }
  store_partials<2>(v, partials, comp * gridDim.x + lb);
}

__global__ void __launch_bounds__(kBlock)
    k_dcg_check(int n, const uint8_t* __restrict__ fcode, float alpha, const float* __restrict__ b,
                const double* __restrict__ x, float* __restrict__ r, int64_t F,
                const int* __restrict__ flags, double* partials) {
  if (flags[F_DONE] == 1 || flags[F_DONE] == 2) return;  // runs after an early stop (3)
  const int comp = blockIdx.y;
  const Dims d = face_dims(n, comp);
  const int64_t sy = d.nx, sz = (int64_t)d.nx * d.ny;
  const uint8_t* __restrict__ code = fcode + comp * F;
  const float* __restrict__ bc = b + comp * F;
  const double* __restrict__ xc = x + comp * F;
  float* __restrict__ rc = r + comp * F;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const Chunk2 ch = chunk_of(F, gridDim.x, lb);
  double v[2] = {0.0, 0.0};
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock) {
    const uint8_t cd = code[idx];
    if (!(cd & FC_ACTIVE)) continue;
    const double rv = (double)bc[idx] - mrow<double>(xc, idx, cd, sy, sz, (double)alpha);
    const float rf = (float)rv;
    rc[idx] = rf;
    v[0] += rv * rv;
    v[1] += (double)rf * rf * mrow_diag_inv(cd, alpha);
  }
  store_partials<2>(v, partials, comp * gridDim.x + lb);
}

// out = (float) x on active faces, 0 elsewhere
__global__ void __launch_bounds__(kBlock)
    k_dcg_finish(const uint8_t* __restrict__ fcode, const double* __restrict__ x, F3 out,
                 int64_t F) {
  const int comp = blockIdx.y;
  const uint8_t* __restrict__ code = fcode + comp * F;
  const double* __restrict__ xc = x + comp * F;
  const Chunk2 ch = chunk_of(F, gridDim.x, xcd_logical_block(blockIdx.x, gridDim.x));
  for (int64_t idx = ch.begin + threadIdx.x; idx < ch.end; idx += kBlock)
    out.c[comp][idx] = (code[idx] & FC_ACTIVE) ? (float)xc[idx] : 0.f;
}

void launch_dcg_init(sim_ctx* c, float alpha) {
  hipLaunchKernelGGL(k_dcg_init, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->n,
                     c->fcode, alpha, c->tmp, c->fx, c->fr, c->fdA, c->F, c->partials);
  launch_finalize(c, 3 * c->grid_faces, 3, FIN_DCG_INIT, tol_sq(c->desc.diff_tol), 1, 0, 0.0, 0);
}

void launch_dcg_dir_spmv(sim_ctx* c, float alpha, const float* d_in, float* d_out) {
  prof_mark(c, SIM_KERN_DCG_DIR_SPMV, true);
  const DcgZmShape sh = dcg_zm_shape(c->n);
  const int nb = sh.tiles * sh.chunks;
  if (3 * nb <= kPartialDoubles) {
    hipLaunchKernelGGL(k_dcg_dir_spmv_zm, dim3(nb, 3), dim3(kBlock), 0, c->stream, c->n, c->fcode,
                       alpha, c->fr, d_in, d_out, c->fq, c->F, c->scal, c->flags, c->partials,
                       c->work + SIM_KERN_DCG_DIR_SPMV);
    prof_mark(c, SIM_KERN_DCG_DIR_SPMV, false);
    launch_finalize(c, 3 * nb, 1, FIN_DQ, 0.0, 0, 0, 0.0, 0);
    return;
  }
  hipLaunchKernelGGL(k_dcg_dir_spmv, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->n,
                     c->fcode, alpha, c->fr, d_in, d_out, c->fq, c->F, c->scal, c->flags,
                     c->partials, c->work + SIM_KERN_DCG_DIR_SPMV);
  prof_mark(c, SIM_KERN_DCG_DIR_SPMV, false);
  launch_finalize(c, 3 * c->grid_faces, 1, FIN_DQ, 0.0, 0, 0, 0.0, 0);
}

void launch_dcg_update(sim_ctx* c, float alpha, const float* d, double tol) {
  prof_mark(c, SIM_KERN_DCG_UPDATE, true);
  hipLaunchKernelGGL(k_dcg_update, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->fcode,
                     alpha, c->fx, c->fr, d, c->fq, c->F, c->scal, c->flags, c->partials,
                     c->work + SIM_KERN_DCG_UPDATE);
  prof_mark(c, SIM_KERN_DCG_UPDATE, false);
  // the iterate is updated every iteration, so the block may end as soon as
  // the recursive |r|^2 meets the tolerance (the FP64 check at its end decides)
  launch_finalize(c, 3 * c->grid_faces, 2, FIN_DCG_UPD, tol_sq(tol), 1, 0, 0.0, 0);
}

void launch_dcg_check(sim_ctx* c, float alpha, double tol) {
  hipLaunchKernelGGL(k_dcg_check, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->n,
                     c->fcode, alpha, c->tmp, c->fx, c->fr, c->F, c->flags, c->partials);
  launch_finalize(c, 3 * c->grid_faces, 2, FIN_CHECK, tol_sq(tol), 1, 0, 0.0, 0);
}

void launch_dcg_finish(sim_ctx* c, F3 out) {
  hipLaunchKernelGGL(k_dcg_finish, dim3(c->grid_faces, 3), dim3(kBlock), 0, c->stream, c->fcode,
                     c->fx, out, c->F);
}

}  // namespace fs
