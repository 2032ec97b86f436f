// MIC(0) preconditioner for the pressure Poisson matrix.
//
// Modified incomplete Cholesky of level 0 with tau = 0.97 and safety
// factor sigma = 0.25, in lexicographic cell order (x fastest), as in the
// fluid-simulation text the paper defers to for its solver details
// (Section 3.2.2).  The factor and both triangular solves have a dependency
// along i+j+k: every cell needs its three lower (or upper) neighbours.
//
// The factor (once per mask) processes one cell hyperplane i+j+k = s per
// launch.  The two triangular solves of every application go by 8^3 tiles:
// tiles on one tile hyperplane I+J+K = S are independent (their cells'
// neighbours across tile faces lie in tiles of S-1, or S+1 going back), so
// one launch per tile hyperplane, 3(n/8)-2 per sweep instead of 3n-2.  A
// tile is one wave: lane (i', j') owns a column and takes cell k' at level
// i'+j'+k'; the three neighbours a cell needs were produced at the level
// before by lanes (i'-1, j'), (i', j'-1) and itself, so a level is two
// cross-lane shuffles (16^3 tiles of four waves, with a barrier per level,
// measured slower).  The order of the operations per cell is the
// sequential one, so the result matches a sequential sweep up to rounding.
#include "common.h"
#include "ctx.h"

namespace fs {

constexpr double kMicTau = 0.97;
constexpr double kMicSigma = 0.25;

struct PlaneRange {
  int k_lo, k_count;
};

static PlaneRange plane_range(int n, int s) {
  int lo = s - 2 * (n - 1);
  if (lo < 0) lo = 0;
  int hi = s < n - 1 ? s : n - 1;
  return PlaneRange{lo, hi - lo + 1};
}

__device__ inline bool plane_cell(int n, int s, int k_lo, int k_count, int& i, int& j, int& k) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * k_count) return false;
  j = t % n;
  k = k_lo + t / n;
  i = s - j - k;
  return i >= 0 && i < n;
}

__device__ inline bool liquid(const uint8_t* cdiag, int n, int i, int j, int k) {
  if ((unsigned)i >= (unsigned)n || (unsigned)j >= (unsigned)n || (unsigned)k >= (unsigned)n)
    return false;
  return cdiag[i + (int64_t)n * (j + (int64_t)n * k)] != 0;
}

__global__ void k_mic0_setup_plane(int n, int s, int k_lo, int k_count,
                                   const uint8_t* __restrict__ cdiag, float* __restrict__ precon) {
  int i, j, k;
  if (!plane_cell(n, s, k_lo, k_count, i, j, k)) return;
  const int64_t c = i + (int64_t)n * (j + (int64_t)n * k);
  const uint8_t dg = cdiag[c];
  if (!dg) {
    precon[c] = 0.f;
    return;
  }
  double e = (double)dg;
  const int di[3] = {1, 0, 0}, dj[3] = {0, 1, 0}, dk[3] = {0, 0, 1};
  for (int a = 0; a < 3; ++a) {
    const int mi = i - di[a], mj = j - dj[a], mk = k - dk[a];
    if (!liquid(cdiag, n, mi, mj, mk)) continue;
    const double pm = (double)precon[mi + (int64_t)n * (mj + (int64_t)n * mk)];
    int other = 0;
    for (int b = 0; b < 3; ++b)
      if (b != a) other += liquid(cdiag, n, mi + di[b], mj + dj[b], mk + dk[b]);
    e -= pm * pm;
    e -= kMicTau * (double)other * pm * pm;
  }
  if (e < kMicSigma * (double)dg) e = (double)dg;
  precon[c] = (float)(1.0 / sqrt(e));
}

constexpr int MT = 8;  // tile edge of the triangular solves: one wave per tile

// Forward substitution on tile (I, J, S - I - J): q_c = (r_c + sum over the
// lower liquid neighbours m of precon_m q_m) precon_c, zero off liquid.
// Block = one wave, lane (i', j') = (lane % 8, lane / 8); grid (tiles_x,
// tiles_y), the blocks off the hyperplane return at once (a grid of just the
// hyperplane's tiles, found by a loop over rows, measured slower).  Each
// lane's column inputs (r, precon, and what the neighbours across the tile's
// x- and y-faces contribute) sit in LDS, one 16-byte word per cell, so that a level reads its cell with one LDS load; the x- and
// y-neighbours inside the tile come from the lanes beside it by shuffles.
__global__ void __launch_bounds__(64)
    k_mic0_fwd_tile(int n, int S, const uint8_t* __restrict__ cdiag,
                    const float* __restrict__ precon, const float* __restrict__ r,
                    float* __restrict__ q, const int* __restrict__ flags) {
  if (flags && flags[F_DONE]) return;
  __shared__ float4 in_l[MT][64];
  __shared__ float out_l[MT][64];
  const int tn = (n + MT - 1) / MT;
  const int I = blockIdx.x, J = blockIdx.y, K = S - I - J;
  if (K < 0 || K >= tn) return;
  const int lane = threadIdx.x, li = lane % MT, lj = lane / MT;
  const int x = I * MT + li, y = J * MT + lj, z0 = K * MT;
  const bool col_ok = x < n && y < n;
  const int64_t sy = n, sz = (int64_t)n * n;
  // precon_m q_m of the neighbours across the tile's faces (zero outside
  // the box and off liquid, where precon and q are zero).  Every load is
  // issued from a valid (clamped) address and masked afterwards, so that the
  // wave waits for one load latency, not one per conditional load.
  const bool fx = col_ok && li == 0 && x > 0, fy = col_ok && lj == 0 && y > 0;
  const bool fz = col_ok && z0 > 0;
  float rv[MT], pv[MT], pxm[MT], qxm[MT], pym[MT], qym[MT];
  uint8_t cv[MT];
#pragma unroll
  for (int k = 0; k < MT; ++k) {
    const bool ok = col_ok && z0 + k < n;
    const int64_t c = x + sy * y + sz * (z0 + k);
    const int64_t a = ok ? c : 0, ax = ok && fx ? c - 1 : 0, ay = ok && fy ? c - sy : 0;
    rv[k] = r[a];
    pv[k] = precon[a];
    cv[k] = cdiag[a];
    pxm[k] = precon[ax];
    qxm[k] = q[ax];
    pym[k] = precon[ay];
    qym[k] = q[ay];
  }
  const int64_t az = fz ? x + sy * y + sz * (z0 - 1) : 0;
  const float pzm = precon[az], qzm = q[az];
#pragma unroll
  for (int k = 0; k < MT; ++k) {
    const bool ok = col_ok && z0 + k < n;
    float4 v;
    v.x = ok && cv[k] ? rv[k] : 0.f;
    v.y = ok ? pv[k] : 0.f;
    v.z = ok && fx ? pxm[k] * qxm[k] : 0.f;
    v.w = ok && fy ? pym[k] * qym[k] : 0.f;
    in_l[k][lane] = v;
  }
  const float wz = fz ? pzm * qzm : 0.f;
  wave_sync();
  float w_last = 0.f;  // precon q of this lane's previous cell
#pragma unroll
  for (int L = 0; L < 3 * MT - 2; ++L) {
    const float from_x = __shfl(w_last, (lane + 63) & 63);  // lane (i' - 1, j')
    const float from_y = __shfl(w_last, (lane + 56) & 63);  // lane (i', j' - 1)
    const int k = L - li - lj;
    if (k >= 0 && k < MT) {
      const float4 v = in_l[k][lane];
      float t = v.x;
      t += li > 0 ? from_x : v.z;
      t += lj > 0 ? from_y : v.w;
      t += k > 0 ? w_last : wz;
      const float qc = t * v.y;
      out_l[k][lane] = qc;
      w_last = v.y * qc;
    }
  }
  wave_sync();
  if (col_ok) {
#pragma unroll
    for (int k = 0; k < MT; ++k)
      if (z0 + k < n) q[x + sy * y + sz * (z0 + k)] = out_l[k][lane];
  }
}

// Back substitution on tile (I, J, S - I - J): z_c = (q_c + precon_c sum over
// the upper liquid neighbours m of z_m) precon_c, zero off liquid; the levels
// in reverse, the neighbours from lanes (i' + 1, j'), (i', j' + 1).
__global__ void __launch_bounds__(64)
    k_mic0_bwd_tile(int n, int S, const uint8_t* __restrict__ cdiag,
                    const float* __restrict__ precon, const float* __restrict__ q,
                    float* __restrict__ zout, const int* __restrict__ flags) {
  if (flags && flags[F_DONE]) return;
  __shared__ float4 in_l[MT][64];
  __shared__ float out_l[MT][64];
  const int tn = (n + MT - 1) / MT;
  const int I = blockIdx.x, J = blockIdx.y, K = S - I - J;
  if (K < 0 || K >= tn) return;
  const int lane = threadIdx.x, li = lane % MT, lj = lane / MT;
  const int x = I * MT + li, y = J * MT + lj, z0 = K * MT;
  const bool col_ok = x < n && y < n;
  const int64_t sy = n, sz = (int64_t)n * n;
  // all loads from valid (clamped) addresses first, masked afterwards (as in
  // the forward sweep)
  const bool fx = col_ok && li == MT - 1 && x + 1 < n, fy = col_ok && lj == MT - 1 && y + 1 < n;
  const int ztop = z0 + MT;
  const bool fz = col_ok && ztop < n;
  float qv[MT], pv[MT], zxm[MT], zym[MT];
#pragma unroll
  for (int k = 0; k < MT; ++k) {
    const bool ok = col_ok && z0 + k < n;
    const int64_t c = x + sy * y + sz * (z0 + k);
    const int64_t a = ok ? c : 0, ax = ok && fx ? c + 1 : 0, ay = ok && fy ? c + sy : 0;
    qv[k] = q[a];
    pv[k] = precon[a];
    zxm[k] = zout[ax];
    zym[k] = zout[ay];
  }
  const float zzm = zout[fz ? x + sy * y + sz * ztop : 0];
#pragma unroll
  for (int k = 0; k < MT; ++k) {
    const bool ok = col_ok && z0 + k < n;
    float4 v;
    v.x = ok ? qv[k] : 0.f;
    v.y = ok ? pv[k] : 0.f;
    v.z = ok && fx ? zxm[k] : 0.f;
    v.w = ok && fy ? zym[k] : 0.f;
    in_l[k][lane] = v;
  }
  const float uz = fz ? zzm : 0.f;
  wave_sync();
  float z_last = 0.f;  // z of this lane's previous (upper) cell
#pragma unroll
  for (int L = 3 * MT - 3; L >= 0; --L) {
    const float from_x = __shfl(z_last, (lane + 1) & 63);  // lane (i' + 1, j')
    const float from_y = __shfl(z_last, (lane + 8) & 63);  // lane (i', j' + 1)
    const int k = L - li - lj;
    if (k >= 0 && k < MT) {
      const float4 v = in_l[k][lane];
      float acc = 0.f;
      acc += li < MT - 1 ? from_x : v.z;
      acc += lj < MT - 1 ? from_y : v.w;
      acc += k < MT - 1 ? z_last : uz;
      const float zc = (v.x + v.y * acc) * v.y;
      out_l[k][lane] = zc;
      z_last = zc;
    }
  }
  wave_sync();
  if (col_ok) {
#pragma unroll
    for (int k = 0; k < MT; ++k)
      if (z0 + k < n) zout[x + sy * y + sz * (z0 + k)] = out_l[k][lane];
  }
}

void launch_mic0_setup(sim_ctx* c) {
  const int n = c->n;
  for (int s = 0; s <= 3 * (n - 1); ++s) {
    PlaneRange pr = plane_range(n, s);
    int threads = n * pr.k_count;
    hipLaunchKernelGGL(k_mic0_setup_plane, dim3((threads + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       c->stream, n, s, pr.k_lo, pr.k_count, c->cdiag, c->precon);
  }
}

void launch_mic0_apply(sim_ctx* c, const float* r, float* z, const int* flags) {
  const int n = c->n;
  const int tn = (n + MT - 1) / MT;
  prof_mark(c, SIM_KERN_MIC0, true);
  for (int S = 0; S <= 3 * (tn - 1); ++S)
    hipLaunchKernelGGL(k_mic0_fwd_tile, dim3(tn, tn), dim3(64), 0, c->stream, n, S, c->cdiag,
                       c->precon, r, c->mq, flags);
  for (int S = 3 * (tn - 1); S >= 0; --S)
    hipLaunchKernelGGL(k_mic0_bwd_tile, dim3(tn, tn), dim3(64), 0, c->stream, n, S, c->cdiag,
                       c->precon, c->mq, z, flags);
  prof_mark(c, SIM_KERN_MIC0, false);
}

}  // namespace fs
