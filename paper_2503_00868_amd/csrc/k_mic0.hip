// MIC(0) preconditioner for the pressure Poisson matrix.
//
// Modified incomplete Cholesky of level 0 with tau = 0.97 and safety
// factor sigma = 0.25, in lexicographic cell order (x fastest), as in the
// fluid-simulation text the paper defers to for its solver details
// (Section 3.2.2).  The factor and both triangular solves have a dependency
// along i+j+k: every cell needs its three lower (or upper) neighbours.  The
// GPU processes one hyperplane i+j+k = s per launch; all cells of a plane
// are independent.  That reproduces the sequential order exactly, so the
// iterates match a sequential implementation up to rounding, at the cost of
// 3n-2 dependent launches per sweep (latency-bound, not bandwidth-bound).
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

// q_c = (r_c + sum over lower liquid neighbours m of precon_m q_m) precon_c
__global__ void k_mic0_fwd_plane(int n, int s, int k_lo, int k_count,
                                 const uint8_t* __restrict__ cdiag,
                                 const float* __restrict__ precon, const float* __restrict__ r,
                                 float* __restrict__ q, const int* __restrict__ flags) {
  if (flags && flags[F_DONE]) return;
  int i, j, k;
  if (!plane_cell(n, s, k_lo, k_count, i, j, k)) return;
  const int64_t c = i + (int64_t)n * (j + (int64_t)n * k);
  if (!cdiag[c]) {
    q[c] = 0.f;
    return;
  }
  float t = r[c];
  const int64_t sy = n, sz = (int64_t)n * n;
  if (i > 0 && cdiag[c - 1]) t += precon[c - 1] * q[c - 1];
  if (j > 0 && cdiag[c - sy]) t += precon[c - sy] * q[c - sy];
  if (k > 0 && cdiag[c - sz]) t += precon[c - sz] * q[c - sz];
  q[c] = t * precon[c];
}

// z_c = (q_c + precon_c * sum over upper liquid neighbours m of z_m) precon_c
__global__ void k_mic0_bwd_plane(int n, int s, int k_lo, int k_count,
                                 const uint8_t* __restrict__ cdiag,
                                 const float* __restrict__ precon, const float* __restrict__ q,
                                 float* __restrict__ z, const int* __restrict__ flags) {
  if (flags && flags[F_DONE]) return;
  int i, j, k;
  if (!plane_cell(n, s, k_lo, k_count, i, j, k)) return;
  const int64_t c = i + (int64_t)n * (j + (int64_t)n * k);
  if (!cdiag[c]) {
    z[c] = 0.f;
    return;
  }
  const int64_t sy = n, sz = (int64_t)n * n;
  float acc = 0.f;
  if (i < n - 1 && cdiag[c + 1]) acc += z[c + 1];
  if (j < n - 1 && cdiag[c + sy]) acc += z[c + sy];
  if (k < n - 1 && cdiag[c + sz]) acc += z[c + sz];
  const float p = precon[c];
  z[c] = (q[c] + p * acc) * p;
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
  prof_mark(c, SIM_KERN_MIC0, true);
  for (int s = 0; s <= 3 * (n - 1); ++s) {
    PlaneRange pr = plane_range(n, s);
    int threads = n * pr.k_count;
    hipLaunchKernelGGL(k_mic0_fwd_plane, dim3((threads + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       c->stream, n, s, pr.k_lo, pr.k_count, c->cdiag, c->precon, r, c->mq, flags);
  }
  for (int s = 3 * (n - 1); s >= 0; --s) {
    PlaneRange pr = plane_range(n, s);
    int threads = n * pr.k_count;
    hipLaunchKernelGGL(k_mic0_bwd_plane, dim3((threads + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       c->stream, n, s, pr.k_lo, pr.k_count, c->cdiag, c->precon, c->mq, z, flags);
  }
  prof_mark(c, SIM_KERN_MIC0, false);
}

}  // namespace fs
