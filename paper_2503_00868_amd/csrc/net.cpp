// Learned preconditioner: workspace layout, weight packing, the U-Net forward
// pass used inside flexible CG, and one batched training step (forward,
// A-norm loss, backward, Adam) on (residual, error) pairs.
//
// Architecture (a reading of the paper's learned pressure solver, Section
// 3.4.1, used here as a preconditioner):
//   x0 = (r/rms(r), mask) -> c1 2->16 -> c2 16->16 = e1          (level 1, n^3)
//   pool -> c3 16->32 -> c4 32->32 = e2                          (level 2)
//   pool -> c5 32->64 -> c6 64->64 = e3                          (level 3)
//   cat(up e3, e2) -> c7 96->32 -> c8 32->32 = d2                (level 2)
//   cat(up d2, e1) -> c9 48->16 -> c10 16->16 = d1               (level 1)
//   c11 16->1 -> o ; z = mask * rms * o
// ReLU after every convolution except c11; all convolutions 3x3x3, bias free.
#include "net.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "common.h"

namespace fs {

struct Layer {
  int cin, cout;   // real channel counts
  int cin_p;       // forward input channels as stored (multiple of 8)
  int cout_p;      // forward output channels as computed (multiple of 16)
  int cout_pd;     // data-gradient input channels (multiple of 8)
};

static const Layer kLayers[11] = {
    {2, 16, 8, 16, 16},   {16, 16, 16, 16, 16}, {16, 32, 16, 32, 32}, {32, 32, 32, 32, 32},
    {32, 64, 32, 64, 64}, {64, 64, 64, 64, 64}, {96, 32, 96, 32, 32}, {32, 32, 32, 32, 32},
    {48, 16, 48, 16, 16}, {16, 16, 16, 16, 16}, {16, 1, 16, 16, 8},
};

static int64_t param_offset(int l) {
  int64_t o = 0;
  for (int q = 0; q < l; ++q) o += 27LL * kLayers[q].cin * kLayers[q].cout;
  return o;
}

static int64_t param_total() { return param_offset(11); }

// Activity maps of the inference pass: map Mi_r covers the level with i
// halvings (0: full resolution) and radius r in fine voxels (see
// activity_maps for what the radii are).
enum MapId { M0_0, M0_1, M0_2, M1_2, M1_3, M1_5, M1_7, M2_5, kNetMaps };
constexpr int kMaps = kNetMaps;
constexpr int kMapLevel[kMaps] = {0, 0, 0, 1, 1, 1, 1, 2};
constexpr int kMapRadius[kMaps] = {0, 1, 2, 2, 3, 5, 7, 5};

}  // namespace fs

struct UNetState {
  int n1, n2, n3;
  // activations (bf16, channels-last)
  __bf16 *X0, *A1, *E1, *B1, *D1, *P1, *A2, *E2, *B2, *D2, *P2, *A3, *E3;
  // gradients
  __bf16 *G11, *L1a, *L1b, *L1T, *L2a, *L2b, *L2T, *L2c, *L3a, *L3b, *L3c;
  // weights: forward and data-gradient layouts
  __bf16* wf[11];
  __bf16* wd[11];
  // decoder layers c7 (index 6) and c9 (index 8) in the forward pass: the
  // upsampled half as per-parity coarse weights, the skip half separately,
  // and the fp16 partial sums of the upsampled half (fine layout)
  __bf16 *weff7, *wskip7, *weff9, *wskip9;
  _Float16 *T2, *T1;
  // tile-plane activity maps (device), and whether the inference pass uses
  // them
  uint8_t* act[fs::kNetMaps];
  bool skip_tiles = true;
  float* dW;
  float* zbuf;
  float* Az;
  bool ready = false;
};

namespace fs {

namespace {

struct Carve {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    size_t o = off;
    off = (off + count * sizeof(T) + 255) / 256 * 256;
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

size_t carve_net(int n, char* base, UNetState* s) {
  Carve cv{base};
  UNetState dummy;
  UNetState* t = s ? s : &dummy;
  const int64_t V1 = (int64_t)n * n * n, V2 = V1 / 8, V3 = V1 / 64;
  t->n1 = n;
  t->n2 = n / 2;
  t->n3 = n / 4;
  t->X0 = cv.take<__bf16>(V1 * 8);
  t->A1 = cv.take<__bf16>(V1 * 16);
  t->E1 = cv.take<__bf16>(V1 * 16);
  t->B1 = cv.take<__bf16>(V1 * 16);
  t->D1 = cv.take<__bf16>(V1 * 16);
  t->P1 = cv.take<__bf16>(V2 * 16);
  t->A2 = cv.take<__bf16>(V2 * 32);
  t->E2 = cv.take<__bf16>(V2 * 32);
  t->B2 = cv.take<__bf16>(V2 * 32);
  t->D2 = cv.take<__bf16>(V2 * 32);
  t->P2 = cv.take<__bf16>(V3 * 32);
  t->A3 = cv.take<__bf16>(V3 * 64);
  t->E3 = cv.take<__bf16>(V3 * 64);
  t->G11 = cv.take<__bf16>(V1 * 8);
  t->L1a = cv.take<__bf16>(V1 * 16);
  t->L1b = cv.take<__bf16>(V1 * 16);
  t->L1T = cv.take<__bf16>(V1 * 48);
  t->L2a = cv.take<__bf16>(V2 * 32);
  t->L2b = cv.take<__bf16>(V2 * 32);
  t->L2T = cv.take<__bf16>(V2 * 96);
  t->L2c = cv.take<__bf16>(V2 * 16);
  t->L3a = cv.take<__bf16>(V3 * 64);
  t->L3b = cv.take<__bf16>(V3 * 64);
  t->L3c = cv.take<__bf16>(V3 * 32);
  for (int l = 0; l < 11; ++l) {
    const Layer& L = kLayers[l];
    t->wf[l] = cv.take<__bf16>((size_t)L.cout_p * 28 * L.cin_p);
    t->wd[l] = cv.take<__bf16>((size_t)L.cin * 28 * L.cout_pd);
  }
  t->weff7 = cv.take<__bf16>((size_t)8 * 8 * 32 * 64);
  t->wskip7 = cv.take<__bf16>((size_t)32 * 28 * 32);
  t->weff9 = cv.take<__bf16>((size_t)8 * 8 * 16 * 32);
  t->wskip9 = cv.take<__bf16>((size_t)16 * 28 * 16);
  t->T2 = cv.take<_Float16>(V2 * 32);
  t->T1 = cv.take<_Float16>(V1 * 16);
  // each sized for the full-resolution level (n^3 / 256 bytes)
  for (int k = 0; k < kNetMaps; ++k) {
    const int64_t m = n, tpr = (m + 15) / 16;
    t->act[k] = cv.take<uint8_t>(tpr * tpr * m);
  }
  t->dW = cv.take<float>(param_total());
  t->zbuf = cv.take<float>(V1);
  t->Az = cv.take<float>(V1);
  return cv.off;
}

NetSrc src1(const __bf16* a, int ca, const uint8_t* act = nullptr) {
  return NetSrc{a, nullptr, ca, 0, 0, act};
}
NetSrc srcup(const __bf16* coarse, int cc, const __bf16* skip, int cs) {
  return NetSrc{coarse, skip, cc, cs, 1};
}
NetOut out_bf(__bf16* p, const uint8_t* act = nullptr) {
  return NetOut{p, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, act};
}
NetOut out_pool(__bf16* p, __bf16* pooled, const uint8_t* act) {
  return NetOut{p, nullptr, nullptr, nullptr, nullptr, nullptr, pooled, act};
}
NetOut out_mask(__bf16* p, const __bf16* relu_of) { return NetOut{p, nullptr, nullptr, nullptr, relu_of}; }

int conv(sim_ctx* c, int n, int l, int epi, NetSrc src, NetOut out, const int* flags) {
  const Layer& L = kLayers[l];
  if (!net_conv(c, n, L.cin_p, L.cout_p, epi, src, c->net->wf[l], out, flags)) {
    c->err = "no convolution kernel for this channel configuration";
    return SIM_ERR_INVALID_ARG;
  }
  return SIM_OK;
}

int dgrad(sim_ctx* c, int n, int l, int epi, const __bf16* G, NetOut out) {
  const Layer& L = kLayers[l];
  if (!net_conv(c, n, L.cout_pd, L.cin, epi, src1(G, L.cout_pd), c->net->wd[l], out, nullptr)) {
    c->err = "no data-gradient kernel for this channel configuration";
    return SIM_ERR_INVALID_ARG;
  }
  return SIM_OK;
}

// Concatenating layer: fp16 partial sums of the upsampled channels from the
// coarse grid, then the skip channels' convolution adds them before the ReLU.
// act_c, act_f (nullable): activity maps of the coarse and the fine level.
int split_conv(sim_ctx* c, int n, int cc, int cout, const __bf16* coarse, const __bf16* weff,
               _Float16* T, NetSrc skip, const __bf16* wskip, __bf16* out, const int* flags,
               const uint8_t* act_c, const uint8_t* act_f) {
  // the fine layer (32 coarse + 16 skip channels) in one pass
  if (cc == 32 && cout == 16 && skip.ca == 16 && !skip.b &&
      net_conv_cat(c, n, coarse, skip.a, weff, wskip, out, flags, act_f))
    return SIM_OK;
  if (!(net_upconv_cls(c, n, cc, cout, coarse, weff, T, flags, act_f) ||
        net_upconv(c, n, cc, cout, coarse, weff, T, flags, act_c)) ||
      !net_conv(c, n, skip.ca, cout, NET_EPI_RELU_ADD, skip, wskip,
                NetOut{out, nullptr, nullptr, nullptr, nullptr, T, nullptr, act_f}, flags)) {
    c->err = "no split convolution kernel for this channel configuration";
    return SIM_ERR_INVALID_ARG;
  }
  return SIM_OK;
}

void wgrad(sim_ctx* c, int n, int l, NetSrc src, const __bf16* G, int g_stride, float* dW) {
  const Layer& L = kLayers[l];
  net_wgrad(c, n, src, L.cin, L.cin_p, G, g_stride, L.cout, dW + param_offset(l));
}

// U-Net forward pass into z (fp32, n^3); activations stay in the workspace.
// keep_input (training): store the 2-channel input tensor (the weight
// gradient of c1 reads it) and compute every tile; otherwise c1 reads r and
// the mask directly, and the tiles the activity maps mark as zero are
// skipped.
int forward(sim_ctx* c, const float* r, float* z, const int* flags, bool keep_input,
            bool have_sumsq = false, const float* qdot = nullptr) {
  UNetState* s = c->net;
  const int n1 = s->n1, n2 = s->n2, n3 = s->n3;
  const bool skip = !keep_input && s->skip_tiles;
  auto A = [&](int id) -> const uint8_t* { return skip ? s->act[id] : nullptr; };
  if (!have_sumsq) launch_dot_cells_slot(c, r, r, S_NET_SUMSQ, flags);
  int rc = SIM_OK;
  if (keep_input) {
    net_input(c, r, c->scal + S_NET_SUMSQ, c->scal + S_NET_RMS, s->X0, flags);
    rc |= conv(c, n1, 0, NET_EPI_RELU, src1(s->X0, 8), out_bf(s->A1), flags);
  } else {
    net_conv_in(c, r, c->scal + S_NET_SUMSQ, c->scal + S_NET_RMS, s->wf[0], s->A1, flags, A(M0_1),
                c->work + SIM_KERN_NET);
  }
  // c2 and c4 also write the 2x2x2 average pool of their output
  rc |= conv(c, n1, 1, NET_EPI_RELU_POOL, src1(s->A1, 16), out_pool(s->E1, s->P1, A(M0_2)), flags);
  rc |= conv(c, n2, 2, NET_EPI_RELU, src1(s->P1, 16), out_bf(s->A2, A(M1_5)), flags);
  rc |= conv(c, n2, 3, NET_EPI_RELU_POOL, src1(s->A2, 32), out_pool(s->E2, s->P2, A(M1_7)), flags);
  rc |= conv(c, n3, 4, NET_EPI_RELU, src1(s->P2, 32), out_bf(s->A3), flags);
  rc |= conv(c, n3, 5, NET_EPI_RELU, src1(s->A3, 64), out_bf(s->E3), flags);
  // c7 = ReLU(upsampled half, on the coarse grid + skip half), likewise c9
  rc |= split_conv(c, n2, 64, 32, s->E3, s->weff7, s->T2, src1(s->E2, 32, A(M1_7)), s->wskip7, s->B2,
                   flags, A(M2_5), A(M1_5));
  rc |= conv(c, n2, 7, NET_EPI_RELU, src1(s->B2, 32, A(M1_5)), out_bf(s->D2, A(M1_3)), flags);
  rc |= split_conv(c, n1, 32, 16, s->D2, s->weff9, s->T1, src1(s->E1, 16, A(M0_2)), s->wskip9, s->B1,
                   flags, A(M1_2), A(M0_2));
  rc |= conv(c, n1, 9, NET_EPI_RELU, src1(s->B1, 16, A(M0_2)), out_bf(s->D1, A(M0_1)), flags);
  net_conv_out(c, n1, s->D1, s->wf[10], z, c->scal + S_NET_RMS, flags, A(M0_1), A(M0_0), qdot);
  return rc ? SIM_ERR_INVALID_ARG : SIM_OK;
}

// Gradient of the loss of one pair with respect to every weight, added to dW.
int backward(sim_ctx* c) {
  UNetState* s = c->net;
  const int n1 = s->n1, n2 = s->n2, n3 = s->n3;
  float* dW = s->dW;
  int rc = SIM_OK;
  // output convolution
  wgrad(c, n1, 10, src1(s->D1, 16), s->G11, 8, dW);
  rc |= dgrad(c, n1, 10, NET_EPI_MASKGRAD, s->G11, out_mask(s->L1a, s->D1));   // G10
  wgrad(c, n1, 9, src1(s->B1, 16), s->L1a, 16, dW);
  rc |= dgrad(c, n1, 9, NET_EPI_MASKGRAD, s->L1a, out_mask(s->L1b, s->B1));    // G9
  wgrad(c, n1, 8, srcup(s->D2, 32, s->E1, 16), s->L1b, 16, dW);
  rc |= dgrad(c, n1, 8, NET_EPI_RAW, s->L1b, out_bf(s->L1T));                  // T48
  net_upsum_mask(c, n1, 32, 48, s->L1T, s->D2, s->L2a);                        // G8
  wgrad(c, n2, 7, src1(s->B2, 32), s->L2a, 32, dW);
  rc |= dgrad(c, n2, 7, NET_EPI_MASKGRAD, s->L2a, out_mask(s->L2b, s->B2));    // G7
  wgrad(c, n2, 6, srcup(s->E3, 64, s->E2, 32), s->L2b, 32, dW);
  rc |= dgrad(c, n2, 6, NET_EPI_RAW, s->L2b, out_bf(s->L2T));                  // T96
  net_upsum_mask(c, n2, 64, 96, s->L2T, s->E3, s->L3a);                        // G6
  wgrad(c, n3, 5, src1(s->A3, 64), s->L3a, 64, dW);
  rc |= dgrad(c, n3, 5, NET_EPI_MASKGRAD, s->L3a, out_mask(s->L3b, s->A3));    // G5
  wgrad(c, n3, 4, src1(s->P2, 32), s->L3b, 64, dW);
  rc |= dgrad(c, n3, 4, NET_EPI_RAW, s->L3b, out_bf(s->L3c));                  // grad P2
  net_skip_grad(c, n2, 32, s->L2T, 96, 64, s->L3c, s->E2, s->L2a);             // G4
  wgrad(c, n2, 3, src1(s->A2, 32), s->L2a, 32, dW);
  rc |= dgrad(c, n2, 3, NET_EPI_MASKGRAD, s->L2a, out_mask(s->L2b, s->A2));    // G3
  wgrad(c, n2, 2, src1(s->P1, 16), s->L2b, 32, dW);
  rc |= dgrad(c, n2, 2, NET_EPI_RAW, s->L2b, out_bf(s->L2c));                  // grad P1
  net_skip_grad(c, n1, 16, s->L1T, 48, 32, s->L2c, s->E1, s->L1a);             // G2
  wgrad(c, n1, 1, src1(s->A1, 16), s->L1a, 16, dW);
  rc |= dgrad(c, n1, 1, NET_EPI_MASKGRAD, s->L1a, out_mask(s->L1b, s->A1));    // G1
  wgrad(c, n1, 0, src1(s->X0, 8), s->L1b, 16, dW);
  return rc ? SIM_ERR_INVALID_ARG : SIM_OK;
}

void pack_all(sim_ctx* c, const float* master) {
  for (int l = 0; l < 11; ++l) {
    const Layer& L = kLayers[l];
    net_pack_weights(c, master + param_offset(l), L.cin, L.cout, L.cin_p, L.cout_p, L.cout_pd,
                     c->net->wf[l], c->net->wd[l]);
  }
  net_pack_split(c, master + param_offset(6), 96, 32, 64, 32, c->net->weff7, c->net->wskip7);
  net_pack_split(c, master + param_offset(8), 48, 16, 32, 16, c->net->weff9, c->net->wskip9);
}

// Which tiles the inference pass computes.  Distances are Chebyshev
// distances d, in fine voxels, to the nearest liquid cell; a voxel of a
// coarser level stands for its fine block.
//
// Non-zero bound: the convolutions are bias-free, every activation but the
// output is a ReLU or a pooling of one, and the input (r / rms, mask)
// vanishes off liquid, so an activation is zero wherever its receptive field
// holds no liquid cell.  A 3x3x3 convolution at level l reaches 2^(l-1)
// fine voxels further, a 2x2x2 pooling adds 1 (level 2) or 2 (level 3) for
// the alignment to its block, nearest upsampling adds nothing: c1 <= 1,
// c2 <= 2, c3 <= 5, c4 <= 7, c6 <= 17, c8 <= 21, c10 <= 23.
//
// Needed bound: z is masked to liquid, so c11 needs c10's output only within
// d <= 1, which needs c9's within 2, whose upsampled half needs c8's within
// 3 (of a fine voxel of its block), which needs c7's within 3 + 2 = 5, which
// needs c4's within 7.  Values outside these sets never reach z.
//
// Each layer computes the tiles that hold a voxel within the smaller of its
// two bounds.  Skipped tiles of layers limited by the non-zero bound hold
// zeros (the workspace is cleared once and no pass writes anything else
// there); skipped tiles of layers limited by the needed bound may hold stale
// values, which only ever feed other unneeded values.
// (the maps, MapId, are listed with the network's constants above)

// dilation of a 0/1 volume by a cube of half-width r along one axis
void dilate_axis(std::vector<uint8_t>& a, int n, int axis, int r) {
  const int64_t s1 = axis == 0 ? n : 1, s2 = axis == 2 ? n : (int64_t)n * n;
  const int64_t st = axis == 0 ? 1 : axis == 1 ? n : (int64_t)n * n;
  std::vector<int> pre(n + 1);
  for (int64_t b = 0; b < n; ++b)
    for (int64_t a1 = 0; a1 < n; ++a1) {
      const int64_t base = a1 * s1 + b * s2;
      pre[0] = 0;
      for (int i = 0; i < n; ++i) pre[i + 1] = pre[i] + (a[base + i * st] != 0);
      for (int i = 0; i < n; ++i)
        a[base + i * st] = pre[std::min(n, i + r + 1)] - pre[std::max(0, i - r)] > 0;
    }
}

// Activity maps: maps[k][(z * tpr + ty) * tpr + tx] = 1 when a voxel of the
// 16 x 16 tile (tx, ty) of plane z of level kMapLevel[k], or of its
// one-voxel halo, has a fine block voxel within kMapRadius[k] of liquid.
void activity_maps(int n, const uint8_t* cell, std::vector<uint8_t> maps[kMaps]) {
  const int64_t C = (int64_t)n * n * n;
  std::vector<uint8_t> near(C);
  for (int64_t q = 0; q < C; ++q) near[q] = cell[q] == 1;
  int radius = 0;
  for (int r : {0, 1, 2, 3, 5, 7}) {
    // near: within r of liquid (dilations by a cube compose)
    for (int axis = 0; axis < 3 && r > radius; ++axis) dilate_axis(near, n, axis, r - radius);
    radius = r;
    for (int k = 0; k < kMaps; ++k) {
      if (kMapRadius[k] != r) continue;
      const int l = kMapLevel[k], m = n >> l, b = 1 << l, tpr = (m + 15) / 16;
      // level voxel live when any voxel of its fine block is
      std::vector<uint8_t> lv((size_t)m * m * m, 0);
      for (int z = 0; z < m * b; ++z)
        for (int y = 0; y < m * b; ++y)
          for (int x = 0; x < m * b; ++x)
            if (near[x + (int64_t)n * (y + (int64_t)n * z)])
              lv[x / b + (int64_t)m * (y / b + (int64_t)m * (z / b))] = 1;
      maps[k].assign((size_t)tpr * tpr * m, 0);
      for (int z = 0; z < m; ++z)
        for (int y = 0; y < m; ++y)
          for (int x = 0; x < m; ++x) {
            if (!lv[x + (int64_t)m * (y + (int64_t)m * z)]) continue;
            // every tile whose halo-extended square holds (x, y)
            for (int ty = std::max(0, (y - 16) / 16); ty <= std::min(tpr - 1, (y + 1) / 16); ++ty)
              for (int tx = std::max(0, (x - 16) / 16); tx <= std::min(tpr - 1, (x + 1) / 16); ++tx)
                if (x >= 16 * tx - 1 && x <= 16 * tx + 16 && y >= 16 * ty - 1 && y <= 16 * ty + 16)
                  maps[k][((size_t)z * tpr + ty) * tpr + tx] = 1;
          }
    }
  }
}

}  // namespace

size_t net_workspace_bytes(int n) { return carve_net(n, nullptr, nullptr); }

int net_init(sim_ctx* c, const uint8_t* h_cell) {
  UNetState* s = new (std::nothrow) UNetState();
  if (!s) return SIM_ERR_INVALID_ARG;
  carve_net(c->n, reinterpret_cast<char*>(c->net_ws), s);
  c->net = s;
  // the inference pass never writes the tiles it skips: clear the whole
  // network workspace once, so they read as zero
  std::vector<uint8_t> maps[kMaps];
  activity_maps(c->n, h_cell, maps);
  if (hipMemsetAsync(c->net_ws, 0, c->net_ws_bytes, c->stream) != hipSuccess) return SIM_ERR_HIP;
  for (int k = 0; k < kMaps; ++k)
    if (hipMemcpyAsync(s->act[k], maps[k].data(), maps[k].size(), hipMemcpyHostToDevice,
                       c->stream) != hipSuccess)
      return SIM_ERR_HIP;
  // the host vectors must outlive the copies
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SIM_ERR_HIP;
  return SIM_OK;
}

void net_destroy(sim_ctx* c) {
  delete c->net;
  c->net = nullptr;
}

bool net_ready(const sim_ctx* c) { return c->net && c->net->ready; }

int net_apply(sim_ctx* c, const float* r, float* z, const int* flags, bool have_sumsq,
              const float* qdot) {
  prof_mark(c, SIM_KERN_NET, true);
  int rc = forward(c, r, z, flags, false, have_sumsq, qdot);
  prof_mark(c, SIM_KERN_NET, false);
  return rc;
}

}  // namespace fs

using namespace fs;

extern "C" {

int sim_net_param_count(int64_t* count) {
  if (!count) return SIM_ERR_INVALID_ARG;
  *count = param_total();
  return SIM_OK;
}

int sim_net_set_weights(sim_ctx* c, const float* w, int64_t count) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!c->net) {
    c->err = "context was not created with the learned preconditioner";
    return SIM_ERR_STATE;
  }
  if (!w || count != param_total()) {
    c->err = "weights must be a device float32 blob of sim_net_param_count entries";
    return SIM_ERR_INVALID_ARG;
  }
  pack_all(c, w);
  if (hipGetLastError() != hipSuccess) {
    c->err = "weight packing launch failed";
    return SIM_ERR_HIP;
  }
  c->net->ready = true;
  return SIM_OK;
}

int sim_net_set_tile_skip(sim_ctx* c, int32_t on) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!c->net) {
    c->err = "context was not created with the learned preconditioner";
    return SIM_ERR_STATE;
  }
  if (on != 0 && on != 1) {
    c->err = "on must be 0 or 1";
    return SIM_ERR_INVALID_ARG;
  }
  c->net->skip_tiles = on != 0;
  return SIM_OK;
}

int sim_net_forward(sim_ctx* c, const float* r, float* z) {
  if (!c) return SIM_ERR_INVALID_ARG;
  if (!net_ready(c)) {
    c->err = "learned preconditioner has no weights";
    return SIM_ERR_STATE;
  }
  if (!r || !z) {
    c->err = "NULL pointer";
    return SIM_ERR_INVALID_ARG;
  }
  int rc = net_apply(c, r, z, nullptr);
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_ERR_HIP;
}

// Loss and gradient (added into s->dW after zeroing it) of a batch.
static int batch_grad(sim_ctx* c, const float* r, const float* e, int batch, double* loss_out) {
  UNetState* s = c->net;
  const int64_t P = param_total();
  if (hipMemsetAsync(s->dW, 0, sizeof(float) * P, c->stream) != hipSuccess) return SIM_ERR_HIP;
  double loss_sum = 0.0;
  for (int b = 0; b < batch; ++b) {
    const float* rb = r + (int64_t)b * c->C;
    const float* eb = e + (int64_t)b * c->C;
    int rc = forward(c, rb, s->zbuf, nullptr, true);
    if (rc) return rc;
    launch_poisson_apply(c, s->zbuf, s->Az);
    launch_dot_cells_slot(c, rb, s->zbuf, S_NET_RZ, nullptr);
    launch_dot_cells_slot(c, rb, eb, S_NET_RE, nullptr);
    launch_dot_cells_slot(c, s->zbuf, s->Az, S_NET_ZAZ, nullptr);
    net_loss_grad(c, rb, s->Az, c->scal + S_NET_RZ, c->scal + S_NET_RMS, s->G11);
    rc = backward(c);
    if (rc) return rc;
    double d[3];
    if (hipMemcpyAsync(d, c->scal + S_NET_RZ, sizeof d, hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      c->err = "device error in the training step";
      return SIM_ERR_HIP;
    }
    loss_sum += 1.0 - d[0] * d[0] / (d[1] * d[2]);
  }
  if (hipGetLastError() != hipSuccess) {
    c->err = "training launch failed";
    return SIM_ERR_HIP;
  }
  *loss_out = loss_sum / batch;
  return SIM_OK;
}

static int check_train_args(sim_ctx* c, const float* r, const float* e, int32_t batch,
                            const double* h_loss) {
  if (!c->net) {
    c->err = "context was not created with the learned preconditioner";
    return SIM_ERR_STATE;
  }
  if (!r || !e || !h_loss || batch < 1) {
    c->err = "invalid training arguments";
    return SIM_ERR_INVALID_ARG;
  }
  return SIM_OK;
}

int sim_net_grad(sim_ctx* c, const float* r, const float* e, int32_t batch, float* grad,
                 double* h_loss) {
  if (!c) return SIM_ERR_INVALID_ARG;
  int rc = check_train_args(c, r, e, batch, h_loss);
  if (rc) return rc;
  if (!grad) {
    c->err = "NULL gradient output";
    return SIM_ERR_INVALID_ARG;
  }
  if (!net_ready(c)) {
    c->err = "learned preconditioner has no weights";
    return SIM_ERR_STATE;
  }
  rc = batch_grad(c, r, e, batch, h_loss);
  if (rc) return rc;
  const int64_t P = param_total();
  launch_scale_copy(c, c->net->dW, grad, P, 1.f / (float)batch);
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_ERR_HIP;
}

int sim_net_train_step(sim_ctx* c, const float* r, const float* e, int32_t batch, float* master,
                       float* adam, int32_t step, float lr, double* h_loss) {
  if (!c) return SIM_ERR_INVALID_ARG;
  int rc = check_train_args(c, r, e, batch, h_loss);
  if (rc) return rc;
  if (!master || !adam || step < 1 || !(lr > 0.f)) {
    c->err = "invalid optimiser arguments";
    return SIM_ERR_INVALID_ARG;
  }
  UNetState* s = c->net;
  const int64_t P = param_total();
  pack_all(c, master);
  s->ready = true;
  rc = batch_grad(c, r, e, batch, h_loss);
  if (rc) return rc;
  net_adam(c, P, master, adam, adam + P, s->dW, 1.f / (float)batch, lr, step);
  pack_all(c, master);
  return hipGetLastError() == hipSuccess ? SIM_OK : SIM_ERR_HIP;
}

}  // extern "C"
