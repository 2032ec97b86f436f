// Learned preconditioner (3-level 3-D U-Net) used inside flexible CG, and the
// launchers of its kernels (k_unet.hip).
#pragma once

#include <stddef.h>

#include "ctx.h"

namespace fs {

// Input of a convolution: channels [0, ca) from a (nearest-upsampled from the
// half-resolution level when up != 0), channels [ca, ca+cb) from b.
struct NetSrc {
  const __bf16* a;
  const __bf16* b;
  int ca, cb, up;
  // activity map of the input (nullable: the output's, NetOut::act): input
  // planes of a tile marked 0 are read as zero
  const uint8_t* act;
};

enum NetEpi {
  NET_EPI_RELU = 0,
  NET_EPI_RAW = 1,
  NET_EPI_MASKGRAD = 2,
  NET_EPI_OUT = 3,
  NET_EPI_RELU_ADD = 4,  // ReLU(conv + out.add): the skip part of a concatenating layer
  NET_EPI_RELU_POOL = 5  // ReLU, and the 2x2x2 average of the output into out.pool
};

struct NetOut {
  __bf16* bf;               // bf16 output [voxel][c_out] (RELU, RAW, MASKGRAD)
  float* f32;               // OUT: z = mask * rms * o
  const uint8_t* mask;      // OUT: liquid where non-zero
  const double* rms;        // OUT: device scalar
  const __bf16* relu_of;    // MASKGRAD: post-activation whose ReLU the gradient passes
  const _Float16* add;      // RELU_ADD: fp16 partial sums [voxel][c_out] added before ReLU
  __bf16* pool;             // RELU_POOL: pooled output at half resolution [voxel][c_out]
  // Tile-plane activity map of the output (nullable: every tile is live),
  // index (z * tiles_per_row + ty) * tiles_per_row + tx over the 16 x 16
  // xy-tiles.  Where it holds 0, no voxel of that tile and plane (with its
  // one-voxel halo) is needed: its values are zero, or nothing downstream
  // that reaches the network's output reads them.  The z-marching kernels
  // neither compute nor store such a tile; the output layer stores zeros.
  const uint8_t* act;
};

size_t net_workspace_bytes(int n);
// h_cell: host copy of the cell types (the activity maps derive from it)
int net_init(sim_ctx* c, const uint8_t* h_cell);
void net_destroy(sim_ctx* c);
bool net_ready(const sim_ctx* c);
// z = mask * rms(r) * U(r / rms(r), mask); returns at once when flags (nullable)
// has the done flag raised.  have_sumsq: the caller has already placed |r|^2
// in the context's S_NET_SUMSQ slot (the flexible-CG update reduces it), so
// the pass does not read r once more for it.  qdot (nullable): the output
// layer also reduces z . qdot into net_conv_out_blocks(n) block partials.
int net_apply(sim_ctx* c, const float* r, float* z, const int* flags, bool have_sumsq = false,
              const float* qdot = nullptr);

// kernel launchers
int conv_tiles(int n);
// z-marching kernels for the configurations (c_in, c_out) = (8|16|48, 16),
// (16, 32), (32, 32) and (16, 48); false for any other
// configuration
bool net_conv_zm(sim_ctx* c, int n, int cin, int cout, int epi, NetSrc src, const __bf16* w,
                 NetOut out, const int* flags);
bool net_conv(sim_ctx* c, int n, int cin, int cout, int epi, NetSrc src, const __bf16* w,
              NetOut out, const int* flags);
void net_wgrad(sim_ctx* c, int n, NetSrc src, int cin_real, int cin_pad, const __bf16* G,
               int g_stride, int cout_real, float* dW);
void net_pool(sim_ctx* c, int n, int C, const __bf16* in, __bf16* out, const int* flags);
// Upsampled half of a concatenating layer, evaluated on the coarse grid: for
// the fine level n, out[v][co] (fp16) = sum over taps and coarse channels of
// the 3x3x3 convolution of up(coarse) (nearest x2), through the per-parity
// 2x2x2 weights weff [8 parities][8 taps][cout][cc] (k_pack_subpixel).
// act (nullable): activity map of the coarse level; the fine outputs of a
// coarse tile-plane marked 0 are not computed (they stay zero).
bool net_upconv(sim_ctx* c, int n, int cc, int cout, const __bf16* coarse, const __bf16* weff,
                _Float16* out, const int* flags, const uint8_t* act);
// The same for 64 coarse channels and 32 outputs with one parity class per
// wave (k_upconv_cls).  act (nullable): activity map of the fine output
// level; the tile-planes marked 0 are not computed (the layer that adds the
// sums does not read them).  False for another channel configuration or
// when n is not a multiple of 16.
bool net_upconv_cls(sim_ctx* c, int n, int cc, int cout, const __bf16* coarse, const __bf16* weff,
                    _Float16* out, const int* flags, const uint8_t* act);
// The fine decoder layer with 32 coarse and 16 skip channels and 16 outputs
// in one pass: out = ReLU(conv(cat(up(coarse), skip))) (bf16), the upsampled
// half through weff as net_upconv, the skip half through wskip ([16][28][16]).
// act (nullable): activity map of the fine output (also read for the skip
// input).  False when n is not a multiple of the 16-voxel tile.
bool net_conv_cat(sim_ctx* c, int n, const __bf16* coarse, const __bf16* skip, const __bf16* weff,
                  const __bf16* wskip, __bf16* out, const int* flags, const uint8_t* act);
// Packs weff from the fp32 master weights W [cout][cin][27] of a layer whose
// first cc input channels are the upsampled ones; and the skip channels
// [cc, cin) into the forward layout [cout_p][28][cin - cc].
void net_pack_split(sim_ctx* c, const float* W, int cin, int cout, int cc, int cout_p,
                    __bf16* weff, __bf16* wskip);
void net_input(sim_ctx* c, const float* r, const double* sumsq, double* rms_out, __bf16* x0,
               const int* flags);
// c11 (16 -> 1) fused with the output map: z = mask * rms * conv(D), on the
// vector ALU (bf16 dot products); w is the layer's packed forward weights.
// act_in, act (nullable, both or neither): activity maps of D and of z.
// qdot (nullable): also reduce z . qdot into net_conv_out_blocks(n) FP64
// block partials (the context's partials buffer).
void net_conv_out(sim_ctx* c, int n, const __bf16* D, const __bf16* w, float* z, const double* rms,
                  const int* flags, const uint8_t* act_in, const uint8_t* act,
                  const float* qdot = nullptr);
int net_conv_out_blocks(int n);
// c1 fused with the input: ReLU(conv(r / rms, mask)) -> out (16 channels),
// rms written to rms_out; the 2-channel input is never stored.  r is read on
// liquid cells only.  act (nullable): activity map of the level.  work
// (nullable): counter of applications that did work.
void net_conv_in(sim_ctx* c, const float* r, const double* sumsq, double* rms_out,
                 const __bf16* w, __bf16* out, const int* flags, const uint8_t* act,
                 int* work);
void net_loss_grad(sim_ctx* c, const float* r, const float* Az, const double* dots,
                   const double* rms, __bf16* g11);
void net_upsum_mask(sim_ctx* c, int n_fine, int Cc, int Ct, const __bf16* T, const __bf16* P,
                    __bf16* out);
void net_skip_grad(sim_ctx* c, int n, int C, const __bf16* T, int Ct, int off, const __bf16* gp,
                   const __bf16* E, __bf16* out);
void net_pack_weights(sim_ctx* c, const float* W, int cin, int cout, int cin_p, int cout_p,
                      int cout_pd, __bf16* wf, __bf16* wd);
void net_adam(sim_ctx* c, int64_t count, float* W, float* m, float* v, const float* dW,
              float inv_batch, float lr, int step);
void launch_scale_copy(sim_ctx* c, const float* a, float* out, int64_t count, float s);

// cell-domain helpers from k_pcg.hip used by the network
// scal[slot] = a.b over cells (skipped when flags, nullable, has done raised)
void launch_dot_cells_slot(sim_ctx* c, const float* a, const float* b, int slot,
                           const int* flags);

}  // namespace fs
