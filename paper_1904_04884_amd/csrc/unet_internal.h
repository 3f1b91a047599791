// Internal declarations of the warm-start U-Net kernels (unet.hip) used by the
// network driver (unet.cpp).  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rihvr {

// Gather modes of the convolution-like GEMM (see unet.hip).
enum GatherMode {
  GG_CONV3_FWD = 0,  // rows: voxels; tap t reads voxel r + offset(t) (zero outside)
  GG_CONV3_BWD = 1,  // rows: voxels; tap t reads voxel r - offset(t)
  GG_UP_FWD = 2,     // rows: coarse voxels; one tap; column d*Cout + co writes fine voxel 2q + d
  GG_UP_BWD = 3,     // rows: coarse voxels; tap d reads fine voxel 2q + d
  GG_POINT = 4,      // rows: voxels; one tap, same voxel (1x1x1 convolution)
};

struct GatherGemmArgs {
  int mode;
  int D, H, W;             // grid of the rows (coarse grid for the up modes)
  const uint16_t* src;     // BF16 channels-last source
  int src_cs, src_c0;      // channel stride / offset of the source view
  int T, C;                // taps, channels per tap (multiple of 8)
  const uint16_t* wt;      // packed BF16 B[t][Npad][C]
  int N, Npad;             // real and padded (multiple of 16) output columns
  int up_cout;             // GG_UP_FWD: output channels (N = 8 * up_cout)
  const float* bias;       // nullable, indexed by output channel
  int relu, out_f32, accumulate;
  void* dst;               // BF16 or FP32 channels-last destination
  int dst_cs, dst_c0;
};
hipError_t launch_gather_gemm(const GatherGemmArgs& a, hipStream_t s);

struct WgradArgs {
  int mode;                // GG_CONV3_FWD, GG_UP_FWD (coarse rows) or GG_POINT
  int D, H, W;             // row grid
  const uint16_t* g;       // gradient w.r.t. the layer output (masked), channel view
  int g_cs, g_c0, N, Npad;
  const uint16_t* s;       // layer input, channel view
  int s_cs, s_c0, C, Cpad;
  float* dw;               // FP32 [t][C][N], accumulated
  long rows_per_block;     // set by launch_wgrad
  int taps;                // set by launch_wgrad
  float* part;             // per-row-chunk partials [chunk][t][C][N] (set by launch_wgrad)
};
// Weight and bias gradients are reduced without floating-point atomics: each
// block writes the partial sum of its chunk of rows (at most kReduceBlocks
// chunks) to `part`, and one ordered pass adds the chunks, so a training step
// gives the same bits on every run.
constexpr long kReduceBlocks = 256;
long wgrad_rows_per_block(long nrows);
long bias_rows_per_block(long nrows);
hipError_t launch_wgrad(WgradArgs a, int taps, float* part, hipStream_t s);
hipError_t launch_bias_grad(const uint16_t* g, int cs, int c0, int N, long nrows, float* db, float* part,
                            hipStream_t s);

hipError_t launch_pool_fwd(const uint16_t* x, int xcs, int xc0, uint16_t* y, int ycs, uint8_t* idx, int C, int D,
                           int H, int W, hipStream_t s);
hipError_t launch_pool_bwd(const uint16_t* gy, int gycs, const uint8_t* idx, uint16_t* gx, int gxcs, int gxc0, int C,
                           int D, int H, int W, hipStream_t s);
hipError_t launch_relu_mask(uint16_t* g, int gcs, int gc0, const uint16_t* y, int ycs, int yc0, int C, long nvox,
                            hipStream_t s);
hipError_t launch_zero_u16(uint16_t* p, size_t n, hipStream_t s);
hipError_t launch_input(const float* in, float scale, uint16_t* x, int cs, long nvox, hipStream_t s);
hipError_t launch_mse(const float* y, const float* t, long n, float pos_w, uint16_t* g, int gcs, float* loss,
                      float* part, hipStream_t s);   // part: one float per block (<= 16384)
hipError_t launch_adam(float* w, const float* g, float* m, float* v, size_t n, float lr, double b1, double b2,
                       double eps, int step, hipStream_t s);
hipError_t launch_pack(const float* w, int T, int cin, int cout, int transpose, int Npad, int Cpad, uint16_t* out,
                       hipStream_t s);
hipError_t launch_pack_up_fwd(const float* u, int cin, int cout, uint16_t* out, hipStream_t s);

}  // namespace rihvr
