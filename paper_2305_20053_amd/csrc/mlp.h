// MR-DINO network layout shared by the HIP kernels and the host runtime.
#pragma once
#include <stdint.h>

#define MLP_MAX_DEPTH 8

// Device weight views of one network.  Layer L = 0 maps the encoded input
// (r_m KL coordinates; the control part of W_0 is folded into an effective
// bias per call) to width W, layers 1..depth-1 are W x W, layer `depth` maps W
// to the r_u reduced state coordinates (rows padded to W with zeros).
struct MlpDev {
  int r_m, d_z, r_u, width, depth, kin;  // kin: columns of the BF16 layer-0 operand (r_m zero padded)
  // FP32 master parameters, packed: W_0 (width x (r_m+d_z)), b_0, W_1, b_1, ...
  const float* master;
  int64_t off_w[MLP_MAX_DEPTH + 1];      // offsets of W_L and b_L in `master`
  int64_t off_b[MLP_MAX_DEPTH + 1];
  // BF16 MFMA operands (see mlp.hip for the k-permutation and the fragment
  // order), stored back to back in the order the kernel reads them:
  // wp[0..depth], wt[depth..1], w0z.
  const void* ws;                        // the whole weight stream (BF16)
  const void* ws8;                       // the same in FP8 (E4M3), 16 x 128 fragments of 2 KB
  const float* wsc_inv;                  // FP8: 1 / scale of each operand, stream order
  int64_t ws_frags;                      // its length in 1 KB fragments
  const void* wp[MLP_MAX_DEPTH + 1];     // forward: rows = outputs, cols = inputs
  const void* wt[MLP_MAX_DEPTH + 1];     // backward (L >= 1): rows = inputs, cols = outputs
  const void* w0z;                       // 32 x width: d_Z rows of W_0^T
  const float* bias[MLP_MAX_DEPTH + 1];  // FP32 biases, padded to width
  const float* b0eff;                    // b_0 + W_0[:, r_m:] z (per call)
  const float* c;                        // reduced-QoI shift, padded to width
  const float* bc;                       // output bias + c, zero padded to width
  double c0;
  // FP32 reference operands: natural W_L (out x in) and its transpose (in x out)
  const float* wn[MLP_MAX_DEPTH + 1];
  const float* wtn[MLP_MAX_DEPTH + 1];
};
