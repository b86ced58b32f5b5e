// Spin surrogate network: shared constants, kernel arguments and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace st {

constexpr int kMlpWidth = 256;
constexpr int kMlpMaxIn = 8;
constexpr float kAdamBeta1 = 0.9f, kAdamBeta2 = 0.999f, kAdamEps = 1e-8f;

// Offsets of the tensors in the flat parameter (and gradient) vector:
// W1 [256][n_in], b1 [256], W2 [256][256], b2, W3 [256][256], b3, W4 [4][256], b4 [4].
struct MlpOffsets {
  int64_t W1, b1, W2, b2, W3, b3, W4, b4, total;
};

inline MlpOffsets mlp_offsets(int n_in) {
  MlpOffsets o;
  const int64_t w = kMlpWidth;
  o.W1 = 0;
  o.b1 = o.W1 + w * n_in;
  o.W2 = o.b1 + w;
  o.b2 = o.W2 + w * w;
  o.W3 = o.b2 + w;
  o.b3 = o.W3 + w * w;
  o.W4 = o.b3 + w;
  o.b4 = o.W4 + 4 * w;
  o.total = o.b4 + 4;
  return o;
}

struct MlpArgs {
  int64_t batch;          // samples
  int64_t ld;             // padded batch: leading dimension of the feature-major arrays
  int n_in;
  MlpOffsets off;
  int64_t n_params;
  const float* params;    // fp32 master weights (flat)
  float* params_rw;
  const __bf16* W2b;      // bf16 [256][256] copies of W2, W3 and their transposes
  const __bf16* W3b;
  const __bf16* W2Tb;
  const __bf16* W3Tb;
  __bf16* W2b_rw;
  __bf16* W3b_rw;
  __bf16* W2Tb_rw;
  __bf16* W3Tb_rw;
  const __bf16* W4s;      // bf16 [16][256]: W4 split into three bf16 parts (rows j, 4 + j,
  __bf16* W4s_rw;         //   8 + j; rows 12-15 zero), W4 = hi + mid + lo to fp32 precision
  const float* x;         // [batch][n_in]
  const float* target;    // [batch][4]
  float* q_out;           // [batch][4]
  float out_ref[4];       // output frame: u = out_ref + out_lin x + out_scale ⊙ y, q = u/|u|
  float out_scale[4];
  float out_lin[4][kMlpMaxIn];
  float inv_loss_norm;    // 1/batch
  float* loss_part;       // [blocks]
  __bf16* hT1;            // [256][ld] activations, feature-major
  __bf16* hT2;
  __bf16* dsT2;           // [256][ld] silu'(z2) (bf16), from the forward half to the backward
  __bf16* dzT2;           // [256][ld] gradients at the pre-activations
  __bf16* dzT3;
  float* gpart_W1;        // per-block partial gradients
  float* gpart_b1;
  float* gpart_b2;
  float* gpart_b3;
  float* gpart_W4;
  float* gpart_b4;
  float* gpart_W2;        // [splits][256][256]
  float* gpart_W3;
  int n_splits;
  int64_t split_chunk;    // samples per split (multiple of 32)
  float* grad;            // flat gradient, same layout as params
  float* adam_m;
  float* adam_v;
};

// Network inputs from coordinates: (z_i - center_i) * inv_scale_i, then extra.
struct FeatureMap {
  double center[6], inv_scale[6], extra;
};

int mlp_tile();
hipError_t launch_features(const double* z, int64_t n, const FeatureMap& f, int n_in, float* x,
                           hipStream_t s);
hipError_t launch_targets(const double* q, int64_t n, const double* ref, float* t, hipStream_t s);
// train: the fused forward and backward pass of one batch (activations, dz2,
// dz3 and the per-tile partials); otherwise inference into q_out.
hipError_t launch_mlp_forward(const MlpArgs& a, bool train, hipStream_t s);
// dW2, dW3 split-K partials from the feature-major activations and gradients.
hipError_t launch_mlp_weight_grad(const MlpArgs& a, hipStream_t s);
// Several independent column sums of row-major partials part[parts][len] into
// out[len], reduced 64 rows per pass until one row is left; the segments
// share one launch per pass.  tmp: the sum over segments of
// sum_partials_tmp(len, parts) floats (a double buffer per segment).
struct SumSegment {
  const float* part;
  int64_t len;
  int parts;
  float* out;
};
constexpr int kMaxSumSegments = 12;
size_t sum_partials_tmp(int64_t len, int parts);
// What a reduction stopped after `max_passes` passes still has to add: rows
// partial rows of len values at src (rows == 0: the segment is complete in
// its out).
struct SumLeft {
  const float* src;
  int64_t len;
  int rows;
};
hipError_t launch_sum_partials_multi(const SumSegment* segs, int nseg, float* tmp, hipStream_t s,
                                     int max_passes = 1 << 30, SumLeft* left = nullptr);
// Adam over the flat parameters, taking the gradient of the parameters at
// [off, off + len) of a pending segment as the sum of its remaining rows (in
// row order; written to grad as well), and the loss likewise.
struct AdamPending {
  int n;
  struct {
    const float* src;
    int64_t off, len;
    int rows;
  } seg[kMaxSumSegments];
  const float* loss_src;
  int loss_rows;
  float* loss_out;
};
// Least-squares fit of targets t [n][4] on the inputs augmented with a
// constant, [1, x] (D = n_in + 1 columns), in double precision.  Pass 1:
// per-block partial sums of the normal equations, D*D entries of [1,x][1,x]ᵀ
// then D*4 of [1,x] tᵀ (row-major), kFitBlocks blocks.  Pass 2: per-block
// sums of squared residuals of each component and their largest magnitude,
// for coefficients coef[4][D].
constexpr int kFitBlocks = 512;
struct FitCoef {
  double c[4][kMlpMaxIn + 1];
};
hipError_t launch_fit_normal(const float* x, const float* t, int64_t n, int n_in, double* partials,
                             hipStream_t s);
hipError_t launch_fit_residual(const float* x, const float* t, int64_t n, int n_in,
                               const FitCoef& coef, double* partials, hipStream_t s);
hipError_t launch_adam(const MlpArgs& a, float lr, float c1, float c2, hipStream_t s,
                       const AdamPending* pending = nullptr);
hipError_t launch_refresh_bf16(const MlpArgs& a, hipStream_t s);

}  // namespace st
