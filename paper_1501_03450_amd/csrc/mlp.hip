// Spin surrogate network: MLP n_in -> 256 -> 256 -> 256 -> 4 with SiLU
// activations and a normalised output q = y/|y|, trained on the mean squared
// error against one-turn quaternions with Adam.
//
// The two 256×256 layers run on the matrix cores: bf16 operands, fp32
// accumulation, v_mfma_f32_16x16x32_bf16 (A[i][k] in lane i + 16(k/8),
// element k%8; B[k][j] in lane j + 16(k/8); D[i][j] in lane j + 16(i/4),
// element i%4).  The n_in -> 256 layer (and its recomputation and weight
// gradient in the backward pass) runs on the fp32 matrix cores,
// v_mfma_f32_16x16x4_f32 (A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
// D as above), so its operands stay fp32.  The 256 -> 4 layer and its weight
// gradient use the bf16 matrix cores with the fp32 operand (W4, dL/dy) split
// into three bf16 parts whose sum is exact, so those products keep fp32
// precision too.
//
// Kernels (one batch, 64 samples per workgroup of four waves):
//   forward        inference: all four layers fused, activations kept in LDS
//   forward<TRAIN> the training step's forward and backward passes of one
//                  tile in one kernel: it stores the two hidden activations
//                  the weight gradients need and silu'(z2) (bf16,
//                  feature-major, straight from the accumulators), keeps
//                  silu'(z3) and dL/dy in LDS, fuses the loss,
//                  then runs dL/dy -> dz3 -> dz2 -> dz1 through the transposed
//                  bf16 weights with z1 recomputed by the same matrix-core
//                  products, stores dz3 and dz2 feature-major, and forms the
//                  per-workgroup partial sums of the b1..b4, W1 and W4
//                  gradients
//   weight_grad    dW2, dW3 = dzᵀ hᵀ as split-K MFMA GEMMs over the batch
//   reduce         fixed-order sum of the partials (deterministic)
//   adam           fp32 master weights, then the bf16 copies W and Wᵀ
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include "mlp_kernels.h"

namespace st {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int W = kMlpWidth;       // 256
constexpr int TM = 64;             // samples per workgroup
constexpr int LDA = W + 8;         // padded LDS row (bf16 elements)
constexpr int NT = 256;            // threads per workgroup

// σ(z) = 1/(1 + e^-z) with the hardware exponential and reciprocal
// (about 1 ulp each): the activations are rounded to bf16 right after.
__device__ __forceinline__ float sigmoid(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = sigmoid(z);
  return s * (1.0f + z * (1.0f - s));
}

// acc[mt][nt] += A[16 MT x 256] (LDS, row stride LDA) · B'[n_base + 16 nt + j][k]
// (global, row-major [256][256]) for the wave's 64 output columns.  Each
// 16x16 output tile accumulates over k in the same order whatever MT and
// UNROLL are, so a tile computed in a smaller call has the same bits.  With
// the loop unrolled (UNROLL = 8) the compiler issues the B loads of later k
// steps ahead of the MFMAs; the L2 latency that remains is covered by the
// other waves on the SIMD.  Callers short of registers unroll by 2.
template <int MT, int UNROLL = 8>
__device__ __forceinline__ void gemm_tiles(const __bf16* A, const __bf16* Bg, int n_base,
                                           f32x4 acc[MT][4], int lane) {
  const int r = lane & 15, kb = 8 * (lane >> 4);
  const __bf16* brow = Bg + (size_t)(n_base + r) * W + kb;
#pragma unroll UNROLL
  for (int k0 = 0; k0 < W; k0 += 32) {
    bf16x8 a[MT], b[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) b[nt] = *reinterpret_cast<const bf16x8*>(brow + nt * 16 * W + k0);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      a[mt] = *reinterpret_cast<const bf16x8*>(A + (mt * 16 + r) * LDA + k0 + kb);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
  }
}

template <int UNROLL = 8>
__device__ __forceinline__ void gemm_64x64(const __bf16* A, const __bf16* Bg, int n_base,
                                           f32x4 acc[4][4], int lane) {
  gemm_tiles<4, UNROLL>(A, Bg, n_base, acc, lane);
}

__device__ __forceinline__ void zero_acc(f32x4 acc[4][4]) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// Layer 1 for the 16 features n0 .. n0 + 15 on the fp32 matrix cores:
// acc[mt] = x[16 mt + i][k] W1[n0 + j][k] summed over the eight zero-padded
// inputs, two steps of four.  The backward pass recomputes z1 with the same
// call, so both passes see the same bits.
__device__ __forceinline__ void layer1_cols(const float (*xs)[kMlpMaxIn], const float* W1, int nin,
                                            int n0, f32x4 acc[4], int lane) {
  const int r = lane & 15, kq = lane >> 4;
  const float w0 = kq < nin ? W1[(n0 + r) * nin + kq] : 0.0f;
  const float w1 = 4 + kq < nin ? W1[(n0 + r) * nin + 4 + kq] : 0.0f;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 d = {0.f, 0.f, 0.f, 0.f};
    d = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[mt * 16 + r][kq], w0, d, 0, 0, 0);
    acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[mt * 16 + r][4 + kq], w1, d, 0, 0, 0);
  }
}

// Part `part` (0, 1 or 2) of v split into three bf16 values that sum to v
// exactly: hi = bf16(v), mid = bf16(v - hi), lo = v - hi - mid (each
// difference is exact in fp32, and the last fits in bf16).
__device__ __forceinline__ __bf16 split3(float v, int part) {
  const __bf16 hi = (__bf16)v;
  if (part == 0) return hi;
  const float r = v - (float)hi;
  const __bf16 mid = (__bf16)r;
  if (part == 1) return mid;
  return (__bf16)(r - (float)mid);
}

// Hidden-layer epilogue: z = acc + b, h = silu(z) into LDS (bf16, row-major),
// and when hT is set also to HBM feature-major [256][ld] from the registers
// (a lane holds four consecutive samples of one feature: one 8-byte store per
// 16x16 tile).
__device__ __forceinline__ void hidden_epilogue(const f32x4 acc[4][4], const float* bias,
                                                __bf16* out_lds, int rows, int n_base, int lane,
                                                __bf16* hT, int64_t ld, int64_t b0) {
  const int c = lane & 15, rq = 4 * (lane >> 4);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int n = n_base + nt * 16 + c;
    const float bn = bias[n];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const int m0 = mt * 16 + rq;
      bf16x4 h;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float z = acc[mt][nt][i] + bn;
        // padded samples (beyond the batch) carry zero activations
        h[i] = (__bf16)(m0 + i < rows ? silu(z) : 0.0f);
        out_lds[(m0 + i) * LDA + n] = h[i];
      }
      if (hT) *reinterpret_cast<bf16x4*>(hT + (size_t)n * ld + b0 + m0) = h;
    }
  }
}

// silu'(z3) of a wave's 64x64 tile kept in LDS between the forward and
// backward halves of the training kernel, in the accumulator layout: lane
// `lane` of the wave stores the four bf16 values of (nt, mt) (samples
// 16 mt + rq .. + 3 of feature 16 nt + c) as one 8-byte word at
// [(4 nt + mt) * 64 + lane] of the wave's 8 KB, and reads back only its own.

__device__ __forceinline__ uint32_t pack_bf16x2(__bf16 lo, __bf16 hi) {
  return (uint32_t)__builtin_bit_cast(unsigned short, lo) |
         ((uint32_t)__builtin_bit_cast(unsigned short, hi) << 16);
}
// element i (0..3) of a packed quadruple, as float
__device__ __forceinline__ float ds_at(uint2 q, int i) {
  const uint32_t w = (i >> 1) ? q.y : q.x;
  return __builtin_bit_cast(float, (i & 1) ? (w & 0xffff0000u) : (w << 16));
}

// Training epilogue of layers 2 and 3: as hidden_epilogue, and silu'(z)
// rounded to bf16 (zero for padded samples) either to HBM feature-major
// [256][ld] from the registers (dsT set) or to the wave's LDS words (ds).
__device__ __forceinline__ void hidden_epilogue_dsilu(const f32x4 acc[4][4], const float* bias,
                                                      __bf16* out_lds, int rows, int n_base,
                                                      int lane, __bf16* dsT, uint2* ds,
                                                      __bf16* hT, int64_t ld, int64_t b0) {
  const int c = lane & 15, rq = 4 * (lane >> 4);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int n = n_base + nt * 16 + c;
    const float bn = bias[n];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const int m0 = mt * 16 + rq;
      bf16x4 d, h;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float z = acc[mt][nt][i] + bn;
        const float sg = sigmoid(z);
        const bool in = m0 + i < rows;
        h[i] = (__bf16)(in ? z * sg : 0.0f);
        out_lds[(m0 + i) * LDA + n] = h[i];
        d[i] = (__bf16)(in ? sg * (1.0f + z * (1.0f - sg)) : 0.0f);
      }
      if (dsT) {
        *reinterpret_cast<bf16x4*>(dsT + (size_t)n * ld + b0 + m0) = d;
      } else {
        ds[(nt * 4 + mt) * 64 + lane] = make_uint2(pack_bf16x2(d[0], d[1]), pack_bf16x2(d[2], d[3]));
      }
      if (hT) *reinterpret_cast<bf16x4*>(hT + (size_t)n * ld + b0 + m0) = h;
    }
  }
}

// A wave's 64 x 64 block of gradients into LDS (bf16, row-major); samples
// beyond the batch get zeros.  With dzT set, the same bf16 values also go to
// HBM feature-major from the registers, and gb[n] receives their sum over
// the tile's samples (the bias gradient partial).
__device__ __forceinline__ void store_grad_tile(const f32x4 acc[4][4], __bf16* out_lds, int rows,
                                                int n_base, int lane, __bf16* dzT = nullptr,
                                                int64_t ld = 0, int64_t b0 = 0,
                                                float* gb = nullptr) {
  const int c = lane & 15, rq = 4 * (lane >> 4);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int n = n_base + nt * 16 + c;
    float sum = 0.0f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const int m0 = mt * 16 + rq;
      bf16x4 v;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[i] = (__bf16)(m0 + i < rows ? acc[mt][nt][i] : 0.0f);
        out_lds[(m0 + i) * LDA + n] = v[i];
        sum += (float)v[i];
      }
      if (dzT) *reinterpret_cast<bf16x4*>(dzT + (size_t)n * ld + b0 + m0) = v;
    }
    if (gb) {
      // the four lane groups hold samples rq = 0, 4, 8, 12 of every 16
      sum += __shfl_xor(sum, 16, 64);
      sum += __shfl_xor(sum, 32, 64);
      if (lane < 16) gb[n] = sum;
    }
  }
}

// One activation buffer per workgroup (34 KB of LDS, so four workgroups fit
// on a CU): each layer's GEMM reads it, a barrier, then the epilogue
// overwrites it with the layer's output.  Inference is compiled for four
// waves per SIMD (128 registers), so that four workgroups are resident per
// CU and the whole batch of 1024 tiles of a 65536-sample batch is on the
// chip at once.
//
// TRAIN: the same tile then runs the backward pass through the layers, with
// silu'(z3) kept in LDS from the forward epilogue (bf16, in the accumulator
// layout the backward products use), silu'(z2) read back from HBM and dL/dy
// in LDS: dz3 = (dL/dy W4) ⊙ silu'(z3), dz2 = (dz3 W3) ⊙ silu'(z2) and
// dz1 = (dz2 W2) ⊙ silu'(z1) with z1 recomputed by the same matrix-core
// products as in the forward half.  h1, h2, dz2 and dz3 go to HBM
// feature-major for the weight-gradient kernel; the bias, W1 and W4 gradient
// partials of the tile are formed here.  Two waves per SIMD, 180 registers
// without spills and 68 KB of LDS (two workgroups per CU); with silu'(z3)
// in registers instead the kernel spilled 32 bytes per lane, and with
// silu'(z2) there as well 368.
#ifndef ST_MLP_TRAIN_WAVES
#define ST_MLP_TRAIN_WAVES 2
#endif
template <bool TRAIN>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(TRAIN ? ST_MLP_TRAIN_WAVES : 4, TRAIN ? ST_MLP_TRAIN_WAVES : 4)))
mlp_forward_kernel(const MlpArgs a) {
  __shared__ __align__(16) __bf16 bufA[TM * LDA];
  __shared__ float xs[TM][kMlpMaxIn];
  __shared__ float ys[TM][4];
  __shared__ float red[NT / 64];
  // training: silu'(z3) of the four waves' tiles (32 KB; inference: unused)
  __shared__ uint2 ds3s[TRAIN ? (NT / 64) * 16 * 64 : 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint2* const ds3 = ds3s + (TRAIN ? wv * 16 * 64 : 0);
  const int64_t B = a.batch, b0 = (int64_t)blockIdx.x * TM;
  const int rows = (int)min((int64_t)TM, B - b0);
  const int nin = a.n_in;
  const float* P = a.params;

  for (int i = tid; i < TM * kMlpMaxIn; i += NT) {
    const int m = i / kMlpMaxIn, k = i % kMlpMaxIn;
    xs[m][k] = (m < rows && k < nin) ? a.x[(b0 + m) * nin + k] : 0.0f;
  }
  __syncthreads();

  // layer 1 (fp32 matrix cores): the wave's 64 features
  f32x4 acc[4][4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    f32x4 col[4];
    layer1_cols(xs, P + a.off.W1, nin, wv * 64 + nt * 16, col, lane);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) acc[mt][nt] = col[mt];
  }
  hidden_epilogue(acc, P + a.off.b1, bufA, rows, wv * 64, lane, TRAIN ? a.hT1 : nullptr, a.ld, b0);
  __syncthreads();

  // layer 2 (MFMA)
  zero_acc(acc);
  gemm_64x64<2>(bufA, a.W2b, wv * 64, acc, lane);
  __syncthreads();
  if (TRAIN)
    hidden_epilogue_dsilu(acc, P + a.off.b2, bufA, rows, wv * 64, lane, a.dsT2, ds3, a.hT2, a.ld,
                          b0);
  else
    hidden_epilogue(acc, P + a.off.b2, bufA, rows, wv * 64, lane, nullptr, 0, 0);
  __syncthreads();
  // layer 3 (MFMA)
  zero_acc(acc);
  gemm_64x64<2>(bufA, a.W3b, wv * 64, acc, lane);
  __syncthreads();
  if (TRAIN)
    hidden_epilogue_dsilu(acc, P + a.off.b3, bufA, rows, wv * 64, lane, nullptr, ds3, nullptr, a.ld,
                          b0);
  else
    hidden_epilogue(acc, P + a.off.b3, bufA, rows, wv * 64, lane, nullptr, 0, 0);
  __syncthreads();

  // layer 4 (bf16 matrix cores, W4 in three parts: operand rows j, 4 + j and
  // 8 + j): wave wv takes samples 16 wv .. 16 wv + 15, and the three partial
  // outputs of (sample, j) sit in lanes c = j, j + 4, j + 8 of a lane group
  {
    const int r = lane & 15, kb = 8 * (lane >> 4), rq = 4 * (lane >> 4);
    f32x4 y4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < W; k0 += 32) {
      const bf16x8 av = *reinterpret_cast<const bf16x8*>(bufA + (wv * 16 + r) * LDA + k0 + kb);
      const bf16x8 bv = *reinterpret_cast<const bf16x8*>(a.W4s + r * W + k0 + kb);
      y4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, y4, 0, 0, 0);
    }
    const float bj = P[a.off.b4 + (r & 3)];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float mid = __shfl(y4[i], lane + 4, 64), lo = __shfl(y4[i], lane + 8, 64);
      if (r < 4) ys[wv * 16 + rq + i][r] = bj + ((y4[i] + mid) + lo);
    }
  }
  __syncthreads();

  // normalised output; when training, the loss and dL/dy (into ys, zero for
  // padded samples)
  float l = 0.0f;
  if (tid < TM) {
    const int m = tid;
    // frame base ref + lin x (zero columns past n_in: xs is zero-padded)
    float base[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float b = a.out_ref[j];
#pragma unroll
      for (int k = 0; k < kMlpMaxIn; ++k) b = fmaf(a.out_lin[j][k], xs[m][k], b);
      base[j] = b;
    }
    const float y0 = fmaf(a.out_scale[0], ys[m][0], base[0]);
    const float y1 = fmaf(a.out_scale[1], ys[m][1], base[1]);
    const float y2 = fmaf(a.out_scale[2], ys[m][2], base[2]);
    const float y3 = fmaf(a.out_scale[3], ys[m][3], base[3]);
    const float ny = sqrtf(y0 * y0 + y1 * y1 + y2 * y2 + y3 * y3);
    const float inv = 1.0f / ny;
    const float q[4] = {y0 * inv, y1 * inv, y2 * inv, y3 * inv};
    if (!TRAIN) {
      if (m < rows)
        for (int j = 0; j < 4; ++j) a.q_out[(b0 + m) * 4 + j] = q[j];
    } else if (m < rows) {
      const float* t = a.target + (b0 + m) * 4;
      float dq[4], qd = 0.0f;
      for (int j = 0; j < 4; ++j) {
        const float d = q[j] - t[j];
        l += d * d;
        dq[j] = 2.0f * d * a.inv_loss_norm;
        qd += q[j] * dq[j];
      }
      for (int j = 0; j < 4; ++j) ys[m][j] = a.out_scale[j] * ((dq[j] - q[j] * qd) * inv);
    } else {
      for (int j = 0; j < 4; ++j) ys[m][j] = 0.0f;
    }
  }
  if (!TRAIN) return;
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
  if (lane == 0) red[wv] = l;
  __syncthreads();
  if (tid == 0) a.loss_part[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) * a.inv_loss_norm;
  const int blk = blockIdx.x;

  // dW4 and db4 partials of this tile.
  // gW4[j][k] = sum over m of dL/dy[m][j] h3[m][k] on the bf16 matrix cores
  // with dL/dy in three parts (operand rows j, 4 + j, 8 + j; rows 12-15
  // zero; padded samples have dL/dy = 0): wave wv takes features 64 wv ..
  // 64 wv + 63, and the parts of row j come out in lane groups 0, 1 and 2
  {
    const int r = lane & 15, kb = 8 * (lane >> 4);
    f32x4 g[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) g[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s0 = 0; s0 < TM; s0 += 32) {
      bf16x8 av;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        av[e] = r < 12 ? split3(ys[s0 + kb + e][r & 3], r >> 2) : (__bf16)0.0f;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int n = wv * 64 + t * 16 + r;
        bf16x8 bv;
#pragma unroll
        for (int e = 0; e < 8; ++e) bv[e] = bufA[(s0 + kb + e) * LDA + n];
        g[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, g[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float mid = __shfl(g[t][i], lane + 16, 64), lo = __shfl(g[t][i], lane + 32, 64);
        if (lane < 16)
          a.gpart_W4[((size_t)blk * 4 + i) * W + wv * 64 + t * 16 + r] = (g[t][i] + mid) + lo;
      }
    if (tid < 4) {
      float sb = 0.0f;
      for (int m = 0; m < rows; ++m) sb += ys[m][tid];
      a.gpart_b4[(size_t)blk * 4 + tid] = sb;
    }
  }
  __syncthreads();   // h3 in bufA read by every wave before dz3 replaces it

  // backward half
  const int n_base = wv * 64, c = lane & 15, rq = 4 * (lane >> 4);
  // dz3 = (dL/dy W4) ⊙ silu'(z3) in the accumulator layout (a lane: four
  // consecutive samples of one feature, silu'(z3) one 8-byte load), its bias
  // gradient partial before rounding, and dz3 in bf16 into LDS (zero past the
  // batch, where dL/dy is zero)
  {
    float gb[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int n = n_base + nt * 16 + c;
      const float w0 = P[a.off.W4 + 0 * W + n], w1 = P[a.off.W4 + 1 * W + n];
      const float w2 = P[a.off.W4 + 2 * W + n], w3 = P[a.off.W4 + 3 * W + n];
      float sum = 0.0f;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        bf16x4 v;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = mt * 16 + rq + i;
          const float dh = w0 * ys[m][0] + w1 * ys[m][1] + w2 * ys[m][2] + w3 * ys[m][3];
          const float dz = dh * ds_at(ds3[(nt * 4 + mt) * 64 + lane], i);
          sum += dz;
          v[i] = (__bf16)dz;
          bufA[m * LDA + n] = v[i];
        }
        *reinterpret_cast<bf16x4*>(a.dzT3 + (size_t)n * a.ld + b0 + mt * 16 + rq) = v;
      }
      gb[nt] = sum;
    }
    // sum the four lane groups (samples rq = 0, 4, 8, 12 of every 16)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      gb[nt] += __shfl_xor(gb[nt], 16, 64);
      gb[nt] += __shfl_xor(gb[nt], 32, 64);
    }
    if (lane < 16)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) a.gpart_b3[(size_t)blk * W + n_base + nt * 16 + c] = gb[nt];
  }
  __syncthreads();

  // dz2 = (dz3 W3) ⊙ silu'(z2): a lane's four consecutive samples of one
  // feature are one 8-byte load of the feature-major silu'(z2)
  zero_acc(acc);
  gemm_64x64<2>(bufA, a.W3Tb, n_base, acc, lane);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const __bf16* dsrow = a.dsT2 + (size_t)(n_base + nt * 16 + c) * a.ld + b0;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const bf16x4 d = *reinterpret_cast<const bf16x4*>(dsrow + mt * 16 + rq);
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[mt][nt][i] = acc[mt][nt][i] * (float)d[i];
    }
  }
  __syncthreads();   // bufA: dz3 -> dz2
  store_grad_tile(acc, bufA, rows, n_base, lane, a.dzT2, a.ld, b0, a.gpart_b2 + (size_t)blk * W);
  __syncthreads();
  // dz1 = (dz2 W2) ⊙ silu'(z1), z1 = W1 x + b1 by the forward pass's products
  zero_acc(acc);
  gemm_64x64<2>(bufA, a.W2Tb, n_base, acc, lane);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    f32x4 z1[4];
    layer1_cols(xs, P + a.off.W1, nin, n_base + nt * 16, z1, lane);
    const float bn = P[a.off.b1 + n_base + nt * 16 + c];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[mt][nt][i] = acc[mt][nt][i] * dsilu(z1[mt][i] + bn);
  }
  __syncthreads();   // bufA: dz2 -> dz1
  store_grad_tile(acc, bufA, rows, n_base, lane);
  __syncthreads();
  // W1 and b1 gradient partials on the fp32 matrix cores: D[n][k] = sum over
  // m of dz1[m][n] [x | 1][m][k], A = dz1ᵀ (the wave's 64 features, from
  // LDS), B = the inputs with a column of ones after them, steps of four
  // samples (padded samples have dz1 = 0)
  {
    const int r = lane & 15, kq = lane >> 4;
    f32x4 g[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) g[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int s0 = 0; s0 < TM; s0 += 4) {
      const int m = s0 + kq;
      const float bx = r < nin ? xs[m][r] : (r == nin ? 1.0f : 0.0f);
#pragma unroll
      for (int t = 0; t < 4; ++t)
        g[t] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)bufA[m * LDA + n_base + t * 16 + r], bx,
                                                    g[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int n = n_base + t * 16 + rq + i;
        if (c < nin) a.gpart_W1[((size_t)blk * W + n) * nin + c] = g[t][i];
        else if (c == nin) a.gpart_b1[(size_t)blk * W + n] = g[t][i];
      }
  }
}

// Weight gradients of the two 256×256 layers: gW[n][k] = Σ_b dzT[n][b] hT[k][b]
// over one split (a contiguous range of samples).  A workgroup computes a
// 128×128 tile of one split, each wave a 64×64 quarter of it; every 32-sample
// step stages the tile's 128 rows of both operands in LDS (double-buffered,
// rows padded to 40 elements so that the fragment reads hit distinct banks),
// and the next step's global loads are in flight during the current step's
// sixteen MFMAs.  The four tiles of a (layer, split) group read the same
// operands, so the launch keeps a group on one XCD (workgroups are dealt to
// the 8 XCDs in turn), where they share the XCD's L2.
constexpr int kWgTile = 128, kWgRow = 40;
__global__ void __launch_bounds__(NT) mlp_weight_grad_kernel(const MlpArgs a) {
  __shared__ __align__(16) __bf16 As[2][kWgTile * kWgRow];
  __shared__ __align__(16) __bf16 Bs[2][kWgTile * kWgRow];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int id = blockIdx.x, xcd = id % 8, slot = id / 8;
  const int group = xcd + 8 * (slot / 4), tile = slot % 4;
  const int which = group & 1, split = group >> 1;
  const __bf16* dzT = which == 0 ? a.dzT2 : a.dzT3;
  const __bf16* hT = which == 0 ? a.hT1 : a.hT2;
  float* out = (which == 0 ? a.gpart_W2 : a.gpart_W3) + (size_t)split * W * W;
  const int n0 = (tile >> 1) * kWgTile, k0 = (tile & 1) * kWgTile;
  const int wn = (wv >> 1) * 64, wk = (wv & 1) * 64;
  const int64_t ld = a.ld;
  const int64_t bs = (int64_t)split * a.split_chunk, be = min(ld, bs + a.split_chunk);
  const int nsteps = be > bs ? (int)((be - bs) / 32) : 0;
  // staging: thread t moves 16 bytes of rows t/4 and 64 + t/4, chunk t%4
  const int sr = tid >> 2, sc = (tid & 3) * 8;
  const __bf16* ga0 = dzT + (size_t)(n0 + sr) * ld + bs + sc;
  const __bf16* ga1 = dzT + (size_t)(n0 + 64 + sr) * ld + bs + sc;
  const __bf16* gb0 = hT + (size_t)(k0 + sr) * ld + bs + sc;
  const __bf16* gb1 = hT + (size_t)(k0 + 64 + sr) * ld + bs + sc;
  const int so0 = sr * kWgRow + sc, so1 = (64 + sr) * kWgRow + sc;
  const int r = lane & 15, kq = 8 * (lane >> 4);
  f32x4 acc[4][4];
  zero_acc(acc);
  bf16x8 xa0, xa1, xb0, xb1;
  if (nsteps > 0) {
    xa0 = *reinterpret_cast<const bf16x8*>(ga0);
    xa1 = *reinterpret_cast<const bf16x8*>(ga1);
    xb0 = *reinterpret_cast<const bf16x8*>(gb0);
    xb1 = *reinterpret_cast<const bf16x8*>(gb1);
    *reinterpret_cast<bf16x8*>(&As[0][so0]) = xa0;
    *reinterpret_cast<bf16x8*>(&As[0][so1]) = xa1;
    *reinterpret_cast<bf16x8*>(&Bs[0][so0]) = xb0;
    *reinterpret_cast<bf16x8*>(&Bs[0][so1]) = xb1;
  }
  __syncthreads();
  for (int st = 0; st < nsteps; ++st) {
    const int cur = st & 1;
    const bool more = st + 1 < nsteps;
    if (more) {
      const int64_t off = (int64_t)(st + 1) * 32;
      xa0 = *reinterpret_cast<const bf16x8*>(ga0 + off);
      xa1 = *reinterpret_cast<const bf16x8*>(ga1 + off);
      xb0 = *reinterpret_cast<const bf16x8*>(gb0 + off);
      xb1 = *reinterpret_cast<const bf16x8*>(gb1 + off);
    }
    bf16x8 av[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      av[i] = *reinterpret_cast<const bf16x8*>(&As[cur][(wn + i * 16 + r) * kWgRow + kq]);
      bv[i] = *reinterpret_cast<const bf16x8*>(&Bs[cur][(wk + i * 16 + r) * kWgRow + kq]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    if (more) {
      *reinterpret_cast<bf16x8*>(&As[cur ^ 1][so0]) = xa0;
      *reinterpret_cast<bf16x8*>(&As[cur ^ 1][so1]) = xa1;
      *reinterpret_cast<bf16x8*>(&Bs[cur ^ 1][so0]) = xb0;
      *reinterpret_cast<bf16x8*>(&Bs[cur ^ 1][so1]) = xb1;
    }
    __syncthreads();
  }
  const int c = lane & 15, rq = 4 * (lane >> 4);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        out[(size_t)(n0 + wn + i * 16 + rq + e) * W + k0 + wk + j * 16 + c] = acc[i][j][e];
}

// Column sums of row-major partials [rows][len], 64 rows per workgroup and
// pass: a workgroup covers C columns (C = 64, or fewer for short rows) with
// 256/C threads per column; every thread sums a strided subset of the rows
// and the subsets are combined in LDS in thread order, so the result does not
// depend on scheduling.  Several independent sums share a launch: the blocks
// of segment k are numbered from first[k].
struct SumPass {
  int nseg;
  struct {
    const float* src;
    float* dst;
    int64_t len, first;
    int rows, C, gx;
  } seg[kMaxSumSegments];
};

__global__ void __launch_bounds__(256) sum_partials_multi_kernel(const SumPass p) {
  __shared__ float acc[256];
  int k = 0;
  while (k + 1 < p.nseg && (int64_t)blockIdx.x >= p.seg[k + 1].first) ++k;
  const int64_t b = (int64_t)blockIdx.x - p.seg[k].first;
  const int C = p.seg[k].C, gx = p.seg[k].gx, rows = p.seg[k].rows;
  const int64_t len = p.seg[k].len;
  const int64_t bx = b % gx, by = b / gx;
  const int t = threadIdx.x, c = t % C, g = t / C, G = 256 / C;
  const int64_t i = bx * C + c;
  const int r0 = (int)by * 64, r1 = min(rows, r0 + 64);
  const float* part = p.seg[k].src;
  float s = 0.0f;
  if (i < len)
#pragma unroll 4
    for (int r = r0 + g; r < r1; r += G) s += part[(size_t)r * len + i];
  acc[t] = s;
  __syncthreads();
  if (g == 0 && i < len) {
    float v = 0.0f;
    for (int q = 0; q < G; ++q) v += acc[q * C + c];
    p.seg[k].dst[(size_t)by * len + i] = v;
  }
}

__global__ void __launch_bounds__(256) adam_kernel(const MlpArgs a, float lr, float c1, float c2,
                                                   const AdamPending pend) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i == 0 && pend.loss_rows > 0) {
    float l = 0.0f;
    for (int r = 0; r < pend.loss_rows; ++r) l += pend.loss_src[r];
    *pend.loss_out = l;
  }
  if (i >= a.n_params) return;
  float g = a.grad[i];
  for (int k = 0; k < pend.n; ++k) {
    const int64_t e = i - pend.seg[k].off;
    if (e >= 0 && e < pend.seg[k].len) {
      g = 0.0f;
      for (int r = 0; r < pend.seg[k].rows; ++r) g += pend.seg[k].src[(int64_t)r * pend.seg[k].len + e];
      a.grad[i] = g;
    }
  }
  const float m = fmaf(kAdamBeta1, a.adam_m[i] - g, g);      // β1 m + (1 - β1) g
  const float v = fmaf(kAdamBeta2, a.adam_v[i] - g * g, g * g);
  a.adam_m[i] = m;
  a.adam_v[i] = v;
  const float p = a.params_rw[i] - lr * (m * c1) / (sqrtf(v * c2) + kAdamEps);
  a.params_rw[i] = p;
  if (i >= a.off.W2 && i < a.off.W2 + W * W) {
    const int64_t e = i - a.off.W2, n = e / W, k = e % W;
    a.W2b_rw[n * W + k] = (__bf16)p;
    a.W2Tb_rw[k * W + n] = (__bf16)p;
  } else if (i >= a.off.W3 && i < a.off.W3 + W * W) {
    const int64_t e = i - a.off.W3, n = e / W, k = e % W;
    a.W3b_rw[n * W + k] = (__bf16)p;
    a.W3Tb_rw[k * W + n] = (__bf16)p;
  } else if (i >= a.off.W4 && i < a.off.W4 + 4 * W) {
    const int64_t e = i - a.off.W4, j = e / W, k = e % W;
#pragma unroll
    for (int part = 0; part < 3; ++part) a.W4s_rw[(4 * part + j) * W + k] = split3(p, part);
  }
}

// Rewrite the bf16 copies from the master weights (after a parameter upload):
// W2, W3, their transposes and the three-part W4.
__global__ void __launch_bounds__(256) refresh_bf16_kernel(const MlpArgs a) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= W * W) return;
  const int64_t n = e / W, k = e % W;
  const float p2 = a.params[a.off.W2 + e], p3 = a.params[a.off.W3 + e];
  a.W2b_rw[n * W + k] = (__bf16)p2;
  a.W2Tb_rw[k * W + n] = (__bf16)p2;
  a.W3b_rw[n * W + k] = (__bf16)p3;
  a.W3Tb_rw[k * W + n] = (__bf16)p3;
  if (e < 16 * W) {        // W4 in three parts, rows 12-15 zero
    const int64_t row = e / W;
    a.W4s_rw[e] = row < 12 ? split3(a.params[a.off.W4 + (row & 3) * W + k], (int)(row >> 2))
                           : (__bf16)0.0f;
  }
}

}  // namespace

int mlp_tile() { return TM; }

hipError_t launch_mlp_forward(const MlpArgs& a, bool train, hipStream_t s) {
  const dim3 grid((unsigned)((a.batch + TM - 1) / TM)), block(NT);
  if (train) hipLaunchKernelGGL(mlp_forward_kernel<true>, grid, block, 0, s, a);
  else       hipLaunchKernelGGL(mlp_forward_kernel<false>, grid, block, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mlp_weight_grad(const MlpArgs& a, hipStream_t s) {
  // 4 tiles × 2 layers × n_splits splits; the kernel maps the linear block
  // index to (group, tile) so that each group stays on one XCD
  if (a.n_splits % 4 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp_weight_grad_kernel, dim3(4u * 2u * (unsigned)a.n_splits), dim3(NT), 0, s, a);
  return hipGetLastError();
}

size_t sum_partials_tmp(int64_t len, int parts) {
  return parts > 64 ? 2 * (size_t)len * (size_t)((parts + 63) / 64) : 0;
}

hipError_t launch_sum_partials_multi(const SumSegment* segs, int nseg, float* tmp, hipStream_t s,
                                     int max_passes, SumLeft* left) {
  if (nseg < 0 || nseg > kMaxSumSegments) return hipErrorInvalidValue;
  struct State { const float* src; int rows; float* tmp; size_t half; int C; int gx; bool done; };
  State st[kMaxSumSegments];
  size_t off = 0;
  for (int k = 0; k < nseg; ++k) {
    const SumSegment& g = segs[k];
    int C = 64;
    while (C > 1 && C / 2 >= g.len) C /= 2;
    st[k] = {g.part, g.parts, tmp + off, sum_partials_tmp(g.len, g.parts) / 2, C,
             (int)((g.len + C - 1) / C), g.len <= 0};
    off += sum_partials_tmp(g.len, g.parts);
  }
  for (int pass = 0;; ++pass) {
    if (pass == max_passes) {
      for (int k = 0; k < nseg; ++k)
        if (left) left[k] = {st[k].src, segs[k].len, st[k].done ? 0 : st[k].rows};
      return hipSuccess;
    }
    SumPass p;
    p.nseg = 0;
    int64_t blocks = 0;
    int idx[kMaxSumSegments];
    for (int k = 0; k < nseg; ++k) {
      if (st[k].done) continue;
      const bool last = st[k].rows <= 64;
      const int next = last ? 1 : (st[k].rows + 63) / 64;
      auto& q = p.seg[p.nseg];
      q.src = st[k].src;
      q.dst = last ? segs[k].out : st[k].tmp + (pass & 1) * st[k].half;
      q.len = segs[k].len;
      q.first = blocks;
      q.rows = st[k].rows;
      q.C = st[k].C;
      q.gx = st[k].gx;
      idx[p.nseg++] = k;
      blocks += (int64_t)st[k].gx * next;
    }
    if (p.nseg == 0) {
      if (left)
        for (int k = 0; k < nseg; ++k) left[k] = {st[k].src, segs[k].len, 0};
      return hipSuccess;
    }
    hipLaunchKernelGGL(sum_partials_multi_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int j = 0; j < p.nseg; ++j) {
      State& x = st[idx[j]];
      if (x.rows <= 64) {
        x.done = true;
      } else {
        x.src = p.seg[j].dst;
        x.rows = (x.rows + 63) / 64;
      }
    }
  }
}

hipError_t launch_adam(const MlpArgs& a, float lr, float c1, float c2, hipStream_t s,
                       const AdamPending* pending) {
  AdamPending none{};
  const AdamPending& p = pending ? *pending : none;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((a.n_params + 255) / 256)), dim3(256), 0, s, a, lr,
                     c1, c2, p);
  return hipGetLastError();
}

hipError_t launch_refresh_bf16(const MlpArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(refresh_bf16_kernel, dim3((W * W + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace st

namespace st {
namespace {

__global__ void __launch_bounds__(256) features_kernel(const double* z, int64_t n, FeatureMap f,
                                                       int n_in, float* x) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  for (int i = 0; i < 6 && i < n_in; ++i)
    x[j * n_in + i] = (float)((z[(size_t)i * n + j] - f.center[i]) * f.inv_scale[i]);
  if (n_in == 7) x[j * n_in + 6] = (float)f.extra;
}

__global__ void __launch_bounds__(256) targets_kernel(const double* q, int64_t n, double r0, double r1,
                                                      double r2, double r3, float* t) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const double w = q[j], x = q[n + j], y = q[2 * n + j], z = q[3 * n + j];
  const double s = (w * r0 + x * r1 + y * r2 + z * r3) < 0.0 ? -1.0 : 1.0;
  t[j * 4 + 0] = (float)(s * w);
  t[j * 4 + 1] = (float)(s * x);
  t[j * 4 + 2] = (float)(s * y);
  t[j * 4 + 3] = (float)(s * z);
}

// Normal equations of the frame fit, one block per contiguous range of
// samples: rows [1, x, t] of 256 samples at a time in LDS, thread v owns one
// entry of [1,x][1,x]ᵀ (v < D*D) or of [1,x] tᵀ and sums it over the range in
// sample order.
__global__ void __launch_bounds__(256) fit_normal_kernel(const float* x, const float* t, int64_t n,
                                                         int n_in, double* partials) {
  constexpr int C = kMlpMaxIn + 1 + 4;
  __shared__ double rows[256][C];
  const int D = n_in + 1, V = D * D + 4 * D, tid = threadIdx.x;
  const int64_t per = (n + kFitBlocks - 1) / kFitBlocks;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = min(n, lo + per);
  const int p = tid < D * D ? tid / D : (tid - D * D) / 4;
  const int q = tid < D * D ? tid % D : D + (tid - D * D) % 4;
  double acc = 0.0;
  for (int64_t c0 = lo; c0 < hi; c0 += 256) {
    const int64_t j = c0 + tid;
    const bool in = j < hi;
    rows[tid][0] = in ? 1.0 : 0.0;
    for (int k = 0; k < n_in; ++k) rows[tid][1 + k] = in ? (double)x[j * n_in + k] : 0.0;
    for (int c = 0; c < 4; ++c) rows[tid][D + c] = in ? (double)t[j * 4 + c] : 0.0;
    __syncthreads();
    if (tid < V) {
      const int m = (int)min((int64_t)256, hi - c0);
      for (int i = 0; i < m; ++i) acc = fma(rows[i][p], rows[i][q], acc);
    }
    __syncthreads();
  }
  if (tid < V) partials[(int64_t)blockIdx.x * V + tid] = acc;
}

// Squared residuals of each component and their largest magnitude over one
// block's range; tree reduction in a fixed order.
__global__ void __launch_bounds__(256) fit_residual_kernel(const float* x, const float* t, int64_t n,
                                                           int n_in, FitCoef cf, double* partials) {
  __shared__ double red[256][8];
  const int tid = threadIdx.x;
  const int64_t per = (n + kFitBlocks - 1) / kFitBlocks;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = min(n, lo + per);
  double ss[4] = {0.0, 0.0, 0.0, 0.0}, mx[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t j = lo + tid; j < hi; j += 256) {
    for (int c = 0; c < 4; ++c) {
      double f = cf.c[c][0];
      for (int k = 0; k < n_in; ++k) f = fma(cf.c[c][1 + k], (double)x[j * n_in + k], f);
      const double r = (double)t[j * 4 + c] - f;
      ss[c] = fma(r, r, ss[c]);
      mx[c] = fmax(mx[c], fabs(r));
    }
  }
  for (int c = 0; c < 4; ++c) { red[tid][c] = ss[c]; red[tid][4 + c] = mx[c]; }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w)
      for (int c = 0; c < 4; ++c) {
        red[tid][c] += red[tid + w][c];
        red[tid][4 + c] = fmax(red[tid][4 + c], red[tid + w][4 + c]);
      }
    __syncthreads();
  }
  if (tid < 8) partials[(int64_t)blockIdx.x * 8 + tid] = red[0][tid];
}

}  // namespace

hipError_t launch_fit_normal(const float* x, const float* t, int64_t n, int n_in, double* partials,
                             hipStream_t s) {
  hipLaunchKernelGGL(fit_normal_kernel, dim3(kFitBlocks), dim3(256), 0, s, x, t, n, n_in, partials);
  return hipGetLastError();
}

hipError_t launch_fit_residual(const float* x, const float* t, int64_t n, int n_in,
                               const FitCoef& coef, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(fit_residual_kernel, dim3(kFitBlocks), dim3(256), 0, s, x, t, n, n_in, coef,
                     partials);
  return hipGetLastError();
}

hipError_t launch_features(const double* z, int64_t n, const FeatureMap& f, int n_in, float* x,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, z, n, f,
                     n_in, x);
  return hipGetLastError();
}

hipError_t launch_targets(const double* q, int64_t n, const double* ref, float* t, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(targets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, q, n, ref[0],
                     ref[1], ref[2], ref[3], t);
  return hipGetLastError();
}

}  // namespace st
