// Microbenchmarks of the chip's peaks: the denominators of the roofline
// fractions, measured on the device the library runs on.  Not a step of the
// method.
//
//   FP64 vector FMA   every lane runs eight independent v_fma_f64 chains
//   FP32 vector FMA   the same with v_fma_f32 (unpacked: the library is built
//                     without packed single-precision instructions)
//   bf16 MFMA         every wave runs four independent chains of
//                     v_mfma_f32_16x16x32_bf16 (16·16·32 multiply-adds each)
//   HBM copy          16-byte loads and stores over two device buffers
//
// Each is launched with enough workgroups to fill all compute units several
// times over and timed with HIP events over repeated launches, after one
// warm-up launch.  Each kernel ends in a store to a small device buffer,
// guarded by a test on its result that the arguments never meet, so that the
// compiler keeps the arithmetic.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include "spintrack.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kFmaIters = 2048;    // per chain
constexpr int kMfmaIters = 1024;   // per chain
constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) fp64_fma_kernel(double b, double c, double* out) {
  double x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = (double)(threadIdx.x + j) * 1e-3;
  for (int i = 0; i < kFmaIters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = fma(x[j], b, c);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += x[j];
  if (s == 12345.678) out[0] = s;   // never true for the arguments used; keeps the chains live
}

__global__ void __launch_bounds__(kBlock) fp32_fma_kernel(float b, float c, float* out) {
  float x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = (float)(threadIdx.x + j) * 1e-3f;
  for (int i = 0; i < kFmaIters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = fmaf(x[j], b, c);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += x[j];
  if (s == 12345.678f) out[0] = s;
}

__global__ void __launch_bounds__(kBlock) mfma_bf16_kernel(float seed, float* out) {
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(seed * (float)(e + 1));
    b[e] = (__bf16)(seed * (float)(8 - e));
  }
  f32x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = f32x4{(float)j, 0.f, 0.f, 0.f};   // distinct chains
  for (int i = 0; i < kMfmaIters; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  if (s == 12345.678f) out[0] = s;
}

// Four 16-byte loads in flight per lane before their stores, then the tail
// one at a time.
__global__ void __launch_bounds__(kBlock) copy_kernel(const float4* __restrict__ src,
                                                      float4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    float4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) dst[i + u * stride] = v[u];
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace

extern "C" st_status st_measure_peaks(int device, st_peaks* out) {
  if (!out) return ST_EINVAL;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return ST_EINVAL;
  int old = -1;
  if (hipGetDevice(&old) != hipSuccess) old = -1;
  if (hipSetDevice(device) != hipSuccess) return ST_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return ST_EDEVICE;
  const int cus = prop.multiProcessorCount;
  st_status st = ST_OK;
  Events ev;
  double* dsink = nullptr;
  float4 *src = nullptr, *dst = nullptr;
  const int64_t copy_bytes = (int64_t)1 << 30;      // per buffer
  const int64_t n4 = copy_bytes / 16;
  hipError_t e = hipEventCreate(&ev.a);
  if (e == hipSuccess) e = hipEventCreate(&ev.b);
  if (e == hipSuccess) e = hipMalloc(&dsink, 64);
  if (e == hipSuccess) e = hipMalloc(&src, copy_bytes);
  if (e == hipSuccess) e = hipMalloc(&dst, copy_bytes);
  if (e == hipSuccess) e = hipMemset(src, 0, copy_bytes);
  auto timed = [&](auto launch, int reps, float* ms) -> hipError_t {
    launch();
    hipError_t r = hipGetLastError();
    if (r == hipSuccess) r = hipEventRecord(ev.a, nullptr);
    for (int i = 0; r == hipSuccess && i < reps; ++i) {
      launch();
      r = hipGetLastError();
    }
    if (r == hipSuccess) r = hipEventRecord(ev.b, nullptr);
    if (r == hipSuccess) r = hipEventSynchronize(ev.b);
    if (r == hipSuccess) r = hipEventElapsedTime(ms, ev.a, ev.b);
    return r;
  };
  const int reps = 10;
  float ms = 0.f;
  // FP64: 16 workgroups of 256 lanes per CU
  const int fma_blocks = 16 * cus;
  if (e == hipSuccess)
    e = timed([&] { hipLaunchKernelGGL(fp64_fma_kernel, dim3(fma_blocks), dim3(kBlock), 0, nullptr,
                                       0.999999, 1e-9, dsink); }, reps, &ms);
  if (e == hipSuccess)
    out->fp64_fma_tflops = 2.0 * 8 * kFmaIters * (double)fma_blocks * kBlock * reps / (ms * 1e-3) / 1e12;
  if (e == hipSuccess)
    e = timed([&] { hipLaunchKernelGGL(fp32_fma_kernel, dim3(fma_blocks), dim3(kBlock), 0, nullptr,
                                       0.999999f, 1e-9f, (float*)dsink); }, reps, &ms);
  if (e == hipSuccess)
    out->fp32_fma_tflops = 2.0 * 8 * kFmaIters * (double)fma_blocks * kBlock * reps / (ms * 1e-3) / 1e12;
  // bf16 MFMA: 16 workgroups of four waves per CU
  const int mfma_blocks = 16 * cus;
  if (e == hipSuccess)
    e = timed([&] { hipLaunchKernelGGL(mfma_bf16_kernel, dim3(mfma_blocks), dim3(kBlock), 0, nullptr,
                                       0.001f, (float*)dsink); }, reps, &ms);
  if (e == hipSuccess)
    out->bf16_mfma_tflops = 2.0 * 16 * 16 * 32 * 4.0 * kMfmaIters * (double)mfma_blocks * (kBlock / 64) *
                            reps / (ms * 1e-3) / 1e12;
  // HBM: 1 GiB read and 1 GiB written per launch
  const int copy_blocks = 64 * cus;
  if (e == hipSuccess)
    e = timed([&] { hipLaunchKernelGGL(copy_kernel, dim3(copy_blocks), dim3(kBlock), 0, nullptr, src, dst,
                                       n4); }, reps, &ms);
  if (e == hipSuccess) out->copy_gbps = 2.0 * (double)copy_bytes * reps / (ms * 1e-3) / 1e9;
  if (e != hipSuccess) st = ST_EDEVICE;
  (void)hipDeviceSynchronize();
  if (dsink) (void)hipFree(dsink);
  if (src) (void)hipFree(src);
  if (dst) (void)hipFree(dst);
  if (old >= 0) (void)hipSetDevice(old);
  return st;
}
