// Per-particle kernels around the surrogate turns of st_track_surrogate:
// the network's spin rotation, the audit against the tracked quaternion,
// rollback and replay bookkeeping, the lane-order partition, and the
// polarization partials of a surrogate turn.  All are elementwise over the
// particles (or a stable partition of them) and bound by HBM.
#include <hip/hip_runtime.h>

#include "fp64_maps.h"
#include "track_kernels.h"

namespace st {

namespace {

// S <- q S q* with the network's quaternion (float [n][4], normalised again in
// double) for alive particles that are not on the fallback path.
__global__ void __launch_bounds__(256) surrogate_spin_kernel(double* spin, const int32_t* alive,
                                                             const int32_t* fallback,
                                                             const float* qnn, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n || alive[j] != 1 || fallback[j] != 0) return;
  Quat q = {qnn[4 * j], qnn[4 * j + 1], qnn[4 * j + 2], qnn[4 * j + 3]};
  const double inv = rsqrt_nr(fma(q.w, q.w, fma(q.x, q.x, fma(q.y, q.y, q.z * q.z))));
  q.w *= inv; q.x *= inv; q.y *= inv; q.z *= inv;
  double sx = spin[j], sy = spin[n + j], sz = spin[2 * n + j];
  qrotate(q, sx, sy, sz);
  spin[j] = sx; spin[n + j] = sy; spin[2 * n + j] = sz;
}

// The same over the turns of a multi-turn launch, for the n_net particles on
// the network (lanes g < n_net of the lane order perm): the particle that
// completed turns_done[g] turns is rotated by the network's quaternion of each
// of them (qnn [turn * n_net + g][4]), in turn order.
__global__ void __launch_bounds__(256) surrogate_spin_turns_kernel(double* spin,
                                                                   const int32_t* perm,
                                                                   const int32_t* turns_done,
                                                                   const float* qnn, int64_t n_net,
                                                                   int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= n_net) return;
  const int k_end = turns_done[g];
  if (k_end <= 0) return;
  const int64_t j = perm[g];
  double sx = spin[j], sy = spin[n + j], sz = spin[2 * n + j];
  for (int k = 0; k < k_end; ++k) {
    const float* f = qnn + ((int64_t)k * n_net + g) * 4;
    Quat q = {f[0], f[1], f[2], f[3]};
    const double inv = rsqrt_nr(fma(q.w, q.w, fma(q.x, q.x, fma(q.y, q.y, q.z * q.z))));
    q.w *= inv; q.x *= inv; q.y *= inv; q.z *= inv;
    qrotate(q, sx, sy, sz);
  }
  spin[j] = sx; spin[n + j] = sy; spin[2 * n + j] = sz;
}

// Audit: largest component difference between the network's quaternion and
// the tracked one (sign aligned); above the threshold the particle falls back
// (fallback[j] = turn) and is flagged in failed[j] for the rollback and
// replay of this audit.  Every particle's flag is written, so a flag never
// survives from an earlier audit or call.
__global__ void __launch_bounds__(256) audit_kernel(const int32_t* alive, int32_t* fallback,
                                                    int32_t* failed, const float* qnn,
                                                    const double* q64, int64_t n,
                                                    double threshold, int32_t turn) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  if (alive[j] != 1 || fallback[j] != 0) {
    failed[j] = 0;
    return;
  }
  const double a[4] = {qnn[4 * j], qnn[4 * j + 1], qnn[4 * j + 2], qnn[4 * j + 3]};
  const double na = rsqrt_nr(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
  const double b[4] = {q64[j], q64[n + j], q64[2 * n + j], q64[3 * n + j]};
  const double dot = a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
  const double s = dot < 0.0 ? -1.0 : 1.0;
  double d = 0.0;
  for (int c = 0; c < 4; ++c) d = fmax(d, fabs(a[c] * na - s * b[c]));
  const bool fail = !(d <= threshold);
  if (fail) fallback[j] = turn;
  failed[j] = fail ? 1 : 0;
}

// Rollback of the particles that failed the last audit (failed[j] != 0):
// their orbit, spin and status go back to the checkpoint of the previous
// audit, and ralive marks exactly them as the live set of the replay launch.
__global__ void __launch_bounds__(256) replay_prepare_kernel(const int32_t* failed, double* z,
                                                             double* spin, const double* ck_z,
                                                             const double* ck_spin,
                                                             const int32_t* ck_alive,
                                                             int32_t* ralive, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  if (failed[j] == 0) {
    ralive[j] = 0;
    return;
  }
  for (int c = 0; c < 6; ++c) z[c * n + j] = ck_z[c * n + j];
  for (int c = 0; c < 3; ++c) spin[c * n + j] = ck_spin[c * n + j];
  ralive[j] = ck_alive[j];
}

// After the replay: the replayed particles take their status from it.
__global__ void __launch_bounds__(256) replay_finish_kernel(const int32_t* failed,
                                                            const int32_t* ralive, int32_t* alive,
                                                            int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < n && failed[j] != 0) alive[j] = ralive[j];
}

// Stable three-way partition of the particle indices into a lane order.
// key 0 first, then 1, then 2; within a key the original order is kept.
// mode 0 (surrogate turns): 0 = alive on the network, 1 = alive on the
// fallback path, 2 = lost.  mode 1 (replay after an audit; `flag` is the
// audit's failed[] array): 0 = failed this audit, 1 = every other particle.
__device__ __forceinline__ int partition_key(int mode, const int32_t* flag, const int32_t* alive,
                                             const int32_t* fallback, int64_t j) {
  if (mode == 1) return flag[j] != 0 ? 0 : 1;
  if (alive[j] != 1) return 2;
  return fallback[j] == 0 ? 0 : 1;
}

__global__ void __launch_bounds__(256) partition_count_kernel(int mode, const int32_t* flag,
                                                              const int32_t* alive,
                                                              const int32_t* fallback, int64_t n,
                                                              int32_t* counts) {
  __shared__ int32_t c[3];
  if (threadIdx.x < 3) c[threadIdx.x] = 0;
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < n) atomicAdd(&c[partition_key(mode, flag, alive, fallback, j)], 1);
  __syncthreads();
  if (threadIdx.x < 3) counts[(int64_t)blockIdx.x * 3 + threadIdx.x] = c[threadIdx.x];
}

// Exclusive offsets of every (block, key): key-major over the whole array.
__global__ void __launch_bounds__(256) partition_scan_kernel(const int32_t* counts, int64_t nb,
                                                             int32_t* offsets) {
  __shared__ int64_t part[256][3];
  // each thread sums a contiguous range of blocks, then a fixed-order scan
  const int64_t per = (nb + 255) / 256;
  const int64_t b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
  int64_t s[3] = {0, 0, 0};
  for (int64_t b = b0; b < b1; ++b)
    for (int k = 0; k < 3; ++k) s[k] += counts[b * 3 + k];
  for (int k = 0; k < 3; ++k) part[threadIdx.x][k] = s[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t base = 0;
    for (int k = 0; k < 3; ++k)
      for (int t = 0; t < 256; ++t) {
        const int64_t v = part[t][k];
        part[t][k] = base;
        base += v;
      }
  }
  __syncthreads();
  int64_t o[3] = {part[threadIdx.x][0], part[threadIdx.x][1], part[threadIdx.x][2]};
  for (int64_t b = b0; b < b1; ++b)
    for (int k = 0; k < 3; ++k) {
      offsets[b * 3 + k] = (int32_t)o[k];
      o[k] += counts[b * 3 + k];
    }
}

__global__ void __launch_bounds__(256) partition_scatter_kernel(int mode, const int32_t* flag,
                                                                const int32_t* alive,
                                                                const int32_t* fallback,
                                                                int64_t n, const int32_t* offsets,
                                                                int32_t* perm) {
  __shared__ int32_t wave_count[4][3];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int key = j < n ? partition_key(mode, flag, alive, fallback, j) : 3;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int rank = 0;
  for (int k = 0; k < 3; ++k) {
    const uint64_t m = __ballot(key == k);
    if (key == k) rank = __popcll(m & below);
    if (lane == 0) wave_count[wv][k] = __popcll(m);
  }
  __syncthreads();
  if (key < 3) {
    int before = 0;
    for (int w = 0; w < wv; ++w) before += wave_count[w][key];
    perm[offsets[(int64_t)blockIdx.x * 3 + key] + before + rank] = (int32_t)j;
  }
}

// Per-block sums (Sx, Sy, Sz, N) over alive particles for one report.
__global__ void __launch_bounds__(256) polarization_partials_kernel(const double* spin,
                                                                    const int32_t* alive, int64_t n,
                                                                    double* partials) {
  __shared__ double red[4][4];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = j < n && alive[j] == 1;
  double v[4] = {live ? spin[j] : 0.0, live ? spin[n + j] : 0.0, live ? spin[2 * n + j] : 0.0,
                 live ? 1.0 : 0.0};
  for (int c = 0; c < 4; ++c)
    for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off, 64);
  if ((threadIdx.x & 63) == 0)
    for (int c = 0; c < 4; ++c) red[threadIdx.x >> 6][c] = v[c];
  __syncthreads();
  if (threadIdx.x < 4)
    partials[(int64_t)blockIdx.x * 4 + threadIdx.x] =
        red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

}  // namespace

hipError_t launch_surrogate_spin(double* spin, const int32_t* alive, const int32_t* fallback,
                                 const float* qnn, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(surrogate_spin_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, spin,
                     alive, fallback, qnn, n);
  return hipGetLastError();
}

hipError_t launch_surrogate_spin_turns(double* spin, const int32_t* perm,
                                       const int32_t* turns_done, const float* qnn, int64_t n_net,
                                       int64_t n, hipStream_t s) {
  if (n_net <= 0) return hipSuccess;
  hipLaunchKernelGGL(surrogate_spin_turns_kernel, dim3((unsigned)((n_net + 255) / 256)), dim3(256), 0,
                     s, spin, perm, turns_done, qnn, n_net, n);
  return hipGetLastError();
}

hipError_t launch_audit(const int32_t* alive, int32_t* fallback, int32_t* failed, const float* qnn,
                        const double* q64, int64_t n, double threshold, int32_t turn,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(audit_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, alive, fallback,
                     failed, qnn, q64, n, threshold, turn);
  return hipGetLastError();
}

hipError_t launch_replay_prepare(const int32_t* failed, double* z, double* spin,
                                 const double* ck_z, const double* ck_spin, const int32_t* ck_alive,
                                 int32_t* ralive, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(replay_prepare_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     failed, z, spin, ck_z, ck_spin, ck_alive, ralive, n);
  return hipGetLastError();
}

hipError_t launch_replay_finish(const int32_t* failed, const int32_t* ralive, int32_t* alive,
                                int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(replay_finish_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     failed, ralive, alive, n);
  return hipGetLastError();
}

hipError_t launch_partition(int mode, const int32_t* flag, const int32_t* alive,
                            const int32_t* fallback, int64_t n, int32_t* counts, int32_t* offsets,
                            int32_t* perm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(partition_count_kernel, dim3((unsigned)nb), dim3(256), 0, s, mode, flag, alive,
                     fallback, n, counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(partition_scan_kernel, dim3(1), dim3(256), 0, s, counts, nb, offsets);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(partition_scatter_kernel, dim3((unsigned)nb), dim3(256), 0, s, mode, flag,
                     alive, fallback, n, offsets, perm);
  return hipGetLastError();
}

hipError_t launch_polarization_partials(const double* spin, const int32_t* alive, int64_t n,
                                        double* partials, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(polarization_partials_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     spin, alive, n, partials);
  return hipGetLastError();
}

}  // namespace st
