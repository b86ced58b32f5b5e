// Launchers of the tracking kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "lattice_table.h"

namespace st {

int track_block_size();

// nt: number of series terms of the double-precision quaternion half-angle
// series (5, 6, 8, 12, 16); mixed: the kernel with single-precision spin
// arithmetic in the elements flagged for it.
// ext: the lattice uses drift-kick (TEAPOT) bends or piece-wise constant
// spin placements (run in double precision).
hipError_t launch_track(const TrackArgs& a, int nt, bool mixed, bool ext, hipStream_t stream);

// a.fallback non-null selects surrogate tracking: an orbit-only launch for the
// a.feat_n particles on the network, then the full kernel for the others.

hipError_t launch_surrogate_spin(double* spin, const int32_t* alive, const int32_t* fallback,
                                 const float* qnn, int64_t n, hipStream_t s);
// Network rotations of a multi-turn surrogate launch for the n_net particles
// on the network, lanes g < n_net of the lane order perm (qnn [turn][n_net][4]
// and turns_done [n_net] from the launch).
hipError_t launch_surrogate_spin_turns(double* spin, const int32_t* perm,
                                       const int32_t* turns_done, const float* qnn, int64_t n_net,
                                       int64_t n, hipStream_t s);
// Audit of the network quaternions against the tracked ones: failures get
// fallback[j] = turn and failed[j] = 1; every other particle failed[j] = 0.
hipError_t launch_audit(const int32_t* alive, int32_t* fallback, int32_t* failed, const float* qnn,
                        const double* q64, int64_t n, double threshold, int32_t turn,
                        hipStream_t s);
// Rollback to the checkpoint, and status after the replay, of the particles
// with failed[j] != 0.
hipError_t launch_replay_prepare(const int32_t* failed, double* z, double* spin,
                                 const double* ck_z, const double* ck_spin, const int32_t* ck_alive,
                                 int32_t* ralive, int64_t n, hipStream_t s);
hipError_t launch_replay_finish(const int32_t* failed, const int32_t* ralive, int32_t* alive,
                                int64_t n, hipStream_t s);
// Lane order for surrogate tracking: a stable partition of 0..n-1 (see
// partition_key; flag is the audit's failed[] array in mode 1); counts and
// offsets hold 3 ints per 256 particles.
hipError_t launch_partition(int mode, const int32_t* flag, const int32_t* alive,
                            const int32_t* fallback, int64_t n, int32_t* counts, int32_t* offsets,
                            int32_t* perm, hipStream_t s);
hipError_t launch_polarization_partials(const double* spin, const int32_t* alive, int64_t n,
                                        double* partials, hipStream_t s);

hipError_t launch_reduce_polarization(const double* partials, int n_blocks, int n_reports,
                                      double* out, hipStream_t stream);

}  // namespace st
