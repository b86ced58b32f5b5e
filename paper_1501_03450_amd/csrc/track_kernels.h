// Launchers of the tracking kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "lattice_table.h"

namespace st {

int track_block_size();

// nt: number of series terms of the quaternion half-angle polynomial (6, 8, 12, 16).
hipError_t launch_track_fp64(const TrackArgs& a, int nt, hipStream_t stream);

hipError_t launch_reduce_polarization(const double* partials, int n_blocks, int n_reports,
                                      double* out, hipStream_t stream);

}  // namespace st
