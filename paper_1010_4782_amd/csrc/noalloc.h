// The fixed device workspace behind stag_apply_m_noalloc (noalloc.hip).
#pragma once

#include "launch.h"

namespace stag {

constexpr size_t kNoAllocBytes = size_t(64) << 20;  // per GPU, held until the process ends
constexpr size_t kNoAllocParamBytes = 16384;        // parameter block at the start of the array
constexpr int kNoAllocMaxRhs = 64;

// Look up (once per device, with that device current) the device address of the array.
hipError_t noalloc_init(int device);
// The array's address on `device` (looked up first if needed).
hipError_t noalloc_address(int device, unsigned char** out);
// Write the problem table and the per-RHS scalars (4 m^2 per RHS) of a single-problem launch to the
// parameter block at `base`, with one kernel on `st`.
hipError_t noalloc_write_params(unsigned char* base, const ProbDev& pd, const double* mass, int nrhs,
                                hipStream_t st);
size_t noalloc_scal_offset();

}  // namespace stag
