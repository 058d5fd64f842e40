// amrmg_noalloc.hpp -- the statically sized device array behind
// amrmg_solve_noalloc (amrmg_noalloc.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace amrmg {

// bytes of the array; a solve whose workspace needs more is refused
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

// Resolve the array's address on device `device` (with that device current),
// once per device; returns the status of the lookup (kept for later calls).
hipError_t noalloc_setup(int device);
// The device address of the array on `device`, or nullptr when noalloc_setup
// has not succeeded for it; *err receives the lookup's status.
void *noalloc_scratch(int device, hipError_t *err);

}  // namespace amrmg
