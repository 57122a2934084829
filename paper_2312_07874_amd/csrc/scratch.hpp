// Fixed-size device workspace of esd_residual_noalloc (see scratch.hip).
#pragma once

#include <cstddef>

namespace esd {

// bytes of the per-GPU scratch array; plans whose residual workspace exceeds
// it are rejected by esd_residual_noalloc
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;

// device address of the current device's scratch array (looked up once per
// device and cached); returns 0 or a hipError_t
int scratch_address(void** out, int* device);

}  // namespace esd
