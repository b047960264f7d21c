// scratch.h -- the static device scratch area (scratch.hip).
#pragma once

#include <stddef.h>

namespace nep {

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;   // per GPU
constexpr int SCRATCH_MAX_DEVICES = 64;

// Device address and size of the current device's scratch array (resolved
// once per device). 0 on success, < 0 if the device or the symbol lookup fails.
int scratch_area(void **base, size_t *bytes);

}  // namespace nep
