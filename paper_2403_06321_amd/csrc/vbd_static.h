// The fixed device scratch of vbd_step_static (vbd_static.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace vbd {

// 96 MiB per device, held from the library's load until the process ends:
// x, x^t, y (16 B each per vertex), the Chebyshev history (2 x 16 B, only
// when acceleration is on) and one contact byte, each section 256-B aligned,
// so about 1.2M vertices with acceleration and 2M without.
constexpr size_t kStaticScratchBytes = size_t(96) << 20;

// Device address of the scratch array on `device`, which must be the current
// device; looked up on the first call per device and kept.
hipError_t static_scratch(int device, void **ptr);

}  // namespace vbd
