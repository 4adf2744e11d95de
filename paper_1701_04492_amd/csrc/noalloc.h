// Fixed device scratch of the allocation-free entry point.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

// Size of the per-device scratch array and the problem sizes it serves
// (nufft3_exec_noalloc: M samples, N frequencies).  Worst case in FP64 with the
// largest rank: 16 M + 72 N bytes of type-III temporaries, about 60 N of the
// inner type-I plan's sample data, K L 16 <= 20 * 2^15 * 16 of its exchange
// buffer, the twiddle tables and 256-byte alignment per block: below 32 MiB.
#define NUFFT_NOALLOC_BYTES ((size_t)48 << 20)
#define NUFFT_NOALLOC_MAX_M ((int64_t)1 << 20)
#define NUFFT_NOALLOC_MAX_N ((int64_t)1 << 15)
#define NUFFT_NOALLOC_MAX_DEVICES 64

namespace nufft {
// Device address and size of the current device's scratch array (looked up
// once per device).
hipError_t noalloc_scratch(void **ptr, size_t *bytes);
}  // namespace nufft
