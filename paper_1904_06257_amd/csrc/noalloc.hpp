// The fixed device buffer of shaken_sweep_noalloc (noalloc.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace shaken {

// field classes the device-side log reduction takes (lambda values)
constexpr int kNoallocClasses = 32;

// what turns a slot's partial lines into H and M (see k_log_reduce)
struct LogReduceArgs {
    int64_t lam2[kNoallocClasses];  // 2 * lambda of each class (integers)
    int64_t c0;                     // sum_k lam2[k] * (sites of class k)
    int64_t n;                      // sites
    int32_t ncls;
    int32_t pad;
};

// int64 entries of the buffer
int64_t noalloc_capacity();

// device address of the buffer on `device`, which must be the current device;
// looked up once per device, then cached
hipError_t noalloc_scratch(int device, int64_t **out);

// H[t], M[t] (either may be null) for t < slots from the partial lines at raw
// (slot t: kLogParts lines of `line` int64)
hipError_t launch_log_reduce(const int64_t *raw, int64_t slots, int64_t line, const LogReduceArgs &a,
                             int64_t *H, int64_t *M, hipStream_t stream);

}  // namespace shaken
