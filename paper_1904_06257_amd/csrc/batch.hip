// Persistent batch kernel of libshaken (one workgroup per chain, spins in LDS).
#include "shaken_internal.hpp"

namespace shaken {

bool persistent_fits(const ChainDesc &) { return false; }

hipError_t launch_persistent(const ChainDesc *, int, const int32_t *, int32_t *, uint32_t, int64_t,
                             int, int, int, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace shaken
