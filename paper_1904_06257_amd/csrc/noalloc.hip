// Fixed device buffer behind shaken_sweep_noalloc, the sweep variant for
// callers that cannot allocate device memory.
//
// The observables of a recorded sweep are accumulated as partial sums
// (kLogParts lines of a context's line width per logged full step); the
// allocating sweep keeps them in log space it grows on demand, this variant
// keeps them in `scratch`, a file-scope device array of fixed size that every
// context on a device shares.  The host never passes the array's name to a
// kernel: its device address is looked up once per device with
// hipGetSymbolAddress (at context creation, with the device current) and that
// address is what the kernels receive.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "shaken_internal.hpp"
#include "noalloc.hpp"

namespace shaken {

namespace {

constexpr int64_t kScratchI64 = (int64_t)(4u << 20) / 8;  // 4 MiB
static __device__ __align__(256) int64_t scratch[kScratchI64];

std::mutex g_mu;
std::vector<int64_t *> g_ptr;  // per device ordinal; nullptr = not looked up yet

// H and M of every logged slot from its partial lines (one thread per slot):
// E_J = sum of the parts' entry 0, plus_k = sum of the parts' entry 1 + k;
// M = 2 sum_k plus_k - n,  H = -E_J - sum_k lam2_k (2 plus_k - size_k)
//   = -E_J - 2 sum_k lam2_k plus_k + c0   with c0 = sum_k lam2_k size_k.
__global__ void k_log_reduce(const int64_t *__restrict__ raw, int64_t slots, int64_t line,
                             LogReduceArgs a, int64_t *__restrict__ H, int64_t *__restrict__ M) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= slots) return;
    const int64_t *r = raw + t * (int64_t)kLogParts * line;
    int64_t ej = 0, plus = 0, lp = 0;
    for (int p = 0; p < kLogParts; ++p) {
        ej += r[p * line];
        for (int k = 0; k < a.ncls; ++k) {
            const int64_t v = r[p * line + 1 + k];
            plus += v;
            lp += a.lam2[k] * v;
        }
    }
    if (H) H[t] = -ej - 2 * lp + a.c0;
    if (M) M[t] = 2 * plus - a.n;
}

}  // namespace

int64_t noalloc_capacity() { return kScratchI64; }

hipError_t noalloc_scratch(int device, int64_t **out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (device < 0) return hipErrorInvalidDevice;
    if ((size_t)device >= g_ptr.size()) g_ptr.resize((size_t)device + 1, nullptr);
    if (!g_ptr[(size_t)device]) {
        // the caller made `device` current; each device holds its own copy
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[(size_t)device] = static_cast<int64_t *>(p);
    }
    *out = g_ptr[(size_t)device];
    return hipSuccess;
}

hipError_t launch_log_reduce(const int64_t *raw, int64_t slots, int64_t line, const LogReduceArgs &a,
                             int64_t *H, int64_t *M, hipStream_t stream) {
    if (slots <= 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(k_log_reduce, dim3((unsigned)((slots + b - 1) / b)), dim3(b), 0, stream, raw, slots,
                       line, a, H, M);
    return hipGetLastError();
}

}  // namespace shaken
