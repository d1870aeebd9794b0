// Internal declarations shared by the host runtime (api.cpp) and the HIP
// kernels (kernels.hip) of libshaken.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shaken.h"

namespace shaken {

constexpr uint32_t kGraphStream = 0x80000000u;  // fourth counter word, graph uniforms
constexpr uint32_t kInitStep = 0xFFFFFFFFu;     // half-step index of the random start
constexpr int kLogParts = 8;   // partial accumulators per logged value (spread atomics)
constexpr int kRows = 8;       // rows of one word column per lane (bit-packed torus)

enum Kind : int32_t { KIND_TORUS = 0, KIND_GRAPH = 1 };
enum Format : int32_t { FMT_INT8 = 1, FMT_BITPACKED = 2 };

// Everything a kernel needs to advance one chain.  Lives in device memory for
// batches and is passed by value for single-chain launches.
struct ChainDesc {
    uint64_t seed;
    uint32_t replica;
    int32_t kind;
    int32_t format;
    int32_t L;        // torus side
    int32_t W;        // torus words per row (ceil(L/32))
    int32_t n;        // sites (L*L or graph vertices)
    void *spin[2];    // spin[0] holds the configuration read at even offsets
    // bit-packed torus: classes j = (#plus neighbours in the half) + 3*(own spin is +1)
    // triangular torus: j = n_plus + 4*(own spin is +1), eight classes
    uint32_t tsmall[8];  // t of the class: floor(p_small * 2^32), p_small = min(p, 1-p)
    uint32_t sgn;        // bit j: class j compares flipped (field >= 0; either way where T = 2^31)
    int32_t fold3;       // mirror classes share t and have opposite flips (3 classes
                         // after folding; 4 on the triangular torus)
    int32_t tri;         // triangular torus (section 4): third oriented edge (x, x + e1 + e2)
    uint32_t wdiv;       // bit-packed torus: ceil(2^32 / W), so that g / W = umulhi(g, wdiv)
                         // for every g with g W < 2^32 (g < rows * W / kRows here)
    int32_t J;           // uniform torus coupling
    // generic threshold table (int8 torus, graph): ((S+smax)*2 + (sigma>0))*ncls + cls
    const uint64_t *lut;
    int32_t smax;
    int32_t ncls;
    // graph: CSR per half (0 = in-half, read in half-step 1; 1 = out-half)
    const int32_t *rowptr[2];
    const int32_t *col[2];
    const int8_t *jw[2];     // coupling per CSR entry
    const uint8_t *cls;      // field class per vertex (never NULL on device)
    int32_t maxdeg;          // largest half-degree
    int32_t ell_k;           // ELL: slots per vertex (0 = no ELL layout)
    // ELL (couplings +-1, degree <= 4): ell[k * ell_stride + v] = index (bits
    // 0-28) | half (bits 29-30: 1 = in-half, 2 = out-half, 0 = empty slot,
    // whose index is v itself) | J < 0 (bit 31)
    const uint32_t *ell;
    int64_t ell_stride;      // n rounded up to a multiple of 4
    // packed record per vertex (couplings +-1, degree <= 3, n <= 65536, at most
    // 16 classes), ell_stride entries: bits 0-47 three 16-bit neighbour
    // indices; bit 48+k: slot k is in the in-half; 51+k: in the out-half;
    // 54+k: J < 0; bits 57-60 field class.  Unused slots and padding vertices
    // have index 0 and no half bit.
    const uint64_t *pell;
    // +-J torus (couplings of one magnitude J, any signs): two L x W bit planes,
    // plane 0 bit (r, c) set iff J((r,c), up) < 0, plane 1 iff J((r,c), right)
    // < 0; null for a uniform coupling.  Flipping a neighbour's bit where its
    // edge is negative turns the field into J (2 n_plus - 2) + q sigma + lambda
    // with n_plus counted on the flipped bits, so the classes and thresholds of
    // the uniform torus apply unchanged.
    const uint32_t *jneg;
    // 1: reversed order P^{sh'} (section 3): the half read at half-step s is
    // (s & 1) ^ 1, the out-half (torus ur) first
    int32_t rev;
    // frozen set B (section 3.1) as bits in the layout of the bit-packed spins
    // (torus L x W words, graph ceil(n/32)): these sites are written +1 by
    // every half-step and by the start; null if B is empty
    const uint32_t *frozen;
    // observables log: slot t is kLogParts lines of log_line int64; line p holds
    // partial sums [E_J, plus_0 .. plus_{ncls-1}] (a block adds into line
    // blockIdx % kLogParts, so that thousands of blocks do not queue on one
    // address); the host adds the lines.
    int64_t *log;
    int64_t log_line;        // 1 + ncls rounded up to 16 (one 128-byte line)
    int64_t log_stride;      // kLogParts * log_line
    // best-energy tracking (persistent batches): H = -E_J - sum_c lam2[c] *
    // (2 plus_c - csize[c]); track[0] = H of the last configuration, track[1] =
    // lowest H of the call; best = that configuration as bits
    int64_t *track;
    uint32_t *best;
    int32_t lam2[16];
    int32_t csize[16];
    // int8 graph chains small enough for the LDS-staged kernel: a bit-packed
    // copy of spin[i] (one bit per vertex, layout of the bit-packed spins),
    // written by that kernel beside its int8 output; null otherwise
    uint32_t *mirror[2];
    // graphs the LDS-staged kernel takes (n < 2^21): each CSR entry as one
    // word, index | (v & 3) << 21 | J << 24 with v the entry's row vertex,
    // padded by 16 zero entries past a multiple of four; null otherwise
    const int32_t *cj[2];
    // graphs the LDS-staged kernel takes whose half-degrees are at most three
    // and whose couplings share one magnitude j0: three slots per vertex
    // (vertex v at 3v .. 3v+2), each (index & 31) | (index >> 5) << 7 | J < 0
    // << 31, so that bits 5-22 are the byte offset of the index's word in
    // LDS and bits 0-4 its bit; slot 0 also holds the vertex's degree in the
    // half (bits 23-24); empty slots point at a zero word past the
    // configuration (word graph_lds_max_words()); null otherwise
    const uint32_t *e3[2];
    int32_t j0;
};

// workgroup size of the LDS-staged graph kernel; as a launch's block size it
// selects that kernel
constexpr int kLdsGraphBlock = 1024;

// can chain d run in the LDS-staged graph kernel (graph, at most 1,179,648
// vertices, bit-packed or with a packed mirror)?
bool graph_lds_fits(const ChainDesc &d);

// words of a packed mirror the LDS-staged kernel can hold (n <= 32 * this)
int graph_lds_max_words();

// mirror[idx] = spin[idx] packed, for every int8 chain with a mirror
hipError_t launch_pack_mirror(const ChainDesc *dev_descs, const ChainDesc *host_descs, int nchains, int idx,
                              hipStream_t stream);

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `stream` and return the hipError_t of the launch.

// random / constant initial state of one chain into buffer `dst`
hipError_t launch_init(const ChainDesc &d, void *dst, int mode, hipStream_t stream);

// One half-step of every chain in dev_descs[0..nchains) (device array, all of
// one kind and format; host_descs mirrors it for launch shapes).  The
// half-step index is s = dstate[0] + s_add if dstate is non-null, else s_add;
// `even` must equal (s % 2 == 0).  Chain configurations at half-step s live in
// spin[s & 1].  With log_on, the observables of a configuration read at an
// even s are accumulated into log slot (s - base) / 2, base = dstate[1] or
// s_log0.
hipError_t launch_half_step_grid(const ChainDesc *dev_descs, const ChainDesc *host_descs,
                                 int nchains, const uint32_t *dstate, uint32_t s_add,
                                 uint32_t s_log0, int log_on, bool even, int block,
                                 hipStream_t stream);

// d[0] = a, d[1] = b (two uint32 words)
hipError_t launch_set_state(uint32_t *d, uint32_t a, uint32_t b, hipStream_t stream);

// dstate[0] += by
hipError_t launch_advance(uint32_t *dstate, uint32_t by, hipStream_t stream);

// observables of spin[idx] of every chain into log slot `slot`
hipError_t launch_observe(const ChainDesc *dev_descs, const ChainDesc *host_descs, int nchains,
                          int idx, int slot, hipStream_t stream);

// zero `count` int64 at p
hipError_t launch_fill_i64(int64_t *p, int64_t count, int64_t value, hipStream_t stream);

// persistent batch: run n_full full steps of every chain, starting at
// half-step s0 (when sp is not null, s0 = sp[0] and n_full = sp[1], read on
// the device: one captured HIP graph serves every call) with the
// configuration in spin[0]; chains are taken from a device queue in the order
// given by `order`; counter must be zero on entry.  Writes the final
// configuration back into spin[0].
hipError_t launch_persistent(const ChainDesc *dev_descs, int nchains, const int32_t *order,
                             int32_t *counter, uint32_t s0, const uint32_t *sp, int64_t n_full,
                             int record, int track, int block, int grid, hipStream_t stream);

// can chain d run in the persistent kernel?
bool persistent_fits(const ChainDesc &d);

// workgroups of the persistent kernel resident on one compute unit at once
int persistent_resident_blocks();

// record the thread-local message returned by shaken_last_error()
shaken_status set_error(shaken_status s, const char *msg);

}  // namespace shaken
