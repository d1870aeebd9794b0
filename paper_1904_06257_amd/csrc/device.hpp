// Device helpers shared by the HIP kernels of libshaken (gfx950): Philox,
// bit-plane helpers, reductions and the 32-site bit-packed update.
#pragma once

#include "shaken_internal.hpp"

namespace shaken {

// words in the global address space
typedef __attribute__((address_space(1))) uint32_t gmem_u32;
typedef __attribute__((address_space(1))) char gmem_char;

// word idx of a global array through a 32-bit byte offset (idx < 2^30), so
// that the access takes the scalar-base form
__device__ __forceinline__ gmem_u32 &gword(gmem_u32 *base, uint32_t idx) {
    return *(gmem_u32 *)((gmem_char *)base + (idx << 2));
}
__device__ __forceinline__ uint32_t gload(const gmem_u32 *base, uint32_t idx) {
    return *(const gmem_u32 *)((const gmem_char *)base + (idx << 2));
}

// ------------------------------------------------------------------ Philox

struct U4 {
    uint32_t x, y, z, w;
};

// Philox4x32 with ten rounds (Salmon et al., SC'11).  The three-input xors
// are single v_bitop3_b32 instructions (truth table 0x96).
__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t a = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t b = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), c3, k1, 0x96);
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// The same call when c1, c2, c3 and the key are the same in every lane and
// only c0 varies (the graph kernels' (vertex group, s, replica, stream)):
// what rounds one and two compute from the shared words alone -- round one's
// product of c2, round two's product of the new c0 -- is done once per call
// site with plain integer arithmetic, which the compiler keeps on the scalar
// unit (philox10_shared), and each lane finishes from its c0 (philox10_c0):
// two products and three xors for the first two rounds instead of four and
// four.  philox10_c0(c0, philox10_shared(c1, c2, c3, k0, k1), k0, k1) equals
// philox10(c0, c1, c2, c3, k0, k1).
struct PhiloxShared {
    uint32_t x3;  // c3 ^ k1: round one's xor into the new c2
    uint32_t x0;  // round one's low c2 product ^ round two's k0: into round two's new c0
    uint32_t x2;  // high half of round two's c0 product ^ its k1: into round two's new c2
    uint32_t c3;  // round two's new c3 (low half of that product)
};

__device__ __forceinline__ PhiloxShared philox10_shared(uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                        uint32_t k1) {
    const uint64_t b0 = (uint64_t)c2 * 0xCD9E8D57u;
    const uint32_t c0r1 = (uint32_t)(b0 >> 32) ^ c1 ^ k0;
    const uint64_t a1 = (uint64_t)c0r1 * 0xD2511F53u;
    PhiloxShared p;
    p.x3 = c3 ^ k1;
    p.x0 = (uint32_t)b0 ^ (k0 + 0x9E3779B9u);
    p.x2 = (uint32_t)(a1 >> 32) ^ (k1 + 0xBB67AE85u);
    p.c3 = (uint32_t)a1;
    return p;
}

__device__ __forceinline__ U4 philox10_c0(uint32_t c0, const PhiloxShared &p, uint32_t k0, uint32_t k1) {
    const uint64_t a0 = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t b1 = (uint64_t)((uint32_t)(a0 >> 32) ^ p.x3) * 0xCD9E8D57u;
    uint32_t x0 = (uint32_t)(b1 >> 32) ^ p.x0, x1 = (uint32_t)b1, x2 = (uint32_t)a0 ^ p.x2, x3 = p.c3;
    k0 += 2u * 0x9E3779B9u;
    k1 += 2u * 0xBB67AE85u;
#pragma unroll
    for (int i = 2; i < 10; ++i) {
        const uint64_t a = (uint64_t)x0 * 0xD2511F53u;
        const uint64_t b = (uint64_t)x2 * 0xCD9E8D57u;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), x1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), x3, k1, 0x96);
        x1 = (uint32_t)b;
        x3 = (uint32_t)a;
        x0 = n0;
        x2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{x0, x1, x2, x3};
}

// The same call with words x and z of the result xored with a per-lane word
// v: the last round's key xor takes (k ^ v) in their place, so the xor costs
// nothing there.  kx0, kx1 = the tenth round's keys xor v.  SH: c2 is the
// same in every lane, so round two's c1 (the low half of round one's c2
// product) is too, and c1 ^ k0 there is one scalar operand (one instruction
// per call fewer; faster in the triangular and persistent kernels, slower
// in the square-lattice grid kernel, which keeps the plain form).
template <bool SH = false>
__device__ __forceinline__ U4 philox10_xv(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1, uint32_t kx0, uint32_t kx1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t a = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t b = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t n0 = (SH && i == 1)
                                ? (uint32_t)(b >> 32) ^ (c1 ^ k0)
                                : __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), c1, i == 9 ? kx0 : k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), c3, i == 9 ? kx1 : k1, 0x96);
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t bfi(uint32_t m, uint32_t x, uint32_t y) {
    return (m & x) | (~m & y);
}

// all-ones if bit `sh` of v is set, else zero
__device__ __forceinline__ uint32_t bitmask(uint32_t v, int sh) {
    return 0u - ((v >> sh) & 1u);
}

// ------------------------------------------------------------ reductions

// Sum over the 64 lanes, returned in every lane: prefix sums within each
// row of 16 lanes by row shifts, the row totals carried by the row
// broadcasts of lanes 15 and 31, lane 63's total read out.  All DPP (VALU);
// lane shuffles would be six dependent LDS round trips.
__device__ __forceinline__ int wave_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
    return __builtin_amdgcn_readlane(v, 63);
}

// line of log slot `slot` that block `blk` adds into
__device__ __forceinline__ int64_t *log_part(const ChainDesc &d, int slot, int blk) {
    return d.log + (int64_t)slot * d.log_stride + (int64_t)(blk & (kLogParts - 1)) * d.log_line;
}

// block-level sum of two ints into log[0] and log[1] (one atomic per block)
__device__ __forceinline__ void block_accumulate2(int e, int p, int64_t *log) {
    __shared__ int sh_e[16], sh_p[16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    e = wave_sum(e);
    p = wave_sum(p);
    if (lane == 0) {
        sh_e[wv] = e;
        sh_p[wv] = p;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long se = 0, sp = 0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) {
            se += sh_e[i];
            sp += sh_p[i];
        }
        if (se) atomicAdd((unsigned long long *)&log[0], (unsigned long long)se);
        if (sp) atomicAdd((unsigned long long *)&log[1], (unsigned long long)sp);
    }
}

// XCD-aware block order: the hardware deals consecutive workgroups round-robin
// over the 8 XCDs; give each XCD a contiguous run of tiles so that rows shared
// as halos stay in one L2.
__device__ __forceinline__ int xcd_block(int bx, int nb) {
    if ((nb & 7) != 0) return bx;
    return (bx & 7) * (nb >> 3) + (bx >> 3);
}

// ------------------------------------------------------ bit-packed torus

// Truth table of a three-input bit function for v_bitop3_b32 (bit a*4 + b*2 + c).
template <typename F>
constexpr int bitop3_table(F f) {
    int t = 0;
    for (int i = 0; i < 8; ++i)
        if (f((i >> 2) & 1, (i >> 1) & 1, i & 1)) t |= 1 << i;
    return t;
}
constexpr int kT_nor_and = bitop3_table([](int a, int b, int c) { return !a && !b && c; });
constexpr int kT_and_or = bitop3_table([](int a, int b, int c) { return (a && b) || c; });
constexpr int kT_xor3 = bitop3_table([](int a, int b, int c) { return a ^ b ^ c; });
constexpr int kT_or_and = bitop3_table([](int a, int b, int c) { return a || (b && c); });
constexpr int kT_bfi = bitop3_table([](int a, int b, int c) { return a ? b : c; });
constexpr int kT_xor_and = bitop3_table([](int a, int b, int c) { return (a ^ b) & c; });

// The eight level masks of the folded table's rest class (levels 0..7) in
// vector registers: with one of the three masks of a level there, the class
// select takes two instructions (each may read only one scalar operand).  A
// lane permute of the uniform value makes it a per-lane value.
struct BpRestMasks {
    uint32_t m[8];
};

__device__ __forceinline__ BpRestMasks bp_rest_masks(uint32_t rest) {
    BpRestMasks r;
    const int self = (int)(threadIdx.x & 63u) << 2;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        r.m[k] = (uint32_t)__builtin_amdgcn_ds_bpermute(self, (int)bitmask(rest, 31 - k));
    return r;
}

// Bit-planes of a word for the six-class table: the two neighbours of the
// half (a, b) and the sites themselves (c).  With a uniform coupling a site
// belongs to class j = n_plus + 3c; the sign plane says where h >= 0 (from
// the per-chain mask sgn).
struct BpPlanes {
    uint32_t one, both, c, smask;
};

__device__ __forceinline__ BpPlanes bp_planes(uint32_t a, uint32_t b, uint32_t c, uint32_t sgn) {
    BpPlanes p;
    p.both = a & b;
    p.one = a ^ b;
    // sign of h per class, one scalar operand per instruction: classes with no,
    // one and two +1 neighbours, then the site's own spin picks the row
    uint32_t slo = __builtin_amdgcn_bitop3_b32(p.one, p.both, bitmask(sgn, 0), kT_nor_and);
    slo = __builtin_amdgcn_bitop3_b32(p.one, bitmask(sgn, 1), slo, kT_and_or);
    slo = __builtin_amdgcn_bitop3_b32(p.both, bitmask(sgn, 2), slo, kT_and_or);
    uint32_t shi = __builtin_amdgcn_bitop3_b32(p.one, p.both, bitmask(sgn, 3), kT_nor_and);
    shi = __builtin_amdgcn_bitop3_b32(p.one, bitmask(sgn, 4), shi, kT_and_or);
    shi = __builtin_amdgcn_bitop3_b32(p.both, bitmask(sgn, 5), shi, kT_and_or);
    p.smask = bfi(c, shi, slo);
    p.c = c;
    return p;
}

// MSB-first comparison of the 32 bit-sliced uniforms of RNG word w with the
// thresholds of their classes, level groups [G0, G1) (group g = levels
// 4g..4g+3 = Philox((w, s, rep, g))), stopping once every site is decided.
// und: sites still undecided; res: sites decided with v < t, where v = u with
// the bits flipped where h >= 0 (u < 2^32 - t  <=>  not (~u < t)), so only
// t <= 2^31 is compared.
template <int G0, int G1>
__device__ __forceinline__ void bp_groups(const BpPlanes &p, uint32_t &und, uint32_t &res,
                                          uint32_t w, uint32_t s, uint32_t rep, uint32_t k0,
                                          uint32_t k1, const uint32_t *__restrict__ ts) {
    const uint32_t t0 = ts[0], t1 = ts[1], t2 = ts[2], t3 = ts[3], t4 = ts[4], t5 = ts[5];
#define SHAKEN_LEVEL(K, R)                                                                    \
    {                                                                                         \
        const int sh_ = 31 - (K);                                                             \
        const uint32_t lo_ = bfi(p.both, bitmask(t2, sh_),                                    \
                                 bfi(p.one, bitmask(t1, sh_), bitmask(t0, sh_)));             \
        const uint32_t hi_ = bfi(p.both, bitmask(t5, sh_),                                    \
                                 bfi(p.one, bitmask(t4, sh_), bitmask(t3, sh_)));             \
        const uint32_t t_ = bfi(p.c, hi_, lo_);                                               \
        const uint32_t d_ = __builtin_amdgcn_bitop3_b32((R), p.smask, t_, kT_xor3);          \
        const uint32_t y_ = und & d_; /* decided at this level */                             \
        res = __builtin_amdgcn_bitop3_b32(res, y_, t_, kT_or_and);                            \
        und &= ~d_;                                                                           \
    }
#pragma unroll
    for (int g = G0; g < G1; ++g) {
        const U4 r = philox10(w, s, rep, (uint32_t)g, k0, k1);
        SHAKEN_LEVEL(4 * g + 0, r.x)
        SHAKEN_LEVEL(4 * g + 1, r.y)
        SHAKEN_LEVEL(4 * g + 2, r.z)
        SHAKEN_LEVEL(4 * g + 3, r.w)
        if (und == 0) break;
    }
#undef SHAKEN_LEVEL
}

// ------------------------------------------- folded table (uniform coupling)
// With the thresholds equal in mirror classes j and 5 - j three classes
// remain: `one` (exactly one +1 neighbour: classes 1 and 4), `al` (the
// neighbours agree with the site: 0 and 5) and `rest` (2 and 3).  The host
// keeps this table only where mirror classes also have opposite signs of h
// (a class with T = 2^31 decides alike with either sign), so the flip plane
// is smask = c ^ F(class), F the sign bit of the member whose site is -1.
// F is folded into the class words, tf = t ^ F, and a site compares u with
// y = tf ^ c = t ^ smask: u < T holds exactly when (u ^ smask) < t, whose
// value is t's bit at the most significant level where the two differ, that
// is y's bit at the most significant level where u and y differ (smask when
// all 32 levels agree).
struct FoldT {
    uint32_t one, al, rest;
};

__device__ __forceinline__ FoldT fold_t(const uint32_t *__restrict__ ts, uint32_t sgn) {
    return FoldT{ts[1] ^ bitmask(sgn, 1), ts[0] ^ bitmask(sgn, 0), ts[2] ^ bitmask(sgn, 2)};
}

struct FoldPlanes {
    uint32_t one, al, c;
};

constexpr int kT_al = bitop3_table([](int a, int c, int one) { return a == c && !one; });
// o' = y where u and y differ, else o
constexpr int kT_first = bitop3_table([](int u, int y, int o) { return u != y ? y : o; });
// eq' = eq where u and y agree
constexpr int kT_and_eq = bitop3_table([](int e, int u, int y) { return e && u == y; });
// out' = out, or ~u where newly decided (there y = ~u)
constexpr int kT_or_andn = bitop3_table([](int o, int e, int u) { return o || (e && !u); });

__device__ __forceinline__ FoldPlanes fold_planes(uint32_t a, uint32_t b, uint32_t c) {
    FoldPlanes p;
    p.one = a ^ b;
    p.al = __builtin_amdgcn_bitop3_b32(a, c, p.one, kT_al);
    p.c = c;
    return p;
}

// tf's bit `sh` of each site's class, one scalar operand per instruction
__device__ __forceinline__ uint32_t fold_select(const FoldPlanes &p, const FoldT &ft, int sh) {
    uint32_t x = __builtin_amdgcn_bitop3_b32(p.one, p.al, bitmask(ft.rest, sh), kT_nor_and);
    x = __builtin_amdgcn_bitop3_b32(p.al, bitmask(ft.al, sh), x, kT_and_or);
    return __builtin_amdgcn_bitop3_b32(p.one, bitmask(ft.one, sh), x, kT_and_or);
}

// Class-word selectors of the folded tables: sel(k) is the bit of level k
// (0 = most significant) of each site's class word tf, c() the sites, and
// smask(sgn) the flip plane (needed only where all 32 levels agree).
struct SqSel {  // square lattice, the three class words scalar
    FoldPlanes p;
    FoldT ft;
    __device__ __forceinline__ uint32_t c() const { return p.c; }
    __device__ __forceinline__ uint32_t sel(int k) const { return fold_select(p, ft, 31 - k); }
    __device__ __forceinline__ uint32_t smask(uint32_t sgn) const {
        uint32_t f = __builtin_amdgcn_bitop3_b32(p.one, p.al, bitmask(sgn, 2), kT_nor_and);
        f = __builtin_amdgcn_bitop3_b32(p.al, bitmask(sgn, 0), f, kT_and_or);
        f = __builtin_amdgcn_bitop3_b32(p.one, bitmask(sgn, 1), f, kT_and_or);
        return f ^ p.c;
    }
};

struct SqSelV : SqSel {  // rest-class words of levels 0..7 in vector registers
    const BpRestMasks *rm;
    __device__ __forceinline__ uint32_t sel(int k) const {
        const uint32_t x = __builtin_amdgcn_bitop3_b32(p.al, bitmask(ft.al, 31 - k), rm->m[k], kT_bfi);
        return __builtin_amdgcn_bitop3_b32(p.one, bitmask(ft.one, 31 - k), x, kT_bfi);
    }
};

// Levels 0..7 (groups 0 and 1) least significant first: afterwards o holds
// y's bit at the most significant differing level of every site whose top
// eight bits of u and y differ, and eq marks the sites where all eight agree
// (o is not meaningful there).  A level costs the class select, y = tf ^ c
// and one instruction each for o and eq; the MSB-first form needs one more
// (decided sites, result, undecided sites).
//
// The levels run on x = u ^ c against tf: u and y differ where x and tf do,
// and the state kept is o ^ c, whose update is then `tf where x != tf`.  Two
// of the four words of each Philox call come out already xored with c.
template <bool SH = false, class S>
__device__ __forceinline__ void fold_top8(const S &sl, uint32_t &o, uint32_t &eq, uint32_t w, uint32_t s,
                                          uint32_t rep, uint32_t k0, uint32_t k1) {
#define SHAKEN_FLEVEL(K, X)                                                                       \
    {                                                                                             \
        const uint32_t x_ = (X);                                                                  \
        const uint32_t t_ = sl.sel(K);                                                            \
        oc = __builtin_amdgcn_bitop3_b32(x_, t_, oc, kT_first);                                   \
        eq = __builtin_amdgcn_bitop3_b32(eq, x_, t_, kT_and_eq);                                  \
    }
    const uint32_t c = sl.c();
    const uint32_t kx0 = (k0 + 9u * 0x9E3779B9u) ^ c, kx1 = (k1 + 9u * 0xBB67AE85u) ^ c;
    uint32_t oc = 0;
    const U4 r1 = philox10_xv<SH>(w, s, rep, 1u, k0, k1, kx0, kx1);
    SHAKEN_FLEVEL(7, r1.w ^ c)
    SHAKEN_FLEVEL(6, r1.z)
    SHAKEN_FLEVEL(5, r1.y ^ c)
    SHAKEN_FLEVEL(4, r1.x)
    const U4 r0 = philox10_xv<SH>(w, s, rep, 0u, k0, k1, kx0, kx1);
    SHAKEN_FLEVEL(3, r0.w ^ c)
    SHAKEN_FLEVEL(2, r0.z)
    SHAKEN_FLEVEL(1, r0.y ^ c)
    SHAKEN_FLEVEL(0, r0.x)
#undef SHAKEN_FLEVEL
    o = oc ^ c;
}

// Levels of groups [G0, G1) most significant first for the sites in und;
// out collects the new spins of the sites decided.
template <class S, int G0, int G1>
__device__ __forceinline__ void fold_groups(const S &sl, uint32_t &und, uint32_t &out, uint32_t w,
                                            uint32_t s, uint32_t rep, uint32_t k0, uint32_t k1) {
#define SHAKEN_GLEVEL(K, R)                                                                       \
    {                                                                                             \
        const uint32_t d_ = __builtin_amdgcn_bitop3_b32((R), sl.c(), sl.sel(K), kT_xor3); /* u != y */ \
        const uint32_t e_ = und & d_;                                                             \
        out = __builtin_amdgcn_bitop3_b32(out, e_, (R), kT_or_andn);                              \
        und &= ~d_;                                                                               \
    }
#pragma unroll
    for (int g = G0; g < G1; ++g) {
        const U4 r = philox10(w, s, rep, (uint32_t)g, k0, k1);
        SHAKEN_GLEVEL(4 * g + 0, r.x)
        SHAKEN_GLEVEL(4 * g + 1, r.y)
        SHAKEN_GLEVEL(4 * g + 2, r.z)
        SHAKEN_GLEVEL(4 * g + 3, r.w)
        if (und == 0) break;
    }
#undef SHAKEN_GLEVEL
}

// Finish a word on a folded table from level group G0 on: und the sites
// still undecided, out the new spins of the others.
template <class S, int G0>
__device__ __forceinline__ uint32_t fold_finish(const S &sl, uint32_t und, uint32_t out, uint32_t vm,
                                                uint32_t w, uint32_t s, uint32_t rep, uint32_t k0,
                                                uint32_t k1, uint32_t sgn) {
    fold_groups<S, G0, 8>(sl, und, out, w, s, rep, k0, k1);
    if (und) out |= und & sl.smask(sgn);
    return out & vm;
}

// Groups 3..7 of one word by a quad of lanes (qlane = the lane's place in
// it, 0..3; all four lanes active, the same word in each): lane i evaluates
// level group 3 + i for every site in und at once, and the quad's first lane
// combines the four -- a site takes the outcome of the lowest group that
// decides it --, finishes the rare sites still undecided after group 6 and
// passes the word's new spins (masked by vm) to store.  One group's latency
// instead of a chain of five.
template <class S, class F>
__device__ __forceinline__ void fold_quad_finish(const S &sl, uint32_t und, uint32_t res, int qlane,
                                                 uint32_t vm, uint32_t w, uint32_t s, uint32_t rep,
                                                 uint32_t k0, uint32_t k1, uint32_t sgn, F &&store) {
    const int g = 3 + qlane;
    const U4 r = philox10(w, s, rep, (uint32_t)g, k0, k1);
    const uint32_t rr[4] = {r.x, r.y, r.z, r.w};
    uint32_t ug = und, og = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t dd = __builtin_amdgcn_bitop3_b32(rr[k], sl.c(), sl.sel(4 * g + k), kT_xor3);  // u != y
        og = __builtin_amdgcn_bitop3_b32(og, ug & dd, rr[k], kT_or_andn);
        ug &= ~dd;
    }
    const uint32_t dg = und & ~ug;  // decided within group g
    // lanes 1..3 of the quad (groups 4..6) to lane 0
    const uint32_t d4 = (uint32_t)__builtin_amdgcn_mov_dpp((int)dg, 0x55, 0xF, 0xF, false);
    const uint32_t o4 = (uint32_t)__builtin_amdgcn_mov_dpp((int)og, 0x55, 0xF, 0xF, false);
    const uint32_t d5 = (uint32_t)__builtin_amdgcn_mov_dpp((int)dg, 0xAA, 0xF, 0xF, false);
    const uint32_t o5 = (uint32_t)__builtin_amdgcn_mov_dpp((int)og, 0xAA, 0xF, 0xF, false);
    const uint32_t d6 = (uint32_t)__builtin_amdgcn_mov_dpp((int)dg, 0xFF, 0xF, 0xF, false);
    const uint32_t o6 = (uint32_t)__builtin_amdgcn_mov_dpp((int)og, 0xFF, 0xF, 0xF, false);
    if (qlane == 0) {
        const uint32_t d34 = dg | d4, d345 = d34 | d5;
        res |= og | (o4 & ~dg) | (o5 & ~d34) | (o6 & ~d345);
        const uint32_t left = und & ~(d345 | d6);
        if (left) res = fold_finish<S, 7>(sl, left, res, vm, w, s, rep, k0, k1, sgn);
        store(res & vm);
    }
}

// a whole word on a folded table
template <class S>
__device__ __forceinline__ uint32_t fold_word(const S &sl, uint32_t vm, uint32_t w, uint32_t s, uint32_t rep,
                                              uint32_t k0, uint32_t k1, uint32_t sgn) {
    uint32_t o = 0, eq = ~0u;
    fold_top8(sl, o, eq, w, s, rep, k0, k1);
    const uint32_t und = eq & vm;
    if (und == 0) return o & vm;
    return fold_finish<S, 2>(sl, und, o & ~eq, vm, w, s, rep, k0, k1, sgn);
}

// New word of 32 sites: a, b neighbour planes of the half, c the sites, vm the
// valid bits, w the RNG word, s the half-step index.
template <bool FOLD3>
__device__ __forceinline__ uint32_t bp_word(uint32_t a, uint32_t b, uint32_t c, uint32_t vm,
                                            uint32_t w, uint32_t s, uint32_t rep, uint32_t k0,
                                            uint32_t k1, const uint32_t *__restrict__ ts,
                                            uint32_t sgn) {
    if constexpr (FOLD3) {
        return fold_word(SqSel{fold_planes(a, b, c), fold_t(ts, sgn)}, vm, w, s, rep, k0, k1, sgn);
    } else {
        const BpPlanes p = bp_planes(a, b, c, sgn);
        uint32_t und = vm, res = 0;
        bp_groups<0, 8>(p, und, res, w, s, rep, k0, k1, ts);
        return (res ^ p.smask) & vm;
    }
}

// ------------------------------------------ bit-packed triangular lattice
// Three neighbour planes a, b, e per half (section 4: three "left"
// neighbours in half-step 1, three "right" ones in half-step 2); a site
// belongs to class j = n_plus + 4c (n_plus = number of +1 neighbours, c =
// the site), eight classes.  s1 = a ^ b ^ e (n_plus odd) and s2 = maj(a, b, e)
// (n_plus >= 2) code n_plus = s1 + 2 s2.  When the thresholds depend on |h|
// only (lambda = 0), classes (n, c) and (3 - n, 1 - c) share one: the class is
// then the number k of neighbours that agree with the site, coded the same
// way over the agreement planes (TriSel below).
struct TriPlanes {
    uint32_t s1, s2, c, smask;
};

__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t e) {
    return (a & b) | (a & e) | (b & e);
}

// eight-class planes: n_plus coded by s1, s2; the flip plane from sgn
__device__ __forceinline__ TriPlanes tri_planes(uint32_t a, uint32_t b, uint32_t e, uint32_t c,
                                                uint32_t sgn) {
    TriPlanes p;
    p.c = c;
    p.s1 = a ^ b ^ e;
    p.s2 = maj3(a, b, e);
    const uint32_t slo = bfi(p.s2, bfi(p.s1, bitmask(sgn, 3), bitmask(sgn, 2)),
                             bfi(p.s1, bitmask(sgn, 1), bitmask(sgn, 0)));
    const uint32_t shi = bfi(p.s2, bfi(p.s1, bitmask(sgn, 7), bitmask(sgn, 6)),
                             bfi(p.s1, bitmask(sgn, 5), bitmask(sgn, 4)));
    p.smask = bfi(c, shi, slo);
    return p;
}

// Folded table in the flipped domain (same contract as the square lattice's
// SqSel): agreement class k holds the mirror classes (3 - k, -1) and (k, +1)
// of the same t; the host keeps the table only where their signs are
// opposite, so the flip plane is c ^ F_k with F_k the sign of (3 - k, -1),
// bit 3 - k of sgn, and the class words are tf_k = t_{4+k} ^ F_k.
struct TriSel {
    uint32_t s1, s2, k1, k2, k3, cc;
    uint32_t tf[4];
    __device__ __forceinline__ uint32_t c() const { return cc; }
    __device__ __forceinline__ uint32_t sel(int k) const {
        const int sh = 31 - k;
        uint32_t x = __builtin_amdgcn_bitop3_b32(s1, s2, bitmask(tf[0], sh), kT_nor_and);
        x = __builtin_amdgcn_bitop3_b32(k1, bitmask(tf[1], sh), x, kT_and_or);
        x = __builtin_amdgcn_bitop3_b32(k2, bitmask(tf[2], sh), x, kT_and_or);
        return __builtin_amdgcn_bitop3_b32(k3, bitmask(tf[3], sh), x, kT_and_or);
    }
    __device__ __forceinline__ uint32_t smask(uint32_t sgn) const {
        uint32_t f = __builtin_amdgcn_bitop3_b32(s1, s2, bitmask(sgn, 3), kT_nor_and);
        f = __builtin_amdgcn_bitop3_b32(k1, bitmask(sgn, 2), f, kT_and_or);
        f = __builtin_amdgcn_bitop3_b32(k2, bitmask(sgn, 1), f, kT_and_or);
        f = __builtin_amdgcn_bitop3_b32(k3, bitmask(sgn, 0), f, kT_and_or);
        return f ^ cc;
    }
};

constexpr int kT_xnor = bitop3_table([](int a, int b, int) { return a == b; });

// the agreement planes of a word: s1 = odd agreement count, s2 = at least
// two; n_plus's parity and majority xnor the site (three complements of
// a ^ c, b ^ c, e ^ c)
__device__ __forceinline__ TriSel tri_sel(uint32_t a, uint32_t b, uint32_t e, uint32_t c,
                                          const uint32_t *__restrict__ ts, uint32_t sgn) {
    TriSel t;
    t.cc = c;
    t.s1 = ~(a ^ b ^ e ^ c);
    t.s2 = __builtin_amdgcn_bitop3_b32(maj3(a, b, e), c, 0u, kT_xnor);
    t.k1 = t.s1 & ~t.s2;
    t.k2 = ~t.s1 & t.s2;
    t.k3 = t.s1 & t.s2;
#pragma unroll
    for (int k = 0; k < 4; ++k) t.tf[k] = ts[4 + k] ^ bitmask(sgn, 3 - k);
    return t;
}

// MSB-first compare of the 32 bit-sliced uniforms with the eight class
// thresholds, level groups [G0, G1); same contract as bp_groups.
template <int G0, int G1>
__device__ __forceinline__ void tri_groups(const TriPlanes &p, uint32_t &und, uint32_t &res,
                                           uint32_t w, uint32_t s, uint32_t rep, uint32_t k0,
                                           uint32_t k1, const uint32_t *__restrict__ ts) {
    const uint32_t t0 = ts[0], t1 = ts[1], t2 = ts[2], t3 = ts[3];
    const uint32_t t4 = ts[4], t5 = ts[5], t6 = ts[6], t7 = ts[7];
#define SHAKEN_TLEVEL(K, R)                                                                       \
    {                                                                                             \
        const int sh_ = 31 - (K);                                                                 \
        const uint32_t lo_ = bfi(p.s2, bfi(p.s1, bitmask(t3, sh_), bitmask(t2, sh_)),             \
                                 bfi(p.s1, bitmask(t1, sh_), bitmask(t0, sh_)));                  \
        const uint32_t hi_ = bfi(p.s2, bfi(p.s1, bitmask(t7, sh_), bitmask(t6, sh_)),             \
                                 bfi(p.s1, bitmask(t5, sh_), bitmask(t4, sh_)));                  \
        const uint32_t t_ = bfi(p.c, hi_, lo_);                                                   \
        const uint32_t d_ = __builtin_amdgcn_bitop3_b32((R), p.smask, t_, kT_xor3);              \
        const uint32_t y_ = und & d_; /* decided at this level */                                 \
        res = __builtin_amdgcn_bitop3_b32(res, y_, t_, kT_or_and);                                \
        und &= ~d_;                                                                               \
    }
#pragma unroll
    for (int g = G0; g < G1; ++g) {
        const U4 r = philox10(w, s, rep, (uint32_t)g, k0, k1);
        SHAKEN_TLEVEL(4 * g + 0, r.x)
        SHAKEN_TLEVEL(4 * g + 1, r.y)
        SHAKEN_TLEVEL(4 * g + 2, r.z)
        SHAKEN_TLEVEL(4 * g + 3, r.w)
        if (und == 0) break;
    }
#undef SHAKEN_TLEVEL
}

// new word of 32 triangular-lattice sites (neighbour planes a, b, e)
template <bool FOLD>
__device__ __forceinline__ uint32_t tri_word(uint32_t a, uint32_t b, uint32_t e, uint32_t c,
                                             uint32_t vm, uint32_t w, uint32_t s, uint32_t rep,
                                             uint32_t k0, uint32_t k1,
                                             const uint32_t *__restrict__ ts, uint32_t sgn) {
    if constexpr (FOLD) {
        return fold_word(tri_sel(a, b, e, c, ts, sgn), vm, w, s, rep, k0, k1, sgn);
    } else {
        const TriPlanes p = tri_planes(a, b, e, c, sgn);
        uint32_t und = vm, res = 0;
        tri_groups<0, 8>(p, und, res, w, s, rep, k0, k1, ts);
        return (res ^ p.smask) & vm;
    }
}

// +-J torus: flip the neighbour planes a (vertical) and b (horizontal) of
// word (r, wd) where the coupling of the edge to that neighbour is negative.
// dl (phase 0): the edges come from the row below, (x_down, x), and from the
// left, (x_left, x), so the right-edge plane is shifted like b; ur (phase 1):
// the edges (x, x_up) and (x, x_right) belong to the word itself.
__device__ __forceinline__ void bp_jflip(const uint32_t *__restrict__ jn, int L, int W, int r,
                                         int wd, int phase, uint32_t &a, uint32_t &b) {
    const uint32_t *__restrict__ up = jn;
    const uint32_t *__restrict__ rt = jn + (size_t)L * W;
    if (phase == 0) {
        // (the indices selected first, each word read unconditionally)
        const int rd = (r == 0) ? L - 1 : r - 1;
        a ^= up[rd * W + wd];
        const uint32_t cw = rt[r * W + (wd > 0 ? wd - 1 : W - 1)];
        b ^= (rt[r * W + wd] << 1) | ((cw >> (wd > 0 ? 31 : ((L - 1) & 31))) & 1u);
    } else {
        a ^= up[r * W + wd];
        b ^= rt[r * W + wd];
    }
}

// sign (+1 / -1) of the coupling of torus site (r, c) to its up (plane 0) or
// right (plane 1) neighbour; +1 without sign planes
__device__ __forceinline__ int torus_jsign(const uint32_t *__restrict__ jn, int L, int W, int plane,
                                           int r, int c) {
    if (!jn) return 1;
    return ((jn[(size_t)plane * L * W + r * W + (c >> 5)] >> (c & 31)) & 1u) ? -1 : 1;
}

// frozen set B: word w of the frozen bit-plane (0 when B is empty)
__device__ __forceinline__ uint32_t frozen_word(const ChainDesc &d, int w) {
    return d.frozen ? d.frozen[w] : 0u;
}

// frozen bits of the four vertices v0..v0+3 of a graph (bit j = v0 + j)
__device__ __forceinline__ uint32_t frozen4(const ChainDesc &d, int v0) {
    return d.frozen ? ((d.frozen[v0 >> 5] >> (v0 & 31)) & 0xFu) : 0u;
}

__device__ __forceinline__ uint32_t bp_valid(int L, int W, int wd) {
    const int rem = L & 31;
    return (wd == W - 1 && rem) ? ((1u << rem) - 1u) : 0xFFFFFFFFu;
}

}  // namespace shaken
