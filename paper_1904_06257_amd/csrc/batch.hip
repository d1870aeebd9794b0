// Persistent batch kernel of libshaken (gfx950).
//
// Many independent shaken-dynamics chains (arXiv:1904.06257; each chain is the
// paper's dynamics with its own graph, beta, q and seed) in one launch.  A
// workgroup takes a whole chain from a device queue (longest first), copies
// its configuration into LDS as bits, runs every half-step of the call with
// workgroup barriers only, and writes the configuration back.  Both halves of
// the double buffer live in LDS (2 x 2048 words = 16 KiB): tori up to
// 256 x 256 and graphs up to 65536 vertices.  The randomness and thresholds
// are those of the grid kernels, so a chain gives the same trajectory either
// way.  Adjacency (CSR) and the threshold table stay in global memory.
#include "device.hpp"

namespace shaken {

#ifndef SHAKEN_PBLOCK
#define SHAKEN_PBLOCK 1024
#endif
constexpr int kPBlock = SHAKEN_PBLOCK;  // threads per chain
constexpr int kPWords = 2048;
constexpr int kPClasses = 16;
constexpr int kPLut = 512;  // threshold entries kept in LDS

bool persistent_fits(const ChainDesc &d) {
    if (d.kind == KIND_TORUS) return d.format == FMT_BITPACKED && d.L * d.W <= kPWords;
    // the ELL and packed paths read the threshold table from LDS only
    const bool lut_lds = (2 * d.smax + 1) * 2 * d.ncls <= kPLut;
    return d.n <= 32 * kPWords && d.ncls <= kPClasses && (lut_lds || (!d.ell && !d.pell));
}

// Sum e and p over the workgroup; the totals are valid in thread 0.
__device__ __forceinline__ void block_sum2(int &e, int &p, int *sh) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    e = wave_sum(e);
    p = wave_sum(p);
    if (lane == 0) {
        sh[2 * wv] = e;
        sh[2 * wv + 1] = p;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kPBlock / 64; ++i) {
            e += sh[2 * i];
            p += sh[2 * i + 1];
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------- torus

// One half-step (or, with dst == nullptr, only the observables of src) of an
// L x L bit-packed torus held in LDS.
// Observables of one configuration, valid in thread 0: E_J and the +1 count of
// every field class.
struct Obs {
    int e;
    int plus[kPClasses];
};

// Row of word w: w / W as a multiply-high by the descriptor's reciprocal
// wdiv (W = 1: the row is w itself).
__device__ __forceinline__ int torus_row(int W, uint32_t wdiv, int w) {
    return W == 1 ? w : (int)__umulhi((uint32_t)w, wdiv);
}

// Neighbour planes of word w (row r, word column wd) read in half `phase`
// (0 = dl, 1 = ur): a the vertical neighbours, b the horizontal ones, e
// (triangular lattice) the diagonal ones, flipped by the coupling signs where
// there are any.  Every index is selected first and each word then read
// unconditionally (a read inside a select becomes a branch and a wait).
template <bool TRI, bool EXT>
__device__ __forceinline__ void lds_planes(const ChainDesc &d, const uint32_t *src, const uint32_t *jn, int w,
                                           int r, int wd, int phase, uint32_t &a, uint32_t &b, uint32_t &e) {
    const int L = d.L, W = d.W;
    const uint32_t own = src[w];
    const int lastbits = (L - 1) & 31;
    e = 0;
    if (phase == 0) {
        // down and left neighbours (the in-half); triangular: down-left too.
        // The left carry is bit 31 of the word to the left, or at the row's
        // start the last valid bit of the row's last word
        const int ia = (r == 0 ? L - 1 : r - 1) * W + wd;
        const int sh = wd > 0 ? 31 : lastbits;
        a = src[ia];
        const uint32_t sw = src[wd > 0 ? w - 1 : w + W - 1];
        b = (own << 1) | ((sw >> sh) & 1u);
        if (TRI) {
            const uint32_t as = src[wd > 0 ? ia - 1 : ia + W - 1];
            e = (a << 1) | ((as >> sh) & 1u);
        }
    } else {
        // up and right: the right carry is bit 0 of the word to the right
        // (to bit 31), or at the row's end bit 0 of the row's first word (to
        // the last valid bit)
        const int ia = (r == L - 1 ? 0 : r + 1) * W + wd;
        const int sh = wd < W - 1 ? 31 : lastbits;
        a = src[ia];
        const uint32_t sw = src[wd < W - 1 ? w + 1 : w - wd];
        b = (own >> 1) | ((sw & 1u) << sh);
        if (TRI) {
            const uint32_t as = src[wd < W - 1 ? ia + 1 : ia - wd];
            e = (a >> 1) | ((as & 1u) << sh);
        }
    }
    if (EXT && !TRI && jn) bp_jflip(jn, L, W, r, wd, phase, a, b);
}

// Words of a torus half-step whose top eight levels left sites undecided,
// finished after the pass over all words by the whole workgroup, so that the
// rare deeper levels run in a few wavefronts instead of in every one.
constexpr int kPTail = 512;
struct TailQ {
    int n;
    uint32_t w[kPTail], und[kPTail], out[kPTail];
    uint32_t a[kPTail], b[kPTail], e[kPTail];  // neighbour planes (no coupling-sign reads in the tail)
};

// One half-step (or, with dst == nullptr, only the observables of src) of an
// L x L bit-packed torus held in LDS.
template <bool FOLD3, bool TRI, bool EXT>
__device__ __forceinline__ void torus_lds_half(const ChainDesc &d, const uint32_t *src, uint32_t *dst, uint32_t s,
                                               bool obs, int *sh_red, Obs *o, TailQ *tq, const uint32_t *jn) {
    const int L = d.L, W = d.W, nw = L * W;
    const uint32_t wdiv = d.wdiv;
    const int phase = (int)(s & 1u) ^ d.rev;  // half read: 0 = dl, 1 = ur
    const uint32_t k0 = (uint32_t)d.seed, k1 = (uint32_t)(d.seed >> 32);
    int e_acc = 0, p_acc = 0;
    for (int w = threadIdx.x; w < nw; w += kPBlock) {
        const uint32_t own = src[w];
        const int r = torus_row(W, wdiv, w), wd = w - __mul24(r, W);
        const uint32_t vm = bp_valid(L, W, wd);
        uint32_t a, b, e;
        if (obs) {
            lds_planes<TRI, EXT>(d, src, jn, w, r, wd, 0, a, b, e);
            e_acc += d.J * (2 * __popc(vm) - 2 * __popc((own ^ a) & vm) - 2 * __popc((own ^ b) & vm));
            if (TRI) e_acc += d.J * (__popc(vm) - 2 * __popc((own ^ e) & vm));
            p_acc += __popc(own & vm);
        }
        if (!dst) continue;
        if (!obs || phase == 1) lds_planes<TRI, EXT>(d, src, jn, w, r, wd, phase, a, b, e);
        uint32_t nw_bits;
        if constexpr (FOLD3) {
            uint32_t ob = 0, eq = ~0u;
            if constexpr (TRI)
                fold_top8<true>(tri_sel(a, b, e, own, d.tsmall, d.sgn), ob, eq, (uint32_t)w, s, d.replica, k0, k1);
            else
                fold_top8<true>(SqSel{fold_planes(a, b, own), fold_t(d.tsmall, d.sgn)}, ob, eq, (uint32_t)w, s,
                                d.replica, k0, k1);
            const uint32_t und = eq & vm;
            nw_bits = ob & vm;
            if (und != 0) {
                const int qi = atomicAdd(&tq->n, 1);
                if (qi < kPTail) {
                    tq->w[qi] = (uint32_t)w;
                    tq->und[qi] = und;
                    tq->out[qi] = ob & ~eq;
                    tq->a[qi] = a;
                    tq->b[qi] = b;
                    if (TRI) tq->e[qi] = e;
                    continue;
                }
                if constexpr (TRI)
                    nw_bits = fold_finish<TriSel, 2>(tri_sel(a, b, e, own, d.tsmall, d.sgn), und, ob & ~eq, vm,
                                                     (uint32_t)w, s, d.replica, k0, k1, d.sgn);
                else
                    nw_bits = fold_finish<SqSel, 2>(SqSel{fold_planes(a, b, own), fold_t(d.tsmall, d.sgn)}, und,
                                                    ob & ~eq, vm, (uint32_t)w, s, d.replica, k0, k1, d.sgn);
            }
        } else if constexpr (TRI) {
            nw_bits = tri_word<false>(a, b, e, own, vm, (uint32_t)w, s, d.replica, k0, k1, d.tsmall, d.sgn);
        } else {
            nw_bits = bp_word<false>(a, b, own, vm, (uint32_t)w, s, d.replica, k0, k1, d.tsmall, d.sgn);
        }
        dst[w] = EXT ? (nw_bits | frozen_word(d, w)) : nw_bits;
    }
    if (FOLD3 && dst) {
        // the queued words
        __syncthreads();
        const int Q = min(tq->n, kPTail);
        for (int it = threadIdx.x; it < Q; it += kPBlock) {
            const int w = (int)tq->w[it];
            const uint32_t own = src[w];
            const uint32_t vm = bp_valid(L, W, w - __mul24(torus_row(W, wdiv, w), W));
            const uint32_t a = tq->a[it], b = tq->b[it], e = TRI ? tq->e[it] : 0u;
            uint32_t nw_bits;
            if constexpr (TRI)
                nw_bits = fold_finish<TriSel, 2>(tri_sel(a, b, e, own, d.tsmall, d.sgn), tq->und[it], tq->out[it],
                                                 vm, (uint32_t)w, s, d.replica, k0, k1, d.sgn);
            else
                nw_bits = fold_finish<SqSel, 2>(SqSel{fold_planes(a, b, own), fold_t(d.tsmall, d.sgn)},
                                                tq->und[it], tq->out[it], vm, (uint32_t)w, s, d.replica, k0, k1,
                                                d.sgn);
            dst[w] = EXT ? (nw_bits | frozen_word(d, w)) : nw_bits;
        }
        // every lane has read the count: the next half-step starts from zero
        // (the caller's barrier orders the reset before its first append)
        __syncthreads();
        if (threadIdx.x == 0) tq->n = 0;
    }
    if (obs) {
        block_sum2(e_acc, p_acc, sh_red);
        if (threadIdx.x == 0) {
            o->e = e_acc;
            o->plus[0] = p_acc;
        }
    }
}

// Record and / or track one observation (thread 0 holds `o`).  Tracking keeps
// the lowest H in *best_h (thread 0) and copies the configuration `cfg`
// (nwords words of bits) to d.best when it improves.
__device__ void observe_step(const ChainDesc &d, const Obs &o, int64_t *log_slot, bool track,
                             int64_t *best_h, int64_t *last_h, const uint32_t *cfg, int nwords,
                             int *sh_flag) {
    if (threadIdx.x == 0) {
        if (log_slot) {
            log_slot[0] = o.e;
            for (int c = 0; c < d.ncls; ++c) log_slot[1 + c] = o.plus[c];
        }
        int improved = 0;
        if (track) {
            int64_t h = -(int64_t)o.e;
            for (int c = 0; c < d.ncls; ++c)
                h -= (int64_t)d.lam2[c] * (2 * (int64_t)o.plus[c] - d.csize[c]);
            *last_h = h;
            if (h < *best_h) {
                *best_h = h;
                improved = 1;
            }
        }
        *sh_flag = improved;
    }
    __syncthreads();
    if (*sh_flag)
        for (int w = threadIdx.x; w < nwords; w += kPBlock) d.best[w] = cfg[w];
    __syncthreads();
}

// A descriptor reference made wave-uniform and constant-addressed.  Inside a
// called (not inlined) function the compiler cannot see that an argument is
// the same for every lane; without this it loads every field into vector
// registers.
// The builtin returns a signed int: each half goes through uint32_t before it
// is widened, or the low half would be sign-extended into the high one.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}

__device__ __forceinline__ const ChainDesc &uniform_desc(const ChainDesc &d) {
    const uint64_t u = uniform_u64(reinterpret_cast<uint64_t>(&d));
    typedef const __attribute__((address_space(4))) ChainDesc *ConstDescPtr;
    return *(const ChainDesc *)(ConstDescPtr)u;
}

__device__ __forceinline__ int64_t uniform_i64(int64_t x) { return (int64_t)uniform_u64((uint64_t)x); }

template <bool FOLD3, bool TRI, bool EXT>
__device__ __attribute__((noinline)) void run_torus(const ChainDesc &d_arg, uint32_t (*buf)[kPWords], uint32_t s0_arg,
                                                    int64_t n_full_arg, int record_arg, int track_arg,
                                                    int *sh_red, int *sh_flag, Obs &o, TailQ *tq,
                                                    uint32_t *jn_lds) {
    const ChainDesc &d = uniform_desc(d_arg);
    const uint32_t s0 = (uint32_t)__builtin_amdgcn_readfirstlane(s0_arg);
    const int64_t n_full = uniform_i64(n_full_arg);
    const int record = __builtin_amdgcn_readfirstlane(record_arg);
    const int track = __builtin_amdgcn_readfirstlane(track_arg);
    const int nw = d.L * d.W;
    const bool obs = record || track;
    const uint32_t *g = (const uint32_t *)d.spin[0];
    for (int w = threadIdx.x; w < nw; w += kPBlock) buf[0][w] = g[w];
    // +-J: the two coupling-sign planes copied into LDS once for the whole run
    const uint32_t *jn = nullptr;
    if (EXT && !TRI && d.jneg) {
        for (int w = threadIdx.x; w < 2 * nw; w += kPBlock) jn_lds[w] = d.jneg[w];
        jn = jn_lds;
    }
    if (threadIdx.x == 0) tq->n = 0;
    __syncthreads();
    int64_t best_h = INT64_MAX, last_h = 0;
    for (int64_t t = 0; t < n_full; ++t) {
        const uint32_t s = s0 + 2u * (uint32_t)t;
        torus_lds_half<FOLD3, TRI, EXT>(d, buf[0], buf[1], s, obs, sh_red, &o, tq, jn);
        if (obs)
            observe_step(d, o, record ? d.log + t * d.log_stride : nullptr, track, &best_h, &last_h,
                         buf[0], nw, sh_flag);
        __syncthreads();
        torus_lds_half<FOLD3, TRI, EXT>(d, buf[1], buf[0], s + 1u, false, sh_red, nullptr, tq, jn);
        __syncthreads();
    }
    if (obs) {
        torus_lds_half<FOLD3, TRI, EXT>(d, buf[0], nullptr, s0, true, sh_red, &o, tq, jn);
        observe_step(d, o, record ? d.log + n_full * d.log_stride : nullptr, track, &best_h, &last_h,
                     buf[0], nw, sh_flag);
        if (track && threadIdx.x == 0) {
            d.track[0] = last_h;
            d.track[1] = best_h;
        }
    }
    uint32_t *go = (uint32_t *)d.spin[0];
    for (int w = threadIdx.x; w < nw; w += kPBlock) go[w] = buf[0][w];
}

// ------------------------------------------------------------------- graph

__device__ __forceinline__ int lds_spin(const uint32_t *bits, int v) {
    return ((bits[v >> 5] >> (v & 31)) & 1u) ? 1 : -1;
}

// One half-step (or, with dst == nullptr, only the observables of src) of a
// graph whose spins are bits in LDS.  A lane takes 4 consecutive vertices (one
// Philox call); 8 consecutive lanes own one 32-vertex output word and merge
// their 4-bit pieces with lane shuffles.
// Adjacency layouts of a graph chain (one instantiation each, so that every
// path gets its own register allocation).
enum GraphLayout : int { GL_CSR = 0, GL_ELL = 1, GL_PACKED = 2 };

template <int LAY>
__device__ __forceinline__ void graph_lds_half(const ChainDesc &d, const uint32_t *src, uint32_t *dst, uint32_t s,
                               bool obs, int *sh_red, int *sh_plus, Obs *o, const uint64_t *lut) {
    const int n = d.n;
    const int half = dst ? ((int)(s & 1u) ^ d.rev) : 0;  // observables use the in-half
    const int32_t *__restrict__ rp = d.rowptr[half];
    const int32_t *__restrict__ col = d.col[half];
    const int8_t *__restrict__ jw = d.jw[half];
    const int ncls = d.ncls, smax = d.smax;
    const uint32_t k0 = (uint32_t)d.seed, k1 = (uint32_t)(d.seed >> 32);
    const int nq = (n + 3) / 4;
    const int nq_pad = (nq + kPBlock - 1) / kPBlock * kPBlock;
    if (obs) {
        if (threadIdx.x < kPClasses) sh_plus[threadIdx.x] = 0;
        __syncthreads();
    }
    int e_acc = 0;
    // +1 counts per field class: for up to four classes one byte each of a
    // register (a lane counts at most 4 kPWords * 32 / (4 kPBlock) vertices),
    // summed per wavefront and class at the end; else LDS atomics per vertex
    uint32_t pcb = 0;
    static_assert(kPWords * 32 / kPBlock < 256, "a lane's class counts fit a byte");
    const bool pc_reg = ncls <= 4;
    const PhiloxShared ps = philox10_shared(s, d.replica, kGraphStream, k0, k1);
    for (int q4 = threadIdx.x; q4 < nq_pad; q4 += kPBlock) {
        uint32_t bits = 0;
        if (q4 < nq) {
            const int v0 = 4 * q4;
            int S0 = 0, S1 = 0, S2 = 0, S3 = 0;
            int cl[4];
            uint32_t pq[4] = {0u, 0u, 0u, 0u};  // packed: the table index's (p, q) bits
            if constexpr (LAY == GL_PACKED) {
                // packed: one 8-byte record per vertex holds neighbours, the
                // slots of each half, signs and class (two 16-byte loads per
                // thread).  With b_k the spin bits of the neighbours as 0/1,
                // S = sum over the half's slots of J_k (2 b_k - 1)
                //   = 2 popc((b ^ neg) & sel) - popc(sel).
                const uint4 a = *(const uint4 *)(d.pell + v0);
                const uint4 b = *(const uint4 *)(d.pell + v0 + 2);
                const uint32_t lo[4] = {a.x, a.z, b.x, b.z};
                const uint32_t hi[4] = {a.y, a.w, b.y, b.w};
                const uint32_t selsh = half ? 19u : 16u;
                int t[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t w0 = src[(lo[j] & 0xFFFFu) >> 5];
                    const uint32_t w1 = src[lo[j] >> 21];
                    const uint32_t w2 = src[(hi[j] & 0xFFFFu) >> 5];
                    // the bit extracts read the low five bits of their offset
                    // operand only: the record words themselves are the offsets
                    // of slots 0 and 2
                    const uint32_t b0 = __builtin_amdgcn_ubfe(w0, lo[j], 1u);
                    const uint32_t b2 = __builtin_amdgcn_ubfe(w2, hi[j], 1u);
                    const uint32_t t1 = w1 >> ((lo[j] >> 16) & 31u);
                    const uint32_t x = (b2 << 2) | (((t1 & 1u) << 1) | b0);
                    const uint32_t sel = (hi[j] >> selsh) & 7u;
                    const uint32_t y = (x ^ (hi[j] >> 22)) & sel;
                    const uint32_t pc = __popc(y), qc = __popc(sel);
                    t[j] = 2 * (int)pc - (int)qc;
                    pq[j] = (pc << 7) | (qc << 5);
                    cl[j] = (int)((hi[j] >> 25) & 15u);
                }
                S0 = t[0];
                S1 = t[1];
                S2 = t[2];
                S3 = t[3];
            } else if constexpr (LAY == GL_ELL) {
                // ELL: one 16-byte record per slot for the 4 vertices, no row pointers
                const int K = d.ell_k;
                const uint32_t want = (uint32_t)(half + 1);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint4 rec = *(const uint4 *)(d.ell + min(k, K - 1) * d.ell_stride + v0);
                    const uint32_t e[4] = {rec.x, rec.y, rec.z, rec.w};
                    int t[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int sv = lds_spin(src, (int)(e[j] & 0x1FFFFFFFu));
                        const int v = (e[j] >> 31) ? -sv : sv;
                        t[j] = (k < K && ((e[j] >> 29) & 3u) == want) ? v : 0;
                    }
                    S0 += t[0];
                    S1 += t[1];
                    S2 += t[2];
                    S3 += t[3];
                }
            } else {
            int rpv[5];
#pragma unroll
            for (int j = 0; j < 5; ++j) rpv[j] = rp[min(v0 + j, n)];
            const int last = rpv[4] - 1;
            for (int base = rpv[0]; base <= last; base += 8) {
                // clamped indices: all eight loads issue before any is used
                int cc[8], jj[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int e = min(base + k, last);
                    cc[k] = col[e];
                    jj[k] = (int)jw[e];
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int e = base + k;
                    const int t = e <= last ? jj[k] * lds_spin(src, cc[k]) : 0;
                    S0 += e < rpv[1] ? t : 0;
                    S1 += (e >= rpv[1] && e < rpv[2]) ? t : 0;
                    S2 += (e >= rpv[2] && e < rpv[3]) ? t : 0;
                    S3 += (e >= rpv[3]) ? t : 0;
                }
            }
            }
            const int Sv[4] = {S0, S1, S2, S3};
            if constexpr (LAY != GL_PACKED) {
                if (v0 + 3 < n) {
                    const uint32_t c4 = *(const uint32_t *)(d.cls + v0);
#pragma unroll
                    for (int j = 0; j < 4; ++j) cl[j] = (int)((c4 >> (8 * j)) & 0xFFu);
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) cl[j] = v0 + j < n ? d.cls[v0 + j] : 0;
                }
            }
            // own spins of the four vertices: bits (v0 & 31) .. +3 of one word.
            // Vertices past n (the last group's padding) have no edges in any
            // layout (S = 0, class 0): they are computed like the others and
            // their bits masked, with no test per vertex
            const uint32_t vmask = n - v0 >= 4 ? 0xFu : (1u << (n - v0)) - 1u;
            const uint32_t ownw = (src[v0 >> 5] >> (v0 & 31)) & vmask;
            if (dst) {
                const U4 r = philox10_c0((uint32_t)q4, ps, k0, k1);
                const uint32_t u[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int own = (int)((ownw >> j) & 1u);
                    // packed: the table is indexed by (p, q, own, class) with
                    // power-of-two strides (built by run_graph), no multiply
                    const uint64_t T = LAY == GL_PACKED
                                           ? lut[pq[j] | ((uint32_t)own << 4) | (uint32_t)cl[j]]
                                           : lut[__mul24((Sv[j] + smax) * 2 + own, ncls) + cl[j]];
                    bits |= (uint32_t)((uint64_t)u[j] < T) << j;
                }
                bits = (bits | frozen4(d, v0)) & vmask;
            }
            if (obs) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const bool up = (ownw >> j) & 1u;
                    e_acc += up ? Sv[j] : -Sv[j];
                    if (pc_reg)
                        pcb += (uint32_t)up << (8 * cl[j]);
                    else if (up)
                        atomicAdd(&sh_plus[cl[j]], 1);
                }
            }
        }
        if (dst) {
            // the eight lanes' 4-bit pieces OR-ed into the group's last lane
            // (DPP row shifts; every lane of the workgroup is here)
            uint32_t val = bits << (4 * (q4 & 7));
            val |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)val, 0x111, 0xF, 0xF, true);   // row_shr:1
            val |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)val, 0x112, 0xF, 0xF, true);   // row_shr:2
            val |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)val, 0x114, 0xF, 0xF, true);   // row_shr:4
            if ((q4 & 7) == 7 && (q4 & ~7) < nq) dst[q4 >> 3] = val;
        }
    }
    if (obs) {
        if (pc_reg) {
            const int lane = threadIdx.x & 63;
            for (int k = 0; k < ncls; ++k) {
                const int t = wave_sum((int)((pcb >> (8 * k)) & 0xFFu));
                if (lane == 0 && t) atomicAdd(&sh_plus[k], t);
            }
        }
        int dummy = 0;
        block_sum2(e_acc, dummy, sh_red);  // ends with a barrier: sh_plus is complete
        if (threadIdx.x == 0) {
            o->e = e_acc;
            for (int c = 0; c < ncls; ++c) o->plus[c] = sh_plus[c];
        }
    }
}

template <int LAY>
__device__ __attribute__((noinline)) void run_graph(const ChainDesc &d_arg, uint32_t (*buf)[kPWords], uint32_t s0_arg,
                                                    int64_t n_full_arg, int record_arg, int track_arg,
                                                    int *sh_red, int *sh_plus, int *sh_flag,
                                                    uint64_t *sh_lut, Obs &o) {
    const ChainDesc &d = uniform_desc(d_arg);
    const uint32_t s0 = (uint32_t)__builtin_amdgcn_readfirstlane(s0_arg);
    const int64_t n_full = uniform_i64(n_full_arg);
    const int record = __builtin_amdgcn_readfirstlane(record_arg);
    const int track = __builtin_amdgcn_readfirstlane(track_arg);
    const int n = d.n, nw = (n + 31) / 32;
    const bool obs = record || track;
    // the chain's threshold table in LDS when it fits (constant during the call)
    const int nlut = (2 * d.smax + 1) * 2 * d.ncls;
    const uint64_t *lut = d.lut;
    if constexpr (LAY == GL_PACKED) {
        // re-indexed for the packed record (couplings +-1, at most three
        // slots, at most 16 classes): entry ((p * 4 + q) * 2 + own) * 16 +
        // class holds the threshold of the field S = 2p - q, p of the q slots
        // of the half having J sigma_y = +1; combinations that cannot occur
        // (p > q, or |S| beyond the table) stay 0
        static_assert(kPLut == 4 * 4 * 2 * 16, "the packed table fills the LDS table");
        for (int i = threadIdx.x; i < kPLut; i += kPBlock) {
            const int cl = i & 15, own = (i >> 4) & 1, q = (i >> 5) & 3, p = (i >> 7) & 3;
            const int S = 2 * p - q;
            uint64_t T = 0;
            if (cl < d.ncls && p <= q && S >= -d.smax && S <= d.smax)
                T = d.lut[((S + d.smax) * 2 + own) * d.ncls + cl];
            sh_lut[i] = T;
        }
    } else if (LAY != GL_CSR || nlut <= kPLut) {
        for (int i = threadIdx.x; i < nlut; i += kPBlock) sh_lut[i] = d.lut[i];
        lut = sh_lut;
    }
    if constexpr (LAY != GL_CSR) lut = sh_lut;  // always LDS (checked on the host)
    const bool bp = d.format == FMT_BITPACKED;
    if (bp) {
        const uint32_t *g = (const uint32_t *)d.spin[0];
        for (int w = threadIdx.x; w < nw; w += kPBlock) buf[0][w] = g[w];
    } else {
        const int8_t *g = (const int8_t *)d.spin[0];
        for (int w = threadIdx.x; w < nw; w += kPBlock) {
            uint32_t word = 0;
            for (int b = 0; b < 32; ++b) {
                const int v = 32 * w + b;
                if (v < n && g[v] > 0) word |= 1u << b;
            }
            buf[0][w] = word;
        }
    }
    __syncthreads();
    int64_t best_h = INT64_MAX, last_h = 0;
    for (int64_t t = 0; t < n_full; ++t) {
        const uint32_t s = s0 + 2u * (uint32_t)t;
        graph_lds_half<LAY>(d, buf[0], buf[1], s, obs, sh_red, sh_plus, &o, lut);
        if (obs)
            observe_step(d, o, record ? d.log + t * d.log_stride : nullptr, track, &best_h, &last_h,
                         buf[0], nw, sh_flag);
        __syncthreads();
        graph_lds_half<LAY>(d, buf[1], buf[0], s + 1u, false, sh_red, sh_plus, nullptr, lut);
        __syncthreads();
    }
    if (obs) {
        graph_lds_half<LAY>(d, buf[0], nullptr, s0, true, sh_red, sh_plus, &o, lut);
        observe_step(d, o, record ? d.log + n_full * d.log_stride : nullptr, track, &best_h, &last_h,
                     buf[0], nw, sh_flag);
        if (track && threadIdx.x == 0) {
            d.track[0] = last_h;
            d.track[1] = best_h;
        }
    }
    if (bp) {
        uint32_t *go = (uint32_t *)d.spin[0];
        for (int w = threadIdx.x; w < nw; w += kPBlock)
            go[w] = buf[0][w] & (32 * w + 32 <= n ? 0xFFFFFFFFu : ((1u << (n & 31)) - 1u));
    } else {
        int8_t *go = (int8_t *)d.spin[0];
        for (int v = threadIdx.x; v < n; v += kPBlock) go[v] = (int8_t)lds_spin(buf[0], v);
    }
}

// ------------------------------------------------------------------ kernel

// At least 8 waves per SIMD: two 1024-thread workgroups per CU, 64 VGPRs.
// Twice the occupancy of the unconstrained allocation (120 VGPRs) outweighs
// the few spills it costs.
#ifndef SHAKEN_PWAVES
#define SHAKEN_PWAVES 8
#endif
__global__ __launch_bounds__(kPBlock, SHAKEN_PWAVES) void k_persistent(const ChainDesc *__restrict__ descs,
                                                        int nchains,
                                                        const int32_t *__restrict__ order,
                                                        int32_t *counter, uint32_t s0_arg,
                                                        const uint32_t *__restrict__ sp,
                                                        int64_t n_full_arg, int record, int track) {
    // start half-step and full steps from device memory under a replayed HIP graph
    const uint32_t s0 = sp ? (uint32_t)__builtin_amdgcn_readfirstlane(sp[0]) : s0_arg;
    const int64_t n_full = sp ? (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane(sp[1]) : n_full_arg;
    __shared__ uint32_t buf[2][kPWords];
    __shared__ int sh_item;
    __shared__ int sh_flag;
    __shared__ int sh_red[2 * (kPBlock / 64)];
    __shared__ int sh_plus[kPClasses];
    __shared__ uint64_t sh_lut[kPLut];
    __shared__ Obs sh_obs;  // observables of the current configuration (thread 0)
    __shared__ TailQ sh_tail;
    __shared__ uint32_t sh_jn[2 * kPWords];  // +-J torus: its coupling-sign planes
    for (;;) {
        if (threadIdx.x == 0) {
            const int k = atomicAdd(counter, 1);
            sh_item = k < nchains ? order[k] : -1;
        }
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(sh_item);
        __syncthreads();
        if (item < 0) break;  // queue drained: every wave of the block leaves
        const ChainDesc &d = descs[item];
        if (d.kind == KIND_TORUS) {
            // the plain square torus reads neither coupling-sign nor frozen planes
            const bool ext = d.jneg || d.frozen;
            if (d.tri) {
                if (d.fold3)
                    run_torus<true, true, true>(d, buf, s0, n_full, record, track, sh_red, &sh_flag, sh_obs, &sh_tail, sh_jn);
                else
                    run_torus<false, true, true>(d, buf, s0, n_full, record, track, sh_red, &sh_flag, sh_obs, &sh_tail, sh_jn);
            } else if (ext) {
                if (d.fold3)
                    run_torus<true, false, true>(d, buf, s0, n_full, record, track, sh_red, &sh_flag, sh_obs, &sh_tail, sh_jn);
                else
                    run_torus<false, false, true>(d, buf, s0, n_full, record, track, sh_red, &sh_flag, sh_obs, &sh_tail, sh_jn);
            } else if (d.fold3) {
                run_torus<true, false, false>(d, buf, s0, n_full, record, track, sh_red, &sh_flag, sh_obs, &sh_tail, sh_jn);
            } else {
                run_torus<false, false, false>(d, buf, s0, n_full, record, track, sh_red, &sh_flag, sh_obs, &sh_tail, sh_jn);
            }
        } else {
            if (d.pell)
                run_graph<GL_PACKED>(d, buf, s0, n_full, record, track, sh_red, sh_plus, &sh_flag, sh_lut, sh_obs);
            else if (d.ell)
                run_graph<GL_ELL>(d, buf, s0, n_full, record, track, sh_red, sh_plus, &sh_flag, sh_lut, sh_obs);
            else
                run_graph<GL_CSR>(d, buf, s0, n_full, record, track, sh_red, sh_plus, &sh_flag, sh_lut, sh_obs);
        }
        __syncthreads();
    }
}

int persistent_resident_blocks() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent, kPBlock, 0) != hipSuccess || nb < 1)
        nb = 1;
    return nb;
}

hipError_t launch_persistent(const ChainDesc *dev_descs, int nchains, const int32_t *order,
                             int32_t *counter, uint32_t s0, const uint32_t *sp, int64_t n_full,
                             int record, int track, int block, int grid, hipStream_t stream) {
    (void)block;
    if (nchains <= 0) return hipSuccess;
    const int g = grid > 0 ? grid : nchains;
    hipLaunchKernelGGL(k_persistent, dim3(g), dim3(kPBlock), 0, stream, dev_descs, nchains, order,
                       counter, s0, sp, n_full, record, track);
    return hipGetLastError();
}

}  // namespace shaken
