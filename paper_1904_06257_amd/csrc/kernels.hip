// HIP kernels of libshaken for gfx950 (MI355X).
//
// The half-steps of shaken dynamics (arXiv:1904.06257, section 2: kernels
// P^{1->2} and P^{2->1}; section 3: P^dl and P^ur on the torus).  Every kernel
// reads one configuration and writes the other buffer: a half-step is a
// parallel update, never an in-place one.
//
// Bit-packed torus ("multi-spin coding"): one lane owns one 32-site word.
// The neighbour words of the half (down/left for dl, up/right for ur) give
// three bit-planes a, b, c (two neighbours and the site itself).  With a
// uniform coupling the field is h = J(2 n_plus - 2) + q sigma + lambda, so a
// site belongs to one of six classes j = n_plus + 3 c.  The comparison
// u < T is done bit-serially from the most significant level, 32 sites at a
// time: level k of the 32 uniforms is one Philox output word (the bit-sliced
// uniform of the contract), the matching threshold bit-plane is assembled from
// the class masks, and a site drops out of the comparison as soon as its
// uniform bit differs from its threshold bit.  Thresholds are folded by the
// sign of h (u < 2^32 - t  <=>  not(~u < t)), so only t <= 2^31 is compared.
#include <climits>

#include "device.hpp"

namespace shaken {

// neighbour bit-planes of word (r, wd) for half `phase` (0 = down/left,
// 1 = up/right) on an L x L torus with W words per row
__device__ __forceinline__ void bp_neighbours(const uint32_t *__restrict__ sp, int L, int W, int r,
                                              int wd, int phase, uint32_t own, uint32_t &a,
                                              uint32_t &b) {
    const int lastbits = ((L - 1) & 31);  // bit index of column L-1 in the last word
    if (phase == 0) {
        const int rd = (r == 0) ? L - 1 : r - 1;
        a = sp[rd * W + wd];
        uint32_t carry;
        if (wd > 0)
            carry = sp[r * W + wd - 1] >> 31;
        else
            carry = (sp[r * W + W - 1] >> lastbits) & 1u;
        b = (own << 1) | carry;
    } else {
        const int ru = (r == L - 1) ? 0 : r + 1;
        a = sp[ru * W + wd];
        if (wd < W - 1)
            b = (own >> 1) | (sp[r * W + wd + 1] << 31);
        else
            b = (own >> 1) | ((sp[r * W] & 1u) << lastbits);
    }
}


// Half-step index and log slot of a launch.  The index is dstate[0] + s_add
// when the launch reads it from device memory (replayable HIP graphs), else
// s_add; the configuration at half-step s lives in spin[s & 1].  Observables
// of the configuration read at an even s go to slot (s - base) / 2.
struct StepArgs {
    const uint32_t *dstate;  // [0] = half-step base, [1] = log base (or null)
    uint32_t s_add;
    uint32_t s_log0;
    int log_on;
};

__device__ __forceinline__ uint32_t step_s(const StepArgs &a) {
    return (a.dstate ? a.dstate[0] : 0u) + a.s_add;
}
__device__ __forceinline__ int step_slot(const StepArgs &a, uint32_t s) {
    return (int)((s - (a.dstate ? a.dstate[1] : a.s_log0)) >> 1);
}

// Finish a word whose first level groups left sites undecided (groups
// G0..7).  Six-class table: res holds the sites decided with v < t; folded
// table: the new spins of the sites decided.
template <bool FOLD3, int G0 = 2>
__device__ __noinline__ uint32_t bp_finish(uint32_t a, uint32_t b, uint32_t c, uint32_t und,
                                           uint32_t res, uint32_t vm, uint32_t w, uint32_t s,
                                           uint32_t rep, uint32_t k0, uint32_t k1,
                                           const uint32_t *__restrict__ ts, uint32_t sgn) {
    if constexpr (FOLD3) {
        return fold_finish<SqSel, G0>(SqSel{fold_planes(a, b, c), fold_t(ts, sgn)}, und, res, vm, w, s, rep, k0,
                                      k1, sgn);
    } else {
        static_assert(G0 == 2, "six-class words are finished from group 2");
        const BpPlanes p = bp_planes(a, b, c, sgn);
        bp_groups<2, 8>(p, und, res, w, s, rep, k0, k1, ts);
        return (res ^ p.smask) & vm;
    }
}

// One lane owns a strip of kRows words of one word column: it loads the strip,
// the halo row below (dl) or above (ur) and the adjacent words that supply the
// wrap-around bit; the vertical neighbour of a row is the strip's next or
// previous row, already in registers.
//
// Tail compaction: every word first runs level groups 0 and 1 (8 levels, after
// which a word is still undecided with probability 1 - (1 - 2^-8)^32 = 0.118).
// Undecided words are appended to a queue in LDS and finished afterwards by
// all lanes of the workgroup together, so that a wavefront does not idle while
// its slowest lane runs the rare deep levels.  Each wavefront appends to a
// region of its own at a slot it computes from its ballot (no shared counter,
// no broadcast); a region that fills up finishes its words in place.
constexpr int kQCap = 512;
// Folded table: words still undecided after level group 2 of the tail move to
// a second, short queue (about 1 in 15 of the first queue's), so that the rare
// deeper groups run in the few wavefronts those words fill (four lanes per
// word, one level group each) instead of in all of them.
constexpr int kQ2Cap = 128;
// A queued word index carries this flag where the word is the last of its row
// with bits past the side (its valid-bit mask is the row end's).
constexpr uint32_t kLastWord = 0x80000000u;

// Tail queue in wavefront regions of qcap_w entries, cnt[r] of them used:
// the entries in region order.  The region boundaries are read once (the
// same in every lane); the slot of the it-th entry is then three compares
// and adds, with no loop and no LDS read per entry.
struct TailMap {
    int total;             // entries queued in all regions
    int b1, b2, b3;        // first entry of regions 1, 2, 3 (past the total if absent)
    int d1, d2, d3;        // slot offset added on entering regions 1, 2, 3
};
__device__ __forceinline__ TailMap tail_map(const int *cnt, int nwav, int qcap_w) {
    const int c0 = cnt[0], c1 = nwav > 1 ? cnt[1] : 0, c2 = nwav > 2 ? cnt[2] : 0, c3 = nwav > 3 ? cnt[3] : 0;
    TailMap m;
    m.total = c0 + c1 + c2 + c3;
    m.b1 = nwav > 1 ? c0 : m.total;
    m.b2 = nwav > 2 ? c0 + c1 : m.total;
    m.b3 = nwav > 3 ? c0 + c1 + c2 : m.total;
    m.d1 = qcap_w - c0;
    m.d2 = qcap_w - c1;
    m.d3 = qcap_w - c2;
    return m;
}
__device__ __forceinline__ int tail_slot(const TailMap &m, int it) {
    return it + (it >= m.b1 ? m.d1 : 0) + (it >= m.b2 ? m.d2 : 0) + (it >= m.b3 ? m.d3 : 0);
}

// EXT: instantiation for chains with +-J sign planes or a frozen set (the
// plain instantiation reads neither).  ALIGN: every chain's side is a
// multiple of 32 (no padding bits, whole strips, the wrap-around bit always
// at bit 31), which spares the per-row masks and selects.  FULL (with ALIGN):
// every chain has exactly as many strips as the grid has lanes, so every
// lane is live and no row needs its activity select.
template <bool OBS, bool FOLD3, bool EXT, bool ALIGN = false, bool FULL = false>
__global__ __launch_bounds__(256) void k_torus_bp(const ChainDesc *__restrict__ descs, StepArgs sa) {
    static_assert(ALIGN || !FULL, "FULL grids are aligned ones");
    __shared__ uint32_t q_w[kQCap], q_a[kQCap], q_b[kQCap], q_c[kQCap], q_und[kQCap], q_res[kQCap];
    __shared__ int q_cnt[4];  // entries queued per wavefront region
    __shared__ uint32_t q2_w[FOLD3 ? kQ2Cap : 1], q2_a[FOLD3 ? kQ2Cap : 1], q2_b[FOLD3 ? kQ2Cap : 1],
        q2_c[FOLD3 ? kQ2Cap : 1], q2_und[FOLD3 ? kQ2Cap : 1], q2_res[FOLD3 ? kQ2Cap : 1];
    __shared__ int q2_cnt;
    const ChainDesc &d = descs[blockIdx.y];
    const uint32_t s = step_s(sa);
    const int bufp = (int)(s & 1u);      // configuration at s lives in spin[s & 1]
    const int phase = bufp ^ d.rev;      // half read: 0 = dl, 1 = ur
    const int slot = OBS ? step_slot(sa, s) : 0;
    const int L = d.L, W = d.W;
    const int nrb = (L + kRows - 1) / kRows;
    const int total = nrb * W;
    const int bx = xcd_block(blockIdx.x, gridDim.x);
    const int gid = bx * blockDim.x + threadIdx.x;
    // global (not generic) pointers: stores and loads address through a
    // scalar base, and they do not count against the LDS wait counter
    const gmem_u32 *__restrict__ in = (const gmem_u32 *)d.spin[bufp];
    gmem_u32 *__restrict__ out = (gmem_u32 *)d.spin[bufp ^ 1];
    const uint32_t k0 = (uint32_t)d.seed, k1 = (uint32_t)(d.seed >> 32);
    const uint32_t rep = d.replica, sgn = d.sgn;
    const uint32_t *ts = d.tsmall;
    // tail queue: each wavefront fills a region of its own (no shared counter)
    // block sizes are 64, 128 or 256: one, two or four wavefronts
    const int nwav = (int)(blockDim.x + 63) >> 6, wv = (int)threadIdx.x >> 6;
    const int qcap_w = kQCap >> (nwav == 4 ? 2 : (nwav == 2 ? 1 : 0)), qbase = wv * qcap_w;
    int wq = 0;  // entries this wavefront has queued (the same in every lane)
    int dis_acc = 0, p_acc = 0;  // disagreeing in-half bonds and +1 sites
    const bool live = FULL || gid < total;
    // row block and word column: gid / W as a multiply-high (W = 1: the
    // reciprocal 2^32 does not fit, and gid is the row block itself)
    const int rb = !live ? 0 : (W == 1 ? gid : (int)__umulhi((uint32_t)gid, d.wdiv));
    const int wd = live ? gid - rb * W : 0;
    const int r0 = rb * kRows;
    const int nr = live ? (ALIGN ? kRows : min(kRows, L - r0)) : 0;
    const uint32_t vm = ALIGN ? ~0u : bp_valid(L, W, wd);
    const int lastbits = (L - 1) & 31;
    // adjacent word supplying the carry bit: left word (dl) / right word (ur)
    const int wside = phase == 0 ? (wd > 0 ? wd - 1 : W - 1) : (wd < W - 1 ? wd + 1 : 0);
    // position of the wrap-around bit: the adjacent word's bit brought to bit 0
    // (dl) or the bit it lands on (ur); 31 inside a row, the last valid bit at
    // the row's end
    const int csh = (ALIGN || (phase == 0 ? wd > 0 : wd < W - 1)) ? 31 : lastbits;
    // rows past the side are the buffer's zero padding (no sites)
    uint32_t own[kRows], side[kRows];
    const uint32_t obase = (uint32_t)(r0 * W + wd), sbase = (uint32_t)(r0 * W + wside);
    // row i of the strip: a scalar base (row offsets are the same in every
    // lane) plus the lane's byte offsets, so no address arithmetic per load
    const uint32_t ob4 = obase << 2, sb4 = sbase << 2;
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
        const gmem_char *rowb = (const gmem_char *)in + (size_t)i * (size_t)W * 4u;
        own[i] = *(const gmem_u32 *)(rowb + ob4);
        side[i] = *(const gmem_u32 *)(rowb + sb4);
    }
    uint32_t halo = 0;
    if (live) {
        const int rh = phase == 0 ? (r0 == 0 ? L - 1 : r0 - 1) : (r0 + nr == L ? 0 : r0 + nr);
        halo = gload(in, (uint32_t)(rh * W + wd));
    }
    BpRestMasks rm;
    FoldT ft;
    if constexpr (FOLD3) {
        ft = fold_t(ts, sgn);
        rm = bp_rest_masks(ft.rest);
    }
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
        // rows past the strip (and lanes past the grid) are computed with no
        // valid sites: nothing undecided, nothing stored
        const bool act = ALIGN ? live : i < nr;
        const uint32_t vmi = act ? vm : 0u;
        // i * W on the scalar unit (EXT: the sign planes' index shares (r0 + i) * W)
        const int widx = EXT ? (r0 + i) * W + wd : (int)obase + i * W;
        uint32_t a, b;
        if (phase == 0) {
            a = (i == 0) ? halo : own[i > 0 ? i - 1 : 0];
            b = ALIGN ? __builtin_amdgcn_alignbit(own[i], side[i], 31) : (own[i] << 1) | ((side[i] >> csh) & 1u);
        } else {
            a = (ALIGN ? i == kRows - 1 : i == nr - 1) ? halo : own[i < kRows - 1 ? i + 1 : 0];
            b = ALIGN ? __builtin_amdgcn_alignbit(side[i], own[i], 1) : (own[i] >> 1) | ((side[i] & 1u) << csh);
        }
        if (EXT && d.jneg && act) bp_jflip(d.jneg, L, W, r0 + i, wd, phase, a, b);
        if (OBS) {
            // disagreeing in-half bonds and +1 sites of the configuration read
            dis_acc += __popc(__builtin_amdgcn_bitop3_b32(own[i], a, vmi, kT_xor_and));
            dis_acc += __popc(__builtin_amdgcn_bitop3_b32(own[i], b, vmi, kT_xor_and));
            p_acc += __popc(own[i] & vmi);
            // count here: left to the compiler, the counts sink to their use
            // after the tail and keep every row's planes live across it
            asm volatile("" : "+v"(dis_acc), "+v"(p_acc));
        }
        // folded table: res = new spins of the sites decided; six classes:
        // the sites decided with v < t (the flip plane applied at the store)
        uint32_t und, res, smask = 0;
        if constexpr (FOLD3) {
            uint32_t o = 0, eq = ~0u;
            SqSelV sl;
            sl.p = fold_planes(a, b, own[i]);
            sl.ft = ft;
            sl.rm = &rm;
            fold_top8(sl, o, eq, (uint32_t)widx, s, rep, k0, k1);
            und = eq & vmi;
            res = o & ~eq;
        } else {
            // under the row's own branch: merged across rows, the scalar
            // level masks of the six classes would not fit the scalar registers
            und = 0;
            res = 0;
            if (act) {
                const BpPlanes p = bp_planes(a, b, own[i], sgn);
                smask = p.smask;
                und = vm;
                bp_groups<0, 2>(p, und, res, (uint32_t)widx, s, rep, k0, k1, ts);
            }
        }
        const bool pend = und != 0;
        const unsigned long long bal = __ballot(pend);
        if (pend) {
            // slot in the wavefront's region: entries queued so far + pending lanes below
            const int q = wq + (int)__builtin_amdgcn_mbcnt_hi(
                                   (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            if (q < qcap_w) {
                const int qs = qbase + q;
                q_w[qs] = (uint32_t)widx | (vm != ~0u ? kLastWord : 0u);
                q_a[qs] = a;
                q_b[qs] = b;
                q_c[qs] = own[i];
                q_und[qs] = und;
                q_res[qs] = res;
            } else {
                gword(out, (uint32_t)widx) = bp_finish<FOLD3>(a, b, own[i], und, res, vm, (uint32_t)widx, s, rep, k0, k1, ts, sgn) |
                            (EXT ? frozen_word(d, widx) : 0u);
            }
        } else if (act) {
            gword(out, (uint32_t)widx) = ((res ^ smask) & vm) | (EXT ? frozen_word(d, widx) : 0u);
        }
        wq += (int)__popcll(bal);
    }
    if ((threadIdx.x & 63) == 0) q_cnt[wv] = min(wq, qcap_w);
    if (FOLD3 && threadIdx.x == 0) q2_cnt = 0;
    __syncthreads();
    const TailMap tm = tail_map(q_cnt, nwav, qcap_w);
    const int Q = tm.total;
    const uint32_t vlast = bp_valid(L, W, W - 1);
    if constexpr (FOLD3) {
        // stage 1: level group 2 of every queued word
        for (int it = threadIdx.x; it < Q; it += blockDim.x) {
            const int qs = tail_slot(tm, it);
            const uint32_t wf = q_w[qs], w = wf & ~kLastWord;
            const uint32_t vw = (wf & kLastWord) ? vlast : ~0u;
            const uint32_t a = q_a[qs], b = q_b[qs], c = q_c[qs];
            uint32_t und = q_und[qs], o = q_res[qs];
            fold_groups<SqSel, 2, 3>(SqSel{fold_planes(a, b, c), ft}, und, o, w, s, rep, k0, k1);
            if (und == 0) {
                gword(out, w) = (o & vw) | (EXT ? frozen_word(d, (int)w) : 0u);
            } else {
                const int q2 = atomicAdd(&q2_cnt, 1);
                if (q2 < kQ2Cap) {
                    q2_w[q2] = wf;
                    q2_a[q2] = a;
                    q2_b[q2] = b;
                    q2_c[q2] = c;
                    q2_und[q2] = und;
                    q2_res[q2] = o;
                } else {
                    gword(out, w) = bp_finish<true, 3>(a, b, c, und, o, vw, w, s, rep, k0, k1, ts, sgn) |
                                    (EXT ? frozen_word(d, (int)w) : 0u);
                }
            }
        }
        __syncthreads();
        // stage 2: groups 3..7 of the words still undecided, four lanes per
        // word (whole quads: 4 Q2 and the block size are multiples of four)
        const int Q2 = min(q2_cnt, kQ2Cap);
        for (int it = threadIdx.x; it < 4 * Q2; it += blockDim.x) {
            const int wi = it >> 2;
            const uint32_t wf = q2_w[wi], w = wf & ~kLastWord;
            const uint32_t vw = (wf & kLastWord) ? vlast : ~0u;
            fold_quad_finish(SqSel{fold_planes(q2_a[wi], q2_b[wi], q2_c[wi]), ft}, q2_und[wi], q2_res[wi], it & 3, vw,
                             w, s, rep, k0, k1, sgn,
                             [&](uint32_t word) { gword(out, w) = word | (EXT ? frozen_word(d, (int)w) : 0u); });
        }
    } else {
        for (int it = threadIdx.x; it < Q; it += blockDim.x) {
            const int qs = tail_slot(tm, it);
            const uint32_t wf = q_w[qs], w = wf & ~kLastWord;
            const uint32_t vw = (wf & kLastWord) ? vlast : ~0u;
            gword(out, w) = bp_finish<false>(q_a[qs], q_b[qs], q_c[qs], q_und[qs], q_res[qs], vw, w, s, rep, k0,
                                             k1, ts, sgn) | (EXT ? frozen_word(d, (int)w) : 0u);
        }
    }
    if (OBS && bx * (int)blockDim.x < total) {
        // each site has two in-half bonds, J sigma sigma' = J (1 - 2 [disagree])
        const int e_acc = d.J * (2 * nr * __popc(vm) - 2 * dis_acc);
        block_accumulate2(e_acc, p_acc, log_part(d, slot, bx));
    }
}

// ------------------------------------------------ triangular bit-packed torus
// Same strip structure and tail queue as k_torus_bp; the third neighbour plane
// e is the vertical neighbour row shifted like b (dl: the down-left
// neighbours, the row below shifted left with the carry of its left word; ur:
// the up-right neighbours, the row above shifted right with the carry of its
// right word).

template <bool FOLD, int G0 = 2>
__device__ __noinline__ uint32_t tri_finish(uint32_t a, uint32_t b, uint32_t e, uint32_t c,
                                            uint32_t und, uint32_t res, uint32_t vm, uint32_t w,
                                            uint32_t s, uint32_t rep, uint32_t k0, uint32_t k1,
                                            const uint32_t *__restrict__ ts, uint32_t sgn) {
    if constexpr (FOLD) {
        return fold_finish<TriSel, G0>(tri_sel(a, b, e, c, ts, sgn), und, res, vm, w, s, rep, k0, k1, sgn);
    } else {
        static_assert(G0 == 2, "eight-class words are finished from group 2");
        const TriPlanes p = tri_planes(a, b, e, c, sgn);
        tri_groups<2, 8>(p, und, res, w, s, rep, k0, k1, ts);
        return (res ^ p.smask) & vm;
    }
}

template <bool OBS, bool FOLD, bool ALIGN = false, bool FULL = false>
__global__ __launch_bounds__(256) void k_tri_bp(const ChainDesc *__restrict__ descs, StepArgs sa) {
    static_assert(ALIGN || !FULL, "FULL grids are aligned ones");  // as in k_torus_bp
    __shared__ uint32_t q_w[kQCap], q_a[kQCap], q_b[kQCap], q_e[kQCap], q_c[kQCap], q_und[kQCap],
        q_res[kQCap];
    __shared__ int q_cnt[4];  // entries queued per wavefront region
    __shared__ uint32_t q2_w[FOLD ? kQ2Cap : 1], q2_a[FOLD ? kQ2Cap : 1], q2_b[FOLD ? kQ2Cap : 1],
        q2_e[FOLD ? kQ2Cap : 1], q2_c[FOLD ? kQ2Cap : 1], q2_und[FOLD ? kQ2Cap : 1], q2_res[FOLD ? kQ2Cap : 1];
    __shared__ int q2_cnt;
    const ChainDesc &d = descs[blockIdx.y];
    const uint32_t s = step_s(sa);
    const int bufp = (int)(s & 1u);
    const int phase = bufp ^ d.rev;
    const int slot = OBS ? step_slot(sa, s) : 0;
    const int L = d.L, W = d.W;
    const int nrb = (L + kRows - 1) / kRows;
    const int total = nrb * W;
    const int bx = xcd_block(blockIdx.x, gridDim.x);
    const int gid = bx * blockDim.x + threadIdx.x;
    // global (not generic) pointers: stores and loads address through a
    // scalar base, and they do not count against the LDS wait counter
    const gmem_u32 *__restrict__ in = (const gmem_u32 *)d.spin[bufp];
    gmem_u32 *__restrict__ out = (gmem_u32 *)d.spin[bufp ^ 1];
    const uint32_t k0 = (uint32_t)d.seed, k1 = (uint32_t)(d.seed >> 32);
    const uint32_t rep = d.replica, sgn = d.sgn;
    const uint32_t *ts = d.tsmall;
    // tail queue: each wavefront fills a region of its own (no shared counter)
    // block sizes are 64, 128 or 256: one, two or four wavefronts
    const int nwav = (int)(blockDim.x + 63) >> 6, wv = (int)threadIdx.x >> 6;
    const int qcap_w = kQCap >> (nwav == 4 ? 2 : (nwav == 2 ? 1 : 0)), qbase = wv * qcap_w;
    int wq = 0;  // entries this wavefront has queued (the same in every lane)
    int e_acc = 0, p_acc = 0;
    const bool live = FULL || gid < total;
    // row block and word column (gid / W as a multiply-high, as in k_torus_bp)
    const int rb = !live ? 0 : (W == 1 ? gid : (int)__umulhi((uint32_t)gid, d.wdiv));
    const int wd = live ? gid - rb * W : 0;
    const int r0 = rb * kRows;
    const int nr = live ? (ALIGN ? kRows : min(kRows, L - r0)) : 0;
    const uint32_t vm = ALIGN ? ~0u : bp_valid(L, W, wd);
    const int lastbits = (L - 1) & 31;
    const int wside = phase == 0 ? (wd > 0 ? wd - 1 : W - 1) : (wd < W - 1 ? wd + 1 : 0);
    // position of the wrap-around bit: the adjacent word's bit brought to bit 0
    // (dl) or the bit it lands on (ur); 31 inside a row, the last valid bit at
    // the row's end
    const int csh = (ALIGN || (phase == 0 ? wd > 0 : wd < W - 1)) ? 31 : lastbits;
    // rows past the side are the buffer's zero padding (no sites)
    uint32_t own[kRows], side[kRows];
    const uint32_t obase = (uint32_t)(r0 * W + wd), sbase = (uint32_t)(r0 * W + wside);
    // row i of the strip: a scalar base (row offsets are the same in every
    // lane) plus the lane's byte offsets, so no address arithmetic per load
    const uint32_t ob4 = obase << 2, sb4 = sbase << 2;
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
        const gmem_char *rowb = (const gmem_char *)in + (size_t)i * (size_t)W * 4u;
        own[i] = *(const gmem_u32 *)(rowb + ob4);
        side[i] = *(const gmem_u32 *)(rowb + sb4);
    }
    uint32_t halo = 0, halo_side = 0;
    if (live) {
        const int rh = phase == 0 ? (r0 == 0 ? L - 1 : r0 - 1) : (r0 + nr == L ? 0 : r0 + nr);
        halo = gload(in, (uint32_t)(rh * W + wd));
        halo_side = gload(in, (uint32_t)(rh * W + wside));
    }
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
        // rows past the strip (and lanes past the grid) are computed with no
        // valid sites: nothing undecided, nothing stored
        const bool act = ALIGN ? live : i < nr;
        const uint32_t vmi = act ? vm : 0u;
        const int widx = (int)obase + i * W;   // i * W on the scalar unit
        uint32_t a, b, e;
        if (phase == 0) {
            a = (i == 0) ? halo : own[i > 0 ? i - 1 : 0];
            const uint32_t as = (i == 0) ? halo_side : side[i > 0 ? i - 1 : 0];
            b = ALIGN ? __builtin_amdgcn_alignbit(own[i], side[i], 31) : (own[i] << 1) | ((side[i] >> csh) & 1u);
            e = ALIGN ? __builtin_amdgcn_alignbit(a, as, 31) : (a << 1) | ((as >> csh) & 1u);
        } else {
            const bool top = ALIGN ? i == kRows - 1 : i == nr - 1;
            a = top ? halo : own[i < kRows - 1 ? i + 1 : 0];
            const uint32_t as = top ? halo_side : side[i < kRows - 1 ? i + 1 : 0];
            b = ALIGN ? __builtin_amdgcn_alignbit(side[i], own[i], 1) : (own[i] >> 1) | ((side[i] & 1u) << csh);
            e = ALIGN ? __builtin_amdgcn_alignbit(as, a, 1) : (a >> 1) | ((as & 1u) << csh);
        }
        if (OBS) {
            e_acc += d.J * (3 * __popc(vmi) - 2 * __popc((own[i] ^ a) & vmi) -
                            2 * __popc((own[i] ^ b) & vmi) - 2 * __popc((own[i] ^ e) & vmi));
            p_acc += __popc(own[i] & vmi);
            asm volatile("" : "+v"(e_acc), "+v"(p_acc));  // count here (as in k_torus_bp)
        }
        // folded table: res = new spins of the sites decided; eight classes:
        // the sites decided with v < t (the flip plane applied at the store)
        uint32_t und, res, smask = 0;
        if constexpr (FOLD) {
            uint32_t o = 0, eq = ~0u;
            fold_top8<true>(tri_sel(a, b, e, own[i], ts, sgn), o, eq, (uint32_t)widx, s, rep, k0, k1);
            und = eq & vmi;
            res = o & ~eq;
        } else {
            // under the row's own branch: merged across rows, the scalar
            // level masks of the eight classes would not fit the scalar registers
            und = 0;
            res = 0;
            if (act) {
                const TriPlanes p = tri_planes(a, b, e, own[i], sgn);
                smask = p.smask;
                und = vm;
                tri_groups<0, 2>(p, und, res, (uint32_t)widx, s, rep, k0, k1, ts);
            }
        }
        const bool pend = und != 0;
        const unsigned long long bal = __ballot(pend);
        if (pend) {
            // slot in the wavefront's region: entries queued so far + pending lanes below
            const int q = wq + (int)__builtin_amdgcn_mbcnt_hi(
                                   (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            if (q < qcap_w) {
                const int qs = qbase + q;
                q_w[qs] = (uint32_t)widx | (vm != ~0u ? kLastWord : 0u);
                q_a[qs] = a;
                q_b[qs] = b;
                q_e[qs] = e;
                q_c[qs] = own[i];
                q_und[qs] = und;
                q_res[qs] = res;
            } else {
                gword(out, (uint32_t)widx) = tri_finish<FOLD>(a, b, e, own[i], und, res, vm, (uint32_t)widx, s,
                                                              rep, k0, k1, ts, sgn) | frozen_word(d, widx);
            }
        } else if (act) {
            gword(out, (uint32_t)widx) = ((res ^ smask) & vm) | frozen_word(d, widx);
        }
        wq += (int)__popcll(bal);
    }
    if ((threadIdx.x & 63) == 0) q_cnt[wv] = min(wq, qcap_w);
    if (FOLD && threadIdx.x == 0) q2_cnt = 0;
    __syncthreads();
    const TailMap tm = tail_map(q_cnt, nwav, qcap_w);
    const int Q = tm.total;
    const uint32_t vlast = bp_valid(L, W, W - 1);
    if constexpr (FOLD) {
        // stage 1: level group 2 of every queued word; the words still
        // undecided move to the second queue
        for (int it = threadIdx.x; it < Q; it += blockDim.x) {
            const int qs = tail_slot(tm, it);
            const uint32_t wf = q_w[qs], w = wf & ~kLastWord;
            const uint32_t vw = (wf & kLastWord) ? vlast : ~0u;
            const uint32_t a = q_a[qs], b = q_b[qs], e = q_e[qs], c = q_c[qs];
            uint32_t und = q_und[qs], o = q_res[qs];
            fold_groups<TriSel, 2, 3>(tri_sel(a, b, e, c, ts, sgn), und, o, w, s, rep, k0, k1);
            if (und == 0) {
                gword(out, w) = (o & vw) | frozen_word(d, (int)w);
            } else {
                const int q2 = atomicAdd(&q2_cnt, 1);
                if (q2 < kQ2Cap) {
                    q2_w[q2] = wf;
                    q2_a[q2] = a;
                    q2_b[q2] = b;
                    q2_e[q2] = e;
                    q2_c[q2] = c;
                    q2_und[q2] = und;
                    q2_res[q2] = o;
                } else {
                    gword(out, w) = tri_finish<true, 3>(a, b, e, c, und, o, vw, w, s, rep, k0, k1, ts, sgn) |
                                    frozen_word(d, (int)w);
                }
            }
        }
        __syncthreads();
        // stage 2: groups 3..7 of the words still undecided, four lanes per
        // word as on the square lattice
        const int Q2 = min(q2_cnt, kQ2Cap);
        for (int it = threadIdx.x; it < 4 * Q2; it += blockDim.x) {
            const int wi = it >> 2;
            const uint32_t wf = q2_w[wi], w = wf & ~kLastWord;
            const uint32_t vw = (wf & kLastWord) ? vlast : ~0u;
            fold_quad_finish(tri_sel(q2_a[wi], q2_b[wi], q2_e[wi], q2_c[wi], ts, sgn), q2_und[wi], q2_res[wi], it & 3,
                             vw, w, s, rep, k0, k1, sgn, [&](uint32_t word) { gword(out, w) = word | frozen_word(d, (int)w); });
        }
    } else {
        for (int it = threadIdx.x; it < Q; it += blockDim.x) {
            const int qs = tail_slot(tm, it);
            const uint32_t wf = q_w[qs], w = wf & ~kLastWord;
            const uint32_t vw = (wf & kLastWord) ? vlast : ~0u;
            gword(out, w) = tri_finish<false>(q_a[qs], q_b[qs], q_e[qs], q_c[qs], q_und[qs], q_res[qs], vw, w, s,
                                              rep, k0, k1, ts, sgn) | frozen_word(d, (int)w);
        }
    }
    if (OBS && bx * (int)blockDim.x < total)
        block_accumulate2(e_acc, p_acc, log_part(d, slot, bx));
}

// ------------------------------------------------------------- int8 torus

// u < T for the bit-sliced uniform of bit b of RNG word w, decided from the
// most significant level down
__device__ __forceinline__ bool sliced_less(uint64_t T, uint32_t w, int b, uint32_t s,
                                            uint32_t rep, uint32_t k0, uint32_t k1) {
    if (T >> 32) return true;  // T = 2^32
    const uint32_t t = (uint32_t)T;
    for (int g = 0; g < 8; ++g) {
        const U4 r = philox10(w, s, rep, (uint32_t)g, k0, k1);
        const uint32_t rr[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * g + j;
            const uint32_t ub = (rr[j] >> b) & 1u;
            const uint32_t tb = (t >> (31 - k)) & 1u;
            if (ub != tb) return ub < tb;
        }
    }
    return false;  // u == t
}

template <bool OBS>
__global__ __launch_bounds__(256) void k_torus_i8(const ChainDesc *__restrict__ descs, StepArgs sa) {
    const ChainDesc &d = descs[blockIdx.y];
    const uint32_t s = step_s(sa);
    const int in_idx = (int)(s & 1u);
    const int slot = OBS ? step_slot(sa, s) : 0;
    const int L = d.L, n = d.n;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int8_t *__restrict__ in = (const int8_t *)d.spin[in_idx];
    int8_t *__restrict__ out = (int8_t *)d.spin[in_idx ^ 1];
    int e_acc = 0, p_acc = 0;
    if (gid < n) {
        const int r = gid / L, c = gid - r * L;
        int n1, n2, n3 = 0;
        if (((s & 1u) ^ (uint32_t)d.rev) == 0) {
            const int rd = r == 0 ? L - 1 : r - 1, cl = c == 0 ? L - 1 : c - 1;
            n1 = in[rd * L + c] * torus_jsign(d.jneg, L, d.W, 0, rd, c);
            n2 = in[r * L + cl] * torus_jsign(d.jneg, L, d.W, 1, r, cl);
            if (d.tri) n3 = in[rd * L + cl];   // down-left (triangular lattice)
        } else {
            const int ru = r == L - 1 ? 0 : r + 1, cr = c == L - 1 ? 0 : c + 1;
            n1 = in[ru * L + c] * torus_jsign(d.jneg, L, d.W, 0, r, c);
            n2 = in[r * L + cr] * torus_jsign(d.jneg, L, d.W, 1, r, c);
            if (d.tri) n3 = in[ru * L + cr];   // up-right
        }
        const int own = in[gid];
        const int S = d.J * (n1 + n2 + n3);
        const uint64_t T = d.lut[((S + d.smax) * 2 + (own > 0)) * d.ncls];
        const uint32_t w = (uint32_t)(r * d.W + (c >> 5));
        const bool up = sliced_less(T, w, c & 31, s, d.replica, (uint32_t)d.seed,
                                    (uint32_t)(d.seed >> 32));
        const bool fz = (frozen_word(d, r * d.W + (c >> 5)) >> (c & 31)) & 1u;
        out[gid] = (up || fz) ? 1 : -1;
        if (OBS) {
            e_acc = own * S;
            p_acc = own > 0;
        }
    }
    if (OBS && blockIdx.x < (unsigned)((n + blockDim.x - 1) / blockDim.x))
        block_accumulate2(e_acc, p_acc, log_part(d, slot, blockIdx.x));
}

// ------------------------------------------------------------------ graph

// Lane = 4 consecutive vertices = one Philox call.  S_v sums the CSR row of
// the half (in-half for s even, out-half for s odd).  The rows of the four
// vertices are contiguous in the CSR arrays, so the lane walks them as one
// edge range in chunks of 8 whose loads are all issued before any is used;
// an edge is attributed to its vertex by comparing with the row bounds.
constexpr int kEdgeChunk = 8;
constexpr int kLdsLut = 512;  // threshold entries kept in LDS

// Spins of a graph chain: int8 (+1/-1 per vertex) or bit-packed (bit v & 31
// of word v >> 5; the whole configuration of 2^20 vertices is 128 KiB and
// stays in every XCD's L2).  A bit-packed word is written by the 8 lanes of
// its 32 vertices together (4-bit pieces merged with lane shuffles).
template <bool BP>
__device__ __forceinline__ int graph_spin(const void *sp, int v) {
    if (BP) return ((((const uint32_t *)sp)[v >> 5] >> (v & 31)) & 1u) ? 1 : -1;
    return (int)((const int8_t *)sp)[v];
}

// own spins of vertices v0..v0+3 (v0 + 3 < n unless `full` is false)
template <bool BP>
__device__ __forceinline__ void graph_own4(const void *sp, int v0, int n, bool full, int own[4]) {
    if (BP) {
        const uint32_t w = ((const uint32_t *)sp)[v0 >> 5] >> (v0 & 31);
#pragma unroll
        for (int j = 0; j < 4; ++j) own[j] = ((w >> j) & 1u) ? 1 : -1;
    } else if (full) {
        const uint32_t o4 = *(const uint32_t *)((const int8_t *)sp + v0);
#pragma unroll
        for (int j = 0; j < 4; ++j) own[j] = (int)(int8_t)(o4 >> (8 * j));
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) own[j] = v0 + j < n ? ((const int8_t *)sp)[v0 + j] : 1;
    }
}

// store the new spins of v0..v0+3: `up` bit j = vertex v0+j is +1.  Every lane
// of the wavefront must call this (bit-packed words are merged by shuffles).
template <bool BP>
__device__ __forceinline__ void graph_store4(void *sp, int q4, int n, uint32_t up) {
    const int v0 = 4 * q4;
    if (BP) {
        uint32_t val = (v0 < n ? up : 0u) << (4 * (q4 & 7));
        val |= __shfl_xor(val, 1, 64);
        val |= __shfl_xor(val, 2, 64);
        val |= __shfl_xor(val, 4, 64);
        if ((q4 & 7) == 0 && v0 < n) ((uint32_t *)sp)[q4 >> 3] = val;
        return;
    }
    if (v0 >= n) return;
    uint32_t packed = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) packed |= (((up >> j) & 1u) ? 0x01u : 0xFFu) << (8 * j);
    int8_t *out = (int8_t *)sp;
    if (v0 + 3 < n) {
        *(uint32_t *)(out + v0) = packed;
    } else {
        for (int j = 0; j < 4 && v0 + j < n; ++j) out[v0 + j] = (int8_t)(packed >> (8 * j));
    }
}

template <bool OBS, bool BP>
__global__ __launch_bounds__(256) void k_graph(const ChainDesc *__restrict__ descs, StepArgs sa) {
    const ChainDesc &d = descs[blockIdx.y];
    const uint32_t s = step_s(sa);
    const int bufp = (int)(s & 1u);
    const int half = bufp ^ d.rev;   // 0 = in-half, 1 = out-half
    const int slot = OBS ? step_slot(sa, s) : 0;
    const int n = d.n;
    const int q4 = blockIdx.x * blockDim.x + threadIdx.x;
    const int v0 = q4 * 4;
    const void *__restrict__ in = d.spin[bufp];
    void *__restrict__ out = d.spin[bufp ^ 1];
    const int32_t *__restrict__ rp = d.rowptr[half];
    const int32_t *__restrict__ col = d.col[half];
    const int8_t *__restrict__ jw = d.jw[half];
    const uint8_t *__restrict__ cls = d.cls;
    const int ncls = d.ncls, smax = d.smax;
    int e_acc = 0;
    // threshold table in LDS when it is small (every 3-regular +-J graph: 14 entries)
    __shared__ uint64_t sh_lut[kLdsLut];
    const int nlut = (2 * smax + 1) * 2 * ncls;
    const bool lut_lds = nlut <= kLdsLut;
    if (lut_lds) {
        for (int i = threadIdx.x; i < nlut; i += blockDim.x) sh_lut[i] = d.lut[i];
    }
    extern __shared__ int sh_plus[];  // ncls counters (OBS only)
    if (OBS) {
        for (int i = threadIdx.x; i < ncls; i += blockDim.x) sh_plus[i] = 0;
    }
    // (the barrier that publishes sh_lut / sh_plus comes after this lane's
    // loads are issued, so the table load overlaps them)
    const int active = v0 < n;
    int Sv[4] = {0, 0, 0, 0}, own[4] = {1, 1, 1, 1}, cl[4] = {0, 0, 0, 0};
    U4 r = {0u, 0u, 0u, 0u};
    if (active) {
        const bool full = v0 + 3 < n;
        int rpv[5];
        if (full) {
            const int4 r4 = *(const int4 *)(rp + v0);
            rpv[0] = r4.x;
            rpv[1] = r4.y;
            rpv[2] = r4.z;
            rpv[3] = r4.w;
            rpv[4] = rp[v0 + 4];
        } else {
#pragma unroll
            for (int j = 0; j < 5; ++j) rpv[j] = rp[min(v0 + j, n)];
        }
        graph_own4<BP>(in, v0, n, full, own);
        if (full) {
            const uint32_t c4 = *(const uint32_t *)(cls + v0);
#pragma unroll
            for (int j = 0; j < 4; ++j) cl[j] = (int)((c4 >> (8 * j)) & 0xFFu);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) cl[j] = v0 + j < n ? cls[v0 + j] : 0;
        }
        r = philox10_c0((uint32_t)q4,
                        philox10_shared(s, d.replica, kGraphStream, (uint32_t)d.seed, (uint32_t)(d.seed >> 32)),
                        (uint32_t)d.seed, (uint32_t)(d.seed >> 32));
        int S0 = 0, S1 = 0, S2 = 0, S3 = 0;
        const int last = rpv[4] - 1;
        for (int base = rpv[0]; base <= last; base += kEdgeChunk) {
            // clamped indices: every load is valid and issued before any is used
            int cc[kEdgeChunk], jj[kEdgeChunk], sv[kEdgeChunk];
#pragma unroll
            for (int k = 0; k < kEdgeChunk; ++k) {
                const int e = min(base + k, last);
                cc[k] = col[e];
                jj[k] = (int)jw[e];
            }
#pragma unroll
            for (int k = 0; k < kEdgeChunk; ++k) sv[k] = graph_spin<BP>(in, cc[k]);
#pragma unroll
            for (int k = 0; k < kEdgeChunk; ++k) {
                const int e = base + k;
                const int t = e <= last ? jj[k] * sv[k] : 0;
                S0 += e < rpv[1] ? t : 0;
                S1 += (e >= rpv[1] && e < rpv[2]) ? t : 0;
                S2 += (e >= rpv[2] && e < rpv[3]) ? t : 0;
                S3 += (e >= rpv[3]) ? t : 0;
            }
        }
        Sv[0] = S0;
        Sv[1] = S1;
        Sv[2] = S2;
        Sv[3] = S3;
    }
    __syncthreads();
    uint32_t up = 0;
    if (active) {
        const uint32_t u[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int key = ((Sv[j] + smax) * 2 + (own[j] > 0)) * ncls + cl[j];
            const uint64_t T = lut_lds ? sh_lut[key] : d.lut[key];
            if (v0 + j < n && (uint64_t)u[j] < T) up |= 1u << j;
            if (OBS && v0 + j < n) {
                e_acc += own[j] * Sv[j];
                if (own[j] > 0) atomicAdd(&sh_plus[cl[j]], 1);
            }
        }
    }
    if (v0 < n) up |= frozen4(d, v0);
    graph_store4<BP>(out, q4, n, up);
    if (OBS && blockIdx.x < (unsigned)((n + 4 * blockDim.x - 1) / (4 * blockDim.x))) {
        int64_t *lg = log_part(d, slot, blockIdx.x);
        __shared__ int sh_e[16];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        e_acc = wave_sum(e_acc);
        if (lane == 0) sh_e[wv] = e_acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            long long se = 0;
            for (int i = 0; i < (int)((blockDim.x + 63) >> 6); ++i) se += sh_e[i];
            if (se) atomicAdd((unsigned long long *)&lg[0], (unsigned long long)se);
        }
        for (int i = threadIdx.x; i < ncls; i += blockDim.x)
            if (sh_plus[i]) atomicAdd((unsigned long long *)&lg[1 + i], (unsigned long long)sh_plus[i]);
    }
}

// ------------------------------------------- graph, gathers served from LDS
//
// Every edge of a half-step gathers one neighbour spin.  From global memory a
// random gather costs a whole cache line between L2 and the compute unit, so
// on a large graph those lines, not the bytes of the CSR arrays, bound the
// kernel.  Here each workgroup first copies the bit-packed configuration
// (2^20 vertices: 128 KiB) into LDS with coalesced loads, issued while the
// row pointers and the first edges are still in flight, and the gathers
// become LDS reads.  The bit-packed source is the state itself (bit-packed
// chains) or, for int8 chains, its packed mirror: the kernel writes the new
// int8 spins and the mirror of them, and each call starts by packing the
// configuration it reads (launch_pack_mirror).  One workgroup of 1024 lanes
// per compute unit (the LDS holds one configuration), four vertices per lane
// as in k_graph.
constexpr int kLdsGraphWords = 36864;                 // 144 KiB: up to 1,179,648 vertices
constexpr int kLdsGraphStage = kLdsGraphWords / 4 / kLdsGraphBlock;  // uint4 loads per lane
constexpr int kLdsGraphClasses = 256;
constexpr int kPlusCopies = 8;
constexpr int kLdsEdgeChunk = 12;
static_assert(32 * kLdsGraphWords <= (1 << 21), "edge words hold 21-bit vertex indices");
static_assert(kLdsGraphWords < (1 << 16), "three-slot words hold 16-bit word indices");

// Loads through the global address space (not flat), unconditional at
// clamped indices: a load under a divergent branch makes the compiler wait
// for it before the branch joins, which would serialise the staging.
typedef uint32_t gl_u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t gl_i32x4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ T gld(const void *base, int64_t i) {
    return ((const __attribute__((address_space(1))) T *)base)[i];
}
template <class T>
__device__ __forceinline__ void gst(void *base, int64_t i, T v) {
    ((__attribute__((address_space(1))) T *)base)[i] = v;
}

// The twelve edge words from position e0 on: four aligned 16-byte loads
// from e0 rounded down to a multiple of four, then a shift by e0 & 3 in two
// bitwise selects per word.  Entries past the half's last edge are padding or other
// rows' edges; the caller masks them.
__device__ __forceinline__ void lds_edge_window(const int32_t *cj, int e0, int (&ew)[kLdsEdgeChunk]) {
    const int a = e0 >> 2, o = e0 & 3;
    int w[16];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const gl_i32x4 v = gld<gl_i32x4>(cj, a + i);
        w[4 * i] = v.x;
        w[4 * i + 1] = v.y;
        w[4 * i + 2] = v.z;
        w[4 * i + 3] = v.w;
    }
    // bitwise selects (written as selects, they become a dynamically
    // indexed array in scratch memory)
    const int m2 = -((o >> 1) & 1), m1 = -(o & 1);
    int w1[14];
#pragma unroll
    for (int i = 0; i < 14; ++i) w1[i] = (w[i + 2] & m2) | (w[i] & ~m2);
#pragma unroll
    for (int k = 0; k < kLdsEdgeChunk; ++k) ew[k] = (w1[k + 1] & m1) | (w1[k] & ~m1);
}

// E3: the three-slot layout (half-degrees at most three, couplings of one
// magnitude): each lane loads its twelve slots from a fixed position, and a
// slot costs one LDS read and four instructions with no edge test.
template <bool OBS, bool BP, bool E3>
__global__ __launch_bounds__(kLdsGraphBlock) void k_graph_lds(const ChainDesc *__restrict__ descs, StepArgs sa) {
    // the configuration, and one group of zero words past it (E3's empty slots)
    __shared__ gl_u32x4 sh_sp4[kLdsGraphWords / 4 + 1];
    __shared__ uint64_t sh_lut[kLdsLut];
    __shared__ int sh_plus[kLdsGraphClasses];
    __shared__ int sh_e[kLdsGraphBlock / 64];
    const ChainDesc &d = descs[blockIdx.y];
    const int n = d.n;
    // a chain smaller than the grid: its surplus workgroups leave at once
    if ((int)blockIdx.x * (4 * kLdsGraphBlock) >= n) return;
    const uint32_t s = step_s(sa);
    const int bufp = (int)(s & 1u);
    const int half = bufp ^ d.rev;   // 0 = in-half, 1 = out-half
    const int slot = OBS ? step_slot(sa, s) : 0;
    const int tid = threadIdx.x;
    const int q4 = blockIdx.x * kLdsGraphBlock + tid;
    const int v0 = q4 * 4;
    void *__restrict__ out = d.spin[bufp ^ 1];
    const uint32_t *bits_in = BP ? (const uint32_t *)d.spin[bufp] : d.mirror[bufp];
    uint32_t *__restrict__ bits_out = BP ? (uint32_t *)out : d.mirror[bufp ^ 1];
    const int ncls = d.ncls, smax = d.smax;
    const int nw = (n + 31) >> 5;
    const int ng = (nw + 3) >> 2;     // groups of four words, the last padded
    const bool active = v0 < n;
    const int va = active ? v0 : 0;   // row pointers and classes are padded
                                      // to a multiple of four vertices
    const int nlut = (2 * smax + 1) * 2 * ncls;
    // +1 counts per class in kPlusCopies copies (lane & 7 picks one) where
    // they fit, so that the lanes of one LDS atomic meet on fewer addresses
    const int pcopies = ncls * kPlusCopies <= kLdsGraphClasses ? kPlusCopies : 1;
    const bool lut_lds = nlut <= kLdsLut;
    if (OBS)   // (first: later, its stores would wait for the loads below)
        for (int i = tid; i < ncls * pcopies; i += kLdsGraphBlock) sh_plus[i] = 0;
    if (E3 && tid == 0) sh_sp4[kLdsGraphWords / 4] = gl_u32x4{0u, 0u, 0u, 0u};
    // 1. row bounds (E3: the lane's twelve slots), classes, the lane's
    // threshold entry and frozen bits (every load of steps 1-3
    // unconditional, at clamped indices: a load under a branch makes the
    // compiler wait for all loads before the next dependent one)
    int rpv[5] = {0, 0, 0, 0, 0};
    gl_u32x4 sl[3];
    if constexpr (E3) {
#pragma unroll
        for (int i = 0; i < 3; ++i) sl[i] = gld<gl_u32x4>(d.e3[half], 3 * (int64_t)(va >> 2) + i);
    } else {
        const gl_i32x4 r4 = gld<gl_i32x4>(d.rowptr[half], va >> 2);
        const int rp4 = gld<int32_t>(d.rowptr[half], va + 4);
        rpv[0] = r4.x;
        rpv[1] = r4.y;
        rpv[2] = r4.z;
        rpv[3] = r4.w;
        rpv[4] = rp4;
    }
    const uint32_t c4 = gld<uint32_t>(d.cls, va >> 2);
    const uint64_t lutv = gld<uint64_t>(d.lut, min(tid, nlut - 1));
    // (no frozen set: a valid word of the class bytes, discarded)
    const uint32_t fzw0 = gld<uint32_t>(d.frozen ? (const void *)d.frozen : (const void *)d.cls, va >> 5);
    const uint32_t fzw = d.frozen ? fzw0 : 0u;
    // the lane's four uniforms while those loads are in flight
    U4 r = {0u, 0u, 0u, 0u};
    if (active)
        r = philox10_c0((uint32_t)q4,
                        philox10_shared(s, d.replica, kGraphStream, (uint32_t)d.seed, (uint32_t)(d.seed >> 32)),
                        (uint32_t)d.seed, (uint32_t)(d.seed >> 32));
    // (these loads stay ahead of the rest, and the row bounds are waited
    // for here, before the loads into LDS are issued)
    __builtin_amdgcn_sched_barrier(0);
    const int e_first = rpv[0], last = rpv[4] - 1;
    if constexpr (!E3) asm volatile("" ::"v"(e_first), "v"(last));
    __builtin_amdgcn_sched_barrier(0);
    // 2. the configuration, coalesced, straight into LDS (global_load_lds:
    // lane l of a wavefront loads 16 bytes into the wavefront's 1 KiB LDS
    // segment at 16 l, the same offset as in global memory).  Each group of
    // four words is loaded by exactly one lane, the last group with the
    // buffer's padding, so no other write to the array is needed -- a wait
    // on the vector memory counter covers only the waiting wavefront's own
    // loads, and the barrier below is what orders them for everyone.  Lanes
    // past the last group load it again into LDS no vertex reads; wavefronts
    // wholly past it load nothing.  Issued
    // after the wait for the row bounds (with loads into LDS in flight the
    // compiler no longer counts vector loads as returning in order, and that
    // wait would cover these too) and before the edges (whose registers
    // would otherwise be reused here, each reuse a wait for the edges).
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
#pragma unroll
    for (int k = 0; k < kLdsGraphStage; ++k) {
        const int base = k * kLdsGraphBlock + wv * 64;
        const int g = min(base + lane, ng - 1);
        if (base < ng)   // wave-uniform
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(bits_in + 4 * g),
                                             (__attribute__((address_space(3))) void *)(sh_sp4 + base), 16, 0, 0);
    }
    // 3. the first chunk of the lane's edges (needs the row bounds): twelve
    // edge words (index, row slot, J) from four aligned 16-byte loads (the
    // array is padded past them), which covers four vertices of degree up
    // to three in one round trip and few cache-line requests
    __builtin_amdgcn_sched_barrier(0);
    int ew[kLdsEdgeChunk];
    if constexpr (!E3) lds_edge_window(d.cj[half], e_first, ew);
    // 4. this wavefront's direct loads have landed (vector memory counter),
    // then the barrier: every lane sees the whole configuration
    __builtin_amdgcn_s_waitcnt(0);
    uint32_t *sh_sp = (uint32_t *)sh_sp4;
    if (lut_lds && tid < nlut) sh_lut[tid] = lutv;
    __syncthreads();
    // 5. own spins and field sums from LDS
    // (the lane's four vertices share one word; bits past n are padding
    // and their results are discarded)
    int own[4], cl[4];
    const uint32_t ow = sh_sp[min(v0, n - 1) >> 5] >> (v0 & 31);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        own[j] = ((ow >> j) & 1u) ? 1 : -1;
        cl[j] = (int)((c4 >> (8 * j)) & 0xFFu);
    }
    int S0 = 0, S1 = 0, S2 = 0, S3 = 0;
    const int cnt = last + 1 - e_first;   // the lane's edges
    if constexpr (E3) {
        // all twelve LDS reads first (every slot names a word: a vertex's or
        // the zero word), then per slot the neighbour's bit xor the sign of
        // J: the count of edges with J sigma_y > 0, so that the field is
        // j0 (2 count - degree); vertices past n have only empty slots.  The
        // bit extract reads the low five bits of its offset operand only, so
        // the slot word itself is the offset.
        const uint32_t w[12] = {sl[0].x, sl[0].y, sl[0].z, sl[0].w, sl[1].x, sl[1].y,
                                sl[1].z, sl[1].w, sl[2].x, sl[2].y, sl[2].z, sl[2].w};
        uint32_t x[12];
#pragma unroll
        for (int k = 0; k < 12; ++k)
            x[k] = *(const uint32_t *)((const char *)sh_sp4 + __builtin_amdgcn_ubfe(w[k], 5u, 18u));
        int Sj[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint32_t pc = 0;
#pragma unroll
            for (int k = 3 * j; k < 3 * j + 3; ++k) pc += __builtin_amdgcn_ubfe(x[k], w[k], 1u) ^ (w[k] >> 31);
            Sj[j] = __mul24(d.j0, 2 * (int)pc - (int)__builtin_amdgcn_ubfe(w[3 * j], 23u, 2u));
        }
        S0 = Sj[0];
        S1 = Sj[1];
        S2 = Sj[2];
        S3 = Sj[3];
    } else if (active && cnt <= kLdsEdgeChunk) {
        // all of them in the window: each edge adds J sigma_y + 128 into the
        // 16-bit field of its row vertex (the slot in the word), so the four
        // sums cost one shift and one add per edge; no field can carry (at
        // most twelve terms below 2^9)
        uint64_t acc = 0;
#pragma unroll
        for (int k = 0; k < kLdsEdgeChunk; ++k) {
            if (k < cnt) {
                const uint32_t w = (uint32_t)ew[k];
                const uint32_t c = w & 0x1FFFFFu;
                const int jv = (int)w >> 24;
                const int t = ((sh_sp[c >> 5] >> (c & 31)) & 1u) ? jv : -jv;
                acc += (uint64_t)(uint32_t)(t + 128) << ((w >> 17) & 0x30u);
            }
        }
        S0 = (int)(acc & 0xFFFFu) - 128 * (rpv[1] - rpv[0]);
        S1 = (int)((acc >> 16) & 0xFFFFu) - 128 * (rpv[2] - rpv[1]);
        S2 = (int)((acc >> 32) & 0xFFFFu) - 128 * (rpv[3] - rpv[2]);
        S3 = (int)((acc >> 48) & 0xFFFFu) - 128 * (rpv[4] - rpv[3]);
    } else if (active) {
        // longer edge ranges: window after window, each edge assigned to its
        // vertex by the row bounds
        for (int base = rpv[0]; base <= last; base += kLdsEdgeChunk) {
            if (base != rpv[0]) lds_edge_window(d.cj[half], base, ew);
#pragma unroll
            for (int k = 0; k < kLdsEdgeChunk; ++k) {
                const int e = base + k;
                const int c = ew[k] & 0x1FFFFF;
                const int sv = ((sh_sp[c >> 5] >> (c & 31)) & 1u) ? 1 : -1;
                const int t = e <= last ? (ew[k] >> 24) * sv : 0;
                S0 += e < rpv[1] ? t : 0;
                S1 += (e >= rpv[1] && e < rpv[2]) ? t : 0;
                S2 += (e >= rpv[2] && e < rpv[3]) ? t : 0;
                S3 += (e >= rpv[3]) ? t : 0;
            }
        }
    }
    // 6. thresholds, the new spins and their packed copy
    const int Sv[4] = {S0, S1, S2, S3};
    uint32_t up = 0;
    int e_acc = 0;
    if (active) {
        const uint32_t u[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int key = ((Sv[j] + smax) * 2 + (own[j] > 0)) * ncls + cl[j];
            const uint64_t T = lut_lds ? sh_lut[key] : d.lut[key];
            if (v0 + j < n && (uint64_t)u[j] < T) up |= 1u << j;
            if (OBS && v0 + j < n) {
                e_acc += own[j] * Sv[j];
                if (own[j] > 0) atomicAdd(&sh_plus[cl[j] * pcopies + (tid & (pcopies - 1))], 1);
            }
        }
        up |= (fzw >> (v0 & 31)) & 0xFu;
    }
    // the observables first: their atomics are then in flight with the
    // stores instead of after them
    if (OBS) {
        int64_t *lg = log_part(d, slot, blockIdx.x);
        const int lane = tid & 63, wv = tid >> 6;
        e_acc = wave_sum(e_acc);
        if (lane == 0) sh_e[wv] = e_acc;
        __syncthreads();
        if (tid == 0) {
            long long se = 0;
            for (int i = 0; i < kLdsGraphBlock / 64; ++i) se += sh_e[i];
            if (se) atomicAdd((unsigned long long *)&lg[0], (unsigned long long)se);
        }
        for (int i = tid; i < ncls; i += kLdsGraphBlock) {
            int v = 0;
            for (int c = 0; c < pcopies; ++c) v += sh_plus[i * pcopies + c];
            if (v) atomicAdd((unsigned long long *)&lg[1 + i], (unsigned long long)v);
        }
    }
    // stores through the global address space (flat stores would also
    // count against the LDS wait counter)
    if (!BP && active) {
        uint32_t packed = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) packed |= (((up >> j) & 1u) ? 0x01u : 0xFFu) << (8 * j);
        if (v0 + 3 < n) {
            gst<uint32_t>(out, q4, packed);
        } else {
            for (int j = 0; j < 4 && v0 + j < n; ++j) gst<int8_t>(out, v0 + j, (int8_t)(packed >> (8 * j)));
        }
    }
    // packed word of 32 vertices: the eight lanes' 4-bit pieces OR-ed into
    // the group's last lane by row shifts (DPP, no LDS traffic)
    {
        uint32_t val = (active ? up : 0u) << (4 * (q4 & 7));
        val |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)val, 0x111, 0xF, 0xF, true);   // row_shr:1
        val |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)val, 0x112, 0xF, 0xF, true);   // row_shr:2
        val |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)val, 0x114, 0xF, 0xF, true);   // row_shr:4
        if ((q4 & 7) == 7 && 4 * (q4 & ~7) < n) gst<uint32_t>(bits_out, q4 >> 3, val);
    }
}

// mirror[idx] = the configuration spin[idx] of an int8 graph chain, packed
// (one word of 32 vertices per lane); chains without a mirror are skipped
__global__ __launch_bounds__(256) void k_pack_mirror(const ChainDesc *__restrict__ descs, int idx) {
    const ChainDesc &d = descs[blockIdx.y];
    uint32_t *mir = d.mirror[idx];
    if (!mir || d.format == FMT_BITPACKED) return;
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = d.n;
    if (w >= ((n + 31) >> 5)) return;
    const int8_t *sp = (const int8_t *)d.spin[idx];
    uint32_t bits = 0;
    const int v0 = 32 * w;
    if (v0 + 31 < n) {
        const uint4 *p = (const uint4 *)(sp + v0);
        const uint4 a = p[0], b = p[1];
        const uint32_t x[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) bits |= (((x[k] >> (8 * j)) & 0xFFu) == 1u ? 1u : 0u) << (4 * k + j);
    } else {
        for (int j = 0; v0 + j < n; ++j) bits |= (sp[v0 + j] > 0 ? 1u : 0u) << j;
    }
    mir[w] = bits;
}

// ELL variant (couplings +-1, at most 4 neighbours): a lane loads the slot
// records of its 4 vertices as one 16-byte load per slot, gathers every
// neighbour spin at once (empty slots point to the vertex itself) and keeps
// those of the half being updated.  Two dependent memory levels instead of
// three (no row pointers).
template <bool OBS, int K, bool BP>
__global__ __launch_bounds__(256) void k_graph_ell(const ChainDesc *__restrict__ descs, StepArgs sa) {
    const ChainDesc &d = descs[blockIdx.y];
    const uint32_t s = step_s(sa);
    const int bufp = (int)(s & 1u);
    const int half = bufp ^ d.rev;
    const uint32_t want = (uint32_t)(half + 1);
    const int slot = OBS ? step_slot(sa, s) : 0;
    const int n = d.n;
    const int q4 = blockIdx.x * blockDim.x + threadIdx.x;
    const int v0 = q4 * 4;
    const void *__restrict__ in = d.spin[bufp];
    void *__restrict__ out = d.spin[bufp ^ 1];
    const uint32_t *__restrict__ ell = d.ell;
    const int64_t stride = d.ell_stride;
    const uint8_t *__restrict__ cls = d.cls;
    const int ncls = d.ncls, smax = d.smax;
    int e_acc = 0;
    __shared__ uint64_t sh_lut[kLdsLut];
    const int nlut = (2 * smax + 1) * 2 * ncls;
    const bool lut_lds = nlut <= kLdsLut;
    if (lut_lds) {
        for (int i = threadIdx.x; i < nlut; i += blockDim.x) sh_lut[i] = d.lut[i];
    }
    extern __shared__ int sh_plus[];
    if (OBS) {
        for (int i = threadIdx.x; i < ncls; i += blockDim.x) sh_plus[i] = 0;
    }
    __syncthreads();
    uint32_t up = 0;
    if (v0 < n) {
        const bool full = v0 + 3 < n;
        uint4 rec[K];
#pragma unroll
        for (int k = 0; k < K; ++k) rec[k] = *(const uint4 *)(ell + k * stride + v0);
        int own[4], cl[4];
        graph_own4<BP>(in, v0, n, full, own);
        if (full) {
            const uint32_t c4 = *(const uint32_t *)(cls + v0);
#pragma unroll
            for (int j = 0; j < 4; ++j) cl[j] = (int)((c4 >> (8 * j)) & 0xFFu);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) cl[j] = v0 + j < n ? cls[v0 + j] : 0;
        }
        const U4 r = philox10_c0((uint32_t)q4,
                                 philox10_shared(s, d.replica, kGraphStream, (uint32_t)d.seed,
                                                 (uint32_t)(d.seed >> 32)),
                                 (uint32_t)d.seed, (uint32_t)(d.seed >> 32));
        int sv[K][4];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            sv[k][0] = graph_spin<BP>(in, (int)(rec[k].x & 0x1FFFFFFFu));
            sv[k][1] = graph_spin<BP>(in, (int)(rec[k].y & 0x1FFFFFFFu));
            sv[k][2] = graph_spin<BP>(in, (int)(rec[k].z & 0x1FFFFFFFu));
            sv[k][3] = graph_spin<BP>(in, (int)(rec[k].w & 0x1FFFFFFFu));
        }
        int Sv[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t e[4] = {rec[k].x, rec[k].y, rec[k].z, rec[k].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int t = (int)(e[j] >> 31) ? -sv[k][j] : sv[k][j];
                Sv[j] += ((e[j] >> 29) & 3u) == want ? t : 0;
            }
        }
        const uint32_t u[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int key = ((Sv[j] + smax) * 2 + (own[j] > 0)) * ncls + cl[j];
            const uint64_t T = lut_lds ? sh_lut[key] : d.lut[key];
            if (v0 + j < n && (uint64_t)u[j] < T) up |= 1u << j;
            if (OBS && v0 + j < n) {
                e_acc += own[j] * Sv[j];
                if (own[j] > 0) atomicAdd(&sh_plus[cl[j]], 1);
            }
        }
    }
    if (v0 < n) up |= frozen4(d, v0);
    graph_store4<BP>(out, q4, n, up);
    if (OBS && blockIdx.x < (unsigned)((n + 4 * blockDim.x - 1) / (4 * blockDim.x))) {
        int64_t *lg = log_part(d, slot, blockIdx.x);
        __shared__ int sh_e[16];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        e_acc = wave_sum(e_acc);
        if (lane == 0) sh_e[wv] = e_acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            long long se = 0;
            for (int i = 0; i < (int)((blockDim.x + 63) >> 6); ++i) se += sh_e[i];
            if (se) atomicAdd((unsigned long long *)&lg[0], (unsigned long long)se);
        }
        for (int i = threadIdx.x; i < ncls; i += blockDim.x)
            if (sh_plus[i]) atomicAdd((unsigned long long *)&lg[1 + i], (unsigned long long)sh_plus[i]);
    }
}

// ------------------------------------------------------------ observables

__global__ __launch_bounds__(256) void k_observe(const ChainDesc *__restrict__ descs, int idx,
                                                 int slot) {
    const ChainDesc &d = descs[blockIdx.y];
    int64_t *lg = log_part(d, slot, blockIdx.x);
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    int e_acc = 0, p_acc = 0;
    bool active_block;
    if (d.kind == KIND_TORUS && d.format == FMT_BITPACKED) {
        const int total = d.L * d.W;
        active_block = blockIdx.x * blockDim.x < (unsigned)total;
        if (gid < total) {
            const uint32_t *sp = (const uint32_t *)d.spin[idx];
            const int r = gid / d.W, wd = gid - r * d.W;
            const uint32_t own = sp[gid];
            uint32_t a, b;
            bp_neighbours(sp, d.L, d.W, r, wd, 0, own, a, b);
            if (d.jneg) bp_jflip(d.jneg, d.L, d.W, r, wd, 0, a, b);
            const uint32_t vm = bp_valid(d.L, d.W, wd);
            e_acc = d.J * (2 * __popc(vm) - 2 * __popc((own ^ a) & vm) - 2 * __popc((own ^ b) & vm));
            if (d.tri) {
                // down-left neighbours: the row below shifted like b
                const int L = d.L, W = d.W, rd = r == 0 ? L - 1 : r - 1;
                const uint32_t as = wd > 0 ? sp[rd * W + wd - 1] : sp[rd * W + W - 1];
                const uint32_t e = (a << 1) | (wd > 0 ? (as >> 31) : ((as >> ((L - 1) & 31)) & 1u));
                e_acc += d.J * (__popc(vm) - 2 * __popc((own ^ e) & vm));
            }
            p_acc = __popc(own & vm);
        }
        if (active_block) block_accumulate2(e_acc, p_acc, lg);
        return;
    }
    if (d.kind == KIND_TORUS) {
        active_block = blockIdx.x * blockDim.x < (unsigned)d.n;
        if (gid < d.n) {
            const int8_t *sp = (const int8_t *)d.spin[idx];
            const int L = d.L, r = gid / L, c = gid - r * L;
            const int own = sp[gid];
            const int rd = r == 0 ? L - 1 : r - 1, cl = c == 0 ? L - 1 : c - 1;
            e_acc = d.J * own * (sp[rd * L + c] * torus_jsign(d.jneg, L, d.W, 0, rd, c) +
                                 sp[r * L + cl] * torus_jsign(d.jneg, L, d.W, 1, r, cl) +
                                 (d.tri ? sp[rd * L + cl] : 0));
            p_acc = own > 0;
        }
        if (active_block) block_accumulate2(e_acc, p_acc, lg);
        return;
    }
    // graph: E_J via the in-half of every vertex, plus counts per class (LDS
    // counters, one atomic per class and block)
    __shared__ int sh_cls[256];
    const int ncls = d.ncls;
    for (int i = threadIdx.x; i < ncls; i += blockDim.x) sh_cls[i] = 0;
    __syncthreads();
    if (gid < d.n) {
        const void *sp = d.spin[idx];
        const bool bp = d.format == FMT_BITPACKED;
        int S = 0;
        for (int e = d.rowptr[0][gid]; e < d.rowptr[0][gid + 1]; ++e)
            S += d.jw[0][e] * (bp ? graph_spin<true>(sp, d.col[0][e]) : graph_spin<false>(sp, d.col[0][e]));
        const int own = bp ? graph_spin<true>(sp, gid) : graph_spin<false>(sp, gid);
        e_acc = own * S;
        if (own > 0) atomicAdd(&sh_cls[d.cls[gid]], 1);
    }
    e_acc = wave_sum(e_acc);
    if ((threadIdx.x & 63) == 0 && e_acc)
        atomicAdd((unsigned long long *)&lg[0], (unsigned long long)(long long)e_acc);
    __syncthreads();
    for (int i = threadIdx.x; i < ncls; i += blockDim.x)
        if (sh_cls[i]) atomicAdd((unsigned long long *)&lg[1 + i], (unsigned long long)sh_cls[i]);
}

// ---------------------------------------------------------------- helpers

__global__ void k_fill_i64(int64_t *p, int64_t count, int64_t value) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

// mode: 0 random, 1 all up, 2 all down
__global__ void k_init(ChainDesc d, void *dst, int mode) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t k0 = (uint32_t)d.seed, k1 = (uint32_t)(d.seed >> 32);
    if (d.kind == KIND_TORUS && d.format == FMT_BITPACKED) {
        const int total = d.L * d.W;
        if (gid >= total) return;
        const uint32_t vm = bp_valid(d.L, d.W, gid % d.W);
        uint32_t v;
        if (mode == 0)
            v = philox10((uint32_t)gid, kInitStep, d.replica, 0u, k0, k1).x;
        else
            v = (mode == 1) ? 0xFFFFFFFFu : 0u;
        ((uint32_t *)dst)[gid] = (v & vm) | frozen_word(d, gid);
        return;
    }
    if (d.kind == KIND_GRAPH && d.format == FMT_BITPACKED) {
        // word gid: vertices 32 gid .. 32 gid + 31, each +1 iff bit 31 of its u
        const int nwords = (d.n + 31) / 32;
        if (gid >= nwords) return;
        uint32_t v = 0;
        for (int b = 0; b < 32; ++b) {
            const int x = 32 * gid + b;
            if (x >= d.n) break;
            bool upx;
            if (mode == 0) {
                const U4 r = philox10((uint32_t)(x >> 2), kInitStep, d.replica, kGraphStream, k0, k1);
                const uint32_t u[4] = {r.x, r.y, r.z, r.w};
                upx = (u[x & 3] >> 31) != 0;
            } else {
                upx = mode == 1;
            }
            if (upx) v |= 1u << b;
        }
        ((uint32_t *)dst)[gid] = v | frozen_word(d, gid);
        return;
    }
    if (gid >= d.n) return;
    int8_t v;
    if (mode == 0) {
        if (d.kind == KIND_TORUS) {
            const int r = gid / d.L, c = gid - r * d.L;
            const uint32_t x = philox10((uint32_t)(r * d.W + (c >> 5)), kInitStep, d.replica, 0u, k0, k1).x;
            v = ((x >> (c & 31)) & 1u) ? 1 : -1;
        } else {
            const U4 r = philox10((uint32_t)(gid >> 2), kInitStep, d.replica, kGraphStream, k0, k1);
            const uint32_t u[4] = {r.x, r.y, r.z, r.w};
            v = (u[gid & 3] >> 31) ? 1 : -1;
        }
    } else {
        v = (mode == 1) ? 1 : -1;
    }
    const int fw = d.kind == KIND_TORUS ? (gid / d.L) * d.W + ((gid % d.L) >> 5) : gid >> 5;
    const int fb = d.kind == KIND_TORUS ? (gid % d.L) & 31 : gid & 31;
    if ((frozen_word(d, fw) >> fb) & 1u) v = 1;
    ((int8_t *)dst)[gid] = v;
}

// -------------------------------------------------------------- launchers

hipError_t launch_fill_i64(int64_t *p, int64_t count, int64_t value, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    const int b = 256;
    const int64_t g = (count + b - 1) / b;
    hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)g), dim3(b), 0, stream, p, count, value);
    return hipGetLastError();
}

hipError_t launch_init(const ChainDesc &d, void *dst, int mode, hipStream_t stream) {
    const int total = d.format != FMT_BITPACKED ? d.n : (d.kind == KIND_TORUS ? d.L * d.W : (d.n + 31) / 32);
    const int b = 256;
    hipLaunchKernelGGL(k_init, dim3((total + b - 1) / b), dim3(b), 0, stream, d, dst, mode);
    return hipGetLastError();
}

static int units_of(const ChainDesc &d) {
    if (d.kind == KIND_TORUS)
        return d.format == FMT_BITPACKED ? ((d.L + kRows - 1) / kRows) * d.W : d.n;
    return (d.n + 3) / 4;
}

hipError_t launch_half_step_grid(const ChainDesc *dev_descs, const ChainDesc *host_descs,
                                 int nchains, const uint32_t *dstate, uint32_t s_add,
                                 uint32_t s_log0, int log_on, bool even, int block,
                                 hipStream_t stream) {
    if (nchains <= 0) return hipSuccess;
    // the chains of one launch share a kind and a format (the runtime groups them)
    const ChainDesc &h0 = host_descs[0];
    int maxu = 0, minu = INT_MAX, fold = 1, maxcls = 1, jpl = 0, aligned = 1;
    for (int i = 0; i < nchains; ++i) {
        maxu = maxu > units_of(host_descs[i]) ? maxu : units_of(host_descs[i]);
        minu = minu < units_of(host_descs[i]) ? minu : units_of(host_descs[i]);
        fold &= host_descs[i].fold3;
        aligned &= host_descs[i].kind == KIND_TORUS && host_descs[i].L % 32 == 0;
        maxcls = maxcls > host_descs[i].ncls ? maxcls : host_descs[i].ncls;
        jpl |= host_descs[i].jneg != nullptr || host_descs[i].frozen != nullptr;
    }
    const bool obs = log_on && even;
    const StepArgs sa{dstate, s_add, s_log0, log_on};
    const int b = block > 0 ? block : 256;
    // the torus kernels split their tail queue over one, two or four
    // wavefronts; 1024 selects the LDS-staged graph kernel
    if (b == kLdsGraphBlock) {
        if (h0.kind != KIND_GRAPH) return hipErrorInvalidValue;
        for (int i = 0; i < nchains; ++i)
            if (!graph_lds_fits(host_descs[i])) return hipErrorInvalidValue;
    } else if (b != 64 && b != 128 && b != 256) {
        return hipErrorInvalidValue;
    }
    const dim3 grid((maxu + b - 1) / b, nchains);
    if (h0.kind == KIND_TORUS && h0.format == FMT_BITPACKED && h0.tri) {
        // the runtime groups triangular tori apart from square ones
        if (fold && aligned && minu == maxu && maxu % b == 0) {
            if (obs) hipLaunchKernelGGL((k_tri_bp<true, true, true, true>), grid, dim3(b), 0, stream, dev_descs, sa);
            else hipLaunchKernelGGL((k_tri_bp<false, true, true, true>), grid, dim3(b), 0, stream, dev_descs, sa);
        } else if (fold && aligned) {
            if (obs) hipLaunchKernelGGL((k_tri_bp<true, true, true>), grid, dim3(b), 0, stream, dev_descs, sa);
            else hipLaunchKernelGGL((k_tri_bp<false, true, true>), grid, dim3(b), 0, stream, dev_descs, sa);
        } else if (obs) { if (fold) hipLaunchKernelGGL((k_tri_bp<true, true>), grid, dim3(b), 0, stream, dev_descs, sa);
                   else hipLaunchKernelGGL((k_tri_bp<true, false>), grid, dim3(b), 0, stream, dev_descs, sa); }
        else { if (fold) hipLaunchKernelGGL((k_tri_bp<false, true>), grid, dim3(b), 0, stream, dev_descs, sa);
               else hipLaunchKernelGGL((k_tri_bp<false, false>), grid, dim3(b), 0, stream, dev_descs, sa); }
    } else if (h0.kind == KIND_TORUS && h0.format == FMT_BITPACKED) {
#define SHAKEN_BP(O, F, JP) hipLaunchKernelGGL((k_torus_bp<O, F, JP>), grid, dim3(b), 0, stream, dev_descs, sa)
        if (jpl) {
            // +-J sign planes or frozen sets (chains without them in the same
            // launch skip them)
            if (obs) { if (fold) SHAKEN_BP(true, true, true); else SHAKEN_BP(true, false, true); }
            else { if (fold) SHAKEN_BP(false, true, true); else SHAKEN_BP(false, false, true); }
        } else if (fold && aligned && minu == maxu && maxu % b == 0) {
            // every lane of the grid is a strip of every chain
            if (obs) hipLaunchKernelGGL((k_torus_bp<true, true, false, true, true>), grid, dim3(b), 0, stream, dev_descs, sa);
            else hipLaunchKernelGGL((k_torus_bp<false, true, false, true, true>), grid, dim3(b), 0, stream, dev_descs, sa);
        } else if (fold && aligned) {
            if (obs) hipLaunchKernelGGL((k_torus_bp<true, true, false, true>), grid, dim3(b), 0, stream, dev_descs, sa);
            else hipLaunchKernelGGL((k_torus_bp<false, true, false, true>), grid, dim3(b), 0, stream, dev_descs, sa);
        } else {
            if (obs) { if (fold) SHAKEN_BP(true, true, false); else SHAKEN_BP(true, false, false); }
            else { if (fold) SHAKEN_BP(false, true, false); else SHAKEN_BP(false, false, false); }
        }
#undef SHAKEN_BP
    } else if (h0.kind == KIND_TORUS) {
        if (obs) hipLaunchKernelGGL((k_torus_i8<true>), grid, dim3(b), 0, stream, dev_descs, sa);
        else hipLaunchKernelGGL((k_torus_i8<false>), grid, dim3(b), 0, stream, dev_descs, sa);
    } else if (b == kLdsGraphBlock) {
        // the three-slot layout where every chain of the launch has it
        bool e3 = true;
        for (int i = 0; i < nchains; ++i) e3 = e3 && host_descs[i].e3[0] != nullptr;
#define SHAKEN_LDS(O, BPF, E) hipLaunchKernelGGL((k_graph_lds<O, BPF, E>), grid, dim3(b), 0, stream, dev_descs, sa)
        if (h0.format == FMT_BITPACKED) {
            if (e3) { if (obs) SHAKEN_LDS(true, true, true); else SHAKEN_LDS(false, true, true); }
            else { if (obs) SHAKEN_LDS(true, true, false); else SHAKEN_LDS(false, true, false); }
        } else {
            if (e3) { if (obs) SHAKEN_LDS(true, false, true); else SHAKEN_LDS(false, false, true); }
            else { if (obs) SHAKEN_LDS(true, false, false); else SHAKEN_LDS(false, false, false); }
        }
#undef SHAKEN_LDS
    } else {
        const size_t shm = obs ? sizeof(int) * (size_t)maxcls : 0;
        int ellk = host_descs[0].ell_k;
        for (int i = 0; i < nchains; ++i)
            if (host_descs[i].ell_k != ellk || !host_descs[i].ell) ellk = 0;
#define SHAKEN_ELL(KK, BPF)                                                                            \
    if (obs) hipLaunchKernelGGL((k_graph_ell<true, KK, BPF>), grid, dim3(b), shm, stream, dev_descs, sa); \
    else hipLaunchKernelGGL((k_graph_ell<false, KK, BPF>), grid, dim3(b), 0, stream, dev_descs, sa);
#define SHAKEN_GRAPH(BPF)                                                                              \
    if (ellk == 1) { SHAKEN_ELL(1, BPF) }                                                              \
    else if (ellk == 2) { SHAKEN_ELL(2, BPF) }                                                         \
    else if (ellk == 3) { SHAKEN_ELL(3, BPF) }                                                         \
    else if (ellk == 4) { SHAKEN_ELL(4, BPF) }                                                         \
    else if (obs) hipLaunchKernelGGL((k_graph<true, BPF>), grid, dim3(b), shm, stream, dev_descs, sa); \
    else hipLaunchKernelGGL((k_graph<false, BPF>), grid, dim3(b), 0, stream, dev_descs, sa);
        if (h0.format == FMT_BITPACKED) { SHAKEN_GRAPH(true) }
        else { SHAKEN_GRAPH(false) }
#undef SHAKEN_GRAPH
#undef SHAKEN_ELL
    }
    return hipGetLastError();
}

bool graph_lds_fits(const ChainDesc &d) {
    return d.kind == KIND_GRAPH && d.n <= 32 * kLdsGraphWords && d.cj[0] && (d.format == FMT_BITPACKED || d.mirror[0]);
}

int graph_lds_max_words() { return kLdsGraphWords; }

hipError_t launch_pack_mirror(const ChainDesc *dev_descs, const ChainDesc *host_descs, int nchains, int idx,
                              hipStream_t stream) {
    int maxw = 0;
    for (int i = 0; i < nchains; ++i)
        if (host_descs[i].mirror[idx] && host_descs[i].format != FMT_BITPACKED)
            maxw = maxw > ((host_descs[i].n + 31) >> 5) ? maxw : ((host_descs[i].n + 31) >> 5);
    if (maxw == 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(k_pack_mirror, dim3((maxw + b - 1) / b, nchains), dim3(b), 0, stream, dev_descs, idx);
    return hipGetLastError();
}

// advance the device half-step counter by `by` (end of a replayed graph)
__global__ void k_advance(uint32_t *dstate, uint32_t by) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dstate[0] += by;
}

__global__ void k_set_state(uint32_t *d, uint32_t a, uint32_t b) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        d[0] = a;
        d[1] = b;
    }
}

hipError_t launch_set_state(uint32_t *d, uint32_t a, uint32_t b, hipStream_t stream) {
    hipLaunchKernelGGL(k_set_state, dim3(1), dim3(64), 0, stream, d, a, b);
    return hipGetLastError();
}

hipError_t launch_advance(uint32_t *dstate, uint32_t by, hipStream_t stream) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, stream, dstate, by);
    return hipGetLastError();
}

hipError_t launch_observe(const ChainDesc *dev_descs, const ChainDesc *host_descs, int nchains,
                          int idx, int slot, hipStream_t stream) {
    if (nchains <= 0) return hipSuccess;
    int maxu = 0;
    for (int i = 0; i < nchains; ++i) {
        const ChainDesc &d = host_descs[i];
        const int u = (d.kind == KIND_TORUS && d.format == FMT_BITPACKED) ? d.L * d.W : d.n;
        maxu = maxu > u ? maxu : u;
    }
    const int b = 256;
    hipLaunchKernelGGL(k_observe, dim3((maxu + b - 1) / b, nchains), dim3(b), 0, stream, dev_descs, idx, slot);
    return hipGetLastError();
}

}  // namespace shaken
