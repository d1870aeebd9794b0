// Host runtime and C ABI of libshaken: argument validation, the layout of the
// oriented graph (in-half and out-half CSR), the threshold tables, chain
// contexts and the batch executor.  Every half-step runs in the HIP kernels of
// kernels.hip; this file only prepares data and enqueues launches.
#include "shaken.h"
#include "shaken_internal.hpp"
#include "noalloc.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

using namespace shaken;

namespace {

thread_local std::string g_err;

shaken_status fail(shaken_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(e_ == hipErrorOutOfMemory ? SHAKEN_ENOMEM : SHAKEN_EDEVICE,           \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                   \
    } while (0)

#define CHK(expr)                                                                             \
    do {                                                                                      \
        shaken_status s_ = (expr);                                                            \
        if (s_ != SHAKEN_OK) return s_;                                                       \
    } while (0)

// Make the context's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (dev >= 0 && dev != prev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

template <class T>
shaken_status dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? SHAKEN_ENOMEM : SHAKEN_EDEVICE,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return SHAKEN_OK;
}

template <class T>
void dfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

// ---------------------------------------------------------------- thresholds

// Local field h = S + q sigma + lambda, evaluated left to right in double.
double field_h(int64_t S, int sigma, double q, double lam) {
    double h = (double)S;
    h = h + q * (double)sigma;
    h = h + lam;
    return h;
}

// T in [0, 2^32] with P(+1) = T / 2^32 ~ 1 / (1 + exp(-2 beta h)) (the
// heat-bath factor exp(beta h s') / (2 cosh(beta h)) of section 2).  The small
// tail e/(1+e) is rounded down and mirrored, so T(h) + T(-h) = 2^32 exactly.
uint64_t threshold_T(double h, double beta) {
    const double e = std::exp(-((2.0 * beta) * std::fabs(h)));
    const double p = e / (1.0 + e);
    const uint64_t t = (uint64_t)std::floor(p * 4294967296.0);
    return (h >= 0.0) ? ((uint64_t)1 << 32) - t : t;
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

}  // namespace

namespace shaken {
shaken_status set_error(shaken_status s, const char *msg) {
    g_err = msg ? msg : "";
    return s;
}
}  // namespace shaken

// ------------------------------------------------------------------ context

struct shaken_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    int kind = KIND_TORUS;
    int format = FMT_BITPACKED;
    int L = 0, W = 0, n = 0;
    int64_t m = 0;
    double q = 0, beta = 0;
    uint64_t seed = 0;
    uint32_t replica = 0;
    int J = 1;  // uniform torus coupling
    std::vector<double> lam;
    std::vector<int64_t> class_size;
    bool lam2_int = true;
    std::vector<int64_t> lam2;  // 2*lambda as integers (valid iff lam2_int)
    int smax = 0;
    int maxdeg = 0;
    std::vector<uint64_t> lut;
    uint32_t s = 0;  // half-step counter; configuration at s is in spin[s & 1]
    void *spin[2] = {nullptr, nullptr};
    uint64_t *lut_dev = nullptr;
    int32_t *rp[2] = {nullptr, nullptr};
    int32_t *col[2] = {nullptr, nullptr};
    int8_t *jw[2] = {nullptr, nullptr};
    uint8_t *cls_dev = nullptr;
    uint32_t *ell_dev = nullptr;
    uint64_t *pell_dev = nullptr;
    uint32_t *jneg_dev = nullptr;  // +-J torus sign planes (2 x L x W words)
    uint32_t *frozen_dev = nullptr;  // frozen set B as bits (layout of the bit-packed spins)
    uint32_t *mirror[2] = {nullptr, nullptr};  // packed copies of int8 graph spins (LDS-staged kernel)
    int32_t *cj[2] = {nullptr, nullptr};       // edge words of the LDS-staged kernel (index, row slot, J)
    uint32_t *e3[2] = {nullptr, nullptr};      // its three slots per vertex (half-degrees <= 3, one |J|)
    int j0 = 0;                                // that common |J|
    bool tri = false;                // triangular torus
    std::vector<uint8_t> frozen_host;  // per site, nonzero = frozen
    int ell_k = 0;
    int64_t ell_stride = 0;
    int64_t *log_dev = nullptr;
    int64_t log_cap = 0;  // slots
    int64_t *obs_dev = nullptr;
    bool lut_stale = false;  // a batch changed beta/q: re-upload before a call of its own
    // degree statistics over the sites (schedule network features): mean of
    // in-half + out-half size, root mean square of in-half - out-half size
    double deg_mean = 0, deg_spread = 0;
    ChainDesc hd{};
    ChainDesc *dd = nullptr;
    // the same descriptor with its log pointer at the device's fixed buffer
    // (shaken_sweep_noalloc); kept in step with dd by upload_desc
    ChainDesc *dd_static = nullptr;
    int64_t *scratch = nullptr;  // device address of that buffer (not owned)
    int block = 256;

    size_t spin_bytes() const {
        if (format == FMT_BITPACKED) return (kind == KIND_TORUS ? (size_t)L * W : ((size_t)n + 31) / 32) * 4;
        return (size_t)n;
    }
    int64_t nvals() const { return 1 + (int64_t)lam.size(); }               // values per slot
    int64_t line() const { return (nvals() + 15) / 16 * 16; }                 // one partial line
    int64_t stride() const { return (int64_t)kLogParts * line(); }            // int64 per slot
};

namespace {

void release(shaken_ctx *c) {
    dfree(c->spin[0]);
    dfree(c->spin[1]);
    dfree(c->lut_dev);
    for (int h = 0; h < 2; ++h) {
        dfree(c->rp[h]);
        dfree(c->col[h]);
        dfree(c->jw[h]);
        dfree(c->cj[h]);
        dfree(c->e3[h]);
    }
    dfree(c->cls_dev);
    dfree(c->ell_dev);
    dfree(c->pell_dev);
    dfree(c->jneg_dev);
    dfree(c->frozen_dev);
    dfree(c->mirror[0]);
    dfree(c->mirror[1]);
    dfree(c->log_dev);
    dfree(c->obs_dev);
    dfree(c->dd);
    dfree(c->dd_static);
}

size_t bit_words(const shaken_ctx *c) {
    if (c->kind == KIND_TORUS) return (size_t)c->L * c->W;
    return ((size_t)c->n + 31) / 32;
}

// Build the host threshold table and the bit-packed torus class tables.
void build_tables(shaken_ctx *c) {
    const int ncls = (int)c->lam.size();
    const int nS = 2 * c->smax + 1;
    c->lut.assign((size_t)nS * 2 * ncls, 0);
    for (int S = -c->smax; S <= c->smax; ++S)
        for (int sb = 0; sb < 2; ++sb)
            for (int k = 0; k < ncls; ++k) {
                const double h = field_h(S, sb ? 1 : -1, c->q, c->lam[k]);
                c->lut[((size_t)(S + c->smax) * 2 + sb) * ncls + k] = threshold_T(h, c->beta);
            }
    if (c->kind == KIND_TORUS) {
        // classes j = n_plus + k (own spin +1), k = 3 (square: 2 neighbours per
        // half) or 4 (triangular: 3 neighbours)
        const int nb = c->tri ? 3 : 2, ncl = 2 * (nb + 1);
        uint32_t sgn = 0;
        uint64_t Tc[8];
        for (int j = 0; j < ncl; ++j) {
            const int nplus = j % (nb + 1), cb = j / (nb + 1);
            const int64_t S = (int64_t)c->J * (2 * nplus - nb);
            const double h = field_h(S, cb ? 1 : -1, c->q, c->lam[0]);
            const uint64_t T = threshold_T(h, c->beta);
            const uint64_t t = (h >= 0.0) ? ((uint64_t)1 << 32) - T : T;
            Tc[j] = T;
            c->hd.tsmall[j] = (uint32_t)t;
            if (h >= 0.0) sgn |= 1u << j;
        }
        // Folded table: mirror classes j and ncl-1-j (the neighbour count
        // reversed, the site flipped) with equal t and opposite signs.  A
        // class with T = 2^31 has t = 2^31 and decides alike with either sign,
        // so it takes the sign opposite to its mirror's.
        const uint32_t *t = c->hd.tsmall;
        const uint64_t half = (uint64_t)1 << 31;
        bool fold = true;
        for (int j = 0; j < ncl / 2; ++j) {
            const int k = ncl - 1 - j;
            fold = fold && t[j] == t[k];
            if (((sgn >> j) ^ (sgn >> k)) & 1u) continue;
            if (Tc[k] == half)
                sgn ^= 1u << k;
            else if (Tc[j] == half)
                sgn ^= 1u << j;
            else
                fold = false;
        }
        c->hd.sgn = sgn;
        c->hd.fold3 = fold ? 1 : 0;
    }
}

// copy the host descriptor to the device: dd as it is, dd_static with the log
// pointed at the fixed buffer (synchronises the stream)
shaken_status upload_desc(shaken_ctx *c) {
    ChainDesc ds = c->hd;
    ds.log = c->scratch;
    HIPCHK(hipMemcpyAsync(c->dd, &c->hd, sizeof(ChainDesc), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->dd_static, &ds, sizeof(ChainDesc), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return SHAKEN_OK;
}

shaken_status upload_tables(shaken_ctx *c) {
    HIPCHK(hipMemcpyAsync(c->lut_dev, c->lut.data(), c->lut.size() * sizeof(uint64_t),
                          hipMemcpyHostToDevice, c->stream));
    return upload_desc(c);
}

// refresh the device tables of a chain whose parameters a batch changed
shaken_status refresh_if_stale(shaken_ctx *c) {
    if (!c->lut_stale) return SHAKEN_OK;
    c->lut_stale = false;
    return upload_tables(c);
}

void refresh_desc_spins(shaken_ctx *c) {
    c->hd.spin[0] = c->spin[0];
    c->hd.spin[1] = c->spin[1];
    c->hd.log = c->log_dev;
}

shaken_status ensure_log(shaken_ctx *c, int64_t slots) {
    if (slots <= c->log_cap) return SHAKEN_OK;
    dfree(c->log_dev);
    c->log_cap = 0;
    CHK(dalloc(&c->log_dev, (size_t)(slots * c->stride())));
    c->log_cap = slots;
    refresh_desc_spins(c);
    return upload_desc(c);
}

// pack / unpack host int8 <-> bit-packed rows (rows x cols spins, W words per
// row; the torus is L x L, a graph one row of n)
void pack_rows(const int8_t *in, int rows, int cols, int W, std::vector<uint32_t> &out) {
    out.assign((size_t)rows * W, 0u);
    for (int r = 0; r < rows; ++r)
        for (int c = 0; c < cols; ++c)
            if (in[(size_t)r * cols + c] > 0) out[(size_t)r * W + (c >> 5)] |= 1u << (c & 31);
}

void unpack_rows(const std::vector<uint32_t> &in, int rows, int cols, int W, int8_t *out) {
    for (int r = 0; r < rows; ++r)
        for (int c = 0; c < cols; ++c)
            out[(size_t)r * cols + c] = ((in[(size_t)r * W + (c >> 5)] >> (c & 31)) & 1u) ? 1 : -1;
}

void unpack_torus(const std::vector<uint32_t> &in, int L, int W, int8_t *out) { unpack_rows(in, L, L, W, out); }

// the spins of a context as bit-packed rows: (rows, cols, words per row)
void spin_rows(const shaken_ctx *c, int &rows, int &cols, int &W) {
    rows = c->kind == KIND_TORUS ? c->L : 1;
    cols = c->kind == KIND_TORUS ? c->L : c->n;
    W = c->kind == KIND_TORUS ? c->W : (c->n + 31) / 32;
}

// Convert a device log (slots x stride) to H and M per slot.
// raw holds `parts` partial lines per slot (kLogParts for the grid kernels, 1
// for the persistent kernel, which owns a chain's whole slot).
// raw: slots x parts lines of `ln` int64 (ln = 0: the context's line width)
void convert_log(const shaken_ctx *c, const std::vector<int64_t> &raw, int64_t slots, int parts,
                 int64_t *H, int64_t *M, int64_t *EJ_out = nullptr, int64_t ln = 0) {
    if (ln == 0) ln = c->line();
    const int64_t st = parts * ln;
    auto val = [&](int64_t t, int64_t v) {
        int64_t a = 0;
        for (int p = 0; p < parts; ++p) a += raw[t * st + p * ln + v];
        return a;
    };
    for (int64_t t = 0; t < slots; ++t) {
        const int64_t EJ = val(t, 0);
        int64_t m = 0, l2 = 0;
        for (size_t k = 0; k < c->lam.size(); ++k) {
            const int64_t mk = 2 * val(t, 1 + (int64_t)k) - c->class_size[k];
            m += mk;
            if (c->lam2_int) l2 += c->lam2[k] * mk;
        }
        if (H) H[t] = -EJ - l2;
        if (M) M[t] = m;
        if (EJ_out) EJ_out[t] = EJ;
    }
}

// Validate and lay out an oriented graph as in-half and out-half CSR.
shaken_status build_graph(shaken_ctx *c, const shaken_graph *g, const int8_t *J, bool split,
                          std::vector<int32_t> rp[2], std::vector<int32_t> col[2],
                          std::vector<int8_t> jw[2]) {
    const int n = g->n;
    const int64_t m = g->m;
    if (n < 1) return fail(SHAKEN_EINVAL, "graph: n must be >= 1");
    if (m < 0 || m > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(SHAKEN_EINVAL, "graph: m out of range");
    if (m > 0 && (!g->src || !g->dst)) return fail(SHAKEN_EINVAL, "graph: src/dst are NULL");
    std::vector<int64_t> key((size_t)m);
    for (int64_t e = 0; e < m; ++e) {
        const int32_t a = g->src[e], b = g->dst[e];
        if (a < 0 || a >= n || b < 0 || b >= n)
            return fail(SHAKEN_EINVAL, "graph: vertex id out of range at edge " + std::to_string(e));
        if (a == b) return fail(SHAKEN_EINVAL, "graph: self-loop at edge " + std::to_string(e));
        // the generalised split keys the oriented pair, Definition 2.1 the undirected one
        key[e] = split ? (int64_t)a * n + b : (int64_t)std::min(a, b) * n + std::max(a, b);
    }
    std::sort(key.begin(), key.end());
    for (int64_t e = 1; e < m; ++e)
        if (key[e] == key[e - 1])
            return fail(SHAKEN_EINVAL, split ? "graph: an oriented edge is given twice"
                                             : "graph: an edge is given twice (the graph must be simple; "
                                               "SHAKEN_GRAPH_SPLIT allows both orientations of a pair)");
    // half 0: in-half (row = head dst, entries = tails src); half 1: out-half
    for (int h = 0; h < 2; ++h) {
        rp[h].assign((size_t)n + 1, 0);
        const int32_t *row = (h == 0) ? g->dst : g->src;
        const int32_t *other = (h == 0) ? g->src : g->dst;
        for (int64_t e = 0; e < m; ++e) rp[h][row[e] + 1]++;
        for (int v = 0; v < n; ++v) rp[h][v + 1] += rp[h][v];
        col[h].assign((size_t)m, 0);
        jw[h].assign((size_t)m, 1);
        std::vector<int32_t> pos(rp[h].begin(), rp[h].end() - 1);
        for (int64_t e = 0; e < m; ++e) {
            const int32_t p = pos[row[e]]++;
            col[h][p] = other[e];
            jw[h][p] = J ? J[e] : (int8_t)1;
        }
    }
    int64_t smax = 0;
    int maxdeg = 0;
    for (int h = 0; h < 2; ++h)
        for (int v = 0; v < n; ++v) {
            int64_t a = 0;
            for (int32_t e = rp[h][v]; e < rp[h][v + 1]; ++e) a += std::abs((int)jw[h][e]);
            smax = std::max(smax, a);
            maxdeg = std::max(maxdeg, rp[h][v + 1] - rp[h][v]);
        }
    if (smax > (1 << 22)) return fail(SHAKEN_EINVAL, "graph: coupling sums too large for the threshold table");
    c->smax = (int)smax;
    c->maxdeg = maxdeg;
    return SHAKEN_OK;
}

struct HostLayout {
    std::vector<uint8_t> cls_host;
    std::vector<int32_t> rp[2], col[2];
    std::vector<int8_t> jw[2];
    std::vector<uint32_t> ell;  // slot-major, ell_k * ell_stride entries
    std::vector<uint64_t> pell; // packed record per vertex, ell_stride entries
    std::vector<uint32_t> jneg; // +-J torus: sign planes of J(x, x_up) and J(x, x_right)
    std::vector<uint32_t> frozen; // frozen set B, bits laid out like bit-packed spins
    int ell_k = 0;
    int64_t ell_stride = 0;
};

// ELL layout when every coupling is +-1 and every vertex has at most 4
// neighbours: slot k of vertex v holds the neighbour index, the half it belongs
// to (1 = in-half, 2 = out-half) and the sign of J; empty slots point to v
// itself with half 0.  Returns false when the layout does not apply.
bool build_ell(int n, HostLayout &hl) {
    if (n >= (1 << 29)) return false;
    int kmax = 0;
    for (int v = 0; v < n; ++v) {
        const int deg = (hl.rp[0][v + 1] - hl.rp[0][v]) + (hl.rp[1][v + 1] - hl.rp[1][v]);
        kmax = std::max(kmax, deg);
    }
    if (kmax == 0 || kmax > 4) return false;
    for (int h = 0; h < 2; ++h)
        for (int8_t j : hl.jw[h])
            if (j != 1 && j != -1) return false;
    hl.ell_k = kmax;
    hl.ell_stride = ((int64_t)n + 3) / 4 * 4;
    hl.ell.assign((size_t)kmax * hl.ell_stride, 0u);
    for (int64_t v = 0; v < hl.ell_stride; ++v)
        for (int k = 0; k < kmax; ++k) hl.ell[k * hl.ell_stride + v] = (uint32_t)std::min<int64_t>(v, n - 1);
    for (int v = 0; v < n; ++v) {
        int k = 0;
        for (int h = 0; h < 2; ++h)
            for (int32_t e = hl.rp[h][v]; e < hl.rp[h][v + 1]; ++e, ++k)
                hl.ell[k * hl.ell_stride + v] = (uint32_t)hl.col[h][e] | ((uint32_t)(h + 1) << 29) |
                                                (hl.jw[h][e] < 0 ? 0x80000000u : 0u);
    }
    return true;
}

// Packed record per vertex for the persistent kernel (layout in ChainDesc::pell):
// needs the ELL layout with at most 3 slots, n <= 65536 and classes < 16.
bool build_pell(int n, HostLayout &hl) {
    if (hl.ell_k == 0 || hl.ell_k > 3 || n > 65536) return false;
    for (int v = 0; v < n; ++v)
        if (hl.cls_host[v] >= 16) return false;
    hl.pell.assign((size_t)hl.ell_stride, 0ull);
    for (int v = 0; v < n; ++v) {
        uint64_t r = (uint64_t)hl.cls_host[v] << 57;
        int k = 0;
        for (int h = 0; h < 2; ++h)
            for (int32_t e = hl.rp[h][v]; e < hl.rp[h][v + 1]; ++e, ++k) {
                r |= (uint64_t)(uint32_t)hl.col[h][e] << (16 * k);
                r |= 1ull << (48 + 3 * h + k);
                r |= (uint64_t)(hl.jw[h][e] < 0) << (54 + k);
            }
        hl.pell[v] = r;
    }
    return true;
}

// Host phase of shaken_init: validation, layout and tables; touches no device.
shaken_status init_host(shaken_ctx *c, const shaken_graph *g, const int8_t *J,
                        const shaken_field *lambda, const shaken_opts *o, HostLayout &hl) {
    std::vector<uint8_t> &cls_host = hl.cls_host;
    std::vector<int32_t> *rp = hl.rp, *col = hl.col;
    std::vector<int8_t> *jw = hl.jw;
    // field
    if (lambda) {
        if (lambda->n_classes < 1 || lambda->n_classes > 256 || !lambda->value)
            return fail(SHAKEN_EINVAL, "field: n_classes must be in [1, 256] with values");
        c->lam.assign(lambda->value, lambda->value + lambda->n_classes);
        for (double v : c->lam)
            if (!std::isfinite(v)) return fail(SHAKEN_EINVAL, "field: non-finite lambda");
    } else {
        c->lam.assign(1, 0.0);
    }
    c->lam2.assign(c->lam.size(), 0);
    c->lam2_int = true;
    for (size_t k = 0; k < c->lam.size(); ++k) {
        const double v2 = 2.0 * c->lam[k];
        if (v2 != std::floor(v2) || std::fabs(v2) > 1e15)
            c->lam2_int = false;
        else
            c->lam2[k] = (int64_t)v2;
    }
    if (g->kind == SHAKEN_TORUS || g->kind == SHAKEN_TRIANGULAR) {
        const bool tri = g->kind == SHAKEN_TRIANGULAR;
        c->tri = tri;
        if (g->L < 3 || g->L > 32768) return fail(SHAKEN_EINVAL, "torus: L must be in [3, 32768]");
        if (o->flags & ~SHAKEN_ORDER_REVERSED)
            return fail(SHAKEN_EINVAL, "SHAKEN_GRAPH_SPLIT, SHAKEN_GRAPH_LDS and SHAKEN_GRAPH_NO_LDS apply to graphs only");
        if (lambda && (lambda->n_classes != 1 || lambda->class_of_vertex))
            return fail(SHAKEN_EINVAL, "torus: the field must be uniform (one class, no class map)");
        c->kind = KIND_TORUS;
        c->L = g->L;
        c->W = (g->L + 31) / 32;
        c->n = g->L * g->L;
        c->m = (tri ? 3 : 2) * (int64_t)c->n;
        c->J = 1;
        if (J && tri) {
            for (int64_t e = 1; e < c->m; ++e)
                if (J[e] != J[0])
                    return fail(SHAKEN_EINVAL, "triangular torus: the coupling must be uniform "
                                               "(pass other couplings as SHAKEN_EDGES)");
            c->J = J[0];
        } else if (J) {
            // uniform coupling, or +-J (one magnitude, any signs: the
            // Edwards-Anderson couplings of section 6) as two sign planes
            const int mag = std::abs((int)J[0]);
            bool mixed = false;
            for (int64_t e = 1; e < c->m; ++e) {
                if (std::abs((int)J[e]) != mag)
                    return fail(SHAKEN_EINVAL, "torus: every coupling must have the same magnitude "
                                               "(uniform or +-J; pass other tori as SHAKEN_EDGES)");
                mixed |= J[e] != J[0];
            }
            c->J = J[0];
            if (mixed) {
                c->J = mag;
                const int L = c->L, W = c->W;
                hl.jneg.assign((size_t)2 * L * W, 0u);
                for (int r = 0; r < L; ++r)
                    for (int col = 0; col < L; ++col) {
                        const int64_t x = (int64_t)r * L + col;
                        const uint32_t bit = 1u << (col & 31);
                        if (J[2 * x] < 0) hl.jneg[(size_t)r * W + (col >> 5)] |= bit;
                        if (J[2 * x + 1] < 0) hl.jneg[(size_t)L * W + (size_t)r * W + (col >> 5)] |= bit;
                    }
            }
        }
        c->smax = (tri ? 3 : 2) * std::abs(c->J);
        c->maxdeg = tri ? 3 : 2;
        if (o->format == SHAKEN_FMT_INT8)
            c->format = FMT_INT8;
        else if (o->format == SHAKEN_FMT_AUTO || o->format == SHAKEN_FMT_BITPACKED)
            c->format = FMT_BITPACKED;
        else
            return fail(SHAKEN_EINVAL, "unknown format");
        c->class_size.assign(1, c->n);
    } else if (g->kind == SHAKEN_EDGES) {
        c->kind = KIND_GRAPH;
        c->n = g->n;
        c->m = g->m;
        if (o->format != SHAKEN_FMT_AUTO && o->format != SHAKEN_FMT_INT8 && o->format != SHAKEN_FMT_BITPACKED)
            return fail(SHAKEN_EINVAL, "unknown format");
        c->format = o->format == SHAKEN_FMT_BITPACKED ? FMT_BITPACKED : FMT_INT8;
        c->W = (g->n + 31) / 32;
        if (o->flags & ~(SHAKEN_GRAPH_SPLIT | SHAKEN_ORDER_REVERSED | SHAKEN_GRAPH_LDS | SHAKEN_GRAPH_NO_LDS))
            return fail(SHAKEN_EINVAL, "unknown opts.flags bits");
        if ((o->flags & SHAKEN_GRAPH_LDS) && (o->flags & SHAKEN_GRAPH_NO_LDS))
            return fail(SHAKEN_EINVAL, "SHAKEN_GRAPH_LDS and SHAKEN_GRAPH_NO_LDS exclude each other");
        CHK(build_graph(c, g, J, (o->flags & SHAKEN_GRAPH_SPLIT) != 0, rp, col, jw));
        if (o->graph_layout < SHAKEN_LAYOUT_AUTO || o->graph_layout > SHAKEN_LAYOUT_PACKED)
            return fail(SHAKEN_EINVAL, "unknown graph layout");
        if (o->graph_layout != SHAKEN_LAYOUT_CSR) {
            const bool ok = build_ell(c->n, hl);
            if (!ok && o->graph_layout != SHAKEN_LAYOUT_AUTO)
                return fail(SHAKEN_EINVAL, "ELL layout needs couplings +-1 and at most 4 neighbours per vertex");
        }
        cls_host.assign((size_t)c->n, 0);
        if (lambda && lambda->class_of_vertex) {
            for (int v = 0; v < c->n; ++v) {
                if (lambda->class_of_vertex[v] >= lambda->n_classes)
                    return fail(SHAKEN_EINVAL, "field: class id out of range");
                cls_host[v] = lambda->class_of_vertex[v];
            }
        }
        c->class_size.assign(c->lam.size(), 0);
        for (int v = 0; v < c->n; ++v) c->class_size[cls_host[v]]++;
        if (o->graph_layout == SHAKEN_LAYOUT_AUTO || o->graph_layout == SHAKEN_LAYOUT_PACKED) {
            const bool ok = build_pell(c->n, hl);
            if (!ok && o->graph_layout == SHAKEN_LAYOUT_PACKED)
                return fail(SHAKEN_EINVAL, "packed layout needs couplings +-1, at most 3 neighbours per "
                                           "vertex, n <= 65536 and at most 16 field classes");
            // AUTO on a graph larger than the persistent kernel takes: CSR
            // (the grid kernels run faster on it than on ELL from 2^17
            // vertices on, and on every batch of such graphs)
            if (!ok && o->graph_layout == SHAKEN_LAYOUT_AUTO && c->n > 65536) {
                hl.ell.clear();
                hl.ell_k = 0;
            }
        }
    } else {
        return fail(SHAKEN_EINVAL, "unknown graph kind");
    }
    if (o->frozen) {
        // frozen set B (section 3.1): bits in the layout of the bit-packed spins
        const bool torus = c->kind == KIND_TORUS;
        const int W = torus ? c->W : (c->n + 31) / 32, rows = torus ? c->L : 1, cols = torus ? c->L : c->n;
        hl.frozen.assign((size_t)rows * W, 0u);
        c->frozen_host.assign((size_t)c->n, 0);
        for (int r = 0; r < rows; ++r)
            for (int col = 0; col < cols; ++col)
                if (o->frozen[(size_t)r * cols + col]) {
                    hl.frozen[(size_t)r * W + (col >> 5)] |= 1u << (col & 31);
                    c->frozen_host[(size_t)r * cols + col] = 1;
                }
    }
    const size_t lut_entries = (size_t)(2 * c->smax + 1) * 2 * c->lam.size();
    if (lut_entries > ((size_t)1 << 24))
        return fail(SHAKEN_EINVAL, "threshold table would exceed 2^24 entries");
    if (o->init == SHAKEN_INIT_USER) {
        if (!o->init_spins) return fail(SHAKEN_EINVAL, "init: SHAKEN_INIT_USER needs init_spins");
        for (int64_t i = 0; i < c->n; ++i)
            if (o->init_spins[i] != 1 && o->init_spins[i] != -1)
                return fail(SHAKEN_EINVAL, "init: spins must be +1 or -1");
    } else if (o->init != SHAKEN_INIT_RANDOM && o->init != SHAKEN_INIT_ALL_UP &&
               o->init != SHAKEN_INIT_ALL_DOWN) {
        return fail(SHAKEN_EINVAL, "unknown init mode");
    }
    return SHAKEN_OK;
}

// Device phase of shaken_init: buffers, uploads, descriptor, initial state.
int default_block(const ChainDesc &d);

shaken_status init_device(shaken_ctx *c, const shaken_opts *o, HostLayout &hl) {
    std::vector<uint8_t> &cls_host = hl.cls_host;
    std::vector<int32_t> *rp = hl.rp, *col = hl.col;
    std::vector<int8_t> *jw = hl.jw;
    const size_t lut_entries = (size_t)(2 * c->smax + 1) * 2 * c->lam.size();

    // device buffers
    // whole 16-byte units (the LDS-staged graph kernel reads bit-packed
    // configurations four words at a time); a bit-packed torus has kRows
    // more rows of zeros, so that the strip loads of the half-step kernels
    // need no bounds test (rows past the side read as no sites)
    size_t sbytes = (c->spin_bytes() + 15) / 16 * 16;
    const size_t pad_bytes = (c->kind == KIND_TORUS && c->format == FMT_BITPACKED) ? (size_t)kRows * c->W * 4 : 0;
    CHK(dalloc((uint8_t **)&c->spin[0], sbytes + pad_bytes));
    CHK(dalloc((uint8_t **)&c->spin[1], sbytes + pad_bytes));
    if (pad_bytes) {
        HIPCHK(hipMemsetAsync((uint8_t *)c->spin[0] + c->spin_bytes(), 0, sbytes + pad_bytes - c->spin_bytes(), c->stream));
        HIPCHK(hipMemsetAsync((uint8_t *)c->spin[1] + c->spin_bytes(), 0, sbytes + pad_bytes - c->spin_bytes(), c->stream));
    }
    CHK(dalloc(&c->lut_dev, lut_entries));
    CHK(dalloc(&c->obs_dev, (size_t)c->stride()));
    CHK(dalloc(&c->dd, 1));
    CHK(dalloc(&c->dd_static, 1));
    // set-up of the fixed buffer's device address (the device is current)
    HIPCHK(noalloc_scratch(c->device, &c->scratch));
    if (c->kind == KIND_GRAPH) {
        // padding read by the LDS-staged kernel's unconditional vector loads:
        // row pointers to a multiple of four vertices plus one (value m_h,
        // empty rows), eight zero edges, class bytes to a multiple of four
        const size_t n4 = ((size_t)c->n + 3) / 4 * 4;
        for (int h = 0; h < 2; ++h) {
            rp[h].resize(n4 + 1, rp[h][(size_t)c->n]);
            col[h].resize(col[h].size() + 8, 0);
            jw[h].resize(jw[h].size() + 8, 0);
        }
        cls_host.resize(n4, 0);
        for (int h = 0; h < 2; ++h) {
            CHK(dalloc(&c->rp[h], rp[h].size()));
            CHK(dalloc(&c->col[h], col[h].size()));
            CHK(dalloc(&c->jw[h], jw[h].size()));
            HIPCHK(hipMemcpyAsync(c->rp[h], rp[h].data(), rp[h].size() * 4, hipMemcpyHostToDevice, c->stream));
            HIPCHK(hipMemcpyAsync(c->col[h], col[h].data(), col[h].size() * 4, hipMemcpyHostToDevice, c->stream));
            HIPCHK(hipMemcpyAsync(c->jw[h], jw[h].data(), jw[h].size(), hipMemcpyHostToDevice, c->stream));
        }
        CHK(dalloc(&c->cls_dev, cls_host.size()));
        HIPCHK(hipMemcpyAsync(c->cls_dev, cls_host.data(), cls_host.size(), hipMemcpyHostToDevice, c->stream));
        if (hl.ell_k > 0) {
            CHK(dalloc(&c->ell_dev, hl.ell.size()));
            HIPCHK(hipMemcpyAsync(c->ell_dev, hl.ell.data(), hl.ell.size() * 4, hipMemcpyHostToDevice, c->stream));
            c->ell_k = hl.ell_k;
            c->ell_stride = hl.ell_stride;
        }
        if (!hl.pell.empty()) {
            CHK(dalloc(&c->pell_dev, hl.pell.size()));
            HIPCHK(hipMemcpyAsync(c->pell_dev, hl.pell.data(), hl.pell.size() * 8, hipMemcpyHostToDevice, c->stream));
        }
    }
    if (!hl.frozen.empty()) {
        CHK(dalloc(&c->frozen_dev, hl.frozen.size()));
        HIPCHK(hipMemcpyAsync(c->frozen_dev, hl.frozen.data(), hl.frozen.size() * 4, hipMemcpyHostToDevice, c->stream));
    }
    if (c->kind == KIND_GRAPH && (c->n + 31) / 32 <= graph_lds_max_words()) {
        if (c->format != FMT_BITPACKED) {
            const size_t mw = ((size_t)(c->n + 31) / 32 + 3) / 4 * 4;
            CHK(dalloc(&c->mirror[0], mw));
            CHK(dalloc(&c->mirror[1], mw));
        }
        // the LDS-staged kernel's edge words: index (< 2^21), the slot of the
        // edge's row vertex in its group of four (v & 3) and J, read four at a
        // time from aligned positions
        for (int h = 0; h < 2; ++h) {
            const size_t mh = (size_t)rp[h][(size_t)c->n];
            std::vector<int32_t> cj((mh + 3) / 4 * 4 + 16, 0);
            for (int v = 0; v < c->n; ++v)
                for (int32_t e = rp[h][(size_t)v]; e < rp[h][(size_t)v + 1]; ++e)
                    cj[(size_t)e] = (int32_t)(((uint32_t)col[h][(size_t)e] & 0x1FFFFFu) | ((uint32_t)(v & 3) << 21) |
                                              ((uint32_t)(uint8_t)jw[h][(size_t)e] << 24));
            CHK(dalloc(&c->cj[h], cj.size()));
            HIPCHK(hipMemcpyAsync(c->cj[h], cj.data(), cj.size() * 4, hipMemcpyHostToDevice, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
        }
        // three slots per vertex where every half-degree is at most three and
        // every coupling has one magnitude: the kernel then needs no row
        // bounds, no window shift and no masks (empty slots read a zero word)
        int j0 = 0;
        bool e3ok = c->maxdeg <= 3;
        for (int h = 0; h < 2 && e3ok; ++h)
            for (int32_t e = 0; e < rp[h][(size_t)c->n] && e3ok; ++e) {
                const int a = std::abs((int)jw[h][(size_t)e]);
                if (j0 == 0) j0 = a;
                e3ok = a > 0 && a == j0;
            }
        if (e3ok) {
            const uint32_t zw = (uint32_t)graph_lds_max_words() << 7;  // the zero word, bit 0
            const size_t nq = ((size_t)c->n + 3) / 4;
            for (int h = 0; h < 2; ++h) {
                std::vector<uint32_t> e3(nq * 12, zw);
                for (int v = 0; v < c->n; ++v) {
                    const int32_t e0 = rp[h][(size_t)v], deg = rp[h][(size_t)v + 1] - e0;
                    for (int k = 0; k < deg; ++k) {
                        const uint32_t cv = (uint32_t)col[h][(size_t)(e0 + k)];
                        e3[(size_t)3 * v + k] = (cv & 31u) | ((cv >> 5) << 7) |
                                                (jw[h][(size_t)(e0 + k)] < 0 ? 0x80000000u : 0u);
                    }
                    e3[(size_t)3 * v] |= (uint32_t)deg << 23;
                }
                CHK(dalloc(&c->e3[h], e3.size()));
                HIPCHK(hipMemcpyAsync(c->e3[h], e3.data(), e3.size() * 4, hipMemcpyHostToDevice, c->stream));
                HIPCHK(hipStreamSynchronize(c->stream));
            }
            c->j0 = j0 > 0 ? j0 : 1;
        }
    }
    if (!hl.jneg.empty()) {
        CHK(dalloc(&c->jneg_dev, hl.jneg.size()));
        HIPCHK(hipMemcpyAsync(c->jneg_dev, hl.jneg.data(), hl.jneg.size() * 4, hipMemcpyHostToDevice, c->stream));
    }

    // descriptor
    ChainDesc &d = c->hd;
    std::memset(&d, 0, sizeof(d));
    d.seed = c->seed;
    d.replica = c->replica;
    d.kind = c->kind;
    d.format = c->format;
    d.L = c->L;
    d.W = c->W;
    d.wdiv = c->W > 0 ? (uint32_t)((((uint64_t)1 << 32) + (uint64_t)c->W - 1) / (uint64_t)c->W) : 0u;
    d.n = c->n;
    d.J = c->J;
    d.lut = c->lut_dev;
    d.smax = c->smax;
    d.ncls = (int32_t)c->lam.size();
    for (int h = 0; h < 2; ++h) {
        d.rowptr[h] = c->rp[h];
        d.col[h] = c->col[h];
        d.jw[h] = c->jw[h];
    }
    d.cls = c->cls_dev;
    d.maxdeg = c->maxdeg;
    d.ell = c->ell_dev;
    d.ell_k = c->ell_k;
    d.ell_stride = c->ell_stride;
    d.pell = c->pell_dev;
    d.jneg = c->jneg_dev;
    d.rev = (o->flags & SHAKEN_ORDER_REVERSED) ? 1 : 0;
    d.tri = c->tri ? 1 : 0;
    d.frozen = c->frozen_dev;
    d.mirror[0] = c->mirror[0];
    d.mirror[1] = c->mirror[1];
    d.cj[0] = c->cj[0];
    d.cj[1] = c->cj[1];
    d.e3[0] = c->e3[0];
    d.e3[1] = c->e3[1];
    d.j0 = c->j0;
    d.log_line = c->line();
    d.log_stride = c->stride();
    for (size_t k = 0; k < c->lam.size() && k < 16; ++k) {
        d.lam2[k] = c->lam2_int ? (int32_t)c->lam2[k] : 0;
        d.csize[k] = (int32_t)c->class_size[k];
    }
    refresh_desc_spins(c);
    build_tables(c);
    CHK(upload_tables(c));
    c->block = (o->flags & SHAKEN_GRAPH_NO_LDS) ? 256
               : ((o->flags & SHAKEN_GRAPH_LDS) && graph_lds_fits(c->hd)) ? kLdsGraphBlock
                                                                          : default_block(c->hd);

    // degree statistics (integer sums; the in - out differences sum to zero
    // over the sites, so their root mean square is their standard deviation)
    if (c->kind == KIND_GRAPH) {
        int64_t sdeg = 0, s2 = 0;
        for (int v = 0; v < c->n; ++v) {
            const int64_t din = rp[0][(size_t)v + 1] - rp[0][(size_t)v];
            const int64_t dout = rp[1][(size_t)v + 1] - rp[1][(size_t)v];
            sdeg += din + dout;
            s2 += (din - dout) * (din - dout);
        }
        c->deg_mean = (double)sdeg / (double)c->n;
        c->deg_spread = std::sqrt((double)s2 / (double)c->n);
    } else {
        c->deg_mean = c->tri ? 6.0 : 4.0;
        c->deg_spread = 0.0;
    }

    // initial state into spin[0] (s = 0)
    switch (o->init) {
    case SHAKEN_INIT_RANDOM:
    case SHAKEN_INIT_ALL_UP:
    case SHAKEN_INIT_ALL_DOWN: {
        const int mode = o->init == SHAKEN_INIT_RANDOM ? 0 : (o->init == SHAKEN_INIT_ALL_UP ? 1 : 2);
        HIPCHK(launch_init(c->hd, c->spin[0], mode, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        break;
    }
    default:
        CHK(shaken_set_spins(c, o->init_spins));
        break;
    }
    return SHAKEN_OK;
}

// The launch shape a graph chain starts with: the LDS-staged kernel from
// kLdsGraphMinN vertices on (where staging the packed configuration costs
// less than the cache lines of its random gathers), else the plain kernel's
// 256-lane blocks.  Batches with autotuning measure both.
constexpr int kLdsGraphMinN = 1 << 17;

int default_block(const ChainDesc &d) {
    return graph_lds_fits(d) && d.n >= kLdsGraphMinN ? kLdsGraphBlock : 256;
}

// before the first half-step of a call on the LDS-staged kernel: the packed
// mirror of the configuration it reads (int8 chains)
shaken_status prepare_mirror(shaken_ctx *c, const ChainDesc *dev) {
    if (c->block == kLdsGraphBlock && c->mirror[0])
        HIPCHK(launch_pack_mirror(dev, &c->hd, 1, (int)(c->s & 1u), c->stream));
    return SHAKEN_OK;
}

// one half-step at the context's counter (descriptor dd, or dd_static with
// the log in the fixed buffer)
shaken_status half_step_once(shaken_ctx *c, int log_on, uint32_t s_log0, bool fixed_log = false) {
    if (c->s >= kInitStep - 1) return fail(SHAKEN_ESTATE, "half-step counter exhausted");
    CHK(refresh_if_stale(c));
    HIPCHK(launch_half_step_grid(fixed_log ? c->dd_static : c->dd, &c->hd, 1, nullptr, c->s, s_log0, log_on,
                                 (c->s & 1u) == 0, c->block, c->stream));
    c->s += 1;
    return SHAKEN_OK;
}

}  // namespace

// ====================================================================== ABI

extern "C" {

shaken_status shaken_init(shaken_ctx **out, const shaken_graph *g, const int8_t *J,
                          const shaken_field *lambda, double q, double beta, uint64_t seed,
                          const shaken_opts *opts) {
    g_err.clear();
    if (!out || !g) return fail(SHAKEN_EINVAL, "out and g must be non-NULL");
    *out = nullptr;
    if (!finite_nonneg(q)) return fail(SHAKEN_EINVAL, "q must be finite and >= 0");
    if (!finite_nonneg(beta)) return fail(SHAKEN_EINVAL, "beta must be finite and >= 0");
    shaken_opts o{};
    o.format = SHAKEN_FMT_AUTO;
    o.init = SHAKEN_INIT_RANDOM;
    o.device = -1;
    o.graph_layout = SHAKEN_LAYOUT_AUTO;
    if (opts) o = *opts;
    shaken_ctx *c = new (std::nothrow) shaken_ctx();
    if (!c) return fail(SHAKEN_ENOMEM, "host allocation failed");
    c->stream = (hipStream_t)o.stream;
    c->q = q;
    c->beta = beta;
    c->seed = seed;
    c->replica = o.replica;
    shaken_status st;
    HostLayout hl;
    try {
        st = init_host(c, g, J, lambda, &o, hl);
    } catch (const std::bad_alloc &) {
        st = fail(SHAKEN_ENOMEM, "host allocation failed");
    }
    if (st != SHAKEN_OK) {
        delete c;
        return st;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        delete c;
        return fail(SHAKEN_EDEVICE, "no HIP device");
    }
    if (o.device >= ndev) {
        delete c;
        return fail(SHAKEN_EINVAL, "device ordinal out of range");
    }
    if (o.device >= 0) {
        c->device = o.device;
    } else if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(SHAKEN_EDEVICE, "no current HIP device");
    }
    DeviceGuard guard(c->device);
    try {
        st = init_device(c, &o, hl);
    } catch (const std::bad_alloc &) {
        st = fail(SHAKEN_ENOMEM, "host allocation failed");
    }
    if (st != SHAKEN_OK) {
        release(c);
        delete c;
        return st;
    }
    *out = c;
    return SHAKEN_OK;
}

shaken_status shaken_free(shaken_ctx *ctx) {
    if (!ctx) return SHAKEN_OK;
    DeviceGuard guard(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    release(ctx);
    delete ctx;
    return SHAKEN_OK;
}

shaken_status shaken_half_step(shaken_ctx *ctx, int64_t n) {
    if (!ctx) return fail(SHAKEN_EINVAL, "ctx is NULL");
    if (n < 0) return fail(SHAKEN_EINVAL, "n must be >= 0");
    DeviceGuard guard(ctx->device);
    if ((int64_t)ctx->s + n >= (int64_t)kInitStep) return fail(SHAKEN_ESTATE, "half-step counter would overflow");
    if (n > 0) CHK(prepare_mirror(ctx, ctx->dd));
    for (int64_t i = 0; i < n; ++i) CHK(half_step_once(ctx, 0, 0));
    return SHAKEN_OK;
}

shaken_status shaken_sweep(shaken_ctx *ctx, int64_t n_full, int64_t *H_out, int64_t *M_out) {
    if (!ctx) return fail(SHAKEN_EINVAL, "ctx is NULL");
    if (n_full < 0) return fail(SHAKEN_EINVAL, "n_full must be >= 0");
    if (ctx->s & 1u) return fail(SHAKEN_ESTATE, "shaken_sweep needs an even half-step counter");
    if (H_out && !ctx->lam2_int) return fail(SHAKEN_EINVAL, "H_out needs every 2*lambda to be an integer");
    if ((int64_t)ctx->s + 2 * n_full >= (int64_t)kInitStep) return fail(SHAKEN_ESTATE, "half-step counter would overflow");
    DeviceGuard guard(ctx->device);
    const bool logs = H_out || M_out;
    const uint32_t s0 = ctx->s;
    if (logs) {
        CHK(ensure_log(ctx, n_full + 1));
        HIPCHK(launch_fill_i64(ctx->log_dev, (n_full + 1) * ctx->stride(), 0, ctx->stream));
    }
    if (n_full > 0) CHK(prepare_mirror(ctx, ctx->dd));
    for (int64_t t = 0; t < n_full; ++t) {
        CHK(half_step_once(ctx, logs ? 1 : 0, s0));
        CHK(half_step_once(ctx, 0, s0));
    }
    if (logs) {
        HIPCHK(launch_observe(ctx->dd, &ctx->hd, 1, (int)(ctx->s & 1u), (int)n_full, ctx->stream));
        std::vector<int64_t> raw((size_t)((n_full + 1) * ctx->stride()));
        HIPCHK(hipMemcpyAsync(raw.data(), ctx->log_dev, raw.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        convert_log(ctx, raw, n_full + 1, kLogParts, H_out, M_out);
    }
    return SHAKEN_OK;
}

shaken_status shaken_sweep_noalloc(shaken_ctx *ctx, int64_t n_full, int64_t *H_dev, int64_t *M_dev) {
    if (!ctx) return fail(SHAKEN_EINVAL, "ctx is NULL");
    if (n_full < 0) return fail(SHAKEN_EINVAL, "n_full must be >= 0");
    if (ctx->s & 1u) return fail(SHAKEN_ESTATE, "shaken_sweep_noalloc needs an even half-step counter");
    if (H_dev && !ctx->lam2_int) return fail(SHAKEN_EINVAL, "H_dev needs every 2*lambda to be an integer");
    if ((int64_t)ctx->s + 2 * n_full >= (int64_t)kInitStep) return fail(SHAKEN_ESTATE, "half-step counter would overflow");
    if (!ctx->scratch || !ctx->dd_static) return fail(SHAKEN_ESTATE, "context has no fixed log buffer");
    const bool logs = H_dev || M_dev;
    const int64_t max_full = noalloc_capacity() / ctx->stride() - 1;
    if (logs) {
        if ((int64_t)ctx->lam.size() > kNoallocClasses)
            return fail(SHAKEN_EINVAL, "shaken_sweep_noalloc logs at most " + std::to_string(kNoallocClasses) +
                                           " field classes");
        if (n_full > max_full)
            return fail(SHAKEN_EINVAL, "n_full = " + std::to_string(n_full) + " exceeds the fixed log buffer: at most " +
                                           std::to_string(max_full) + " full steps per call with logs for this context");
    }
    DeviceGuard guard(ctx->device);
    const uint32_t s0 = ctx->s;
    const int64_t slots = n_full + 1;
    // partial sums accumulate into the slots: clear them with a fill kernel
    if (logs) HIPCHK(launch_fill_i64(ctx->scratch, slots * ctx->stride(), 0, ctx->stream));
    if (n_full > 0) CHK(prepare_mirror(ctx, ctx->dd_static));
    for (int64_t t = 0; t < n_full; ++t) {
        CHK(half_step_once(ctx, logs ? 1 : 0, s0, true));
        CHK(half_step_once(ctx, 0, s0, true));
    }
    if (logs) {
        HIPCHK(launch_observe(ctx->dd_static, &ctx->hd, 1, (int)(ctx->s & 1u), (int)n_full, ctx->stream));
        LogReduceArgs a{};
        a.ncls = (int32_t)ctx->lam.size();
        a.n = ctx->n;
        for (size_t k = 0; k < ctx->lam.size(); ++k) {
            a.lam2[k] = ctx->lam2_int ? ctx->lam2[k] : 0;
            a.c0 += a.lam2[k] * ctx->class_size[k];
        }
        HIPCHK(launch_log_reduce(ctx->scratch, slots, ctx->line(), a, H_dev, M_dev, ctx->stream));
    }
    return SHAKEN_OK;
}

shaken_status shaken_observables(shaken_ctx *ctx, shaken_obs *out) {
    if (!ctx || !out) return fail(SHAKEN_EINVAL, "ctx and out must be non-NULL");
    DeviceGuard guard(ctx->device);
    // the observe kernel writes slot `slot` of d.log: point a temporary desc at obs_dev
    ChainDesc d = ctx->hd;
    d.log = ctx->obs_dev;
    ChainDesc *dtmp = nullptr;
    CHK(dalloc(&dtmp, 1));
    shaken_status st = SHAKEN_OK;
    std::vector<int64_t> raw((size_t)ctx->stride());
    do {
        hipError_t e;
        if ((e = hipMemcpyAsync(dtmp, &d, sizeof(d), hipMemcpyHostToDevice, ctx->stream)) != hipSuccess ||
            (e = launch_fill_i64(ctx->obs_dev, ctx->stride(), 0, ctx->stream)) != hipSuccess ||
            (e = launch_observe(dtmp, &d, 1, (int)(ctx->s & 1u), 0, ctx->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(raw.data(), ctx->obs_dev, raw.size() * 8, hipMemcpyDeviceToHost, ctx->stream)) != hipSuccess ||
            (e = hipStreamSynchronize(ctx->stream)) != hipSuccess) {
            st = fail(SHAKEN_EDEVICE, std::string("observables: ") + hipGetErrorString(e));
        }
    } while (0);
    dfree(dtmp);
    if (st != SHAKEN_OK) return st;
    auto val = [&](int64_t v) {
        int64_t a = 0;
        for (int p = 0; p < kLogParts; ++p) a += raw[p * ctx->line() + v];
        return a;
    };
    out->half_step = ctx->s;
    out->n_sites = ctx->n;
    out->E_J = val(0);
    int64_t m = 0, l2 = 0;
    double l2d = 0;
    for (size_t k = 0; k < ctx->lam.size(); ++k) {
        const int64_t mk = 2 * val(1 + (int64_t)k) - ctx->class_size[k];
        m += mk;
        l2 += ctx->lam2[k] * mk;
        l2d += 2.0 * ctx->lam[k] * (double)mk;
    }
    out->M = m;
    out->E_lambda2 = ctx->lam2_int ? l2 : 0;
    out->H = ctx->lam2_int ? (double)(-out->E_J - l2) : -(double)out->E_J - l2d;
    out->flags = ctx->lam2_int ? 1 : 0;
    out->reserved = 0;
    return SHAKEN_OK;
}

shaken_status shaken_set_params(shaken_ctx *ctx, double beta, double q) {
    if (!ctx) return fail(SHAKEN_EINVAL, "ctx is NULL");
    if (!finite_nonneg(q)) return fail(SHAKEN_EINVAL, "q must be finite and >= 0");
    if (!finite_nonneg(beta)) return fail(SHAKEN_EINVAL, "beta must be finite and >= 0");
    DeviceGuard guard(ctx->device);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->beta = beta;
    ctx->q = q;
    build_tables(ctx);
    return upload_tables(ctx);
}

shaken_status shaken_get_spins(shaken_ctx *ctx, int8_t *out) {
    if (!ctx || !out) return fail(SHAKEN_EINVAL, "ctx and out must be non-NULL");
    DeviceGuard guard(ctx->device);
    const void *src = ctx->spin[ctx->s & 1u];
    if (ctx->format == FMT_BITPACKED) {
        int rows, cols, W;
        spin_rows(ctx, rows, cols, W);
        std::vector<uint32_t> w((size_t)rows * W);
        HIPCHK(hipMemcpyAsync(w.data(), src, w.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        unpack_rows(w, rows, cols, W, out);
    } else {
        HIPCHK(hipMemcpyAsync(out, src, (size_t)ctx->n, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return SHAKEN_OK;
}

shaken_status shaken_set_spins(shaken_ctx *ctx, const int8_t *in) {
    if (!ctx || !in) return fail(SHAKEN_EINVAL, "ctx and in must be non-NULL");
    for (int64_t i = 0; i < ctx->n; ++i)
        if (in[i] != 1 && in[i] != -1) return fail(SHAKEN_EINVAL, "spins must be +1 or -1");
    std::vector<int8_t> forced;
    if (!ctx->frozen_host.empty()) {  // sites of the frozen set stay +1
        forced.assign(in, in + ctx->n);
        for (int64_t i = 0; i < ctx->n; ++i)
            if (ctx->frozen_host[(size_t)i]) forced[(size_t)i] = 1;
        in = forced.data();
    }
    DeviceGuard guard(ctx->device);
    void *dst = ctx->spin[ctx->s & 1u];
    if (ctx->format == FMT_BITPACKED) {
        int rows, cols, W;
        spin_rows(ctx, rows, cols, W);
        std::vector<uint32_t> w;
        pack_rows(in, rows, cols, W, w);
        HIPCHK(hipMemcpyAsync(dst, w.data(), w.size() * 4, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    } else {
        HIPCHK(hipMemcpyAsync(dst, in, (size_t)ctx->n, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return SHAKEN_OK;
}

shaken_status shaken_set_half_step(shaken_ctx *ctx, int64_t s) {
    if (!ctx) return fail(SHAKEN_EINVAL, "ctx is NULL");
    if (s < 0 || s >= (int64_t)kInitStep) return fail(SHAKEN_EINVAL, "s out of range");
    DeviceGuard guard(ctx->device);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (((uint32_t)s & 1u) != (ctx->s & 1u)) {
        // keep the configuration where the new parity expects it
        std::swap(ctx->spin[0], ctx->spin[1]);
        refresh_desc_spins(ctx);
        CHK(upload_desc(ctx));
    }
    ctx->s = (uint32_t)s;
    return SHAKEN_OK;
}

shaken_status shaken_get_lut(const shaken_ctx *ctx, uint64_t *out, size_t *n, int32_t *smax) {
    if (!ctx || !n) return fail(SHAKEN_EINVAL, "ctx and n must be non-NULL");
    if (smax) *smax = ctx->smax;
    if (!out) {
        *n = ctx->lut.size();
        return SHAKEN_OK;
    }
    if (*n < ctx->lut.size()) return fail(SHAKEN_EINVAL, "capacity too small");
    std::memcpy(out, ctx->lut.data(), ctx->lut.size() * sizeof(uint64_t));
    *n = ctx->lut.size();
    return SHAKEN_OK;
}

shaken_status shaken_spins_device(shaken_ctx *ctx, void **ptr, int32_t *format) {
    if (!ctx || !ptr) return fail(SHAKEN_EINVAL, "ctx and ptr must be non-NULL");
    *ptr = ctx->spin[ctx->s & 1u];
    if (format) *format = ctx->format == FMT_BITPACKED ? SHAKEN_FMT_BITPACKED : SHAKEN_FMT_INT8;
    return SHAKEN_OK;
}

shaken_status shaken_synchronize(shaken_ctx *ctx) {
    if (!ctx) return fail(SHAKEN_EINVAL, "ctx is NULL");
    DeviceGuard guard(ctx->device);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return SHAKEN_OK;
}

const char *shaken_strerror(shaken_status s) {
    switch (s) {
    case SHAKEN_OK: return "ok";
    case SHAKEN_EINVAL: return "invalid argument";
    case SHAKEN_ENOMEM: return "out of memory";
    case SHAKEN_EDEVICE: return "device error";
    case SHAKEN_ESTATE: return "invalid state";
    }
    return "unknown status";
}

const char *shaken_last_error(void) { return g_err.c_str(); }

int32_t shaken_version(void) { return (SHAKEN_VERSION_MAJOR << 16) | SHAKEN_VERSION_MINOR; }

}  // extern "C"

// ====================================================================== batches

namespace {

// full steps of half-step launches per captured HIP graph (grid strategy)
constexpr int kGraphChunk = 16;

struct Group {
    int kind = 0, format = 0, tri = 0;
    std::vector<int> members;  // indices into the batch's contexts
    std::vector<ChainDesc> hd;
    ChainDesc *dd = nullptr;
    int block = 256;
};

}  // namespace

struct shaken_batch {
    std::vector<shaken_ctx *> ctx;
    int device = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int strategy = SHAKEN_BATCH_GRID;
    int use_graph = 0;
    int autotune = 0;
    bool tuned = false;
    int record = 0;
    int track = 0;
    std::vector<Group> groups;
    // batch-wide pools: thresholds of every chain, tracking pairs, best configurations
    uint64_t *lut_pool = nullptr;
    std::vector<size_t> lut_off;
    std::vector<uint64_t> lut_host;
    int64_t *track_pool = nullptr;
    uint32_t *best_pool = nullptr;
    std::vector<size_t> best_off;
    // observables log, slot-major: slot t of chain i starts at
    // log_pool + t * log_row + log_off[i] and holds log_parts lines
    int64_t *log_pool = nullptr;
    int64_t log_cap = 0;  // slots
    int64_t log_row = 0;  // entries per slot over all chains
    std::vector<int64_t> log_off;
    int log_parts = kLogParts;
    uint32_t *dstate = nullptr;  // [0] half-step base, [1] log base
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int chunk = 0;          // full steps per graph replay
    // spin buffers of every chain as the device descriptors hold them
    std::vector<std::pair<void *, void *>> up_spin;
    // host-side work done so far (shaken_batch_counters)
    int64_t n_captures = 0, n_log_allocs = 0, n_autotunes = 0, n_uploads = 0, n_sweeps = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
    int64_t last_n_full = -1;
    // persistent strategy
    ChainDesc *pdescs = nullptr;
    std::vector<ChainDesc> phd;
    int32_t *order = nullptr;
    int32_t *counter = nullptr;
    int pblock = 256, pgrid = 0;
    bool ptuned = false;
    hipGraphExec_t pgexec = nullptr;  // captured persistent launch (use_hipgraph)
    hipGraph_t pgraph = nullptr;
    int pg_grid = 0;                  // workgroup count it was captured with
};

namespace {

void batch_release(shaken_batch *b) {
    for (auto &g : b->groups) dfree(g.dd);
    dfree(b->dstate);
    dfree(b->lut_pool);
    dfree(b->track_pool);
    dfree(b->best_pool);
    dfree(b->log_pool);
    dfree(b->pdescs);
    dfree(b->order);
    dfree(b->counter);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->pgexec) (void)hipGraphExecDestroy(b->pgexec);
    if (b->pgraph) (void)hipGraphDestroy(b->pgraph);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

// refresh every group's device descriptors from the contexts (spin and log
// pointers may have changed)
// the descriptor chain i uses inside the batch (pool pointers)
ChainDesc batch_desc(shaken_batch *b, size_t i) {
    shaken_ctx *c = b->ctx[i];
    refresh_desc_spins(c);
    ChainDesc d = c->hd;
    d.lut = b->lut_pool + b->lut_off[i];
    d.track = b->track_pool ? b->track_pool + 2 * i : nullptr;
    d.best = b->best_pool ? b->best_pool + b->best_off[i] : nullptr;
    d.log = b->log_pool ? b->log_pool + b->log_off[i] : nullptr;
    d.log_stride = b->log_row;
    return d;
}

// log space for `slots` slots of every chain (one allocation for the batch)
shaken_status batch_ensure_log(shaken_batch *b, int64_t slots, bool *changed) {
    if (slots <= b->log_cap) return SHAKEN_OK;
    dfree(b->log_pool);
    b->log_pool = nullptr;
    b->log_cap = 0;
    b->log_off.assign(b->ctx.size(), 0);
    int64_t row = 0;
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        b->log_off[i] = row;
        row += b->log_parts * b->ctx[i]->line();
    }
    b->log_row = row;
    CHK(dalloc(&b->log_pool, (size_t)(slots * row)));
    b->log_cap = slots;
    b->n_log_allocs += 1;
    *changed = true;
    return SHAKEN_OK;
}

shaken_status batch_upload(shaken_batch *b) {
    b->up_spin.resize(b->ctx.size());
    for (size_t i = 0; i < b->ctx.size(); ++i) b->up_spin[i] = {b->ctx[i]->spin[0], b->ctx[i]->spin[1]};
    b->n_uploads += 1;
    for (auto &g : b->groups) {
        for (size_t i = 0; i < g.members.size(); ++i) g.hd[i] = batch_desc(b, g.members[i]);
        HIPCHK(hipMemcpyAsync(g.dd, g.hd.data(), g.hd.size() * sizeof(ChainDesc),
                              hipMemcpyHostToDevice, b->stream));
    }
    if (b->pdescs) {
        for (size_t i = 0; i < b->ctx.size(); ++i) b->phd[i] = batch_desc(b, i);
        HIPCHK(hipMemcpyAsync(b->pdescs, b->phd.data(), b->phd.size() * sizeof(ChainDesc),
                              hipMemcpyHostToDevice, b->stream));
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    return SHAKEN_OK;
}

// all groups, one half-step at s (explicit) or dstate[0] + s_add
shaken_status batch_half(shaken_batch *b, const uint32_t *dstate, uint32_t s_add, uint32_t s_log0,
                         bool even) {
    for (auto &g : b->groups)
        HIPCHK(launch_half_step_grid(g.dd, g.hd.data(), (int)g.hd.size(), dstate, s_add, s_log0,
                                     b->record, even, g.block, b->stream));
    return SHAKEN_OK;
}

// can every chain of the group run in the LDS-staged graph kernel?
bool group_lds_fits(const Group &g) {
    for (const auto &d : g.hd)
        if (!graph_lds_fits(d)) return false;
    return !g.hd.empty();
}

// launch shape a group starts with: the LDS-staged kernel when every chain
// takes it on its own
int group_default_block(const shaken_batch *b, const Group &g) {
    for (int i : g.members)
        if (b->ctx[(size_t)i]->block != kLdsGraphBlock) return 256;
    return kLdsGraphBlock;
}

// packed mirrors of the configurations the next half-step reads (groups on
// the LDS-staged kernel, or all that fit it when `all_fitting`)
shaken_status batch_pack_mirrors(shaken_batch *b, uint32_t s, bool all_fitting) {
    for (auto &g : b->groups)
        if (g.block == kLdsGraphBlock || (all_fitting && group_lds_fits(g)))
            HIPCHK(launch_pack_mirror(g.dd, g.hd.data(), (int)g.hd.size(), (int)(s & 1u), b->stream));
    return SHAKEN_OK;
}

// `reps` launches of the same half-step at the (even) counter s for one
// group and block size, captured in a HIP graph: trial launches are
// idempotent (they read spin[0], write spin[1]) and run as a sweep runs them,
// replayed from a graph (timed eagerly, the host's launch rate would hide
// differences of a few microseconds per launch)
struct TrialGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    ~TrialGraph() {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
    }
};

shaken_status trial_graph(shaken_batch *b, Group &g, int block, uint32_t s, int reps, TrialGraph &t) {
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int i = 0; i < reps && e == hipSuccess; ++i)
        e = launch_half_step_grid(g.dd, g.hd.data(), (int)g.hd.size(), nullptr, s, s, 0, (s & 1u) == 0, block,
                                  b->stream);
    const hipError_t e2 = hipStreamEndCapture(b->stream, &t.g);
    if (e != hipSuccess || e2 != hipSuccess)
        return fail(SHAKEN_EDEVICE, std::string("autotune capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    HIPCHK(hipGraphInstantiate(&t.x, t.g, nullptr, nullptr, 0));
    return SHAKEN_OK;
}

// GPU time of one replay of a trial graph (milliseconds)
shaken_status time_replay(shaken_batch *b, TrialGraph &t, float *ms) {
    HIPCHK(hipEventRecord(b->ev0, b->stream));
    HIPCHK(hipGraphLaunch(t.x, b->stream));
    HIPCHK(hipEventRecord(b->ev1, b->stream));
    HIPCHK(hipEventSynchronize(b->ev1));
    HIPCHK(hipEventElapsedTime(ms, b->ev0, b->ev1));
    return SHAKEN_OK;
}

// GPU time the autotuners spend on trial launches before they compare
// candidates: an idle GPU takes some tens of milliseconds of work to reach its
// steady clocks (measured on MI355X: half-step launches of the 4096^2 x 24
// batch run 74 us at first, 66 us after ~30 ms, 63 us in long runs), and a
// comparison made while the clocks rise favours whichever candidate runs last.
constexpr float kWarmMs = 40.0f;
constexpr int kWarmMaxTrials = 400;
// timed replays per candidate of the grid autotuner (the fastest counts)
constexpr int kTimedRounds = 3;

// Launch shapes the autotuners measured, kept for the process (opts.autotune
// = 2 reuses them).  The key is the device and every chain's shape: kind,
// format, lattice, sizes, table folding, sign planes, frozen set, field
// classes, graph layout and the kernel the chain may run on.
std::mutex g_tune_mu;
std::unordered_map<std::string, int> g_tune_cache;

std::string chain_shape(const shaken_ctx *c, const ChainDesc &d) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "%d.%d.%d.%d.%d.%lld.%d.%d.%d.%d.%d.%d.%d.%d.%d.%d;", d.kind, d.format, d.tri, d.L,
                  d.n, (long long)c->m, d.fold3, d.jneg != nullptr, d.frozen != nullptr, d.ncls, d.smax, d.ell_k,
                  d.pell != nullptr, d.cj[0] != nullptr, d.e3[0] != nullptr, c->block);
    return buf;
}

std::string tune_key(const shaken_batch *b, const char *what, const std::vector<int> &members) {
    std::string k = std::string(what) + "@" + std::to_string(b->device) + ":";
    for (int i : members) k += chain_shape(b->ctx[(size_t)i], b->ctx[(size_t)i]->hd);
    return k;
}

bool tune_lookup(const std::string &key, int *out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it == g_tune_cache.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(const std::string &key, int v) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = v;
}

shaken_status batch_autotune(shaken_batch *b) {
    const uint32_t s = b->ctx[0]->s;
    // shapes already measured in this process (autotune = 2)
    std::vector<std::string> keys;
    bool all_cached = true;
    for (auto &g : b->groups) {
        keys.push_back(tune_key(b, "grid", g.members));
        int blk = 0;
        if (b->autotune == 2 && tune_lookup(keys.back(), &blk)) continue;
        all_cached = false;
    }
    if (all_cached) {
        for (size_t k = 0; k < b->groups.size(); ++k) (void)tune_lookup(keys[k], &b->groups[k].block);
        b->tuned = true;
        return SHAKEN_OK;
    }
    CHK(batch_pack_mirrors(b, s, true));
    const int reps = 10;
    size_t gi = 0;
    for (auto &g : b->groups) {
        const std::string &key = keys[gi++];
        int cached = 0;
        if (b->autotune == 2 && tune_lookup(key, &cached)) {
            g.block = cached;
            continue;
        }
        std::vector<int> cands{64, 128, 256};
        if (group_lds_fits(g)) cands.push_back(kLdsGraphBlock);
        std::vector<TrialGraph> tg(cands.size());
        size_t def = 0;
        for (size_t k = 0; k < cands.size(); ++k) {
            CHK(trial_graph(b, g, cands[k], s, reps, tg[k]));
            if (cands[k] == g.block) def = k;
        }
        // warm phase with the default shape, one untimed replay per
        // candidate, then kTimedRounds rounds of one timed replay each, the
        // candidates in turn; each keeps its fastest.  (A replay of a
        // microsecond-scale launch lasts tens of microseconds, so one
        // disturbed replay could otherwise decide.)
        float warm = 0;
        for (int k = 0; k < kWarmMaxTrials && warm < kWarmMs; ++k) {
            float ms = 0;
            CHK(time_replay(b, tg[def], &ms));
            warm += ms;
        }
        std::vector<float> tmin(cands.size(), 1e30f);
        for (size_t k = 0; k < cands.size(); ++k) {
            float ms = 0;
            CHK(time_replay(b, tg[k], &ms));
        }
        for (int round = 0; round < kTimedRounds; ++round)
            for (size_t k = 0; k < cands.size(); ++k) {
                float ms = 0;
                CHK(time_replay(b, tg[k], &ms));
                tmin[k] = std::min(tmin[k], ms);
            }
        int best_b = g.block;
        float best = 1e30f;
        for (size_t k = 0; k < cands.size(); ++k)
            if (tmin[k] < best) {
                best = tmin[k];
                best_b = cands[k];
            }
        g.block = best_b;
        tune_store(key, best_b);
    }
    b->tuned = true;
    b->n_autotunes += 1;
    return SHAKEN_OK;
}

shaken_status batch_build_graph(shaken_batch *b, int chunk) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    shaken_status st = SHAKEN_OK;
    for (int k = 0; k < 2 * chunk && st == SHAKEN_OK; ++k)
        st = batch_half(b, b->dstate, (uint32_t)k, 0, (k & 1) == 0);
    if (st == SHAKEN_OK) {
        hipError_t e = launch_advance(b->dstate, (uint32_t)(2 * chunk), b->stream);
        if (e != hipSuccess) st = fail(SHAKEN_EDEVICE, hipGetErrorString(e));
    }
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &gr);
    if (st != SHAKEN_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return st;
    }
    if (e != hipSuccess) return fail(SHAKEN_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    b->graph = gr;
    HIPCHK(hipGraphInstantiate(&b->gexec, gr, nullptr, nullptr, 0));
    b->chunk = chunk;
    b->n_captures += 1;
    return SHAKEN_OK;
}

// Persistent strategy: capture the queue reset and the persistent launch; the
// start half-step and the number of full steps are read from dstate[0..1],
// so one capture serves every call.
shaken_status batch_build_pgraph(shaken_batch *b) {
    if (b->pgexec) (void)hipGraphExecDestroy(b->pgexec);
    if (b->pgraph) (void)hipGraphDestroy(b->pgraph);
    b->pgexec = nullptr;
    b->pgraph = nullptr;
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_set_state((uint32_t *)b->counter, 0u, 0u, b->stream);
    if (e == hipSuccess)
        e = launch_persistent(b->pdescs, (int)b->ctx.size(), b->order, b->counter, 0u, b->dstate, 0,
                              b->record, b->track, b->pblock, b->pgrid, b->stream);
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->stream, &gr);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return fail(SHAKEN_EDEVICE, std::string("persistent graph capture: ") +
                                        hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->pgraph = gr;
    HIPCHK(hipGraphInstantiate(&b->pgexec, gr, nullptr, nullptr, 0));
    b->pg_grid = b->pgrid;
    b->n_captures += 1;
    return SHAKEN_OK;
}

// Persistent strategy: pick the number of resident workgroups (the occupancy
// bound, or one per compute unit) by timing eight full steps of the batch
// with each; the occupancy bound stays unless the other is at least 3 %
// faster (run-to-run noise is about that size).  Every chain's configuration
// is saved before the trials and restored after the last one (a trial's
// timing does not depend on which configuration it starts from), so tuning
// leaves the chains as they were.
shaken_status batch_autotune_persistent(shaken_batch *b) {
    const int n = (int)b->ctx.size();
    std::vector<int> all(n);
    for (int i = 0; i < n; ++i) all[(size_t)i] = i;
    const std::string key = tune_key(b, "persistent", all);
    int cached = 0;
    if (b->autotune == 2 && tune_lookup(key, &cached)) {
        b->pgrid = cached;
        b->ptuned = true;
        return SHAKEN_OK;
    }
    int ncu = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) ncu = prop.multiProcessorCount;
    std::vector<int> cands{b->pgrid};
    if (std::min(n, ncu) != b->pgrid) cands.push_back(std::min(n, ncu));
    std::vector<size_t> off;
    size_t tot = 0;
    for (auto *c : b->ctx) {
        off.push_back(tot);
        tot += (c->spin_bytes() + 255) / 256 * 256;
    }
    uint8_t *save = nullptr;
    CHK(dalloc(&save, tot));
    auto copy_all = [&](bool to_save) -> hipError_t {
        for (int i = 0; i < n; ++i) {
            void *dev = b->ctx[i]->spin[0];
            const hipError_t e = to_save ? hipMemcpyAsync(save + off[i], dev, b->ctx[i]->spin_bytes(),
                                                          hipMemcpyDeviceToDevice, b->stream)
                                         : hipMemcpyAsync(dev, save + off[i], b->ctx[i]->spin_bytes(),
                                                          hipMemcpyDeviceToDevice, b->stream);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    const uint32_t s0 = b->ctx[0]->s;
    // one trial: eight full steps with `grid` workgroups (GPU milliseconds)
    auto trial = [&](int grid, float *ms) -> hipError_t {
        hipError_t e = launch_set_state((uint32_t *)b->counter, 0u, 0u, b->stream);
        if (e == hipSuccess) e = hipEventRecord(b->ev0, b->stream);
        if (e == hipSuccess)
            e = launch_persistent(b->pdescs, n, b->order, b->counter, s0, nullptr, 8, 0, 0, b->pblock, grid,
                                  b->stream);
        if (e == hipSuccess) e = hipEventRecord(b->ev1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(b->ev1);
        if (e == hipSuccess) e = hipEventElapsedTime(ms, b->ev0, b->ev1);
        return e;
    };
    shaken_status st = SHAKEN_OK;
    hipError_t e = copy_all(true);
    // warm phase (steady clocks before the comparison) with the occupancy-bound grid
    float warm = 0;
    for (int k = 0; k < kWarmMaxTrials && warm < kWarmMs && e == hipSuccess; ++k) {
        float ms = 0;
        e = trial(b->pgrid, &ms);
        warm += ms;
    }
    float best = 1e30f;
    int best_g = b->pgrid;
    for (size_t k = 0; k < cands.size() && e == hipSuccess; ++k) {
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first run warms the caches
            float ms = 0;
            e = trial(cands[k], &ms);
            if (e == hipSuccess && rep == 1 && (k == 0 || ms < 0.97f * best)) {
                best = ms;
                best_g = cands[k];
            }
        }
    }
    if (e == hipSuccess) e = copy_all(false);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) st = fail(SHAKEN_EDEVICE, std::string("persistent autotune: ") + hipGetErrorString(e));
    dfree(save);
    if (st != SHAKEN_OK) return st;
    b->pgrid = best_g;
    b->ptuned = true;
    b->n_autotunes += 1;
    tune_store(key, best_g);
    return SHAKEN_OK;
}

shaken_status batch_sweep_grid(shaken_batch *b, int64_t n_full) {
    const uint32_t s0 = b->ctx[0]->s;
    uint32_t s = s0;
    int64_t t = 0;
    if (n_full > 0) CHK(batch_pack_mirrors(b, s0, false));
    if (b->use_graph) {
        // one graph of kGraphChunk full steps, captured on the first call
        // whatever its length, replayed as often as it fits; the remainder
        // runs eagerly (a call never captures again unless the log space or
        // the launch shapes changed)
        if (!b->gexec) CHK(batch_build_graph(b, kGraphChunk));
        const int64_t reps = n_full / kGraphChunk;
        if (reps > 0) {
            HIPCHK(launch_set_state(b->dstate, s0, s0, b->stream));
            for (int64_t r = 0; r < reps; ++r) HIPCHK(hipGraphLaunch(b->gexec, b->stream));
        }
        t = reps * kGraphChunk;
        s = s0 + (uint32_t)(2 * t);
    }
    for (; t < n_full; ++t) {
        CHK(batch_half(b, nullptr, s, s0, true));
        CHK(batch_half(b, nullptr, s + 1, s0, false));
        s += 2;
    }
    return SHAKEN_OK;
}

}  // namespace

extern "C" {

shaken_status shaken_batch_create(shaken_batch **out, shaken_ctx *const *ctx, int32_t n,
                                  const shaken_batch_opts *opts) {
    g_err.clear();
    if (!out || !ctx || n < 1) return fail(SHAKEN_EINVAL, "need out, ctx and n >= 1");
    *out = nullptr;
    shaken_batch_opts o{};
    if (opts) o = *opts;
    for (int i = 0; i < n; ++i) {
        if (!ctx[i]) return fail(SHAKEN_EINVAL, "ctx[" + std::to_string(i) + "] is NULL");
        if (ctx[i]->device != ctx[0]->device) return fail(SHAKEN_EINVAL, "contexts on different devices");
        if (ctx[i]->s != ctx[0]->s) return fail(SHAKEN_ESTATE, "contexts have different half-step counters");
        for (int j = 0; j < i; ++j)
            if (ctx[j] == ctx[i]) return fail(SHAKEN_EINVAL, "a context appears twice");
    }
    if (ctx[0]->s & 1u) return fail(SHAKEN_ESTATE, "batches need an even half-step counter");
    if (o.strategy < SHAKEN_BATCH_AUTO || o.strategy > SHAKEN_BATCH_PERSISTENT)
        return fail(SHAKEN_EINVAL, "unknown batch strategy");
    if (o.log_reserve < 0) return fail(SHAKEN_EINVAL, "log_reserve must be >= 0");
    if (o.autotune < 0 || o.autotune > 2) return fail(SHAKEN_EINVAL, "autotune must be 0, 1 or 2");
    shaken_batch *b = new (std::nothrow) shaken_batch();
    if (!b) return fail(SHAKEN_ENOMEM, "host allocation failed");
    b->ctx.assign(ctx, ctx + n);
    b->device = ctx[0]->device;
    DeviceGuard guard(b->device);
    b->use_graph = o.use_hipgraph;
    b->autotune = o.autotune;
    b->record = o.record;
    b->track = o.track;
    b->stream = o.stream ? (hipStream_t)o.stream : ctx[0]->stream;
    shaken_status st = SHAKEN_OK;
    auto bail = [&](shaken_status s) {
        batch_release(b);
        delete b;
        return s;
    };
    // HIP graphs (and the autotuner's trial graphs) cannot be captured on the
    // legacy null stream: such a batch gets a stream of its own (a blocking
    // one, ordered with the null stream the chains may use on their own)
    if (!b->stream && (b->use_graph || b->autotune)) {
        if (hipStreamCreate(&b->stream) != hipSuccess) return bail(fail(SHAKEN_EDEVICE, "hipStreamCreate failed"));
        b->own_stream = true;
    }
    // work queued on the chains' own streams must finish first
    for (int i = 0; i < n; ++i)
        if (hipStreamSynchronize(ctx[i]->stream) != hipSuccess) return bail(fail(SHAKEN_EDEVICE, "stream sync failed"));
    if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess)
        return bail(fail(SHAKEN_EDEVICE, "hipEventCreate failed"));
    bool all_fit = true;
    for (int i = 0; i < n; ++i) all_fit = all_fit && persistent_fits(ctx[i]->hd);
    int strat = o.strategy;
    // AUTO: LDS-resident spins win wherever every chain fits (measured 4.6x
    // over the grid kernels on 1024 graphs of 1K-64K vertices, 1.2-1.9x on
    // batches of 32^2..256^2 square, +-J and triangular tori); larger tori
    // run on the grid kernels.
    if (strat == SHAKEN_BATCH_AUTO) strat = all_fit ? SHAKEN_BATCH_PERSISTENT : SHAKEN_BATCH_GRID;
    if (strat == SHAKEN_BATCH_PERSISTENT && !all_fit)
        return bail(fail(SHAKEN_EINVAL, "a chain does not fit the persistent strategy"));
    if (b->track && strat != SHAKEN_BATCH_PERSISTENT)
        return bail(fail(SHAKEN_EINVAL, "tracking needs the persistent strategy"));
    b->strategy = strat;
    b->log_parts = strat == SHAKEN_BATCH_PERSISTENT ? 1 : kLogParts;
    if (b->record && o.log_reserve > 0) {
        bool changed = false;
        if ((st = batch_ensure_log(b, (int64_t)o.log_reserve + 1, &changed)) != SHAKEN_OK) return bail(st);
    }
    // threshold pool (current tables of every chain)
    {
        size_t tot = 0;
        for (int i = 0; i < n; ++i) {
            b->lut_off.push_back(tot);
            tot += ctx[i]->lut.size();
        }
        b->lut_host.resize(tot);
        for (int i = 0; i < n; ++i)
            std::copy(ctx[i]->lut.begin(), ctx[i]->lut.end(), b->lut_host.begin() + b->lut_off[i]);
        if ((st = dalloc(&b->lut_pool, tot)) != SHAKEN_OK) return bail(st);
        if (hipMemcpy(b->lut_pool, b->lut_host.data(), tot * 8, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(SHAKEN_EDEVICE, "threshold upload failed"));
    }
    if (b->track) {
        size_t tot = 0;
        for (int i = 0; i < n; ++i) {
            if (!ctx[i]->lam2_int) return bail(fail(SHAKEN_EINVAL, "tracking needs every 2*lambda to be an integer"));
            b->best_off.push_back(tot);
            tot += bit_words(ctx[i]);
        }
        if ((st = dalloc(&b->track_pool, 2 * (size_t)n)) != SHAKEN_OK) return bail(st);
        if ((st = dalloc(&b->best_pool, tot)) != SHAKEN_OK) return bail(st);
    }
    if ((st = dalloc(&b->dstate, 2)) != SHAKEN_OK) return bail(st);
    if (strat == SHAKEN_BATCH_GRID) {
        // group by (kind, format): one launch per group and half-step
        for (int i = 0; i < n; ++i) {
            Group *g = nullptr;
            for (auto &x : b->groups)
                if (x.kind == ctx[i]->kind && x.format == ctx[i]->format && x.tri == (int)ctx[i]->tri) g = &x;
            if (!g) {
                b->groups.emplace_back();
                g = &b->groups.back();
                g->kind = ctx[i]->kind;
                g->format = ctx[i]->format;
                g->tri = ctx[i]->tri;
            }
            g->members.push_back(i);
            g->hd.push_back(ctx[i]->hd);
        }
        for (auto &g : b->groups) {
            if ((st = dalloc(&g.dd, g.hd.size())) != SHAKEN_OK) return bail(st);
            g.block = group_default_block(b, g);
        }
    } else {
        b->phd.resize(n);
        if ((st = dalloc(&b->pdescs, (size_t)n)) != SHAKEN_OK) return bail(st);
        if ((st = dalloc(&b->order, (size_t)n)) != SHAKEN_OK) return bail(st);
        if ((st = dalloc(&b->counter, 2)) != SHAKEN_OK) return bail(st);
        // longest first: cost ~ sites (tori) or sites + edges (graphs)
        std::vector<std::pair<double, int>> cost;
        for (int i = 0; i < n; ++i) {
            const shaken_ctx *c = ctx[i];
            const double w = c->kind == KIND_TORUS ? (double)c->n : 3.0 * (double)(c->n + c->m);
            cost.push_back({-w, i});
        }
        std::sort(cost.begin(), cost.end());
        std::vector<int32_t> ord;
        for (auto &p : cost) ord.push_back(p.second);
        if (hipMemcpy(b->order, ord.data(), ord.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(SHAKEN_EDEVICE, "order upload failed"));
        int ncu = 256;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) ncu = prop.multiProcessorCount;
        // as many workgroups as are resident at once: each loops over the queue
        b->pgrid = std::min(n, persistent_resident_blocks() * ncu);
    }
    if ((st = batch_upload(b)) != SHAKEN_OK) return bail(st);
    *out = b;
    return SHAKEN_OK;
}

shaken_status shaken_batch_sweep(shaken_batch *b, int64_t n_full) {
    if (!b) return fail(SHAKEN_EINVAL, "batch is NULL");
    if (n_full < 0) return fail(SHAKEN_EINVAL, "n_full must be >= 0");
    DeviceGuard guard(b->device);
    const uint32_t s0 = b->ctx[0]->s;
    if ((int64_t)s0 + 2 * n_full >= (int64_t)kInitStep) return fail(SHAKEN_ESTATE, "half-step counter would overflow");
    if (s0 & 1u) return fail(SHAKEN_ESTATE, "batches need an even half-step counter");
    bool moved = false;
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        shaken_ctx *c = b->ctx[i];
        if (c->s != s0) return fail(SHAKEN_ESTATE, "a context of the batch was stepped on its own");
        // a checkpoint restore on a member (shaken_set_half_step) can swap its
        // two spin buffers: the device descriptors must follow
        moved |= b->up_spin[i].first != c->spin[0] || b->up_spin[i].second != c->spin[1];
    }
    if (moved) CHK(batch_upload(b));
    if (b->record) {
        bool changed = false;
        CHK(batch_ensure_log(b, n_full + 1, &changed));
        // the grid kernels add partial sums into the slots; the persistent
        // kernel writes every slot it logs
        if (b->strategy == SHAKEN_BATCH_GRID)
            HIPCHK(launch_fill_i64(b->log_pool, (n_full + 1) * b->log_row, 0, b->stream));
        if (changed) {
            CHK(batch_upload(b));
            if (b->gexec) {
                (void)hipGraphExecDestroy(b->gexec);
                b->gexec = nullptr;
            }
        }
    }
    if (b->strategy == SHAKEN_BATCH_GRID && b->autotune && !b->tuned) {
        CHK(batch_autotune(b));
        if (b->gexec) {
            (void)hipGraphExecDestroy(b->gexec);
            b->gexec = nullptr;
        }
    }
    if (b->strategy == SHAKEN_BATCH_PERSISTENT && b->autotune && !b->ptuned) CHK(batch_autotune_persistent(b));
    HIPCHK(hipEventRecord(b->ev0, b->stream));
    if (b->strategy == SHAKEN_BATCH_GRID) {
        CHK(batch_sweep_grid(b, n_full));
    } else if (b->use_graph) {
        // captured on the first call (n_full = 0 included): the start
        // half-step and the length come from device memory
        if (!b->pgexec || b->pg_grid != b->pgrid) CHK(batch_build_pgraph(b));
        HIPCHK(launch_set_state(b->dstate, s0, (uint32_t)n_full, b->stream));
        HIPCHK(hipGraphLaunch(b->pgexec, b->stream));
    } else {
        HIPCHK(launch_set_state((uint32_t *)b->counter, 0u, 0u, b->stream));
        HIPCHK(launch_persistent(b->pdescs, (int)b->ctx.size(), b->order, b->counter, s0, nullptr, n_full,
                                 b->record, b->track, b->pblock, b->pgrid, b->stream));
    }
    const uint32_t s1 = s0 + (uint32_t)(2 * n_full);
    if (b->record) {
        // observables of the final configuration (spin[s1 & 1]) into slot n_full
        // (the persistent kernel records the final slot itself)
        if (b->strategy == SHAKEN_BATCH_GRID) {
            for (auto &g : b->groups)
                HIPCHK(launch_observe(g.dd, g.hd.data(), (int)g.hd.size(), (int)(s1 & 1u), (int)n_full, b->stream));
        }
    }
    HIPCHK(hipEventRecord(b->ev1, b->stream));
    b->timed = true;
    for (auto *c : b->ctx) c->s = s1;
    b->last_n_full = n_full;
    b->n_sweeps += 1;
    return SHAKEN_OK;
}

namespace {

shaken_status batch_read_log(shaken_batch *b, int32_t i, int64_t *H_out, int64_t *M_out, int64_t *EJ_out,
                             int64_t cap) {
    if (!b || i < 0 || i >= (int32_t)b->ctx.size()) return fail(SHAKEN_EINVAL, "bad batch or index");
    if (!b->record || b->last_n_full < 0) return fail(SHAKEN_ESTATE, "no recorded sweep");
    shaken_ctx *c = b->ctx[i];
    if (H_out && !c->lam2_int) return fail(SHAKEN_EINVAL, "H_out needs every 2*lambda to be an integer");
    const int64_t slots = b->last_n_full + 1;
    if (cap < slots) return fail(SHAKEN_EINVAL, "capacity too small");
    DeviceGuard guard(b->device);
    // one line per slot (persistent): only its used values cross the bus
    const int64_t ln = b->log_parts == 1 ? c->nvals() : c->line();
    const int64_t width = b->log_parts == 1 ? ln : b->log_parts * c->line();
    std::vector<int64_t> raw((size_t)(slots * width));
    HIPCHK(hipMemcpy2DAsync(raw.data(), (size_t)width * 8, b->log_pool + b->log_off[i], (size_t)b->log_row * 8,
                            (size_t)width * 8, (size_t)slots, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    convert_log(c, raw, slots, b->log_parts, H_out, M_out, EJ_out, ln);
    return SHAKEN_OK;
}

}  // namespace

shaken_status shaken_batch_get_log(shaken_batch *b, int32_t i, int64_t *H_out, int64_t *M_out,
                                   int64_t cap) {
    return batch_read_log(b, i, H_out, M_out, nullptr, cap);
}

shaken_status shaken_batch_get_log_ej(shaken_batch *b, int32_t i, int64_t *EJ_out, int64_t *M_out,
                                      int64_t cap) {
    if (!EJ_out) return fail(SHAKEN_EINVAL, "EJ_out is NULL");
    return batch_read_log(b, i, nullptr, M_out, EJ_out, cap);
}

shaken_status shaken_batch_get_logs(shaken_batch *b, int64_t *H_out, int64_t *M_out, int64_t *EJ_out,
                                    int64_t cap) {
    if (!b) return fail(SHAKEN_EINVAL, "batch is NULL");
    if (!H_out && !M_out && !EJ_out) return fail(SHAKEN_EINVAL, "every output is NULL");
    if (!b->record || b->last_n_full < 0) return fail(SHAKEN_ESTATE, "no recorded sweep");
    const int64_t slots = b->last_n_full + 1;
    if (cap < slots) return fail(SHAKEN_EINVAL, "capacity too small");
    if (H_out)
        for (auto *c : b->ctx)
            if (!c->lam2_int) return fail(SHAKEN_EINVAL, "H_out needs every 2*lambda to be an integer");
    DeviceGuard guard(b->device);
    // the slots of this call are contiguous in the slot-major pool: one copy
    std::vector<int64_t> pool((size_t)(slots * b->log_row));
    HIPCHK(hipMemcpyAsync(pool.data(), b->log_pool, pool.size() * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        shaken_ctx *c = b->ctx[i];
        const int64_t width = b->log_parts * c->line();
        std::vector<int64_t> raw((size_t)(slots * width));
        for (int64_t t = 0; t < slots; ++t)
            std::copy_n(pool.begin() + t * b->log_row + b->log_off[i], width, raw.begin() + t * width);
        const int64_t o = (int64_t)i * cap;
        convert_log(c, raw, slots, b->log_parts, H_out ? H_out + o : nullptr, M_out ? M_out + o : nullptr,
                    EJ_out ? EJ_out + o : nullptr);
    }
    return SHAKEN_OK;
}

shaken_status shaken_batch_set_params(shaken_batch *b, const double *beta, const double *q) {
    if (!b || !beta || !q) return fail(SHAKEN_EINVAL, "batch, beta and q must be non-NULL");
    const size_t n = b->ctx.size();
    for (size_t i = 0; i < n; ++i)
        if (!finite_nonneg(beta[i]) || !finite_nonneg(q[i]))
            return fail(SHAKEN_EINVAL, "beta and q must be finite and >= 0 (chain " + std::to_string(i) + ")");
    DeviceGuard guard(b->device);
    HIPCHK(hipStreamSynchronize(b->stream));
    bool fold_changed = false;
    for (size_t i = 0; i < n; ++i) {
        shaken_ctx *c = b->ctx[i];
        const int fold_before = c->hd.fold3;
        c->beta = beta[i];
        c->q = q[i];
        build_tables(c);
        c->lut_stale = true;
        fold_changed |= fold_before != c->hd.fold3;
        std::copy(c->lut.begin(), c->lut.end(), b->lut_host.begin() + b->lut_off[i]);
    }
    HIPCHK(hipMemcpyAsync(b->lut_pool, b->lut_host.data(), b->lut_host.size() * 8,
                          hipMemcpyHostToDevice, b->stream));
    CHK(batch_upload(b));
    if (fold_changed && b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    return SHAKEN_OK;
}

shaken_status shaken_batch_get_track(shaken_batch *b, int64_t *H_last, int64_t *H_best,
                                     int8_t *best_spins) {
    if (!b) return fail(SHAKEN_EINVAL, "batch is NULL");
    if (!b->track || b->last_n_full < 0) return fail(SHAKEN_ESTATE, "no tracked sweep");
    DeviceGuard guard(b->device);
    const size_t n = b->ctx.size();
    std::vector<int64_t> tr(2 * n);
    HIPCHK(hipMemcpyAsync(tr.data(), b->track_pool, tr.size() * 8, hipMemcpyDeviceToHost, b->stream));
    std::vector<uint32_t> w;
    if (best_spins) {
        w.resize(b->best_off.back() + bit_words(b->ctx.back()));
        HIPCHK(hipMemcpyAsync(w.data(), b->best_pool, w.size() * 4, hipMemcpyDeviceToHost, b->stream));
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    size_t off = 0;
    for (size_t i = 0; i < n; ++i) {
        if (H_last) H_last[i] = tr[2 * i];
        if (H_best) H_best[i] = tr[2 * i + 1];
        if (best_spins) {
            shaken_ctx *c = b->ctx[i];
            const uint32_t *wi = w.data() + b->best_off[i];
            if (c->kind == KIND_TORUS) {
                std::vector<uint32_t> tmp(wi, wi + bit_words(c));
                unpack_torus(tmp, c->L, c->W, best_spins + off);
            } else {
                for (int v = 0; v < c->n; ++v) best_spins[off + v] = ((wi[v >> 5] >> (v & 31)) & 1u) ? 1 : -1;
            }
            off += (size_t)c->n;
        }
    }
    return SHAKEN_OK;
}

shaken_status shaken_batch_info(shaken_batch *b, int32_t *strategy, double *last_ms) {
    if (!b) return fail(SHAKEN_EINVAL, "batch is NULL");
    if (strategy) *strategy = b->strategy;
    if (last_ms) {
        *last_ms = 0;
        if (b->timed) {
            DeviceGuard guard(b->device);
            float ms = 0;
            HIPCHK(hipEventSynchronize(b->ev1));
            HIPCHK(hipEventElapsedTime(&ms, b->ev0, b->ev1));
            *last_ms = ms;
        }
    }
    return SHAKEN_OK;
}

shaken_status shaken_batch_counters(shaken_batch *b, shaken_batch_counts *out) {
    if (!b || !out) return fail(SHAKEN_EINVAL, "batch and out must be non-NULL");
    out->sweeps = b->n_sweeps;
    out->captures = b->n_captures;
    out->log_allocs = b->n_log_allocs;
    out->autotunes = b->n_autotunes;
    out->uploads = b->n_uploads;
    return SHAKEN_OK;
}

shaken_status shaken_batch_launch_shape(shaken_batch *b, int32_t i, int32_t *block) {
    if (!b || !block || i < 0 || i >= (int32_t)b->ctx.size()) return fail(SHAKEN_EINVAL, "bad batch, index or output");
    *block = 0;
    for (const auto &g : b->groups)
        for (int m : g.members)
            if (m == i) *block = g.block;
    return SHAKEN_OK;
}

shaken_status shaken_batch_free(shaken_batch *b) {
    if (!b) return SHAKEN_OK;
    DeviceGuard guard(b->device);
    (void)hipStreamSynchronize(b->stream);
    batch_release(b);
    delete b;
    return SHAKEN_OK;
}

}  // extern "C"

// =========================================================== one-call runs

namespace shaken {
// the network's device and stream (defined with the network)
int mlp_device(const shaken_mlp *m);
hipStream_t mlp_stream(const shaken_mlp *m);
}  // namespace shaken

namespace {

constexpr int kFeat = SHAKEN_MLP_IN;

// the geometric schedule at chunk c of C: (log beta, log q)
void geometric_at(const shaken_schedule &s, int64_t c, int64_t C, double *lb, double *lq) {
    const double t = ((double)c + 0.5) / (double)C;
    const double l0 = std::log(s.beta0), l1 = std::log(s.beta1);
    *lb = l0 + t * (l1 - l0);
    *lq = std::log(s.q);
}

// energies after a sweep: H of the last configuration and the lowest H over
// the call's full-step configurations, per chain (track on the persistent
// strategy, the observables log on the grid strategy)
shaken_status call_energies(shaken_batch *b, int64_t n_full, std::vector<int64_t> &last,
                            std::vector<int64_t> &best) {
    const size_t n = b->ctx.size();
    last.resize(n);
    best.resize(n);
    if (b->track) return shaken_batch_get_track(b, last.data(), best.data(), nullptr);
    const int64_t cap = n_full + 1;
    std::vector<int64_t> H((size_t)(n * cap));
    CHK(shaken_batch_get_logs(b, H.data(), nullptr, nullptr, cap));
    for (size_t i = 0; i < n; ++i) {
        const int64_t *h = H.data() + i * cap;
        last[i] = h[cap - 1];
        best[i] = *std::min_element(h, h + cap);
    }
    return SHAKEN_OK;
}

struct RunState {
    shaken_batch *b = nullptr;
    float *x = nullptr, *y = nullptr;  // network features and outputs (device)
    ~RunState() {
        if (b) shaken_batch_free(b);
        dfree(x);
        dfree(y);
    }
};

}  // namespace

extern "C" {

shaken_status shaken_batch_run(shaken_ctx *const *ctx, int32_t n, int64_t n_full,
                               const shaken_batch_opts *opts, const shaken_schedule *sched,
                               shaken_run_result *res) {
    g_err.clear();
    if (!ctx || n < 1) return fail(SHAKEN_EINVAL, "need ctx and n >= 1");
    if (n_full < 0) return fail(SHAKEN_EINVAL, "n_full must be >= 0");
    for (int i = 0; i < n; ++i)
        if (!ctx[i]) return fail(SHAKEN_EINVAL, "ctx[" + std::to_string(i) + "] is NULL");
    shaken_schedule sc{};
    if (sched) sc = *sched;
    if (sc.kind < SHAKEN_SCHEDULE_NONE || sc.kind > SHAKEN_SCHEDULE_MLP)
        return fail(SHAKEN_EINVAL, "unknown schedule kind");
    const bool scheduled = sc.kind != SHAKEN_SCHEDULE_NONE;
    int64_t chunk = n_full, chunks = 1;
    if (scheduled) {
        if (sc.chunk_sweeps < 1) return fail(SHAKEN_EINVAL, "chunk_sweeps must be >= 1");
        if (n_full % sc.chunk_sweeps) return fail(SHAKEN_EINVAL, "n_full must be a multiple of chunk_sweeps");
        chunk = sc.chunk_sweeps;
        chunks = n_full / chunk;
        if (!(std::isfinite(sc.beta0) && sc.beta0 > 0 && std::isfinite(sc.beta1) && sc.beta1 > 0))
            return fail(SHAKEN_EINVAL, "geometric schedule: beta0 and beta1 must be finite and > 0");
        if (!finite_nonneg(sc.q) || sc.q == 0.0)
            return fail(SHAKEN_EINVAL, "geometric schedule: q must be finite and > 0");
        if (sc.kind == SHAKEN_SCHEDULE_MLP) {
            if (!sc.mlp) return fail(SHAKEN_EINVAL, "schedule MLP needs the network");
            if (shaken::mlp_device(sc.mlp) != ctx[0]->device)
                return fail(SHAKEN_EINVAL, "the network is on another device");
        }
    }
    const bool want_best = res && (res->H_best || res->best_spins);
    const bool energies = (res && (res->H_final || want_best)) || sc.kind == SHAKEN_SCHEDULE_MLP;
    shaken_batch_opts o{};
    if (opts) o = *opts;
    if (energies) {
        for (int i = 0; i < n; ++i)
            if (!ctx[i]->lam2_int) return fail(SHAKEN_EINVAL, "energies need every 2*lambda to be an integer");
        bool all_fit = true;
        for (int i = 0; i < n; ++i) all_fit = all_fit && persistent_fits(ctx[i]->hd);
        int strat = o.strategy == SHAKEN_BATCH_AUTO ? (all_fit ? SHAKEN_BATCH_PERSISTENT : SHAKEN_BATCH_GRID)
                                                    : o.strategy;
        o.strategy = strat;
        if (strat == SHAKEN_BATCH_PERSISTENT) {
            o.track = 1;
        } else {
            if (res && res->best_spins) return fail(SHAKEN_EINVAL, "best_spins needs the persistent strategy");
            o.record = 1;
            o.log_reserve = (int32_t)std::min<int64_t>(std::max<int64_t>(o.log_reserve, chunk), INT32_MAX);
        }
    }
    RunState rs;
    CHK(shaken_batch_create(&rs.b, ctx, n, &o));
    shaken_batch *b = rs.b;
    DeviceGuard guard(b->device);
    const size_t N = (size_t)n;
    // the run's energies: current and lowest so far, and the best configurations
    std::vector<int64_t> e_cur(N, 0), e_best(N, 0), last, best;
    std::vector<int8_t> best_sp;
    std::vector<size_t> sp_off(N + 1, 0);
    for (size_t i = 0; i < N; ++i) sp_off[i + 1] = sp_off[i] + (size_t)ctx[i]->n;
    auto take_best = [&](bool first) -> shaken_status {
        bool improved = first;
        for (size_t i = 0; i < N && !improved; ++i) improved = best[i] < e_best[i];
        if (res && res->best_spins && improved) {
            std::vector<int8_t> sp(sp_off[N]);
            CHK(shaken_batch_get_track(b, nullptr, nullptr, sp.data()));
            for (size_t i = 0; i < N; ++i)
                if (first || best[i] < e_best[i])
                    std::copy(sp.begin() + (ptrdiff_t)sp_off[i], sp.begin() + (ptrdiff_t)sp_off[i + 1],
                              best_sp.begin() + (ptrdiff_t)sp_off[i]);
        }
        for (size_t i = 0; i < N; ++i) e_best[i] = first ? best[i] : std::min(e_best[i], best[i]);
        for (size_t i = 0; i < N; ++i) e_cur[i] = last[i];
        return SHAKEN_OK;
    };
    if (res && res->best_spins) best_sp.assign(sp_off[N], 0);
    if (energies) {
        // energies of the start (a sweep of no steps)
        CHK(shaken_batch_sweep(b, 0));
        CHK(call_energies(b, 0, last, best));
        CHK(take_best(true));
    }
    const bool use_mlp = sc.kind == SHAKEN_SCHEDULE_MLP;
    std::vector<float> F, Y;
    hipStream_t ms = nullptr;
    if (use_mlp) {
        F.assign(N * kFeat, 0.f);
        Y.assign(N * kFeat, 0.f);
        CHK(dalloc(&rs.x, N * kFeat));
        CHK(dalloc(&rs.y, N * kFeat));
        ms = shaken::mlp_stream(sc.mlp);
    }
    const double lb_lo = std::log(0.05), lb_hi = std::log(20.0);
    const double lq_lo = std::log(0.05), lq_hi = std::log(8.0);
    std::vector<double> lb_prev(N, 0.0), lq_prev(N, 0.0), beta(N), q(N);
    int64_t fallbacks = 0;
    for (int64_t c = 0; c < chunks; ++c) {
        if (scheduled) {
            double glb, glq;
            geometric_at(sc, c, chunks, &glb, &glq);
            std::vector<double> lb(N, glb), lq(N, glq);
            if (use_mlp) {
                for (size_t i = 0; i < N; ++i) {
                    const shaken_ctx *x = ctx[i];
                    const double sites = (double)x->n;
                    float *f = F.data() + i * kFeat;
                    f[0] = (float)(std::log2(sites) / 16.0);
                    f[1] = (float)(x->deg_mean / 4.0);
                    f[2] = (float)(x->deg_spread / 2.0);
                    f[3] = (float)((double)c / (double)chunks);
                    f[4] = (float)((double)e_cur[i] / sites);
                    f[5] = (float)((double)e_best[i] / sites);
                    f[6] = (float)(lb_prev[i] / 3.0);
                    f[7] = (float)(lq_prev[i] / 3.0);
                    f[8] = 1.0f;
                }
                HIPCHK(hipMemcpyAsync(rs.x, F.data(), F.size() * 4, hipMemcpyHostToDevice, ms));
                CHK(shaken_mlp_forward(sc.mlp, rs.x, n, rs.y));
                HIPCHK(hipMemcpyAsync(Y.data(), rs.y, Y.size() * 4, hipMemcpyDeviceToHost, ms));
                HIPCHK(hipStreamSynchronize(ms));
                for (size_t i = 0; i < N; ++i) {
                    const double a = (double)Y[i * kFeat], bq = (double)Y[i * kFeat + 1];
                    if (std::isfinite(a) && std::isfinite(bq)) {
                        lb[i] = a;
                        lq[i] = bq;
                    } else {
                        ++fallbacks;
                    }
                }
            }
            for (size_t i = 0; i < N; ++i) {
                lb[i] = std::min(std::max(lb[i], lb_lo), lb_hi);
                lq[i] = std::min(std::max(lq[i], lq_lo), lq_hi);
                beta[i] = std::exp(lb[i]);
                q[i] = std::exp(lq[i]);
                if (res && res->beta_used) res->beta_used[(size_t)c * N + i] = beta[i];
                if (res && res->q_used) res->q_used[(size_t)c * N + i] = q[i];
            }
            CHK(shaken_batch_set_params(b, beta.data(), q.data()));
            lb_prev = lb;
            lq_prev = lq;
        }
        CHK(shaken_batch_sweep(b, chunk));
        if (energies) {
            CHK(call_energies(b, chunk, last, best));
            CHK(take_best(false));
        }
    }
    if (!energies || chunks == 0) HIPCHK(hipStreamSynchronize(b->stream));
    if (res) {
        res->chunks = scheduled ? chunks : (n_full > 0 ? 1 : 0);
        res->fallbacks = fallbacks;
        for (size_t i = 0; i < N; ++i) {
            if (res->H_final) res->H_final[i] = e_cur[i];
            if (res->H_best) res->H_best[i] = e_best[i];
        }
        if (res->best_spins) std::copy(best_sp.begin(), best_sp.end(), res->best_spins);
    }
    return SHAKEN_OK;
}

}  // extern "C"
