/*
 * Plain, single-threaded CPU oracle of shaken dynamics (Apollonio, D'Autilia,
 * Scoppola, Scoppola, Troiani, "Shaken dynamics: an easy way to parallel Markov
 * Chain Monte Carlo", arXiv:1904.06257).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * implementation: every formula below is written out again from the paper and
 * from the randomness contract stated in this header.
 *
 * What is computed (paper section 2, equations ham21 and the two half-step
 * kernels P^{1->2}, P^{2->1}; section 3, equations hur, hdl, pasymm, pasymm1):
 *
 *   half-step 1 (1->2):  sigma'_x ~ exp(beta h_x sigma'_x) / (2 cosh(beta h_x)),
 *                        h_x = sum_{y:(y,x) in E^o} J_yx sigma_y + q sigma_x + lambda_x
 *   half-step 2 (2->1):  tau_x    ~ exp(beta h_x tau_x)    / (2 cosh(beta h_x)),
 *                        h_x = sum_{y:(x,y) in E^o} J_xy sigma'_y + q sigma'_x + lambda_x
 *
 * i.e. P(new spin = +1) = 1 / (1 + exp(-2 beta h_x)), every site redrawn at once
 * from the previous configuration only (double buffering, never in place).
 * On the L x L torus E^o = {(x, x_up), (x, x_right)}, so half-step 1 reads the
 * down and left neighbours (P^dl) and half-step 2 the up and right ones (P^ur);
 * a full step is P^dl followed by P^ur (section 3, definition of P^sh).
 * Sites are (row, col) with row-major index row*L + col; "up" is row+1 and
 * "right" is col+1, both modulo L.  This is the reading under which the
 * zero-temperature diagonal growth printed in the proof of Theorem 3.3 is
 * reproduced.
 *
 * Randomness contract (the paper fixes none; this is the project's own).
 *   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = (lo32(seed),
 *   hi32(seed)), counter = (c0, c1, c2, c3).
 *   Threshold of a site with local field h (IEEE double, h evaluated as
 *   ((double)S + q*sigma) + lambda, no contraction):
 *       e = exp(-((2 beta) |h|)),  t = floor(e / (1 + e) * 2^32),
 *       T = 2^32 - t if h >= 0 else t;   new spin = +1 iff u < T.
 *   Torus site (r, c), W = ceil(L/32) words per row, word w = r*W + (c>>5),
 *   bit b = c & 31, half-step index s, replica id p:
 *       R_k = word (k & 3) of Philox((w, s, p, k >> 2)),  k = 0..31
 *       u   = sum_k ((R_k >> b) & 1) * 2^(31-k)        (bit-sliced uniform)
 *   Graph vertex v:
 *       u   = word (v & 3) of Philox((v >> 2, s, p, 0x80000000))
 *   Random initial state: half-step index s = 0xFFFFFFFF; torus site is +1 iff
 *   bit b of R_0 is set; graph vertex is +1 iff bit 31 of its u is set.
 *
 * Observables of a configuration: M = sum_x sigma_x,
 * E_J = sum_{(x,y) in E^o} J_xy sigma_x sigma_y (each undirected edge once), so
 * that H(sigma) = -E_J - sum_x 2 lambda_x sigma_x (equation ham1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TWO32 4294967296.0
#define GRAPH_STREAM 0x80000000u
#define INIT_STEP 0xFFFFFFFFu

/* ---------------------------------------------------------------- Philox -- */

/* Ten rounds of the Philox-4x32 bijection.  One round multiplies counter words
 * 0 and 2 by the two round constants, keeps the low halves, and xors the high
 * halves with the other two counter words and the round key; the key is then
 * advanced by the two Weyl constants. */
void oracle_philox4x32_10(const uint32_t ctr[4], uint64_t seed, uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t a = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t b = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(b >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)b;
        uint32_t y2 = (uint32_t)(a >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------- threshold -- */

/* 33-bit threshold T in [0, 2^32] with P(+1) = T / 2^32 ~ 1/(1+exp(-2 beta h)). */
uint64_t oracle_threshold(double h, double beta)
{
    double e = exp(-((2.0 * beta) * fabs(h)));
    double p_small = e / (1.0 + e);
    uint64_t t = (uint64_t)floor(p_small * TWO32);
    return (h >= 0.0) ? ((uint64_t)1 << 32) - t : t;
}

/* local field h = S + q*sigma + lambda, evaluated left to right in double */
double oracle_field(int64_t S, int sigma, double q, double lam)
{
    double h = (double)S;
    h = h + q * (double)sigma;
    h = h + lam;
    return h;
}

/* ----------------------------------------------------------------- torus -- */

static int torus_words(int L) { return (L + 31) / 32; }

/* the 32 level words R_0..R_31 of torus RNG word w at half-step s */
static void torus_levels(uint64_t seed, uint32_t replica, uint32_t s, uint32_t w,
                         uint32_t R[32])
{
    uint32_t g;
    for (g = 0; g < 8; ++g) {
        uint32_t ctr[4] = {w, s, replica, g};
        oracle_philox4x32_10(ctr, seed, &R[4 * g]);
    }
}

/* bit-sliced uniform of bit b from the 32 level words */
static uint32_t torus_u_from_levels(const uint32_t R[32], int b)
{
    uint32_t u = 0;
    int k;
    for (k = 0; k < 32; ++k)
        u |= ((R[k] >> b) & 1u) << (31 - k);
    return u;
}

uint32_t oracle_torus_uniform(int L, uint64_t seed, uint32_t replica, uint32_t s,
                              int r, int c)
{
    uint32_t R[32];
    uint32_t w = (uint32_t)(r * torus_words(L) + (c >> 5));
    torus_levels(seed, replica, s, w, R);
    return torus_u_from_levels(R, c & 31);
}

void oracle_torus_init_random(int L, uint64_t seed, uint32_t replica, int8_t *spins)
{
    int W = torus_words(L), r, c;
    for (r = 0; r < L; ++r)
        for (c = 0; c < L; ++c) {
            uint32_t ctr[4] = {(uint32_t)(r * W + (c >> 5)), INIT_STEP, replica, 0};
            uint32_t out[4];
            oracle_philox4x32_10(ctr, seed, out);
            spins[r * L + c] = ((out[0] >> (c & 31)) & 1u) ? 1 : -1;
        }
}

/* Coupling-weighted neighbour sum of site (r,c).  The oriented edges of the
 * torus are (x, x_up) with coupling Jup[x] and (x, x_right) with Jr[x]
 * (row-major site index); Jup == NULL means every coupling equals J.
 *   phase 0 (in-half, dl):  Jup[x_down] sigma(x_down) + Jr[x_left] sigma(x_left)
 *   phase 1 (out-half, ur): Jup[x] sigma(x_up) + Jr[x] sigma(x_right)
 * Triangular lattice (section 4; skewed coordinates, uniform J): the third
 * oriented edge (x, x_up_right) adds the diagonal neighbour, down-left in the
 * in-half and up-right in the out-half. */
static int64_t torus_fsum(int L, int J, const int8_t *Jup, const int8_t *Jr, int tri,
                          const int8_t *sp, int r, int c, int phase)
{
    int x = r * L + c;
    if (phase == 0) {
        int xd = ((r - 1 + L) % L) * L + c, xl = r * L + (c - 1 + L) % L;
        if (tri) return (int64_t)J * (sp[xd] + sp[xl] + sp[((r - 1 + L) % L) * L + (c - 1 + L) % L]);
        if (!Jup) return (int64_t)J * (sp[xd] + sp[xl]);
        return (int64_t)Jup[xd] * sp[xd] + (int64_t)Jr[xl] * sp[xl];
    } else {
        int xu = ((r + 1) % L) * L + c, xr = r * L + (c + 1) % L;
        if (tri) return (int64_t)J * (sp[xu] + sp[xr] + sp[((r + 1) % L) * L + (c + 1) % L]);
        if (!Jup) return (int64_t)J * (sp[xu] + sp[xr]);
        return (int64_t)Jup[x] * sp[xu] + (int64_t)Jr[x] * sp[xr];
    }
}

/* new value of one site at half-step s, read from configuration `in` */
/* mode bit 0: the reversed order P^{sh'} = P^{ur} P^{dl} (section 3): the half
 * read at half-step s is (s & 1) ^ 1, i.e. the out-half (ur) at even s.
 * mode bit 1: the triangular lattice (uniform J; Jup must be NULL). */
int oracle_torus_site_j(int L, int J, const int8_t *Jup, const int8_t *Jr, int mode, double lam,
                        double q, double beta, uint64_t seed, uint32_t replica, uint32_t s,
                        const int8_t *in, int r, int c)
{
    int64_t S = torus_fsum(L, J, Jup, Jr, (mode >> 1) & 1, in, r, c, (int)(s & 1u) ^ (mode & 1));
    double h = oracle_field(S, in[r * L + c], q, lam);
    uint64_t T = oracle_threshold(h, beta);
    uint32_t u = oracle_torus_uniform(L, seed, replica, s, r, c);
    return ((uint64_t)u < T) ? 1 : -1;
}

int oracle_torus_site(int L, int J, double lam, double q, double beta, uint64_t seed,
                      uint32_t replica, uint32_t s, const int8_t *in, int r, int c)
{
    return oracle_torus_site_j(L, J, NULL, NULL, 0, lam, q, beta, seed, replica, s, in, r, c);
}

/* one half-step: every site redrawn from `in` into `out` (in != out) */
void oracle_torus_half_step_j(int L, int J, const int8_t *Jup, const int8_t *Jr, int mode,
                              double lam, double q, double beta, uint64_t seed, uint32_t replica,
                              uint32_t s, const int8_t *in, int8_t *out)
{
    int W = torus_words(L), r, wd, b;
    uint32_t R[32];
    for (r = 0; r < L; ++r)
        for (wd = 0; wd < W; ++wd) {
            torus_levels(seed, replica, s, (uint32_t)(r * W + wd), R);
            for (b = 0; b < 32 && 32 * wd + b < L; ++b) {
                int c = 32 * wd + b;
                int64_t S = torus_fsum(L, J, Jup, Jr, (mode >> 1) & 1, in, r, c,
                                       (int)(s & 1u) ^ (mode & 1));
                double h = oracle_field(S, in[r * L + c], q, lam);
                uint64_t T = oracle_threshold(h, beta);
                uint32_t u = torus_u_from_levels(R, b);
                out[r * L + c] = ((uint64_t)u < T) ? 1 : -1;
            }
        }
}

void oracle_torus_half_step(int L, int J, double lam, double q, double beta,
                            uint64_t seed, uint32_t replica, uint32_t s,
                            const int8_t *in, int8_t *out)
{
    oracle_torus_half_step_j(L, J, NULL, NULL, 0, lam, q, beta, seed, replica, s, in, out);
}

/* E_J over the oriented edge set {(x, x_up), (x, x_right)} and M */
void oracle_torus_observe_j(int L, int J, const int8_t *Jup, const int8_t *Jr, int mode,
                            const int8_t *sp, int64_t *EJ, int64_t *M)
{
    int64_t e = 0, m = 0;
    int r, c;
    for (r = 0; r < L; ++r)
        for (c = 0; c < L; ++c) {
            int x = r * L + c;
            int ju = Jup ? Jup[x] : J, jr = Jup ? Jr[x] : J;
            e += (int64_t)ju * sp[x] * sp[((r + 1) % L) * L + c];
            e += (int64_t)jr * sp[x] * sp[r * L + (c + 1) % L];
            if (mode & 2) e += (int64_t)J * sp[x] * sp[((r + 1) % L) * L + (c + 1) % L];
            m += sp[x];
        }
    *EJ = e;
    *M = m;
}

void oracle_torus_observe(int L, int J, const int8_t *sp, int64_t *EJ, int64_t *M)
{
    oracle_torus_observe_j(L, J, NULL, NULL, 0, sp, EJ, M);
}

/* n_full full steps from half-step index s0 (must be even); spins updated in
 * place (through a private second buffer); logs hold n_full+1 entries
 * (configuration at the start and after every full step); NULL skips a log.
 * Returns 0, or -1 on allocation failure / odd s0. */
int oracle_torus_run_j(int L, int J, const int8_t *Jup, const int8_t *Jr, int mode, double lam,
                       double q, double beta, uint64_t seed, uint32_t replica, uint32_t s0,
                       int8_t *spins, int64_t n_full, int64_t *EJ_log, int64_t *M_log)
{
    int8_t *tmp;
    int64_t t;
    uint32_t s = s0;
    if (s0 & 1u) return -1;
    tmp = (int8_t *)malloc((size_t)L * L);
    if (!tmp) return -1;
    for (t = 0; t <= n_full; ++t) {
        int64_t e, m;
        if (EJ_log || M_log) {
            oracle_torus_observe_j(L, J, Jup, Jr, mode, spins, &e, &m);
            if (EJ_log) EJ_log[t] = e;
            if (M_log) M_log[t] = m;
        }
        if (t == n_full) break;
        oracle_torus_half_step_j(L, J, Jup, Jr, mode, lam, q, beta, seed, replica, s, spins, tmp);
        oracle_torus_half_step_j(L, J, Jup, Jr, mode, lam, q, beta, seed, replica, s + 1, tmp, spins);
        s += 2;
    }
    free(tmp);
    return 0;
}

int oracle_torus_run(int L, int J, double lam, double q, double beta, uint64_t seed,
                     uint32_t replica, uint32_t s0, int8_t *spins, int64_t n_full,
                     int64_t *EJ_log, int64_t *M_log)
{
    return oracle_torus_run_j(L, J, NULL, NULL, 0, lam, q, beta, seed, replica, s0, spins, n_full,
                              EJ_log, M_log);
}

/* ----------------------------------------------------------------- graph -- */

uint32_t oracle_graph_uniform(uint64_t seed, uint32_t replica, uint32_t s, uint32_t v)
{
    uint32_t ctr[4] = {v >> 2, s, replica, GRAPH_STREAM};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, seed, out);
    return out[v & 3u];
}

void oracle_graph_init_random(int n, uint64_t seed, uint32_t replica, int8_t *spins)
{
    int v;
    for (v = 0; v < n; ++v)
        spins[v] = (oracle_graph_uniform(seed, replica, INIT_STEP, (uint32_t)v) >> 31) ? 1 : -1;
}

/* One half-step on an arbitrary oriented graph, straight from the definition:
 * S_x accumulates J_e * sigma_tail over the oriented edges e = (tail, head) with
 * x as the head (half-step 1, s even) or, with the roles swapped, as the tail
 * (half-step 2, s odd).  J == NULL means every J_e = +1.  lam_of_class[cls[x]]
 * is lambda_x (cls == NULL means class 0 for all). */
int oracle_graph_half_step(int n, int64_t m, const int32_t *src, const int32_t *dst,
                           const int8_t *J, const uint8_t *cls, const double *lam_of_class,
                           double q, double beta, uint64_t seed, uint32_t replica,
                           uint32_t s, const int8_t *in, int8_t *out)
{
    int64_t *S = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int64_t e;
    int v;
    if (!S) return -1;
    for (e = 0; e < m; ++e) {
        int64_t j = J ? J[e] : 1;
        if ((s & 1u) == 0)
            S[dst[e]] += j * in[src[e]];
        else
            S[src[e]] += j * in[dst[e]];
    }
    for (v = 0; v < n; ++v) {
        double lam = lam_of_class ? lam_of_class[cls ? cls[v] : 0] : 0.0;
        double h = oracle_field(S[v], in[v], q, lam);
        uint64_t T = oracle_threshold(h, beta);
        uint32_t u = oracle_graph_uniform(seed, replica, s, (uint32_t)v);
        out[v] = ((uint64_t)u < T) ? 1 : -1;
    }
    free(S);
    return 0;
}

/* E_J = sum over oriented edges of J_e sigma_src sigma_dst; plus[c] = number of
 * +1 spins in lambda class c (n_classes entries) */
void oracle_graph_observe(int n, int64_t m, const int32_t *src, const int32_t *dst,
                          const int8_t *J, const uint8_t *cls, int n_classes,
                          const int8_t *sp, int64_t *EJ, int64_t *plus)
{
    int64_t e, acc = 0;
    int v;
    for (e = 0; e < m; ++e)
        acc += (int64_t)(J ? J[e] : 1) * sp[src[e]] * sp[dst[e]];
    *EJ = acc;
    for (v = 0; v < n_classes; ++v) plus[v] = 0;
    for (v = 0; v < n; ++v)
        if (sp[v] > 0) plus[cls ? cls[v] : 0] += 1;
}

/* n_full full steps from even s0; EJ_log gets n_full+1 entries, plus_log gets
 * (n_full+1)*n_classes entries (row t = configuration after t full steps). */
int oracle_graph_run(int n, int64_t m, const int32_t *src, const int32_t *dst,
                     const int8_t *J, const uint8_t *cls, int n_classes,
                     const double *lam_of_class, double q, double beta, uint64_t seed,
                     uint32_t replica, uint32_t s0, int8_t *spins, int64_t n_full,
                     int64_t *EJ_log, int64_t *plus_log)
{
    int8_t *tmp;
    int64_t t;
    uint32_t s = s0;
    if (s0 & 1u) return -1;
    tmp = (int8_t *)malloc((size_t)(n > 0 ? n : 1));
    if (!tmp) return -1;
    for (t = 0; t <= n_full; ++t) {
        if (EJ_log || plus_log) {
            int64_t e;
            int64_t pl[256];
            oracle_graph_observe(n, m, src, dst, J, cls, n_classes, spins, &e, pl);
            if (EJ_log) EJ_log[t] = e;
            if (plus_log) memcpy(plus_log + t * n_classes, pl, sizeof(int64_t) * n_classes);
        }
        if (t == n_full) break;
        if (oracle_graph_half_step(n, m, src, dst, J, cls, lam_of_class, q, beta, seed,
                                   replica, s, spins, tmp) ||
            oracle_graph_half_step(n, m, src, dst, J, cls, lam_of_class, q, beta, seed,
                                   replica, s + 1, tmp, spins)) {
            free(tmp);
            return -1;
        }
        s += 2;
    }
    free(tmp);
    return 0;
}
