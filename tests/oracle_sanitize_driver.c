/* Host sanitizer run of the C oracle (AddressSanitizer + UndefinedBehavior-
 * Sanitizer): every exported routine on small and ragged inputs, including the
 * torus wrap-around at L = 3 and 33, +-J couplings, an empty edge list, split
 * (anti-parallel) edges and zero temperature.  Exits non-zero on any
 * inconsistency; the sanitizers abort on any invalid access.  The +-J cases
 * also run the reversed order; the triangular lattice runs too. */
#include "../oracle/shaken_oracle.c"

#include <stdio.h>

/* pm: 0 uniform J, 1 +-J couplings with the reversed order, 2 triangular */
static int check_torus(int L, int pm)
{
    int8_t *sp = malloc((size_t)L * L), *a = malloc((size_t)L * L), *b = malloc((size_t)L * L);
    int8_t *ju = malloc((size_t)L * L), *jr = malloc((size_t)L * L);
    int64_t ej[6], m[6], e1, m1;
    int i, rc = 0;
    for (i = 0; i < L * L; ++i) {
        ju[i] = (i * 7 + 3) % 5 < 2 ? -1 : 1;
        jr[i] = (i * 11 + 1) % 3 == 0 ? -1 : 1;
    }
    oracle_torus_init_random(L, 9, 1, sp);
    memcpy(a, sp, (size_t)L * L);
    if (oracle_torus_run_j(L, 1, pm == 1 ? ju : NULL, pm == 1 ? jr : NULL, pm, 0.25, 0.7, 0.6, 9, 1, 0, a, 5, ej, m))
        return 1;
    /* the same five steps as ten half-steps */
    memcpy(b, sp, (size_t)L * L);
    for (i = 0; i < 10; ++i) {
        int8_t *t = malloc((size_t)L * L);
        oracle_torus_half_step_j(L, 1, pm == 1 ? ju : NULL, pm == 1 ? jr : NULL, pm, 0.25, 0.7, 0.6, 9, 1,
                                 (uint32_t)i, b, t);
        memcpy(b, t, (size_t)L * L);
        free(t);
    }
    if (memcmp(a, b, (size_t)L * L)) rc = 2;
    oracle_torus_observe_j(L, 1, pm == 1 ? ju : NULL, pm == 1 ? jr : NULL, pm, a, &e1, &m1);
    if (e1 != ej[5] || m1 != m[5]) rc = 3;
    /* zero temperature and a single site */
    (void)oracle_torus_site_j(L, 1, pm == 1 ? ju : NULL, pm == 1 ? jr : NULL, pm, 0.1, 0.3, 1e9, 9, 1, 4, a,
                              L - 1, L - 1);
    free(sp); free(a); free(b); free(ju); free(jr);
    return rc;
}

static int check_graph(void)
{
    /* a 5-cycle plus one chord, the chord in both orientations (split) */
    int32_t src[7] = {0, 1, 2, 3, 4, 0, 2}, dst[7] = {1, 2, 3, 4, 0, 2, 0};
    int8_t J[7] = {1, -1, 2, 1, -2, 1, 1};
    uint8_t cls[5] = {0, 1, 0, 1, 0};
    double lam[2] = {0.5, -0.5};
    int8_t sp[5], a[5];
    int64_t ej[4], plus[8], e1, p1[2];
    oracle_graph_init_random(5, 3, 2, sp);
    memcpy(a, sp, 5);
    if (oracle_graph_run(5, 7, src, dst, J, cls, 2, lam, 0.9, 0.4, 3, 2, 0, a, 3, ej, plus)) return 10;
    oracle_graph_observe(5, 7, src, dst, J, cls, 2, a, &e1, p1);
    if (e1 != ej[3] || p1[0] != plus[6] || p1[1] != plus[7]) return 11;
    /* no edges at all */
    if (oracle_graph_half_step(5, 0, src, dst, NULL, NULL, NULL, 0.0, 0.0, 1, 0, 0, sp, a)) return 12;
    return 0;
}

int main(void)
{
    int L[4] = {3, 4, 33, 65}, i, pm, rc;
    for (i = 0; i < 4; ++i)
        for (pm = 0; pm < 3; ++pm)
            if ((rc = check_torus(L[i], pm)) != 0) {
                printf("torus L=%d pm=%d: %d\n", L[i], pm, rc);
                return rc;
            }
    if ((rc = check_graph()) != 0) {
        printf("graph: %d\n", rc);
        return rc;
    }
    printf("ok\n");
    return 0;
}
