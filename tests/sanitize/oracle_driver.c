/* The CPU oracle (oracle/oracle.c) under AddressSanitizer /
 * UndefinedBehaviorSanitizer, built with gcc and run by
 * tests/test_sanitizers.py.  Test infrastructure of test infrastructure:
 * it includes the oracle's source and calls every entry point on dirty
 * random graphs with patterns of every kind (edges, anti-edges,
 * anti-vertices, labels), checking a few identities between routes.  Exits
 * 0 when every check holds (the sanitizers abort on a finding). */
#include <stdio.h>

#include "../../oracle/oracle.c"

static int failures = 0;
#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            failures++;                                                      \
        }                                                                    \
    } while (0)

static uint64_t state = 88172645463325252ull;
static uint64_t rnd(void) { /* xorshift64 */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
}

/* canonical adjacency bitmask of every labelled k-vertex graph (pairs in
 * lexicographic order), by trying every permutation */
static void canon_table(int k, uint16_t *out) {
    int pa[10], pb[10], np = 0;
    for (int a = 0; a < k; a++)
        for (int b = a + 1; b < k; b++) { pa[np] = a; pb[np] = b; np++; }
    int perm[6] = {0, 1, 2, 3, 4, 5};
    for (int mask = 0; mask < (1 << np); mask++) out[mask] = (uint16_t)mask;
    /* Heap's algorithm over permutations of 0..k-1 */
    int c[6] = {0};
    for (int step = 0;; step++) {
        if (step) {
            int i = 1;
            while (i < k && c[i] >= i) { c[i] = 0; i++; }
            if (i >= k) break;
            int j = (i % 2) ? c[i] : 0;
            int t = perm[j]; perm[j] = perm[i]; perm[i] = t;
            c[i]++;
        }
        for (int mask = 0; mask < (1 << np); mask++) {
            int r = 0;
            for (int e = 0; e < np; e++) {
                if (!(mask >> e & 1)) continue;
                int x = perm[pa[e]], y = perm[pb[e]];
                if (x > y) { int t = x; x = y; y = t; }
                for (int f = 0; f < np; f++)
                    if (pa[f] == x && pb[f] == y) r |= 1 << f;
            }
            if (r < out[mask]) out[mask] = (uint16_t)r;
        }
    }
}

static void pattern(orc_pattern *p, int k) {
    memset(p, 0, sizeof(*p));
    p->k = k;
    for (int i = 0; i < 16; i++) p->label[i] = -1;
    for (int a = 0; a < 4; a++) p->av_label[a] = -1;
}

static void edge(orc_pattern *p, int a, int b) { p->edge[a] |= 1u << b; p->edge[b] |= 1u << a; }
static void anti(orc_pattern *p, int a, int b) { p->anti[a] |= 1u << b; p->anti[b] |= 1u << a; }

int main(void) {
    uint16_t canon3[8], canon4[64], canon5[1024];
    canon_table(3, canon3);
    canon_table(4, canon4);
    canon_table(5, canon5);
    for (int t = 0; t < 40; t++) {
        const int32_t n = 1 + (int32_t)(rnd() % 120);
        const int64_t m = (int64_t)(rnd() % 900);
        int32_t *src = malloc(sizeof(int32_t) * (size_t)(m + 1)), *dst = malloc(sizeof(int32_t) * (size_t)(m + 1));
        int16_t *lab = malloc(sizeof(int16_t) * (size_t)n);
        for (int64_t i = 0; i < m; i++) {
            src[i] = (int32_t)(rnd() % (uint64_t)n);
            dst[i] = rnd() % 5 == 0 ? src[i] : (int32_t)(rnd() % (1 + rnd() % (uint64_t)n));
        }
        for (int32_t v = 0; v < n; v++) lab[v] = (int16_t)(rnd() % 3);
        orc_graph *g = orc_graph_build(n, m, src, dst, (t % 2) ? lab : NULL);
        CHECK(g != NULL);
        int64_t *deg = calloc((size_t)n + 1, sizeof(int64_t)), *off = calloc((size_t)n + 1, sizeof(int64_t));
        orc_graph_degrees(g, deg);
        int64_t sum = 0;
        for (int32_t v = 0; v < n; v++) sum += deg[v];
        CHECK(sum == 2 * orc_graph_m(g));
        int32_t *adj = malloc(sizeof(int32_t) * (size_t)(sum + 1));
        orc_graph_csr(g, off, adj);
        int64_t *te = calloc((size_t)sum + 1, sizeof(int64_t)), *tv = calloc((size_t)n, sizeof(int64_t));
        orc_edge_triangles(g, 4, te);
        orc_triangles_per_vertex(g, tv);

        orc_pattern ps[8];
        int np = 0;
        pattern(&ps[np], 3); edge(&ps[np], 0, 1); edge(&ps[np], 1, 2); edge(&ps[np], 0, 2); np++;  /* triangle */
        pattern(&ps[np], 4); edge(&ps[np], 0, 1); edge(&ps[np], 0, 2); edge(&ps[np], 0, 3);
        anti(&ps[np], 1, 2); anti(&ps[np], 1, 3); anti(&ps[np], 2, 3); np++;                     /* induced 3-star */
        pattern(&ps[np], 4); edge(&ps[np], 0, 1); edge(&ps[np], 1, 2); edge(&ps[np], 2, 3);
        edge(&ps[np], 3, 0); anti(&ps[np], 1, 3); np++;                                           /* 4-cycle + anti-edge */
        pattern(&ps[np], 3); edge(&ps[np], 0, 1); edge(&ps[np], 1, 2); edge(&ps[np], 0, 2);
        ps[np].n_av = 1; ps[np].av[0] = 7u; np++;                                                  /* triangle in no K4 */
        pattern(&ps[np], 3); edge(&ps[np], 0, 1); edge(&ps[np], 1, 2);
        ps[np].label[0] = 1; ps[np].label[2] = 0; ps[np].n_av = 1; ps[np].av[0] = 2u;
        ps[np].av_label[0] = 2; np++;                                                              /* labelled, anti-vertex */
        pattern(&ps[np], 5); for (int a = 0; a < 5; a++) for (int b = a + 1; b < 5; b++) edge(&ps[np], a, b); np++;
        for (int i = 0; i < np; i++) {
            uint64_t lo, hi, a, vlo, vhi;
            const int rc = orc_count(g, &ps[i], 4, &lo, &hi, &a);
            CHECK(rc == 0);
            CHECK(orc_valid_maps(g, &ps[i], 3, &vlo, &vhi) == 0);
            const u128 cnt = ((u128)hi << 64) | lo, vm = ((u128)vhi << 64) | vlo;
            CHECK(cnt * a == vm);
            CHECK(orc_exists(g, &ps[i], 4) == (cnt > 0));
            int32_t roots[7] = {0, n - 1, n / 2, 0, 1 % n, n / 3, n - 1};
            CHECK(orc_valid_maps_roots(g, &ps[i], 2, roots, 7, &vlo, &vhi) == 0);
            CHECK(orc_valid_maps_roots(g, &ps[i], 2, roots, 0, &vlo, &vhi) == 0 && vlo == 0 && vhi == 0);
            int64_t sizes[16];
            uint8_t *mem = malloc((size_t)ps[i].k * (size_t)n);
            CHECK(orc_domains(g, &ps[i], 3, sizes, mem) == 0);
            for (int u = 0; u < ps[i].k; u++) CHECK(sizes[u] >= 0 && sizes[u] <= n && ((sizes[u] > 0) == (cnt > 0)));
            free(mem);
        }
        uint64_t c3[8], c4[64], c5[1024], nl[6], nh[6];
        CHECK(orc_esu_census(g, 3, canon3, 4, c3) == 0);
        CHECK(orc_esu_census(g, 4, canon4, 4, c4) == 0);
        if (n <= 60) CHECK(orc_esu_census(g, 5, canon5, 4, c5) == 0);
        CHECK(orc_noninduced4(g, 4, nl, nh) == 0);
        /* triangles three ways: the closed form, per vertex, per edge */
        int64_t s_tv = 0, s_te = 0;
        for (int32_t v = 0; v < n; v++) s_tv += tv[v];
        for (int64_t e = 0; e < sum; e++) s_te += te[e];
        CHECK((uint64_t)(s_tv / 3) == nl[0] && (uint64_t)(s_te / 6) == nl[0] && c3[7] == nl[0]);
        free(src); free(dst); free(lab); free(deg); free(off); free(adj); free(te); free(tv);
        orc_graph_free(g);
    }
    /* a disconnected pattern is refused */
    {
        int32_t s[1] = {0}, d[1] = {1};
        orc_graph *g = orc_graph_build(3, 1, s, d, NULL);
        orc_pattern p;
        pattern(&p, 3);
        edge(&p, 0, 1);
        uint64_t lo, hi, a;
        CHECK(orc_count(g, &p, 2, &lo, &hi, &a) == -1);
        CHECK(orc_exists(g, &p, 2) == -1);
        orc_graph_free(g);
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle driver ok\n");
    return 0;
}
