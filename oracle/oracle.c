/*
 * CPU oracle for pattern-aware subgraph counting (Peregrine, EuroSys 2020).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load or call
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code with the HIP library: it builds its own
 * adjacency, has its own pattern type and uses a different algorithm
 * (no symmetry breaking, no vertex cover, no degree ordering, no set-size
 * arithmetic).  Every routine is a plain, slow, obviously correct reading of
 * a definition in the paper:
 *
 *  - orc_count: the number of matches of a pattern as
 *      |valid maps| / |Aut_t(p)|
 *    where a valid map is an injective m: V_regular(p) -> V(G) that keeps
 *    every true edge (problem statement, Sec. 2.1), keeps every anti-edge
 *    absent (Sec. 3.1.1, anti-edge constraint), keeps labels, and satisfies
 *    each anti-vertex constraint (Sec. 3.1.2: the sets adj(m(u)) minus the
 *    images of u's pattern neighbours, intersected over the anti-vertex's
 *    neighbours u, must be empty).  Aut_t is the group of permutations of the
 *    regular vertices that preserve edges, anti-edges, labels and the
 *    anti-vertex neighbourhoods (Sec. 4.3 treats anti-vertex anti-edges as
 *    their own kind when finding symmetries).
 *    Vertex-induced counting is the same count with an anti-edge on every
 *    non-adjacent regular pair (the Theorem of Sec. 3.1.3).
 *  - orc_esu_census: every connected k-vertex set exactly once (Wernicke's
 *    ESU enumeration), classified by its induced subgraph; this is motif
 *    counting as defined in Sec. 2.1, done pattern-unaware.
 *  - orc_noninduced4: textbook closed forms for non-induced 4-vertex
 *    subgraph counts (triangle, 3-star, 4-path, 4-cycle, paw, diamond).
 *
 * Graph semantics: undirected simple graph (Sec. 2.1); loops are dropped and
 * duplicates collapsed.
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

typedef struct {
    int32_t n;
    int64_t m;        /* distinct undirected edges */
    int64_t *off;     /* n + 1 */
    int32_t *adj;     /* each row sorted ascending by vertex id */
    int16_t *label;   /* n entries or NULL */
} orc_graph;

typedef struct {
    int32_t k;             /* regular vertices 0..k-1, k <= 16 */
    int32_t n_av;          /* anti-vertices, <= 4 */
    uint32_t edge[16];     /* true-edge neighbour masks */
    uint32_t anti[16];     /* anti-edge neighbour masks */
    uint32_t av[4];        /* regular neighbours (via anti-edges) of each anti-vertex */
    int16_t label[16];     /* -1 = any */
    int16_t av_label[4];   /* -1 = any */
} orc_pattern;

/* ------------------------------------------------------------------ graph */

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

orc_graph *orc_graph_build(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                           const int16_t *labels) {
    orc_graph *g = calloc(1, sizeof(*g));
    int64_t *keys = malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
    int64_t nk = 0;
    for (int64_t i = 0; i < m; i++) {
        int64_t a = src[i], b = dst[i];
        if (a == b || a < 0 || b < 0 || a >= n || b >= n) continue;
        keys[nk++] = a * (int64_t)n + b;
        keys[nk++] = b * (int64_t)n + a;
    }
    qsort(keys, (size_t)nk, sizeof(int64_t), cmp_i64);
    int64_t w = 0;
    for (int64_t i = 0; i < nk; i++)
        if (i == 0 || keys[i] != keys[i - 1]) keys[w++] = keys[i];
    g->n = n;
    g->m = w / 2;
    g->off = calloc((size_t)n + 1, sizeof(int64_t));
    g->adj = malloc(sizeof(int32_t) * (size_t)(w + 1));
    for (int64_t i = 0; i < w; i++) {
        g->off[keys[i] / n + 1]++;
        g->adj[i] = (int32_t)(keys[i] % n);
    }
    for (int32_t v = 0; v < n; v++) g->off[v + 1] += g->off[v];
    free(keys);
    if (labels) {
        g->label = malloc(sizeof(int16_t) * (size_t)(n + 1));
        memcpy(g->label, labels, sizeof(int16_t) * (size_t)n);
    }
    return g;
}

void orc_graph_free(orc_graph *g) {
    if (!g) return;
    free(g->off);
    free(g->adj);
    free(g->label);
    free(g);
}

int64_t orc_graph_m(const orc_graph *g) { return g->m; }

void orc_graph_degrees(const orc_graph *g, int64_t *out) {
    for (int32_t v = 0; v < g->n; v++) out[v] = g->off[v + 1] - g->off[v];
}

/* copy of the canonical adjacency (for invariant checks in tests) */
void orc_graph_csr(const orc_graph *g, int64_t *off, int32_t *adj) {
    memcpy(off, g->off, sizeof(int64_t) * ((size_t)g->n + 1));
    memcpy(adj, g->adj, sizeof(int32_t) * (size_t)g->off[g->n]);
}

static int has_edge(const orc_graph *g, int32_t a, int32_t b) {
    int64_t lo = g->off[a], hi = g->off[a + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (g->adj[mid] < b) lo = mid + 1;
        else hi = mid;
    }
    return lo < g->off[a + 1] && g->adj[lo] == b;
}

/* --------------------------------------------------------------- patterns */

static int pair_type(const orc_pattern *p, int i, int j) {
    if (p->edge[i] >> j & 1u) return 1;
    if (p->anti[i] >> j & 1u) return 2;
    return 0;
}

/* The regular vertex set's image of an anti-vertex neighbourhood under perm. */
static uint32_t map_mask(uint32_t mask, const int *perm, int k) {
    uint32_t r = 0;
    for (int i = 0; i < k; i++)
        if (mask >> i & 1u) r |= 1u << perm[i];
    return r;
}

static int av_multiset_kept(const orc_pattern *p, const int *perm) {
    int used[4] = {0, 0, 0, 0};
    for (int a = 0; a < p->n_av; a++) {
        uint32_t img = map_mask(p->av[a], perm, p->k);
        int found = 0;
        for (int b = 0; b < p->n_av && !found; b++)
            if (!used[b] && p->av[b] == img && p->av_label[b] == p->av_label[a]) {
                used[b] = 1;
                found = 1;
            }
        if (!found) return 0;
    }
    return 1;
}

typedef struct {
    const orc_pattern *p;
    int perm[16];
    int used[16];
    uint64_t count;
} aut_state;

static void aut_rec(aut_state *s, int i) {
    const orc_pattern *p = s->p;
    if (i == p->k) {
        if (av_multiset_kept(p, s->perm)) s->count++;
        return;
    }
    for (int c = 0; c < p->k; c++) {
        if (s->used[c]) continue;
        if (p->label[i] != p->label[c]) continue;
        int ok = 1;
        for (int j = 0; j < i && ok; j++)
            if (pair_type(p, i, j) != pair_type(p, c, s->perm[j])) ok = 0;
        if (!ok) continue;
        s->used[c] = 1;
        s->perm[i] = c;
        aut_rec(s, i + 1);
        s->used[c] = 0;
    }
}

/* |Aut_t(p)|: permutations of the regular vertices preserving every pair's
 * type (none / edge / anti-edge), every label, and the multiset of
 * anti-vertex neighbourhoods.  Exhaustive search; a pattern whose pairs are
 * all true edges (a clique with no labels and no anti-vertices) has k!
 * automorphisms by inspection, which avoids listing 14! permutations.
 * Returns 0 when the search would be too large (k > 11 otherwise). */
uint64_t orc_aut(const orc_pattern *p) {
    int all_edges = p->n_av == 0;
    for (int i = 0; i < p->k && all_edges; i++) {
        if (p->label[i] != -1) all_edges = 0;
        for (int j = 0; j < p->k; j++)
            if (i != j && pair_type(p, i, j) != 1) all_edges = 0;
    }
    if (all_edges) {
        uint64_t f = 1;
        for (int i = 2; i <= p->k; i++) f *= (uint64_t)i;
        return f;
    }
    if (p->k > 11) return 0;
    aut_state s;
    memset(&s, 0, sizeof(s));
    s.p = p;
    aut_rec(&s, 0);
    return s.count;
}

/* ------------------------------------------------------- generic matcher */

typedef struct {
    const orc_graph *g;
    const orc_pattern *p;
    int order[16];    /* BFS order over true edges */
    int parent[16];   /* an earlier position that is a true neighbour */
    const int32_t *roots;  /* NULL: every vertex is a start vertex */
    int64_t n_roots;
    atomic_int_fast64_t cursor;
    u128 total;
    pthread_mutex_t mu;
} match_job;

/* Anti-vertex constraint for anti-vertex a under map img[] (img indexed by
 * pattern vertex): no data vertex lies in every set
 * adj(img[u]) \ img(N_E(u)) for u in the anti-vertex's neighbourhood. */
static int av_ok(const orc_graph *g, const orc_pattern *p, int a, const int32_t *img) {
    uint32_t nb = p->av[a];
    int first = -1;
    for (int u = 0; u < p->k; u++)
        if (nb >> u & 1u) { first = u; break; }
    int32_t x = img[first];
    for (int64_t e = g->off[x]; e < g->off[x + 1]; e++) {
        int32_t w = g->adj[e];
        if (p->av_label[a] != -1 && (!g->label || g->label[w] != p->av_label[a])) continue;
        int in_all = 1;
        for (int u = 0; u < p->k && in_all; u++) {
            if (!(nb >> u & 1u)) continue;
            /* w must be in adj(img[u]) and not the image of a true neighbour of u */
            if (!has_edge(g, img[u], w)) in_all = 0;
            for (int y = 0; y < p->k && in_all; y++)
                if ((p->edge[u] >> y & 1u) && img[y] == w) in_all = 0;
        }
        if (in_all) return 0;
    }
    return 1;
}

static u128 match_rec(match_job *J, int32_t *img, int pos) {
    const orc_graph *g = J->g;
    const orc_pattern *p = J->p;
    if (pos == p->k) {
        for (int a = 0; a < p->n_av; a++)
            if (!av_ok(g, p, a, img)) return 0;
        return 1;
    }
    int u = J->order[pos];
    int32_t par = img[J->order[J->parent[pos]]];
    u128 c = 0;
    for (int64_t e = g->off[par]; e < g->off[par + 1]; e++) {
        int32_t x = g->adj[e];
        int ok = 1;
        if (p->label[u] != -1 && (!g->label || g->label[x] != p->label[u])) ok = 0;
        for (int q = 0; q < pos && ok; q++) {
            int w = J->order[q];
            if (img[w] == x) ok = 0;                                           /* injective */
            else if ((p->edge[u] >> w & 1u) && !has_edge(g, x, img[w])) ok = 0;  /* true edge */
            else if ((p->anti[u] >> w & 1u) && has_edge(g, x, img[w])) ok = 0;  /* anti-edge */
        }
        if (!ok) continue;
        img[u] = x;
        c += match_rec(J, img, pos + 1);
    }
    return c;
}

static void *match_worker(void *arg) {
    match_job *J = arg;
    const orc_pattern *p = J->p;
    int32_t img[16];
    u128 local = 0;
    for (;;) {
        int64_t v = atomic_fetch_add(&J->cursor, 1);
        if (v >= J->n_roots) break;
        if (J->roots) v = J->roots[v];
        int u0 = J->order[0];
        if (p->label[u0] != -1 && (!J->g->label || J->g->label[v] != p->label[u0])) continue;
        img[u0] = (int32_t)v;
        local += match_rec(J, img, 1);
    }
    pthread_mutex_lock(&J->mu);
    J->total += local;
    pthread_mutex_unlock(&J->mu);
    return NULL;
}

/* Number of valid maps of p into g whose first pattern vertex (vertex 0)
 * is mapped to one of roots[0..n_roots) (roots == NULL: any vertex).  Used
 * whole by orc_count and on a bounded sample of start vertices to time the
 * oracle.  Returns -1 if the regular vertices are not connected by true
 * edges. */
int orc_valid_maps_roots(const orc_graph *g, const orc_pattern *p, int nthreads, const int32_t *roots,
                         int64_t n_roots, uint64_t *lo, uint64_t *hi) {
    match_job J;
    memset(&J, 0, sizeof(J));
    J.g = g;
    J.p = p;
    J.roots = roots;
    J.n_roots = roots ? n_roots : g->n;
    /* BFS over true edges from regular vertex 0 */
    int seen[16] = {0};
    int head = 0, tail = 0;
    J.order[tail++] = 0;
    seen[0] = 1;
    J.parent[0] = -1;
    while (head < tail) {
        int x = J.order[head++];
        for (int y = 0; y < p->k; y++)
            if ((p->edge[x] >> y & 1u) && !seen[y]) {
                seen[y] = 1;
                J.parent[tail] = head - 1;
                J.order[tail++] = y;
            }
    }
    if (tail != p->k) return -1;
    atomic_init(&J.cursor, 0);
    pthread_mutex_init(&J.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, match_worker, &J);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.mu);
    *lo = (uint64_t)J.total;
    *hi = (uint64_t)(J.total >> 64);
    return 0;
}

/* Number of valid maps of p into g (see the file header). */
int orc_valid_maps(const orc_graph *g, const orc_pattern *p, int nthreads, uint64_t *lo,
                   uint64_t *hi) {
    return orc_valid_maps_roots(g, p, nthreads, NULL, 0, lo, hi);
}

/* ---------------------------------------------------------- MNI domains */

/* Sec. 2 (support of a pattern): dom(u) is the set of data vertices that u
 * is mapped to by at least one valid map.  Written from that definition:
 * for every pattern vertex u and every data vertex v, search for one valid
 * map with u -> v (the same checks as match_rec, stopping at the first).
 * This is test infrastructure: it shares nothing with the GPU path. */
typedef struct {
    match_job J;          /* order[0] = u, BFS order over true edges from u */
    uint8_t *member;      /* n entries: 1 if v in dom(u) */
} dom_job;

static int exists_rec(match_job *J, int32_t *img, int pos) {
    const orc_graph *g = J->g;
    const orc_pattern *p = J->p;
    if (pos == p->k) {
        for (int a = 0; a < p->n_av; a++)
            if (!av_ok(g, p, a, img)) return 0;
        return 1;
    }
    int u = J->order[pos];
    int32_t par = img[J->order[J->parent[pos]]];
    for (int64_t e = g->off[par]; e < g->off[par + 1]; e++) {
        int32_t x = g->adj[e];
        int ok = 1;
        if (p->label[u] != -1 && (!g->label || g->label[x] != p->label[u])) ok = 0;
        for (int q = 0; q < pos && ok; q++) {
            int w = J->order[q];
            if (img[w] == x) ok = 0;
            else if ((p->edge[u] >> w & 1u) && !has_edge(g, x, img[w])) ok = 0;
            else if ((p->anti[u] >> w & 1u) && has_edge(g, x, img[w])) ok = 0;
        }
        if (!ok) continue;
        img[u] = x;
        if (exists_rec(J, img, pos + 1)) return 1;
    }
    return 0;
}

static void *dom_worker(void *arg) {
    dom_job *D = arg;
    match_job *J = &D->J;
    const orc_pattern *p = J->p;
    int32_t img[16];
    for (;;) {
        int64_t v = atomic_fetch_add(&J->cursor, 1);
        if (v >= J->g->n) break;
        int u0 = J->order[0];
        if (p->label[u0] != -1 && (!J->g->label || J->g->label[v] != p->label[u0])) continue;
        img[u0] = (int32_t)v;
        D->member[v] = (uint8_t)exists_rec(J, img, 1);
    }
    return NULL;
}

/* sizes[u] = |dom(u)| for u = 0..k-1; member: NULL or k*n bytes (row u:
 * membership of each data vertex in dom(u)).  Returns -1 if the regular
 * vertices are not connected by true edges. */
int orc_domains(const orc_graph *g, const orc_pattern *p, int nthreads, int64_t *sizes, uint8_t *member) {
    uint8_t *buf = (uint8_t *)calloc((size_t)(g->n > 0 ? g->n : 1), 1);
    if (!buf) return -2;
    for (int u = 0; u < p->k; u++) {
        dom_job D;
        memset(&D, 0, sizeof(D));
        D.J.g = g;
        D.J.p = p;
        D.member = buf;
        memset(buf, 0, (size_t)g->n);
        int seen[16] = {0};
        int head = 0, tail = 0;
        D.J.order[tail++] = u;
        seen[u] = 1;
        D.J.parent[0] = -1;
        while (head < tail) {
            int x = D.J.order[head++];
            for (int y = 0; y < p->k; y++)
                if ((p->edge[x] >> y & 1u) && !seen[y]) {
                    seen[y] = 1;
                    D.J.parent[tail] = head - 1;
                    D.J.order[tail++] = y;
                }
        }
        if (tail != p->k) { free(buf); return -1; }
        atomic_init(&D.J.cursor, 0);
        int nt = nthreads < 1 ? 1 : (nthreads > 256 ? 256 : nthreads);
        pthread_t th[256];
        for (int t = 0; t < nt; t++) pthread_create(&th[t], NULL, dom_worker, &D);
        for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
        int64_t c = 0;
        for (int32_t v = 0; v < g->n; v++) c += buf[v];
        sizes[u] = c;
        if (member) memcpy(member + (size_t)u * (size_t)g->n, buf, (size_t)g->n);
    }
    free(buf);
    return 0;
}

/* exists(G, p): is there at least one valid map (Sec. 3.2.2, existence
 * queries)?  The same search as the valid-map count, from every start
 * vertex in turn, ending at the first valid map any thread finds.  Returns
 * 1 / 0, or -1 for a disconnected pattern. */
typedef struct {
    match_job J;
    atomic_int found;
} exists_job;

static void *exists_worker(void *arg) {
    exists_job *E = arg;
    match_job *J = &E->J;
    const orc_pattern *p = J->p;
    int32_t img[16];
    while (!atomic_load(&E->found)) {
        int64_t v = atomic_fetch_add(&J->cursor, 1);
        if (v >= J->g->n) break;
        int u0 = J->order[0];
        if (p->label[u0] != -1 && (!J->g->label || J->g->label[v] != p->label[u0])) continue;
        img[u0] = (int32_t)v;
        if (exists_rec(J, img, 1)) atomic_store(&E->found, 1);
    }
    return NULL;
}

int orc_exists(const orc_graph *g, const orc_pattern *p, int nthreads) {
    exists_job E;
    memset(&E, 0, sizeof(E));
    E.J.g = g;
    E.J.p = p;
    int seen[16] = {0};
    int head = 0, tail = 0;
    E.J.order[tail++] = 0;
    seen[0] = 1;
    E.J.parent[0] = -1;
    while (head < tail) {
        int x = E.J.order[head++];
        for (int y = 0; y < p->k; y++)
            if ((p->edge[x] >> y & 1u) && !seen[y]) {
                seen[y] = 1;
                E.J.parent[tail] = head - 1;
                E.J.order[tail++] = y;
            }
    }
    if (tail != p->k) return -1;
    atomic_init(&E.J.cursor, 0);
    atomic_init(&E.found, 0);
    int nt = nthreads < 1 ? 1 : (nthreads > 256 ? 256 : nthreads);
    pthread_t th[256];
    for (int t = 0; t < nt; t++) pthread_create(&th[t], NULL, exists_worker, &E);
    for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
    return atomic_load(&E.found) ? 1 : 0;
}

/* count(G, p) = |valid maps| / |Aut_t(p)|.  Returns 0 on success, -1 for a
 * disconnected pattern, -2 if |Aut_t| is out of the exhaustive range, -3 if
 * the division is not exact (which would mean a bug in this file). */
int orc_count(const orc_graph *g, const orc_pattern *p, int nthreads, uint64_t *lo,
              uint64_t *hi, uint64_t *aut_out) {
    uint64_t a = orc_aut(p);
    if (aut_out) *aut_out = a;
    if (a == 0) return -2;
    uint64_t vl, vh;
    int rc = orc_valid_maps(g, p, nthreads, &vl, &vh);
    if (rc) return rc;
    u128 v = ((u128)vh << 64) | vl;
    if (v % a) return -3;
    v /= a;
    *lo = (uint64_t)v;
    *hi = (uint64_t)(v >> 64);
    return 0;
}

/* ------------------------------------------------------------ ESU census */

typedef struct {
    const orc_graph *g;
    int k;
    const uint16_t *canon;   /* adjacency bitmask -> canonical bitmask */
    atomic_int_fast64_t cursor;
    uint64_t *counts;        /* indexed by canonical bitmask */
    int nbits;
    pthread_mutex_t mu;
} esu_job;

typedef struct {
    esu_job *J;
    int32_t sub[8];
    int32_t *ext[8];
    int64_t cap;
    uint64_t *local;
} esu_thr;

static int pair_bit(int i, int j, int k) {
    /* bit index of pair (i<j) in row-major upper-triangle order */
    int idx = 0;
    for (int a = 0; a < i; a++) idx += k - 1 - a;
    return idx + (j - i - 1);
}

static void esu_classify(esu_thr *T, int k) {
    const orc_graph *g = T->J->g;
    uint32_t mask = 0;
    for (int i = 0; i < k; i++)
        for (int j = i + 1; j < k; j++)
            if (has_edge(g, T->sub[i], T->sub[j])) mask |= 1u << pair_bit(i, j, k);
    T->local[T->J->canon[mask]]++;
}

static void esu_extend(esu_thr *T, int depth, int64_t next, int32_t v) {
    esu_job *J = T->J;
    const orc_graph *g = J->g;
    if (depth == J->k) {
        esu_classify(T, J->k);
        return;
    }
    int32_t *ext = T->ext[depth];
    int64_t cnt = next;
    while (cnt > 0) {
        int32_t w = ext[--cnt];
        /* new extension: ext[0..cnt) plus exclusive neighbours of w above v */
        int32_t *nx = T->ext[depth + 1];
        int64_t nn = 0;
        for (int64_t i = 0; i < cnt; i++) nx[nn++] = ext[i];
        for (int64_t e = g->off[w]; e < g->off[w + 1]; e++) {
            int32_t u = g->adj[e];
            if (u <= v) continue;
            int excl = 1;
            for (int s = 0; s < depth && excl; s++)
                if (T->sub[s] == u || has_edge(g, T->sub[s], u)) excl = 0;
            if (excl) nx[nn++] = u;
        }
        T->sub[depth] = w;
        esu_extend(T, depth + 1, nn, v);
    }
}

static void *esu_worker(void *arg) {
    esu_thr *T = arg;
    esu_job *J = T->J;
    const orc_graph *g = J->g;
    for (;;) {
        int64_t v = atomic_fetch_add(&J->cursor, 1);
        if (v >= g->n) break;
        int64_t nn = 0;
        for (int64_t e = g->off[v]; e < g->off[v + 1]; e++)
            if (g->adj[e] > v) T->ext[1][nn++] = g->adj[e];
        T->sub[0] = (int32_t)v;
        esu_extend(T, 1, nn, (int32_t)v);
    }
    return NULL;
}

/* Census of connected k-vertex induced subgraphs (3 <= k <= 6).  canon maps
 * every adjacency bitmask of k labelled vertices to its class representative;
 * counts[rep] receives the number of vertex sets of that class. */
int orc_esu_census(const orc_graph *g, int k, const uint16_t *canon, int nthreads,
                   uint64_t *counts) {
    if (k < 2 || k > 6) return -1;
    esu_job J;
    memset(&J, 0, sizeof(J));
    J.g = g;
    J.k = k;
    J.canon = canon;
    J.nbits = k * (k - 1) / 2;
    atomic_init(&J.cursor, 0);
    int64_t dmax = 0;
    for (int32_t v = 0; v < g->n; v++)
        if (g->off[v + 1] - g->off[v] > dmax) dmax = g->off[v + 1] - g->off[v];
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    esu_thr *T = calloc((size_t)nthreads, sizeof(esu_thr));
    pthread_t th[256];
    size_t ncls = (size_t)1 << J.nbits;
    for (int t = 0; t < nthreads; t++) {
        T[t].J = &J;
        T[t].cap = (int64_t)k * (dmax + 1);
        for (int d = 0; d <= k; d++) T[t].ext[d] = malloc(sizeof(int32_t) * (size_t)(T[t].cap + 1));
        T[t].local = calloc(ncls, sizeof(uint64_t));
        pthread_create(&th[t], NULL, esu_worker, &T[t]);
    }
    memset(counts, 0, sizeof(uint64_t) * ncls);
    for (int t = 0; t < nthreads; t++) {
        pthread_join(th[t], NULL);
        for (size_t c = 0; c < ncls; c++) counts[c] += T[t].local[c];
        for (int d = 0; d <= k; d++) free(T[t].ext[d]);
        free(T[t].local);
    }
    free(T);
    return 0;
}

/* ---------------------------------------------- 4-vertex closed forms */

typedef struct {
    const orc_graph *g;
    atomic_int_fast64_t cursor;
    int64_t *t_edge;     /* triangles on each adjacency slot (both directions) */
    pthread_mutex_t mu;
    u128 c4_twice;       /* sum over unordered pairs of C(codeg, 2) */
} cf_job;

static int64_t common(const orc_graph *g, int32_t a, int32_t b) {
    int64_t i = g->off[a], ie = g->off[a + 1], j = g->off[b], je = g->off[b + 1], c = 0;
    while (i < ie && j < je) {
        if (g->adj[i] < g->adj[j]) i++;
        else if (g->adj[i] > g->adj[j]) j++;
        else { c++; i++; j++; }
    }
    return c;
}

static void *tri_worker(void *arg) {
    cf_job *J = arg;
    const orc_graph *g = J->g;
    for (;;) {
        int64_t v = atomic_fetch_add(&J->cursor, 1);
        if (v >= g->n) break;
        for (int64_t e = g->off[v]; e < g->off[v + 1]; e++)
            J->t_edge[e] = common(g, (int32_t)v, g->adj[e]);
    }
    return NULL;
}

static void *codeg_worker(void *arg) {
    cf_job *J = arg;
    const orc_graph *g = J->g;
    int64_t *cnt = calloc((size_t)g->n, sizeof(int64_t));
    int32_t *touched = malloc(sizeof(int32_t) * (size_t)(g->n + 1));
    u128 local = 0;
    for (;;) {
        int64_t u = atomic_fetch_add(&J->cursor, 1);
        if (u >= g->n) break;
        int64_t nt = 0;
        for (int64_t e = g->off[u]; e < g->off[u + 1]; e++) {
            int32_t w = g->adj[e];
            for (int64_t f = g->off[w]; f < g->off[w + 1]; f++) {
                int32_t x = g->adj[f];
                if (x <= u) continue;
                if (cnt[x]++ == 0) touched[nt++] = x;
            }
        }
        for (int64_t i = 0; i < nt; i++) {
            int64_t c = cnt[touched[i]];
            local += (u128)(c * (c - 1) / 2);
            cnt[touched[i]] = 0;
        }
    }
    pthread_mutex_lock(&J->mu);
    J->c4_twice += local;
    pthread_mutex_unlock(&J->mu);
    free(cnt);
    free(touched);
    return NULL;
}

/* t[e] = triangles through the edge in adjacency slot e (common neighbours
 * of its two endpoints, counted by a merge of their sorted rows). */
void orc_edge_triangles(const orc_graph *g, int nthreads, int64_t *t) {
    cf_job J;
    memset(&J, 0, sizeof(J));
    J.g = g;
    J.t_edge = t;
    atomic_init(&J.cursor, 0);
    int nt = nthreads < 1 ? 1 : (nthreads > 256 ? 256 : nthreads);
    pthread_t th[256];
    for (int i = 0; i < nt; i++) pthread_create(&th[i], NULL, tri_worker, &J);
    for (int i = 0; i < nt; i++) pthread_join(th[i], NULL);
}

/* out[0..5] (each as lo/hi uint64 pairs in out_lo/out_hi):
 *   0 T       triangles
 *   1 N_star  non-induced 3-stars      sum_v C(d_v, 3)
 *   2 N_P4    non-induced 4-paths      sum_{uv in E} (d_u-1)(d_v-1) - 3T
 *   3 N_C4    non-induced 4-cycles     (1/2) sum_{pairs} C(codeg, 2)
 *   4 N_paw   non-induced paws         sum_v t_v (d_v - 2)
 *   5 N_dia   non-induced diamonds     sum_{uv in E} C(t_uv, 2)
 * Each form counts subgraphs (not maps): a 4-path has a unique middle edge,
 * a paw a unique degree-3 vertex, a diamond a unique chord, and a 4-cycle
 * is seen once from each of its two diagonals. */
int orc_noninduced4(const orc_graph *g, int nthreads, uint64_t *out_lo, uint64_t *out_hi) {
    cf_job J;
    memset(&J, 0, sizeof(J));
    J.g = g;
    J.t_edge = calloc((size_t)g->off[g->n] + 1, sizeof(int64_t));
    pthread_mutex_init(&J.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    atomic_init(&J.cursor, 0);
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, tri_worker, &J);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    atomic_store(&J.cursor, 0);
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, codeg_worker, &J);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);

    u128 tri3 = 0, star = 0, p4 = 0, paw2 = 0, dia = 0;
    for (int32_t v = 0; v < g->n; v++) {
        int64_t d = g->off[v + 1] - g->off[v];
        u128 tv2 = 0;   /* 2 * t_v */
        if (d >= 3) star += (u128)d * (u128)(d - 1) * (u128)(d - 2) / 6;
        for (int64_t e = g->off[v]; e < g->off[v + 1]; e++) {
            int32_t w = g->adj[e];
            int64_t t = J.t_edge[e];
            tv2 += (u128)t;
            if (w > v) {
                int64_t dw = g->off[w + 1] - g->off[w];
                p4 += (u128)(d - 1) * (u128)(dw - 1);
                dia += (u128)t * (u128)(t > 0 ? t - 1 : 0) / 2;
                tri3 += (u128)t;
            }
        }
        if (d >= 2) paw2 += tv2 * (u128)(d - 2);
    }
    u128 T = tri3 / 3;
    u128 res[6];
    res[0] = T;
    res[1] = star;
    res[2] = p4 - 3 * T;
    res[3] = J.c4_twice / 2;
    res[4] = paw2 / 2;
    res[5] = dia;
    for (int i = 0; i < 6; i++) {
        out_lo[i] = (uint64_t)res[i];
        out_hi[i] = (uint64_t)(res[i] >> 64);
    }
    free(J.t_edge);
    pthread_mutex_destroy(&J.mu);
    return 0;
}

/* Per-vertex triangle counts (for small-graph invariants). */
void orc_triangles_per_vertex(const orc_graph *g, int64_t *out) {
    for (int32_t v = 0; v < g->n; v++) {
        int64_t t2 = 0;
        for (int64_t e = g->off[v]; e < g->off[v + 1]; e++) t2 += common(g, v, g->adj[e]);
        out[v] = t2 / 2;
    }
}
