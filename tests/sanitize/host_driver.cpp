// Host code of libpg under AddressSanitizer / UndefinedBehaviorSanitizer on
// the CPU: the plan compiler (csrc/plan.cpp) and the host part of ingest
// (csrc/ingest.cpp), built with g++ and run by tests/test_sanitizers.py.
// Plans every connected pattern on up to 5 vertices (edge- and
// vertex-induced, anchored, with anti-vertices and labels) and the trie of
// batches of them; ingests dirty random graphs and checks the CSR, the
// row splits and the root tasks; and drives the error paths.  Exits 0 when
// every check holds (the sanitizers abort on a finding).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../../paper_2004_02369_amd/csrc/pg_internal.hpp"

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            failures++;                                                       \
        }                                                                     \
    } while (0)

static bool connected(int k, const std::vector<pg_edge> &E) {
    std::vector<int> seen(k, 0), stack{0};
    seen[0] = 1;
    while (!stack.empty()) {
        int x = stack.back();
        stack.pop_back();
        for (const pg_edge &e : E) {
            if (e.type != PG_EDGE) continue;
            int y = e.u == x ? e.v : e.v == x ? e.u : -1;
            if (y >= 0 && !seen[y]) {
                seen[y] = 1;
                stack.push_back(y);
            }
        }
    }
    for (int i = 0; i < k; i++)
        if (!seen[i]) return false;
    return true;
}

static pg_status plan(int k, int nav, const std::vector<pg_edge> &E, int induced, const int16_t *labels,
                      const pg_plan_options *opt, pg::PlanImpl *out) {
    pg_pattern_desc d{};
    d.k = k;
    d.n_anti_vertices = nav;
    d.n_edges = (int32_t)E.size();
    d.induced = induced;
    d.edges = E.data();
    d.labels = labels;
    std::string err;
    return pg::compile_plan(&d, opt, out, &err);
}

static void patterns() {
    std::vector<pg::PlanImpl> keep;
    keep.reserve(4096);
    for (int k = 2; k <= 5; k++) {
        std::vector<std::pair<int, int>> pairs;
        for (int a = 0; a < k; a++)
            for (int b = a + 1; b < k; b++) pairs.push_back({a, b});
        const int np = (int)pairs.size();
        for (int mask = 1; mask < (1 << np); mask++) {
            std::vector<pg_edge> E;
            for (int i = 0; i < np; i++)
                if (mask >> i & 1) E.push_back({pairs[i].first, pairs[i].second, PG_EDGE});
            if (!connected(k, E)) continue;
            for (int induced = 0; induced < 2; induced++) {
                for (int mode = 0; mode < 3; mode++) {
                    pg_plan_options o{};
                    o.mode = mode;
                    pg::PlanImpl p;
                    CHECK(plan(k, 0, E, induced, nullptr, &o, &p) == PG_OK);
                    CHECK(p.info.aut >= 1 && !p.count_progs.empty() && !p.enum_progs.empty());
                    if (mode == 0) keep.push_back(std::move(p));
                }
                // anchored at every vertex
                for (int a = 0; a < k; a++) {
                    pg_plan_options o{};
                    o.anchored = 1;
                    o.anchor = a;
                    pg::PlanImpl p;
                    CHECK(plan(k, 0, E, induced, nullptr, &o, &p) == PG_OK);
                }
            }
            // an anti-vertex on the first two vertices, and labels
            std::vector<pg_edge> Av = E;
            Av.push_back({0, k, PG_ANTI_EDGE});
            Av.push_back({1, k, PG_ANTI_EDGE});
            pg::PlanImpl pav;
            CHECK(plan(k, 1, Av, 0, nullptr, nullptr, &pav) == PG_OK);
            std::vector<int16_t> lab(k + 1);
            for (int i = 0; i <= k; i++) lab[i] = (int16_t)(i % 3 == 2 ? -1 : i % 2);
            pg::PlanImpl pl;
            CHECK(plan(k, 1, Av, 0, lab.data(), nullptr, &pl) == PG_OK);
        }
    }
    // cliques up to 14 (orbit search without listing automorphisms)
    for (int k = 6; k <= 14; k++) {
        std::vector<pg_edge> E;
        for (int a = 0; a < k; a++)
            for (int b = a + 1; b < k; b++) E.push_back({a, b, PG_EDGE});
        pg::PlanImpl p;
        CHECK(plan(k, 0, E, 0, nullptr, nullptr, &p) == PG_OK);
    }
    // tries of batches of up to 64 plans, counting and enumerating
    std::mt19937 rng(5);
    for (int t = 0; t < 200; t++) {
        std::vector<const pg::PlanImpl *> batch;
        const int nb = 1 + (int)(rng() % 64);
        for (int i = 0; i < nb; i++) batch.push_back(&keep[rng() % keep.size()]);
        for (int emit = 0; emit < 2; emit++) {
            const pg::Trie T = pg::build_trie(emit ? std::vector<const pg::PlanImpl *>{batch[0]} : batch, emit);
            CHECK(T.consistent);
            for (int32_t r : T.roots) CHECK(r >= 0 && r < (int32_t)T.nodes.size());
            for (const pg::Node &n : T.nodes) {
                CHECK(n.child_begin >= 0 && n.child_begin + n.child_count <= (int32_t)T.nodes.size());
                CHECK(n.list_begin >= 0 && n.list_begin + n.list_count <= (int32_t)T.lists.size());
            }
        }
    }
    // error paths: disconnected, too many vertices, an edge both true and anti
    {
        pg::PlanImpl p;
        CHECK(plan(3, 0, {{0, 1, PG_EDGE}}, 0, nullptr, nullptr, &p) == PG_EINVAL);
        CHECK(plan(17, 0, {{0, 1, PG_EDGE}}, 0, nullptr, nullptr, &p) == PG_EINVAL);
        CHECK(plan(2, 0, {{0, 1, PG_EDGE}, {0, 1, PG_ANTI_EDGE}}, 0, nullptr, nullptr, &p) == PG_EINVAL);
        CHECK(plan(2, 0, {{0, 5, PG_EDGE}}, 0, nullptr, nullptr, &p) == PG_EINVAL);
    }
}

static void graphs() {
    std::mt19937 rng(11);
    for (int t = 0; t < 60; t++) {
        const int n = 1 + (int)(rng() % 400);
        const int m = (int)(rng() % 3000);
        std::vector<int32_t> src(m), dst(m);
        for (int i = 0; i < m; i++) {
            // skewed endpoints, loops and repeats included
            src[i] = (int32_t)(rng() % n);
            dst[i] = (int32_t)((rng() % 4 == 0) ? src[i] : (int32_t)(rng() % (1 + rng() % n)));
        }
        std::vector<int16_t> lab(n);
        for (int i = 0; i < n; i++) lab[i] = (int16_t)(rng() % 5);
        pg::HostGraph h;
        std::string err;
        CHECK(pg::ingest(n, m, src.data(), dst.data(), t % 2 ? lab.data() : nullptr, &h, &err) == PG_OK);
        // rows sorted and simple, symmetric, split at the owner, degree order
        int64_t adj = 0;
        std::vector<std::vector<int32_t>> rows(n);
        for (int r = 0; r < n; r++) {
            rows[r].assign(h.col.begin() + h.rp[r], h.col.begin() + h.rp[r + 1]);
            adj += (int64_t)rows[r].size();
            for (size_t i = 0; i < rows[r].size(); i++) {
                CHECK(rows[r][i] != r && rows[r][i] >= 0 && rows[r][i] < n);
                if (i) CHECK(rows[r][i - 1] < rows[r][i]);
            }
            const int32_t up = h.up[r];
            CHECK(up >= 0 && up <= (int32_t)rows[r].size());
            for (int i = 0; i < (int)rows[r].size(); i++) CHECK((rows[r][i] > r) == (i >= up));
            if (r) CHECK(rows[r - 1].size() <= rows[r].size());
        }
        CHECK(adj == 2 * h.m);
        for (int r = 0; r < n; r++)
            for (int32_t c : rows[r]) CHECK(std::binary_search(rows[c].begin(), rows[c].end(), r));
        // every edge once as a task u < v, costliest (d(u) + d(v)) first
        CHECK((int64_t)h.tsrc.size() == h.m);
        int64_t prev = INT64_MAX;
        for (size_t i = 0; i < h.tsrc.size(); i++) {
            const int32_t u = h.tsrc[i], v = h.tdst[i];
            CHECK(u < v && std::binary_search(rows[u].begin(), rows[u].end(), v));
            const int64_t c = (int64_t)rows[u].size() + (int64_t)rows[v].size();
            CHECK(c <= prev);
            prev = c;
        }
        // perm is a bijection and labels follow it
        std::vector<int> seen(n, 0);
        for (int r = 0; r < n; r++) seen[h.perm[r]]++;
        for (int v = 0; v < n; v++) CHECK(seen[v] == 1);
        if (t % 2)
            for (int r = 0; r < n; r++) CHECK(h.lab[r] == lab[h.perm[r]]);
    }
    // error paths
    pg::HostGraph h;
    std::string err;
    const int32_t s[1] = {0}, d[1] = {7};
    CHECK(pg::ingest(5, 1, s, d, nullptr, &h, &err) == PG_EINVAL);
    const int16_t bad[2] = {0, -1};
    const int32_t s2[1] = {0}, d2[1] = {1};
    CHECK(pg::ingest(2, 1, s2, d2, bad, &h, &err) == PG_EINVAL);
    CHECK(pg::ingest(3, 0, nullptr, nullptr, nullptr, &h, &err) == PG_OK && h.m == 0);
}

int main() {
    patterns();
    graphs();
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host driver ok\n");
    return 0;
}
