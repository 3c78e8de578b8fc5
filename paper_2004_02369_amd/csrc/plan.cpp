// Exploration-plan compiler (host).
//
// Follows Sec. 4.1 (Fig. "Computing exploration plan"): break the pattern's
// symmetries with a partial order (Grochow-Kellis), take the core as the
// subgraph induced by a minimum connected vertex cover, and enumerate the
// matching orders as the linear extensions of the order restricted to the
// core.  Sec. 4.2: the cover also covers anti-edges, which are matched by
// set differences.  Sec. 4.3: anti-vertices stay out of the core, their
// checks run once the vertices they depend on are matched, and they take
// part in symmetry breaking as their own kind of vertex.
//
// The output is a set of "programs" the GPU interprets level by level: each
// level is one pattern vertex, with the earlier levels it must be adjacent
// to (intersections), non-adjacent to (differences), above / below (order
// ranges) and different from.  Vertices outside the core come last; the
// final level counts a group of interchangeable non-core vertices by set
// size, C(|S|, j), instead of enumerating them.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "pg_internal.hpp"

namespace pg {
namespace {

constexpr int kMaxLinearExtensions = 720;

struct Typed {
    int k = 0, nav = 0;
    uint32_t E[kMaxK] = {};   // true edges among regular vertices
    uint32_t A[kMaxK] = {};   // anti-edges among regular vertices
    uint32_t AV[kMaxAV] = {}; // regular neighbours of each anti-vertex
    int lab[kMaxK];
    int avlab[kMaxAV];
};

inline int popc(uint32_t x) { return __builtin_popcount(x); }

int ptype(const Typed &t, int i, int j) {
    if (t.E[i] >> j & 1u) return 1;
    if (t.A[i] >> j & 1u) return 2;
    return 0;
}

bool parse(const pg_pattern_desc *d, Typed *t, std::string *err) {
    if (!d) { *err = "pattern is NULL"; return false; }
    if (d->k < 2 || d->k > kMaxK) { *err = "k must be in [2, 16]"; return false; }
    if (d->n_anti_vertices < 0 || d->n_anti_vertices > kMaxAV) { *err = "at most 4 anti-vertices"; return false; }
    if (d->n_edges < 0 || (d->n_edges > 0 && !d->edges)) { *err = "bad edge list"; return false; }
    t->k = d->k;
    t->nav = d->n_anti_vertices;
    const int tot = t->k + t->nav;
    for (int i = 0; i < kMaxK; i++) t->lab[i] = -1;
    for (int a = 0; a < kMaxAV; a++) t->avlab[a] = -1;
    if (d->labels) {
        for (int i = 0; i < tot; i++) {
            if (d->labels[i] < -1) { *err = "labels must be >= -1"; return false; }
            if (i < t->k) t->lab[i] = d->labels[i];
            else t->avlab[i - t->k] = d->labels[i];
        }
    }
    for (int e = 0; e < d->n_edges; e++) {
        int u = d->edges[e].u, v = d->edges[e].v, ty = d->edges[e].type;
        if (u < 0 || v < 0 || u >= tot || v >= tot || u == v) { *err = "edge endpoint out of range"; return false; }
        if (ty != PG_EDGE && ty != PG_ANTI_EDGE) { *err = "unknown edge type"; return false; }
        bool ru = u < t->k, rv = v < t->k;
        if (ru && rv) {
            if (ty == PG_EDGE) { t->E[u] |= 1u << v; t->E[v] |= 1u << u; }
            else { t->A[u] |= 1u << v; t->A[v] |= 1u << u; }
        } else if (!ru && !rv) {
            *err = "an edge between two anti-vertices";
            return false;
        } else {
            if (ty != PG_ANTI_EDGE) { *err = "an anti-vertex may only have anti-edges"; return false; }
            int a = ru ? v - t->k : u - t->k, r = ru ? u : v;
            t->AV[a] |= 1u << r;
        }
    }
    for (int i = 0; i < t->k; i++)
        if (t->E[i] & t->A[i]) { *err = "a pair is both an edge and an anti-edge"; return false; }
    for (int a = 0; a < t->nav; a++)
        if (!t->AV[a]) { *err = "an anti-vertex without anti-edges"; return false; }
    if (d->induced) {
        for (int i = 0; i < t->k; i++)
            for (int j = 0; j < t->k; j++)
                if (i != j && !(t->E[i] >> j & 1u)) t->A[i] |= 1u << j;
    }
    // regular vertices connected by true edges
    uint32_t seen = 1, frontier = 1;
    while (frontier) {
        uint32_t nx = 0;
        for (int i = 0; i < t->k; i++)
            if (frontier >> i & 1u) nx |= t->E[i];
        frontier = nx & ~seen;
        seen |= nx;
    }
    if (seen != ((1u << t->k) - 1u)) { *err = "regular vertices are not connected by true edges"; return false; }
    return true;
}

// ------------------------------------------------ typed automorphism search

uint64_t vertex_sig(const Typed &t, int i) {
    uint64_t n_av = 0, av_sz = 0;
    for (int a = 0; a < t.nav; a++)
        if (t.AV[a] >> i & 1u) { n_av++; av_sz += (uint64_t)popc(t.AV[a]) * 16 + (uint64_t)(t.avlab[a] + 1); }
    return (uint64_t)(t.lab[i] + 1) | (uint64_t)popc(t.E[i]) << 16 | (uint64_t)popc(t.A[i]) << 21 |
           n_av << 26 | av_sz << 30;
}

// Searches for an automorphism pi of the typed pattern with pi(f) = f for
// every f in `fixed` and pi(v) = w.  Backtracking over vertices in an order
// that keeps each newly placed vertex adjacent (edge or anti-edge) to placed
// ones, so type mismatches prune early; the anti-vertex neighbourhood
// multiset is checked on complete permutations.
struct AutSearch {
    const Typed &t;
    uint64_t sig[kMaxK];
    int order[kMaxK];
    int img[kMaxK];
    bool used[kMaxK];
    uint32_t fixed;
    int v, w;

    explicit AutSearch(const Typed &tt) : t(tt) {
        for (int i = 0; i < t.k; i++) sig[i] = vertex_sig(t, i);
    }

    bool av_ok() const {
        bool taken[kMaxAV] = {false, false, false, false};
        for (int a = 0; a < t.nav; a++) {
            uint32_t im = 0;
            for (int i = 0; i < t.k; i++)
                if (t.AV[a] >> i & 1u) im |= 1u << img[i];
            bool found = false;
            for (int b = 0; b < t.nav && !found; b++)
                if (!taken[b] && t.AV[b] == im && t.avlab[b] == t.avlab[a]) { taken[b] = true; found = true; }
            if (!found) return false;
        }
        return true;
    }

    bool rec(int pos) {
        if (pos == t.k) return av_ok();
        int x = order[pos];
        int cands[kMaxK], nc = 0;
        if (x == v) cands[nc++] = w;
        else if (fixed >> x & 1u) cands[nc++] = x;
        else
            for (int c = 0; c < t.k; c++)
                if (!used[c] && sig[c] == sig[x]) cands[nc++] = c;
        for (int ci = 0; ci < nc; ci++) {
            int c = cands[ci];
            if (used[c] || sig[c] != sig[x]) continue;
            bool ok = true;
            for (int p = 0; p < pos && ok; p++) {
                int y = order[p];
                if (ptype(t, x, y) != ptype(t, c, img[y])) ok = false;
            }
            if (!ok) continue;
            used[c] = true;
            img[x] = c;
            if (rec(pos + 1)) return true;
            used[c] = false;
        }
        return false;
    }

    bool exists(uint32_t fixed_, int v_, int w_) {
        fixed = fixed_;
        v = v_;
        w = w_;
        if (sig[v] != sig[w]) return false;
        if ((fixed >> v & 1u) && v != w) return false;
        if ((fixed >> w & 1u) && v != w) return false;
        // placement order: v, fixed vertices, then breadth-first over typed adjacency
        uint32_t placed = 0;
        int n = 0;
        order[n++] = v;
        placed |= 1u << v;
        for (int i = 0; i < t.k; i++)
            if ((fixed >> i & 1u) && !(placed >> i & 1u)) { order[n++] = i; placed |= 1u << i; }
        while (n < t.k) {
            int best = -1, best_links = -1;
            for (int i = 0; i < t.k; i++) {
                if (placed >> i & 1u) continue;
                int links = popc((t.E[i] | t.A[i]) & placed);
                if (links > best_links) { best_links = links; best = i; }
            }
            order[n++] = best;
            placed |= 1u << best;
        }
        for (int i = 0; i < t.k; i++) used[i] = false;
        return rec(0);
    }
};

// ------------------------------------------------------ symmetry breaking

struct SymmetryBreak {
    uint32_t lt[kMaxK] = {};  // lt[a] bit b: m(a) < m(b) required
    std::vector<std::pair<int, int>> pairs;
    std::vector<int> orbit_size, orbit_vertex;
    uint64_t aut = 1;
};

void close_order(uint32_t lt[kMaxK], int k) {
    for (int m = 0; m < k; m++)
        for (int i = 0; i < k; i++)
            if (lt[i] >> m & 1u) lt[i] |= lt[m];
}

// Grochow-Kellis: while the (pointwise stabiliser) group is not trivial,
// take the largest orbit, order its smallest vertex below every other
// member, and fix that vertex.  |Aut_t| is the product of the orbit sizes.
// (Any choice breaks the symmetry exactly; this one reproduces the paper's
// diamond example.)
SymmetryBreak break_symmetries(const Typed &t, uint32_t fixed0) {
    SymmetryBreak sb;
    AutSearch S(t);
    uint32_t fixed = fixed0;  // vertices every automorphism used must fix
    for (;;) {
        int orbit_of[kMaxK];
        for (int i = 0; i < t.k; i++) orbit_of[i] = -1;
        std::vector<uint32_t> orbits;
        for (int v = 0; v < t.k; v++) {
            if (orbit_of[v] >= 0) continue;
            uint32_t o = 1u << v;
            orbit_of[v] = (int)orbits.size();
            if (!(fixed >> v & 1u))
                for (int w = v + 1; w < t.k; w++)
                    if (orbit_of[w] < 0 && !(fixed >> w & 1u) && S.exists(fixed, v, w)) {
                        o |= 1u << w;
                        orbit_of[w] = (int)orbits.size();
                    }
            orbits.push_back(o);
        }
        int best = -1;
        for (size_t i = 0; i < orbits.size(); i++)
            if (best < 0 || popc(orbits[i]) > popc(orbits[best])) best = (int)i;  // ties: lowest vertex
        if (popc(orbits[best]) <= 1) break;
        int v = __builtin_ctz(orbits[best]);
        for (int w = 0; w < t.k; w++)
            if ((orbits[best] >> w & 1u) && w != v) {
                sb.lt[v] |= 1u << w;
                sb.pairs.push_back({v, w});
            }
        sb.orbit_size.push_back(popc(orbits[best]));
        sb.orbit_vertex.push_back(v);
        sb.aut *= (uint64_t)popc(orbits[best]);
        fixed |= 1u << v;
    }
    close_order(sb.lt, t.k);
    return sb;
}

// --------------------------------------------------------- core selection

bool connected_in(const Typed &t, uint32_t mask) {
    if (!mask) return false;
    uint32_t seen = mask & (~mask + 1u), frontier = seen;
    while (frontier) {
        uint32_t nx = 0;
        for (int i = 0; i < t.k; i++)
            if (frontier >> i & 1u) nx |= t.E[i] & mask;
        frontier = nx & ~seen;
        seen |= nx;
    }
    return seen == mask;
}

bool covers(const Typed &t, uint32_t mask) {
    for (int i = 0; i < t.k; i++) {
        if (mask >> i & 1u) continue;
        if ((t.E[i] | t.A[i]) & ~mask) return false;  // an edge/anti-edge with both ends outside
    }
    return true;
}

// Minimum vertex cover of true edges and anti-edges that is connected by
// true edges (anti-vertices excluded).  Among minimum covers: most true
// edges inside the core (fewer core matches), then the smallest vertex set.
uint32_t min_connected_cover(const Typed &t, uint32_t must) {
    const uint32_t full = (1u << t.k) - 1u;
    for (int s = 1; s <= t.k; s++) {
        uint32_t best = 0;
        int best_edges = -1;
        uint32_t m = (1u << s) - 1u;
        while (m <= full) {
            if ((m & must) == must && covers(t, m) && connected_in(t, m)) {
                int e = 0;
                for (int i = 0; i < t.k; i++)
                    if (m >> i & 1u) e += popc(t.E[i] & m);
                if (e > best_edges) { best_edges = e; best = m; }
            }
            uint32_t c = m & (~m + 1u), r = m + c;  // next mask with s bits (Gosper)
            if (r == 0) break;
            m = (((r ^ m) >> 2) / c) | r;
        }
        if (best) return best;
    }
    return full;
}

// --------------------------------------------------------- matching orders

void linear_extensions(const uint32_t lt[kMaxK], uint32_t core, int k, uint32_t placed,
                       std::vector<int> &seq, std::vector<std::vector<int>> &out, size_t cap) {
    if (out.size() > cap) return;
    if (placed == core) { out.push_back(seq); return; }
    for (int v = 0; v < k; v++) {
        if (!(core >> v & 1u) || (placed >> v & 1u)) continue;
        bool ready = true;
        for (int u = 0; u < k && ready; u++)
            if ((core >> u & 1u) && !(placed >> u & 1u) && (lt[u] >> v & 1u)) ready = false;
        if (!ready) continue;
        seq.push_back(v);
        linear_extensions(lt, core, k, placed | 1u << v, seq, out, cap);
        seq.pop_back();
    }
}

// Score of an exploration sequence of the core: prefer levels whose new
// vertex has a true neighbour already matched *below* it in the order (its
// candidates then come from the upper part of a degree-ordered row), and
// more intersections early.
long long sequence_score(const Typed &t, const std::vector<int> &seq, const uint32_t lt[kMaxK]) {
    long long s = 0;
    int c = (int)seq.size();
    for (int i = 1; i < c; i++) {
        int x = seq[i];
        bool oriented = false;
        int isect = 0;
        for (int j = 0; j < i; j++) {
            int y = seq[j];
            if (t.E[x] >> y & 1u) {
                isect++;
                if (lt[y] >> x & 1u) oriented = true;
            }
        }
        if (i >= 2 && oriented) s += 1000;
        s += (long long)isect * (c - i) * 10;
    }
    return s;
}

bool seq_connected(const Typed &t, const std::vector<int> &seq) {
    for (size_t i = 1; i < seq.size(); i++) {
        bool ok = false;
        for (size_t j = 0; j < i && !ok; j++)
            if (t.E[seq[i]] >> seq[j] & 1u) ok = true;
        if (!ok) return false;
    }
    return true;
}

std::vector<int> choose_sequence(const Typed &t, uint32_t core, const uint32_t lt[kMaxK], int first = -1) {
    std::vector<int> verts;
    for (int i = 0; i < t.k; i++)
        if (core >> i & 1u) verts.push_back(i);
    if (verts.size() <= 7) {
        std::vector<int> best;
        long long best_s = -1;
        std::vector<int> p = verts;
        do {
            if (!seq_connected(t, p)) continue;
            // anchored: the anchor is one of the root vertices
            if (first >= 0 && p[0] != first && !(p.size() > 1 && p[1] == first)) continue;
            long long s = sequence_score(t, p, lt);
            if (s > best_s) { best_s = s; best = p; }
        } while (std::next_permutation(p.begin(), p.end()));
        return best;
    }
    // greedy for large cores: start at the lowest vertex in the order that
    // has a core neighbour, then repeatedly add the best-scoring neighbour
    std::vector<int> seq;
    uint32_t placed = 0;
    int start = verts[0];
    for (int v : verts) {
        bool minimal = true;
        for (int u : verts)
            if (lt[u] >> v & 1u) minimal = false;
        if (minimal) { start = v; break; }
    }
    if (first >= 0) start = first;
    seq.push_back(start);
    placed |= 1u << start;
    while (seq.size() < verts.size()) {
        int best = -1;
        long long best_s = -1;
        for (int v : verts) {
            if (placed >> v & 1u) continue;
            if (!(t.E[v] & placed)) continue;
            std::vector<int> s2 = seq;
            s2.push_back(v);
            long long s = sequence_score(t, s2, lt);
            if (s > best_s) { best_s = s; best = v; }
        }
        seq.push_back(best);
        placed |= 1u << best;
    }
    return seq;
}

// --------------------------------------------------------- program builder

uint32_t involvement(const Typed &t) {
    uint32_t inv = 0;
    for (int a = 0; a < t.nav; a++) {
        inv |= t.AV[a];
        for (int u = 0; u < t.k; u++)
            if (t.AV[a] >> u & 1u) inv |= t.E[u];
    }
    return inv;
}

// Groups of interchangeable non-core vertices: identical neighbours,
// anti-neighbours, label and order relations to every vertex outside the
// group, totally ordered among themselves.  Vertices an anti-vertex check
// depends on stay alone.
std::vector<std::vector<int>> noncore_groups(const Typed &t, uint32_t core, const uint32_t lt[kMaxK],
                                             bool singletons) {
    const uint32_t full = (1u << t.k) - 1u, noncore = full & ~core;
    const uint32_t inv = involvement(t);
    auto pred = [&](int x) {
        uint32_t p = 0;
        for (int y = 0; y < t.k; y++)
            if (lt[y] >> x & 1u) p |= 1u << y;
        return p;
    };
    std::map<std::tuple<uint32_t, uint32_t, int, int, uint32_t, uint32_t>, std::vector<int>> init;
    for (int x = 0; x < t.k; x++) {
        if (!(noncore >> x & 1u)) continue;
        int tag = (singletons || (inv >> x & 1u)) ? x : -1;
        init[{t.E[x], t.A[x], t.lab[x], tag, lt[x] & core, pred(x) & core}].push_back(x);
    }
    std::vector<std::vector<int>> cls;
    for (auto &kv : init) cls.push_back(kv.second);
    bool changed = true;
    while (changed) {
        changed = false;
        std::vector<std::vector<int>> nx;
        for (auto &c : cls) {
            if (c.size() < 2) { nx.push_back(c); continue; }
            uint32_t cm = 0;
            for (int x : c) cm |= 1u << x;
            std::map<std::pair<uint32_t, uint32_t>, std::vector<int>> sp;
            for (int x : c) sp[{lt[x] & noncore & ~cm, pred(x) & noncore & ~cm}].push_back(x);
            if (sp.size() > 1) changed = true;
            for (auto &kv : sp) nx.push_back(kv.second);
        }
        cls.swap(nx);
    }
    std::vector<std::vector<int>> out;
    for (auto &c : cls) {
        bool chain = true;
        for (int x : c)
            for (int y : c)
                if (x != y && !(lt[x] >> y & 1u) && !(lt[y] >> x & 1u)) chain = false;
        if (!chain) {
            for (int x : c) out.push_back({x});
            continue;
        }
        std::sort(c.begin(), c.end(), [&](int a, int b) { return (lt[a] >> b & 1u) != 0; });
        out.push_back(c);
    }
    return out;
}

struct BuiltProgram {
    Program prog;
    bool need_split = false;  // level 0 / 1 unordered: caller retries with each order added
    int root_a = -1, root_b = -1;
};

BuiltProgram build_program(const Typed &t, const std::vector<int> &core_seq, uint32_t core,
                           const uint32_t lt_in[kMaxK], bool emit) {
    BuiltProgram bp;
    uint32_t lt[kMaxK];
    std::memcpy(lt, lt_in, sizeof(lt));
    auto groups = noncore_groups(t, core, lt, emit);
    const uint32_t inv = involvement(t);
    // last group: not tied to an anti-vertex, largest, least constrained
    int last = -1;
    for (int g = 0; g < (int)groups.size(); g++) {
        auto key = [&](int gi) {
            int x = groups[gi][0];
            bool tied = (inv >> x & 1u) != 0;
            return std::make_tuple(!tied, (int)groups[gi].size(), -(popc(t.E[x]) + popc(t.A[x])), -x);
        };
        if (last < 0 || key(g) > key(last)) last = g;
    }
    std::vector<int> order_groups;
    for (int g = 0; g < (int)groups.size(); g++)
        if (g != last) order_groups.push_back(g);
    std::sort(order_groups.begin(), order_groups.end(), [&](int a, int b) {
        int xa = groups[a][0], xb = groups[b][0];
        int ca = popc(t.E[xa]) + popc(t.A[xa]), cb = popc(t.E[xb]) + popc(t.A[xb]);
        if (ca != cb) return ca > cb;
        return xa < xb;
    });
    // Count programs: a group whose fixed label no other non-core vertex
    // can carry, with no anti-vertex and no order relation to another
    // non-core vertex beyond what the core's order implies, never shares an
    // image with the other non-core vertices, so its C(|S|, j) multiplies
    // the rest instead of being enumerated (the set-size counting of
    // non-core vertices, Sec. 4, applied to each independent group)
    std::vector<int> fac_groups;
    if (!emit) {
        const uint32_t noncore = ((1u << t.k) - 1u) & ~core;
        auto implied = [&](int a, int b) {  // a < b follows from a < c < b, c in the core
            for (int c = 0; c < t.k; c++)
                if ((core >> c & 1u) && (lt[a] >> c & 1u) && (lt[c] >> b & 1u)) return true;
            return false;
        };
        std::vector<int> keep;
        for (int g : order_groups) {
            uint32_t gm = 0;
            for (int x : groups[g]) gm |= 1u << x;
            const int lab = t.lab[groups[g][0]];
            bool ok = lab >= 0 && !(gm & inv);
            for (int y = 0; ok && y < t.k; y++) {
                if (!(noncore >> y & 1u) || (gm >> y & 1u)) continue;
                if (t.lab[y] < 0 || t.lab[y] == lab) ok = false;
                for (int x : groups[g]) {
                    if ((lt[x] >> y & 1u) && !implied(x, y)) ok = false;
                    if ((lt[y] >> x & 1u) && !implied(y, x)) ok = false;
                }
            }
            (ok ? fac_groups : keep).push_back(g);
        }
        order_groups.swap(keep);
    }
    std::vector<int> seq = core_seq;
    for (int g : order_groups)
        for (int x : groups[g]) seq.push_back(x);
    seq.push_back(groups[last][0]);
    const int F = (int)seq.size() - 1;
    const int jgroup = (int)groups[last].size();

    if (F >= 2) {
        int a = seq[0], b = seq[1];
        if (lt[b] >> a & 1u) std::swap(seq[0], seq[1]);
        else if (!(lt[a] >> b & 1u)) {
            bp.need_split = true;
            bp.root_a = a;
            bp.root_b = b;
            return bp;
        }
    }
    int level_of[kMaxK];
    for (int i = 0; i < kMaxK; i++) level_of[i] = -1;
    for (int x = 0; x <= F; x++) level_of[seq[x]] = x;
    // pattern vertex u matched at level x, against the images of levels < x
    auto make_level = [&](int u, int x, int group) {
        Level L;
        for (int y = 0; y < x; y++) {
            int w = seq[y];
            uint32_t bit = 1u << y;
            if (t.E[u] >> w & 1u) L.isect |= bit;
            if (t.A[u] >> w & 1u) L.diff |= bit;
            if (lt[w] >> u & 1u) L.lo |= bit;
            if (lt[u] >> w & 1u) L.hi |= bit;
        }
        L.excl = ((1u << x) - 1u) & ~(L.isect | L.lo | L.hi);
        for (int y = 0; y < x && L.isect; y++) {
            if (!(L.excl >> y & 1u)) continue;
            const int w = seq[y];
            bool in = t.lab[u] < 0 || t.lab[w] == t.lab[u];
            for (int z = 0; z < x && in; z++) {
                if ((L.isect >> z & 1u) && !(t.E[w] >> seq[z] & 1u)) in = false;
                if ((L.diff >> z & 1u) && !(t.A[w] >> seq[z] & 1u)) in = false;
            }
            if (in) L.excl_in |= 1u << y;
        }
        L.label = t.lab[u];
        L.pv = u;
        L.group = group;
        return L;
    };
    bp.prog.lev.resize(F + 1);
    for (int x = 0; x <= F; x++) bp.prog.lev[x] = make_level(seq[x], x, x == F ? jgroup : 1);
    for (int g : fac_groups) bp.prog.factors.push_back(make_level(groups[g][0], F, (int)groups[g].size()));
    // anti-vertex checks: evaluated at the deepest level they depend on
    for (int a = 0; a < t.nav; a++) {
        uint32_t deps = t.AV[a];
        for (int u = 0; u < t.k; u++)
            if (t.AV[a] >> u & 1u) deps |= t.E[u];
        int trig = 0;
        for (int u = 0; u < t.k; u++)
            if (deps >> u & 1u) trig = std::max(trig, level_of[u]);
        AVCheck c;
        std::memset(&c, 0, sizeof(c));
        c.label = t.avlab[a];
        for (int u = 0; u < t.k; u++) {
            if (!(t.AV[a] >> u & 1u)) continue;
            int lu = level_of[u];
            c.nbr |= 1u << lu;
            for (int w = 0; w < t.k; w++)
                if (t.E[u] >> w & 1u) c.xmask[lu] |= 1u << level_of[w];
        }
        bp.prog.lev[trig].avs.push_back(c);
    }
    // base sets: a materialised earlier level (>= 2, below the final level's
    // parent chain) whose candidates contain every candidate of this level
    auto pick_base = [&](Level &L, int x) {
        int best = -1, best_cov = -1;
        for (int b = 2; b < x; b++) {
            const Level &B = bp.prog.lev[b];
            if ((B.isect & ~L.isect) || (B.diff & ~L.diff) || (B.lo & ~L.lo) || (B.hi & ~L.hi)) continue;
            if (B.label != -1 && B.label != L.label) continue;
            if (!B.avs.empty()) continue;
            int cov = popc(B.isect) + popc(B.diff);
            if (cov >= best_cov) { best_cov = cov; best = b; }
        }
        L.base = best;
        if (best >= 0) {
            L.t_isect = L.isect & ~bp.prog.lev[best].isect;
            L.t_diff = L.diff & ~bp.prog.lev[best].diff;
        } else {
            L.t_isect = L.isect;
            L.t_diff = L.diff;
        }
    };
    for (int x = 2; x <= F; x++) pick_base(bp.prog.lev[x], x);
    for (Level &L : bp.prog.factors) pick_base(L, F);
    for (int x = 0; x < 2 && x <= F; x++) {
        bp.prog.lev[x].t_isect = bp.prog.lev[x].isect;
        bp.prog.lev[x].t_diff = bp.prog.lev[x].diff;
    }
    return bp;
}

void add_programs(const Typed &t, const std::vector<int> &core_seq, uint32_t core, const uint32_t lt[kMaxK],
                  bool emit, std::vector<Program> &out, int depth = 0) {
    BuiltProgram bp = build_program(t, core_seq, core, lt, emit);
    if (!bp.need_split) {
        out.push_back(std::move(bp.prog));
        return;
    }
    // The two root vertices are unordered: they are adjacent, hence always
    // distinct, so the maps split into m(a) < m(b) and m(b) < m(a).
    if (depth > 2) return;  // cannot happen: each split orders the root pair
    uint32_t l1[kMaxK], l2[kMaxK];
    std::memcpy(l1, lt, sizeof(l1));
    std::memcpy(l2, lt, sizeof(l2));
    l1[bp.root_a] |= 1u << bp.root_b;
    l2[bp.root_b] |= 1u << bp.root_a;
    close_order(l1, t.k);
    close_order(l2, t.k);
    add_programs(t, core_seq, core, l1, emit, out, depth + 1);
    add_programs(t, core_seq, core, l2, emit, out, depth + 1);
}

std::string program_key(const Program &p, int anchor) {
    std::string s;
    auto put = [&](uint64_t v) { s.append(reinterpret_cast<const char *>(&v), sizeof(v)); };
    put(p.lev.size());
    // anchored: programs that hold the anchor at different levels mark
    // different vertices and must stay apart
    for (size_t y = 0; anchor >= 0 && y < p.lev.size(); y++)
        if (p.lev[y].pv == anchor) put(y);
    put(p.factors.size());
    for (const std::vector<Level> *ls : {&p.lev, &p.factors})
        for (const Level &L : *ls) {
            put(L.isect); put(L.diff); put(L.lo); put(L.hi); put(L.excl);
            put((uint64_t)(int64_t)L.label); put((uint64_t)L.group); put(L.avs.size());
            for (const AVCheck &c : L.avs) {
                put(c.nbr); put((uint64_t)(int64_t)c.label);
                for (int i = 0; i < kMaxLevels; i++) put(c.xmask[i]);
            }
        }
    return s;
}

std::string mo_key(const Typed &t, const std::vector<int> &L) {
    std::string s;
    for (size_t i = 0; i < L.size(); i++)
        for (size_t j = i + 1; j < L.size(); j++) s.push_back((char)('0' + ptype(t, L[i], L[j])));
    for (int v : L) s += "," + std::to_string(t.lab[v]);
    return s;
}

}  // namespace

pg_status compile_plan(const pg_pattern_desc *desc, const pg_plan_options *opt, PlanImpl *out,
                       std::string *err) {
    auto t0 = std::chrono::steady_clock::now();
    Typed t;
    if (!parse(desc, &t, err)) return PG_EINVAL;
    int mode = opt ? opt->mode : PG_PLAN_AUTO;
    if (mode < PG_PLAN_AUTO || mode > PG_PLAN_PARTIAL_ORDER) { *err = "unknown plan mode"; return PG_EINVAL; }

    const bool anchored = opt && opt->anchored;
    if (opt && (opt->anchored < 0 || opt->anchored > 1)) { *err = "anchored must be 0 or 1"; return PG_EINVAL; }
    if (anchored && (opt->anchor < 0 || opt->anchor >= t.k)) { *err = "anchor out of range"; return PG_EINVAL; }
    const uint32_t must = anchored ? 1u << opt->anchor : 0u;
    uint32_t core = min_connected_cover(t, must);
    SymmetryBreak sb = break_symmetries(t, must);

    std::vector<std::vector<int>> les;
    std::vector<int> seq;
    linear_extensions(sb.lt, core, t.k, 0, seq, les, kMaxLinearExtensions);
    int mode_used = mode;
    if (mode == PG_PLAN_AUTO)
        mode_used = les.size() <= (size_t)kMaxLinearExtensions ? PG_PLAN_LINEAR_EXT : PG_PLAN_PARTIAL_ORDER;
    if (mode_used == PG_PLAN_LINEAR_EXT && les.size() > (size_t)kMaxLinearExtensions) {
        *err = "too many matching orders; use the partial-order plan mode";
        return PG_EUNSUPPORTED;
    }

    PlanImpl &P = *out;
    P.k = t.k;
    std::vector<Program> cprogs, eprogs;
    int n_mo = 0;
    if (mode_used == PG_PLAN_LINEAR_EXT) {
        std::map<std::string, int> mos;
        for (const auto &L : les) {
            mos[mo_key(t, L)]++;
            // relations: the partial order plus the total order of this extension
            uint32_t lt[kMaxK];
            std::memcpy(lt, sb.lt, sizeof(lt));
            for (size_t i = 0; i + 1 < L.size(); i++) lt[L[i]] |= 1u << L[i + 1];
            close_order(lt, t.k);
            std::vector<int> cs = choose_sequence(t, core, lt, anchored ? opt->anchor : -1);
            add_programs(t, cs, core, lt, false, cprogs);
            add_programs(t, cs, core, lt, true, eprogs);
        }
        n_mo = (int)mos.size();
    } else {
        std::vector<int> cs = choose_sequence(t, core, sb.lt, anchored ? opt->anchor : -1);
        add_programs(t, cs, core, sb.lt, false, cprogs);
        add_programs(t, cs, core, sb.lt, true, eprogs);
        n_mo = 1;
    }
    // merge identical count programs (their counts are equal)
    std::map<std::string, size_t> idx;
    for (auto &p : cprogs) {
        std::string key = program_key(p, anchored ? opt->anchor : -1);
        auto it = idx.find(key);
        if (it == idx.end()) {
            idx[key] = P.count_progs.size();
            P.count_progs.push_back(std::move(p));
        } else {
            P.count_progs[it->second].mult += p.mult;
        }
    }
    P.enum_progs = std::move(eprogs);

    pg_plan_info_t &I = P.info;
    std::memset(&I, 0, sizeof(I));
    I.aut = sb.aut;
    I.k = t.k;
    I.core_mask = core;
    I.core_size = popc(core);
    I.n_matching_orders = n_mo;
    I.n_programs = (int32_t)P.count_progs.size();
    int maxlev = 0;
    for (auto &p : P.count_progs) maxlev = std::max(maxlev, (int)p.lev.size());
    for (auto &p : P.enum_progs) maxlev = std::max(maxlev, (int)p.lev.size());
    I.n_levels = maxlev;
    I.n_order = (int32_t)std::min<size_t>(sb.pairs.size(), 120);
    for (int i = 0; i < I.n_order; i++) {
        I.order[2 * i] = sb.pairs[i].first;
        I.order[2 * i + 1] = sb.pairs[i].second;
    }
    I.n_orbit_steps = (int32_t)sb.orbit_size.size();
    for (int i = 0; i < I.n_orbit_steps && i < 16; i++) {
        I.orbit_size[i] = sb.orbit_size[i];
        I.orbit_vertex[i] = sb.orbit_vertex[i];
    }
    I.mode_used = mode_used;
    I.anchor = anchored ? opt->anchor : -1;
    P.anchor = I.anchor;
    I.plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return PG_OK;
}

// ------------------------------------------------------------------- trie

namespace {

struct HostNode {
    Node n;
    std::vector<AVCheck> avs;
    std::vector<int> children;
    std::string key;
    bool product = false;  // a factor node, or the count node closing a product
};

std::string node_key(const Node &n, const std::vector<AVCheck> &avs) {
    std::string s;
    auto put = [&](uint64_t v) { s.append(reinterpret_cast<const char *>(&v), sizeof(v)); };
    put((uint64_t)n.kind); put((uint64_t)n.level); put(n.isect); put(n.diff); put(n.lo); put(n.hi);
    put(n.excl); put(n.excl_in); put(n.t_isect); put(n.t_diff); put((uint64_t)(int64_t)n.base);
    put((uint64_t)(int64_t)n.label); put((uint64_t)n.group); put((uint64_t)(int64_t)n.label0);
    put((uint64_t)(int64_t)n.label1);
    if (n.kind == kCount || n.kind == kEmit || n.kind == kFactor || n.anchor_level >= 0) {
        put((uint64_t)n.plan);
        put(n.mult);
        put((uint64_t)(int64_t)n.anchor_level);
        for (int i = 0; i < kMaxLevels; i++) put((uint64_t)(int64_t)n.pv[i]);
    }
    put(avs.size());
    for (const AVCheck &c : avs) {
        put(c.nbr); put((uint64_t)(int64_t)c.label);
        for (int i = 0; i < kMaxLevels; i++) put(c.xmask[i]);
    }
    return s;
}

Node blank_node() {
    Node n;
    std::memset(&n, 0, sizeof(n));
    n.base = -1;
    n.label = -1;
    n.label0 = -1;
    n.label1 = -1;
    n.group = 1;
    n.mult = 1;
    for (int i = 0; i < kMaxLevels; i++) n.pv[i] = -1;
    n.anchor_level = -1;
    n.share = -1;
    return n;
}

}  // namespace

// Enumeration nodes whose count children each add a term that does not
// depend on the node's own vertex (see kIndepCounts): the count child has one
// row of an earlier level as its only operand, no range, and excludes this
// level's image, which the pattern places inside that row.
void mark_independent_counts(Trie &T, const std::vector<bool> &product) {
    for (size_t i = 0; i < T.nodes.size(); i++) {
        Node &E = T.nodes[i];
        if (E.kind != kEnum || E.child_count == 0 || E.av_count) continue;
        const int x = E.level;
        bool ok = true;
        for (int c = E.child_begin; c < E.child_begin + E.child_count && ok; c++) {
            const Node &N = T.nodes[c];
            ok = N.kind == kCount && !product[c] && __builtin_popcount(N.t_isect) == 1 && N.t_diff == 0 &&
                 N.base < 0 && N.lo == 0 && N.hi == 0 && N.label < 0 && N.av_count == 0 && N.anchor_level < 0 &&
                 !(N.isect >> x & 1u) && !(N.diff >> x & 1u) && (N.excl_in >> x & 1u);
        }
        if (ok) E.flags |= kIndepCounts;
    }
}

// Share groups.  Children of an edge root at level 2 that apply the same set
// operation (true-edge rows, anti-edge rows, exclusions) and differ only in
// their id ranges -- count nodes, and enumeration nodes whose children only
// count -- form a group when there are two or more of them.  The group gets
// a leader: an enumeration node outside the tree with the ranges every
// member shares (the intersection of their lo / hi level masks), whose
// candidates contain every member's.  The engine materialises the leader's
// candidates once per root task and reads each member's range out of them.
// Members with a base set, a label, anti-vertex checks, a domain anchor or
// a part in a product are left alone.
void share_groups(Trie &T, const std::vector<bool> &product) {
    const size_t n0 = T.nodes.size();
    for (size_t r = 0; r < T.roots.size(); r++) {
        const int rid = T.roots[r];
        if (T.nodes[rid].kind != kRootEdge) continue;
        const Node R = T.nodes[rid];
        std::map<std::vector<uint32_t>, std::vector<int>> groups;
        for (int c = R.child_begin; c < R.child_begin + R.child_count; c++) {
            const Node &N = T.nodes[c];
            if (N.level != 2 || N.base >= 0 || N.label >= 0 || N.av_count || N.anchor_level >= 0 || product[c])
                continue;
            if (N.kind == kEnum) {
                bool leaf = true;
                for (int d = N.child_begin; d < N.child_begin + N.child_count; d++)
                    if (T.nodes[d].kind == kEnum) leaf = false;
                if (!leaf) continue;
            } else if (N.kind != kCount) {
                continue;
            }
            groups[{N.isect, N.diff, N.excl, N.t_isect, N.t_diff}].push_back(c);
        }
        std::vector<int32_t> leaders;
        for (auto &kv : groups) {
            const std::vector<int> &mem = kv.second;
            if (mem.size() < 2) continue;
            Node L = T.nodes[mem[0]];
            L.kind = kEnum;
            L.flags = 0;
            L.group = 1;
            L.plan = 0;
            L.mult = 1;
            L.child_begin = L.child_count = 0;
            for (int m : mem) {
                L.lo &= T.nodes[m].lo;
                L.hi &= T.nodes[m].hi;
            }
            L.share = -1;
            L.list_begin = (int32_t)T.lists.size();
            L.list_count = (int32_t)mem.size();
            const int lid = (int)T.nodes.size();
            for (int m : mem) {
                T.lists.push_back(m);
                T.nodes[m].share = lid;
            }
            T.nodes.push_back(L);
            leaders.push_back(lid);
        }
        if (!leaders.empty()) {
            T.nodes[rid].list_begin = (int32_t)T.lists.size();
            T.nodes[rid].list_count = (int32_t)leaders.size();
            for (int32_t l : leaders) T.lists.push_back(l);
        }
    }
    (void)n0;
}

Trie build_trie(const std::vector<const PlanImpl *> &plans, bool emit) {
    std::vector<HostNode> H;
    std::vector<int> roots;
    // find or add a child of `parent` (-1: a root); H may reallocate, so the
    // parent's child list is looked up again after the insertion
    auto child = [&](int parent, HostNode &&hn) -> int {
        const std::vector<int> &kids = parent < 0 ? roots : H[parent].children;
        for (int c : kids)
            if (H[c].key == hn.key) return c;
        H.push_back(std::move(hn));
        const int id = (int)H.size() - 1;
        if (parent < 0) roots.push_back(id);
        else H[parent].children.push_back(id);
        return id;
    };
    size_t n_programs = 0;
    int max_level = 0;
    for (size_t pi = 0; pi < plans.size(); pi++) {
        const auto &progs = emit ? plans[pi]->enum_progs : plans[pi]->count_progs;
        for (const Program &p : progs) {
            const int F = (int)p.lev.size() - 1;
            max_level = std::max(max_level, F + 1);
            HostNode r;
            r.n = blank_node();
            r.n.kind = F == 1 ? kRootVertex : kRootEdge;
            r.n.level = F == 1 ? 0 : 1;
            r.n.label0 = p.lev[0].label;
            r.n.label1 = F == 1 ? -1 : p.lev[1].label;
            // an anchored plan's root knows where its anchor is, so a root
            // task whose anchor image is already in the domain is skipped
            if (plans[pi]->anchor >= 0)
                for (int y = 0; y <= r.n.level; y++)
                    if (p.lev[y].pv == plans[pi]->anchor) {
                        r.n.anchor_level = y;
                        r.n.plan = (int32_t)pi;
                    }
            for (int x = 0; x <= r.n.level; x++)
                for (const AVCheck &c : p.lev[x].avs) r.avs.push_back(c);
            r.key = node_key(r.n, r.avs);
            int cur = child(-1, std::move(r));
            n_programs++;
            int anchor_level = -1;
            for (int y = 0; y < F; y++)
                if (plans[pi]->anchor >= 0 && p.lev[y].pv == plans[pi]->anchor) anchor_level = y;
            auto level_node = [&](const Level &L, int x, int32_t kind) {
                HostNode h;
                h.n = blank_node();
                h.n.kind = kind;
                h.n.level = x;
                h.n.isect = L.isect; h.n.diff = L.diff; h.n.lo = L.lo; h.n.hi = L.hi; h.n.excl = L.excl;
                h.n.excl_in = L.excl_in;
                h.n.t_isect = L.t_isect; h.n.t_diff = L.t_diff; h.n.base = L.base;
                h.n.label = L.label;
                h.n.group = L.group;
                h.avs = L.avs;
                if (kind != kEnum) {
                    h.n.plan = (int32_t)pi;
                    h.n.anchor_level = anchor_level;
                }
                return h;
            };
            for (int x = H[cur].n.level + 1; x < F; x++) {
                HostNode h = level_node(p.lev[x], x, kEnum);
                h.key = node_key(h.n, h.avs);
                cur = child(cur, std::move(h));
            }
            // a product: its factor nodes, then the count node that closes
            // it, as consecutive siblings of their own (keys never shared)
            const std::string own = p.factors.empty() ? std::string() : "#" + std::to_string(n_programs);
            for (const Level &L : p.factors) {
                HostNode h = level_node(L, F, kFactor);
                h.key = node_key(h.n, h.avs) + own;
                h.product = true;
                child(cur, std::move(h));
            }
            if (F > H[cur].n.level) {
                HostNode h = level_node(p.lev[F], F, emit ? kEmit : kCount);
                h.n.mult = p.mult;
                h.n.k = plans[pi]->k;
                for (int y = 0; y <= F; y++) h.n.pv[y] = (int8_t)p.lev[y].pv;
                h.key = node_key(h.n, h.avs) + own;
                h.product = !own.empty();
                child(cur, std::move(h));
            }
        }
    }
    // flatten breadth-first so every node's children are contiguous,
    // count / emit children before enumeration children
    Trie T;
    T.max_level = max_level;
    {
        std::vector<int> order2;
        for (int r : roots) order2.push_back(r);
        for (size_t i = 0; i < order2.size(); i++) {
            std::vector<int> kids = H[order2[i]].children;
            std::stable_sort(kids.begin(), kids.end(), [&](int a, int b) {
                return (H[a].n.kind == kEnum) < (H[b].n.kind == kEnum);
            });
            for (int c : kids) order2.push_back(c);
        }
        std::vector<int> id2(H.size(), -1);
        for (size_t i = 0; i < order2.size(); i++) id2[order2[i]] = (int)i;
        T.nodes.assign(order2.size(), Node{});
        T.avs.clear();
        for (size_t i = 0; i < order2.size(); i++) {
            HostNode &h = H[order2[i]];
            Node n = h.n;
            n.av_begin = (int32_t)T.avs.size();
            n.av_count = (int32_t)h.avs.size();
            for (const AVCheck &c : h.avs) T.avs.push_back(c);
            std::vector<int> kids = h.children;
            std::stable_sort(kids.begin(), kids.end(), [&](int a, int b) {
                return (H[a].n.kind == kEnum) < (H[b].n.kind == kEnum);
            });
            n.child_count = (int32_t)kids.size();
            n.child_begin = kids.empty() ? 0 : id2[kids[0]];
            T.nodes[i] = n;
        }
        for (size_t r = 0; r < roots.size(); r++) {
            T.roots.push_back(id2[roots[r]]);
            if (H[roots[r]].n.kind == kRootVertex) T.has_vertex_root = true;
            else T.has_edge_root = true;
        }
        if (!emit) {
            std::vector<bool> product(T.nodes.size(), false);
            for (size_t i = 0; i < order2.size(); i++) product[i] = H[order2[i]].product;
            mark_independent_counts(T, product);
            share_groups(T, product);
        }
    }
    // every program ends in its own leaf (count programs are merged before,
    // so two leaves never share a key)
    size_t leaves = 0;
    for (const Node &n : T.nodes) leaves += (n.kind == kCount || n.kind == kEmit) ? 1 : 0;
    T.consistent = leaves == n_programs;
    return T;
}

}  // namespace pg
