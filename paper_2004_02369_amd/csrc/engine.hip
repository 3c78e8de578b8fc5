// GPU matching engine for gfx950 (CDNA4, wave64).
//
// One persistent kernel.  Every workgroup is one wavefront that repeatedly
// claims a chunk of root tasks from a global atomic cursor (the shared
// "next vertex" counter of Sec. 5.5; tasks pre-sorted so the costliest roots
// go first, Sec. 5.2) and interprets the program trie built by the plan
// compiler:
//
//  * root tasks are oriented edges (u < v in degree rank) for programs with
//    two or more levels before the final one, and single vertices otherwise;
//  * an enumeration node materialises its candidate set -- the intersection
//    of neighbour rows for true edges minus rows for anti-edges (Sec. 4.2),
//    restricted to the (lo, hi) id range the matching / partial order
//    allows (Sec. 5.1) -- wave-cooperatively into per-wave scratch: each
//    lane takes one element of the shortest positive operand, tests it by
//    binary search against the other sorted rows, and a ballot + popcount
//    compacts the survivors in order, so the set stays sorted;
//  * a count node completes the non-core vertices by set size (Sec. 5.1
//    completes them by intersections; here only |S| is needed): its work is
//    flattened over up to 64 prefixes at once -- per prefix, one or more
//    segments of driver elements are laid end to end and the wave's lanes
//    walk the concatenation, so short rows do not leave lanes idle.  When
//    the only positive operand is long and the differences are short the
//    count is taken by complement, |P| - |P & (D1 u D2 ...)|, driven by the
//    short difference rows;
//  * counts are reduced per wave in 64-bit and added to the per-plan
//    counters once per wave at exit.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "engine.hpp"

namespace pg {

constexpr int kP = 64;       // prefixes per flattened batch (one per lane)
constexpr int kSegPerPrefix = 3;
constexpr int kSeg = kP * kSegPerPrefix;
constexpr int kBaseOp = 31;  // operand id of the base set

struct Lds {
    int32_t m[kMaxLevels];
    long long roff[kMaxLevels];
    int32_t rlen[kMaxLevels];
    int32_t set_len[kMaxLevels];
    int32_t st_node[kMaxLevels];
    int32_t st_idx[kMaxLevels];
    int32_t st_child[kMaxLevels];
    // root tasks of the current batch
    int32_t tu[kP], tv[kP];
    // prefix batch: values of the (at most two) varying levels
    int32_t pv0[kP], pv1[kP];
    long long po0[kP], po1[kP];
    int32_t pl0[kP], pl1[kP];
    int32_t plo[kP], phi[kP];
    const int32_t *bptr[kP];
    int32_t blen[kP];
    const int32_t *p1ptr[kP];
    int32_t p1len[kP];
    int32_t pmode[kP];       // -1 skip, 0 direct, 1 complement
    int32_t pdrv[kP];
    uint32_t pcnt[kP];
    int32_t pconst[kP];
    int32_t seg_start[kSeg + 1];
    int16_t seg_prefix[kSeg];
    int16_t seg_op[kSeg];
    const int32_t *seg_ptr[kSeg];
    unsigned long long acc[kMaxPlansPerLaunch];
    int32_t nseg;
    int32_t total;
    int32_t stop;
    unsigned long long bytes;
};

__device__ __forceinline__ void wsync() { __syncthreads(); }

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// first index i in [0, n) with a[i] >= key (n if none)
__device__ __forceinline__ int32_t lower_bound(const int32_t *__restrict__ a, int32_t n, int32_t key) {
    int32_t lo = 0;
    while (n > 0) {
        int32_t half = n >> 1;
        if (a[lo + half] < key) {
            lo += half + 1;
            n -= half + 1;
        } else {
            n = half;
        }
    }
    return lo;
}

__device__ __forceinline__ bool contains(const int32_t *__restrict__ a, int32_t n, int32_t key) {
    int32_t i = lower_bound(a, n, key);
    return i < n && a[i] == key;
}

// restrict sorted a[0, n) to values in (lo, hi): returns begin, sets len
__device__ __forceinline__ int32_t restrict_range(const int32_t *a, int32_t n, int32_t lo, int32_t hi,
                                                  int32_t *len) {
    if (lo >= hi - 1 || n == 0) {
        *len = 0;
        return 0;
    }
    int32_t b = (lo < 0) ? 0 : lower_bound(a, n, lo + 1);
    int32_t e = (hi == INT_MAX) ? n : lower_bound(a, n, hi);
    *len = e > b ? e - b : 0;
    return b;
}

__device__ __forceinline__ unsigned long long choose(unsigned long long n, int j, bool *ovf) {
    if ((long long)j > (long long)n) return 0;
    unsigned long long r = 1;
    for (int t = 1; t <= j; t++) {
        unsigned long long f = n - (unsigned long long)j + (unsigned long long)t;
        unsigned long long q;
        if (__builtin_mul_overflow(r, f, &q)) {
            *ovf = true;
            return 0;
        }
        r = q / (unsigned long long)t;
    }
    return r;
}

struct Ctx {
    const KParams &P;
    Lds &L;
    int32_t *buf0;  // this wave's scratch (level 2 at offset 0)
    int lane;
    int vl0, vl1;   // varying levels of the current prefix batch (-1 none)

    __device__ Ctx(const KParams &p, Lds &l, int32_t *b, int ln) : P(p), L(l), buf0(b), lane(ln), vl0(-1), vl1(-1) {}

    __device__ __forceinline__ int32_t *setbuf(int level) const { return buf0 + (long long)(level - 2) * P.set_cap; }

    __device__ __forceinline__ int32_t val(int y, int l) const {
        if (y == vl0) return L.pv0[l];
        if (y == vl1) return L.pv1[l];
        return L.m[y];
    }
    __device__ __forceinline__ void row(int y, int l, const int32_t **p, int32_t *n) const {
        if (y == vl0) {
            *p = P.col + L.po0[l];
            *n = L.pl0[l];
        } else if (y == vl1) {
            *p = P.col + L.po1[l];
            *n = L.pl1[l];
        } else {
            *p = P.col + L.roff[y];
            *n = L.rlen[y];
        }
    }

    // anti-vertex check for candidate e at level x under prefix l (l < 0:
    // the fixed assignment only): the sets N(m(a)) \ m(xmask[a]) over the
    // anti-vertex's neighbour levels a must have an empty intersection.
    __device__ bool av_pass(const AVCheck &c, int x, int l, int32_t e) const {
        const int32_t *best = nullptr;
        int32_t best_n = INT_MAX;
        int best_a = -1;
        for (int a = 0; a < kMaxLevels; a++) {
            if (!(c.nbr >> a & 1u)) continue;
            int32_t v = (a == x) ? e : (l >= 0 ? val(a, l) : L.m[a]);
            const int32_t *p = P.col + P.rp[v];
            int32_t n = (int32_t)(P.rp[v + 1] - P.rp[v]);
            if (n < best_n) {
                best_n = n;
                best = p;
                best_a = a;
            }
        }
        for (int32_t i = 0; i < best_n; i++) {
            int32_t w = best[i];
            if (c.label >= 0 && (P.lab == nullptr || P.lab[w] != c.label)) continue;
            bool in_all = true;
            for (int a = 0; a < kMaxLevels && in_all; a++) {
                if (!(c.nbr >> a & 1u)) continue;
                // w must not be the image of a true neighbour of a
                uint32_t xm = c.xmask[a];
                for (int y = 0; y < kMaxLevels && in_all; y++) {
                    if (!(xm >> y & 1u)) continue;
                    int32_t vy = (y == x) ? e : (l >= 0 ? val(y, l) : L.m[y]);
                    if (vy == w) in_all = false;
                }
                if (!in_all || a == best_a) continue;
                int32_t v = (a == x) ? e : (l >= 0 ? val(a, l) : L.m[a]);
                if (!contains(P.col + P.rp[v], (int32_t)(P.rp[v + 1] - P.rp[v]), w)) in_all = false;
            }
            if (in_all) return false;
        }
        return true;
    }

    // direct test of candidate e of node N at level x (driver operand drv
    // already satisfied), prefix l or -1
    __device__ bool test_direct(const Node &N, int x, int l, int drv, int32_t e, const int32_t *bp,
                                int32_t bn) const {
        bool ok = true;
        if (N.base >= 0 && drv != kBaseOp) ok = contains(bp, bn, e);
        uint32_t ti = N.t_isect;
        while (ti && ok) {
            int y = __builtin_ctz(ti);
            ti &= ti - 1;
            if (y == drv) continue;
            const int32_t *p;
            int32_t n;
            if (l >= 0) row(y, l, &p, &n);
            else {
                p = P.col + L.roff[y];
                n = L.rlen[y];
            }
            ok = contains(p, n, e);
        }
        uint32_t td = N.t_diff;
        while (td && ok) {
            int y = __builtin_ctz(td);
            td &= td - 1;
            const int32_t *p;
            int32_t n;
            if (l >= 0) row(y, l, &p, &n);
            else {
                p = P.col + L.roff[y];
                n = L.rlen[y];
            }
            ok = !contains(p, n, e);
        }
        uint32_t ex = N.excl;
        while (ex && ok) {
            int y = __builtin_ctz(ex);
            ex &= ex - 1;
            ok = e != (l >= 0 ? val(y, l) : L.m[y]);
        }
        if (ok && N.label >= 0) ok = P.lab != nullptr && P.lab[e] == N.label;
        for (int i = 0; i < N.av_count && ok; i++) ok = av_pass(P.avs[N.av_begin + i], x, l, e);
        return ok;
    }

    // ---------------------------------------------------------------
    // Materialise the candidate set of enumeration node N (level x) for the
    // fixed assignment m[0..x): returns its length, elements in setbuf(x).
    __device__ int32_t materialise(const Node &N) {
        const int x = N.level;
        int32_t lo = -1, hi = INT_MAX;
        for (uint32_t s = N.lo; s; s &= s - 1) lo = max(lo, L.m[__builtin_ctz(s)]);
        for (uint32_t s = N.hi; s; s &= s - 1) hi = min(hi, L.m[__builtin_ctz(s)]);
        const int32_t *dptr = nullptr, *bp = nullptr;
        int32_t dlen = INT_MAX, bn = 0;
        int drv = -1;
        long long bytes = 0;
        if (N.base >= 0) {
            const int32_t *B = setbuf(N.base);
            int32_t n;
            int32_t b = restrict_range(B, L.set_len[N.base], lo, hi, &n);
            bp = B + b;
            bn = n;
            dptr = bp;
            dlen = n;
            drv = kBaseOp;
            bytes += n;
        }
        for (uint32_t s = N.t_isect; s; s &= s - 1) {
            int y = __builtin_ctz(s);
            int32_t n;
            int32_t b = restrict_range(P.col + L.roff[y], L.rlen[y], lo, hi, &n);
            bytes += n;
            if (n < dlen) {
                dlen = n;
                dptr = P.col + L.roff[y] + b;
                drv = y;
            }
        }
        if (P.run_flags & PG_RUN_COUNT_BYTES) {
            for (uint32_t s = N.t_diff; s; s &= s - 1) {
                int y = __builtin_ctz(s);
                int32_t n;
                restrict_range(P.col + L.roff[y], L.rlen[y], lo, hi, &n);
                bytes += n;
            }
            if (lane == 0) L.bytes += 4ull * (unsigned long long)bytes;
        }
        int32_t *out = setbuf(x);
        int32_t total = 0;
        if (dlen == INT_MAX) dlen = 0;
        for (int32_t base = 0; base < dlen; base += 64) {
            int32_t i = base + lane;
            bool ok = false;
            int32_t e = 0;
            if (i < dlen) {
                e = dptr[i];
                ok = test_direct(N, x, -1, drv, e, bp, bn);
            }
            unsigned long long bal = __ballot(ok);
            if (ok) {
                int32_t pos = total + (int32_t)__popcll(bal & ((1ull << lane) - 1ull));
                out[pos] = e;
            }
            total += (int32_t)__popcll(bal);
        }
        return total;
    }

    // ---------------------------------------------------------------
    // Flattened evaluation of count / emit node N (level x) over np
    // prefixes already loaded into the batch arrays (pv*, po*, pl*, pmode).
    __device__ void count_batch(const Node &N, int np) {
        const int x = N.level;
        const bool emit = N.kind == kEmit;
        // per-prefix setup: one lane per prefix
        if (lane < np && L.pmode[lane] >= 0) {
            const int l = lane;
            int32_t lo = -1, hi = INT_MAX;
            for (uint32_t s = N.lo; s; s &= s - 1) lo = max(lo, val(__builtin_ctz(s), l));
            for (uint32_t s = N.hi; s; s &= s - 1) hi = min(hi, val(__builtin_ctz(s), l));
            L.plo[l] = lo;
            L.phi[l] = hi;
            const int32_t *dptr = nullptr;
            int32_t dlen = INT_MAX;
            int drv = -1;
            long long bytes = 0;
            if (N.base >= 0) {
                const int32_t *B = setbuf(N.base);
                int32_t n;
                int32_t b = restrict_range(B, L.set_len[N.base], lo, hi, &n);
                L.bptr[l] = B + b;
                L.blen[l] = n;
                dptr = B + b;
                dlen = n;
                drv = kBaseOp;
                bytes += n;
            }
            for (uint32_t s = N.t_isect; s; s &= s - 1) {
                int y = __builtin_ctz(s);
                const int32_t *p;
                int32_t rn;
                row(y, l, &p, &rn);
                int32_t n;
                int32_t b = restrict_range(p, rn, lo, hi, &n);
                bytes += n;
                if (n < dlen) {
                    dlen = n;
                    dptr = p + b;
                    drv = y;
                }
            }
            if (dlen == INT_MAX) dlen = 0;
            int npos = (N.base >= 0 ? 1 : 0) + __builtin_popcount(N.t_isect);
            int ndiff = __builtin_popcount(N.t_diff);
            bool complement = false;
            if (!emit && npos == 1 && N.label < 0 && N.av_count == 0 && ndiff >= 1 && ndiff <= kSegPerPrefix &&
                !(P.run_flags & PG_RUN_NO_MODE_B)) {
                long long cost = 0;
                for (uint32_t s = N.t_diff; s; s &= s - 1) {
                    const int32_t *p;
                    int32_t rn, n;
                    row(__builtin_ctz(s), l, &p, &rn);
                    restrict_range(p, rn, lo, hi, &n);
                    cost += n;
                }
                complement = cost < dlen;
            }
            if ((P.run_flags & PG_RUN_COUNT_BYTES)) {
                for (uint32_t s = N.t_diff; s; s &= s - 1) {
                    const int32_t *p;
                    int32_t rn, n;
                    row(__builtin_ctz(s), l, &p, &rn);
                    restrict_range(p, rn, lo, hi, &n);
                    bytes += n;
                }
                atomicAdd(&L.bytes, 4ull * (unsigned long long)bytes);
            }
            L.pcnt[l] = 0;
            if (!complement) {
                L.pmode[l] = 0;
                L.pdrv[l] = drv;
                L.p1ptr[l] = dptr;
                L.p1len[l] = dlen;
                L.pconst[l] = 0;
            } else {
                // the single positive operand P1 (restricted) is the driver
                // found above; excluded images inside P1 \ (D...) are removed
                L.pmode[l] = 1;
                L.pdrv[l] = drv;
                L.p1ptr[l] = dptr;
                L.p1len[l] = dlen;
                int32_t c = dlen;
                for (uint32_t s = N.excl; s; s &= s - 1) {
                    int32_t v = val(__builtin_ctz(s), l);
                    if (v <= lo || v >= hi) continue;
                    if (!contains(dptr, dlen, v)) continue;
                    bool in_d = false;
                    for (uint32_t t = N.t_diff; t && !in_d; t &= t - 1) {
                        const int32_t *p;
                        int32_t rn;
                        row(__builtin_ctz(t), l, &p, &rn);
                        in_d = contains(p, rn, v);
                    }
                    if (!in_d) c--;
                }
                L.pconst[l] = c;
            }
        }
        wsync();
        // segments, laid out by lane 0 (at most kSeg)
        if (lane == 0) {
            int ns = 0;
            int32_t total = 0;
            for (int l = 0; l < np; l++) {
                if (L.pmode[l] < 0) continue;
                if (L.pmode[l] == 0) {
                    if (L.p1len[l] > 0) {
                        L.seg_start[ns] = total;
                        L.seg_prefix[ns] = (int16_t)l;
                        L.seg_op[ns] = -1;
                        L.seg_ptr[ns] = L.p1ptr[l];
                        total += L.p1len[l];
                        ns++;
                    }
                } else {
                    int k = 0;
                    for (uint32_t s = N.t_diff; s; s &= s - 1, k++) {
                        const int32_t *p;
                        int32_t rn, n;
                        row(__builtin_ctz(s), l, &p, &rn);
                        int32_t b = restrict_range(p, rn, L.plo[l], L.phi[l], &n);
                        if (n > 0) {
                            L.seg_start[ns] = total;
                            L.seg_prefix[ns] = (int16_t)l;
                            L.seg_op[ns] = (int16_t)k;
                            L.seg_ptr[ns] = p + b;
                            total += n;
                            ns++;
                        }
                    }
                }
            }
            L.seg_start[ns] = total;
            L.nseg = ns;
            L.total = total;
        }
        wsync();
        const int nseg = L.nseg;
        const int32_t total = L.total;
        for (int32_t tb = 0; tb < total; tb += 64) {
            int32_t t = tb + lane;
            bool ok = false;
            int l = 0;
            int32_t e = 0;
            if (t < total) {
                // segment holding flat index t
                int s_lo = 0, s_n = nseg;
                while (s_n > 1) {
                    int half = s_n >> 1;
                    if (L.seg_start[s_lo + half] <= t) {
                        s_lo += half;
                        s_n -= half;
                    } else {
                        s_n = half;
                    }
                }
                const int s = s_lo;
                l = L.seg_prefix[s];
                e = L.seg_ptr[s][t - L.seg_start[s]];
                if (L.pmode[l] == 0) {
                    ok = test_direct(N, x, l, L.pdrv[l], e, L.bptr[l], L.blen[l]);
                } else {
                    // complement term k: e in D_k, count it if e in P1 and in no earlier D
                    const int k = L.seg_op[s];
                    ok = contains(L.p1ptr[l], L.p1len[l], e);
                    int kk = 0;
                    for (uint32_t d = N.t_diff; d && ok && kk < k; d &= d - 1, kk++) {
                        const int32_t *p;
                        int32_t rn;
                        row(__builtin_ctz(d), l, &p, &rn);
                        ok = !contains(p, rn, e);
                    }
                }
            }
            if (emit) {
                unsigned long long bal = __ballot(ok);
                unsigned long long base = 0;
                if (lane == 0 && bal) base = atomicAdd(P.emit_ctr, (unsigned long long)__popcll(bal));
                base = __shfl(base, 0);
                if (ok) {
                    unsigned long long slot = base + (unsigned long long)__popcll(bal & ((1ull << lane) - 1ull));
                    if (slot < P.cap) {
                        int32_t *o = P.out + slot * (unsigned long long)N.k;
                        for (int y = 0; y < x; y++) o[N.pv[y]] = P.perm[val(y, l)];
                        o[N.pv[x]] = P.perm[e];
                    }
                }
            } else if (ok) {
                atomicAdd(&L.pcnt[l], 1u);
            }
        }
        wsync();
        if (!emit) {
            unsigned long long contrib = 0;
            bool ovf = false;
            if (lane < np && L.pmode[lane] >= 0) {
                unsigned long long c = L.pmode[lane] == 0 ? (unsigned long long)L.pcnt[lane]
                                                          : (unsigned long long)(L.pconst[lane] - (int32_t)L.pcnt[lane]);
                contrib = choose(c, N.group, &ovf);
                unsigned long long q;
                if (__builtin_mul_overflow(contrib, N.mult, &q)) ovf = true;
                contrib = q;
            }
            for (int off = 32; off > 0; off >>= 1) {
                unsigned long long o = __shfl_xor(contrib, off);
                unsigned long long s = contrib + o;
                if (s < contrib) ovf = true;
                contrib = s;
            }
            if (__ballot(ovf)) {
                if (lane == 0) atomicOr(P.flags, 1);
            }
            if (lane == 0) {
                unsigned long long a = L.acc[N.plan];
                unsigned long long s = a + contrib;
                if (s < a) atomicOr(P.flags, 1);
                L.acc[N.plan] = s;
                if (P.mode == kModeExists && s > 0) {
                    atomicOr(P.flags + 1, 1);
                    L.stop = 1;
                }
            }
        }
        wsync();
    }

    // run every count / emit child of node id `nid` over the candidates of
    // level x held in setbuf(x) (length len), in batches of 64 prefixes
    __device__ void counts_over_set(int nid, int x, int32_t len) {
        const Node &N = P.nodes[nid];
        const int cb = uni(N.child_begin), cc = uni(N.child_count);
        int first_enum = cc;
        for (int c = 0; c < cc; c++)
            if (P.nodes[cb + c].kind == kEnum) {
                first_enum = c;
                break;
            }
        if (first_enum == 0) return;
        const int32_t *S = setbuf(x);
        vl0 = x;
        vl1 = -1;
        for (int32_t s = 0; s < len; s += kP) {
            int np = min(kP, len - s);
            if (lane < np) {
                int32_t v = S[s + lane];
                L.pv0[lane] = v;
                L.po0[lane] = P.rp[v];
                L.pl0[lane] = (int32_t)(P.rp[v + 1] - P.rp[v]);
                L.pmode[lane] = 0;
            }
            wsync();
            for (int c = 0; c < first_enum; c++) {
                if (lane < np) L.pmode[lane] = 0;
                wsync();
                count_batch(P.nodes[cb + c], np);
            }
        }
        vl0 = -1;
    }

    __device__ void set_level(int x, int32_t v) {
        if (lane == 0) {
            L.m[x] = v;
            L.roff[x] = P.rp[v];
            L.rlen[x] = (int32_t)(P.rp[v + 1] - P.rp[v]);
        }
        wsync();
    }

    __device__ bool stopped() {
        if (P.mode != kModeExists) return false;
        if (lane == 0) {
            int f = __atomic_load_n(P.flags + 1, __ATOMIC_RELAXED);
            if (f) L.stop = 1;
        }
        wsync();
        return L.stop != 0;
    }

    // depth-first walk of the enumeration children of root node rid, with
    // levels 0..1 already assigned in m[]
    __device__ void dfs(int rid) {
        const Node &R = P.nodes[rid];
        const int cb = uni(R.child_begin), cc = uni(R.child_count);
        for (int c = 0; c < cc; c++) {
            const int e0 = cb + c;
            if (P.nodes[e0].kind != kEnum) continue;
            if (stopped()) return;
            int32_t len = materialise(P.nodes[e0]);
            if (lane == 0) L.set_len[2] = len;
            wsync();
            if (len == 0) continue;
            counts_over_set(e0, 2, len);
            // stack of enumeration frames
            int sp = 0;
            auto push = [&](int nid, int x) {
                if (lane == 0) {
                    L.st_node[sp] = nid;
                    L.st_idx[sp] = 0;
                    L.st_child[sp] = 0;
                }
                sp++;
                wsync();
                (void)x;
            };
            push(e0, 2);
            while (sp > 0) {
                if (stopped()) return;
                const int f = sp - 1;
                const int nid = uni(L.st_node[f]);
                const Node &N = P.nodes[nid];
                const int x = N.level;
                const int ncb = uni(N.child_begin), ncc = uni(N.child_count);
                int ch = uni(L.st_child[f]);
                int idx = uni(L.st_idx[f]);
                // advance to the next enumeration child
                while (ch < ncc && P.nodes[ncb + ch].kind != kEnum) ch++;
                if (ch >= ncc) {
                    idx++;
                    if (idx >= L.set_len[x]) {
                        sp--;
                        wsync();
                        continue;
                    }
                    if (lane == 0) {
                        L.st_idx[f] = idx;
                        L.st_child[f] = 0;
                    }
                    wsync();
                    continue;
                }
                if (lane == 0) L.st_child[f] = ch + 1;
                wsync();
                set_level(x, setbuf(x)[idx]);
                const int nid2 = ncb + ch;
                int32_t len2 = materialise(P.nodes[nid2]);
                if (lane == 0) L.set_len[x + 1] = len2;
                wsync();
                if (len2 == 0) continue;
                counts_over_set(nid2, x + 1, len2);
                bool has_enum = false;
                const Node &N2 = P.nodes[nid2];
                for (int c2 = 0; c2 < N2.child_count; c2++)
                    if (P.nodes[N2.child_begin + c2].kind == kEnum) has_enum = true;
                if (has_enum) push(nid2, x + 1);
            }
        }
    }
};

// Root checks (labels and anti-vertex checks on levels 0 / 1) for prefix l.
__device__ bool root_ok(Ctx &C, const Node &R, int l) {
    const KParams &P = C.P;
    if (R.label0 >= 0 && (P.lab == nullptr || P.lab[C.L.pv0[l]] != R.label0)) return false;
    if (R.kind == kRootEdge && R.label1 >= 0 && (P.lab == nullptr || P.lab[C.L.pv1[l]] != R.label1))
        return false;
    for (int i = 0; i < R.av_count; i++) {
        const AVCheck &c = P.avs[R.av_begin + i];
        // the deepest root level is the "candidate" of the check
        int x = R.level;
        if (!C.av_pass(c, x, l, C.val(x, l))) return false;
    }
    return true;
}

__global__ void __launch_bounds__(64) match_kernel(KParams P) {
    __shared__ Lds L;
    const int lane = threadIdx.x;
    int32_t *buf0 = P.scratch ? P.scratch + (long long)blockIdx.x * P.wave_stride : nullptr;
    Ctx C(P, L, buf0, lane);
    for (int i = lane; i < kMaxPlansPerLaunch; i += 64) L.acc[i] = 0;
    if (lane == 0) {
        L.stop = 0;
        L.bytes = 0;
    }
    wsync();
    const long long total_tasks = P.n_etasks + P.n_vtasks;
    for (;;) {
        if (C.stopped()) break;
        unsigned long long t0 = 0;
        if (lane == 0) t0 = atomicAdd(P.cursor, (unsigned long long)P.chunk);
        t0 = __shfl(t0, 0);
        if ((long long)t0 >= total_tasks) break;
        const long long c_end = min((long long)t0 + P.chunk, total_tasks);
        for (long long tb = (long long)t0; tb < c_end;) {
            // edge tasks occupy [0, n_etasks), vertex tasks the rest; a chunk
            // may straddle the boundary
            const bool edge_phase = tb < P.n_etasks;
            const long long t_end = edge_phase ? min(c_end, P.n_etasks) : c_end;
            const int np = (int)min((long long)kP, t_end - tb);
            for (int r = 0; r < P.n_roots; r++) {
                const int rid = uni(P.roots[r]);
                const Node &R = P.nodes[rid];
                if ((R.kind == kRootEdge) != edge_phase) continue;
                // load the prefix batch: tasks tb .. tb + np
                if (lane < np) {
                    long long t = tb + lane;
                    int32_t u, v = 0;
                    if (edge_phase) {
                        u = P.tsrc[t];
                        v = P.tdst[t];
                    } else {
                        u = P.n - 1 - (int32_t)(t - P.n_etasks);
                    }
                    L.tu[lane] = u;
                    L.tv[lane] = v;
                    L.pv0[lane] = u;
                    L.po0[lane] = P.rp[u];
                    L.pl0[lane] = (int32_t)(P.rp[u + 1] - P.rp[u]);
                    L.pv1[lane] = v;
                    if (edge_phase) {
                        L.po1[lane] = P.rp[v];
                        L.pl1[lane] = (int32_t)(P.rp[v + 1] - P.rp[v]);
                    }
                }
                wsync();
                C.vl0 = 0;
                C.vl1 = edge_phase ? 1 : -1;
                bool okr = false;
                if (lane < np) okr = root_ok(C, R, lane);
                const unsigned long long okmask = __ballot(okr);
                const int cb = uni(R.child_begin), cc = uni(R.child_count);
                for (int c = 0; c < cc; c++) {
                    const Node &N = P.nodes[cb + c];
                    if (N.kind == kEnum) break;
                    if (lane < np) L.pmode[lane] = okr ? 0 : -1;
                    wsync();
                    C.count_batch(N, np);
                }
                C.vl0 = -1;
                C.vl1 = -1;
                // enumeration children: one task at a time
                bool any_enum = false;
                for (int c = 0; c < cc; c++)
                    if (P.nodes[cb + c].kind == kEnum) any_enum = true;
                if (!any_enum || !edge_phase) continue;
                for (int l = 0; l < np; l++) {
                    if (!(okmask >> l & 1ull)) continue;
                    const int32_t u = L.tu[l], v = L.tv[l];
                    wsync();
                    C.set_level(0, u);
                    C.set_level(1, v);
                    C.dfs(rid);
                    if (C.stopped()) break;
                }
                wsync();
            }
            tb += np;
        }
    }
    wsync();
    if (lane < P.n_plans && L.acc[lane]) {
        unsigned long long old = atomicAdd(P.counts + lane, L.acc[lane]);
        if (old + L.acc[lane] < old) atomicOr(P.flags, 1);
    }
    if (lane == 0 && L.bytes) atomicAdd(P.bytes_ctr, L.bytes);
}

hipError_t launch_match(const KParams &P, int grid, hipStream_t s) {
    hipLaunchKernelGGL(match_kernel, dim3(grid), dim3(64), 0, s, P);
    return hipGetLastError();
}

}  // namespace pg
