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
//    flattened over up to 64 prefixes at once -- each lane sets up one
//    prefix and emits one or more segments of driver elements, a wave
//    prefix scan lays the segments end to end, and the lanes walk the
//    concatenation, so short rows do not leave lanes idle.  When the only
//    positive operand is long and the differences are short the count is
//    taken by complement, |P| - |P & (D1 u D2 ...)|, driven by the short
//    difference rows;
//  * counts are reduced per wave in 64-bit and added to the per-plan
//    counters once per wave at exit.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <mutex>

#include "engine.hpp"

namespace pg {

constexpr int kP = 64;        // prefixes per flattened batch (one per lane)
constexpr int kMaxDiffB = 3;  // complement counting handles up to this many difference rows
constexpr int kSeg = kP * kMaxDiffB;
constexpr int kBaseOp = 31;   // operand id of the base set

struct Lds {
    // the fixed assignment (levels matched so far) and their rows
    int32_t m[kMaxLevels];
    int32_t roff[kMaxLevels];     // row offsets in col (the graph has < 2^31 entries)
    int32_t rlen[kMaxLevels];
    int32_t rup[kMaxLevels];      // index of the first neighbour above the row's owner
    int32_t cur_idx[kMaxLevels];  // index of m[level] in that level's materialised set
    int32_t set_len[kMaxLevels];
    int32_t st_node[kMaxLevels];
    int32_t st_idx[kMaxLevels];
    int32_t st_child[kMaxLevels];
    // parent slots: root tasks (levels 0 and 1) or elements of a
    // materialised set (one level), with their rows
    int32_t tu[kP], tv[kP];
    int32_t tidx[kP];             // set parents: index of the parent in its set
    int32_t tro0[kP], tro1[kP];
    int32_t trl0[kP], trl1[kP], tru0[kP], tru1[kP];
    // level-2 candidates of a whole task batch, in the arena: task t owns
    // [tstart[t], tstart[t] + tcnt[t]); prefixes of a task batch record their task
    int32_t tstart[kP + 1];
    int32_t tcnt[kP];
    int32_t ptask[kP];            // parent slot of each prefix
    // prefix batch: value and row of the varying level
    int32_t pv0[kP];
    int32_t po0[kP];
    int32_t pl0[kP];
    int32_t pu0[kP];
    int32_t pidx[kP];             // index of the prefix in its own set (set batches)
    int32_t boff[kP];             // direct: the base range; complement: the single positive operand (enc)
    int32_t blen[kP];
    int32_t p1own[kP];            // complement: owner of that operand's row, -1 for a set
    int8_t pmode[kP];             // -1 skip, 0 direct, 1 complement
    int8_t pdrv[kP];
    uint32_t pcnt[kP];
    int32_t pconst[kP];
    int32_t seg_start[kSeg + 1];
    uint8_t seg_prefix[kSeg];
    int32_t seg_off[kSeg];        // segment start (enc)
    int32_t seg_own[kSeg];
    int32_t stop;
    unsigned long long bytes;
    unsigned long long t_start;
};

struct RowRef {
    const int32_t *p;
    int32_t n;
    int32_t up;     // index of the first element above `owner`
    int32_t owner;
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

// restrict a row to values in (lo, hi); a bound equal to the row's owner is
// the precomputed split between its lower and upper neighbours
__device__ __forceinline__ int32_t restrict_row(const RowRef &r, int32_t lo, int32_t hi, int32_t *len) {
    if (lo >= hi - 1 || r.n == 0) {
        *len = 0;
        return 0;
    }
    int32_t b, e;
    if (lo < 0) b = 0;
    else if (lo == r.owner) b = r.up;
    else if (lo > r.owner) b = r.up + lower_bound(r.p + r.up, r.n - r.up, lo + 1);
    else b = lower_bound(r.p, r.up, lo + 1);
    if (hi == INT_MAX) e = r.n;
    else if (hi == r.owner) e = r.up;
    else if (hi > r.owner) e = r.up + lower_bound(r.p + r.up, r.n - r.up, hi);
    else e = lower_bound(r.p, r.up, hi);
    *len = e > b ? e - b : 0;
    return b;
}

// C(n, j) exactly.  After step t, r = C(n - j + t, t) (each step's quotient
// is an integer: C(n-j+t, t) = C(n-j+t-1, t-1) * f / t).  The product r * f
// is formed in 64 bits when it fits and in 128 bits otherwise, so only a
// result of 2^64 or more sets the flag.
__device__ __forceinline__ unsigned long long choose(unsigned long long n, int j, bool *ovf) {
    if ((long long)j > (long long)n) return 0;
    if (j == 1) return n;
    unsigned long long r = 1;
    for (int t = 1; t <= j; t++) {
        const unsigned long long f = n - (unsigned long long)j + (unsigned long long)t;
        unsigned long long q;
        if (!__builtin_mul_overflow(r, f, &q)) {
            r = q / (unsigned long long)t;
        } else {
            const unsigned __int128 w = (unsigned __int128)r * f / (unsigned __int128)t;
            if (w >> 64) {
                *ovf = true;
                return 0;
            }
            r = (unsigned long long)w;
        }
    }
    return r;
}

// First task of claim i: claims hold 1 + floor(j / ramp) tasks (claim j),
// capped at `chunk`, so they grow linearly over the costliest tasks and
// stay at `chunk` after that.  With q = floor(i / ramp), r = i mod ramp the
// sum of the first i sizes is i + ramp q (q - 1) / 2 + r q while q < chunk.
__device__ __forceinline__ long long claim_start(long long i, int chunk, long long ramp) {
    const long long full = ramp * (long long)(chunk - 1);  // claims before the cap is reached
    if (i <= full) {
        const long long q = i / ramp, r = i - (i / ramp) * ramp;
        return i + ramp * (q * (q - 1) / 2) + r * q;
    }
    const long long q = chunk - 1;
    return full + ramp * (q * (q - 1) / 2) + (i - full) * (long long)chunk;
}

// exclusive prefix sum over the wave; *tot receives the wave total
__device__ __forceinline__ int wave_scan_excl(int x, int lane, int *tot) {
    int inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    *tot = __shfl(inc, 63, 64);
    return inc - x;
}

// In a pass over laid-out segments, lane t holds an element of segment s(t)
// with s non-decreasing in t, and segments of one prefix are adjacent, so
// the lanes' prefixes form runs.  Adds each run's number of lanes with ok
// to cnt[prefix]: one LDS atomic per run (distinct addresses) instead of
// one per passing lane on the same address.
template <class T>
__device__ __forceinline__ void add_runs(T *cnt, int l, bool valid, bool ok, int lane) {
    const int lp = __shfl_up(l, 1, 64);
    const bool head = valid && (lane == 0 || lp != l);
    const unsigned long long heads = __ballot(head), bal = __ballot(ok);
    if (head && bal) {
        const unsigned long long later = heads & ~((2ull << lane) - 1ull);  // 2 << 63 wraps to 0: no later head
        const unsigned long long upto = later ? (1ull << __builtin_ctzll(later)) - 1ull : ~0ull;
        const unsigned long long run = upto & ~((1ull << lane) - 1ull);
        const int c = __popcll(bal & run);
        if (c) atomicAdd(&cnt[l], (T)c);
    }
}

// membership of e in the row of r.owner: one load for a hub (dense bitmap),
// a binary search otherwise (the variant per degree bucket: hub_start is a
// launch knob)
__device__ __forceinline__ bool in_row(const KParams &P, const RowRef &r, int32_t e) {
    if (r.owner >= P.hub_start) {
        const uint32_t w = P.hub_bits[(long long)(r.owner - P.hub_start) * P.hub_words + (e >> 5)];
        return (w >> (e & 31)) & 1u;
    }
    return contains(r.p, r.n, e);
}

// membership in a sorted range whose elements are a row's (owner >= 0) or a
// materialised set's (owner < 0); the caller knows e lies in the range's bounds
__device__ __forceinline__ bool in_range(const KParams &P, const int32_t *p, int32_t n, int32_t owner, int32_t e) {
    if (owner >= P.hub_start) {
        const uint32_t w = P.hub_bits[(long long)(owner - P.hub_start) * P.hub_words + (e >> 5)];
        return (w >> (e & 31)) & 1u;
    }
    return contains(p, n, e);
}

// Products of independent groups, prefix p: the factor nodes' product so
// far (1 between products).  Only the variant that evaluates factor nodes
// references it, so only that kernel allocates it.
__shared__ unsigned long long fac_lds[kP];

// kFac: the trie may hold kFactor nodes
// kCnt: the build for long count launches (no existence stop, emission or
// domain marks), where those paths fold away at compile time
template <bool kAV, bool kFac, bool kCnt = false>
struct Ctx {
    const KParams P;  // by value: a reference to the kernel argument would force a private copy
    Lds &L;
    int32_t *buf0;  // this wave's scratch (level 2 at offset 0)
    int lane;
    int vl0;        // the level whose value varies per prefix (-1 none)
    int plev0;      // levels taken from each prefix's parent slot (-1 none):
    int plev1;      //   root tasks give levels 0 and 1, set parents one level
    int amode;      // 1: the vl0 level's set is the arena slice of the prefix's parent
    int anc_level;  // domains: the current root's anchor level (0 / 1, -1 none) and plan
    int anc_plan;
    int32_t *arena; // this wave's arena for batched expansions
    unsigned long long acc;  // lane p: running count of plan p

    __device__ Ctx(const KParams &p, Lds &l, int32_t *b, int ln)
        : P(p), L(l), buf0(b), lane(ln), vl0(-1), plev0(-1), plev1(-1), amode(0), anc_level(-1), anc_plan(0),
          arena(nullptr), acc(0) {}

    __device__ __forceinline__ int32_t *setbuf(int level) const { return buf0 + (long long)(level - 2) * P.set_cap; }

    // 32-bit addresses kept in LDS: rows as offsets into col, sets as the
    // complement of their offset in this wave's scratch
    __device__ __forceinline__ int32_t enc(const int32_t *p) const {
        return (p >= P.col && p < P.col + P.ncol) ? (int32_t)(p - P.col) : ~(int32_t)(p - buf0);
    }
    __device__ __forceinline__ const int32_t *dec(int32_t o) const {
        return o >= 0 ? P.col + o : buf0 + (long long)(~o);
    }

    __device__ __forceinline__ int32_t val(int y, int l) const {
        if (l < 0) return L.m[y];
        if (y == plev0) return L.tu[L.ptask[l]];
        if (y == plev1) return L.tv[L.ptask[l]];
        if (y == vl0) return L.pv0[l];
        return L.m[y];
    }

    __device__ __forceinline__ RowRef row(int y, int l) const {
        RowRef r;
        if (l >= 0 && (y == plev0 || y == plev1)) {
            const int t = L.ptask[l];
            const bool a = y == plev0;
            r.p = P.col + (a ? L.tro0[t] : L.tro1[t]);
            r.n = a ? L.trl0[t] : L.trl1[t];
            r.up = a ? L.tru0[t] : L.tru1[t];
            r.owner = a ? L.tu[t] : L.tv[t];
        } else if (l >= 0 && y == vl0) {
            r.p = P.col + L.po0[l];
            r.n = L.pl0[l];
            r.up = L.pu0[l];
            r.owner = L.pv0[l];
        } else {
            r.p = P.col + L.roff[y];
            r.n = L.rlen[y];
            r.up = L.rup[y];
            r.owner = L.m[y];
        }
        return r;
    }

    // Range of node N's base set for prefix l (-1: fixed assignment) within
    // (lo, hi).  The base set is the prefix's own set (level vl0, in the
    // arena slice of its parent when amode), the parent's set (level
    // plev0), or a fixed level's set; a bound equal to the element the
    // prefix holds in that set is its known index.
    __device__ __forceinline__ int32_t base_range(const Node &N, int l, int32_t lo, int32_t hi,
                                                  const int32_t **bp) const {
        const int bl = N.base;
        const int32_t *B;
        int32_t Bn, cur, ci;
        if (l >= 0 && bl == vl0) {
            B = amode ? arena + L.tstart[L.ptask[l]] : setbuf(bl);
            Bn = amode ? L.tcnt[L.ptask[l]] : L.set_len[bl];
            cur = L.pv0[l];
            ci = L.pidx[l];
        } else if (l >= 0 && bl == plev0) {
            B = setbuf(bl);
            Bn = L.set_len[bl];
            cur = L.tu[L.ptask[l]];
            ci = L.tidx[L.ptask[l]];
        } else {
            B = setbuf(bl);
            Bn = L.set_len[bl];
            cur = L.m[bl];
            ci = L.cur_idx[bl];
        }
        if (lo >= hi - 1) {
            *bp = B;
            return 0;
        }
        const int32_t b = lo < 0 ? 0 : (lo == cur ? ci + 1 : lower_bound(B, Bn, lo + 1));
        const int32_t e = hi == INT_MAX ? Bn : (hi == cur ? ci : lower_bound(B, Bn, hi));
        *bp = B + b;
        return e > b ? e - b : 0;
    }

    // The candidates of a level with a fixed label, drawn from y's row: in
    // the variant for labelled plans, the part of the row's label-sorted
    // copy that holds the label (id order, so ranges restrict as usual;
    // no owner, so no bitmap and no owner split)
    __device__ __forceinline__ RowRef drow(const Node &N, int y, int l) const {
        RowRef r = row(y, l);
        if constexpr (kFac) {
            if (N.label >= 0 && P.lab_off) {
                RowRef s;
                s.up = 0;
                s.owner = -1;
                s.p = r.p + P.lab_copy;
                s.n = 0;
                if (N.label < P.n_labels) {
                    const int32_t *o = P.lab_off + (long long)r.owner * (P.n_labels + 1);
                    const int32_t a = o[N.label];
                    s.p += a;
                    s.n = o[N.label + 1] - a;
                }
                return s;
            }
        }
        return r;
    }

    __device__ __forceinline__ RowRef vrow(int32_t v) const {
        RowRef r;
        long long o = P.rp[v];
        r.p = P.col + o;
        r.n = (int32_t)(P.rp[v + 1] - o);
        r.up = P.up[v];
        r.owner = v;
        return r;
    }

    __device__ bool av_pass(const AVCheck &c, int x, int l, int32_t e) const;

    // direct test of candidate e of node N at level x (driver operand drv
    // already satisfied), prefix l or -1 (fixed assignment, base range bp/bn)
    __device__ __forceinline__ bool test_direct(const Node &N, int x, int l, int drv, int32_t e, const int32_t *bp,
                                                int32_t bn) const {
        bool ok = true;
        if (N.base >= 0 && drv != kBaseOp) ok = contains(bp, bn, e);
        for (uint32_t ti = N.t_isect; ti && ok; ti &= ti - 1) {
            int y = __builtin_ctz(ti);
            if (y == drv) continue;
            ok = in_row(P, row(y, l), e);
        }
        for (uint32_t td = N.t_diff; td && ok; td &= td - 1) ok = !in_row(P, row(__builtin_ctz(td), l), e);
        for (uint32_t ex = N.excl; ex && ok; ex &= ex - 1) ok = e != val(__builtin_ctz(ex), l);
        if (ok && N.label >= 0) ok = P.lab != nullptr && P.lab[e] == N.label;
        if constexpr (kAV)
            for (int i = 0; i < N.av_count && ok; i++) ok = av_pass(P.avs[N.av_begin + i], x, l, e);
        return ok;
    }

    // ---------------------------------------------------------------
    // Materialise the candidate set of enumeration node N (level x) for the
    // fixed assignment m[0..x): returns its length, elements in setbuf(x).
    __device__ __forceinline__ int32_t materialise(const Node &N) {
        const int x = N.level;
        int32_t lo = -1, hi = INT_MAX;
        for (uint32_t s = N.lo; s; s &= s - 1) lo = max(lo, L.m[__builtin_ctz(s)]);
        for (uint32_t s = N.hi; s; s &= s - 1) hi = min(hi, L.m[__builtin_ctz(s)]);
        const int32_t *dptr = nullptr, *bp = nullptr;
        int32_t dlen = INT_MAX, bn = 0;
        int drv = -1;
        long long bytes = 0;
        if (N.base >= 0) {
            bn = base_range(N, -1, lo, hi, &bp);
            dptr = bp;
            dlen = bn;
            drv = kBaseOp;
            bytes += bn;
        }
        for (uint32_t s = N.t_isect; s; s &= s - 1) {
            int y = __builtin_ctz(s);
            RowRef r = drow(N, y, -1);
            int32_t n;
            int32_t b = restrict_row(r, lo, hi, &n);
            bytes += n;
            if (n < dlen) {
                dlen = n;
                dptr = r.p + b;
                drv = y;
            }
        }
        if (P.run_flags & PG_RUN_COUNT_BYTES) {
            for (uint32_t s = N.t_diff; s; s &= s - 1) {
                int32_t n;
                restrict_row(row(__builtin_ctz(s), -1), lo, hi, &n);
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
    // prefixes already loaded into the batch arrays (pv0/po0/pl0/pu0 and
    // pidx for the varying level vl0, ptask for parent-slot levels, pmode).
    __device__ __forceinline__ void count_batch(const Node &N, int np) {
        const int x = N.level;
        const bool emit = !kCnt && N.kind == kEmit;
        int my_nseg = 0, my_tot = 0;
        const int32_t *sp0 = nullptr, *sp1 = nullptr, *sp2 = nullptr;
        int32_t sl0 = 0, sl1 = 0, sl2 = 0;
        int so0 = -1, so1 = -1, so2 = -1;  // segment owners (row owner, -1 = a set)
        // domains: a prefix whose anchor image is already in the domain
        // adds nothing
        if (!kCnt && P.mark && N.anchor_level >= 0 && lane < np && L.pmode[lane] >= 0) {
            const int32_t v = val(N.anchor_level, lane);
            const uint32_t w =
                __atomic_load_n(P.mark + (long long)N.plan * P.mark_words + (v >> 5), __ATOMIC_RELAXED);
            if ((w >> (v & 31)) & 1u) L.pmode[lane] = -1;
        }
        // products: a prefix with an empty factor set adds nothing
        if constexpr (kFac)
            if (lane < np && fac_lds[lane] == 0) L.pmode[lane] = -1;
        if (lane < np && L.pmode[lane] >= 0) {
            const int l = lane;
            int32_t lo = -1, hi = INT_MAX;
            for (uint32_t s = N.lo; s; s &= s - 1) lo = max(lo, val(__builtin_ctz(s), l));
            for (uint32_t s = N.hi; s; s &= s - 1) hi = min(hi, val(__builtin_ctz(s), l));
            const int32_t *dptr = nullptr;
            int32_t dlen = INT_MAX;
            int drv = -1, downer = -1;
            long long bytes = 0;
            if (N.base >= 0) {
                const int32_t *bp;
                const int32_t n = base_range(N, l, lo, hi, &bp);
                L.boff[l] = enc(bp);
                L.blen[l] = n;
                dptr = bp;
                dlen = n;
                drv = kBaseOp;
                bytes += n;
            }
            for (uint32_t s = N.t_isect; s; s &= s - 1) {
                const int y = __builtin_ctz(s);
                RowRef r = drow(N, y, l);
                int32_t n;
                int32_t b = restrict_row(r, lo, hi, &n);
                bytes += n;
                if (n < dlen) {
                    dlen = n;
                    dptr = r.p + b;
                    drv = y;
                    downer = r.owner;
                }
            }
            if (dlen == INT_MAX) dlen = 0;
            const int npos = (N.base >= 0 ? 1 : 0) + __builtin_popcount(N.t_isect);
            const int ndiff = __builtin_popcount(N.t_diff);
            bool complement = false;
            // with one positive operand and no difference rows the count is
            // |P| less the excluded images in it (no walk); in labelled plans
            // a label part as that operand already holds only candidates
            // with the label
            const bool lab_part = kFac && N.label >= 0 && P.lab_off && drv != kBaseOp;
            if (!emit && npos == 1 && (N.label < 0 || lab_part) && N.av_count == 0 && ndiff <= kMaxDiffB &&
                !(P.run_flags & PG_RUN_NO_MODE_B) && dlen > 0) {
                // restricted difference rows become the complement's segments
                int k = 0;
                for (uint32_t s = N.t_diff; s; s &= s - 1, k++) {
                    RowRef r = row(__builtin_ctz(s), l);
                    int32_t n;
                    int32_t b = restrict_row(r, lo, hi, &n);
                    if (k == 0) {
                        sp0 = r.p + b;
                        sl0 = n;
                        so0 = r.owner;
                    } else if (k == 1) {
                        sp1 = r.p + b;
                        sl1 = n;
                        so1 = r.owner;
                    } else {
                        sp2 = r.p + b;
                        sl2 = n;
                        so2 = r.owner;
                    }
                }
                // an element of D_k is also probed against D_0..D_k-1: longest
                // rows first keeps those extra probes on the short rows
                if (ndiff > 1) {
                    auto order = [](const int32_t *&pa, int32_t &la, int &oa, const int32_t *&pb, int32_t &lb,
                                    int &ob) {
                        if (la < lb) {
                            const int32_t *tp = pa;
                            pa = pb;
                            pb = tp;
                            const int32_t tl = la;
                            la = lb;
                            lb = tl;
                            const int to = oa;
                            oa = ob;
                            ob = to;
                        }
                    };
                    order(sp0, sl0, so0, sp1, sl1, so1);
                    if (ndiff > 2) {
                        order(sp1, sl1, so1, sp2, sl2, so2);
                        order(sp0, sl0, so0, sp1, sl1, so1);
                    }
                }
                // direct: every element of P is probed against each D; by
                // complement: an element of D_k against P and D_0..D_k-1
                complement = ndiff == 0 || (long long)sl0 + 2ll * sl1 + 3ll * sl2 < (long long)ndiff * dlen;
            }
            if (P.run_flags & PG_RUN_COUNT_BYTES) {
                // a count taken from a length (one operand, no difference
                // rows) executes no set operation: it moves no merge bytes
                if (complement && ndiff == 0) bytes = 0;
                for (uint32_t s = N.t_diff; s; s &= s - 1) {
                    int32_t n;
                    restrict_row(row(__builtin_ctz(s), l), lo, hi, &n);
                    bytes += n;
                }
                atomicAdd(&L.bytes, 4ull * (unsigned long long)bytes);
            }
            L.pcnt[l] = 0;
            L.pdrv[l] = (int8_t)drv;
            L.p1own[l] = downer;
            if (complement) {
                // the single positive operand is the base or a row: keep it in
                // the base slots
                L.boff[l] = enc(dptr);
                L.blen[l] = dlen;
            }
            if (!complement) {
                L.pmode[l] = 0;
                L.pconst[l] = 0;
                sp0 = dptr;
                sl0 = dlen;
                so0 = downer;
                my_nseg = dlen > 0 ? 1 : 0;
                my_tot = dlen;
            } else {
                // excluded images inside P1 \ (D...) were counted in |P1|
                L.pmode[l] = 1;
                int32_t c = dlen;
                for (uint32_t s = N.excl; s; s &= s - 1) {
                    const int y = __builtin_ctz(s);
                    int32_t v = val(y, l);
                    if (v <= lo || v >= hi) continue;
                    // the pattern puts this image in the row and outside every difference row
                    if ((N.excl_in >> y & 1u) && drv != kBaseOp) {
                        c--;
                        continue;
                    }
                    if (!in_range(P, dptr, dlen, downer, v)) continue;
                    bool in_d = false;
                    for (uint32_t t = N.t_diff; t && !in_d; t &= t - 1) in_d = in_row(P, row(__builtin_ctz(t), l), v);
                    if (!in_d) c--;
                }
                L.pconst[l] = c;
                // pack the non-empty difference segments, keeping their order
                int k = 0;
                const int32_t *q0 = nullptr, *q1 = nullptr, *q2 = nullptr;
                int32_t m0 = 0, m1 = 0, m2 = 0;
                int o0 = -1, o1 = -1, o2 = -1;
                if (sl0 > 0) {
                    q0 = sp0;
                    m0 = sl0;
                    o0 = so0;
                    k++;
                }
                if (ndiff > 1 && sl1 > 0) {
                    if (k == 0) {
                        q0 = sp1;
                        m0 = sl1;
                        o0 = so1;
                    } else {
                        q1 = sp1;
                        m1 = sl1;
                        o1 = so1;
                    }
                    k++;
                }
                if (ndiff > 2 && sl2 > 0) {
                    if (k == 0) {
                        q0 = sp2;
                        m0 = sl2;
                        o0 = so2;
                    } else if (k == 1) {
                        q1 = sp2;
                        m1 = sl2;
                        o1 = so2;
                    } else {
                        q2 = sp2;
                        m2 = sl2;
                        o2 = so2;
                    }
                    k++;
                }
                sp0 = q0;
                sl0 = m0;
                so0 = o0;
                sp1 = q1;
                sl1 = m1;
                so1 = o1;
                sp2 = q2;
                sl2 = m2;
                so2 = o2;
                my_nseg = k;
                my_tot = m0 + m1 + m2;
            }
        }
        // lay the segments end to end with wave scans (no serial pass)
        int nseg = 0, total = 0;
        const int sbase = wave_scan_excl(my_nseg, lane, &nseg);
        int obase = wave_scan_excl(my_tot, lane, &total);
        if (my_nseg > 0) {
            L.seg_start[sbase] = obase;
            L.seg_prefix[sbase] = (uint8_t)lane;
            L.seg_own[sbase] = so0;
            L.seg_off[sbase] = enc(sp0);
            obase += sl0;
        }
        if (my_nseg > 1) {
            L.seg_start[sbase + 1] = obase;
            L.seg_prefix[sbase + 1] = (uint8_t)lane;
            L.seg_own[sbase + 1] = so1;
            L.seg_off[sbase + 1] = enc(sp1);
            obase += sl1;
        }
        if (my_nseg > 2) {
            L.seg_start[sbase + 2] = obase;
            L.seg_prefix[sbase + 2] = (uint8_t)lane;
            L.seg_own[sbase + 2] = so2;
            L.seg_off[sbase + 2] = enc(sp2);
        }
        if (lane == 0) L.seg_start[nseg] = total;
        wsync();
        // lane t walks elements t, t + 64, ... of the concatenated segments;
        // the element of the next pass is loaded before this pass's probes,
        // so its load overlaps them
        int s = 0;  // this lane's segment, advanced monotonically
        int32_t e_next = 0;
        if (lane < total) {
            // first visit: binary search for the segment holding the lane
            int s_lo = 0, s_n = nseg;
            while (s_n > 1) {
                const int half = s_n >> 1;
                if (L.seg_start[s_lo + half] <= lane) {
                    s_lo += half;
                    s_n -= half;
                } else {
                    s_n = half;
                }
            }
            s = s_lo;
            e_next = dec(L.seg_off[s])[lane - L.seg_start[s]];
        }
        for (int32_t tb = 0; tb < total; tb += 64) {
            const int32_t t = tb + lane;
            bool ok = false;
            int l = 0;
            const int32_t e = e_next;
            const int s_cur = s;
            if (t + 64 < total) {
                while (L.seg_start[s + 1] <= t + 64) s++;
                e_next = dec(L.seg_off[s])[t + 64 - L.seg_start[s]];
            }
            if (t < total) {
                const int s = s_cur;
                l = L.seg_prefix[s];
                if (L.pmode[l] == 0) {
                    ok = test_direct(N, x, l, L.pdrv[l], e, dec(L.boff[l]), L.blen[l]);
                } else {
                    // complement term: e in D_k counts if e in P1 and in no
                    // earlier D of this prefix (the segments just before)
                    ok = in_range(P, dec(L.boff[l]), L.blen[l], L.p1own[l], e);
                    for (int s2 = s - 1; ok && s2 >= 0 && L.seg_prefix[s2] == l; s2--)
                        ok = !in_range(P, dec(L.seg_off[s2]), L.seg_start[s2 + 1] - L.seg_start[s2], L.seg_own[s2], e);
                }
            }
            if (emit) {
                const unsigned long long bal = __ballot(ok);
                unsigned long long base = 0;
                if (lane == 0 && bal) base = atomicAdd(P.emit_ctr, (unsigned long long)__popcll(bal));
                base = __shfl(base, 0);
                if (ok) {
                    const unsigned long long slot = base + (unsigned long long)__popcll(bal & ((1ull << lane) - 1ull));
                    if (slot < P.cap) {
                        int32_t *o = P.out + slot * (unsigned long long)N.k;
                        for (int y = 0; y < x; y++) o[N.pv[y]] = P.perm[val(y, l)];
                        o[N.pv[x]] = P.perm[e];
                    }
                }
            } else {
                add_runs(L.pcnt, l, t < total, ok, lane);
            }
        }
        wsync();
        if (!emit) {
            unsigned long long contrib = 0;
            bool ovf = false;
            // a factor node only multiplies into its prefix's product; the
            // count node after it closes the product
            const bool factor = kFac && N.kind == kFactor;
            if (lane < np && L.pmode[lane] >= 0) {
                const unsigned long long c = L.pmode[lane] == 0
                                                 ? (unsigned long long)L.pcnt[lane]
                                                 : (unsigned long long)(L.pconst[lane] - (int32_t)L.pcnt[lane]);
                contrib = choose(c, N.group, &ovf);
                if constexpr (kFac) {
                    unsigned long long q;
                    if (__builtin_mul_overflow(contrib, fac_lds[lane], &q)) ovf = true;
                    contrib = q;
                }
                if (!factor) {
                    // domains: this prefix has a match, so its anchor's image
                    // is in the anchor's domain
                    if (!kCnt && P.mark && contrib && N.anchor_level >= 0) {
                        const int32_t v = val(N.anchor_level, lane);
                        atomicOr(P.mark + (long long)N.plan * P.mark_words + (v >> 5), 1u << (v & 31));
                    }
                    unsigned long long q;
                    if (__builtin_mul_overflow(contrib, N.mult, &q)) ovf = true;
                    contrib = q;
                }
            }
            if constexpr (kFac) fac_lds[lane] = factor ? contrib : 1ull;
            if (factor) {
                if (__ballot(ovf) && lane == 0) atomicOr(P.flags, 1);
            } else {
                for (int off = 32; off > 0; off >>= 1) {
                    const unsigned long long o = __shfl_xor(contrib, off);
                    const unsigned long long s = contrib + o;
                    if (s < contrib) ovf = true;
                    contrib = s;
                }
                if (__ballot(ovf) && lane == 0) atomicOr(P.flags, 1);
                // every lane holds the batch total; lane N.plan keeps that plan's sum
                if (lane == N.plan) {
                    const unsigned long long s = acc + contrib;
                    if (s < acc) atomicOr(P.flags, 1);
                    acc = s;
                    if (!kCnt && P.mode == kModeExists && s > 0) {
                        atomicOr(P.flags + 1, 1);
                        L.stop = 1;
                    }
                }
            }
        }
        wsync();
    }

    // run every count / emit child of node `nid` over the candidates of
    // level x held in setbuf(x) at positions [begin, end), in batches of 64
    // prefixes
    __device__ __forceinline__ void counts_over_set(int nid, int x, int32_t begin, int32_t end) {
        const Node &N = P.nodes[nid];
        const int cb = uni(N.child_begin), cc = uni(N.child_count);
        int first_enum = cc;
        for (int c = 0; c < cc; c++)
            if (P.nodes[cb + c].kind == kEnum) {
                first_enum = c;
                break;
            }
        if (first_enum == 0) return;
        const int sp0 = plev0, sp1 = plev1;
        if (N.flags & kIndepCounts) {
            // one parent (the fixed assignment): its candidates each add the same term
            plev0 = plev1 = -1;
            indep_counts(N, -1, end - begin, lane == 0);
            plev0 = sp0;
            plev1 = sp1;
            return;
        }
        const int32_t *S = setbuf(x);
        plev0 = plev1 = -1;
        amode = 0;
        vl0 = x;
        for (int32_t s = begin; s < end; s += kP) {
            if (stopped()) break;
            const int np = min(kP, end - s);
            if (lane < np) {
                const int32_t v = S[s + lane];
                const long long o = P.rp[v];
                L.pv0[lane] = v;
                L.po0[lane] = (int32_t)o;
                L.pl0[lane] = (int32_t)(P.rp[v + 1] - o);
                L.pu0[lane] = P.up[v];
                L.pidx[lane] = s + lane;
            }
            for (int c = 0; c < first_enum; c++) {
                if (lane < np) L.pmode[lane] = 0;
                wsync();
                count_batch(P.nodes[cb + c], np);
            }
        }
        vl0 = -1;
        plev0 = sp0;
        plev1 = sp1;
    }

    __device__ __forceinline__ void set_level(int x, int32_t v, int32_t idx) {
        if (lane == 0) {
            const long long o = P.rp[v];
            L.m[x] = v;
            L.roff[x] = (int32_t)o;
            L.rlen[x] = (int32_t)(P.rp[v + 1] - o);
            L.rup[x] = P.up[v];
            L.cur_idx[x] = idx;
        }
        wsync();
    }

    // early exit: another wavefront found a match (existence) or the
    // launch's time limit has passed (then every wavefront is told to stop)
    __device__ __forceinline__ bool stopped() {
        if ((kCnt || P.mode != kModeExists) && !P.time_budget) return false;
        if (lane == 0) {
            if (__atomic_load_n(P.flags + 1, __ATOMIC_RELAXED)) {
                L.stop = 1;
            } else if (P.time_budget && (long long)(wall_clock64() - L.t_start) > P.time_budget) {
                L.stop = 1;
                atomicOr(P.flags + 2, 1);
                atomicOr(P.flags + 1, 1);
            }
        }
        wsync();
        return L.stop != 0;
    }

    __device__ __forceinline__ bool has_enum_child(const Node &N) const {
        for (int c = 0; c < N.child_count; c++)
            if (P.nodes[N.child_begin + c].kind == kEnum) return true;
        return false;
    }

    __device__ __forceinline__ bool is_leaf_enum(const Node &E) const {
        return E.kind == kEnum && !has_enum_child(E) && !(P.run_flags & PG_RUN_NO_TASK_BATCH);
    }

    // Phase 2 of a batched expansion: the count / emit children of node nid
    // over the candidates in [rb, re) of every parent's slice of the arena
    // (lane t gives parent t's range), flattened 64 (parent, candidate)
    // prefixes at a time.  A flat index belongs to the last parent whose
    // range starts at or before it (a search over the lanes' starts).
    __device__ __forceinline__ void expand_over(int nid, int x, int np, int32_t rb, int32_t re) {
        const int32_t len = lane < np && re > rb ? re - rb : 0;
        if (P.nodes[nid].flags & kIndepCounts) {
            // every candidate adds the same term: no per-candidate pass
            indep_counts(P.nodes[nid], lane, len, lane < np);
            return;
        }
        int ntot = 0;
        const int32_t ms = wave_scan_excl(len, lane, &ntot);
        const int32_t ms_key = lane < np ? ms : INT_MAX;
        vl0 = x;
        amode = 1;
        const Node &N = P.nodes[nid];
        const int cb = uni(N.child_begin), cc = uni(N.child_count);
        for (int32_t s0 = 0; s0 < ntot; s0 += kP) {
            const int np2 = min(kP, ntot - s0);
            const int32_t idx = s0 + lane;
            int t = 0;
            for (int step = 32; step > 0; step >>= 1)
                if (__shfl(ms_key, t + step) <= idx) t += step;
            const int32_t tb = __shfl(rb, t), tm = __shfl(ms, t);
            if (lane < np2) {
                const int32_t k = tb + (idx - tm);
                const int32_t v = arena[L.tstart[t] + k];
                const long long o = P.rp[v];
                L.ptask[lane] = t;
                L.pidx[lane] = k;
                L.pv0[lane] = v;
                L.po0[lane] = (int32_t)o;
                L.pl0[lane] = (int32_t)(P.rp[v + 1] - o);
                L.pu0[lane] = P.up[v];
            }
            for (int c = 0; c < cc; c++) {
                if (lane < np2) L.pmode[lane] = 0;
                wsync();
                count_batch(P.nodes[cb + c], np2);
            }
        }
        amode = 0;
        vl0 = -1;
        // the next round's setup reads parent slots through ptask
        if (lane < np) L.ptask[lane] = lane;
        wsync();
    }

    // A share group's count member M: lane t's parent has n candidates in
    // M's range (mine: the lane holds a parent), so it adds
    // C(n, group) * mult to M's plan.
    __device__ __forceinline__ void count_member(const Node &M, int32_t n, bool mine) {
        unsigned long long contrib = 0;
        bool ovf = false;
        if (mine && n > 0) {
            contrib = choose((unsigned long long)n, M.group, &ovf);
            unsigned long long q;
            if (__builtin_mul_overflow(contrib, M.mult, &q)) ovf = true;
            contrib = q;
        }
        add_to_plan(M.plan, contrib, ovf);
    }

    // Count children of an enumeration node flagged kIndepCounts: every
    // candidate of the node adds the same term, C(|row| - excluded, group)
    // * mult, the node's own image being one of the excluded ones (the
    // pattern puts it in the row).  Lane l (mine) holds a parent with n
    // candidates; l is also the prefix slot val() and row() read.
    __device__ __forceinline__ void indep_counts(const Node &E, int l, int32_t n, bool mine) {
        const int x = E.level;
        const int cb = uni(E.child_begin), cc = uni(E.child_count);
        for (int c = 0; c < cc; c++) {
            const Node &N = P.nodes[cb + c];
            unsigned long long contrib = 0;
            bool ovf = false;
            if (mine && n > 0) {
                const RowRef r = row(__builtin_ctz(N.t_isect), l);
                int32_t k = r.n;
                for (uint32_t s = N.excl; s; s &= s - 1) {
                    const int y = __builtin_ctz(s);
                    if (y == x || (N.excl_in >> y & 1u)) k--;
                    else if (in_row(P, r, val(y, l))) k--;
                }
                unsigned long long q;
                contrib = choose((unsigned long long)max(k, 0), N.group, &ovf);
                if (__builtin_mul_overflow(contrib, N.mult, &q)) ovf = true;
                if (__builtin_mul_overflow(q, (unsigned long long)n, &contrib)) ovf = true;
            }
            add_to_plan(N.plan, contrib, ovf);
        }
    }

    // add every lane's contrib to plan `plan` (wave reduction, overflow flag,
    // existence stop); the sum lands in lane plan's accumulator
    __device__ __forceinline__ void add_to_plan(int plan, unsigned long long contrib, bool ovf) {
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(contrib, off);
            const unsigned long long sum = contrib + o;
            if (sum < contrib) ovf = true;
            contrib = sum;
        }
        if (__ballot(ovf) && lane == 0) atomicOr(P.flags, 1);
        if (lane == plan) {
            const unsigned long long sum = acc + contrib;
            if (sum < acc) atomicOr(P.flags, 1);
            acc = sum;
            if (!kCnt && P.mode == kModeExists && sum > 0) {
                atomicOr(P.flags + 1, 1);
                L.stop = 1;
            }
        }
    }

    // the positions [*rb, *re) of the sorted set S (n elements) that lie in
    // node M's id range for prefix l (-1: the fixed assignment)
    __device__ __forceinline__ void member_range(const Node &M, int l, const int32_t *S, int32_t n, int32_t *rb,
                                                 int32_t *re) const {
        int32_t lo = -1, hi = INT_MAX;
        for (uint32_t s = M.lo; s; s &= s - 1) lo = max(lo, val(__builtin_ctz(s), l));
        for (uint32_t s = M.hi; s; s &= s - 1) hi = min(hi, val(__builtin_ctz(s), l));
        *rb = lo < 0 ? 0 : lower_bound(S, n, lo + 1);
        *re = hi == INT_MAX ? n : lower_bound(S, n, hi);
        if (*re < *rb) *re = *rb;
    }

    // Enumeration node E whose children are all count / emit nodes, for a
    // batch of np parents at once (slots 0..np-1: root tasks with plev0/1 =
    // levels 0/1, or elements of a materialised set with plev0 = its
    // level): one flattened pass materialises every parent's candidates
    // into the arena (parent order, each slice sorted), then the count
    // children run flattened over all (parent, candidate) prefixes.
    // Parents whose driver does not fit the arena take the one-parent path.
    __device__ __forceinline__ void leaf_batch(int eid, int np, unsigned long long okmask) {
        const Node &E = P.nodes[eid];
        const int x = E.level;
        // a share group's leader lists its members (0 for any other node)
        const int mcount = uni(E.list_count), mbegin = uni(E.list_begin);
        if (lane < np) L.ptask[lane] = lane;
        wsync();
        vl0 = -1;
        amode = 0;
        int32_t dlen = 0;
        const int32_t *dptr = nullptr;
        const int32_t *my_bp = nullptr;  // this parent's base range (kept across rounds)
        int32_t my_bn = 0;
        int drv = -1;
        bool ok = lane < np && (okmask >> lane & 1ull);
        // domains: a parent whose anchor image is already in the domain adds nothing
        if (!kCnt && ok && anc_level >= 0) {
            const int32_t v = val(anc_level, lane);
            const uint32_t w =
                __atomic_load_n(P.mark + (long long)anc_plan * P.mark_words + (v >> 5), __ATOMIC_RELAXED);
            ok = !((w >> (v & 31)) & 1u);
        }
        if (ok) {
            int32_t lo = -1, hi = INT_MAX;
            for (uint32_t s = E.lo; s; s &= s - 1) lo = max(lo, val(__builtin_ctz(s), lane));
            for (uint32_t s = E.hi; s; s &= s - 1) hi = min(hi, val(__builtin_ctz(s), lane));
            dlen = INT_MAX;
            long long bytes = 0;
            if (E.base >= 0) {
                my_bn = base_range(E, lane, lo, hi, &my_bp);
                dlen = my_bn;
                dptr = my_bp;
                drv = kBaseOp;
                bytes += my_bn;
            }
            for (uint32_t s = E.t_isect; s; s &= s - 1) {
                const int y = __builtin_ctz(s);
                RowRef r = drow(E, y, lane);
                int32_t n;
                const int32_t b = restrict_row(r, lo, hi, &n);
                bytes += n;
                if (n < dlen) {
                    dlen = n;
                    dptr = r.p + b;
                    drv = y;
                }
            }
            if (dlen == INT_MAX) dlen = 0;
            if (P.run_flags & PG_RUN_COUNT_BYTES) {
                for (uint32_t s = E.t_diff; s; s &= s - 1) {
                    int32_t n;
                    restrict_row(row(__builtin_ctz(s), lane), lo, hi, &n);
                    bytes += n;
                }
                atomicAdd(&L.bytes, 4ull * (unsigned long long)bytes);
            }
        }
        // parents whose own driver exceeds the arena go one at a time below;
        // the rest run in rounds of as many parents as fit the arena.  With
        // a batching limit, a batch whose parents average more candidates
        // than the limit goes one parent at a time as a whole: long lists
        // already fill the wave, and the flattened pass would only add work.
        bool big = ok && dlen > P.arena_cap;
        if (P.batch_max_avg > 0) {
            int tot = 0;
            wave_scan_excl(ok && !big ? dlen : 0, lane, &tot);
            const int nsmall = __popcll(__ballot(ok && !big));
            if ((long long)tot > (long long)P.batch_max_avg * nsmall) big = ok;
        }
        const unsigned long long bigmask = __ballot(big);
        unsigned long long remaining = __ballot(ok && !big);
        while (remaining) {
            if (stopped()) break;
            // parent slots as the materialisation pass reads them (a previous
            // round's count phase reused these arrays)
            L.pdrv[lane] = (int8_t)drv;
            L.boff[lane] = my_bp ? enc(my_bp) : 0;
            L.blen[lane] = my_bn;
            const bool mine = (remaining >> lane) & 1ull;
            int tot = 0;
            const int off = wave_scan_excl(mine ? dlen : 0, lane, &tot);
            const bool sel = mine && (long long)off + dlen <= P.arena_cap;
            const unsigned long long selmask = __ballot(sel);
            remaining &= ~selmask;
            const int32_t flen = sel ? dlen : 0;
            int total = 0, nseg = 0;
            const int obase = wave_scan_excl(flen, lane, &total);
            const int sidx = wave_scan_excl(flen > 0 ? 1 : 0, lane, &nseg);
            wsync();
            if (flen > 0) {
                L.seg_start[sidx] = obase;
                L.seg_prefix[sidx] = (uint8_t)lane;
                L.seg_off[sidx] = enc(dptr);
            }
            L.tcnt[lane] = 0;
            if (lane == 0) L.seg_start[nseg] = total;
            wsync();
            int32_t out_n = 0;
            // as in count_batch: the next pass's element loads before this
            // pass's probes
            int s = 0;
            int32_t e_next = 0;
            if (lane < total) {
                int s_lo = 0, s_n = nseg;
                while (s_n > 1) {
                    const int half = s_n >> 1;
                    if (L.seg_start[s_lo + half] <= lane) {
                        s_lo += half;
                        s_n -= half;
                    } else {
                        s_n = half;
                    }
                }
                s = s_lo;
                e_next = dec(L.seg_off[s])[lane - L.seg_start[s]];
            }
            for (int32_t tb = 0; tb < total; tb += 64) {
                const int32_t t = tb + lane;
                bool pass = false;
                int l = 0;
                const int32_t e = e_next;
                const int s_cur = s;
                if (t + 64 < total) {
                    while (L.seg_start[s + 1] <= t + 64) s++;
                    e_next = dec(L.seg_off[s])[t + 64 - L.seg_start[s]];
                }
                if (t < total) {
                    l = L.seg_prefix[s_cur];
                    pass = test_direct(E, x, l, L.pdrv[l], e, dec(L.boff[l]), L.blen[l]);
                }
                const unsigned long long bal = __ballot(pass);
                if (pass) arena[out_n + (int32_t)__popcll(bal & ((1ull << lane) - 1ull))] = e;
                add_runs(L.tcnt, l, t < total, pass, lane);
                out_n += (int32_t)__popcll(bal);
            }
            wsync();
            // survivors are in parent order: slices start at the scan of the counts
            int ntot = 0;
            const int32_t tc = lane < np ? L.tcnt[lane] : 0;
            const int32_t st = wave_scan_excl(tc, lane, &ntot);
            if (lane < np) L.tstart[lane] = st;
            if (lane == 0) L.tstart[np] = ntot;
            wsync();
            if (mcount == 0) {
                expand_over(eid, x, np, 0, tc);
            } else {
                // a share group's leader: every member reads its own range
                // out of each parent's slice
                for (int k = 0; k < mcount; k++) {
                    const int mid = uni(P.lists[mbegin + k]);
                    const Node &M = P.nodes[mid];
                    int32_t rb = 0, re = 0;
                    if (lane < np && tc > 0) member_range(M, lane, arena + st, tc, &rb, &re);
                    if (M.kind == kEnum) expand_over(mid, x, np, rb, re);
                    else count_member(M, re - rb, lane < np);
                }
            }
        }
        // parents too large for the arena: one at a time into setbuf(x)
        if (bigmask) {
            const int sp0 = plev0, sp1 = plev1;
            for (int l = 0; l < np; l++) {
                if (!(bigmask >> l & 1ull)) continue;
                if (stopped()) break;
                if (sp0 >= 0) set_level(sp0, L.tu[l], L.tidx[l]);
                if (sp1 >= 0) set_level(sp1, L.tv[l], 0);
                plev0 = plev1 = -1;
                const int32_t len = materialise(E);
                if (lane == 0) L.set_len[x] = len;
                wsync();
                if (mcount == 0) {
                    if (len > 0) counts_over_set(eid, x, 0, len);
                } else {
                    for (int k = 0; k < mcount; k++) {
                        const int mid = uni(P.lists[mbegin + k]);
                        const Node &M = P.nodes[mid];
                        int32_t rb, re;
                        member_range(M, -1, setbuf(x), len, &rb, &re);
                        if (M.kind == kEnum) {
                            if (re > rb) counts_over_set(mid, x, rb, re);
                        } else {
                            count_member(M, re - rb, lane == 0);
                        }
                    }
                }
                plev0 = sp0;
                plev1 = sp1;
            }
        }
    }

    // the leaf enumeration children of node nid (level x, set S_x of length
    // len materialised), batched over S_x in groups of 64 parents
    __device__ __forceinline__ void leaf_children_over_set(int nid, int x, int32_t len) {
        const Node &N = P.nodes[nid];
        const int cb = uni(N.child_begin), cc = uni(N.child_count);
        const int32_t *S = setbuf(x);
        for (int c = 0; c < cc; c++) {
            const int eid = cb + c;
            if (!is_leaf_enum(P.nodes[eid])) continue;
            for (int32_t s0 = 0; s0 < len; s0 += kP) {
                if (stopped()) return;
                const int np = min(kP, len - s0);
                if (lane < np) {
                    const int32_t v = S[s0 + lane];
                    const long long o = P.rp[v];
                    L.tu[lane] = v;
                    L.tidx[lane] = s0 + lane;
                    L.tro0[lane] = (int32_t)o;
                    L.trl0[lane] = (int32_t)(P.rp[v + 1] - o);
                    L.tru0[lane] = P.up[v];
                }
                wsync();
                plev0 = x;
                plev1 = -1;
                leaf_batch(eid, np, np == 64 ? ~0ull : ((1ull << np) - 1ull));
                plev0 = -1;
            }
        }
    }

    __device__ __forceinline__ bool has_deep_enum_child(const Node &N) const {
        for (int c = 0; c < N.child_count; c++) {
            const Node &E = P.nodes[N.child_begin + c];
            if (E.kind == kEnum && !is_leaf_enum(E)) return true;
        }
        return false;
    }

    // depth-first walk of the deep enumeration children of root node rid
    // (those with enumeration children of their own; leaf ones run as
    // batches), with levels 0..1 already assigned in m[].  Each frame holds a
    // materialised set; its count children and leaf enumeration children run
    // batched over the whole set, its deep enumeration children per element.
    __device__ __forceinline__ void dfs(int rid) {
        const Node &R = P.nodes[rid];
        const int cb = uni(R.child_begin), cc = uni(R.child_count);
        for (int c = 0; c < cc; c++) {
            const int e0 = cb + c;
            const Node &E0 = P.nodes[e0];
            if (E0.kind != kEnum || is_leaf_enum(E0)) continue;
            if (stopped()) return;
            const int32_t len = materialise(E0);
            if (lane == 0) L.set_len[2] = len;
            wsync();
            if (len == 0) continue;
            counts_over_set(e0, 2, 0, len);
            leaf_children_over_set(e0, 2, len);
            if (!has_deep_enum_child(E0)) continue;
            // stack of enumeration frames
            if (lane == 0) {
                L.st_node[0] = e0;
                L.st_idx[0] = 0;
                L.st_child[0] = 0;
            }
            int sp = 1;
            wsync();
            while (sp > 0) {
                if (stopped()) return;
                const int f = sp - 1;
                const int nid = uni(L.st_node[f]);
                const Node &N = P.nodes[nid];
                const int x = N.level;
                const int ncb = uni(N.child_begin), ncc = uni(N.child_count);
                int ch = uni(L.st_child[f]);
                const int idx = uni(L.st_idx[f]);
                // advance to the next deep enumeration child
                while (ch < ncc && (P.nodes[ncb + ch].kind != kEnum || is_leaf_enum(P.nodes[ncb + ch]))) ch++;
                if (ch >= ncc) {
                    if (idx + 1 >= L.set_len[x]) {
                        sp--;
                        wsync();
                        continue;
                    }
                    if (lane == 0) {
                        L.st_idx[f] = idx + 1;
                        L.st_child[f] = 0;
                    }
                    wsync();
                    continue;
                }
                if (lane == 0) L.st_child[f] = ch + 1;
                set_level(x, setbuf(x)[idx], idx);
                const int nid2 = ncb + ch;
                const int32_t len2 = materialise(P.nodes[nid2]);
                if (lane == 0) L.set_len[x + 1] = len2;
                wsync();
                if (len2 == 0) continue;
                counts_over_set(nid2, x + 1, 0, len2);
                leaf_children_over_set(nid2, x + 1, len2);
                if (has_deep_enum_child(P.nodes[nid2])) {
                    if (lane == 0) {
                        L.st_node[sp] = nid2;
                        L.st_idx[sp] = 0;
                        L.st_child[sp] = 0;
                    }
                    sp++;
                    wsync();
                }
            }
        }
    }
};

// Anti-vertex check: vals[y] is the image of level y (the candidate
// included).  The sets N(vals[a]) \ {vals[y] : y in xmask[a]} over the
// anti-vertex's neighbour levels a must have an empty intersection.  Kept
// out of line: rare, and large enough to crowd the hot loops' registers.
__device__ __noinline__ bool av_check(const KParams &P, const int32_t *vals, const AVCheck &c) {
    const int32_t *best = nullptr;
    int32_t best_n = INT_MAX;
    int best_a = -1;
    for (int a = 0; a < kMaxLevels; a++) {
        if (!(c.nbr >> a & 1u)) continue;
        const int32_t v = vals[a];
        const int32_t n = (int32_t)(P.rp[v + 1] - P.rp[v]);
        if (n < best_n) {
            best_n = n;
            best = P.col + P.rp[v];
            best_a = a;
        }
    }
    for (int32_t i = 0; i < best_n; i++) {
        const int32_t w = best[i];
        if (c.label >= 0 && (P.lab == nullptr || P.lab[w] != c.label)) continue;
        bool in_all = true;
        for (int a = 0; a < kMaxLevels && in_all; a++) {
            if (!(c.nbr >> a & 1u)) continue;
            // w must not be the image of a true pattern neighbour of a
            for (uint32_t xm = c.xmask[a]; xm && in_all; xm &= xm - 1)
                if (vals[__builtin_ctz(xm)] == w) in_all = false;
            if (!in_all || a == best_a) continue;
            const int32_t v = vals[a];
            RowRef r;
            r.p = P.col + P.rp[v];
            r.n = (int32_t)(P.rp[v + 1] - P.rp[v]);
            r.up = P.up[v];
            r.owner = v;
            if (!in_row(P, r, w)) in_all = false;
        }
        if (in_all) return false;
    }
    return true;
}

// every level value comes from Ctx::val, which knows the batch layout
// (fixed assignment, root batch, set batch or task batch)
template <bool kAV, bool kFac, bool kCnt>
__device__ bool Ctx<kAV, kFac, kCnt>::av_pass(const AVCheck &c, int x, int l, int32_t e) const {
    int32_t vals[kMaxLevels];
    for (int y = 0; y < kMaxLevels; y++) vals[y] = y < x ? val(y, l) : (y == x ? e : 0);
    return av_check(P, vals, c);
}

// Root checks (labels and anti-vertex checks on levels 0 / 1) for prefix l.
// root filters that need only the task's vertices (u, v = -1 for a vertex
// task's second slot): labels, and for domains a root whose anchor image is
// already in the domain (another wave may have just set the bit: a stale
// read only costs the work)
__device__ __forceinline__ bool root_pre(const KParams &P, const Node &R, int32_t u, int32_t v) {
    if (R.label0 >= 0 && (P.lab == nullptr || P.lab[u] != R.label0)) return false;
    if (R.kind == kRootEdge && R.label1 >= 0 && (P.lab == nullptr || P.lab[v] != R.label1)) return false;
    if (P.mark && R.anchor_level >= 0) {
        const int32_t a = R.anchor_level == 0 ? u : v;
        const uint32_t w = __atomic_load_n(P.mark + (long long)R.plan * P.mark_words + (a >> 5), __ATOMIC_RELAXED);
        if ((w >> (a & 31)) & 1u) return false;
    }
    return true;
}

// anti-vertex checks of a root (the task's rows are loaded)
template <bool kAV, bool kFac, bool kCnt>
__device__ __forceinline__ bool root_ok(Ctx<kAV, kFac, kCnt> &C, const Node &R, int l) {
    if constexpr (kAV)
        for (int i = 0; i < R.av_count; i++) {
            const AVCheck &c = C.P.avs[R.av_begin + i];
            // the deepest root level is the "candidate" of the check
            const int x = R.level;
            if (!C.av_pass(c, x, l, C.val(x, l))) return false;
        }
    return true;
}

// kAV: the trie holds anti-vertex checks (the variant without them keeps
// the out-of-line check and its call frame out of the hot loops)
template <bool kAV, bool kPre, bool kCnt = false>
__device__ __forceinline__ void match_body(const KParams P) {
    __shared__ Lds L;
    const int lane = threadIdx.x;
    int32_t *buf0 = P.scratch ? P.scratch + (long long)blockIdx.x * P.wave_stride : nullptr;
    Ctx<kAV, kPre, kCnt> C(P, L, buf0, lane);
    C.arena = buf0 ? buf0 + P.wave_stride - P.arena_cap : nullptr;
    if (lane < kMaxLevels) {
        // a valid vertex in every slot of the fixed assignment
        L.m[lane] = 0;
        L.roff[lane] = 0;
        L.rlen[lane] = 0;
        L.rup[lane] = 0;
        L.cur_idx[lane] = 0;
        L.set_len[lane] = 0;
    }
    if constexpr (kPre) fac_lds[lane] = 1;
    if (lane == 0) {
        L.stop = 0;
        L.bytes = 0;
        L.t_start = 0;
        if (P.time_budget || (P.run_flags & PG_RUN_WAVE_TIMES)) {
            const unsigned long long now = wall_clock64();
            const unsigned long long old = atomicCAS(P.t_start, 0ull, now);
            L.t_start = old ? old : now;
        }
    }
    wsync();
    // share groups apply to batched count and existence launches (not to
    // emission, domain marks, or level-2 expansion one root task at a time)
    const bool share_on =
        !(P.run_flags & (PG_RUN_NO_TASK_BATCH | PG_RUN_NO_SHARE)) && (kCnt || (!P.mark && P.mode != kModeEmit));
    // this launch's window of root tasks: [t_lo, t_hi) of the edge tasks
    // followed by the vertex tasks
    const long long t_lo = P.task_begin;
    const long long t_hi = P.task_end > 0 ? P.task_end : P.n_etasks + P.n_vtasks;
    for (;;) {
        if (C.stopped()) break;
        // guided claiming: tasks are sorted costliest first, so claims grow
        // from one task at the head to P.chunk at the tail.  The cursor
        // counts claims; claim i covers a fixed range of tasks (a function
        // of i alone), so every launch forms the same task batches.
        long long c_beg = 0, c_end = 0;
        if (lane == 0) {
            const long long i = (long long)atomicAdd(P.cursor, 1ull);
            c_beg = claim_start(i, P.chunk, P.chunk_ramp);
            c_end = claim_start(i + 1, P.chunk, P.chunk_ramp);
        }
        c_beg = t_lo + (long long)__shfl(c_beg, 0);
        c_end = min(t_lo + (long long)__shfl(c_end, 0), t_hi);
        if (c_beg >= t_hi) break;
        const long long t0 = c_beg;
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
                // the batch's tasks tb .. tb + np
                int32_t u = 0, v = 0;
                if (lane < np) {
                    const long long t = tb + lane;
                    if (edge_phase) {
                        u = P.tsrc[t];
                        v = P.tdst[t];
                    } else {
                        u = P.n - 1 - (int32_t)(t - P.n_etasks);
                    }
                }
                bool okr = false;
                if constexpr (kPre) {
                    // labelled roots / domains: a root no task passes costs
                    // no row loads
                    okr = lane < np && root_pre(P, R, u, v);
                    if (!__ballot(okr)) continue;
                }
                if (lane < np) {
                    L.tu[lane] = u;
                    L.tv[lane] = v;
                    L.tidx[lane] = 0;
                    L.ptask[lane] = lane;
                    const long long ou = P.rp[u];
                    L.tro0[lane] = (int32_t)ou;
                    L.trl0[lane] = (int32_t)(P.rp[u + 1] - ou);
                    L.tru0[lane] = P.up[u];
                    if (edge_phase) {
                        const long long ov = P.rp[v];
                        L.tro1[lane] = (int32_t)ov;
                        L.trl1[lane] = (int32_t)(P.rp[v + 1] - ov);
                        L.tru1[lane] = P.up[v];
                    }
                }
                wsync();
                // the batch's root tasks also stay in registers (lane l holds
                // task l): deeper batches reuse the parent slots
                const int32_t task_u = lane < np ? L.tu[lane] : 0;
                const int32_t task_v = lane < np ? L.tv[lane] : 0;
                C.plev0 = 0;
                C.plev1 = edge_phase ? 1 : -1;
                C.vl0 = -1;
                C.anc_level = !kCnt && P.mark ? uni(R.anchor_level) : -1;
                C.anc_plan = uni(R.plan);
                if constexpr (!kPre) okr = lane < np && root_pre(P, R, task_u, task_v);
                if constexpr (kAV)
                    if (okr) okr = root_ok(C, R, lane);
                const unsigned long long okmask = __ballot(okr);
                const int cb = uni(R.child_begin), cc = uni(R.child_count);
                bool any_enum = false;
                for (int c = 0; c < cc; c++) {
                    const Node &N = P.nodes[cb + c];
                    if (N.kind == kEnum) {
                        any_enum = true;
                        break;
                    }
                    if (share_on && N.share >= 0) continue;  // counted by its share group
                    if (lane < np) L.pmode[lane] = okr ? (int8_t)0 : (int8_t)-1;
                    wsync();
                    C.count_batch(N, np);
                }
                // share groups: one materialisation per root task for all members
                if (share_on && edge_phase) {
                    const int lb = uni(R.list_begin), lc = uni(R.list_count);
                    for (int g = 0; g < lc; g++) {
                        if (C.stopped()) break;
                        C.leaf_batch(uni(P.lists[lb + g]), np, okmask);
                    }
                }
                if (!any_enum || !edge_phase) {
                    C.plev0 = C.plev1 = -1;
                    continue;
                }
                // enumeration children with only count children: whole batch
                bool any_deep = false;
                for (int c = 0; c < cc; c++) {
                    const int eid = cb + c;
                    if (P.nodes[eid].kind != kEnum) continue;
                    if (!C.is_leaf_enum(P.nodes[eid])) {
                        any_deep = true;
                        continue;
                    }
                    if (share_on && P.nodes[eid].share >= 0) continue;  // expanded by its share group
                    if (C.stopped()) break;
                    C.leaf_batch(eid, np, okmask);
                }
                C.plev0 = C.plev1 = -1;
                // deeper enumeration children: one task at a time
                if (!any_deep) continue;
                for (int l = 0; l < np; l++) {
                    if (!(okmask >> l & 1ull)) continue;
                    const int32_t u = __shfl(task_u, l), v = __shfl(task_v, l);
                    wsync();
                    C.set_level(0, u, 0);
                    C.set_level(1, v, 0);
                    C.dfs(rid);
                    if (C.stopped()) break;
                }
                wsync();
            }
            tb += np;
        }
    }
    wsync();
    if (lane < P.n_plans && C.acc) {
        const unsigned long long old = atomicAdd(P.counts + lane, C.acc);
        if (old + C.acc < old) atomicOr(P.flags, 1);
    }
    if (lane == 0 && L.bytes) atomicAdd(P.bytes_ctr, L.bytes);
    // load balance: when this wavefront ran out of tasks, after the first
    // wavefront's start (the earliest is kept complemented, so a max finds it)
    if ((P.run_flags & PG_RUN_WAVE_TIMES) && lane == 0) {
        const unsigned long long t = wall_clock64() - L.t_start;
        atomicMax(P.wave_done, ~t);
        atomicMax(P.wave_done + 1, t);
    }
}

// Long count launches: held to 96 VGPRs (five wavefronts per SIMD by
// registers; 8.9 KB of LDS per wave then allows 18 per CU).  The kernel is
// bound by load latency, so resident waves are what hides it; most of the
// few spills this costs sit in the task-claim loop.  Its launches only
// count (no existence stop, emission or domain marks), so those paths are
// compiled out.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) match_kernel(KParams P) {
    match_body<false, false, true>(P);
}

// The same program at 128 VGPRs and four wavefronts per SIMD, without
// spills, for launches that end quickly (existence, emission, tries without
// enumeration levels, small task sets), where it measured faster
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) match_kernel_light(KParams P) {
    match_body<false, false>(P);
}

// labelled roots or domain marks: roots are filtered before their rows load;
// also the variant that evaluates factor nodes.  Held to 128 VGPRs (four
// waves per SIMD): its launches, e.g. 64 anchored labelled plans of a
// mining round, are short, and there five waves measured slower
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) match_kernel_pre(KParams P) {
    match_body<false, true>(P);
}

// anti-vertex checks: held to 128 VGPRs (four waves per SIMD) like the
// light build.  Left free it takes about 190 and two waves per SIMD; the
// spills of the out-of-line check's image table cost less than the halved
// residency (p7 on a 1M-edge Chung-Lu graph 32.7 -> 27.0 ms)
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) match_kernel_av(KParams P) {
    match_body<true, true>(P);
}

static const void *variant_fn(int variant) {
    switch (variant) {
    case kVarAV: return reinterpret_cast<const void *>(match_kernel_av);
    case kVarPre: return reinterpret_cast<const void *>(match_kernel_pre);
    case kVarLight: return reinterpret_cast<const void *>(match_kernel_light);
    default: return reinterpret_cast<const void *>(match_kernel);
    }
}

int match_blocks_per_cu(int variant) {
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, variant_fn(variant), 64, 0);
    if (e != hipSuccess || nb < 1) nb = 8;
    return nb;
}

// rows of bits: out[r] += popcount(bits[r * words .. (r + 1) * words)); one
// row per blockIdx.y, a grid-stride loop over its words
__global__ void __launch_bounds__(256) popcount_rows(const uint32_t *bits, long long words,
                                                     unsigned long long *out) {
    const uint32_t *row = bits + (long long)blockIdx.y * words;
    unsigned long long c = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (long long)gridDim.x * blockDim.x)
        c += (unsigned long long)__popc(row[i]);
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out + blockIdx.y, c);
}

hipError_t launch_popcount(const uint32_t *bits, long long words, int rows, unsigned long long *out,
                           hipStream_t s) {
    const long long blocks = std::min<long long>(std::max<long long>(1, (words + 255) / 256), 1024);
    hipLaunchKernelGGL(popcount_rows, dim3((unsigned)blocks, (unsigned)rows), dim3(256), 0, s, bits, words, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// Device memory for callers that cannot allocate (pg_count_noalloc): one
// fixed array per device, [control block | program trie | per-wavefront
// scratch], held from the library's first use on a device until the
// process ends.  Every such call on a device shares it, so calls that
// overlap on one device race.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};
}  // namespace

// The array's device address on the current device (looked up once per
// device, with that device current; host code never uses the symbol
// itself, only this address).
hipError_t static_scratch(void **ptr, size_t *bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_static_ptr[dev] = p;
    }
    *ptr = g_static_ptr[dev];
    *bytes = kStaticScratchBytes;
    return hipSuccess;
}

// words 64-bit zeros from p on: a kernel rather than a memset, so the
// clear is an ordinary kernel node for callers that capture the stream
__global__ void __launch_bounds__(256) zero_words(unsigned long long *p, long long words) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

hipError_t launch_zero(unsigned long long *p, long long words, hipStream_t s) {
    hipLaunchKernelGGL(zero_words, dim3(1), dim3(256), 0, s, p, words);
    return hipGetLastError();
}

// Hub bitmaps: row r of bits (words 32-bit words) is the adjacency of
// vertex first + r.  One workgroup per row: clear it, then set the bit of
// every neighbour (rows are sorted, but neighbours share words, so OR).
__global__ void __launch_bounds__(256) build_hub_bits(const int64_t *rp, const int32_t *col, int32_t first,
                                                      long long words, uint32_t *bits) {
    const int32_t v = first + (int32_t)blockIdx.x;
    uint32_t *row = bits + (long long)blockIdx.x * words;
    for (long long i = threadIdx.x; i < words; i += blockDim.x) row[i] = 0u;
    __syncthreads();
    for (long long e = rp[v] + threadIdx.x; e < rp[v + 1]; e += blockDim.x) {
        const int32_t c = col[e];
        atomicOr(row + (c >> 5), 1u << (c & 31));
    }
}

hipError_t launch_hub_bits(const int64_t *rp, const int32_t *col, int32_t first, int32_t rows, long long words,
                           uint32_t *bits, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(build_hub_bits, dim3((unsigned)rows), dim3(256), 0, s, rp, col, first, words, bits);
    return hipGetLastError();
}

hipError_t launch_match(const KParams &P, int grid, int variant, hipStream_t s) {
    // the long-count build has no existence, emission or domain paths
    if (variant == kVarPlain && (P.mode != kModeCount || P.mark || P.out)) return hipErrorInvalidValue;
    if (variant == kVarAV) hipLaunchKernelGGL(match_kernel_av, dim3(grid), dim3(64), 0, s, P);
    else if (variant == kVarPre) hipLaunchKernelGGL(match_kernel_pre, dim3(grid), dim3(64), 0, s, P);
    else if (variant == kVarLight) hipLaunchKernelGGL(match_kernel_light, dim3(grid), dim3(64), 0, s, P);
    else hipLaunchKernelGGL(match_kernel, dim3(grid), dim3(64), 0, s, P);
    return hipGetLastError();
}

}  // namespace pg
