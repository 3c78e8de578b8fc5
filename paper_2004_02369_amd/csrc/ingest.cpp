// Host part of graph ingest (no device code): the canonical undirected
// simple edge set, the degree order, the CSR in rank ids with sorted rows,
// each row's split into lower and upper neighbours, the oriented-edge root
// tasks sorted costliest first, and labels in rank order.  pg_load_graph
// uploads the result.
#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "pg_internal.hpp"

namespace pg {

namespace {

// LSD radix sort of 64-bit keys, 16 bits per pass.
void radix_sort_u64(std::vector<uint64_t> &a, int key_bits) {
    std::vector<uint64_t> tmp(a.size());
    std::vector<size_t> cnt(1 << 16);
    for (int shift = 0; shift < key_bits; shift += 16) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (uint64_t x : a) cnt[(x >> shift) & 0xFFFF]++;
        size_t s = 0;
        for (auto &c : cnt) {
            size_t t = c;
            c = s;
            s += t;
        }
        for (uint64_t x : a) tmp[cnt[(x >> shift) & 0xFFFF]++] = x;
        a.swap(tmp);
    }
}

int bits_for(uint64_t v) {
    int b = 0;
    while (b < 64 && (v >> b)) b++;
    return b;
}

}  // namespace

pg_status ingest(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int16_t *labels,
                 HostGraph *out, std::string *err) {
    auto fail = [&](const std::string &msg) { *err = msg; };
    // 1. canonical undirected simple edge set (Sec. 2.1)
    std::vector<uint64_t> keys;
    keys.reserve((size_t)m);
    for (int64_t i = 0; i < m; i++) {
        int32_t a = src[i], b = dst[i];
        if (a < 0 || b < 0 || a >= n || b >= n) {
            fail("edge endpoint out of range at index " + std::to_string(i));
            return PG_EINVAL;
        }
        if (a == b) continue;
        if (a > b) std::swap(a, b);
        keys.push_back((uint64_t)(uint32_t)a << 32 | (uint32_t)b);
    }
    radix_sort_u64(keys, 32 + bits_for((uint64_t)n));
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    const int64_t mu = (int64_t)keys.size();
    if (2 * mu > (int64_t)INT32_MAX) {
        fail("graph too large: more than 2^31 - 1 adjacency entries");
        return PG_EUNSUPPORTED;
    }

    // 2. degree order: rank by (degree, original id) ascending (Sec. 5.2)
    std::vector<int64_t> deg(n, 0);
    for (uint64_t k : keys) {
        deg[k >> 32]++;
        deg[k & 0xFFFFFFFFu]++;
    }
    int64_t dmax = 0;
    for (int64_t d : deg) dmax = std::max(dmax, d);
    if (dmax > INT32_MAX / 2) { fail("degree too large"); return PG_EUNSUPPORTED; }
    std::vector<int64_t> dstart(dmax + 2, 0);
    for (int64_t d : deg) dstart[d + 1]++;
    for (int64_t d = 0; d <= dmax; d++) dstart[d + 1] += dstart[d];
    std::vector<int32_t> rank(n), perm(n);
    for (int32_t v = 0; v < n; v++) {
        int32_t r = (int32_t)dstart[deg[v]]++;
        rank[v] = r;
        perm[r] = v;
    }

    // 3. CSR in rank ids, rows sorted ascending
    std::vector<int64_t> rp(n + 1, 0);
    for (int32_t r = 0; r < n; r++) rp[r + 1] = rp[r] + deg[perm[r]];
    std::vector<int32_t> col((size_t)(2 * mu));
    {
        std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
        for (uint64_t k : keys) {
            int32_t a = rank[k >> 32], b = rank[k & 0xFFFFFFFFu];
            col[fill[a]++] = b;
            col[fill[b]++] = a;
        }
    }
    keys.clear();
    keys.shrink_to_fit();
    for (int32_t r = 0; r < n; r++) std::sort(col.begin() + rp[r], col.begin() + rp[r + 1]);
    // split of each row into lower and upper neighbours (degree-oriented part)
    std::vector<int32_t> up(n);
    for (int32_t r = 0; r < n; r++)
        up[r] = (int32_t)(std::lower_bound(col.begin() + rp[r], col.begin() + rp[r + 1], r) - (col.begin() + rp[r]));

    // 4. root edge tasks u < v, costliest first (Sec. 5.2: start with the
    //    highest-degree vertices); cost estimate d(u) + d(v)
    std::vector<int32_t> tsrc((size_t)mu), tdst((size_t)mu);
    {
        std::vector<int64_t> cstart(2 * dmax + 3, 0);
        for (int32_t u = 0; u < n; u++)
            for (int64_t e = rp[u]; e < rp[u + 1]; e++)
                if (col[e] > u) cstart[2 * dmax - (deg[perm[u]] + deg[perm[col[e]]]) + 1]++;
        for (size_t i = 1; i < cstart.size(); i++) cstart[i] += cstart[i - 1];
        for (int32_t u = 0; u < n; u++)
            for (int64_t e = rp[u]; e < rp[u + 1]; e++)
                if (col[e] > u) {
                    int64_t slot = cstart[2 * dmax - (deg[perm[u]] + deg[perm[col[e]]])]++;
                    tsrc[slot] = u;
                    tdst[slot] = col[e];
                }
    }
    std::vector<int16_t> lab;
    if (labels) {
        lab.resize(n);
        for (int32_t v = 0; v < n; v++) {
            if (labels[v] < 0) { fail("labels must be >= 0"); return PG_EINVAL; }
            lab[rank[v]] = labels[v];
        }
    }

    out->n = n;
    out->m = mu;
    out->d_max = (int32_t)dmax;
    out->rp = std::move(rp);
    out->col = std::move(col);
    out->up = std::move(up);
    out->perm = std::move(perm);
    out->tsrc = std::move(tsrc);
    out->tdst = std::move(tdst);
    out->lab = std::move(lab);
    return PG_OK;
}

}  // namespace pg
