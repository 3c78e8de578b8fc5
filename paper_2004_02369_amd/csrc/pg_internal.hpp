// Internal types of libpg shared by the host plan compiler, the graph
// store and the HIP engine.  Nothing here is part of the C ABI.
#pragma once

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pg.h"

namespace pg {

constexpr int kMaxK = 16;       // regular pattern vertices
constexpr int kMaxAV = 4;       // anti-vertices
constexpr int kMaxLevels = 16;  // GPU levels per program (one per matched pattern vertex)
constexpr int kMaxPlansPerLaunch = 64;

// Kinds of program-trie nodes.  A "level" is one pattern vertex matched on
// the GPU; level 0 and 1 of edge-rooted programs come from a root task.
enum NodeKind : int32_t {
    kRootVertex = 0,  // root task = one vertex (level 0); children are count nodes at level 1
    kRootEdge = 1,    // root task = one oriented edge u < v (levels 0, 1)
    kEnum = 2,        // materialise this level's candidate set, then descend per candidate
    kCount = 3,       // add C(|candidates|, group) * mult to counts[plan]
    kEmit = 4,        // write one match row per candidate
    kFactor = 5,      // C(|candidates|, group) multiplies the next count sibling's term
};

// Anti-vertex constraint (Sec. 3.1.2 / Sec. 4.3), evaluated for a candidate
// once every vertex it depends on is matched: no data vertex lies in all
// sets N(m(a)) \ m(true pattern neighbours of a), a over its neighbours.
struct AVCheck {
    uint32_t nbr;                 // levels of the anti-vertex's regular neighbours
    int32_t label;                // -1 = any
    uint32_t xmask[kMaxLevels];   // per neighbour level a: levels of a's true pattern neighbours
};

// One node of the program trie, laid out for the device.  All masks are
// over levels strictly below `level`.
struct Node {
    int32_t kind;
    int32_t level;
    uint32_t isect;    // candidates must be adjacent to these levels' images (true edges)
    uint32_t diff;     // ... and not adjacent to these (anti-edges)
    uint32_t lo;       // ... and larger than these images (partial / matching order)
    uint32_t hi;       // ... and smaller than these
    uint32_t excl;     // ... and different from these (injectivity not implied otherwise)
    uint32_t excl_in;  // excl levels whose images certainly lie in every isect row and no diff row
    uint32_t t_isect;  // isect levels still to test once the base set is used
    uint32_t t_diff;   // diff levels still to test once the base set is used
    int32_t base;      // materialised ancestor level whose set contains every candidate; -1 none
    int32_t label;     // -1 = any
    int32_t group;     // count: number of interchangeable vertices counted as C(n, group)
    int32_t av_begin;  // anti-vertex checks applied to this node's candidates
    int32_t av_count;
    int32_t plan;      // count / emit: output slot
    int32_t child_begin;
    int32_t child_count;
    int32_t k;         // emit: pattern size
    uint64_t mult;     // count: multiplicity (identical programs merged)
    int32_t label0;    // root nodes: labels of level 0 and level 1
    int32_t label1;
    int8_t pv[kMaxLevels];  // emit: pattern vertex matched at each level
    int32_t anchor_level;   // count: level holding the plan's anchored vertex (-1 none)
    // share groups (siblings under an edge root with one set operation and
    // different id ranges): a member's `share` is its group's leader, an
    // enumeration node outside the tree that holds the widest range; a
    // leader lists its members, an edge root its leaders, at
    // lists[list_begin .. list_begin + list_count)
    int32_t share;
    int32_t list_begin;
    int32_t list_count;
    int32_t flags;     // kIndepCounts
};

// Enumeration node flag: every child is a count node whose candidates do not
// depend on this node's vertex except through excluding it, and the pattern
// puts that vertex inside the count's one row (excl_in), with no id range,
// base set, difference row, label, anti-vertex check or domain anchor.  Each
// candidate of this node then adds the same C(|row| - excluded, group), so a
// parent's total is its number of candidates times that term.
constexpr int32_t kIndepCounts = 1;

// A program: one matching order with its completion, as a sequence of levels.
struct Level {
    uint32_t isect = 0, diff = 0, lo = 0, hi = 0, excl = 0;
    // excluded levels whose pattern vertex has a true edge to every isect
    // level's and an anti-edge to every diff level's (and the label): their
    // images are in every isect row and in no diff row of any valid prefix
    uint32_t excl_in = 0;
    uint32_t t_isect = 0, t_diff = 0;
    int32_t base = -1;
    int32_t label = -1;
    int32_t group = 1;
    int32_t pv = -1;
    std::vector<AVCheck> avs;  // checks applied to this level's candidates
};

struct Program {
    std::vector<Level> lev;    // last level is the count / emit level
    // count programs: further non-core groups, each independent of every
    // other non-core vertex (its own fixed label, no order relation to
    // them, no anti-vertex), counted at the last level's depth; the
    // program's count per prefix is the product of their C(|S|, j) and
    // the last level's
    std::vector<Level> factors;
    uint64_t mult = 1;
};

struct PlanImpl {
    pg_plan_info_t info{};
    int32_t k = 0;
    int32_t anchor = -1;  // anchored regular vertex (domain plans), -1 none
    std::vector<Program> count_progs;  // merged, with multiplicities
    std::vector<Program> enum_progs;   // one per matching order, every vertex its own level
};

// The trie of all programs of one launch, flattened for upload.
struct Trie {
    std::vector<Node> nodes;
    std::vector<AVCheck> avs;
    std::vector<int32_t> roots;   // node ids of root nodes
    std::vector<int32_t> lists;   // share groups: leaders of a root, members of a leader (node ids)
    int32_t max_level = 0;        // deepest level index + 1
    bool has_vertex_root = false;
    bool has_edge_root = false;
    bool consistent = false;      // one leaf per program
};

Trie build_trie(const std::vector<const PlanImpl *> &plans, bool emit);

// A graph after the host part of ingest, in rank ids (degree order).
struct HostGraph {
    int32_t n = 0;
    int64_t m = 0;                // distinct undirected edges
    int32_t d_max = 0;
    std::vector<int64_t> rp;      // n + 1 row offsets
    std::vector<int32_t> col;     // 2m entries, each row ascending
    std::vector<int32_t> up;      // per row: index of its first neighbour above it
    std::vector<int32_t> perm;    // rank -> original id
    std::vector<int32_t> tsrc, tdst;  // oriented edges u < v, costliest first
    std::vector<int16_t> lab;     // labels in rank order (empty: unlabelled)
};

// Host part of pg_load_graph (see ingest.cpp); *err describes a failure.
pg_status ingest(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int16_t *labels,
                 HostGraph *out, std::string *err);

// Plan compiler entry (host only).
pg_status compile_plan(const pg_pattern_desc *desc, const pg_plan_options *opt, PlanImpl *out,
                       std::string *err);

void set_error(const std::string &msg);

}  // namespace pg

struct pg_plan {
    pg::PlanImpl impl;
    uint64_t uid = 0;  // unique per plan object (cache key; addresses get reused)
};
