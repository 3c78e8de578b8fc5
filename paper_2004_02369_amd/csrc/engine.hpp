// Launch interface of the matching kernel (host <-> device parameter block).
#pragma once

#include <hip/hip_runtime.h>

#include "pg_internal.hpp"

namespace pg {

enum RunMode : int32_t { kModeCount = 0, kModeExists = 1, kModeEmit = 2 };

struct KParams {
    const int64_t *rp;
    const int32_t *col;
    long long ncol;            // entries of col (2m, < 2^31)
    const int32_t *up;         // per vertex: index in its row of the first neighbour above it
    const uint32_t *hub_bits;  // dense adjacency bitmaps of vertices hub_start..n-1 (hub_words each)
    long long hub_words;
    int32_t hub_start;
    const int16_t *lab;
    const int32_t *perm;
    const int32_t *tsrc;
    const int32_t *tdst;
    const Node *nodes;
    const AVCheck *avs;
    const int32_t *roots;
    const int32_t *lists;      // share groups (leaders of a root, members of a leader)
    unsigned long long *cursor;
    unsigned long long *counts;
    int32_t *flags;            // [0] overflow, [1] stop, [2] time limit reached
    unsigned long long *t_start; // device wall clock when the first wavefront started (0 = not yet)
    unsigned long long *wave_done; // PG_RUN_WAVE_TIMES: [0] ~earliest, [1] latest finish (ticks after t_start)
    unsigned long long *emit_ctr;
    int32_t *out;
    unsigned long long *bytes_ctr;
    int32_t *scratch;
    long long wave_stride;     // ints per wave
    long long set_cap;         // ints per materialised level
    long long arena_cap;       // ints of the level-2 arena at the end of each wave's scratch
    long long n_etasks;
    long long n_vtasks;
    unsigned long long cap;    // emit capacity (rows)
    long long time_budget;     // wall-clock ticks from the first wavefront's start; 0 = unlimited
    int32_t n;
    int32_t n_roots;
    int32_t chunk;             // largest claim of root tasks
    long long chunk_ramp;      // claims per step of claim growth (claim j holds 1 + j / chunk_ramp tasks, at most chunk)
    int32_t n_plans;
    int32_t mode;
    int32_t run_flags;
    int32_t batch_max_avg;     // leaf batching only while parents average at most this many candidates; 0 = always
    uint32_t *mark;            // domains: per plan, a bitmap of mark_words words over rank ids (nullptr = off)
    long long mark_words;
    long long task_begin;      // root tasks [task_begin, task_end) of this launch; task_end 0 = to the last
    long long task_end;
    // labelled graphs: col[lab_copy + rp[v] ..) is v's row sorted by (label,
    // id); label l's part starts lab_off[v * (n_labels + 1) + l] entries in
    // (nullptr / 0 = no copy)
    const int32_t *lab_off;
    int32_t n_labels;
    long long lab_copy;
};

// Kernel variants: plain (long count launches; 96 VGPRs, 18 waves per CU);
// "pre" for labelled roots, domain marks or factor nodes (roots are
// filtered before their rows load); anti-vertex checks; light (the plain
// program at 128 VGPRs, 16 waves per CU, for launches that end quickly).
enum Variant : int { kVarPlain = 0, kVarPre = 1, kVarAV = 2, kVarLight = 3 };
constexpr int kNumVariants = 4;

hipError_t launch_match(const KParams &P, int grid, int variant, hipStream_t s);

// Dense adjacency bitmaps of the rows of vertices first .. first+rows-1
// (words 32-bit words each) from the CSR, on stream s.
hipError_t launch_hub_bits(const int64_t *rp, const int32_t *col, int32_t first, int32_t rows, long long words,
                           uint32_t *bits, hipStream_t s);

// Size of the fixed per-device array behind pg_count_noalloc.
constexpr size_t kStaticScratchBytes = size_t(256) << 20;

// Device address and size of that array on the current device.
hipError_t static_scratch(void **ptr, size_t *bytes);

// Zero `words` 64-bit words at p with a kernel on stream s.
hipError_t launch_zero(unsigned long long *p, long long words, hipStream_t s);

// out[r] += number of set bits in row r of `rows` bitmaps of `words` words each
hipError_t launch_popcount(const uint32_t *bits, long long words, int rows, unsigned long long *out,
                           hipStream_t s);

// resident wavefronts (one per workgroup) per compute unit of a variant
int match_blocks_per_cu(int variant);

}  // namespace pg
