/*
 * pg.h -- C ABI of libpg, a pattern-aware subgraph matcher for AMD MI355X
 * (gfx950), after Peregrine (Jamshidi, Mahadasa, Vora; EuroSys 2020).
 *
 * The library turns a pattern into an exploration plan on the host
 * (Sec. 4.1, Fig. "Computing exploration plan": symmetry-breaking partial
 * order, core = minimum connected vertex cover, matching orders) and runs
 * that plan on the GPU over a degree-ordered CSR graph resident in HBM
 * (Sec. 5.1-5.2), counting the vertices outside the core by set sizes.
 *
 * Conventions shared by every entry point:
 *  - Every call returns pg_status: PG_OK (0), PG_STOPPED (1, early exit),
 *    or a negative error.  On error, pg_last_error() returns a message for
 *    the calling thread.  No C++ exception crosses this interface.
 *  - Pointers are host pointers unless the comment says "device".
 *  - The caller owns every input array; the library copies what it keeps
 *    during the call.  Objects returned through an out-pointer are owned by
 *    the library until the matching pg_free_* call.
 *  - hip_stream is a hipStream_t (NULL = the null stream).  Calls that take
 *    one enqueue their GPU work on it and return after it completed.
 *  - Vertex ids in results are the caller's original ids.
 *  - Counts are exact unsigned 64-bit integers; a count that does not fit
 *    returns PG_EOVERFLOW.
 */
#ifndef PG_H
#define PG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pg_status;
#define PG_OK 0
#define PG_STOPPED 1
#define PG_EINVAL (-1)        /* bad argument, malformed or unsupported pattern shape */
#define PG_ENOMEM (-2)        /* host or device allocation failed */
#define PG_EDEVICE (-3)       /* HIP runtime error */
#define PG_EOVERFLOW (-4)     /* a count exceeds 2^64 - 1 */
#define PG_EUNSUPPORTED (-5)  /* valid request this build does not handle */
#define PG_ETIMEDOUT (-6)     /* the run's time limit passed; counts are partial (lower bounds) */

typedef struct pg_graph pg_graph;
typedef struct pg_plan pg_plan;

/* ------------------------------------------------------------------ graph */

typedef struct {
    int32_t device;         /* HIP device ordinal; -1 = the current device */
    int32_t hub_min_degree; /* rows of this degree or more also get a dense adjacency bitmap
                               (membership in one load instead of a binary search);
                               0 = 16, -1 = no bitmaps */
    int32_t hub_budget_mib; /* HBM for those bitmaps, highest degrees first; 0 = a sixteenth of
                               the device memory (at least 1024 MiB) */
    int32_t reserved[5];    /* must be zero */
} pg_options;

typedef struct {
    int32_t n;            /* vertices (ids 0..n-1, isolated ones kept) */
    int32_t d_max;        /* largest degree */
    int64_t m;            /* distinct undirected edges after ingest */
    int64_t device_bytes; /* HBM held by the resident graph */
    int32_t labelled;     /* 1 if vertex labels were given */
    int32_t device;       /* HIP device holding the graph */
    const int32_t *perm;  /* host, n entries: perm[rank] = original id; owned by the graph */
    int32_t resident_waves[2]; /* wavefronts of the matching kernel resident at once on the device:
                                  [0] the build for long count launches, [1] the anti-vertex
                                  build.  A launch's default grid is the residency of the build
                                  it runs on (shorter and labelled launches use a four-wave build,
                                  at most [0]) */
    int32_t hub_count;      /* rows held as bitmaps too (the hub_count highest ranks) */
    int32_t hub_min_degree; /* smallest degree among them (0 if none) */
} pg_graph_info_t;

/* Ingest an undirected graph and make it resident on the GPU (Sec. 5.1,
 * 5.2): self-loops are dropped, duplicate and reversed pairs collapse into
 * one edge, vertices are renumbered by ascending (degree, original id) --
 * the degree order of Sec. 5.2 with ties broken by id -- and every
 * adjacency list is sorted.
 *   n       number of vertices, >= 1
 *   m       number of input pairs, >= 0
 *   src,dst m entries each, ids in [0, n)        (PG_EINVAL otherwise)
 *   labels  n entries or NULL (unlabelled graph); values >= 0
 *   opt     NULL for defaults
 *   out     receives the graph; release with pg_free_graph */
pg_status pg_load_graph(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                        const int16_t *labels, const pg_options *opt, pg_graph **out);

/* Sizes of the resident graph and its degree order (Sec. 5.2: vertices are
 * ranked by degree; perm maps a rank back to the caller's id), plus the
 * launch residency the engine sizes its grids from.  out: host. */
pg_status pg_graph_info(const pg_graph *g, pg_graph_info_t *out);

/* Copy the resident CSR back to the host in rank ids: row_ptr n+1 entries,
 * col 2m entries (each row ascending).  Either pointer may be NULL. */
pg_status pg_graph_csr(const pg_graph *g, int64_t *row_ptr, int32_t *col);

void pg_free_graph(pg_graph *g);

/* ---------------------------------------------------------------- patterns */

#define PG_EDGE 0       /* true edge: the two images must be adjacent (Sec. 2.1) */
#define PG_ANTI_EDGE 1  /* anti-edge: the two images must not be adjacent (Sec. 3.1.1) */

typedef struct {
    int32_t u, v, type;  /* pattern vertex ids; type PG_EDGE or PG_ANTI_EDGE */
} pg_edge;

/* A pattern (Sec. 3.1, Fig. "Pattern Interface").
 *   Regular vertices are 0..k-1 (2 <= k <= 16) and must be connected by
 *   true edges.  Anti-vertices are k..k+n_anti_vertices-1 (at most 4); an
 *   anti-vertex has only anti-edges, to regular vertices, at least one
 *   (Sec. 3.1.2).  labels: k + n_anti_vertices entries or NULL; -1 = any.
 *   induced = 1 adds an anti-edge between every pair of non-adjacent
 *   regular vertices, which makes the count vertex-induced (the Theorem of
 *   Sec. 3.1.3). */
typedef struct {
    int32_t k;
    int32_t n_anti_vertices;
    int32_t n_edges;
    int32_t induced;
    const pg_edge *edges;
    const int16_t *labels;
} pg_pattern_desc;

/* ------------------------------------------------------------------- plans */

#define PG_PLAN_AUTO 0          /* matching orders = linear extensions when few, else partial order only */
#define PG_PLAN_LINEAR_EXT 1    /* always enumerate linear extensions of the core order (Sec. 4.1) */
#define PG_PLAN_PARTIAL_ORDER 2 /* one program constrained only by the partial order */

typedef struct {
    int32_t mode;          /* PG_PLAN_* */
    int32_t anchored;      /* 1: plan for the domain of regular vertex `anchor` (MNI support,
                              Sec. 2 and 5.5): the anchor is kept in the core and symmetry
                              is broken only by automorphisms that fix it, so every data
                              vertex the anchor can map to is reached; counts are then
                              valid maps / |stabiliser of the anchor| */
    int32_t anchor;        /* the anchored regular vertex, 0..k-1 */
    int32_t reserved[5];   /* must be zero */
} pg_plan_options;

typedef struct {
    uint64_t aut;             /* |Aut_t|: permutations of the regular vertices preserving
                                 edges, anti-edges, labels and anti-vertex neighbourhoods */
    int32_t k;
    int32_t core_size;
    uint32_t core_mask;       /* bit u set: regular vertex u is in the core */
    int32_t n_matching_orders;/* distinct matching orders (Sec. 4.1) */
    int32_t n_programs;       /* count-mode programs after merging identical ones */
    int32_t n_levels;         /* deepest program (levels evaluated on the GPU) */
    int32_t n_order;          /* pairs in order[] */
    int32_t order[240];       /* pairs (a, b): m(a) < m(b) is required (Grochow-Kellis) */
    int32_t n_orbit_steps;    /* orbit_size[i]: orbit of the vertex fixed at step i */
    int32_t orbit_size[16];   /* |Aut_t| = product of orbit_size[0..n_orbit_steps) */
    int32_t orbit_vertex[16];
    int32_t mode_used;        /* PG_PLAN_LINEAR_EXT or PG_PLAN_PARTIAL_ORDER */
    double plan_ms;           /* host time to build the plan */
    int32_t anchor;           /* anchored vertex, -1 if none (then aut is its stabiliser's order) */
} pg_plan_info_t;

/* Build the exploration plan of a pattern (Sec. 4.1 Fig. "Computing
 * exploration plan", Sec. 4.2-4.3).  Pure host computation.
 * PG_EINVAL: k out of range, disconnected regular vertices, an edge that
 * is both true and anti, an anti-vertex with a true edge or no anti-edge,
 * ids out of range. */
pg_status pg_plan_pattern(const pg_pattern_desc *p, pg_plan **out);
pg_status pg_plan_pattern_ex(const pg_pattern_desc *p, const pg_plan_options *opt, pg_plan **out);
pg_status pg_plan_info(const pg_plan *plan, pg_plan_info_t *out);
void pg_free_plan(pg_plan *plan);

/* Serialise the level programs the GPU interprets, for inspection and
 * host-side checking.  enum_mode = 0: the count programs (merged, with
 * multiplicities); 1: the enumeration programs.  buf: host, cap int32
 * entries; *len receives the number of entries needed (PG_EINVAL with
 * *len set when cap is too small).  Layout: n_programs, then per program
 *   n_levels, mult_lo, mult_hi, n_levels levels, n_factors, n_factors levels,
 * each level being
 *   isect diff lo hi excl t_isect t_diff base label group pv n_av,
 *   then per anti-vertex check: nbr label xmask[16].
 * Level masks are over earlier levels (bit y = level y); pv is the pattern
 * vertex matched at the level; the last level counts C(|S|, group).
 * Factors (count programs only) are further non-core groups evaluated at
 * the last level's depth, each independent of every other non-core vertex
 * (a label none of them can carry, no order relation or anti-vertex between
 * them): a prefix's count is the product of every factor's C(|S|, group)
 * and the last level's (Sec. 4, non-core vertices counted from set sizes). */
pg_status pg_plan_programs(const pg_plan *plan, int32_t enum_mode, int32_t *buf, int64_t cap, int64_t *len);

/* ---------------------------------------------------------------- counting */

typedef struct {
    int32_t grid_waves;    /* persistent wavefronts; 0 = auto: the resident wavefronts of the
                              kernel build the launch runs on, fewer for small launches (about
                              64 root tasks per program leaf per wave, at least one per CU) */
    int32_t chunk;         /* largest claim of root tasks (claims grow from 1 over the costliest
                              tasks); 0 = auto (64) */
    int32_t flags;         /* PG_RUN_* */
    int32_t time_limit_ms; /* stop every wavefront once this long has passed on the device clock
                              since the launch's first wavefront started, and return
                              PG_ETIMEDOUT; 0 = no limit */
    int32_t hub_min_degree;/* membership tests use the bitmap of rows of at least this degree
                              (among those the graph holds bitmaps for) and binary search
                              below it; 0 = every bitmap the graph holds, -1 = none */
    int32_t batch_max_avg; /* an enumeration level whose children only count is expanded for
                              up to 64 parents in one flattened pass while those parents
                              average at most this many candidates, else parent by parent;
                              0 = always flattened */
    int32_t task_begin;    /* count over root tasks [task_begin, task_end) of the launch only
                              (pg_launch_tasks gives their number): every match is found from
                              exactly one root task (Sec. 5.1: matches grow from a start vertex),
                              so counts over windows that partition the tasks sum to the full
                              counts; tasks come costliest first.  0, 0 = every task */
    int32_t task_end;      /* 0 = to the last task */
    int32_t reserved[2];   /* must be zero */
} pg_run_config;

#define PG_RUN_COUNT_BYTES 1  /* also count the merge-model bytes of every set operation */
#define PG_RUN_NO_MODE_B 2    /* never count by complement (|A| - |A & B|) */
#define PG_RUN_NO_TASK_BATCH 4  /* expand level 2 one root task at a time only */
#define PG_RUN_LIGHT_KERNEL 8   /* run a long counting launch on the four-waves-per-SIMD build of
                                   the kernel (128 VGPRs, no spills) instead of the five-wave one;
                                   shorter launches always use it */
#define PG_RUN_WAVE_TIMES 32     /* record the first and last wavefront finish times (pg_run_stats) */
#define PG_RUN_NO_SHARE 16      /* evaluate every level-2 node of an edge root on its own, without the
                                   share groups that read several nodes' candidates from one
                                   materialised set (Sec. 3.2: several patterns in one call) */

typedef struct {
    double kernel_ms;        /* device time of the matching kernel (HIP events) */
    double total_ms;         /* host wall time of the call */
    uint64_t logical_bytes;  /* sum over set operations of 4 (|A| + |B|), if requested */
    uint64_t root_tasks;     /* root tasks processed */
    int32_t grid_waves;
    int32_t chunk;
    uint64_t tasks_started;  /* root tasks of the window in claims the wavefronts made: all of
                                them after a complete run, the part reached before the stop
                                when a time limit ended the run */
    double wave_done_first_ms; /* with PG_RUN_WAVE_TIMES: when the first and the last wavefront */
    double wave_done_last_ms;  /* finished, after the first one started (device clock); their
                                  difference is the launch's load imbalance */
} pg_run_stats;

/* Count the matches of each plan (Sec. 3.2: count() is match() with a
 * counting callback).  All plans run in one launch over one shared root
 * frontier.  counts: host, n_plans entries, receives exact counts in the
 * order of plans[].  Synchronous on hip_stream. */
pg_status pg_count(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, uint64_t *counts,
                   void *hip_stream);

/* pg_count with launch knobs (NULL = defaults) and run statistics
 * (NULL = not wanted).  Results do not depend on the knobs.  Plans whose
 * programs are identical (different patterns can compile to the same
 * plan, as K5 and the induced K5 do) are counted once per launch and their
 * counts copied; the statistics describe that launch. */
pg_status pg_count_ex(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, uint64_t *counts,
                      const pg_run_config *cfg, pg_run_stats *stats, void *hip_stream);

/* pg_count_ex for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops and harnesses that must not call
 * hipMalloc): the control block, the program trie and the per-wavefront
 * scratch come from one fixed device array of 256 MiB that the library
 * holds on every device it runs on until the process ends.  Makes no
 * device allocation.  The grid (cfg->grid_waves, or the default) is
 * reduced to the wavefronts whose scratch fits the array; PG_ENOMEM with a
 * message when not even one wavefront's scratch fits (enumeration levels x
 * the largest degree, plus a 128 KB arena) or the trie does not.  Every
 * call on one device shares that array and leaves its contents behind:
 * calls that overlap on one device race, so callers serialise them (one
 * stream, or their own lock).  counts: host, n_plans entries.  Synchronous
 * on hip_stream; no run statistics. */
pg_status pg_count_noalloc(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, uint64_t *counts,
                           const pg_run_config *cfg, void *hip_stream);

/* Existence query with early termination (Sec. 3.2.2, Sec. 5.3): found = 1
 * if the pattern has at least one match.  Returns PG_OK either way. */
pg_status pg_exists(pg_graph *g, const pg_plan *plan, int32_t *found, void *hip_stream);

/* Enumerate every match once (one canonical representative per set of
 * automorphic matches): match(G, p, f) of Sec. 3.2 (Fig. "program
 * examples") with the matches written to device memory instead of passed
 * to a callback.  out: device memory of cap * k int32, row i holds
 * match i as original vertex ids indexed by pattern vertex.  n_total
 * receives the number of matches even when it exceeds cap (then only the
 * first cap rows, in unspecified order, are written). */
pg_status pg_enumerate(pg_graph *g, const pg_plan *plan, int32_t *out, uint64_t cap,
                       uint64_t *n_total, void *hip_stream);

/* Callback form of matching (Fig. "program examples", match(G, p, f)):
 * ids holds k original vertex ids indexed by pattern vertex.  A nonzero
 * return stops the exploration and the call returns PG_STOPPED.
 * n_matches receives the number of callbacks made.  Matches stream through
 * one device buffer of about 64 MB: windows of root tasks are enumerated
 * in turn and the callback sees each window's matches before the next
 * window is launched, so a stop takes effect within one window.  Runs on
 * the null stream; the callback runs on the calling host thread. */
typedef int (*pg_match_cb)(const int32_t *ids, int32_t k, void *user);
pg_status pg_match(pg_graph *g, const pg_plan *plan, pg_match_cb cb, void *user, uint64_t *n_matches);
/* pg_match with the device buffer's capacity in rows (0 = about 64 MB). */
pg_status pg_match_ex(pg_graph *g, const pg_plan *plan, pg_match_cb cb, void *user, uint64_t *n_matches,
                      uint64_t buffer_rows);

/* Root tasks of a plan's enumeration on a graph: every match is found from
 * exactly one of them, so windows of tasks partition the matches.  Tasks
 * are the graph's edges (each once, oriented by rank) when the plan's cores
 * have two vertices or more, then the vertices when some core has one; the
 * edges come costliest first. */
pg_status pg_root_tasks(pg_graph *g, const pg_plan *plan, int64_t *n_tasks);

/* Root tasks of one counting launch of these plans (the edges when some
 * plan's cores have two vertices or more, then the vertices when some core
 * has one): the range of pg_run_config.task_begin / task_end. */
pg_status pg_launch_tasks(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, int64_t *n_tasks);

/* pg_enumerate over the root tasks [task_begin, task_end) only (0 <=
 * task_begin < task_end <= pg_root_tasks). */
pg_status pg_enumerate_range(pg_graph *g, const pg_plan *plan, int64_t task_begin, int64_t task_end, int32_t *out,
                             uint64_t cap, uint64_t *n_total, void *hip_stream);

/* MNI domains (Sec. 2, frequent subgraph mining; Sec. 5.5): for each plan p,
 * compiled anchored at regular vertex u_p (pg_plan_options.anchored), the
 * number of distinct data vertices v such that some valid map sends u_p to
 * v, i.e. |dom(u_p)| over all embeddings.  The MNI support of a pattern is
 * the minimum of |dom(u)| over its vertices; one anchor per automorphism
 * orbit suffices.  sizes: host, n_plans entries.  One launch over all
 * plans (at most 64); the graph holds n_plans n-bit bitmaps for it.  Root
 * tasks whose anchor image is already in the domain are skipped, so the
 * launch counts nothing (pg_count of an anchored plan counts valid maps /
 * |stabiliser of the anchor|).  PG_EINVAL if a plan is not anchored.
 * Synchronous on hip_stream. */
pg_status pg_domain_sizes(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, uint64_t *sizes,
                          const pg_run_config *cfg, void *hip_stream);

/* ------------------------------------------------------ asynchronous jobs
 *
 * For request loops that keep several queries in flight (serving): a job is
 * one launch of one or more plans (one plan for an existence query) on the
 * caller's stream, using device memory the caller provides, so admission
 * can be decided by memory and launches on different streams overlap.  No
 * call below allocates device memory. */

typedef struct pg_job pg_job;

#define PG_JOB_COUNT 0   /* exact counts of every plan */
#define PG_JOB_EXISTS 1  /* one plan; stops at the first match (Sec. 5.3) */

/* Device bytes a job of these plans needs (control words, the program trie
 * and per-wavefront scratch for cfg's grid; cfg NULL = whole-GPU grid). */
pg_status pg_job_workspace_size(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, int32_t mode,
                                const pg_run_config *cfg, uint64_t *bytes);

/* Enqueue a job on hip_stream and return without waiting.  workspace:
 * device memory of at least pg_job_workspace_size() bytes, 256-byte
 * aligned, owned by the caller and not touched by anything else until
 * pg_job_finish returns (PG_ENOMEM if too small).  The plans must stay
 * alive until then.  Jobs on different streams run concurrently. */
pg_status pg_submit(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, int32_t mode,
                    const pg_run_config *cfg, void *workspace, uint64_t workspace_bytes, void *hip_stream,
                    pg_job **out);

/* Non-blocking: done = 1 once the job's kernel has completed and its counts
 * have reached host memory.  At most 64 jobs per graph are in flight
 * (pg_submit returns PG_ENOMEM beyond that); finish every job before
 * pg_free_graph. */
pg_status pg_job_poll(pg_job *job, int32_t *done);

/* Wait for the job, write its counts (host, n_plans entries; for an
 * existence job counts[0] = 1 if a match exists, else 0) and release the
 * job handle (not the workspace).  After pg_job_poll has reported done,
 * this makes no further GPU call and does not wait. */
pg_status pg_job_finish(pg_job *job, uint64_t *counts, pg_run_stats *stats);

/* Thread-local message for the last error on this thread ("" if none). */
const char *pg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PG_H */
