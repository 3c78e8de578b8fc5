// C ABI of libpg: graph store (ingest to a degree-ordered CSR resident in
// HBM), plan handles, and the count / exists / enumerate / match calls that
// launch the matching kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "engine.hpp"
#include "pg_internal.hpp"

namespace pg {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string &msg) { g_err = msg; }

}  // namespace pg

using pg::set_error;

#define PG_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            set_error(std::string(#call) + ": " + hipGetErrorString(e_));             \
            return PG_EDEVICE;                                                        \
        }                                                                             \
    } while (0)

namespace {
// Host-side preparation of one launch: the program trie, its upload image
// and the launch shape.
struct LaunchPlan {
    pg::Trie trie;
    std::vector<char> image;  // nodes | anti-vertex checks | roots | share-group lists
    size_t a_off = 0, r_off = 0, x_off = 0;
    bool with_av = false;
    int variant = pg::kVarPlain;
    int grid = 0, chunk = 0;
    long long n_et = 0, n_vt = 0;
    int enum_levels = 0;
    long long set_cap = 0, arena_cap = 0;
    size_t scratch_ints = 0;
};

inline void dfree(void *p) {
    if (p) (void)hipFree(p);
}
inline void edestroy(hipEvent_t e) { (void)hipEventDestroy(e); }
}  // namespace

struct pg_job {
    pg_graph *g = nullptr;
    LaunchPlan L;
    int32_t n_plans = 0;
    int32_t mode = 0;
    unsigned long long *ctl = nullptr;  // in the caller's workspace
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, ek = nullptr, e1 = nullptr;  // kernel start, kernel end, counts on the host
    std::chrono::steady_clock::time_point t_submit;
    bool enqueued = false;  // work is on the stream that reads L.image
    int ctl_slot = -1;      // this job's block of the graph's pinned control blocks
    long long tasks = 0;    // root tasks of its window
    ~pg_job();
};

struct pg_graph {
    int32_t n = 0;
    int64_t m = 0;
    int32_t d_max = 0;
    int32_t device = 0;
    int32_t n_cu = 0;
    int64_t wall_khz = 0;  // device wall-clock ticks per millisecond
    int32_t blocks_per_cu[pg::kNumVariants] = {};  // resident wavefronts per CU of each kernel variant (pg::Variant)
    bool labelled = false;
    std::vector<int32_t> perm;  // rank -> original id
    // device arrays
    int64_t *rp = nullptr;
    int32_t *col = nullptr;
    int32_t *up = nullptr;
    uint32_t *hub_bits = nullptr;  // dense adjacency bitmaps of ranks hub_start..n-1
    int32_t hub_start = 0;
    int64_t hub_min_deg = 0;
    std::vector<int64_t> hub_deg;  // host: degrees of ranks hub_start..n-1 (ascending)
    int64_t hub_words = 0;
    int16_t *lab = nullptr;
    // labelled graphs: col holds, after the 2m row entries, a copy of every
    // row sorted by (label, id) at the same offsets; lab_off[v * (n_labels
    // + 1) + l] is where label l starts within v's row of that copy
    int32_t *lab_off = nullptr;
    int32_t n_labels = 0;
    int32_t *dperm = nullptr;
    int32_t *tsrc = nullptr;
    int32_t *tdst = nullptr;
    int64_t device_bytes = 0;
    // per-call buffers, grown on demand
    std::mutex mu;
    uint32_t *marks = nullptr;              // domain bitmaps (pg_domain_sizes)
    unsigned long long *mark_cnt = nullptr;
    size_t mark_cap = 0;                    // words held by marks
    // asynchronous jobs: each copies its control block back into one of
    // these pinned host blocks on its own stream, so finishing it needs no
    // further GPU call
    unsigned long long *ctl_host = nullptr;
    std::vector<int> ctl_free;
    std::mutex job_mu;
    int32_t *scratch = nullptr;
    size_t scratch_ints = 0;
    void *trie_buf = nullptr;
    size_t trie_bytes = 0;
    unsigned long long *ctl = nullptr;  // control block: counts[64], cursor, emit counter, bytes, flags, start clock
    // cached launch preparation of the last pg_count / pg_enumerate call
    std::vector<uint64_t> trie_key;
    bool trie_emit = false;
    LaunchPlan launch;
    bool trie_valid = false;

    ~pg_graph() {
        dfree(rp);
        dfree(col);
        dfree(up);
        dfree(hub_bits);
        dfree(lab);
        dfree(lab_off);
        dfree(dperm);
        dfree(tsrc);
        dfree(tdst);
        dfree(scratch);
        dfree(trie_buf);
        dfree(ctl);
        dfree(marks);
        dfree(mark_cnt);
        if (ctl_host) (void)hipHostFree(ctl_host);
    }
};

inline pg_job::~pg_job() {
    if (enqueued) (void)hipStreamSynchronize(s);
    if (e0) edestroy(e0);
    if (ek) edestroy(ek);
    if (e1) edestroy(e1);
    if (ctl_slot >= 0) {
        std::lock_guard<std::mutex> lock(g->job_mu);
        g->ctl_free.push_back(ctl_slot);
    }
}

namespace {

constexpr int64_t kHubMinDegree = 16;
constexpr long long kArenaInts = 32768;  // per wavefront
constexpr int64_t kHubBudgetBytes = int64_t(1) << 30;
// label-sorted row copy: at most this many label offsets (4 bytes each)
constexpr int64_t kLabelOffsetBudget = int64_t(1) << 28;

constexpr int kCtlCounts = 0;
constexpr int kCtlCursor = 64;
constexpr int kCtlEmit = 65;
constexpr int kCtlBytes = 66;
constexpr int kCtlFlags = 67;  // four int32 in two slots: overflow, stop, timed out, unused
constexpr int kCtlStart = 69;  // device wall clock at the first wavefront's start
constexpr int kCtlDoneFirst = 70;  // wave finish times (PG_RUN_WAVE_TIMES): ~(earliest), latest, in ticks
constexpr int kCtlDoneLast = 71;
constexpr int kCtlWords = 72;
constexpr int kJobSlots = 64;  // asynchronous jobs in flight per graph

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

template <class T>
pg_status upload(T **dst, const std::vector<T> &src, int64_t *bytes) {
    size_t nb = std::max<size_t>(1, src.size()) * sizeof(T);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), nb);
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
        return PG_ENOMEM;
    }
    if (!src.empty()) PG_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    *bytes += (int64_t)nb;
    return PG_OK;
}

}  // namespace

extern "C" {

const char *pg_last_error(void) { return pg::g_err.c_str(); }

pg_status pg_load_graph(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int16_t *labels,
                        const pg_options *opt, pg_graph **out) {
    try {
        if (!out) { set_error("out is NULL"); return PG_EINVAL; }
        *out = nullptr;
        if (n < 1) { set_error("n must be >= 1"); return PG_EINVAL; }
        if (m < 0 || (m > 0 && (!src || !dst))) { set_error("bad edge arrays"); return PG_EINVAL; }
        int64_t hub_min = kHubMinDegree, hub_budget = 0;  // 0: set from the device's memory below
        if (opt) {
            for (int i = 0; i < 5; i++)
                if (opt->reserved[i]) { set_error("pg_options.reserved must be zero"); return PG_EINVAL; }
            if (opt->hub_min_degree < -1 || opt->hub_budget_mib < 0) {
                set_error("bad hub bitmap options");
                return PG_EINVAL;
            }
            if (opt->hub_min_degree == -1) hub_min = INT64_MAX;
            else if (opt->hub_min_degree > 0) hub_min = opt->hub_min_degree;
            if (opt->hub_budget_mib > 0) hub_budget = (int64_t)opt->hub_budget_mib << 20;
        }
        int dev = opt ? opt->device : -1;
        if (dev < 0) PG_HIP(hipGetDevice(&dev));
        int ndev = 0;
        PG_HIP(hipGetDeviceCount(&ndev));
        if (dev >= ndev) { set_error("device out of range"); return PG_EINVAL; }
        DeviceGuard guard(dev);

        // host part of ingest: canonical edges, degree order, CSR, tasks
        pg::HostGraph h;
        {
            std::string err;
            const pg_status ist = pg::ingest(n, m, src, dst, labels, &h, &err);
            if (ist) {
                set_error(err);
                return ist;
            }
        }
        const int64_t mu = h.m, dmax = h.d_max;
        std::vector<int64_t> &rp = h.rp;
        std::vector<int32_t> &col = h.col, &up = h.up, &perm = h.perm, &tsrc = h.tsrc, &tdst = h.tdst;
        std::vector<int16_t> &lab = h.lab;

        std::unique_ptr<pg_graph> g(new pg_graph());
        g->n = n;
        g->m = mu;
        g->d_max = (int32_t)dmax;
        g->device = dev;
        g->labelled = labels != nullptr;
        hipDeviceProp_t prop;
        PG_HIP(hipGetDeviceProperties(&prop, dev));
        g->n_cu = prop.multiProcessorCount;
        int khz = 0;
        PG_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        if (khz <= 0) { set_error("device reports no wall-clock rate"); return PG_EDEVICE; }
        g->wall_khz = khz;
        for (int v = 0; v < pg::kNumVariants; v++) g->blocks_per_cu[v] = pg::match_blocks_per_cu(v);
        pg_status st;
        if ((st = upload(&g->rp, rp, &g->device_bytes))) return st;
        // labelled levels drive from the part of a row that holds their
        // label: each row again, sorted by (label, id), after the rows
        // (so one 32-bit offset into col addresses both), and per vertex
        // the start of every label's part
        int32_t n_labels = 0;
        if (labels && 4 * mu <= (int64_t)INT32_MAX) {
            for (int16_t l : lab) n_labels = std::max<int32_t>(n_labels, l + 1);
            if ((int64_t)n * (n_labels + 1) > kLabelOffsetBudget) n_labels = 0;
        }
        if (n_labels > 0) {
            const int32_t stride = n_labels + 1;
            std::vector<int32_t> ext((size_t)(4 * mu));
            std::copy(col.begin(), col.end(), ext.begin());
            std::vector<int32_t> off((size_t)n * (size_t)stride, 0);
            for (int32_t r = 0; r < n; r++) {
                int32_t *o = off.data() + (size_t)r * (size_t)stride;
                for (int64_t e = rp[r]; e < rp[r + 1]; e++) o[lab[col[e]] + 1]++;
                for (int32_t l = 0; l < n_labels; l++) o[l + 1] += o[l];
                std::vector<int32_t> pos(o, o + n_labels);
                // the row is in id order, so a stable placement by label
                // leaves every label's part in id order
                for (int64_t e = rp[r]; e < rp[r + 1]; e++) ext[(size_t)(2 * mu + rp[r] + pos[lab[col[e]]]++)] = col[e];
            }
            if ((st = upload(&g->col, ext, &g->device_bytes))) return st;
            if ((st = upload(&g->lab_off, off, &g->device_bytes))) return st;
            g->n_labels = n_labels;
        } else if ((st = upload(&g->col, col, &g->device_bytes))) {
            return st;
        }
        if ((st = upload(&g->up, up, &g->device_bytes))) return st;
        // hub rows also as dense bitmaps: the highest-degree vertices (rank
        // order is degree order) with degree >= hub_min, within a budget
        // (default: a sixteenth of the device's memory), built on the device
        // from the uploaded rows
        {
            if (hub_budget == 0) hub_budget = std::max<int64_t>(kHubBudgetBytes, (int64_t)(prop.totalGlobalMem / 16));
            const int64_t words = ((int64_t)n + 31) / 32;
            int32_t hs = n;
            while (hs > 0 && rp[hs] - rp[hs - 1] >= hub_min && (int64_t)(n - hs + 1) * words * 4 <= hub_budget)
                hs--;
            g->hub_start = hs;
            g->hub_words = words;
            g->hub_min_deg = hs < n ? rp[hs + 1] - rp[hs] : 0;
            for (int32_t r = hs; r < n; r++) g->hub_deg.push_back(rp[r + 1] - rp[r]);
            if (hs < n) {
                const size_t nb = (size_t)(n - hs) * (size_t)words * sizeof(uint32_t);
                if (hipMalloc(reinterpret_cast<void **>(&g->hub_bits), nb) != hipSuccess) {
                    set_error("hipMalloc hub bitmaps");
                    return PG_ENOMEM;
                }
                g->device_bytes += (int64_t)nb;
                PG_HIP(pg::launch_hub_bits(g->rp, g->col, hs, n - hs, words, g->hub_bits, nullptr));
                PG_HIP(hipDeviceSynchronize());
            }
        }
        if ((st = upload(&g->dperm, perm, &g->device_bytes))) return st;
        if ((st = upload(&g->tsrc, tsrc, &g->device_bytes))) return st;
        if ((st = upload(&g->tdst, tdst, &g->device_bytes))) return st;
        if (labels && (st = upload(&g->lab, lab, &g->device_bytes))) return st;
        PG_HIP(hipMalloc(reinterpret_cast<void **>(&g->ctl), kCtlWords * sizeof(unsigned long long)));
        g->perm = std::move(perm);
        *out = g.release();
        return PG_OK;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PG_ENOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return PG_EINVAL;
    }
}

pg_status pg_graph_info(const pg_graph *g, pg_graph_info_t *out) {
    if (!g || !out) { set_error("NULL argument"); return PG_EINVAL; }
    std::memset(out, 0, sizeof(*out));
    out->n = g->n;
    out->m = g->m;
    out->d_max = g->d_max;
    out->device_bytes = g->device_bytes;
    out->labelled = g->labelled ? 1 : 0;
    out->device = g->device;
    out->perm = g->perm.data();
    out->resident_waves[0] = g->n_cu * g->blocks_per_cu[pg::kVarPlain];
    out->resident_waves[1] = g->n_cu * g->blocks_per_cu[pg::kVarAV];
    out->hub_count = g->n - g->hub_start;
    out->hub_min_degree = g->hub_start < g->n ? (int32_t)g->hub_min_deg : 0;
    return PG_OK;
}

pg_status pg_graph_csr(const pg_graph *g, int64_t *row_ptr, int32_t *col) {
    if (!g) { set_error("NULL graph"); return PG_EINVAL; }
    DeviceGuard guard(g->device);
    if (row_ptr) PG_HIP(hipMemcpy(row_ptr, g->rp, sizeof(int64_t) * (size_t)(g->n + 1), hipMemcpyDeviceToHost));
    if (col && g->m) PG_HIP(hipMemcpy(col, g->col, sizeof(int32_t) * (size_t)(2 * g->m), hipMemcpyDeviceToHost));
    return PG_OK;
}

void pg_free_graph(pg_graph *g) {
    if (!g) return;
    DeviceGuard guard(g->device);
    delete g;
}

pg_status pg_plan_pattern_ex(const pg_pattern_desc *p, const pg_plan_options *opt, pg_plan **out) {
    try {
        if (!out) { set_error("out is NULL"); return PG_EINVAL; }
        *out = nullptr;
        if (opt)
            for (int i = 0; i < 5; i++)
                if (opt->reserved[i]) { set_error("pg_plan_options.reserved must be zero"); return PG_EINVAL; }
        static std::atomic<uint64_t> next_uid{1};
        std::unique_ptr<pg_plan> plan(new pg_plan());
        plan->uid = next_uid.fetch_add(1);
        std::string err;
        pg_status st = pg::compile_plan(p, opt, &plan->impl, &err);
        if (st) {
            set_error(err);
            return st;
        }
        *out = plan.release();
        return PG_OK;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PG_ENOMEM;
    }
}

pg_status pg_plan_pattern(const pg_pattern_desc *p, pg_plan **out) { return pg_plan_pattern_ex(p, nullptr, out); }

pg_status pg_plan_info(const pg_plan *plan, pg_plan_info_t *out) {
    if (!plan || !out) { set_error("NULL argument"); return PG_EINVAL; }
    *out = plan->impl.info;
    return PG_OK;
}

void pg_free_plan(pg_plan *plan) { delete plan; }

pg_status pg_plan_programs(const pg_plan *plan, int32_t enum_mode, int32_t *buf, int64_t cap, int64_t *len) {
    if (!plan || !len) { set_error("NULL argument"); return PG_EINVAL; }
    const auto &progs = enum_mode ? plan->impl.enum_progs : plan->impl.count_progs;
    std::vector<int32_t> v;
    v.push_back((int32_t)progs.size());
    for (const pg::Program &p : progs) {
        v.push_back((int32_t)p.lev.size());
        v.push_back((int32_t)(uint32_t)(p.mult & 0xFFFFFFFFu));
        v.push_back((int32_t)(uint32_t)(p.mult >> 32));
        auto put = [&](const pg::Level &L) {
            for (uint32_t x : {L.isect, L.diff, L.lo, L.hi, L.excl, L.t_isect, L.t_diff}) v.push_back((int32_t)x);
            v.push_back(L.base);
            v.push_back(L.label);
            v.push_back(L.group);
            v.push_back(L.pv);
            v.push_back((int32_t)L.avs.size());
            for (const pg::AVCheck &c : L.avs) {
                v.push_back((int32_t)c.nbr);
                v.push_back(c.label);
                for (int i = 0; i < pg::kMaxLevels; i++) v.push_back((int32_t)c.xmask[i]);
            }
        };
        for (const pg::Level &L : p.lev) put(L);
        v.push_back((int32_t)p.factors.size());
        for (const pg::Level &L : p.factors) put(L);
    }
    *len = (int64_t)v.size();
    if (!buf || cap < (int64_t)v.size()) { set_error("buffer too small"); return PG_EINVAL; }
    std::memcpy(buf, v.data(), v.size() * sizeof(int32_t));
    return PG_OK;
}

}  // extern "C"

namespace {

struct LaunchArgs {
    int mode = pg::kModeCount;
    int32_t *out = nullptr;
    uint64_t cap = 0;
    uint64_t *sizes = nullptr;     // domains: host, n_plans domain sizes (marks on)
    int64_t task_begin = 0;        // root-task window; task_end 0 = all tasks
    int64_t task_end = 0;
    uint32_t *mark_dev = nullptr;  // set by run(): the graph's mark bitmaps
    long long mark_words = 0;
};

pg_status check_args(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, const pg_run_config *cfg) {
    if (!g) { set_error("NULL graph"); return PG_EINVAL; }
    if (n_plans < 1 || n_plans > pg::kMaxPlansPerLaunch) { set_error("n_plans must be in [1, 64]"); return PG_EINVAL; }
    if (!plans) { set_error("plans is NULL"); return PG_EINVAL; }
    for (int i = 0; i < n_plans; i++)
        if (!plans[i]) { set_error("a plan is NULL"); return PG_EINVAL; }
    if (cfg) {
        if (cfg->grid_waves < 0 || cfg->chunk < 0 || cfg->time_limit_ms < 0 || cfg->hub_min_degree < -1 ||
            cfg->batch_max_avg < 0) {
            set_error("negative launch knob");
            return PG_EINVAL;
        }
        if (cfg->task_begin < 0 || cfg->task_end < 0 || (cfg->task_end > 0 && cfg->task_end <= cfg->task_begin)) {
            set_error("bad root-task window");
            return PG_EINVAL;
        }
        if (cfg->reserved[0] || cfg->reserved[1]) {
            set_error("pg_run_config.reserved must be zero");
            return PG_EINVAL;
        }
    }
    return PG_OK;
}

// root tasks from which a count launch with enumeration levels takes the
// five-wave kernel variant
constexpr long long kLongLaunchTasks = 1ll << 18;
// small launches: root tasks (times program leaves) per wave of the grid
constexpr long long kTasksPerWave = 64;

// shape of a launch for a built trie (mode: pg::RunMode; marks: domain
// bitmaps are on)
void shape(const pg_graph *g, const pg_run_config *cfg, LaunchPlan &L, int mode, bool marks) {
    const pg::Trie &T = L.trie;
    L.with_av = !T.avs.empty();
    L.n_et = T.has_edge_root ? (long long)g->m : 0;
    L.n_vt = T.has_vertex_root ? (long long)g->n : 0;
    bool pre = marks, enums = false;
    for (int32_t r : T.roots)
        if (T.nodes[r].label0 >= 0 || T.nodes[r].label1 >= 0) pre = true;
    for (const pg::Node &n : T.nodes) {
        if (n.kind == pg::kFactor) pre = true;
        if (n.kind == pg::kEnum) enums = true;
    }
    // five waves per SIMD pay off on long counts that enumerate; shorter
    // launches measured faster at four (no spills)
    const bool long_count = mode == pg::kModeCount && enums && L.n_et + L.n_vt >= kLongLaunchTasks &&
                            !(cfg && (cfg->flags & PG_RUN_LIGHT_KERNEL));
    L.variant = L.with_av ? pg::kVarAV : pre ? pg::kVarPre : long_count ? pg::kVarPlain : pg::kVarLight;
    // persistent grid: the wavefronts of this variant that can be resident
    // at once, fewer for small launches (about kTasksPerWave root tasks per
    // program leaf and wave, at least one wave per CU): there, starting and
    // draining idle waves costs more than the matching
    long long leaves = 0;
    for (const pg::Node &n : T.nodes) leaves += (n.kind == pg::kCount || n.kind == pg::kEmit) ? 1 : 0;
    const long long resident = (long long)g->n_cu * g->blocks_per_cu[L.variant];
    const long long want = ((L.n_et + L.n_vt) * std::max(1ll, leaves) + kTasksPerWave - 1) / kTasksPerWave;
    L.grid = cfg && cfg->grid_waves ? cfg->grid_waves
                                    : (int)std::min(resident, std::max<long long>(g->n_cu, want));
    L.chunk = cfg && cfg->chunk ? cfg->chunk : 64;
    // scratch: one set per enumeration level (levels 2 .. max_level-2) plus
    // the arena of batched expansions
    L.enum_levels = std::max(0, T.max_level - 3);
    L.set_cap = std::max<long long>(1, g->d_max);
    L.arena_cap = L.enum_levels ? kArenaInts : 0;
    L.scratch_ints = (size_t)L.grid * ((size_t)L.enum_levels * (size_t)L.set_cap + (size_t)L.arena_cap);
    const size_t nb = T.nodes.size() * sizeof(pg::Node), ab = T.avs.size() * sizeof(pg::AVCheck),
                 rb = T.roots.size() * sizeof(int32_t), xb = T.lists.size() * sizeof(int32_t);
    L.a_off = (nb + 15) & ~size_t(15);
    L.r_off = (L.a_off + ab + 15) & ~size_t(15);
    L.x_off = (L.r_off + rb + 15) & ~size_t(15);
    L.image.assign(L.x_off + xb + 64, 0);
    std::memcpy(L.image.data(), T.nodes.data(), nb);
    std::memcpy(L.image.data() + L.a_off, T.avs.data(), ab);
    std::memcpy(L.image.data() + L.r_off, T.roots.data(), rb);
    if (xb) std::memcpy(L.image.data() + L.x_off, T.lists.data(), xb);
}

pg_status check_trie(const pg::Trie &T) {
    if (T.max_level > pg::kMaxLevels) { set_error("plan too deep"); return PG_EUNSUPPORTED; }
    if (!T.consistent) { set_error("internal: program trie lost a program"); return PG_EUNSUPPORTED; }
    return PG_OK;
}

// Claims grow from 1 task to `chunk` over a window's costliest tasks: claim
// j holds 1 + j / ramp tasks (at most chunk), and the growth spans the
// window when ramp = 2 span / (chunk (chunk - 1)).
long long chunk_ramp(long long span, int chunk) {
    const long long c = std::max(1, chunk);
    return c > 1 ? std::max(1ll, 2 * span / (c * (c - 1))) : 1;
}

// tasks covered by the first i claims (the kernel's claim_start)
long long claim_start_host(long long i, int chunk, long long ramp) {
    const long long full = ramp * (long long)(chunk - 1);
    if (i <= full) {
        const long long q = i / ramp, r = i - q * ramp;
        return i + ramp * (q * (q - 1) / 2) + r * q;
    }
    const long long q = chunk - 1;
    return full + ramp * (q * (q - 1) / 2) + (i - full) * (long long)chunk;
}

// The effective root-task window of a launch: the call's own (enumeration
// windows) if set, else the run configuration's; end 0 = every task.
void effective_window(const LaunchPlan &L, const LaunchArgs &la, const pg_run_config *cfg, long long *b, long long *e) {
    *b = 0;
    *e = 0;
    if (la.task_begin || la.task_end) {
        *b = la.task_begin;
        *e = la.task_end;
    } else if (cfg) {
        *b = cfg->task_begin;
        *e = cfg->task_end;
    }
    if (*e == 0) *e = L.n_et + L.n_vt;
}

long long window_tasks(const LaunchPlan &L, const LaunchArgs &la, const pg_run_config *cfg) {
    long long b, e;
    effective_window(L, la, cfg, &b, &e);
    return e > b ? e - b : 0;
}

pg_status check_window(const LaunchPlan &L, const LaunchArgs &la, const pg_run_config *cfg) {
    long long b, e;
    effective_window(L, la, cfg, &b, &e);
    if (b < 0 || e > L.n_et + L.n_vt || (e <= b && L.n_et + L.n_vt > 0)) {
        set_error("bad root-task window (the launch has " + std::to_string(L.n_et + L.n_vt) + " root tasks)");
        return PG_EINVAL;
    }
    return PG_OK;
}

pg::KParams params(const pg_graph *g, const LaunchPlan &L, const void *trie_dev, unsigned long long *ctl,
                   int32_t *scratch, const LaunchArgs &la, int32_t n_plans, const pg_run_config *cfg) {
    pg::KParams P;
    std::memset(&P, 0, sizeof(P));
    P.rp = g->rp;
    P.col = g->col;
    P.ncol = (g->n_labels > 0 ? 4 : 2) * g->m;
    P.lab_off = g->lab_off;
    P.n_labels = g->n_labels;
    P.lab_copy = 2 * g->m;
    P.up = g->up;
    // bitmaps are held for ranks hub_start..n-1 (degree order); a launch may
    // use them from a later rank on, binary search below it
    int32_t hs = g->hub_start;
    if (cfg && cfg->hub_min_degree == -1) {
        hs = g->n;
    } else if (cfg && cfg->hub_min_degree > 0) {
        const auto it = std::lower_bound(g->hub_deg.begin(), g->hub_deg.end(), (int64_t)cfg->hub_min_degree);
        hs = g->hub_start + (int32_t)(it - g->hub_deg.begin());
    }
    P.hub_bits = hs < g->n ? g->hub_bits + (size_t)(hs - g->hub_start) * (size_t)g->hub_words : nullptr;
    P.hub_words = g->hub_words;
    P.hub_start = hs;
    P.lab = g->lab;
    P.perm = g->dperm;
    P.tsrc = g->tsrc;
    P.tdst = g->tdst;
    P.nodes = reinterpret_cast<const pg::Node *>(trie_dev);
    P.avs = reinterpret_cast<const pg::AVCheck *>(static_cast<const char *>(trie_dev) + L.a_off);
    P.roots = reinterpret_cast<const int32_t *>(static_cast<const char *>(trie_dev) + L.r_off);
    P.lists = reinterpret_cast<const int32_t *>(static_cast<const char *>(trie_dev) + L.x_off);
    P.cursor = ctl + kCtlCursor;
    P.counts = ctl + kCtlCounts;
    P.flags = reinterpret_cast<int32_t *>(ctl + kCtlFlags);
    P.emit_ctr = ctl + kCtlEmit;
    P.out = la.out;
    P.bytes_ctr = ctl + kCtlBytes;
    P.t_start = ctl + kCtlStart;
    P.wave_done = ctl + kCtlDoneFirst;
    P.time_budget = cfg && cfg->time_limit_ms ? (long long)cfg->time_limit_ms * g->wall_khz : 0;
    P.scratch = L.enum_levels ? scratch : nullptr;
    P.wave_stride = (long long)L.enum_levels * L.set_cap + L.arena_cap;
    P.set_cap = L.set_cap;
    P.arena_cap = L.arena_cap;
    P.n_etasks = L.n_et;
    P.n_vtasks = L.n_vt;
    P.cap = la.cap;
    P.n = g->n;
    P.n_roots = (int32_t)L.trie.roots.size();
    P.chunk = L.chunk;
    // this launch's root-task window: the call's own (enumeration windows),
    // else the run configuration's
    if (la.task_begin || la.task_end) {
        P.task_begin = la.task_begin;
        P.task_end = la.task_end;
    } else if (cfg) {
        P.task_begin = cfg->task_begin;
        P.task_end = cfg->task_end;
    }
    P.chunk_ramp = chunk_ramp((P.task_end > 0 ? P.task_end : L.n_et + L.n_vt) - P.task_begin, L.chunk);
    P.n_plans = n_plans;
    P.mode = la.mode;
    P.run_flags = cfg ? cfg->flags : 0;
    P.batch_max_avg = cfg ? cfg->batch_max_avg : 0;
    P.mark = la.mark_dev;
    P.mark_words = la.mark_words;

    return P;
}

pg_status read_ctl(const unsigned long long *ctl, int32_t n_plans, uint64_t *counts, uint64_t *emitted) {
    const int32_t *flags = reinterpret_cast<const int32_t *>(ctl + kCtlFlags);
    if (counts)
        for (int i = 0; i < n_plans; i++) counts[i] = ctl[kCtlCounts + i];
    if (emitted) *emitted = ctl[kCtlEmit];
    if (flags[2]) {
        set_error("time limit reached; counts are partial");
        return PG_ETIMEDOUT;
    }
    if (flags[0]) {
        set_error("a count exceeds 2^64 - 1");
        return PG_EOVERFLOW;
    }
    return PG_OK;
}

pg_status run(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, uint64_t *counts, const pg_run_config *cfg,
              pg_run_stats *stats, void *hip_stream, const LaunchArgs &la, uint64_t *emitted) {
    auto t_start = std::chrono::steady_clock::now();
    pg_status st = check_args(g, plans, n_plans, cfg);
    if (st) return st;
    std::lock_guard<std::mutex> lock(g->mu);
    DeviceGuard guard(g->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const bool emit = la.mode == pg::kModeEmit;

    // program trie (cached for a repeated plan list)
    std::vector<uint64_t> key;
    for (int i = 0; i < n_plans; i++) key.push_back(plans[i]->uid);
    if (!g->trie_valid || g->trie_key != key || g->trie_emit != emit) {
        std::vector<const pg::PlanImpl *> impls;
        for (int i = 0; i < n_plans; i++) impls.push_back(&plans[i]->impl);
        g->launch.trie = pg::build_trie(impls, emit);
        if ((st = check_trie(g->launch.trie))) {
            g->trie_valid = false;
            return st;
        }
        shape(g, cfg, g->launch, la.mode, la.sizes != nullptr);
        g->trie_key = key;
        g->trie_emit = emit;
        g->trie_valid = true;
    }
    LaunchPlan &L = g->launch;
    shape(g, cfg, L, la.mode, la.sizes != nullptr);  // the knobs may differ between calls
    if ((st = check_window(L, la, cfg))) return st;

    if (L.image.size() > g->trie_bytes) {
        dfree(g->trie_buf);
        g->trie_buf = nullptr;
        g->trie_bytes = 0;
        if (hipMalloc(&g->trie_buf, L.image.size()) != hipSuccess) { set_error("hipMalloc trie"); return PG_ENOMEM; }
        g->trie_bytes = L.image.size();
    }
    PG_HIP(hipMemcpyAsync(g->trie_buf, L.image.data(), L.image.size(), hipMemcpyHostToDevice, s));
    if (L.scratch_ints > g->scratch_ints) {
        dfree(g->scratch);
        g->scratch = nullptr;
        g->scratch_ints = 0;
        if (hipMalloc(reinterpret_cast<void **>(&g->scratch), L.scratch_ints * sizeof(int32_t)) != hipSuccess) {
            set_error("hipMalloc scratch");
            return PG_ENOMEM;
        }
        g->scratch_ints = L.scratch_ints;
    }
    PG_HIP(hipMemsetAsync(g->ctl, 0, kCtlWords * sizeof(unsigned long long), s));
    LaunchArgs la2 = la;
    const long long words = ((long long)g->n + 31) / 32;
    if (la.sizes) {
        // one n-bit bitmap per plan, plus its popcount
        const size_t need = (size_t)n_plans * (size_t)words;
        if (need > g->mark_cap) {
            dfree(g->marks);
            dfree(g->mark_cnt);
            g->marks = nullptr;
            g->mark_cnt = nullptr;
            g->mark_cap = 0;
            if (hipMalloc(reinterpret_cast<void **>(&g->marks), need * sizeof(uint32_t)) != hipSuccess ||
                hipMalloc(reinterpret_cast<void **>(&g->mark_cnt),
                          pg::kMaxPlansPerLaunch * sizeof(unsigned long long)) != hipSuccess) {
                set_error("hipMalloc domain bitmaps");
                return PG_ENOMEM;
            }
            g->mark_cap = need;
        }
        PG_HIP(hipMemsetAsync(g->marks, 0, need * sizeof(uint32_t), s));
        la2.mark_dev = g->marks;
        la2.mark_words = words;
    }
    const pg::KParams P = params(g, L, g->trie_buf, g->ctl, g->scratch, la2, n_plans, cfg);

    hipEvent_t e0, e1;
    PG_HIP(hipEventCreate(&e0));
    PG_HIP(hipEventCreate(&e1));
    PG_HIP(hipEventRecord(e0, s));
    hipError_t le = pg::launch_match(P, L.grid, L.variant, s);
    if (le != hipSuccess) {
        edestroy(e0);
        edestroy(e1);
        set_error(std::string("kernel launch: ") + hipGetErrorString(le));
        return PG_EDEVICE;
    }
    PG_HIP(hipEventRecord(e1, s));
    std::vector<unsigned long long> dsz;
    if (la.sizes) {
        PG_HIP(hipMemsetAsync(g->mark_cnt, 0, (size_t)n_plans * sizeof(unsigned long long), s));
        hipError_t pe = pg::launch_popcount(g->marks, words, n_plans, g->mark_cnt, s);
        if (pe != hipSuccess) {
            edestroy(e0);
            edestroy(e1);
            set_error(std::string("popcount launch: ") + hipGetErrorString(pe));
            return PG_EDEVICE;
        }
        dsz.resize(n_plans);
        PG_HIP(hipMemcpyAsync(dsz.data(), g->mark_cnt, (size_t)n_plans * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s));
    }
    unsigned long long ctl[kCtlWords];
    PG_HIP(hipMemcpyAsync(ctl, g->ctl, sizeof(ctl), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < dsz.size(); i++) la.sizes[i] = dsz[i];
    float ms = 0.f;
    PG_HIP(hipEventElapsedTime(&ms, e0, e1));
    edestroy(e0);
    edestroy(e1);
    if (stats) {
        stats->kernel_ms = ms;
        stats->total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        stats->logical_bytes = ctl[kCtlBytes];
        const long long wt = window_tasks(L, la, cfg);
        stats->root_tasks = (uint64_t)wt;
        stats->grid_waves = L.grid;
        stats->chunk = L.chunk;
        stats->tasks_started =
            (uint64_t)std::min(wt, claim_start_host((long long)ctl[kCtlCursor], L.chunk, chunk_ramp(wt, L.chunk)));
        if (cfg && (cfg->flags & PG_RUN_WAVE_TIMES)) {
            stats->wave_done_first_ms = (double)(~ctl[kCtlDoneFirst]) / (double)g->wall_khz;
            stats->wave_done_last_ms = (double)ctl[kCtlDoneLast] / (double)g->wall_khz;
        }
    }
    return read_ctl(ctl, n_plans, counts, emitted);
}

// Everything the counting kernel reads of a plan, written out: two plans
// with equal keys count the same subgraphs on every graph.
std::vector<int64_t> count_key(const pg::PlanImpl &P) {
    std::vector<int64_t> v{P.k, P.anchor, (int64_t)P.count_progs.size()};
    auto put = [&](const pg::Level &L) {
        for (uint32_t x : {L.isect, L.diff, L.lo, L.hi, L.excl, L.excl_in, L.t_isect, L.t_diff}) v.push_back(x);
        for (int32_t x : {L.base, L.label, L.group, L.pv, (int32_t)L.avs.size()}) v.push_back(x);
        for (const pg::AVCheck &c : L.avs) {
            v.push_back(c.nbr);
            v.push_back(c.label);
            for (int i = 0; i < pg::kMaxLevels; i++) v.push_back(c.xmask[i]);
        }
    };
    for (const pg::Program &pr : P.count_progs) {
        v.push_back((int64_t)pr.lev.size());
        v.push_back((int64_t)pr.factors.size());
        v.push_back((int64_t)(pr.mult >> 1));  // split: mult may exceed INT64_MAX
        v.push_back((int64_t)(pr.mult & 1u));
        for (const pg::Level &L : pr.lev) put(L);
        for (const pg::Level &L : pr.factors) put(L);
    }
    return v;
}

// The distinct plans of a call, and where each plan's count comes from.
// Different patterns can compile to the same programs (K5 and the induced
// K5: a clique has no non-adjacent pair to add an anti-edge to); such plans
// are counted once per launch.
void distinct_plans(const pg_plan *const *plans, int32_t n, std::vector<const pg_plan *> *uniq,
                    std::vector<int32_t> *from) {
    std::vector<std::vector<int64_t>> keys;
    from->assign((size_t)n, 0);
    for (int32_t i = 0; i < n; i++) {
        std::vector<int64_t> k = count_key(plans[i]->impl);
        size_t j = 0;
        while (j < keys.size() && keys[j] != k) j++;
        if (j == keys.size()) {
            keys.push_back(std::move(k));
            uniq->push_back(plans[i]);
        }
        (*from)[(size_t)i] = (int32_t)j;
    }
}

constexpr size_t kWsAlign = 256;
inline size_t align_up(size_t x) { return (x + kWsAlign - 1) & ~(kWsAlign - 1); }

// workspace layout of an asynchronous job: control words | trie image | scratch
size_t workspace_bytes(const LaunchPlan &L) {
    return align_up(kCtlWords * sizeof(unsigned long long)) + align_up(L.image.size()) +
           L.scratch_ints * sizeof(int32_t);
}

}  // namespace

extern "C" {

pg_status pg_count_ex(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, uint64_t *counts,
                      const pg_run_config *cfg, pg_run_stats *stats, void *hip_stream) {
    if (!counts) { set_error("counts is NULL"); return PG_EINVAL; }
    try {
        pg_status st = check_args(g, plans, n_plans, cfg);
        if (st) return st;
        std::vector<const pg_plan *> uniq;
        std::vector<int32_t> from;
        distinct_plans(plans, n_plans, &uniq, &from);
        if ((int32_t)uniq.size() == n_plans)
            return run(g, plans, n_plans, counts, cfg, stats, hip_stream, LaunchArgs{}, nullptr);
        std::vector<uint64_t> c(uniq.size(), 0);
        st = run(g, uniq.data(), (int32_t)uniq.size(), c.data(), cfg, stats, hip_stream, LaunchArgs{}, nullptr);
        if (st == PG_OK || st == PG_ETIMEDOUT || st == PG_EOVERFLOW)
            for (int32_t i = 0; i < n_plans; i++) counts[i] = c[(size_t)from[(size_t)i]];
        return st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PG_ENOMEM;
    }
}

pg_status pg_count_noalloc(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, uint64_t *counts,
                           const pg_run_config *cfg, void *hip_stream) {
    if (!counts) { set_error("counts is NULL"); return PG_EINVAL; }
    try {
        pg_status st = check_args(g, plans, n_plans, cfg);
        if (st) return st;
        DeviceGuard guard(g->device);
        hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
        LaunchPlan L;
        std::vector<const pg::PlanImpl *> impls;
        for (int i = 0; i < n_plans; i++) impls.push_back(&plans[i]->impl);
        L.trie = pg::build_trie(impls, false);
        if ((st = check_trie(L.trie))) return st;
        shape(g, cfg, L, pg::kModeCount, false);
        if ((st = check_window(L, LaunchArgs{}, cfg))) return st;
        void *base = nullptr;
        size_t cap = 0;
        PG_HIP(pg::static_scratch(&base, &cap));
        // [control block | trie | scratch of as many wavefronts as fit]
        const size_t ctl_b = align_up(kCtlWords * sizeof(unsigned long long)), trie_b = align_up(L.image.size());
        if (ctl_b + trie_b > cap) {
            set_error("the program trie (" + std::to_string(L.image.size()) + " bytes) does not fit the fixed " +
                      std::to_string(cap >> 20) + " MiB device array");
            return PG_ENOMEM;
        }
        const size_t per_wave = ((size_t)L.enum_levels * (size_t)L.set_cap + (size_t)L.arena_cap) * sizeof(int32_t);
        if (per_wave > 0) {
            const size_t fit = (cap - ctl_b - trie_b) / per_wave;
            if (fit < 1) {
                set_error("one wavefront's scratch (" + std::to_string(per_wave) + " bytes for " +
                          std::to_string(L.enum_levels) + " levels of up to " + std::to_string(L.set_cap) +
                          " vertices) exceeds the fixed " + std::to_string(cap >> 20) + " MiB device array");
                return PG_ENOMEM;
            }
            if ((size_t)L.grid > fit) L.grid = (int)fit;
        }
        char *ctl = static_cast<char *>(base);
        char *trie = ctl + ctl_b;
        int32_t *scratch = reinterpret_cast<int32_t *>(trie + trie_b);
        unsigned long long *c = reinterpret_cast<unsigned long long *>(ctl);
        PG_HIP(hipMemcpyAsync(trie, L.image.data(), L.image.size(), hipMemcpyHostToDevice, s));
        PG_HIP(pg::launch_zero(c, kCtlWords, s));
        const pg::KParams P = params(g, L, trie, c, scratch, LaunchArgs{}, n_plans, cfg);
        PG_HIP(pg::launch_match(P, L.grid, L.variant, s));
        unsigned long long h[kCtlWords];
        PG_HIP(hipMemcpyAsync(h, c, sizeof(h), hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
        return read_ctl(h, n_plans, counts, nullptr);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PG_ENOMEM;
    }
}

pg_status pg_count(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, uint64_t *counts, void *hip_stream) {
    return pg_count_ex(g, plans, n_plans, counts, nullptr, nullptr, hip_stream);
}

pg_status pg_exists(pg_graph *g, const pg_plan *plan, int32_t *found, void *hip_stream) {
    if (!found || !plan) { set_error("NULL argument"); return PG_EINVAL; }
    LaunchArgs la;
    la.mode = pg::kModeExists;
    uint64_t c = 0;
    const pg_plan *plans[1] = {plan};
    pg_run_config cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    cfg.chunk = 1;
    try {
        pg_status st = run(g, plans, 1, &c, &cfg, nullptr, hip_stream, la, nullptr);
        if (st == PG_EOVERFLOW) st = PG_OK;  // partial sums may wrap once a match is found
        if (st) return st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PG_ENOMEM;
    }
    *found = c > 0 ? 1 : 0;
    return PG_OK;
}

pg_status pg_domain_sizes(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, uint64_t *sizes,
                          const pg_run_config *cfg, void *hip_stream) {
    if (!sizes) { set_error("sizes is NULL"); return PG_EINVAL; }
    if (plans && n_plans > 0)
        for (int i = 0; i < n_plans && i < pg::kMaxPlansPerLaunch; i++)
            if (plans[i] && plans[i]->impl.anchor < 0) {
                set_error("every plan must be anchored (pg_plan_options.anchored)");
                return PG_EINVAL;
            }
    LaunchArgs la;
    la.sizes = sizes;
    std::vector<uint64_t> c((size_t)std::max(0, n_plans));
    try {
        pg_status st = run(g, plans, n_plans, c.data(), cfg, nullptr, hip_stream, la, nullptr);
        if (st) return st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PG_ENOMEM;
    }
    return PG_OK;
}

pg_status pg_enumerate(pg_graph *g, const pg_plan *plan, int32_t *out, uint64_t cap, uint64_t *n_total,
                       void *hip_stream) {
    if (!plan || !n_total) { set_error("NULL argument"); return PG_EINVAL; }
    if (cap > 0 && !out) { set_error("out is NULL with cap > 0"); return PG_EINVAL; }
    LaunchArgs la;
    la.mode = pg::kModeEmit;
    la.out = out;
    la.cap = cap;
    const pg_plan *plans[1] = {plan};
    try {
        return run(g, plans, 1, nullptr, nullptr, nullptr, hip_stream, la, n_total);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PG_ENOMEM;
    }
}

pg_status pg_root_tasks(pg_graph *g, const pg_plan *plan, int64_t *n_tasks) {
    if (!g || !plan || !n_tasks) { set_error("NULL argument"); return PG_EINVAL; }
    try {
        std::vector<const pg::PlanImpl *> impls{&plan->impl};
        const pg::Trie T = pg::build_trie(impls, true);
        *n_tasks = (T.has_edge_root ? g->m : 0) + (T.has_vertex_root ? (int64_t)g->n : 0);
        return PG_OK;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PG_ENOMEM;
    }
}

pg_status pg_launch_tasks(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, int64_t *n_tasks) {
    if (!n_tasks) { set_error("n_tasks is NULL"); return PG_EINVAL; }
    pg_status st = check_args(g, plans, n_plans, nullptr);
    if (st) return st;
    try {
        std::vector<const pg::PlanImpl *> impls;
        for (int i = 0; i < n_plans; i++) impls.push_back(&plans[i]->impl);
        const pg::Trie T = pg::build_trie(impls, false);
        *n_tasks = (T.has_edge_root ? g->m : 0) + (T.has_vertex_root ? (int64_t)g->n : 0);
        return PG_OK;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PG_ENOMEM;
    }
}

pg_status pg_enumerate_range(pg_graph *g, const pg_plan *plan, int64_t task_begin, int64_t task_end, int32_t *out,
                             uint64_t cap, uint64_t *n_total, void *hip_stream) {
    if (!plan || !n_total) { set_error("NULL argument"); return PG_EINVAL; }
    if (cap > 0 && !out) { set_error("out is NULL with cap > 0"); return PG_EINVAL; }
    if (task_end <= task_begin || task_begin < 0) { set_error("bad root-task window"); return PG_EINVAL; }
    LaunchArgs la;
    la.mode = pg::kModeEmit;
    la.out = out;
    la.cap = cap;
    la.task_begin = task_begin;
    la.task_end = task_end;
    const pg_plan *plans[1] = {plan};
    try {
        return run(g, plans, 1, nullptr, nullptr, nullptr, hip_stream, la, n_total);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PG_ENOMEM;
    }
}

// Streams the matches through one device buffer: windows of root tasks are
// enumerated one after another (every match is found from exactly one root
// task), a window whose matches overflow the buffer is halved and redone,
// and the callback sees each window's rows before the next launch.
pg_status pg_match(pg_graph *g, const pg_plan *plan, pg_match_cb cb, void *user, uint64_t *n_matches) {
    return pg_match_ex(g, plan, cb, user, n_matches, 0);
}

pg_status pg_match_ex(pg_graph *g, const pg_plan *plan, pg_match_cb cb, void *user, uint64_t *n_matches,
                      uint64_t buffer_rows) {
    if (!g || !plan || !cb) { set_error("NULL argument"); return PG_EINVAL; }
    if (n_matches) *n_matches = 0;
    int64_t total = 0;
    pg_status st = pg_root_tasks(g, plan, &total);
    if (st) return st;
    if (total == 0) return PG_OK;
    const int k = plan->impl.k;
    const uint64_t kMaxRows = (uint64_t)1 << 26;
    uint64_t cap = buffer_rows ? buffer_rows
                               : std::max<uint64_t>((uint64_t)1 << 16, ((uint64_t)64 << 20) / (4u * (uint64_t)k));
    DeviceGuard guard(g->device);
    int32_t *d = nullptr;
    auto grow = [&](uint64_t rows) -> pg_status {
        dfree(d);
        d = nullptr;
        if (hipMalloc(reinterpret_cast<void **>(&d), rows * (uint64_t)k * sizeof(int32_t)) != hipSuccess) {
            set_error("hipMalloc match rows");
            return PG_ENOMEM;
        }
        cap = rows;
        return PG_OK;
    };
    if ((st = grow(cap))) return st;
    std::vector<int32_t> h;
    int64_t begin = 0, width = total;
    while (begin < total) {
        const int64_t end = std::min(total, begin + width);
        uint64_t got = 0;
        st = pg_enumerate_range(g, plan, begin, end, d, cap, &got, nullptr);
        if (st) break;
        if (got > cap) {
            if (end - begin > 1) {
                // too many for the buffer: a narrower window, sized from this one
                width = std::max<int64_t>(1, (int64_t)((double)(end - begin) * (double)cap / (2.0 * (double)got)));
                continue;
            }
            if (got > kMaxRows) {
                set_error("one root task yields more matches than the callback form buffers");
                st = PG_EUNSUPPORTED;
                break;
            }
            if ((st = grow(got))) break;
            continue;
        }
        h.resize(got * (uint64_t)k);
        if (got && hipMemcpy(h.data(), d, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
            set_error("copy of match rows failed");
            st = PG_EDEVICE;
            break;
        }
        bool stop = false;
        for (uint64_t i = 0; i < got && !stop; i++) {
            if (n_matches) (*n_matches)++;
            if (cb(h.data() + i * (uint64_t)k, k, user)) stop = true;
        }
        if (stop) {
            st = PG_STOPPED;
            break;
        }
        begin = end;
        // widen again while windows come back well under the buffer
        if (got < cap / 4) width = std::min<int64_t>(total, width * 2);
    }
    dfree(d);
    return st;
}

// ----------------------------------------------------------- asynchronous jobs

static pg_status prepare_job(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, int32_t mode,
                             const pg_run_config *cfg, LaunchPlan *L) {
    pg_status st = check_args(g, plans, n_plans, cfg);
    if (st) return st;
    if (mode != PG_JOB_COUNT && mode != PG_JOB_EXISTS) { set_error("unknown job mode"); return PG_EINVAL; }
    if (mode == PG_JOB_EXISTS && n_plans != 1) { set_error("an existence job takes one plan"); return PG_EINVAL; }
    std::vector<const pg::PlanImpl *> impls;
    for (int i = 0; i < n_plans; i++) impls.push_back(&plans[i]->impl);
    L->trie = pg::build_trie(impls, false);
    if ((st = check_trie(L->trie))) return st;
    pg_run_config c;
    std::memset(&c, 0, sizeof(c));
    if (cfg) c = *cfg;
    if (mode == PG_JOB_EXISTS && !c.chunk) c.chunk = 1;  // poll the stop flag often
    shape(g, &c, *L, mode == PG_JOB_EXISTS ? pg::kModeExists : pg::kModeCount, false);
    return check_window(*L, LaunchArgs{}, cfg);
}

pg_status pg_job_workspace_size(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, int32_t mode,
                                const pg_run_config *cfg, uint64_t *bytes) {
    if (!bytes) { set_error("bytes is NULL"); return PG_EINVAL; }
    try {
        LaunchPlan L;
        pg_status st = prepare_job(g, plans, n_plans, mode, cfg, &L);
        if (st) return st;
        *bytes = workspace_bytes(L);
        return PG_OK;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PG_ENOMEM;
    }
}

pg_status pg_submit(pg_graph *g, const pg_plan *const *plans, int32_t n_plans, int32_t mode,
                    const pg_run_config *cfg, void *workspace, uint64_t workspace_bytes_, void *hip_stream,
                    pg_job **out) {
    if (!out) { set_error("out is NULL"); return PG_EINVAL; }
    *out = nullptr;
    try {
        std::unique_ptr<pg_job> j(new pg_job());
        pg_status st = prepare_job(g, plans, n_plans, mode, cfg, &j->L);
        if (st) return st;
        const uint64_t need = workspace_bytes(j->L);
        if (!workspace || workspace_bytes_ < need) {
            set_error("workspace too small: need " + std::to_string(need) + " bytes");
            return PG_ENOMEM;
        }
        if (reinterpret_cast<uintptr_t>(workspace) % kWsAlign) {
            set_error("workspace must be 256-byte aligned");
            return PG_EINVAL;
        }
        DeviceGuard guard(g->device);
        j->g = g;
        {
            std::lock_guard<std::mutex> lock(g->job_mu);
            if (!g->ctl_host) {
                void *h = nullptr;
                PG_HIP(hipHostMalloc(&h, (size_t)kJobSlots * kCtlWords * sizeof(unsigned long long),
                                     hipHostMallocDefault));
                g->ctl_host = static_cast<unsigned long long *>(h);
                for (int i = kJobSlots - 1; i >= 0; i--) g->ctl_free.push_back(i);
            }
            if (g->ctl_free.empty()) {
                set_error("too many jobs in flight on this graph (64)");
                return PG_ENOMEM;
            }
            j->ctl_slot = g->ctl_free.back();
            g->ctl_free.pop_back();
        }
        j->n_plans = n_plans;
        j->mode = mode;
        j->tasks = window_tasks(j->L, LaunchArgs{}, cfg);
        j->s = reinterpret_cast<hipStream_t>(hip_stream);
        j->t_submit = std::chrono::steady_clock::now();
        char *base = static_cast<char *>(workspace);
        j->ctl = reinterpret_cast<unsigned long long *>(base);
        char *trie = base + align_up(kCtlWords * sizeof(unsigned long long));
        int32_t *scratch = reinterpret_cast<int32_t *>(trie + align_up(j->L.image.size()));
        j->enqueued = true;
        PG_HIP(hipMemcpyAsync(trie, j->L.image.data(), j->L.image.size(), hipMemcpyHostToDevice, j->s));
        PG_HIP(hipMemsetAsync(j->ctl, 0, kCtlWords * sizeof(unsigned long long), j->s));
        LaunchArgs la;
        la.mode = mode == PG_JOB_EXISTS ? pg::kModeExists : pg::kModeCount;
        const pg::KParams P = params(g, j->L, trie, j->ctl, scratch, la, n_plans, cfg);
        PG_HIP(hipEventCreate(&j->e0));
        PG_HIP(hipEventCreate(&j->ek));
        PG_HIP(hipEventCreate(&j->e1));
        PG_HIP(hipEventRecord(j->e0, j->s));
        hipError_t le = pg::launch_match(P, j->L.grid, j->L.variant, j->s);
        if (le != hipSuccess) {
            set_error(std::string("kernel launch: ") + hipGetErrorString(le));
            return PG_EDEVICE;
        }
        PG_HIP(hipEventRecord(j->ek, j->s));
        PG_HIP(hipMemcpyAsync(g->ctl_host + (size_t)j->ctl_slot * kCtlWords, j->ctl,
                              kCtlWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, j->s));
        PG_HIP(hipEventRecord(j->e1, j->s));
        *out = j.release();
        return PG_OK;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return PG_ENOMEM;
    }
}

pg_status pg_job_poll(pg_job *j, int32_t *done) {
    if (!j || !done) { set_error("NULL argument"); return PG_EINVAL; }
    DeviceGuard guard(j->g->device);
    hipError_t e = hipEventQuery(j->e1);
    if (e == hipSuccess) *done = 1;
    else if (e == hipErrorNotReady) *done = 0;
    else {
        set_error(std::string("hipEventQuery: ") + hipGetErrorString(e));
        return PG_EDEVICE;
    }
    return PG_OK;
}

pg_status pg_job_finish(pg_job *j, uint64_t *counts, pg_run_stats *stats) {
    if (!j) { set_error("NULL job"); return PG_EINVAL; }
    std::unique_ptr<pg_job> own(j);
    DeviceGuard guard(j->g->device);
    PG_HIP(hipEventSynchronize(j->e1));
    j->enqueued = false;
    const unsigned long long *ctl = j->g->ctl_host + (size_t)j->ctl_slot * kCtlWords;
    float ms = 0.f;
    PG_HIP(hipEventElapsedTime(&ms, j->e0, j->ek));
    if (stats) {
        stats->kernel_ms = ms;
        stats->total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - j->t_submit).count();
        stats->logical_bytes = ctl[kCtlBytes];
        stats->root_tasks = (uint64_t)j->tasks;
        stats->grid_waves = j->L.grid;
        stats->chunk = j->L.chunk;
        stats->tasks_started = (uint64_t)std::min(
            j->tasks, claim_start_host((long long)ctl[kCtlCursor], j->L.chunk, chunk_ramp(j->tasks, j->L.chunk)));
    }
    if (j->mode == PG_JOB_EXISTS) {
        // partial sums of an early-stopped search may wrap; only > 0 matters
        const int32_t *flags = reinterpret_cast<const int32_t *>(ctl + kCtlFlags);
        if (flags[2] && ctl[kCtlCounts] == 0) {
            set_error("time limit reached before a match was found");
            return PG_ETIMEDOUT;
        }
        if (counts) counts[0] = ctl[kCtlCounts] > 0 ? 1 : 0;
        return PG_OK;
    }
    return read_ctl(ctl, j->n_plans, counts, nullptr);
}

}  // extern "C"
