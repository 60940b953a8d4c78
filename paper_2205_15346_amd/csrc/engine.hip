// Host side of batched and served evolution (te_engine_*, te_batch_* in include/te.h).
//
// An engine holds a pool of device memory for job workspaces, a table of job slots (device
// solver states) and at most two round plans.  A plan is the resident set of one stretch of
// rounds: the jobs' views, their grouping by Hamiltonian (multi-vector sparse products), the
// (group, tile) and (job, tile) work lists of the batched kernels, and the hipGraph of one
// round.  The scheduler keeps up to two rounds queued on the device, waits for the older one,
// reads the per-round job records the device wrote into mapped host memory, retires completed
// jobs and, at that round boundary, admits queued jobs that fit (slot free, footprint fits the
// pool) by building the next plan.  Every decision of the method itself is taken on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "pool.h"
#include "te_internal.h"

using namespace te;

namespace {

constexpr int kRing = 4;        // round events in the ring
constexpr int kDepth = 2;       // rounds on the device at once (one queued behind the running one)
constexpr int kTileRows = kBlock;  // rows per tile of the multi-vector product
constexpr int kMaxEngineJobs = 16384;
const int kClasses[4] = {1, 2, 4, 8};

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int nv_class_index(int nv) { return nv <= 1 ? 0 : nv <= 2 ? 1 : nv <= 4 ? 2 : 3; }

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// device workspace of one job inside the pool
struct JobLayout {
    uint64_t v, y, part, npart, red, total;
};

JobLayout job_layout(int dim, int m) {
    JobLayout L{};
    const uint64_t ld = basis_ld(dim);
    const uint64_t tiles = (uint64_t)ceil_div(dim, kTileRows);
    uint64_t o = 0;
    L.v = o;
    o += (uint64_t)m * ld * sizeof(double2);
    o = align_up(o, 256);
    L.y = o;
    o += ld * sizeof(double2);
    o = align_up(o, 256);
    L.part = o;
    o += (uint64_t)kMaxVals * tiles * sizeof(double2);
    o = align_up(o, 256);
    L.npart = o;
    o += tiles * sizeof(double);
    o = align_up(o, 256);
    L.red = o;
    o += (uint64_t)kMaxVals * sizeof(double2);
    L.total = align_up(o, 256);
    return L;
}

struct JobRec {
    te_job id = 0;
    te_hamiltonian h = nullptr;
    const double2* v0 = nullptr;
    double2* out = nullptr;
    double t = 0.0, tol = 0.0;
    int m = 0, dim = 0;
    int state = TE_JOB_QUEUED;
    te_status status = TE_OK;
    te_result res{};
    double t_sub = 0.0, t_adm = 0.0, t_fin = 0.0;
    int64_t round_adm = 0;
    int rounds = 0, steps = 0;
    double t_now = 0.0;
    int slot = -1;
    uint64_t off = 0, bytes = 0;
    bool fresh = false;  // admitted, set-up work not yet enqueued
};

struct Plan {
    char* dev = nullptr;
    size_t dev_cap = 0;
    char* host = nullptr;  // pinned staging of the device arrays
    size_t host_cap = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t last_use = nullptr;
    bool used = false;
    // device views
    JobView* jobs = nullptr;
    GroupView* groups = nullptr;
    int2* pitems[4] = {nullptr, nullptr, nullptr, nullptr};
    int n_pitems[4] = {0, 0, 0, 0};
    int2* uitems = nullptr;
    int n_uitems = 0;
    int2* ditems = nullptr;  // (job, tile) projections of jobs in groups of two or more
    int n_ditems = 0;
    JobView* new_jobs = nullptr;
    Problem* probs = nullptr;
    int2* new_items = nullptr;
    int n_new = 0, n_new_items = 0;
    int n_jobs = 0, n_groups = 0, rpt_u = 1, m = 0;
    std::vector<te_job> job_ids;               // JobView order
    std::vector<std::vector<int>> group_jobs;  // plan job indices per group
    int64_t weight = 0;                        // rows of all jobs (retirement threshold)
    int64_t retired_weight = 0;

    void release_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

}  // namespace

struct te_engine_s {
    te_engine_config cfg{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    char* pool_base = nullptr;
    PoolAlloc pool;
    DevState* states = nullptr;
    int* rounds_dev = nullptr;
    SlotOut* slots_host = nullptr;  // [2][max_jobs], mapped
    SlotOut* slots_dev = nullptr;
    RoundOut* ro_host = nullptr;
    RoundOut* ro_dev = nullptr;
    Plan plans[2];
    int cur = -1;
    int64_t n_plans = 0;
    hipEvent_t ev[kRing] = {};
    std::vector<hipEvent_t> pev;  // profiling: one event per kernel class boundary
    int64_t launched = 0, observed = 0;
    std::vector<int> free_slots;
    std::deque<JobRec> jobs;  // by id
    std::deque<te_job> queue;
    std::vector<te_job> resident;
    bool tuned = false;
    te_tuning tuning{4, 4, 2, 2, 0, 0.0};
    te_profile prof{};
    double busy = 0.0, busy_since = -1.0;
    te_status err = TE_OK;
    std::string err_msg;
    bool need_plan = false;
    int64_t done_count = 0, failed_count = 0;
    // threading
    std::mutex mu;        // job table, queue, counters
    std::mutex sched_mu;  // one scheduler at a time
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    // two lanes (cfg.lane_rows > 0): this engine only routes; lane[0] takes jobs below lane_rows
    // rows, lane[1] the others; route[id] = (lane, id in that lane)
    te_engine_s* lane[2] = {nullptr, nullptr};
    std::vector<std::pair<int, te_job>> route;

    ~te_engine_s();
};

namespace {

te_status hip_fail(hipError_t e, const char* what) {
    return set_error(e == hipErrorOutOfMemory ? TE_ERR_OUT_OF_MEMORY : TE_ERR_DEVICE,
                     std::string(what) + ": " + hipGetErrorString(e));
}

#define EHIP(call)                                       \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

bool profiling(const te_engine_s* e) { return (e->cfg.flags & TE_ENGINE_PROFILE) != 0; }

JobView job_view(te_engine_s* e, const JobRec& j, int rpt_u) {
    const JobLayout L = job_layout(j.dim, j.m);
    char* base = e->pool_base + j.off;
    JobView v{};
    v.rp = j.h->csr.row_ptr;
    v.ci = j.h->csr.col;
    v.val = j.h->csr.val;
    v.rval = j.h->csr.rval;
    v.pk = j.h->csr.pk;
    v.V = (double2*)(base + L.v);
    v.y = (double2*)(base + L.y);
    v.st = e->states + j.slot;
    v.rb.part = (double2*)(base + L.part);
    v.rb.npart = (double*)(base + L.npart);
    v.rb.red = (double2*)(base + L.red);
    v.rb.n_tiles = (int)ceil_div(j.dim, (int64_t)kBlock * e->tuning.rows_per_thread);
    v.rb.n_norm = (int)ceil_div(j.dim, (int64_t)kBlock * rpt_u);
    v.v0 = j.v0;
    v.out = j.out;
    v.ld = (int64_t)basis_ld(j.dim);
    v.id = j.id;
    v.dim = j.dim;
    v.slot = j.slot;
    return v;
}

// Enqueues one round of the plan on stream s: for every Krylov iteration the grouped
// projections (one launch per group-size class), the fold and the update; then the step
// kernel, the recombination, the output of completed jobs and the round records.  With
// events (profiling), E receives 3m + 3 boundaries.
hipError_t enqueue_round(te_engine_s* e, const Plan& p, hipStream_t s, std::vector<hipEvent_t>* E) {
    hipError_t r = hipSuccess;
    auto mark = [&](size_t i) {
        if (E && r == hipSuccess) r = hipEventRecord((*E)[i], s);
    };
    const te_tuning& t = e->tuning;
    mark(0);
    for (int j = 0; j < p.m && r == hipSuccess; ++j) {
        for (int c = 0; c < 4 && r == hipSuccess; ++c)
            r = launch_gproject(t.lanes_per_row, t.nnz_per_lane, t.rows_per_thread, kClasses[c], p.jobs, p.groups,
                                p.pitems[c], p.n_pitems[c], j, s);
        if (r == hipSuccess) r = launch_bdots(t.rows_per_thread, p.jobs, p.ditems, p.n_ditems, j, s);
        mark(3 * j + 1);
        if (r == hipSuccess) r = launch_bfold(p.jobs, p.n_jobs, j, s);
        mark(3 * j + 2);
        if (r == hipSuccess) r = launch_bupdate(p.rpt_u, p.jobs, p.uitems, p.n_uitems, j, s);
        mark(3 * j + 3);
    }
    if (r == hipSuccess) r = launch_bstep(p.jobs, p.n_jobs, s);
    mark(3 * p.m + 1);
    if (r == hipSuccess) r = launch_bcombine(p.rpt_u, p.jobs, p.uitems, p.n_uitems, s);
    if (r == hipSuccess) r = launch_bcopy_out(p.rpt_u, p.jobs, p.uitems, p.n_uitems, s);
    if (r == hipSuccess)
        r = launch_bflag(p.jobs, p.n_jobs, e->rounds_dev, e->slots_dev, e->cfg.max_jobs, e->ro_dev, s);
    mark(3 * p.m + 2);
    return r;
}

// Times every supported projection shape on plan p (iteration m/2) and keeps the
// fastest.  Runs after the set-up of p's jobs and before their initial vectors are copied in:
// it only writes the product vectors and partials, which the first round overwrites.
te_status autotune(te_engine_s* e, const Plan& p) {
    const int J = std::min(p.m / 2, p.m - 1);  // mid-restart: the mean cost over j = 0..m-1
    const int shapes[4][2] = {{4, 1}, {4, 4}, {8, 2}, {1, 8}};
    hipEvent_t e0, e1;
    EHIP(hipEventCreate(&e0));
    EHIP(hipEventCreate(&e1));
    double best = 1e30;
    te_tuning bt = e->tuning;
    hipError_t r = hipSuccess;
    for (const auto& sh : shapes) {
        auto launch_all = [&]() {
            for (int c = 0; c < 4 && r == hipSuccess; ++c)
                r = launch_gproject(sh[0], sh[1], e->tuning.rows_per_thread, kClasses[c], p.jobs, p.groups,
                                    p.pitems[c], p.n_pitems[c], J, e->stream);
            if (r == hipSuccess) r = launch_bdots(e->tuning.rows_per_thread, p.jobs, p.ditems, p.n_ditems, J, e->stream);
        };
        launch_all();
        if (r == hipSuccess) r = hipEventRecord(e0, e->stream);
        for (int q = 0; q < 3 && r == hipSuccess; ++q) launch_all();
        if (r == hipSuccess) r = hipEventRecord(e1, e->stream);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        float ms = 0.f;
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
        if (r != hipSuccess) break;
        const double us = 1e3 * ms / 3.0;
        if (us < best) {
            best = us;
            bt.lanes_per_row = sh[0];
            bt.nnz_per_lane = sh[1];
            bt.project_us = us;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != hipSuccess) return hip_fail(r, "engine autotune");
    e->tuning.lanes_per_row = bt.lanes_per_row;
    e->tuning.nnz_per_lane = bt.nnz_per_lane;
    e->tuning.project_us = bt.project_us;
    e->tuned = true;
    return TE_OK;
}

te_status ensure_plan_buffers(Plan& p, size_t bytes) {
    if (p.dev_cap < bytes) {
        dev_free(p.dev);
        p.dev = (char*)dev_alloc(bytes);
        p.dev_cap = p.dev ? bytes : 0;
        if (!p.dev) return set_error(TE_ERR_OUT_OF_MEMORY, "plan buffer allocation failed");
    }
    if (p.host_cap < bytes) {
        if (p.host) (void)hipHostFree(p.host);
        p.host = nullptr;
        p.host_cap = 0;
        EHIP(hipHostMalloc((void**)&p.host, bytes, hipHostMallocDefault));
        p.host_cap = bytes;
    }
    if (!p.last_use) EHIP(hipEventCreateWithFlags(&p.last_use, hipEventDisableTiming));
    return TE_OK;
}

// Admits queued jobs in submission order while a slot is free and the footprint fits.
// Called with e->mu held.
void admit(te_engine_s* e) {
    while (!e->queue.empty() && !e->free_slots.empty()) {
        JobRec& j = e->jobs[(size_t)e->queue.front()];
        uint64_t off = 0;
        if (!e->pool.alloc(j.bytes, &off)) break;
        e->queue.pop_front();
        j.off = off;
        j.slot = e->free_slots.back();
        e->free_slots.pop_back();
        j.state = TE_JOB_RUNNING;
        j.t_adm = now_s();
        j.round_adm = e->observed;
        j.fresh = true;
        e->resident.push_back(j.id);
    }
}

// Builds the plan of the resident set into the buffer not used by the current plan,
// enqueues the set-up of freshly admitted jobs and captures the round graph.  e->mu held.
te_status build_plan(te_engine_s* e) {
    admit(e);
    const int pi = (e->cur < 0) ? 0 : 1 - e->cur;
    Plan& p = e->plans[pi];
    if (p.used) EHIP(hipEventSynchronize(p.last_use));  // no queued round still reads it
    p.release_graph();
    p.used = false;

    // group the resident jobs by Hamiltonian (up to kMaxGroup per group), larger first
    std::vector<te_job> ids = e->resident;
    std::stable_sort(ids.begin(), ids.end(), [&](te_job a, te_job b) {
        const JobRec& x = e->jobs[(size_t)a];
        const JobRec& y = e->jobs[(size_t)b];
        if (x.dim != y.dim) return x.dim > y.dim;
        if (x.h != y.h) return std::less<const void*>()(x.h, y.h);
        return a < b;
    });
    int max_dim = 0;
    for (te_job id : ids) max_dim = std::max(max_dim, e->jobs[(size_t)id].dim);
    const int rpt_u = e->tuning.update_rows_per_thread;
    const int rpt_p = e->tuning.rows_per_thread;
    (void)max_dim;

    p.job_ids = ids;
    p.group_jobs.clear();
    p.n_jobs = (int)ids.size();
    p.rpt_u = rpt_u;
    p.m = 0;
    p.weight = 0;
    p.retired_weight = 0;
    for (size_t i = 0; i < ids.size();) {
        size_t k = i + 1;
        while (k < ids.size() && k - i < (size_t)kMaxGroup && e->jobs[(size_t)ids[k]].h == e->jobs[(size_t)ids[i]].h)
            ++k;
        std::vector<int> g;
        for (size_t q = i; q < k; ++q) g.push_back((int)q);
        p.group_jobs.push_back(g);
        i = k;
    }
    p.n_groups = (int)p.group_jobs.size();
    int n_new = 0;
    int64_t n_items_c[4] = {0, 0, 0, 0}, n_u = 0, n_new_items = 0, n_d = 0;
    for (const auto& g : p.group_jobs) {
        const JobRec& j0 = e->jobs[(size_t)ids[(size_t)g[0]]];
        const int64_t ptiles = ceil_div(j0.dim, (int64_t)kBlock * rpt_p);  // projection tiles
        if (g.size() == 1) {
            n_items_c[0] += ptiles;
        } else {
            n_items_c[nv_class_index((int)g.size())] += ceil_div(j0.dim, kTileRows);
            n_d += ptiles * (int64_t)g.size();
        }
    }
    for (te_job id : ids) {
        const JobRec& j = e->jobs[(size_t)id];
        p.m = std::max(p.m, j.m);
        p.weight += j.dim;
        n_u += ceil_div(j.dim, (int64_t)kBlock * rpt_u);
        if (j.fresh) {
            ++n_new;
            n_new_items += ceil_div(j.dim, (int64_t)kBlock * rpt_u);
        }
    }
    const int64_t n_p = n_items_c[0] + n_items_c[1] + n_items_c[2] + n_items_c[3];
    if (n_p >= ((int64_t)1 << 31) / kBlock || n_u >= ((int64_t)1 << 31) / kBlock || n_d >= ((int64_t)1 << 31) / kBlock)
        return set_error(TE_ERR_CAPACITY, "round work list too long");

    // layout of the plan buffer
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    const size_t o_jobs = take(sizeof(JobView) * std::max(p.n_jobs, 1));
    const size_t o_groups = take(sizeof(GroupView) * std::max(p.n_groups, 1));
    size_t o_p[4];
    for (int c = 0; c < 4; ++c) o_p[c] = take(sizeof(int2) * std::max<int64_t>(n_items_c[c], 1));
    const size_t o_u = take(sizeof(int2) * std::max<int64_t>(n_u, 1));
    const size_t o_d = take(sizeof(int2) * std::max<int64_t>(n_d, 1));
    const size_t o_nj = take(sizeof(JobView) * std::max(n_new, 1));
    const size_t o_pr = take(sizeof(Problem) * std::max(n_new, 1));
    const size_t o_ni = take(sizeof(int2) * std::max<int64_t>(n_new_items, 1));
    const size_t total = o;
    te_status rc = ensure_plan_buffers(p, total);
    if (rc != TE_OK) return rc;

    char* H = p.host;
    JobView* hj = (JobView*)(H + o_jobs);
    GroupView* hg = (GroupView*)(H + o_groups);
    int2* hp[4];
    for (int c = 0; c < 4; ++c) hp[c] = (int2*)(H + o_p[c]);
    int2* hu = (int2*)(H + o_u);
    int2* hd = (int2*)(H + o_d);
    JobView* hnj = (JobView*)(H + o_nj);
    Problem* hpr = (Problem*)(H + o_pr);
    int2* hni = (int2*)(H + o_ni);

    for (int i = 0; i < p.n_jobs; ++i) hj[i] = job_view(e, e->jobs[(size_t)ids[(size_t)i]], rpt_u);
    int fill_c[4] = {0, 0, 0, 0};
    int fill_d = 0;
    for (int gi = 0; gi < p.n_groups; ++gi) {
        const auto& g = p.group_jobs[(size_t)gi];
        const JobRec& j0 = e->jobs[(size_t)ids[(size_t)g[0]]];
        GroupView gv{};
        gv.rp = j0.h->csr.row_ptr;
        gv.ci = j0.h->csr.col;
        gv.val = j0.h->csr.val;
        gv.rval = j0.h->csr.rval;
        gv.pk = j0.h->csr.pk;
        gv.dim = j0.dim;
        gv.nv = (int)g.size();
        for (int q = 0; q < kMaxGroup; ++q) gv.job[q] = q < gv.nv ? g[(size_t)q] : 0;
        hg[gi] = gv;
        const int c = nv_class_index(gv.nv);
        const int ptiles = (int)ceil_div(j0.dim, (int64_t)kBlock * rpt_p);
        if (gv.nv == 1) {
            for (int t = 0; t < ptiles; ++t) hp[0][fill_c[0]++] = make_int2(gi, t);
        } else {
            const int tiles = (int)ceil_div(j0.dim, kTileRows);
            for (int t = 0; t < tiles; ++t) hp[c][fill_c[c]++] = make_int2(gi, t);
            for (int t = 0; t < ptiles; ++t)
                for (int q = 0; q < gv.nv; ++q) hd[fill_d++] = make_int2(g[(size_t)q], t);
        }
    }
    int fu = 0, fn = 0, fni = 0;
    for (int i = 0; i < p.n_jobs; ++i) {
        JobRec& j = e->jobs[(size_t)ids[(size_t)i]];
        const int tiles = (int)ceil_div(j.dim, (int64_t)kBlock * rpt_u);
        for (int t = 0; t < tiles; ++t) hu[fu++] = make_int2(i, t);
        if (j.fresh) {
            hnj[fn] = hj[i];
            hpr[fn] = make_problem(j.h, e->cfg.opt, j.t, j.tol, j.m);
            for (int t = 0; t < tiles; ++t) hni[fni++] = make_int2(fn, t);
            ++fn;
        }
    }
    for (int c = 0; c < 4; ++c) p.n_pitems[c] = (int)n_items_c[c];
    p.n_uitems = (int)n_u;
    p.n_ditems = (int)n_d;
    p.n_new = n_new;
    p.n_new_items = (int)n_new_items;

    char* D = p.dev;
    p.jobs = (JobView*)(D + o_jobs);
    p.groups = (GroupView*)(D + o_groups);
    for (int c = 0; c < 4; ++c) p.pitems[c] = (int2*)(D + o_p[c]);
    p.uitems = (int2*)(D + o_u);
    p.ditems = (int2*)(D + o_d);
    p.new_jobs = (JobView*)(D + o_nj);
    p.probs = (Problem*)(D + o_pr);
    p.new_items = (int2*)(D + o_ni);
    EHIP(hipMemcpyAsync(p.dev, p.host, total, hipMemcpyHostToDevice, e->stream));

    // set-up of the admitted jobs (stream-ordered after every round already queued)
    if (n_new > 0) {
        EHIP(launch_bsetup(p.new_jobs, p.probs, n_new, e->stream));
        if (!e->tuned && p.n_jobs > 0) {
            rc = autotune(e, p);
            if (rc != TE_OK) return rc;
        }
        EHIP(launch_bcopy_in(p.rpt_u, p.new_jobs, p.new_items, p.n_new_items, e->stream));
        for (te_job id : ids) e->jobs[(size_t)id].fresh = false;
    }

    if (!profiling(e) && p.n_jobs > 0) {
        EHIP(hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t le = enqueue_round(e, p, e->cap_stream, nullptr);
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(e->cap_stream, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(le, "kernel launch during round capture");
        }
        if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
        p.graph = g;
        EHIP(hipGraphInstantiate(&p.exec, g, nullptr, nullptr, 0));
    }
    e->cur = pi;
    e->n_plans += 1;
    e->need_plan = false;
    return TE_OK;
}

// algorithmic bytes of one round of plan p for the jobs whose restart in that round had
// Krylov dimension k (k = 0: the job did not run); per kernel class as in te_evolve
void round_bytes(const te_engine_s* e, const Plan& p, const std::vector<int>& kk, te_profile* pr) {
    const bool three = (e->cfg.opt.flags & TE_OPT_LANCZOS3) != 0;
    for (const auto& g : p.group_jobs) {
        const JobRec& j0 = e->jobs[(size_t)p.job_ids[(size_t)g[0]]];
        const double d = (double)j0.dim, nnz = (double)j0.h->csr.nnz;
        for (int j = 0; j < p.m; ++j) {
            bool any = false;
            for (int q : g) {
                const int k = kk[(size_t)q];
                const int m = e->jobs[(size_t)p.job_ids[(size_t)q]].m;
                if (k <= 0) continue;
                const int cols = (three && j >= 1) ? 2 : j + 1;  // basis columns the iteration reads
                if (j < std::min(k + 1, m)) {
                    any = true;
                    pr->bytes[TE_KERNEL_PROJECT] += 16.0 * d * (cols + 1);
                }
                if (j < k) pr->bytes[TE_KERNEL_UPDATE] += 16.0 * d * (cols + 1) + ((j + 1 < m) ? 16.0 * d : 0.0);
            }
            if (any) pr->bytes[TE_KERNEL_PROJECT] += csr_entries_bytes(j0.h->csr) + 4.0 * (d + 1);
        }
        for (int q : g)
            if (kk[(size_t)q] > 0) pr->bytes[TE_KERNEL_COMBINE] += 16.0 * d * (kk[(size_t)q] + 1);
    }
}

te_status accumulate_round_profile(te_engine_s* e, const Plan& p, const std::vector<int>& kk) {
    auto span = [&](size_t a, size_t b, double* out) {
        float ms = 0.f;
        hipError_t r = hipEventElapsedTime(&ms, e->pev[a], e->pev[b]);
        *out = 1e-3 * (double)ms;
        return r;
    };
    double t = 0.0;
    for (int j = 0; j < p.m; ++j) {
        EHIP(span(3 * j, 3 * j + 1, &t));
        e->prof.launches[TE_KERNEL_PROJECT] += 1;
        e->prof.seconds[TE_KERNEL_PROJECT] += t;
        EHIP(span(3 * j + 1, 3 * j + 2, &t));
        e->prof.launches[TE_KERNEL_FOLD] += 1;
        e->prof.seconds[TE_KERNEL_FOLD] += t;
        EHIP(span(3 * j + 2, 3 * j + 3, &t));
        e->prof.launches[TE_KERNEL_UPDATE] += 1;
        e->prof.seconds[TE_KERNEL_UPDATE] += t;
    }
    EHIP(span(3 * p.m, 3 * p.m + 1, &t));
    e->prof.launches[TE_KERNEL_STEP] += 1;
    e->prof.seconds[TE_KERNEL_STEP] += t;
    EHIP(span(3 * p.m + 1, 3 * p.m + 2, &t));
    e->prof.launches[TE_KERNEL_COMBINE] += 1;
    e->prof.seconds[TE_KERNEL_COMBINE] += t;
    round_bytes(e, p, kk, &e->prof);
    return TE_OK;
}

void finish_job(te_engine_s* e, JobRec& j, const SlotOut& o) {
    j.res.steps = o.steps;
    j.res.matvecs = o.matvecs;
    j.res.breakdown_dim = o.breakdown_dim;
    j.res.warnings = (uint32_t)o.warnings;
    j.res.err_bound = o.beta0 * o.err_acc;
    j.res.num_err_estimate = o.beta0 * o.num_acc;
    j.res.t_reached = (o.beta0 == 0.0) ? j.t : o.t_now;
    j.steps = o.steps;
    j.t_now = j.res.t_reached;
    j.status = o.status;
    if (j.status == TE_OK && o.beta0 != 0.0 && o.t_now != j.t) j.status = TE_ERR_DEVICE;
    j.state = (j.status == TE_OK) ? TE_JOB_DONE : TE_JOB_FAILED;
    j.t_fin = now_s();
    j.rounds = (int)(e->observed - j.round_adm);
    if (j.state == TE_JOB_DONE) e->done_count += 1;
    else e->failed_count += 1;
    (void)e->pool.release(j.off, j.bytes);
    e->free_slots.push_back(j.slot);
}

// Reads the records of round r (just observed) and retires completed jobs.  e->mu held.
void harvest(te_engine_s* e, int64_t r, std::vector<int>* kk) {
    const SlotOut* bank = e->slots_host + (size_t)(r & 1) * e->cfg.max_jobs;
    Plan& p = e->plans[e->cur];
    std::map<te_job, int> pos;
    if (kk) {
        kk->assign(p.job_ids.size(), 0);
        for (size_t i = 0; i < p.job_ids.size(); ++i) pos[p.job_ids[i]] = (int)i;
    }
    std::vector<te_job> keep;
    bool retired = false;
    for (te_job id : e->resident) {
        JobRec& j = e->jobs[(size_t)id];
        const SlotOut o = bank[j.slot];
        if (o.id != id || o.round != (int)r) {
            keep.push_back(id);
            continue;
        }
        if (kk && pos.count(id) && o.steps == j.steps + 1) (*kk)[(size_t)pos[id]] = o.last_k;
        j.steps = o.steps;
        j.t_now = o.t_now;
        if (o.done) {
            finish_job(e, j, o);
            retired = true;
            for (size_t i = 0; i < p.job_ids.size(); ++i)
                if (p.job_ids[i] == id) p.retired_weight += j.dim;
        } else {
            keep.push_back(id);
        }
    }
    e->resident.swap(keep);
    if (retired) e->cv_done.notify_all();
    // scheduling point: admission possible, or enough of the plan retired to compact it
    const bool can_admit = !e->queue.empty() && !e->free_slots.empty() &&
                           e->pool.fits(e->jobs[(size_t)e->queue.front()].bytes);
    const bool compact = retired && (p.retired_weight * 10 >= p.weight || e->resident.empty());
    if (can_admit || compact) e->need_plan = true;
}

void fail_all(te_engine_s* e, te_status s, const std::string& msg) {
    e->err = s;
    e->err_msg = msg;
    for (te_job id : e->resident) {
        JobRec& j = e->jobs[(size_t)id];
        j.state = TE_JOB_FAILED;
        j.status = s;
        j.t_fin = now_s();
        e->failed_count += 1;
    }
    e->resident.clear();
    e->cv_done.notify_all();
}

// One scheduling iteration.  Returns false when there is nothing to run.  Called with lk
// (on e->mu) held; releases it while waiting for the device.
bool schedule_once(te_engine_s* e, std::unique_lock<std::mutex>& lk) {
    if (e->err != TE_OK) return false;
    const int64_t in_flight = e->launched - e->observed;
    if (in_flight == 0 && e->resident.empty() && e->queue.empty()) return false;
    if (e->need_plan || e->cur < 0 || (in_flight == 0 && e->plans[e->cur].n_jobs == 0)) {
        if (in_flight == 0 && e->resident.empty()) e->need_plan = true;
        te_status rc = build_plan(e);
        if (rc != TE_OK) {
            fail_all(e, rc, te_last_error());
            return false;
        }
    }
    Plan& p = e->plans[e->cur];
    const int depth = profiling(e) ? 1 : kDepth;
    while (!e->resident.empty() && p.n_jobs > 0 && e->launched - e->observed < depth) {
        hipError_t r;
        if (profiling(e)) {
            while ((int)e->pev.size() < 3 * p.m + 3) {
                hipEvent_t ev;
                r = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence);  // timing only
                if (r != hipSuccess) break;
                e->pev.push_back(ev);
            }
            r = enqueue_round(e, p, e->stream, &e->pev);
        } else {
            r = hipGraphLaunch(p.exec, e->stream);
        }
        if (r == hipSuccess) r = hipEventRecord(e->ev[e->launched % kRing], e->stream);
        if (r == hipSuccess) r = hipEventRecord(p.last_use, e->stream);
        if (r != hipSuccess) {
            fail_all(e, TE_ERR_DEVICE, std::string("round launch: ") + hipGetErrorString(r));
            return false;
        }
        p.used = true;
        if (e->busy_since < 0.0) e->busy_since = now_s();
        e->launched += 1;
    }
    if (e->launched == e->observed) return false;
    const int64_t r = e->observed;
    hipEvent_t ev = e->ev[r % kRing];
    lk.unlock();
    hipError_t w = hipEventSynchronize(ev);
    lk.lock();
    if (w != hipSuccess) {
        fail_all(e, TE_ERR_DEVICE, std::string("round: ") + hipGetErrorString(w));
        return false;
    }
    e->observed += 1;
    std::vector<int> kk;
    harvest(e, r + 1, profiling(e) ? &kk : nullptr);
    if (profiling(e)) {
        te_status rc = accumulate_round_profile(e, p, kk);
        if (rc != TE_OK) {
            fail_all(e, rc, te_last_error());
            return false;
        }
    }
    if (e->resident.empty() && e->launched == e->observed && e->busy_since >= 0.0) {
        e->busy += now_s() - e->busy_since;
        e->busy_since = -1.0;
    }
    return true;
}

bool job_finished(const JobRec& j) { return j.state == TE_JOB_DONE || j.state == TE_JOB_FAILED; }

bool all_finished(te_engine_s* e, te_job id) {
    if (id >= 0) return job_finished(e->jobs[(size_t)id]);
    return e->queue.empty() && e->resident.empty();
}

void worker_main(te_engine_s* e) {
    (void)hipSetDevice(e->device);
    std::unique_lock<std::mutex> lk(e->mu);
    while (!e->stop) {
        bool progressed;
        {
            std::unique_lock<std::mutex> sl(e->sched_mu);
            progressed = schedule_once(e, lk);
        }
        if (!progressed && !e->stop) e->cv_work.wait(lk);
    }
}

te_status check_config(const te_engine_config& c) {
    if (c.m < 2) return set_error(TE_ERR_INVALID_ARG, "m must be >= 2");
    if (c.m > TE_MAX_KRYLOV) return set_error(TE_ERR_UNSUPPORTED, "m > TE_MAX_KRYLOV");
    if (c.max_jobs < 1 || c.max_jobs > kMaxEngineJobs) return set_error(TE_ERR_INVALID_ARG, "max_jobs out of range");
    if (c.lanes_per_row != 0 && !gproject_supported(c.lanes_per_row, c.nnz_per_lane))
        return set_error(TE_ERR_INVALID_ARG, "unsupported projection shape (4 lanes with 1 or 4 nonzeros, 8 with 2, 1 with 8)");
    if (c.update_rows_per_thread < 0 || c.update_rows_per_thread > 2)
        return set_error(TE_ERR_INVALID_ARG, "update_rows_per_thread must be 0, 1 or 2");
    if (c.rows_per_thread != 0 && c.rows_per_thread != 1 && c.rows_per_thread != 2 && c.rows_per_thread != 4)
        return set_error(TE_ERR_INVALID_ARG, "rows_per_thread must be 0, 1, 2 or 4");
    if (c.flags & ~(TE_ENGINE_THREADED | TE_ENGINE_PROFILE)) return set_error(TE_ERR_INVALID_ARG, "unknown flags");
    if (c.opt.flags & ~TE_OPT_LANCZOS3)
        return set_error(TE_ERR_INVALID_ARG, "engine options take only TE_OPT_LANCZOS3 (profiling: TE_ENGINE_PROFILE)");
    if (c.lane_rows < 0 || c.lane_jobs < 0 || c.lane_jobs > c.max_jobs)
        return set_error(TE_ERR_INVALID_ARG, "lane_rows must be >= 0 and lane_jobs within 0..max_jobs");
    return check_options(c.opt);
}

}  // namespace

te_engine_s::~te_engine_s() {
    for (auto* l : lane)
        if (l) (void)te_engine_destroy(l);  // stops the lane's scheduler thread first
    for (auto& p : plans) {
        p.release_graph();
        if (p.last_use) (void)hipEventDestroy(p.last_use);
        dev_free(p.dev);
        if (p.host) (void)hipHostFree(p.host);
    }
    for (auto& v : ev)
        if (v) (void)hipEventDestroy(v);
    for (auto& v : pev) (void)hipEventDestroy(v);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
    if (slots_host) (void)hipHostFree(slots_host);
    if (ro_host) (void)hipHostFree(ro_host);
    dev_free(rounds_dev);
    dev_free(states);
    dev_free(pool_base);
}

// ============================================================================== C ABI
extern "C" {

uint64_t te_job_footprint(int64_t dim, int32_t m) {
    if (dim < 1 || dim >= ((int64_t)1 << 31) - 1 || m < 1 || m > TE_MAX_KRYLOV) return 0;
    return job_layout((int)dim, (int)std::min<int64_t>(m, dim)).total;
}

void te_engine_default_config(te_engine_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->m = 40;
    c->max_jobs = 1024;
    c->hbm_budget = 0;
    c->lanes_per_row = 0;
    c->nnz_per_lane = 0;
    c->rows_per_thread = 0;
    c->update_rows_per_thread = 0;
    c->flags = TE_ENGINE_THREADED;
    te_default_options(&c->opt);
}

te_status te_engine_create(te_engine* out, const te_engine_config* cfg, void* stream) {
    if (!out || !cfg) return set_error(TE_ERR_INVALID_ARG, "null pointer");
    *out = nullptr;
    te_status rc = check_config(*cfg);
    if (rc != TE_OK) return rc;
    if (cfg->hbm_budget < PoolAlloc::kAlign) return set_error(TE_ERR_INVALID_ARG, "hbm_budget too small");
    if (cfg->lane_rows > 0) {  // two lanes: a router over two engines, each with half the budget
        auto* r = new (std::nothrow) te_engine_s();
        if (!r) return set_error(TE_ERR_OUT_OF_MEMORY, "host allocation failed");
        r->cfg = *cfg;
        te_engine_config c = *cfg;
        c.lane_rows = 0;
        c.lane_jobs = 0;
        c.hbm_budget = cfg->hbm_budget / 2 / PoolAlloc::kAlign * PoolAlloc::kAlign;
        rc = te_engine_create(&r->lane[0], &c, stream);  // small jobs: the caller's stream, if any
        if (rc == TE_OK) {
            c.max_jobs = cfg->lane_jobs ? cfg->lane_jobs : std::min(2, cfg->max_jobs);
            rc = te_engine_create(&r->lane[1], &c, nullptr);  // large jobs: a stream of its own
        }
        if (rc != TE_OK) {
            delete r;
            return rc;
        }
        *out = r;
        return TE_OK;
    }
    auto* e = new (std::nothrow) te_engine_s();
    if (!e) return set_error(TE_ERR_OUT_OF_MEMORY, "host allocation failed");
    e->cfg = *cfg;
    if (cfg->lanes_per_row != 0) {
        e->tuning.lanes_per_row = cfg->lanes_per_row;
        e->tuning.nnz_per_lane = cfg->nnz_per_lane;
        e->tuned = true;
    }
    e->tuning.rows_per_thread = cfg->rows_per_thread ? cfg->rows_per_thread : 4;
    e->tuning.update_rows_per_thread = cfg->update_rows_per_thread ? cfg->update_rows_per_thread : 2;
    auto chk = [&](hipError_t r, const char* what) {
        if (r != hipSuccess && rc == TE_OK) rc = hip_fail(r, what);
    };
    chk(hipGetDevice(&e->device), "hipGetDevice");
    if (rc == TE_OK) {
        e->pool_base = (char*)dev_alloc(cfg->hbm_budget, (hipStream_t)stream);
        if (!e->pool_base) rc = set_error(TE_ERR_OUT_OF_MEMORY, "pool allocation of " + std::to_string(cfg->hbm_budget) + " bytes failed");
    }
    if (rc == TE_OK) {
        e->pool.reset(cfg->hbm_budget);
        e->states = (DevState*)dev_alloc(sizeof(DevState) * (size_t)cfg->max_jobs, (hipStream_t)stream);
        e->rounds_dev = (int*)dev_alloc(256, (hipStream_t)stream);
        if (!e->states || !e->rounds_dev) rc = set_error(TE_ERR_OUT_OF_MEMORY, "slot allocation failed");
    }
    if (rc == TE_OK) {
        chk(hipMemset(e->states, 0, sizeof(DevState) * (size_t)cfg->max_jobs), "hipMemset");
        chk(hipMemset(e->rounds_dev, 0, 256), "hipMemset");
        const size_t sb = sizeof(SlotOut) * 2 * (size_t)cfg->max_jobs;
        chk(hipHostMalloc((void**)&e->slots_host, sb, hipHostMallocMapped | hipHostMallocCoherent), "hipHostMalloc");
        if (rc == TE_OK) {
            std::memset(e->slots_host, 0, sb);
            for (size_t i = 0; i < 2 * (size_t)cfg->max_jobs; ++i) e->slots_host[i].id = -1;
            chk(hipHostGetDevicePointer((void**)&e->slots_dev, e->slots_host, 0), "hipHostGetDevicePointer");
        }
        chk(hipHostMalloc((void**)&e->ro_host, sizeof(RoundOut), hipHostMallocMapped | hipHostMallocCoherent),
            "hipHostMalloc");
        if (rc == TE_OK) {
            std::memset(e->ro_host, 0, sizeof(RoundOut));
            chk(hipHostGetDevicePointer((void**)&e->ro_dev, e->ro_host, 0), "hipHostGetDevicePointer");
        }
    }
    if (rc == TE_OK) {
        if (stream) {
            e->stream = (hipStream_t)stream;
        } else {
            chk(hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking), "hipStreamCreate");
            e->own_stream = true;
        }
        chk(hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
        for (auto& v : e->ev) chk(hipEventCreateWithFlags(&v, hipEventDisableTiming), "hipEventCreate");
        chk(hipDeviceSynchronize(), "hipDeviceSynchronize");
    }
    if (rc != TE_OK) {
        delete e;
        return rc;
    }
    for (int s = cfg->max_jobs - 1; s >= 0; --s) e->free_slots.push_back(s);
    if (cfg->flags & TE_ENGINE_THREADED) {
        try {
            e->worker = std::thread(worker_main, e);
        } catch (...) {
            delete e;
            return set_error(TE_ERR_DEVICE, "could not start the scheduler thread");
        }
    }
    *out = e;
    return TE_OK;
}

te_status te_engine_submit(te_engine e, te_hamiltonian h, const te_c128* v0, te_c128* v_out, double t, double tol,
                           te_job* id) {
    if (!e || !h || !v0 || !v_out) return set_error(TE_ERR_INVALID_ARG, "null pointer");
    if (e->lane[0]) {
        const int l = (int64_t)h->csr.dim >= e->cfg.lane_rows ? 1 : 0;
        std::lock_guard<std::mutex> lk(e->mu);  // ids in submission order over both lanes
        te_job local = -1;
        te_status rc = te_engine_submit(e->lane[l], h, v0, v_out, t, tol, &local);
        if (rc != TE_OK) return rc;
        e->route.emplace_back(l, local);
        if (id) *id = (te_job)e->route.size() - 1;
        return TE_OK;
    }
    if (!std::isfinite(t) || t < 0.0) return set_error(TE_ERR_INVALID_ARG, "t must be finite and >= 0");
    if (!std::isfinite(tol) || !(tol > 0.0)) return set_error(TE_ERR_INVALID_ARG, "tol must be finite and > 0");
    const int dim = h->csr.dim;
    const int m = std::min(e->cfg.m, dim);
    const uint64_t bytes = job_layout(dim, m).total;
    if (bytes > e->pool.size())
        return set_error(TE_ERR_CAPACITY, "job footprint " + std::to_string(bytes) + " B exceeds the pool (" +
                                              std::to_string(e->pool.size()) + " B)");
    std::unique_lock<std::mutex> lk(e->mu);
    if (e->err != TE_OK) return set_error(e->err, "engine failed: " + e->err_msg);
    JobRec j;
    j.id = (te_job)e->jobs.size();
    j.h = h;
    j.v0 = (const double2*)v0;
    j.out = (double2*)v_out;
    j.t = t;
    j.tol = tol;
    j.m = m;
    j.dim = dim;
    j.bytes = bytes;
    j.t_sub = now_s();
    if (t == 0.0) {
        hipError_t r = hipSuccess;
        if ((const void*)v0 != (const void*)v_out)
            r = hipMemcpy(v_out, v0, (size_t)dim * sizeof(te_c128), hipMemcpyDeviceToDevice);
        if (r != hipSuccess) return hip_fail(r, "copy v0");
        j.state = TE_JOB_DONE;
        j.t_adm = j.t_fin = j.t_sub;
        e->done_count += 1;
        e->jobs.push_back(j);
    } else {
        e->jobs.push_back(j);
        e->queue.push_back(j.id);
        e->cv_work.notify_all();
    }
    if (id) *id = j.id;
    return TE_OK;
}

// the lane and the lane's id of a routed job
static bool routed(te_engine e, te_job id, te_engine* l, te_job* local) {
    std::lock_guard<std::mutex> lk(e->mu);
    if (id < 0 || id >= (te_job)e->route.size()) return false;
    *l = e->lane[e->route[(size_t)id].first];
    *local = e->route[(size_t)id].second;
    return true;
}

te_status te_engine_poll(te_engine e, te_job id, te_job_info* info, te_result* res) {
    if (!e) return set_error(TE_ERR_INVALID_ARG, "null engine");
    if (e->lane[0]) {
        te_engine l;
        te_job local;
        if (!routed(e, id, &l, &local)) return set_error(TE_ERR_INVALID_ARG, "unknown job id");
        return te_engine_poll(l, local, info, res);
    }
    std::lock_guard<std::mutex> lk(e->mu);
    if (id < 0 || id >= (te_job)e->jobs.size()) return set_error(TE_ERR_INVALID_ARG, "unknown job id");
    const JobRec& j = e->jobs[(size_t)id];
    if (info) {
        info->state = j.state;
        info->status = j.status;
        info->rounds = job_finished(j) ? j.rounds : (j.state == TE_JOB_RUNNING ? (int)(e->observed - j.round_adm) : 0);
        info->steps = j.steps;
        info->t_now = j.t_now;
        info->submitted = j.t_sub;
        info->admitted = j.t_adm;
        info->finished = j.t_fin;
    }
    if (res) {
        if (job_finished(j)) *res = j.res;
        else std::memset(res, 0, sizeof(*res));
    }
    return TE_OK;
}

te_status te_engine_wait(te_engine e, te_job id, double timeout_s) {
    if (!e) return set_error(TE_ERR_INVALID_ARG, "null engine");
    const double deadline = timeout_s < 0.0 ? 1e300 : now_s() + timeout_s;
    if (e->lane[0]) {
        if (id == -1) {
            for (te_engine l : e->lane) {
                const double left = timeout_s < 0.0 ? -1.0 : std::max(0.0, deadline - now_s());
                te_status rc = te_engine_wait(l, -1, left);
                if (rc != TE_OK) return rc;
            }
            return TE_OK;
        }
        te_engine l;
        te_job local;
        if (!routed(e, id, &l, &local)) return set_error(TE_ERR_INVALID_ARG, "unknown job id");
        return te_engine_wait(l, local, timeout_s);
    }
    std::unique_lock<std::mutex> lk(e->mu);
    if (id >= (te_job)e->jobs.size() || id < -1) return set_error(TE_ERR_INVALID_ARG, "unknown job id");
    const bool threaded = (e->cfg.flags & TE_ENGINE_THREADED) != 0;
    while (!all_finished(e, id)) {
        if (e->err != TE_OK) return set_error(e->err, "engine failed: " + e->err_msg);
        if (now_s() >= deadline) return set_error(TE_ERR_TIMEOUT, "jobs not done before the timeout");
        if (threaded) {
            e->cv_done.wait_for(lk, std::chrono::milliseconds(50));
        } else {
            std::unique_lock<std::mutex> sl(e->sched_mu);
            if (!schedule_once(e, lk) && !all_finished(e, id) && e->err == TE_OK)
                return set_error(TE_ERR_DEVICE, "scheduler made no progress");
        }
    }
    if (e->err != TE_OK) return set_error(e->err, "engine failed: " + e->err_msg);
    return TE_OK;
}

te_status te_engine_get_stats(te_engine e, te_engine_stats* out) {
    if (!e || !out) return set_error(TE_ERR_INVALID_ARG, "null pointer");
    if (e->lane[0]) {
        te_engine_stats a, b;
        te_status rc = te_engine_get_stats(e->lane[0], &a);
        if (rc == TE_OK) rc = te_engine_get_stats(e->lane[1], &b);
        if (rc != TE_OK) return rc;
        *out = a;
        out->rounds += b.rounds;
        out->plans += b.plans;
        out->jobs_submitted += b.jobs_submitted;
        out->jobs_done += b.jobs_done;
        out->jobs_failed += b.jobs_failed;
        out->jobs_queued += b.jobs_queued;
        out->jobs_running += b.jobs_running;
        out->pool_bytes += b.pool_bytes;
        out->pool_used += b.pool_used;
        out->pool_peak += b.pool_peak;
        out->busy_seconds = std::max(a.busy_seconds, b.busy_seconds);
        for (int k = 0; k < TE_KERNEL_CLASSES; ++k) {
            out->prof.launches[k] += b.prof.launches[k];
            out->prof.seconds[k] += b.prof.seconds[k];
            out->prof.bytes[k] += b.prof.bytes[k];
        }
        return TE_OK;
    }
    std::lock_guard<std::mutex> lk(e->mu);
    std::memset(out, 0, sizeof(*out));
    out->rounds = e->observed;
    out->plans = e->n_plans;
    out->jobs_submitted = (int64_t)e->jobs.size();
    out->jobs_done = e->done_count;
    out->jobs_failed = e->failed_count;
    out->jobs_queued = (int64_t)e->queue.size();
    out->jobs_running = (int64_t)e->resident.size();
    out->pool_bytes = e->pool.size();
    out->pool_used = e->pool.used();
    out->pool_peak = e->pool.peak();
    out->busy_seconds = e->busy + (e->busy_since >= 0.0 ? now_s() - e->busy_since : 0.0);
    out->tuning = e->tuning;
    out->prof = e->prof;
    return TE_OK;
}

te_status te_engine_destroy(te_engine e) {
    if (!e) return set_error(TE_ERR_INVALID_ARG, "null engine");
    if (e->lane[0]) {
        te_status rc = TE_OK;
        for (te_engine& l : e->lane) {
            const te_status r = te_engine_destroy(l);
            if (rc == TE_OK) rc = r;
            l = nullptr;
        }
        delete e;
        return rc;
    }
    {
        std::lock_guard<std::mutex> lk(e->mu);
        e->stop = true;
        e->cv_work.notify_all();
    }
    if (e->worker.joinable()) e->worker.join();
    (void)hipStreamSynchronize(e->stream);
    delete e;
    return TE_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------ batch
struct te_batch_s {
    te_engine_config cfg{};
    void* stream = nullptr;
    struct Item {
        te_hamiltonian h;
        const te_c128* v0;
        te_c128* out;
        double t, tol;
        te_job id;
    };
    std::vector<Item> items;
    te_engine eng = nullptr;
};

extern "C" {

te_status te_batch_create(te_batch* out, const te_engine_config* cfg, void* stream) {
    if (!out || !cfg) return set_error(TE_ERR_INVALID_ARG, "null pointer");
    *out = nullptr;
    te_engine_config c = *cfg;
    c.flags &= ~TE_ENGINE_THREADED;
    c.lane_rows = 0;  // a batch runs as one lane
    c.lane_jobs = 0;
    if (c.max_jobs == 0) c.max_jobs = 1;
    c.hbm_budget = 0;
    te_status rc = check_config(c);
    if (rc != TE_OK) return rc;
    auto* b = new (std::nothrow) te_batch_s();
    if (!b) return set_error(TE_ERR_OUT_OF_MEMORY, "host allocation failed");
    b->cfg = *cfg;
    b->cfg.flags &= ~TE_ENGINE_THREADED;
    b->stream = stream;
    *out = b;
    return TE_OK;
}

te_status te_batch_add(te_batch b, te_hamiltonian h, int32_t n, const te_c128* const* v0, te_c128* const* v_out,
                       double t, double tol, int32_t* first) {
    if (!b || !h || !v0 || !v_out) return set_error(TE_ERR_INVALID_ARG, "null pointer");
    if (b->eng) return set_error(TE_ERR_INVALID_ARG, "batch already launched");
    if (n < 1) return set_error(TE_ERR_INVALID_ARG, "n must be >= 1");
    if (!std::isfinite(t) || t < 0.0) return set_error(TE_ERR_INVALID_ARG, "t must be finite and >= 0");
    if (!std::isfinite(tol) || !(tol > 0.0)) return set_error(TE_ERR_INVALID_ARG, "tol must be finite and > 0");
    if (b->items.size() + (size_t)n > (size_t)kMaxEngineJobs * 64) return set_error(TE_ERR_CAPACITY, "too many jobs");
    for (int32_t i = 0; i < n; ++i)
        if (!v0[i] || !v_out[i]) return set_error(TE_ERR_INVALID_ARG, "null vector pointer");
    if (first) *first = (int32_t)b->items.size();
    for (int32_t i = 0; i < n; ++i) b->items.push_back({h, v0[i], v_out[i], t, tol, -1});
    return TE_OK;
}

te_status te_batch_launch(te_batch b, uint64_t hbm_budget, te_engine_stats* stats) {
    if (!b) return set_error(TE_ERR_INVALID_ARG, "null batch");
    if (b->eng) return set_error(TE_ERR_INVALID_ARG, "batch already launched");
    te_engine_config c = b->cfg;
    uint64_t total = 0, largest = 0;
    for (const auto& it : b->items) {
        const uint64_t f = te_job_footprint(it.h->csr.dim, c.m);
        total += f;
        largest = std::max(largest, f);
    }
    c.hbm_budget = hbm_budget ? hbm_budget : std::max<uint64_t>(total, PoolAlloc::kAlign);
    if (c.hbm_budget < largest) return set_error(TE_ERR_CAPACITY, "hbm_budget below the largest job footprint");
    if (b->cfg.max_jobs == 0) c.max_jobs = (int32_t)std::min<size_t>(std::max<size_t>(b->items.size(), 1), kMaxEngineJobs);
    te_status rc = te_engine_create(&b->eng, &c, b->stream);
    if (rc != TE_OK) return rc;
    for (auto& it : b->items) {
        rc = te_engine_submit(b->eng, it.h, it.v0, it.out, it.t, it.tol, &it.id);
        if (rc != TE_OK) return rc;
    }
    rc = te_engine_wait(b->eng, -1, -1.0);
    if (stats) (void)te_engine_get_stats(b->eng, stats);
    return rc;
}

te_status te_batch_result(te_batch b, int32_t i, te_result* res, te_status* status) {
    if (!b) return set_error(TE_ERR_INVALID_ARG, "null batch");
    if (i < 0 || (size_t)i >= b->items.size()) return set_error(TE_ERR_INVALID_ARG, "index out of range");
    if (!b->eng) return set_error(TE_ERR_INVALID_ARG, "batch not launched");
    te_job_info info;
    te_status rc = te_engine_poll(b->eng, b->items[(size_t)i].id, &info, res);
    if (rc != TE_OK) return rc;
    if (status) *status = (info.state == TE_JOB_DONE || info.state == TE_JOB_FAILED) ? info.status : TE_ERR_TIMEOUT;
    return TE_OK;
}

te_status te_batch_info(te_batch b, int32_t i, te_job_info* info) {
    if (!b || !info) return set_error(TE_ERR_INVALID_ARG, "null pointer");
    if (i < 0 || (size_t)i >= b->items.size()) return set_error(TE_ERR_INVALID_ARG, "index out of range");
    if (!b->eng) return set_error(TE_ERR_INVALID_ARG, "batch not launched");
    return te_engine_poll(b->eng, b->items[(size_t)i].id, info, nullptr);
}

te_status te_batch_destroy(te_batch b) {
    if (!b) return set_error(TE_ERR_INVALID_ARG, "null batch");
    te_status rc = TE_OK;
    if (b->eng) rc = te_engine_destroy(b->eng);
    delete b;
    return rc;
}

}  // extern "C"
