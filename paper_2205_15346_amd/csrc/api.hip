// Host side of the C ABI declared in include/te.h.
//
// te_evolve enqueues, per restart, the 2m row-parallel kernels of one Krylov build, the
// one-block step kernel and the recombination (captured once as a hipGraph per workspace).
// All decisions are taken on the device; the host keeps one restart queued ahead of the
// one that is running and stops launching when the step kernel has raised its done flag
// (written to mapped pinned memory).  Restarts launched after completion are no-ops.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "te_internal.h"

using namespace te;

namespace {

thread_local std::string g_last_error;

// te_set_allocator hook.  Every block it supplies is recorded with the free function, context
// and stream it came with, so a block always goes back to the allocator that supplied it.
te_alloc_fn g_alloc = nullptr;
te_free_fn g_free = nullptr;
void* g_alloc_ctx = nullptr;
struct AllocRecord {
    te_free_fn free_fn;
    void* ctx;
    void* stream;
};
std::mutex g_alloc_mu;
std::unordered_map<void*, AllocRecord> g_alloc_records;

te_status fail(te_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define TE_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(e_ == hipErrorOutOfMemory ? TE_ERR_OUT_OF_MEMORY : TE_ERR_DEVICE,              \
                        std::string(#call) + ": " + hipGetErrorString(e_));                            \
    } while (0)

}  // namespace

namespace te {

te_status set_error(te_status s, const std::string& msg) { return fail(s, msg); }

void* dev_alloc(size_t bytes, hipStream_t stream) {
    if (bytes == 0) bytes = 1;
    te_alloc_fn a;
    AllocRecord rec;
    {
        std::lock_guard<std::mutex> lock(g_alloc_mu);
        a = g_alloc;
        rec = AllocRecord{g_free, g_alloc_ctx, (void*)stream};
    }
    if (a) {  // the callback runs without the lock held
        void* p = a(bytes, (void*)stream, rec.ctx);
        if (p) {
            std::lock_guard<std::mutex> lock(g_alloc_mu);
            g_alloc_records[p] = rec;
        }
        return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void dev_free(void* p) {
    if (!p) return;
    AllocRecord rec{};
    bool hooked = false;
    {
        std::lock_guard<std::mutex> lock(g_alloc_mu);
        auto it = g_alloc_records.find(p);
        if (it != g_alloc_records.end()) {
            rec = it->second;
            g_alloc_records.erase(it);
            hooked = true;
        }
    }
    if (!hooked) {
        (void)hipFree(p);
        return;
    }
    // hipFree waits for the device; a caching allocator may hand the block out at once, so
    // wait here the same way before returning it
    (void)hipDeviceSynchronize();
    rec.free_fn(p, rec.stream, rec.ctx);
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t basis_ld(int64_t dim) { return align_up((size_t)dim, 64); }

}  // namespace te

// ------------------------------------------------------------------------- workspace
namespace te {

struct Workspace {
    int dim = 0, m = 0;
    int64_t ld = 0;
    Tiling tl{};
    char* base = nullptr;  // one device allocation
    double2* V = nullptr;
    double2* y = nullptr;
    RedBuf rb{};
    DevState* st = nullptr;
    int* host_flag = nullptr;  // mapped pinned
    int* host_flag_dev = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> pev[2];  // per-kernel timing events (profiling mode)
    size_t bytes = 0;

    static size_t layout(int dim, int m, const Tiling& tl, size_t* off_y, size_t* off_part, size_t* off_npart,
                         size_t* off_red, size_t* off_st) {
        const size_t ld = basis_ld(dim);
        size_t o = 0;
        o += (size_t)m * ld * sizeof(double2);
        *off_y = o;
        o += ld * sizeof(double2);
        o = align_up(o, 256);
        *off_part = o;
        o += (size_t)kMaxVals * max_tiles(dim) * sizeof(double2);  // any tiling fits
        o = align_up(o, 256);
        *off_npart = o;
        o += (size_t)max_tiles(dim) * sizeof(double);
        o = align_up(o, 256);
        *off_red = o;  // folded values
        o += (size_t)kMaxVals * sizeof(double2);
        o = align_up(o, 256);
        *off_st = o;
        o += sizeof(DevState);
        return align_up(o, 256);
    }

    ~Workspace() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto& v : pev)
            for (auto& e : v) (void)hipEventDestroy(e);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (host_flag) (void)hipHostFree(host_flag);
        dev_free(base);
    }
};

}  // namespace te

te_hamiltonian_s::~te_hamiltonian_s() {
    delete ws;
    dev_free(row_ptr);
    dev_free(col);
    dev_free(val);
    dev_free(rval);
    dev_free(code);
    dev_free(slice);
    dev_free(toff);
    dev_free(tval);
    dev_free(diag);
}

namespace {

Tiling handle_tiling(te_hamiltonian h) {
    if (!h->tuned) return default_tiling(h->csr.dim);
    const te_tuning& t = h->tuning;
    return make_tiling(h->csr.dim, t.rows_per_thread, t.lanes_per_row, t.nnz_per_lane, t.update_rows_per_thread,
                       t.split_projection);
}

te_status make_workspace(te_hamiltonian h, int m, hipStream_t s, Workspace** out) {
    auto* w = new (std::nothrow) Workspace();
    if (!w) return fail(TE_ERR_OUT_OF_MEMORY, "host allocation failed");
    w->dim = h->csr.dim;
    w->m = m;
    w->ld = (int64_t)basis_ld(w->dim);
    w->tl = handle_tiling(h);
    size_t oy, op, on, orr, os;
    w->bytes = Workspace::layout(w->dim, m, w->tl, &oy, &op, &on, &orr, &os);
    w->base = (char*)dev_alloc(w->bytes, s);
    if (!w->base) {
        delete w;
        return fail(TE_ERR_OUT_OF_MEMORY, "workspace allocation of " + std::to_string(w->bytes) + " bytes failed");
    }
    w->V = (double2*)w->base;
    w->y = (double2*)(w->base + oy);
    w->rb.part = (double2*)(w->base + op);
    w->rb.npart = (double*)(w->base + on);
    w->rb.red = (double2*)(w->base + orr);
    w->rb.n_tiles = w->tl.n_tiles_p;
    w->rb.n_norm = w->tl.n_tiles_u;
    w->st = (DevState*)(w->base + os);
    te_status rc = TE_OK;
    auto chk = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == TE_OK) rc = fail(TE_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    chk(hipMemset(w->rb.red, 0, (size_t)kMaxVals * sizeof(double2)), "hipMemset");
    chk(hipMemset(w->st, 0, sizeof(DevState)), "hipMemset");
    chk(hipHostMalloc((void**)&w->host_flag, 64, hipHostMallocMapped | hipHostMallocCoherent), "hipHostMalloc");
    if (rc == TE_OK) chk(hipHostGetDevicePointer((void**)&w->host_flag_dev, w->host_flag, 0), "hipHostGetDevicePointer");
    chk(hipStreamCreateWithFlags(&w->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    chk(hipEventCreateWithFlags(&w->ev[0], hipEventDisableTiming), "hipEventCreate");
    chk(hipEventCreateWithFlags(&w->ev[1], hipEventDisableTiming), "hipEventCreate");
    chk(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (rc != TE_OK) {
        delete w;
        return rc;
    }
    *out = w;
    return TE_OK;
}

// enqueue one restart (2m kernels + step + combine) on stream s
hipError_t enqueue_restart(te_hamiltonian h, Workspace* w, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int j = 0; j < w->m && e == hipSuccess; ++j) {
        e = launch_project(w->tl, h->csr, w->V, w->ld, j, w->y, w->st, w->rb, s);
        if (e == hipSuccess) e = launch_fold(j, w->st, w->rb, s);
        if (e == hipSuccess) e = launch_update(w->tl, w->V, w->ld, w->dim, j, w->y, w->st, w->rb, s);
    }
    if (e == hipSuccess) e = launch_step(w->st, w->rb, w->host_flag_dev, s);
    if (e == hipSuccess) e = launch_combine(w->tl, w->V, w->ld, w->dim, w->st, s);
    return e;
}

// restart with an event before the first and after every kernel (profiling mode)
// restart with an event before the first and after every kernel (profiling mode);
// iteration j: E[3j] project E[3j+1] fold E[3j+2] update E[3j+3]; then step, combine
// Events are bound to the dispatches (E[0]: start of the first projection; E[3j+1], E[3j+2],
// E[3j+3]: ends of projection, fold and update j; E[3m+1], E[3m+2]: ends of step and
// recombination), so timing adds no packets between the kernels.
hipError_t enqueue_restart_profiled(te_hamiltonian h, Workspace* w, hipStream_t s, std::vector<hipEvent_t>& E) {
    hipError_t e = hipSuccess;
    for (int j = 0; j < w->m && e == hipSuccess; ++j) {
        e = launch_project(w->tl, h->csr, w->V, w->ld, j, w->y, w->st, w->rb, s, j == 0 ? E[0] : nullptr,
                           E[3 * j + 1]);
        if (e == hipSuccess) e = launch_fold(j, w->st, w->rb, s, E[3 * j + 2]);
        if (e == hipSuccess) e = launch_update(w->tl, w->V, w->ld, w->dim, j, w->y, w->st, w->rb, s, E[3 * j + 3]);
    }
    if (e == hipSuccess) e = launch_step(w->st, w->rb, w->host_flag_dev, s, E[3 * w->m + 1]);
    if (e == hipSuccess) e = launch_combine(w->tl, w->V, w->ld, w->dim, w->st, s, E[3 * w->m + 2]);
    return e;
}

size_t profile_events(int m) { return (size_t)(3 * m + 3); }

// add one finished restart with Krylov dimension k to the profile.  A build that broke down
// at k < m still ran the projection of iteration k (its fold detected the breakdown).
hipError_t accumulate_profile(te_hamiltonian h, Workspace* w, std::vector<hipEvent_t>& E, int k, bool three_term,
                              te_profile* p) {
    const double d = (double)w->dim, nnz = (double)h->csr.nnz;
    auto span = [&](int a, int b, double* out) {
        float ms = 0.f;
        hipError_t e = hipEventElapsedTime(&ms, E[a], E[b]);
        *out = 1e-3 * (double)ms;
        return e;
    };
    double t;
    const int jp = std::min(k + 1, w->m);  // projections that ran
    for (int j = 0; j < jp; ++j) {
        hipError_t e = span(3 * j, 3 * j + 1, &t);
        if (e != hipSuccess) return e;
        p->launches[TE_KERNEL_PROJECT] += 1;
        p->seconds[TE_KERNEL_PROJECT] += t;
        // CSR (values, columns, row pointers), columns i_lo..j of V, y written
        const int cols = (three_term && j >= 1) ? 2 : j + 1;
        p->bytes[TE_KERNEL_PROJECT] += csr_entries_bytes(h->csr) + 4.0 * (d + 1) + 16.0 * d * (cols + 1);
        e = span(3 * j + 1, 3 * j + 2, &t);
        if (e != hipSuccess) return e;
        p->launches[TE_KERNEL_FOLD] += 1;
        p->seconds[TE_KERNEL_FOLD] += t;
        if (j >= k) continue;
        e = span(3 * j + 2, 3 * j + 3, &t);
        if (e != hipSuccess) return e;
        p->launches[TE_KERNEL_UPDATE] += 1;
        p->seconds[TE_KERNEL_UPDATE] += t;
        // y and columns i_lo..j read, column j+1 written unless this is the last iteration
        p->bytes[TE_KERNEL_UPDATE] += 16.0 * d * (cols + 1) + ((j + 1 < w->m) ? 16.0 * d : 0.0);
    }
    hipError_t e = span(3 * w->m, 3 * w->m + 1, &t);
    if (e != hipSuccess) return e;
    p->launches[TE_KERNEL_STEP] += 1;
    p->seconds[TE_KERNEL_STEP] += t;
    e = span(3 * w->m + 1, 3 * w->m + 2, &t);
    if (e != hipSuccess) return e;
    p->launches[TE_KERNEL_COMBINE] += 1;
    p->seconds[TE_KERNEL_COMBINE] += t;
    p->bytes[TE_KERNEL_COMBINE] += 16.0 * d * (k + 1);
    return hipSuccess;
}

bool graphs_enabled() {
    const char* v = std::getenv("TE_NO_GRAPH");
    return !(v && v[0] == '1');
}

te_status ensure_graph(te_hamiltonian h, Workspace* w) {
    if (w->exec || !graphs_enabled()) return TE_OK;
    TE_HIP(hipStreamBeginCapture(w->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = enqueue_restart(h, w, w->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(w->cap_stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(TE_ERR_DEVICE, std::string("kernel launch during capture: ") + hipGetErrorString(le));
    }
    if (ce != hipSuccess) return fail(TE_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
    w->graph = g;
    TE_HIP(hipGraphInstantiate(&w->exec, g, nullptr, nullptr, 0));
    return TE_OK;
}

// re-point a workspace at a new tiling (the partial buffers fit every tiling)
te_status retile(te_hamiltonian h, Workspace* w, const Tiling& t) {
    w->tl = t;
    w->rb.n_tiles = t.n_tiles_p;
    w->rb.n_norm = t.n_tiles_u;
    if (w->exec) {
        (void)hipGraphExecDestroy(w->exec);
        w->exec = nullptr;
    }
    if (w->graph) {
        (void)hipGraphDestroy(w->graph);
        w->graph = nullptr;
    }
    return ensure_graph(h, w);
}

// "gfx950/<storage> dim nnz m": the best shape depends on how the entries are stored
std::string tune_key(te_hamiltonian h, int m) {
    const Csr& c = h->csr;
    const bool coded = c.pk.col || c.pk.col16;
    const char* storage = c.pk.c8 ? (coded ? "coded8" : "packed8") : c.pk.c16 ? (coded ? "coded16" : "packed16")
                          : c.rval ? "real" : "complex";
    return std::string("gfx950/") + storage + " " + std::to_string(c.dim) + " " + std::to_string(c.nnz) + " " +
           std::to_string(m);
}

bool tune_cache_lookup(const std::string& key, te_tuning* t) {
    const char* path = std::getenv("TE_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char arch[32];
        long long dim, nnz;
        int m, g, u, rp, ru, sp;
        double us;
        if (std::sscanf(line, "%31s %lld %lld %d %d %d %d %d %d %lf", arch, &dim, &nnz, &m, &g, &u, &rp, &ru, &sp,
                        &us) != 10)
            continue;
        const std::string k = std::string(arch) + " " + std::to_string(dim) + " " + std::to_string(nnz) + " " +
                              std::to_string(m);
        if (k == key && tiling_supported(rp, g, u, ru, sp)) {
            *t = te_tuning{g, u, rp, ru, sp, us};
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_cache_store(const std::string& key, const te_tuning& t) {
    const char* path = std::getenv("TE_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %d %.3f\n", key.c_str(), t.lanes_per_row, t.nnz_per_lane, t.rows_per_thread,
                 t.update_rows_per_thread, t.split_projection, t.project_us);
    std::fclose(f);
}

// Times the projection kernel (iteration j = m/2, zero basis) for every supported shape, then
// the update kernel with one and two rows per thread.
te_status run_autotune(te_hamiltonian h, Workspace* w, hipStream_t s) {
    const std::string key = tune_key(h, w->m);
    te_tuning best{};
    if (tune_cache_lookup(key, &best)) {
        h->tuning = best;
        h->tuned = true;
        return retile(h, w, handle_tiling(h));
    }
    const int J = std::min(w->m / 2, w->m - 1);  // mid-restart: the mean cost over j = 0..m-1
    te_options o;
    te_default_options(&o);
    const Problem prob = make_problem(h, o, 1.0, 1.0, w->m);
    TE_HIP(hipMemsetAsync(w->V, 0, (size_t)(J + 1) * w->ld * sizeof(double2), s));
    TE_HIP(launch_setup(w->st, prob, s));
    hipEvent_t e0, e1;
    TE_HIP(hipEventCreate(&e0));
    TE_HIP(hipEventCreate(&e1));
    const int rpt_u = default_tiling(w->dim).rpt_u;
    const int shapes[6][2] = {{4, 1}, {4, 4}, {8, 2}, {2, 8}, {1, 8}, {1, 16}};
    double best_us = 1e30;
    hipError_t err = hipSuccess;
    for (int sp = 0; sp <= 1 && err == hipSuccess; ++sp)
    for (int rp = 1; rp <= 4 && err == hipSuccess; rp *= 2) {
        for (const auto& sh : shapes) {
            const Tiling t = make_tiling(w->dim, rp, sh[0], sh[1], rpt_u, sp);
            RedBuf rb = w->rb;
            rb.n_tiles = t.n_tiles_p;
            err = launch_project(t, h->csr, w->V, w->ld, J, w->y, w->st, rb, s);
            if (err == hipSuccess) err = hipEventRecord(e0, s);
            for (int q = 0; q < 3 && err == hipSuccess; ++q) err = launch_project(t, h->csr, w->V, w->ld, J, w->y, w->st, rb, s);
            if (err == hipSuccess) err = hipEventRecord(e1, s);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (err != hipSuccess) break;
            const double us = 1e3 * ms / 3.0;
            if (us < best_us) {
                best_us = us;
                best = te_tuning{sh[0], sh[1], rp, rpt_u, sp, us};
            }
        }
    }
    // Rows per thread of the update (and recombination), timed at the same iteration.  The
    // squared norm of column J is set to 1 so that the update streams its columns instead of
    // taking the breakdown exit (its results in the workspace are not used).
    const double2 one = make_double2(1.0, 0.0);
    if (err == hipSuccess) err = hipMemcpyAsync(&w->rb.red[2 * J + 1], &one, sizeof(one), hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);  // `one` lives on this stack frame
    double best_u = 1e30;
    for (int ru = 1; ru <= 2 && err == hipSuccess; ++ru) {
        const Tiling t = make_tiling(w->dim, best.rows_per_thread, best.lanes_per_row, best.nnz_per_lane, ru,
                                     best.split_projection);
        RedBuf rb = w->rb;
        rb.n_tiles = t.n_tiles_p;
        rb.n_norm = t.n_tiles_u;
        err = launch_update(t, w->V, w->ld, w->dim, J, w->y, w->st, rb, s);
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        for (int q = 0; q < 3 && err == hipSuccess; ++q) err = launch_update(t, w->V, w->ld, w->dim, J, w->y, w->st, rb, s);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err == hipSuccess && 1e3 * ms / 3.0 < best_u) {
            best_u = 1e3 * ms / 3.0;
            best.update_rows_per_thread = ru;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(TE_ERR_DEVICE, std::string("autotune: ") + hipGetErrorString(err));
    h->tuning = best;
    h->tuned = true;
    tune_cache_store(key, best);
    return retile(h, w, handle_tiling(h));
}

bool autotune_enabled() {
    const char* v = std::getenv("TE_AUTOTUNE");
    return !(v && v[0] == '0');
}

te_status get_workspace(te_hamiltonian h, int m, hipStream_t s, Workspace** out) {
    if (h->ws && h->ws->m == m) {
        *out = h->ws;
        return TE_OK;
    }
    delete h->ws;
    h->ws = nullptr;
    Workspace* w = nullptr;
    te_status rc = make_workspace(h, m, s, &w);
    if (rc != TE_OK) return rc;
    h->ws = w;
    rc = ensure_graph(h, w);
    if (rc != TE_OK) return rc;
    *out = w;
    return TE_OK;
}

}  // namespace

namespace te {

Problem make_problem(const te_hamiltonian_s* h, const te_options& o, double t, double tol, int m) {
    Problem p{};
    p.t = t;
    p.tol_rate = tol / t;
    p.numerr_per_step = (double)h->csr.dim * h->norm1 * std::ldexp(1.0, -52);
    p.t_init = o.t_init;
    p.shrink = o.shrink;
    p.quad_rel_tol = o.quad_rel_tol;
    p.m = m;
    p.dim = h->csr.dim;
    p.n_substeps = o.n_substeps;
    p.quad_max_level = o.quad_max_level;
    p.quad_min_level = o.quad_min_level;
    p.max_halvings = o.max_halvings;
    p.three_term = (o.flags & TE_OPT_LANCZOS3) ? 1 : 0;
    p.gauss_n = o.quad_gauss_points;
    return p;
}

te_status check_options(const te_options& o) {
    if (o.n_substeps < 1 || !(o.t_init > 0.0) || !std::isfinite(o.t_init) || !(o.shrink > 0.0) || !(o.shrink <= 1.0) ||
        !(o.quad_rel_tol > 0.0) || o.quad_max_level < 0 || o.quad_max_level > 20 || o.quad_min_level < 0 ||
        o.max_halvings < 0 || (o.flags & ~(TE_OPT_PROFILE | TE_OPT_LANCZOS3)) != 0 || o.quad_gauss_points < 0 ||
        o.quad_gauss_points > TE_MAX_KRYLOV)
        return fail(TE_ERR_INVALID_ARG, "invalid te_options");
    return TE_OK;
}

}  // namespace te

// ============================================================================== C ABI
extern "C" {

void te_default_options(te_options* o) {
    if (!o) return;
    o->n_substeps = 10;
    o->t_init = 0.1;
    o->shrink = 0.97;
    o->quad_rel_tol = 1e-3;
    o->quad_max_level = 15;
    o->quad_min_level = 3;
    o->max_halvings = 64;
    o->flags = 0;
    o->quad_gauss_points = 0;
}

const char* te_status_string(te_status s) {
    switch (s) {
        case TE_OK: return "ok";
        case TE_ERR_INVALID_ARG: return "invalid argument";
        case TE_ERR_INVALID_CSR: return "invalid CSR matrix";
        case TE_ERR_NOT_HERMITIAN: return "matrix is not Hermitian";
        case TE_ERR_UNSUPPORTED: return "unsupported parameter";
        case TE_ERR_OUT_OF_MEMORY: return "out of device memory";
        case TE_ERR_DEVICE: return "HIP device error";
        case TE_ERR_STEP_UNDERFLOW: return "step-size search underflow";
        case TE_ERR_NONFINITE: return "non-finite value";
        case TE_ERR_CAPACITY: return "capacity exceeded";
        default: return "unknown status";
    }
}

const char* te_last_error(void) { return g_last_error.c_str(); }

te_status te_set_allocator(te_alloc_fn alloc, te_free_fn free_fn, void* ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(TE_ERR_INVALID_ARG, "alloc and free must be set together");
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    g_alloc = alloc;
    g_free = free_fn;
    g_alloc_ctx = ctx;
    return TE_OK;
}

size_t te_workspace_bytes(te_hamiltonian h, int32_t m) {
    if (!h || m < 1 || m > TE_MAX_KRYLOV) return 0;
    const int dim = h->csr.dim;
    const int mm = std::min(m, dim);
    size_t a, b, c, d, e;
    return Workspace::layout(dim, mm, default_tiling(dim), &a, &b, &c, &d, &e);
}

// Validates a handle's CSR on the device (structure, column range, finite entries, optionally
// Hermitian with sorted columns) and stores its 1-norm.  err (>= 4 bytes) and rowsum (dim + 8
// doubles) are device scratch; *herr receives the error bits (32: an imaginary part is nonzero).
static te_status validate_handle(te_hamiltonian h, int check_hermitian, int* err, double* rowsum, int* herr,
                                 hipStream_t s) {
    const int dim = h->csr.dim;
    double norm1 = 0.0;
    TE_HIP(hipMemsetAsync(err, 0, sizeof(int), s));
    TE_HIP(launch_validate(h->csr, check_hermitian, err, rowsum, s));
    TE_HIP(launch_norm1(rowsum, dim, rowsum + dim, s));
    TE_HIP(hipMemcpyAsync(herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    TE_HIP(hipMemcpyAsync(&norm1, rowsum + dim, sizeof(double), hipMemcpyDeviceToHost, s));
    TE_HIP(hipStreamSynchronize(s));
    if (*herr & (1 | 2 | 4 | 8))
        return fail(TE_ERR_INVALID_CSR, "invalid CSR (code " + std::to_string(*herr) + ": 1 structure, 2 column range, "
                                        "4 non-finite value, 8 unsorted columns)");
    if (*herr & 16) return fail(TE_ERR_NOT_HERMITIAN, "H differs from its conjugate transpose");
    h->norm1 = norm1;
    return TE_OK;
}

// Every imaginary part is zero: keep the real parts only (8-byte entries).
static te_status keep_real_entries(te_hamiltonian h, hipStream_t s) {
    const int64_t nnz = h->csr.nnz;
    h->rval = (double*)dev_alloc((size_t)nnz * sizeof(double));
    if (!h->rval) return fail(TE_ERR_OUT_OF_MEMORY, "device allocation for the real entries failed");
    TE_HIP(launch_real_part(h->val, h->rval, nnz, s));
    TE_HIP(hipStreamSynchronize(s));
    dev_free(h->val);
    h->val = nullptr;
    h->csr.val = nullptr;
    h->csr.rval = h->rval;
    return TE_OK;
}

// Packing of the stored entries (te::Packed).  One host pass over the entries, read back from
// the device in chunks, collects the distinct (column - row, value) pairs and the distinct
// values off the diagonal in two open-addressing tables (values compared bit for bit).  At most
// 65535 pairs: codes of pairs, no columns.  Else at most 65535 values: value codes beside the
// columns.  The matrix stays in CSR form (*packed = false) when both are exceeded, a diagonal
// entry has an imaginary part other than +0, or a row stores its diagonal twice.
namespace {

struct PairKey {
    int32_t off;
    uint64_t re, im;
};

inline uint64_t mix64(uint64_t x) {  // the splitmix64 finaliser
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

constexpr int kMaxCodes = 65535;     // codes 0..65534 off the diagonal, 65535 for the diagonal
constexpr int kCodeSlots = 1 << 17;  // load factor <= 1/2
constexpr int64_t kPackChunk = (int64_t)1 << 22;
constexpr size_t kCodePad = 64;  // >= the largest batch of codes + 4 bytes

// Distinct keys -> codes in first-seen order; full once kMaxCodes keys are held.
struct CodeTable {
    std::vector<int32_t> slot;
    std::vector<PairKey> keys;
    std::vector<int> off;
    std::vector<double2> val;
    bool full = false;
    CodeTable() : slot(kCodeSlots, -1), keys(kCodeSlots) {}
    // code of the key, or -1 when the table is (or just became) full
    int code(int32_t o, uint64_t re, uint64_t im, double2 v) {
        if (full) return -1;
        uint32_t q = (uint32_t)mix64(((uint64_t)(uint32_t)o << 32) ^ mix64(re) ^ (mix64(im) * 3u)) & (kCodeSlots - 1);
        while (slot[q] >= 0 && !(keys[q].off == o && keys[q].re == re && keys[q].im == im)) q = (q + 1) & (kCodeSlots - 1);
        if (slot[q] >= 0) return slot[q];
        if ((int)off.size() == kMaxCodes) {
            full = true;
            return -1;
        }
        slot[q] = (int32_t)off.size();
        keys[q] = PairKey{o, re, im};
        off.push_back(o);
        val.push_back(v);
        return slot[q];
    }
};

}  // namespace

static te_status try_pack(te_hamiltonian h, hipStream_t s, bool* packed) {
    *packed = false;
    const int dim = h->csr.dim;
    const int64_t nnz = h->csr.nnz;
    const bool real = h->csr.val == nullptr;  // real CSR entries (rval)
    std::vector<int> rp;
    std::vector<uint16_t> pcode, vcode;  // codes of pairs, codes of values
    std::vector<double> diag;
    std::vector<int> cbuf;
    std::vector<double2> vbuf;
    std::vector<double> rbuf;
    CodeTable pairs, values;
    try {
        rp.resize((size_t)dim + 1);
        pcode.resize((size_t)nnz);
        vcode.resize((size_t)nnz);
        diag.assign((size_t)dim, 0.0);
        cbuf.resize((size_t)std::min(nnz, kPackChunk));
        if (real) rbuf.resize((size_t)std::min(nnz, kPackChunk));
        else vbuf.resize((size_t)std::min(nnz, kPackChunk));
    } catch (...) {
        return TE_OK;  // no host memory for the pass: keep CSR
    }
    constexpr uint16_t kDiag = 0xFFFF;  // placeholder until the diagonal's code is known
    TE_HIP(hipMemcpyAsync(rp.data(), h->csr.row_ptr, ((size_t)dim + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
    TE_HIP(hipStreamSynchronize(s));
    int r = 0, diag_row = -1;
    for (int64_t k0 = 0; k0 < nnz; k0 += kPackChunk) {
        const int64_t n = std::min(kPackChunk, nnz - k0);
        TE_HIP(hipMemcpyAsync(cbuf.data(), h->csr.col + k0, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, s));
        if (real) TE_HIP(hipMemcpyAsync(rbuf.data(), h->csr.rval + k0, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
        else TE_HIP(hipMemcpyAsync(vbuf.data(), h->csr.val + k0, (size_t)n * sizeof(double2), hipMemcpyDeviceToHost, s));
        TE_HIP(hipStreamSynchronize(s));
        for (int64_t i = 0; i < n; ++i) {
            const int64_t k = k0 + i;
            while (rp[(size_t)r + 1] <= k) ++r;
            const int c = cbuf[(size_t)i];
            const double2 v = real ? make_double2(rbuf[(size_t)i], 0.0) : vbuf[(size_t)i];
            uint64_t re, im;
            std::memcpy(&re, &v.x, 8);
            std::memcpy(&im, &v.y, 8);
            if (c == r) {
                if (im != 0 || diag_row == r) return TE_OK;
                diag_row = r;
                diag[(size_t)r] = v.x;
                pcode[(size_t)k] = vcode[(size_t)k] = kDiag;
                continue;
            }
            const int pq = pairs.code(c - r, re, im, v);
            const int vq = values.code(0, re, im, v);
            if (pq < 0 && vq < 0) return TE_OK;
            pcode[(size_t)k] = (uint16_t)std::max(pq, 0);
            vcode[(size_t)k] = (uint16_t)std::max(vq, 0);
        }
    }
    const bool by_pairs = !pairs.full;
    CodeTable& tab = by_pairs ? pairs : values;
    std::vector<uint16_t>& code = by_pairs ? pcode : vcode;
    const int dcode = (int)tab.off.size();  // the diagonal's code follows the table's
    tab.off.push_back(0);
    tab.val.push_back(make_double2(0.0, 0.0));
    for (auto& q : code)
        if (q == kDiag) q = (uint16_t)dcode;
    // value codes: codes and columns sliced in chunks of 64 rows (te::Packed)
    const int nch = (dim + 63) / 64;
    std::vector<int> slice, scol, cbase;
    std::vector<uint16_t> scol16;  // with cbase: the 16-bit form of scol
    if (!by_pairs) {
        std::vector<int> cols;
        std::vector<uint16_t> scode;
        int64_t total = 0;
        try {
            slice.resize((size_t)nch);
            for (int c = 0; c < nch; ++c) {
                int w = 0;
                for (int rr = 64 * c; rr < std::min(dim, 64 * c + 64); ++rr) w = std::max(w, rp[(size_t)rr + 1] - rp[(size_t)rr]);
                slice[(size_t)c] = (int)total;
                total += 64 * (int64_t)w;
                if (total >= ((int64_t)1 << 31)) return TE_OK;  // positions would not fit int32: keep CSR
            }
            cols.resize((size_t)nnz);
            scol.assign((size_t)total, 0);
            scode.assign((size_t)total, 0);
        } catch (...) {
            return TE_OK;
        }
        TE_HIP(hipMemcpyAsync(cols.data(), h->csr.col, (size_t)nnz * sizeof(int), hipMemcpyDeviceToHost, s));
        TE_HIP(hipStreamSynchronize(s));
        for (int rr = 0; rr < dim; ++rr) {
            const int64_t at = slice[(size_t)(rr >> 6)] + (rr & 63);
            for (int k = rp[(size_t)rr]; k < rp[(size_t)rr + 1]; ++k) {
                const int64_t i = at + 64 * (int64_t)(k - rp[(size_t)rr]);
                scol[(size_t)i] = cols[(size_t)k];
                scode[(size_t)i] = code[(size_t)k];
            }
        }
        code.swap(scode);
        // 16-bit columns when the entries q of every chunk of 64 rows (a group) lie within 65535
        // columns of the group's smallest: a base per group, an offset per entry
        try {
            const int64_t groups = total / 64;
            cbase.assign((size_t)groups, INT32_MAX);
            std::vector<int> cmax((size_t)groups, -1);
            for (int rr = 0; rr < dim; ++rr) {
                const int64_t g0 = slice[(size_t)(rr >> 6)] / 64;
                for (int k = rp[(size_t)rr]; k < rp[(size_t)rr + 1]; ++k) {
                    const size_t g = (size_t)(g0 + (k - rp[(size_t)rr]));
                    const int c = cols[(size_t)k];
                    cbase[g] = std::min(cbase[g], c);
                    cmax[g] = std::max(cmax[g], c);
                }
            }
            bool fits = true;
            for (size_t g = 0; g < cbase.size() && fits; ++g) {
                if (cmax[g] < 0) cbase[g] = 0;  // no entry in the group (a chunk narrower than its slot count)
                else fits = (int64_t)cmax[g] - cbase[g] <= 65535;
            }
            if (fits) {
                scol16.assign((size_t)total, 0);
                for (int rr = 0; rr < dim; ++rr) {
                    const int64_t at = slice[(size_t)(rr >> 6)] + (rr & 63);
                    const int64_t g0 = slice[(size_t)(rr >> 6)] / 64;
                    for (int k = rp[(size_t)rr]; k < rp[(size_t)rr + 1]; ++k) {
                        const int64_t q = k - rp[(size_t)rr];
                        scol16[(size_t)(at + 64 * q)] = (uint16_t)(cols[(size_t)k] - cbase[(size_t)(g0 + q)]);
                    }
                }
            } else {
                cbase.clear();
            }
        } catch (...) {
            cbase.clear();
            scol16.clear();
        }
    }
    const int64_t ncode = (int64_t)code.size();
    const bool narrow = dcode <= 255;
    const size_t cbytes = (size_t)ncode * (narrow ? 1 : 2);
    // padded (zero bytes): a batch of 1-byte codes is read as whole dwords and may run past the end
    void* d_code = dev_alloc(cbytes + kCodePad);
    int* d_toff = (int*)dev_alloc(tab.off.size() * sizeof(int));
    double2* d_tval = (double2*)dev_alloc(tab.val.size() * sizeof(double2));
    double* d_diag = (double*)dev_alloc((size_t)dim * sizeof(double));
    // value codes: the columns, 32-bit or (one buffer) the group bases followed by 16-bit offsets
    const bool cols16 = !by_pairs && !scol16.empty();
    const size_t col_bytes =
        by_pairs ? 0 : cols16 ? cbase.size() * sizeof(int) + scol16.size() * sizeof(uint16_t) : scol.size() * sizeof(int);
    int* d_scol = by_pairs ? nullptr : (int*)dev_alloc(col_bytes);
    int* d_slice = by_pairs ? nullptr : (int*)dev_alloc(slice.size() * sizeof(int));
    auto release = [&]() {
        dev_free(d_code);
        dev_free(d_toff);
        dev_free(d_tval);
        dev_free(d_diag);
        dev_free(d_scol);
        dev_free(d_slice);
    };
    if (!d_code || !d_toff || !d_tval || !d_diag || (!by_pairs && (!d_scol || !d_slice))) {
        release();
        return TE_OK;  // no device memory for the packed copy: keep CSR
    }
    std::vector<uint8_t> code8;
    if (narrow) {
        code8.resize((size_t)ncode);
        for (int64_t k = 0; k < ncode; ++k) code8[(size_t)k] = (uint8_t)code[(size_t)k];
    }
    hipError_t e = hipMemsetAsync((char*)d_code + cbytes, 0, kCodePad, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_code, narrow ? (const void*)code8.data() : (const void*)code.data(), cbytes,
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_toff, tab.off.data(), tab.off.size() * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_tval, tab.val.data(), tab.val.size() * sizeof(double2), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_diag, diag.data(), (size_t)dim * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !by_pairs && !cols16)
        e = hipMemcpyAsync(d_scol, scol.data(), scol.size() * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && cols16)
        e = hipMemcpyAsync(d_scol, cbase.data(), cbase.size() * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && cols16)
        e = hipMemcpyAsync(d_scol + cbase.size(), scol16.data(), scol16.size() * sizeof(uint16_t),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !by_pairs)
        e = hipMemcpyAsync(d_slice, slice.data(), slice.size() * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        release();
        return fail(TE_ERR_DEVICE, std::string("packing the entries: ") + hipGetErrorString(e));
    }
    h->code = d_code;
    h->toff = d_toff;
    h->tval = d_tval;
    h->diag = d_diag;
    h->slice = d_slice;
    Packed pk;
    if (narrow) pk.c8 = (const uint8_t*)d_code;
    else pk.c16 = (const uint16_t*)d_code;
    if (cols16) {  // value codes: the sliced columns as group bases + 16-bit offsets
        pk.cbase = d_scol;
        pk.col16 = (const uint16_t*)(d_scol + cbase.size());
    } else {
        pk.col = d_scol;  // value codes: the sliced columns
    }
    pk.slice = d_slice;
    pk.toff = d_toff;
    pk.tval = d_tval;
    pk.diag = d_diag;
    pk.dcode = dcode;
    h->csr.pk = pk;
    dev_free(h->col);  // CSR columns: dropped (pairs) or replaced by the sliced copy (either form)
    h->col = d_scol;
    h->csr.col = nullptr;
    dev_free(h->val);
    dev_free(h->rval);
    h->val = nullptr;
    h->rval = nullptr;
    h->csr.val = nullptr;
    h->csr.rval = nullptr;
    *packed = true;
    return TE_OK;
}

te_status te_hamiltonian_create(te_hamiltonian* out, int64_t dim, int64_t nnz, const int32_t* row_ptr,
                                const int32_t* col_idx, const te_c128* values, uint32_t flags, void* stream) {
    if (!out || !row_ptr || !col_idx || !values) return fail(TE_ERR_INVALID_ARG, "null pointer");
    *out = nullptr;
    if (dim < 1 || dim >= ((int64_t)1 << 31) - 1) return fail(TE_ERR_INVALID_ARG, "dim out of range");
    if (nnz < 1 || nnz >= ((int64_t)1 << 31)) return fail(TE_ERR_INVALID_CSR, "nnz out of range (1..2^31-1)");
    if (flags & ~(TE_PTR_DEVICE | TE_CHECK_HERMITIAN | TE_STORE_COMPLEX | TE_STORE_CSR))
        return fail(TE_ERR_INVALID_ARG, "unknown flags");
    hipStream_t s = (hipStream_t)stream;
    auto* h = new (std::nothrow) te_hamiltonian_s();
    if (!h) return fail(TE_ERR_OUT_OF_MEMORY, "host allocation failed");
    h->row_ptr = (int*)dev_alloc((dim + 1) * sizeof(int), s);
    h->col = (int*)dev_alloc(nnz * sizeof(int), s);
    h->val = (double2*)dev_alloc(nnz * sizeof(double2), s);
    double* rowsum = (double*)dev_alloc(dim * sizeof(double) + 64, s);
    int* err = (int*)dev_alloc(64, s);
    if (!h->row_ptr || !h->col || !h->val || !rowsum || !err) {
        dev_free(rowsum);
        dev_free(err);
        delete h;
        return fail(TE_ERR_OUT_OF_MEMORY, "device allocation for the matrix failed");
    }
    const hipMemcpyKind kind = (flags & TE_PTR_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    te_status rc = TE_OK;
    int herr = 0;
    auto chk = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == TE_OK)
            rc = fail(e == hipErrorOutOfMemory ? TE_ERR_OUT_OF_MEMORY : TE_ERR_DEVICE,
                      std::string(what) + ": " + hipGetErrorString(e));
    };
    chk(hipMemcpyAsync(h->row_ptr, row_ptr, (dim + 1) * sizeof(int), kind, s), "copy row_ptr");
    chk(hipMemcpyAsync(h->col, col_idx, nnz * sizeof(int), kind, s), "copy col_idx");
    chk(hipMemcpyAsync(h->val, values, nnz * sizeof(double2), kind, s), "copy values");
    chk(hipMemsetAsync(err, 0, sizeof(int), s), "hipMemsetAsync");
    h->csr.row_ptr = h->row_ptr;
    h->csr.col = h->col;
    h->csr.val = h->val;
    h->csr.rval = nullptr;
    h->csr.dim = (int)dim;
    h->csr.nnz = nnz;
    if (rc == TE_OK) rc = validate_handle(h, (flags & TE_CHECK_HERMITIAN) ? 1 : 0, err, rowsum, &herr, s);
    dev_free(rowsum);
    dev_free(err);
    bool packed = false;
    if (rc == TE_OK && !(flags & TE_STORE_CSR)) rc = try_pack(h, s, &packed);
    if (rc == TE_OK && !packed && !(herr & 32) && !(flags & TE_STORE_COMPLEX)) rc = keep_real_entries(h, s);
    if (rc != TE_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return TE_OK;
}

te_status te_hamiltonian_destroy(te_hamiltonian h) {
    if (!h) return fail(TE_ERR_INVALID_ARG, "null handle");
    (void)hipDeviceSynchronize();
    delete h;
    return TE_OK;
}

te_status te_hamiltonian_real_values(te_hamiltonian h, int32_t* real_values) {
    if (!h || !real_values) return fail(TE_ERR_INVALID_ARG, "null pointer");
    *real_values = h->csr.rval ? 1 : 0;
    return TE_OK;
}

te_status te_hamiltonian_storage(te_hamiltonian h, int32_t* kind) {
    if (!h || !kind) return fail(TE_ERR_INVALID_ARG, "null pointer");
    const Packed& pk = h->csr.pk;
    const bool coded = pk.col || pk.col16;
    if (pk.c8) *kind = coded ? TE_STORAGE_CODED8 : TE_STORAGE_PACKED8;
    else if (pk.c16) *kind = coded ? TE_STORAGE_CODED16 : TE_STORAGE_PACKED16;
    else *kind = h->csr.rval ? TE_STORAGE_REAL : TE_STORAGE_COMPLEX;
    return TE_OK;
}

te_status te_hamiltonian_pack(te_hamiltonian h, int32_t* kind, void* stream) {
    if (!h) return fail(TE_ERR_INVALID_ARG, "null handle");
    {
        std::lock_guard<std::mutex> lock(h->mu);
        if (!is_packed(h->csr.pk)) {
            TE_HIP(hipDeviceSynchronize());  // no work in flight may still read the arrays freed below
            bool packed = false;
            const te_status rc = try_pack(h, (hipStream_t)stream, &packed);
            if (rc != TE_OK) return rc;
            if (packed) {
                // the workspace's restart graph holds the CSR arrays: drop it with the workspace
                delete h->ws;
                h->ws = nullptr;
                h->tuned = false;  // the best shape depends on the storage
            }
        }
    }
    return kind ? te_hamiltonian_storage(h, kind) : TE_OK;
}

te_status te_hamiltonian_copy_csr(te_hamiltonian h, int32_t* row_ptr, int32_t* col_idx, te_c128* values,
                                  uint32_t flags, void* stream) {
    if (!h) return fail(TE_ERR_INVALID_ARG, "null handle");
    if (flags & ~TE_PTR_DEVICE) return fail(TE_ERR_INVALID_ARG, "unknown flags");
    hipStream_t s = (hipStream_t)stream;
    const bool dev = (flags & TE_PTR_DEVICE) != 0;
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const int64_t dim = h->csr.dim, nnz = h->csr.nnz;
    if (is_packed(h->csr.pk)) {  // expand into device scratch, then copy out
        int* c = (int*)dev_alloc((size_t)nnz * sizeof(int));
        double2* v = (double2*)dev_alloc((size_t)nnz * sizeof(double2));
        hipError_t e = (c && v) ? launch_expand_packed(h->csr.row_ptr, h->csr.pk, h->csr.dim, c, v, s) : hipErrorOutOfMemory;
        if (e == hipSuccess && row_ptr) e = hipMemcpyAsync(row_ptr, h->csr.row_ptr, (dim + 1) * sizeof(int), kind, s);
        if (e == hipSuccess && col_idx) e = hipMemcpyAsync(col_idx, c, nnz * sizeof(int), kind, s);
        if (e == hipSuccess && values) e = hipMemcpyAsync(values, v, nnz * sizeof(double2), kind, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        dev_free(c);
        dev_free(v);
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? TE_ERR_OUT_OF_MEMORY : TE_ERR_DEVICE,
                        std::string("expanding the packed entries: ") + hipGetErrorString(e));
        return TE_OK;
    }
    if (row_ptr) TE_HIP(hipMemcpyAsync(row_ptr, h->csr.row_ptr, (dim + 1) * sizeof(int), kind, s));
    if (col_idx) TE_HIP(hipMemcpyAsync(col_idx, h->csr.col, nnz * sizeof(int), kind, s));
    if (values) {
        if (h->csr.val) {
            TE_HIP(hipMemcpyAsync(values, h->csr.val, nnz * sizeof(double2), kind, s));
        } else if (dev) {
            TE_HIP(launch_expand_real(h->csr.rval, (double2*)values, nnz, s));
        } else {
            std::vector<double> tmp;
            try {
                tmp.resize((size_t)nnz);
            } catch (...) {
                return fail(TE_ERR_OUT_OF_MEMORY, "host buffer for the real entries");
            }
            TE_HIP(hipMemcpyAsync(tmp.data(), h->csr.rval, nnz * sizeof(double), hipMemcpyDeviceToHost, s));
            TE_HIP(hipStreamSynchronize(s));
            for (int64_t k = 0; k < nnz; ++k) {
                values[k].re = tmp[(size_t)k];
                values[k].im = 0.0;
            }
        }
    }
    TE_HIP(hipStreamSynchronize(s));
    return TE_OK;
}

void te_memory_burden_defaults(te_memory_burden* p) {
    if (!p) return;
    p->K = 4;
    p->Kp = 4;
    p->N0 = 20;
    p->Nm = 2;
    p->eps_m = std::sqrt(20.0);
    p->Nc = 20.0;
    p->dNc = 12.0;
    p->C0 = 1.0;
    p->Cm = 1.0;
}

te_status te_hamiltonian_create_memory_burden(te_hamiltonian* out, const te_memory_burden* p,
                                              int64_t* initial_index, void* stream) {
    if (!out || !p) return fail(TE_ERR_INVALID_ARG, "null pointer");
    *out = nullptr;
    const te_memory_burden P = *p;
    const int n = P.K + P.Kp;
    if (P.K < 1 || P.Kp < 0 || n > 63 || P.N0 < 0 || P.Nm < 0 || P.Nm > P.K)
        return fail(TE_ERR_INVALID_ARG, "need K >= 1, K' >= 0, K + K' <= 63, N_0 >= 0, 0 <= N_m <= K");
    if (!std::isfinite(P.eps_m) || !std::isfinite(P.Nc) || !std::isfinite(P.dNc) || !std::isfinite(P.C0) ||
        !std::isfinite(P.Cm) || !(P.dNc > 0.0) || !(P.dNc < P.Nc))
        return fail(TE_ERR_INVALID_ARG, "need finite parameters and 0 < dN_c < N_c");
    // binomials (exact in int64 up to binom(63, 31) < 2^63)
    std::vector<int64_t> binom(64 * 64, 0);
    for (int a = 0; a < 64; ++a) {
        binom[(size_t)a * 64] = 1;
        for (int b = 1; b <= a; ++b)
            binom[(size_t)a * 64 + b] = binom[(size_t)(a - 1) * 64 + b - 1] + (b <= a - 1 ? binom[(size_t)(a - 1) * 64 + b] : 0);
    }
    const int64_t C = binom[(size_t)n * 64 + P.Nm];
    const int64_t Q = (int64_t)P.Nm * (n - P.Nm);
    const int64_t max_len = 1 + Q + (P.N0 > 0 ? 2 : 0);
    if (C > ((int64_t)1 << 31) / (P.N0 + 1)) return fail(TE_ERR_UNSUPPORTED, "dimension does not fit int32");
    const int64_t dim = C * (P.N0 + 1);
    const int64_t nnz = C * ((int64_t)(P.N0 + 1) * (1 + Q) + 2 * (int64_t)P.N0);
    if (dim > kMaxModelRows || nnz >= ((int64_t)1 << 31))
        return fail(TE_ERR_UNSUPPORTED, "more than 2^26 rows, or nnz that does not fit int32");
    int slots = 1;
    while (slots < max_len) slots <<= 1;
    if (slots > 512) return fail(TE_ERR_UNSUPPORTED, "a row would exceed 512 entries");
    // hopping amplitudes C_m f_i of the qubit pairs, on the host as the paper writes them
    auto f = [&](int i, int k, int l) {
#pragma clang fp contract(off)
        const int dk = (i == 3) ? P.K + 1 : 1;
        const int dl = (i == 2) ? 1 : P.K + 1;
        const double x = (double)(k + dk), y = (double)(l + dl);
        const double a = std::sqrt(2.0) * (x * x * x);
        const double b = std::sqrt(7.0) * (y * y * y * y * y);
        const double F = std::fmod(a + b, 1.0);
        return F < 0.5 ? F - 1.0 : F;
    };
    std::vector<double> hop(64 * 64, 0.0);
    auto set_pair = [&](int u, int v, double amp) {
        hop[(size_t)u * 64 + v] = amp;
        hop[(size_t)v * 64 + u] = amp;
    };
    for (int k = 1; k <= P.K; ++k)
        for (int kp = 1; kp <= P.Kp; ++kp) set_pair(k - 1, P.K + kp - 1, P.Cm * f(1, k, kp));
    for (int k = 1; k <= P.K; ++k)
        for (int l = k + 1; l <= P.K; ++l) set_pair(k - 1, l - 1, P.Cm * f(2, k, l));
    for (int kp = 1; kp <= P.Kp; ++kp)
        for (int lp = kp + 1; lp <= P.Kp; ++lp) set_pair(P.K + kp - 1, P.K + lp - 1, P.Cm * f(3, kp, lp));

    hipStream_t s = (hipStream_t)stream;
    auto* h = new (std::nothrow) te_hamiltonian_s();
    if (!h) return fail(TE_ERR_OUT_OF_MEMORY, "host allocation failed");
    h->row_ptr = (int*)dev_alloc((size_t)(dim + 1) * sizeof(int));
    h->col = (int*)dev_alloc((size_t)nnz * sizeof(int));
    h->rval = (double*)dev_alloc((size_t)nnz * sizeof(double));
    int64_t* d_binom = (int64_t*)dev_alloc(binom.size() * sizeof(int64_t));
    double* d_hop = (double*)dev_alloc(hop.size() * sizeof(double));
    double* rowsum = (double*)dev_alloc((size_t)dim * sizeof(double) + 64);
    int* err = (int*)dev_alloc(64);
    auto cleanup = [&]() {
        dev_free(d_binom);
        dev_free(d_hop);
        dev_free(rowsum);
        dev_free(err);
    };
    if (!h->row_ptr || !h->col || !h->rval || !d_binom || !d_hop || !rowsum || !err) {
        cleanup();
        delete h;
        return fail(TE_ERR_OUT_OF_MEMORY, "device allocation for the matrix failed");
    }
    h->csr.row_ptr = h->row_ptr;
    h->csr.col = h->col;
    h->csr.val = nullptr;
    h->csr.rval = h->rval;
    h->csr.dim = (int)dim;
    h->csr.nnz = nnz;
    MemoryBurdenDev M;
    M.n = n;
    M.K = P.K;
    M.Nm = P.Nm;
    M.N0 = P.N0;
    M.C = C;
    M.slots = slots;
    M.dim = dim;
    M.eps_m = P.eps_m;
    M.Nc = P.Nc;
    M.NcMinusDNc = P.Nc - P.dNc;
    M.C0 = P.C0;
    M.binom = d_binom;
    M.hop = d_hop;
    te_status rc = TE_OK;
    hipError_t e = hipMemcpyAsync(d_binom, binom.data(), binom.size() * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_hop, hop.data(), hop.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_memory_burden(M, h->row_ptr, h->col, h->rval, s);
    if (e != hipSuccess) rc = fail(TE_ERR_DEVICE, std::string("building the matrix: ") + hipGetErrorString(e));
    int herr = 0;
    // the construction is checked like any uploaded matrix (sorted, in range, Hermitian)
    if (rc == TE_OK) rc = validate_handle(h, 1, err, rowsum, &herr, s);
    cleanup();
    if (rc != TE_OK) {
        delete h;
        return rc;
    }
    if (initial_index) *initial_index = 0;  // n_0 = N_0 (block 0) and the first configuration
    *out = h;
    return TE_OK;
}

te_status te_hamiltonian_create_bose_chain(te_hamiltonian* out, int32_t K, int32_t N, const double* U,
                                          const te_c128* hop, uint32_t flags, void* stream) {
    if (!out || !U || (K > 1 && !hop)) return fail(TE_ERR_INVALID_ARG, "null pointer");
    *out = nullptr;
    if (K < 1 || K > 64 || N < 0 || N > 65535) return fail(TE_ERR_INVALID_ARG, "need 1 <= K <= 64 and 0 <= N <= 65535");
    if (flags & ~TE_STORE_COMPLEX) return fail(TE_ERR_INVALID_ARG, "unknown flags");
    for (int k = 0; k < K; ++k)
        if (!std::isfinite(U[k]) || (k < K - 1 && (!std::isfinite(hop[k].re) || !std::isfinite(hop[k].im))))
            return fail(TE_ERR_INVALID_ARG, "non-finite parameter");
    // binomials C(a, b), a <= N + K, b <= K, saturated (entries beyond the dimension are never used)
    const int bw = K + 1, rows = N + K + 1;
    const int64_t cap = (int64_t)1 << 61;  // the sum of two saturated entries stays in range
    std::vector<int64_t> binom((size_t)rows * bw, 0);
    for (int a = 0; a < rows; ++a) {
        binom[(size_t)a * bw] = 1;
        for (int b = 1; b <= std::min(a, K); ++b) {
            const int64_t x = binom[(size_t)(a - 1) * bw + b - 1] + (b <= a - 1 ? binom[(size_t)(a - 1) * bw + b] : 0);
            binom[(size_t)a * bw + b] = std::min(x, cap);
        }
    }
    const int64_t dim = binom[(size_t)(N + K - 1) * bw + (K - 1)];  // compositions of N into K parts
    if (dim > kMaxModelRows) return fail(TE_ERR_UNSUPPORTED, "more than 2^26 rows");
    int slots = 1;
    while (slots < 2 * K - 1) slots <<= 1;
    hipStream_t s = (hipStream_t)stream;
    auto* h = new (std::nothrow) te_hamiltonian_s();
    if (!h) return fail(TE_ERR_OUT_OF_MEMORY, "host allocation failed");
    const int64_t nb = (dim + 4 * kBlock - 1) / (4 * kBlock);
    h->row_ptr = (int*)dev_alloc((size_t)(dim + 1) * sizeof(int));
    int* cnt = (int*)dev_alloc((size_t)dim * sizeof(int));
    int64_t* scratch = (int64_t*)dev_alloc((size_t)(nb + 2) * sizeof(int64_t));
    int64_t* d_binom = (int64_t*)dev_alloc(binom.size() * sizeof(int64_t));
    double* d_U = (double*)dev_alloc((size_t)K * sizeof(double));
    double2* d_hop = (double2*)dev_alloc((size_t)std::max(K - 1, 1) * sizeof(double2));
    double* rowsum = (double*)dev_alloc((size_t)dim * sizeof(double) + 64);
    int* err = (int*)dev_alloc(64);
    auto cleanup = [&]() {
        dev_free(cnt);
        dev_free(scratch);
        dev_free(d_binom);
        dev_free(d_U);
        dev_free(d_hop);
        dev_free(rowsum);
        dev_free(err);
    };
    if (!h->row_ptr || !cnt || !scratch || !d_binom || !d_U || !d_hop || !rowsum || !err) {
        cleanup();
        delete h;
        return fail(TE_ERR_OUT_OF_MEMORY, "device allocation for the matrix failed");
    }
    BoseChainDev B;
    B.K = K;
    B.N = N;
    B.slots = slots;
    B.dim = dim;
    B.bw = bw;
    B.binom = d_binom;
    B.U = d_U;
    B.hop = d_hop;
    te_status rc = TE_OK;
    int64_t nnz = 0;
    hipError_t e = hipMemcpyAsync(d_binom, binom.data(), binom.size() * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_U, U, (size_t)K * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && K > 1) e = hipMemcpyAsync(d_hop, hop, (size_t)(K - 1) * sizeof(double2), hipMemcpyHostToDevice, s);
    // the column and value arrays are sized by the counted entries: count + scan, then fill
    if (e == hipSuccess) e = launch_bose_row_ptr(B, h->row_ptr, cnt, scratch, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&nnz, scratch + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && nnz >= ((int64_t)1 << 31)) rc = fail(TE_ERR_UNSUPPORTED, "nnz does not fit int32");
    if (e == hipSuccess && rc == TE_OK) {
        h->col = (int*)dev_alloc((size_t)nnz * sizeof(int));
        h->val = (double2*)dev_alloc((size_t)nnz * sizeof(double2));
        if (!h->col || !h->val) rc = fail(TE_ERR_OUT_OF_MEMORY, "device allocation for the matrix failed");
    }
    if (e == hipSuccess && rc == TE_OK) e = launch_bose_fill(B, h->row_ptr, h->col, h->val, s);
    if (e != hipSuccess && rc == TE_OK) rc = fail(TE_ERR_DEVICE, std::string("building the matrix: ") + hipGetErrorString(e));
    h->csr.row_ptr = h->row_ptr;
    h->csr.col = h->col;
    h->csr.val = h->val;
    h->csr.rval = nullptr;
    h->csr.dim = (int)dim;
    h->csr.nnz = nnz;
    int herr = 0;
    if (rc == TE_OK) rc = validate_handle(h, 1, err, rowsum, &herr, s);
    cleanup();
    if (rc == TE_OK && !(herr & 32) && !(flags & TE_STORE_COMPLEX)) rc = keep_real_entries(h, s);
    if (rc != TE_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return TE_OK;
}

te_status te_hamiltonian_info(te_hamiltonian h, int64_t* dim, int64_t* nnz, double* norm1) {
    if (!h) return fail(TE_ERR_INVALID_ARG, "null handle");
    if (dim) *dim = h->csr.dim;
    if (nnz) *nnz = h->csr.nnz;
    if (norm1) *norm1 = h->norm1;
    return TE_OK;
}

}  // extern "C"

namespace {

// Device buffers of one sampled evolution (te_evolve_sampled).
struct SampleBuffers {
    int n = 0, n_obs = 0;
    double* t = nullptr;        // [n] sample times
    double2* omega = nullptr;   // [n][kMaxM]
    double* bound = nullptr;    // [n]
    double* obs_part = nullptr; // [n][n_obs][tiles]
    double* obs_val = nullptr;  // [n][n_obs]
    double2* states = nullptr;  // caller's [n][dim] or null
    const double* obs = nullptr;
    int tiles = 0;
};

hipError_t enqueue_restart_sampled(te_hamiltonian h, Workspace* w, const SampleBuffers& sb, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int j = 0; j < w->m && e == hipSuccess; ++j) {
        e = launch_project(w->tl, h->csr, w->V, w->ld, j, w->y, w->st, w->rb, s);
        if (e == hipSuccess) e = launch_fold(j, w->st, w->rb, s);
        if (e == hipSuccess) e = launch_update(w->tl, w->V, w->ld, w->dim, j, w->y, w->st, w->rb, s);
    }
    if (e == hipSuccess) e = launch_step(w->st, w->rb, w->host_flag_dev, s);
    if (e == hipSuccess)  // the samples read the basis before the recombination overwrites column 0
        e = launch_samples(w->tl.rpt_u, w->V, w->ld, w->dim, w->st, sb.states, sb.obs, sb.n_obs, sb.obs_part,
                           sb.tiles, s);
    if (e == hipSuccess) e = launch_combine(w->tl, w->V, w->ld, w->dim, w->st, s);
    return e;
}

// The result record of a finished evolution from the device state's header, and the state's
// own failure status (step underflow, non-finite values, eigensolver failure).
te_status finish_result(const DevState& hs, double t, te_result* res) {
    if (res) {
        res->steps = hs.steps;
        res->matvecs = hs.matvecs;
        res->breakdown_dim = hs.breakdown_dim;
        res->warnings = (uint32_t)hs.warnings;
        res->err_bound = hs.beta0 * hs.err_acc;
        res->num_err_estimate = hs.beta0 * hs.num_acc;
        res->t_reached = hs.t_now;
    }
    if (hs.status != TE_OK) {
        if (hs.status == TE_ERR_STEP_UNDERFLOW)
            return fail(hs.status, "no admissible step after max_halvings halvings (t_now=" + std::to_string(hs.t_now) + ")");
        if (hs.status == TE_ERR_NONFINITE) return fail(hs.status, "non-finite value in v0 or during the iteration");
        return fail(hs.status, "device-side failure (eigensolver did not converge)");
    }
    if (hs.beta0 == 0.0 && res) res->t_reached = t;
    return TE_OK;
}

te_status reached_end(const DevState& hs, double t) {
    if (hs.beta0 != 0.0 && hs.t_now != t)
        return fail(TE_ERR_DEVICE, "evolution stopped at t=" + std::to_string(hs.t_now) + " before reaching t");
    return TE_OK;
}

// The argument rules shared by te_evolve and te_evolve_noalloc.
te_status check_evolve_args(te_hamiltonian h, const te_c128* v0, const te_c128* v_out, double t, double tol,
                            int32_t m, const te_options* opt, te_options* o) {
    if (!h || !v0 || !v_out) return fail(TE_ERR_INVALID_ARG, "null pointer");
    if (!std::isfinite(t) || t < 0.0) return fail(TE_ERR_INVALID_ARG, "t must be finite and >= 0");
    if (!std::isfinite(tol) || !(tol > 0.0)) return fail(TE_ERR_INVALID_ARG, "tol must be finite and > 0");
    if (m < 2) return fail(TE_ERR_INVALID_ARG, "m must be >= 2");
    if (m > TE_MAX_KRYLOV) return fail(TE_ERR_UNSUPPORTED, "m > TE_MAX_KRYLOV");
    te_default_options(o);
    if (opt) *o = *opt;
    return check_options(*o);
}

te_status evolve_impl(te_hamiltonian h, const te_c128* v0, te_c128* v_out, double t, double tol, int32_t m,
                      const te_options* opt, te_result* res, void* stream, SampleBuffers* sb,
                      DevState* header_out) {
    te_options o;
    te_status rc = check_evolve_args(h, v0, v_out, t, tol, m, opt, &o);
    if (rc != TE_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int dim = h->csr.dim;
    std::lock_guard<std::mutex> lock(h->mu);
    if (res) std::memset(res, 0, sizeof(*res));
    if (t == 0.0) {
        if (v_out != v0) TE_HIP(hipMemcpyAsync(v_out, v0, (size_t)dim * sizeof(te_c128), hipMemcpyDeviceToDevice, s));
        TE_HIP(hipStreamSynchronize(s));
        if (header_out) header_out->beta0 = -1.0;  // not evolved
        return TE_OK;
    }
    if (sb && (o.flags & TE_OPT_PROFILE)) return fail(TE_ERR_INVALID_ARG, "sampled evolution takes no TE_OPT_PROFILE");
    const int mm = std::min(m, dim);
    Workspace* w = nullptr;
    rc = get_workspace(h, mm, s, &w);
    if (rc != TE_OK) return rc;
    if (!h->tuned && autotune_enabled()) {
        rc = run_autotune(h, w, s);
        if (rc != TE_OK) return rc;
    }
    const Problem prob = make_problem(h, o, t, tol, mm);
    volatile int* flag = (volatile int*)w->host_flag;
    for (int i = 0; i < 16; ++i) flag[i] = 0;
    const bool profile = (o.flags & TE_OPT_PROFILE) != 0;
    if (profile) {
        h->prof = te_profile{};
        for (auto& v : w->pev) {
            while (v.size() < profile_events(mm)) {
                hipEvent_t e;
                // timing only: no system-scope fence (no cache writeback per record); the
                // restart's own event, recorded after these, is what the host waits on
                TE_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
                v.push_back(e);
            }
        }
    }
    TE_HIP(launch_setup(w->st, prob, s));
    TE_HIP(launch_copy((const double2*)v0, w->V, dim, s));
    if (sb) {
        sb->tiles = w->tl.n_tiles_u;
        const size_t part = (size_t)sb->n * (size_t)std::max(sb->n_obs, 1) * (size_t)sb->tiles * sizeof(double);
        sb->obs_part = (double*)dev_alloc(part);
        if (!sb->obs_part) return fail(TE_ERR_OUT_OF_MEMORY, "sample scratch allocation failed");
        SampleState ss{sb->t, sb->omega, sb->bound, sb->n, 0, 0, 0};
        TE_HIP(hipMemcpyAsync(&w->st->smp, &ss, sizeof(ss), hipMemcpyHostToDevice, s));
        TE_HIP(hipStreamSynchronize(s));  // ss lives on this stack frame
    }
    const long max_restarts = 100000000L;
    long r = 0;
    for (;; ++r) {
        if (sb) TE_HIP(enqueue_restart_sampled(h, w, *sb, s));
        else if (profile) TE_HIP(enqueue_restart_profiled(h, w, s, w->pev[r & 1]));
        else if (w->exec) TE_HIP(hipGraphLaunch(w->exec, s));
        else TE_HIP(enqueue_restart(h, w, s));
        TE_HIP(hipEventRecord(w->ev[r & 1], s));
        if (r >= 1) {
            TE_HIP(hipEventSynchronize(w->ev[(r - 1) & 1]));
            if (profile && r - 1 < flag[1]) TE_HIP(accumulate_profile(h, w, w->pev[(r - 1) & 1], flag[8 + ((r - 1) & 7)], prob.three_term != 0, &h->prof));
            if (flag[0]) break;
        }
        if (r >= max_restarts) return fail(TE_ERR_DEVICE, "restart limit reached");
    }
    if (profile) {
        TE_HIP(hipEventSynchronize(w->ev[r & 1]));
        if (r < flag[1]) TE_HIP(accumulate_profile(h, w, w->pev[r & 1], flag[8 + (r & 7)], prob.three_term != 0, &h->prof));
    }
    TE_HIP(launch_output(w->V, (double2*)v_out, dim, w->st, s));
    DevState hs;
    TE_HIP(hipMemcpyAsync(&hs, w->st, offsetof(DevState, alpha), hipMemcpyDeviceToHost, s));
    if (sb) {
        TE_HIP(hipMemcpyAsync(&hs.smp, &w->st->smp, sizeof(SampleState), hipMemcpyDeviceToHost, s));
        if (sb->n_obs > 0) TE_HIP(launch_obs_fold(sb->obs_part, sb->tiles, sb->n * sb->n_obs, sb->obs_val, s));
    }
    TE_HIP(hipStreamSynchronize(s));
    if (header_out) *header_out = hs;
    rc = finish_result(hs, t, res);
    if (rc != TE_OK) return rc;
    if (std::getenv("TE_TRACE")) {
        DevState* full = new (std::nothrow) DevState();
        if (full && hipMemcpy(full, w->st, sizeof(DevState), hipMemcpyDeviceToHost) == hipSuccess) {
            const int n = std::min(hs.steps, kTrace);
            std::fprintf(stderr, "[te trace] restarts=%d matvecs=%d bound=%.3e status=%d\n", hs.steps, hs.matvecs,
                         hs.err_acc, hs.status);
            for (int q = std::max(0, hs.steps - n); q < hs.steps; ++q) {
                const double* tr = full->trace[q % kTrace];
                std::fprintf(stderr,
                             "[te trace] %3d t_now=%.6f tau=%.6f err=%.3e h=%.3e k=%d bd=%d qok=%d t_rem=%.6f "
                             "eig_us=%.1f search_us=%.1f integrals=%d maxlev=%d\n",
                             q, tr[0], tr[1], tr[2], tr[3], (int)tr[4], (int)tr[5], (int)tr[6], tr[7], tr[8], tr[9],
                             (int)tr[10], (int)tr[11]);
            }
        }
        delete full;
    }
    return reached_end(hs, t);
}

// ------------------------------------------------------------ evolution without allocation
// te_evolve_noalloc runs the same kernels as te_evolve with its workspace (basis, product
// vector, reduction partials, device state, done flag) carved out of one file-scope device
// array instead of device memory the library allocates.  The array exists once per device
// (each device's code object holds its own copy, for the life of the process); host code
// never names it in a launch or copy, only through the address hipGetSymbolAddress returns
// for the current device on the first call there.
constexpr size_t kNoallocScratchBytes = (size_t)TE_NOALLOC_SCRATCH_BYTES;
constexpr int kNoallocMaxDevices = 64;
constexpr size_t kNoallocFlagBytes = 256;  // the done flag and restart records, first in the array

__device__ __align__(256) char scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu[kNoallocMaxDevices];     // one caller at a time per device
char* g_scratch_ptr[kNoallocMaxDevices] = {};     // device address of `scratch`, per device

// the scratch address on the current device (looked up once per device; caller holds the
// device's mutex)
te_status scratch_address(int dev, char** out) {
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TE_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (char*)p;
    }
    *out = g_scratch_ptr[dev];
    return TE_OK;
}

// Workspace view over the scratch array.  base stays null so that nothing is ever freed.
te_status noalloc_workspace(te_hamiltonian h, int m, char* sp, Workspace* w) {
    w->dim = h->csr.dim;
    w->m = m;
    w->ld = (int64_t)basis_ld(w->dim);
    w->tl = handle_tiling(h);
    size_t oy, op, on, orr, os;
    const size_t bytes = Workspace::layout(w->dim, m, w->tl, &oy, &op, &on, &orr, &os);
    if (bytes + kNoallocFlagBytes > kNoallocScratchBytes)
        return fail(TE_ERR_CAPACITY, "te_evolve_noalloc: dim " + std::to_string(w->dim) + " with m " +
                                         std::to_string(m) + " needs " + std::to_string(bytes + kNoallocFlagBytes) +
                                         " bytes of scratch, the maximum is " + std::to_string(kNoallocScratchBytes));
    char* ws = sp + kNoallocFlagBytes;
    w->bytes = bytes;
    w->V = (double2*)ws;
    w->y = (double2*)(ws + oy);
    w->rb.part = (double2*)(ws + op);
    w->rb.npart = (double*)(ws + on);
    w->rb.red = (double2*)(ws + orr);
    w->rb.n_tiles = w->tl.n_tiles_p;
    w->rb.n_norm = w->tl.n_tiles_u;
    w->st = (DevState*)(ws + os);
    w->host_flag_dev = (int*)sp;  // device memory here, read back with a copy
    return TE_OK;
}

te_status evolve_noalloc_locked(te_hamiltonian h, const te_c128* v0, te_c128* v_out, double t, double tol,
                                int32_t m, const te_options& o, te_result* res, hipStream_t s, char* sp) {
    const int dim = h->csr.dim;
    if (t == 0.0) {
        if (v_out != v0) TE_HIP(hipMemcpyAsync(v_out, v0, (size_t)dim * sizeof(te_c128), hipMemcpyDeviceToDevice, s));
        TE_HIP(hipStreamSynchronize(s));
        return TE_OK;
    }
    const int mm = std::min(m, dim);
    Workspace w;
    te_status rc = noalloc_workspace(h, mm, sp, &w);
    if (rc != TE_OK) return rc;
    // the array keeps the previous call's contents: clear the flags, the folded values and the
    // device state, as a fresh workspace starts
    TE_HIP(hipMemsetAsync(sp, 0, kNoallocFlagBytes, s));
    TE_HIP(hipMemsetAsync(w.rb.red, 0, (size_t)kMaxVals * sizeof(double2), s));
    TE_HIP(hipMemsetAsync(w.st, 0, sizeof(DevState), s));
    const Problem prob = make_problem(h, o, t, tol, mm);
    TE_HIP(launch_setup(w.st, prob, s));
    TE_HIP(launch_copy((const double2*)v0, w.V, dim, s));
    // Two restarts per check of the done flag: the second is a no-op when the first finished.
    const long max_restarts = 100000000L;
    for (long r = 0;; r += 2) {
        TE_HIP(enqueue_restart(h, &w, s));
        TE_HIP(enqueue_restart(h, &w, s));
        int done = 0;
        TE_HIP(hipMemcpyAsync(&done, w.host_flag_dev, sizeof(int), hipMemcpyDeviceToHost, s));
        TE_HIP(hipStreamSynchronize(s));
        if (done) break;
        if (r >= max_restarts) return fail(TE_ERR_DEVICE, "restart limit reached");
    }
    TE_HIP(launch_output(w.V, (double2*)v_out, dim, w.st, s));
    DevState hs;
    TE_HIP(hipMemcpyAsync(&hs, w.st, offsetof(DevState, alpha), hipMemcpyDeviceToHost, s));
    TE_HIP(hipStreamSynchronize(s));
    rc = finish_result(hs, t, res);
    if (rc != TE_OK) return rc;
    return reached_end(hs, t);
}

}  // namespace

extern "C" {

te_status te_evolve(te_hamiltonian h, const te_c128* v0, te_c128* v_out, double t, double tol, int32_t m,
                    const te_options* opt, te_result* res, void* stream) {
    return evolve_impl(h, v0, v_out, t, tol, m, opt, res, stream, nullptr, nullptr);
}

te_status te_evolve_noalloc(te_hamiltonian h, const te_c128* v0, te_c128* v_out, double t, double tol,
                            int32_t m, const te_options* opt, te_result* res, void* stream) {
    te_options o;
    te_status rc = check_evolve_args(h, v0, v_out, t, tol, m, opt, &o);
    if (rc != TE_OK) return rc;
    if (o.flags & TE_OPT_PROFILE) return fail(TE_ERR_INVALID_ARG, "te_evolve_noalloc takes no TE_OPT_PROFILE");
    if (res) std::memset(res, 0, sizeof(*res));
    int dev = -1;
    TE_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoallocMaxDevices) return fail(TE_ERR_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
    char* sp = nullptr;
    rc = scratch_address(dev, &sp);
    if (rc != TE_OK) return rc;
    std::lock_guard<std::mutex> hlock(h->mu);
    return evolve_noalloc_locked(h, v0, v_out, t, tol, m, o, res, (hipStream_t)stream, sp);
}

te_status te_evolve_sampled(te_hamiltonian h, const te_c128* v0, te_c128* v_out, double t, double tol,
                            int32_t m, const te_options* opt, const te_samples* smp, te_result* res,
                            void* stream) {
    if (!h || !v0 || !v_out || !smp) return fail(TE_ERR_INVALID_ARG, "null pointer");
    const int n = smp->n_times, n_obs = smp->n_obs;
    if (n < 0 || n_obs < 0) return fail(TE_ERR_INVALID_ARG, "negative sample or observable count");
    if (n == 0) return te_evolve(h, v0, v_out, t, tol, m, opt, res, stream);
    if (!smp->times) return fail(TE_ERR_INVALID_ARG, "null sample times");
    if (n_obs > 0 && (!smp->obs || !smp->obs_out)) return fail(TE_ERR_INVALID_ARG, "null observable pointer");
    if (!std::isfinite(t) || t < 0.0) return fail(TE_ERR_INVALID_ARG, "t must be finite and >= 0");
    for (int i = 0; i < n; ++i) {
        const double ti = smp->times[i];
        if (!(ti >= 0.0 && ti <= t) || (i > 0 && ti < smp->times[i - 1]))
            return fail(TE_ERR_INVALID_ARG, "sample times must be ascending and within [0, t]");
    }
    hipStream_t s = (hipStream_t)stream;
    const int dim = h->csr.dim;
    SampleBuffers sb;
    sb.n = n;
    sb.n_obs = n_obs;
    sb.states = (double2*)smp->states;
    sb.obs = smp->obs;
    sb.t = (double*)dev_alloc((size_t)n * sizeof(double));
    sb.omega = (double2*)dev_alloc((size_t)n * kMaxM * sizeof(double2));
    sb.bound = (double*)dev_alloc((size_t)n * sizeof(double));
    sb.obs_val = (double*)dev_alloc((size_t)n * std::max(n_obs, 1) * sizeof(double));
    auto release = [&]() {
        (void)hipStreamSynchronize(s);
        dev_free(sb.t);
        dev_free(sb.omega);
        dev_free(sb.bound);
        dev_free(sb.obs_part);
        dev_free(sb.obs_val);
    };
    if (!sb.t || !sb.omega || !sb.bound || !sb.obs_val) {
        release();
        return fail(TE_ERR_OUT_OF_MEMORY, "sample buffer allocation failed");
    }
    te_status rc = TE_OK;
    auto chk = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == TE_OK) rc = fail(TE_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    chk(hipMemcpyAsync(sb.t, smp->times, (size_t)n * sizeof(double), hipMemcpyHostToDevice, s), "copy times");
    chk(hipStreamSynchronize(s), "hipStreamSynchronize");
    DevState hs;
    std::memset(&hs, 0, offsetof(DevState, alpha));
    if (rc == TE_OK) rc = evolve_impl(h, v0, v_out, t, tol, m, opt, res, stream, &sb, &hs);
    if (rc == TE_OK && (hs.beta0 == -1.0 || hs.beta0 == 0.0)) {
        // t = 0: every sample is v0; ||v0|| = 0: every sample is zero
        const bool zero = hs.beta0 == 0.0;
        for (int i = 0; i < n && smp->states; ++i) {
            double2* dst = (double2*)smp->states + (size_t)i * dim;
            if (zero) chk(hipMemsetAsync(dst, 0, (size_t)dim * sizeof(double2), s), "clear state");
            else chk(hipMemcpyAsync(dst, v0, (size_t)dim * sizeof(double2), hipMemcpyDeviceToDevice, s), "copy v0");
        }
        std::vector<double> vals((size_t)std::max(n_obs, 1), 0.0);
        if (!zero && n_obs > 0 && rc == TE_OK) {
            const int tiles = (dim + kBlock - 1) / kBlock;
            sb.obs_part = (double*)dev_alloc((size_t)n_obs * tiles * sizeof(double));
            if (!sb.obs_part) rc = fail(TE_ERR_OUT_OF_MEMORY, "sample scratch allocation failed");
            if (rc == TE_OK) chk(launch_expect((const double2*)v0, dim, sb.obs, n_obs, sb.obs_part, tiles, s), "expect");
            if (rc == TE_OK) chk(launch_obs_fold(sb.obs_part, tiles, n_obs, sb.obs_val, s), "fold");
            if (rc == TE_OK)
                chk(hipMemcpyAsync(vals.data(), sb.obs_val, (size_t)n_obs * sizeof(double), hipMemcpyDeviceToHost, s),
                    "copy observables");
            chk(hipStreamSynchronize(s), "hipStreamSynchronize");
        }
        for (int i = 0; i < n && rc == TE_OK; ++i) {
            for (int o = 0; o < n_obs; ++o) smp->obs_out[(size_t)i * n_obs + o] = vals[(size_t)o];
            if (smp->bound_out) smp->bound_out[i] = 0.0;
        }
    } else if (rc == TE_OK) {
        if (hs.smp.next != n) rc = fail(TE_ERR_DEVICE, "not every sample time was reached");
        if (rc == TE_OK && n_obs > 0)
            chk(hipMemcpyAsync(smp->obs_out, sb.obs_val, (size_t)n * n_obs * sizeof(double), hipMemcpyDeviceToHost, s),
                "copy observables");
        if (rc == TE_OK && smp->bound_out)
            chk(hipMemcpyAsync(smp->bound_out, sb.bound, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s),
                "copy bounds");
    }
    release();
    return rc;
}

te_status te_autotune(te_hamiltonian h, int32_t m, te_tuning* out, void* stream) {
    if (!h) return fail(TE_ERR_INVALID_ARG, "null handle");
    if (m < 1 || m > TE_MAX_KRYLOV) return fail(TE_ERR_INVALID_ARG, "m out of range");
    std::lock_guard<std::mutex> lock(h->mu);
    Workspace* w = nullptr;
    te_status rc = get_workspace(h, std::min<int>(m, h->csr.dim), (hipStream_t)stream, &w);
    if (rc != TE_OK) return rc;
    h->tuned = false;
    rc = run_autotune(h, w, (hipStream_t)stream);
    if (rc == TE_OK && out) *out = h->tuning;
    return rc;
}

te_status te_get_tuning(te_hamiltonian h, te_tuning* out) {
    if (!h || !out) return fail(TE_ERR_INVALID_ARG, "null pointer");
    std::lock_guard<std::mutex> lock(h->mu);
    if (h->tuned) {
        *out = h->tuning;
    } else {
        const Tiling t = default_tiling(h->csr.dim);
        *out = te_tuning{t.g, t.u, t.rpt_p, t.rpt_u, t.split, 0.0};
    }
    return TE_OK;
}

te_status te_set_tuning(te_hamiltonian h, const te_tuning* t) {
    if (!h || !t) return fail(TE_ERR_INVALID_ARG, "null pointer");
    if (!tiling_supported(t->rows_per_thread, t->lanes_per_row, t->nnz_per_lane, t->update_rows_per_thread,
                          t->split_projection))
        return fail(TE_ERR_INVALID_ARG, "unsupported tuning (lanes x nonzeros 4x1, 4x4, 8x2, 2x8, 1x8 or 1x16; "
                                        "rows per thread 1, 2 or 4; update rows 1 or 2; split 0 or 1)");
    std::lock_guard<std::mutex> lock(h->mu);
    h->tuning = *t;
    h->tuned = true;
    if (h->ws) return retile(h, h->ws, handle_tiling(h));
    return TE_OK;
}

te_status te_last_profile(te_hamiltonian h, te_profile* out) {
    if (!h || !out) return fail(TE_ERR_INVALID_ARG, "null pointer");
    std::lock_guard<std::mutex> lock(h->mu);
    *out = h->prof;
    return TE_OK;
}

// ------------------------------------------------------------------ component entry points
te_status te_spmv(te_hamiltonian h, const te_c128* x, te_c128* y, te_c128* xhy, void* stream) {
    if (!h || !x || !y) return fail(TE_ERR_INVALID_ARG, "null pointer");
    if ((const void*)x == (void*)y) return fail(TE_ERR_INVALID_ARG, "x and y must not alias");
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(h->mu);
    Workspace* w = nullptr;
    te_status rc = get_workspace(h, h->ws ? h->ws->m : std::min(2, h->csr.dim), s, &w);
    if (rc != TE_OK) return rc;
    TE_HIP(launch_spmv_only(w->tl, h->csr, (const double2*)x, (double2*)y, w->st, w->rb, s));
    double2 dot;
    TE_HIP(hipMemcpyAsync(&dot, &w->st->ceff[0], sizeof(double2), hipMemcpyDeviceToHost, s));
    TE_HIP(hipStreamSynchronize(s));
    if (xhy) {
        xhy->re = dot.x;
        xhy->im = dot.y;
    }
    return TE_OK;
}

}  // extern "C"

extern "C" {

te_status te_arnoldi(te_hamiltonian h, const te_c128* u, int32_t m, double tol_rate, te_c128* V, double* alpha,
                     double* beta, int32_t* k_out, void* stream) {
    if (!h || !u || !V || !alpha || !beta || !k_out) return fail(TE_ERR_INVALID_ARG, "null pointer");
    if (m < 1 || m > TE_MAX_KRYLOV) return fail(TE_ERR_INVALID_ARG, "m out of range");
    if (!(tol_rate >= 0.0) || !std::isfinite(tol_rate)) return fail(TE_ERR_INVALID_ARG, "tol_rate must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(h->mu);
    const int dim = h->csr.dim;
    const int mm = std::min<int>(m, dim);
    Workspace* w = nullptr;
    te_status rc = get_workspace(h, mm, s, &w);
    if (rc != TE_OK) return rc;
    te_options o;
    te_default_options(&o);
    Problem prob = make_problem(h, o, 1.0, 1.0, mm);
    prob.tol_rate = tol_rate;
    TE_HIP(launch_setup(w->st, prob, s));
    TE_HIP(launch_copy((const double2*)u, w->V, dim, s));
    for (int j = 0; j < mm; ++j) {
        TE_HIP(launch_project(w->tl, h->csr, w->V, w->ld, j, w->y, w->st, w->rb, s));
        TE_HIP(launch_fold(j, w->st, w->rb, s));
        TE_HIP(launch_update(w->tl, w->V, w->ld, dim, j, w->y, w->st, w->rb, s));
    }
    TE_HIP(launch_last_norm(w->st, w->rb, s));
    DevState hs;
    TE_HIP(hipMemcpyAsync(&hs, w->st, offsetof(DevState, ceff), hipMemcpyDeviceToHost, s));
    TE_HIP(hipStreamSynchronize(s));
    if (hs.status != TE_OK) return fail(hs.status, "non-finite value during the Krylov build");
    if (hs.done) return fail(TE_ERR_INVALID_ARG, "start vector has zero norm");
    const int k = hs.k_limit;
    TE_HIP(launch_scale_columns(w->V, (double2*)V, w->ld, dim, k, w->st, s));
    TE_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < mm; ++i) {
        alpha[i] = (i < k) ? hs.alpha[i] : 0.0;
        beta[i] = (i < k) ? hs.beta[i] : 0.0;
    }
    *k_out = k;
    return TE_OK;
}

te_status te_tridiag_eig(int32_t k, const double* alpha, const double* beta, double* lambda, double* Q, void* stream) {
    if (!alpha || !lambda || !Q || (k > 1 && !beta)) return fail(TE_ERR_INVALID_ARG, "null pointer");
    if (k < 1 || k > TE_MAX_KRYLOV) return fail(TE_ERR_INVALID_ARG, "k out of range");
    for (int i = 0; i < k; ++i)
        if (!std::isfinite(alpha[i]) || (i < k - 1 && !std::isfinite(beta[i])))
            return fail(TE_ERR_NONFINITE, "non-finite tridiagonal entry");
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)k;
    double* d = (double*)dev_alloc((4 * n + n * n) * sizeof(double) + 64);
    if (!d) return fail(TE_ERR_OUT_OF_MEMORY, "device allocation failed");
    double *da = d, *db = d + n, *dl = d + 2 * n, *dq = d + 4 * n;
    int* dst = (int*)(d + 3 * n);
    te_status rc = TE_OK;
    int status = 0;
    auto chk = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == TE_OK) rc = fail(TE_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    chk(hipMemcpyAsync(da, alpha, n * sizeof(double), hipMemcpyHostToDevice, s), "copy");
    if (k > 1) chk(hipMemcpyAsync(db, beta, (n - 1) * sizeof(double), hipMemcpyHostToDevice, s), "copy");
    if (rc == TE_OK) chk(launch_eig_only(k, da, db, dl, dq, dst, s), "launch");
    if (rc == TE_OK) chk(hipMemcpyAsync(lambda, dl, n * sizeof(double), hipMemcpyDeviceToHost, s), "copy");
    if (rc == TE_OK) chk(hipMemcpyAsync(Q, dq, n * n * sizeof(double), hipMemcpyDeviceToHost, s), "copy");
    if (rc == TE_OK) chk(hipMemcpyAsync(&status, dst, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    if (rc == TE_OK) chk(hipStreamSynchronize(s), "sync");
    dev_free(d);
    if (rc == TE_OK && status) rc = fail(TE_ERR_DEVICE, "QL iteration did not converge");
    return rc;
}

te_status te_error_integral(int32_t k, const double* lambda, const double* coef, double h, double a, double b,
                            const te_options* opt, double* value, int32_t* level, int32_t* converged, void* stream) {
    if (!lambda || !coef || !value) return fail(TE_ERR_INVALID_ARG, "null pointer");
    if (k < 1 || k > TE_MAX_KRYLOV) return fail(TE_ERR_INVALID_ARG, "k out of range");
    if (!std::isfinite(a) || !std::isfinite(b) || b < a || !std::isfinite(h) || h < 0.0)
        return fail(TE_ERR_INVALID_ARG, "need finite a <= b and h >= 0");
    te_options o;
    te_default_options(&o);
    if (opt) o = *opt;
    te_status rc = check_options(o);
    if (rc != TE_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    Problem p{};
    p.quad_rel_tol = o.quad_rel_tol;
    p.quad_max_level = o.quad_max_level;
    p.quad_min_level = o.quad_min_level;
    p.gauss_n = o.quad_gauss_points;
    const size_t n = (size_t)k;
    double* d = (double*)dev_alloc((2 * n + 4) * sizeof(double));
    if (!d) return fail(TE_ERR_OUT_OF_MEMORY, "device allocation failed");
    double out[3] = {0, 0, 0};
    auto chk = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == TE_OK) rc = fail(TE_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    chk(hipMemcpyAsync(d, lambda, n * sizeof(double), hipMemcpyHostToDevice, s), "copy");
    chk(hipMemcpyAsync(d + n, coef, n * sizeof(double), hipMemcpyHostToDevice, s), "copy");
    if (rc == TE_OK) chk(launch_integral_only(k, d, d + n, h, a, b, p, d + 2 * n, s), "launch");
    if (rc == TE_OK) chk(hipMemcpyAsync(out, d + 2 * n, 3 * sizeof(double), hipMemcpyDeviceToHost, s), "copy");
    if (rc == TE_OK) chk(hipStreamSynchronize(s), "sync");
    dev_free(d);
    if (rc != TE_OK) return rc;
    *value = out[0];
    if (level) *level = (int32_t)out[1];
    if (converged) *converged = (int32_t)out[2];
    return TE_OK;
}

te_status te_step_search(int32_t k, const double* alpha, const double* beta, double h, double tol_rate, double t_rem,
                         int32_t first, double tau_prev, int32_t breakdown, const te_options* opt, double* tau,
                         double* err, te_c128* omega, uint32_t* warnings, void* stream) {
    if (!alpha || !tau || !err || !omega || (k > 1 && !beta)) return fail(TE_ERR_INVALID_ARG, "null pointer");
    if (k < 1 || k > TE_MAX_KRYLOV) return fail(TE_ERR_INVALID_ARG, "k out of range");
    if (!(t_rem > 0.0) || !std::isfinite(t_rem) || !(tol_rate > 0.0) || !std::isfinite(tol_rate) || !(h >= 0.0) ||
        !std::isfinite(h) || (!first && !(tau_prev > 0.0)))
        return fail(TE_ERR_INVALID_ARG, "invalid scalar argument");
    te_options o;
    te_default_options(&o);
    if (opt) o = *opt;
    te_status rc = check_options(o);
    if (rc != TE_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    DevState* hs = new (std::nothrow) DevState();
    if (!hs) return fail(TE_ERR_OUT_OF_MEMORY, "host allocation failed");
    std::memset(hs, 0, sizeof(DevState));
    Problem& p = hs->p;
    p.t = t_rem;
    p.tol_rate = tol_rate;
    p.t_init = o.t_init;
    p.shrink = o.shrink;
    p.quad_rel_tol = o.quad_rel_tol;
    p.m = k;
    p.n_substeps = o.n_substeps;
    p.quad_max_level = o.quad_max_level;
    p.quad_min_level = o.quad_min_level;
    p.max_halvings = o.max_halvings;
    p.gauss_n = o.quad_gauss_points;
    hs->k_limit = k;
    hs->h = h;
    hs->breakdown = breakdown ? 1 : 0;
    hs->first = first ? 1 : 0;
    hs->tau_prev = tau_prev;
    for (int i = 0; i < k; ++i) {
        hs->alpha[i] = alpha[i];
        hs->beta[i] = (i < k - 1) ? beta[i] : 0.0;
        hs->s[i] = 1.0;
    }
    DevState* d = (DevState*)dev_alloc(sizeof(DevState));
    if (!d) {
        delete hs;
        return fail(TE_ERR_OUT_OF_MEMORY, "device allocation failed");
    }
    auto chk = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == TE_OK) rc = fail(TE_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    chk(hipMemcpyAsync(d, hs, sizeof(DevState), hipMemcpyHostToDevice, s), "copy");
    if (rc == TE_OK) chk(launch_step_only(d, s), "launch");
    if (rc == TE_OK) chk(hipMemcpyAsync(hs, d, sizeof(DevState), hipMemcpyDeviceToHost, s), "copy");
    if (rc == TE_OK) chk(hipStreamSynchronize(s), "sync");
    dev_free(d);
    if (rc == TE_OK) {
        *tau = hs->last_tau;
        *err = hs->last_err;
        for (int i = 0; i < k; ++i) {
            omega[i].re = hs->omega[i].x;
            omega[i].im = hs->omega[i].y;
        }
        if (warnings) *warnings = (uint32_t)hs->warnings;
        if (hs->status == TE_ERR_STEP_UNDERFLOW) rc = fail(TE_ERR_STEP_UNDERFLOW, "no admissible step");
        else if (hs->status != TE_OK) rc = fail(hs->status, "device-side failure in the step search");
    }
    delete hs;
    return rc;
}

}  // extern "C"
