// Internal declarations shared by the HIP sources of libtimeevolve (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>

#include "te.h"

namespace te {

constexpr int kBlock = 256;      // threads per workgroup of the row-parallel kernels
constexpr int kWaves = kBlock / 64;
constexpr int kMaxM = TE_MAX_KRYLOV;
constexpr int kGroup = 16;       // tiles per first-level reduction group
constexpr int kMaxVals = 2 * (kMaxM + 1);  // values one tile contributes to a reduction
constexpr int kTrace = 64;                 // restarts kept in the device trace ring
constexpr int kTraceFields = 12;  // t_now, tau, err, h, k, breakdown, quad_ok, t_rem,
                                  // eigensolve us, step-search us, integrals, max level

// ---------------------------------------------------------------------------------------
// Solver state kept in device memory for one evolution.  Written only by the single
// "finisher" workgroup of a kernel (the last one to arrive) or by the one-block step kernel.
struct Problem {
    double t, tol_rate, numerr_per_step;
    double t_init, shrink, quad_rel_tol;
    int32_t m, dim;
    int32_t n_substeps, quad_max_level, quad_min_level, max_halvings;
    int32_t three_term;  // Krylov step: 0 full re-orthogonalisation, 1 three-term recurrence only
    int32_t gauss_n;     // error integral: 0 adaptive tanh-sinh, n > 0 the n-point Gauss-Legendre rule
};

// Intermediate-time sampling (second remark after Alg. 1): the step kernel computes the Krylov
// coefficients of the sample times its step covers; the sample kernel forms those states.
struct SampleState {
    const double* t;   // [n] ascending sample times (device)
    double2* omega;    // [n][kMaxM] coefficients on the raw basis columns
    double* bound;     // [n] bound at the end of the step holding the sample (times ||v0||)
    int32_t n;         // 0: no sampling
    int32_t next;      // first sample not yet assigned to a step
    int32_t lo, hi;    // samples of the current step
};

struct DevState {
    Problem p;  // set by the setup kernel
    double beta0;
    // progress
    double t_now, tau_prev, err_acc, num_acc;
    int32_t first, done, do_combine, status;
    int32_t steps, matvecs, breakdown_dim, warnings;
    // current Krylov build
    int32_t k_limit;   // iterations j < k_limit still run (m, or k after a breakdown)
    int32_t breakdown; // lucky breakdown in this build
    int32_t k_comb;    // columns the recombination uses
    int32_t norm_init; // column 0 is the raw v0: take s[0] = 1/||column 0|| at the next projection
    int32_t counted;   // batched engine: completion already reported to the host
    int32_t pad_;
    double h;          // residual norm h_{k+1,k}
    double ys;         // scale of the raw product y = H V[:, j] (s[j])
    double last_tau, last_err;
    double alpha[kMaxM];
    double beta[kMaxM];
    double s[kMaxM + 1];        // column scales: normalised v_i = s[i] * V[:, i]
    double2 ceff[kMaxM];        // orthogonalisation coefficients on the raw columns
    double2 omega[kMaxM];       // recombination coefficients on the raw columns
    double2 gcol[2][kMaxM + 1]; // Gram column v_i^H v_j of iteration j in gcol[j & 1]
    double trace[kTrace][kTraceFields];  // restart r in row r % kTrace
    SampleState smp;                     // cleared by the setup kernel
};

// Reduction scratch: every tile of a row-parallel kernel writes its partial sums with plain
// stores and a later kernel folds them in a fixed order.  All cross-workgroup communication
// goes through kernel boundaries: no atomics or device-scope fences on the hot path.
struct RedBuf {
    double2* part;   // [kMaxVals][n_tiles] projection partials
    double* npart;   // [n_tiles] squared-norm partials of the last residual
    double2* red;    // [kMaxVals] folded projection values
    int n_tiles;     // tiles of the projection kernel (rows of part)
    int n_norm;      // tiles of the update kernel (entries of npart)
};

// -------------------------------------------------------------------- batched engine
// Packed entries: entry k of row r holds a code q; q stands for column r + toff[q] and value
// tval[q], except q = dcode, the row's diagonal: column r, value (diag[r], 0).  Codes are one
// byte when there are at most 255 distinct (column offset, value) pairs off the diagonal, else
// two bytes.  Value codes: when the pairs are too many but the values few, col keeps every
// entry's column and the codes index values only (toff is then all zero); codes and columns
// are then sliced: rows in chunks of 64, entry q of row r at slice[r / 64] + 64 q + r % 64
// (a chunk is as wide as its longest row).
struct Packed {
    const uint8_t* c8 = nullptr;    // 1-byte codes, or
    const uint16_t* c16 = nullptr;  // 2-byte codes (at most one is set)
    const int* col = nullptr;       // value codes: the columns (sliced), or
    const uint16_t* col16 = nullptr;  // value codes: column - cbase[group] (sliced), with
    const int* cbase = nullptr;     //   one base per group (chunk of 64 rows, entry position)
    const int* slice = nullptr;     // value codes: [ceil(dim / 64)] chunk offsets (multiples of 64)
    const int* toff = nullptr;      // [dcode + 1] column offsets, toff[dcode] = 0
    const double2* tval = nullptr;  // [dcode + 1] values
    const double* diag = nullptr;   // [dim] real diagonal (0 where a row has none)
    int dcode = 0;
};

// One evolution job of a batched round: its matrix, basis, state and reduction scratch.
struct JobView {
    const int* rp;
    const int* ci;
    const double2* val;  // complex entries, or
    const double* rval;  // real entries, or
    Packed pk;           // packed entries (exactly one of the three is set)
    double2* V;          // basis columns, leading dimension ld
    double2* y;          // raw product H V[:, j]
    DevState* st;
    RedBuf rb;           // n_tiles = projection tiles (kBlock * rows per thread rows each)
    const double2* v0;   // caller's initial vector (read at admission)
    double2* out;        // caller's output vector (written when the job completes)
    int64_t ld;
    int64_t id;          // engine job id, echoed in the completion record
    int dim;
    int slot;            // index of the completion record
};

constexpr int kMaxGroup = 8;  // vectors sharing one sparse-matrix stream

// Jobs of one matrix whose sparse products run as one multi-vector product.
struct GroupView {
    const int* rp;
    const int* ci;
    const double2* val;    // complex entries, or
    const double* rval;    // real entries, or
    Packed pk;             // packed entries (exactly one of the three is set)
    int dim;
    int nv;                // jobs in the group (1..kMaxGroup)
    int job[kMaxGroup];    // indices into the round's JobView array
};

// Per-round record of a running job, written by the device into host-mapped memory at the end
// of every round until the round in which the job completes (done = 1).  Records alternate
// between two banks by round parity, so the host reads the bank of a finished round while the
// next round writes the other one.
struct SlotOut {
    int64_t id;
    int32_t done, status;
    int32_t steps, matvecs, breakdown_dim, warnings;
    int32_t last_k, round;  // Krylov dimension of the job's last restart; round (1-based)
    double beta0, err_acc, num_acc, t_now;
};

// Round bookkeeping written by the device into host-mapped memory.
struct RoundOut {
    int32_t rounds;   // rounds completed since the engine started
    int32_t active;   // jobs of the finished round still running
    int32_t pad_[14];
};

// -------------------------------------------------------------------- complex helpers
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// a*b
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// acc + a*b
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc + conj(a)*b
__device__ __forceinline__ double2 cfma_conj(double2 a, double2 b, double2 acc) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
// acc - a*b
__device__ __forceinline__ double2 cfms(double2 a, double2 b, double2 acc) {
    acc.x = fma(-a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(-a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}

// Basis columns are streamed once per pass and not reused before the pass ends, so they are
// read with non-temporal loads: they then do not evict the CSR arrays and the product vector
// from the caches, which the next sparse product reads again (measured: a sparse product after a
// 40-column pass runs 14% faster when that pass used non-temporal loads).
__device__ __forceinline__ double2 load_stream(const double2* p) {
    double2 v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Block-wide sum in a fixed order; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* lds /* kWaves */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += lds[w];
    return s;
}

// Block-wide maximum; every thread gets the result.
__device__ __forceinline__ double block_max(double v, double* lds /* kWaves */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = lds[0];
    for (int w = 1; w < kWaves; ++w) s = fmax(s, lds[w]);
    return s;
}

// ----------------------------------------------------------------------- launchers
struct Workspace;  // defined in api.hip

// Exactly one of val (complex entries with columns), rval (real entries with columns) and
// pk (packed entries, col unset) is set.
struct Csr {
    const int* row_ptr;
    const int* col;
    const double2* val;
    const double* rval;
    Packed pk;
    int dim;
    int64_t nnz;
};

inline bool is_packed(const Packed& p) { return p.c8 != nullptr || p.c16 != nullptr; }

// bytes a sparse product streams for the stored entries (row pointers and vectors aside):
// value + column index per entry, or a code (and with value codes a column) per entry and the
// real diagonal per row
inline double csr_entries_bytes(const Csr& c) {
    const double nnz = (double)c.nnz, d = (double)c.dim;
    // the sliced padding and the 16-bit form's bases (one per 64 entry slots) are not counted
    const double cols = c.pk.col ? 4.0 * nnz : c.pk.col16 ? 2.0 * nnz : 0.0;
    if (c.pk.c8) return 1.0 * nnz + cols + 8.0 * d;
    if (c.pk.c16) return 2.0 * nnz + cols + 8.0 * d;
    return (c.rval ? 12.0 : 20.0) * nnz;
}

// Row tiling of the row-parallel kernels.  The projection kernel's shape is chosen per matrix
// by the autotuner: g lanes share a row of the sparse product, each keeping u nonzeros in
// flight, and every thread owns rpt_p rows of the dense passes.
struct Tiling {
    int rpt_p;      // rows per thread, projection kernel (1, 2 or 4)
    int g;          // lanes per row in the sparse product (1, 2, 4 or 8)
    int u;          // nonzeros per lane in flight (g = 1: 8 or 16; 2: 8; 4: 1 or 4; 8: 2)
    int n_tiles_p;  // tiles (workgroups) of the projection kernel
    int rpt_u;      // rows per thread, update and recombination kernels (1 or 2)
    int n_tiles_u;
    int split;      // 1: sparse product and projections as two launches (y read back)
};
Tiling make_tiling(int dim, int rpt_p, int g, int u, int rpt_u, int split);
Tiling default_tiling(int dim);
bool tiling_supported(int rpt_p, int g, int u, int rpt_u, int split);
int max_tiles(int dim);  // tiles of the finest tiling (rpt = 1): sizes the partial buffers

hipError_t launch_setup(DevState* st, const Problem& prob, hipStream_t s);
hipError_t launch_copy(const double2* src, double2* dst, int dim, hipStream_t s);
// The optional events of the single-solve launchers are bound to the dispatches themselves
// (profiling: `start` at the first kernel's start, `done` at the last kernel's end).
hipError_t launch_project(const Tiling& tl, const Csr& H, const double2* V, int64_t ld, int j, double2* y,
                          const DevState* st, const RedBuf& rb, hipStream_t s, hipEvent_t start = nullptr,
                          hipEvent_t done = nullptr);
hipError_t launch_fold(int j, const DevState* st, const RedBuf& rb, hipStream_t s, hipEvent_t done = nullptr);
hipError_t launch_update(const Tiling& tl, double2* V, int64_t ld, int dim, int j, const double2* y,
                         DevState* st, const RedBuf& rb, hipStream_t s, hipEvent_t done = nullptr);
hipError_t launch_last_norm(DevState* st, const RedBuf& rb, hipStream_t s);
hipError_t launch_combine(const Tiling& tl, double2* V, int64_t ld, int dim, const DevState* st, hipStream_t s,
                          hipEvent_t done = nullptr);
hipError_t launch_output(const double2* V, double2* out, int dim, const DevState* st, hipStream_t s);
hipError_t launch_step(DevState* st, const RedBuf& rb, int* host_flag, hipStream_t s, hipEvent_t done = nullptr);
hipError_t launch_spmv_only(const Tiling& tl, const Csr& H, const double2* x, double2* y, DevState* st,
                            const RedBuf& rb, hipStream_t s);
hipError_t launch_scale_columns(const double2* src, double2* dst, int64_t ld, int dim, int k, const DevState* st,
                                hipStream_t s);
hipError_t launch_validate(const Csr& H, int check_hermitian, int* err, double* rowsum, hipStream_t s);
hipError_t launch_norm1(const double* rowsum, int dim, double* out, hipStream_t s);
hipError_t launch_real_part(const double2* val, double* rval, int64_t n, hipStream_t s);
hipError_t launch_expand_real(const double* rval, double2* val, int64_t n, hipStream_t s);
// Columns and complex values of packed entries (inverse of the packing).
hipError_t launch_expand_packed(const int* row_ptr, const Packed& pk, int dim, int* col, double2* val, hipStream_t s);

// Device construction of the paper's exemplary Hamiltonian (models.hip): sizes, parameters and
// device tables prepared by te_hamiltonian_create_memory_burden.
struct MemoryBurdenDev {
    int n, K, Nm, N0;      // qubit modes (K + K'), a-type qubits, excitations, bosons
    int64_t C;             // qubit configurations binom(n, Nm)
    int slots;             // power of two >= longest row, <= 512
    int64_t dim;
    double eps_m, Nc, NcMinusDNc, C0;
    const int64_t* binom;  // [64 * 64] binomials
    const double* hop;     // [64 * 64] symmetric hopping amplitudes of the qubit pairs
};
hipError_t launch_memory_burden(const MemoryBurdenDev& M, int* row_ptr, int* col, double* val, hipStream_t s);

// Device construction of the Bose chain (models.hip): K modes, N bosons, on-site interaction and
// nearest-neighbour hopping; tables prepared by te_hamiltonian_create_bose_chain.
struct BoseChainDev {
    int K, N;
    int slots;             // power of two >= 2K - 1, <= 128
    int64_t dim;           // <= kMaxModelRows
    int bw;                // row stride of binom
    const int64_t* binom;  // [(N + K + 1) * bw] binomials C(a, b), b <= K
    const double* U;       // [K]
    const double2* hop;    // [K - 1]
};
// Row counts and their exclusive scan: row_ptr[dim + 1]; cnt: dim ints; scratch: dim / 1024 + 2
// int64, whose entry [ceil(dim / 1024)] receives the number of entries.
hipError_t launch_bose_row_ptr(const BoseChainDev& B, int* row_ptr, int* cnt, int64_t* scratch, hipStream_t s);
// Columns (ascending per row) and values of every row, into arrays of row_ptr[dim] entries.
hipError_t launch_bose_fill(const BoseChainDev& B, const int* row_ptr, int* col, double2* val, hipStream_t s);
// Rows of a matrix built on the device: one wavefront per row, 4 rows per 256-thread workgroup,
// so the grid's thread count stays below 2^32.
constexpr int64_t kMaxModelRows = (int64_t)1 << 26;

// batched launchers: items are (group or job, tile) pairs, one workgroup each
hipError_t launch_gproject(int g, int u, int rpt, int nv_class, const JobView* jobs, const GroupView* groups,
                           const int2* items, int n_items, int j, hipStream_t s);
hipError_t launch_bdots(int rpt, const JobView* jobs, const int2* items, int n_items, int j, hipStream_t s);
hipError_t launch_bfold(const JobView* jobs, int n_jobs, int j, hipStream_t s);
hipError_t launch_bupdate(int rpt, const JobView* jobs, const int2* items, int n_items, int j, hipStream_t s);
hipError_t launch_bstep(const JobView* jobs, int n_jobs, hipStream_t s);
hipError_t launch_bcombine(int rpt, const JobView* jobs, const int2* items, int n_items, hipStream_t s);
hipError_t launch_bsetup(const JobView* jobs, const Problem* probs, int n_jobs, hipStream_t s);
hipError_t launch_bcopy_in(int rpt, const JobView* jobs, const int2* items, int n_items, hipStream_t s);
hipError_t launch_bcopy_out(int rpt, const JobView* jobs, const int2* items, int n_items, hipStream_t s);
hipError_t launch_bflag(const JobView* jobs, int n_jobs, int* rounds_dev, SlotOut* slots, int max_slots,
                        RoundOut* ro, hipStream_t s);
bool gproject_supported(int g, int u);

// component kernels (one block)
hipError_t launch_eig_only(int k, const double* alpha, const double* beta, double* lambda, double* Q,
                           int* status, hipStream_t s);
hipError_t launch_integral_only(int k, const double* lambda, const double* coef, double h, double a, double b,
                                const Problem& opt, double* out, hipStream_t s);
hipError_t launch_step_only(DevState* st, hipStream_t s);

// sampling: states / diagonal-observable partials of the current step's samples, and the fold
hipError_t launch_samples(int rpt, const double2* V, int64_t ld, int dim, const DevState* st, double2* states,
                          const double* obs, int n_obs, double* obs_part, int n_tiles, hipStream_t s);
hipError_t launch_expect(const double2* v, int dim, const double* obs, int n_obs, double* obs_part, int n_tiles,
                         hipStream_t s);
hipError_t launch_obs_fold(const double* obs_part, int n_tiles, int n_values, double* out, hipStream_t s);

// ------------------------------------------------------------- host-side shared helpers
te_status set_error(te_status s, const std::string& msg);  // thread-local te_last_error text
// te_set_allocator hook or hipMalloc; the stream is the one the memory is first used on
void* dev_alloc(size_t bytes, hipStream_t stream = nullptr);
void dev_free(void* p);  // returns a block to the allocator that supplied it
te_status check_options(const te_options& o);
size_t align_up(size_t x, size_t a);
// leading dimension (elements) of a basis: one column per Krylov vector
size_t basis_ld(int64_t dim);

}  // namespace te

// A Hamiltonian handle: device CSR, its 1-norm, and the single-solve workspace and tuning.
struct te_hamiltonian_s {
    te::Csr csr{};
    int* row_ptr = nullptr;
    int* col = nullptr;
    double2* val = nullptr;
    double* rval = nullptr;
    void* code = nullptr;      // packed entries: codes, table and diagonal
    int* slice = nullptr;      // value codes: chunk offsets
    int* toff = nullptr;
    double2* tval = nullptr;
    double* diag = nullptr;
    double norm1 = 0.0;
    std::mutex mu;
    te::Workspace* ws = nullptr;
    te_profile prof{};
    bool tuned = false;  // tuning measured or set explicitly
    te_tuning tuning{4, 4, 1, 1, 0, 0.0};
    ~te_hamiltonian_s();
};

namespace te {

// Per-solve constants of Alg. 1 for one (H, t, tol, m).
Problem make_problem(const te_hamiltonian_s* h, const te_options& o, double t, double tol, int m);

// Whole block: fold the squared-norm partials of the last residual (iteration m-1) into
// h = ||p|| and test it for a lucky breakdown.  No-op when a breakdown already set k < m.
__device__ inline void finish_last_norm(DevState* st, const RedBuf& rb, double* lds) {
    if (st->done || st->breakdown) return;
    double acc = 0.0;
    for (int t = threadIdx.x; t < rb.n_norm; t += kBlock) acc += rb.npart[t];
    const double h2 = block_sum(acc, lds);
    if (threadIdx.x == 0) {
        const double h = sqrt(h2);
        st->beta[st->p.m - 1] = h;
        st->h = h;
        if (!isfinite(h)) {
            st->status = TE_ERR_NONFINITE;
            st->done = 1;
        } else if (h < st->p.tol_rate) {
            st->breakdown = 1;
        }
    }
    __threadfence_block();
    __syncthreads();
}

}  // namespace te
