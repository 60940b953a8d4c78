// Internal declarations shared by the HIP sources of libtimeevolve (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "te.h"

namespace te {

constexpr int kBlock = 256;      // threads per workgroup of the row-parallel kernels
constexpr int kWaves = kBlock / 64;
constexpr int kMaxM = TE_MAX_KRYLOV;
constexpr int kGroup = 16;       // tiles per first-level reduction group
constexpr int kMaxVals = 2 * (kMaxM + 1);  // values one tile contributes to a reduction

// ---------------------------------------------------------------------------------------
// Solver state kept in device memory for one evolution.  Written only by the single
// "finisher" workgroup of a kernel (the last one to arrive) or by the one-block step kernel.
struct Problem {
    double t, tol_rate, numerr_per_step;
    double t_init, shrink, quad_rel_tol;
    int32_t m, dim;
    int32_t n_substeps, quad_max_level, quad_min_level, max_halvings;
};

struct DevState {
    Problem p;  // set by the init kernel
    double beta0;
    // progress
    double t_now, tau_prev, err_acc, num_acc;
    int32_t first, done, do_combine, status;
    int32_t steps, matvecs, breakdown_dim, warnings;
    // current Krylov build
    int32_t k_limit;   // iterations j < k_limit still run (m, or k after a breakdown)
    int32_t breakdown; // lucky breakdown in this build
    int32_t k_comb;    // columns the recombination uses
    int32_t pad0;
    double h;          // residual norm h_{k+1,k}
    double last_tau, last_err;
    double alpha[kMaxM];
    double beta[kMaxM];
    double s[kMaxM + 1];      // column scales: normalised v_i = s[i] * V[:, i]
    double2 ceff[kMaxM];      // orthogonalisation coefficients on the raw columns
    double2 omega[kMaxM];     // recombination coefficients on the raw columns
    double2 G[kMaxM * kMaxM]; // Gram matrix of the normalised basis, G[i*kMaxM + j]
};

// Scratch of the deterministic two-level grid reduction: tiles write partials, the last
// tile of each group of kGroup folds its group, the last group folds the groups.
struct RedBuf {
    double2* part;   // [kMaxVals][n_tiles]
    double2* gpart;  // [kMaxVals][n_groups]
    unsigned* gcnt;  // [n_groups], zero between kernels
    unsigned* fcnt;  // [1], zero between kernels
    int n_tiles, n_groups;
};

// -------------------------------------------------------------------- complex helpers
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sums `nv` values that every thread of the block holds in vals[] (identical layout),
// result in out[] (LDS, visible to all threads after return).  Fixed order.
template <int NV>
__device__ __forceinline__ void block_sum(const double (&vals)[NV], double* out, double* lds /* kWaves*NV */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double s = wave_sum(vals[v]);
        if (lane == 0) lds[wave * NV + v] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += lds[w * NV + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Two-level deterministic grid reduction of `nv` complex values per tile.  Every block
// calls it with its tile partials in `vals` (LDS).  Returns true in exactly one block
// (the last to arrive), which then holds the grid totals in `vals`.
__device__ inline bool grid_reduce(double2* vals, int nv, int tile, const RedBuf& rb) {
    __shared__ unsigned ticket;
    __shared__ double2 tmp[kBlock];
    const int tid = threadIdx.x;
    for (int v = tid; v < nv; v += kBlock) rb.part[(size_t)v * rb.n_tiles + tile] = vals[v];
    __threadfence();
    __syncthreads();
    const int group = tile / kGroup;
    const int g0 = group * kGroup;
    const int gs = min(kGroup, rb.n_tiles - g0);
    if (tid == 0) ticket = atomicAdd(&rb.gcnt[group], 1u);
    __syncthreads();
    if (ticket != (unsigned)(gs - 1)) return false;
    __threadfence();
    // fold this group's gs tiles: thread -> (value, stripe), fixed order
    {
        const int stripes = max(1, min(gs, kBlock / max(nv, 1)));
        for (int v0 = 0; v0 < nv; v0 += kBlock / stripes) {
            const int v = v0 + tid % (kBlock / stripes);
            const int st = tid / (kBlock / stripes);
            double2 acc = make_double2(0.0, 0.0);
            if (v < nv && st < stripes) {
                for (int t = st; t < gs; t += stripes) acc = cadd(acc, rb.part[(size_t)v * rb.n_tiles + g0 + t]);
            }
            tmp[tid] = acc;
            __syncthreads();
            if (tid < kBlock / stripes && v0 + tid < nv) {
                double2 s = make_double2(0.0, 0.0);
                for (int q = 0; q < stripes; ++q) s = cadd(s, tmp[q * (kBlock / stripes) + tid]);
                rb.gpart[(size_t)(v0 + tid) * rb.n_groups + group] = s;
            }
            __syncthreads();
        }
    }
    if (tid == 0) rb.gcnt[group] = 0u;
    __threadfence();
    __syncthreads();
    if (tid == 0) ticket = atomicAdd(rb.fcnt, 1u);
    __syncthreads();
    if (ticket != (unsigned)(rb.n_groups - 1)) return false;
    __threadfence();
    {
        const int ng = rb.n_groups;
        const int stripes = max(1, min(ng, kBlock / max(nv, 1)));
        for (int v0 = 0; v0 < nv; v0 += kBlock / stripes) {
            const int v = v0 + tid % (kBlock / stripes);
            const int st = tid / (kBlock / stripes);
            double2 acc = make_double2(0.0, 0.0);
            if (v < nv && st < stripes) {
                for (int g = st; g < ng; g += stripes) acc = cadd(acc, rb.gpart[(size_t)v * ng + g]);
            }
            tmp[tid] = acc;
            __syncthreads();
            if (tid < kBlock / stripes && v0 + tid < nv) {
                double2 s = make_double2(0.0, 0.0);
                for (int q = 0; q < stripes; ++q) s = cadd(s, tmp[q * (kBlock / stripes) + tid]);
                vals[v0 + tid] = s;
            }
            __syncthreads();
        }
    }
    if (tid == 0) *rb.fcnt = 0u;
    __syncthreads();
    return true;
}

// ----------------------------------------------------------------------- launchers
struct Workspace;  // defined in api.hip

struct Csr {
    const int* row_ptr;
    const int* col;
    const double2* val;
    int dim;
    int64_t nnz;
};

// Row tiling of the row-parallel kernels.
struct Tiling {
    int rpt;      // rows per thread
    int g;        // lanes per row in the sparse product
    int rows;     // rows per tile = kBlock * rpt
    int n_tiles;
    int n_groups;
};
Tiling choose_tiling(int dim);

hipError_t launch_init(const Tiling& tl, const double2* v0, double2* V, int dim, DevState* st,
                       const RedBuf& rb, const Problem& prob, hipStream_t s);
hipError_t launch_project(const Tiling& tl, const Csr& H, double2* V, int64_t ld, int j, double2* y,
                          DevState* st, const RedBuf& rb, hipStream_t s);
hipError_t launch_update(const Tiling& tl, double2* V, int64_t ld, int dim, int j, const double2* y,
                         DevState* st, const RedBuf& rb, hipStream_t s);
hipError_t launch_combine(const Tiling& tl, double2* V, int64_t ld, int dim, DevState* st, hipStream_t s);
hipError_t launch_output(const Tiling& tl, const double2* V, double2* out, int dim, const DevState* st,
                         hipStream_t s);
hipError_t launch_step(DevState* st, int* host_flag, hipStream_t s);
hipError_t launch_spmv_only(const Tiling& tl, const Csr& H, const double2* x, double2* y, DevState* st,
                            const RedBuf& rb, hipStream_t s);
hipError_t launch_validate(const Csr& H, int check_hermitian, int* err, double* rowsum, hipStream_t s);
hipError_t launch_norm1(const double* rowsum, int dim, double* out, hipStream_t s);

// component kernels (one block)
hipError_t launch_eig_only(int k, const double* alpha, const double* beta, double* lambda, double* Q,
                           int* status, hipStream_t s);
hipError_t launch_integral_only(int k, const double* lambda, const double* coef, double h, double a, double b,
                                const Problem& opt, double* out, hipStream_t s);
hipError_t launch_step_only(DevState* st, hipStream_t s);

}  // namespace te
