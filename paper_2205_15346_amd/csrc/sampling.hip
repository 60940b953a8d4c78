// Intermediate-time sampling (second remark after Alg. 1): the states and diagonal-observable
// reductions of the sample times a step covers, from that step's basis and coefficients (the
// step kernel writes the coefficients; see sample_coefficients in stepper.hip).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "te_internal.h"

namespace te {

// ------------------------------------------------------------------- sampled states
// Samples of the current step, four per pass over the basis: w_s = sum_i omega_s,i V[:, i]
// on this tile's rows; writes ||v0|| w_s to states[s] (if given) and, for every diagonal
// observable o, the tile's partial sum of D_o[r] |w_s[r]|^2 ||v0||^2.
constexpr int kSampleChunk = 4;

template <int RPT>
__global__ __launch_bounds__(kBlock) void k_samples(const double2* __restrict__ V, int64_t ld, int dim,
                                                     const DevState* __restrict__ st, double2* __restrict__ states,
                                                     const double* __restrict__ obs, int n_obs,
                                                     double* __restrict__ obs_part, int n_tiles) {
    __shared__ double lds[kWaves];
    const int lo = st->smp.lo, hi = st->smp.hi;
    if (lo >= hi) return;
    const int k = st->k_comb;
    const double b0 = st->beta0;
    const double2* __restrict__ om = st->smp.omega;
    const int r0 = blockIdx.x * (kBlock * RPT);
    for (int s0 = lo; s0 < hi; s0 += kSampleChunk) {
        const int ns = min(kSampleChunk, hi - s0);
        double2 w[kSampleChunk][RPT];
#pragma unroll
        for (int c = 0; c < kSampleChunk; ++c)
#pragma unroll
            for (int q = 0; q < RPT; ++q) w[c][q] = make_double2(0.0, 0.0);
        for (int i = 0; i < k; ++i) {
            const double2* __restrict__ vi = V + (int64_t)i * ld;
            double2 v[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int r = r0 + threadIdx.x + q * kBlock;
                v[q] = (r < dim) ? load_stream(vi + r) : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int c = 0; c < kSampleChunk; ++c) {
                if (c >= ns) break;
                const double2 a = om[(size_t)(s0 + c) * kMaxM + i];
#pragma unroll
                for (int q = 0; q < RPT; ++q) w[c][q] = cfma(a, v[q], w[c][q]);
            }
        }
#pragma unroll
        for (int c = 0; c < kSampleChunk; ++c) {
            if (c >= ns) break;
            const int smp = s0 + c;
            double p2[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const double2 x = cscale(w[c][q], b0);
                p2[q] = x.x * x.x + x.y * x.y;
                const int r = r0 + threadIdx.x + q * kBlock;
                if (states && r < dim) states[(size_t)smp * dim + r] = x;
            }
            for (int o = 0; o < n_obs; ++o) {
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const int r = r0 + threadIdx.x + q * kBlock;
                    if (r < dim) acc = fma(obs[(size_t)o * dim + r], p2[q], acc);
                }
                const double sum = block_sum(acc, lds);
                if (threadIdx.x == 0) obs_part[((size_t)smp * n_obs + o) * n_tiles + blockIdx.x] = sum;
                __syncthreads();
            }
        }
    }
}

// partials of <v| D_o |v> for one vector (sample slot 0 of obs_part), tiles of kBlock rows
__global__ __launch_bounds__(kBlock) void k_expect(const double2* __restrict__ v, int dim,
                                                    const double* __restrict__ obs, int n_obs,
                                                    double* __restrict__ obs_part, int n_tiles) {
    __shared__ double lds[kWaves];
    const int r = blockIdx.x * kBlock + threadIdx.x;
    double p2 = 0.0;
    if (r < dim) {
        const double2 x = v[r];
        p2 = x.x * x.x + x.y * x.y;
    }
    for (int o = 0; o < n_obs; ++o) {
        const double sum = block_sum(r < dim ? obs[(size_t)o * dim + r] * p2 : 0.0, lds);
        if (threadIdx.x == 0) obs_part[(size_t)o * n_tiles + blockIdx.x] = sum;
        __syncthreads();
    }
}

// out[value] = sum over tiles of obs_part[value][tile], one workgroup per value
__global__ __launch_bounds__(kBlock) void k_obs_fold(const double* __restrict__ obs_part, int n_tiles,
                                                      double* __restrict__ out) {
    __shared__ double lds[kWaves];
    double acc = 0.0;
    for (int t = threadIdx.x; t < n_tiles; t += kBlock) acc += obs_part[(size_t)blockIdx.x * n_tiles + t];
    const double sum = block_sum(acc, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = sum;
}

template <typename F>
static hipError_t by_rpt(int rpt, F&& f) {
    if (rpt == 1) f(std::integral_constant<int, 1>{});
    else f(std::integral_constant<int, 2>{});
    return hipGetLastError();
}

hipError_t launch_samples(int rpt, const double2* V, int64_t ld, int dim, const DevState* st, double2* states,
                          const double* obs, int n_obs, double* obs_part, int n_tiles, hipStream_t s) {
    return by_rpt(rpt, [&](auto r) {
        k_samples<decltype(r)::value><<<n_tiles, kBlock, 0, s>>>(V, ld, dim, st, states, obs, n_obs, obs_part,
                                                                  n_tiles);
    });
}

hipError_t launch_expect(const double2* v, int dim, const double* obs, int n_obs, double* obs_part, int n_tiles,
                         hipStream_t s) {
    k_expect<<<n_tiles, kBlock, 0, s>>>(v, dim, obs, n_obs, obs_part, n_tiles);
    return hipGetLastError();
}

hipError_t launch_obs_fold(const double* obs_part, int n_tiles, int n_values, double* out, hipStream_t s) {
    if (n_values <= 0) return hipSuccess;
    k_obs_fold<<<n_values, kBlock, 0, s>>>(obs_part, n_tiles, out);
    return hipGetLastError();
}

}  // namespace te
