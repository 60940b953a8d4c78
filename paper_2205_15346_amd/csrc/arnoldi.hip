// Row-parallel kernels of one Krylov build (paper, eq. arnoldi / Alg. 1 step 1, carried out
// as Lanczos on H with full re-orthogonalisation) and of the restart recombination
// (Alg. 1 step 3, w = V omega).
//
// Orthogonalisation scheme (differs from the paper's modified Gram-Schmidt, same result in
// exact arithmetic): iteration j makes two passes over the basis.
//   pass A  y = H v_j fused with all projections c'_i = v_i^H y and the Gram column
//           g_i = v_i^H v_j (i <= j), one read of V_j;
//   pass B  v_{j+1} = y - sum_i c_i v_i with c = G^{-1} c' (G = V^H V, first-order
//           corrections), plus ||v_{j+1}||^2, one read of V_j and one write.
// Using the measured Gram matrix keeps the new vector orthogonal to O(eps ||H||/beta)
// without a second classical Gram-Schmidt sweep.  Normalisation is deferred: column i is
// stored unnormalised and s[i] = 1/||column|| is applied on use.
#include <algorithm>
#include <type_traits>

#include "te_internal.h"

namespace te {

Tiling choose_tiling(int dim) {
    Tiling t;
    // aim for >= ~512 tiles on large problems (two per CU), more rows per thread only
    // when the tile count stays high
    int rpt = 1;
    while (rpt < 8 && (int64_t)dim >= (int64_t)kBlock * rpt * 2 * 512) rpt *= 2;
    t.rpt = rpt;
    t.g = 4;
    t.rows = kBlock * rpt;
    t.n_tiles = (dim + t.rows - 1) / t.rows;
    t.n_groups = (t.n_tiles + kGroup - 1) / kGroup;
    return t;
}

// ------------------------------------------------------------------------ init
// V[:,0] = v0, ||v0||^2 -> beta0, s[0] = 1/beta0; the finisher also sets up the state.
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_init(const double2* __restrict__ v0, double2* __restrict__ V,
                                                  int dim, DevState* __restrict__ st, RedBuf rb, Problem prob) {
    __shared__ double lds[kWaves];
    __shared__ double2 vals[1];
    const int rows = kBlock * RPT;
    const int r0 = blockIdx.x * rows;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = r0 + threadIdx.x + q * kBlock;
        if (r < dim) {
            const double2 v = v0[r];
            V[r] = v;
            acc = fma(v.x, v.x, acc);
            acc = fma(v.y, v.y, acc);
        }
    }
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        double s = wave_sum(acc);
        if (lane == 0) lds[wave] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double b = 0.0;
            for (int w = 0; w < kWaves; ++w) b += lds[w];
            vals[0] = make_double2(b, 0.0);
        }
        __syncthreads();
    }
    if (!grid_reduce(vals, 1, blockIdx.x, rb)) return;
    if (threadIdx.x == 0) {
        const double nrm2 = vals[0].x;
        st->p = prob;
        st->t_now = 0.0;
        st->tau_prev = prob.t_init;
        st->err_acc = 0.0;
        st->num_acc = 0.0;
        st->first = 1;
        st->done = 0;
        st->do_combine = 0;
        st->status = TE_OK;
        st->steps = 0;
        st->matvecs = 0;
        st->breakdown_dim = 0;
        st->warnings = 0;
        st->k_limit = prob.m;
        st->breakdown = 0;
        st->k_comb = 0;
        st->h = 0.0;
        const double beta0 = sqrt(nrm2);
        st->beta0 = beta0;
        if (!isfinite(nrm2)) {
            st->status = TE_ERR_NONFINITE;
            st->done = 1;
        } else if (beta0 == 0.0) {
            st->done = 1;
        } else {
            st->s[0] = 1.0 / beta0;
        }
    }
}

// -------------------------------------------------------------- pass A: SpMV + projections
template <int RPT, int G>
__global__ __launch_bounds__(kBlock) void k_project(const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const double2* __restrict__ val, double2* __restrict__ V,
                                                     int64_t ld, int dim, int j, double2* __restrict__ y,
                                                     DevState* __restrict__ st, RedBuf rb) {
    constexpr int R = kBlock * RPT;
    __shared__ double2 ytile[R];
    __shared__ double2 wpart[kWaves][kMaxVals];
    __shared__ double2 vals[kMaxVals];
    if (st->done || j >= st->k_limit) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = blockIdx.x * R;
    const int r1 = min(r0 + R, dim);
    const double sj = st->s[j];
    const double2* __restrict__ x = V + (int64_t)j * ld;

    // y = s_j * H * V[:, j]  (G lanes per row, coalesced CSR stream)
    {
        const int lg = tid % G, grp = tid / G;
        for (int r = r0 + grp; r < r1; r += kBlock / G) {
            double2 acc = make_double2(0.0, 0.0);
            const int kb = rp[r], ke = rp[r + 1];
            for (int k = kb + lg; k < ke; k += G) acc = cfma(val[k], x[ci[k]], acc);
#pragma unroll
            for (int o = G / 2; o > 0; o >>= 1) {
                acc.x += __shfl_xor(acc.x, o);
                acc.y += __shfl_xor(acc.y, o);
            }
            if (lg == 0) {
                const double2 yy = cscale(acc, sj);
                y[r] = yy;
                ytile[r - r0] = yy;
            }
        }
    }
    __syncthreads();

    // projections of y and of x on every stored column i <= j
    double2 yq[RPT], xq[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = r0 + tid + q * kBlock;
        if (r < r1) {
            yq[q] = ytile[r - r0];
            xq[q] = x[r];
        } else {
            yq[q] = make_double2(0.0, 0.0);
            xq[q] = make_double2(0.0, 0.0);
        }
    }
    for (int i = 0; i <= j; ++i) {
        const double2* __restrict__ vi = V + (int64_t)i * ld;
        double2 cy = make_double2(0.0, 0.0), cx = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = r0 + tid + q * kBlock;
            if (r < r1) {
                const double2 v = vi[r];
                cy = cfma_conj(v, yq[q], cy);
                cx = cfma_conj(v, xq[q], cx);
            }
        }
        cy.x = wave_sum(cy.x);
        cy.y = wave_sum(cy.y);
        cx.x = wave_sum(cx.x);
        cx.y = wave_sum(cx.y);
        if (lane == 0) {
            wpart[wave][2 * i] = cy;
            wpart[wave][2 * i + 1] = cx;
        }
    }
    __syncthreads();
    const int nv = 2 * (j + 1);
    for (int v = tid; v < nv; v += kBlock) {
        double2 s = make_double2(0.0, 0.0);
        for (int w = 0; w < kWaves; ++w) s = cadd(s, wpart[w][v]);
        vals[v] = s;
    }
    __syncthreads();
    if (!grid_reduce(vals, nv, blockIdx.x, rb)) return;

    // finisher: scale, Gram column, corrected coefficients c = (I + E)^{-1} c'
    __shared__ double2 cp[kMaxM + 1], c1[kMaxM + 1];
    if (tid <= j) {
        const double si = st->s[tid];
        const double2 cy = cscale(vals[2 * tid], si);              // c'_i = v_i^H y
        const double2 gx = cscale(vals[2 * tid + 1], si * sj);     // g_i  = v_i^H v_j
        cp[tid] = cy;
        st->G[tid * kMaxM + j] = gx;
        st->G[j * kMaxM + tid] = make_double2(gx.x, -gx.y);
    }
    __threadfence_block();
    __syncthreads();
    // two sweeps of c <- c' - E c with E = G - I
    for (int sweep = 0; sweep < 2; ++sweep) {
        double2 acc = make_double2(0.0, 0.0);
        if (tid <= j) {
            acc = (sweep == 0) ? cp[tid] : c1[tid];
            double2 corr = make_double2(0.0, 0.0);
            for (int l = 0; l <= j; ++l) {
                double2 e = st->G[tid * kMaxM + l];
                if (l == tid) e.x -= 1.0;
                corr = cfma(e, (sweep == 0) ? cp[l] : c1[l], corr);
            }
            acc.x = cp[tid].x - corr.x;
            acc.y = cp[tid].y - corr.y;
        }
        __syncthreads();
        if (tid <= j) c1[tid] = acc;
        __syncthreads();
    }
    if (tid <= j) {
        const double2 c = c1[tid];
        st->ceff[tid] = cscale(c, st->s[tid]);
        if (tid == j) {
            st->alpha[j] = c.x;
            if (!isfinite(c.x) || !isfinite(c.y)) {
                st->status = TE_ERR_NONFINITE;
                st->done = 1;
            }
        }
    }
}

// ------------------------------------------------------------- pass B: update + norm
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_update(double2* __restrict__ V, int64_t ld, int dim, int j,
                                                    const double2* __restrict__ y, DevState* __restrict__ st,
                                                    RedBuf rb) {
    __shared__ double lds[kWaves];
    __shared__ double2 vals[1];
    if (st->done || j >= st->k_limit) return;
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * (kBlock * RPT);
    const bool store = (j + 1) < st->p.m;
    double2 p[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = r0 + tid + q * kBlock;
        p[q] = (r < dim) ? y[r] : make_double2(0.0, 0.0);
    }
    for (int i = 0; i <= j; ++i) {
        const double2 c = st->ceff[i];
        const double2* __restrict__ vi = V + (int64_t)i * ld;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = r0 + tid + q * kBlock;
            if (r < dim) p[q] = cfms(c, vi[r], p[q]);
        }
    }
    double acc = 0.0;
    double2* __restrict__ vn = V + (int64_t)(j + 1) * ld;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = r0 + tid + q * kBlock;
        if (r < dim) {
            if (store) vn[r] = p[q];
            acc = fma(p[q].x, p[q].x, acc);
            acc = fma(p[q].y, p[q].y, acc);
        }
    }
    {
        const int lane = tid & 63, wave = tid >> 6;
        const double s = wave_sum(acc);
        if (lane == 0) lds[wave] = s;
        __syncthreads();
        if (tid == 0) {
            double b = 0.0;
            for (int w = 0; w < kWaves; ++w) b += lds[w];
            vals[0] = make_double2(b, 0.0);
        }
        __syncthreads();
    }
    if (!grid_reduce(vals, 1, blockIdx.x, rb)) return;
    if (tid == 0) {
        const double beta = sqrt(vals[0].x);
        st->beta[j] = beta;
        if (!isfinite(beta)) {
            st->status = TE_ERR_NONFINITE;
            st->done = 1;
        } else if (beta < st->p.tol_rate) {  // lucky breakdown (Alg. 1: no < tol_rate)
            st->k_limit = j + 1;
            st->breakdown = 1;
            st->h = beta;
        } else if (j + 1 == st->p.m) {
            st->h = beta;
        } else {
            st->s[j + 1] = 1.0 / beta;
        }
    }
}

// ------------------------------------------------------------- recombination w = V omega
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_combine(double2* __restrict__ V, int64_t ld, int dim,
                                                     const DevState* __restrict__ st) {
    if (!st->do_combine) return;
    const int k = st->k_comb;
    const int r0 = blockIdx.x * (kBlock * RPT);
    double2 w[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) w[q] = make_double2(0.0, 0.0);
    for (int i = 0; i < k; ++i) {
        const double2 c = st->omega[i];
        const double2* __restrict__ vi = V + (int64_t)i * ld;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = r0 + threadIdx.x + q * kBlock;
            if (r < dim) w[q] = cfma(c, vi[r], w[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = r0 + threadIdx.x + q * kBlock;
        if (r < dim) V[r] = w[q];
    }
}

// dst[:, i] = s[i] * src[:, i] for i < k (normalised basis in the caller's layout)
__global__ __launch_bounds__(kBlock) void k_scale_columns(const double2* __restrict__ src, double2* __restrict__ dst,
                                                           int64_t ld, int dim, int k, const DevState* __restrict__ st) {
    for (int i = blockIdx.y; i < k; i += gridDim.y) {
        const double sc = st->s[i];
        for (int r = blockIdx.x * kBlock + threadIdx.x; r < dim; r += gridDim.x * kBlock)
            dst[(int64_t)i * dim + r] = cscale(src[(int64_t)i * ld + r], sc);
    }
}

__global__ __launch_bounds__(kBlock) void k_output(const double2* __restrict__ V, double2* __restrict__ out,
                                                    int dim, const DevState* __restrict__ st) {
    // after the last recombination column 0 is the normalised state (s[0] == 1)
    const double b = (st->beta0 == 0.0) ? 0.0 : st->beta0 * st->s[0];
    for (int r = blockIdx.x * kBlock + threadIdx.x; r < dim; r += gridDim.x * kBlock) out[r] = cscale(V[r], b);
}

// ---------------------------------------------------------- standalone sparse product
template <int G>
__global__ __launch_bounds__(kBlock) void k_spmv(const int* __restrict__ rp, const int* __restrict__ ci,
                                                  const double2* __restrict__ val, const double2* __restrict__ x,
                                                  double2* __restrict__ y, int dim, DevState* __restrict__ st,
                                                  RedBuf rb, int rows_per_tile) {
    __shared__ double2 wpart[kWaves];
    __shared__ double2 vals[1];
    const int tid = threadIdx.x, lg = tid % G, grp = tid / G;
    const int r0 = blockIdx.x * rows_per_tile;
    const int r1 = min(r0 + rows_per_tile, dim);
    double2 dot = make_double2(0.0, 0.0);
    for (int r = r0 + grp; r < r1; r += kBlock / G) {
        double2 acc = make_double2(0.0, 0.0);
        for (int k = rp[r] + lg; k < rp[r + 1]; k += G) acc = cfma(val[k], x[ci[k]], acc);
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
            acc.x += __shfl_xor(acc.x, o);
            acc.y += __shfl_xor(acc.y, o);
        }
        if (lg == 0) {
            y[r] = acc;
            dot = cfma_conj(x[r], acc, dot);
        }
    }
    dot.x = wave_sum(dot.x);
    dot.y = wave_sum(dot.y);
    if ((tid & 63) == 0) wpart[tid >> 6] = dot;
    __syncthreads();
    if (tid == 0) {
        double2 s = make_double2(0.0, 0.0);
        for (int w = 0; w < kWaves; ++w) s = cadd(s, wpart[w]);
        vals[0] = s;
    }
    __syncthreads();
    if (!grid_reduce(vals, 1, blockIdx.x, rb)) return;
    if (tid == 0) st->ceff[0] = vals[0];
}

// ------------------------------------------------------------------ CSR validation
// err bits: 1 structure, 2 column range, 4 non-finite, 8 unsorted (Hermitian check), 16 not Hermitian
__global__ __launch_bounds__(kBlock) void k_validate(const int* __restrict__ rp, const int* __restrict__ ci,
                                                      const double2* __restrict__ val, int dim, int64_t nnz,
                                                      int check_herm, int* err, double* rowsum) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= dim) return;
    int e = 0;
    const int kb = rp[r], ke = rp[r + 1];
    if (r == 0 && kb != 0) e |= 1;
    if (r == dim - 1 && (int64_t)ke != nnz) e |= 1;
    if (ke < kb || kb < 0 || (int64_t)ke > nnz) {
        atomicOr(err, e | 1);
        rowsum[r] = 0.0;
        return;
    }
    double sum = 0.0;
    for (int k = kb; k < ke; ++k) {
        const int c = ci[k];
        const double2 v = val[k];
        if (c < 0 || c >= dim) {
            e |= 2;
            continue;
        }
        if (!isfinite(v.x) || !isfinite(v.y)) e |= 4;
        sum += hypot(v.x, v.y);
        if (check_herm) {
            if (k > kb && ci[k - 1] >= c) e |= 8;
            // binary search column r in row c (sorted columns required)
            // clamp: row c's own pointers may be invalid (reported by that row's thread)
            int lo = max(rp[c], 0), hi = (int)min((int64_t)rp[c + 1], nnz) - 1;
            bool found = false;
            double2 w = make_double2(0.0, 0.0);
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int cm = ci[mid];
                if (cm == r) {
                    found = true;
                    w = val[mid];
                    break;
                }
                if (cm < r) lo = mid + 1;
                else hi = mid - 1;
            }
            const double scale = fmax(hypot(v.x, v.y), hypot(w.x, w.y));
            if (!found || fabs(v.x - w.x) > 8.0 * 2.220446049250313e-16 * scale ||
                fabs(v.y + w.y) > 8.0 * 2.220446049250313e-16 * scale)
                e |= 16;
        }
    }
    rowsum[r] = sum;
    if (e) atomicOr(err, e);
}

__global__ __launch_bounds__(kBlock) void k_max(const double* __restrict__ a, int n, double* out) {
    __shared__ double lds[kWaves];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) m = fmax(m, a[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int w = 0; w < kWaves; ++w) r = fmax(r, lds[w]);
        *out = r;
    }
}

// --------------------------------------------------------------------------- launchers
template <typename F>
static hipError_t by_rpt(int rpt, F&& f) {
    switch (rpt) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        default: f(std::integral_constant<int, 8>{}); break;
    }
    return hipGetLastError();
}

hipError_t launch_init(const Tiling& tl, const double2* v0, double2* V, int dim, DevState* st,
                       const RedBuf& rb, const Problem& prob, hipStream_t s) {
    return by_rpt(tl.rpt, [&](auto r) {
        k_init<decltype(r)::value><<<tl.n_tiles, kBlock, 0, s>>>(v0, V, dim, st, rb, prob);
    });
}

hipError_t launch_project(const Tiling& tl, const Csr& H, double2* V, int64_t ld, int j, double2* y,
                          DevState* st, const RedBuf& rb, hipStream_t s) {
    return by_rpt(tl.rpt, [&](auto r) {
        k_project<decltype(r)::value, 4><<<tl.n_tiles, kBlock, 0, s>>>(H.row_ptr, H.col, H.val, V, ld, H.dim, j, y,
                                                                        st, rb);
    });
}

hipError_t launch_update(const Tiling& tl, double2* V, int64_t ld, int dim, int j, const double2* y,
                         DevState* st, const RedBuf& rb, hipStream_t s) {
    return by_rpt(tl.rpt, [&](auto r) {
        k_update<decltype(r)::value><<<tl.n_tiles, kBlock, 0, s>>>(V, ld, dim, j, y, st, rb);
    });
}

hipError_t launch_combine(const Tiling& tl, double2* V, int64_t ld, int dim, DevState* st, hipStream_t s) {
    return by_rpt(tl.rpt, [&](auto r) {
        k_combine<decltype(r)::value><<<tl.n_tiles, kBlock, 0, s>>>(V, ld, dim, st);
    });
}

hipError_t launch_output(const Tiling&, const double2* V, double2* out, int dim, const DevState* st, hipStream_t s) {
    const int blocks = (int)std::min<int64_t>(((int64_t)dim + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_output, dim3(blocks), dim3(kBlock), 0, s, V, out, dim, st);
    return hipGetLastError();
}

hipError_t launch_scale_columns(const double2* src, double2* dst, int64_t ld, int dim, int k, const DevState* st,
                                hipStream_t s) {
    const int bx = (int)std::min<int64_t>(((int64_t)dim + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(k_scale_columns, dim3(bx, std::max(1, std::min(k, 64))), dim3(kBlock), 0, s, src, dst, ld, dim, k, st);
    return hipGetLastError();
}

hipError_t launch_spmv_only(const Tiling& tl, const Csr& H, const double2* x, double2* y, DevState* st,
                            const RedBuf& rb, hipStream_t s) {
    hipLaunchKernelGGL(k_spmv<4>, dim3(tl.n_tiles), dim3(kBlock), 0, s, H.row_ptr, H.col, H.val, x, y, H.dim, st, rb,
                       tl.rows);
    return hipGetLastError();
}

hipError_t launch_validate(const Csr& H, int check_hermitian, int* err, double* rowsum, hipStream_t s) {
    const int blocks = (H.dim + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_validate, dim3(blocks), dim3(kBlock), 0, s, H.row_ptr, H.col, H.val, H.dim, H.nnz,
                       check_hermitian, err, rowsum);
    return hipGetLastError();
}

hipError_t launch_norm1(const double* rowsum, int dim, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_max, dim3(1), dim3(kBlock), 0, s, rowsum, dim, out);
    return hipGetLastError();
}

}  // namespace te
