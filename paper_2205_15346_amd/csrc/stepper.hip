// One-workgroup kernel that closes every restart on the device (paper, Alg. 1 step 2 and the
// bookkeeping of step 3):
//   1. diagonalise the k x k real symmetric tridiagonal J = V^H H V (Sec. "Pseudocode", first
//      remark) by the implicit QL method with Wilkinson shifts: wave 0 runs the rotation
//      chain, lane q owns row q of Q (k <= 64);
//   2. f(tau) = h |e_k^T exp(-iJ tau) e_1| = h |sum_n Q[k-1][n] Q[0][n] exp(-i lam_n tau)|
//      (eq. errorIntegral in Lanczos form: |e_k^T exp(M tau) e_1| is unchanged by the
//      diagonal phase similarity between M = -i J-like Hessenberg and J);
//   3. its integrals by the tanh-sinh rule, all 256 threads evaluating nodes;
//   4. the step-size search of eq. stepSize (first-step doubling, 0.97 shrink, halving,
//      substeps, end snap);
//   5. omega = exp(-iJ tau) e_1 scaled to the raw basis columns, and the restart controller:
//      time, accumulated bound, roundoff estimate (eq. numericalError), warnings, done flag.
#include "te_internal.h"

namespace te {

namespace {

constexpr int QS = kMaxM + 1;  // padded row stride of Q in LDS
constexpr double kEps = 2.220446049250313e-16;
constexpr double kHalfPi = 1.5707963267948966;

struct StepShared {
    double Q[kMaxM * QS];
    double d[kMaxM], e[kMaxM];
    double lam[kMaxM], cf[kMaxM];
    double red[kWaves * 8];
    double bcast[8];
    int ibcast[4];
};

// ---------------------------------------------------------------- eigen-decomposition
// Wave 0 only.  On return d[] holds the eigenvalues and column n of Q the eigenvector of
// d[n].  Returns false if an eigenvalue needed more than 64 QL iterations.
__device__ bool tridiag_ql(int k, double* d, double* e, double* Q) {
    const int lane = threadIdx.x;  // < 64
    for (int c = 0; c < k; ++c)
        if (lane < k) Q[lane * QS + c] = (lane == c) ? 1.0 : 0.0;
    e[k - 1] = 0.0;
    bool ok = true;
    for (int l = 0; l < k; ++l) {
        int iter = 0;
        while (true) {
            int mm = l;
            while (mm < k - 1) {
                const double dd = fabs(d[mm]) + fabs(d[mm + 1]);
                if (fabs(e[mm]) <= kEps * dd) break;
                ++mm;
            }
            if (mm == l) break;
            if (++iter > 64) {
                ok = false;
                break;
            }
            // Wilkinson shift from the leading 2x2 block
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = sqrt(fma(g, g, 1.0));
            g = d[mm] - d[l] + e[l] / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            double carry = (lane < k) ? Q[lane * QS + mm] : 0.0;
            int i = mm - 1;
            bool underflow = false;
            for (; i >= l; --i) {
                const double qi = (lane < k) ? Q[lane * QS + i] : 0.0;
                const double f = s * e[i];
                const double b = c * e[i];
                r = sqrt(fma(f, f, g * g));
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[mm] = 0.0;
                    underflow = true;
                    break;
                }
                const double rinv = 1.0 / r;
                s = f * rinv;
                c = g * rinv;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                if (lane < k) {
                    Q[lane * QS + i + 1] = s * qi + c * carry;
                    carry = c * qi - s * carry;
                }
            }
            if (underflow) {
                if (lane < k) Q[lane * QS + i + 1] = carry;
                continue;
            }
            if (lane < k) Q[lane * QS + l] = carry;
            d[l] -= p;
            e[l] = g;
            e[mm] = 0.0;
        }
        if (!ok) break;
    }
    return ok;
}

// ------------------------------------------------------------------------- quadrature
// node t of the flattened levels 0..5 (t < 193): level and abscissa u
__device__ __forceinline__ void flat_node(int t, int* level, double* u) {
    if (t < 7) {
        *level = 0;
        *u = (double)(t - 3);
        return;
    }
    int lev = 1;
    while (t >= 3 * (1 << (lev + 1)) + 1) ++lev;
    const int p = t - (3 * (1 << lev) + 1);
    const int half = 3 * (1 << (lev - 1));
    const double step = ldexp(1.0, -lev);
    *level = lev;
    *u = (p < half) ? -(2.0 * (half - 1 - p) + 1.0) * step : (2.0 * (p - half) + 1.0) * step;
}

__device__ __forceinline__ double integrand(double x, int k, const double* lam, const double* cf, double h) {
    double re = 0.0, im = 0.0;
    for (int n = 0; n < k; ++n) {
        double sn, cn;
        sincos(lam[n] * x, &sn, &cn);
        re = fma(cf[n], cn, re);
        im = fma(-cf[n], sn, im);
    }
    return h * sqrt(fma(re, re, im * im));
}

__device__ __forceinline__ double node_value(double u, double center, double radius, int k, const double* lam,
                                             const double* cf, double h) {
    const double sh = kHalfPi * sinh(u);
    const double x = center + radius * tanh(sh);
    const double ch = cosh(sh);
    const double w = radius * kHalfPi * cosh(u) / (ch * ch);
    return w * integrand(x, k, lam, cf, h);
}

struct QuadOut {
    double value;
    int level;
    int converged;
};

// Whole block.  Integral of f over [a, b] by the adaptive tanh-sinh rule: stop at the first
// level >= max(1, min_level) whose change is <= max(rel_tol |I|, noise_rate (b - a)).
__device__ QuadOut integrate(double a, double b, const Problem& P, int k, const double* lam, const double* cf,
                             double h, double noise_rate, StepShared& sh) {
    QuadOut out;
    if (b == a) {
        out.value = 0.0;
        out.level = 0;
        out.converged = 1;
        return out;
    }
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double center = 0.5 * (a + b), radius = 0.5 * (b - a);
    const double abs_tol = noise_rate * (b - a);
    const int L0 = min(5, P.quad_max_level);
    const int n0 = 6 * (1 << L0) + 1;
    // levels 0..L0 in one pass (<= 193 nodes <= blockDim)
    double val = 0.0;
    int my_level = -1;
    if (tid < n0) {
        double u;
        flat_node(tid, &my_level, &u);
        val = node_value(u, center, radius, k, lam, cf, h);
    }
    for (int lev = 0; lev <= L0; ++lev) {
        const double s = wave_sum(my_level == lev ? val : 0.0);
        if (lane == 0) sh.red[wave * 8 + lev] = s;
    }
    __syncthreads();
    if (tid == 0) {
        double total = 0.0, prev = 0.0, value = 0.0;
        int conv = 0, lev_out = L0;
        for (int lev = 0; lev <= L0; ++lev) {
            double ls = 0.0;
            for (int w = 0; w < kWaves; ++w) ls += sh.red[w * 8 + lev];
            total += ls;
            value = total * ldexp(1.0, -lev);
            if (lev >= 1 && lev >= P.quad_min_level && fabs(value - prev) <= fmax(P.quad_rel_tol * fabs(value), abs_tol)) {
                conv = 1;
                lev_out = lev;
                break;
            }
            prev = value;
        }
        sh.bcast[0] = value;
        sh.bcast[1] = total;
        sh.bcast[2] = prev;
        sh.ibcast[0] = conv;
        sh.ibcast[1] = lev_out;
    }
    __syncthreads();
    out.value = sh.bcast[0];
    out.converged = sh.ibcast[0];
    out.level = sh.ibcast[1];
    double total = sh.bcast[1];
    double prev = sh.bcast[0];
    __syncthreads();
    for (int lev = L0 + 1; !out.converged && lev <= P.quad_max_level; ++lev) {
        const int n = 3 * (1 << lev), half = n / 2;
        const double step = ldexp(1.0, -lev);
        double acc = 0.0;
        for (int p = tid; p < n; p += kBlock) {
            const double u = (p < half) ? -(2.0 * (half - 1 - p) + 1.0) * step : (2.0 * (p - half) + 1.0) * step;
            acc += node_value(u, center, radius, k, lam, cf, h);
        }
        const double s = wave_sum(acc);
        if (lane == 0) sh.red[wave] = s;
        __syncthreads();
        if (tid == 0) {
            double ls = 0.0;
            for (int w = 0; w < kWaves; ++w) ls += sh.red[w];
            sh.bcast[0] = ls;
        }
        __syncthreads();
        total += sh.bcast[0];
        const double value = total * step;
        out.value = value;
        out.level = lev;
        if (lev >= P.quad_min_level && fabs(value - prev) <= fmax(P.quad_rel_tol * fabs(value), abs_tol))
            out.converged = 1;
        prev = value;
        __syncthreads();
    }
    return out;
}

// --------------------------------------------------------------------- step search
struct StepOut {
    double tau, err;
    int quad_ok;
    int underflow;
};

// Whole block; every thread returns the same result (decisions are taken on values
// broadcast through LDS).  Follows eq. stepSize / Alg. 1 step 2 with the readings of the
// CPU reference (clipping to t_rem, doubling only from an admissible first guess, substep
// integrals over [tau + (n-1)s, tau + n s] accepted with '<', halving on '>', end snap).
__device__ StepOut step_search(const Problem& P, int k, double h, int breakdown, int first, double tau_prev,
                               double t_rem, StepShared& sh) {
    const double rate = P.tol_rate;
    const double noise = h * (double)k * kEps;
    StepOut o;
    o.quad_ok = 1;
    o.underflow = 0;
    auto I = [&](double a, double b) {
        QuadOut q = integrate(a, b, P, k, sh.lam, sh.cf, h, noise, sh);
        o.quad_ok &= q.converged;
        return q.value;
    };
    if (breakdown) {
        o.tau = t_rem;
        o.err = I(0.0, t_rem);
        return o;
    }
    double tau, err;
    if (first) {
        tau = fmin(P.t_init, t_rem);
        err = I(0.0, tau);
        while (err <= __dmul_rn(rate, tau) && __dmul_rn(2.0, tau) <= t_rem) {
            const double tau2 = __dmul_rn(2.0, tau);
            const double e2 = I(0.0, tau2);
            if (e2 <= __dmul_rn(rate, tau2)) {
                tau = tau2;
                err = e2;
            } else {
                break;
            }
        }
    } else {
        tau = fmin(__dmul_rn(P.shrink, tau_prev), t_rem);
        err = I(0.0, tau);
    }
    int halvings = 0;
    while (err > __dmul_rn(rate, tau)) {
        if (halvings == P.max_halvings) {
            o.underflow = 1;
            o.tau = tau;
            o.err = err;
            return o;
        }
        tau = 0.5 * tau;
        err = I(0.0, tau);
        ++halvings;
    }
    const double s = tau / (double)P.n_substeps;
    int n = 1;
    while (true) {
        const double b = __dadd_rn(tau, __dmul_rn((double)n, s));
        if (b > t_rem) break;
        const double delta = I(__dadd_rn(tau, __dmul_rn((double)(n - 1), s)), b);
        if (__dadd_rn(err, delta) < __dmul_rn(rate, b)) {
            err = __dadd_rn(err, delta);
            ++n;
        } else {
            break;
        }
    }
    tau = __dadd_rn(tau, __dmul_rn((double)(n - 1), s));
    if (tau < t_rem && __dadd_rn(t_rem, -tau) < s) {
        const double ef = I(0.0, t_rem);
        if (ef <= __dmul_rn(rate, t_rem)) {
            tau = t_rem;
            err = ef;
        }
    }
    o.tau = tau;
    o.err = err;
    return o;
}

// Loads J from the state, diagonalises it and prepares lam/cf.  Returns false on failure.
__device__ bool prepare_spectrum(const DevState* st, int k, StepShared& sh) {
    const int tid = threadIdx.x;
    if (tid < k) {
        sh.d[tid] = st->alpha[tid];
        sh.e[tid] = (tid < k - 1) ? st->beta[tid] : 0.0;
    }
    __syncthreads();
    __shared__ int ok_sh;
    if (tid < 64) {
        const bool ok = tridiag_ql(k, sh.d, sh.e, sh.Q);
        if (tid == 0) ok_sh = ok ? 1 : 0;
    }
    __syncthreads();
    if (tid < k) {
        sh.lam[tid] = sh.d[tid];
        sh.cf[tid] = sh.Q[(k - 1) * QS + tid] * sh.Q[tid];
    }
    __syncthreads();
    return ok_sh != 0;
}

// omega_i = sum_n Q[i][n] exp(-i lam_n tau) Q[0][n], scaled by s_i for the raw columns
__device__ void write_omega(DevState* st, int k, double tau, bool scale_raw, StepShared& sh) {
    const int tid = threadIdx.x;
    if (tid < k) {
        double re = 0.0, im = 0.0;
        for (int n = 0; n < k; ++n) {
            double sn, cn;
            sincos(sh.lam[n] * tau, &sn, &cn);
            const double a = sh.Q[tid * QS + n] * sh.Q[n];
            re = fma(a, cn, re);
            im = fma(-a, sn, im);
        }
        const double sc = scale_raw ? st->s[tid] : 1.0;
        st->omega[tid] = make_double2(re * sc, im * sc);
    }
}

__device__ void step_body(DevState* st, int* host_flag, bool controller) {
    __shared__ StepShared sh;
    const int tid = threadIdx.x;
    if (st->done) {
        if (tid == 0) {
            st->do_combine = 0;
            if (host_flag) __hip_atomic_store(host_flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        return;
    }
    const Problem P = st->p;
    const int k = st->k_limit;
    const double h = st->h;
    const int breakdown = st->breakdown;
    const double t_now = st->t_now;
    const double t_rem = P.t - t_now;
    const bool ok = prepare_spectrum(st, k, sh);
    if (!ok) {
        if (tid == 0) {
            st->status = TE_ERR_DEVICE;
            st->done = 1;
            st->do_combine = 0;
            if (host_flag) __hip_atomic_store(host_flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        return;
    }
    const StepOut so = step_search(P, k, h, breakdown, st->first, st->tau_prev, t_rem, sh);
    if (so.underflow) {
        if (tid == 0) {
            st->status = TE_ERR_STEP_UNDERFLOW;
            st->done = 1;
            st->do_combine = 0;
            st->last_tau = so.tau;
            st->last_err = so.err;
            if (host_flag) __hip_atomic_store(host_flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        return;
    }
    write_omega(st, k, so.tau, controller, sh);
    __syncthreads();
    if (tid == 0) {
        st->last_tau = so.tau;
        st->last_err = so.err;
        if (!so.quad_ok) st->warnings |= TE_WARN_QUADRATURE;
        if (!controller) return;
        st->err_acc += so.err;
        st->num_acc += P.numerr_per_step;
        if (st->num_acc > st->err_acc) st->warnings |= TE_WARN_NUMERICAL;
        st->steps += 1;
        st->matvecs += k;
        st->tau_prev = so.tau;
        st->first = 0;
        double tn = (so.tau == t_rem) ? P.t : t_now + so.tau;
        if (breakdown) {
            st->breakdown_dim = k;
            tn = P.t;
        }
        st->t_now = tn;
        {
            double* tr = st->trace[(st->steps - 1) % kTrace];
            tr[0] = t_now;
            tr[1] = so.tau;
            tr[2] = so.err;
            tr[3] = h;
            tr[4] = (double)k;
            tr[5] = (double)breakdown;
            tr[6] = (double)so.quad_ok;
            tr[7] = t_rem;
        }
        st->k_comb = k;
        st->norm_init = 0;
        st->do_combine = 1;
        st->s[0] = 1.0;
        if (tn >= P.t) st->done = 1;
        st->k_limit = P.m;
        st->breakdown = 0;
        if (host_flag) {
            // host_flag[0] done, [1] restarts completed, [8 + r % 8] Krylov dimension of restart r
            const int r = st->steps - 1;
            __hip_atomic_store(host_flag + 8 + (r & 7), k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(host_flag + 1, st->steps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(host_flag, st->done, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_step(DevState* st, RedBuf rb, int* host_flag) {
    __shared__ double lds[kWaves];
    finish_last_norm(st, rb, lds);  // h of a build that ran all m iterations
    step_body(st, host_flag, true);
}

// step search alone on a state prepared by the host (component entry point)
__global__ __launch_bounds__(kBlock) void k_step_only(DevState* st) { step_body(st, nullptr, false); }

__global__ __launch_bounds__(kBlock) void k_eig_only(int k, const double* alpha, const double* beta, double* lambda,
                                                      double* Q, int* status) {
    __shared__ StepShared sh;
    const int tid = threadIdx.x;
    if (tid < k) {
        sh.d[tid] = alpha[tid];
        sh.e[tid] = (tid < k - 1) ? beta[tid] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
        const bool ok = tridiag_ql(k, sh.d, sh.e, sh.Q);
        if (tid == 0) *status = ok ? 0 : 1;
    }
    __syncthreads();
    if (tid < k) {
        lambda[tid] = sh.d[tid];
        for (int n = 0; n < k; ++n) Q[n * k + tid] = sh.Q[tid * QS + n];  // column-major
    }
}

__global__ __launch_bounds__(kBlock) void k_integral_only(int k, const double* lambda, const double* coef, double h,
                                                           double a, double b, Problem P, double* out) {
    __shared__ StepShared sh;
    const int tid = threadIdx.x;
    if (tid < k) {
        sh.lam[tid] = lambda[tid];
        sh.cf[tid] = coef[tid];
    }
    __syncthreads();
    const QuadOut q = integrate(a, b, P, k, sh.lam, sh.cf, h, h * (double)k * kEps, sh);
    if (tid == 0) {
        out[0] = q.value;
        out[1] = (double)q.level;
        out[2] = (double)q.converged;
    }
}

}  // namespace

hipError_t launch_step(DevState* st, const RedBuf& rb, int* host_flag, hipStream_t s) {
    hipLaunchKernelGGL(k_step, dim3(1), dim3(kBlock), 0, s, st, rb, host_flag);
    return hipGetLastError();
}

hipError_t launch_step_only(DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_step_only, dim3(1), dim3(kBlock), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_eig_only(int k, const double* alpha, const double* beta, double* lambda, double* Q, int* status,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_eig_only, dim3(1), dim3(kBlock), 0, s, k, alpha, beta, lambda, Q, status);
    return hipGetLastError();
}

hipError_t launch_integral_only(int k, const double* lambda, const double* coef, double h, double a, double b,
                                const Problem& opt, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_integral_only, dim3(1), dim3(kBlock), 0, s, k, lambda, coef, h, a, b, opt, out);
    return hipGetLastError();
}

}  // namespace te
