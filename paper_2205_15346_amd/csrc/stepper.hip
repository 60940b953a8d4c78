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
#include <hip/hip_ext.h>

#include "te_internal.h"

namespace te {

namespace {

constexpr double kEps = 2.220446049250313e-16;
constexpr double kHalfPi = 1.5707963267948966;
constexpr uint64_t kWallClockHz = 100000000ull;  // wall_clock64() runs at a constant 100 MHz on gfx9
constexpr int kMaxTpn = 8;                       // threads sharing one quadrature node

struct StepShared {
    double Qt[kMaxM * 64];  // eigenvectors: column n (eigenvalue n) at Qt[n * 64 + row]
    // divide and conquer: halves' inputs, merge arrays (sorted poles, kept poles, roots)
    double U[kMaxM * 64];   // eigenvectors of the rank-one problem, U[j * 64 + i]
    double dca[kMaxM], dcb[kMaxM], dd[kMaxM], dz[kMaxM], ds[kMaxM], zs[kMaxM];
    double dk[kMaxM], zk[kMaxM], zh[kMaxM], tau[kMaxM];
    double rc[kMaxM], rs[kMaxM];
    int perm[kMaxM], keep[kMaxM], org[kMaxM], r1[kMaxM], r2[kMaxM], defl[kMaxM];
    int dc_ok[2], dc_K, dc_nrot;
    double dc_rho, dc_tol;
    double gx[kMaxM], gw[kMaxM];  // Gauss-Legendre nodes and weights on [-1, 1] (fast option)
    double d[kMaxM], e[kMaxM];
    double lam[kMaxM], cf[kMaxM];
    double pre[kBlock], pim[kBlock];
    double red[kWaves * 8];
    double lev_sum[8];
    double bcast[8];
    int ibcast[4];
};

// ---------------------------------------------------------------- eigen-decomposition
// 1/sqrt(t) for t > 0: hardware estimate refined by one Newton step (relative error ~1 ulp).
__device__ __forceinline__ double rsqrt_nr(double t) {
    const double y = __builtin_amdgcn_rsq(t);
    return y * fma(-0.5 * t * y, y, 1.5);
}

// 1/x: hardware estimate refined by one Newton step (relative error ~1 ulp).
__device__ __forceinline__ double rcp_nr(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    return y * fma(-x, y, 2.0);
}

// Value of a wave-distributed register array at a wave-uniform lane index.
__device__ __forceinline__ double lane_get(double x, int i) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), i);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), i);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Implicit QL with Wilkinson shifts on the k x k symmetric tridiagonal (diagonal a, off-diagonal
// b): the textbook method of Bowdler, Martin, Reinsch and Wilkinson (Numer. Math. 11, 1968; the
// procedure EISPACK publishes as tql2), restructured for one wave.  Run by wave 0: lane i holds
// d_i and e_i in registers, lane q owns row q of the eigenvector
// matrix (Qt, transposed in LDS).  Within a sweep every d/e value read is a pre-sweep value, so
// the reads sit off the rotation chain; deflation points come from one ballot.  On return lam[]
// holds the eigenvalues (unsorted) and Qt[n * 64 + q] = Q[q][n].  False if an eigenvalue needed
// more than 64 iterations.
__device__ bool tridiag_ql(int k, const double* a, const double* b, double* lam, double* Qt) {
    const int lane = threadIdx.x & 63;  // run by one whole wave
    double dr = (lane < k) ? a[lane] : 0.0;
    double er = (lane < k - 1) ? b[lane] : 0.0;
    for (int c = 0; c < k; ++c) Qt[c * 64 + lane] = (lane == c) ? 1.0 : 0.0;
    bool ok = true;
    for (int l = 0; l < k && ok; ++l) {
        int iter = 0;
        while (true) {
            const double dn = __shfl_down(dr, 1);
            const bool small = (lane >= k - 1) || (fabs(er) <= kEps * (fabs(dr) + fabs(dn)));
            const unsigned long long mask = __ballot(small) & (~0ull << l);
            const int mm = __ffsll((long long)mask) - 1;
            if (mm == l) break;
            if (++iter > 64) {
                ok = false;
                break;
            }
            const double dl = lane_get(dr, l), el = lane_get(er, l);
            double g = (lane_get(dr, l + 1) - dl) / (2.0 * el);
            double r = sqrt(fma(g, g, 1.0));
            g = lane_get(dr, mm) - dl + el / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            double carry = Qt[mm * 64 + lane];
            int i = mm - 1;
            int underflow = 0;
            // operands of the next rotation are fetched one step ahead (all pre-sweep values)
            double ei_n = lane_get(er, i), di_n = lane_get(dr, i), di1_n = lane_get(dr, i + 1);
            double qi_n = Qt[i * 64 + lane];
            for (; i >= l; --i) {
                const double ei = ei_n, di = di_n, di1 = di1_n, qi = qi_n;
                if (i > l) {
                    ei_n = lane_get(er, i - 1);
                    di1_n = di;
                    di_n = lane_get(dr, i - 1);
                    qi_n = Qt[(i - 1) * 64 + lane];
                }
                const double f = s * ei;
                const double bb = c * ei;
                const double t = fma(f, f, g * g);
                // wave-uniform test: the compare mask itself drives a scalar branch
                if (__builtin_amdgcn_ballot_w64(t == 0.0) != 0) {
                    if (lane == i + 1) dr = di1 - p;
                    if (lane == mm) er = 0.0;
                    underflow = 1;
                    break;
                }
                const double rinv = rsqrt_nr(t);
                if (lane == i + 1) er = t * rinv;
                s = f * rinv;
                c = g * rinv;
                g = di1 - p;
                r = (di - g) * s + 2.0 * c * bb;
                p = s * r;
                if (lane == i + 1) dr = g + p;
                g = c * r - bb;
                Qt[(i + 1) * 64 + lane] = s * qi + c * carry;
                carry = c * qi - s * carry;
            }
            if (underflow) {
                Qt[(i + 1) * 64 + lane] = carry;
                continue;
            }
            Qt[l * 64 + lane] = carry;
            if (lane == l) {
                dr = dl - p;
                er = g;
            }
            if (lane == mm) er = 0.0;
        }
    }
    if (lane < k) lam[lane] = dr;
    return ok;
}

// sum over the 4 lanes of a quad (lanes 4q..4q+3)
__device__ __forceinline__ double quad_sum(double v) {
    v += __shfl_xor(v, 1);
    return v + __shfl_xor(v, 2);
}

// Root i of the secular equation 1 + rho sum_j z_j^2 / (d_j - lam) = 0 over the K kept poles
// d (ascending, rho > 0): lam in (d_i, d_{i+1}), the last in (d_{K-1}, d_{K-1} + rho sum z^2),
// solved by the 4 lanes of a quad (lane part = 0..3 sums terms j = part, part + 4, ...; every
// lane then takes the same steps).  Coordinates are shifted to the nearer pole (chosen by the
// sign at the midpoint), so d_j - lam is formed as (d_j - d_org) - tau without cancellation.
// Iteration of Bunch, Nielsen and Sorensen: the sums over the poles below and above the root are
// each replaced by one pole plus a constant matching value and slope at the iterate, and the
// resulting quadratic is solved; bisection of the bracket when its root falls outside.  Stops
// when the secular function is at its rounding level.  Returns tau; *org receives the origin.
__device__ double secular_root(int i, int part, int K, const double* d, const double* z, double rho, int* org) {
    const bool last = i == K - 1;
    double lo, hi;
    int o;
    if (!last) {
        const double mid = 0.5 * (d[i] + d[i + 1]);
        double f = 0.0;
        for (int j = part; j < K; j += 4) f += z[j] * z[j] * rcp_nr(d[j] - mid);
        f = 1.0 + rho * quad_sum(f);
        if (f >= 0.0) {
            o = i;
            lo = 0.0;
            hi = mid - d[i];
        } else {
            o = i + 1;
            lo = mid - d[i + 1];
            hi = 0.0;
        }
    } else {
        o = K - 1;
        double s2 = 0.0;
        for (int j = part; j < K; j += 4) s2 += z[j] * z[j];
        lo = 0.0;
        hi = rho * quad_sum(s2);
    }
    const double dorg = d[o];
    const double di = d[i] - dorg, dn = last ? 0.0 : d[i + 1] - dorg;
    double tau = 0.5 * (lo + hi);
    for (int it = 0; it < 64; ++it) {
        double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
        for (int j = part; j < K; j += 4) {
            const double r = rcp_nr((d[j] - dorg) - tau);
            const double w = z[j] * z[j] * r;
            if (j <= i) {
                psi += w;
                dpsi += w * r;
            } else {
                phi += w;
                dphi += w * r;
            }
        }
        psi = quad_sum(psi);
        dpsi = quad_sum(dpsi);
        phi = quad_sum(phi);
        dphi = quad_sum(dphi);
        const double f = 1.0 + rho * (psi + phi);
        if (fabs(f) <= 2.0 * kEps * (1.0 + rho * (fabs(psi) + fabs(phi)))) break;
        if (f < 0.0) lo = tau;
        else hi = tau;
        const double Q = dpsi * (di - tau) * (di - tau);
        const double P = psi - Q / (di - tau);
        double nt;
        if (!last) {
            const double S = dphi * (dn - tau) * (dn - tau);
            const double R = phi - S / (dn - tau);
            const double c = 1.0 + rho * (P + R);
            const double a2 = c;
            const double a1 = -c * (di + dn) - rho * (Q + S);
            const double a0 = c * di * dn + rho * (Q * dn + S * di);
            const double sq = sqrt(fmax(a1 * a1 - 4.0 * a2 * a0, 0.0));
            double x1, x2;
            if (a1 <= 0.0) {
                x1 = (a2 != 0.0) ? (-a1 + sq) / (2.0 * a2) : HUGE_VAL;
                x2 = (-a1 + sq != 0.0) ? 2.0 * a0 / (-a1 + sq) : HUGE_VAL;
            } else {
                x1 = (-a1 - sq != 0.0) ? 2.0 * a0 / (-a1 - sq) : HUGE_VAL;
                x2 = (a2 != 0.0) ? (-a1 - sq) / (2.0 * a2) : HUGE_VAL;
            }
            if (x1 > lo && x1 < hi) nt = x1;
            else if (x2 > lo && x2 < hi) nt = x2;
            else nt = 0.5 * (lo + hi);
        } else {
            const double c = 1.0 + rho * P;
            nt = (c != 0.0) ? di + rho * Q / c : 0.5 * (lo + hi);
            if (!(nt > lo && nt < hi)) nt = 0.5 * (lo + hi);
        }
        if (nt == tau || fabs(nt - tau) <= 2.0 * kEps * fabs(nt)) {
            tau = nt;
            break;
        }
        tau = nt;
    }
    *org = o;
    return tau;
}

// Divide and conquer (Cuppen) on the k x k symmetric tridiagonal, run by the whole workgroup:
// T = diag(T1', T2') + rho v v^T with v = e_m + sign(beta) e_{m+1}, rho = |beta| (beta the
// coupling of the halves, removed from their touching diagonal entries).  Waves 0 and 1 solve
// T1' and T2' by QL at the same time; the merge solves D + rho z z^T, z = [last row of Q1;
// sign(beta) first row of Q2]: poles sorted, deflation (a negligible z component, or two poles
// close enough that a rotation zeroes one z component, LAPACK's criteria), one secular root
// per thread, the z of Gu and Eisenstat recomputed from the roots (orthogonal eigenvectors by
// construction), and the rank-one problem's eigenvectors applied to the halves' ones in place,
// one component per wave.  Output as for tridiag_ql (eigenvalues unsorted).  False if a half's
// QL failed.
__device__ bool tridiag_dc(int k, const double* a, const double* b, double* lam, StepShared& sh) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = k / 2, k2 = k - m;
    const double beta = b[m - 1];
    const double rho0 = fabs(beta), sg = beta >= 0.0 ? 1.0 : -1.0;
    double* Qt = sh.Qt;
    if (tid < k) sh.dca[tid] = a[tid] - ((tid == m - 1 || tid == m) ? rho0 : 0.0);
    if (tid < k - 1) sh.dcb[tid] = (tid == m - 1) ? 0.0 : b[tid];
    __syncthreads();
    if (wave == 0) {
        const bool o = tridiag_ql(m, sh.dca, sh.dcb, sh.lam, Qt);
        if (lane == 0) sh.dc_ok[0] = o ? 1 : 0;
    } else if (wave == 1) {
        const bool o = tridiag_ql(k2, sh.dca + m, sh.dcb + m, sh.lam + m, Qt + m * 64);
        if (lane == 0) sh.dc_ok[1] = o ? 1 : 0;
    }
    __syncthreads();
    if (!sh.dc_ok[0] || !sh.dc_ok[1]) return false;
    // second half's vectors to global components: x -> x + m (one row per wave at a time)
    for (int n = m + wave; n < k; n += kWaves) {
        const double v = Qt[n * 64 + lane];
        const double sft = __shfl(v, (lane - m) & 63);
        Qt[n * 64 + lane] = (lane >= m && lane < k) ? sft : 0.0;
    }
    __syncthreads();
    if (tid < k) {
        sh.dd[tid] = sh.lam[tid];
        sh.dz[tid] = (tid < m) ? Qt[tid * 64 + m - 1] : sg * Qt[tid * 64 + m];
    }
    __syncthreads();
    if (tid < k) {  // rank sort of the poles (ties by index)
        const double dn = sh.dd[tid];
        int r = 0;
        for (int j = 0; j < k; ++j) r += (sh.dd[j] < dn || (sh.dd[j] == dn && j < tid)) ? 1 : 0;
        sh.perm[r] = tid;
    }
    __syncthreads();
    if (tid < k) {
        sh.ds[tid] = sh.dd[sh.perm[tid]];
        sh.zs[tid] = sh.dz[sh.perm[tid]];
    }
    __syncthreads();
    {  // normalisation: ||z||^2 and max |d| over the block
        const double z2 = (tid < k) ? sh.zs[tid] * sh.zs[tid] : 0.0;
        const double da = (tid < k) ? fabs(sh.ds[tid]) : 0.0;
        const double nz2 = block_sum(z2, sh.red);
        const double dmax = block_max(da, sh.red + kWaves);
        if (tid < k) sh.zs[tid] *= rsqrt_nr(nz2);
        if (tid == 0) {
            sh.dc_rho = rho0 * nz2;
            sh.dc_tol = 8.0 * kEps * fmax(dmax, rho0 * nz2);
        }
    }
    __syncthreads();
    if (tid == 0) {  // deflation in sorted order (each pair test depends on the previous kept pole)
        const double rho = sh.dc_rho, tol = sh.dc_tol;
        int nrot = 0, lastj = -1;
        for (int j = 0; j < k; ++j) {
            const double zj = sh.zs[j];
            if (rho * fabs(zj) <= tol) {
                sh.defl[j] = 1;
                continue;
            }
            sh.defl[j] = 0;
            if (lastj >= 0) {
                const double zl = sh.zs[lastj];
                const double r = hypot(zl, zj);
                const double c = zj / r, s = -zl / r;
                const double t = sh.ds[j] - sh.ds[lastj];
                if (fabs(t * c * s) <= tol) {
                    sh.zs[j] = r;
                    sh.zs[lastj] = 0.0;
                    const double dl = sh.ds[lastj], dj = sh.ds[j];
                    sh.ds[lastj] = dl * c * c + dj * s * s;
                    sh.ds[j] = dl * s * s + dj * c * c;
                    sh.r1[nrot] = sh.perm[lastj];
                    sh.r2[nrot] = sh.perm[j];
                    sh.rc[nrot] = c;
                    sh.rs[nrot] = s;
                    ++nrot;
                    sh.defl[lastj] = 1;
                }
            }
            lastj = j;
        }
        sh.dc_nrot = nrot;
    }
    __syncthreads();
    if (tid < k && !sh.defl[tid]) {  // compaction of the kept poles, in sorted order
        int pos = 0;
        for (int j = 0; j < tid; ++j) pos += sh.defl[j] ? 0 : 1;
        sh.keep[pos] = tid;
        sh.dk[pos] = sh.ds[tid];
        sh.zk[pos] = sh.zs[tid];
    }
    if (tid == 0) {
        int K = 0;
        for (int j = 0; j < k; ++j) K += sh.defl[j] ? 0 : 1;
        sh.dc_K = K;
    }
    __syncthreads();
    const int K = sh.dc_K;
    const double rho = sh.dc_rho;
    if (wave == 0) {  // deflation rotations, in order, on the vector rows
        for (int q = 0; q < sh.dc_nrot; ++q) {
            const int p1 = sh.r1[q], p2 = sh.r2[q];
            const double c = sh.rc[q], s = sh.rs[q];
            if (lane < k) {
                const double vl = Qt[p1 * 64 + lane], vj = Qt[p2 * 64 + lane];
                Qt[p1 * 64 + lane] = c * vl + s * vj;
                Qt[p2 * 64 + lane] = -s * vl + c * vj;
            }
        }
    }
    // roots: root q on the quad of threads 4q..4q+3 (the quad's lanes stay together: K <= 64)
    {
        const int q = tid >> 2, part = tid & 3;
        if (q < K) {
            int o;
            const double t = secular_root(q, part, K, sh.dk, sh.zk, rho, &o);
            if (part == 0) {
                sh.tau[q] = t;
                sh.org[q] = o;
            }
        }
    }
    __syncthreads();
    // per-root work below: root i on lane i / 4 of wave i % 4
    const int ri = lane * kWaves + wave;
    if (ri < K) {  // z recomputed from the roots: zh_j^2 = prod_i (lam_i - d_j) / prod_{i != j} (d_i - d_j) / rho
        const double dj = sh.dk[ri];
        double num = 1.0;
        for (int i = 0; i < K; ++i) {
            num *= (sh.dk[sh.org[i]] - dj) + sh.tau[i];
            if (i != ri) num *= rcp_nr(sh.dk[i] - dj);
        }
        sh.zh[ri] = copysign(sqrt(fabs(num / rho)), sh.zk[ri]);
    }
    __syncthreads();
    if (ri < K) {  // eigenvector ri of the rank-one problem: zh_j / (d_j - lam_ri), normalised
        const double dorg = sh.dk[sh.org[ri]], t = sh.tau[ri];
        double n2 = 0.0;
        for (int j = 0; j < K; ++j) {
            const double u = sh.zh[j] * rcp_nr((sh.dk[j] - dorg) - t);
            sh.U[j * 64 + ri] = u;
            n2 += u * u;
        }
        const double inv = rsqrt_nr(n2);
        for (int j = 0; j < K; ++j) sh.U[j * 64 + ri] *= inv;
    }
    __syncthreads();
    // kept vector rows <- (kept rows) U, component by component (component x on wave x % 4):
    // lane j holds component x of kept row j, broadcast to all lanes by readlane
    const int rowj = (lane < K) ? sh.perm[sh.keep[lane]] : 0;
    for (int x = wave; x < k; x += kWaves) {
        const double vj = (lane < K) ? Qt[rowj * 64 + x] : 0.0;
        double acc = 0.0;
#pragma unroll 4
        for (int j = 0; j < K; ++j) acc = fma(lane_get(vj, j), sh.U[j * 64 + lane], acc);
        if (lane < K) Qt[rowj * 64 + x] = acc;
    }
    if (tid < k) {
        const int sj = tid;  // sorted position
        if (sh.defl[sj]) lam[sh.perm[sj]] = sh.ds[sj];
    }
    if (ri < K) lam[sh.perm[sh.keep[ri]]] = sh.dk[sh.org[ri]] + sh.tau[ri];
    __syncthreads();
    return true;
}

// Eigen-decomposition of the tridiagonal (a, b) by the whole workgroup: divide and conquer from
// k = 16 on, QL (wave 0) below it or should a half fail.
__device__ bool tridiag_eig(int k, const double* a, const double* b, double* lam, StepShared& sh) {
    __shared__ int ok_sh;
    if (k >= 16 && tridiag_dc(k, a, b, lam, sh)) return true;
    if (threadIdx.x < 64) {
        const bool q = tridiag_ql(k, a, b, lam, sh.Qt);
        if (threadIdx.x == 0) ok_sh = q ? 1 : 0;
    }
    __syncthreads();
    return ok_sh != 0;
}

// ------------------------------------------------------------------------- quadrature
// node p (0 <= p < 3 * 2^lev) of refinement level lev >= 1: odd multiples of 2^-lev in (-3, 3)
__device__ __forceinline__ double level_abscissa(int lev, int p) {
    const int half = 3 * (1 << (lev - 1));
    const double step = ldexp(1.0, -lev);
    return (p < half) ? -(2.0 * (half - 1 - p) + 1.0) * step : (2.0 * (p - half) + 1.0) * step;
}

// node t of the flattened levels 0..L (t < 6 * 2^L + 1): level and abscissa u
__device__ __forceinline__ void flat_node(int t, int* level, double* u) {
    if (t < 7) {
        *level = 0;
        *u = (double)(t - 3);
        return;
    }
    int lev = 1;
    while (t >= 3 * (1 << (lev + 1)) + 1) ++lev;
    const int p = t - (3 * (1 << lev) + 1);
    *level = lev;
    *u = level_abscissa(lev, p);
}

struct QuadOut {
    double value;
    int level;
    int converged;
};

// Whole block.  Evaluates `count` nodes (abscissae from node_u(q) -> (u, level)), each shared
// by tpn threads that split the k-term sum; leaves in sh.lev_sum[lev - lev0] the per-level sums
// of w(u) f(x(u)) for levels lev0..lev0+nlev-1.  Fixed order.
template <typename NodeFn>
__device__ void eval_nodes(int count, int lev0, int nlev, NodeFn node_u, double center, double radius, int k,
                           const double* lam, const double* cf, double h, StepShared& sh) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tpn = max(1, min(kMaxTpn, kBlock / max(count, 1)));
    const int per_round = kBlock / tpn;
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    for (int base = 0; base < count; base += per_round) {
        const int node = base + tid / tpn, part = tid % tpn;
        double re = 0.0, im = 0.0, w = 0.0;
        int lev = -1;
        if (node < count) {
            double u;
            node_u(node, &u, &lev);
            const double shu = kHalfPi * sinh(u);
            const double x = center + radius * tanh(shu);
            const double ch = cosh(shu);
            w = radius * kHalfPi * cosh(u) / (ch * ch);
            for (int n = part; n < k; n += tpn) {
                double sn, cn;
                sincos(lam[n] * x, &sn, &cn);
                re = fma(cf[n], cn, re);
                im = fma(-cf[n], sn, im);
            }
        }
        if (tpn > 1) {
            sh.pre[tid] = re;
            sh.pim[tid] = im;
            __syncthreads();
            if (part == 0 && node < count) {
                for (int q = 1; q < tpn; ++q) {
                    re += sh.pre[tid + q];
                    im += sh.pim[tid + q];
                }
            }
            __syncthreads();
        }
        if (part == 0 && node < count) {
            const double val = w * h * sqrt(fma(re, re, im * im));
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (lev - lev0 == q) acc[q] += val;
        }
    }
    for (int q = 0; q < nlev; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0) sh.red[wave * 8 + q] = s;
    }
    __syncthreads();
    if (threadIdx.x < nlev) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t += sh.red[w * 8 + threadIdx.x];
        sh.lev_sum[threadIdx.x] = t;
    }
    __syncthreads();
}

// Nodes and weights of the n-point Gauss-Legendre rule on [-1, 1] into sh.gx / sh.gw, thread i
// computing root i: Newton's method on P_n from the estimate cos(pi (i + 3/4) / (n + 1/2)),
// P_n and P_n' by the three-term recurrence, weight 2 / ((1 - x^2) P_n'(x)^2).  Whole block.
__device__ void gauss_legendre_nodes(int n, StepShared& sh) {
    const int i = threadIdx.x;
    if (i < n) {
        double x = cos(3.141592653589793 * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 64; ++it) {
            double p0 = 1.0, p1 = x;
            for (int q = 2; q <= n; ++q) {
                const double p2 = ((2.0 * q - 1.0) * x * p1 - (q - 1.0) * p0) / q;
                p0 = p1;
                p1 = p2;
            }
            dp = (n == 1) ? 1.0 : n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) <= 2e-16) break;
        }
        // derivative at the converged root
        double p0 = 1.0, p1 = x;
        for (int q = 2; q <= n; ++q) {
            const double p2 = ((2.0 * q - 1.0) * x * p1 - (q - 1.0) * p0) / q;
            p0 = p1;
            p1 = p2;
        }
        dp = (n == 1) ? 1.0 : n * (x * p1 - p0) / (x * x - 1.0);
        sh.gx[i] = x;
        sh.gw[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    __syncthreads();
}

// Whole block.  Integral of f over [a, b] by the n-point Gauss-Legendre rule (sh.gx, sh.gw),
// tpn threads per node as in eval_nodes; fixed order.
__device__ double gauss_integral(double a, double b, int n, int k, const double* lam, const double* cf, double h,
                                 StepShared& sh) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double center = 0.5 * (a + b), radius = 0.5 * (b - a);
    const int tpn = max(1, min(kMaxTpn, kBlock / n));
    const int node = tid / tpn, part = tid % tpn;
    double re = 0.0, im = 0.0;
    if (node < n) {
        const double x = center + radius * sh.gx[node];
        for (int q = part; q < k; q += tpn) {
            double sn, cn;
            sincos(lam[q] * x, &sn, &cn);
            re = fma(cf[q], cn, re);
            im = fma(-cf[q], sn, im);
        }
    }
    if (tpn > 1) {
        sh.pre[tid] = re;
        sh.pim[tid] = im;
        __syncthreads();
        if (part == 0 && node < n) {
            for (int q = 1; q < tpn; ++q) {
                re += sh.pre[tid + q];
                im += sh.pim[tid + q];
            }
        }
        __syncthreads();
    }
    const double val = (part == 0 && node < n) ? radius * sh.gw[node] * h * sqrt(fma(re, re, im * im)) : 0.0;
    const double s = wave_sum(val);
    if (lane == 0) sh.red[wave * 8] = s;
    __syncthreads();
    double total = 0.0;
    for (int w = 0; w < kWaves; ++w) total += sh.red[w * 8];
    __syncthreads();
    return total;
}

// Whole block.  Integral of f over [a, b] by the adaptive tanh-sinh rule: stop at the first
// level >= max(1, min_level) whose change is <= max(rel_tol |I|, noise_rate (b - a)).
// Levels 0..L1 (L1 = min(3, max_level), 49 nodes) are evaluated in one pass, later levels one
// at a time.
__device__ __noinline__ QuadOut integrate(double a, double b, const Problem& P, int k, const double* lam, const double* cf,
                             double h, double noise_rate, StepShared& sh) {
    QuadOut out;
    out.value = 0.0;
    out.level = 0;
    out.converged = 1;
    if (b == a) return out;
    if (P.gauss_n > 0) {  // the fast option: fixed rule, no error estimate
        out.value = gauss_integral(a, b, P.gauss_n, k, lam, cf, h, sh);
        return out;
    }
    const double center = 0.5 * (a + b), radius = 0.5 * (b - a);
    const double abs_tol = noise_rate * (b - a);
    const int L1 = min(3, P.quad_max_level);
    eval_nodes(6 * (1 << L1) + 1, 0, L1 + 1, [](int q, double* u, int* lev) { flat_node(q, lev, u); }, center, radius,
               k, lam, cf, h, sh);
    double total = 0.0, prev = 0.0, value = 0.0;
    out.converged = 0;
    for (int lev = 0; lev <= P.quad_max_level; ++lev) {
        if (lev > L1) {
            eval_nodes(3 * (1 << lev), lev, 1, [lev](int q, double* u, int* l) {
                *u = level_abscissa(lev, q);
                *l = lev;
            }, center, radius, k, lam, cf, h, sh);
            total += sh.lev_sum[0];
            __syncthreads();
        } else {
            total += sh.lev_sum[lev];
        }
        value = total * ldexp(1.0, -lev);
        out.level = lev;
        if (lev >= 1 && lev >= P.quad_min_level && fabs(value - prev) <= fmax(P.quad_rel_tol * fabs(value), abs_tol)) {
            out.converged = 1;
            break;
        }
        prev = value;
    }
    out.value = value;
    return out;
}

// --------------------------------------------------------------------- step search
struct StepOut {
    double tau, err;
    int quad_ok;
    int underflow;
    int integrals;
    int max_level;
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
    o.integrals = 0;
    o.max_level = 0;
    auto I = [&](double a, double b) {
        QuadOut q = integrate(a, b, P, k, sh.lam, sh.cf, h, noise, sh);
        o.quad_ok &= q.converged;
        o.integrals += 1;
        o.max_level = max(o.max_level, q.level);
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
    const bool ok = tridiag_eig(k, sh.d, sh.e, sh.lam, sh);
    if (tid < k) sh.cf[tid] = sh.Qt[tid * 64 + k - 1] * sh.Qt[tid * 64];
    __syncthreads();
    return ok;
}

// omega_i = sum_n Q[i][n] exp(-i lam_n tau) Q[0][n], scaled by s_i for the raw columns
__device__ void write_omega(DevState* st, int k, double tau, bool scale_raw, StepShared& sh) {
    const int tid = threadIdx.x;
    if (tid < k) {
        double re = 0.0, im = 0.0;
        for (int n = 0; n < k; ++n) {
            double sn, cn;
            sincos(sh.lam[n] * tau, &sn, &cn);
            const double a = sh.Qt[n * 64 + tid] * sh.Qt[n * 64];
            re = fma(a, cn, re);
            im = fma(-a, sn, im);
        }
        const double sc = scale_raw ? st->s[tid] : 1.0;
        st->omega[tid] = make_double2(re * sc, im * sc);
    }
}

// Krylov coefficients of the sample times this step covers (t_s <= t_end), computed like
// omega with tau = t_s - t_now, and the bound at the end of the step for each of them.
__device__ void sample_coefficients(DevState* st, int k, double t_now, double t_end, double bound,
                                    StepShared& sh) {
    __shared__ int lo_sh, hi_sh;
    if (threadIdx.x == 0) {
        const int n = st->smp.n;
        int s = st->smp.next;
        while (s < n && st->smp.t[s] <= t_end) ++s;
        lo_sh = st->smp.next;
        hi_sh = s;
        st->smp.lo = lo_sh;
        st->smp.hi = s;
        st->smp.next = s;
    }
    __syncthreads();
    const int lo = lo_sh, cnt = hi_sh - lo_sh;
    for (int p = threadIdx.x; p < cnt * k; p += blockDim.x) {
        const int smp = lo + p / k, i = p % k;
        const double dt = st->smp.t[smp] - t_now;
        double re = 0.0, im = 0.0;
        for (int n = 0; n < k; ++n) {
            double sn, cn;
            sincos(sh.lam[n] * dt, &sn, &cn);
            const double a = sh.Qt[n * 64 + i] * sh.Qt[n * 64];
            re = fma(a, cn, re);
            im = fma(-a, sn, im);
        }
        const double sc = st->s[i];
        st->smp.omega[(size_t)smp * kMaxM + i] = make_double2(re * sc, im * sc);
        if (i == 0) st->smp.bound[smp] = bound;
    }
}

__device__ void step_body(DevState* st, int* host_flag, bool controller) {
    __shared__ StepShared sh;
    const int tid = threadIdx.x;
    if (tid == 0) {  // no samples unless this step assigns some
        st->smp.lo = 0;
        st->smp.hi = 0;
    }
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
    const uint64_t c0 = wall_clock64();
    const bool ok = prepare_spectrum(st, k, sh);
    if (P.gauss_n > 0) gauss_legendre_nodes(P.gauss_n, sh);
    const uint64_t c1 = wall_clock64();
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
    const uint64_t c2 = wall_clock64();
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
    if (controller && st->smp.n > 0) {
        const double t_end = (so.tau == t_rem || breakdown) ? P.t : t_now + so.tau;
        sample_coefficients(st, k, t_now, t_end, st->beta0 * (st->err_acc + so.err), sh);
    }
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
            const double tick_us = 1e6 / (double)kWallClockHz;
            tr[8] = (double)(c1 - c0) * tick_us;
            tr[9] = (double)(c2 - c1) * tick_us;
            tr[10] = (double)so.integrals;
            tr[11] = (double)so.max_level;
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

// batched: one workgroup per job of the round
__global__ __launch_bounds__(kBlock) void k_bstep(const JobView* __restrict__ jobs) {
    __shared__ double lds[kWaves];
    const JobView& J = jobs[blockIdx.x];
    finish_last_norm(J.st, J.rb, lds);
    step_body(J.st, nullptr, true);
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
    const bool ok = tridiag_eig(k, sh.d, sh.e, sh.lam, sh);
    if (tid == 0) *status = ok ? 0 : 1;
    if (tid < k) {
        lambda[tid] = sh.lam[tid];
        for (int n = 0; n < k; ++n) Q[n * k + tid] = sh.Qt[n * 64 + tid];  // column-major
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
    if (P.gauss_n > 0) gauss_legendre_nodes(P.gauss_n, sh);
    const QuadOut q = integrate(a, b, P, k, sh.lam, sh.cf, h, h * (double)k * kEps, sh);
    if (tid == 0) {
        out[0] = q.value;
        out[1] = (double)q.level;
        out[2] = (double)q.converged;
    }
}

}  // namespace

hipError_t launch_step(DevState* st, const RedBuf& rb, int* host_flag, hipStream_t s, hipEvent_t done) {
    if (done) hipExtLaunchKernelGGL(k_step, dim3(1), dim3(kBlock), 0, s, nullptr, done, 0, st, rb, host_flag);
    else hipLaunchKernelGGL(k_step, dim3(1), dim3(kBlock), 0, s, st, rb, host_flag);
    return hipGetLastError();
}

hipError_t launch_bstep(const JobView* jobs, int n_jobs, hipStream_t s) {
    if (n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bstep, dim3(n_jobs), dim3(kBlock), 0, s, jobs);
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
