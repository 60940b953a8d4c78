// Device construction of the paper's exemplary Hamiltonian (Sec. "Exemplary System", eq.
// fullHamiltonianSimple): two bosonic modes a_0, b_0 with N_0 = n_0 + m_0 conserved and K + K'
// memory qubits with N_m excitations (eq. subsetOccupations).  Matrix creation is the paper's
// memory limit (Sec. "Analysis of Performance"); here the CSR is written directly in device
// memory, one wavefront per row, with no host-side basis, lookup table or triplet list.
//
// Basis (the paper's product of the two conserved sectors, each enumerated in descending
// lexicographic order of the occupation tuples): row = i0 * C + i1 with i0 = N_0 - n_0 and i1
// the rank of the qubit configuration among the C = binom(K + K', N_m) configurations.  A
// configuration is a bit mask, bit q = occupation of qubit mode q (a_1..a_K, then a'_1..a'_K').
//
// Row r holds, sorted by column: its diagonal; for every pair of qubit modes (u, v) with
// different occupations the entry of the pair's hopping term at the configuration with u and v
// exchanged; the C_0 term's entries at i0 - 1 (a boson moved from b_0 to a_0) and i0 + 1.  Its
// length is 1 + N_m (K + K' - N_m) + [n_0 < N_0] + [n_0 > 0], so row pointers have a closed form.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "te_internal.h"

namespace te {
namespace {

constexpr int kModelSlots = 512;  // sorted entries per row (power of two, >= longest row)
constexpr int kRowsPerBlock = kBlock / 64;

struct ModelArgs {
    int n;             // qubit modes K + K'
    int K;             // first K qubit modes are a_1..a_K
    int Nm, N0;
    int C;             // qubit configurations
    int slots;         // power of two >= longest row
    int64_t dim;
    double eps_m, Nc, NcMinusDNc, C0;
    const int64_t* binom;  // binom[a * 64 + b] = binomial(a, b), 0 <= b <= a < 64
    const double* hop;     // hop[u * 64 + v]: amplitude of (a_u^+ a_v + h.c.), symmetric
};

__device__ __forceinline__ int64_t binom_at(const ModelArgs& A, int a, int b) {
    return (b < 0 || b > a) ? 0 : A.binom[a * 64 + b];
}

// rank of a configuration in descending lexicographic order: every zero at position i with r
// ones still to place is preceded by the configurations that put a one there
__device__ int64_t config_rank(const ModelArgs& A, unsigned long long mask) {
    int64_t rank = 0;
    int r = A.Nm;
    for (int i = 0; i < A.n && r > 0; ++i) {
        if ((mask >> i) & 1ull) --r;
        else rank += binom_at(A, A.n - 1 - i, r - 1);
    }
    return rank;
}

__device__ unsigned long long config_unrank(const ModelArgs& A, int64_t rank) {
    unsigned long long mask = 0;
    int r = A.Nm;
    for (int i = 0; i < A.n && r > 0; ++i) {
        const int64_t c = binom_at(A, A.n - 1 - i, r - 1);
        if (rank < c) {
            mask |= 1ull << i;
            --r;
        } else {
            rank -= c;
        }
    }
    return mask;
}

// first stored entry of row r (closed form of the row lengths)
__device__ __forceinline__ int64_t row_start(const ModelArgs& A, int64_t r) {
    const int64_t Q = (int64_t)A.Nm * (A.n - A.Nm);
    const int64_t i0 = r / A.C, i1 = r - i0 * A.C;
    // entries per configuration in blocks 0..i0-1: 1 + Q each, plus [i > 0] + [i < N_0] for block i
    const int64_t before = i0 * (1 + Q) + (i0 > 0 ? i0 - 1 : 0) + (i0 < A.N0 ? i0 : (int64_t)A.N0);
    const int64_t len = 1 + Q + (i0 > 0 ? 1 : 0) + (i0 < A.N0 ? 1 : 0);
    return (int64_t)A.C * before + i1 * len;
}

__global__ __launch_bounds__(kBlock) void k_model_row_ptr(ModelArgs A, int* __restrict__ row_ptr) {
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r <= A.dim; r += (int64_t)gridDim.x * kBlock)
        row_ptr[r] = (int)row_start(A, r);
}

// The diagonal, evaluated left to right as the paper's term is written (no contraction, so
// the value does not depend on the compiler's choice of fused operations).
__device__ double diag_value(const ModelArgs& A, int n0, int nk, int nkp) {
#pragma clang fp contract(off)
    const double a = A.eps_m * (1.0 - (double)n0 / A.Nc) * (double)nk;
    const double b = A.eps_m * (1.0 - (double)n0 / A.NcMinusDNc) * (double)nkp;
    return a + b;
}

// amplitude * sqrt(n_src (n_dst + 1)) of a boson hop out of a mode with n_src into one with n_dst
__device__ double hop_value(double amp, int n_src, int n_dst) {
#pragma clang fp contract(off)
    return amp * sqrt((double)n_src * ((double)n_dst + 1.0));
}

// one wavefront per row: generate, sort by column (bitonic network in LDS), store
__global__ __launch_bounds__(kBlock) void k_model_fill(ModelArgs A, int* __restrict__ col, double* __restrict__ val) {
    __shared__ int skey[kRowsPerBlock][kModelSlots];
    __shared__ double sval[kRowsPerBlock][kModelSlots];
    __shared__ unsigned char ones[kRowsPerBlock][64], zeros[kRowsPerBlock][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * kRowsPerBlock + w;
    const bool live = r < A.dim;  // dead waves still take part in the block's barriers
    const int64_t rr = live ? r : A.dim - 1;
    const int i0 = (int)(rr / A.C);
    const int64_t i1 = rr - (int64_t)i0 * A.C;
    const int n0 = A.N0 - i0, m0 = i0;
    const unsigned long long mask = config_unrank(A, i1);
    if (lane < A.n) {
        const int bit = (int)((mask >> lane) & 1ull);
        const int below = __popcll(mask & ((1ull << lane) - 1ull));
        if (bit) ones[w][below] = (unsigned char)lane;
        else zeros[w][lane - below] = (unsigned char)lane;
    }
    __syncthreads();
    const int nz = A.n - A.Nm;
    const int Q = A.Nm * nz;
    const int len = 1 + Q + (n0 > 0 ? 1 : 0) + (n0 < A.N0 ? 1 : 0);
    const int64_t base_col = (int64_t)i0 * A.C;
    for (int e = lane; e < A.slots; e += 64) {
        int key = INT_MAX;
        double v = 0.0;
        if (e == 0) {
            const int nk = __popcll(mask & ((A.K >= 64) ? ~0ull : ((1ull << A.K) - 1ull)));
            key = (int)rr;
            v = diag_value(A, n0, nk, A.Nm - nk);
        } else if (e <= Q) {
            const int a = (e - 1) / nz, b = (e - 1) - a * nz;
            const int u = ones[w][a], q = zeros[w][b];
            const unsigned long long src = mask ^ (1ull << u) ^ (1ull << q);
            key = (int)(base_col + config_rank(A, src));
            v = hop_value(A.hop[u * 64 + q], 1, 0);
        } else {
            int extra = e - Q - 1;  // 0: the n_0 - 1 source (if any), then the n_0 + 1 source
            if (extra == 0 && n0 > 0) {  // a_0^+ b_0 from (n_0 - 1, m_0 + 1): block i0 + 1
                key = (int)(rr + A.C);
                v = hop_value(A.C0, m0 + 1, n0 - 1);
            } else {
                if (n0 > 0) --extra;
                if (extra == 0 && n0 < A.N0) {  // b_0^+ a_0 from (n_0 + 1, m_0 - 1): block i0 - 1
                    key = (int)(rr - A.C);
                    v = hop_value(A.C0, n0 + 1, m0 - 1);
                }
            }
        }
        skey[w][e] = key;
        sval[w][e] = v;
    }
    __syncthreads();
    for (int k = 2; k <= A.slots; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < A.slots; i += 64) {
                const int l = i ^ j;
                if (l > i) {
                    const int ki = skey[w][i], kl = skey[w][l];
                    const bool up = (i & k) == 0;
                    if ((ki > kl) == up) {
                        skey[w][i] = kl;
                        skey[w][l] = ki;
                        const double t = sval[w][i];
                        sval[w][i] = sval[w][l];
                        sval[w][l] = t;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (!live) return;
    const int64_t start = row_start(A, rr);
    for (int e = lane; e < len; e += 64) {
        col[start + e] = skey[w][e];
        val[start + e] = sval[w][e];
    }
}

// ------------------------------------------------------------------------ Bose chain
// Fock states |n_1..n_K> with sum n_k = N (Sec. "Creation of Hamiltonian Matrix", eqs.
// basisState and totalOccupationNumber) in descending lexicographic order.  The index map and
// its inverse (eq. findIndices) are closed forms of the combinatorial number system instead of
// a hash table: with R_i = N - sum_{l<i} n_l, rank = sum_i comp(R_i - n_i - 1, K - i), where
// comp(s, m) = binom(s + m - 1, m - 1) counts the compositions of s into m parts (the states
// that agree up to i and hold more bosons in mode i).  A hop between modes k and k + 1 changes
// only the terms i = k, k + 1 of that sum, so the partner's rank is the row's own rank plus or
// minus one comp() term.
struct BoseArgs {
    int K, N;
    int slots;             // power of two >= 2K - 1
    int64_t dim;
    int bw;                // row stride of the binomial table
    const int64_t* binom;  // binom[a * bw + b], a <= N + K, b <= K
    const double* U;       // on-site interaction U_k n_k (n_k - 1)
    const double2* hop;    // a_k of a_k b_k^+ b_{k+1} + conj(a_k) b_{k+1}^+ b_k
};

__device__ __forceinline__ int64_t comp(const BoseArgs& A, int s, int m) {
    if (m == 0) return s == 0 ? 1 : 0;
    if (s < 0) return 0;
    return A.binom[(int64_t)(s + m - 1) * A.bw + (m - 1)];
}

// occupation of mode i of the state of rank `rank` (lanes = modes; every lane runs the same walk
// and keeps its own mode), and R_i = bosons left for modes i..K-1.  Within the block of states
// that agree before mode i, comp(R_i - v - 1, K - i) of them hold more than v bosons in mode i,
// a count that falls as v grows: n_i is the smallest v whose count does not exceed the rank left,
// found by bisection, so a row costs O(K log N) table reads.
__device__ void bose_unrank(const BoseArgs& A, int64_t rank, int lane, int* n_lane, int* R_lane) {
    int R = A.N, mine = 0, mineR = 0;
    for (int i = 0; i < A.K; ++i) {
        const int m = A.K - i;
        int lo = 0, hi = R;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (comp(A, R - mid - 1, m) <= rank)
                hi = mid;
            else
                lo = mid + 1;
        }
        rank -= comp(A, R - lo - 1, m);
        if (lane == i) {
            mine = lo;
            mineR = R;
        }
        R -= lo;
    }
    *n_lane = mine;
    *R_lane = mineR;
}

// entries per row: diagonal + a hop out of each occupied mode to each neighbour
__global__ __launch_bounds__(kBlock) void k_bose_count(BoseArgs A, int* __restrict__ cnt) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * kRowsPerBlock + w;
    if (r >= A.dim) return;
    int n, R;
    bose_unrank(A, r, lane, &n, &R);
    const bool occ = lane < A.K && n > 0;
    const unsigned long long m = __ballot(occ);
    const int nz = __popcll(m);
    if (lane == 0) cnt[r] = 1 + 2 * nz - (int)(m & 1ull) - (int)((m >> (A.K - 1)) & 1ull);
}

// exclusive scan of the row counts into row_ptr: per-block scans of 1024 rows, a scan of the
// block totals, and the block offsets added back
constexpr int kScanRows = 4 * kBlock;

__global__ __launch_bounds__(kBlock) void k_scan_blocks(const int* __restrict__ cnt, int* __restrict__ out,
                                                        int64_t* __restrict__ bsum, int64_t n) {
    __shared__ int64_t sh[kBlock];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanRows + 4 * tid;
    int v[4];
    int64_t t = 0;
    for (int q = 0; q < 4; ++q) {
        v[q] = (base + q < n) ? cnt[base + q] : 0;
        t += v[q];
    }
    sh[tid] = t;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {  // inclusive scan of the thread totals
        const int64_t x = (tid >= o) ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += x;
        __syncthreads();
    }
    int64_t run = sh[tid] - t;
    for (int q = 0; q < 4; ++q) {
        if (base + q < n) out[base + q] = (int)run;
        run += v[q];
    }
    if (tid == kBlock - 1) bsum[blockIdx.x] = sh[tid];
}

__global__ __launch_bounds__(kBlock) void k_scan_totals(int64_t* __restrict__ bsum, int64_t nb, int64_t* __restrict__ total) {
    __shared__ int64_t sh[kBlock];
    const int tid = threadIdx.x;
    int64_t off = 0;
    for (int64_t c = 0; c < nb; c += kBlock) {
        const int64_t x = (c + tid < nb) ? bsum[c + tid] : 0;
        sh[tid] = x;
        __syncthreads();
        for (int o = 1; o < kBlock; o <<= 1) {
            const int64_t y = (tid >= o) ? sh[tid - o] : 0;
            __syncthreads();
            sh[tid] += y;
            __syncthreads();
        }
        if (c + tid < nb) bsum[c + tid] = off + sh[tid] - x;  // exclusive
        off += sh[kBlock - 1];
        __syncthreads();
    }
    if (tid == 0) *total = off;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int* __restrict__ out, const int64_t* __restrict__ bsum,
                                                     int64_t n, const int64_t* __restrict__ total) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] += (int)bsum[i / kScanRows];
    if (i == n) out[n] = (int)*total;
}

// one wavefront per row: the row's entries (lane k: the hops between modes k and k + 1),
// sorted by column in LDS, stored at row_ptr[r]
__global__ __launch_bounds__(kBlock) void k_bose_fill(BoseArgs A, const int* __restrict__ row_ptr,
                                                      int* __restrict__ col, double2* __restrict__ val) {
    __shared__ int skey[kRowsPerBlock][128];
    __shared__ double2 sval[kRowsPerBlock][128];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * kRowsPerBlock + w;
    const bool live = r < A.dim;
    const int64_t rr = live ? r : A.dim - 1;
    int n, R;
    bose_unrank(A, rr, lane, &n, &R);
    const int n1 = __shfl_down(n, 1);  // occupation of mode lane + 1
    // diagonal sum_k U_k n_k (n_k - 1), summed in mode order
    const double term = (lane < A.K) ? (double)n * ((double)n - 1.0) * A.U[lane] : 0.0;
    double diag = 0.0;
    for (int k = 0; k < A.K; ++k) diag += __shfl(term, k);
    for (int e = lane; e < A.slots; e += 64) {
        skey[w][e] = INT_MAX;
        sval[w][e] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (lane < A.K - 1) {
        const double2 a = A.hop[lane];
        // a_k b_k^+ b_{k+1} from the state with (n_k - 1, n_{k+1} + 1)
        if (n > 0) {
            const double sq = sqrt((double)(n1 + 1) * ((double)(n - 1) + 1.0));
            skey[w][2 * lane] = (int)(rr + comp(A, R - n, A.K - lane - 1));
            sval[w][2 * lane] = make_double2(a.x * sq, a.y * sq);
        }
        // conj(a_k) b_{k+1}^+ b_k from the state with (n_k + 1, n_{k+1} - 1)
        if (n1 > 0) {
            const double sq = sqrt((double)(n + 1) * ((double)(n1 - 1) + 1.0));
            skey[w][2 * lane + 1] = (int)(rr - comp(A, R - n - 1, A.K - lane - 1));
            sval[w][2 * lane + 1] = make_double2(a.x * sq, -a.y * sq);
        }
    }
    if (lane == 0) {
        skey[w][2 * (A.K - 1)] = (int)rr;
        sval[w][2 * (A.K - 1)] = make_double2(diag, 0.0);
    }
    __syncthreads();
    for (int k = 2; k <= A.slots; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < A.slots; i += 64) {
                const int l = i ^ j;
                if (l > i) {
                    const int ki = skey[w][i], kl = skey[w][l];
                    const bool up = (i & k) == 0;
                    if ((ki > kl) == up) {
                        skey[w][i] = kl;
                        skey[w][l] = ki;
                        const double2 t = sval[w][i];
                        sval[w][i] = sval[w][l];
                        sval[w][l] = t;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (!live) return;
    const int start = row_ptr[rr], len = row_ptr[rr + 1] - start;
    for (int e = lane; e < len; e += 64) {
        col[start + e] = skey[w][e];
        val[start + e] = sval[w][e];
    }
}

}  // namespace

static BoseArgs bose_args(const BoseChainDev& B) {
    BoseArgs A;
    A.K = B.K;
    A.N = B.N;
    A.slots = B.slots;
    A.dim = B.dim;
    A.bw = B.bw;
    A.binom = B.binom;
    A.U = B.U;
    A.hop = B.hop;
    return A;
}

hipError_t launch_bose_row_ptr(const BoseChainDev& B, int* row_ptr, int* cnt, int64_t* scratch, hipStream_t s) {
    const BoseArgs A = bose_args(B);
    const int64_t blocks = (B.dim + kRowsPerBlock - 1) / kRowsPerBlock;
    k_bose_count<<<(unsigned)blocks, kBlock, 0, s>>>(A, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nb = (B.dim + kScanRows - 1) / kScanRows;
    k_scan_blocks<<<(unsigned)nb, kBlock, 0, s>>>(cnt, row_ptr, scratch, B.dim);
    k_scan_totals<<<1, kBlock, 0, s>>>(scratch, nb, scratch + nb);
    k_scan_add<<<(unsigned)((B.dim + 1 + kBlock - 1) / kBlock), kBlock, 0, s>>>(row_ptr, scratch, B.dim, scratch + nb);
    return hipGetLastError();
}

hipError_t launch_bose_fill(const BoseChainDev& B, const int* row_ptr, int* col, double2* val, hipStream_t s) {
    const BoseArgs A = bose_args(B);
    const int64_t blocks = (B.dim + kRowsPerBlock - 1) / kRowsPerBlock;
    k_bose_fill<<<(unsigned)blocks, kBlock, 0, s>>>(A, row_ptr, col, val);
    return hipGetLastError();
}

hipError_t launch_memory_burden(const MemoryBurdenDev& M, int* row_ptr, int* col, double* val, hipStream_t s) {
    ModelArgs A;
    A.n = M.n;
    A.K = M.K;
    A.Nm = M.Nm;
    A.N0 = M.N0;
    A.C = (int)M.C;
    A.slots = M.slots;
    A.dim = M.dim;
    A.eps_m = M.eps_m;
    A.Nc = M.Nc;
    A.NcMinusDNc = M.NcMinusDNc;
    A.C0 = M.C0;
    A.binom = M.binom;
    A.hop = M.hop;
    const int g1 = (int)std::min<int64_t>((M.dim + 1 + kBlock - 1) / kBlock, 65536);
    k_model_row_ptr<<<g1, kBlock, 0, s>>>(A, row_ptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t blocks = (M.dim + kRowsPerBlock - 1) / kRowsPerBlock;
    k_model_fill<<<(unsigned)blocks, kBlock, 0, s>>>(A, col, val);
    return hipGetLastError();
}

}  // namespace te
