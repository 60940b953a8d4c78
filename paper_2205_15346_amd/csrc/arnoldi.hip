// Row-parallel kernels of one Krylov build (paper, eq. arnoldi / Alg. 1 step 1, carried out
// as Lanczos on H with full re-orthogonalisation) and of the restart recombination
// (Alg. 1 step 3, w = V omega).
//
// Orthogonalisation scheme (differs from the paper's modified Gram-Schmidt, same result in
// exact arithmetic).  Iteration j makes two passes over the stored basis:
//   project  y = H V[:, j] fused with c'_i = V[:, i]^H y and g_i = V[:, i]^H V[:, j] for all
//            i <= j (one read of columns 0..j, raw = unnormalised);
//   fold     (small) reduces the tile partials; ||V[:, j]|| = sqrt(g_j) is the norm of the
//            previous residual (beta_{j-1}, breakdown test, scale s_j); corrects the
//            coefficients with the measured Gram matrix, c = c' - E_{:,j} c'_j - E_{:,j-1} c'_{j-1}
//            (E = G - I; the other columns of E multiply O(eps) coefficients);
//   update   V[:, j+1] = s_j y - sum_i c_i s_i V[:, i] (one read of columns 0..j, one write).
// The Gram correction keeps the new vector orthogonal to O(eps ||H|| / beta) without a
// second classical Gram-Schmidt sweep.  Normalisation is deferred: column i is stored
// unnormalised and s[i] = 1/||column i|| is applied where it is used.
//
// Tile partials are written with plain stores and folded by a later kernel, so the streaming
// kernels carry no device-scope fences or atomics.
#include <algorithm>
#include <type_traits>

#include <hip/hip_ext.h>

#include "te_internal.h"

namespace te {

int max_tiles(int dim) { return (dim + kBlock - 1) / kBlock; }

bool tiling_supported(int rpt_p, int g, int u, int rpt_u, int split) {
    const bool shape = (g == 4 && (u == 1 || u == 4)) || (g == 8 && u == 2) || (g == 2 && u == 8) ||
                       (g == 1 && (u == 8 || u == 16));
    return shape && (rpt_p == 1 || rpt_p == 2 || rpt_p == 4) && (rpt_u == 1 || rpt_u == 2) && (split == 0 || split == 1);
}

Tiling make_tiling(int dim, int rpt_p, int g, int u, int rpt_u, int split) {
    Tiling t;
    t.split = split;
    t.rpt_p = rpt_p;
    t.g = g;
    t.u = u;
    t.n_tiles_p = (dim + kBlock * rpt_p - 1) / (kBlock * rpt_p);
    t.rpt_u = rpt_u;
    t.n_tiles_u = (dim + kBlock * rpt_u - 1) / (kBlock * rpt_u);
    return t;
}

// Without tuning: two rows per thread once that still leaves >= 1024 tiles (4 workgroups per
// CU); measured on MI355X, 1-2 rows per thread stream at ~6.5 TB/s, 8 rows per thread at ~3.9.
Tiling default_tiling(int dim) {
    const int rpt = ((int64_t)dim >= (int64_t)kBlock * 2 * 1024) ? 2 : 1;
    return make_tiling(dim, rpt, 4, 4, rpt, 0);
}

// ------------------------------------------------------------------- setup / copy
__device__ __forceinline__ void setup_state(DevState* __restrict__ st, const Problem& prob) {
    st->p = prob;
    st->beta0 = 0.0;
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
    st->norm_init = 1;
    st->counted = 0;
    st->h = 0.0;
    st->ys = 1.0;
    st->s[0] = 1.0;
    st->smp.t = nullptr;
    st->smp.omega = nullptr;
    st->smp.bound = nullptr;
    st->smp.n = 0;
    st->smp.next = 0;
    st->smp.lo = 0;
    st->smp.hi = 0;
}

__global__ void k_setup(DevState* __restrict__ st, Problem prob) {
    if (threadIdx.x == 0) setup_state(st, prob);
}

__global__ __launch_bounds__(kBlock) void k_copy(const double2* __restrict__ src, double2* __restrict__ dst, int dim) {
    for (int r = blockIdx.x * kBlock + threadIdx.x; r < dim; r += gridDim.x * kBlock) dst[r] = src[r];
}

// -------------------------------------------------------------- project: SpMV + projections
// Cross-lane reduction of 32 doubles per lane (8 columns x {Re, Im} x {y, x}).  Five halving
// steps: in each, a lane keeps one half of its values, sends the other half to a partner lane
// and adds what the partner sent, so after step s each lane carries 32 / 2^s partial sums.
// The partners are chosen so that four of the five exchanges are DPP lane permutations of a
// plain VALU move (mirror within 16 lanes, mirror within 8, then the two quad swaps) and one
// is an LDS swizzle (lane ^ 16 within 32); a last exchange across the halves of the wave
// (lane ^ 32) completes the sums.  31 + 1 exchanges for 32 values instead of 6 per value for
// independent butterflies.  A partner must hold the same value set: each permutation flips
// the bit that decides which half a lane keeps and only bits not used by an earlier step.
// Every index is a compile-time constant so the array stays in registers.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double swizzle_xor16(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_ds_swizzle((int)b, 0x401F);  // bitmask mode: and 31, xor 16
    const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x401F);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

constexpr int kDppRowMirror = 0x140;      // lane i <-> 15 - i within 16
constexpr int kDppRowHalfMirror = 0x141;  // lane i <-> 7 - i within 8
constexpr int kDppQuadXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppQuadXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]

// H values move; BIT of the lane id decides which half is kept; EX selects the exchange
template <int N, int H, int BIT, int EX>
__device__ __forceinline__ void halve(double (&a)[N], int lane) {
    const bool hi = ((lane >> BIT) & 1) != 0;
#pragma unroll
    for (int v = 0; v < H; ++v) {
        const double send = hi ? a[v] : a[v + H];
        const double keep = hi ? a[v + H] : a[v];
        double got;
        if (EX == 0) got = dpp_move<kDppRowMirror>(send);
        else if (EX == 1) got = dpp_move<kDppRowHalfMirror>(send);
        else if (EX == 2) got = dpp_move<kDppQuadXor2>(send);
        else if (EX == 3) got = dpp_move<kDppQuadXor1>(send);
        else got = swizzle_xor16(send);
        a[v] = keep + got;
    }
}

// Returns, in every lane, the full sum of value halving_value(lane & 31).
__device__ __forceinline__ double halving_reduce32(double (&a)[32], int lane) {
    halve<32, 16, 3, 0>(a, lane);
    halve<32, 8, 2, 1>(a, lane);
    halve<32, 4, 1, 2>(a, lane);
    halve<32, 2, 0, 3>(a, lane);
    halve<32, 1, 4, 4>(a, lane);
    return a[0] + __shfl_xor(a[0], 32);
}

// index (0..31) of the value whose sum lanes l and l + 32 hold after halving_reduce32
__device__ __forceinline__ int halving_value(int lane) {
    return ((lane >> 3) & 1) * 16 + ((lane >> 2) & 1) * 8 + ((lane >> 1) & 1) * 4 + (lane & 1) * 2 + ((lane >> 4) & 1);
}

// The same for 16 values (4 columns): four DPP halvings inside each row of 16 lanes, then the
// rows are added pairwise (lane ^ 16, lane ^ 32).  Every lane returns the full sum of value
// halving_value16(lane & 15).
__device__ __forceinline__ double halving_reduce16(double (&a)[16], int lane) {
    halve<16, 8, 3, 0>(a, lane);
    halve<16, 4, 2, 1>(a, lane);
    halve<16, 2, 1, 2>(a, lane);
    halve<16, 1, 0, 3>(a, lane);
    const double v = a[0] + swizzle_xor16(a[0]);
    return v + __shfl_xor(v, 32);
}

__device__ __forceinline__ int halving_value16(int lane) {
    return ((lane >> 3) & 1) * 8 + ((lane >> 2) & 1) * 4 + ((lane >> 1) & 1) * 2 + (lane & 1);
}

// One stored entry times an entry of x, added to acc: complex entries, or real ones (a matrix
// whose imaginary parts are all zero is stored with 8-byte entries; the products are the same
// values, since the imaginary part would only add exact zeros).
__device__ __forceinline__ double2 entry_fma(double2 v, double2 x, double2 acc) { return cfma(v, x, acc); }
__device__ __forceinline__ double2 entry_fma(double v, double2 x, double2 acc) {
    acc.x = fma(v, x.x, acc.x);
    acc.y = fma(v, x.y, acc.y);
    return acc;
}
template <typename VT>
__device__ __forceinline__ VT entry_zero();
template <>
__device__ __forceinline__ double2 entry_zero<double2>() { return make_double2(0.0, 0.0); }
template <>
__device__ __forceinline__ double entry_zero<double>() { return 0.0; }

// The build of this restart is over at iteration j (finished, or broken down before j): both
// fields are loaded before either is tested, so the test costs one round trip.
__device__ __forceinline__ bool build_over(const DevState* __restrict__ st, int j) {
    const int done = st->done, limit = st->k_limit;
    return (done != 0) | (j >= limit);
}

// Sources of a row's stored entries: (column, value) of entry k.  CSR keeps both per entry;
// packed entries keep a code into a table of (column offset, value) pairs and, for the
// diagonal, the row's real diagonal (the sum runs over the same entries in the same order, so
// the products are bitwise those of the CSR they were packed from).
template <typename VT>
struct CsrSrc {
    const int* __restrict__ ci;
    const VT* __restrict__ val;
    using V = VT;
    __device__ __forceinline__ CsrSrc row(int, int) const { return *this; }
    __device__ __forceinline__ void load(int k, int& c, VT& v) const {
        c = ci[k];
        v = val[k];
    }
};

// Columns of value codes, stored sliced like the codes (entry q of row r at slice[r / 64] +
// 64 q + r % 64, so that the rows of a wave read consecutive addresses): kCols32 keeps every
// column, kCols16 a 16-bit offset per entry from a base per group (the entries q of one chunk
// of 64 rows: group slice[r / 64] / 64 + q).  kColsNone: codes of (column offset, value) pairs
// in CSR order.
enum { kColsNone = 0, kCols32 = 1, kCols16 = 2 };

template <typename CT, int COLS>
struct PackSrc {
    const CT* __restrict__ code;
    const int* __restrict__ cols;
    const uint16_t* __restrict__ cols16;
    const int* __restrict__ cbase;
    const int* __restrict__ slice;
    const int* __restrict__ toff;
    const double2* __restrict__ tval;
    const double* __restrict__ diag;
    int dcode;
    int r = 0;
    int at = 0;  // sliced: position of the row's first entry (entry k at at + 64 (k - kb))
    int kb = 0;
    int cb = 0;  // kCols16: the chunk's first group
    double dg = 0.0;
    using V = double2;
    __device__ __forceinline__ PackSrc row(int rr, int kb_) const {
        PackSrc p = *this;
        p.r = rr;
        p.dg = diag[rr];
        if constexpr (COLS != kColsNone) {
            const int s0 = slice[rr >> 6];
            p.at = s0 + (rr & 63);
            p.kb = kb_;
            if constexpr (COLS == kCols16) p.cb = s0 >> 6;
        }
        return p;
    }
    __device__ __forceinline__ void load(int k, int& c, double2& v) const {
        int q;
        if constexpr (COLS == kCols32) {
            const int i = at + 64 * (k - kb);
            q = code[i];
            c = cols[i];
        } else if constexpr (COLS == kCols16) {
            const int i = at + 64 * (k - kb);
            q = code[i];
            c = cbase[cb + (k - kb)] + (int)cols16[i];
        } else {
            q = code[k];
            c = r + toff[q];
        }
        const double2 t = tval[q];
        v = (q == dcode) ? make_double2(dg, 0.0) : t;
    }
};

// the entry source of packed entries with the given code array and (pair or value) table
template <typename CT, int COLS>
__device__ __forceinline__ PackSrc<CT, COLS> pack_src(const CT* code, const Packed& pk, const int* toff,
                                                      const double2* tval) {
    return PackSrc<CT, COLS>{code, pk.col, pk.col16, pk.cbase, pk.slice, toff, tval, pk.diag, pk.dcode};
}

// Calls f with the packed source of the given codes, by how the columns are kept.
template <typename CT, typename F>
__device__ __forceinline__ void with_packed(const CT* code, const Packed& pk, const int* toff, const double2* tval,
                                            F&& f) {
    if (pk.col16) f(pack_src<CT, kCols16>(code, pk, toff, tval));
    else if (pk.col) f(pack_src<CT, kCols32>(code, pk, toff, tval));
    else f(pack_src<CT, kColsNone>(code, pk, toff, tval));
}

// Calls f with the source of the matrix's storage kind.
template <typename F>
__device__ __forceinline__ void with_entries(const int* ci, const double2* val, const double* rval, const Packed& pk,
                                             F&& f) {
    if (pk.c8) with_packed(pk.c8, pk, pk.toff, pk.tval, f);
    else if (pk.c16) with_packed(pk.c16, pk, pk.toff, pk.tval, f);
    else if (rval) f(CsrSrc<double>{ci, rval});
    else f(CsrSrc<double2>{ci, val});
}

// y = H V[:, j] (raw) on rows [r0, r1): G lanes per row stream the stored entries, each with U
// entries in flight; results to y and, if ytile is given, to LDS.
template <int G, int U, typename Src>
__device__ __forceinline__ void tile_spmv_t(const int* __restrict__ rp, const Src& src,
                                            const double2* __restrict__ x,
                                            int r0, int r1, double2* __restrict__ y, double2* ytile) {
    using VT = typename Src::V;
    const int tid = threadIdx.x;
    const int lg = tid % G, grp = tid / G;
    for (int r = r0 + grp; r < r1; r += kBlock / G) {
        double2 acc = make_double2(0.0, 0.0);
        const int kb = rp[r], ke = rp[r + 1];
        const Src rs = src.row(r, kb);
        for (int k0 = kb + lg; k0 < ke; k0 += G * U) {
            VT vv[U];
            int cc[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int k = k0 + q * G;
                if (k < ke) {
                    rs.load(k, cc[q], vv[q]);
                } else {
                    vv[q] = entry_zero<VT>();
                    cc[q] = -1;
                }
            }
#pragma unroll
            for (int q = 0; q < U; ++q)
                if (cc[q] >= 0) acc = entry_fma(vv[q], x[cc[q]], acc);
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
            acc.x += __shfl_xor(acc.x, o);
            acc.y += __shfl_xor(acc.y, o);
        }
        if (lg == 0) {
            y[r] = acc;
            if (ytile) ytile[r - r0] = acc;
        }
    }
}

// One row per thread, 1-byte codes.  The U * H codes of a batch come from U * H / 4 + 1 aligned
// dword loads (the code array is padded so that the last batch's over-read stays inside it),
// byte-aligned with v_alignbyte; their gathers follow in H groups of U.  A row of up to U * H
// entries thus costs one round trip for its codes and the gathers behind it.  Entries past the
// row's end gather x[r] (in bounds, unused), so a group's gathers carry no branches.
template <int U, int H>
__device__ __forceinline__ void tile_spmv_p8_rows(const int* __restrict__ rp, const uint8_t* __restrict__ code,
                                                  const int* toff, const double2* tval,
                                                  const double* __restrict__ diag, int dcode,
                                                  const double2* __restrict__ x, int r0, int r1,
                                                  double2* __restrict__ y, double2* ytile) {
    constexpr int CB = U * H;
    static_assert(CB % 4 == 0, "batches of whole dwords");
    const uint32_t* __restrict__ words = reinterpret_cast<const uint32_t*>(code);
    for (int r = r0 + (int)threadIdx.x; r < r1; r += kBlock) {
        double2 acc = make_double2(0.0, 0.0);
        const int kb = rp[r], ke = rp[r + 1];
        const double dg = diag[r];
        for (int k0 = kb; k0 < ke; k0 += CB) {
            uint32_t w[CB / 4 + 1];
#pragma unroll
            for (int i = 0; i <= CB / 4; ++i) w[i] = words[(k0 >> 2) + i];
            uint32_t b[CB / 4];
#pragma unroll
            for (int i = 0; i < CB / 4; ++i) b[i] = __builtin_amdgcn_alignbyte(w[i + 1], w[i], (uint32_t)(k0 & 3));
#pragma unroll
            for (int h = 0; h < H; ++h) {
                double2 vv[U];
                int cc[U];
#pragma unroll
                for (int q = 0; q < U; ++q) {
                    const int e = h * U + q;
                    const int c8 = (int)((b[e >> 2] >> (8 * (e & 3))) & 0xffu);
                    const bool live = k0 + e < ke;
                    cc[q] = live ? r + toff[c8] : r;
                    const double2 t = tval[live ? c8 : dcode];
                    vv[q] = (c8 == dcode) ? make_double2(dg, 0.0) : t;
                }
                double2 xv[U];
#pragma unroll
                for (int q = 0; q < U; ++q) xv[q] = x[cc[q]];
#pragma unroll
                for (int q = 0; q < U; ++q)
                    if (k0 + h * U + q < ke) acc = entry_fma(vv[q], xv[q], acc);
            }
        }
        y[r] = acc;
        if (ytile) ytile[r - r0] = acc;
    }
}

// Whole block; false (and nothing computed) when the build is over at iteration j.  A table of
// 1-byte codes (at most 256 pairs) is staged in LDS first, while the state is tested.
template <int G, int U>
__device__ __forceinline__ bool tile_spmv(const int* __restrict__ rp, const int* __restrict__ ci,
                                          const double2* __restrict__ val, const double* __restrict__ rval,
                                          const Packed& pk, const double2* __restrict__ x, int r0, int r1,
                                          double2* __restrict__ y, double2* ytile, const DevState* __restrict__ st,
                                          int j) {
    if (pk.c8) {
        __shared__ int s_toff[256];
        __shared__ double2 s_tval[256];
        for (int i = threadIdx.x; i <= pk.dcode; i += kBlock) {
            s_toff[i] = pk.toff[i];
            s_tval[i] = pk.tval[i];
        }
        if (build_over(st, j)) return false;  // the same for every thread of the block
        __syncthreads();
        if (pk.col16)
            tile_spmv_t<G, U>(rp, pack_src<uint8_t, kCols16>(pk.c8, pk, s_toff, s_tval), x, r0, r1, y, ytile);
        else if (pk.col)
            tile_spmv_t<G, U>(rp, pack_src<uint8_t, kCols32>(pk.c8, pk, s_toff, s_tval), x, r0, r1, y, ytile);
        else if constexpr (G == 1 && U % 4 == 0)
            tile_spmv_p8_rows<U, 1>(rp, pk.c8, s_toff, s_tval, pk.diag, pk.dcode, x, r0, r1, y, ytile);
        else
            tile_spmv_t<G, U>(rp, pack_src<uint8_t, kColsNone>(pk.c8, pk, s_toff, s_tval), x, r0, r1, y, ytile);
        return true;
    }
    if (build_over(st, j)) return false;
    with_entries(ci, val, rval, pk, [&](const auto& src) { tile_spmv_t<G, U>(rp, src, x, r0, r1, y, ytile); });
    return true;
}

// Projection of iteration j on one tile.  FROM_Y: the sparse product already ran (k_yspmv)
// and y is read back; otherwise it is computed here and kept in LDS.
template <int RPT, int G, int U, bool FROM_Y>
__device__ __forceinline__ void project_body(const int* __restrict__ rp, const int* __restrict__ ci,
                                             const double2* __restrict__ val, const double* __restrict__ rval,
                                             const Packed& pk, const double2* __restrict__ V,
                                             int64_t ld, int dim, int j, double2* __restrict__ y,
                                             const DevState* __restrict__ st, const RedBuf& rb, int tile) {
    constexpr int R = kBlock * RPT;
    __shared__ double2 ytile[FROM_Y ? 1 : R];
    __shared__ double2 wpart[kWaves][kMaxVals];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r0 = tile * R;
    const int r1 = min(r0 + R, dim);
    const double2* __restrict__ x = V + (int64_t)j * ld;

    if (FROM_Y) {
        if (build_over(st, j)) return;
    } else {
        if (!tile_spmv<G, U>(rp, ci, val, rval, pk, x, r0, r1, y, ytile, st, j)) return;
        __syncthreads();
    }
    // Rows past the end of a ragged tile read row r1 - 1 and are weighted by zero, so the loads
    // of a batch carry no branches and are all issued before the first one is used.
    double2 yq[RPT], xq[RPT];
    int rr[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = r0 + tid + q * kBlock;
        rr[q] = min(r, r1 - 1);
        if (r < r1) {
            yq[q] = FROM_Y ? y[r] : ytile[r - r0];
            xq[q] = x[r];
        } else {
            yq[q] = make_double2(0.0, 0.0);
            xq[q] = make_double2(0.0, 0.0);
        }
    }
    // projections on columns i_lo..j (i_lo = j - 1 in three-term mode) in batches of CB: with
    // four rows per thread, batches of 4 keep the loads of a batch in flight without spilling
    // the occupancy below four waves per SIMD.  Columns past j in the last batch re-read
    // column j (cached); their sums are not stored.
    constexpr int CB = RPT >= 4 ? 4 : 8;
    const int i_lo = (st->p.three_term && j >= 1) ? j - 1 : 0;
    for (int i0 = i_lo; i0 <= j; i0 += CB) {
        double a[4 * CB];
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            double2 cy = make_double2(0.0, 0.0), cx = make_double2(0.0, 0.0);
            const double2* __restrict__ vi = V + (int64_t)min(i0 + b, j) * ld;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const double2 v = load_stream(vi + rr[q]);
                cy = cfma_conj(v, yq[q], cy);
                cx = cfma_conj(v, xq[q], cx);
            }
            a[4 * b] = cy.x;
            a[4 * b + 1] = cy.y;
            a[4 * b + 2] = cx.x;
            a[4 * b + 3] = cx.y;
        }
        double s;
        int v;  // 4 * column-in-batch + component
        if constexpr (CB == 8) {
            s = halving_reduce32(a, lane);
            v = halving_value(lane);
        } else {
            s = halving_reduce16(a, lane);
            v = halving_value16(lane);
        }
        if (lane < 4 * CB) {
            const int i = i0 + (v >> 2);
            if (i <= j) {
                double* dst = (double*)&wpart[wave][2 * i + ((v >> 1) & 1)];
                dst[v & 1] = s;
            }
        }
    }
    __syncthreads();
    const int nv = 2 * (j + 1);
    for (int v = 2 * i_lo + tid; v < nv; v += kBlock) {
        double2 s = make_double2(0.0, 0.0);
        for (int w = 0; w < kWaves; ++w) s = cadd(s, wpart[w][v]);
        rb.part[(size_t)v * rb.n_tiles + tile] = s;
    }
}

template <int RPT, int G, int U, bool FROM_Y>
__global__ __launch_bounds__(kBlock) void k_project(const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const double2* __restrict__ val, const double* __restrict__ rval,
                                                     Packed pk, const double2* __restrict__ V, int64_t ld, int dim,
                                                     int j, double2* __restrict__ y, const DevState* __restrict__ st,
                                                     RedBuf rb) {
    project_body<RPT, G, U, FROM_Y>(rp, ci, val, rval, pk, V, ld, dim, j, y, st, rb, blockIdx.x);
}

// sparse product alone (split projection): y = H V[:, j] on the rows of one projection tile
template <int RPT, int G, int U>
__global__ __launch_bounds__(kBlock) void k_yspmv(const int* __restrict__ rp, const int* __restrict__ ci,
                                                   const double2* __restrict__ val, const double* __restrict__ rval,
                                                   Packed pk, const double2* __restrict__ V, int64_t ld, int dim,
                                                   int j, double2* __restrict__ y, const DevState* __restrict__ st) {
    const int r0 = blockIdx.x * kBlock * RPT;
    tile_spmv<G, U>(rp, ci, val, rval, pk, V + (int64_t)j * ld, r0, min(r0 + kBlock * RPT, dim), y, nullptr, st, j);
}

// Batched projection.  Jobs that share H form a group; a group of one runs the fused kernel
// below (sparse product into LDS, then the projections), a larger group runs the multi-vector
// sparse product (tiles of kBlock rows), which streams each (column, value) pair of H once for
// every vector of the group, followed by the projections as a separate launch over (job, tile)
// items.  Both run the single-solve projection's own code per job (fused, or split with y read
// back), so a job's results do not depend on its group.

// live vectors of a group at iteration j (bit v: job gv.job[v] still builds its basis)
template <int NV>
__device__ __forceinline__ unsigned group_mask(const JobView* __restrict__ jobs, const GroupView& gv, int j,
                                               const double2* (&xs)[NV], double2* (&ys)[NV]) {
    unsigned mask = 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        xs[v] = nullptr;
        ys[v] = nullptr;
        if (v < gv.nv) {
            const JobView& J = jobs[gv.job[v]];
            const DevState* st = J.st;
            if (!st->done && j < st->k_limit) {
                mask |= 1u << v;
                xs[v] = J.V + (int64_t)j * J.ld;
                ys[v] = J.y;
            }
        }
    }
    return mask;
}

// y_v = H V_v[:, j] on rows [r0, r1) for every live vector: G lanes per row, U nonzeros in
// flight each; results to y_v and, if ytile is given, to LDS (NV = 1).
template <int G, int U, int NV, typename Src>
__device__ __forceinline__ void group_spmv(const GroupView& gv, const Src& src, int r0, int r1,
                                           unsigned mask, const double2* const (&xs)[NV],
                                           double2* const (&ys)[NV], double2* ytile) {
    using VT = typename Src::V;
    const int* __restrict__ rp = gv.rp;
    const int tid = threadIdx.x;
    const int lg = tid % G, grp = tid / G;
    for (int r = r0 + grp; r < r1; r += kBlock / G) {
        double2 acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = make_double2(0.0, 0.0);
        const int kb = rp[r], ke = rp[r + 1];
        const Src rs = src.row(r, kb);
        for (int k0 = kb + lg; k0 < ke; k0 += G * U) {
            VT vv[U];
            int cc[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int k = k0 + q * G;
                if (k < ke) {
                    rs.load(k, cc[q], vv[q]);
                } else {
                    vv[q] = entry_zero<VT>();
                    cc[q] = -1;
                }
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if (cc[q] < 0) continue;
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (mask & (1u << v)) acc[v] = entry_fma(vv[q], xs[v][cc[q]], acc[v]);
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
#pragma unroll
            for (int o = G / 2; o > 0; o >>= 1) {
                acc[v].x += __shfl_xor(acc[v].x, o);
                acc[v].y += __shfl_xor(acc[v].y, o);
            }
            if (lg == 0 && (mask & (1u << v))) {
                ys[v][r] = acc[v];
                if (ytile) ytile[r - r0] = acc[v];
            }
        }
    }
}

// fused projection of a group of one: one workgroup per (group, tile of kBlock * RPT rows)
template <int RPT, int G, int U>
__global__ __launch_bounds__(kBlock) void k_gproject(const JobView* __restrict__ jobs,
                                                      const GroupView* __restrict__ groups,
                                                      const int2* __restrict__ items, int j) {
    const int2 it = items[blockIdx.x];
    const JobView& J = jobs[groups[it.x].job[0]];
    project_body<RPT, G, U, false>(J.rp, J.ci, J.val, J.rval, J.pk, J.V, J.ld, J.dim, j, J.y, J.st, J.rb, it.y);
}

// multi-vector sparse product of a group: one workgroup per (group, tile)
template <int G, int U, int NV>
__global__ __launch_bounds__(kBlock) void k_gspmm(const JobView* __restrict__ jobs,
                                                   const GroupView* __restrict__ groups,
                                                   const int2* __restrict__ items, int j) {
    const int2 it = items[blockIdx.x];
    const GroupView& gv = groups[it.x];
    const double2* xs[NV];
    double2* ys[NV];
    const unsigned mask = group_mask<NV>(jobs, gv, j, xs, ys);
    if (mask == 0) return;
    const int r0 = it.y * kBlock;
    const int r1 = min(r0 + kBlock, gv.dim);
    const Packed& pk = gv.pk;
    if (pk.c8) {  // the 1-byte code table staged in LDS, as for the single-vector product
        __shared__ int s_toff[256];
        __shared__ double2 s_tval[256];
        for (int i = threadIdx.x; i <= pk.dcode; i += kBlock) {
            s_toff[i] = pk.toff[i];
            s_tval[i] = pk.tval[i];
        }
        __syncthreads();
        with_packed(pk.c8, pk, s_toff, s_tval,
                    [&](const auto& src) { group_spmv<G, U, NV>(gv, src, r0, r1, mask, xs, ys, nullptr); });
        return;
    }
    with_entries(gv.ci, gv.val, gv.rval, pk, [&](const auto& src) {
        group_spmv<G, U, NV>(gv, src, r0, r1, mask, xs, ys, nullptr);
    });
}

// projections after a multi-vector product: one workgroup per (job, tile of kBlock * RPT rows)
template <int RPT>
__global__ __launch_bounds__(kBlock) void k_bdots(const JobView* __restrict__ jobs, const int2* __restrict__ items,
                                                  int j) {
    const int2 it = items[blockIdx.x];
    const JobView& J = jobs[it.x];
    project_body<RPT, 4, 4, true>(J.rp, J.ci, J.val, J.rval, J.pk, J.V, J.ld, J.dim, j, J.y, J.st, J.rb, it.y);
}

// ---------------------------------------------------- fold of the projection partials
// Folds value v of iteration j over all tiles in a fixed order (whole block).
__device__ __forceinline__ void fold_value(const DevState* __restrict__ st, const RedBuf& rb, int j, int v) {
    __shared__ double lds[kWaves];
    if (build_over(st, j)) return;
    if (st->p.three_term && v < 2 * (j - 1)) return;  // columns the three-term recurrence skips
    double2 acc = make_double2(0.0, 0.0);
    for (int t = threadIdx.x; t < rb.n_tiles; t += kBlock) acc = cadd(acc, rb.part[(size_t)v * rb.n_tiles + t]);
    const double sx = block_sum(acc.x, lds);
    const double sy = block_sum(acc.y, lds);
    if (threadIdx.x == 0) rb.red[v] = make_double2(sx, sy);
}

__global__ __launch_bounds__(kBlock) void k_fold(const DevState* __restrict__ st, RedBuf rb, int j) {
    fold_value(st, rb, j, blockIdx.x);
}

// batched: grid (2(j+1), jobs)
__global__ __launch_bounds__(kBlock) void k_bfold(const JobView* __restrict__ jobs, int j) {
    const JobView& J = jobs[blockIdx.y];
    fold_value(J.st, J.rb, j, blockIdx.x);
}

// ----------------------------------------------------------------- update: new column
// Prologue (every block, identical arithmetic; block 0 also records the state):
//   ||V[:, j]|| = sqrt(g_j raw) is beta_{j-1} (or ||v0|| at the first projection) -> breakdown
//   test and s_j; c'_i = s_i s_j (V_i^H y)_raw, g_i = s_i s_j (V_i^H V_j)_raw;
//   c_i = c'_i - E_{i,j} c'_j - E_{i,j-1} c'_{j-1}, E = G - I, column j-1 of G from iteration j-1.
// Body: V[:, j+1] = s_j y - sum_i c_i s_i V[:, i]; the last residual only yields its norm.
template <int RPT>
__device__ __forceinline__ void update_body(double2* __restrict__ V, int64_t ld, int dim, int j,
                                            const double2* __restrict__ y, DevState* __restrict__ st,
                                            const RedBuf& rb, int tile) {
    __shared__ double lds[kWaves];
    __shared__ double2 cp[kMaxM + 1], g[kMaxM + 1], cs[kMaxM + 1];
    __shared__ double sj_sh;
    __shared__ int stop_sh;
    const int tid = threadIdx.x;
    const int r0 = tile * (kBlock * RPT);
    // this tile's rows of y, loaded while the prologue below waits on the state
    double2 yl[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = r0 + tid + q * kBlock;
        yl[q] = (r < dim) ? load_stream(y + r) : make_double2(0.0, 0.0);  // last reader of y
    }
    if (build_over(st, j)) return;
    const bool rec = tile == 0;
    if (tid == 0) {
        int stop = 0;
        double sj;
        if (j == 0) {
            sj = st->s[0];
            if (st->norm_init) {  // column 0 holds the raw v0
                const double n2 = rb.red[1].x;
                const double b0 = sqrt(n2);
                if (!isfinite(n2)) {
                    stop = 1;
                    if (rec) {
                        st->status = TE_ERR_NONFINITE;
                        st->done = 1;
                    }
                } else if (b0 == 0.0) {
                    stop = 1;
                    if (rec) st->done = 1;
                } else {
                    sj = 1.0 / b0;
                }
                if (rec) {  // norm_init itself is cleared by the step kernel: other blocks read it
                    st->beta0 = b0;
                    st->s[0] = sj;
                }
            }
        } else {
            const double b = sqrt(rb.red[2 * j + 1].x);  // ||V[:, j]|| = beta_{j-1}
            sj = 1.0 / b;
            if (rec) st->beta[j - 1] = b;
            if (!isfinite(b)) {
                stop = 1;
                if (rec) {
                    st->status = TE_ERR_NONFINITE;
                    st->done = 1;
                }
            } else if (b < st->p.tol_rate) {  // lucky breakdown (Alg. 1: no < tol_rate)
                stop = 1;
                if (rec) {
                    st->k_limit = j;
                    st->breakdown = 1;
                    st->h = b;
                }
            } else if (rec) {
                st->s[j] = sj;
            }
        }
        sj_sh = sj;
        stop_sh = stop;
    }
    __syncthreads();
    if (stop_sh) return;
    const double sj = sj_sh;
    const bool three = st->p.three_term != 0;
    const int i_lo = (three && j >= 1) ? j - 1 : 0;  // first column of this iteration
    if (tid >= i_lo && tid <= j) {
        const double si = (tid == j) ? sj : st->s[tid];
        const double sc = si * sj;
        cp[tid] = cscale(rb.red[2 * tid], sc);     // c'_i = v_i^H y
        g[tid] = cscale(rb.red[2 * tid + 1], sc);  // g_i  = v_i^H v_j
    }
    __syncthreads();
    if (tid >= i_lo && tid <= j) {
        double2 c;
        if (three) {
            // the recurrence as printed (eq. arnoldi, Lanczos form): w = H v_j - beta_{j-1} v_{j-1},
            // alpha_j = v_j^H w, w -= alpha_j v_j; beta_{j-1} = 1 / s_j
            const double bprev = (j >= 1) ? 1.0 / sj : 0.0;
            if (tid == j) c = (j >= 1) ? cfms(make_double2(bprev, 0.0), cconj(g[j - 1]), cp[j]) : cp[j];
            else c = make_double2(bprev, 0.0);
        } else {
            double2 e = g[tid];
            if (tid == j) e.x -= 1.0;
            c = cfms(e, cp[j], cp[tid]);
            if (j >= 1) {
                double2 f;
                if (tid < j) {
                    f = st->gcol[(j - 1) & 1][tid];
                    if (tid == j - 1) f.x -= 1.0;
                } else {
                    f = cconj(g[j - 1]);
                }
                c = cfms(f, cp[j - 1], c);
            }
        }
        const double si = (tid == j) ? sj : st->s[tid];
        cs[tid] = cscale(c, si);
        if (rec) {
            st->gcol[j & 1][tid] = g[tid];
            if (tid == j) {
                st->alpha[j] = c.x;
                if (!isfinite(c.x) || !isfinite(c.y)) {
                    st->status = TE_ERR_NONFINITE;
                    st->done = 1;
                }
            }
        }
    }
    __syncthreads();

    const bool last = (j + 1) == st->p.m;
    double2 p[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) p[q] = cscale(yl[q], sj);
    for (int i = i_lo; i <= j; ++i) {
        const double2 c = cs[i];
        const double2* __restrict__ vi = V + (int64_t)i * ld;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = r0 + tid + q * kBlock;
            if (r < dim) p[q] = cfms(c, load_stream(vi + r), p[q]);
        }
    }
    if (!last) {
        double2* __restrict__ vn = V + (int64_t)(j + 1) * ld;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = r0 + tid + q * kBlock;
            if (r < dim) vn[r] = p[q];
        }
    } else {  // the last residual is not stored; its norm is h of eq. errorIntegral
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            acc = fma(p[q].x, p[q].x, acc);
            acc = fma(p[q].y, p[q].y, acc);
        }
        const double s = block_sum(acc, lds);
        if (tid == 0) rb.npart[tile] = s;
    }
}

template <int RPT>
__global__ __launch_bounds__(kBlock) void k_update(double2* __restrict__ V, int64_t ld, int dim, int j,
                                                    const double2* __restrict__ y, DevState* __restrict__ st,
                                                    RedBuf rb) {
    update_body<RPT>(V, ld, dim, j, y, st, rb, blockIdx.x);
}

template <int RPT>
__global__ __launch_bounds__(kBlock) void k_bupdate(const JobView* __restrict__ jobs, const int2* __restrict__ items,
                                                     int j) {
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;
    const JobView& J = jobs[it.x];
    update_body<RPT>(J.V, J.ld, J.dim, j, J.y, J.st, J.rb, it.y);
}

__global__ __launch_bounds__(kBlock) void k_last_norm(DevState* st, RedBuf rb) {
    __shared__ double lds[kWaves];
    finish_last_norm(st, rb, lds);
}

// ------------------------------------------------------------- recombination w = V omega
template <int RPT>
__device__ __forceinline__ void combine_body(double2* __restrict__ V, int64_t ld, int dim,
                                             const DevState* __restrict__ st, int tile) {
    if (!st->do_combine) return;
    const int k = st->k_comb;
    const int r0 = tile * (kBlock * RPT);
    double2 w[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) w[q] = make_double2(0.0, 0.0);
    for (int i = 0; i < k; ++i) {
        const double2 c = st->omega[i];
        const double2* __restrict__ vi = V + (int64_t)i * ld;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = r0 + threadIdx.x + q * kBlock;
            if (r < dim) w[q] = cfma(c, load_stream(vi + r), w[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = r0 + threadIdx.x + q * kBlock;
        if (r < dim) V[r] = w[q];
    }
}

template <int RPT>
__global__ __launch_bounds__(kBlock) void k_combine(double2* __restrict__ V, int64_t ld, int dim,
                                                     const DevState* __restrict__ st) {
    combine_body<RPT>(V, ld, dim, st, blockIdx.x);
}

template <int RPT>
__global__ __launch_bounds__(kBlock) void k_bcombine(const JobView* __restrict__ jobs, const int2* __restrict__ items) {
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;
    const JobView& J = jobs[it.x];
    combine_body<RPT>(J.V, J.ld, J.dim, J.st, it.y);
}

// ------------------------------------------------------- batched setup, copy, output
__global__ void k_bsetup(const JobView* __restrict__ jobs, const Problem* __restrict__ probs, int n) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) setup_state(jobs[r].st, probs[r]);
}

// rows of one update tile (rpt rows per thread): V[:, 0] = v0 or out = beta0 s_0 V[:, 0]
__global__ __launch_bounds__(kBlock) void k_bcopy_in(const JobView* __restrict__ jobs, const int2* __restrict__ items,
                                                      int rpt) {
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;
    const JobView& J = jobs[it.x];
    for (int q = 0; q < rpt; ++q) {
        const int r = it.y * kBlock * rpt + q * kBlock + threadIdx.x;
        if (r < J.dim) J.V[r] = J.v0[r];
    }
}

__global__ __launch_bounds__(kBlock) void k_bcopy_out(const JobView* __restrict__ jobs, const int2* __restrict__ items,
                                                       int rpt) {
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;
    const JobView& J = jobs[it.x];
    const DevState* st = J.st;
    if (!st->done || st->counted) return;  // only jobs that completed in this round
    const double b = (st->beta0 == 0.0) ? 0.0 : st->beta0 * st->s[0];
    for (int q = 0; q < rpt; ++q) {
        const int r = it.y * kBlock * rpt + q * kBlock + threadIdx.x;
        if (r < J.dim) J.out[r] = cscale(J.V[r], b);
    }
}

// End of a batched round (one workgroup): write the round record of every job that has not
// yet reported its completion into bank (round & 1) of the host-mapped records, mark the jobs
// that completed in this round as reported, and advance the round counter.
__global__ __launch_bounds__(kBlock) void k_bflag(const JobView* __restrict__ jobs, int n, int* __restrict__ rounds,
                                                   SlotOut* __restrict__ slots, int max_slots,
                                                   RoundOut* __restrict__ ro) {
    __shared__ double lds[kWaves];
    const int round = *rounds + 1;
    SlotOut* bank = slots + (size_t)(round & 1) * max_slots;
    double live = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) {
        const JobView& J = jobs[i];
        DevState* st = J.st;
        if (st->counted) continue;
        SlotOut o;
        o.id = J.id;
        o.done = st->done;
        o.status = st->status;
        o.steps = st->steps;
        o.matvecs = st->matvecs;
        o.breakdown_dim = st->breakdown_dim;
        o.warnings = st->warnings;
        o.last_k = st->k_comb;
        o.round = round;
        o.beta0 = st->beta0;
        o.err_acc = st->err_acc;
        o.num_acc = st->num_acc;
        o.t_now = st->t_now;
        bank[J.slot] = o;
        if (st->done) st->counted = 1;
        else live += 1.0;
    }
    const double total = block_sum(live, lds);
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) {
        *rounds = round;
        __hip_atomic_store(&ro->active, (int)total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&ro->rounds, round, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
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
template <int G, typename Src>
__device__ __forceinline__ double2 spmv_rows(const int* __restrict__ rp, const Src& src,
                                             const double2* __restrict__ x, double2* __restrict__ y, int r0, int r1) {
    using VT = typename Src::V;
    const int tid = threadIdx.x, lg = tid % G, grp = tid / G;
    double2 dot = make_double2(0.0, 0.0);
    for (int r = r0 + grp; r < r1; r += kBlock / G) {
        double2 acc = make_double2(0.0, 0.0);
        const int kb = rp[r], ke = rp[r + 1];
        const Src rs = src.row(r, kb);
        for (int k = kb + lg; k < ke; k += G) {
            int c;
            VT v;
            rs.load(k, c, v);
            acc = entry_fma(v, x[c], acc);
        }
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
    return dot;
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_spmv(const int* __restrict__ rp, const int* __restrict__ ci,
                                                  const double2* __restrict__ val, const double* __restrict__ rval,
                                                  Packed pk, const double2* __restrict__ x,
                                                  double2* __restrict__ y, int dim, RedBuf rb, int rows_per_tile) {
    __shared__ double lds[kWaves];
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * rows_per_tile;
    const int r1 = min(r0 + rows_per_tile, dim);
    double2 dot = make_double2(0.0, 0.0);
    with_entries(ci, val, rval, pk, [&](const auto& src) { dot = spmv_rows<G>(rp, src, x, y, r0, r1); });
    const double sx = block_sum(dot.x, lds);
    const double sy = block_sum(dot.y, lds);
    if (tid == 0) rb.part[blockIdx.x] = make_double2(sx, sy);
}

// one block: sum of rb.part[0..n_tiles) into st->ceff[0]
__global__ __launch_bounds__(kBlock) void k_sum_part(DevState* st, RedBuf rb) {
    __shared__ double lds[kWaves];
    double2 acc = make_double2(0.0, 0.0);
    for (int t = threadIdx.x; t < rb.n_tiles; t += kBlock) acc = cadd(acc, rb.part[t]);
    const double sx = block_sum(acc.x, lds);
    const double sy = block_sum(acc.y, lds);
    if (threadIdx.x == 0) st->ceff[0] = make_double2(sx, sy);
}

// ------------------------------------------------------------------ CSR validation
// err bits: 1 structure, 2 column range, 4 non-finite, 8 unsorted (Hermitian check), 16 not Hermitian;
// bit 32 (not an error) marks a nonzero imaginary part
__device__ __forceinline__ double2 as_complex(double2 v) { return v; }
__device__ __forceinline__ double2 as_complex(double v) { return make_double2(v, 0.0); }

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_validate(const int* __restrict__ rp, const int* __restrict__ ci,
                                                      const VT* __restrict__ val, int dim, int64_t nnz,
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
        const double2 v = as_complex(val[k]);
        if (c < 0 || c >= dim) {
            e |= 2;
            continue;
        }
        if (!isfinite(v.x) || !isfinite(v.y)) e |= 4;
        if (v.y != 0.0) e |= 32;
        sum += hypot(v.x, v.y);
        if (check_herm) {
            if (k > kb && ci[k - 1] >= c) e |= 8;
            // binary search column r in row c (sorted columns required); clamp: row c's own
            // pointers may be invalid (reported by that row's thread)
            int lo = max(rp[c], 0), hi = (int)min((int64_t)rp[c + 1], nnz) - 1;
            bool found = false;
            double2 w = make_double2(0.0, 0.0);
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int cm = ci[mid];
                if (cm == r) {
                    found = true;
                    w = as_complex(val[mid]);
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

__global__ __launch_bounds__(kBlock) void k_expand_real(const double* __restrict__ rval, double2* __restrict__ val,
                                                         int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock)
        val[k] = make_double2(rval[k], 0.0);
}

// one thread per row: columns and values of the row's packed entries
__global__ __launch_bounds__(kBlock) void k_expand_packed(const int* __restrict__ rp, Packed pk, int dim,
                                                          int* __restrict__ col, double2* __restrict__ val) {
    for (int r = blockIdx.x * kBlock + threadIdx.x; r < dim; r += gridDim.x * kBlock)
        with_entries(nullptr, nullptr, nullptr, pk, [&](const auto& src) {
            const int kb = rp[r], ke = rp[r + 1];
            const auto rs = src.row(r, kb);
            for (int k = kb; k < ke; ++k) {
                typename std::decay_t<decltype(src)>::V v;
                rs.load(k, col[k], v);
                val[k] = as_complex(v);
            }
        });
}

__global__ __launch_bounds__(kBlock) void k_real_part(const double2* __restrict__ val, double* __restrict__ rval,
                                                       int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock)
        rval[k] = val[k].x;
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
    if (rpt == 1) f(std::integral_constant<int, 1>{});
    else f(std::integral_constant<int, 2>{});
    return hipGetLastError();
}

// the projections also come with four rows per thread
template <typename F>
static hipError_t by_rpt_p(int rpt, F&& f) {
    if (rpt == 1) f(std::integral_constant<int, 1>{});
    else if (rpt == 2) f(std::integral_constant<int, 2>{});
    else f(std::integral_constant<int, 4>{});
    return hipGetLastError();
}

// Launch with optional timing events bound to the dispatch (hipExtLaunchKernelGGL records the
// kernel's own start/end, no marker packet of its own in the queue).
template <typename... KArgs, typename... Args>
static void launch_timed(void (*kernel)(KArgs...), dim3 grid, hipStream_t s, hipEvent_t start, hipEvent_t done,
                         Args... args) {
    if (start || done) hipExtLaunchKernelGGL(kernel, grid, dim3(kBlock), 0, s, start, done, 0, args...);
    else hipLaunchKernelGGL(kernel, grid, dim3(kBlock), 0, s, args...);
}

static int grid_for(int dim) { return (int)std::min<int64_t>(((int64_t)dim + kBlock - 1) / kBlock, 4096); }

// ----------------------------------------------------------------- batched launchers
bool gproject_supported(int g, int u) { return (g == 4 && (u == 1 || u == 4)) || (g == 8 && u == 2) || (g == 1 && u == 8); }

template <int RPT, int G, int U>
static void gproject_nv(int nv_class, dim3 grid, hipStream_t s, const JobView* jobs, const GroupView* groups,
                        const int2* items, int j) {
    switch (nv_class) {
        case 1: k_gproject<RPT, G, U><<<grid, kBlock, 0, s>>>(jobs, groups, items, j); break;
        case 2: k_gspmm<G, U, 2><<<grid, kBlock, 0, s>>>(jobs, groups, items, j); break;
        case 4: k_gspmm<G, U, 4><<<grid, kBlock, 0, s>>>(jobs, groups, items, j); break;
        default: k_gspmm<G, U, 8><<<grid, kBlock, 0, s>>>(jobs, groups, items, j); break;
    }
}

// nv_class 1: fused product + projections (tiles of kBlock * rpt rows); 2, 4, 8: the
// multi-vector product only (tiles of kBlock rows; the projections follow with launch_bdots)
hipError_t launch_gproject(int g, int u, int rpt, int nv_class, const JobView* jobs, const GroupView* groups,
                           const int2* items, int n_items, int j, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    const dim3 grid(n_items);
    return by_rpt_p(rpt, [&](auto r) {
        constexpr int RPT = decltype(r)::value;
        if (g == 8) gproject_nv<RPT, 8, 2>(nv_class, grid, s, jobs, groups, items, j);
        else if (g == 1) gproject_nv<RPT, 1, 8>(nv_class, grid, s, jobs, groups, items, j);
        else if (u == 1) gproject_nv<RPT, 4, 1>(nv_class, grid, s, jobs, groups, items, j);
        else gproject_nv<RPT, 4, 4>(nv_class, grid, s, jobs, groups, items, j);
    });
}

hipError_t launch_bdots(int rpt, const JobView* jobs, const int2* items, int n_items, int j, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    return by_rpt_p(rpt, [&](auto r) { k_bdots<decltype(r)::value><<<n_items, kBlock, 0, s>>>(jobs, items, j); });
}

hipError_t launch_bfold(const JobView* jobs, int n_jobs, int j, hipStream_t s) {
    if (n_jobs <= 0) return hipSuccess;
    k_bfold<<<dim3(2 * (j + 1), n_jobs), kBlock, 0, s>>>(jobs, j);
    return hipGetLastError();
}

hipError_t launch_bupdate(int rpt, const JobView* jobs, const int2* items, int n_items, int j, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    return by_rpt(rpt, [&](auto r) { k_bupdate<decltype(r)::value><<<n_items, kBlock, 0, s>>>(jobs, items, j); });
}

hipError_t launch_bcombine(int rpt, const JobView* jobs, const int2* items, int n_items, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    return by_rpt(rpt, [&](auto r) { k_bcombine<decltype(r)::value><<<n_items, kBlock, 0, s>>>(jobs, items); });
}

hipError_t launch_bsetup(const JobView* jobs, const Problem* probs, int n_jobs, hipStream_t s) {
    if (n_jobs <= 0) return hipSuccess;
    k_bsetup<<<(n_jobs + 63) / 64, 64, 0, s>>>(jobs, probs, n_jobs);
    return hipGetLastError();
}

hipError_t launch_bcopy_in(int rpt, const JobView* jobs, const int2* items, int n_items, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_bcopy_in<<<n_items, kBlock, 0, s>>>(jobs, items, rpt);
    return hipGetLastError();
}

hipError_t launch_bcopy_out(int rpt, const JobView* jobs, const int2* items, int n_items, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_bcopy_out<<<n_items, kBlock, 0, s>>>(jobs, items, rpt);
    return hipGetLastError();
}

hipError_t launch_bflag(const JobView* jobs, int n_jobs, int* rounds_dev, SlotOut* slots, int max_slots,
                        RoundOut* ro, hipStream_t s) {
    k_bflag<<<1, kBlock, 0, s>>>(jobs, n_jobs, rounds_dev, slots, max_slots, ro);
    return hipGetLastError();
}

hipError_t launch_setup(DevState* st, const Problem& prob, hipStream_t s) {
    k_setup<<<1, 64, 0, s>>>(st, prob);
    return hipGetLastError();
}

hipError_t launch_copy(const double2* src, double2* dst, int dim, hipStream_t s) {
    k_copy<<<grid_for(dim), kBlock, 0, s>>>(src, dst, dim);
    return hipGetLastError();
}

// Calls f with the (lanes per row, nonzeros per lane) of a supported sparse-product shape.
template <typename F>
void by_spmv_shape(int g, int u, F&& f) {
    using std::integral_constant;
    if (g == 8) f(integral_constant<int, 8>{}, integral_constant<int, 2>{});
    else if (g == 2) f(integral_constant<int, 2>{}, integral_constant<int, 8>{});
    else if (g == 1 && u == 16) f(integral_constant<int, 1>{}, integral_constant<int, 16>{});
    else if (g == 1) f(integral_constant<int, 1>{}, integral_constant<int, 8>{});
    else if (u == 1) f(integral_constant<int, 4>{}, integral_constant<int, 1>{});
    else f(integral_constant<int, 4>{}, integral_constant<int, 4>{});
}

hipError_t launch_project(const Tiling& tl, const Csr& H, const double2* V, int64_t ld, int j, double2* y,
                          const DevState* st, const RedBuf& rb, hipStream_t s, hipEvent_t start, hipEvent_t done) {
    return by_rpt_p(tl.rpt_p, [&](auto r) {
        constexpr int RPT = decltype(r)::value;
        const dim3 grid(tl.n_tiles_p);
        by_spmv_shape(tl.g, tl.u, [&](auto g, auto u) {
            constexpr int G = decltype(g)::value, U = decltype(u)::value;
            if (tl.split) {  // the sparse product keeps one row per thread; rpt_p shapes the projections
                const dim3 g1((H.dim + kBlock - 1) / kBlock);
                launch_timed(k_yspmv<1, G, U>, g1, s, start, nullptr, H.row_ptr, H.col, H.val, H.rval, H.pk, V, ld,
                             H.dim, j, y, st);
                launch_timed(k_project<RPT, 4, 4, true>, grid, s, nullptr, done, H.row_ptr, H.col, H.val, H.rval, H.pk,
                             V, ld, H.dim, j, y, st, rb);
            } else {
                launch_timed(k_project<RPT, G, U, false>, grid, s, start, done, H.row_ptr, H.col, H.val, H.rval, H.pk,
                             V, ld, H.dim, j, y, st, rb);
            }
        });
    });
}

hipError_t launch_fold(int j, const DevState* st, const RedBuf& rb, hipStream_t s, hipEvent_t done) {
    launch_timed(k_fold, dim3(2 * (j + 1)), s, nullptr, done, st, rb, j);
    return hipGetLastError();
}

hipError_t launch_update(const Tiling& tl, double2* V, int64_t ld, int dim, int j, const double2* y,
                         DevState* st, const RedBuf& rb, hipStream_t s, hipEvent_t done) {
    return by_rpt(tl.rpt_u, [&](auto r) {
        launch_timed(k_update<decltype(r)::value>, dim3(tl.n_tiles_u), s, nullptr, done, V, ld, dim, j, y, st, rb);
    });
}

hipError_t launch_last_norm(DevState* st, const RedBuf& rb, hipStream_t s) {
    k_last_norm<<<1, kBlock, 0, s>>>(st, rb);
    return hipGetLastError();
}

hipError_t launch_combine(const Tiling& tl, double2* V, int64_t ld, int dim, const DevState* st, hipStream_t s,
                          hipEvent_t done) {
    return by_rpt(tl.rpt_u, [&](auto r) {
        launch_timed(k_combine<decltype(r)::value>, dim3(tl.n_tiles_u), s, nullptr, done, V, ld, dim, st);
    });
}

hipError_t launch_output(const double2* V, double2* out, int dim, const DevState* st, hipStream_t s) {
    k_output<<<grid_for(dim), kBlock, 0, s>>>(V, out, dim, st);
    return hipGetLastError();
}

hipError_t launch_scale_columns(const double2* src, double2* dst, int64_t ld, int dim, int k, const DevState* st,
                                hipStream_t s) {
    const int bx = (int)std::min<int64_t>(((int64_t)dim + kBlock - 1) / kBlock, 1024);
    k_scale_columns<<<dim3(bx, std::max(1, std::min(k, 64))), kBlock, 0, s>>>(src, dst, ld, dim, k, st);
    return hipGetLastError();
}

hipError_t launch_spmv_only(const Tiling& tl, const Csr& H, const double2* x, double2* y, DevState* st,
                            const RedBuf& rb, hipStream_t s) {
    k_spmv<4><<<tl.n_tiles_p, kBlock, 0, s>>>(H.row_ptr, H.col, H.val, H.rval, H.pk, x, y, H.dim, rb, kBlock * tl.rpt_p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sum_part<<<1, kBlock, 0, s>>>(st, rb);
    return hipGetLastError();
}

hipError_t launch_validate(const Csr& H, int check_hermitian, int* err, double* rowsum, hipStream_t s) {
    const int blocks = (H.dim + kBlock - 1) / kBlock;
    if (H.rval) k_validate<double><<<blocks, kBlock, 0, s>>>(H.row_ptr, H.col, H.rval, H.dim, H.nnz, check_hermitian, err, rowsum);
    else k_validate<double2><<<blocks, kBlock, 0, s>>>(H.row_ptr, H.col, H.val, H.dim, H.nnz, check_hermitian, err, rowsum);
    return hipGetLastError();
}

hipError_t launch_real_part(const double2* val, double* rval, int64_t n, hipStream_t s) {
    const int blocks = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 8192);
    k_real_part<<<blocks, kBlock, 0, s>>>(val, rval, n);
    return hipGetLastError();
}

hipError_t launch_expand_real(const double* rval, double2* val, int64_t n, hipStream_t s) {
    const int blocks = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 8192);
    k_expand_real<<<blocks, kBlock, 0, s>>>(rval, val, n);
    return hipGetLastError();
}

hipError_t launch_expand_packed(const int* row_ptr, const Packed& pk, int dim, int* col, double2* val, hipStream_t s) {
    const int blocks = (int)std::min<int64_t>(((int64_t)dim + kBlock - 1) / kBlock, 8192);
    k_expand_packed<<<blocks, kBlock, 0, s>>>(row_ptr, pk, dim, col, val);
    return hipGetLastError();
}

hipError_t launch_norm1(const double* rowsum, int dim, double* out, hipStream_t s) {
    k_max<<<1, kBlock, 0, s>>>(rowsum, dim, out);
    return hipGetLastError();
}

}  // namespace te
