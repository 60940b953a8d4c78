/*
 * te.h - C ABI of libtimeevolve: restarted Krylov evolution v(t) = exp(-iHt) v0 on one
 * AMD Instinct MI355X (gfx950), with the a-posteriori error bound of
 * M. Michel & S. Zell, "TimeEvolver: A Program for Time Evolution With Improved
 * Error Bound", Comput. Phys. Commun. (2022).
 *
 * Problem statement (paper, Sec. "Time Evolution in a Generic Physical Quantum System",
 * eq. vOfT; Alg. 1 input/output): given a Hermitian sparse d x d matrix H, a complex
 * vector v0, a time t and a maximal error err_max, return an approximation of
 * exp(-iHt) v0 whose 2-norm error is bounded by the integral of eq. errorIntegral,
 * summed over restarts, up to roundoff (eq. numericalError).
 *
 * Conventions for every call
 *  - Complex numbers are interleaved (re, im) doubles, i.e. te_c128 has the layout of
 *    std::complex<double>, hipDoubleComplex and torch.complex128.
 *  - "device" pointers are HIP device pointers on the current device; "host" pointers are
 *    ordinary host memory.  Ownership never transfers unless stated.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued on it; calls
 *    documented as synchronous return only after that work completed.
 *  - Every call returns a te_status; on failure te_last_error() gives a thread-local
 *    message and output buffers are left unspecified.  Calls never abort the process.
 *  - All arithmetic is FP64 / complex FP64; indices are int32.
 */
#ifndef TE_H
#define TE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct te_hamiltonian_s* te_hamiltonian; /* opaque; owns a device copy of the CSR */
typedef struct {
    double re, im;
} te_c128;
typedef int32_t te_status;

enum {
    TE_OK = 0,
    TE_ERR_INVALID_ARG = 1,    /* null pointer, t<0, tol<=0, non-finite scalars, m<2, ... */
    TE_ERR_INVALID_CSR = 2,    /* row_ptr not monotone / not 0..nnz, column out of range,
                                  non-finite value, nnz >= 2^31 */
    TE_ERR_NOT_HERMITIAN = 3,  /* only with TE_CHECK_HERMITIAN */
    TE_ERR_UNSUPPORTED = 4,    /* m > TE_MAX_KRYLOV */
    TE_ERR_OUT_OF_MEMORY = 5,
    TE_ERR_DEVICE = 6,         /* a HIP runtime error; te_last_error() holds its text */
    TE_ERR_STEP_UNDERFLOW = 7, /* the step search halved max_halvings times without success */
    TE_ERR_NONFINITE = 8,      /* NaN/Inf met in v0 or during the iteration */
    TE_ERR_CAPACITY = 9,       /* batch / engine capacity or memory budget exceeded */
    TE_ERR_TIMEOUT = 10        /* te_engine_wait: the jobs waited for are not done yet */
};

/* warning bits of te_result.warnings (they never change the status) */
#define TE_WARN_NUMERICAL 1u  /* accumulated roundoff estimate d*||H||_1*eps exceeds the
                                 accumulated analytic bound (Sec. "Pseudocode", third remark) */
#define TE_WARN_QUADRATURE 2u /* an error integral did not meet its stopping test within
                                 quad_max_level refinements (Sec. "Description of Program") */

/* flags of te_hamiltonian_create */
#define TE_PTR_DEVICE 1u      /* row_ptr/col_idx/values are device pointers (else host) */
#define TE_CHECK_HERMITIAN 2u /* verify H == H^H on the device (needs sorted columns) */
#define TE_STORE_COMPLEX 4u   /* keep 16-byte complex entries even when all are real */
#define TE_STORE_CSR 8u       /* keep column indices and values per entry (no packing) */

#define TE_MAX_KRYLOV 64 /* largest Krylov dimension m: a row of the small eigenproblem is held
                            by one 64-lane wavefront */

/* Tunable constants of the step-size search (Alg. 1 step 2).  te_default_options()
 * fills: n_substeps=10, t_init=0.1, shrink=0.97, quad_rel_tol=1e-3, quad_max_level=15,
 * quad_min_level=3, max_halvings=64, flags=0, quad_gauss_points=0. */
typedef struct {
    int32_t n_substeps;     /* N_SUBSTEPS of Alg. 1 */
    double t_init;          /* first step-size guess (Alg. 1 line 1) */
    double shrink;          /* later restarts start from shrink * previous step */
    double quad_rel_tol;    /* relative stopping test of the error integral */
    int32_t quad_max_level; /* refinements before TE_WARN_QUADRATURE */
    int32_t quad_min_level; /* refinements always taken */
    int32_t max_halvings;   /* cap of the halving loop (TE_ERR_STEP_UNDERFLOW) */
    uint32_t flags;         /* TE_OPT_* bits (below); other bits must be 0 */
    int32_t quad_gauss_points; /* 0: adaptive tanh-sinh (rigorous to its tolerance); 1..64: the
                                  paper's fast option (Sec. "Description of Program"), an
                                  n-point Gauss-Legendre rule per integral with no error
                                  estimate, so the reported bound is approximate */
} te_options;

typedef struct {
    int32_t steps;           /* restarts taken */
    int32_t matvecs;         /* products H*x */
    int32_t breakdown_dim;   /* Krylov dimension at a lucky breakdown, else 0 */
    uint32_t warnings;       /* TE_WARN_* bits */
    double err_bound;        /* ||v0|| * sum of per-step integrals of eq. errorIntegral */
    double num_err_estimate; /* ||v0|| * accumulated d*||H||_1*2^-52 (eq. numericalError) */
    double t_reached;        /* == t on success */
} te_result;

/* te_options.flags bit: time every kernel of te_evolve with HIP events on the caller's
 * stream (restarts are then launched directly instead of as a graph; the events are bound to
 * the kernel dispatches, so the timed solve runs at the graph's speed) and record the
 * per-kernel durations and algorithmic bytes, read back with te_last_profile().  A class's
 * duration runs from the end of the kernel before it to its own end. */
#define TE_OPT_PROFILE 1u

/* te_options.flags bit: build each Krylov basis with the three-term recurrence exactly as
 * printed (eq. arnoldi / Alg. 1, step 1: subtract beta_{j-1} v_{j-1}, project on v_j, subtract)
 * and no re-orthogonalisation against older vectors.  Moves 2 instead of j + 1 basis columns
 * per pass (about 3x fewer bytes at m = 40).  The bound of eq. errorIntegral rests on the
 * Arnoldi relation and a unit residual vector, which the recurrence keeps to rounding error,
 * not on orthogonality; the basis loses orthogonality as j grows, so results differ from the
 * default mode by up to the two bounds.  Also accepted by te_engine_config.opt. */
#define TE_OPT_LANCZOS3 2u

/* Kernel classes of one restart, in te_profile order. */
enum {
    TE_KERNEL_PROJECT = 0, /* sparse product fused with all projections and the Gram column */
    TE_KERNEL_UPDATE = 1,  /* new basis vector and its norm */
    TE_KERNEL_STEP = 2,    /* eigensolve, error integrals, step search, restart control */
    TE_KERNEL_COMBINE = 3, /* recombination w = V omega */
    TE_KERNEL_FOLD = 4,    /* fold of the projection partials + Gram correction (small) */
    TE_KERNEL_CLASSES = 5
};

/* Per-kernel-class totals of the last profiled te_evolve on a handle.  bytes are the
 * algorithmic bytes of each launch (one read of every operand and one write of every
 * result it must touch); launches after a lucky breakdown that do no work are excluded. */
typedef struct {
    int64_t launches[TE_KERNEL_CLASSES];
    double seconds[TE_KERNEL_CLASSES];
    double bytes[TE_KERNEL_CLASSES];
} te_profile;

void te_default_options(te_options* opt);
const char* te_status_string(te_status s);
const char* te_last_error(void);

/* ---------------------------------------------------------------------------------------
 * Hamiltonian handle (paper: the Hermitian matrix H handed to the evolver, Sec.
 * "Description of Program"; CSR is the sparse format of the problem statement).
 *   dim, nnz     : matrix size and stored entries; 1 <= dim, 0 < nnz < 2^31.
 *   row_ptr      : int32[dim+1], row_ptr[0] = 0, non-decreasing, row_ptr[dim] = nnz.
 *   col_idx      : int32[nnz], 0 <= col < dim (sorted per row if TE_CHECK_HERMITIAN).
 *   values       : te_c128[nnz], finite.
 * The arrays are copied; the caller keeps ownership.  Validation runs on the device and
 * returns TE_ERR_INVALID_CSR / TE_ERR_NOT_HERMITIAN.  Synchronous.  The 1-norm
 * max_i sum_j |H_ij| (equal to the column-sum norm for Hermitian H) is computed here.
 * When every imaginary part is exactly zero (real symmetric H, as for the spin and boson
 * models of the paper's examples) the device copy keeps only the real parts, 8 bytes per
 * entry instead of 16: the sparse products then stream 12 instead of 20 bytes per entry and
 * give the same values (a zero imaginary part adds exact zeros).  TE_STORE_COMPLEX keeps
 * the complex copy regardless.
 * Packing: the Hamiltonians of lattice models are sums of a few local terms, so their entries
 * off the diagonal take few distinct (column - row, value) pairs (the XXZ ring: 2 per bond).
 * When there are at most 65535 such pairs, every diagonal entry is real (imaginary part +0)
 * and no row stores its diagonal twice, the device copy keeps per entry only a 1-byte (at most
 * 255 pairs) or 2-byte code into a table of the pairs, plus the real diagonal per row, and
 * drops the column indices and values: a sparse product then streams 1 or 2 bytes per entry
 * and 8 per row instead of 20 (or 12) per entry, and gives bitwise the values of the CSR it
 * was packed from (same entries, same order).  With more pairs but at most 65535 distinct
 * values off the diagonal (the paper's model: its couplings), the columns stay and the codes
 * index the values ("value codes": 5 or 6 bytes per entry).  The test is one host pass over
 * the entries (read back from the device in chunks).  TE_STORE_CSR keeps the CSR regardless. */
te_status te_hamiltonian_create(te_hamiltonian* out, int64_t dim, int64_t nnz,
                                const int32_t* row_ptr, const int32_t* col_idx,
                                const te_c128* values, uint32_t flags, void* stream);

/* *real_values = 1 when the handle stores real entries (see te_hamiltonian_create), else 0. */
te_status te_hamiltonian_real_values(te_hamiltonian h, int32_t* real_values);

/* Storage of the handle's entries (see te_hamiltonian_create). */
enum {
    TE_STORAGE_COMPLEX = 0,   /* column + complex value per entry (20 bytes) */
    TE_STORAGE_REAL = 1,      /* column + real value per entry (12 bytes) */
    TE_STORAGE_PACKED8 = 2,   /* 1-byte code per entry + real diagonal per row */
    TE_STORAGE_PACKED16 = 3,  /* 2-byte code per entry + real diagonal per row */
    TE_STORAGE_CODED8 = 4,    /* column + 1-byte value code per entry + real diagonal per row */
    TE_STORAGE_CODED16 = 5    /* column + 2-byte value code per entry + real diagonal per row */
};
te_status te_hamiltonian_storage(te_hamiltonian h, int32_t* kind);

/* Packs the entries of a handle held as CSR (one built on the device, or created with
 * TE_STORE_CSR) as te_hamiltonian_create would; a no-op for a packed handle or a matrix that
 * does not pack.  *kind (may be NULL) receives the storage afterwards.  The handle's kernel
 * shape is tuned again on its next use.  Not while the handle is in use by a solve, a batch or
 * an engine.  Synchronous on `stream`. */
te_status te_hamiltonian_pack(te_hamiltonian h, int32_t* kind, void* stream);

/* Copies the handle's CSR out: row_ptr[dim+1], col_idx[nnz], values[nnz] (complex; real
 * entries are returned with zero imaginary parts; packed entries are expanded back, bit for
 * bit, in their stored order; the expansion takes nnz * 20 bytes of device scratch).  Device pointers with TE_PTR_DEVICE, else
 * host.  Any of the three may be NULL (not copied).  Synchronous. */
te_status te_hamiltonian_copy_csr(te_hamiltonian h, int32_t* row_ptr, int32_t* col_idx, te_c128* values,
                                  uint32_t flags, void* stream);

/* ---------------------------------------------------------------------------------------
 * The paper's exemplary Hamiltonian built on the device (Sec. "Exemplary System", eq.
 * fullHamiltonianSimple with the conserved totals of eq. subsetOccupations): modes a_0, b_0
 * with N_0 = n_0 + m_0 bosons and K + K' memory qubits a_1..a_K, a'_1..a'_K' with N_m
 * excitations,
 *   H = C_0 (a_0^+ b_0 + h.c.) + eps_m (1 - n_0/N_c) sum_k n_k + eps_m (1 - n_0/(N_c - dN_c)) sum_k' n'_k'
 *     + C_m [ sum_{k,k'} f_1(k,k') (a_k^+ a'_k' + h.c.) + sum_{k<l} f_2(k,l) (a_k^+ a_l + h.c.)
 *             + sum_{k'<l'} f_3(k',l') (a'_k'^+ a'_l' + h.c.) ],
 * f_i = F_i - 1 if F_i < 1/2 else F_i, F_i(k,l) = (sqrt(2) (k + dk_i)^3 + sqrt(7) (l + dl_i)^5) mod 1,
 * dk_1 = dk_2 = 1, dk_3 = K + 1, dl_1 = dl_3 = K + 1, dl_2 = 1 (the f_i are evaluated on the
 * host; every matrix entry on the device).  Basis: row = (N_0 - n_0) binom(K+K', N_m) + rank
 * of the qubit configuration, both sectors in descending lexicographic order of the occupation
 * tuples (modes ordered a_1..a_K, a'_1..a'_K').  The matrix is real: the handle stores 8-byte
 * entries.  Matrix creation is the memory limit of the paper's CPU program (Sec. "Analysis of
 * Performance"); here no basis, lookup table or triplet list exists on the host. */
typedef struct {
    int32_t K, Kp;  /* memory qubits a_k and a'_k' (K >= 1, K + K' <= 63) */
    int32_t N0;     /* bosons in a_0, b_0 (>= 0) */
    int32_t Nm;     /* memory excitations, 0 <= N_m <= K */
    double eps_m;   /* memory-mode energy */
    double Nc;      /* critical occupation N_c */
    double dNc;     /* 0 < dN_c < N_c */
    double C0, Cm;  /* couplings */
} te_memory_burden;

/* The paper's parameters of its Fig. 1 system: K = K' = 4, N_0 = 20, N_m = 2, eps_m = sqrt(20),
 * N_c = 20, dN_c = 12, C_0 = C_m = 1. */
void te_memory_burden_defaults(te_memory_burden* p);

/* Builds the matrix in device memory and returns its handle; *initial_index (may be NULL)
 * receives the basis index of the initial state of eq. initialStateSimple
 * (n_0 = N_0, a_1..a_{N_m} occupied).  TE_ERR_INVALID_ARG for parameters out of range,
 * TE_ERR_UNSUPPORTED when dim exceeds 2^26, nnz does not fit int32 or a row exceeds 512
 * entries.  Synchronous. */
te_status te_hamiltonian_create_memory_burden(te_hamiltonian* out, const te_memory_burden* p,
                                              int64_t* initial_index, void* stream);

/* ---------------------------------------------------------------------------------------
 * Open Bose chain of K modes with N bosons built on the device, in the number-state basis of
 * Sec. "Creation of Hamiltonian Matrix" (eqs. basisState, totalOccupationNumber):
 *   H = sum_{k<K-1} ( hop[k] b_k^+ b_{k+1} + conj(hop[k]) b_{k+1}^+ b_k ) + sum_k U[k] n_k (n_k - 1).
 * Basis: all (n_0..n_{K-1}) with sum N in descending lexicographic order, index 0 =
 * (N, 0, ..., 0).  The index of a state and its inverse (eq. findIndices) are closed forms of
 * the combinatorial number system; no basis, lookup table or triplet list is built.  Every row
 * stores its diagonal (also when zero) and its hops, columns ascending.
 *   K    : 1..64 modes;  N : 0..65535 bosons;  dim = binom(N + K - 1, K - 1) <= 2^26.
 *   U    : host double[K], finite.
 *   hop  : host te_c128[K - 1], finite (may be NULL when K == 1).
 *   flags: 0 or TE_STORE_COMPLEX (as for te_hamiltonian_create: without it a matrix whose
 *          hops are all real keeps 8-byte entries).
 * TE_ERR_INVALID_ARG for arguments out of range, TE_ERR_UNSUPPORTED when dim exceeds 2^26 or
 * nnz does not fit int32.  Synchronous on `stream`. */
te_status te_hamiltonian_create_bose_chain(te_hamiltonian* out, int32_t K, int32_t N, const double* U,
                                          const te_c128* hop, uint32_t flags, void* stream);
te_status te_hamiltonian_destroy(te_hamiltonian h); /* frees everything the handle owns */
te_status te_hamiltonian_info(te_hamiltonian h, int64_t* dim, int64_t* nnz, double* norm1);

/* Device bytes of the workspace that te_evolve keeps inside handle h for Krylov dimension m
 * (Krylov basis min(m, dim)*dim complex, one work vector, reduction partials, device state):
 * what admission control has to reserve besides the handle's own matrix.  0 for a null
 * handle or m outside 1..TE_MAX_KRYLOV.  Host only. */
size_t te_workspace_bytes(te_hamiltonian h, int32_t m);

/* Optional allocator hook for the device memory the library allocates (handle copies of the
 * matrix, workspaces, engine pools and plans; not te_evolve_noalloc, which allocates nothing).
 *   alloc(bytes, stream, ctx): returns device memory of at least bytes (NULL on failure);
 *       stream is the hipStream_t the memory is first used on (NULL = default stream).
 *   free_(ptr, stream, ctx): returns a block; called after the device has finished with it
 *       (the library waits for the device first, as hipFree would), with the stream and ctx
 *       the block was allocated with.
 * Both NULL restore hipMalloc/hipFree; one NULL is TE_ERR_INVALID_ARG.  Every block goes back
 * to the allocator that supplied it, also after the hook has been changed.  The callbacks may
 * be called from the engine's scheduler thread.  Host only; thread-safe. */
typedef void* (*te_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*te_free_fn)(void* ptr, void* stream, void* ctx);
te_status te_set_allocator(te_alloc_fn alloc, te_free_fn free_fn, void* ctx);

/* ---------------------------------------------------------------------------------------
 * te_evolve: Alg. 1 ("Krylov-method") end to end on the device.
 *   v0     : device, dim complex; need not be normalised (the result and the bound scale
 *            with ||v0||, the method itself runs on v0/||v0||).
 *   v_out  : device, dim complex; may equal v0.
 *   t >= 0, tol > 0 (err_max, the bound on the 2-norm of the final error), finite.
 *   m      : Krylov dimension, 2 <= m <= TE_MAX_KRYLOV; clamped to dim.
 *   opt    : NULL for defaults.   res : host, may be NULL.
 * Every restart (Arnoldi steps, diagonalisation of the small Hessenberg matrix, error
 * integral, step-size search, recombination) runs on the device; the host only enqueues
 * restarts ahead of the device and stops once the device reports completion.
 * t == 0 copies v0; ||v0|| == 0 returns zeros with a zero bound.  Synchronous.
 * Calls on one handle are serialised (the handle holds one workspace). */
te_status te_evolve(te_hamiltonian h, const te_c128* v0, te_c128* v_out, double t, double tol,
                    int32_t m, const te_options* opt, te_result* res, void* stream);

/* te_evolve_noalloc: for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation).  The same evolution as
 * te_evolve, with the same arguments, results, errors and kernels (the handle's current
 * kernel shape; this call never autotunes), but the workspace (Krylov basis, product vector,
 * reduction partials, device state, done flag) lives in one static device array of
 * TE_NOALLOC_SCRATCH_BYTES per device, set up on the first call on each device, instead of
 * memory the library allocates: the call makes no device or pinned-host allocation.
 * Limit: te_workspace_bytes(h, m) + 256 must not exceed TE_NOALLOC_SCRATCH_BYTES (64 MiB:
 * dim up to ~100,000 at m = 40, e.g. the XXZ ring up to L = 16), else TE_ERR_CAPACITY before
 * any device work.  TE_OPT_PROFILE is rejected (TE_ERR_INVALID_ARG).  The array keeps the
 * last call's contents, which the call clears as needed.  Every call on one device shares the
 * array, so calls that overlapped on one device would race: the library serialises them with a
 * per-device lock (each process holds its own copy of the array).  The host checks the
 * device's done flag every two restarts with a 4-byte copy.  Synchronous. */
#define TE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
te_status te_evolve_noalloc(te_hamiltonian h, const te_c128* v0, te_c128* v_out, double t, double tol,
                            int32_t m, const te_options* opt, te_result* res, void* stream);

/* Intermediate-time sampling (second remark after Alg. 1): inside the step that holds t_s,
 * v(t_s) = V exp(-i J (t_s - t_now)) e_1 from the step's own basis and small matrix, so the
 * samples cost no extra Krylov builds.  Each sample carries the bound accumulated up to the
 * end of its step (an upper bound at t_s).  Diagonal observables (e.g. number operators in a
 * Fock basis) are reduced on the device without writing the states.
 *   times    : host, n_times ascending values in [0, t].
 *   states   : device, n_times x dim complex (state s at states + s*dim), or NULL.
 *   obs      : device, n_obs x dim real diagonals D_o (D_o at obs + o*dim), or NULL if n_obs == 0.
 *   obs_out  : host, n_times x n_obs: <v(t_s)| D_o |v(t_s)>.
 *   bound_out: host, n_times, or NULL. */
typedef struct {
    int32_t n_times;
    const double* times;
    te_c128* states;
    int32_t n_obs;
    const double* obs;
    double* obs_out;
    double* bound_out;
} te_samples;

/* te_evolve plus samples (see te_samples).  Same arguments, results and errors as te_evolve;
 * TE_ERR_INVALID_ARG for unsorted or out-of-range times and with TE_OPT_PROFILE.  Allocates
 * O(n_times * (64 + n_obs * dim / 256)) scratch for the call.  Synchronous. */
te_status te_evolve_sampled(te_hamiltonian h, const te_c128* v0, te_c128* v_out, double t, double tol,
                            int32_t m, const te_options* opt, const te_samples* samples,
                            te_result* res, void* stream);

/* Totals recorded by the last te_evolve on h that ran with TE_OPT_PROFILE (zeros if none). */
te_status te_last_profile(te_hamiltonian h, te_profile* out);

/* ---------------------------------------------------------------------------------------
 * Autotuning of the kernel shapes (per Hamiltonian handle).  The projection kernel (sparse
 * product fused with the projections) is timed on the handle's own matrix for every supported
 * shape and the fastest is kept; te_evolve tunes a handle on first use unless the environment
 * sets TE_AUTOTUNE=0.  If TE_TUNE_CACHE names a file, results are read from / appended to it
 * (one line per "gfx950/<storage> dim nnz m" key, storage as named by TE_STORAGE_*). */
typedef struct {
    int32_t lanes_per_row;          /* lanes sharing one row of the sparse product: 1, 2, 4 or 8 */
    int32_t nnz_per_lane;           /* nonzeros per lane in flight: 8 (1 or 2 lanes), 1 or 4
                                       (4 lanes), 2 (8 lanes) */
    int32_t rows_per_thread;        /* projection kernel: 1, 2 or 4 (4: batches of 4 columns) */
    int32_t update_rows_per_thread; /* update and recombination kernels: 1 or 2 */
    int32_t split_projection;       /* 0: sparse product fused with the projections in one kernel;
                                       1: two launches, the product vector read back (same results) */
    double project_us;              /* measured time of one projection launch, 0 if not measured */
} te_tuning;

/* Times every supported projection shape for Krylov dimension m, then the update kernel with one
 * and two rows per thread in the chosen shape, and keeps the fastest in h (out may be NULL).
 * Synchronous. */
te_status te_autotune(te_hamiltonian h, int32_t m, te_tuning* out, void* stream);
te_status te_get_tuning(te_hamiltonian h, te_tuning* out); /* the shape te_evolve will use */
te_status te_set_tuning(te_hamiltonian h, const te_tuning* t); /* TE_ERR_INVALID_ARG if unsupported */

/* ---------------------------------------------------------------------------------------
 * Component entry points: each runs one step of the hot path with the same kernels that
 * te_evolve uses, for testing and for callers that assemble their own loop.
 *
 * te_spmv (eq. arnoldi, first line: w_j = H v_j, fused with the projection <v_j, w_j>):
 *   x, y: device, dim complex, must not alias.  xhy: host, receives x^H y (may be NULL).
 *   Synchronous. */
te_status te_spmv(te_hamiltonian h, const te_c128* x, te_c128* y, te_c128* xhy, void* stream);

/* te_arnoldi (Alg. 1 step 1, with full re-orthogonalisation): builds the Krylov basis of
 * u (device, dim, assumed normalised) for Lanczos on H.
 *   V      : device, m*dim complex, column-major (column i at V + i*dim), receives the
 *            orthonormal basis v_1..v_k (columns >= k are unspecified).
 *   alpha  : host double[m], diagonal of the real symmetric tridiagonal J = V^H H V.
 *   beta   : host double[m], beta[i] = ||residual|| after step i (off-diagonal J_{i+1,i}
 *            for i < k-1; beta[k-1] = h, the h_{k+1,k} of eq. errorIntegral).
 *   k_out  : host, Krylov dimension reached (< m after a lucky breakdown, no < tol_rate).
 *   Synchronous. */
te_status te_arnoldi(te_hamiltonian h, const te_c128* u, int32_t m, double tol_rate,
                     te_c128* V, double* alpha, double* beta, int32_t* k_out, void* stream);

/* te_tridiag_eig (Sec. "Pseudocode", first remark: diagonalise H_m once per restart):
 * J = Q diag(lambda) Q^T for the k x k real symmetric tridiagonal with diagonal alpha[k]
 * and off-diagonal beta[k-1].  Host arrays in/out; Q is column-major k*k (column n is the
 * eigenvector of lambda[n]); eigenvalues are not sorted.  Runs on the device in one
 * workgroup (divide and conquer from k = 16, implicit QL below), the same code the step kernel
 * of te_evolve runs.  1 <= k <= TE_MAX_KRYLOV.  Synchronous. */
te_status te_tridiag_eig(int32_t k, const double* alpha, const double* beta, double* lambda,
                         double* Q, void* stream);

/* te_error_integral (eq. errorIntegral on [a, b]): integral of
 * f(tau) = h |sum_n coef[n] exp(-i lambda[n] tau)| by the device tanh-sinh rule.
 *   lambda, coef: host double[k]; value/level/converged: host outputs.  Synchronous. */
te_status te_error_integral(int32_t k, const double* lambda, const double* coef, double h,
                            double a, double b, const te_options* opt, double* value,
                            int32_t* level, int32_t* converged, void* stream);

/* te_step_search (Alg. 1 step 2 and the coefficients omega of its last line): from the
 * tridiagonal (alpha[k], beta[k-1]), residual norm h and the rate tol_rate = err_max/t
 * (eq. errorRate), the largest admissible step tau <= t_rem (eq. stepSize) with its
 * integral err, and omega = exp(-iJ tau) e_1 (host te_c128[k]).
 *   first   : nonzero on the first restart (doubling from t_init), else tau_prev is used.
 *   breakdown: nonzero when the Krylov space is invariant (tau = t_rem).
 *   warnings: host, TE_WARN_QUADRATURE if an integral did not converge.
 * Returns TE_ERR_STEP_UNDERFLOW when no admissible step is found.  Synchronous. */
te_status te_step_search(int32_t k, const double* alpha, const double* beta, double h,
                         double tol_rate, double t_rem, int32_t first, double tau_prev,
                         int32_t breakdown, const te_options* opt, double* tau, double* err,
                         te_c128* omega, uint32_t* warnings, void* stream);

/* ---------------------------------------------------------------------------------------
 * Batched and served evolution.  An engine advances many jobs, each one te_evolve problem
 * (H, v0, t, tol) with the engine's m and options, together in rounds: one round runs one
 * restart of Alg. 1 (Krylov build, step-size choice, recombination) for every resident job,
 * with batched kernels whose workgroups are (job, row tile) items of all jobs at once.  Jobs
 * sharing one Hamiltonian handle stream its CSR once per Krylov iteration for up to 8 vectors
 * (a multi-vector sparse product).  A round is one hipGraph launch; all step decisions stay on
 * the device, the host only keeps rounds queued and reads completion records written by the
 * device into mapped host memory.
 *
 * Scheduling points are round boundaries.  There, completed jobs leave (their workspace is
 * returned to the pool) and queued jobs are admitted in submission order while a slot is free
 * and te_job_footprint(dim, m) bytes fit in the pool (first fit).  H, the basis and the job
 * state stay resident across restarts.  A job's arithmetic does not depend on the other jobs
 * of a round: with one kernel shape its result is bitwise the same alone and in any mix.
 *
 * Lanes (te_engine_config.lane_rows > 0).  Every job of a round advances by one restart, so a
 * job whose restarts are cheap but many (a small matrix, a long time, a tight tolerance) moves
 * at the pace of the largest job beside it.  With two lanes, jobs of at least lane_rows rows
 * run in a lane of their own, at most lane_jobs at a time in submission order, on a second
 * stream, while the smaller jobs go round in the other lane at their own pace; the device runs
 * both lanes' kernels side by side.  Job ids stay one sequence over both lanes; the statistics
 * add up both lanes (busy_seconds: the larger of the two; tuning: the small-job lane's).  The
 * lanes run side by side only with TE_ENGINE_THREADED (otherwise te_engine_wait drives one lane,
 * then the other).
 *
 * Job buffers: v0 and v_out are device pointers of dim complex owned by the caller; v0 must
 * hold its data when te_engine_submit is called and stay unchanged until the job is admitted,
 * v_out must stay valid until the job is done (it is complete once te_engine_poll reports
 * TE_JOB_DONE); v_out may equal v0.  The Hamiltonian handle must outlive its jobs; a handle in
 * use by an engine must not be passed to te_evolve concurrently (it is only read, but
 * te_hamiltonian_destroy would free it). */
typedef struct te_engine_s* te_engine;
typedef int64_t te_job;

#define TE_ENGINE_THREADED 1u /* a worker thread schedules rounds; otherwise rounds advance
                                 inside te_engine_wait / te_batch_launch */
#define TE_ENGINE_PROFILE 2u  /* no graphs, no lookahead: an event around every kernel class;
                                 te_engine_stats.prof accumulates times and algorithmic bytes */

typedef struct {
    int32_t m;                      /* Krylov dimension, 2..TE_MAX_KRYLOV (clamped per job to dim) */
    int32_t max_jobs;               /* resident jobs at most, 1..16384 */
    uint64_t hbm_budget;            /* bytes of device memory for job workspaces, allocated once */
    int32_t lanes_per_row;          /* sparse-product shape: 1, 4 or 8 lanes per row; 0 = autotune */
    int32_t nnz_per_lane;           /* 8 with 1 lane, 1 or 4 with 4 lanes, 2 with 8 lanes */
    int32_t rows_per_thread;        /* projections: 1, 2 or 4 rows per thread; 0 = 4 */
    int32_t update_rows_per_thread; /* update and recombination: 1 or 2; 0 = 2 */
    uint32_t flags;                 /* TE_ENGINE_* */
    te_options opt;                 /* step-size / quadrature options; opt.flags: 0 or TE_OPT_LANCZOS3 */
    int64_t lane_rows;              /* 0: one lane.  > 0: two lanes, each an engine of its own (own
                                       rounds and half of hbm_budget; the small-job lane on the
                                       given stream, the large-job lane on a stream of its own)
                                       running concurrently: jobs of at least lane_rows rows go to
                                       the large-job lane, which keeps at most lane_jobs of them
                                       resident (admitted in submission order), the others to the
                                       small-job lane.  A job must fit half of hbm_budget. */
    int32_t lane_jobs;              /* resident jobs of the large-job lane, 1..max_jobs (0: two, or
                                       max_jobs if that is smaller) */
} te_engine_config;

enum { TE_JOB_QUEUED = 0, TE_JOB_RUNNING = 1, TE_JOB_DONE = 2, TE_JOB_FAILED = 3 };

typedef struct {
    int32_t state;      /* TE_JOB_* */
    te_status status;   /* TE_OK, or why the job failed */
    int32_t rounds;     /* rounds the job was resident for */
    int32_t steps;      /* restarts completed so far */
    double t_now;       /* time reached so far */
    double submitted, admitted, finished; /* host monotonic clock (seconds; 0 = not yet) */
} te_job_info;

typedef struct {
    int64_t rounds;       /* rounds completed */
    int64_t plans;        /* round graphs built (one per change of the resident set) */
    int64_t jobs_submitted, jobs_done, jobs_failed, jobs_queued, jobs_running;
    uint64_t pool_bytes, pool_used, pool_peak;
    double busy_seconds;  /* wall time with at least one job resident */
    te_tuning tuning;     /* shape in use (project_us: autotuned time of one projection round) */
    te_profile prof;      /* TE_ENGINE_PROFILE only: per kernel class, summed over rounds */
} te_engine_stats;

/* Device bytes one job of dimension dim takes from the pool (basis m x dim, product vector,
 * reduction partials); 0 for invalid arguments.  Host-only. */
uint64_t te_job_footprint(int64_t dim, int32_t m);

/* Fills the defaults: m=40, max_jobs=1024, hbm_budget=0 (must be set), autotuned sparse-product
 * shape, 2 rows per thread, threaded, te_default_options.  A job's results are bitwise those of
 * te_evolve with the same shape (te_set_tuning with the same lanes, nonzeros, rows per thread
 * and update rows per thread). */
void te_engine_default_config(te_engine_config* cfg);

/* Allocates the pool (hbm_budget bytes) and the job slots on the current device.  stream:
 * the engine's work stream (NULL: the engine creates a non-blocking stream of its own).
 * TE_ENGINE_THREADED starts the scheduler thread. */
te_status te_engine_create(te_engine* out, const te_engine_config* cfg, void* stream);

/* Queues one job; returns its id (ids increase from 0).  Thread-safe, never blocks on the
 * device.  TE_ERR_CAPACITY if the job's footprint exceeds the whole pool (it could never be
 * admitted); TE_ERR_INVALID_ARG for the te_evolve argument rules.  t == 0 completes at once
 * (v_out = v0). */
te_status te_engine_submit(te_engine e, te_hamiltonian h, const te_c128* v0, te_c128* v_out,
                           double t, double tol, te_job* id);

/* State of a job; res (may be NULL) is filled once the job is done or failed. */
te_status te_engine_poll(te_engine e, te_job id, te_job_info* info, te_result* res);

/* Waits until job id (or every job submitted so far, for id = -1) is done or failed, or the
 * timeout (seconds; < 0 = none) expires: TE_ERR_TIMEOUT.  Without TE_ENGINE_THREADED the
 * rounds run inside this call.  Returns TE_ERR_DEVICE if the engine failed. */
te_status te_engine_wait(te_engine e, te_job id, double timeout_s);

te_status te_engine_get_stats(te_engine e, te_engine_stats* out);

/* Stops the scheduler, waits for the device, frees the pool.  Jobs not done are dropped. */
te_status te_engine_destroy(te_engine e);

/* Batch: a fixed set of jobs run to completion by an engine without a scheduler thread.
 * te_batch_add appends n jobs on one H (v0[i], v_out[i]: host arrays of n device pointers)
 * and returns the index of the first; te_batch_launch runs every job (hbm_budget 0: the sum
 * of the footprints, so all jobs are resident from the first round) and returns once all are
 * done; te_batch_result gives a job's result and status, te_batch_info its timing (submitted
 * = start of te_batch_launch).  cfg: as for te_engine_create
 * (max_jobs 0 = all jobs, hbm_budget ignored; TE_ENGINE_THREADED ignored). */
typedef struct te_batch_s* te_batch;
te_status te_batch_create(te_batch* out, const te_engine_config* cfg, void* stream);
te_status te_batch_add(te_batch b, te_hamiltonian h, int32_t n, const te_c128* const* v0,
                       te_c128* const* v_out, double t, double tol, int32_t* first);
te_status te_batch_launch(te_batch b, uint64_t hbm_budget, te_engine_stats* stats);
te_status te_batch_result(te_batch b, int32_t i, te_result* res, te_status* status);
te_status te_batch_info(te_batch b, int32_t i, te_job_info* info); /* times, rounds, state */
te_status te_batch_destroy(te_batch b);

#ifdef __cplusplus
}
#endif

#endif /* TE_H */
