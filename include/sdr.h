/*
 * sdr.h -- C interface of the GMRES-SDR library for MI355X (gfx950).
 *
 * GMRES-SDR (Burke, Guettel, Soodhalter, "GMRES with randomized sketching and
 * deflated restarting", arXiv 2311.14206) solves A x = b for a sparse,
 * nonsymmetric, real or complex A, and sequences A_i x_i = b_i, by restarted
 * cycles of Algorithm 1: truncated Arnoldi (each new basis vector is
 * orthogonalised against the t previous ones only, Section 3.2), a sparse-sign
 * sketch S of every basis vector (Section 3, eq. (3.1)), the sketched least
 * squares problem min_y ||S r0 - S A [U V] y|| (eq. (3.2), Section 3.3), the
 * safety-factor residual control of Section 3.4, and the sketched
 * harmonic-Ritz compression of [U V] into the next recycle space (Section 3.5,
 * eq. (3.6)).  Sequences reuse U, SU, SAU (Section 3.6).
 *
 * Conventions
 *  - Every vector / matrix pointer passed to a solve is a DEVICE pointer on the
 *    current HIP device.  Complex data are interleaved (re, im) pairs.
 *  - CSR: int32 row_ptr[n+1] (row_ptr[0] = 0, non-decreasing), int32
 *    col_idx[nnz] in [0, n), values[nnz] of the stated dtype.
 *  - The handle copies the matrix (it owns its copies); b, x, g, lambda and
 *    output buffers are borrowed for the duration of a call only.
 *  - Calls are ordered on the handle's stream (sdr_set_stream) and return after
 *    the work has completed.  A handle must be used by one thread at a time.
 *  - Return codes: 0 success, 1 not converged (x holds the last iterate),
 *    negative values are errors; sdr_last_error() gives a message (thread
 *    local).
 */
#ifndef SDR_H
#define SDR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SDR_F64 = 0,   /* real float64 */
  SDR_F32 = 1,   /* real float32 (only as a basis precision, see "precision") */
  SDR_C128 = 2,  /* complex128 */
  SDR_C64 = 3    /* complex64 (only as a basis precision) */
} sdr_dtype;

enum {
  SDR_OK = 0,
  SDR_NOT_CONVERGED = 1,
  SDR_EINVAL = -1,      /* bad sizes or parameters, non-finite input */
  SDR_EPATTERN = -2,    /* sdr_update_matrix: sparsity pattern differs */
  SDR_EDEVICE = -3,     /* a HIP call failed */
  SDR_EBREAKDOWN = -4,  /* no progress possible (breakdown at the first step) */
  SDR_ENOMEM = -5       /* device allocation failed */
};

/* Sparse matrix in CSR form, device pointers.  dtype is SDR_F64 or SDR_C128. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const void* values;
  sdr_dtype dtype;
} sdr_csr;

/* Counters and timings of the last solve (Section 6 counts MV and IP). */
typedef struct {
  int32_t cycles;          /* restart cycles run */
  int32_t iters;           /* Arnoldi steps (accepted) */
  int32_t matvecs;         /* products with A, incl. residual checks */
  int32_t inner_products;  /* length-N inner products and norms */
  int32_t sketches;        /* length-N vectors sketched */
  int32_t res_checks;      /* true-residual evaluations (Section 3.4) */
  int32_t status;          /* return code of the solve */
  int32_t k_eff;           /* recycle dimension after the solve */
  double relres;           /* ||b - A x|| / ||b|| at exit (FP64) */
  double sres;             /* last sketched residual */
  double safety;           /* safety factor at exit (0 with the Givens control) */
  double seconds;          /* wall time of the solve */
  double host_eig_seconds; /* host time in the harmonic-Ritz eigen-step */
  double eps;              /* fitted eps of the Givens residual control (0 otherwise) */
} sdr_stats;

/* Per-cycle decision record of the last solve. */
typedef struct {
  int32_t j_stop;     /* Arnoldi steps taken in the cycle */
  int32_t n_checks;   /* true-residual checks in the cycle */
  int32_t ell;        /* numerical rank used in the harmonic-Ritz step */
  int32_t k_eff;      /* recycle dimension produced */
  int32_t flags;      /* 1 converged, 2 Arnoldi breakdown, 4 rank loss */
  int32_t pad;
  double sres;        /* sketched residual at the stop */
  double res;         /* true residual at the stop (absolute) */
} sdr_cycle_record;

typedef struct sdr_handle sdr_handle;

/*
 * Create a solver for the n x n matrix A (Algorithm 1 inputs m, t, k, s).
 *   m      Arnoldi steps per cycle (>= 1); the search space is [U, V(:,1:j)].
 *   k      recycle dimension (>= 0); real problems may keep k+1 so that a
 *          complex-conjugate harmonic-Ritz pair is never split.
 *   t      truncation window (1 <= t <= min(m, 4)).
 *   s_dim  sketch rows; s_dim > m + k and s_dim % zeta == 0 (zeta = 8 by
 *          default, option "zeta"); at most 2048 for real and 1024 for
 *          complex matrices (per-wave sketch accumulators in LDS).
 *   seed   64-bit seed of the sketching operator.
 * The CSR arrays are copied.  Returns NULL on error (see sdr_last_error()).
 */
sdr_handle* sdr_create(const sdr_csr* A, int m, int k, int t, int s_dim, uint64_t seed);

/*
 * Set an option (before the first solve for "precision" and "zeta").
 *   "zeta"           nonzeros per sketch column (default 8)
 *   "max_cycles"     restart limit (default 10000)
 *   "safety0"        initial safety factor (default 1.4, Section 3.4)
 *   "persist_safety" 1: keep safety across cycles (default 0: reset per cycle)
 *   "precision"      0: basis in the matrix precision (FP64 / complex128);
 *                    1: basis, SpMV and sketches in FP32 / complex64 with the
 *                    least squares, eigen-step and residual in FP64 / c128
 *   "variant"        0: exact sequences (recompute S A_i U), 1: inexact
 *   "breakdown_rtol" Arnoldi breakdown threshold (default 1e-14; 1e-6 FP32)
 *   "rank_rtol"      rank-loss threshold of the sketched LSQ (default 1e-12)
 *   "lsq_chunk"      Arnoldi steps per least-squares launch (default 8)
 *   "lsq_kernel"     least-squares kernel: 0 (default) keeps the QR factor in
 *                    registers where the sketch and the basis are small
 *                    enough, else block Gram-Schmidt (blocks of up to 8
 *                    steps, Q swept four times per block) with the sweeps
 *                    spread over many workgroups; 1: the block method in
 *                    one workgroup; 2: one launch per step (reference
 *                    form); 3: the block method on many workgroups.  The
 *                    same decisions and, up to rounding, the same factor.
 *   "dia"            1 (default): a pattern whose entries lie on at most 16
 *                    diagonals (padding at most nnz/4) is stored by diagonals
 *                    for the basis SpMV; 0: always CSR
 *   "precond"        1: right Jacobi preconditioning of the forward solve
 *                    (Section 6 solves its Stokes systems preconditioned; a
 *                    diagonal right preconditioner is the cheapest such
 *                    case): A x = b is solved as (A D^-1) u = b, x = D^-1 u,
 *                    D = diag(A).  D^-1 is folded into the stored values
 *                    (A D^-1 on the same pattern, refreshed by
 *                    sdr_update_matrix), so an Arnoldi step costs the same.
 *                    Every diagonal entry must be stored and nonzero, else
 *                    the solve or update returns SDR_EINVAL (and, after a
 *                    rejected update, every solve until a valid matrix).  Residuals,
 *                    tolerances and stats refer to A x = b (the same vector
 *                    b - A D^-1 u); the recycle space, basis and sketches
 *                    (sdr_get_recycle, sdr_get_basis) belong to A D^-1.
 *                    sdr_spmv and the adjoint solve use A unpreconditioned.
 *                    2: right ILU(0) preconditioning (Section 6 solves its
 *                    Stokes systems with ILU; zero fill, the right side and
 *                    the elimination order are this library's readings):
 *                    (A M^-1) u = b, x = M^-1 u, M = L U the ILU(0)
 *                    factorisation of A with the unknowns taken colour by
 *                    colour in a greedy colouring of the symmetrised pattern
 *                    (each row, in increasing index, takes the smallest
 *                    colour none of its lower-indexed neighbours holds).
 *                    The factors live on A's entries and are refreshed by
 *                    sdr_update_matrix; every diagonal entry must be stored
 *                    and every pivot nonzero, else SDR_EINVAL as for 1.  An
 *                    Arnoldi step applies M^-1 (2C - 1 launches for C
 *                    colours, 3 for a 5-point stencil) before its SpMV.
 *                    Residuals, basis and recycle space as for 1, with
 *                    A M^-1 in place of A D^-1.
 *                    Default 0, set before the first solve.
 *   "sketch"         0 (default): the sparse-sign operator (zeta nonzeros
 *                    per column, drawn from seed); 1: the subsampled
 *                    randomised DCT S = sqrt(N/s) P F E of Section 6 (F the
 *                    orthonormal DCT-II, E random signs, P s distinct random
 *                    rows, all drawn from seed; s_dim <= n, any s_dim).  Set
 *                    before the first solve.  The DCT sketch costs s
 *                    multiply-adds per entry (ALU-bound), the sparse sign a
 *                    few LDS adds.
 *   "resid_control"  0 (default): the safety-factor rule of Section 3.4, a
 *                    true residual once the sketched one is below tol /
 *                    safety; 1: the Givens-rotation estimate of Sections 4.5
 *                    and 5: each step's sine is the ratio of consecutive
 *                    sketched residuals, the estimate of the true residual
 *                    grows by sqrt((s^2 + 2 eps (1 + c)) / (1 - eps^2)) from
 *                    ||r0|| (or the sketched residual over span(U) / sqrt(1 -
 *                    eps)), a true residual is computed once the estimate is
 *                    below tol, and eps is raised (by bisection) to the
 *                    smallest value whose estimate reaches a true residual
 *                    that exceeded it; the estimate then restarts from that
 *                    residual.  eps persists across the cycles of a solve
 *                    (stats.eps)
 *   "givens_eps0"    initial eps of the Givens control, in [0, 1) (default 0)
 *   "kernel_timing"  n > 0: HIP events around the SpMV and update kernels of
 *                    one Arnoldi step in n, at positions that move by 13 from
 *                    cycle to cycle (sdr_kernel_times); default 0
 * Returns 0 or SDR_EINVAL.
 */
int sdr_set_option(sdr_handle* h, const char* key, double value);

/*
 * Run the handle's calls on this HIP stream (hipStream_t as void*).  NULL
 * means the device's null stream: the handle then runs on a non-blocking
 * stream of its own that waits, at each call, for the work queued on the
 * null stream before the call.  Either way inputs written by earlier work on
 * the given stream are read in order.  Until this is called the handle uses
 * its own stream without that wait: inputs must then be complete on the
 * device before a call.
 */
int sdr_set_stream(sdr_handle* h, void* hip_stream);

/*
 * Solve A x = b to ||b - A x|| <= tol * ||b||.  If A_or_null is not NULL it
 * replaces the matrix first (as sdr_update_matrix).  x holds the initial guess
 * on entry and the solution on exit.  The recycle space of the previous solve
 * is reused (Section 3.6).  stats may be NULL.
 * Returns 0, SDR_NOT_CONVERGED, or an error code.
 */
int sdr_solve(sdr_handle* h, const sdr_csr* A_or_null, const void* b, void* x, double tol,
              sdr_stats* stats);

/*
 * Replace the matrix values (same n, nnz, row_ptr, col_idx) for the next solve
 * of a sequence.  With the exact variant the next solve recomputes S A_i U
 * (k extra products and sketches); the inexact variant keeps the stale one.
 * Returns 0, SDR_EPATTERN, or an error code.
 */
int sdr_update_matrix(sdr_handle* h, const sdr_csr* A_i);

/*
 * Adjoint solve A^T lambda = g (A^H for complex) with its own recycle space,
 * kept across calls.  tol is relative to ||g||.  Returns as sdr_solve.
 */
int sdr_solve_adjoint(sdr_handle* h, const void* g, void* lambda, double tol, sdr_stats* stats);

/*
 * For every stored entry e = (i, j): grad_vals[e] = -lambda[i] * x[j] (real)
 * or -lambda[i] * conj(x[j]) (complex).  With A x = b and lambda solving the
 * adjoint system A^T lambda = dL/dx (A^H lambda = dL/d conj(x) for complex
 * data) this is the derivative of the loss L with respect to the stored
 * entries of A (with respect to conj(A_ij) for complex data); dL/db = lambda.
 * lambda, x: n device vectors, grad_vals: nnz device vector, matrix dtype.
 */
int sdr_grad_values(sdr_handle* h, const void* lambda, const void* x, void* grad_vals);

/* Copy the per-cycle records of the last solve; returns the number written. */
int sdr_get_trace(sdr_handle* h, sdr_cycle_record* out, int cap);

/* Current recycle dimension, and a copy of U (n x k, ld = n), SU, SAU
 * (s x k, ld = s) into device buffers (any may be NULL).  Real handles write
 * float64; complex handles complex128. */
int sdr_get_recycle(sdr_handle* h, void* U, void* SU, void* SAU, int* k_out);

/* y = S X for ncols device columns X (ld = n) in the handle's FP64/c128
 * type; Y is s x ncols (ld = s).  The operator Section 3 describes, drawn
 * from the handle's seed. */
int sdr_sketch(sdr_handle* h, const void* X, int ncols, void* Y);

/*
 * Allocation-free form of sdr_sketch, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  Y = S X for ncols device columns X (n x ncols, ld = n) of
 * dtype SDR_F64 or SDR_C128 (interleaved), Y s_dim x ncols (ld = s_dim): the
 * sparse-sign operator with zeta nonzeros per column drawn from seed, the
 * same operator and the same kernels as sdr_sketch on a handle created with
 * that seed, s_dim and option "zeta".  No handle, no allocation: the partial
 * sums live in a static device array of SDR_NOALLOC_SCRATCH_BYTES (16 MiB),
 * one per GPU, held until the process ends; the array's device address is
 * looked up on the first call on each device.
 *   Limits: 1 <= n < 2^31, s_dim a multiple of zeta, s_dim <= 2048 (real) or
 *   1024 (complex), and n * (s_dim + 1) * element size / 2048 within the
 *   scratch (about n <= 17e6 at s_dim = 240 real, 5.9e6 at 360 complex);
 *   beyond them SDR_EINVAL with a message.
 * The work is queued on hip_stream (hipStream_t as void*, NULL = the null
 * stream) and the call returns without waiting: Y is complete when that
 * stream's work is.  Every call on one GPU shares that GPU's scratch: calls
 * whose work overlaps on one GPU (other streams, other threads) race and
 * must be ordered by the caller.  Returns 0 or a negative error code.
 */
#define SDR_NOALLOC_SCRATCH_BYTES (16u << 20)
int sdr_sketch_noalloc(int64_t n, int s_dim, int zeta, uint64_t seed, sdr_dtype dtype, const void* X,
                       int ncols, void* Y, void* hip_stream);

/* y = A x with the handle's matrix (FP64 / complex128 device vectors). */
int sdr_spmv(sdr_handle* h, const void* x, void* y);

/* z = M^-1 v for the handle's preconditioner (option "precond": 0 the
 * identity, 1 D^-1, 2 the ILU(0) solve; Section 6), FP64 / complex128 device
 * vectors of length n.  Factors the current matrix first if no solve has.
 * SDR_EINVAL if that factorisation failed (zero diagonal entry or pivot).
 * The apply is queued on the handle's stream (sdr_set_stream) and the call
 * returns without waiting: z is complete when that stream's work is.  With
 * the null stream set, the null stream's later work waits for the apply (on
 * the device). */
int sdr_precond_apply(sdr_handle* h, const void* v, void* z);

/* Basis data of the last cycle for inspection: the first ncols normalised
 * basis vectors V (n x ncols, FP64/c128 device), H ((m+1) x m host, column
 * major), SV (s x ncols host).  Any pointer may be NULL. */
int sdr_get_basis(sdr_handle* h, int ncols, void* V, void* H_host, void* SV_host);

/* Sketched residual norms ||S r0 - SAW y_j|| of the last cycle of the last
 * solve, by Arnoldi step (the quantity Section 3.3's least squares
 * minimises): out[0] over span(U) alone (||S r0|| without a recycled block),
 * out[j] after step j.  Writes min(cap, count) host doubles and returns
 * count (j_stop + 1; 0 before the first solve). */
int sdr_get_step_sres(sdr_handle* h, double* out, int cap);

/* Drop the recycle spaces of the forward and the adjoint solver (the next
 * solve of either starts without U).  Returns 0. */
int sdr_reset(sdr_handle* h);

/*
 * Per-step kernel timings gathered with HIP events on the handle's stream
 * when the option "kernel_timing" is n > 0 (one step in n), accumulated since the last call and
 * then cleared.  ms[0]: SpMV + window products + sketch kernel, ms[1]:
 * orthogonalisation update kernel, ms[2]: the kernels of the step, from the
 * start of the first to the end of the update (the least squares runs on a
 * second stream), ms[3]: the subsampled-DCT sketch kernel (option sketch=1,
 * launched between them; 0 otherwise).  counts[0..2]: launches timed; counts[3 + tw]:
 * steps whose truncation window held tw vectors (tw <= 4).  cap is the
 * length of both arrays (8 covers everything).
 */
int sdr_kernel_times(sdr_handle* h, double* ms, int64_t* counts, int cap);

/*
 * Storage of the matrix in the basis SpMV: returns the number of diagonals
 * when the pattern is stored by diagonals (option "dia") and writes their
 * offsets (column - row, ascending) to offsets[0 .. min(that, cap) - 1];
 * returns 0 for CSR.  Negative: error code.
 */
int sdr_spmv_layout(sdr_handle* h, int* offsets, int cap);

/*
 * Diagonals of that storage found constant when the matrix was last packed
 * (every entry inside the matrix with the same bits, as in a constant-
 * coefficient stencil): bit d set for diagonal d of sdr_spmv_layout's order.
 * The step kernel takes their values from its arguments instead of reading
 * them; the products are the same.  Option "dia_const": 1 on, 0 off; by
 * default on for complex data and off for real data (whose step kernel at
 * the 1024^2 stencil ran no faster without the streams).
 * Packing happens at the first solve after the matrix is set or updated, so
 * the mask describes the matrix of the last solve (0 before the first, or
 * for CSR).  Negative: error code.
 */
int sdr_spmv_const_diagonals(sdr_handle* h);

void sdr_destroy(sdr_handle* h);

/* Message of the last error on this thread ("" if none). */
const char* sdr_last_error(void);

/*
 * Host-only helper used by the library's cycle end and exported for testing:
 * the sketched harmonic-Ritz step (Section 3.5).  Given the triangular factor
 * R (l0 x l0, column major, upper) of SAW = Q R and C = Q^H [SU, SV] (l0 x l0),
 * computes G (l0 x k_eff, column major, ld = l0) whose columns span the
 * invariant subspace of the k largest-modulus eigenvalues of the sketched
 * pencil, with the truncated-SVD regularisation when R is numerically rank
 * deficient.  is_complex selects complex128 data; for real data G is real and
 * a conjugate pair is never split.  Returns k_eff (>= 0) and writes ell, or a
 * negative error code.  G must hold l0 * (k+1) elements.
 */
int sdr_host_harmonic_ritz(int l0, const void* R, const void* C, int s, int k, int is_complex,
                           void* G, int* ell);

#ifdef __cplusplus
}
#endif

#endif /* SDR_H */
