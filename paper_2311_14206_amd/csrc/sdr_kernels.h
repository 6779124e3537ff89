// Launch wrappers of the GMRES-SDR device kernels (gfx950).
#pragma once

#include <string>

#include "sdr_common.h"

namespace sdr {

// Set the thread-local message that sdr_last_error() returns.
void set_last_error(const std::string& msg);

constexpr int kBlock = 256;        // threads per block of the streaming kernels
constexpr int kWaves = kBlock / 64;
constexpr int kLsqBlock = 512;     // threads of the single-block least-squares kernels
constexpr int kMaxWindow = 4;      // largest truncation window t
constexpr int kRowsSpmv = 1536;    // rows per tile, SpMV + window products + sketch
constexpr int kSpmvThreads = 512;  // threads of the diagonal-storage SpMV (3 rows each); 256 when
                                   // 8 waves of sketch bins exceed kSpmvLds
constexpr int kRowsUpdate = 2048;  // rows per block of the other streaming kernels
constexpr int kUpdateRows = 8;     // rows per thread of the update
constexpr int kUpdateThreads = 512;  // threads per update block for complex data (4096 rows)
constexpr int kPartRounds = 3;     // SpMV partials per thread the update loads up front (768 tiles)
constexpr int kWaveTileNnz = 512;  // largest staged chunk (entries of 64 rows) per wave of the SpMV
constexpr int kSpmvLds = 64 * 1024;  // LDS budget of the SpMV kernel: sketch bins + staged chunks
constexpr int kMaxDiag = 16;       // most diagonals of the stencil (diagonal-storage) SpMV

template <class T> struct Window { const T* p[kMaxWindow]; };

// A matrix whose nonzeros lie on ndiag diagonals (offsets off[d] = column -
// row), stored diagonal by diagonal: val[d * n + r] = A(r, r + off[d]), zero
// where r + off[d] falls outside the matrix or the entry is not stored.
template <class T> struct DiaView {
  int ndiag;
  int off[kMaxDiag];
  const T* val;
  // diagonals whose stored entries are one value wherever the diagonal lies
  // in the matrix (bit d of cmask; the value in cval[d]): the step kernel
  // takes that value from here instead of reading its stream
  unsigned cmask;
  T cval[kMaxDiag];
};

// Record of one Arnoldi step, written by the least-squares kernels with
// plain stores (host-mapped memory; read by the host after the streams are
// synchronised).
struct StepRec {
  double sres;
  double nu;
  int32_t j;
  int32_t flags;  // 1 halt, 2 breakdown, 4 rank loss
  int32_t pad[2];
};

// Written once by the step that raises the halt flag: its fields, a
// system-scope fence, then seq (the host resets seq to -1 and waits for it).
struct HaltRec {
  double sres;
  int32_t j;
  int32_t flags;
  int32_t seq;
  int32_t pad;
};

// Device control block of a cycle.
struct Ctrl {
  int32_t halt;     // != 0: step kernels return immediately
  int32_t halt_j;
  int32_t flags;
  int32_t mode;     // residual control: 0 safety factor, 1 Givens estimate
  double thresh;    // tol_abs / safety (mode 0), tol_abs (mode 1)
  // Givens estimate (mode 1): eps, the running estimate of the true
  // residual and the previous step's sketched residual (its sine is the
  // ratio of consecutive sketched residuals).  Written by the least-squares
  // kernels on their stream, and by the host's resume after a check.
  double eps, est, sprev;
};

// Residual control of a cycle start, for the least-squares init: mode, eps
// and ||r0|| (the estimate's anchor when no recycled block precedes V).
struct GivensInit {
  int mode;
  double eps;
  double beta;
};

// Work arrays of the block least squares on several workgroups (device,
// allocated by the solver): the block W (s x 8, ld s; then Q1, then W2),
// the projections P (rows x 8, row major), the in-block factors R1 and R2
// (8 x 8, column major), and the block's step headers (H columns, norms,
// breakdown flags, column norms of W).
template <class A> struct BlkWork {
  A* W = nullptr;
  A* P = nullptr;
  A* R1 = nullptr;
  A* R2 = nullptr;
  A* hc = nullptr;      // 8 x (kMaxWindow + 1)
  double* nuj = nullptr;
  double* n0 = nullptr;
  int* brk = nullptr;
};

// Small dense state of the sketched least squares (FP64 / complex128).
template <class A> struct LsqState {
  A* Q;    int ldq;   // s x Lmax orthonormal factor of SAW
  A* R;    int ldr;   // Lmax x Lmax upper triangular, column major
  A* z;               // Q^H S r0
  A* rho;             // S r0 - Q Q^H S r0 (projected sketched residual)
  A* SB;   int ldsb;  // [SU, SV]       s x (khat + m + 1)
  A* SAW;  int ldsaw; // [SAU, SAV]     s x (khat + m)
  A* H;    int ldh;   // (m+1) x m Hessenberg (banded), column major
  double* nu;         // norms of the stored basis vectors p_i
  double* sres_hist;
  Ctrl* ctrl;
  StepRec* rec;       // host-mapped records, one per step
  HaltRec* halt;      // host-mapped record of the halting step
  BlkWork<A> bw;      // the block least squares' work arrays
};

// w = A x (if spmv) with per-block partial sums in part (nb blocks of
// kRowsSpmv rows), columns: S x (sk.s of them, unscaled sparse-sign sums) and
// ||x||^2 when sk.s > 0, then <p_q, w> for the tw window vectors and ||w||^2.
// With sk.s = 0 only the window products and ||w||^2 are written; with spmv
// false only the sketch and ||x||^2 (w, win unused).  With events e0/e1 the
// dispatch records its own start and end (kernel timing).
template <class T>
void launch_spmv_sketch(hipStream_t st, int n, const int* rp, const int* ci, const T* val, const T* x,
                        T* w, Window<T> win, int tw, SketchSpec sk, bool spmv,
                        typename traits<T>::acc* part, int nb, const Ctrl* ctrl,
                        hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// The same kernel for a matrix in diagonal storage: w = A x with x read at
// the shifted row r + off[d] (coalesced for every diagonal), no index arrays.
template <class T>
void launch_spmv_dia_sketch(hipStream_t st, int n, DiaView<T> A, const T* x, T* w, Window<T> win, int tw,
                            SketchSpec sk, bool spmv, typename traits<T>::acc* part, int nb,
                            const Ctrl* ctrl, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// dst[map[e]] = src[e] rounded to T (CSR values into diagonal storage; the
// other positions of dst keep their zeros).
template <class T>
void launch_pack_dia(hipStream_t st, int64_t nnz, const typename traits<T>::acc* src, const int* map,
                     T* dst);
// Constant diagonals of a packed matrix: flags[d] = 1 and vals[d] = the value
// when every entry of diagonal d inside the matrix has the same bits.
template <class T>
void launch_dia_const(hipStream_t st, int n, DiaView<T> M, int* flags, T* vals);

// Prologue: nu[jprev] = ||p_jprev|| and d_q from this step's SpMV partials
// (part, nb1 blocks, sketch length s: columns s, s+1 .. s+tw).  Then
// w <- (w - sum_q (d_q / nu_{i0+q}^2) p_{i0+q}) / nu[jprev] in place.
template <class T>
void launch_update(hipStream_t st, int n, T* w, Window<T> win, int tw,
                   const typename traits<T>::acc* part, int nb1, int s, double* nu, int i0, int jprev,
                   const Ctrl* ctrl, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// out = [reduced columns of pa (first nscaled scaled by scl), reduced columns of pb].
template <class A>
void launch_reduce2(hipStream_t st, const A* pa, int nba, int ca, int nscaled, double scl,
                    const A* pb, int nbb, int cb, A* out, const Ctrl* ctrl);

// nu[0] and SV(:, 0) from a reduced sketch of p_0 ([s values, ||p_0||^2]).
template <class A>
void launch_init_v0(hipStream_t st, const A* red, int s, A* svcol, double* nu);

// out[c] = scale_c * sum_b part[c * nb + b] (fixed order); scale 1/sqrt(zeta) for c < nscaled.
// With mirror (host-mapped coherent memory) the sums are also stored there.
template <class A>
void launch_reduce_cols(hipStream_t st, const A* part, int nb, int ncols, int nscaled,
                        double scale, A* out, const Ctrl* ctrl, A* mirror = nullptr);

// One Arnoldi step's small work: H column, SV column, SAV column, QR append,
// projected residual and the halt decision.
// red: [S p_j (s), ||p_j||^2, window products (tw), ||A p_{j-1}||^2]; the
// first two come from step j+1's SpMV partials, the others from step j's.
template <class A>
void launch_lsq_step(hipStream_t st, LsqState<A> S, int j, int khat, int m, int t, int s,
                     const A* red, double brtol, double rank_rtol);

// Steps j0 .. j1 of the least squares, step j reading its reduced inputs at
// redb + slotr * (j % nslot) (layout of launch_lsq_step's red).  kind 0: one
// launch with the QR factor held in registers where the register shape
// allows, else block Gram-Schmidt over several workgroups (blocks of up to 8
// steps, seven launches per block), else in one workgroup; kind 1: block
// Gram-Schmidt in one workgroup (one launch); kind 2: one launch per step;
// kind 3: the several-workgroup block kernels.  A shape the chosen kernel
// cannot take falls back to one launch per step.  Stops after a step that raises the
// halt flag.
template <class A>
void launch_lsq_steps(hipStream_t st, LsqState<A> S, int j0, int j1, int khat, int m, int t, int s,
                      const A* redb, int64_t slotr, int nslot, double brtol, double rank_rtol,
                      int kind = 0);

// The reduced inputs of steps j0 .. j1 into their slots of redb (slot
// j % nslot): [S p_j scaled by scl, ||p_j||^2] from the SpMV partial slot of
// step j+1, then [<p_q, w> (tw), ||w||^2] from the slot of step j.
template <class A>
void launch_reduce_steps(hipStream_t st, const A* part1, int64_t slot1, int nb1, int s, int j0, int j1,
                         int t, int nslot, double scl, A* redb, int64_t slotr, const Ctrl* ctrl);

// Initialise the QR of SAW with its first khat columns (SAU) and rho = S r0.
// Also seeds the control block's residual estimate (gv.mode 1) and writes
// the sketched residual over span(U) alone to the step record 0.  kind as
// for launch_lsq_steps: the register kernel or the several-workgroup block
// kernels where the steps take them, else one workgroup.
template <class A>
void launch_lsq_init(hipStream_t st, LsqState<A> S, int khat, int s, const A* Sr,
                     double rank_rtol, int m, GivensInit gv, int kind = 0);

// y = R(0:n,0:n)^{-1} z(0:n); coefficients for [U, P]: y_i (U part), y_i / nu_i (P part).
template <class A>
void launch_backsolve(hipStream_t st, LsqState<A> S, int n, int khat, A* ycoef);

// One kept row of the subsampled randomised DCT sketch S = sqrt(N/s) P F E
// (Section 6), with what its kernel needs to run the cosines cos(phi + q b)
// along the entries, b = pi p / N, by Reinsch's two-term recurrence (c += d,
// d -= lam c): for b <= pi/2 directly; for b > pi/2 as (-1)^q cos(phi - q b')
// with b' = pi - b, so that lam = 4 sin^2(b'/2) stays small.  sh, ch: sin and
// cos of b'/2; a: the row's scale sqrt(N/s) c_p; out: its output row (rows
// are processed grouped by mode).
struct DctRow {
  int64_t p;
  double lam, sh, ch, a;
  int32_t out, mode;  // mode 1: the alternating form (b > pi/2)
};
struct DctSpec {
  const DctRow* rows;  // s rows, device
  int s;
  int64_t n4;          // 4 N: phases p (2r + 1) are reduced mod 4N exactly
  double ang;          // pi / (2N)
  uint64_t sign_seed;  // seed of E's signs (SplitMix64 keys, bit 0)
};

// S x for the subsampled DCT: per-tile partial sums (tiles of kRowsSpmv rows,
// those of the step kernels) into rows 0 .. s-1 of part, the rows already
// scaled; with with_norm also ||x||^2 into row s (nb = ceil(n / kRowsSpmv)).
template <class X>
void launch_dct_sketch(hipStream_t st, int n, const X* x, DctSpec d, typename traits<X>::acc* part, int nb,
                       bool with_norm, const Ctrl* ctrl, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Batched sketch of cc columns of X (ld) plus column norms: partials
// [(cc*s + cc) x nb], then reduced by launch_reduce_cols.
template <class X>
void launch_sketch_cols(hipStream_t st, int n, const X* x, int64_t ld, int cc, SketchSpec sk,
                        typename traits<X>::acc* part, int nb);

// xt = U yU + P yP (ku + jp columns), output in the accumulation type.
template <class T>
void launch_gemv_basis(hipStream_t st, int n, const T* U, int64_t ldu, int ku, const T* P,
                       int64_t ldp, int jp, const typename traits<T>::acc* y,
                       typename traits<T>::acc* out);

// rnew = r0 - A x (full precision values), nb = ceil(n/kRowsUpdate) blocks.
// Partials per block: with sk.s > 0 the sketch of rnew in rows 0 .. s-1 and
// ||rnew||^2 in row s (k_sketch_cols' layout for one column, the same sums
// in the same order); with sk.s = 0 ||rnew||^2 in row 0.
template <class A>
void launch_spmv_residual(hipStream_t st, int n, const int* rp, const int* ci, const A* val,
                          const A* x, const A* r0, A* rnew, A* part, int nb, SketchSpec sk);

// The same with A in diagonal storage (values in the accumulation type).
template <class A>
void launch_spmv_dia_residual(hipStream_t st, int n, DiaView<A> M, const A* x, const A* r0, A* rnew, A* part,
                              int nb, SketchSpec sk);

// Row width of G for launch_gemm_basis: kc rounded up to a multiple of 8.
int gemm_basis_width(int kc);

// C = [U P] G (n x kc), G (ku + jp) x kc stored row major with
// gemm_basis_width(kc) entries a row, zero beyond column kc.
template <class T>
void launch_gemm_basis(hipStream_t st, int n, const T* U, int64_t ldu, int ku, const T* P,
                       int64_t ldp, int jp, const typename traits<T>::acc* G, int kc, T* C,
                       int64_t ldc);

// C (M x N) = op(A) B with op(A) = A^H (A stored K x M) or A (M x K); small sizes.
// y = R^{-1} z over the leading nls columns of the upper triangular R (ld
// ldr), scaled into coefficients of the stored basis: y_i for i < khat,
// y_i / nu[i - khat] after.  One wavefront on stream st.  Returns false
// (nothing launched) when nls > 512.
template <class A>
bool launch_back_subst(hipStream_t st, int nls, int khat, const A* R, int ldr, const A* z, const double* nu,
                       A* y);

// Ri = R^{-1} for the upper triangular n x n leading block of R (ld ldr),
// one wavefront per column, and fro2[j] = ||Ri(:, j)||^2; false (nothing
// launched) when n exceeds 512.
template <class A>
bool launch_tri_inverse(hipStream_t st, int n, const A* R, int ldr, A* Ri, int ldri, double* fro2);

template <class A>
void launch_small_gemm(hipStream_t st, bool conjtrans, int M, int N, int K, const A* a, int lda,
                       const A* b, int ldb, A* c, int ldc);

template <class A> void launch_axpy(hipStream_t st, int n, A alpha, const A* x, A* y);
// Right Jacobi preconditioning A D^-1, D = diag(A): d[r] = A(r, r) (zero if
// row r stores no diagonal entry, which sets *flag to 1) and
// scaled[e] = val[e] * (1 / d[col[e]]).
template <class A>
void launch_jacobi(hipStream_t st, int n, int64_t nnz, const int* rp, const int* ci, const A* val, A* d,
                   A* scaled, int* flag);
// x <- x * d (divide false) or x * (1 / d) (divide true), elementwise.
template <class A>
void launch_scale_by_diag(hipStream_t st, int n, const A* d, A* x, bool divide);

// ILU(0) right preconditioning in a multicolour elimination order (Section 6
// preconditions by ILU; zero fill and the greedy colour order are readings).
// The factors live on A's own entries: F[e] is l_ik for an entry left of the
// diagonal in the elimination order (kind 0), u_ii (kind 1) or u_ij (kind 2).
// Rows of one colour are never neighbours, so the factorisation and both
// triangular solves advance a colour per launch.
struct IluView {
  int n = 0;
  int ncolours = 0;
  const int* crow = nullptr;     // the rows, colour by colour (device)
  const int* coff = nullptr;     // ncolours + 1 offsets into crow (host)
  const int* rp = nullptr;       // A's pattern (device)
  const int* ci = nullptr;
  const uint8_t* kind = nullptr; // per entry: 0 lower, 1 diagonal, 2 upper
  const int* dpos = nullptr;     // per row: its diagonal entry
  const void* F = nullptr;       // factor values, A's value type
  // The factors packed for the solves, by colour in sliced ELL form (64 rows
  // of a colour per slice; a slice's entries column-major, so lane l of a
  // wave reads row l of every entry column): the entries left of the
  // diagonal for the forward solve of colours 1.., right of it for the
  // backward solve of colours ..C-2.  Padding has value 0 and column 0.
  const int* lslice = nullptr;   // per slice: first packed slot (host index by colour: lsl0)
  const int* lw = nullptr;       // per slice: width
  const int* lcol = nullptr;
  const void* lval = nullptr;
  const int* uslice = nullptr;
  const int* uw = nullptr;
  const int* ucol = nullptr;
  const void* uval = nullptr;
  const int* lsl0 = nullptr;     // host: ncolours + 1 first slice of each colour (forward)
  const int* usl0 = nullptr;     // host: ncolours + 1 (backward)
  const void* dinv = nullptr;    // 1 / u_ii by position in crow
};

// The elimination, colour by colour: per row, its entries left of the
// diagonal in elimination order, lo[l] = (entry (i,k), diagonal entry of k),
// each followed by its updates up[up_off[l] .. up_off[l+1]) = (target entry
// (i,j), source entry (k,j)).  F holds A's values on entry and the factors on
// return; *flag is set if a pivot is zero.
template <class A>
void launch_ilu_factor(hipStream_t st, const IluView& v, const int* lo_off, const int2* lo, const int* up_off,
                       const int2* up, A* F, int* flag);

// The packed copies of the factors (lval, uval from F through the slot maps
// lsrc, usrc, -1 for padding) and dinv.
template <class A>
void launch_ilu_pack(hipStream_t st, const IluView& v, int64_t nl, const int* lsrc, int64_t nu,
                     const int* usrc);

// out = M^-1 in (forward solve with L into y, backward solve with U), one
// thread per row of a colour; y holds the forward solution (acc type).  With
// ctrl, a launch returns at once when its halt flag is set.
template <class T>
void launch_ilu_apply(hipStream_t st, const IluView& v, const T* in, typename traits<T>::acc* y, T* out,
                      const Ctrl* ctrl);

// out = M x = L (U x), t = U x.
template <class A>
void launch_ilu_mult(hipStream_t st, const IluView& v, const A* x, A* t, A* out);
// dst (T) = scale * src (acc type), rounding to T; with ctrl, the control
// block is also reset for a new cycle (not halted, threshold thresh).
template <class T>
void launch_cast_scale(hipStream_t st, int n, const typename traits<T>::acc* src, double scale,
                       T* dst, Ctrl* ctrl = nullptr, double thresh = 0.0);
// The same with scale = 1 / sqrt(Re nrm2[0]) read on the device (1 if that
// is not positive): the norm of a reduction still on the device.
template <class T>
void launch_cast_rscale(hipStream_t st, int n, const typename traits<T>::acc* src,
                        const typename traits<T>::acc* nrm2, T* dst, Ctrl* ctrl = nullptr,
                        double thresh = 0.0);
// dst (T) = src (T) cast from full precision A values (matrix copy)
template <class T>
void launch_narrow_values(hipStream_t st, int64_t n, const typename traits<T>::acc* src, T* dst);
template <class A>
void launch_gather_conj(hipStream_t st, int64_t nnz, const A* src, const int* perm, A* dst);
template <class A>
void launch_grad_values(hipStream_t st, int n, const int* rp, const int* ci, const A* lam,
                        const A* x, A* g);
// widen T -> acc (for basis inspection)
template <class T>
void launch_widen_scale(hipStream_t st, int n, const T* src, double scale,
                        typename traits<T>::acc* dst);

void launch_set_ctrl(hipStream_t st, Ctrl* c, int halt, double thresh);
// Resume under the Givens control: halt cleared, threshold tol, eps and the
// estimate restarted from the true residual est at the step whose sketched
// residual is sprev.
void launch_set_ctrl_givens(hipStream_t st, Ctrl* c, double thresh, double eps, double est, double sprev);

}  // namespace sdr
