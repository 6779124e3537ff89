// GMRES-SDR host driver and C interface.
//
// One restart cycle follows Algorithm 1 for A x = r0 with the readings listed
// in the library documentation: m Arnoldi steps on top of the recycle block
// U, truncated orthogonalisation against the last t vectors, one sketch per
// step, the sketched least squares updated by one QR column per step, the
// safety-factor residual control of Section 3.4, and the sketched
// harmonic-Ritz update of U, SU, SAU after every cycle (Section 3.5).  The
// restart loop applies x += xt, r = r0 - A xt (Section 3.6 for sequences).
//
// The Arnoldi steps are queued on the stream ahead of the host; each step's
// least-squares kernel writes its sketched residual to host-mapped memory and
// raises a device halt flag when a true-residual check is due, which turns the
// queued steps behind it into no-ops.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <condition_variable>
#include <type_traits>
#include <future>
#include <mutex>
#include <thread>
#include <memory>
#include <string>
#include <vector>

#include "../../include/sdr.h"
#include "dense.h"
#include "sdr_kernels.h"

using namespace sdr;

namespace {

thread_local std::string g_err;

void set_err(const std::string& s) { g_err = s; }

struct HipError {
  int code;
};

#define HIPCHK(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) {                                                                \
      set_err(std::string("HIP error ") + hipGetErrorString(e_) + " at " #call);          \
      throw HipError{SDR_EDEVICE};                                                         \
    }                                                                                      \
  } while (0)

#define LAUNCHCHK() HIPCHK(hipGetLastError())

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <class P>
P* dalloc(size_t count) {
  if (count == 0) count = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, count * sizeof(P));
  if (e != hipSuccess) {
    set_err(std::string("hipMalloc failed: ") + hipGetErrorString(e));
    throw HipError{SDR_ENOMEM};
  }
  return static_cast<P*>(p);
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

struct Options {
  int zeta = 8;
  int max_cycles = 10000;
  double safety0 = 1.4;
  bool persist_safety = false;
  int precision = 0;
  int variant = 0;
  double brtol = -1.0;  // < 0: default for the basis precision
  double rank_rtol = 1e-12;
  int lsq_chunk = 8;      // steps per least-squares launch
  int lsq_kernel = 0;     // 0: register kernel where the shape allows, else block; 1: block in one
                          // workgroup; 2: per step; 3: block over several workgroups
  int kernel_timing = 0;  // 0: off; n: time the SpMV and update kernels of every n-th step
  int dia = 1;            // 1: diagonal storage for stencil patterns; 0: always CSR
  int dia_const = -1;     // 1: constant diagonals passed to the step kernel as values; 0: read;
                          // -1: 1 for complex data (their 16-byte streams), 0 for real
  int precond = 0;        // 0: none; 1: right Jacobi (A D^-1); 2: right ILU(0), multicolour order
  int resid_control = 0;  // 0: safety factor (Section 3.4); 1: Givens estimate (Sections 4.5, 5)
  int sketch = 0;         // 0: sparse sign; 1: subsampled randomised DCT (Section 6)
  double givens_eps0 = 0.0;  // initial eps of the Givens estimate
};

// Diagonal layout of a CSR pattern: the distinct offsets column - row (at
// most kMaxDiag, sorted) and, per stored entry, its position d * n + row in
// diagonal storage.  Refused (false) for more offsets, for diagonals padded
// beyond a quarter of nnz, for repeated entries or an index range past int32.
bool dia_layout(int n, const std::vector<int>& rp, const std::vector<int>& ci, std::vector<int>* offs,
                std::vector<int>* map) {
  const int64_t nnz = (int64_t)ci.size();
  std::vector<int> o;
  for (int r = 0; r < n; ++r)
    for (int e = rp[r]; e < rp[r + 1]; ++e) {
      const int off = ci[e] - r;
      if (std::find(o.begin(), o.end(), off) == o.end()) {
        if ((int)o.size() == kMaxDiag) return false;
        o.push_back(off);
      }
    }
  if (o.empty() || (int64_t)o.size() * n > nnz + nnz / 4 || (int64_t)o.size() * n >= ((int64_t)1 << 31))
    return false;
  std::sort(o.begin(), o.end());
  std::vector<char> seen((size_t)o.size() * n, 0);
  map->assign((size_t)nnz, 0);
  for (int r = 0; r < n; ++r)
    for (int e = rp[r]; e < rp[r + 1]; ++e) {
      const int d = (int)(std::lower_bound(o.begin(), o.end(), ci[e] - r) - o.begin());
      const int64_t pos = (int64_t)d * n + r;
      if (seen[pos]) return false;
      seen[pos] = 1;
      (*map)[e] = (int)pos;
    }
  *offs = o;
  return true;
}

// Matrix view (device, full precision values).
template <class A>
struct MatView {
  int n = 0;
  int64_t nnz = 0;
  const int* rp = nullptr;
  const int* ci = nullptr;
  const A* val = nullptr;
};

inline double to_double_re(double v) { return v; }
inline double to_double_re(cx<double> v) { return v.x; }

template <class A> A from_cd(std::complex<double> z);
template <> double from_cd<double>(std::complex<double> z) { return z.real(); }
template <> cx<double> from_cd<cx<double>>(std::complex<double> z) { return {z.real(), z.imag()}; }
inline std::complex<double> to_cd(double v) { return {v, 0.0}; }
inline std::complex<double> to_cd(cx<double> v) { return {v.x, v.y}; }

struct SolverBase {
  virtual ~SolverBase() {}
  virtual int solve(const void* b, void* x, double tol, sdr_stats* st,
                    std::vector<sdr_cycle_record>* trace) = 0;
  virtual void matrix_changed() = 0;
  virtual int get_recycle(void* U, void* SU, void* SAU, int* k) = 0;
  virtual int get_basis(int ncols, void* V, void* H, void* SV) = 0;
  virtual int step_sres(double* out, int cap) = 0;
  virtual int sketch(const void* X, int ncols, void* Y) = 0;
  virtual void set_stream(hipStream_t s) = 0;
  virtual void set_options(const Options& o) = 0;
  // Right ILU(0) preconditioning: the solver runs on A M^-1 (null: on A).
  virtual void set_ilu(const IluView* v) = 0;
  virtual void reset() = 0;
  virtual int kernel_times(double* ms, int64_t* counts, int cap) = 0;
  virtual int spmv_layout(int* offsets, int cap) = 0;
  virtual unsigned const_diagonals() const = 0;
};

template <class T>
class Solver final : public SolverBase {
 public:
  using A = typename traits<T>::acc;
  static constexpr bool kSame = sizeof(T) == sizeof(A);

  Solver(MatView<A> mat, int m, int k, int t, int s, uint64_t seed, const Options& opt,
         hipStream_t st)
      : M_(mat), m_(m), k_(k), t_(t), s_(s), opt_(opt), stream_(st) {
    n_ = mat.n;
    sk_.seed = seed;
    sk_.s = s;
    sk_.zeta = opt.zeta;
    sk_.bsz = s / opt.zeta;
    sk_.words = (opt.zeta + 3) / 4;
    dct_on_ = opt.sketch == 1;
    sk_.ext = dct_on_ ? 1 : 0;
    // the sparse sign's sums are scaled by 1/sqrt(zeta) when reduced; the DCT
    // kernel scales its own rows
    sk_scl_ = dct_on_ ? 1.0 : 1.0 / std::sqrt((double)opt.zeta);
    brtol_ = opt.brtol >= 0.0 ? opt.brtol : (kSame ? 1e-14 : 1e-6);
    nb1_ = (n_ + kRowsSpmv - 1) / kRowsSpmv;
    nb2_ = (n_ + kRowsUpdate - 1) / kRowsUpdate;
    kmax_ = k + 1;
    lmax_ = kmax_ + m + 1;
    const size_t N = (size_t)n_;
    try {
      Pbuf_[0] = dalloc<T>(N * (m + 1));
      Pbuf_[1] = dalloc<T>(N * (m + 1));
      P_ = Pbuf_[0];
      U_ = dalloc<T>(N * kmax_);
      Unew_ = dalloc<T>(N * kmax_);
      SU_ = dalloc<A>((size_t)s * kmax_);
      SAU_ = dalloc<A>((size_t)s * kmax_);
      Q_ = dalloc<A>((size_t)s * lmax_);
      R_ = dalloc<A>((size_t)lmax_ * lmax_);
      z_ = dalloc<A>(lmax_);
      rho_ = dalloc<A>(s);
      for (int b = 0; b < 2; ++b) {
        SBbuf_[b] = dalloc<A>((size_t)s * (lmax_ + 1));
        SAWbuf_[b] = dalloc<A>((size_t)s * lmax_);
      }
      SB_ = SBbuf_[0];
      SAW_ = SAWbuf_[0];
      H_ = dalloc<A>((size_t)(m + 1) * m);
      nu_ = dalloc<double>(m + 2);
      sres_hist_ = dalloc<double>(m + 2);
      ctrl_ = dalloc<Ctrl>(1);
      ctrl_free_ = dalloc<Ctrl>(1);
      nslot_ = m + 2;  // one partial slot per step: the least squares may lag a whole cycle
      // SpMV partial columns per step: S p_{j-1} (s), ||p_{j-1}||^2, window products, ||w||^2
      slot1_ = (size_t)(s + 1 + kMaxWindow + 1) * nb1_;
      slotr_ = (size_t)(s + 1 + kMaxWindow + 1);
      part1_ = dalloc<A>(slot1_ * nslot_);
      redb_ = dalloc<A>(slotr_ * nslot_);
      red0_ = dalloc<A>(s + 1);
      psk_ = dalloc<A>((size_t)(8 * s + 8 + 1) * nb2_);
      red2_ = dalloc<A>(8 * s + 8 + 1);
      if (dct_on_) build_dct(seed);
      HIPCHK(hipStreamCreateWithFlags(&streamB_, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&ev_copy_, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&ev_res_, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&ev_bs_, hipEventDisableTiming));
      evs_.assign(nslot_ + 1, nullptr);
      // Step events order stream B's least squares after stream A's SpMV
      // launches on the same device: a device-scope release suffices, and
      // the default system-scope fence (an L2 writeback each time) is skipped.
      for (auto& e : evs_) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventDisableSystemFence));
      red3_ = dalloc<A>(4);
      // the eigen-step's R^{-1} and R^{-1} C, formed on the device for complex data
      if (traits<T>::cpx) {
        Ri_ = dalloc<A>((size_t)lmax_ * lmax_);
        RiC_ = dalloc<A>((size_t)lmax_ * lmax_);
        fro2_ = dalloc<double>(lmax_);
        HIPCHK(hipHostMalloc((void**)&hRiC_, sizeof(A) * (size_t)lmax_ * lmax_, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&hfro2_, sizeof(double) * lmax_, hipHostMallocDefault));
      }
      // block least-squares work: W (s x 8), P ((lmax + 8) x 8), R1, R2, the H columns
      blkA_ = dalloc<A>((size_t)s * 8 + (size_t)(lmax_ + 8) * 8 + 2 * 64 + 8 * (kMaxWindow + 1));
      blkD_ = dalloc<double>(16);
      blkI_ = dalloc<int>(8);
      Sr_ = dalloc<A>(s);
      ycoef_ = dalloc<A>(lmax_);
      xt_ = dalloc<A>(N);
      r_ = dalloc<A>(N);
      rnew_ = dalloc<A>(N);
      G_ = dalloc<A>((size_t)lmax_ * gemm_basis_width(kmax_));
      Gs_ = dalloc<A>((size_t)lmax_ * kmax_);
      C_ = dalloc<A>((size_t)lmax_ * lmax_);
      if (opt.kernel_timing) {
        for (auto& evp : ev_) {
          evp.assign(m + 2, std::array<hipEvent_t, 6>{});
          // (timing only: no system-scope fence at each record)
          for (auto& a : evp)
            for (auto& e : a) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        }
      }
      HIPCHK(hipHostMalloc((void**)&rec_host_, sizeof(StepRec) * (m + 2),
                           hipHostMallocMapped | hipHostMallocCoherent));
      HIPCHK(hipHostGetDevicePointer((void**)&rec_dev_, rec_host_, 0));
      HIPCHK(hipHostMalloc((void**)&halt_host_, sizeof(HaltRec), hipHostMallocMapped | hipHostMallocCoherent));
      HIPCHK(hipHostGetDevicePointer((void**)&halt_dev_, halt_host_, 0));
      HIPCHK(hipHostMalloc((void**)&hR_, sizeof(A) * (size_t)lmax_ * lmax_, hipHostMallocDefault));
      HIPCHK(hipHostMalloc((void**)&hC_, sizeof(A) * (size_t)lmax_ * lmax_, hipHostMallocDefault));
      HIPCHK(hipHostMalloc((void**)&hz_, sizeof(A) * (size_t)lmax_, hipHostMallocDefault));
      HIPCHK(hipHostMalloc((void**)&hy_, sizeof(A) * (size_t)lmax_, hipHostMallocDefault));
      HIPCHK(hipHostMalloc((void**)&hnu_, sizeof(double) * (size_t)(m + 2), hipHostMallocDefault));
      HIPCHK(hipHostMalloc((void**)&hRc_, sizeof(A) * (size_t)lmax_ * lmax_, hipHostMallocDefault));
      HIPCHK(hipHostMalloc((void**)&hnuc_, sizeof(double) * (size_t)(m + 2), hipHostMallocDefault));
      HIPCHK(hipHostMalloc((void**)&hG_, sizeof(A) * (size_t)lmax_ * (2 * kmax_ + gemm_basis_width(kmax_)),
                           hipHostMallocDefault));
      HIPCHK(hipHostMalloc((void**)&hscal_, sizeof(A) * 8, hipHostMallocDefault));
      HIPCHK(hipHostMalloc((void**)&hres_, sizeof(A) * 2, hipHostMallocMapped | hipHostMallocCoherent));
      HIPCHK(hipHostGetDevicePointer((void**)&hres_dev_, hres_, 0));
      HIPCHK(hipMemsetAsync(ctrl_free_, 0, sizeof(Ctrl), stream_));
      HIPCHK(hipMemsetAsync(nu_, 0, sizeof(double) * (m + 2), stream_));
      HIPCHK(hipMemsetAsync(H_, 0, sizeof(A) * (m + 1) * m, stream_));
      HIPCHK(hipStreamSynchronize(stream_));
      HIPCHK(hipMemsetAsync(redb_, 0, sizeof(A) * slotr_ * nslot_, stream_));
      HIPCHK(hipStreamSynchronize(stream_));
      if (opt.dia) {
        std::vector<int> rp(n_ + 1), ci((size_t)mat.nnz), offs, map;
        HIPCHK(hipMemcpy(rp.data(), mat.rp, sizeof(int) * (n_ + 1), hipMemcpyDeviceToHost));
        if (mat.nnz) HIPCHK(hipMemcpy(ci.data(), mat.ci, sizeof(int) * mat.nnz, hipMemcpyDeviceToHost));
        if (mat.nnz && dia_layout(n_, rp, ci, &offs, &map)) {
          dia_.ndiag = (int)offs.size();
          for (int d = 0; d < dia_.ndiag; ++d) dia_.off[d] = offs[d];
          dia_map_ = dalloc<int>(map.size());
          diaval_ = dalloc<T>((size_t)dia_.ndiag * n_);
          HIPCHK(hipMemcpy(dia_map_, map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice));
          // Null-stream copies need not have reached the device when they
          // return, and the solver's kernels run on non-blocking streams:
          // finish the copy, then zero the padding on the solver's stream.
          HIPCHK(hipStreamSynchronize(nullptr));
          HIPCHK(hipMemsetAsync(diaval_, 0, sizeof(T) * (size_t)dia_.ndiag * n_, stream_));
          HIPCHK(hipStreamSynchronize(stream_));
          dia_.val = diaval_;
          dcflag_ = dalloc<int>(kMaxDiag);
          dcval_ = dalloc<T>(kMaxDiag);
        }
      }
      if (!kSame && !dia()) valB_ = dalloc<T>((size_t)mat.nnz);  // CSR values in the basis precision
    } catch (...) {
      release();
      throw;
    }
    low_dirty_ = true;
  }

  ~Solver() override { release(); }

  void set_stream(hipStream_t s) override { stream_ = s; }

  // Options that may change between solves (the others are refused once the
  // solver exists).
  void set_options(const Options& o) override {
    opt_.max_cycles = o.max_cycles;
    opt_.safety0 = o.safety0;
    opt_.persist_safety = o.persist_safety;
    opt_.resid_control = o.resid_control;
    opt_.givens_eps0 = o.givens_eps0;
    opt_.lsq_kernel = o.lsq_kernel;
  }

  void set_ilu(const IluView* v) override {
    ilu_ = v;
    if (v && !izb_) {
      izb_ = dalloc<T>(n_);
      iy_ = dalloc<A>(n_);
      izA_ = dalloc<A>(n_);
      iyA_ = dalloc<A>(n_);
    }
  }

  void set_matrix(MatView<A> mat) { M_ = mat; }

  void matrix_changed() override {
    low_dirty_ = true;
    if (opt_.variant == 0) sau_stale_ = true;
  }

  bool dia() const { return dia_.ndiag > 0; }

  // After a packing: which diagonals hold one value inside the matrix (the
  // host waits for the answer, once per matrix change; the step kernel then
  // takes those values from its arguments).
  void find_constant_diagonals() {
    dia_.cmask = 0;
    if (opt_.dia_const == 0 || (opt_.dia_const < 0 && !traits<T>::cpx)) return;
    launch_dia_const<T>(stream_, n_, dia_, dcflag_, dcval_);
    LAUNCHCHK();
    int fl[kMaxDiag] = {};
    T cv[kMaxDiag];
    HIPCHK(hipMemcpyAsync(fl, dcflag_, sizeof(int) * dia_.ndiag, hipMemcpyDeviceToHost, stream_));
    HIPCHK(hipMemcpyAsync(cv, dcval_, sizeof(T) * dia_.ndiag, hipMemcpyDeviceToHost, stream_));
    HIPCHK(hipStreamSynchronize(stream_));
    for (int d = 0; d < dia_.ndiag; ++d)
      if (fl[d]) {
        dia_.cmask |= 1u << d;
        dia_.cval[d] = cv[d];
      }
  }

  unsigned const_diagonals() const override { return dia_.cmask; }

  // Matrix values for the basis SpMV: diagonal storage (packed on change) or
  // CSR values in the basis precision.
  const T* basis_values() {
    if (dia()) {
      if (low_dirty_) {
        launch_pack_dia<T>(stream_, M_.nnz, M_.val, dia_map_, diaval_);
        LAUNCHCHK();
        low_dirty_ = false;
        find_constant_diagonals();
      }
      return diaval_;
    }
    if (kSame) return reinterpret_cast<const T*>(M_.val);
    if (low_dirty_) {
      launch_narrow_values<T>(stream_, M_.nnz, M_.val, valB_);
      LAUNCHCHK();
      low_dirty_ = false;
    }
    return valB_;
  }

  // The subsampled randomised DCT S = sqrt(N/s) P F E (Section 6): the kept
  // rows P are the s indices with the smallest SplitMix64 keys of seed ^
  // kDctRowSalt (ties by index), in increasing order; E's sign of row r is
  // bit 0 of the key of seed ^ kDctSignSalt.  Per kept row the kernel needs
  // its frequency, the phase step pi p / N and the scale sqrt(N/s) c_p.
  void build_dct(uint64_t seed) {
    static constexpr uint64_t kDctSignSalt = 0x5851F42D4C957F2Dull;
    static constexpr uint64_t kDctRowSalt = 0x14057B7EF767814Full;
    if (s_ > n_) {
      set_err("the subsampled DCT sketch needs s_dim <= n");
      throw HipError{SDR_EINVAL};
    }
    std::vector<std::pair<uint64_t, int>> keys(n_);
    const uint64_t base = seed ^ kDctRowSalt;
    for (int i = 0; i < n_; ++i) keys[i] = {mix64(base + kGamma * (uint64_t)(i + 1)), i};
    std::nth_element(keys.begin(), keys.begin() + (s_ - 1), keys.end());
    std::vector<int> rows(s_);
    for (int i = 0; i < s_; ++i) rows[i] = keys[i].second;
    std::sort(rows.begin(), rows.end());
    std::vector<DctRow> h(s_);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < s_; ++i) {
      const int p = rows[i];
      // step b = pi p / N; b > pi/2 (2p > N) runs the alternating form with b' = pi - b
      const int mode = 2 * (int64_t)p > (int64_t)n_ ? 1 : 0;
      const double half = pi * (double)(mode ? n_ - p : p) / (2.0 * n_);  // b/2 or b'/2
      h[i].p = p;
      h[i].sh = std::sin(half);
      h[i].ch = std::cos(half);
      h[i].lam = 4.0 * h[i].sh * h[i].sh;
      h[i].a = std::sqrt((double)n_ / s_) * (p == 0 ? std::sqrt(1.0 / n_) : std::sqrt(2.0 / n_));
      h[i].out = i;
      h[i].mode = mode;
    }
    // processed grouped by mode, so that a wavefront's lanes read one LDS array
    std::stable_sort(h.begin(), h.end(), [](const DctRow& a, const DctRow& b) { return a.mode < b.mode; });
    dct_rows_ = dalloc<DctRow>(s_);
    HIPCHK(hipMemcpy(dct_rows_, h.data(), sizeof(DctRow) * s_, hipMemcpyHostToDevice));
    dct_.rows = dct_rows_;
    dct_.s = s_;
    dct_.n4 = 4 * (int64_t)n_;
    dct_.ang = pi / (2.0 * n_);
    dct_.sign_seed = seed ^ kDctSignSalt;
  }

  // out[c] = S X(:, c) for c < nc (X with leading dimension n), norms^2 in nrm2.
  template <class X>
  void sketch_cols(const X* x, int nc, A* out, int ldo, double* nrm2) {
    sr_of_ = nullptr;  // (the partials below replace a residual's sketch)
    if (dct_on_) {
      for (int c = 0; c < nc; ++c) {
        launch_dct_sketch<X>(stream_, n_, x + (size_t)c * n_, dct_, psk_, nb1_, true, nullptr);
        LAUNCHCHK();
        launch_reduce_cols<A>(stream_, psk_, nb1_, s_ + 1, s_, 1.0, red2_, nullptr);
        LAUNCHCHK();
        HIPCHK(hipMemcpyAsync(out + (size_t)c * ldo, red2_, sizeof(A) * s_, hipMemcpyDeviceToDevice, stream_));
        if (nrm2) {
          HIPCHK(hipMemcpyAsync(hscal_, red2_ + s_, sizeof(A), hipMemcpyDeviceToHost, stream_));
          HIPCHK(hipStreamSynchronize(stream_));
          nrm2[c] = to_double_re(hscal_[0]);
        }
      }
      return;
    }
    const int maxcc = std::max(1, std::min(8, (int)(48 * 1024 / (kWaves * s_ * sizeof(A)))));
    for (int c0 = 0; c0 < nc; c0 += maxcc) {
      const int cc = std::min(maxcc, nc - c0);
      launch_sketch_cols<X>(stream_, n_, x + (size_t)c0 * n_, (int64_t)n_, cc, sk_, psk_, nb2_);
      LAUNCHCHK();
      launch_reduce_cols<A>(stream_, psk_, nb2_, cc * s_ + cc, cc * s_,
                            sk_scl_, red2_, nullptr);
      LAUNCHCHK();
      for (int c = 0; c < cc; ++c)
        HIPCHK(hipMemcpyAsync(out + (size_t)(c0 + c) * ldo, red2_ + (size_t)c * s_, sizeof(A) * s_,
                              hipMemcpyDeviceToDevice, stream_));
      if (nrm2) {
        HIPCHK(hipMemcpyAsync(hscal_, red2_ + (size_t)cc * s_, sizeof(A) * cc,
                              hipMemcpyDeviceToHost, stream_));
        HIPCHK(hipStreamSynchronize(stream_));
        for (int c = 0; c < cc; ++c) nrm2[c0 + c] = to_double_re(hscal_[c]);
      }
    }
  }

  int sketch(const void* X, int ncols, void* Y) override {
    sketch_cols<A>(static_cast<const A*>(X), ncols, static_cast<A*>(Y), s_, nullptr);
    HIPCHK(hipStreamSynchronize(stream_));
    return SDR_OK;
  }

  // r = b - A x and ||r||^2 to the host, queued on stream A; finish_residual()
  // waits for it.
  void enqueue_residual(const A* x, const A* b, A* r) {
    // The residual kernel also sketches r (when its bins fit), so that a
    // cycle starting from r reduces these partials instead of sketching r
    // in a pass of its own.  Right ILU(0): r = b - A (M^-1 x).
    if (ilu_) {
      launch_ilu_apply<A>(stream_, *ilu_, x, iyA_, izA_, nullptr);
      LAUNCHCHK();
      x = izA_;
    }
    const bool fuse = !dct_on_ && (size_t)kWaves * s_ * sizeof(A) <= 48 * 1024;
    SketchSpec skr = sk_;
    if (!fuse) skr.s = 0;
    if constexpr (std::is_same<T, A>::value) {
      // the diagonal storage holds the matrix in full precision: same sums
      if (dia()) {
        (void)basis_values();  // (packed if the values changed)
        launch_spmv_dia_residual<A>(stream_, n_, dia_, x, b, r, psk_, nb2_, skr);
      } else {
        launch_spmv_residual<A>(stream_, n_, M_.rp, M_.ci, M_.val, x, b, r, psk_, nb2_, skr);
      }
    } else {
      launch_spmv_residual<A>(stream_, n_, M_.rp, M_.ci, M_.val, x, b, r, psk_, nb2_, skr);
    }
    LAUNCHCHK();
    sr_of_ = fuse ? r : nullptr;
    // ||r||^2 to red3_ (the next cycle's start scales by it on the device)
    // and straight into host-mapped memory for the host
    launch_reduce_cols<A>(stream_, psk_ + (size_t)skr.s * nb2_, nb2_, 1, 0, 1.0, red3_, nullptr, hres_dev_);
    LAUNCHCHK();
    HIPCHK(hipEventRecord(ev_res_, stream_));
  }
  double finish_residual() {
    HIPCHK(hipEventSynchronize(ev_res_));  // (not the stream: later work may be queued)
    return std::sqrt(to_double_re(hres_[0]));
  }
  double residual(const A* x, const A* b, A* r) {
    enqueue_residual(x, b, r);
    return finish_residual();
  }

  LsqState<A> lsq() {
    LsqState<A> S;
    S.Q = Q_;
    S.ldq = s_;
    S.R = R_;
    S.ldr = lmax_;
    S.z = z_;
    S.rho = rho_;
    // recycled columns right-aligned before column kmax: SV(:, i) sits at kmax + i
    S.SB = SB_ + (size_t)(kmax_ - khat_) * s_;
    S.ldsb = s_;
    S.SAW = SAW_ + (size_t)(kmax_ - khat_) * s_;
    S.ldsaw = s_;
    S.H = H_;
    S.ldh = m_ + 1;
    S.nu = nu_;
    S.sres_hist = sres_hist_;
    S.ctrl = ctrl_;
    S.rec = rec_dev_;
    S.halt = halt_dev_;
    S.bw.W = blkA_;
    S.bw.P = blkA_ + (size_t)s_ * 8;
    S.bw.R1 = S.bw.P + (size_t)(lmax_ + 8) * 8;
    S.bw.R2 = S.bw.R1 + 64;
    S.bw.hc = S.bw.R2 + 64;
    S.bw.nuj = blkD_;
    S.bw.n0 = blkD_ + 8;
    S.bw.brk = blkI_;
    return S;
  }

  // Arnoldi part of step j on stream A: the SpMV of p_{j-1} with its window
  // products and its sketch, an event for the least squares of step j-1,
  // then the update to p_j.  Step m+1 is the sketch of p_m alone.
  // With ev, an event after the SpMV for the least squares on stream B.
  void enqueue_step_a(int j, const T* vals, bool ev) {
    const int sl = j % nslot_;
    A* p1 = part1_ + slot1_ * sl;
    const T* x = P_ + (size_t)(j - 1) * n_;
    if (j > m_) {
      // sketch of p_m only (the diagonal-storage kernel's sketch pass needs far
      // less LDS than the CSR kernel's staging, so more of its blocks run at once)
      Window<T> none{};
      if (dct_on_) {  // S p_m and ||p_m||^2 by the DCT kernel
        launch_dct_sketch<T>(stream_, n_, x, dct_, p1, nb1_, true, ctrl_);
        LAUNCHCHK();
        HIPCHK(hipEventRecord(evs_[sl], stream_));
        return;
      }
      if (dia())
        launch_spmv_dia_sketch<T>(stream_, n_, dia_, x, nullptr, none, 0, sk_, false, p1, nb1_, ctrl_);
      else
        launch_spmv_sketch<T>(stream_, n_, M_.rp, M_.ci, vals, x, nullptr, none, 0, sk_, false, p1, nb1_,
                              ctrl_);
      LAUNCHCHK();
      HIPCHK(hipEventRecord(evs_[sl], stream_));
      return;
    }
    const int i0 = std::max(j - t_, 0);
    const int tw = j - i0;
    Window<T> win{};
    for (int q = 0; q < tw; ++q) win.p[q] = P_ + (size_t)(i0 + q) * n_;
    T* w = P_ + (size_t)j * n_;
    const bool tm = timed(j, evp_);
    hipEvent_t* te = tm ? ev_[evp_][j].data() : nullptr;
    // right ILU(0): the SpMV multiplies z = M^-1 p_{j-1}, the sketch and the
    // norm stay those of p_{j-1}
    const T* xin = x;
    SketchSpec skj = sk_;
    if (ilu_) {
      launch_ilu_apply<T>(stream_, *ilu_, x, iy_, izb_, ctrl_);
      LAUNCHCHK();
      xin = izb_;
      skj.src = x;
    }
    if (dia())
      launch_spmv_dia_sketch<T>(stream_, n_, dia_, xin, w, win, tw, skj, true, p1, nb1_, ctrl_,
                                tm ? te[0] : nullptr, tm ? te[1] : nullptr);
    else
      launch_spmv_sketch<T>(stream_, n_, M_.rp, M_.ci, vals, xin, w, win, tw, skj, true, p1, nb1_, ctrl_,
                            tm ? te[0] : nullptr, tm ? te[1] : nullptr);
    LAUNCHCHK();
    if (dct_on_) {  // S p_{j-1} into the sketch rows the step kernel left alone
      launch_dct_sketch<T>(stream_, n_, x, dct_, p1, nb1_, false, ctrl_, tm ? te[4] : nullptr,
                           tm ? te[5] : nullptr);
      LAUNCHCHK();
    }
    if (ev) HIPCHK(hipEventRecord(evs_[sl], stream_));
    launch_update<T>(stream_, n_, w, win, tw, p1, nb1_, s_, nu_, i0, j - 1, ctrl_,
                     tm ? te[2] : nullptr, tm ? te[3] : nullptr);
    LAUNCHCHK();
  }

  // Step j of a cycle of parity par is timed when (j + offset) is a multiple
  // of kernel_timing; the offset moves by 13 each cycle, so the samples
  // cover every step position rather than always the same one.
  bool timed(int j, int par) const {
    return opt_.kernel_timing > 0 && (j + ev_ofs_[par]) % opt_.kernel_timing == 0;
  }

  // Kernel times of a finished cycle, read while the GPU runs the next one
  // (the events alternate between two sets by cycle, so a set is read
  // before it is recorded again).
  void drain_timing() {
    if (ev_pend_j_ <= 0) return;
    auto& evs = ev_[ev_pend_p_];
    for (int j = 1; j <= ev_pend_j_; ++j) {
      if (!timed(j, ev_pend_p_)) continue;
      float a = 0.f, b2 = 0.f, c = 0.f;
      HIPCHK(hipEventElapsedTime(&a, evs[j][0], evs[j][1]));
      HIPCHK(hipEventElapsedTime(&b2, evs[j][2], evs[j][3]));
      HIPCHK(hipEventElapsedTime(&c, evs[j][0], evs[j][3]));
      kt_ms_[0] += a;
      kt_ms_[1] += b2;
      kt_ms_[2] += c;
      if (dct_on_) {
        float dd = 0.f;
        HIPCHK(hipEventElapsedTime(&dd, evs[j][4], evs[j][5]));
        kt_ms_[3] += dd;
      }
      kt_n_[0]++;
      kt_n_[1]++;
      kt_n_[2]++;
      kt_bytes_tw_[std::min(j, t_)]++;
    }
    ev_pend_j_ = 0;
  }

  // The least squares of steps j0 .. j1 runs behind the SpMV of step j1 + 1;
  // chunks start at base, base + chunk, ... so that only their last SpMV
  // records an event.
  bool needs_event(int j, int base) const {
    return j == m_ + 1 || (j > base && (j - base) % opt_.lsq_chunk == 0);
  }

  // Least squares of steps j0 .. j1 on stream B, behind the SpMV of step
  // j1 + 1 (which sketches p_{j1}); the window products of step j come from
  // step j's SpMV.
  void enqueue_chunk(int j0, int j1) {
    HIPCHK(hipStreamWaitEvent(streamB_, evs_[(j1 + 1) % nslot_], 0));
    launch_reduce_steps<A>(streamB_, part1_, (int64_t)slot1_, nb1_, s_, j0, j1, t_, nslot_,
                           sk_scl_, redb_, (int64_t)slotr_, ctrl_);
    launch_lsq_steps<A>(streamB_, lsq(), j0, j1, khat_, m_, t_, s_, redb_, (int64_t)slotr_, nslot_,
                        brtol_, opt_.rank_rtol, opt_.lsq_kernel);
    LAUNCHCHK();
  }

  void sync_both() {
    HIPCHK(hipStreamSynchronize(stream_));
    HIPCHK(hipStreamSynchronize(streamB_));
  }

  // Wait for the halt record; returns false if the streams drain without one.
  bool wait_halt(HaltRec& out) {
    long spins = 0;
    for (;;) {
      if (__atomic_load_n(&halt_host_->seq, __ATOMIC_ACQUIRE) >= 0) {
        volatile HaltRec* h = halt_host_;
        out.sres = h->sres;
        out.j = h->j;
        out.flags = h->flags;
        return true;
      }
      if (++spins % 4096 == 0) {
        const hipError_t qa = hipStreamQuery(stream_);
        const hipError_t qb = hipStreamQuery(streamB_);
        if (qa != hipSuccess && qa != hipErrorNotReady) {
          set_err(std::string("stream error: ") + hipGetErrorString(qa));
          throw HipError{SDR_EDEVICE};
        }
        if (qb != hipSuccess && qb != hipErrorNotReady) {
          set_err(std::string("stream error: ") + hipGetErrorString(qb));
          throw HipError{SDR_EDEVICE};
        }
        if (qa == hipSuccess && qb == hipSuccess) {
          if (__atomic_load_n(&halt_host_->seq, __ATOMIC_ACQUIRE) >= 0) continue;
          return false;
        }
      }
    }
  }

  // Queue the rest of the cycle from step j0: the Arnoldi steps (with
  // events at chunk ends) and the least-squares chunks behind them.
  // Chunks whose steps the chain has already finished (their events are
  // complete when queued, as after a late eigen-step) share one reduction
  // launch: the same sums per step, one bandwidth-bound pass instead of a
  // latency-bound launch per chunk.
  void enqueue_from(int j0, int& enqA, const T* vals) {
    const int base = j0;
    while (enqA < m_ + 1) {
      ++enqA;
      enqueue_step_a(enqA, vals, needs_event(enqA, base));
    }
    int done_to = j0 - 1;
    for (int c0 = j0; c0 <= m_; c0 += opt_.lsq_chunk) {
      const int c1 = std::min(c0 + opt_.lsq_chunk - 1, m_);
      if (hipEventQuery(evs_[(c1 + 1) % nslot_]) != hipSuccess) break;
      done_to = c1;
    }
    int c0 = j0;
    if (done_to > j0) {
      HIPCHK(hipStreamWaitEvent(streamB_, evs_[(done_to + 1) % nslot_], 0));  // (complete: no wait)
      launch_reduce_steps<A>(streamB_, part1_, (int64_t)slot1_, nb1_, s_, j0, done_to, t_, nslot_, sk_scl_,
                             redb_, (int64_t)slotr_, ctrl_);
      for (; c0 <= done_to; c0 += opt_.lsq_chunk)
        launch_lsq_steps<A>(streamB_, lsq(), c0, std::min(c0 + opt_.lsq_chunk - 1, m_), khat_, m_, t_, s_, redb_,
                            (int64_t)slotr_, nslot_, brtol_, opt_.rank_rtol, opt_.lsq_kernel);
      LAUNCHCHK();
    }
    for (; c0 <= m_; c0 += opt_.lsq_chunk) enqueue_chunk(c0, std::min(c0 + opt_.lsq_chunk - 1, m_));
  }

  // y = R^{-1} z for the leading (khat + j) block; coefficients of the stored
  // basis [U, P]: y_i for U, y_i / nu_i for the unnormalised P.  On the device
  // (one wavefront, no host round trip before the basis product); on the host
  // beyond 512 columns.
  void solve_coefficients(int j) {
    const int nls = khat_ + j;
    // On stream B, where R and z were formed (the host has seen that stream
    // finish the steps up to j): it runs beside stream A's remaining work,
    // such as the recycled-basis product, and the check's product waits for it.
    if (launch_back_subst<A>(streamB_, nls, khat_, R_, lmax_, z_, nu_, ycoef_)) {
      LAUNCHCHK();
      HIPCHK(hipEventRecord(ev_bs_, streamB_));
      HIPCHK(hipStreamWaitEvent(stream_, ev_bs_, 0));
      return;
    }
    // (own staging: the eigen-step's copies of R and nu may be in use on a worker thread)
    HIPCHK(hipMemcpyAsync(hRc_, R_, sizeof(A) * (size_t)lmax_ * nls, hipMemcpyDeviceToHost, stream_));
    HIPCHK(hipMemcpyAsync(hz_, z_, sizeof(A) * nls, hipMemcpyDeviceToHost, stream_));
    HIPCHK(hipMemcpyAsync(hnuc_, nu_, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, stream_));
    HIPCHK(hipStreamSynchronize(stream_));
    std::vector<std::complex<double>> y(nls);
    for (int i = 0; i < nls; ++i) y[i] = to_cd(hz_[i]);
    for (int i = nls - 1; i >= 0; --i) {
      const std::complex<double> rii = to_cd(hRc_[(size_t)i * lmax_ + i]);
      y[i] = std::abs(rii) > 0.0 ? y[i] / rii : std::complex<double>(0.0);
      for (int k = 0; k < i; ++k) y[k] -= to_cd(hRc_[(size_t)i * lmax_ + k]) * y[i];
    }
    for (int i = 0; i < nls; ++i)
      hy_[i] = from_cd<A>(i < khat_ ? y[i] : y[i] / hnuc_[i - khat_]);
    HIPCHK(hipMemcpyAsync(ycoef_, hy_, sizeof(A) * nls, hipMemcpyHostToDevice, stream_));
  }

  // Which inputs of a failed residual check hold non-finite values (host copies).
  std::string nonfinite_report(int j) {
    const int nls = khat_ + j;
    auto bad = [](const std::vector<A>& v) {
      size_t c = 0;
      for (const A& a : v) {
        const std::complex<double> z = to_cd(a);
        if (!std::isfinite(z.real()) || !std::isfinite(z.imag())) ++c;
      }
      return c;
    };
    std::vector<A> y(nls), R((size_t)lmax_ * nls), z(nls), xt(n_);
    std::vector<double> nu(j + 1);
    HIPCHK(hipMemcpy(y.data(), ycoef_, sizeof(A) * nls, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(R.data(), R_, sizeof(A) * R.size(), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(z.data(), z_, sizeof(A) * nls, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(nu.data(), nu_, sizeof(double) * (j + 1), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(xt.data(), xt_, sizeof(A) * n_, hipMemcpyDeviceToHost));
    size_t rbad = 0;
    for (int c = 0; c < nls; ++c)
      for (int i = 0; i <= c; ++i) {
        const std::complex<double> v = to_cd(R[(size_t)c * lmax_ + i]);
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) ++rbad;
      }
    size_t nubad = 0;
    for (double v : nu)
      if (!std::isfinite(v) || v == 0.0) ++nubad;
    return "non-finite: coefficients " + std::to_string(bad(y)) + "/" + std::to_string(nls) + ", R " +
           std::to_string(rbad) + ", z " + std::to_string(bad(z)) + ", nu (or zero) " +
           std::to_string(nubad) + "/" + std::to_string(j + 1) + ", basis product " +
           std::to_string(bad(xt)) + "/" + std::to_string(n_) + ", k_hat " + std::to_string(khat_);
  }

  // Givens estimate of the true residual at step j (Sections 4.5 and 5),
  // rebuilt on the host from the anchor (the value at step a, divided by
  // sqrt(1 - eps) when it is a sketched residual) and the sketched residuals
  // of steps a .. j in the step records: the same operations in the same
  // order as the least-squares kernels' running estimate.
  double givens_estimate(double eps, double anchor, bool scaled, int a, int j) const {
    double e = scaled ? anchor / std::sqrt(1.0 - eps) : anchor;
    double sp = rec_host_[a].sres;
    for (int i = a + 1; i <= j; ++i) {
      const double sr = rec_host_[i].sres;
      double sn = sp > 0.0 ? sr / sp : 0.0;
      sn = sn < 1.0 ? sn : 1.0;
      const double cs = std::sqrt(std::max(0.0, 1.0 - sn * sn));
      e *= std::sqrt((sn * sn + 2.0 * eps * (1.0 + cs)) / (1.0 - eps * eps));
      sp = sr;
    }
    return e;
  }

  // A true residual res at step j: raise eps to the smallest value (by
  // bisection) whose estimate from the anchor reaches res, if it fell short.
  double givens_refit(double eps, double anchor, bool scaled, int a, int j, double res) const {
    if (!(res > givens_estimate(eps, anchor, scaled, a, j))) return eps;
    double lo = eps, hi = 1.0;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (givens_estimate(mid, anchor, scaled, a, j) >= res)
        hi = mid;
      else
        lo = mid;
    }
    return hi;
  }

  // Residual check after step j: x~ = [U P] y and r_new = r0 - A x~, queued on
  // stream A (finish_residual() returns ||r_new||).
  void enqueue_check(int j) {
    solve_coefficients(j);
    launch_gemv_basis<T>(stream_, n_, U_, n_, khat_, P_, n_, j, ycoef_, xt_);
    LAUNCHCHK();
    enqueue_residual(xt_, r_, rnew_);
  }

  int solve(const void* bv, void* xv, double tol, sdr_stats* st,
            std::vector<sdr_cycle_record>* trace) override {
    const A* b = static_cast<const A*>(bv);
    A* x = static_cast<A*>(xv);
    const double t0 = now();
    double eig_time = 0.0;
    trace->clear();
    ev_pend_j_ = 0;  // (times of a solve that ended in an error are dropped)
    int matvecs = 0, ips = 0, sketches = 0, checks = 0, iters = 0, cycles = 0;
    const T* vals = basis_values();
    double nb2v = 0.0;
    sketch_cols<A>(b, 1, Sr_, s_, &nb2v);  // ||b|| (the sketch is discarded)
    const double nb = std::sqrt(nb2v);
    if (!std::isfinite(nb)) {
      set_err("non-finite right-hand side");
      return SDR_EINVAL;
    }
    double rn = residual(x, b, r_);
    matvecs++;
    ips++;
    if (!std::isfinite(rn)) {
      set_err("non-finite initial residual");
      return SDR_EINVAL;
    }
    if (nb == 0.0) {
      HIPCHK(hipMemsetAsync(x, 0, sizeof(A) * n_, stream_));
      HIPCHK(hipStreamSynchronize(stream_));
      fill_stats(st, 0, 0, matvecs, ips, sketches, checks, SDR_OK, 0.0, 0.0, 1.4, now() - t0, 0.0);
      return SDR_OK;
    }
    const double tol_abs = tol * nb;
    if (sau_stale_ && khat_ > 0) {
      // exact variant: S A_i U with the new matrix (k products and sketches)
      for (int c = 0; c < khat_; ++c) {
        Window<T> win{};
        const T* uc = U_ + (size_t)c * n_;
        if (ilu_) {  // A M^-1 U
          launch_ilu_apply<T>(stream_, *ilu_, uc, iy_, izb_, nullptr);
          LAUNCHCHK();
          uc = izb_;
        }
        if (dia())
          launch_spmv_dia_sketch<T>(stream_, n_, dia_, uc, Unew_ + (size_t)c * n_, win, 0,
                                    SketchSpec{}, true, part1_, nb1_, ctrl_free_);
        else
          launch_spmv_sketch<T>(stream_, n_, M_.rp, M_.ci, vals, uc,
                                Unew_ + (size_t)c * n_, win, 0, SketchSpec{}, true, part1_, nb1_,
                                ctrl_free_);
        LAUNCHCHK();
      }
      sketch_cols<T>(Unew_, khat_, SAU_, s_, nullptr);
      matvecs += khat_;
      sketches += khat_;
    }
    sau_stale_ = false;
    double safety = opt_.safety0;
    // Givens control: eps persists across the cycles of a solve; the
    // threshold is tol itself
    const bool givens = opt_.resid_control == 1;
    double geps = opt_.givens_eps0;
    auto thresh_of = [&](double sf) { return givens ? tol_abs : tol_abs / sf; };
    bool converged = rn <= tol_abs;
    double last_sres = 0.0;
    int status = SDR_NOT_CONVERGED;
    (void)wait_eig();  // left over from a solve that failed
    pend_.active = false;
    bool started = false;  // this cycle's start already queued (at the end of the previous one)
    while (!converged && cycles < opt_.max_cycles) {
      if (!opt_.persist_safety) safety = opt_.safety0;
      sdr_cycle_record rec{};
      if (!started) start_cycle(r_, rn, thresh_of(safety), vals);
      started = false;
      const int cyc_par = cycle_par_;
      sketches++;
      ips++;
      int enqA = 1;
      if (pend_.active) {
        // The Arnoldi basis of this cycle does not depend on the recycle space
        // (V spans K_m(A, r0)): the previous cycle's eigen-step runs on a
        // worker thread while this one queues the cycle's steps.
        for (int j = 2; j <= m_ + 1; ++j) enqueue_step_a(j, vals, needs_event(j, 1));
        enqA = m_ + 1;
        EigResult er = take_eig();
        eig_time += er.seconds;
        finish_recycle_enqueue(er, trace);
      }
      if (khat_ > 0) {
        HIPCHK(hipMemcpyAsync(SB_ + (size_t)(kmax_ - khat_) * s_, SU_, sizeof(A) * s_ * khat_,
                              hipMemcpyDeviceToDevice, streamB_));
        HIPCHK(hipMemcpyAsync(SAW_ + (size_t)(kmax_ - khat_) * s_, SAU_, sizeof(A) * s_ * khat_,
                              hipMemcpyDeviceToDevice, streamB_));
      }
      launch_lsq_init<A>(streamB_, lsq(), khat_, s_, Sr_, opt_.rank_rtol, m_,
                         GivensInit{givens ? 1 : 0, geps, rn}, opt_.lsq_kernel);
      LAUNCHCHK();
      // anchor of the Givens estimate: ||r0||, or the sketched residual over
      // span(U) (step record 0) divided by sqrt(1 - eps)
      const bool g_scaled0 = khat_ > 0;
      double g_anchor = rn;
      bool g_scaled = g_scaled0;
      int g_a = 0;
      // --- truncated Arnoldi with sketched least squares ---
      int done = 0, jstop = 0, flags_stop = 0;
      bool early = false;
      double res = 0.0, sres = 0.0;
      bool cyc_conv = false;
      enqueue_from(1, enqA, vals);
      drain_timing();  // the previous cycle's kernel times, while this one runs
      for (;;) {
        HaltRec hr;
        if (!wait_halt(hr)) {
          set_err("halt record missing");
          throw HipError{SDR_EDEVICE};
        }
        if (hr.j == m_) {
          // the cycle ends here whatever the check says: its eigen-step
          // starts at once (stream B orders it after the least squares)
          begin_recycle(hr.j, (int)trace->size(), streamB_);
          early = true;
        }
        // Every step record up to hr.j is complete (the halt record is
        // published after them), and stream B's queued chunks must have seen
        // the halt before a resume clears it; stream A needs no wait: the
        // check's kernels queue behind its remaining work.
        HIPCHK(hipStreamSynchronize(streamB_));
        StepRec rc{};
        while (done < hr.j) {
          ++done;
          rc = rec_host_[done];
          const int tw = done - std::max(done - t_, 0);
          matvecs++;
          ips += tw + 1;
          iters++;
          if (!(rc.flags & 2)) sketches++;
        }
        sres = rc.sres;
        {
          enqueue_check(done);
          if (done == m_) {
            // Unless this check converges the next cycle starts from the new
            // residual: x += x~ and that start are queued now, ahead of the
            // host's reading of the residual (wasted work if it converges).
            if (!(rc.flags & 6) && !opt_.persist_safety && cycles + 1 < opt_.max_cycles) {
              launch_axpy<A>(stream_, n_, from_cd<A>({1.0, 0.0}), xt_, x);
              LAUNCHCHK();
              cur_ ^= 1;
              start_cycle(rnew_, -1.0, thresh_of(opt_.safety0), vals);
              cur_ ^= 1;
              started = true;
            }
          }
          res = finish_residual();
          matvecs++;
          ips++;
          checks++;
          rec.n_checks++;
          if (!std::isfinite(res)) {
            set_err("non-finite residual at step " + std::to_string(done) + " of cycle " +
                    std::to_string(cycles + 1) + " (" + nonfinite_report(done) + ")");
            throw HipError{SDR_EDEVICE};
          }
          if (res < tol_abs) {
            cyc_conv = true;
            jstop = done;
            break;
          }
          if (rc.flags & 6) {
            jstop = done;
            flags_stop = rc.flags & 6;
            break;
          }
          if (givens) {
            if (g_a == 0 && g_scaled) g_anchor = rec_host_[0].sres;  // (written by this cycle's init)
            geps = givens_refit(geps, g_anchor, g_scaled, g_a, done, res);
            g_anchor = res;
            g_scaled = false;
            g_a = done;
          } else if (sres > 0.0) {
            safety = res / sres;
          }
          if (done == m_) {
            jstop = done;
            break;
          }
          // resume: the steps after `done` may have been skipped by the halt
          if (givens)
            launch_set_ctrl_givens(stream_, ctrl_, tol_abs, geps, res, rec_host_[done].sres);
          else
            launch_set_ctrl(stream_, ctrl_, 0, tol_abs / safety);
          LAUNCHCHK();
          __atomic_store_n(&halt_host_->seq, -1, __ATOMIC_RELEASE);
          enqA = done;
          enqueue_from(done + 1, enqA, vals);
        }
      }
      cycles++;
      last_sres = sres;
      if (opt_.kernel_timing) {
        ev_pend_j_ = jstop;  // read during the next cycle (drain_timing)
        ev_pend_p_ = cyc_par;
      }
      // x += xt, r = r0 - A xt
      if (!started) {
        launch_axpy<A>(stream_, n_, from_cd<A>({1.0, 0.0}), xt_, x);
        LAUNCHCHK();
      }
      std::swap(r_, rnew_);
      rn = res;
      rec.j_stop = jstop;
      rec.flags = (cyc_conv ? 1 : 0) | flags_stop;
      // the cycle's sketched residuals by step (records 0 .. jstop are
      // complete: stream B was synchronised after the last halt)
      step_sres_.assign(jstop + 1, 0.0);
      for (int i = 0; i <= jstop; ++i) step_sres_[i] = rec_host_[i].sres;
      rec.sres = sres;
      rec.res = res;
      trace->push_back(rec);
      converged = cyc_conv;
      // --- sketched harmonic-Ritz update of U, SU, SAU (always) ---
      if (!early) begin_recycle(jstop, (int)trace->size() - 1, stream_);
      cur_ ^= 1;
      const bool more = !converged && cycles < opt_.max_cycles && !(flags_stop && jstop == 1);
      if (!more) {
        EigResult er = take_eig();
        eig_time += er.seconds;
        finish_recycle_enqueue(er, trace);
        break;
      }
    }
    sync_both();
    drain_timing();
    status = converged ? SDR_OK : SDR_NOT_CONVERGED;
    fill_stats(st, cycles, iters, matvecs, ips, sketches, checks, status, rn / nb, last_sres,
               givens ? 0.0 : safety, now() - t0, eig_time);
    if (st) st->eps = givens ? geps : 0.0;
    return status;
  }

  // Cycle start on stream A: S r0 (from the partials of the residual kernel
  // that formed r0, when it did), p_0 = r0 / ||r0|| into the P buffer of cur_
  // with the control block reset in the same launch, and step 1, whose SpMV
  // sketches p_0; stream B follows with SV(:, 0) and nu_0.  ||r0|| comes from
  // the host (rn >= 0) or stays on the device (rn < 0: red3_ holds ||r0||^2
  // from the last check).
  void start_cycle(const A* r0, double rn, double thresh, const T* vals) {
    evp_ ^= 1;
    cycle_par_ = evp_;
    if (opt_.kernel_timing > 0) {
      ev_ofs_[evp_] = ev_ofs_next_;
      ev_ofs_next_ = (ev_ofs_next_ + 13) % opt_.kernel_timing;
    }
    P_ = Pbuf_[cur_];
    SB_ = SBbuf_[cur_];
    SAW_ = SAWbuf_[cur_];
    if (sr_of_ == r0) {  // sketched by the residual kernel that formed r0
      launch_reduce_cols<A>(stream_, psk_, nb2_, s_, s_, sk_scl_, Sr_, nullptr);
      LAUNCHCHK();
    } else {
      sketch_cols<A>(r0, 1, Sr_, s_, nullptr);
    }
    // p_0, and the control block reset for the cycle (same launch)
    if (rn >= 0.0)
      launch_cast_scale<T>(stream_, n_, r0, rn > 0.0 ? 1.0 / rn : 1.0, P_, ctrl_, thresh);
    else
      launch_cast_rscale<T>(stream_, n_, r0, red3_, P_, ctrl_, thresh);
    last_sv_ = SB_ + (size_t)kmax_ * s_;
    __atomic_store_n(&halt_host_->seq, -1, __ATOMIC_RELEASE);
    LAUNCHCHK();
    enqueue_step_a(1, vals, true);
    HIPCHK(hipStreamWaitEvent(streamB_, evs_[1 % nslot_], 0));
    launch_reduce_cols<A>(streamB_, part1_ + slot1_ * (1 % nslot_), nb1_, s_ + 1, s_,
                          sk_scl_, red0_, nullptr);
    launch_init_v0<A>(streamB_, red0_, s_, SB_ + (size_t)kmax_ * s_, nu_);
    LAUNCHCHK();
  }

  // Result of the host eigen-step of a finished cycle.
  struct EigResult {
    int keff = 0, ell = 0;
    double seconds = 0.0;
    std::vector<std::complex<double>> G;
    int code = 0;     // error raised on the worker thread
    std::string err;  // and its message (error strings are per thread)
  };

  // End of a cycle: C = Q^H [SU, SV] on the device (stream st) and the small
  // factors to pinned host memory, then the eigen-step starts on a worker
  // thread; take_eig() collects it.
  void begin_recycle(int j, int trace_idx, hipStream_t st) {
    pend_ = Pending{};
    pend_.active = true;
    pend_.j = j;
    pend_.khat = khat_;
    pend_.l0 = khat_ + j;
    pend_.trace_idx = trace_idx;
    pend_.P = P_;
    pend_.SB = SB_ + (size_t)(kmax_ - khat_) * s_;
    pend_.SAW = SAW_ + (size_t)(kmax_ - khat_) * s_;
    const int l0 = pend_.l0;
    if (k_ == 0 || l0 == 0) return;
    launch_small_gemm<A>(st, true, l0, l0, s_, Q_, s_, pend_.SB, s_, C_, l0);
    LAUNCHCHK();
    // complex data: R^{-1} (a wavefront per column) and R^{-1} C on the
    // device, so that the host's step starts from them (its longest serial
    // part on this data); real data keep the host's own triangular solve
    pend_.gpu_ric = Ri_ != nullptr && launch_tri_inverse<A>(st, l0, R_, lmax_, Ri_, l0, fro2_);
    if (pend_.gpu_ric) {
      launch_small_gemm<A>(st, false, l0, l0, l0, Ri_, l0, C_, l0, RiC_, l0);
      LAUNCHCHK();
      HIPCHK(hipMemcpyAsync(hRiC_, RiC_, sizeof(A) * (size_t)l0 * l0, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(hfro2_, fro2_, sizeof(double) * l0, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipMemcpyAsync(hR_, R_, sizeof(A) * (size_t)lmax_ * l0, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hC_, C_, sizeof(A) * (size_t)l0 * l0, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hnu_, nu_, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(ev_copy_, st));
    // hand the eigen-step to the worker thread (started once, kept)
    if (!eig_thr_.joinable()) eig_thr_ = std::thread([this] { eig_loop(); });
    {
      std::lock_guard<std::mutex> lk(eig_mu_);
      eig_job_ = true;
      eig_done_ = false;
    }
    eig_pending_ = true;
    eig_cv_.notify_all();
  }

  // Worker thread: one eigen-step per hand-over, until release().
  void eig_loop() {
    std::unique_lock<std::mutex> lk(eig_mu_);
    for (;;) {
      eig_cv_.wait(lk, [this] { return eig_job_ || eig_quit_; });
      if (eig_quit_) return;
      eig_job_ = false;
      lk.unlock();
      EigResult r;
      try {
        r = eig_compute();
      } catch (HipError& e) {
        r = EigResult{};
        r.code = e.code;
        r.err = g_err;  // (error strings are per thread)
      }
      lk.lock();
      eig_res_ = std::move(r);
      eig_done_ = true;
      eig_cv_.notify_all();
    }
  }

  // Wait for the pending eigen-step, if any, and return its result.
  EigResult wait_eig() {
    if (!eig_pending_) return EigResult{};
    std::unique_lock<std::mutex> lk(eig_mu_);
    eig_cv_.wait(lk, [this] { return eig_done_; });
    eig_pending_ = false;
    return std::move(eig_res_);
  }

  // The pending eigen-step's result (an empty one if none was started).
  EigResult take_eig() {
    EigResult er = wait_eig();
    if (er.code) {
      set_err(er.err);
      throw HipError{er.code};
    }
    return er;
  }

  // Host eigen-step of the pending cycle (no device work: it may run on a
  // worker thread while the next cycle is queued).
  EigResult eig_compute() {
    EigResult r;
    const int l0 = pend_.l0;
    if (!pend_.active || k_ == 0 || l0 == 0) return r;
    const double t0 = now();
    HIPCHK(hipEventSynchronize(ev_copy_));
    std::vector<std::complex<double>> Rc((size_t)l0 * l0), Cc((size_t)l0 * l0);
    for (int c = 0; c < l0; ++c)
      for (int i = 0; i < l0; ++i) {
        Rc[(size_t)c * l0 + i] = i <= c ? to_cd(hR_[(size_t)c * lmax_ + i]) : std::complex<double>(0.0);
        Cc[(size_t)c * l0 + i] = to_cd(hC_[(size_t)c * l0 + i]);
      }
    if (pend_.gpu_ric) {
      std::vector<std::complex<double>> RiC((size_t)l0 * l0);
      for (size_t i = 0; i < RiC.size(); ++i) RiC[i] = to_cd(hRiC_[i]);
      double fro2 = 0.0;
      for (int c = 0; c < l0; ++c) fro2 += hfro2_[c];
      r.keff = dense::harmonic_ritz(l0, Rc.data(), Cc.data(), s_, k_, !traits<T>::cpx, r.G, &r.ell, RiC.data(),
                                    fro2);
    } else {
      r.keff = dense::harmonic_ritz(l0, Rc.data(), Cc.data(), s_, k_, !traits<T>::cpx, r.G, &r.ell);
    }
    if (r.keff < 0) {
      set_err("Schur iteration did not converge");
      throw HipError{SDR_EDEVICE};
    }
    r.seconds = now() - t0;
    return r;
  }

  // U = [U P] G (stream A) and SU = [SU SV] G, SAU = [SAU SAV] G (stream B)
  // from the eigen-step's result; updates khat_ and the trace record.
  void finish_recycle_enqueue(const EigResult& r, std::vector<sdr_cycle_record>* trace) {
    if (!pend_.active) return;
    pend_.active = false;
    const int l0 = pend_.l0, khat = pend_.khat, keff = r.keff;
    if (keff > 0) {
      A* Gh = hG_;
      A* Gp = hG_ + (size_t)l0 * keff;
      for (int c = 0; c < keff; ++c)
        for (int i = 0; i < l0; ++i) {
          const A g = from_cd<A>(r.G[(size_t)c * l0 + i]);
          Gh[(size_t)c * l0 + i] = g;
          Gp[(size_t)c * l0 + i] = i < khat ? g : scale(g, 1.0 / hnu_[i - khat]);
        }
      // small products on stream B (they feed this cycle's least squares),
      // the N x keff product on stream A behind the cycle's Arnoldi steps (it
      // feeds the first residual check; run beside the steps it slowed them
      // more than it saved)
      HIPCHK(hipMemcpyAsync(Gs_, Gh, sizeof(A) * (size_t)l0 * keff, hipMemcpyHostToDevice, streamB_));
      launch_small_gemm<A>(streamB_, false, s_, keff, l0, pend_.SB, s_, Gs_, l0, SU_, s_);
      launch_small_gemm<A>(streamB_, false, s_, keff, l0, pend_.SAW, s_, Gs_, l0, SAU_, s_);
      // the basis product takes G row major, rows padded with zeros
      const int gw = gemm_basis_width(keff);
      A* Gr = Gp + (size_t)l0 * keff;
      for (int i = 0; i < l0; ++i)
        for (int c = 0; c < gw; ++c) Gr[(size_t)i * gw + c] = c < keff ? Gp[(size_t)c * l0 + i] : A{};
      HIPCHK(hipMemcpyAsync(G_, Gr, sizeof(A) * (size_t)l0 * gw, hipMemcpyHostToDevice, stream_));
      launch_gemm_basis<T>(stream_, n_, U_, n_, khat, pend_.P, n_, pend_.j, G_, keff, Unew_, n_);
      LAUNCHCHK();
      std::swap(U_, Unew_);
    }
    khat_ = keff;
    if (trace && pend_.trace_idx >= 0 && pend_.trace_idx < (int)trace->size()) {
      (*trace)[pend_.trace_idx].ell = r.ell;
      (*trace)[pend_.trace_idx].k_eff = keff;
    }
  }

  void fill_stats(sdr_stats* st, int cycles, int iters, int mv, int ip, int sk, int ch, int status,
                  double relres, double sres, double safety, double secs, double eig) {
    if (!st) return;
    std::memset(st, 0, sizeof(*st));
    st->cycles = cycles;
    st->iters = iters;
    st->matvecs = mv;
    st->inner_products = ip;
    st->sketches = sk;
    st->res_checks = ch;
    st->status = status;
    st->k_eff = khat_;
    st->relres = relres;
    st->sres = sres;
    st->safety = safety;
    st->seconds = secs;
    st->host_eig_seconds = eig;
  }

  int get_recycle(void* U, void* SU, void* SAU, int* k) override {
    if (k) *k = khat_;
    if (khat_ > 0) {
      if (U) {
        launch_widen_scale<T>(stream_, n_ * khat_, U_, 1.0, static_cast<A*>(U));
        LAUNCHCHK();
      }
      if (SU)
        HIPCHK(hipMemcpyAsync(SU, SU_, sizeof(A) * s_ * khat_, hipMemcpyDeviceToDevice, stream_));
      if (SAU)
        HIPCHK(hipMemcpyAsync(SAU, SAU_, sizeof(A) * s_ * khat_, hipMemcpyDeviceToDevice, stream_));
    }
    HIPCHK(hipStreamSynchronize(stream_));
    return SDR_OK;
  }

  int step_sres(double* out, int cap) override {
    const int n = (int)step_sres_.size();
    if (out)
      for (int i = 0; i < std::min(n, cap); ++i) out[i] = step_sres_[i];
    return n;
  }

  int get_basis(int ncols, void* V, void* Hh, void* SVh) override {
    if (ncols < 0 || ncols > m_ + 1) {
      set_err("ncols out of range");
      return SDR_EINVAL;
    }
    std::vector<double> nuh(m_ + 2);
    HIPCHK(hipMemcpyAsync(nuh.data(), nu_, sizeof(double) * (m_ + 2), hipMemcpyDeviceToHost, stream_));
    HIPCHK(hipStreamSynchronize(stream_));
    if (V)
      for (int c = 0; c < ncols; ++c) {
        const double sc = nuh[c] > 0.0 ? 1.0 / nuh[c] : 0.0;
        launch_widen_scale<T>(stream_, n_, Pbuf_[cur_ ^ 1] + (size_t)c * n_, sc,
                              static_cast<A*>(V) + (size_t)c * n_);
        LAUNCHCHK();
      }
    if (Hh)
      HIPCHK(hipMemcpyAsync(Hh, H_, sizeof(A) * (m_ + 1) * m_, hipMemcpyDeviceToHost, stream_));
    if (SVh && ncols > 0 && last_sv_)
      HIPCHK(hipMemcpyAsync(SVh, last_sv_, sizeof(A) * s_ * ncols, hipMemcpyDeviceToHost, stream_));
    HIPCHK(hipStreamSynchronize(stream_));
    return SDR_OK;
  }

 private:
  void release() {
    (void)wait_eig();
    if (eig_thr_.joinable()) {
      {
        std::lock_guard<std::mutex> lk(eig_mu_);
        eig_quit_ = true;
      }
      eig_cv_.notify_all();
      eig_thr_.join();
    }
    for (void* p : {(void*)valB_, (void*)dia_map_, (void*)diaval_, (void*)dcflag_, (void*)dcval_,
                    (void*)Pbuf_[0], (void*)Pbuf_[1],
                    (void*)U_, (void*)Unew_, (void*)SU_,
                    (void*)red0_,
                    (void*)SAU_, (void*)Q_, (void*)R_, (void*)z_, (void*)rho_, (void*)SBbuf_[0],
                    (void*)SBbuf_[1], (void*)SAWbuf_[0], (void*)SAWbuf_[1], (void*)H_,
                    (void*)nu_, (void*)sres_hist_, (void*)ctrl_, (void*)ctrl_free_, (void*)part1_,
                    (void*)redb_, (void*)psk_, (void*)red2_, (void*)red3_, (void*)Sr_,
                    (void*)ycoef_, (void*)xt_, (void*)r_, (void*)rnew_, (void*)G_, (void*)Gs_,
                    (void*)C_, (void*)dct_rows_, (void*)blkA_, (void*)blkD_, (void*)blkI_, (void*)Ri_, (void*)RiC_,
                    (void*)fro2_, (void*)izb_, (void*)iy_, (void*)izA_, (void*)iyA_})
      dfree(p);
    if (rec_host_) (void)hipHostFree(rec_host_);
    rec_host_ = nullptr;
    if (halt_host_) (void)hipHostFree(halt_host_);
    halt_host_ = nullptr;
    for (void* p : {(void*)hR_, (void*)hC_, (void*)hz_, (void*)hy_, (void*)hnu_, (void*)hG_,
                    (void*)hRc_, (void*)hnuc_,
                    (void*)hscal_, (void*)hres_, (void*)hRiC_, (void*)hfro2_})
      if (p) (void)hipHostFree(p);
    hR_ = hC_ = hz_ = hy_ = hG_ = hscal_ = hRc_ = hres_ = hRiC_ = nullptr;
    hfro2_ = nullptr;
    hres_dev_ = nullptr;
    hnu_ = hnuc_ = nullptr;
    for (auto& evp : ev_) {
      for (auto& a : evp)
        for (auto& e : a)
          if (e) (void)hipEventDestroy(e);
      evp.clear();
    }
    for (auto& e : evs_)
      if (e) (void)hipEventDestroy(e);
    evs_.clear();
    if (ev_copy_) (void)hipEventDestroy(ev_copy_);
    ev_copy_ = nullptr;
    if (ev_res_) (void)hipEventDestroy(ev_res_);
    ev_res_ = nullptr;
    if (ev_bs_) (void)hipEventDestroy(ev_bs_);
    ev_bs_ = nullptr;
    if (streamB_) (void)hipStreamDestroy(streamB_);
    streamB_ = nullptr;
  }

  MatView<A> M_;
  int n_ = 0, m_, k_, t_, s_;
  Options opt_;
  std::vector<double> step_sres_;  // sketched residual by step of the last cycle (0: over span(U))
  hipStream_t stream_;
  SketchSpec sk_{};
  double brtol_ = 1e-14;
  int nb1_ = 0, nb2_ = 0, kmax_ = 0, lmax_ = 0;
  int khat_ = 0, khat_prev_ = 0;
  bool sau_stale_ = false, low_dirty_ = true;
  T* valB_ = nullptr;
  DiaView<T> dia_{};      // diagonal storage of the basis-precision matrix (ndiag 0: CSR)
  int* dia_map_ = nullptr;
  T* diaval_ = nullptr;
  int* dcflag_ = nullptr;  // constant-diagonal flags and values (kMaxDiag each)
  T* dcval_ = nullptr;
  T *P_ = nullptr, *U_ = nullptr, *Unew_ = nullptr;
  // right ILU(0): z = M^-1 p for the step SpMV (izb_, forward solve in iy_)
  // and for the residual (izA_, iyA_)
  const IluView* ilu_ = nullptr;
  T* izb_ = nullptr;
  A *iy_ = nullptr, *izA_ = nullptr, *iyA_ = nullptr;
  T* Pbuf_[2] = {nullptr, nullptr};
  A* SBbuf_[2] = {nullptr, nullptr};
  A* SAWbuf_[2] = {nullptr, nullptr};
  int cur_ = 0;  // which of the double buffers the running cycle uses
  // a finished cycle whose recycle update waits for the host eigen-step
  struct Pending {
    bool active = false;
    int j = 0, l0 = 0, khat = 0, trace_idx = -1;
    T* P = nullptr;
    A* SB = nullptr;   // shifted so that column 0 is the first recycled column
    A* SAW = nullptr;
    bool gpu_ric = false;  // R^{-1} C and ||R^{-1}||_F^2 copied to the host by the device
  } pend_;
  hipEvent_t ev_copy_ = nullptr;
  hipEvent_t ev_res_ = nullptr;   // after the residual norm's reduction into host-mapped memory
  hipEvent_t ev_bs_ = nullptr;    // after the check's back substitution (stream B)
  A* last_sv_ = nullptr;  // SV(:, 0) of the last cycle (basis inspection)
  A *SU_ = nullptr, *SAU_ = nullptr, *Q_ = nullptr, *R_ = nullptr, *z_ = nullptr, *rho_ = nullptr;
  A *SB_ = nullptr, *SAW_ = nullptr, *H_ = nullptr;
  double *nu_ = nullptr, *sres_hist_ = nullptr;
  Ctrl *ctrl_ = nullptr, *ctrl_free_ = nullptr;
  const A* sr_of_ = nullptr;  // the vector whose sketch partials psk_ holds (rows 0 .. s-1)
  bool dct_on_ = false;       // subsampled randomised DCT sketch (option "sketch")
  double sk_scl_ = 1.0;       // scale of the reduced sketch rows
  DctRow* dct_rows_ = nullptr;
  DctSpec dct_{};
  A *Ri_ = nullptr, *RiC_ = nullptr, *hRiC_ = nullptr;
  double *fro2_ = nullptr, *hfro2_ = nullptr;
  A *blkA_ = nullptr;
  double* blkD_ = nullptr;
  int* blkI_ = nullptr;
  A *part1_ = nullptr, *redb_ = nullptr, *psk_ = nullptr, *red2_ = nullptr, *red3_ = nullptr,
    *red0_ = nullptr;
  int nslot_ = 0;
  size_t slot1_ = 0, slotr_ = 0;
  hipStream_t streamB_ = nullptr;
  std::vector<hipEvent_t> evs_;
  A *Sr_ = nullptr, *ycoef_ = nullptr, *xt_ = nullptr, *r_ = nullptr, *rnew_ = nullptr;
  A *G_ = nullptr, *Gs_ = nullptr, *C_ = nullptr;
  StepRec *rec_host_ = nullptr, *rec_dev_ = nullptr;
  HaltRec *halt_host_ = nullptr, *halt_dev_ = nullptr;
  // pinned host staging of the small dense data
  A* hres_ = nullptr;      // host-mapped coherent: the last residual's ||r||^2
  A* hres_dev_ = nullptr;  // its device address
  A *hR_ = nullptr, *hC_ = nullptr, *hz_ = nullptr, *hy_ = nullptr, *hG_ = nullptr, *hscal_ = nullptr,
    *hRc_ = nullptr;
  double *hnu_ = nullptr, *hnuc_ = nullptr;
  // the pending cycle's eigen-step on a worker thread
  std::thread eig_thr_;
  std::mutex eig_mu_;
  std::condition_variable eig_cv_;
  bool eig_job_ = false, eig_done_ = false, eig_quit_ = false, eig_pending_ = false;
  EigResult eig_res_;
  std::vector<std::array<hipEvent_t, 6>> ev_[2];  // kernel timing events, by cycle parity
  int evp_ = 0, ev_pend_p_ = 0, ev_pend_j_ = 0, cycle_par_ = 0;
  int ev_ofs_[2] = {0, 0}, ev_ofs_next_ = 0;  // timed-step offsets by cycle parity
  double kt_ms_[4] = {0, 0, 0, 0};  // SpMV, update, step, DCT sketch
  int64_t kt_n_[3] = {0, 0, 0};
  int64_t kt_bytes_tw_[kMaxWindow + 1] = {0, 0, 0, 0, 0};

 public:
  void reset() override {
    khat_ = 0;
    sau_stale_ = false;
  }

  int spmv_layout(int* offsets, int cap) override {
    for (int d = 0; d < dia_.ndiag && d < cap; ++d)
      if (offsets) offsets[d] = dia_.off[d];
    return dia_.ndiag;
  }

  // [0] SpMV + sketch ms, [1] update ms, [2] the kernels of a step (SpMV start to update end),
  // [3] the DCT sketch kernel (sketch=1; its launches are counts[0]);
  // counts[0..2] launches; counts[3 + tw] = launches with window size tw.
  int kernel_times(double* ms, int64_t* counts, int cap) override {
    for (int i = 0; i < 3 && i < cap; ++i) {
      if (ms) ms[i] = kt_ms_[i];
      if (counts) counts[i] = kt_n_[i];
    }
    if (ms && cap > 3) ms[3] = kt_ms_[3];
    kt_ms_[3] = 0;
    for (int tw = 0; tw <= kMaxWindow; ++tw)
      if (counts && 3 + tw < cap) counts[3 + tw] = kt_bytes_tw_[tw];
    for (int i = 0; i < 3; ++i) {
      kt_ms_[i] = 0;
      kt_n_[i] = 0;
    }
    for (auto& v : kt_bytes_tw_) v = 0;
    return SDR_OK;
  }
};

}  // namespace

// The thread-local message of sdr_last_error, for the other C entry points.
void sdr::set_last_error(const std::string& msg) { set_err(msg); }

// ============================================================== C handle ===
struct sdr_handle {
  int n = 0;
  int64_t nnz = 0;
  int m = 0, k = 0, t = 0, s = 0;
  uint64_t seed = 0;
  bool cpx = false;
  Options opt;
  int* rp = nullptr;
  int* ci = nullptr;
  void* vals = nullptr;
  // transpose (adjoint) pattern
  int* rpT = nullptr;
  int* ciT = nullptr;
  int* perm = nullptr;
  void* valsT = nullptr;
  // right Jacobi preconditioning (option "precond"): d = diag(A) and the
  // values of A D^-1 on the same pattern, which the forward solver runs on
  void* d_pc = nullptr;
  void* vals_pc = nullptr;
  int* pc_flag = nullptr;
  bool pc_bad = false;  // the last matrix had a zero diagonal entry (or ILU pivot): the factors are stale
  // right ILU(0) (option "precond" 2): the multicolour order and elimination
  // lists of the pattern (built once) and the factors on A's entries
  IluView ilu;
  std::vector<int> ilu_coff;
  int *ilu_crow = nullptr, *ilu_dpos = nullptr, *ilu_lo_off = nullptr, *ilu_up_off = nullptr;
  int2 *ilu_lo = nullptr, *ilu_up = nullptr;
  uint8_t* ilu_kind = nullptr;
  void* ilu_F = nullptr;
  void *ilu_t = nullptr, *ilu_u = nullptr;  // n-vectors for the change of variable
  // sliced-ELL copies for the solves: slot maps (entry of F or -1), columns,
  // values, slice tables (device) and each colour's first slice (host)
  int *ilu_lsrc = nullptr, *ilu_usrc = nullptr, *ilu_lcol = nullptr, *ilu_ucol = nullptr;
  int *ilu_lslice = nullptr, *ilu_lw = nullptr, *ilu_uslice = nullptr, *ilu_uw = nullptr;
  void *ilu_lval = nullptr, *ilu_uval = nullptr, *ilu_dinv = nullptr;
  std::vector<int> ilu_lsl0, ilu_usl0;
  int64_t ilu_nl = 0, ilu_nu = 0;
  bool ilu_built = false;
  bool adj_ready = false;
  uint64_t pattern_hash = 0;
  hipStream_t own = nullptr;
  hipStream_t stream = nullptr;
  bool follow_null = false;   // run on own, ordered after the null stream's earlier work
  hipEvent_t ev_in = nullptr;
  std::unique_ptr<SolverBase> fwd, adj;
  std::vector<sdr_cycle_record> trace;
  size_t elem() const { return cpx ? 16 : 8; }
};

namespace {

uint64_t hash_pattern(const std::vector<int>& rp, const std::vector<int>& ci) {
  uint64_t h = 1469598103934665603ull;
  auto mixin = [&](uint64_t v) {
    h ^= v;
    h *= 1099511628211ull;
  };
  for (int v : rp) mixin((uint32_t)v);
  for (int v : ci) mixin((uint32_t)v);
  return h;
}

std::unique_ptr<SolverBase> make_solver(sdr_handle* h, bool adjoint) {
  const int* rp = adjoint ? h->rpT : h->rp;
  const int* ci = adjoint ? h->ciT : h->ci;
  const void* v = adjoint ? h->valsT : h->opt.precond == 1 ? h->vals_pc : h->vals;
  if (!h->cpx) {
    MatView<double> mv{h->n, h->nnz, rp, ci, static_cast<const double*>(v)};
    if (h->opt.precision == 1)
      return std::unique_ptr<SolverBase>(new Solver<float>(mv, h->m, h->k, h->t, h->s, h->seed, h->opt, h->stream));
    return std::unique_ptr<SolverBase>(new Solver<double>(mv, h->m, h->k, h->t, h->s, h->seed, h->opt, h->stream));
  }
  MatView<cx<double>> mv{h->n, h->nnz, rp, ci, static_cast<const cx<double>*>(v)};
  if (h->opt.precision == 1)
    return std::unique_ptr<SolverBase>(new Solver<cx<float>>(mv, h->m, h->k, h->t, h->s, h->seed, h->opt, h->stream));
  return std::unique_ptr<SolverBase>(new Solver<cx<double>>(mv, h->m, h->k, h->t, h->s, h->seed, h->opt, h->stream));
}

// The multicolour order and elimination lists of right ILU(0) for the
// handle's pattern (host work, once per pattern): a greedy colouring of the
// symmetrised pattern (each row, in increasing index, takes the smallest
// colour none of its lower-indexed neighbours holds), the rows colour by
// colour, each entry tagged left of / on / right of the diagonal in that
// order, and per row its left entries in elimination order with the updates
// each one makes to the row.  Throws SDR_EINVAL if a diagonal entry is not
// stored.
void build_ilu(sdr_handle* h) {
  const int n = (int)h->n;
  const int64_t nnz = h->nnz;
  std::vector<int> rp(n + 1), ci(std::max<int64_t>(nnz, 1));
  HIPCHK(hipMemcpy(rp.data(), h->rp, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
  if (nnz > 0) HIPCHK(hipMemcpy(ci.data(), h->ci, sizeof(int) * nnz, hipMemcpyDeviceToHost));
  // transpose pattern, for the symmetrised neighbours
  std::vector<int> tp(n + 1, 0), tc(std::max<int64_t>(nnz, 1));
  for (int64_t e = 0; e < nnz; ++e) tp[ci[e] + 1]++;
  for (int i = 0; i < n; ++i) tp[i + 1] += tp[i];
  {
    std::vector<int> fill(tp.begin(), tp.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int e = rp[i]; e < rp[i + 1]; ++e) tc[fill[ci[e]]++] = i;
  }
  std::vector<int> colour(n, -1), mark;
  int ncol = 0;
  for (int i = 0; i < n; ++i) {
    auto note = [&](int j) {
      if (j < i) {
        const int c = colour[j];
        if (c >= (int)mark.size()) mark.resize(c + 1, -1);
        mark[c] = i;
      }
    };
    for (int e = rp[i]; e < rp[i + 1]; ++e) note(ci[e]);
    for (int e = tp[i]; e < tp[i + 1]; ++e) note(tc[e]);
    int c = 0;
    while (c < (int)mark.size() && mark[c] == i) ++c;
    colour[i] = c;
    ncol = std::max(ncol, c + 1);
  }
  // rows by colour (increasing index within a colour) and their ranks
  std::vector<int> coff(ncol + 1, 0), crow(n), rank(n);
  for (int i = 0; i < n; ++i) coff[colour[i] + 1]++;
  for (int c = 0; c < ncol; ++c) coff[c + 1] += coff[c];
  {
    std::vector<int> fill(coff.begin(), coff.end() - 1);
    for (int i = 0; i < n; ++i) crow[fill[colour[i]]++] = i;
  }
  for (int p = 0; p < n; ++p) rank[crow[p]] = p;
  std::vector<uint8_t> kind(std::max<int64_t>(nnz, 1));
  std::vector<int> dpos(n, -1);
  for (int i = 0; i < n; ++i)
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      const int j = ci[e];
      kind[e] = j == i ? 1 : (rank[j] < rank[i] ? 0 : 2);
      if (j == i) dpos[i] = e;
    }
  for (int i = 0; i < n; ++i)
    if (dpos[i] < 0) {
      h->pc_bad = true;
      set_err("ILU(0) preconditioning needs every diagonal entry of A stored");
      throw HipError{SDR_EINVAL};
    }
  // per row: left entries in elimination order, each with its updates
  std::vector<int> lo_off(n + 1, 0), up_off(1, 0);
  std::vector<int2> lo, up;
  std::vector<int> left;
  for (int i = 0; i < n; ++i) {
    left.clear();
    for (int e = rp[i]; e < rp[i + 1]; ++e)
      if (kind[e] == 0) left.push_back(e);
    std::sort(left.begin(), left.end(), [&](int a, int b) { return rank[ci[a]] < rank[ci[b]]; });
    for (int e : left) {
      const int k = ci[e];
      lo.push_back(make_int2(e, dpos[k]));
      for (int f = rp[k]; f < rp[k + 1]; ++f) {
        if (kind[f] != 2) continue;  // u_kj, rank(j) > rank(k)
        const int jc = ci[f];
        for (int g = rp[i]; g < rp[i + 1]; ++g)
          if (ci[g] == jc) {
            up.push_back(make_int2(g, f));
            break;
          }
      }
      up_off.push_back((int)up.size());
    }
    lo_off[i + 1] = (int)lo.size();
  }
  // sliced-ELL packing by colour: kind 0 entries for the forward solve,
  // kind 2 for the backward solve
  auto pack = [&](uint8_t want, std::vector<int>& src, std::vector<int>& col, std::vector<int>& slo,
                  std::vector<int>& sw, std::vector<int>& sl0) {
    sl0.assign(ncol + 1, 0);
    std::vector<int> ent;
    for (int c = 0; c < ncol; ++c) {
      sl0[c] = (int)slo.size();
      const int c0 = coff[c], cnt = coff[c + 1] - c0;
      for (int b0 = 0; b0 < cnt; b0 += 64) {
        int w = 0;
        for (int t = b0; t < std::min(cnt, b0 + 64); ++t) {
          const int i = crow[c0 + t];
          int k = 0;
          for (int e = rp[i]; e < rp[i + 1]; ++e) k += kind[e] == want;
          w = std::max(w, k);
        }
        const int o = (int)src.size();
        slo.push_back(o);
        sw.push_back(w);
        src.resize(o + (size_t)w * 64, -1);
        col.resize(o + (size_t)w * 64, 0);
        for (int t = b0; t < std::min(cnt, b0 + 64); ++t) {
          const int i = crow[c0 + t];
          int k = 0;
          for (int e = rp[i]; e < rp[i + 1]; ++e)
            if (kind[e] == want) {
              src[o + (size_t)k * 64 + (t - b0)] = e;
              col[o + (size_t)k * 64 + (t - b0)] = ci[e];
              ++k;
            }
        }
      }
    }
    sl0[ncol] = (int)slo.size();
  };
  std::vector<int> lsrc, lcolv, lslo, lsw, usrc, ucolv, uslo, usw;
  pack(0, lsrc, lcolv, lslo, lsw, h->ilu_lsl0);
  pack(2, usrc, ucolv, uslo, usw, h->ilu_usl0);
  auto up_vec = [](const std::vector<int>& v) {
    int* d = dalloc<int>(std::max<size_t>(v.size(), 1));
    if (!v.empty()) HIPCHK(hipMemcpy(d, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice));
    return d;
  };
  h->ilu_lsrc = up_vec(lsrc);
  h->ilu_lcol = up_vec(lcolv);
  h->ilu_lslice = up_vec(lslo);
  h->ilu_lw = up_vec(lsw);
  h->ilu_usrc = up_vec(usrc);
  h->ilu_ucol = up_vec(ucolv);
  h->ilu_uslice = up_vec(uslo);
  h->ilu_uw = up_vec(usw);
  h->ilu_nl = (int64_t)lsrc.size();
  h->ilu_nu = (int64_t)usrc.size();
  h->ilu_lval = dalloc<unsigned char>(h->elem() * std::max<size_t>(lsrc.size(), 1));
  h->ilu_uval = dalloc<unsigned char>(h->elem() * std::max<size_t>(usrc.size(), 1));
  h->ilu_dinv = dalloc<unsigned char>(h->elem() * n);
  const size_t nlo = std::max<size_t>(lo.size(), 1), nup = std::max<size_t>(up.size(), 1);
  h->ilu_crow = dalloc<int>(n);
  h->ilu_dpos = dalloc<int>(n);
  h->ilu_lo_off = dalloc<int>(n + 1);
  h->ilu_up_off = dalloc<int>(up_off.size());
  h->ilu_lo = dalloc<int2>(nlo);
  h->ilu_up = dalloc<int2>(nup);
  h->ilu_kind = dalloc<uint8_t>(kind.size());
  h->ilu_F = dalloc<unsigned char>(h->elem() * std::max<int64_t>(nnz, 1));
  h->ilu_t = dalloc<unsigned char>(h->elem() * n);
  h->ilu_u = dalloc<unsigned char>(h->elem() * n);
  HIPCHK(hipMemcpy(h->ilu_crow, crow.data(), sizeof(int) * n, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->ilu_dpos, dpos.data(), sizeof(int) * n, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->ilu_lo_off, lo_off.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->ilu_up_off, up_off.data(), sizeof(int) * up_off.size(), hipMemcpyHostToDevice));
  if (!lo.empty()) HIPCHK(hipMemcpy(h->ilu_lo, lo.data(), sizeof(int2) * lo.size(), hipMemcpyHostToDevice));
  if (!up.empty()) HIPCHK(hipMemcpy(h->ilu_up, up.data(), sizeof(int2) * up.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->ilu_kind, kind.data(), kind.size(), hipMemcpyHostToDevice));
  h->ilu_coff = coff;
  IluView& v = h->ilu;
  v.n = n;
  v.ncolours = ncol;
  v.crow = h->ilu_crow;
  v.coff = h->ilu_coff.data();
  v.rp = h->rp;
  v.ci = h->ci;
  v.kind = h->ilu_kind;
  v.dpos = h->ilu_dpos;
  v.F = h->ilu_F;
  v.lslice = h->ilu_lslice;
  v.lw = h->ilu_lw;
  v.lcol = h->ilu_lcol;
  v.lval = h->ilu_lval;
  v.uslice = h->ilu_uslice;
  v.uw = h->ilu_uw;
  v.ucol = h->ilu_ucol;
  v.uval = h->ilu_uval;
  v.lsl0 = h->ilu_lsl0.data();
  v.usl0 = h->ilu_usl0.data();
  v.dinv = h->ilu_dinv;
  h->ilu_built = true;
}

// Right ILU(0): the factors of the handle's matrix (on A's entries, in the
// multicolour order).  Throws SDR_EINVAL on a zero pivot.
void refresh_ilu(sdr_handle* h) {
  if (!h->ilu_built) build_ilu(h);
  if (!h->pc_flag) h->pc_flag = dalloc<int>(1);
  HIPCHK(hipMemsetAsync(h->pc_flag, 0, sizeof(int), h->stream));
  HIPCHK(hipMemcpyAsync(h->ilu_F, h->vals, h->elem() * h->nnz, hipMemcpyDeviceToDevice, h->stream));
  if (h->cpx) {
    launch_ilu_factor<cx<double>>(h->stream, h->ilu, h->ilu_lo_off, h->ilu_lo, h->ilu_up_off, h->ilu_up,
                                  static_cast<cx<double>*>(h->ilu_F), h->pc_flag);
    launch_ilu_pack<cx<double>>(h->stream, h->ilu, h->ilu_nl, h->ilu_lsrc, h->ilu_nu, h->ilu_usrc);
  } else {
    launch_ilu_factor<double>(h->stream, h->ilu, h->ilu_lo_off, h->ilu_lo, h->ilu_up_off, h->ilu_up,
                              static_cast<double*>(h->ilu_F), h->pc_flag);
    launch_ilu_pack<double>(h->stream, h->ilu, h->ilu_nl, h->ilu_lsrc, h->ilu_nu, h->ilu_usrc);
  }
  HIPCHK(hipGetLastError());
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, h->pc_flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->pc_bad = flag != 0;
  if (flag) {
    set_err("ILU(0) preconditioning met a zero pivot");
    throw HipError{SDR_EINVAL};
  }
}

// x <- M x (to_u) or M^-1 x: the change of variable of right ILU(0).
void ilu_transform(sdr_handle* h, void* x, bool to_u) {
  if (h->cpx) {
    auto* xv = static_cast<cx<double>*>(x);
    auto* t = static_cast<cx<double>*>(h->ilu_t);
    auto* u = static_cast<cx<double>*>(h->ilu_u);
    if (to_u)
      launch_ilu_mult<cx<double>>(h->stream, h->ilu, xv, t, u);
    else
      launch_ilu_apply<cx<double>>(h->stream, h->ilu, xv, t, u, nullptr);
  } else {
    auto* xv = static_cast<double*>(x);
    auto* t = static_cast<double*>(h->ilu_t);
    auto* u = static_cast<double*>(h->ilu_u);
    if (to_u)
      launch_ilu_mult<double>(h->stream, h->ilu, xv, t, u);
    else
      launch_ilu_apply<double>(h->stream, h->ilu, xv, t, u, nullptr);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(x, h->ilu_u, h->elem() * h->n, hipMemcpyDeviceToDevice, h->stream));
}

// Right Jacobi preconditioning, A x = b as (A D^-1) u = b with x = D^-1 u and
// D = diag(A): refresh d and the values of A D^-1 from the handle's matrix.
// Throws SDR_EINVAL if a diagonal entry is zero or not stored.  (Precond 2:
// the ILU(0) factors instead.)
void refresh_precond(sdr_handle* h) {
  if (h->opt.precond == 0) return;
  if (h->opt.precond == 2) return refresh_ilu(h);
  if (!h->vals_pc) {
    h->d_pc = dalloc<unsigned char>(h->elem() * h->n);
    h->vals_pc = dalloc<unsigned char>(h->elem() * std::max<int64_t>(h->nnz, 1));
    h->pc_flag = dalloc<int>(1);
  }
  HIPCHK(hipMemsetAsync(h->pc_flag, 0, sizeof(int), h->stream));
  if (h->cpx)
    launch_jacobi<cx<double>>(h->stream, h->n, h->nnz, h->rp, h->ci, static_cast<const cx<double>*>(h->vals),
                              static_cast<cx<double>*>(h->d_pc), static_cast<cx<double>*>(h->vals_pc),
                              h->pc_flag);
  else
    launch_jacobi<double>(h->stream, h->n, h->nnz, h->rp, h->ci, static_cast<const double*>(h->vals),
                          static_cast<double*>(h->d_pc), static_cast<double*>(h->vals_pc), h->pc_flag);
  HIPCHK(hipGetLastError());
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, h->pc_flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->pc_bad = flag != 0;
  if (flag) {
    set_err("Jacobi preconditioning needs every diagonal entry of A stored and nonzero");
    throw HipError{SDR_EINVAL};
  }
}

// x <- D x (to_u) or D^-1 x: the change of variable of right Jacobi preconditioning.
void precond_scale(sdr_handle* h, void* x, bool to_u) {
  if (h->cpx)
    launch_scale_by_diag<cx<double>>(h->stream, h->n, static_cast<const cx<double>*>(h->d_pc),
                                     static_cast<cx<double>*>(x), !to_u);
  else
    launch_scale_by_diag<double>(h->stream, h->n, static_cast<const double*>(h->d_pc), static_cast<double*>(x),
                                 !to_u);
  HIPCHK(hipGetLastError());
}

SolverBase* fwd(sdr_handle* h) {
  if (h->opt.sketch == 0 && h->s % h->opt.zeta != 0) {
    set_err("s_dim must be a multiple of zeta");
    throw HipError{SDR_EINVAL};
  }
  if (!h->fwd) {
    refresh_precond(h);
    h->fwd = make_solver(h, false);
    if (h->opt.precond == 2) h->fwd->set_ilu(&h->ilu);
  }
  return h->fwd.get();
}

int validate_csr(const sdr_csr* A, std::vector<int>* rp_out, std::vector<int>* ci_out) {
  if (!A || A->n <= 0 || A->nnz < 0 || !A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->values))) {
    set_err("invalid CSR descriptor");
    return SDR_EINVAL;
  }
  if (A->dtype != SDR_F64 && A->dtype != SDR_C128) {
    set_err("matrix dtype must be SDR_F64 or SDR_C128");
    return SDR_EINVAL;
  }
  if (A->n > (int64_t)0x7fffffff || A->nnz > (int64_t)0x7fffffff) {
    set_err("n and nnz must fit in int32");
    return SDR_EINVAL;
  }
  std::vector<int> rp(A->n + 1), ci(A->nnz);
  HIPCHK(hipMemcpy(rp.data(), A->row_ptr, sizeof(int) * (A->n + 1), hipMemcpyDeviceToHost));
  if (A->nnz) HIPCHK(hipMemcpy(ci.data(), A->col_idx, sizeof(int) * A->nnz, hipMemcpyDeviceToHost));
  if (rp[0] != 0 || rp[A->n] != A->nnz) {
    set_err("row_ptr must start at 0 and end at nnz");
    return SDR_EINVAL;
  }
  for (int64_t i = 0; i < A->n; ++i)
    if (rp[i + 1] < rp[i]) {
      set_err("row_ptr must be non-decreasing");
      return SDR_EINVAL;
    }
  for (int64_t e = 0; e < A->nnz; ++e)
    if (ci[e] < 0 || ci[e] >= A->n) {
      set_err("column index out of range");
      return SDR_EINVAL;
    }
  if (rp_out) *rp_out = std::move(rp);
  if (ci_out) *ci_out = std::move(ci);
  return SDR_OK;
}

void build_adjoint(sdr_handle* h) {
  if (h->adj_ready) return;
  std::vector<int> rp(h->n + 1), ci(h->nnz);
  HIPCHK(hipMemcpy(rp.data(), h->rp, sizeof(int) * (h->n + 1), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(ci.data(), h->ci, sizeof(int) * h->nnz, hipMemcpyDeviceToHost));
  std::vector<int> rpT(h->n + 1, 0), ciT(h->nnz), perm(h->nnz);
  for (int64_t e = 0; e < h->nnz; ++e) rpT[ci[e] + 1]++;
  for (int i = 0; i < h->n; ++i) rpT[i + 1] += rpT[i];
  std::vector<int> fill(rpT.begin(), rpT.end() - 1);
  for (int i = 0; i < h->n; ++i)
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      const int d = fill[ci[e]]++;
      ciT[d] = i;
      perm[d] = e;
    }
  h->rpT = dalloc<int>(h->n + 1);
  h->ciT = dalloc<int>(h->nnz);
  h->perm = dalloc<int>(h->nnz);
  h->valsT = dalloc<unsigned char>(h->elem() * h->nnz);
  HIPCHK(hipMemcpy(h->rpT, rpT.data(), sizeof(int) * (h->n + 1), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->ciT, ciT.data(), sizeof(int) * h->nnz, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->perm, perm.data(), sizeof(int) * h->nnz, hipMemcpyHostToDevice));
  HIPCHK(hipStreamSynchronize(nullptr));  // (the adjoint's kernels run on a non-blocking stream)
  h->adj_ready = true;
}

void refresh_adjoint_values(sdr_handle* h) {
  if (!h->adj_ready) return;
  if (h->cpx)
    launch_gather_conj<cx<double>>(h->stream, h->nnz, static_cast<const cx<double>*>(h->vals), h->perm,
                                   static_cast<cx<double>*>(h->valsT));
  else
    launch_gather_conj<double>(h->stream, h->nnz, static_cast<const double*>(h->vals), h->perm,
                               static_cast<double*>(h->valsT));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
}

}  // namespace

extern "C" {

const char* sdr_last_error(void) { return g_err.c_str(); }

sdr_handle* sdr_create(const sdr_csr* A, int m, int k, int t, int s_dim, uint64_t seed) {
  g_err.clear();
  sdr_handle* h = nullptr;
  try {
    std::vector<int> rp, ci;
    if (validate_csr(A, &rp, &ci) != SDR_OK) return nullptr;
    if (m < 1 || k < 0 || t < 1 || t > m || t > kMaxWindow || s_dim <= m + k) {
      set_err("invalid parameters: need m>=1, k>=0, 1<=t<=min(m,4), s_dim>m+k");
      return nullptr;
    }
    {
      // one LDS accumulator copy of the sketch per wave of the streaming kernels
      const size_t esz = A->dtype == SDR_C128 ? 16 : 8;
      if ((size_t)kWaves * (size_t)s_dim * esz > (size_t)kSpmvLds) {
        set_err("s_dim too large: need s_dim <= " + std::to_string(kSpmvLds / (kWaves * esz)));
        return nullptr;
      }
    }
    h = new sdr_handle();
    h->n = (int)A->n;
    h->nnz = A->nnz;
    h->m = m;
    h->k = k;
    h->t = t;
    h->s = s_dim;
    h->seed = seed;
    h->cpx = A->dtype == SDR_C128;
    h->pattern_hash = hash_pattern(rp, ci);
    HIPCHK(hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
    h->stream = h->own;
    h->rp = dalloc<int>(h->n + 1);
    h->ci = dalloc<int>(h->nnz);
    h->vals = dalloc<unsigned char>(h->elem() * h->nnz);
    HIPCHK(hipMemcpy(h->rp, A->row_ptr, sizeof(int) * (h->n + 1), hipMemcpyDeviceToDevice));
    if (h->nnz) {
      HIPCHK(hipMemcpy(h->ci, A->col_idx, sizeof(int) * h->nnz, hipMemcpyDeviceToDevice));
      HIPCHK(hipMemcpy(h->vals, A->values, h->elem() * h->nnz, hipMemcpyDeviceToDevice));
    }
    // device-to-device copies may return before they finish, and the handle's
    // kernels run on non-blocking streams: complete them here
    HIPCHK(hipStreamSynchronize(nullptr));
    return h;
  } catch (HipError&) {
    if (h) sdr_destroy(h);
    return nullptr;
  }
}

int sdr_set_option(sdr_handle* h, const char* key, double v) {
  if (!h || !key) {
    set_err("null handle or key");
    return SDR_EINVAL;
  }
  const std::string k(key);
  const bool built = (bool)h->fwd;
  if (k == "zeta") {
    const int z = (int)v;
    if (built || z < 1 || z > 32) {
      set_err("zeta must divide s_dim, be in [1,32] and be set before the first solve");
      return SDR_EINVAL;
    }
    h->opt.zeta = z;
  } else if (k == "max_cycles") {
    if (v < 1) return set_err("max_cycles >= 1"), SDR_EINVAL;
    h->opt.max_cycles = (int)v;
  } else if (k == "safety0") {
    if (!(v >= 1.0)) return set_err("safety0 >= 1"), SDR_EINVAL;
    h->opt.safety0 = v;
  } else if (k == "persist_safety") {
    h->opt.persist_safety = v != 0.0;
  } else if (k == "precision") {
    if (built || (v != 0.0 && v != 1.0)) {
      set_err("precision is 0 or 1 and must be set before the first solve");
      return SDR_EINVAL;
    }
    h->opt.precision = (int)v;
  } else if (k == "variant") {
    if (built || (v != 0.0 && v != 1.0)) {
      set_err("variant is 0 or 1 and must be set before the first solve");
      return SDR_EINVAL;
    }
    h->opt.variant = (int)v;
  } else if (k == "breakdown_rtol") {
    if (built || !(v >= 0.0)) return set_err("breakdown_rtol >= 0, before the first solve"), SDR_EINVAL;
    h->opt.brtol = v;
  } else if (k == "rank_rtol") {
    if (built || !(v >= 0.0)) return set_err("rank_rtol >= 0, before the first solve"), SDR_EINVAL;
    h->opt.rank_rtol = v;
  } else if (k == "kernel_timing") {
    if (built || !(v >= 0.0 && v <= 1e6)) return set_err("kernel_timing in [0,1e6], before the first solve"), SDR_EINVAL;
    h->opt.kernel_timing = (int)v;
  } else if (k == "dia") {
    if (built || (v != 0.0 && v != 1.0)) return set_err("dia is 0 or 1, before the first solve"), SDR_EINVAL;
    h->opt.dia = (int)v;
  } else if (k == "dia_const") {
    if (built || (v != 0.0 && v != 1.0))
      return set_err("dia_const is 0 or 1, before the first solve"), SDR_EINVAL;
    h->opt.dia_const = (int)v;
  } else if (k == "precond") {
    if (built || (v != 0.0 && v != 1.0 && v != 2.0))
      return set_err("precond is 0, 1 (Jacobi) or 2 (ILU(0)), before the first solve"), SDR_EINVAL;
    h->opt.precond = (int)v;
  } else if (k == "sketch") {
    if (built || (v != 0.0 && v != 1.0))
      return set_err("sketch is 0 (sparse sign) or 1 (subsampled DCT), before the first solve"), SDR_EINVAL;
    h->opt.sketch = (int)v;
  } else if (k == "resid_control") {
    if (v != 0.0 && v != 1.0) return set_err("resid_control is 0 (safety) or 1 (Givens)"), SDR_EINVAL;
    h->opt.resid_control = (int)v;
  } else if (k == "givens_eps0") {
    if (!(v >= 0.0 && v < 1.0)) return set_err("givens_eps0 in [0, 1)"), SDR_EINVAL;
    h->opt.givens_eps0 = v;
  } else if (k == "lsq_kernel") {
    if (v != 0.0 && v != 1.0 && v != 2.0 && v != 3.0)
      return set_err("lsq_kernel is 0 (automatic), 1 (block, one workgroup), 2 (one launch per step) or 3 "
                     "(block, several workgroups)"),
             SDR_EINVAL;
    h->opt.lsq_kernel = (int)v;
  } else if (k == "lsq_chunk") {
    if (built || v < 1 || v > 64) return set_err("lsq_chunk in [1,64], before the first solve"), SDR_EINVAL;
    h->opt.lsq_chunk = (int)v;
  } else {
    set_err("unknown option " + k);
    return SDR_EINVAL;
  }
  if (h->fwd) h->fwd->set_options(h->opt);
  if (h->adj) h->adj->set_options(h->opt);
  return SDR_OK;
}

int sdr_set_stream(sdr_handle* h, void* s) {
  if (!h) return set_err("null handle"), SDR_EINVAL;
  // NULL: the handle's own (non-blocking) stream, made to wait at each call
  // for the work queued on the null stream before it (running the solver on
  // the legacy null stream itself costs launch time)
  h->follow_null = s == nullptr;
  h->stream = s ? static_cast<hipStream_t>(s) : h->own;
  if (h->fwd) h->fwd->set_stream(h->stream);
  if (h->adj) h->adj->set_stream(h->stream);
  return SDR_OK;
}

namespace {
// Order the call's work after the caller's null-stream work (see sdr_set_stream).
void order_after_caller(sdr_handle* h) {
  if (!h->follow_null) return;
  HIPCHK(hipEventRecord(h->ev_in, nullptr));
  HIPCHK(hipStreamWaitEvent(h->own, h->ev_in, 0));
}

// For a call that returns without waiting: the caller's later null-stream
// work is ordered after the call's work on the handle's own stream (a wait
// on the device, not on the host).
void order_caller_after(sdr_handle* h) {
  if (!h->follow_null) return;
  HIPCHK(hipEventRecord(h->ev_in, h->own));
  HIPCHK(hipStreamWaitEvent(nullptr, h->ev_in, 0));
}
}  // namespace

int sdr_update_matrix(sdr_handle* h, const sdr_csr* A) {
  if (!h) return set_err("null handle"), SDR_EINVAL;
  try {
    std::vector<int> rp, ci;
    int rc = validate_csr(A, &rp, &ci);
    if (rc != SDR_OK) return rc;
    if (A->n != h->n || A->nnz != h->nnz || (A->dtype == SDR_C128) != h->cpx ||
        hash_pattern(rp, ci) != h->pattern_hash) {
      set_err("matrix pattern differs from the handle's");
      return SDR_EPATTERN;
    }
    order_after_caller(h);
    HIPCHK(hipMemcpyAsync(h->vals, A->values, h->elem() * h->nnz, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    // Both solvers learn of the new values before the preconditioner is
    // refreshed: a rejected preconditioner (zero diagonal) throws, and the
    // adjoint solve, which uses A itself, must still see the new matrix.
    if (h->fwd) h->fwd->matrix_changed();
    if (h->adj) h->adj->matrix_changed();
    refresh_adjoint_values(h);
    if (h->fwd) refresh_precond(h);
    return SDR_OK;
  } catch (HipError& e) {
    return e.code;
  }
}

int sdr_solve(sdr_handle* h, const sdr_csr* A, const void* b, void* x, double tol, sdr_stats* st) {
  if (!h || !b || !x || !(tol > 0.0)) return set_err("null argument or tol <= 0"), SDR_EINVAL;
  g_err.clear();
  try {
    if (A) {
      int rc = sdr_update_matrix(h, A);
      if (rc != SDR_OK) return rc;
    }
    order_after_caller(h);
    SolverBase* f = fwd(h);
    if (h->opt.precond == 0) return f->solve(b, x, tol, st, &h->trace);
    if (h->pc_bad) {
      set_err(h->opt.precond == 2 ? "ILU(0) preconditioning of the current matrix failed (zero pivot)"
                                  : "Jacobi preconditioning needs every diagonal entry of A stored and nonzero");
      return SDR_EINVAL;
    }
    if (h->opt.precond == 2) {
      ilu_transform(h, x, true);  // the initial guess u0 = M x0
      const int rc = f->solve(b, x, tol, st, &h->trace);
      ilu_transform(h, x, false);  // x = M^-1 u
      HIPCHK(hipStreamSynchronize(h->stream));
      return rc;
    }
    precond_scale(h, x, true);  // the initial guess u0 = D x0
    const int rc = f->solve(b, x, tol, st, &h->trace);
    precond_scale(h, x, false);  // x = D^-1 u
    HIPCHK(hipStreamSynchronize(h->stream));
    return rc;
  } catch (HipError& e) {
    return e.code;
  }
}

int sdr_solve_adjoint(sdr_handle* h, const void* g, void* lam, double tol, sdr_stats* st) {
  if (!h || !g || !lam || !(tol > 0.0)) return set_err("null argument or tol <= 0"), SDR_EINVAL;
  g_err.clear();
  try {
    if (!h->adj_ready) {
      build_adjoint(h);
      refresh_adjoint_values(h);
    }
    if (h->opt.sketch == 0 && h->s % h->opt.zeta != 0)
      return set_err("s_dim must be a multiple of zeta"), SDR_EINVAL;
    if (!h->adj) h->adj = make_solver(h, true);
    std::vector<sdr_cycle_record> tr;
    order_after_caller(h);
    return h->adj->solve(g, lam, tol, st, &tr);
  } catch (HipError& e) {
    return e.code;
  }
}

int sdr_grad_values(sdr_handle* h, const void* lam, const void* x, void* g) {
  if (!h || !lam || !x || !g) return set_err("null argument"), SDR_EINVAL;
  try {
    order_after_caller(h);
    if (h->cpx)
      launch_grad_values<cx<double>>(h->stream, h->n, h->rp, h->ci, static_cast<const cx<double>*>(lam),
                                     static_cast<const cx<double>*>(x), static_cast<cx<double>*>(g));
    else
      launch_grad_values<double>(h->stream, h->n, h->rp, h->ci, static_cast<const double*>(lam),
                                 static_cast<const double*>(x), static_cast<double*>(g));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    return SDR_OK;
  } catch (HipError& e) {
    return e.code;
  }
}

int sdr_get_trace(sdr_handle* h, sdr_cycle_record* out, int cap) {
  if (!h) return set_err("null handle"), SDR_EINVAL;
  const int n = std::min<int>(cap, (int)h->trace.size());
  if (out && n > 0) std::memcpy(out, h->trace.data(), sizeof(sdr_cycle_record) * n);
  return (int)h->trace.size();
}

int sdr_get_recycle(sdr_handle* h, void* U, void* SU, void* SAU, int* k) {
  if (!h) return set_err("null handle"), SDR_EINVAL;
  try {
    order_after_caller(h);
    return fwd(h)->get_recycle(U, SU, SAU, k);
  } catch (HipError& e) {
    return e.code;
  }
}

int sdr_sketch(sdr_handle* h, const void* X, int ncols, void* Y) {
  if (!h || !X || !Y || ncols < 0) return set_err("bad argument"), SDR_EINVAL;
  try {
    order_after_caller(h);
    return fwd(h)->sketch(X, ncols, Y);
  } catch (HipError& e) {
    return e.code;
  }
}

int sdr_precond_apply(sdr_handle* h, const void* v, void* z) {
  if (!h || !v || !z) return set_err("bad argument"), SDR_EINVAL;
  g_err.clear();
  try {
    order_after_caller(h);
    (void)fwd(h);  // (builds and factors the preconditioner)
    if (h->pc_bad) return set_err("the preconditioner of the current matrix failed"), SDR_EINVAL;
    if (h->opt.precond == 2) {  // straight into z, the forward solution in the handle's scratch
      if (h->cpx)
        launch_ilu_apply<cx<double>>(h->stream, h->ilu, static_cast<const cx<double>*>(v),
                                     static_cast<cx<double>*>(h->ilu_t), static_cast<cx<double>*>(z), nullptr);
      else
        launch_ilu_apply<double>(h->stream, h->ilu, static_cast<const double*>(v),
                                 static_cast<double*>(h->ilu_t), static_cast<double*>(z), nullptr);
      HIPCHK(hipGetLastError());
    } else {
      HIPCHK(hipMemcpyAsync(z, v, h->elem() * h->n, hipMemcpyDeviceToDevice, h->stream));
      if (h->opt.precond == 1) precond_scale(h, z, false);
    }
    order_caller_after(h);
    return SDR_OK;  // queued on the handle's stream
  } catch (HipError& e) {
    return e.code;
  }
}

int sdr_spmv(sdr_handle* h, const void* x, void* y) {
  if (!h || !x || !y) return set_err("bad argument"), SDR_EINVAL;
  try {
    order_after_caller(h);
    Ctrl* c = dalloc<Ctrl>(1);
    HIPCHK(hipMemsetAsync(c, 0, sizeof(Ctrl), h->stream));
    const int nb = (h->n + kRowsSpmv - 1) / kRowsSpmv;
    if (h->cpx) {
      auto* part = dalloc<cx<double>>((size_t)nb * (kMaxWindow + 1));
      Window<cx<double>> win{};
      launch_spmv_sketch<cx<double>>(h->stream, h->n, h->rp, h->ci,
                                     static_cast<const cx<double>*>(h->vals),
                                     static_cast<const cx<double>*>(x), static_cast<cx<double>*>(y), win,
                                     0, SketchSpec{}, true, part, nb, c);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(h->stream));
      dfree(part);
    } else {
      auto* part = dalloc<double>((size_t)nb * (kMaxWindow + 1));
      Window<double> win{};
      launch_spmv_sketch<double>(h->stream, h->n, h->rp, h->ci, static_cast<const double*>(h->vals),
                                 static_cast<const double*>(x), static_cast<double*>(y), win, 0,
                                 SketchSpec{}, true, part, nb, c);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(h->stream));
      dfree(part);
    }
    dfree(c);
    return SDR_OK;
  } catch (HipError& e) {
    return e.code;
  }
}

int sdr_get_basis(sdr_handle* h, int ncols, void* V, void* H, void* SV) {
  if (!h) return set_err("null handle"), SDR_EINVAL;
  try {
    order_after_caller(h);
    return fwd(h)->get_basis(ncols, V, H, SV);
  } catch (HipError& e) {
    return e.code;
  }
}

int sdr_get_step_sres(sdr_handle* h, double* out, int cap) {
  if (!h || cap < 0) return set_err("null handle or cap < 0"), SDR_EINVAL;
  if (!h->fwd) return 0;
  return h->fwd->step_sres(out, cap);
}

int sdr_reset(sdr_handle* h) {
  if (!h) return set_err("null handle"), SDR_EINVAL;
  if (h->fwd) h->fwd->reset();
  if (h->adj) h->adj->reset();
  return SDR_OK;
}

int sdr_kernel_times(sdr_handle* h, double* ms, int64_t* counts, int cap) {
  if (!h) return set_err("null handle"), SDR_EINVAL;
  try {
    return fwd(h)->kernel_times(ms, counts, cap);
  } catch (HipError& e) {
    return e.code;
  }
}

int sdr_spmv_layout(sdr_handle* h, int* offsets, int cap) {
  if (!h) return set_err("null handle"), SDR_EINVAL;
  try {
    return fwd(h)->spmv_layout(offsets, cap);
  } catch (HipError& e) {
    return e.code;
  }
}

int sdr_spmv_const_diagonals(sdr_handle* h) {
  if (!h) return set_err("null handle"), SDR_EINVAL;
  try {
    return (int)fwd(h)->const_diagonals();
  } catch (HipError& e) {
    return e.code;
  }
}

void sdr_destroy(sdr_handle* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  h->fwd.reset();
  h->adj.reset();
  for (void* p : {(void*)h->rp, (void*)h->ci, h->vals, (void*)h->rpT, (void*)h->ciT, (void*)h->perm,
                  h->valsT, h->d_pc, h->vals_pc, (void*)h->pc_flag, (void*)h->ilu_crow, (void*)h->ilu_dpos,
                  (void*)h->ilu_lo_off, (void*)h->ilu_up_off, (void*)h->ilu_lo, (void*)h->ilu_up,
                  (void*)h->ilu_kind, h->ilu_F, h->ilu_t, h->ilu_u, (void*)h->ilu_lsrc, (void*)h->ilu_usrc,
                  (void*)h->ilu_lcol, (void*)h->ilu_ucol, (void*)h->ilu_lslice, (void*)h->ilu_lw,
                  (void*)h->ilu_uslice, (void*)h->ilu_uw, h->ilu_lval, h->ilu_uval, h->ilu_dinv})
    dfree(p);
  if (h->own) (void)hipStreamDestroy(h->own);
  if (h->ev_in) (void)hipEventDestroy(h->ev_in);
  delete h;
}

int sdr_host_harmonic_ritz(int l0, const void* R, const void* C, int s, int k, int is_complex,
                           void* G, int* ell) {
  if (l0 < 0 || k < 0 || (l0 > 0 && (!R || !C || !G)) || !ell) return set_err("bad argument"), SDR_EINVAL;
  std::vector<std::complex<double>> Rc((size_t)l0 * l0), Cc((size_t)l0 * l0), Gv;
  for (size_t i = 0; i < Rc.size(); ++i) {
    if (is_complex) {
      Rc[i] = static_cast<const std::complex<double>*>(R)[i];
      Cc[i] = static_cast<const std::complex<double>*>(C)[i];
    } else {
      Rc[i] = static_cast<const double*>(R)[i];
      Cc[i] = static_cast<const double*>(C)[i];
    }
  }
  const int keff = dense::harmonic_ritz(l0, Rc.data(), Cc.data(), s, k, !is_complex, Gv, ell);
  if (keff < 0) return set_err("Schur iteration did not converge"), SDR_EDEVICE;
  for (size_t i = 0; i < Gv.size(); ++i) {
    if (is_complex)
      static_cast<std::complex<double>*>(G)[i] = Gv[i];
    else
      static_cast<double*>(G)[i] = Gv[i].real();
  }
  return keff;
}

}  // extern "C"
