// Host small-dense linear algebra for the sketched harmonic-Ritz step
// (Section 3.5): the ordered generalised Schur decomposition of the pencil
// (M_ell, Sigma_ell) is computed as the ordered Schur decomposition of
// Sigma_ell^{-1} M_ell, whose invariant subspace is the pencil's right
// deflating subspace because Sigma_ell is diagonal and positive.  When the
// triangular factor R of SAW = Q R is comfortably far from the truncation
// threshold, the truncated SVD keeps every singular value and the matrix is
// similar (by the unitary right singular vectors) to R^{-1} Q^H [SU, SV], the
// minimum-norm solution of eq. (3.6); that matrix is used directly and the SVD
// is skipped.
#include "dense.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <limits>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

namespace sdr {
namespace dense {

// Helper threads for the column-parallel loops of the eigen-step (the
// triangular inverse and product, the leading Schur vectors): started on first use and kept for the life of
// the process.  parallel_for(n, fn) calls fn(i) for every i < n, spread over
// the calling thread and the helpers by an atomic counter, and returns when
// all calls are done; concurrent callers take turns.  Each fn(i) writes data
// of its own, so results do not depend on the thread count.  A helper polls
// for the next job for about 0.2 ms before it sleeps, so the loops of one
// eigen-step start without a wake-up each.
class ColumnPool {
 public:
  static ColumnPool& instance() {
    static ColumnPool* p = new ColumnPool();  // (kept: helpers are never joined)
    return *p;
  }
  int helpers() const { return helpers_; }
  void parallel_for(int n, const std::function<void(int)>& fn) {
    if (n <= 1 || helpers_ == 0) {
      for (int i = 0; i < n; ++i) fn(i);
      return;
    }
    std::lock_guard<std::mutex> turn(run_mu_);
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn;
      n_ = n;
      next_.store(0, std::memory_order_relaxed);
      busy_.store(helpers_, std::memory_order_relaxed);
      gen_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
    work();
    for (int spin = 0; busy_.load(std::memory_order_acquire) != 0; ++spin) {
      if (spin > 4096) {
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [this] { return busy_.load(std::memory_order_acquire) == 0; });
        break;
      }
      std::this_thread::yield();
    }
  }

 private:
  ColumnPool() {
    const unsigned hw = std::thread::hardware_concurrency();
    helpers_ = hw >= 8 ? 3 : hw >= 2 ? (int)hw - 1 : 0;
    for (int t = 0; t < helpers_; ++t) std::thread([this] { loop(); }).detach();
  }
  void work() {
    const int n = n_;
    for (int i = next_.fetch_add(1); i < n; i = next_.fetch_add(1)) (*fn_)(i);
  }
  void loop() {
    long seen = 0;
    for (;;) {
      const auto t0 = std::chrono::steady_clock::now();
      while (gen_.load(std::memory_order_acquire) == seen &&
             std::chrono::steady_clock::now() - t0 < std::chrono::microseconds(200)) {
      }
      if (gen_.load(std::memory_order_acquire) == seen) {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return gen_.load(std::memory_order_acquire) != seen; });
      }
      seen = gen_.load(std::memory_order_acquire);
      work();
      if (busy_.fetch_sub(1, std::memory_order_acq_rel) == 1) {
        std::lock_guard<std::mutex> lk(mu_);
        done_cv_.notify_all();
      }
    }
  }
  int helpers_ = 0;
  std::mutex run_mu_, mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)>* fn_ = nullptr;
  int n_ = 0;
  std::atomic<int> next_{0}, busy_{0};
  std::atomic<long> gen_{0};
};

static inline double abs1(cd z) { return std::fabs(z.real()) + std::fabs(z.imag()); }

// Rotation G = [[c, s], [-conj(s), c]] with G [x; y] = [r; 0], c real.
static inline void givens(cd x, cd y, double& c, cd& s) {
  const double ay = std::abs(y);
  if (ay == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  const double ax = std::abs(x);
  if (ax == 0.0) {
    c = 0.0;
    s = std::conj(y) / ay;
    return;
  }
  const double r = std::hypot(ax, ay);
  c = ax / r;
  s = (x / ax) * std::conj(y) / r;
}

bool schur(Mat& T, Mat& Z) {
  const int n = T.n;
  Z = Mat(n, n);
  for (int i = 0; i < n; ++i) Z(i, i) = 1.0;
  if (n <= 1) return true;
  // Householder reduction to upper Hessenberg form, T <- P T P, Z <- Z P.
  std::vector<cd> v(n), wrk(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int len = n - k - 1;
    double xn = 0.0;
    for (int i = 0; i < len; ++i) xn += std::norm(T(k + 1 + i, k));
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const cd x0 = T(k + 1, k);
    const double ax0 = std::abs(x0);
    const cd alpha = -(ax0 > 0.0 ? x0 / ax0 : cd(1.0, 0.0)) * xn;
    for (int i = 0; i < len; ++i) v[i] = T(k + 1 + i, k);
    v[0] -= alpha;
    double vn2 = 0.0;
    for (int i = 0; i < len; ++i) vn2 += std::norm(v[i]);
    if (vn2 == 0.0) continue;
    const double f = 2.0 / vn2;
    for (int j = k; j < n; ++j) {
      cd s = 0.0;
      for (int i = 0; i < len; ++i) s += std::conj(v[i]) * T(k + 1 + i, j);
      s *= f;
      for (int i = 0; i < len; ++i) T(k + 1 + i, j) -= v[i] * s;
    }
    // right: M(:, k+1:) -= f (M(:, k+1:) v) v^H, column by column
    for (Mat* Mp : {&T, &Z}) {
      cd* M = Mp->a.data();
      std::fill(wrk.begin(), wrk.end(), cd(0.0));
      for (int l = 0; l < len; ++l) {
        const cd* col = M + (size_t)(k + 1 + l) * n;
        const cd vl = v[l];
        for (int i = 0; i < n; ++i) wrk[i] += col[i] * vl;
      }
      for (int i = 0; i < n; ++i) wrk[i] *= f;
      for (int l = 0; l < len; ++l) {
        cd* col = M + (size_t)(k + 1 + l) * n;
        const cd cv = std::conj(v[l]);
        for (int i = 0; i < n; ++i) col[i] -= wrk[i] * cv;
      }
    }
    T(k + 1, k) = alpha;
    for (int i = 1; i < len; ++i) T(k + 1 + i, k) = 0.0;
  }
  // Single-shift QR iteration with Wilkinson shifts and deflation.
  const double eps = std::numeric_limits<double>::epsilon();
  double anorm = 0.0;
  for (auto& z : T.a) anorm = std::max(anorm, abs1(z));
  int hi = n - 1, iter = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    for (; l > 0; --l) {
      double sc = abs1(T(l - 1, l - 1)) + abs1(T(l, l));
      if (sc == 0.0) sc = anorm;
      if (abs1(T(l, l - 1)) <= eps * sc) break;
    }
    if (l > 0) T(l, l - 1) = 0.0;
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    cd mu;
    if (iter > 0 && iter % 10 == 0) {
      mu = T(hi, hi) + cd(0.75 * abs1(T(hi, hi - 1)), 0.0);  // exceptional shift
    } else {
      const cd a = T(hi - 1, hi - 1), b = T(hi - 1, hi), c = T(hi, hi - 1), d = T(hi, hi);
      const cd tr = 0.5 * (a + d);
      const cd disc = std::sqrt(0.25 * (a - d) * (a - d) + b * c);
      const cd m1 = tr + disc, m2 = tr - disc;
      mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    }
    cd x = T(l, l) - mu, y = T(l + 1, l);
    for (int k = l; k < hi; ++k) {
      if (k > l) {
        x = T(k, k - 1);
        y = T(k + 1, k - 1);
      }
      double c;
      cd s;
      givens(x, y, c, s);
      for (int j = std::max(l, k - 1); j < n; ++j) {
        const cd t1 = T(k, j), t2 = T(k + 1, j);
        T(k, j) = c * t1 + s * t2;
        T(k + 1, j) = -std::conj(s) * t1 + c * t2;
      }
      const int rmax = std::min(k + 2, hi);
      for (int i = 0; i <= rmax; ++i) {
        const cd t1 = T(i, k), t2 = T(i, k + 1);
        T(i, k) = c * t1 + std::conj(s) * t2;
        T(i, k + 1) = -s * t1 + c * t2;
      }
      for (int i = 0; i < n; ++i) {
        const cd t1 = Z(i, k), t2 = Z(i, k + 1);
        Z(i, k) = c * t1 + std::conj(s) * t2;
        Z(i, k + 1) = -s * t1 + c * t2;
      }
      if (k > l) T(k + 1, k - 1) = 0.0;
    }
    ++iter;
    if (++total > 60 * n) return false;
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) T(i, j) = 0.0;
  return true;
}

// ---------------------------------------------------------------------------
// Complex leading invariant subspace without the Schur vectors of the whole
// matrix.  The Hessenberg reduction keeps its reflectors instead of forming
// Z, the QR iteration updates only its active window (the eigenvalues do not
// need the rest of T) and logs its rotations, and the leading kk Schur
// vectors are formed afterwards from the log and the reflectors alone: Z =
// Q_h G_1 G_2 ... G_N, so Z(:, 1:kk) = Q_h (G_1 (... (G_N E_kk))), an n x kk
// product instead of n x n.  Valid when the selected eigenvalues occupy the
// leading diagonal positions, which the caller checks.
// ---------------------------------------------------------------------------
struct Rot {
  int k;
  double c, sr, si;  // G = [[c, s], [-conj(s), c]], s = sr + i si
};

// Split (real, imaginary) column-major n x n matrix: the loops below run on
// contiguous real arrays, which vectorise where std::complex does not.
struct SplitMat {
  int n = 0;
  std::vector<double> re, im;
  explicit SplitMat(int nn = 0) : n(nn), re((size_t)nn * nn, 0.0), im((size_t)nn * nn, 0.0) {}
  double& r(int i, int j) { return re[(size_t)j * n + i]; }
  double& c(int i, int j) { return im[(size_t)j * n + i]; }
};

// Householder reduction of T to upper Hessenberg form; reflector k (acting
// on rows k+1 .. n-1) is I - f_k v_k v_k^H with v_k in column k of (Vr, Vi),
// rows 0 .. n-k-2.
static void hessenberg_reflectors(SplitMat& T, std::vector<double>& Vr, std::vector<double>& Vi,
                                  std::vector<double>& F) {
  const int n = T.n;
  Vr.assign((size_t)n * n, 0.0);
  Vi.assign((size_t)n * n, 0.0);
  F.assign(n, 0.0);
  std::vector<double> wr(n), wi(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int len = n - k - 1;
    double* __restrict__ cr = T.re.data() + (size_t)k * n + k + 1;
    double* __restrict__ ci = T.im.data() + (size_t)k * n + k + 1;
    double xn = 0.0;
    for (int i = 0; i < len; ++i) xn += cr[i] * cr[i] + ci[i] * ci[i];
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const double ax0 = std::hypot(cr[0], ci[0]);
    const double ar = ax0 > 0.0 ? -cr[0] / ax0 * xn : -xn;
    const double ai = ax0 > 0.0 ? -ci[0] / ax0 * xn : 0.0;
    double* __restrict__ vr = Vr.data() + (size_t)k * n;
    double* __restrict__ vi = Vi.data() + (size_t)k * n;
    for (int i = 0; i < len; ++i) {
      vr[i] = cr[i];
      vi[i] = ci[i];
    }
    vr[0] -= ar;
    vi[0] -= ai;
    double vn2 = 0.0;
    for (int i = 0; i < len; ++i) vn2 += vr[i] * vr[i] + vi[i] * vi[i];
    if (vn2 == 0.0) continue;
    const double f = 2.0 / vn2;
    F[k] = f;
    // left: T(k+1:, j) -= v (f v^H T(k+1:, j)) for j > k
    for (int j = k + 1; j < n; ++j) {
      double* __restrict__ tr = T.re.data() + (size_t)j * n + k + 1;
      double* __restrict__ ti = T.im.data() + (size_t)j * n + k + 1;
      double sr = 0.0, si = 0.0;
      for (int i = 0; i < len; ++i) {
        sr += vr[i] * tr[i] + vi[i] * ti[i];
        si += vr[i] * ti[i] - vi[i] * tr[i];
      }
      sr *= f;
      si *= f;
      for (int i = 0; i < len; ++i) {
        tr[i] -= vr[i] * sr - vi[i] * si;
        ti[i] -= vr[i] * si + vi[i] * sr;
      }
    }
    // right: T(:, k+1:) -= (f T(:, k+1:) v) v^H
    std::fill(wr.begin(), wr.end(), 0.0);
    std::fill(wi.begin(), wi.end(), 0.0);
    for (int l = 0; l < len; ++l) {
      const double* __restrict__ tr = T.re.data() + (size_t)(k + 1 + l) * n;
      const double* __restrict__ ti = T.im.data() + (size_t)(k + 1 + l) * n;
      const double a = vr[l], b = vi[l];
      for (int i = 0; i < n; ++i) {
        wr[i] += tr[i] * a - ti[i] * b;
        wi[i] += tr[i] * b + ti[i] * a;
      }
    }
    for (int i = 0; i < n; ++i) {
      wr[i] *= f;
      wi[i] *= f;
    }
    for (int l = 0; l < len; ++l) {
      double* __restrict__ tr = T.re.data() + (size_t)(k + 1 + l) * n;
      double* __restrict__ ti = T.im.data() + (size_t)(k + 1 + l) * n;
      const double a = vr[l], b = vi[l];  // conj(v_l) = a - i b
      for (int i = 0; i < n; ++i) {
        tr[i] -= wr[i] * a + wi[i] * b;
        ti[i] -= wi[i] * a - wr[i] * b;
      }
    }
    cr[0] = ar;
    ci[0] = ai;
    for (int i = 1; i < len; ++i) cr[i] = ci[i] = 0.0;
  }
}

// Single-shift QR on the Hessenberg matrix T, updating only the active
// window [l, hi]; the diagonal holds the eigenvalues on return, in the
// positions the full iteration gives them.  Rotations are appended to log in
// the order applied.
static bool hessenberg_qr_window(SplitMat& T, std::vector<Rot>& log) {
  const int n = T.n;
  auto at = [&](int i, int j) { return cd(T.r(i, j), T.c(i, j)); };
  auto put = [&](int i, int j, cd v) {
    T.r(i, j) = v.real();
    T.c(i, j) = v.imag();
  };
  const double eps = std::numeric_limits<double>::epsilon();
  double anorm = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= std::min(j + 1, n - 1); ++i) anorm = std::max(anorm, abs1(at(i, j)));
  double* __restrict__ Re = T.re.data();
  double* __restrict__ Im = T.im.data();
  int hi = n - 1, iter = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    for (; l > 0; --l) {
      double sc = abs1(at(l - 1, l - 1)) + abs1(at(l, l));
      if (sc == 0.0) sc = anorm;
      if (abs1(at(l, l - 1)) <= eps * sc) break;
    }
    if (l > 0) put(l, l - 1, 0.0);
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    cd mu;
    if (iter > 0 && iter % 10 == 0) {
      mu = at(hi, hi) + cd(0.75 * abs1(at(hi, hi - 1)), 0.0);  // exceptional shift
    } else {
      const cd a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
      const cd tr = 0.5 * (a + d);
      const cd disc = std::sqrt(0.25 * (a - d) * (a - d) + b * c);
      const cd m1 = tr + disc, m2 = tr - disc;
      mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    }
    cd x = at(l, l) - mu, y = at(l + 1, l);
    for (int k = l; k < hi; ++k) {
      if (k > l) {
        x = at(k, k - 1);
        y = at(k + 1, k - 1);
      }
      double c;
      cd s;
      givens(x, y, c, s);
      const double sr = s.real(), si = s.imag();
      // rows k, k+1 over columns max(l, k-1) .. hi (stride n)
      for (int j = std::max(l, k - 1); j <= hi; ++j) {
        const size_t o = (size_t)j * n + k;
        const double ar = Re[o], ai = Im[o], br = Re[o + 1], bi = Im[o + 1];
        Re[o] = c * ar + (sr * br - si * bi);
        Im[o] = c * ai + (sr * bi + si * br);
        Re[o + 1] = -(sr * ar + si * ai) + c * br;  // -conj(s) a + c b
        Im[o + 1] = -(sr * ai - si * ar) + c * bi;
      }
      // columns k, k+1 over rows l .. min(k+2, hi) (contiguous)
      const int rmax = std::min(k + 2, hi);
      double* __restrict__ r0 = Re + (size_t)k * n;
      double* __restrict__ i0 = Im + (size_t)k * n;
      double* __restrict__ r1 = r0 + n;
      double* __restrict__ i1 = i0 + n;
      for (int i = l; i <= rmax; ++i) {
        const double ar = r0[i], ai = i0[i], br = r1[i], bi = i1[i];
        r0[i] = c * ar + (sr * br + si * bi);  // c a + conj(s) b
        i0[i] = c * ai + (sr * bi - si * br);
        r1[i] = -(sr * ar - si * ai) + c * br;  // -s a + c b
        i1[i] = -(sr * ai + si * ar) + c * bi;
      }
      log.push_back(Rot{k, c, sr, si});
      if (k > l) put(k + 1, k - 1, 0.0);
    }
    ++iter;
    if (++total > 60 * n) return false;
  }
  return true;
}

// Z(:, 0 .. kk-1) of the Schur form reached by the logged iteration, from the
// reflectors (Vr, Vi, F) and the rotation log: Y = Q_h G_1 ... G_N E_kk.
static void leading_schur_vectors(int n, int kk, const std::vector<double>& Vr, const std::vector<double>& Vi,
                                  const std::vector<double>& F, const std::vector<Rot>& log, Mat& Y) {
  // M = G_1 ... G_N E_kk, rows contiguous (n x kk, split): G on rows k, k+1.
  // Columns are independent: parts of up to 8 columns go to the helper
  // threads, each applying the whole log, then the reflectors, to its own.
  constexpr int kPart = 8;
  std::vector<double> Yr((size_t)n * kk), Yi((size_t)n * kk);
  const int parts = (kk + kPart - 1) / kPart;
  ColumnPool::instance().parallel_for(parts, [&](int part) {
    const int j0 = part * kPart, w = std::min(kk, j0 + kPart) - j0;
    // this part's columns of M in a buffer of its own (no cache line shared
    // with another part), rows contiguous
    std::vector<double> Mr((size_t)n * w, 0.0), Mi((size_t)n * w, 0.0);
    for (int j = 0; j < w; ++j) Mr[(size_t)(j0 + j) * w + j] = 1.0;
    int top = j0 + w - 1;  // rows beyond top are zero in these columns
    for (auto it = log.rbegin(); it != log.rend(); ++it) {
      const int k = it->k;
      if (k > top) continue;
      const double c = it->c, sr = it->sr, si = it->si;
      double* __restrict__ ar = Mr.data() + (size_t)k * w;
      double* __restrict__ ai = Mi.data() + (size_t)k * w;
      double* __restrict__ br = ar + w;
      double* __restrict__ bi = ai + w;
      for (int j = 0; j < w; ++j) {
        const double xr = ar[j], xi = ai[j], yr = br[j], yi = bi[j];
        ar[j] = c * xr - (sr * yr - si * yi);  // c a - s b
        ai[j] = c * xi - (sr * yi + si * yr);
        br[j] = (sr * xr + si * xi) + c * yr;  // conj(s) a + c b
        bi[j] = (sr * xi - si * xr) + c * yi;
      }
      if (k + 1 > top) top = k + 1;
    }
    // Y = Q_h M with Q_h = P_0 P_1 ... P_{n-3}: columns of Y split, column major
    for (int j = 0; j < w; ++j)
      for (int i = 0; i < n; ++i) {
        Yr[(size_t)(j0 + j) * n + i] = Mr[(size_t)i * w + j];
        Yi[(size_t)(j0 + j) * n + i] = Mi[(size_t)i * w + j];
      }
    for (int k = n - 3; k >= 0; --k) {
      const double f = F[k];
      if (f == 0.0) continue;
      const int len = n - k - 1;
      const double* __restrict__ vr = Vr.data() + (size_t)k * n;
      const double* __restrict__ vi = Vi.data() + (size_t)k * n;
      for (int j = j0; j < j0 + w; ++j) {
        double* __restrict__ yr = Yr.data() + (size_t)j * n + k + 1;
        double* __restrict__ yi = Yi.data() + (size_t)j * n + k + 1;
        double dr = 0.0, di = 0.0;
        for (int i = 0; i < len; ++i) {
          dr += vr[i] * yr[i] + vi[i] * yi[i];
          di += vr[i] * yi[i] - vi[i] * yr[i];
        }
        dr *= f;
        di *= f;
        for (int i = 0; i < len; ++i) {
          yr[i] -= vr[i] * dr - vi[i] * di;
          yi[i] -= vr[i] * di + vi[i] * dr;
        }
      }
    }
  });
  Y = Mat(n, kk);
  for (size_t i = 0; i < Y.a.size(); ++i) Y.a[i] = cd(Yr[i], Yi[i]);
}

// M(r0 : r0+len, c0 : c1] -= f v (v^T M(r0 : r0+len, c0 : c1]), four columns a
// pass (one sweep of v per four dot products and per four updates).
static void reflect_left(double* __restrict__ M, int n, int r0, int len, const double* __restrict__ v,
                         double f, int c0, int c1) {
  int j = c0;
  for (; j + 4 <= c1; j += 4) {
    double* __restrict__ a0 = M + (size_t)j * n + r0;
    double* __restrict__ a1 = a0 + n;
    double* __restrict__ a2 = a1 + n;
    double* __restrict__ a3 = a2 + n;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma omp simd reduction(+ : s0, s1, s2, s3)
    for (int i = 0; i < len; ++i) {
      s0 += v[i] * a0[i];
      s1 += v[i] * a1[i];
      s2 += v[i] * a2[i];
      s3 += v[i] * a3[i];
    }
    s0 *= f;
    s1 *= f;
    s2 *= f;
    s3 *= f;
    for (int i = 0; i < len; ++i) {
      a0[i] -= v[i] * s0;
      a1[i] -= v[i] * s1;
      a2[i] -= v[i] * s2;
      a3[i] -= v[i] * s3;
    }
  }
  for (; j < c1; ++j) {
    double* __restrict__ a0 = M + (size_t)j * n + r0;
    double s0 = 0.0;
#pragma omp simd reduction(+ : s0)
    for (int i = 0; i < len; ++i) s0 += v[i] * a0[i];
    s0 *= f;
    for (int i = 0; i < len; ++i) a0[i] -= v[i] * s0;
  }
}

// M(0 : n, c0 : c0+len) -= f (M(0 : n, c0 : c0+len) v) v^T, four columns a pass.
static void reflect_right(double* __restrict__ M, int n, int c0, int len, const double* __restrict__ v,
                          double f, double* __restrict__ w) {
  for (int i = 0; i < n; ++i) w[i] = 0.0;
  int l = 0;
  for (; l + 4 <= len; l += 4) {
    const double* __restrict__ a0 = M + (size_t)(c0 + l) * n;
    const double* __restrict__ a1 = a0 + n;
    const double* __restrict__ a2 = a1 + n;
    const double* __restrict__ a3 = a2 + n;
    const double v0 = v[l], v1 = v[l + 1], v2 = v[l + 2], v3 = v[l + 3];
    for (int i = 0; i < n; ++i) w[i] += a0[i] * v0 + a1[i] * v1 + a2[i] * v2 + a3[i] * v3;
  }
  for (; l < len; ++l) {
    const double* __restrict__ a0 = M + (size_t)(c0 + l) * n;
    const double v0 = v[l];
    for (int i = 0; i < n; ++i) w[i] += a0[i] * v0;
  }
  for (int i = 0; i < n; ++i) w[i] *= f;
  l = 0;
  for (; l + 4 <= len; l += 4) {
    double* __restrict__ a0 = M + (size_t)(c0 + l) * n;
    double* __restrict__ a1 = a0 + n;
    double* __restrict__ a2 = a1 + n;
    double* __restrict__ a3 = a2 + n;
    const double v0 = v[l], v1 = v[l + 1], v2 = v[l + 2], v3 = v[l + 3];
    for (int i = 0; i < n; ++i) {
      const double wi = w[i];
      a0[i] -= wi * v0;
      a1[i] -= wi * v1;
      a2[i] -= wi * v2;
      a3[i] -= wi * v3;
    }
  }
  for (; l < len; ++l) {
    double* __restrict__ a0 = M + (size_t)(c0 + l) * n;
    const double v0 = v[l];
    for (int i = 0; i < n; ++i) a0[i] -= w[i] * v0;
  }
}

// Householder reduction of T (n x n, column major) to upper Hessenberg form,
// T <- Z^T T Z with Z = P_0 P_1 ... P_{n-3}; Z is accumulated afterwards from
// the last reflector back (each P_k then acts on a trailing block only).
static void hessenberg(int n, std::vector<double>& T, std::vector<double>& Z) {
  auto t = [&](int i, int j) -> double& { return T[(size_t)j * n + i]; };
  std::vector<double> Vr((size_t)n * n, 0.0), F(n, 0.0), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int len = n - k - 1;
    double xn = 0.0;
    for (int i = 0; i < len; ++i) xn += t(k + 1 + i, k) * t(k + 1 + i, k);
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const double alpha = t(k + 1, k) > 0.0 ? -xn : xn;
    double* v = Vr.data() + (size_t)k * n;
    for (int i = 0; i < len; ++i) v[i] = t(k + 1 + i, k);
    v[0] -= alpha;
    double vn2 = 0.0;
    for (int i = 0; i < len; ++i) vn2 += v[i] * v[i];
    if (vn2 == 0.0) continue;
    const double f = 2.0 / vn2;
    F[k] = f;
    reflect_left(T.data(), n, k + 1, len, v, f, k + 1, n);
    reflect_right(T.data(), n, k + 1, len, v, f, w.data());
    t(k + 1, k) = alpha;
    for (int i = 1; i < len; ++i) t(k + 1 + i, k) = 0.0;
  }
  Z.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  for (int k = n - 3; k >= 0; --k) {
    if (F[k] == 0.0) continue;
    // Z(k+1:, k+1:) <- P_k Z(k+1:, k+1:): columns left of k+1 are untouched
    reflect_left(Z.data(), n, k + 1, n - k - 1, Vr.data() + (size_t)k * n, F[k], k + 1, n);
  }
}

// Real Schur form by Hessenberg reduction and Francis double-shift QR
// (real arithmetic throughout): A = Z T Z^T with T quasi-upper triangular.
// 2 x 2 diagonal blocks with real eigenvalues are split by a rotation, so every
// remaining 2 x 2 block holds a complex-conjugate pair.  T, Z column major.
static bool schur_real(int n, std::vector<double>& T, std::vector<double>& Z) {
  auto t = [&](int i, int j) -> double& { return T[(size_t)j * n + i]; };
  auto z = [&](int i, int j) -> double& { return Z[(size_t)j * n + i]; };
  if (n <= 1) {
    Z.assign((size_t)n * n, 1.0);
    return true;
  }
  hessenberg(n, T, Z);
  // reflector P = I - beta v v^T (len 2 or 3) applied to rows k.. (left) and
  // columns k.. (right) of T, and to columns of Z
  auto left = [&](int k, int len, const double* vv, double beta, int c0, int c1) {
    if (len == 3) {
      for (int j = c0; j <= c1; ++j) {
        double* c = &t(k, j);
        const double sm = (vv[0] * c[0] + vv[1] * c[1] + vv[2] * c[2]) * beta;
        c[0] -= sm * vv[0];
        c[1] -= sm * vv[1];
        c[2] -= sm * vv[2];
      }
    } else {
      for (int j = c0; j <= c1; ++j) {
        double* c = &t(k, j);
        const double sm = (vv[0] * c[0] + vv[1] * c[1]) * beta;
        c[0] -= sm * vv[0];
        c[1] -= sm * vv[1];
      }
    }
  };
  // columns k .. k+len-1 of M, rows 0 .. r1 (contiguous down each column)
  auto right = [&](std::vector<double>& M, int k, int len, const double* vv, double beta, int r1) {
    double* m0 = M.data() + (size_t)k * n;
    double* m1 = m0 + n;
    if (len == 3) {
      double* m2 = m1 + n;
      for (int i = 0; i <= r1; ++i) {
        const double sm = (m0[i] * vv[0] + m1[i] * vv[1] + m2[i] * vv[2]) * beta;
        m0[i] -= sm * vv[0];
        m1[i] -= sm * vv[1];
        m2[i] -= sm * vv[2];
      }
    } else {
      for (int i = 0; i <= r1; ++i) {
        const double sm = (m0[i] * vv[0] + m1[i] * vv[1]) * beta;
        m0[i] -= sm * vv[0];
        m1[i] -= sm * vv[1];
      }
    }
  };
  auto house = [](double* x, int len, double* vv, double& beta) {
    double nr = 0.0;
    for (int i = 0; i < len; ++i) nr += x[i] * x[i];
    nr = std::sqrt(nr);
    for (int i = 0; i < len; ++i) vv[i] = x[i];
    if (nr == 0.0) {
      beta = 0.0;
      return;
    }
    const double alpha = x[0] > 0.0 ? -nr : nr;
    vv[0] -= alpha;
    double vn2 = 0.0;
    for (int i = 0; i < len; ++i) vn2 += vv[i] * vv[i];
    beta = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
  };
  const double eps = std::numeric_limits<double>::epsilon();
  double anorm = 0.0;
  for (double x : T) anorm = std::max(anorm, std::fabs(x));
  int p = n - 1, iter = 0, total = 0;
  while (p > 0) {
    int l = p;
    for (; l > 0; --l) {
      double sc = std::fabs(t(l - 1, l - 1)) + std::fabs(t(l, l));
      if (sc == 0.0) sc = anorm;
      if (std::fabs(t(l, l - 1)) <= eps * sc) break;
    }
    if (l > 0) t(l, l - 1) = 0.0;
    if (l == p) {
      --p;
      iter = 0;
      continue;
    }
    if (l == p - 1) {
      // 2 x 2 block: split it if its eigenvalues are real
      const int i = p - 1;
      const double a = t(i, i), b = t(i, i + 1), c = t(i + 1, i), d = t(i + 1, i + 1);
      const double hp = 0.5 * (a - d), disc = hp * hp + b * c;
      if (disc >= 0.0) {
        const double lam = 0.5 * (a + d) + (hp >= 0.0 ? 1.0 : -1.0) * std::sqrt(disc);
        double v0, v1;
        if (std::fabs(lam - d) + std::fabs(c) >= std::fabs(b) + std::fabs(lam - a)) {
          v0 = lam - d;
          v1 = c;
        } else {
          v0 = b;
          v1 = lam - a;
        }
        const double nr = std::hypot(v0, v1);
        if (nr > 0.0) {
          const double cs = v0 / nr, sn = v1 / nr;  // G = [[cs, -sn], [sn, cs]]
          for (int r = 0; r < n; ++r) {
            const double x0 = t(r, i), x1 = t(r, i + 1);
            t(r, i) = cs * x0 + sn * x1;
            t(r, i + 1) = -sn * x0 + cs * x1;
          }
          for (int cc = 0; cc < n; ++cc) {
            const double x0 = t(i, cc), x1 = t(i + 1, cc);
            t(i, cc) = cs * x0 + sn * x1;
            t(i + 1, cc) = -sn * x0 + cs * x1;
          }
          for (int r = 0; r < n; ++r) {
            const double x0 = z(r, i), x1 = z(r, i + 1);
            z(r, i) = cs * x0 + sn * x1;
            z(r, i + 1) = -sn * x0 + cs * x1;
          }
          t(i + 1, i) = 0.0;
        }
      }
      p -= 2;
      iter = 0;
      continue;
    }
    double tr, det;
    if (iter > 0 && iter % 10 == 0) {  // exceptional shift
      const double sc = std::fabs(t(p, p - 1)) + std::fabs(t(p - 1, p - 2));
      tr = 1.5 * sc;
      det = sc * sc;
    } else {
      tr = t(p - 1, p - 1) + t(p, p);
      det = t(p - 1, p - 1) * t(p, p) - t(p - 1, p) * t(p, p - 1);
    }
    double x[3];
    x[0] = t(l, l) * t(l, l) + t(l, l + 1) * t(l + 1, l) - tr * t(l, l) + det;
    x[1] = t(l + 1, l) * (t(l, l) + t(l + 1, l + 1) - tr);
    x[2] = t(l + 1, l) * t(l + 2, l + 1);
    double vv[3], beta;
    for (int k = l; k <= p - 2; ++k) {
      house(x, 3, vv, beta);
      const int r = std::max(l, k - 1);
      left(k, 3, vv, beta, r, n - 1);
      const int rr = std::min(k + 3, p);
      right(T, k, 3, vv, beta, rr);
      right(Z, k, 3, vv, beta, n - 1);
      if (k > l) {
        t(k + 1, k - 1) = 0.0;
        t(k + 2, k - 1) = 0.0;
      }
      x[0] = t(k + 1, k);
      x[1] = t(k + 2, k);
      if (k < p - 2) x[2] = t(k + 3, k);
    }
    house(x, 2, vv, beta);
    left(p - 1, 2, vv, beta, p - 2, n - 1);
    right(T, p - 1, 2, vv, beta, p);
    right(Z, p - 1, 2, vv, beta, n - 1);
    t(p, p - 2) = 0.0;
    ++iter;
    if (++total > 60 * n) return false;
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 2; i < n; ++i) t(i, j) = 0.0;
  return true;
}

// Complex upper triangular form of a real Schur form: each 2 x 2 block (a
// conjugate pair) is triangularised by a unitary rotation whose first column
// is the block's eigenvector.  partner[i] is the other member of i's pair, or
// -1 for a real eigenvalue.
static void real_to_complex_schur(int n, const std::vector<double>& Tr, const std::vector<double>& Zr,
                                  Mat& T, Mat& Z, std::vector<int>& partner) {
  T = Mat(n, n);
  Z = Mat(n, n);
  for (size_t i = 0; i < Tr.size(); ++i) {
    T.a[i] = Tr[i];
    Z.a[i] = Zr[i];
  }
  partner.assign(n, -1);
  for (int i = 0; i + 1 < n; ++i) {
    if (T(i + 1, i) == cd(0.0)) continue;
    const cd a = T(i, i), b = T(i, i + 1), c = T(i + 1, i), d = T(i + 1, i + 1);
    const cd hp = 0.5 * (a - d);
    const cd lam = 0.5 * (a + d) + std::sqrt(hp * hp + b * c);
    cd v0 = b, v1 = lam - a;
    const double nr = std::hypot(std::abs(v0), std::abs(v1));
    v0 /= nr;
    v1 /= nr;
    for (int r = 0; r < n; ++r) {
      const cd t1 = T(r, i), t2 = T(r, i + 1);
      T(r, i) = t1 * v0 + t2 * v1;
      T(r, i + 1) = -t1 * std::conj(v1) + t2 * std::conj(v0);
    }
    for (int cc = 0; cc < n; ++cc) {
      const cd t1 = T(i, cc), t2 = T(i + 1, cc);
      T(i, cc) = std::conj(v0) * t1 + std::conj(v1) * t2;
      T(i + 1, cc) = -v1 * t1 + v0 * t2;
    }
    for (int r = 0; r < n; ++r) {
      const cd t1 = Z(r, i), t2 = Z(r, i + 1);
      Z(r, i) = t1 * v0 + t2 * v1;
      Z(r, i + 1) = -t1 * std::conj(v1) + t2 * std::conj(v0);
    }
    T(i + 1, i) = 0.0;
    partner[i] = i + 1;
    partner[i + 1] = i;
    ++i;
  }
}

// Exchange the diagonal entries i and i+1 of the upper triangular T by a
// unitary 2 x 2 rotation whose first column is the eigenvector of the
// trailing entry; update Z accordingly.
static void swap_adjacent(Mat& T, Mat& Z, int i) {
  const int n = T.n;
  const cd a = T(i, i), b = T(i + 1, i + 1), c = T(i, i + 1);
  const cd x0 = c, x1 = b - a;
  const double nr = std::hypot(std::abs(x0), std::abs(x1));
  if (nr == 0.0) return;
  const cd z0 = x0 / nr, z1 = x1 / nr;
  for (int r = 0; r <= i + 1; ++r) {
    const cd t1 = T(r, i), t2 = T(r, i + 1);
    T(r, i) = t1 * z0 + t2 * z1;
    T(r, i + 1) = -t1 * std::conj(z1) + t2 * std::conj(z0);
  }
  for (int cc = i; cc < n; ++cc) {
    const cd t1 = T(i, cc), t2 = T(i + 1, cc);
    T(i, cc) = std::conj(z0) * t1 + std::conj(z1) * t2;
    T(i + 1, cc) = -z1 * t1 + z0 * t2;
  }
  for (int r = 0; r < n; ++r) {
    const cd t1 = Z(r, i), t2 = Z(r, i + 1);
    Z(r, i) = t1 * z0 + t2 * z1;
    Z(r, i + 1) = -t1 * std::conj(z1) + t2 * std::conj(z0);
  }
  T(i + 1, i) = 0.0;
  T(i, i) = b;
  T(i + 1, i + 1) = a;
}

int reorder(Mat& T, Mat& Z, std::vector<char> sel) {
  const int n = T.n;
  int ks = 0;
  for (int i = 0; i < n; ++i) {
    if (!sel[i]) continue;
    for (int p = i; p > ks; --p) swap_adjacent(T, Z, p - 1);
    ++ks;
  }
  return ks;
}

static inline double conj_(double v) { return v; }
static inline cd conj_(cd v) { return std::conj(v); }
static inline double norm_(double v) { return v * v; }
static inline double norm_(cd v) { return std::norm(v); }
static inline double phase_re(double g, double ag) { return g / ag; }
static inline cd phase_re(cd g, double ag) { return g / ag; }

// One-sided Jacobi (Hestenes) on the columns of a square matrix in scalar type
// S (double for real data: a quarter of the complex work).  A = P diag(sig) W^H
// with the singular values in decreasing order.
template <class S>
static void jacobi_core(int n, std::vector<S>& A, std::vector<S>& W, std::vector<double>& sig) {
  W.assign((size_t)n * n, S(0.0));
  for (int i = 0; i < n; ++i) W[(size_t)i * n + i] = S(1.0);
  const double eps = std::numeric_limits<double>::epsilon();
  for (int sweep = 0; sweep < 80; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n - 1; ++p) {
      S* ap = &A[(size_t)p * n];
      S* wp = &W[(size_t)p * n];
      for (int q = p + 1; q < n; ++q) {
        S* aq = &A[(size_t)q * n];
        S* wq = &W[(size_t)q * n];
        double al = 0.0, be = 0.0;
        S ga = S(0.0);
        for (int i = 0; i < n; ++i) {
          al += norm_(ap[i]);
          be += norm_(aq[i]);
          ga += conj_(ap[i]) * aq[i];
        }
        const double ag = std::abs(ga);
        if (ag == 0.0 || ag <= eps * std::sqrt(al * be)) continue;
        off = std::max(off, ag / std::sqrt(al * be));
        const S e = phase_re(ga, ag);
        const double zeta = (be - al) / (2.0 * ag);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        const S se = sn * e, sec = sn * conj_(e);
        // [a_p, a_q] <- [a_p, a_q] [[c, s e], [-s conj(e), c]]
        for (int i = 0; i < n; ++i) {
          const S x = ap[i], y = aq[i];
          ap[i] = c * x - sec * y;
          aq[i] = se * x + c * y;
          const S u = wp[i], v = wq[i];
          wp[i] = c * u - sec * v;
          wq[i] = se * u + c * v;
        }
      }
    }
    if (off <= eps * n) break;
  }
  sig.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s2 = 0.0;
    for (int i = 0; i < n; ++i) s2 += norm_(A[(size_t)j * n + i]);
    sig[j] = std::sqrt(s2);
  }
}

// The rotations act on the columns of X = A^H: for the triangular factor of a
// QR decomposition the one-sided method converges in far fewer sweeps on the
// transpose.  X V = U diag(sig) gives A = V diag(sig) U^H, so P = V, W = U.
void svd_jacobi(const Mat& A0, Mat& P, std::vector<double>& sig, Mat& W, bool real) {
  const int n = A0.n;
  std::vector<double> s0;
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  P = Mat(n, n);
  W = Mat(n, n);
  if (real) {
    std::vector<double> X((size_t)n * n), V;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) X[(size_t)j * n + i] = A0(j, i).real();
    jacobi_core(n, X, V, s0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return s0[a] > s0[b]; });
    for (int jj = 0; jj < n; ++jj) {
      const int j = ord[jj];
      const double inv = s0[j] > 0.0 ? 1.0 / s0[j] : 0.0;
      for (int i = 0; i < n; ++i) {
        W(i, jj) = X[(size_t)j * n + i] * inv;
        P(i, jj) = V[(size_t)j * n + i];
      }
    }
  } else {
    std::vector<cd> X((size_t)n * n), V;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) X[(size_t)j * n + i] = std::conj(A0(j, i));
    jacobi_core(n, X, V, s0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return s0[a] > s0[b]; });
    for (int jj = 0; jj < n; ++jj) {
      const int j = ord[jj];
      const double inv = s0[j] > 0.0 ? 1.0 / s0[j] : 0.0;
      for (int i = 0; i < n; ++i) {
        W(i, jj) = X[(size_t)j * n + i] * inv;
        P(i, jj) = V[(size_t)j * n + i];
      }
    }
  }
  sig.resize(n);
  for (int jj = 0; jj < n; ++jj) sig[jj] = s0[ord[jj]];
}

// Real orthonormal basis of the span of the complex columns Zk, assumed closed
// under conjugation: pivoted Gram-Schmidt (twice) on [Re Zk, Im Zk].
static Mat real_basis(const Mat& Zk, int keff) {
  const int n = Zk.n, m = Zk.m;
  std::vector<std::vector<double>> cols;
  for (int j = 0; j < m; ++j) {
    std::vector<double> re(n), im(n);
    for (int i = 0; i < n; ++i) {
      re[i] = Zk(i, j).real();
      im[i] = Zk(i, j).imag();
    }
    cols.push_back(re);
    cols.push_back(im);
  }
  Mat out(n, keff);
  std::vector<char> used(cols.size(), 0);
  for (int k = 0; k < keff; ++k) {
    int best = -1;
    double bn = -1.0;
    for (size_t c = 0; c < cols.size(); ++c) {
      if (used[c]) continue;
      double s = 0.0;
      for (double v : cols[c]) s += v * v;
      if (s > bn) {
        bn = s;
        best = (int)c;
      }
    }
    if (best < 0 || bn <= 0.0) break;
    used[best] = 1;
    std::vector<double> q = cols[best];
    for (int pass = 0; pass < 2; ++pass) {
      for (int p = 0; p < k; ++p) {
        double d = 0.0;
        for (int i = 0; i < n; ++i) d += out(i, p).real() * q[i];
        for (int i = 0; i < n; ++i) q[i] -= d * out(i, p).real();
      }
    }
    double qn = 0.0;
    for (double v : q) qn += v * v;
    qn = std::sqrt(qn);
    for (int i = 0; i < n; ++i) out(i, k) = q[i] / qn;
    for (size_t c = 0; c < cols.size(); ++c) {
      if (used[c]) continue;
      double d = 0.0;
      for (int i = 0; i < n; ++i) d += out(i, k).real() * cols[c][i];
      for (int i = 0; i < n; ++i) cols[c][i] -= d * out(i, k).real();
    }
  }
  return out;
}

// Ri = R^{-1} (R upper triangular, n x n, column major, nonsingular) by
// back substitution, X = Ri C, and the bound ||R||_F ||R^{-1}||_F returned.
// Both run four columns a pass down contiguous columns (one load of a column
// of R or R^{-1} serves four updates).
template <class S>
static double tri_inverse_product(int n, const S* R, S* Ri, const S* C, std::vector<S>& X) {
  // Ri zero on entry; column jc = j0 + c is R^{-1} e_jc, its rows above jc
  // found from the bottom: at step p row p is final, rows 0 .. p-1 take its
  // contribution and row p-1 is then divided by its diagonal entry
  ColumnPool::instance().parallel_for((n + 3) / 4, [&](int g) {
    const int j0 = 4 * g;
    const int jb = std::min(4, n - j0);
    S* col[4];
    for (int c = 0; c < 4; ++c) col[c] = Ri + (size_t)(j0 + std::min(c, jb - 1)) * n;
    for (int c = 0; c < jb; ++c) col[c][j0 + c] = S(1.0) / R[(size_t)(j0 + c) * n + j0 + c];
    for (int p = j0 + jb - 1; p >= 1; --p) {
      const S* __restrict__ rp = R + (size_t)p * n;
      S xp[4];
      for (int c = 0; c < 4; ++c) xp[c] = c < jb && p <= j0 + c ? col[c][p] : S(0.0);
      S* __restrict__ c0 = col[0];
      S* __restrict__ c1 = col[1];
      S* __restrict__ c2 = col[2];
      S* __restrict__ c3 = col[3];
      if (jb == 4) {
        for (int i = 0; i < p; ++i) {
          const S r = rp[i];
          c0[i] -= r * xp[0];
          c1[i] -= r * xp[1];
          c2[i] -= r * xp[2];
          c3[i] -= r * xp[3];
        }
      } else {
        for (int c = 0; c < jb; ++c)
          for (int i = 0; i < p; ++i) col[c][i] -= rp[i] * xp[c];
      }
      const S d = R[(size_t)(p - 1) * n + (p - 1)];
      for (int c = 0; c < jb; ++c)
        if (p <= j0 + c) col[c][p - 1] /= d;
    }
  });
  double f = 0.0, fi = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j; ++i) {
      f += norm_(R[(size_t)j * n + i]);
      fi += norm_(Ri[(size_t)j * n + i]);
    }
  X.assign((size_t)n * n, S(0.0));
  const int nq = n / 4;  // groups of four columns, then the rest one by one
  ColumnPool::instance().parallel_for(nq + (n - 4 * nq), [&](int g) {
    if (g >= nq) {
      const int j = 4 * nq + (g - nq);
      S* xj = X.data() + (size_t)j * n;
      for (int p = 0; p < n; ++p) {
        const S cpj = C[(size_t)j * n + p];
        const S* rip = Ri + (size_t)p * n;
        for (int i = 0; i <= p; ++i) xj[i] += rip[i] * cpj;
      }
      return;
    }
    const int j = 4 * g;
    S* __restrict__ x0 = X.data() + (size_t)j * n;
    S* __restrict__ x1 = x0 + n;
    S* __restrict__ x2 = x1 + n;
    S* __restrict__ x3 = x2 + n;
    for (int p = 0; p < n; ++p) {
      const S a0 = C[(size_t)j * n + p], a1 = C[(size_t)(j + 1) * n + p];
      const S a2 = C[(size_t)(j + 2) * n + p], a3 = C[(size_t)(j + 3) * n + p];
      const S* __restrict__ rip = Ri + (size_t)p * n;  // column p of R^{-1}: rows 0 .. p
      for (int i = 0; i <= p; ++i) {
        const S r = rip[i];
        x0[i] += r * a0;
        x1[i] += r * a1;
        x2[i] += r * a2;
        x3[i] += r * a3;
      }
    }
  });
  return std::sqrt(f * fi);
}

int harmonic_ritz(int l0, const cd* R, const cd* C, int s, int k, bool real, std::vector<cd>& G,
                  int* ell_out, const cd* RiC_in, double ri_fro2) {
  G.clear();
  *ell_out = 0;
  if (l0 <= 0 || k <= 0) return 0;
  const double thr = std::max(s, l0) * std::ldexp(1.0, -52);
  Mat Rm(l0, l0), Cm(l0, l0);
  for (int j = 0; j < l0; ++j)
    for (int i = 0; i < l0; ++i) {
      Rm(i, j) = i <= j ? R[(size_t)j * l0 + i] : cd(0.0);
      Cm(i, j) = C[(size_t)j * l0 + i];
    }
  // triangular inverse of R, the Frobenius condition bound, and R^{-1} C (real
  // arithmetic for real data)
  bool singular = false;
  for (int i = 0; i < l0; ++i)
    if (std::abs(Rm(i, i)) == 0.0) singular = true;
  double cond = std::numeric_limits<double>::infinity();
  Mat RiC;  // R^{-1} C when R is nonsingular
  if (!singular && RiC_in != nullptr && ri_fro2 >= 0.0) {
    double f = 0.0;
    for (int j = 0; j < l0; ++j)
      for (int i = 0; i <= j; ++i) f += std::norm(Rm(i, j));
    cond = std::sqrt(f * ri_fro2);
    RiC = Mat(l0, l0);
    for (size_t i = 0; i < RiC.a.size(); ++i) RiC.a[i] = RiC_in[i];
  } else if (!singular) {
    if (real) {
      std::vector<double> r((size_t)l0 * l0), ri((size_t)l0 * l0, 0.0), c((size_t)l0 * l0), x;
      for (size_t i = 0; i < r.size(); ++i) {
        r[i] = Rm.a[i].real();
        c[i] = Cm.a[i].real();
      }
      cond = tri_inverse_product(l0, r.data(), ri.data(), c.data(), x);
      RiC = Mat(l0, l0);
      for (size_t i = 0; i < x.size(); ++i) RiC.a[i] = x[i];
    } else {
      std::vector<cd> ri((size_t)l0 * l0, cd(0.0)), x;
      cond = tri_inverse_product(l0, Rm.a.data(), ri.data(), Cm.a.data(), x);
      RiC = Mat(l0, l0);
      RiC.a = x;
    }
  }
  const bool svd_path = !(std::isfinite(cond) && cond * thr < 0.5);
  Mat Aeig;
  Mat Wl;  // right singular vectors kept (svd path)
  int ell = l0;
  if (!svd_path) {
    Aeig = RiC;
  } else {
    Mat P, W;
    std::vector<double> sig;
    svd_jacobi(Rm, P, sig, W, real);
    ell = 0;
    if (sig[0] > 0.0)
      for (int i = 0; i < l0; ++i)
        if (sig[i] > sig[0] * thr) ++ell;
    if (ell == 0) return 0;
    Mat PC(ell, l0);  // P_ell^H C
    for (int j = 0; j < l0; ++j)
      for (int i = 0; i < ell; ++i) {
        cd acc = 0.0;
        for (int p = 0; p < l0; ++p) acc += std::conj(P(p, i)) * Cm(p, j);
        PC(i, j) = acc;
      }
    Aeig = Mat(ell, ell);
    for (int j = 0; j < ell; ++j)
      for (int i = 0; i < ell; ++i) {
        cd acc = 0.0;
        for (int p = 0; p < l0; ++p) acc += PC(i, p) * W(p, j);
        Aeig(i, j) = acc / sig[i];
      }
    Wl = Mat(l0, ell);
    for (int j = 0; j < ell; ++j)
      for (int i = 0; i < l0; ++i) Wl(i, j) = W(i, j);
  }
  *ell_out = ell;
  const int n = ell;
  // moduli of the eigenvalues; in the real Schur form a 2 x 2 block holds a
  // conjugate pair whose common modulus is the square root of its determinant
  std::vector<double> mod(n);
  std::vector<int> partner(n, -1);
  std::vector<double> Tr, Zr;
  Mat T, Z;
  SplitMat H;  // complex data: Hessenberg form iterated to triangular (window updates only)
  std::vector<double> hVr, hVi, hF;
  std::vector<Rot> hlog;
  if (real) {
    Tr.resize((size_t)n * n);
    for (size_t i = 0; i < Tr.size(); ++i) Tr[i] = Aeig.a[i].real();
    if (!schur_real(n, Tr, Zr)) return -1;
    auto tr = [&](int i, int j) { return Tr[(size_t)j * n + i]; };
    for (int i = 0; i < n; ++i) {
      if (i + 1 < n && tr(i + 1, i) != 0.0) {
        const double det = tr(i, i) * tr(i + 1, i + 1) - tr(i, i + 1) * tr(i + 1, i);
        mod[i] = mod[i + 1] = std::sqrt(std::fabs(det));
        partner[i] = i + 1;
        partner[i + 1] = i;
        ++i;
      } else {
        mod[i] = std::fabs(tr(i, i));
      }
    }
  } else {
    // eigenvalues by the windowed QR; the Schur vectors only if needed below
    H = SplitMat(n);
    for (size_t i = 0; i < Aeig.a.size(); ++i) {
      H.re[i] = Aeig.a[i].real();
      H.im[i] = Aeig.a[i].imag();
    }
    hessenberg_reflectors(H, hVr, hVi, hF);
    if (!hessenberg_qr_window(H, hlog)) return -1;
    for (int i = 0; i < n; ++i) mod[i] = std::hypot(H.r(i, i), H.c(i, i));
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return mod[a] > mod[b]; });
  const int kk = std::min(k, n);
  std::vector<char> sel(n, 0);
  for (int i = 0; i < kk; ++i) sel[ord[i]] = 1;
  // never split a complex-conjugate pair (the two members of a 2 x 2 block)
  for (int i = 0; i < n; ++i)
    if (sel[i] && partner[i] >= 0) sel[partner[i]] = 1;
  int keff = 0;
  while (keff < n && sel[keff]) ++keff;
  bool leading = true;  // the selection already leads the Schur form
  for (int i = keff; i < n; ++i)
    if (sel[i]) leading = false;
  Mat Y;
  if (!real && leading) {
    // the leading Schur vectors span the selected invariant subspace
    leading_schur_vectors(n, keff, hVr, hVi, hF, hlog, Y);
  } else if (real && leading) {
    // the leading real Schur vectors are an orthonormal real basis of the
    // selected invariant subspace: no reordering, no complex form needed
    Y = Mat(n, keff);
    for (int j = 0; j < keff; ++j)
      for (int i = 0; i < n; ++i) Y(i, j) = Zr[(size_t)j * n + i];
  } else {
    if (real) {
      std::vector<int> pc;
      real_to_complex_schur(n, Tr, Zr, T, Z, pc);
    } else {
      // the full Schur form (T, Z) for the reordering: the same iteration,
      // so the same eigenvalue positions
      T = Aeig;
      if (!schur(T, Z)) return -1;
    }
    keff = reorder(T, Z, sel);
    Mat Zk(n, keff);
    for (int j = 0; j < keff; ++j)
      for (int i = 0; i < n; ++i) Zk(i, j) = Z(i, j);
    Y = real ? real_basis(Zk, keff) : Zk;
  }
  G.assign((size_t)l0 * keff, cd(0.0));
  if (!svd_path) {
    for (int j = 0; j < keff; ++j)
      for (int i = 0; i < l0; ++i) G[(size_t)j * l0 + i] = Y(i, j);
  } else {
    for (int j = 0; j < keff; ++j)
      for (int i = 0; i < l0; ++i) {
        cd acc = 0.0;
        for (int p = 0; p < n; ++p) acc += Wl(i, p) * Y(p, j);
        G[(size_t)j * l0 + i] = real ? cd(acc.real(), 0.0) : acc;
      }
  }
  return keff;
}

}  // namespace dense
}  // namespace sdr
