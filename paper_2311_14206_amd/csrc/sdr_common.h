// Scalar traits and small helpers shared by the GMRES-SDR kernels and host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define SDR_HD __host__ __device__ __forceinline__

namespace sdr {

// Interleaved complex number (matches the C-ABI's (re, im) layout).
template <class R>
struct cx {
  R x, y;
};

template <class R> SDR_HD cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <class R> SDR_HD cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <class R> SDR_HD cx<R> operator-(cx<R> a) { return {-a.x, -a.y}; }
// Each component is one product and one fused multiply-add in a fixed
// order, so a complex product rounds the same in every kernel whatever the
// compiler contracts around it.
template <class R> SDR_HD cx<R> operator*(cx<R> a, cx<R> b) {
  return {fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x)};
}
template <class R> SDR_HD cx<R> operator*(cx<R> a, R s) { return {a.x * s, a.y * s}; }
template <class R> SDR_HD cx<R>& operator+=(cx<R>& a, cx<R> b) { a.x += b.x; a.y += b.y; return a; }
template <class R> SDR_HD cx<R>& operator-=(cx<R>& a, cx<R> b) { a.x -= b.x; a.y -= b.y; return a; }

SDR_HD double conj(double a) { return a; }
SDR_HD float conj(float a) { return a; }
template <class R> SDR_HD cx<R> conj(cx<R> a) { return {a.x, -a.y}; }
SDR_HD double abs2(double a) { return a * a; }
SDR_HD double abs2(float a) { return (double)a * (double)a; }
template <class R> SDR_HD double abs2(cx<R> a) { return fma((double)a.x, (double)a.x, (double)a.y * a.y); }
SDR_HD double re(double a) { return a; }
template <class R> SDR_HD R re(cx<R> a) { return a.x; }

template <class T> struct traits;
template <> struct traits<double> {
  using acc = double;  // accumulation / small-dense type
  static constexpr bool cpx = false;
};
template <> struct traits<float> {
  using acc = double;
  static constexpr bool cpx = false;
};
template <> struct traits<cx<double>> {
  using acc = cx<double>;
  static constexpr bool cpx = true;
};
template <> struct traits<cx<float>> {
  using acc = cx<double>;
  static constexpr bool cpx = true;
};

// widen to the accumulation type / round back to the storage type
SDR_HD double widen(double a) { return a; }
SDR_HD double widen(float a) { return (double)a; }
SDR_HD cx<double> widen(cx<double> a) { return a; }
SDR_HD cx<double> widen(cx<float> a) { return {(double)a.x, (double)a.y}; }

template <class T> SDR_HD T narrow(typename traits<T>::acc a);
template <> SDR_HD double narrow<double>(double a) { return a; }
template <> SDR_HD float narrow<float>(double a) { return (float)a; }
template <> SDR_HD cx<double> narrow<cx<double>>(cx<double> a) { return a; }
template <> SDR_HD cx<float> narrow<cx<float>>(cx<double> a) { return {(float)a.x, (float)a.y}; }

template <class A> SDR_HD A zero();
template <> SDR_HD double zero<double>() { return 0.0; }
template <> SDR_HD cx<double> zero<cx<double>>() { return {0.0, 0.0}; }

SDR_HD double scale(double a, double s) { return a * s; }
SDR_HD cx<double> scale(cx<double> a, double s) { return {a.x * s, a.y * s}; }

// ---------------------------------------------------------------------------
// Sparse-sign sketch generator (Section 3, eq. (3.1)): column n, block b of
// zeta.  Word g = b / 4 of column n is the SplitMix64 output mixer (Steele,
// Lea, Flood 2014) applied to key = seed + GAMMA * (n * G + g + 1); block
// b = 4g + q takes the 16-bit field u = (h >> 16q) & 0xFFFF:
//   row  = b * bsz + (((u >> 1) * bsz) >> 15),   sign = u & 1 ? -1 : +1,
// value sign / sqrt(zeta).  bsz = s / zeta, G = ceil(zeta / 4).
// ---------------------------------------------------------------------------
static constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

SDR_HD uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct SketchSpec {
  uint64_t seed;
  int s;      // rows
  int zeta;   // nonzeros per column
  int bsz;    // s / zeta
  int words;  // ceil(zeta / 4)
  int ext;    // 1: rows 0 .. s-1 are formed by another kernel (the subsampled
              // DCT); a step kernel keeps the partial layout and fills the rest
  const void* src = nullptr;  // a step kernel's sketch and norm input when it is
                              // not the SpMV input (right preconditioning)
};

}  // namespace sdr
