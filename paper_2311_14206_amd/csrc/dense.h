// Host small-dense linear algebra for the sketched harmonic-Ritz step.
#pragma once

#include <complex>
#include <vector>

namespace sdr {
namespace dense {

using cd = std::complex<double>;

// Column-major n x n matrix helper.
struct Mat {
  int n = 0, m = 0;  // rows, cols
  std::vector<cd> a;
  Mat() = default;
  Mat(int rows, int cols) : n(rows), m(cols), a((size_t)rows * cols, cd(0.0, 0.0)) {}
  cd& operator()(int i, int j) { return a[(size_t)j * n + i]; }
  const cd& operator()(int i, int j) const { return a[(size_t)j * n + i]; }
};

// Complex Schur form A = Z T Z^H (T upper triangular); returns false if the
// QR iteration did not converge.
bool schur(Mat& T, Mat& Z);

// Move the eigenvalues flagged in sel to the leading positions of the Schur
// form (T, Z), keeping their relative order.  Returns the number moved.
int reorder(Mat& T, Mat& Z, std::vector<char> sel);

// One-sided Jacobi SVD of a square matrix: A = P diag(sig) W^H, singular
// values in decreasing order; real arithmetic when real is set.
void svd_jacobi(const Mat& A, Mat& P, std::vector<double>& sig, Mat& W, bool real);

// Sketched harmonic-Ritz step (Section 3.5): see sdr_host_harmonic_ritz.
// R: l0 x l0 upper triangular factor of SAW; C = Q^H [SU, SV].  Writes G
// (l0 x k_eff) and returns k_eff, or -1 on failure.  RiC, when given, is
// R^{-1} C formed elsewhere (l0 x l0, column major) and ri_fro2 the squared
// Frobenius norm of R^{-1}: the triangular inverse is then not formed here.
int harmonic_ritz(int l0, const cd* R, const cd* C, int s, int k, bool real, std::vector<cd>& G,
                  int* ell, const cd* RiC = nullptr, double ri_fro2 = -1.0);

}  // namespace dense
}  // namespace sdr
