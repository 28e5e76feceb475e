// Eigen-decomposition of a small complex Hermitian matrix by cyclic Jacobi
// rotations (host code; the calibration step of the channel compression).
// Each off-diagonal element a_pq = |a_pq| e^{i phi} is removed by the unitary
// U = diag(1, e^{-i phi}) R(theta), which turns the 2 x 2 block real and then
// rotates it diagonal (the classical Jacobi method, e.g. Golub and Van Loan,
// Matrix Computations, Sec. 8.5, applied after the phase change).
#pragma once

#include <cmath>
#include <complex>
#include <vector>

namespace nlv {

// A: n x n Hermitian, row-major (overwritten).  On return w[k] are the
// eigenvalues and column k of V (row-major n x n) the eigenvector of w[k].
inline void hermitian_eig(int n, std::vector<std::complex<double>>& A, std::vector<double>& w,
                          std::vector<std::complex<double>>& V) {
  using cd = std::complex<double>;
  V.assign((size_t)n * n, cd(0.0, 0.0));
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> cd& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += std::norm(a(i, i));
      for (int j = i + 1; j < n; ++j) off += std::norm(a(i, j));
    }
    if (off <= 1e-30 * (diag + 1e-300)) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double mag = std::abs(a(p, q));
        if (mag == 0.0) continue;
        const cd ph = a(p, q) / mag;                   // e^{i phi}
        const double app = a(p, p).real(), aqq = a(q, q).real();
        // real symmetric block [[app, mag], [mag, aqq]]: rotation angle
        const double tau = (aqq - app) / (2.0 * mag);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        // U = diag(1, e^{-i phi}) [[c, s], [-s, c]] on rows / columns (p, q)
        const cd eph = std::conj(ph);
        const cd up_p = c, up_q = -s * eph;            // column p of U (rows p, q)
        const cd uq_p = s, uq_q = c * eph;             // column q of U (rows p, q)
        for (int k = 0; k < n; ++k) {                  // A <- A U
          const cd akp = a(k, p), akq = a(k, q);
          a(k, p) = akp * up_p + akq * up_q;
          a(k, q) = akp * uq_p + akq * uq_q;
        }
        for (int k = 0; k < n; ++k) {                  // A <- U^H A
          const cd apk = a(p, k), aqk = a(q, k);
          a(p, k) = std::conj(up_p) * apk + std::conj(up_q) * aqk;
          a(q, k) = std::conj(uq_p) * apk + std::conj(uq_q) * aqk;
        }
        a(p, q) = 0.0;
        a(q, p) = 0.0;
        for (int k = 0; k < n; ++k) {                  // V <- V U
          const cd vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = vkp * up_p + vkq * up_q;
          V[(size_t)k * n + q] = vkp * uq_p + vkq * uq_q;
        }
      }
    }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = a(i, i).real();
}

}  // namespace nlv
