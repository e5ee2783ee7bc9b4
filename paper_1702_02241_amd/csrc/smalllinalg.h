// Small dense FP64 linear algebra on the host (matrices of order <= 64):
// cyclic Jacobi eigensolver for symmetric matrices, Cholesky, triangular
// solves.  Row-major storage, leading dimension = order.
#pragma once

#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

namespace rpca {
namespace la {

// Eigen-decomposition A = W diag(w) W^T of a symmetric n x n matrix by cyclic
// Jacobi rotations.  Eigenvalues are returned in descending order with the
// matching eigenvectors as the columns of W.
inline void sym_eig(const double* A_in, int n, double* w, double* W) {
  std::vector<double> A(A_in, A_in + (size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) W[i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += A[i * n + i] * A[i * n + i];
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    }
    if (off <= 1e-30 * diag || off == 0.0) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double app = A[p * n + p], aqq = A[q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = cs * akp - sn * akq;
          A[k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = cs * apk - sn * aqk;
          A[q * n + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double wkp = W[k * n + p], wkq = W[k * n + q];
          W[k * n + p] = cs * wkp - sn * wkq;
          W[k * n + q] = sn * wkp + cs * wkq;
        }
      }
    }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A[a * n + a] > A[b * n + b]; });
  std::vector<double> Wc(W, W + (size_t)n * n);
  for (int j = 0; j < n; ++j) {
    w[j] = A[idx[j] * n + idx[j]];
    for (int i = 0; i < n; ++i) W[i * n + j] = Wc[i * n + idx[j]];
  }
}

// C = A (ra x ca) * B (ca x cb)
inline void matmul(const double* A, const double* B, double* C, int ra, int ca, int cb) {
  for (int i = 0; i < ra; ++i)
    for (int j = 0; j < cb; ++j) {
      double s = 0.0;
      for (int t = 0; t < ca; ++t) s += A[i * ca + t] * B[t * cb + j];
      C[i * cb + j] = s;
    }
}

// C = A^T (A is r x ca) * B (r x cb)
inline void matmul_tn(const double* A, const double* B, double* C, int r, int ca, int cb) {
  for (int i = 0; i < ca; ++i)
    for (int j = 0; j < cb; ++j) {
      double s = 0.0;
      for (int t = 0; t < r; ++t) s += A[t * ca + i] * B[t * cb + j];
      C[i * cb + j] = s;
    }
}

// Lower Cholesky factor of an SPD matrix (returns false if not positive definite).
inline bool cholesky(const double* A, int n, double* Lo) {
  memset(Lo, 0, sizeof(double) * n * n);
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int t = 0; t < j; ++t) s -= Lo[j * n + t] * Lo[j * n + t];
    if (!(s > 0.0)) return false;
    const double d = sqrt(s);
    Lo[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int t = 0; t < j; ++t) v -= Lo[i * n + t] * Lo[j * n + t];
      Lo[i * n + j] = v / d;
    }
  }
  return true;
}

// Inverse of the upper-triangular R = Lo^T, returned as a full n x n matrix T with R T = I.
inline void inv_upper_from_lower(const double* Lo, int n, double* T) {
  memset(T, 0, sizeof(double) * n * n);
  for (int col = 0; col < n; ++col) {
    // solve R t = e_col by back substitution, R[i][j] = Lo[j][i]
    for (int i = n - 1; i >= 0; --i) {
      double s = (i == col) ? 1.0 : 0.0;
      for (int j = i + 1; j < n; ++j) s -= Lo[j * n + i] * T[j * n + col];
      T[i * n + col] = s / Lo[i * n + i];
    }
  }
}

}  // namespace la
}  // namespace rpca
