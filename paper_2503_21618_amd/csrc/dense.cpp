// Host FP64 dense linear algebra for the L x L projected problems of the
// Rayleigh-Ritz step (Algorithm 1, "Solve the eigenvalue problem").
//
// sym_eig: Householder reduction to tridiagonal form followed by the implicit
// symmetric QR iteration with Wilkinson shifts (Golub and Van Loan, Matrix
// Computations, Sections 8.3.1-8.3.3), eigenvectors accumulated.
//
// projected_pencil: Ritz pairs of (GA, GB) = (U^T A U, U^T B U) without a
// Cholesky factor of GB: GB is scaled to unit diagonal, diagonalised, its
// eigenvalues floored at a tiny fraction of the largest (so a numerically
// rank-deficient filtered block keeps L columns), then the reduced standard
// problem is diagonalised (Stathopoulos and Wu's SVQB orthogonalisation
// folded into the projection).
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace slrf {

// QT holds the transpose of the accumulated orthogonal factor, so that the
// reflections and rotations update contiguous rows.
static void tridiagonalize(int n, double* A, double* QT, double* d, double* e) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) QT[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
  std::vector<double> v(n), p(n), w(n), sr(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double xn = 0;
    for (int i = 0; i < m; ++i) xn += A[(size_t)(k + 1 + i) * n + k] * A[(size_t)(k + 1 + i) * n + k];
    xn = std::sqrt(xn);
    if (xn == 0) continue;
    const double x0 = A[(size_t)(k + 1) * n + k];
    const double alpha = x0 > 0 ? -xn : xn;
    double vn2 = 0;
    for (int i = 0; i < m; ++i) {
      v[i] = A[(size_t)(k + 1 + i) * n + k];
      if (i == 0) v[i] -= alpha;
      vn2 += v[i] * v[i];
    }
    if (vn2 == 0) continue;
    const double beta = 2.0 / vn2;
    // p = beta * A22 v
    for (int i = 0; i < m; ++i) {
      double s = 0;
      const double* row = A + (size_t)(k + 1 + i) * n + (k + 1);
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = beta * s;
    }
    double pv = 0;
    for (int i = 0; i < m; ++i) pv += p[i] * v[i];
    const double K = 0.5 * beta * pv;
    for (int i = 0; i < m; ++i) w[i] = p[i] - K * v[i];
    for (int i = 0; i < m; ++i) {
      double* row = A + (size_t)(k + 1 + i) * n + (k + 1);
      for (int j = 0; j < m; ++j) row[j] -= v[i] * w[j] + w[i] * v[j];
    }
    A[(size_t)(k + 1) * n + k] = A[(size_t)k * n + (k + 1)] = alpha;
    for (int i = 1; i < m; ++i) A[(size_t)(k + 1 + i) * n + k] = A[(size_t)k * n + (k + 1 + i)] = 0;
    // Q <- Q H: with s_r = beta sum_i Q[r][k+1+i] v_i, Q[r][k+1+i] -= s_r v_i
    std::fill(sr.begin(), sr.end(), 0.0);
    for (int i = 0; i < m; ++i) {
      const double* q = QT + (size_t)(k + 1 + i) * n;
      const double vi = v[i];
      for (int r = 0; r < n; ++r) sr[r] += q[r] * vi;
    }
    for (int r = 0; r < n; ++r) sr[r] *= beta;
    for (int i = 0; i < m; ++i) {
      double* q = QT + (size_t)(k + 1 + i) * n;
      const double vi = v[i];
      for (int r = 0; r < n; ++r) q[r] -= sr[r] * vi;
    }
  }
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];
}

// Implicit symmetric QR on (d, e), rotations applied to the columns of Q (rows
// of QT).
static bool tridiag_qr(int n, double* d, double* e, double* QT) {
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  long guard = 0;
  const long max_guard = 60L * n + 100;
  while (hi > 0) {
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0;
      --hi;
      continue;
    }
    if (++guard > max_guard) return false;
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    if (lo > 0) e[lo - 1] = 0;
    // Wilkinson shift from the trailing 2x2 block
    const double delta = 0.5 * (d[hi - 1] - d[hi]);
    const double eh = e[hi - 1];
    const double den = delta + (delta >= 0 ? 1.0 : -1.0) * std::hypot(delta, eh);
    const double mu = d[hi] - (den != 0 ? eh * eh / den : 0.0);
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, z);
      double c = 1, s = 0;
      if (r != 0) {
        c = x / r;
        s = -z / r;
      }
      if (k > lo) e[k - 1] = r;
      const double dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = c * c * dk - 2 * c * s * ek + s * s * dk1;
      d[k + 1] = s * s * dk + 2 * c * s * ek + c * c * dk1;
      e[k] = c * s * dk + (c * c - s * s) * ek - c * s * dk1;
      if (k + 1 < hi) {
        z = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      x = e[k];
      double* qa = QT + (size_t)k * n;
      double* qb = QT + (size_t)(k + 1) * n;
      for (int i = 0; i < n; ++i) {
        const double a = qa[i], b = qb[i];
        qa[i] = c * a - s * b;
        qb[i] = s * a + c * b;
      }
    }
  }
  return true;
}

bool sym_eig(int n, double* A, double* w, double* V) {
  if (n == 1) {
    w[0] = A[0];
    V[0] = 1;
    return true;
  }
  std::vector<double> QT((size_t)n * n), d(n), e(n);
  tridiagonalize(n, A, QT.data(), d.data(), e.data());
  if (!tridiag_qr(n, d.data(), e.data(), QT.data())) return false;
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
  for (int j = 0; j < n; ++j) {
    w[j] = d[idx[j]];
    for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = QT[(size_t)idx[j] * n + i];
  }
  return true;
}

bool projected_pencil(int L, const double* GA, const double* GB, double* theta, double* Z, double floor_rel) {
  for (int i = 0; i < L * L; ++i)
    if (!std::isfinite(GA[i]) || !std::isfinite(GB[i])) return false;
  std::vector<double> s(L), B((size_t)L * L), lam(L), V((size_t)L * L), T((size_t)L * L),
      C((size_t)L * L), tmp((size_t)L * L), th(L), S((size_t)L * L);
  for (int i = 0; i < L; ++i) {
    const double g = GB[(size_t)i * L + i];
    s[i] = g > 0 ? 1.0 / std::sqrt(g) : 1.0;
  }
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < L; ++j)
      B[(size_t)i * L + j] = 0.5 * (GB[(size_t)i * L + j] + GB[(size_t)j * L + i]) * s[i] * s[j];
  if (!sym_eig(L, B.data(), lam.data(), V.data())) return false;
  const double lmax = lam[L - 1];
  if (!(lmax > 0)) return false;
  const double floor_ = floor_rel * lmax;
  // T = diag(s) V diag(max(lam, floor)^-1/2)
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < L; ++j)
      T[(size_t)i * L + j] = s[i] * V[(size_t)i * L + j] / std::sqrt(std::max(lam[j], floor_));
  // C = T^T GA T, with GA symmetrised; the products run row by row over
  // contiguous rows (i, k, j order)
  std::vector<double> As((size_t)L * L);
  for (int i = 0; i < L; ++i)
    for (int k = 0; k < L; ++k) As[(size_t)i * L + k] = 0.5 * (GA[(size_t)i * L + k] + GA[(size_t)k * L + i]);
  std::fill(tmp.begin(), tmp.end(), 0.0);
  for (int i = 0; i < L; ++i) {
    double* out = tmp.data() + (size_t)i * L;
    for (int k = 0; k < L; ++k) {
      const double a = As[(size_t)i * L + k];
      const double* t = T.data() + (size_t)k * L;
      for (int j = 0; j < L; ++j) out[j] += a * t[j];
    }
  }
  std::fill(C.begin(), C.end(), 0.0);
  for (int k = 0; k < L; ++k) {
    const double* t = T.data() + (size_t)k * L;
    const double* m = tmp.data() + (size_t)k * L;
    for (int i = 0; i < L; ++i) {
      const double a = t[i];
      double* out = C.data() + (size_t)i * L;
      for (int j = 0; j < L; ++j) out[j] += a * m[j];
    }
  }
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < i; ++j) {
      const double a = 0.5 * (C[(size_t)i * L + j] + C[(size_t)j * L + i]);
      C[(size_t)i * L + j] = C[(size_t)j * L + i] = a;
    }
  if (!sym_eig(L, C.data(), th.data(), S.data())) return false;
  for (int j = 0; j < L; ++j) theta[j] = th[j];
  // Z = T S
  for (int i = 0; i < L; ++i) {
    double* out = Z + (size_t)i * L;
    std::fill(out, out + L, 0.0);
    for (int k = 0; k < L; ++k) {
      const double a = T[(size_t)i * L + k];
      const double* sr = S.data() + (size_t)k * L;
      for (int j = 0; j < L; ++j) out[j] += a * sr[j];
    }
  }
  return true;
}

}  // namespace slrf
