// Host FP64 dense helpers for the projected (L x L) problems.
#pragma once

namespace slrf {

// Eigen-decomposition of a symmetric n x n row-major matrix A (destroyed):
// w ascending, V row-major with column j the eigenvector of w[j].
bool sym_eig(int n, double* A, double* w, double* V);

// Ritz values theta (ascending) and coefficients Z (L x L row-major) of the
// projected pencil (GA, GB): Z^T GB Z = I, Z^T GA Z = diag(theta).  floor_rel:
// eigenvalues of the unit-diagonal GB below floor_rel times its largest are
// raised to that floor (1e-15 for FP64 Gram matrices; about the Gram's own
// rounding level when it was accumulated in a lower precision).
bool projected_pencil(int L, const double* GA, const double* GB, double* theta, double* Z,
                      double floor_rel = 1e-15);

// SLRF design at gamma = 1 (see slrf.h): xi[N] sorted, omega[2N] (re, im).
bool design_poles_unit(int N, double alpha, double beta, double* xi, double* omega);

// Quadrature-rule filter of Section 3.2 (rule 0 midpoint, 1 Gauss-Legendre,
// 2 Gauss-Chebyshev): sigma[2N], weight[2N] (re, im), sorted by Re(sigma).
bool quadrature_poles(int rule, int N, double gamma, double* sigma, double* weight);

}  // namespace slrf
