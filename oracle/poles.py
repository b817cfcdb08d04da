"""SLRF pole and weight design (paper Section 3.1), separation factor (Def. 3.1),
and the quadrature-rule comparison filters (Section 3.2).  Test infrastructure.

Parity unpinned numerically: the paper prints no pole values.  Pinned by the
invariants listed in the package header.

Readings of the paper used here:
  * The filter drops the 1/(2 pi i) factor: Phi(x) = sum_j 2 Re(w_j / (x - sigma_j))
    (the rational filter equation of Section 3.1; a global scale does not change
    the filtered subspace).
  * h = 1 on [0, gamma], 0 elsewhere; delta = beta on [0, gamma], 1 on
    (gamma, kappa], 0 elsewhere, kappa = 10 gamma.
  * The delta-weighted L2 norm is evaluated by two composite trapezoid rules,
    on [0, 1] and on [1, 10] (gamma = 1), node spacing 1/2000 (``spacing``).
  * For fixed x_j the weights enter linearly, so they are the linear least-squares
    solution (variable projection, Golub and Pereyra 1973); the abscissae
    x_j = sigmoid(theta_j) in (0, 1) minimise the projected residual by
    Levenberg-Marquardt from a fixed set of start points, keeping the smallest
    objective.
  * Poles and weights for gamma follow from the gamma = 1 design by
    sigma_j = gamma xi_j (1 + alpha i), w_j = gamma omega_j.
  * Ridge term.  As stated, the problem has no minimiser with distinct poles:
    the objective keeps decreasing as the x_j merge into one multiple pole, while
    the weights grow without bound and cancel (10^6..10^8 at N = 4).  Such a
    filter cannot be applied with inexact inner solves.  The design therefore
    minimises ||Phi - h||_delta^2 + eta sum_j |w_j|^2 with eta = 1e-6 (at
    gamma = 1), which keeps the poles apart and the weights O(1).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import least_squares

KAPPA = 10.0


def filter_value(t, sigma, w):
    """Phi(t) = sum_j w_j/(t - sigma_j) + conj(w_j)/(t - conj(sigma_j)), real t."""
    t = np.asarray(t, dtype=np.float64)[..., None]
    return (2.0 * np.real(w / (t - sigma))).sum(-1)


def filter_derivative(t, sigma, w):
    """Phi'(t) = -sum_j 2 Re(w_j / (t - sigma_j)^2)."""
    t = np.asarray(t, dtype=np.float64)[..., None]
    return (-2.0 * np.real(w / (t - sigma) ** 2)).sum(-1)


def separation_factor(sigma, w, gamma):
    """|Phi'(gamma)| (Definition 3.1)."""
    return float(abs(filter_derivative(gamma, sigma, w)))


def trapezoid_rows(beta: float, spacing: float = 1.0 / 2000.0):
    """Nodes t, weights sqrt(q_t * delta_t) and targets h_t of the discretised
    delta-norm at gamma = 1 (two composite trapezoid rules)."""
    n1 = int(round(1.0 / spacing))
    n2 = int(round((KAPPA - 1.0) / spacing))
    t1 = np.linspace(0.0, 1.0, n1 + 1)
    q1 = np.full(n1 + 1, 1.0 / n1)
    q1[[0, -1]] *= 0.5
    t2 = np.linspace(1.0, KAPPA, n2 + 1)
    q2 = np.full(n2 + 1, (KAPPA - 1.0) / n2)
    q2[[0, -1]] *= 0.5
    t = np.concatenate([t1, t2])
    sw = np.sqrt(np.concatenate([beta * q1, q2]))
    h = np.concatenate([np.ones(n1 + 1), np.zeros(n2 + 1)])
    return t, sw, h


def _design_matrix(t, xi, alpha):
    """Columns: dPhi/dRe(w_j) = 2 Re(1/(t - s_j)), dPhi/dIm(w_j) = -2 Im(1/(t - s_j))."""
    s = xi * (1.0 + 1j * alpha)
    g = 1.0 / (t[:, None] - s[None, :])
    return np.concatenate([2.0 * g.real, -2.0 * g.imag], axis=1)


ETA = 1e-6


def _ridge_system(xi, alpha, rows, eta):
    t, sw, h = rows
    G = _design_matrix(t, xi, alpha) * sw[:, None]
    m = G.shape[1]
    Ga = np.vstack([G, np.sqrt(eta) * np.eye(m)])
    ha = np.concatenate([h * sw, np.zeros(m)])
    return G, Ga, ha


def _solve_ls(Ga, ha):
    Q, R = np.linalg.qr(Ga)
    return np.linalg.solve(R, Q.T @ ha)


def weights_for(xi, alpha, rows, eta: float = ETA):
    """Optimal complex weights for fixed pole abscissae (ridge least squares).

    Returns (w, data-fit term ||Phi - h||_delta^2)."""
    t, sw, h = rows
    G, Ga, ha = _ridge_system(np.asarray(xi, dtype=np.float64), alpha, rows, eta)
    coef = _solve_ls(Ga, ha)
    N = len(xi)
    w = coef[:N] + 1j * coef[N:]
    res = G @ coef - h * sw
    return w, float(res @ res)


def objective(xi, alpha, rows, eta: float = ETA):
    """J(xi) = min_w ||Phi - h||_delta^2 + eta ||w||^2 (discretised)."""
    r = projected_residual(np.asarray(xi, dtype=np.float64), alpha, rows, eta)
    return float(r @ r)


def projected_residual(xi, alpha, rows, eta: float = ETA):
    """Stacked residual [sqrt(q delta)(Phi - h); sqrt(eta) w] at the optimal w."""
    _, Ga, ha = _ridge_system(xi, alpha, rows, eta)
    return Ga @ _solve_ls(Ga, ha) - ha


def start_points(N: int):
    """Deterministic start abscissae in (0, 1): equispaced, and 8 warped copies."""
    base = (np.arange(N) + 0.5) / N
    pts = [base]
    for p in (0.5, 0.7, 0.85, 1.2, 1.5, 2.0):
        pts.append(base ** p)
    pts.append(0.5 * base + 0.25)
    pts.append(1.0 - (1.0 - base) ** 1.5)
    return pts


def design(N: int, alpha: float, beta: float, gamma: float = 1.0,
           spacing: float = 1.0 / 2000.0, eta: float = ETA):
    """SLRF design: returns (sigma[N], w[N], J_fit) with sigma sorted by real part.

    J_fit is the data-fit term ||Phi - h||_delta^2 at the returned design."""
    rows = trapezoid_rows(beta, spacing)

    def f(theta):
        return projected_residual(1.0 / (1.0 + np.exp(-theta)), alpha, rows, eta)

    best, best_J = None, np.inf
    for x0 in start_points(N):
        th0 = np.log(x0 / (1.0 - x0))
        r = least_squares(f, th0, method="lm", xtol=1e-13, ftol=1e-15, gtol=1e-15,
                          max_nfev=5000 * (N + 1))
        J = float(r.fun @ r.fun)
        if J < best_J:
            best, best_J = r, J
    xi = np.sort(1.0 / (1.0 + np.exp(-best.x)))
    w, J = weights_for(xi, alpha, rows, eta)
    sigma = gamma * xi * (1.0 + 1j * alpha)
    return sigma, gamma * w, J


def circle_quadrature(N: int, rule: str, gamma: float):
    """Upper-half-plane nodes/weights of a quadrature rule on the circle with
    centre gamma/2 and radius gamma/2 (Section 3.2): 'midpoint', 'gauss-legendre'
    or 'gauss-chebyshev' in the angle theta in (0, pi).  The contour integral
    (1/2 pi i) oint f(z)/(z - x) ... of the spectral projector gives, with
    z = c + r e^{i theta}, Phi(x) = sum_j 2 Re(w_j/(x - z_j)) with
    w_j = -(1/(2 pi)) r e^{i theta_j} q_j for angle weights q_j on (0, pi)
    (the lower half follows by conjugation; the sign makes Phi ~ 1 inside)."""
    c = r = gamma / 2.0
    if rule == "midpoint":
        th = (np.arange(N) + 0.5) * np.pi / N
        q = np.full(N, np.pi / N)
    elif rule == "gauss-legendre":
        x, qq = np.polynomial.legendre.leggauss(N)
        th = (x + 1.0) * np.pi / 2.0
        q = qq * np.pi / 2.0
    elif rule == "gauss-chebyshev":
        k = np.arange(1, N + 1)
        x = np.cos((2 * k - 1) * np.pi / (2 * N))
        th = (x + 1.0) * np.pi / 2.0
        # integral of g over [-1, 1] ~ sum pi/N sqrt(1-x^2) g(x_k)
        q = (np.pi / N) * np.sqrt(1.0 - x * x) * np.pi / 2.0
    else:
        raise ValueError(rule)
    z = c + r * np.exp(1j * th)
    w = -(r * np.exp(1j * th)) * q / (2.0 * np.pi)
    order = np.argsort(z.real)
    return z[order], w[order]
