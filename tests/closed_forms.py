"""Closed-form spectra used as test expectations (not part of the oracle)."""
import numpy as np


def closed_1d(n):
    """Eigenpairs of the 1D linear-FE string with n interior nodes, h = 1/(n+1):
    lambda_k = (6/h^2)(1 - cos k pi h)/(2 + cos k pi h),
    x_k(i) = sin(k pi i h) / sqrt((h/6)(4 + 2 cos k pi h)(n+1)/2)  (B-normalised)."""
    h = 1.0 / (n + 1)
    k = np.arange(1, n + 1)
    c = np.cos(k * np.pi * h)
    one_minus_c = 2.0 * np.sin(0.5 * k * np.pi * h) ** 2
    lam = (6.0 / h ** 2) * one_minus_c / (2 + c)
    i = np.arange(1, n + 1)
    X = np.sin(np.outer(i, k) * np.pi * h) / np.sqrt((h / 6) * (4 + 2 * c) * (n + 1) / 2)
    return lam, X


def closed_3d_cc(m):
    """Sorted eigenvalues of the constant-coefficient Q1 pencil on (m-1)^3 interior
    nodes: sums mu_a + mu_b + mu_c of the 1D eigenvalues (Kronecker sums)."""
    mu, _ = closed_1d(m - 1)
    return np.sort((mu[:, None, None] + mu[None, :, None] + mu[None, None, :]).ravel())
