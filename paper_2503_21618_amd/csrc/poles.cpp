// SLRF pole/weight design (paper Section 3.1) at gamma = 1.
//
// Filter Phi(t) = sum_j 2 Re(w_j / (t - xi_j (1 + alpha i))).  Objective: the
// delta-weighted squared L2 distance to the step h (1 on [0, 1], 0 on (1, 10]),
// delta = beta on [0, 1] and 1 on (1, 10], each part by a composite trapezoid
// rule with node spacing 1/2000, plus a ridge term 1e-6 sum |w_j|^2.  Without
// the ridge the problem has no minimiser with distinct poles: merging poles
// lowers the objective while the weights diverge.
//
// The weights enter linearly, so for given abscissae they solve a ridge least
// squares problem (Householder QR here); the abscissae xi_j = 1/(1 + e^-theta_j)
// minimise the projected residual (variable projection) by Levenberg-Marquardt
// with a forward-difference Jacobian, from a fixed set of start points; the
// best result is kept.
#include <algorithm>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "dense.h"

namespace slrf {
namespace {

constexpr double kKappa = 10.0;
constexpr double kEta = 1e-6;
constexpr int kPerUnit = 2000;

struct Rows {
  std::vector<double> t, sw, h;
};

Rows make_rows(double beta) {
  Rows r;
  const int n1 = kPerUnit, n2 = (int)std::lround((kKappa - 1.0) * kPerUnit);
  for (int i = 0; i <= n1; ++i) {
    double q = 1.0 / n1;
    if (i == 0 || i == n1) q *= 0.5;
    r.t.push_back((double)i / n1);
    r.sw.push_back(std::sqrt(beta * q));
    r.h.push_back(1.0);
  }
  for (int i = 0; i <= n2; ++i) {
    double q = (kKappa - 1.0) / n2;
    if (i == 0 || i == n2) q *= 0.5;
    r.t.push_back(1.0 + (kKappa - 1.0) * i / n2);
    r.sw.push_back(std::sqrt(q));
    r.h.push_back(0.0);
  }
  return r;
}

// Ridge least squares for fixed xi; returns the stacked residual in `res`
// (size m + 2N) and the coefficients (Re w, Im w) in `coef`.  Column-major
// Householder QR with caller-owned scratch (one per thread).
struct Scratch {
  std::vector<double> G, Gc, y, yc;
};

void ridge_solve(const Rows& R, const std::vector<double>& xi, double alpha, std::vector<double>& coef,
                 std::vector<double>& res, Scratch& w) {
  const int N = (int)xi.size(), m = (int)R.t.size(), p = 2 * N, M = m + p;
  w.G.assign((size_t)M * p, 0.0);
  w.y.assign(M, 0.0);
  for (int j = 0; j < N; ++j) {
    const double sr = xi[j], si = xi[j] * alpha;
    double* gre = &w.G[(size_t)j * M];
    double* gim = &w.G[(size_t)(N + j) * M];
    for (int i = 0; i < m; ++i) {
      const double dr = R.t[i] - sr, di = -si;  // t - s
      const double den = dr * dr + di * di;
      gre[i] = 2.0 * (dr / den) * R.sw[i];      // 2 Re(1/(t - s))
      gim[i] = -2.0 * (-di / den) * R.sw[i];    // -2 Im(1/(t - s))
    }
  }
  for (int i = 0; i < m; ++i) w.y[i] = R.h[i] * R.sw[i];
  for (int j = 0; j < p; ++j) w.G[(size_t)j * M + m + j] = std::sqrt(kEta);
  w.Gc = w.G;
  w.yc = w.y;
  double* A = w.Gc.data();
  for (int k = 0; k < p; ++k) {
    double* ak = A + (size_t)k * M;
    double nrm = 0;
    for (int i = k; i < M; ++i) nrm += ak[i] * ak[i];
    nrm = std::sqrt(nrm);
    if (nrm == 0) continue;
    const double a = ak[k] > 0 ? -nrm : nrm;
    ak[k] -= a;  // ak[k..M) now holds the Householder vector v
    double vn = 0;
    for (int i = k; i < M; ++i) vn += ak[i] * ak[i];
    if (vn == 0) {
      ak[k] += a;
      continue;
    }
    const double scale = 2.0 / vn;
    for (int j = k + 1; j < p; ++j) {
      double* aj = A + (size_t)j * M;
      double sdot = 0;
      for (int i = k; i < M; ++i) sdot += ak[i] * aj[i];
      sdot *= scale;
      for (int i = k; i < M; ++i) aj[i] -= sdot * ak[i];
    }
    double sdot = 0;
    for (int i = k; i < M; ++i) sdot += ak[i] * w.yc[i];
    sdot *= scale;
    for (int i = k; i < M; ++i) w.yc[i] -= sdot * ak[i];
    ak[k] = a;  // R diagonal (below it: v, no longer needed)
  }
  coef.assign(p, 0.0);
  for (int k = p - 1; k >= 0; --k) {
    double sum = w.yc[k];
    for (int j = k + 1; j < p; ++j) sum -= A[(size_t)j * M + k] * coef[j];
    coef[k] = sum / A[(size_t)k * M + k];
  }
  res.assign(M, 0.0);
  for (int i = 0; i < M; ++i) res[i] = -w.y[i];
  for (int j = 0; j < p; ++j) {
    const double* gj = &w.G[(size_t)j * M];
    const double cj = coef[j];
    for (int i = 0; i < M; ++i) res[i] += gj[i] * cj;
  }
}

double cost_of(const std::vector<double>& r) {
  double s = 0;
  for (double v : r) s += v * v;
  return s;
}

std::vector<double> to_xi(const std::vector<double>& th) {
  std::vector<double> xi(th.size());
  for (size_t j = 0; j < th.size(); ++j) xi[j] = 1.0 / (1.0 + std::exp(-th[j]));
  return xi;
}

// Levenberg-Marquardt on theta; returns the final cost.
double lm(const Rows& R, double alpha, std::vector<double>& th) {
  const int N = (int)th.size();
  Scratch sc;
  std::vector<double> coef, r, rp;
  ridge_solve(R, to_xi(th), alpha, coef, r, sc);
  double cost = cost_of(r);
  double lambda = 1e-3;
  const int M = (int)r.size();
  std::vector<double> J((size_t)M * N);
  for (int it = 0; it < 300; ++it) {
    for (int j = 0; j < N; ++j) {
      std::vector<double> tp = th;
      const double hstep = 1e-7 * std::max(1.0, std::fabs(th[j]));
      tp[j] += hstep;
      ridge_solve(R, to_xi(tp), alpha, coef, rp, sc);
      for (int i = 0; i < M; ++i) J[(size_t)i * N + j] = (rp[i] - r[i]) / hstep;
    }
    std::vector<double> A((size_t)N * N, 0.0), g(N, 0.0);
    for (int i = 0; i < M; ++i)
      for (int a = 0; a < N; ++a) {
        const double ja = J[(size_t)i * N + a];
        g[a] += ja * r[i];
        for (int b = 0; b < N; ++b) A[(size_t)a * N + b] += ja * J[(size_t)i * N + b];
      }
    bool accepted = false;
    for (int tries = 0; tries < 20 && !accepted; ++tries) {
      // solve (A + lambda diag(A)) delta = -g by Gaussian elimination with pivoting
      std::vector<double> Ml = A, rhs(N);
      for (int a = 0; a < N; ++a) {
        Ml[(size_t)a * N + a] += lambda * std::max(A[(size_t)a * N + a], 1e-300);
        rhs[a] = -g[a];
      }
      for (int k = 0; k < N; ++k) {
        int piv = k;
        for (int i = k + 1; i < N; ++i)
          if (std::fabs(Ml[(size_t)i * N + k]) > std::fabs(Ml[(size_t)piv * N + k])) piv = i;
        if (piv != k) {
          for (int j = 0; j < N; ++j) std::swap(Ml[(size_t)k * N + j], Ml[(size_t)piv * N + j]);
          std::swap(rhs[k], rhs[piv]);
        }
        const double d = Ml[(size_t)k * N + k];
        if (d == 0) continue;
        for (int i = k + 1; i < N; ++i) {
          const double f = Ml[(size_t)i * N + k] / d;
          for (int j = k; j < N; ++j) Ml[(size_t)i * N + j] -= f * Ml[(size_t)k * N + j];
          rhs[i] -= f * rhs[k];
        }
      }
      std::vector<double> delta(N, 0.0);
      for (int k = N - 1; k >= 0; --k) {
        double s = rhs[k];
        for (int j = k + 1; j < N; ++j) s -= Ml[(size_t)k * N + j] * delta[j];
        delta[k] = Ml[(size_t)k * N + k] != 0 ? s / Ml[(size_t)k * N + k] : 0.0;
      }
      std::vector<double> tn = th;
      double step = 0, tnorm = 0;
      for (int j = 0; j < N; ++j) {
        tn[j] += delta[j];
        step += delta[j] * delta[j];
        tnorm += th[j] * th[j];
      }
      ridge_solve(R, to_xi(tn), alpha, coef, rp, sc);
      const double cn = cost_of(rp);
      if (cn < cost) {
        const double rel = (cost - cn) / cost;
        th = tn;
        r = rp;
        cost = cn;
        lambda = std::max(lambda / 3.0, 1e-12);
        accepted = true;
        if (rel < 1e-15 || std::sqrt(step) < 1e-13 * (1.0 + std::sqrt(tnorm))) return cost;
      } else {
        lambda *= 4.0;
      }
    }
    if (!accepted) break;
  }
  return cost;
}

}  // namespace

bool design_poles_unit(int N, double alpha, double beta, double* xi_out, double* omega_out) {
  const Rows R = make_rows(beta);
  std::vector<std::vector<double>> starts;
  std::vector<double> base(N);
  for (int j = 0; j < N; ++j) base[j] = (j + 0.5) / N;
  starts.push_back(base);
  for (double pw : {0.5, 0.7, 0.85, 1.2, 1.5, 2.0}) {
    std::vector<double> s(N);
    for (int j = 0; j < N; ++j) s[j] = std::pow(base[j], pw);
    starts.push_back(s);
  }
  {
    std::vector<double> s(N), s2(N);
    for (int j = 0; j < N; ++j) {
      s[j] = 0.5 * base[j] + 0.25;
      s2[j] = 1.0 - std::pow(1.0 - base[j], 1.5);
    }
    starts.push_back(s);
    starts.push_back(s2);
  }
  // independent start points run concurrently; the minimum is taken in start order
  std::vector<std::vector<double>> ths(starts.size());
  std::vector<double> costs(starts.size(), INFINITY);
  std::vector<std::thread> pool;
  for (size_t q = 0; q < starts.size(); ++q) {
    pool.emplace_back([&, q] {
      std::vector<double> th(N);
      for (int j = 0; j < N; ++j) th[j] = std::log(starts[q][j] / (1.0 - starts[q][j]));
      costs[q] = lm(R, alpha, th);
      ths[q] = th;
    });
  }
  for (auto& t : pool) t.join();
  double best = INFINITY;
  std::vector<double> best_th;
  for (size_t q = 0; q < starts.size(); ++q)
    if (costs[q] < best) {
      best = costs[q];
      best_th = ths[q];
    }
  if (best_th.empty()) return false;
  std::vector<double> xi = to_xi(best_th);
  std::sort(xi.begin(), xi.end());
  std::vector<double> coef, res;
  Scratch sc;
  ridge_solve(R, xi, alpha, coef, res, sc);
  for (int j = 0; j < N; ++j) {
    xi_out[j] = xi[j];
    omega_out[2 * j] = coef[j];
    omega_out[2 * j + 1] = coef[N + j];
  }
  return true;
}

// Quadrature-rule filters of Section 3.2 (the comparison systems of its filter
// study): nodes on the circle with centre gamma/2 and radius gamma/2, at angles
// theta_j in (0, pi) from a rule for the integral over theta of the contour
// integral of the spectral projector, z_j = c + r e^{i theta_j}, weights
// w_j = -(r e^{i theta_j} q_j) / (2 pi) for the rule's angle weights q_j (the
// lower half-plane follows by conjugation, Phi(x) = sum_j 2 Re(w_j/(x - z_j))).
// Gauss-Legendre nodes by Newton's method on the three-term recurrence of P_N.
bool quadrature_poles(int rule, int N, double gamma, double* sigma, double* weight) {
  if (N < 1 || N > 64 || !(gamma > 0)) return false;
  const double pi = 3.14159265358979323846;
  std::vector<double> th(N), q(N);
  if (rule == 0) {  // midpoint
    for (int j = 0; j < N; ++j) {
      th[j] = (j + 0.5) * pi / N;
      q[j] = pi / N;
    }
  } else if (rule == 1) {  // Gauss-Legendre on [-1, 1] mapped to (0, pi)
    for (int j = 0; j < N; ++j) {
      double x = std::cos(pi * (j + 0.75) / (N + 0.5));
      double dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= N; ++k) {
          const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        const double pn = N == 1 ? x : p1, pm = N == 1 ? 1.0 : p0;
        dp = N * (x * pn - pm) / (x * x - 1.0);
        const double dx = pn / dp;
        x -= dx;
        if (std::fabs(dx) < 1e-16) break;
      }
      {  // derivative at the converged node
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= N; ++k) {
          const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        const double pn = N == 1 ? x : p1, pm = N == 1 ? 1.0 : p0;
        dp = N * (x * pn - pm) / (x * x - 1.0);
      }
      th[j] = (x + 1.0) * pi / 2.0;
      q[j] = 2.0 / ((1.0 - x * x) * dp * dp) * pi / 2.0;
    }
  } else if (rule == 2) {  // Gauss-Chebyshev (first kind) for a smooth integrand on [-1, 1]
    for (int j = 0; j < N; ++j) {
      const double x = std::cos((2.0 * (j + 1) - 1.0) * pi / (2.0 * N));
      th[j] = (x + 1.0) * pi / 2.0;
      q[j] = (pi / N) * std::sqrt(1.0 - x * x) * pi / 2.0;
    }
  } else {
    return false;
  }
  const double c = gamma / 2.0, r = gamma / 2.0;
  std::vector<std::pair<double, int>> ord(N);
  std::vector<std::complex<double>> z(N), w(N);
  for (int j = 0; j < N; ++j) {
    const std::complex<double> e = std::polar(1.0, th[j]);
    z[j] = c + r * e;
    w[j] = -(r * e) * q[j] / (2.0 * pi);
    ord[j] = {z[j].real(), j};
  }
  std::sort(ord.begin(), ord.end());
  for (int j = 0; j < N; ++j) {
    const int k = ord[j].second;
    sigma[2 * j] = z[k].real();
    sigma[2 * j + 1] = z[k].imag();
    weight[2 * j] = w[k].real();
    weight[2 * j + 1] = w[k].imag();
  }
  return true;
}

}  // namespace slrf
