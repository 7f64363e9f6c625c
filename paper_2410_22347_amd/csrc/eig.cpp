// Host FP64 symmetric eigensolver for the sphering fit.
//
// The fit needs eig(K_Q) (to form W = K_Q^(1/2) and its pseudo-inverse) and
// the leading eigenvectors of W K_{X_c} W for every cluster (Section 3.2 of
// the paper replaces the two SVDs of Algorithm 2 by these decompositions).
// The matrices are D x D with D <= a few thousand, so a dense two-phase
// method is used:
//   1. Householder reduction to tridiagonal form, T = Q^T A Q, with Q formed
//      by backward accumulation of the reflectors;
//   2. implicit symmetric QR steps with the Wilkinson shift on T (bulge
//      chasing with Givens rotations), deflating negligible off-diagonals,
//      the rotations being applied to the rows of Q^T.
// Rows of the returned Vt are unit eigenvectors, sorted by decreasing
// eigenvalue.  Returns false when an off-diagonal entry is still above the
// deflation threshold after the step budget (60 steps per order by default).  Written for clarity and cache-friendly row updates; all
// clusters are solved in parallel by the caller.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <numeric>
#include <vector>

namespace gv {

// QR steps allowed per decomposition before the solver reports failure
// (0: 60 per matrix order)
static std::atomic<long> g_step_limit{0};
void set_eig_step_limit(long max_steps) { g_step_limit = max_steps > 0 ? max_steps : 0; }

bool eigh_desc(int n, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& Vt) {
  lam.assign(n, 0.0);
  Vt.assign((size_t)n * n, 0.0);
  if (n == 1) {
    lam[0] = A[0];
    Vt[0] = 1.0;
    return true;
  }
  auto a_ = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };

  // ---------------------------------------------------------- 1. tridiagonalise
  std::vector<double> diag(n), off(n, 0.0);
  std::vector<std::vector<double>> refl(std::max(0, n - 2));
  std::vector<double> beta(std::max(0, n - 2), 0.0);
  std::vector<double> p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int L = n - k - 1;
    std::vector<double>& v = refl[k];
    v.assign(L, 0.0);
    double norm2 = 0.0;
    for (int r = 0; r < L; ++r) {
      v[r] = a_(k + 1 + r, k);
      norm2 += v[r] * v[r];
    }
    double xnorm = std::sqrt(norm2);
    if (xnorm == 0.0) {
      beta[k] = 0.0;
      off[k] = 0.0;
      continue;
    }
    double alpha = (v[0] > 0.0) ? -xnorm : xnorm;  // H x = alpha e1
    v[0] -= alpha;
    double vtv = 0.0;
    for (int r = 0; r < L; ++r) vtv += v[r] * v[r];
    double b = 2.0 / vtv;
    beta[k] = b;
    off[k] = alpha;
    // p = b S v on the trailing block S = A[k+1.., k+1..]
    for (int r = 0; r < L; ++r) {
      const double* row = &A[(size_t)(k + 1 + r) * n + (k + 1)];
      double s = 0.0;
      for (int c = 0; c < L; ++c) s += row[c] * v[c];
      p[r] = b * s;
    }
    double ptv = 0.0;
    for (int r = 0; r < L; ++r) ptv += p[r] * v[r];
    const double K = 0.5 * b * ptv;
    for (int r = 0; r < L; ++r) w[r] = p[r] - K * v[r];
    // S -= v w^T + w v^T
    for (int r = 0; r < L; ++r) {
      double* row = &A[(size_t)(k + 1 + r) * n + (k + 1)];
      const double vr = v[r], wr = w[r];
      for (int c = 0; c < L; ++c) row[c] -= vr * w[c] + wr * v[c];
    }
  }
  for (int i = 0; i < n; ++i) diag[i] = a_(i, i);
  off[n - 2] = a_(n - 1, n - 2);  // the last off-diagonal is never reflected

  // Q = H_0 H_1 ... H_{n-3}, formed backward so each step touches only the
  // trailing block; Q is stored transposed (rows of Qt are columns of Q).
  std::vector<double> Q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  std::vector<double> u(n);
  for (int k = n - 3; k >= 0; --k) {
    if (beta[k] == 0.0) continue;
    const std::vector<double>& v = refl[k];
    const int L = n - k - 1, o = k + 1;
    // Q[o.., o..] <- (I - b v v^T) Q[o.., o..]: u = v^T Q, Q -= b v u^T
    std::fill(u.begin(), u.begin() + L, 0.0);
    for (int r = 0; r < L; ++r) {
      const double vr = v[r];
      const double* row = &Q[(size_t)(o + r) * n + o];
      for (int c = 0; c < L; ++c) u[c] += vr * row[c];
    }
    for (int r = 0; r < L; ++r) {
      const double s = beta[k] * v[r];
      double* row = &Q[(size_t)(o + r) * n + o];
      for (int c = 0; c < L; ++c) row[c] -= s * u[c];
    }
  }
  // Vt = Q^T
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Vt[(size_t)j * n + i] = Q[(size_t)i * n + j];

  // ---------------------------------------------------------- 2. implicit QR
  const double eps = std::ldexp(1.0, -52);
  auto rotate_rows = [&](int r0, double c, double s) {
    double* x = &Vt[(size_t)r0 * n];
    double* y = &Vt[(size_t)(r0 + 1) * n];
    for (int j = 0; j < n; ++j) {
      const double xj = x[j], yj = y[j];
      x[j] = c * xj + s * yj;
      y[j] = -s * xj + c * yj;
    }
  };
  int hi = n - 1;
  long guard = 0;
  const long lim = g_step_limit.load();
  const long max_steps = lim > 0 ? lim : 60L * n;
  while (hi > 0 && guard < max_steps) {
    if (std::fabs(off[hi - 1]) <= eps * (std::fabs(diag[hi - 1]) + std::fabs(diag[hi]))) {
      off[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(off[lo - 1]) > eps * (std::fabs(diag[lo - 1]) + std::fabs(diag[lo]))) --lo;
    if (lo > 0) off[lo - 1] = 0.0;
    // Wilkinson shift from the trailing 2x2 block
    const double delta = 0.5 * (diag[hi - 1] - diag[hi]);
    const double bb = off[hi - 1];
    const double den = delta + (delta >= 0.0 ? 1.0 : -1.0) * std::hypot(delta, bb);
    const double mu = diag[hi] - (den != 0.0 ? bb * bb / den : 0.0);
    double x = diag[lo] - mu, z = off[lo];
    double bulge = 0.0;
    for (int k = lo; k < hi; ++k) {
      if (k > lo) {
        x = off[k - 1];
        z = bulge;
      }
      const double r = std::hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = x / r;
        s = z / r;
      }
      if (k > lo) off[k - 1] = r;
      const double ak = diag[k], ak1 = diag[k + 1], bk = off[k];
      diag[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
      diag[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
      off[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
      if (k + 1 < hi) {
        bulge = s * off[k + 1];
        off[k + 1] = c * off[k + 1];
      }
      rotate_rows(k, c, s);
    }
    ++guard;
  }
  const bool converged = hi == 0;

  // ---------------------------------------------------------- sort decreasing
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return diag[a] > diag[b]; });
  std::vector<double> sorted((size_t)n * n);
  for (int r = 0; r < n; ++r) {
    lam[r] = diag[order[r]];
    std::copy(&Vt[(size_t)order[r] * n], &Vt[(size_t)order[r] * n] + n, &sorted[(size_t)r * n]);
  }
  Vt.swap(sorted);
  return converged;
}

}  // namespace gv
