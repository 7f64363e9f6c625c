// Host driver for the FP64 eigensolver under AddressSanitizer and
// UndefinedBehaviorSanitizer: decompositions of seeded symmetric matrices of
// several orders (random, zero, identity, rank-one, repeated eigenvalues), each checked by its residual ||A V^T - V^T diag(lam)|| and the
// orthonormality of V, and the non-convergence report under a tiny step limit.
// Prints one line per case; exits non-zero on the first failure.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

namespace gv {
bool eigh_desc(int n, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& Vt);
void set_eig_step_limit(long max_steps);
}  // namespace gv

static uint64_t g_state = 0x2410223470ull;
static double uniform() {  // SplitMix64, mapped to [-1, 1)
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}

static bool check(const char* what, int n, const std::vector<double>& A0) {
  std::vector<double> A = A0, lam, Vt;
  if (!gv::eigh_desc(n, A, lam, Vt)) {
    std::printf("%s n=%d: no convergence\n", what, n);
    return false;
  }
  double scale = 1e-300, res = 0.0, orth = 0.0;
  for (double v : A0) scale = std::fmax(scale, std::fabs(v));
  for (int k = 0; k < n; ++k) {
    if (k > 0 && lam[k] > lam[k - 1]) {
      std::printf("%s n=%d: eigenvalues not in decreasing order\n", what, n);
      return false;
    }
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s += A0[(size_t)i * n + j] * Vt[(size_t)k * n + j];
      res = std::fmax(res, std::fabs(s - lam[k] * Vt[(size_t)k * n + i]));
    }
    for (int l = 0; l < n; ++l) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s += Vt[(size_t)k * n + j] * Vt[(size_t)l * n + j];
      orth = std::fmax(orth, std::fabs(s - (k == l ? 1.0 : 0.0)));
    }
  }
  const double tol = 64.0 * n * 0x1.0p-52;
  std::printf("%s n=%d: residual %.3g (x scale), orthogonality %.3g\n", what, n, res / scale, orth);
  return res <= tol * scale && orth <= tol;
}

int main() {
  const int orders[] = {1, 2, 3, 7, 33, 130};
  for (int n : orders) {
    std::vector<double> A((size_t)n * n), Z((size_t)n * n, 0.0), I((size_t)n * n, 0.0), R((size_t)n * n), U(n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = uniform();
    for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
    for (int i = 0; i < n; ++i) U[i] = uniform();
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) R[(size_t)i * n + j] = U[i] * U[j];
    // repeated eigenvalues: H diag(3, 3, 3, 1, 1, 1, ...) H with a Householder
    // reflection H = I - 2 v v^T / v^T v (so the matrix is not diagonal)
    std::vector<double> P((size_t)n * n), v(n);
    double vv = 0.0;
    for (int i = 0; i < n; ++i) vv += (v[i] = uniform()) * v[i];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) {
          const double hik = (i == k) - 2.0 * v[i] * v[k] / vv, hkj = (k == j) - 2.0 * v[k] * v[j] / vv;
          s += hik * ((k % 6) < 3 ? 3.0 : 1.0) * hkj;
        }
        P[(size_t)i * n + j] = s;
      }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) P[(size_t)i * n + j] = P[(size_t)j * n + i];  // exactly symmetric
    if (!check("random", n, A) || !check("zero", n, Z) || !check("identity", n, I) || !check("rank-one", n, R) ||
        !check("repeated", n, P))
      return 1;
  }
  // a step budget too small to converge is reported, not ignored
  gv::set_eig_step_limit(1);
  std::vector<double> A(33 * 33), lam, Vt;
  for (int i = 0; i < 33; ++i)
    for (int j = 0; j <= i; ++j) A[(size_t)i * 33 + j] = A[(size_t)j * 33 + i] = uniform();
  const bool ok = gv::eigh_desc(33, A, lam, Vt);
  gv::set_eig_step_limit(0);
  std::printf("step limit 1: %s\n", ok ? "converged" : "reported non-convergence");
  if (ok) return 1;
  std::printf("all cases passed\n");
  return 0;
}
