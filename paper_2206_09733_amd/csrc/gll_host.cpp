// gll_host.cpp -- Gauss-Lobatto tables of the library, computed on the host once per order.
//
// Interior Lobatto nodes are the zeros of P_N', i.e. of the Gegenbauer polynomial C^(3/2)_{N-1},
// which are the eigenvalues of its symmetric tridiagonal Jacobi matrix (zero diagonal,
// off-diagonal sqrt(k(k+2)/((2k+1)(2k+3))), k = 1..N-2).  They are found by bisection on the
// Sturm sequence of that matrix.  Weights: 2/(N(N+1) P_N(x_j)^2).  The derivative matrix is the
// barycentric one, D_ij = (l_j/l_i)/(x_i - x_j) with l_j = 1/prod_{k != j}(x_j - x_k), and
// D_ii = -sum_{j != i} D_ij so that every row annihilates constants.
#include <cmath>
#include <vector>

namespace dg {

// number of eigenvalues below x of the (m x m) tridiagonal matrix with zero diagonal and
// squared off-diagonals b2[1..m-1]
static int sturm_count(int m, const std::vector<double>& b2, double x) {
  int count = 0;
  double q = -x;
  if (q < 0) count++;
  for (int k = 1; k < m; k++) {
    if (q == 0.0) q = 1e-300;
    q = -x - b2[k] / q;
    if (q < 0) count++;
  }
  return count;
}

static double legendre_value(int N, double x) {
  if (N == 0) return 1.0;
  double pm = 1.0, pc = x;
  for (int k = 1; k < N; k++) {
    const double pn = ((2.0 * k + 1.0) * x * pc - k * pm) / (k + 1.0);
    pm = pc;
    pc = pn;
  }
  return pc;
}

// xi[n], w[n], D[n*n], Dh[n*n] for order N (n = N + 1)
void gll_tables(int N, double* xi, double* w, double* D, double* Dh) {
  const int n = N + 1;
  std::vector<double> x(n);
  x[0] = -1.0;
  x[N] = 1.0;
  const int m = N - 1;
  if (m > 0) {
    std::vector<double> b2(m, 0.0);
    for (int k = 1; k < m; k++) b2[k] = (double)k * (k + 2) / ((2.0 * k + 1.0) * (2.0 * k + 3.0));
    for (int j = 0; j < m; j++) {
      double lo = -1.0, hi = 1.0;
      for (int it = 0; it < 200 && hi - lo > 0.0; it++) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(m, b2, mid) > j) hi = mid;
        else lo = mid;
      }
      x[1 + j] = 0.5 * (lo + hi);
    }
    for (int j = 1; j <= N / 2; j++) {  // exact symmetry about 0
      const double a = 0.5 * (x[N - j] - x[j]);
      x[j] = -a;
      x[N - j] = a;
    }
    if (N % 2 == 0) x[N / 2] = 0.0;
  }
  for (int j = 0; j < n; j++) {
    xi[j] = x[j];
    const double L = legendre_value(N, x[j]);
    w[j] = 2.0 / (N * (N + 1.0) * L * L);
  }
  std::vector<double> lam(n);
  for (int j = 0; j < n; j++) {
    double p = 1.0;
    for (int k = 0; k < n; k++)
      if (k != j) p *= (x[j] - x[k]);
    lam[j] = 1.0 / p;
  }
  for (int i = 0; i < n; i++) {
    double diag = 0.0;
    for (int j = 0; j < n; j++) {
      if (j == i) continue;
      const double d = (lam[j] / lam[i]) / (x[i] - x[j]);
      D[i * n + j] = d;
      diag -= d;
    }
    D[i * n + i] = diag;
  }
  for (int k = 0; k < n * n; k++) Dh[k] = D[k];
  Dh[N * n + N] -= 1.0 / w[N];
  Dh[0] += 1.0 / w[0];
}

}  // namespace dg
