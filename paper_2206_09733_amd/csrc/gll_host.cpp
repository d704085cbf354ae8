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

namespace dg {

// Gauss-Legendre nodes (zeros of P_n: eigenvalues of the Jacobi matrix with off-diagonals
// k / sqrt(4k^2 - 1)) by Sturm bisection, and weights 2 / ((1 - x^2) P_n'(x)^2).
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  std::vector<double> b2(n, 0.0);
  for (int k = 1; k < n; k++) b2[k] = (double)k * k / (4.0 * k * k - 1.0);
  for (int j = 0; j < n; j++) {
    double lo = -1.0, hi = 1.0;
    for (int it = 0; it < 200; it++) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (sturm_count(n, b2, mid) > j) hi = mid;
      else lo = mid;
    }
    x[j] = 0.5 * (lo + hi);
  }
  for (int j = 0; j < n; j++) {
    double pm = 1.0, pc = x[j], dm = 0.0, dc = 1.0;
    for (int k = 1; k < n; k++) {
      const double pn = ((2.0 * k + 1.0) * x[j] * pc - k * pm) / (k + 1.0);
      const double dn = dm + (2.0 * k + 1.0) * pc;
      pm = pc; pc = pn; dm = dc; dc = dn;
    }
    const double dp = n == 1 ? 1.0 : dc;
    w[j] = 2.0 / ((1.0 - x[j] * x[j]) * dp * dp);
  }
}

// value at y of the j-th Lagrange basis polynomial through nodes x[0..n) (barycentric form)
static double lagrange_at(const double* x, int n, int j, double y) {
  for (int k = 0; k < n; k++)
    if (y == x[k]) return k == j ? 1.0 : 0.0;
  double num = 0.0, den = 0.0, lj = 0.0;
  for (int k = 0; k < n; k++) {
    double l = 1.0;
    for (int r = 0; r < n; r++)
      if (r != k) l /= (x[k] - x[r]);
    const double t = l / (y - x[k]);
    den += t;
    if (k == j) lj = t;
  }
  (void)num;
  return lj / den;
}

// Gauss-Legendre tables of order N (n = N + 1 points): points and weights as above, the
// barycentric derivative matrix (rows annihilate constants), and the Lagrange basis at the ends:
// lb[j] = l_j(-1), lb[n + j] = l_j(+1).
void gl_tables(int N, double* xi, double* w, double* D, double* lb) {
  const int n = N + 1;
  std::vector<double> x, wv;
  gauss_legendre(n, x, wv);
  for (int j = 0; j < n / 2; j++) {  // exact symmetry about 0
    const double a = 0.5 * (x[n - 1 - j] - x[j]);
    x[j] = -a;
    x[n - 1 - j] = a;
    const double ww = 0.5 * (wv[j] + wv[n - 1 - j]);
    wv[j] = wv[n - 1 - j] = ww;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
  std::vector<double> lam(n);
  for (int j = 0; j < n; j++) {
    double p = 1.0;
    for (int k = 0; k < n; k++)
      if (k != j) p *= (x[j] - x[k]);
    lam[j] = 1.0 / p;
  }
  for (int i = 0; i < n; i++) {
    xi[i] = x[i];
    w[i] = wv[i];
    double diag = 0.0;
    for (int j = 0; j < n; j++) {
      if (j == i) continue;
      const double d = (lam[j] / lam[i]) / (x[i] - x[j]);
      D[i * n + j] = d;
      diag -= d;
    }
    D[i * n + i] = diag;
    lb[i] = lagrange_at(x.data(), n, i, -1.0);
    lb[n + i] = lagrange_at(x.data(), n, i, 1.0);
  }
}

// Geometry tables of Gauss-Legendre meshes of order N: the Lobatto nodes xl, the Lobatto
// derivative matrix Dl and I[q*n+l], the Lobatto basis function l at Gauss point q (the points of
// gl_tables).
void lobatto_to_gauss(int N, double* xl, double* Dl, double* I) {
  const int n = N + 1;
  std::vector<double> wl(n), Dhl(n * n), xg(n), wg(n), Dg(n * n), lb(n * n);
  gll_tables(N, xl, wl.data(), Dl, Dhl.data());
  gl_tables(N, xg.data(), wg.data(), Dg.data(), lb.data());
  for (int q = 0; q < n; q++)
    for (int l = 0; l < n; l++) I[q * n + l] = lagrange_at(xl, n, l, xg[q]);
}

// Mortar operators between Lobatto grids of orders N < M:
//   I[p][q] (M+1)x(N+1): value at M-node p of the order-N interpolant of the q-th basis function
//   P[i][q] (N+1)x(M+1): L2 projection onto degree N of the q-th order-M basis function,
//     P = Mass_N^{-1} B, Mass_N[i][j] = int l^N_i l^N_j, B[i][q] = int l^N_i l^M_q, integrated
//     exactly with Gauss-Legendre of N+M+1 points; Mass_N is factored by Cholesky.
void mortar_tables(int N, int M, double* I, double* P) {
  const int n = N + 1, m = M + 1;
  std::vector<double> xn(n), wn(n), xm(m), wm(m), Dn(n * n), Dm(m * m), Dhn(n * n), Dhm(m * m);
  gll_tables(N, xn.data(), wn.data(), Dn.data(), Dhn.data());
  gll_tables(M, xm.data(), wm.data(), Dm.data(), Dhm.data());
  for (int p = 0; p < m; p++)
    for (int q = 0; q < n; q++) I[p * n + q] = lagrange_at(xn.data(), n, q, xm[p]);
  std::vector<double> gx, gw;
  gauss_legendre(N + M + 1, gx, gw);
  const int G = (int)gx.size();
  std::vector<double> A(n * n, 0.0), B(n * m, 0.0);
  for (int g = 0; g < G; g++) {
    std::vector<double> ln(n), lm(m);
    for (int i = 0; i < n; i++) ln[i] = lagrange_at(xn.data(), n, i, gx[g]);
    for (int q = 0; q < m; q++) lm[q] = lagrange_at(xm.data(), m, q, gx[g]);
    for (int i = 0; i < n; i++) {
      for (int j = 0; j < n; j++) A[i * n + j] += gw[g] * ln[i] * ln[j];
      for (int q = 0; q < m; q++) B[i * m + q] += gw[g] * ln[i] * lm[q];
    }
  }
  // Cholesky A = L L^T, then solve for each column of B
  std::vector<double> L(n * n, 0.0);
  for (int i = 0; i < n; i++)
    for (int j = 0; j <= i; j++) {
      double s = A[i * n + j];
      for (int k = 0; k < j; k++) s -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = i == j ? std::sqrt(s) : s / L[j * n + j];
    }
  for (int q = 0; q < m; q++) {
    std::vector<double> y(n);
    for (int i = 0; i < n; i++) {
      double s = B[i * m + q];
      for (int k = 0; k < i; k++) s -= L[i * n + k] * y[k];
      y[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; i--) {
      double s = y[i];
      for (int k = i + 1; k < n; k++) s -= L[k * n + i] * P[k * m + q];
      P[i * m + q] = s / L[i * n + i];
    }
  }
}

}  // namespace dg
