/*
 * dgsem_oracle.c -- plain CPU oracle of the DGSEM residual and low-storage RK3 (HORSES3D,
 * arXiv 2206.09733).  TEST INFRASTRUCTURE ONLY: loaded by tests/, __graft_entry__.smoke()
 * and bench.py's cpu_baseline leg, never by the product path.  It shares no code with the
 * HIP library.
 *
 * The paper states the continuous problem and the weak form but not the discrete formulas.
 * Each step below names the passage it follows and the reading taken where the paper is
 * silent:
 *   - conservation law, Euler and viscous fluxes: section "Compressible Navier-Stokes",
 *     eqs. compressibleNScompact and viscousfluxes (row 1 of F_e read as rho*v3; rho*e read as
 *     total energy per unit volume; H=(rho*e+p)/rho; calorically perfect gas, gamma=1.4,
 *     R=1 so T=p/rho, constant mu=1/Re, kappa=mu*gamma/((gamma-1)Pr));
 *   - curvilinear map, Jacobian, contravariant fluxes: section "Spatial discretisation",
 *     eq. compressibleNScompact_transformed; metric terms in the conservative curl form
 *     (the p-nonconforming geometry rules the paper cites for section "Spatial p-adaptation");
 *   - weak form with numerical flux (eqs. NS2-NS4) on Gauss-Lobatto points, written in the
 *     equivalent SBP strong form with a boundary lift (section "Energy/Entropy stable
 *     versions": the SBP-SAT property of Gauss-Lobatto quadrature);
 *   - split-form volume term with Chandrashekar's entropy-conserving two-point flux and the
 *     averaged metric of the two nodes (same section, list of split forms);
 *   - the other split forms of that list: Ismail-Roe's entropy-conserving flux and the
 *     kinetic-energy-preserving fluxes of Kennedy-Gruber, Pirozzoli, Ducros and Morinishi;
 *   - Riemann fluxes Roe (which is Roe-Pike's wave-strength evaluation), Lax-Friedrichs
 *     (local, i.e. Rusanov), low-dissipation Roe, matrix dissipation, central and the EC flux
 *     at faces (box of convective fluxes in section "Spatial discretisation");
 *   - BR1 for the viscous terms (same box), gradients of (v,T) lifted with the face average;
 *     the same box's BR2 and symmetric interior penalty as the other face viscous fluxes;
 *   - mortar coupling for faces between elements of different orders (section "Spatial
 *     p-adaptation"): interpolate both traces to the finer face grid, flux there, L2-project
 *     back with exactly integrated matrices;
 *   - on Gauss-Legendre nodes (the section's other quadrature), the plain weak form with
 *     interpolated face traces on uniform-order boxes (affine or deformed), with BR1, BR2 or
 *     the interior penalty for the viscous terms;
 *   - Williamson's low-storage RK3 and Carpenter-Kennedy's low-storage RK4 (section "Time
 *     advancement");
 *   - entropy S=-rho*s, s=ln p - gamma ln rho and w=dS/du (section "Shock capturing",
 *     eq. shock:entropy);
 *   - spectral vanishing viscosity (same section, eqs. shock:fluxmatrix and
 *     shock:filteredflux): the Navier-Stokes viscous flux in entropy variables, B = L^T D L,
 *     half-filtered in Legendre modal space with Tadmor's or Maday's kernel, the density sensor;
 *     and the explicit LES closures of the turbulence-models section (Smagorinsky, WALE,
 *     Vreman), as the eddy viscosity added to the artificial one node by node.
 *
 * Parity unpinned (no test fixes the choice; every other function fails a pin under a plausible
 * mistake): the averaged state of the matrix-dissipation surface flux (5), the L^T D L
 * factorisation of the SVV flux matrix (8c), and the interior penalty's use of the smaller of
 * the two traces of J on Gauss-Legendre points (7c; on these boxes the two agree).
 */
#include "dgsem_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORC_LONG_DOUBLE
typedef long double real;
#define RSQRT sqrtl
#define RCBRT cbrtl
#define RLOG logl
#define RSIN sinl
#define RCOS cosl
#define RFABS fabsl
#define REXP expl
#define RPOW powl
#else
typedef double real;
#define RSQRT sqrt
#define RCBRT cbrt
#define RLOG log
#define RSIN sin
#define RCOS cos
#define RFABS fabs
#define REXP exp
#define RPOW pow
#endif

#define PI_L 3.141592653589793238462643383279502884L

/* ------------------------------------------------------------------------------------------
 * 1. Gauss-Lobatto tables.  Nodes: -1, +1 and the roots of L_N' (found by Newton on
 *    L_{N+1}-L_{N-1}, which vanishes exactly at the N+1 Lobatto points); weights
 *    2/(N(N+1) L_N(x_j)^2); derivative matrix of the Lagrange interpolant through the nodes,
 *    D_ij = L_N(x_i)/(L_N(x_j)(x_i-x_j)) off the diagonal, D_00=-N(N+1)/4, D_NN=N(N+1)/4.
 *    All in long double, then rounded to `real`.
 * ---------------------------------------------------------------------------------------- */
static void legendre(int N, long double x, long double* L, long double* dL) {
  if (N == 0) { *L = 1.0L; *dL = 0.0L; return; }
  long double Lm = 1.0L, Lc = x, dLm = 0.0L, dLc = 1.0L;
  for (int k = 1; k < N; k++) {
    long double Ln = ((2.0L * k + 1.0L) * x * Lc - k * Lm) / (k + 1.0L);
    long double dLn = dLm + (2.0L * k + 1.0L) * Lc;
    Lm = Lc; Lc = Ln; dLm = dLc; dLc = dLn;
  }
  *L = Lc; *dL = dLc;
}

typedef struct {
  real xi[ORC_NMAX + 1];
  real w[ORC_NMAX + 1];
  real D[ORC_NMAX + 1][ORC_NMAX + 1];
  long double xl[ORC_NMAX + 1];
  real lb[2][ORC_NMAX + 1];  /* Lagrange basis at xi = -1 (lb[0]) and xi = +1 (lb[1]) */
} gll_t;

static gll_t GLL[ORC_NMAX + 1];  /* Gauss-Lobatto */
static gll_t GL[ORC_NMAX + 1];   /* Gauss-Legendre */
static int GLL_READY = 0;

static void gll_build(int N, gll_t* g) {
  long double x[ORC_NMAX + 1];
  x[0] = -1.0L; x[N] = 1.0L;
  for (int j = 1; j <= N / 2 && j < N; j++) {
    long double t = -cosl(PI_L * j / N);
    for (int it = 0; it < 200; it++) {
      long double a, da, b, db, c, dc;
      legendre(N + 1, t, &a, &da);
      legendre(N - 1, t, &b, &db);
      legendre(N, t, &c, &dc);
      long double q = a - b, dq = (2.0L * N + 1.0L) * c;
      long double dt = q / dq;
      t -= dt;
      if (fabsl(dt) < 1e-21L) break;
    }
    x[j] = t;
    x[N - j] = -t;
  }
  if (N % 2 == 0 && N > 0) x[N / 2] = 0.0L;
  long double LN[ORC_NMAX + 1];
  for (int j = 0; j <= N; j++) {
    long double dd;
    legendre(N, x[j], &LN[j], &dd);
    g->xl[j] = x[j];
    g->xi[j] = (real)x[j];
    g->w[j] = (real)(2.0L / (N * (N + 1.0L) * LN[j] * LN[j]));
  }
  for (int i = 0; i <= N; i++)
    for (int j = 0; j <= N; j++) {
      long double d;
      if (i != j) d = LN[i] / (LN[j] * (x[i] - x[j]));
      else if (i == 0) d = -N * (N + 1.0L) / 4.0L;
      else if (i == N) d = N * (N + 1.0L) / 4.0L;
      else d = 0.0L;
      g->D[i][j] = (real)d;
    }
  for (int j = 0; j <= N; j++) {
    g->lb[0][j] = j == 0 ? 1 : 0;
    g->lb[1][j] = j == N ? 1 : 0;
  }
}

/* Gauss-Legendre points of order N (the N+1 zeros of P_{N+1}, by Newton from the Chebyshev-like
 * guesses), weights 2/((1-x^2) P'^2), derivative matrix D_ij = P'(x_i)/(P'(x_j)(x_i - x_j)),
 * D_ii = x_i/(1 - x_i^2) (P = P_{N+1}), and the Lagrange basis at the ends as products. */
static void gl_build(int N, gll_t* g) {
  const int n = N + 1;
  long double x[ORC_NMAX + 1], dP[ORC_NMAX + 1];
  for (int j = 0; j < n; j++) {
    long double t = -cosl(PI_L * (j + 0.75L) / (n + 0.5L));
    long double L, dL;
    for (int it = 0; it < 200; it++) {
      legendre(n, t, &L, &dL);
      long double dt = L / dL;
      t -= dt;
      if (fabsl(dt) < 1e-21L) break;
    }
    legendre(n, t, &L, &dL);
    x[j] = t;
    dP[j] = dL;
  }
  for (int j = 0; j < n; j++) {
    g->xl[j] = x[j];
    g->xi[j] = (real)x[j];
    g->w[j] = (real)(2.0L / ((1.0L - x[j] * x[j]) * dP[j] * dP[j]));
  }
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++)
      g->D[i][j] = (real)(i != j ? dP[i] / (dP[j] * (x[i] - x[j])) : x[i] / (1.0L - x[i] * x[i]));
  for (int j = 0; j < n; j++)
    for (int side = 0; side < 2; side++) {
      long double y = side ? 1.0L : -1.0L, v = 1.0L;
      for (int r = 0; r < n; r++)
        if (r != j) v *= (y - x[r]) / (x[j] - x[r]);
      g->lb[side][j] = (real)v;
    }
}

static void mortar_tables(void);

static void gll_init(void) {
  if (GLL_READY) return;
  for (int N = 1; N <= ORC_NMAX; N++) {
    gll_build(N, &GLL[N]);
    gl_build(N, &GL[N]);
  }
  mortar_tables();
  GLL_READY = 1;
}

int orc_gl(int N, double* xi, double* w, double* D, double* lb) {
  if (N < 1 || N > ORC_NMAX) return -1;
  gll_init();
  for (int i = 0; i <= N; i++) {
    if (xi) xi[i] = (double)GL[N].xi[i];
    if (w) w[i] = (double)GL[N].w[i];
    if (lb) { lb[i] = (double)GL[N].lb[0][i]; lb[N + 1 + i] = (double)GL[N].lb[1][i]; }
    for (int j = 0; j <= N; j++)
      if (D) D[i * (N + 1) + j] = (double)GL[N].D[i][j];
  }
  return 0;
}

int orc_gll(int N, double* xi, double* w, double* D) {
  if (N < 1 || N > ORC_NMAX) return -1;
  gll_init();
  for (int i = 0; i <= N; i++) {
    if (xi) xi[i] = (double)GLL[N].xi[i];
    if (w) w[i] = (double)GLL[N].w[i];
    for (int j = 0; j <= N; j++)
      if (D) D[i * (N + 1) + j] = (double)GLL[N].D[i][j];
  }
  return 0;
}

/* ------------------------------------------------------------------------------------------
 * 2. Mortar operators (section "Spatial p-adaptation": mortar coupling).  Interpolation from
 *    the Lobatto grid of order N to the one of order M (Lagrange basis evaluated at the M
 *    nodes), and the L2 projection back, P = Mass_N^{-1} B_NM with
 *    Mass_N[i][j] = int l^N_i l^N_j and B_NM[i][j] = int l^N_i l^M_j integrated exactly by a
 *    Gauss-Legendre rule of G = 2*ORC_NMAX+2 points.
 * ---------------------------------------------------------------------------------------- */
static long double lagrange(int N, int j, long double x) {
  long double v = 1.0L;
  for (int r = 0; r <= N; r++)
    if (r != j) v *= (x - GLL[N].xl[r]) / (GLL[N].xl[j] - GLL[N].xl[r]);
  return v;
}

#define GQ (2 * ORC_NMAX + 2)
static long double GQX[GQ], GQW[GQ];
static int GQ_READY = 0;

static void gauss_init(void) {
  if (GQ_READY) return;
  for (int j = 0; j < GQ; j++) {
    long double t = -cosl(PI_L * (j + 0.75L) / (GQ + 0.5L));
    long double L, dL;
    for (int it = 0; it < 200; it++) {
      legendre(GQ, t, &L, &dL);
      long double dt = L / dL;
      t -= dt;
      if (fabsl(dt) < 1e-21L) break;
    }
    legendre(GQ, t, &L, &dL);
    GQX[j] = t;
    GQW[j] = 2.0L / ((1.0L - t * t) * dL * dL);
  }
  GQ_READY = 1;
}

/* I[p][q]: value at node p of grid M of the order-N interpolant through values at node q. */
static void interp_matrix(int N, int M, real I[ORC_NMAX + 1][ORC_NMAX + 1]) {
  for (int p = 0; p <= M; p++)
    for (int q = 0; q <= N; q++) I[p][q] = (real)lagrange(N, q, GLL[M].xl[p]);
}

/* P[i][q]: order-N nodal coefficient i of the L2 projection of the order-M basis function q. */
static void project_matrix(int N, int M, real P[ORC_NMAX + 1][ORC_NMAX + 1]) {
  gauss_init();
  long double A[ORC_NMAX + 1][2 * (ORC_NMAX + 1)];
  int n = N + 1;
  for (int i = 0; i <= N; i++) {
    for (int j = 0; j <= N; j++) {
      long double s = 0.0L;
      for (int g = 0; g < GQ; g++) s += GQW[g] * lagrange(N, i, GQX[g]) * lagrange(N, j, GQX[g]);
      A[i][j] = s;
    }
    for (int j = 0; j <= M; j++) {
      long double s = 0.0L;
      for (int g = 0; g < GQ; g++) s += GQW[g] * lagrange(N, i, GQX[g]) * lagrange(M, j, GQX[g]);
      A[i][n + j] = s;
    }
  }
  /* Gauss-Jordan elimination with partial pivoting: [Mass | B] -> [I | Mass^{-1} B] */
  for (int c = 0; c < n; c++) {
    int piv = c;
    for (int r = c + 1; r < n; r++)
      if (fabsl(A[r][c]) > fabsl(A[piv][c])) piv = r;
    if (piv != c)
      for (int k = 0; k < n + M + 1; k++) { long double t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t; }
    long double d = A[c][c];
    for (int k = 0; k < n + M + 1; k++) A[c][k] /= d;
    for (int r = 0; r < n; r++) {
      if (r == c) continue;
      long double f = A[r][c];
      for (int k = 0; k < n + M + 1; k++) A[r][k] -= f * A[c][k];
    }
  }
  for (int i = 0; i <= N; i++)
    for (int q = 0; q <= M; q++) P[i][q] = (real)A[i][n + q];
}

/* INTERP[N][M]: order N -> order M interpolation, PROJ[N][M]: order M -> order N projection */
static real INTERP[ORC_NMAX + 1][ORC_NMAX + 1][ORC_NMAX + 1][ORC_NMAX + 1];
static real PROJ[ORC_NMAX + 1][ORC_NMAX + 1][ORC_NMAX + 1][ORC_NMAX + 1];

static void mortar_tables(void) {
  for (int N = 1; N <= ORC_NMAX; N++)
    for (int M = N; M <= ORC_NMAX; M++) {
      interp_matrix(N, M, INTERP[N][M]);
      project_matrix(N, M, PROJ[N][M]);
    }
}

int orc_mortar_matrices(int N, int M, double* I, double* P) {
  if (N < 1 || M < N || M > ORC_NMAX) return -1;
  gll_init();
  for (int p = 0; p <= M; p++)
    for (int q = 0; q <= N; q++) I[p * (N + 1) + q] = (double)INTERP[N][M][p][q];
  for (int i = 0; i <= N; i++)
    for (int q = 0; q <= M; q++) P[i * (M + 1) + q] = (double)PROJ[N][M][i][q];
  return 0;
}

/* ------------------------------------------------------------------------------------------
 * 3. Solver state.
 * ---------------------------------------------------------------------------------------- */
struct orc_solver {
  int ex, ey, ez, E;
  real lo[3], hi[3], h[3];
  int deform;
  real amp;
  int (*N)[3];      /* polynomial order per element and reference direction */
  long* off;        /* first node of each element */
  long ntot;
  int* nbr;         /* nbr[6e + 2d + s]: element across face (d, s), s=0 at xi_d=-1, 1 at +1 */
  real gamma, Pr, Ma, Re, mu, kappa;
  int vol, surf, viscous;
  int visc_flux;   /* ORC_VISC_BR1 / BR2 / IP */
  int gauss;       /* Gauss-Legendre nodes (weak form) instead of Gauss-Lobatto */
  real lam_g;      /* global Lax-Friedrichs: max |v| + c of the state being evaluated */
  const gll_t* T;  /* the node tables of this solver: GLL or GL */
  real visc_eta;   /* BR2 lifting factor, or interior-penalty factor */
  int svv;         /* spectral vanishing viscosity on (section 8c) */
  int svv_kernel, svv_cut;
  real svv_mu, svv_kappa, svv_sensor;
  real les_cs;     /* constant of the explicit LES closure; 0 = off */
  int les_model;   /* ORC_LES_SMAGORINSKY / WALE / VREMAN */
  real *Gw, *Fa;   /* entropy-variable gradients (15 per node), filtered fluxes (15 per node) */
  real *X, *Ja, *J; /* coordinates, metric terms, Jacobian */
  real *U, *dU, *G, *R;
};

static inline long nidx(const int n1, const int n2, int i, int j, int k) {
  return i + (long)n1 * (j + (long)n2 * k);
}

/* index of the node of element e with reference indices (i0,i1,i2) */
static inline long node_of(const orc_solver* s, int e, const int ii[3]) {
  const int* N = s->N[e];
  return nidx(N[0] + 1, N[1] + 1, ii[0], ii[1], ii[2]);
}

static inline int nn_of(const orc_solver* s, int e) {
  return (s->N[e][0] + 1) * (s->N[e][1] + 1) * (s->N[e][2] + 1);
}

/* state of node q of element e from array A (5 fields) */
static inline void load5(const orc_solver* s, const real* A, int e, long q, real u[5]) {
  int nn = nn_of(s, e);
  const real* base = A + s->off[e] * 5;
  for (int v = 0; v < 5; v++) u[v] = base[(long)v * nn + q];
}

static inline void load_ja(const orc_solver* s, int e, long q, int d, real n[3]) {
  int nn = nn_of(s, e);
  const real* base = s->Ja + s->off[e] * 9;
  for (int c = 0; c < 3; c++) n[c] = base[(long)(3 * d + c) * nn + q];
}

/* ------------------------------------------------------------------------------------------
 * 4. Mesh: periodic box, optional sin*sin deformation evaluated on the undeformed
 *    coordinates, nodes = map at the Lobatto points (isoparametric).
 * ---------------------------------------------------------------------------------------- */
static void displacement(const orc_solver* s, const real xu[3], real dx[3]) {
  dx[0] = dx[1] = dx[2] = 0;
  if (s->deform) {
    dx[0] = s->amp * RSIN(xu[1]) * RSIN(xu[2]);
    dx[1] = s->amp * RSIN(xu[2]) * RSIN(xu[0]);
    dx[2] = s->amp * RSIN(xu[0]) * RSIN(xu[1]);
  }
}

/* derivative along reference direction d, at node ii of element e, of a nodal field f on the
 * nodes of table set T (the element's orders) */
static real dref_t(const orc_solver* s, const gll_t* T, int e, const real* f, int d, const int ii[3]) {
  int Nd = s->N[e][d];
  real acc = 0;
  int jj[3] = {ii[0], ii[1], ii[2]};
  for (int m = 0; m <= Nd; m++) {
    jj[d] = m;
    acc += T[Nd].D[ii[d]][m] * f[node_of(s, e, jj)];
  }
  return acc;
}

static real dref(const orc_solver* s, int e, const real* f, int d, const int ii[3]) {
  return dref_t(s, s->T, e, f, d, ii);
}

/* Geometry of element e on the nodes of table set T: coordinates X[3][nn], metric terms
 * Ja[9][nn] in the curl form and the map's derivatives dX[9][nn] (dX[3m+d] = d x_m / d xi_d). */
static void element_geometry(const orc_solver* s, int e, const gll_t* T, real* X, real* Ja, real* dX) {
  int a = e % s->ex, b = (e / s->ex) % s->ey, c = e / (s->ex * s->ey);
  int cell[3] = {a, b, c};
  const int* N = s->N[e];
  int nn = nn_of(s, e);
  /* The map is x = corner + Xl, Xl = (1+xi)/2 h + displacement.  The metric terms depend
   * only on derivatives of x and on x up to a constant per element (a constant c added to
   * X_l in the curl form adds c grad X_m, whose discrete curl vanishes because the
   * tensor-product derivative matrices commute), so they are formed from Xl, whose size is
   * the element's, not the box's. */
  real* Xl = (real*)malloc(sizeof(real) * 3 * nn);
  for (int k = 0; k <= N[2]; k++)
    for (int j = 0; j <= N[1]; j++)
      for (int i = 0; i <= N[0]; i++) {
        int ii[3] = {i, j, k};
        real xu[3], loc[3], dx[3];
        for (int d = 0; d < 3; d++) {
          loc[d] = (1 + T[N[d]].xi[ii[d]]) / 2 * s->h[d];
          xu[d] = s->lo[d] + cell[d] * s->h[d] + loc[d];
        }
        displacement(s, xu, dx);
        long q = node_of(s, e, ii);
        for (int d = 0; d < 3; d++) {
          X[(long)d * nn + q] = xu[d] + dx[d];
          Xl[(long)d * nn + q] = loc[d] + dx[d];
        }
      }
  real* A = (real*)malloc(sizeof(real) * 3 * nn);
  for (int k = 0; k <= N[2]; k++)
    for (int j = 0; j <= N[1]; j++)
      for (int i = 0; i <= N[0]; i++) {
        int ii[3] = {i, j, k};
        long q = node_of(s, e, ii);
        for (int m = 0; m < 3; m++)
          for (int d = 0; d < 3; d++) dX[(3 * m + d) * nn + q] = dref_t(s, T, e, Xl + (long)m * nn, d, ii);
      }
  /* curl form: Ja^i_n = -[curl_xi (X_l grad_xi X_m)]_i with (n,m,l) cyclic */
  for (int n = 0; n < 3; n++) {
    int m = (n + 1) % 3, l = (n + 2) % 3;
    for (int q = 0; q < nn; q++)
      for (int d = 0; d < 3; d++) A[d * nn + q] = Xl[(long)l * nn + q] * dX[(3 * m + d) * nn + q];
    for (int k = 0; k <= N[2]; k++)
      for (int j = 0; j <= N[1]; j++)
        for (int i = 0; i <= N[0]; i++) {
          int ii[3] = {i, j, k};
          long q = node_of(s, e, ii);
          /* curl components: (d1 A2 - d2 A1, d2 A0 - d0 A2, d0 A1 - d1 A0) */
          real c0 = dref_t(s, T, e, A + 2 * nn, 1, ii) - dref_t(s, T, e, A + 1 * nn, 2, ii);
          real c1 = dref_t(s, T, e, A + 0 * nn, 2, ii) - dref_t(s, T, e, A + 2 * nn, 0, ii);
          real c2 = dref_t(s, T, e, A + 1 * nn, 0, ii) - dref_t(s, T, e, A + 0 * nn, 1, ii);
          Ja[(long)(3 * 0 + n) * nn + q] = -c0;
          Ja[(long)(3 * 1 + n) * nn + q] = -c1;
          Ja[(long)(3 * 2 + n) * nn + q] = -c2;
        }
  }
  free(A);
  free(Xl);
}

/* J = a_1 . (a_2 x a_3), a_d = dX/dxi_d, at each of the nn nodes */
static void jacobian(const real* dX, int nn, real* J) {
  for (int q = 0; q < nn; q++) {
    real a1[3], a2[3], a3[3];
    for (int m = 0; m < 3; m++) {
      a1[m] = dX[(3 * m + 0) * nn + q];
      a2[m] = dX[(3 * m + 1) * nn + q];
      a3[m] = dX[(3 * m + 2) * nn + q];
    }
    J[q] = a1[0] * (a2[1] * a3[2] - a2[2] * a3[1]) + a1[1] * (a2[2] * a3[0] - a2[0] * a3[2]) +
           a1[2] * (a2[0] * a3[1] - a2[1] * a3[0]);
  }
}

/* Gauss-Legendre solvers: the map and its metric terms are those of the Lobatto grid of the
 * same order (isoparametric there, curl form there), evaluated as the polynomials they are at
 * the Gauss points.  The curl form makes sum_d d(Ja^d)/dxi_d vanish at the (N+1)^3 Lobatto
 * nodes, hence identically for these polynomials, hence at any points; and the normal
 * component on a face depends only on the Lobatto nodes of that face, which both elements
 * share, so the face metric the two sides interpolate is the same (free stream). */
static void element_geometry_gauss(const orc_solver* s, int e, real* X, real* Ja, real* J) {
  const int N = s->N[e][0], n = N + 1, nn = n * n * n;
  real* Xg = (real*)malloc(sizeof(real) * 21 * nn);  /* X, Ja, dX on the Lobatto nodes */
  real* tmp = (real*)malloc(sizeof(real) * 2 * nn);
  real* out = (real*)malloc(sizeof(real) * 21 * nn);
  element_geometry(s, e, GLL, Xg, Xg + 3 * nn, Xg + 12 * nn);
  /* I[g][l]: the Lobatto basis function l at Gauss point g */
  real I[ORC_NMAX + 1][ORC_NMAX + 1];
  for (int g = 0; g < n; g++)
    for (int l = 0; l < n; l++) I[g][l] = (real)lagrange(N, l, GL[N].xl[g]);
  for (int f = 0; f < 21; f++) {
    const real* src = Xg + (long)f * nn;
    real *t1 = tmp, *t2 = tmp + nn;
    for (int k = 0; k < n; k++)  /* along xi_0, then xi_1, then xi_2 */
      for (int j = 0; j < n; j++)
        for (int g = 0; g < n; g++) {
          real acc = 0;
          for (int l = 0; l < n; l++) acc += I[g][l] * src[nidx(n, n, l, j, k)];
          t1[nidx(n, n, g, j, k)] = acc;
        }
    for (int k = 0; k < n; k++)
      for (int g = 0; g < n; g++)
        for (int i = 0; i < n; i++) {
          real acc = 0;
          for (int l = 0; l < n; l++) acc += I[g][l] * t1[nidx(n, n, i, l, k)];
          t2[nidx(n, n, i, g, k)] = acc;
        }
    for (int g = 0; g < n; g++)
      for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
          real acc = 0;
          for (int l = 0; l < n; l++) acc += I[g][l] * t2[nidx(n, n, i, j, l)];
          out[(long)f * nn + nidx(n, n, i, j, g)] = acc;
        }
  }
  memcpy(X, out, sizeof(real) * 3 * nn);
  memcpy(Ja, out + 3 * nn, sizeof(real) * 9 * nn);
  jacobian(out + 12 * nn, nn, J);
  free(Xg);
  free(tmp);
  free(out);
}

static void build_geometry(orc_solver* s) {
#pragma omp parallel for schedule(static)
  for (int e = 0; e < s->E; e++) {
    int nn = nn_of(s, e);
    real* X = s->X + s->off[e] * 3;
    real* Ja = s->Ja + s->off[e] * 9;
    real* J = s->J + s->off[e];
    if (s->gauss) {
      element_geometry_gauss(s, e, X, Ja, J);
      continue;
    }
    real* dX = (real*)malloc(sizeof(real) * 9 * nn);
    element_geometry(s, e, s->T, X, Ja, dX);
    jacobian(dX, nn, J);
    free(dX);
  }
}

static orc_solver* create(int ex, int ey, int ez, const double* lo, const double* hi, int deform, double amp,
                          int n_uniform, const int* orders, double gamma, double Pr, double Ma, double Re,
                          int vol_flux, int surf_flux, int gauss) {
  if (ex < 1 || ey < 1 || ez < 1 || !lo || !hi) return NULL;
  if (vol_flux < 0 || vol_flux > ORC_VOL_MORINISHI || surf_flux < 0 || surf_flux > ORC_SURF_LF_GLOBAL) return NULL;
  gll_init();
  orc_solver* s = (orc_solver*)calloc(1, sizeof(orc_solver));
  s->gauss = gauss;
  s->T = gauss ? GL : GLL;
  s->ex = ex; s->ey = ey; s->ez = ez; s->E = ex * ey * ez;
  for (int d = 0; d < 3; d++) { s->lo[d] = lo[d]; s->hi[d] = hi[d]; }
  s->h[0] = (s->hi[0] - s->lo[0]) / ex;
  s->h[1] = (s->hi[1] - s->lo[1]) / ey;
  s->h[2] = (s->hi[2] - s->lo[2]) / ez;
  s->deform = deform; s->amp = amp;
  s->gamma = gamma; s->Pr = Pr; s->Ma = Ma; s->Re = Re;
  s->viscous = Re > 0;
  s->mu = s->viscous ? (real)1 / (real)Re : 0;
  s->kappa = s->viscous ? s->mu * s->gamma / ((s->gamma - 1) * s->Pr) : 0;
  s->vol = vol_flux; s->surf = surf_flux;
  s->visc_flux = ORC_VISC_BR1;
  s->visc_eta = 0;
  s->N = (int(*)[3])malloc(sizeof(int[3]) * s->E);
  s->off = (long*)malloc(sizeof(long) * (s->E + 1));
  long acc = 0;
  for (int e = 0; e < s->E; e++) {
    for (int d = 0; d < 3; d++) {
      int n = orders ? orders[3 * e + d] : n_uniform;
      if (n < 1 || n > ORC_NMAX) { orc_destroy(s); return NULL; }
      s->N[e][d] = n;
    }
    s->off[e] = acc;
    acc += nn_of(s, e);
  }
  s->off[s->E] = acc;
  s->ntot = acc;
  s->nbr = (int*)malloc(sizeof(int) * 6 * s->E);
  for (int e = 0; e < s->E; e++) {
    int a = e % ex, b = (e / ex) % ey, c = e / (ex * ey);
    s->nbr[6 * e + 0] = ((a + ex - 1) % ex) + ex * (b + ey * c);
    s->nbr[6 * e + 1] = ((a + 1) % ex) + ex * (b + ey * c);
    s->nbr[6 * e + 2] = a + ex * (((b + ey - 1) % ey) + ey * c);
    s->nbr[6 * e + 3] = a + ex * (((b + 1) % ey) + ey * c);
    s->nbr[6 * e + 4] = a + ex * (b + ey * ((c + ez - 1) % ez));
    s->nbr[6 * e + 5] = a + ex * (b + ey * ((c + 1) % ez));
  }
  /* viscous terms are only defined here on conforming faces */
  if (s->viscous)
    for (int e = 0; e < s->E; e++)
      for (int d = 0; d < 3; d++) {
        int r = s->nbr[6 * e + 2 * d + 1];
        for (int t = 0; t < 3; t++)
          if (t != d && s->N[e][t] != s->N[r][t]) { orc_destroy(s); return NULL; }
      }
  s->X = (real*)calloc(3 * acc, sizeof(real));
  s->Ja = (real*)calloc(9 * acc, sizeof(real));
  s->J = (real*)calloc(acc, sizeof(real));
  s->U = (real*)calloc(5 * acc, sizeof(real));
  s->dU = (real*)calloc(5 * acc, sizeof(real));
  s->R = (real*)calloc(5 * acc, sizeof(real));
  s->G = (real*)calloc(12 * acc, sizeof(real));
  if (!s->X || !s->Ja || !s->J || !s->U || !s->dU || !s->R || !s->G) { orc_destroy(s); return NULL; }
  build_geometry(s);
  return s;
}

orc_solver* orc_create(int ex, int ey, int ez, const double* lo, const double* hi, int deform,
                       double amp, int n_uniform, const int* orders, double gamma, double Pr,
                       double Ma, double Re, int vol_flux, int surf_flux) {
  return create(ex, ey, ez, lo, hi, deform, amp, n_uniform, orders, gamma, Pr, Ma, Re, vol_flux, surf_flux, 0);
}

orc_solver* orc_create_gauss(int ex, int ey, int ez, const double* lo, const double* hi, int deform, double amp,
                             int N, double gamma, double Pr, double Ma, double Re, int surf_flux) {
  return create(ex, ey, ez, lo, hi, deform, amp, N, NULL, gamma, Pr, Ma, Re, ORC_VOL_CENTRAL, surf_flux, 1);
}

void orc_destroy(orc_solver* s) {
  if (!s) return;
  free(s->N); free(s->off); free(s->nbr);
  free(s->X); free(s->Ja); free(s->J);
  free(s->U); free(s->dU); free(s->G); free(s->R);
  free(s->Gw); free(s->Fa);
  free(s);
}

long orc_num_nodes(const orc_solver* s) { return s ? s->ntot : -1; }
int orc_num_elements(const orc_solver* s) { return s ? s->E : -1; }
int orc_elem_info(const orc_solver* s, int e, int* n3, long* off) {
  if (!s || e < 0 || e >= s->E) return -1;
  for (int d = 0; d < 3; d++) n3[d] = s->N[e][d];
  *off = s->off[e];
  return 0;
}
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_get_coords(const orc_solver* s, double* X) {
  for (long i = 0; i < 3 * s->ntot; i++) X[i] = (double)s->X[i];
  return 0;
}
int orc_get_metrics(const orc_solver* s, double* Ja, double* J) {
  if (Ja) for (long i = 0; i < 9 * s->ntot; i++) Ja[i] = (double)s->Ja[i];
  if (J) for (long i = 0; i < s->ntot; i++) J[i] = (double)s->J[i];
  return 0;
}

/* ------------------------------------------------------------------------------------------
 * 5. Physics (section "Compressible Navier-Stokes").
 * ---------------------------------------------------------------------------------------- */
typedef struct { real rho, v[3], p, E; } prim_t;

static inline prim_t prim(const real u[5], real gamma) {
  prim_t w;
  w.rho = u[0];
  for (int c = 0; c < 3; c++) w.v[c] = u[1 + c] / u[0];
  w.E = u[4];
  w.p = (gamma - 1) * (u[4] - (real)0.5 * u[0] * (w.v[0] * w.v[0] + w.v[1] * w.v[1] + w.v[2] * w.v[2]));
  return w;
}

/* Euler flux along the (not necessarily unit) vector n: F_e . n */
static void euler_flux(const real u[5], const real n[3], real gamma, real F[5]) {
  prim_t w = prim(u, gamma);
  real vn = w.v[0] * n[0] + w.v[1] * n[1] + w.v[2] * n[2];
  F[0] = w.rho * vn;
  for (int c = 0; c < 3; c++) F[1 + c] = u[1 + c] * vn + w.p * n[c];
  F[4] = (w.E + w.p) * vn;
}

/* logarithmic mean (a-b)/(ln a - ln b), series in u=((a-b)/(a+b))^2 near a=b */
static real logmean(real a, real b) {
  real f = (a - b) / (a + b);
  real u = f * f;
  if (u < (real)1e-4) {
    real s = 1 + u * ((real)1 / 3 + u * ((real)1 / 5 + u * ((real)1 / 7 + u * ((real)1 / 9 +
             u * ((real)1 / 11 + u * ((real)1 / 13))))));
    return (a + b) / (2 * s);
  }
  return (a - b) / (RLOG(a) - RLOG(b));
}

/* Chandrashekar's kinetic-energy-preserving, entropy-conserving two-point flux along n */
static void two_point_ec(const real uL[5], const real uR[5], const real n[3], real gamma, real F[5]) {
  prim_t L = prim(uL, gamma), R = prim(uR, gamma);
  real bL = L.rho / (2 * L.p), bR = R.rho / (2 * R.p);
  real rho_ln = logmean(L.rho, R.rho), b_ln = logmean(bL, bR);
  real rho_a = (L.rho + R.rho) / 2, b_a = (bL + bR) / 2;
  real v_a[3], v2_a = 0;
  for (int c = 0; c < 3; c++) {
    v_a[c] = (L.v[c] + R.v[c]) / 2;
    v2_a += (L.v[c] * L.v[c] + R.v[c] * R.v[c]) / 2;
  }
  real p_hat = rho_a / (2 * b_a);
  real vn = v_a[0] * n[0] + v_a[1] * n[1] + v_a[2] * n[2];
  F[0] = rho_ln * vn;
  for (int c = 0; c < 3; c++) F[1 + c] = F[0] * v_a[c] + p_hat * n[c];
  F[4] = F[0] * (1 / (2 * (gamma - 1) * b_ln) - v2_a / 2) + v_a[0] * F[1] + v_a[1] * F[2] + v_a[2] * F[3];
}

/* Ismail and Roe's entropy-conserving two-point flux along n (one of the entropy-conserving
 * split forms of section "Energy/Entropy stable versions"), written with the parameter vector
 * z = sqrt(rho/p) (1, v1, v2, v3, p): with {.} the arithmetic and (.)^ln the logarithmic mean,
 *   rho^ = {z1} (z5)^ln,  v^ = {z1 v}/{z1},  p1^ = {z5}/{z1},
 *   p2^ = (gamma+1)/(2 gamma) (z5)^ln/(z1)^ln + (gamma-1)/(2 gamma) {z5}/{z1},
 *   H^ = gamma p2^/((gamma-1) rho^) + |v^|^2/2;
 *   F = (rho^ v^.n,  rho^ v^ (v^.n) + p1^ n,  rho^ H^ (v^.n)). */
static void two_point_ir(const real uL[5], const real uR[5], const real n[3], real gamma, real F[5]) {
  prim_t L = prim(uL, gamma), R = prim(uR, gamma);
  real z1L = RSQRT(L.rho / L.p), z1R = RSQRT(R.rho / R.p);
  real z5L = RSQRT(L.rho * L.p), z5R = RSQRT(R.rho * R.p);
  real z1a = (z1L + z1R) / 2, z5a = (z5L + z5R) / 2;
  real z1ln = logmean(z1L, z1R), z5ln = logmean(z5L, z5R);
  real rho = z1a * z5ln;
  real v[3];
  for (int c = 0; c < 3; c++) v[c] = (z1L * L.v[c] + z1R * R.v[c]) / 2 / z1a;
  real p1 = z5a / z1a;
  real p2 = (gamma + 1) / (2 * gamma) * z5ln / z1ln + (gamma - 1) / (2 * gamma) * z5a / z1a;
  real H = gamma * p2 / ((gamma - 1) * rho) + (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / 2;
  real vn = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
  F[0] = rho * vn;
  for (int c = 0; c < 3; c++) F[1 + c] = F[0] * v[c] + p1 * n[c];
  F[4] = F[0] * H;
}

static void two_point_central(const real uL[5], const real uR[5], const real n[3], real gamma, real F[5]) {
  real FL[5], FR[5];
  euler_flux(uL, n, gamma, FL);
  euler_flux(uR, n, gamma, FR);
  for (int v = 0; v < 5; v++) F[v] = (FL[v] + FR[v]) / 2;
}

/* The kinetic-energy-preserving split forms of section "Energy/Entropy stable versions" (list
 * of split forms), written as two-point fluxes along n from products of arithmetic means
 * {a} = (a_L + a_R)/2; vn = v.n, e = rho*E/rho (total energy per unit mass), H = e + p/rho.
 *   Kennedy-Gruber: F_rho = {rho}{vn},  F_m = {rho}{vn}{v} + {p} n,  F_E = {rho}{vn}{e} + {p}{vn}
 *   Pirozzoli:      F_rho = {rho}{vn},  F_m = {rho}{vn}{v} + {p} n,  F_E = {rho}{vn}{H}
 *   Ducros:         F_rho = {rho}{vn},  F_m = {rho v}{vn} + {p} n,   F_E = {rho e + p}{vn}
 *   Morinishi:      F_rho = {rho vn},   F_m = {rho vn}{v} + {p} n,
 *                   F_E = gamma/(gamma-1) {p vn} + {rho vn}({v}.{v}) - {rho vn |v|^2}/2 */
static void two_point_kep(int kind, const real uL[5], const real uR[5], const real n[3], real gamma, real F[5]) {
  prim_t L = prim(uL, gamma), R = prim(uR, gamma);
  real vnL = L.v[0] * n[0] + L.v[1] * n[1] + L.v[2] * n[2];
  real vnR = R.v[0] * n[0] + R.v[1] * n[1] + R.v[2] * n[2];
  real rho_a = (L.rho + R.rho) / 2, vn_a = (vnL + vnR) / 2, p_a = (L.p + R.p) / 2;
  real v_a[3];
  for (int c = 0; c < 3; c++) v_a[c] = (L.v[c] + R.v[c]) / 2;
  switch (kind) {
    case ORC_VOL_KG:
    case ORC_VOL_PIROZZOLI: {
      F[0] = rho_a * vn_a;
      for (int c = 0; c < 3; c++) F[1 + c] = rho_a * vn_a * v_a[c] + p_a * n[c];
      if (kind == ORC_VOL_KG) {
        real e_a = (L.E / L.rho + R.E / R.rho) / 2;
        F[4] = rho_a * vn_a * e_a + p_a * vn_a;
      } else {
        real H_a = ((L.E + L.p) / L.rho + (R.E + R.p) / R.rho) / 2;
        F[4] = rho_a * vn_a * H_a;
      }
      break;
    }
    case ORC_VOL_DUCROS: {
      F[0] = rho_a * vn_a;
      for (int c = 0; c < 3; c++) F[1 + c] = (uL[1 + c] + uR[1 + c]) / 2 * vn_a + p_a * n[c];
      F[4] = ((L.E + L.p) + (R.E + R.p)) / 2 * vn_a;
      break;
    }
    default: { /* Morinishi */
      real m_a = (L.rho * vnL + R.rho * vnR) / 2;
      real v2L = L.v[0] * L.v[0] + L.v[1] * L.v[1] + L.v[2] * L.v[2];
      real v2R = R.v[0] * R.v[0] + R.v[1] * R.v[1] + R.v[2] * R.v[2];
      F[0] = m_a;
      for (int c = 0; c < 3; c++) F[1 + c] = m_a * v_a[c] + p_a * n[c];
      F[4] = gamma / (gamma - 1) * (L.p * vnL + R.p * vnR) / 2 +
             m_a * (v_a[0] * v_a[0] + v_a[1] * v_a[1] + v_a[2] * v_a[2]) -
             (L.rho * vnL * v2L + R.rho * vnR * v2R) / 4;
      break;
    }
  }
}

/* Roe's wave decomposition along the unit normal n: sum_k f(lambda_k) alpha_k r_k with
 * f = |.| (absval=1) or the identity (absval=0, then the sum equals F(uR)-F(uL)).  The wave
 * strengths come from the jumps (Roe and Pike's evaluation, no Roe matrix is formed).  zv
 * scales the velocity jump inside the strengths: 1 for Roe's flux, the Mach-number factor of
 * the low-dissipation variant below. */
static void roe_waves_z(const real uL[5], const real uR[5], const real n[3], real gamma, int absval, real zv,
                        real W[5]) {
  prim_t L = prim(uL, gamma), R = prim(uR, gamma);
  real sL = RSQRT(L.rho), sR = RSQRT(R.rho);
  real HL = (L.E + L.p) / L.rho, HR = (R.E + R.p) / R.rho;
  real v[3], q2 = 0;
  for (int c = 0; c < 3; c++) { v[c] = (sL * L.v[c] + sR * R.v[c]) / (sL + sR); q2 += v[c] * v[c]; }
  real H = (sL * HL + sR * HR) / (sL + sR);
  real rho = sL * sR;
  real c2 = (gamma - 1) * (H - q2 / 2), c = RSQRT(c2);
  real vn = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
  real drho = R.rho - L.rho, dp = R.p - L.p, dv[3];
  for (int k = 0; k < 3; k++) dv[k] = zv * (R.v[k] - L.v[k]);
  real dvn = dv[0] * n[0] + dv[1] * n[1] + dv[2] * n[2];
  real a1 = (dp - rho * c * dvn) / (2 * c2);
  real a2 = drho - dp / c2;
  real a3 = (dp + rho * c * dvn) / (2 * c2);
  real l1 = vn - c, l2 = vn, l3 = vn + c;
  if (absval) { l1 = RFABS(l1); l2 = RFABS(l2); l3 = RFABS(l3); }
  real dvt[3];
  for (int k = 0; k < 3; k++) dvt[k] = dv[k] - dvn * n[k];
  real vdvt = v[0] * dvt[0] + v[1] * dvt[1] + v[2] * dvt[2];
  W[0] = l1 * a1 + l2 * a2 + l3 * a3;
  for (int k = 0; k < 3; k++)
    W[1 + k] = l1 * a1 * (v[k] - c * n[k]) + l2 * (a2 * v[k] + rho * dvt[k]) + l3 * a3 * (v[k] + c * n[k]);
  W[4] = l1 * a1 * (H - vn * c) + l2 * (a2 * q2 / 2 + rho * vdvt) + l3 * a3 * (H + vn * c);
}

static void roe_waves(const real uL[5], const real uR[5], const real n[3], real gamma, int absval, real W[5]) {
  roe_waves_z(uL, uR, n, gamma, absval, 1, W);
}

/* entropy variables w = dS/du of S = -rho s/(gamma-1), s = ln p - gamma ln rho */
static void entropy_vars(const real u[5], real gamma, real w[5]) {
  prim_t q = prim(u, gamma);
  real sp = RLOG(q.p) - gamma * RLOG(q.rho);
  real b = q.rho / (2 * q.p);
  real v2 = q.v[0] * q.v[0] + q.v[1] * q.v[1] + q.v[2] * q.v[2];
  w[0] = (gamma - sp) / (gamma - 1) - b * v2;
  for (int c = 0; c < 3; c++) w[1 + c] = 2 * b * q.v[c];
  w[4] = -2 * b;
}

/* Matrix dissipation for the entropy-stable flux along the unit normal n:
 * D = R |Lambda| T R^T (w_R - w_L), with the eigenvectors R of the Euler flux Jacobian along n
 * and Barth's scaling T = diag(rho/(2 gamma), rho (gamma-1)/gamma, p, p, rho/(2 gamma)), for
 * which R T R^T = du/dw.  Reading: R, Lambda, T are taken at the averaged state
 * rho^ = (rho)^ln, v^ = {v}, p^ = {rho}/(2{beta}) (Chandrashekar's averages), with
 * c^2 = gamma p^/rho^ and H^ = c^2/(gamma-1) + |v^|^2/2.  The two shear waves are summed with the
 * tangential projector I - n n^T, so no tangent basis is needed.  D . (w_R - w_L) >= 0.
 * The structure and scaling are pinned; the choice of the averaged state among consistent
 * averages is parity unpinned (no pin distinguishes them). */
static void matrix_dissipation(const real uL[5], const real uR[5], const real n[3], real gamma, real D[5]) {
  prim_t L = prim(uL, gamma), R = prim(uR, gamma);
  real bL = L.rho / (2 * L.p), bR = R.rho / (2 * R.p);
  real rho = logmean(L.rho, R.rho);
  real p = (L.rho + R.rho) / (2 * (bL + bR));
  real v[3], q2 = 0;
  for (int c = 0; c < 3; c++) { v[c] = (L.v[c] + R.v[c]) / 2; q2 += v[c] * v[c]; }
  real c2 = gamma * p / rho, c = RSQRT(c2);
  real H = c2 / (gamma - 1) + q2 / 2;
  real vn = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
  real wL[5], wR[5], dw[5];
  entropy_vars(uL, gamma, wL);
  entropy_vars(uR, gamma, wR);
  for (int k = 0; k < 5; k++) dw[k] = wR[k] - wL[k];
  real r1[5] = {1, v[0] - c * n[0], v[1] - c * n[1], v[2] - c * n[2], H - c * vn};
  real r2[5] = {1, v[0], v[1], v[2], q2 / 2};
  real r5[5] = {1, v[0] + c * n[0], v[1] + c * n[1], v[2] + c * n[2], H + c * vn};
  real s1 = 0, s2 = 0, s5 = 0;
  for (int k = 0; k < 5; k++) { s1 += r1[k] * dw[k]; s2 += r2[k] * dw[k]; s5 += r5[k] * dw[k]; }
  s1 *= RFABS(vn - c) * rho / (2 * gamma);
  s2 *= RFABS(vn) * rho * (gamma - 1) / gamma;
  s5 *= RFABS(vn + c) * rho / (2 * gamma);
  real q[3], qn = 0;
  for (int k = 0; k < 3; k++) { q[k] = dw[1 + k] + v[k] * dw[4]; qn += q[k] * n[k]; }
  real qt[3], vqt = 0;
  for (int k = 0; k < 3; k++) { qt[k] = q[k] - qn * n[k]; vqt += v[k] * qt[k]; }
  real sh = p * RFABS(vn);
  for (int k = 0; k < 5; k++) D[k] = s1 * r1[k] + s2 * r2[k] + s5 * r5[k];
  for (int k = 0; k < 3; k++) D[1 + k] += sh * qt[k];
  D[4] += sh * vqt;
}

/* numerical flux through a face with scaled normal S (S = |S| n_hat) */
static void riemann(int kind, const real uL[5], const real uR[5], const real S[3], real gamma, real F[5]) {
  real a = RSQRT(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
  real n[3] = {S[0] / a, S[1] / a, S[2] / a};
  real FL[5], FR[5];
  switch (kind) {
    case ORC_SURF_ROE: {
      real W[5];
      euler_flux(uL, n, gamma, FL);
      euler_flux(uR, n, gamma, FR);
      roe_waves(uL, uR, n, gamma, 1, W);
      for (int v = 0; v < 5; v++) F[v] = a * ((FL[v] + FR[v]) / 2 - W[v] / 2);
      break;
    }
    case ORC_SURF_LLF: {
      prim_t L = prim(uL, gamma), R = prim(uR, gamma);
      real vnL = L.v[0] * n[0] + L.v[1] * n[1] + L.v[2] * n[2];
      real vnR = R.v[0] * n[0] + R.v[1] * n[1] + R.v[2] * n[2];
      real lL = RFABS(vnL) + RSQRT(gamma * L.p / L.rho);
      real lR = RFABS(vnR) + RSQRT(gamma * R.p / R.rho);
      real lam = lL > lR ? lL : lR;
      euler_flux(uL, n, gamma, FL);
      euler_flux(uR, n, gamma, FR);
      for (int v = 0; v < 5; v++) F[v] = a * ((FL[v] + FR[v]) / 2 - lam * (uR[v] - uL[v]) / 2);
      break;
    }
    case ORC_SURF_EC: two_point_ec(uL, uR, S, gamma, F); break;
    case ORC_SURF_IR: two_point_ir(uL, uR, S, gamma, F); break;
    case ORC_SURF_ES: {
      /* entropy-stable: Chandrashekar's flux minus local Lax-Friedrichs dissipation; the
       * dissipation (U_R - U_L) has a non-negative inner product with the jump of the entropy
       * variables (S is convex), so every face produces entropy of the right sign */
      prim_t L = prim(uL, gamma), R = prim(uR, gamma);
      real vnL = L.v[0] * n[0] + L.v[1] * n[1] + L.v[2] * n[2];
      real vnR = R.v[0] * n[0] + R.v[1] * n[1] + R.v[2] * n[2];
      real lL = RFABS(vnL) + RSQRT(gamma * L.p / L.rho);
      real lR = RFABS(vnR) + RSQRT(gamma * R.p / R.rho);
      real lam = lL > lR ? lL : lR;
      two_point_ec(uL, uR, S, gamma, F);
      for (int v = 0; v < 5; v++) F[v] -= a * lam * (uR[v] - uL[v]) / 2;
      break;
    }
    case ORC_SURF_ES_MATRIX: {
      /* entropy-stable: Chandrashekar's flux minus the matrix dissipation above */
      real D[5];
      two_point_ec(uL, uR, S, gamma, F);
      matrix_dissipation(uL, uR, n, gamma, D);
      for (int v = 0; v < 5; v++) F[v] -= a * D[v] / 2;
      break;
    }
    case ORC_SURF_LOW_DISS_ROE: {
      /* low-dissipation Roe: Roe's flux with the velocity jump in the wave strengths scaled by
       * z = min(1, max(M_L, M_R)), M = |v|/c the local Mach numbers (reading: the
       * low-Mach-number correction of Oswald et al., which leaves density and pressure jumps
       * and supersonic faces as in Roe's flux) */
      prim_t L = prim(uL, gamma), R = prim(uR, gamma);
      real ML = RSQRT((L.v[0] * L.v[0] + L.v[1] * L.v[1] + L.v[2] * L.v[2]) * L.rho / (gamma * L.p));
      real MR = RSQRT((R.v[0] * R.v[0] + R.v[1] * R.v[1] + R.v[2] * R.v[2]) * R.rho / (gamma * R.p));
      real z = ML > MR ? ML : MR;
      if (z > 1) z = 1;
      real W[5];
      euler_flux(uL, n, gamma, FL);
      euler_flux(uR, n, gamma, FR);
      roe_waves_z(uL, uR, n, gamma, 1, z, W);
      for (int v = 0; v < 5; v++) F[v] = a * ((FL[v] + FR[v]) / 2 - W[v] / 2);
      break;
    }
    default: two_point_central(uL, uR, S, gamma, F); break;
  }
}

/* Lax-Friedrichs with a given wave speed lam: {F} . S - lam |S| (U_R - U_L) / 2 */
static void lax_friedrichs(const real uL[5], const real uR[5], const real S[3], real gamma, real lam, real F[5]) {
  real a = RSQRT(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
  real FL[5], FR[5];
  euler_flux(uL, S, gamma, FL);
  euler_flux(uR, S, gamma, FR);
  for (int v = 0; v < 5; v++) F[v] = (FL[v] + FR[v]) / 2 - a * lam * (uR[v] - uL[v]) / 2;
}

/* the solver's surface flux: Lax-Friedrichs (global) takes the state's largest wave speed,
 * every other flux only the two traces */
static void surface_flux(const orc_solver* s, const real uL[5], const real uR[5], const real S[3], real F[5]) {
  if (s->surf == ORC_SURF_LF_GLOBAL) lax_friedrichs(uL, uR, S, s->gamma, s->lam_g, F);
  else riemann(s->surf, uL, uR, S, s->gamma, F);
}

static void volume_flux(const orc_solver* s, const real uL[5], const real uR[5], const real n[3], real F[5]) {
  if (s->vol == ORC_VOL_EC) two_point_ec(uL, uR, n, s->gamma, F);
  else if (s->vol == ORC_VOL_IR) two_point_ir(uL, uR, n, s->gamma, F);
  else if (s->vol == ORC_VOL_CENTRAL) two_point_central(uL, uR, n, s->gamma, F);
  else two_point_kep(s->vol, uL, uR, n, s->gamma, F);
}

/* viscous flux (eq. viscousfluxes) from the velocity v and the gradients of (v1,v2,v3,T);
 * grad[3c+n] = d g_c / d x_n.  Fv[5n+v]: component v of the flux in physical direction n. */
static void viscous_flux_v(const real vel[3], const real grad[12], real mu, real kappa, real Fv[15]) {
  real divv = grad[0] + grad[4] + grad[8];
  real tau[3][3];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++)
      tau[a][b] = mu * (grad[3 * a + b] + grad[3 * b + a]) - (a == b ? (real)2 / 3 * mu * divv : 0);
  for (int n = 0; n < 3; n++) {
    Fv[5 * n + 0] = 0;
    for (int a = 0; a < 3; a++) Fv[5 * n + 1 + a] = tau[a][n];
    Fv[5 * n + 4] = vel[0] * tau[0][n] + vel[1] * tau[1][n] + vel[2] * tau[2][n] + kappa * grad[9 + n];
  }
}

static void viscous_flux(const real u[5], const real grad[12], real gamma, real mu, real kappa, real Fv[15]) {
  prim_t w = prim(u, gamma);
  viscous_flux_v(w.v, grad, mu, kappa, Fv);
}

/* ------------------------------------------------------------------------------------------
 * 6. Faces.  The face between L (its xi_d=+1 side) and R = nbr(L, +d) (its xi_d=-1 side) is
 *    oriented along +xi_d and uses L's metric Ja^d as the scaled normal S.  Both elements
 *    evaluate it with the same arguments, so the flux is single-valued.  Conforming faces:
 *    pointwise.  Non-conforming faces: mortar of orders (max, max) in the two tangential
 *    directions; traces and L's normal interpolated to it, flux there, projected back to
 *    each side's grid.
 * ---------------------------------------------------------------------------------------- */
static void face_dirs(int d, int* ta, int* tb) {
  *ta = d == 0 ? 1 : 0;
  *tb = d == 2 ? 1 : 2;
}

/* Flux on the face (L, +d), on the whole node grid of one side (want_R = 0: L's grid,
 * 1: R's grid).  F[v*na*nb + p + na*r], (p, r) the indices along the two tangential
 * directions (ta < tb). */
static void face_flux_side(const orc_solver* s, const real* U, int L, int d, int want_R, real* F) {
  int R = s->nbr[6 * L + 2 * d + 1];
  int ta, tb;
  face_dirs(d, &ta, &tb);
  const int* NL = s->N[L];
  const int* NR = s->N[R];
  const int* Ns = want_R ? NR : NL;
  int na = Ns[ta] + 1, nb = Ns[tb] + 1, nf = na * nb;
  if (NL[ta] == NR[ta] && NL[tb] == NR[tb]) {
    for (int r = 0; r < nb; r++)
      for (int p = 0; p < na; p++) {
        int iL[3], iR[3];
        iL[d] = NL[d]; iL[ta] = p; iL[tb] = r;
        iR[d] = 0; iR[ta] = p; iR[tb] = r;
        real uL[5], uR[5], S[3], Fp[5];
        load5(s, U, L, node_of(s, L, iL), uL);
        load5(s, U, R, node_of(s, R, iR), uR);
        load_ja(s, L, node_of(s, L, iL), d, S);
        surface_flux(s, uL, uR, S, Fp);
        for (int v = 0; v < 5; v++) F[v * nf + p + na * r] = Fp[v];
      }
    return;
  }
  int Ma = NL[ta] > NR[ta] ? NL[ta] : NR[ta];
  int Mb = NL[tb] > NR[tb] ? NL[tb] : NR[tb];
  int nma = Ma + 1, nmb = Mb + 1;
  real* Fm = (real*)malloc(sizeof(real) * 5 * nma * nmb);
  for (int rm = 0; rm < nmb; rm++)
    for (int pm = 0; pm < nma; pm++) {
      real uL[5] = {0, 0, 0, 0, 0}, uR[5] = {0, 0, 0, 0, 0}, S[3] = {0, 0, 0};
      for (int r2 = 0; r2 <= NL[tb]; r2++)
        for (int p2 = 0; p2 <= NL[ta]; p2++) {
          int ii[3];
          ii[d] = NL[d]; ii[ta] = p2; ii[tb] = r2;
          real w = INTERP[NL[ta]][Ma][pm][p2] * INTERP[NL[tb]][Mb][rm][r2], u[5], n[3];
          long q = node_of(s, L, ii);
          load5(s, U, L, q, u);
          load_ja(s, L, q, d, n);
          for (int v = 0; v < 5; v++) uL[v] += w * u[v];
          for (int c = 0; c < 3; c++) S[c] += w * n[c];
        }
      for (int r2 = 0; r2 <= NR[tb]; r2++)
        for (int p2 = 0; p2 <= NR[ta]; p2++) {
          int ii[3];
          ii[d] = 0; ii[ta] = p2; ii[tb] = r2;
          real w = INTERP[NR[ta]][Ma][pm][p2] * INTERP[NR[tb]][Mb][rm][r2], u[5];
          load5(s, U, R, node_of(s, R, ii), u);
          for (int v = 0; v < 5; v++) uR[v] += w * u[v];
        }
      real Fp[5];
      surface_flux(s, uL, uR, S, Fp);
      for (int v = 0; v < 5; v++) Fm[v * nma * nmb + pm + nma * rm] = Fp[v];
    }
  for (int r = 0; r < nb; r++)
    for (int p = 0; p < na; p++)
      for (int v = 0; v < 5; v++) {
        real acc = 0;
        for (int rm = 0; rm < nmb; rm++)
          for (int pm = 0; pm < nma; pm++)
            acc += PROJ[Ns[ta]][Ma][p][pm] * PROJ[Ns[tb]][Mb][r][rm] * Fm[v * nma * nmb + pm + nma * rm];
        F[v * nf + p + na * r] = acc;
      }
  free(Fm);
}

/* ------------------------------------------------------------------------------------------
 * 7. BR1 gradients of g = (v1, v2, v3, T), T = p/rho:
 *    J grad g = sum_d Ja^d [ D_d g + (1/w_N)(g*-g) at xi_d=+1 - (1/w_0)(g*-g) at xi_d=-1 ],
 *    g* = average of the two traces.
 * ---------------------------------------------------------------------------------------- */
static inline void gvars(const real u[5], real gamma, real g[4]) {
  prim_t w = prim(u, gamma);
  g[0] = w.v[0]; g[1] = w.v[1]; g[2] = w.v[2];
  g[3] = w.p / w.rho;
}

/* BR1 gradient of nv nodal variables vars(u) (nv <= 5): Gout[off*3nv + (3c+x)*nn + node] */
typedef void (*vars_fn)(const real u[5], real gamma, real* g);

static void br1_gradient(orc_solver* s, const real* U, int nv, vars_fn vars, real* Gout) {
#pragma omp parallel for schedule(static)
  for (int e = 0; e < s->E; e++) {
    const int* N = s->N[e];
    int nn = nn_of(s, e);
    real* G = Gout + s->off[e] * 3 * nv;
    for (int k = 0; k <= N[2]; k++)
      for (int j = 0; j <= N[1]; j++)
        for (int i = 0; i <= N[0]; i++) {
          int ii[3] = {i, j, k};
          long q = node_of(s, e, ii);
          real u[5], g[5];
          load5(s, U, e, q, u);
          vars(u, s->gamma, g);
          real acc[15] = {0};
          for (int d = 0; d < 3; d++) {
            real a[5] = {0, 0, 0, 0, 0};
            int jj[3] = {i, j, k};
            for (int m = 0; m <= N[d]; m++) {
              jj[d] = m;
              real um[5], gm[5];
              load5(s, U, e, node_of(s, e, jj), um);
              vars(um, s->gamma, gm);
              for (int c = 0; c < nv; c++) a[c] += GLL[N[d]].D[ii[d]][m] * gm[c];
            }
            for (int side = 0; side < 2; side++) {
              int at = side ? N[d] : 0;
              if (ii[d] != at) continue;
              int ne = s->nbr[6 * e + 2 * d + side];
              int kk[3] = {i, j, k};
              kk[d] = side ? 0 : s->N[ne][d];
              real un[5], gn[5];
              load5(s, U, ne, node_of(s, ne, kk), un);
              vars(un, s->gamma, gn);
              real wgt = 1 / GLL[N[d]].w[at];
              for (int c = 0; c < nv; c++) {
                real jump = (g[c] + gn[c]) / 2 - g[c];
                a[c] += side ? wgt * jump : -wgt * jump;
              }
            }
            real n[3];
            load_ja(s, e, q, d, n);
            for (int c = 0; c < nv; c++)
              for (int x = 0; x < 3; x++) acc[3 * c + x] += n[x] * a[c];
          }
          real Jq = s->J[s->off[e] + q];
          for (int t = 0; t < 3 * nv; t++) G[(long)t * nn + q] = acc[t] / Jq;
        }
  }
}

static void compute_gradients(orc_solver* s, const real* U, real* Gout) { br1_gradient(s, U, 4, gvars, Gout); }

/* contravariant viscous flux of node q of element e along xi_d */
static void contra_visc(const orc_solver* s, const real* U, const real* Gall, int e, long q, int d, const real* Sopt,
                        real Fd[5]) {
  int nn = nn_of(s, e);
  real u[5], gr[12], Fv[15], n[3];
  load5(s, U, e, q, u);
  for (int t = 0; t < 12; t++) gr[t] = Gall[s->off[e] * 12 + (long)t * nn + q];
  viscous_flux(u, gr, s->gamma, s->mu, s->kappa, Fv);
  if (Sopt) { n[0] = Sopt[0]; n[1] = Sopt[1]; n[2] = Sopt[2]; }
  else load_ja(s, e, q, d, n);
  for (int v = 0; v < 5; v++) Fd[v] = n[0] * Fv[v] + n[1] * Fv[5 + v] + n[2] * Fv[10 + v];
}

/* Gradient of g at node ii of element e from the element's own values (the broken gradient
 * (1/J) sum_d Ja^d D_d g, no lifting); with lift_d >= 0 plus eta times the lift of the jump on
 * the one face (lift_d, lift_side) alone -- BR2's face-local lifting. */
static void broken_gradient(const orc_solver* s, const real* U, int e, const int ii[3], int lift_d, int lift_side,
                            real eta, real gr[12]) {
  const int* N = s->N[e];
  long q = node_of(s, e, ii);
  real u[5], g[4];
  load5(s, U, e, q, u);
  gvars(u, s->gamma, g);
  for (int t = 0; t < 12; t++) gr[t] = 0;
  for (int d = 0; d < 3; d++) {
    real a[4] = {0, 0, 0, 0};
    int jj[3] = {ii[0], ii[1], ii[2]};
    for (int m = 0; m <= N[d]; m++) {
      jj[d] = m;
      real um[5], gm[4];
      load5(s, U, e, node_of(s, e, jj), um);
      gvars(um, s->gamma, gm);
      for (int c = 0; c < 4; c++) a[c] += GLL[N[d]].D[ii[d]][m] * gm[c];
    }
    if (d == lift_d) {
      int at = lift_side ? N[d] : 0;
      int ne = s->nbr[6 * e + 2 * d + lift_side];
      int kk[3] = {ii[0], ii[1], ii[2]};
      kk[d] = lift_side ? 0 : s->N[ne][d];
      real un[5], gn[4];
      load5(s, U, ne, node_of(s, ne, kk), un);
      gvars(un, s->gamma, gn);
      real wgt = eta / GLL[N[d]].w[at];
      for (int c = 0; c < 4; c++) {
        real jump = (g[c] + gn[c]) / 2 - g[c];
        a[c] += lift_side ? wgt * jump : -wgt * jump;
      }
    }
    real n[3];
    load_ja(s, e, q, d, n);
    for (int c = 0; c < 4; c++)
      for (int x = 0; x < 3; x++) gr[3 * c + x] += n[x] * a[c];
  }
  real Jq = s->J[s->off[e] + q];
  for (int t = 0; t < 12; t++) gr[t] /= Jq;
}

/* Face viscous flux along the scaled normal S between the node q of element e (face (d, side))
 * and the matching node qo of its neighbour oth, from the face gradients of the chosen scheme
 * (box of viscous fluxes in section "Spatial discretisation"):
 *   BR1: average of the two sides' fluxes with their fully lifted gradients;
 *   BR2: the same with each side's broken gradient plus eta times the lift of this face's jump;
 *   IP (symmetric interior penalty): the same with the broken gradients, plus the penalty
 *        sigma F_v(v_mean, [g] n^) . S, [g] = g(+ side) - g(- side), n^ = S/|S|,
 *        sigma = eta (N_d + 1)^2 / h, h = 2 min(J_e, J_oth)/|S| (the element size across the
 *        face, exact on affine elements).
 * The volume terms of all three use the fully lifted gradient (for the interior penalty this
 * supplies its symmetrising term). */
static void face_viscous_flux(const orc_solver* s, const real* U, const real* Gall, int e, const int ii[3], int d,
                              int side, int oth, const int kk[3], const real S[3], real Fst[5]) {
  long q = node_of(s, e, ii), qo = node_of(s, oth, kk);
  real Fa[5], Fb[5];
  if (s->visc_flux == ORC_VISC_BR1) {
    contra_visc(s, U, Gall, e, q, d, S, Fa);
    contra_visc(s, U, Gall, oth, qo, d, S, Fb);
  } else {
    const int br2 = s->visc_flux == ORC_VISC_BR2;
    real ga[12], gb[12], ua[5], ub[5], Fv[15];
    broken_gradient(s, U, e, ii, br2 ? d : -1, side, s->visc_eta, ga);
    broken_gradient(s, U, oth, kk, br2 ? d : -1, 1 - side, s->visc_eta, gb);
    load5(s, U, e, q, ua);
    load5(s, U, oth, qo, ub);
    viscous_flux(ua, ga, s->gamma, s->mu, s->kappa, Fv);
    for (int v = 0; v < 5; v++) Fa[v] = S[0] * Fv[v] + S[1] * Fv[5 + v] + S[2] * Fv[10 + v];
    viscous_flux(ub, gb, s->gamma, s->mu, s->kappa, Fv);
    for (int v = 0; v < 5; v++) Fb[v] = S[0] * Fv[v] + S[1] * Fv[5 + v] + S[2] * Fv[10 + v];
  }
  for (int v = 0; v < 5; v++) Fst[v] = (Fa[v] + Fb[v]) / 2;
  if (s->visc_flux == ORC_VISC_IP) {
    real ua[5], ub[5], ga[4], gb[4];
    load5(s, U, e, q, ua);
    load5(s, U, oth, qo, ub);
    gvars(ua, s->gamma, ga);
    gvars(ub, s->gamma, gb);
    /* the + side of the face is the element across +xi_d from the other */
    const real* gp = side ? gb : ga;
    const real* gm = side ? ga : gb;
    real area = RSQRT(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
    real Je = s->J[s->off[e] + q], Jo = s->J[s->off[oth] + qo];
    real h = 2 * (Je < Jo ? Je : Jo) / area;
    real n1 = s->N[e][d] + 1;
    real sigma = s->visc_eta * n1 * n1 / h;
    real vm[3], gr[12], Fv[15];
    for (int c = 0; c < 3; c++) vm[c] = (ga[c] + gb[c]) / 2;
    for (int c = 0; c < 4; c++)
      for (int x = 0; x < 3; x++) gr[3 * c + x] = sigma * (gp[c] - gm[c]) * S[x] / area;
    viscous_flux_v(vm, gr, s->mu, s->kappa, Fv);
    for (int v = 0; v < 5; v++) Fst[v] += S[0] * Fv[v] + S[1] * Fv[5 + v] + S[2] * Fv[10 + v];
  }
}

/* ------------------------------------------------------------------------------------------
 * 8. Residual of one element:
 *    J dU/dt = -[ sum_d sum_m 2 D_im F#(U_i,U_m; avg Ja^d)
 *                 + (1/w_N)(F*-F~(U)) at xi_d=+1 - (1/w_0)(F*-F~(U)) at xi_d=-1 ]
 *              + sum_d D_d F~_v^d + (1/w_N)(F~_v*-F~_v) at +1 - (1/w_0)(F~_v*-F~_v) at -1
 * ---------------------------------------------------------------------------------------- */
static void element_residual(const orc_solver* s, const real* U, const real* Gall, int e, real* R) {
  const int* N = s->N[e];
  int nn = nn_of(s, e);
  /* numerical flux on the six faces, each on this element's face grid */
  real* Ff[6];
  for (int d = 0; d < 3; d++) {
    int ta, tb;
    face_dirs(d, &ta, &tb);
    int nf = (N[ta] + 1) * (N[tb] + 1);
    for (int side = 0; side < 2; side++) {
      Ff[2 * d + side] = (real*)malloc(sizeof(real) * 5 * nf);
      int L = side ? e : s->nbr[6 * e + 2 * d];
      face_flux_side(s, U, L, d, side ? 0 : 1, Ff[2 * d + side]);
    }
  }
  for (int k = 0; k <= N[2]; k++)
    for (int j = 0; j <= N[1]; j++)
      for (int i = 0; i <= N[0]; i++) {
        int ii[3] = {i, j, k};
        long q = node_of(s, e, ii);
        real u[5];
        load5(s, U, e, q, u);
        real V[5] = {0, 0, 0, 0, 0}, Sf[5] = {0, 0, 0, 0, 0};
        real Vv[5] = {0, 0, 0, 0, 0}, Sv[5] = {0, 0, 0, 0, 0};
        for (int d = 0; d < 3; d++) {
          int Nd = N[d];
          real nq[3];
          load_ja(s, e, q, d, nq);
          int jj[3] = {i, j, k};
          for (int m = 0; m <= Nd; m++) {
            jj[d] = m;
            long qm = node_of(s, e, jj);
            real um[5], nm[3], navg[3], F[5];
            load5(s, U, e, qm, um);
            load_ja(s, e, qm, d, nm);
            for (int c = 0; c < 3; c++) navg[c] = (nq[c] + nm[c]) / 2;
            volume_flux(s, u, um, navg, F);
            for (int v = 0; v < 5; v++) V[v] += 2 * GLL[Nd].D[ii[d]][m] * F[v];
            if (s->viscous) {
              real Fd[5];
              contra_visc(s, U, Gall, e, qm, d, NULL, Fd);
              for (int v = 0; v < 5; v++) Vv[v] += GLL[Nd].D[ii[d]][m] * Fd[v];
            }
          }
          for (int side = 0; side < 2; side++) {
            int at = side ? Nd : 0;
            if (ii[d] != at) continue;
            int ta, tb;
            face_dirs(d, &ta, &tb);
            int na = N[ta] + 1, nf = na * (N[tb] + 1);
            real Fs[5], Fo[5];
            for (int v = 0; v < 5; v++) Fs[v] = Ff[2 * d + side][v * nf + ii[ta] + na * ii[tb]];
            euler_flux(u, nq, s->gamma, Fo);
            real wgt = 1 / GLL[Nd].w[at];
            for (int v = 0; v < 5; v++) Sf[v] += (side ? wgt : -wgt) * (Fs[v] - Fo[v]);
            if (s->viscous) {
              /* conforming only: matching node on the other element */
              int oth = s->nbr[6 * e + 2 * d + side];
              int kk[3] = {i, j, k};
              kk[d] = side ? 0 : s->N[oth][d];
              long qo = node_of(s, oth, kk);
              int Lq_e = side ? e : oth;
              long Lq = side ? q : qo;
              real S[3];
              load_ja(s, Lq_e, Lq, d, S);
              real Fst[5], Fown[5];
              face_viscous_flux(s, U, Gall, e, ii, d, side, oth, kk, S, Fst);
              contra_visc(s, U, Gall, e, q, d, NULL, Fown);
              for (int v = 0; v < 5; v++) Sv[v] += (side ? wgt : -wgt) * (Fst[v] - Fown[v]);
            }
          }
        }
        real Jq = s->J[s->off[e] + q];
        for (int v = 0; v < 5; v++) R[(long)v * nn + q] = (-V[v] - Sf[v] + Vv[v] + Sv[v]) / Jq;
      }
  for (int f = 0; f < 6; f++) free(Ff[f]);
}

/* ------------------------------------------------------------------------------------------
 * 8b. Residual of one element on Gauss-Legendre nodes (section "Spatial discretisation": the
 *     weak form NS2-NS4 with Gauss quadrature; no boundary nodes, so no split form).  With the
 *     Lagrange basis l_i, weights w_i and the derivative matrix D on the Gauss points:
 *       J dU_i/dt = -[ sum_d sum_m Dw_im F~^d_m
 *                      + sum_d (l_i(+1) F*(+d face) - l_i(-1) F*(-d face)) / w_i ],
 *     Dw_im = -D_mi w_m / w_i (the quadrature of -int F dl_i/dxi), F~^d = Ja^d . F(U) at the
 *     nodes, F* the numerical flux between the two traces U(+-1) = sum_i l_i(+-1) U_i along the
 *     line through the face point, with the owner's metric interpolated the same way as normal.
 *     With viscosity, the BR1 viscous flux enters the same way with the opposite sign: Ja^d .
 *     F_v(U, grad g) at the nodes, and on the faces the average of the two sides' F_v from their
 *     traces of U and of grad g (gradients from compute_gradients_gauss).  Uniform orders. */
/* trace on the face (d, side) of element e at face point (p, r) of a nodal field with nv
 * components stored [c * nn + node] from base f: sum_i l_i(side) f(node i of the line) */
static void gauss_trace(const orc_solver* s, const real* f, int nv, int e, int d, int side, int p, int r, real* out) {
  const int N = s->N[e][0], n = N + 1, nn = n * n * n;
  const gll_t* T = &s->T[N];
  int ta, tb;
  face_dirs(d, &ta, &tb);
  for (int c = 0; c < nv; c++) out[c] = 0;
  for (int i = 0; i < n; i++) {
    int ii[3];
    ii[d] = i; ii[ta] = p; ii[tb] = r;
    long q = node_of(s, e, ii);
    for (int c = 0; c < nv; c++) out[c] += T->lb[side][i] * f[(long)c * nn + q];
  }
}

/* 7b. BR1 gradients of g = (v, T) on Gauss-Legendre points, weak form with the face values
 *     g* = (g(U_L) + g(U_R)) / 2 of the interpolated traces:
 *       J grad g = sum_d Ja^d (delta_d g),
 *       (delta_d g)_i = -sum_m (w_m / w_i) D_mi g_m + (l_i(+1) g*(+d) - l_i(-1) g*(-d)) / w_i
 *     (the node's metric outside the weak derivative, as in the Lobatto BR1 gradient of 7). */
static void compute_gradients_gauss(orc_solver* s, const real* U, real* Gout) {
#pragma omp parallel for schedule(static)
  for (int e = 0; e < s->E; e++) {
    const int N = s->N[e][0], n = N + 1, nn = n * n * n;
    const gll_t* T = &s->T[N];
    real* G = Gout + s->off[e] * 12;
    for (int k = 0; k < n; k++)
      for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
          int ii[3] = {i, j, k};
          long q = node_of(s, e, ii);
          real acc[12] = {0};
          for (int d = 0; d < 3; d++) {
            int ta, tb;
            face_dirs(d, &ta, &tb);
            real a[4] = {0, 0, 0, 0};
            int jj[3] = {i, j, k};
            for (int m = 0; m < n; m++) {
              jj[d] = m;
              real um[5], gm[4];
              load5(s, U, e, node_of(s, e, jj), um);
              gvars(um, s->gamma, gm);
              real dw = -T->D[m][ii[d]] * T->w[m] / T->w[ii[d]];
              for (int c = 0; c < 4; c++) a[c] += dw * gm[c];
            }
            for (int side = 0; side < 2; side++) {
              int ne = s->nbr[6 * e + 2 * d + side];
              real uo[5], un[5], go[4], gn[4];
              gauss_trace(s, U + s->off[e] * 5, 5, e, d, side, ii[ta], ii[tb], uo);
              gauss_trace(s, U + s->off[ne] * 5, 5, ne, d, 1 - side, ii[ta], ii[tb], un);
              gvars(uo, s->gamma, go);
              gvars(un, s->gamma, gn);
              real l = T->lb[side][ii[d]] / T->w[ii[d]];
              for (int c = 0; c < 4; c++) a[c] += (side ? l : -l) * (go[c] + gn[c]) / 2;
            }
            real nv[3];
            load_ja(s, e, q, d, nv);
            for (int c = 0; c < 4; c++)
              for (int x = 0; x < 3; x++) acc[3 * c + x] += nv[x] * a[c];
          }
          real Jq = s->J[s->off[e] + q];
          for (int t = 0; t < 12; t++) G[(long)t * nn + q] = acc[t] / Jq;
        }
  }
}

/* 7c. BR2 and the symmetric interior penalty on Gauss-Legendre points.  Gauss quadrature is
 *     exact to degree 2N-1, so integrating by parts splits the weak derivative of 7b into the
 *     element's own (broken) derivative and, per face, the lift of g* - g(+-1), where
 *     g(+-1) = sum_j l_j(+-1) g_j is the trace of the element's interpolant of g:
 *       (delta_d g)_i = sum_m D_im g_m + (l_i(+1) (g*(+d) - g(+1)) - l_i(-1) (g*(-d) - g(-1))) / w_i.
 *     On face (d, side), BR2 takes the trace of the broken gradient plus eta times the trace of
 *     that face's lift alone; the interior penalty takes the trace of the broken gradient and
 *     adds its penalty (7, face_viscous_flux) with [g] and the mean velocity from g of the two
 *     interpolated traces of U, and h = 2 min(J_L, J_R)/|S| from the two traces of J.  On the
 *     box's smooth maps the two traces of J agree to interpolation error, so taking the smaller
 *     one is parity unpinned; the rest of 7c is pinned. */
static void gauss_broken_gradient(const orc_solver* s, const real* U, int e, const int ii[3], real gr[12]) {
  const int N = s->N[e][0], n = N + 1;
  const gll_t* T = &s->T[N];
  long q = node_of(s, e, ii);
  for (int t = 0; t < 12; t++) gr[t] = 0;
  for (int d = 0; d < 3; d++) {
    real a[4] = {0, 0, 0, 0};
    int jj[3] = {ii[0], ii[1], ii[2]};
    for (int m = 0; m < n; m++) {
      jj[d] = m;
      real um[5], gm[4];
      load5(s, U, e, node_of(s, e, jj), um);
      gvars(um, s->gamma, gm);
      for (int c = 0; c < 4; c++) a[c] += T->D[ii[d]][m] * gm[c];
    }
    real nv[3];
    load_ja(s, e, q, d, nv);
    for (int c = 0; c < 4; c++)
      for (int x = 0; x < 3; x++) gr[3 * c + x] += nv[x] * a[c];
  }
  real Jq = s->J[s->off[e] + q];
  for (int t = 0; t < 12; t++) gr[t] /= Jq;
}

/* g* - g(side) on face (d, side) of element e at face point (p, r): the jump that face lifts */
static void gauss_face_jump(const orc_solver* s, const real* U, int e, int d, int side, int p, int r, real jump[4]) {
  const int N = s->N[e][0], n = N + 1;
  const gll_t* T = &s->T[N];
  int ta, tb;
  face_dirs(d, &ta, &tb);
  int ne = s->nbr[6 * e + 2 * d + side];
  real uo[5], un[5], go[4], gn[4], gt[4] = {0, 0, 0, 0};
  gauss_trace(s, U + s->off[e] * 5, 5, e, d, side, p, r, uo);
  gauss_trace(s, U + s->off[ne] * 5, 5, ne, d, 1 - side, p, r, un);
  gvars(uo, s->gamma, go);
  gvars(un, s->gamma, gn);
  for (int i = 0; i < n; i++) {
    int ii[3];
    ii[d] = i; ii[ta] = p; ii[tb] = r;
    real ui[5], gi[4];
    load5(s, U, e, node_of(s, e, ii), ui);
    gvars(ui, s->gamma, gi);
    for (int c = 0; c < 4; c++) gt[c] += T->lb[side][i] * gi[c];
  }
  for (int c = 0; c < 4; c++) jump[c] = (go[c] + gn[c]) / 2 - gt[c];
}

/* fac times the lift of the jump of face (d, side), at node ii of the line through the face
 * point, added to the gradient gr */
static void gauss_add_lift(const orc_solver* s, int e, const int ii[3], int d, int side, const real jump[4], real fac,
                           real gr[12]) {
  const gll_t* T = &s->T[s->N[e][0]];
  long q = node_of(s, e, ii);
  real l = fac * T->lb[side][ii[d]] / T->w[ii[d]];
  if (!side) l = -l;
  real nv[3];
  load_ja(s, e, q, d, nv);
  real Jq = s->J[s->off[e] + q];
  for (int c = 0; c < 4; c++)
    for (int x = 0; x < 3; x++) gr[3 * c + x] += l * nv[x] * jump[c] / Jq;
}

/* BR2 (br2 = 1) or interior-penalty (br2 = 0) gradient of element e on its face (d, side) at
 * face point (p, r) */
static void gauss_face_gradient(const orc_solver* s, const real* U, int e, int d, int side, int p, int r, int br2,
                                real eta, real gr[12]) {
  const int N = s->N[e][0], n = N + 1;
  const gll_t* T = &s->T[N];
  int ta, tb;
  face_dirs(d, &ta, &tb);
  real jump[4];
  if (br2) gauss_face_jump(s, U, e, d, side, p, r, jump);
  for (int t = 0; t < 12; t++) gr[t] = 0;
  for (int i = 0; i < n; i++) {
    int ii[3];
    ii[d] = i; ii[ta] = p; ii[tb] = r;
    real gb[12];
    gauss_broken_gradient(s, U, e, ii, gb);
    if (br2) gauss_add_lift(s, e, ii, d, side, jump, eta, gb);
    for (int t = 0; t < 12; t++) gr[t] += T->lb[side][i] * gb[t];
  }
}

/* the traces uL, uR at face point (p, r) of the face between L (its +d face) and its neighbour
 * Rr, and the owner L's metric Ja^d interpolated there, the face's scaled normal S */
static void gauss_face_state(const orc_solver* s, const real* U, int L, int Rr, int d, int p, int r, real uL[5],
                             real uR[5], real S[3]) {
  const int n = s->N[L][0] + 1;
  const gll_t* T = &s->T[s->N[L][0]];
  int ta, tb;
  face_dirs(d, &ta, &tb);
  for (int v = 0; v < 5; v++) uL[v] = uR[v] = 0;
  S[0] = S[1] = S[2] = 0;
  for (int i = 0; i < n; i++) {
    int ii[3];
    ii[d] = i; ii[ta] = p; ii[tb] = r;
    real a[5], b[5], ja[3];
    long qL = node_of(s, L, ii), qR = node_of(s, Rr, ii);
    load5(s, U, L, qL, a);
    load5(s, U, Rr, qR, b);
    load_ja(s, L, qL, d, ja);
    for (int v = 0; v < 5; v++) {
      uL[v] += T->lb[1][i] * a[v];
      uR[v] += T->lb[0][i] * b[v];
    }
    for (int c = 0; c < 3; c++) S[c] += T->lb[1][i] * ja[c];
  }
}

/* the face viscous flux along S at face point (p, r) between L and Rr, from the traces uL, uR
 * (BR1: the two sides' fluxes from their traces of the BR1 gradient Gall; BR2 and the interior
 * penalty: from their face gradients of 7c, plus the penalty) */
static void gauss_face_viscous(const orc_solver* s, const real* U, const real* Gall, int L, int Rr, int d, int p, int r,
                               const real uL[5], const real uR[5], const real S[3], real Fst[5]) {
  real qL[12], qR[12], Fa[15], Fb[15];
  if (s->visc_flux == ORC_VISC_BR1) {
    gauss_trace(s, Gall + s->off[L] * 12, 12, L, d, 1, p, r, qL);
    gauss_trace(s, Gall + s->off[Rr] * 12, 12, Rr, d, 0, p, r, qR);
  } else {
    const int br2 = s->visc_flux == ORC_VISC_BR2;
    gauss_face_gradient(s, U, L, d, 1, p, r, br2, s->visc_eta, qL);
    gauss_face_gradient(s, U, Rr, d, 0, p, r, br2, s->visc_eta, qR);
  }
  viscous_flux(uL, qL, s->gamma, s->mu, s->kappa, Fa);
  viscous_flux(uR, qR, s->gamma, s->mu, s->kappa, Fb);
  for (int v = 0; v < 5; v++)
    Fst[v] = (S[0] * (Fa[v] + Fb[v]) + S[1] * (Fa[5 + v] + Fb[5 + v]) + S[2] * (Fa[10 + v] + Fb[10 + v])) / 2;
  if (s->visc_flux == ORC_VISC_IP) {
    const int N = s->N[L][0], n = N + 1;
    const gll_t* T = &s->T[N];
    int ta, tb;
    face_dirs(d, &ta, &tb);
    real JL = 0, JR = 0;
    for (int i = 0; i < n; i++) {
      int ii[3];
      ii[d] = i; ii[ta] = p; ii[tb] = r;
      JL += T->lb[1][i] * s->J[s->off[L] + node_of(s, L, ii)];
      JR += T->lb[0][i] * s->J[s->off[Rr] + node_of(s, Rr, ii)];
    }
    real gL[4], gR[4], vm[3], gr[12], Fv[15];
    gvars(uL, s->gamma, gL);
    gvars(uR, s->gamma, gR);
    real area = RSQRT(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
    real h = 2 * (JL < JR ? JL : JR) / area;
    real sigma = s->visc_eta * (real)(n * n) / h;
    for (int c = 0; c < 3; c++) vm[c] = (gL[c] + gR[c]) / 2;
    for (int c = 0; c < 4; c++)
      for (int x = 0; x < 3; x++) gr[3 * c + x] = sigma * (gR[c] - gL[c]) * S[x] / area;
    viscous_flux_v(vm, gr, s->mu, s->kappa, Fv);
    for (int v = 0; v < 5; v++) Fst[v] += S[0] * Fv[v] + S[1] * Fv[5 + v] + S[2] * Fv[10 + v];
  }
}

static void element_residual_gauss(const orc_solver* s, const real* U, const real* Gall, int e, real* R) {
  const int N = s->N[e][0], n = N + 1, nn = n * n * n;
  const gll_t* T = &s->T[N];
  /* numerical flux on the six faces, face point (p, r) along the two tangential directions */
  real Ff[6][5][(ORC_NMAX + 1) * (ORC_NMAX + 1)];
  for (int d = 0; d < 3; d++) {
    int ta, tb;
    face_dirs(d, &ta, &tb);
    for (int side = 0; side < 2; side++) {
      int L = side ? e : s->nbr[6 * e + 2 * d];
      int Rr = s->nbr[6 * L + 2 * d + 1];
      for (int r = 0; r < n; r++)
        for (int p = 0; p < n; p++) {
          real uL[5], uR[5], S[3];
          gauss_face_state(s, U, L, Rr, d, p, r, uL, uR, S);
          real F[5];
          surface_flux(s, uL, uR, S, F);
          if (s->viscous) {
            real Fst[5];
            gauss_face_viscous(s, U, Gall, L, Rr, d, p, r, uL, uR, S, Fst);
            for (int v = 0; v < 5; v++) F[v] -= Fst[v];
          }
          for (int v = 0; v < 5; v++) Ff[2 * d + side][v][p + n * r] = F[v];
        }
    }
  }
  for (int k = 0; k < n; k++)
    for (int j = 0; j < n; j++)
      for (int i = 0; i < n; i++) {
        int ii[3] = {i, j, k};
        long q = node_of(s, e, ii);
        real V[5] = {0, 0, 0, 0, 0};
        for (int d = 0; d < 3; d++) {
          int ta, tb;
          face_dirs(d, &ta, &tb);
          int jj[3] = {i, j, k};
          for (int m = 0; m < n; m++) {
            jj[d] = m;
            long qm = node_of(s, e, jj);
            real um[5], nm[3], F[5];
            load5(s, U, e, qm, um);
            load_ja(s, e, qm, d, nm);
            euler_flux(um, nm, s->gamma, F);
            if (s->viscous) {  /* the viscous flux enters with the opposite sign */
              real Fd[5];
              contra_visc(s, U, Gall, e, qm, d, NULL, Fd);
              for (int v = 0; v < 5; v++) F[v] -= Fd[v];
            }
            real dw = -T->D[m][ii[d]] * T->w[m] / T->w[ii[d]];
            for (int v = 0; v < 5; v++) V[v] += dw * F[v];
          }
          int fq = ii[ta] + n * ii[tb];
          for (int v = 0; v < 5; v++)
            V[v] += (T->lb[1][ii[d]] * Ff[2 * d + 1][v][fq] - T->lb[0][ii[d]] * Ff[2 * d][v][fq]) / T->w[ii[d]];
        }
        real Jq = s->J[s->off[e] + q];
        for (int v = 0; v < 5; v++) R[(long)v * nn + q] = -V[v] / Jq;
      }
}

/* ------------------------------------------------------------------------------------------
 * 8c. Spectral vanishing viscosity (section "Shock capturing").
 *     The artificial flux F_a is the Navier-Stokes viscous flux with viscosity mu_a and
 *     conductivity kappa_a = mu_a gamma / ((gamma-1) Pr), written as F_a = B G with G the BR1
 *     gradient of the entropy variables w = (.., rho v/p, -rho/p) (eq. shock:fluxmatrix).
 *     With theta = p/rho, grad v_k = theta (grad w_{k+1} + v_k grad w_5) and grad theta =
 *     theta^2 grad w_5, so B = L^T D L with the eight rows of L
 *       L_m G = <E_m, Z>  (m = 1..5),   Z_kj = d_j w_{k+1} + v_k d_j w_5,
 *       L_m G = d_j w_5   (m = 6..8, j = m - 6),
 *     E_m an orthonormal basis of the symmetric traceless 3x3 matrices, and
 *       D = (2 mu_a theta five times, kappa_a theta^2 three times):
 *     L^T D L G is the stress mu_a (grad v + grad v^T - 2/3 div v I) and the heat flux
 *     kappa_a grad theta, i.e. the Navier-Stokes viscous flux.
 *     The filtered flux (eq. shock:filteredflux): F_a^F = J^{-1/2} L^T D^{1/2} F*(sqrt(J D) L G),
 *     the filter F* applied to each of the eight nodal fields y_m = sqrt(J D_m) L_m G of the
 *     element in the Legendre modal space: transform, multiply mode (a,b,c) by
 *     1 - (1 - s_a)(1 - s_b)(1 - s_c), transform back.  One-direction kernel: s_k = 0 for k <= M;
 *     for k > M, s_k = 1 (Tadmor's step) or exp(-((k-N)/(k-M))^2) (Maday et al.).
 *     Sensor: s_rho = sum over the nodes of w_i w_j w_k J |grad_xi rho|^2 (the element integral of
 *     the paper by the nodal quadrature, grad_xi rho the element's own derivative); an element
 *     with s_rho above the threshold takes the unfiltered flux L^T D L G.
 *     Residual: as the viscous terms of section 8, J R_a = sum_d D_d F~^d
 *     + (1/w_N)(F~* - F~) at xi_d = +1 - (1/w_0)(F~* - F~) at -1, F~^d = Ja^d . F_a^F and F~* the
 *     average of the two sides' filtered fluxes along the owner's Ja^d.
 *     Explicit LES closure (section on turbulence models: Smagorinsky, WALE, Vreman and
 *     SVV-Smagorinsky, whose definitions the paper leaves to its references).  Reading: the
 *     artificial viscosity of the term above becomes, node by node, mu_a + rho nu_t with the
 *     eddy viscosity nu_t of the model from g = grad v (g_kj = d v_k / d x_j) of the same BR1
 *     gradient (grad v_k = theta (grad w_{k+1} + v_k grad w_5)) and the filter width
 *     Delta = 2 (J/n)^(1/3) (the cube root of the element volume per node, n the element's node
 *     count):
 *       Smagorinsky  nu_t = (C Delta)^2 |S|,  S = (g + g^T)/2,  |S| = sqrt(2 S:S);
 *       WALE         nu_t = (C Delta)^2 (Sd:Sd)^(3/2) / ((S:S)^(5/2) + (Sd:Sd)^(5/4)),
 *                    Sd = (g^2 + (g^2)^T)/2 - tr(g^2) I/3  (Nicoud and Ducros);
 *       Vreman       nu_t = C sqrt(B / (g:g)),  b = Delta^2 g g^T,
 *                    B = b11 b22 - b12^2 + b11 b33 - b13^2 + b22 b33 - b23^2  (Vreman);
 *     each zero where its denominator vanishes; the conductivity is that viscosity times
 *     gamma/((gamma-1) Pr).  Filtered by the SVV kernel this is the SVV-Smagorinsky closure (with
 *     Smagorinsky's nu_t); with Tadmor's kernel and cutoff -1 (every mode kept) the plain model.
 *     Since D scales with the viscosity node by node, sqrt(J D) and D^{1/2} carry the local value
 *     and the factorisation above is unchanged.
 * ---------------------------------------------------------------------------------------- */
static real svv_sigma(int N, int kernel, int M, int k) {
  if (k <= M) return 0;
  if (kernel == ORC_SVV_TADMOR) return 1;
  real r = (real)(k - N) / (real)(k - M);
  return REXP(-r * r);
}

/* orthonormal basis of the symmetric traceless 3x3 matrices (Frobenius inner product) */
static void svv_basis(real E[5][3][3]) {
  for (int m = 0; m < 5; m++)
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) E[m][a][b] = 0;
  real r2 = 1 / RSQRT((real)2), r6 = 1 / RSQRT((real)6);
  E[0][0][1] = E[0][1][0] = r2;
  E[1][0][2] = E[1][2][0] = r2;
  E[2][1][2] = E[2][2][1] = r2;
  E[3][0][0] = r2; E[3][1][1] = -r2;
  E[4][0][0] = r6; E[4][1][1] = r6; E[4][2][2] = -2 * r6;
}

/* rows L[8][15] (over G[3c + x], c the entropy variable, x the direction) and D[8] at one state.
 * B is singular, so its L^T D L factorisation is not unique and the filtered flux depends on the
 * one taken: this one (the symmetric traceless basis above and the temperature gradient) is
 * parity unpinned; the pins fix B = L^T D L and the entropy identity, which every such
 * factorisation satisfies. */
static void svv_factors(const real u[5], real gamma, real mu, real kappa, real L[8][15], real D[8]) {
  prim_t q = prim(u, gamma);
  real th = q.p / q.rho;
  real E[5][3][3];
  svv_basis(E);
  for (int m = 0; m < 8; m++)
    for (int t = 0; t < 15; t++) L[m][t] = 0;
  for (int m = 0; m < 5; m++) {
    for (int k = 0; k < 3; k++)
      for (int j = 0; j < 3; j++) {
        L[m][3 * (k + 1) + j] += E[m][k][j];
        L[m][3 * 4 + j] += E[m][k][j] * q.v[k];
      }
    D[m] = 2 * mu * th;
  }
  for (int j = 0; j < 3; j++) {
    L[5 + j][3 * 4 + j] = 1;
    D[5 + j] = kappa * th * th;
  }
}

/* Legendre polynomial P_a at the Lobatto node i of order N, and the discrete norm of P_a */
static real svv_leg(int N, int a, int i) {
  long double L, dL;
  legendre(a, GLL[N].xl[i], &L, &dL);
  return (real)L;
}

static real svv_norm(int N, int a) {
  real g = 0;
  for (int i = 0; i <= N; i++) g += GLL[N].w[i] * svv_leg(N, a, i) * svv_leg(N, a, i);
  return g;
}

/* the modal filter of one nodal field f of an element with orders N[3] */
static void svv_filter_field(const int N[3], int kernel, int M, const real* f, real* out) {
  const int n0 = N[0] + 1, n1 = N[1] + 1, n2 = N[2] + 1, nn = n0 * n1 * n2;
  real* c = (real*)malloc(sizeof(real) * nn);
  for (int cc = 0; cc < n2; cc++)
    for (int b = 0; b < n1; b++)
      for (int a = 0; a < n0; a++) {
        real acc = 0;
        for (int k = 0; k < n2; k++)
          for (int j = 0; j < n1; j++)
            for (int i = 0; i < n0; i++)
              acc += GLL[N[0]].w[i] * svv_leg(N[0], a, i) * GLL[N[1]].w[j] * svv_leg(N[1], b, j) *
                     GLL[N[2]].w[k] * svv_leg(N[2], cc, k) * f[nidx(n0, n1, i, j, k)];
        acc /= svv_norm(N[0], a) * svv_norm(N[1], b) * svv_norm(N[2], cc);
        real sa = svv_sigma(N[0], kernel, M, a), sb = svv_sigma(N[1], kernel, M, b),
             sc = svv_sigma(N[2], kernel, M, cc);
        c[nidx(n0, n1, a, b, cc)] = acc * (1 - (1 - sa) * (1 - sb) * (1 - sc));
      }
  for (int k = 0; k < n2; k++)
    for (int j = 0; j < n1; j++)
      for (int i = 0; i < n0; i++) {
        real acc = 0;
        for (int cc = 0; cc < n2; cc++)
          for (int b = 0; b < n1; b++)
            for (int a = 0; a < n0; a++)
              acc += svv_leg(N[0], a, i) * svv_leg(N[1], b, j) * svv_leg(N[2], cc, k) * c[nidx(n0, n1, a, b, cc)];
        out[nidx(n0, n1, i, j, k)] = acc;
      }
  free(c);
}

/* the eddy viscosity rho nu_t of the explicit LES closure at one node: state u, entropy-variable
 * gradient G[3c + x], model and constant, Jacobian J, n nodes in the element */
static real les_viscosity(const real u[5], const real G[15], real gamma, int model, real cs, real J, int n) {
  prim_t q = prim(u, gamma);
  real th = q.p / q.rho;
  real g[3][3];  /* d v_k / d x_j */
  for (int k = 0; k < 3; k++)
    for (int j = 0; j < 3; j++) g[k][j] = th * (G[3 * (k + 1) + j] + q.v[k] * G[3 * 4 + j]);
  real delta = 2 * RCBRT(J / n);
  real ss = 0;  /* S:S */
  for (int k = 0; k < 3; k++)
    for (int j = 0; j < 3; j++) {
      real sk = (g[k][j] + g[j][k]) / 2;
      ss += sk * sk;
    }
  real nu = 0;
  if (model == ORC_LES_SMAGORINSKY) {
    nu = (cs * delta) * (cs * delta) * RSQRT(2 * ss);
  } else if (model == ORC_LES_WALE) {
    real g2[3][3], tr = 0;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        g2[i][j] = 0;
        for (int k = 0; k < 3; k++) g2[i][j] += g[i][k] * g[k][j];
      }
    for (int i = 0; i < 3; i++) tr += g2[i][i];
    real sd = 0;  /* Sd:Sd */
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        real x = (g2[i][j] + g2[j][i]) / 2 - (i == j ? tr / 3 : 0);
        sd += x * x;
      }
    real den = RPOW(ss, (real)2.5) + RPOW(sd, (real)1.25);
    nu = den > 0 ? (cs * delta) * (cs * delta) * RPOW(sd, (real)1.5) / den : 0;
  } else {  /* Vreman */
    real b[3][3], gg = 0;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        b[i][j] = 0;
        for (int m = 0; m < 3; m++) b[i][j] += delta * delta * g[i][m] * g[j][m];
        gg += g[i][j] * g[i][j];
      }
    real B = b[0][0] * b[1][1] - b[0][1] * b[0][1] + b[0][0] * b[2][2] - b[0][2] * b[0][2] +
             b[1][1] * b[2][2] - b[1][2] * b[1][2];
    nu = gg > 0 && B > 0 ? cs * RSQRT(B / gg) : 0;
  }
  return q.rho * nu;
}

/* the factors of the artificial flux at one node: viscosity mu_a plus (cs > 0) the LES model's eddy
 * viscosity, conductivity that viscosity times gamma/((gamma-1) Pr) */
static void svv_node_factors(const real u[5], const real G[15], real gamma, real Pr, real mu_a, int model,
                             real cs, real J, int n, real L[8][15], real D[8]) {
  real mu = mu_a;
  if (cs > 0) mu += les_viscosity(u, G, gamma, model, cs, J, n);
  svv_factors(u, gamma, mu, mu * gamma / ((gamma - 1) * Pr), L, D);
}

/* the sensor s_rho of element e */
static real svv_sensor(const orc_solver* s, const real* U, int e) {
  const int* N = s->N[e];
  real acc = 0;
  for (int k = 0; k <= N[2]; k++)
    for (int j = 0; j <= N[1]; j++)
      for (int i = 0; i <= N[0]; i++) {
        int ii[3] = {i, j, k};
        long q = node_of(s, e, ii);
        real g2 = 0;
        for (int d = 0; d < 3; d++) {
          real a = 0;
          int jj[3] = {i, j, k};
          for (int m = 0; m <= N[d]; m++) {
            jj[d] = m;
            a += GLL[N[d]].D[ii[d]][m] * U[s->off[e] * 5 + node_of(s, e, jj)];
          }
          g2 += a * a;
        }
        acc += GLL[N[0]].w[i] * GLL[N[1]].w[j] * GLL[N[2]].w[k] * s->J[s->off[e] + q] * g2;
      }
  return acc;
}

/* filtered fluxes of element e into Fa[off*15 + (5n+v)*nn + node] from the entropy-variable
 * gradients Gw; returns sum_m <y_m, F* y_m> (nodal quadrature, the entropy form) */
static real svv_element_flux(const orc_solver* s, const real* U, const real* Gw, int e, real* Fa) {
  const int* N = s->N[e];
  int nn = nn_of(s, e);
  real* y = (real*)malloc(sizeof(real) * 8 * nn);
  real* yf = (real*)malloc(sizeof(real) * 8 * nn);
  real* Dn = (real*)malloc(sizeof(real) * 8 * nn);
  real (*Ln)[8][15] = (real(*)[8][15])malloc(sizeof(real) * 8 * 15 * nn);
  const int trouble = s->svv_sensor >= 0 && svv_sensor(s, U, e) > s->svv_sensor;
  for (long q = 0; q < nn; q++) {
    real u[5], G[15];
    load5(s, U, e, q, u);
    for (int t = 0; t < 15; t++) G[t] = Gw[s->off[e] * 15 + (long)t * nn + q];
    real Jq = s->J[s->off[e] + q];
    svv_node_factors(u, G, s->gamma, s->Pr, s->svv_mu, s->les_model, s->les_cs, Jq, nn, Ln[q], &Dn[8 * q]);
    for (int m = 0; m < 8; m++) {
      real lg = 0;
      for (int t = 0; t < 15; t++) lg += Ln[q][m][t] * G[t];
      y[(long)m * nn + q] = RSQRT(Jq * Dn[8 * q + m]) * lg;
    }
  }
  real form = 0;
  for (int m = 0; m < 8; m++) {
    if (trouble) for (long q = 0; q < nn; q++) yf[(long)m * nn + q] = y[(long)m * nn + q];
    else svv_filter_field(N, s->svv_kernel, s->svv_cut, y + (long)m * nn, yf + (long)m * nn);
  }
  for (int k = 0; k <= N[2]; k++)
    for (int j = 0; j <= N[1]; j++)
      for (int i = 0; i <= N[0]; i++) {
        int ii[3] = {i, j, k};
        long q = node_of(s, e, ii);
        real wq = GLL[N[0]].w[i] * GLL[N[1]].w[j] * GLL[N[2]].w[k];
        for (int m = 0; m < 8; m++) form += wq * y[(long)m * nn + q] * yf[(long)m * nn + q];
        real Jq = s->J[s->off[e] + q];
        for (int x = 0; x < 3; x++)
          for (int c = 0; c < 5; c++) {
            real acc = 0;
            for (int m = 0; m < 8; m++) acc += Ln[q][m][3 * c + x] * RSQRT(Dn[8 * q + m]) * yf[(long)m * nn + q];
            Fa[s->off[e] * 15 + (long)(5 * x + c) * nn + q] = acc / RSQRT(Jq);
          }
      }
  free(y); free(yf); free(Dn); free(Ln);
  return form;
}

/* contravariant filtered flux of node q of element e along S */
static void svv_contra(const orc_solver* s, const real* Fa, int e, long q, const real S[3], real F[5]) {
  int nn = nn_of(s, e);
  for (int v = 0; v < 5; v++) {
    F[v] = 0;
    for (int x = 0; x < 3; x++) F[v] += S[x] * Fa[s->off[e] * 15 + (long)(5 * x + v) * nn + q];
  }
}

/* adds the artificial-viscosity residual of element e to R (R laid out as the state) */
static void svv_element_residual(const orc_solver* s, const real* Fa, int e, real* R) {
  const int* N = s->N[e];
  int nn = nn_of(s, e);
  for (int k = 0; k <= N[2]; k++)
    for (int j = 0; j <= N[1]; j++)
      for (int i = 0; i <= N[0]; i++) {
        int ii[3] = {i, j, k};
        long q = node_of(s, e, ii);
        real Ra[5] = {0, 0, 0, 0, 0};
        for (int d = 0; d < 3; d++) {
          int jj[3] = {i, j, k};
          for (int m = 0; m <= N[d]; m++) {
            jj[d] = m;
            long qm = node_of(s, e, jj);
            real S[3], F[5];
            load_ja(s, e, qm, d, S);
            svv_contra(s, Fa, e, qm, S, F);
            for (int v = 0; v < 5; v++) Ra[v] += GLL[N[d]].D[ii[d]][m] * F[v];
          }
          for (int side = 0; side < 2; side++) {
            int at = side ? N[d] : 0;
            if (ii[d] != at) continue;
            int oth = s->nbr[6 * e + 2 * d + side];
            int kk[3] = {i, j, k};
            kk[d] = side ? 0 : s->N[oth][d];
            long qo = node_of(s, oth, kk);
            real S[3], own[5], Fe[5], Fo[5], nq[3];
            if (side) load_ja(s, e, q, d, S);
            else load_ja(s, oth, qo, d, S);
            svv_contra(s, Fa, e, q, S, Fe);
            svv_contra(s, Fa, oth, qo, S, Fo);
            load_ja(s, e, q, d, nq);
            svv_contra(s, Fa, e, q, nq, own);
            real wgt = 1 / GLL[N[d]].w[at];
            for (int v = 0; v < 5; v++) Ra[v] += (side ? wgt : -wgt) * ((Fe[v] + Fo[v]) / 2 - own[v]);
          }
        }
        real Jq = s->J[s->off[e] + q];
        for (int v = 0; v < 5; v++) R[(long)v * nn + q] += Ra[v] / Jq;
      }
}

/* the artificial-viscosity residual of U added to R; returns the entropy form sum <y, F* y> */
static real svv_residual(orc_solver* s, const real* U, real* R) {
  br1_gradient(s, U, 5, entropy_vars, s->Gw);
  /* per-element terms of the form, summed in element order: the result does not depend on the
   * thread count */
  real* fe = (real*)malloc(sizeof(real) * (size_t)(s->E > 0 ? s->E : 1));
#pragma omp parallel for schedule(dynamic, 4)
  for (int e = 0; e < s->E; e++) fe[e] = svv_element_flux(s, U, s->Gw, e, s->Fa);
#pragma omp parallel for schedule(dynamic, 4)
  for (int e = 0; e < s->E; e++) svv_element_residual(s, s->Fa, e, R + s->off[e] * 5);
  real form = 0;
  for (int e = 0; e < s->E; e++) form += fe[e];
  free(fe);
  return form;
}

static void residual(orc_solver* s, const real* U, real* R) {
  if (s->surf == ORC_SURF_LF_GLOBAL) {
    /* the largest |v| + c over the nodes of the state the residual is taken of */
    real lam = 0;
    for (int e = 0; e < s->E; e++) {
      int nn = nn_of(s, e);
      for (int q = 0; q < nn; q++) {
        real u[5];
        load5(s, U, e, q, u);
        prim_t w = prim(u, s->gamma);
        real l = RSQRT(w.v[0] * w.v[0] + w.v[1] * w.v[1] + w.v[2] * w.v[2]) + RSQRT(s->gamma * w.p / w.rho);
        if (l > lam) lam = l;
      }
    }
    s->lam_g = lam;
  }
  if (s->gauss) {
    if (s->viscous) compute_gradients_gauss(s, U, s->G);
#pragma omp parallel for schedule(dynamic, 4)
    for (int e = 0; e < s->E; e++) element_residual_gauss(s, U, s->G, e, R + s->off[e] * 5);
    return;
  }
  if (s->viscous) compute_gradients(s, U, s->G);
#pragma omp parallel for schedule(dynamic, 4)
  for (int e = 0; e < s->E; e++) element_residual(s, U, s->G, e, R + s->off[e] * 5);
  if (s->svv) svv_residual(s, U, R);
}

int orc_residual(orc_solver* s, double* Rout) {
  if (!s) return -1;
  residual(s, s->U, s->R);
  if (Rout) for (long i = 0; i < 5 * s->ntot; i++) Rout[i] = (double)s->R[i];
  return 0;
}

int orc_gradients(orc_solver* s, double* Gout) {
  if (!s) return -1;
  if (s->gauss) compute_gradients_gauss(s, s->U, s->G);
  else compute_gradients(s, s->U, s->G);
  for (long i = 0; i < 12 * s->ntot; i++) Gout[i] = (double)s->G[i];
  return 0;
}

/* ------------------------------------------------------------------------------------------
 * 9. Low-storage (2N) explicit Runge-Kutta schemes (section "Time advancement"): per stage k,
 *    dU <- A_k dU + dt R(U);  U <- U + B_k dU.
 *    scheme 0: Williamson's RK3 (the default of the paper), A = (0, -5/9, -153/128),
 *              B = (1/3, 15/16, 8/15);
 *    scheme 1: Carpenter and Kennedy's five-stage fourth-order scheme (the paper's RK4 option),
 *              with their published rational coefficients.
 * ---------------------------------------------------------------------------------------- */
int orc_rk(orc_solver* s, int scheme, double dt, int nsteps) {
  if (!s || nsteps < 0 || scheme < 0 || scheme > 1) return -1;
  real A[5], B[5];
  int ns;
  if (scheme == 0) {
    ns = 3;
    A[0] = 0; A[1] = (real)-5 / 9; A[2] = (real)-153 / 128;
    B[0] = (real)1 / 3; B[1] = (real)15 / 16; B[2] = (real)8 / 15;
  } else {
    ns = 5;
    A[0] = 0;
    A[1] = -(real)567301805773.0L / (real)1357537059087.0L;
    A[2] = -(real)2404267990393.0L / (real)2016746695238.0L;
    A[3] = -(real)3550918686646.0L / (real)2091501179385.0L;
    A[4] = -(real)1275806237668.0L / (real)842570457699.0L;
    B[0] = (real)1432997174477.0L / (real)9575080441755.0L;
    B[1] = (real)5161836677717.0L / (real)13612068292357.0L;
    B[2] = (real)1720146321549.0L / (real)2090206949498.0L;
    B[3] = (real)3134564353537.0L / (real)4481467310338.0L;
    B[4] = (real)2277821191437.0L / (real)14882151754819.0L;
  }
  long n5 = 5 * s->ntot;
  for (int step = 0; step < nsteps; step++)
    for (int k = 0; k < ns; k++) {
      residual(s, s->U, s->R);
#pragma omp parallel for schedule(static)
      for (long i = 0; i < n5; i++) {
        s->dU[i] = (k == 0 ? 0 : A[k] * s->dU[i]) + (real)dt * s->R[i];
        s->U[i] += B[k] * s->dU[i];
      }
    }
  return 0;
}

int orc_rk3(orc_solver* s, double dt, int nsteps) { return orc_rk(s, 0, dt, nsteps); }

/* ------------------------------------------------------------------------------------------
 * 10. Initial conditions, evaluated at the node coordinates.
 *   UNIFORM (rho, v1, v2, v3, p);  TGV on [0,2pi]^3 with p0 = 1/(gamma Ma^2), rho = p/p0;
 *   VORTEX (beta, x0, y0, u_inf, v_inf): isentropic vortex on a rho=p=1 free stream;
 *   DENSITY_WAVE (amp, v1, v2, v3, p, k1, k2, k3, phase): rho = 1 + amp sin(k.x + phase).
 * ---------------------------------------------------------------------------------------- */
static void ic_point(const orc_solver* s, int ic, const double* P, const real x[3], real u[5]) {
  real g = s->gamma;
  real rho = 1, v[3] = {0, 0, 0}, p = 1;
  if (ic == ORC_IC_UNIFORM) {
    rho = P[0]; v[0] = P[1]; v[1] = P[2]; v[2] = P[3]; p = P[4];
  } else if (ic == ORC_IC_TGV) {
    real p0 = 1 / (g * s->Ma * s->Ma);
    v[0] = RSIN(x[0]) * RCOS(x[1]) * RCOS(x[2]);
    v[1] = -RCOS(x[0]) * RSIN(x[1]) * RCOS(x[2]);
    v[2] = 0;
    p = p0 + (RCOS(2 * x[0]) + RCOS(2 * x[1])) * (RCOS(2 * x[2]) + 2) / 16;
    rho = p / p0;
  } else if (ic == ORC_IC_VORTEX) {
    real beta = P[0], dx = x[0] - P[1], dy = x[1] - P[2];
    real r2 = dx * dx + dy * dy;
    real pi = (real)PI_L;
    real f = beta / (2 * pi) * REXP((1 - r2) / 2);
    v[0] = P[3] - f * dy;
    v[1] = P[4] + f * dx;
    v[2] = 0;
    real T = 1 - (g - 1) * beta * beta / (8 * g * pi * pi) * REXP(1 - r2);
    rho = RPOW(T, 1 / (g - 1));
    p = rho * T;
  } else if (ic == ORC_IC_DENSITY_WAVE) {
    rho = 1 + P[0] * RSIN(P[5] * x[0] + P[6] * x[1] + P[7] * x[2] + P[8]);
    v[0] = P[1]; v[1] = P[2]; v[2] = P[3]; p = P[4];
  }
  u[0] = rho;
  for (int c = 0; c < 3; c++) u[1 + c] = rho * v[c];
  u[4] = p / (g - 1) + rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / 2;
}

int orc_set_ic(orc_solver* s, int ic, const double* params) {
  if (!s || ic < 0 || ic > 3) return -1;
  if (ic != ORC_IC_TGV && !params) return -1;
  for (int e = 0; e < s->E; e++) {
    int nn = nn_of(s, e);
    for (int q = 0; q < nn; q++) {
      real x[3], u[5];
      for (int d = 0; d < 3; d++) x[d] = s->X[s->off[e] * 3 + (long)d * nn + q];
      ic_point(s, ic, params, x, u);
      for (int v = 0; v < 5; v++) s->U[s->off[e] * 5 + (long)v * nn + q] = u[v];
    }
  }
  memset(s->dU, 0, sizeof(real) * 5 * s->ntot);
  return 0;
}

int orc_set_state(orc_solver* s, const double* U) {
  if (!s || !U) return -1;
  for (long i = 0; i < 5 * s->ntot; i++) s->U[i] = U[i];
  memset(s->dU, 0, sizeof(real) * 5 * s->ntot);
  return 0;
}

int orc_get_state(const orc_solver* s, double* U) {
  if (!s || !U) return -1;
  for (long i = 0; i < 5 * s->ntot; i++) U[i] = (double)s->U[i];
  return 0;
}

/* time step: CFL h_min / ((N_max+1)^2 lambda_max), limited by the viscous bound
 * 0.25 h_min^2 / ((N_max+1)^4 gamma mu / (Pr rho_min)), mu the physical viscosity plus the
 * artificial one of section 8c */
double orc_suggest_dt(const orc_solver* s, double cfl) {
  real hmin = s->h[0];
  if (s->h[1] < hmin) hmin = s->h[1];
  if (s->h[2] < hmin) hmin = s->h[2];
  int Nmax = 1;
  for (int e = 0; e < s->E; e++)
    for (int d = 0; d < 3; d++)
      if (s->N[e][d] > Nmax) Nmax = s->N[e][d];
  real lam = 0, rmin = 1e300;
  for (int e = 0; e < s->E; e++) {
    int nn = nn_of(s, e);
    for (int q = 0; q < nn; q++) {
      real u[5];
      load5(s, s->U, e, q, u);
      prim_t w = prim(u, s->gamma);
      real l = RSQRT(w.v[0] * w.v[0] + w.v[1] * w.v[1] + w.v[2] * w.v[2]) + RSQRT(s->gamma * w.p / w.rho);
      if (l > lam) lam = l;
      if (w.rho < rmin) rmin = w.rho;
    }
  }
  real n1 = Nmax + 1;
  real dt = (real)cfl * hmin / (n1 * n1 * lam);
  real mu = (s->viscous ? s->mu : 0) + (s->svv ? s->svv_mu : 0);  /* physical plus artificial */
  if (mu > 0) {
    real dtv = (real)0.25 * hmin * hmin / (n1 * n1 * n1 * n1 * s->gamma * mu / (s->Pr * rmin));
    if (dtv < dt) dt = dtv;
  }
  return (double)dt;
}

/* ------------------------------------------------------------------------------------------
 * 11. Diagnostics with the Lobatto quadrature w_i w_j w_k J:
 *   out[0..4] integral of U; out[5] integral of -rho s; out[6] integral of -rho s/(gamma-1);
 *   out[7] kinetic energy (volume mean of rho|v|^2/2); out[8] enstrophy (volume mean of
 *   rho|curl v|^2/2, element-local derivative of v); out[9] max(|v|+c); out[10] min rho;
 *   out[11] min p; out[12] number of non-finite state values; out[13] volume.
 * ---------------------------------------------------------------------------------------- */
int orc_diagnostics(const orc_solver* s, double* out) {
  if (!s || !out) return -1;
  real acc[9] = {0};
  real lam = 0, rmin = 1e300, pmin = 1e300;
  long bad = 0;
  for (int e = 0; e < s->E; e++) {
    const int* N = s->N[e];
    int nn = nn_of(s, e);
    real* vel = (real*)malloc(sizeof(real) * 3 * nn);
    for (int q = 0; q < nn; q++) {
      real u[5];
      load5(s, s->U, e, q, u);
      for (int c = 0; c < 3; c++) vel[c * nn + q] = u[1 + c] / u[0];
    }
    for (int k = 0; k <= N[2]; k++)
      for (int j = 0; j <= N[1]; j++)
        for (int i = 0; i <= N[0]; i++) {
          int ii[3] = {i, j, k};
          long q = node_of(s, e, ii);
          real u[5];
          load5(s, s->U, e, q, u);
          for (int v = 0; v < 5; v++)
            if (!isfinite((double)u[v])) bad++;
          prim_t w = prim(u, s->gamma);
          real Jq = s->J[s->off[e] + q];
          real wq = s->T[N[0]].w[i] * s->T[N[1]].w[j] * s->T[N[2]].w[k] * Jq;
          for (int v = 0; v < 5; v++) acc[v] += wq * u[v];
          real sp = RLOG(w.p) - s->gamma * RLOG(w.rho);
          acc[5] += wq * (-w.rho * sp);
          acc[6] += wq * (-w.rho * sp / (s->gamma - 1));
          real v2 = w.v[0] * w.v[0] + w.v[1] * w.v[1] + w.v[2] * w.v[2];
          acc[7] += wq * w.rho * v2 / 2;
          /* grad v: dv_c/dx_n = (1/J) sum_d Ja^d_n D_d v_c */
          real gv[3][3] = {{0}};
          for (int d = 0; d < 3; d++) {
            real n[3];
            load_ja(s, e, q, d, n);
            for (int c = 0; c < 3; c++) {
              real dd = dref(s, e, vel + c * nn, d, ii);
              for (int x = 0; x < 3; x++) gv[c][x] += n[x] * dd / Jq;
            }
          }
          real om[3] = {gv[2][1] - gv[1][2], gv[0][2] - gv[2][0], gv[1][0] - gv[0][1]};
          acc[8] += wq * w.rho * (om[0] * om[0] + om[1] * om[1] + om[2] * om[2]) / 2;
          real l = RSQRT(v2) + RSQRT(s->gamma * w.p / w.rho);
          if (l > lam) lam = l;
          if (w.rho < rmin) rmin = w.rho;
          if (w.p < pmin) pmin = w.p;
        }
    free(vel);
  }
  real vol = 0;
  for (int e = 0; e < s->E; e++) {
    const int* N = s->N[e];
    for (int k = 0; k <= N[2]; k++)
      for (int j = 0; j <= N[1]; j++)
        for (int i = 0; i <= N[0]; i++) {
          int ii[3] = {i, j, k};
          vol += s->T[N[0]].w[i] * s->T[N[1]].w[j] * s->T[N[2]].w[k] * s->J[s->off[e] + node_of(s, e, ii)];
        }
  }
  for (int v = 0; v < 7; v++) out[v] = (double)acc[v];
  out[7] = (double)(acc[7] / vol);
  out[8] = (double)(acc[8] / vol);
  out[9] = (double)lam;
  out[10] = (double)rmin;
  out[11] = (double)pmin;
  out[12] = (double)bad;
  out[13] = (double)vol;
  return 0;
}

/* sum over nodes of w_i w_j w_k J w(U).R: the semi-discrete entropy production rate */
double orc_entropy_production(const orc_solver* s, const double* R) {
  real acc = 0;
  for (int e = 0; e < s->E; e++) {
    const int* N = s->N[e];
    int nn = nn_of(s, e);
    for (int k = 0; k <= N[2]; k++)
      for (int j = 0; j <= N[1]; j++)
        for (int i = 0; i <= N[0]; i++) {
          int ii[3] = {i, j, k};
          long q = node_of(s, e, ii);
          real u[5];
          load5(s, s->U, e, q, u);
          prim_t w = prim(u, s->gamma);
          real sp = RLOG(w.p) - s->gamma * RLOG(w.rho);
          real b = w.rho / (2 * w.p);
          real v2 = w.v[0] * w.v[0] + w.v[1] * w.v[1] + w.v[2] * w.v[2];
          real wv[5] = {(s->gamma - sp) / (s->gamma - 1) - b * v2, 2 * b * w.v[0], 2 * b * w.v[1],
                        2 * b * w.v[2], -2 * b};
          real wq = s->T[N[0]].w[i] * s->T[N[1]].w[j] * s->T[N[2]].w[k] * s->J[s->off[e] + q];
          for (int v = 0; v < 5; v++) acc += wq * wv[v] * (real)R[s->off[e] * 5 + (long)v * nn + q];
        }
  }
  return (double)acc;
}

/* ------------------------------------------------------------------------------------------
 * 12. Point functions exported for the pins.
 * ---------------------------------------------------------------------------------------- */
static void to_real(const double* a, real* b, int n) { for (int i = 0; i < n; i++) b[i] = a[i]; }
static void to_dbl(const real* a, double* b, int n) { for (int i = 0; i < n; i++) b[i] = (double)a[i]; }

int orc_euler_flux(const double* U, const double* n, double gamma, double* F) {
  real u[5], nn[3], f[5];
  to_real(U, u, 5); to_real(n, nn, 3);
  euler_flux(u, nn, gamma, f);
  to_dbl(f, F, 5);
  return 0;
}
int orc_two_point_ec(const double* UL, const double* UR, const double* n, double gamma, double* F) {
  real a[5], b[5], nn[3], f[5];
  to_real(UL, a, 5); to_real(UR, b, 5); to_real(n, nn, 3);
  two_point_ec(a, b, nn, gamma, f);
  to_dbl(f, F, 5);
  return 0;
}
int orc_two_point_ir(const double* UL, const double* UR, const double* n, double gamma, double* F) {
  real a[5], b[5], nn[3], f[5];
  to_real(UL, a, 5); to_real(UR, b, 5); to_real(n, nn, 3);
  two_point_ir(a, b, nn, gamma, f);
  to_dbl(f, F, 5);
  return 0;
}
int orc_two_point_central(const double* UL, const double* UR, const double* n, double gamma, double* F) {
  real a[5], b[5], nn[3], f[5];
  to_real(UL, a, 5); to_real(UR, b, 5); to_real(n, nn, 3);
  two_point_central(a, b, nn, gamma, f);
  to_dbl(f, F, 5);
  return 0;
}
/* Gauss-Legendre meshes: the broken gradient Gb and the sum Gl of the six face lifts of 7c at
 * every node (layout of orc_gradients); Gb + Gl is the BR1 gradient of 7b */
int orc_gauss_gradient_parts(const orc_solver* s, double* Gb, double* Gl) {
  if (!s || !s->gauss) return -1;
  for (int e = 0; e < s->E; e++) {
    const int N = s->N[e][0], n = N + 1, nn = n * n * n;
    for (int k = 0; k < n; k++)
      for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
          int ii[3] = {i, j, k};
          long q = node_of(s, e, ii);
          real gb[12], gl[12] = {0};
          gauss_broken_gradient(s, s->U, e, ii, gb);
          for (int d = 0; d < 3; d++) {
            int ta, tb;
            face_dirs(d, &ta, &tb);
            for (int side = 0; side < 2; side++) {
              real jump[4];
              gauss_face_jump(s, s->U, e, d, side, ii[ta], ii[tb], jump);
              gauss_add_lift(s, e, ii, d, side, jump, 1, gl);
            }
          }
          for (int t = 0; t < 12; t++) {
            Gb[s->off[e] * 12 + (long)t * nn + q] = (double)gb[t];
            Gl[s->off[e] * 12 + (long)t * nn + q] = (double)gl[t];
          }
        }
  }
  return 0;
}

/* Gauss-Legendre Navier-Stokes meshes: the face viscous flux of the current state on every face
 * of every element, F[((e * 6 + f) * 5 + v) * nf + q] for face f = 2 d + side and face point
 * q = p + n r (the flux along the owner's scaled normal; both elements of a face hold the same) */
int orc_gauss_face_viscous(orc_solver* s, double* F) {
  if (!s || !s->gauss || !s->viscous) return -1;
  compute_gradients_gauss(s, s->U, s->G);
  for (int e = 0; e < s->E; e++) {
    const int n = s->N[e][0] + 1, nf = n * n;
    for (int d = 0; d < 3; d++)
      for (int side = 0; side < 2; side++) {
        int L = side ? e : s->nbr[6 * e + 2 * d];
        int Rr = s->nbr[6 * L + 2 * d + 1];
        for (int r = 0; r < n; r++)
          for (int p = 0; p < n; p++) {
            real uL[5], uR[5], S[3], Fst[5];
            gauss_face_state(s, s->U, L, Rr, d, p, r, uL, uR, S);
            gauss_face_viscous(s, s->U, s->G, L, Rr, d, p, r, uL, uR, S, Fst);
            for (int v = 0; v < 5; v++) F[(((long)e * 6 + 2 * d + side) * 5 + v) * nf + p + n * r] = (double)Fst[v];
          }
      }
  }
  return 0;
}

int orc_set_viscous_flux(orc_solver* s, int kind, double eta) {
  if (!s || kind < ORC_VISC_BR1 || kind > ORC_VISC_IP || !(eta >= 0)) return -1;
  s->visc_flux = kind;
  s->visc_eta = eta > 0 ? (real)eta : (kind == ORC_VISC_BR2 ? 2 : 1);
  return 0;
}
int orc_two_point(int vol_kind, const double* UL, const double* UR, const double* n, double gamma, double* F) {
  if (vol_kind < 0 || vol_kind > ORC_VOL_MORINISHI) return -1;
  real a[5], b[5], nn[3], f[5];
  to_real(UL, a, 5); to_real(UR, b, 5); to_real(n, nn, 3);
  if (vol_kind == ORC_VOL_EC) two_point_ec(a, b, nn, gamma, f);
  else if (vol_kind == ORC_VOL_IR) two_point_ir(a, b, nn, gamma, f);
  else if (vol_kind == ORC_VOL_CENTRAL) two_point_central(a, b, nn, gamma, f);
  else two_point_kep(vol_kind, a, b, nn, gamma, f);
  to_dbl(f, F, 5);
  return 0;
}
int orc_lax_friedrichs(const double* UL, const double* UR, const double* S, double gamma, double lam, double* F) {
  real a[5], b[5], nn[3], f[5];
  to_real(UL, a, 5); to_real(UR, b, 5); to_real(S, nn, 3);
  lax_friedrichs(a, b, nn, gamma, lam, f);
  to_dbl(f, F, 5);
  return 0;
}
int orc_riemann(int kind, const double* UL, const double* UR, const double* S, double gamma, double* F) {
  if (kind < 0 || kind > ORC_SURF_LOW_DISS_ROE) return -1;
  real a[5], b[5], nn[3], f[5];
  to_real(UL, a, 5); to_real(UR, b, 5); to_real(S, nn, 3);
  riemann(kind, a, b, nn, gamma, f);
  to_dbl(f, F, 5);
  return 0;
}
int orc_roe_waves(const double* UL, const double* UR, const double* nhat, double gamma, int absval, double* W) {
  real a[5], b[5], nn[3], f[5];
  to_real(UL, a, 5); to_real(UR, b, 5); to_real(nhat, nn, 3);
  roe_waves(a, b, nn, gamma, absval, f);
  to_dbl(f, W, 5);
  return 0;
}
int orc_entropy_vars(const double* U, double gamma, double* wout) {
  real u[5], w[5];
  to_real(U, u, 5);
  entropy_vars(u, gamma, w);
  to_dbl(w, wout, 5);
  return 0;
}
double orc_entropy(const double* U, double gamma) {
  real u[5];
  to_real(U, u, 5);
  prim_t w = prim(u, gamma);
  real sp = RLOG(w.p) - (real)gamma * RLOG(w.rho);
  return (double)(-w.rho * sp / ((real)gamma - 1));
}
double orc_logmean(double a, double b) { return (double)logmean(a, b); }
int orc_viscous_flux(const double* U, const double* grad, double gamma, double Pr, double Re, double* Fv) {
  real u[5], g[12], f[15];
  to_real(U, u, 5); to_real(grad, g, 12);
  real mu = (real)1 / (real)Re;
  real kappa = mu * (real)gamma / (((real)gamma - 1) * (real)Pr);
  viscous_flux(u, g, gamma, mu, kappa, f);
  to_dbl(f, Fv, 15);
  return 0;
}

/* ------------------------------------------------------------------------------------------
 * 13. Spectral vanishing viscosity (section 8c) exports.
 * ---------------------------------------------------------------------------------------- */
int orc_set_svv(orc_solver* s, double mu_a, int kernel, int cutoff, double sensor_threshold) {
  if (!s || s->gauss || !(mu_a >= 0) || kernel < ORC_SVV_TADMOR || kernel > ORC_SVV_MADAY) return -1;
  if (mu_a == 0 && !(s->les_cs > 0)) { s->svv = 0; return 0; }
  for (int e = 0; e < s->E; e++)
    for (int d = 0; d < 3; d++) {
      if (cutoff < -1 || cutoff > s->N[e][d]) return -1;
      int r = s->nbr[6 * e + 2 * d + 1];
      for (int t = 0; t < 3; t++)
        if (t != d && s->N[e][t] != s->N[r][t]) return -1;  /* conforming faces only */
    }
  if (!s->Gw) s->Gw = (real*)calloc(15 * s->ntot, sizeof(real));
  if (!s->Fa) s->Fa = (real*)calloc(15 * s->ntot, sizeof(real));
  if (!s->Gw || !s->Fa) return -1;
  s->svv = 1;
  s->svv_mu = mu_a;
  s->svv_kappa = s->svv_mu * s->gamma / ((s->gamma - 1) * s->Pr);
  s->svv_kernel = kernel;
  s->svv_cut = cutoff;
  s->svv_sensor = sensor_threshold;
  return 0;
}

/* the explicit LES closure: model (ORC_LES_*) and its constant cs (0 = off); call before
 * orc_set_svv, which then sets the filter (and may take mu_a = 0) */
int orc_set_les(orc_solver* s, int model, double cs) {
  if (!s || s->gauss || !(cs >= 0) || !isfinite(cs) || model < ORC_LES_SMAGORINSKY || model > ORC_LES_VREMAN)
    return -1;
  s->les_cs = cs;
  s->les_model = model;
  return 0;
}

/* the eddy viscosity rho nu_t of the explicit LES closure at one state: U the conservative state,
 * Gw[3c+x] the entropy-variable gradient, model and constant, J the Jacobian and n the element's
 * node count */
int orc_les_viscosity(const double* U, const double* Gw, double gamma, int model, double cs, double J, int n,
                      double* mu) {
  if (!U || !Gw || !mu || n < 1 || !(J > 0) || model < ORC_LES_SMAGORINSKY || model > ORC_LES_VREMAN) return -1;
  real u[5], G[15];
  to_real(U, u, 5);
  to_real(Gw, G, 15);
  *mu = (double)les_viscosity(u, G, gamma, model, cs, J, n);
  return 0;
}

/* the artificial-viscosity part of the residual of the current state; *form (if given) receives
 * sum_m <y_m, F* y_m> over the elements */
int orc_svv_residual(orc_solver* s, double* Ra, double* form) {
  if (!s || !s->svv) return -1;
  real* R = (real*)calloc(5 * s->ntot, sizeof(real));
  if (!R) return -1;
  real f = svv_residual(s, s->U, R);
  for (long i = 0; i < 5 * s->ntot; i++) Ra[i] = (double)R[i];
  if (form) *form = (double)f;
  free(R);
  return 0;
}

int orc_svv_sensor(orc_solver* s, double* sens) {
  if (!s) return -1;
  for (int e = 0; e < s->E; e++) sens[e] = (double)svv_sensor(s, s->U, e);
  return 0;
}

int orc_svv_filter(int N, int kernel, int cutoff, const double* f, double* out) {
  if (N < 1 || N > ORC_NMAX || cutoff < -1 || cutoff > N || kernel < ORC_SVV_TADMOR || kernel > ORC_SVV_MADAY)
    return -1;
  gll_init();
  int n = N + 1, nn = n * n * n, Ns[3] = {N, N, N};
  real* a = (real*)malloc(sizeof(real) * 2 * nn);
  to_real(f, a, nn);
  svv_filter_field(Ns, kernel, cutoff, a, a + nn);
  to_dbl(a + nn, out, nn);
  free(a);
  return 0;
}

/* the unfiltered flux L^T D L G at one state, G[3c+x] = d w_c / d x_x; F[5x+v]; with cs > 0 the
 * viscosity gains Smagorinsky's at Jacobian J in an element of n nodes */
int orc_les_flux(const double* U, const double* Gw, double gamma, double Pr, double mu_a, int model, double cs,
                 double J, int n, double* F) {
  if (n < 1 || !(J > 0) || model < ORC_LES_SMAGORINSKY || model > ORC_LES_VREMAN) return -1;
  real u[5], G[15], L[8][15], D[8];
  to_real(U, u, 5);
  to_real(Gw, G, 15);
  svv_node_factors(u, G, gamma, Pr, mu_a, model, cs, J, n, L, D);
  for (int x = 0; x < 3; x++)
    for (int c = 0; c < 5; c++) {
      real acc = 0;
      for (int m = 0; m < 8; m++) {
        real lg = 0;
        for (int t = 0; t < 15; t++) lg += L[m][t] * G[t];
        acc += L[m][3 * c + x] * D[m] * lg;
      }
      F[5 * x + c] = (double)acc;
    }
  return 0;
}

int orc_svv_flux(const double* U, const double* Gw, double gamma, double Pr, double mu_a, double* F) {
  return orc_les_flux(U, Gw, gamma, Pr, mu_a, ORC_LES_SMAGORINSKY, 0.0, 1.0, 1, F);
}
