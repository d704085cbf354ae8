// kernels_gauss.hip -- DGSEM on Gauss-Legendre nodes, the other quadrature that section "Spatial
// discretisation" allows: the plain weak form (no boundary nodes, so no split form), with BR1,
// BR2 or interior-penalty viscous terms for Navier-Stokes, on uniform-order boxes (undeformed or
// deformed), FP64.
//
// Two launches per RK stage (three with viscosity: gauss_grad_kernel between them).
// gauss_trace_kernel interpolates each element's state to its six
// faces, U(+-1) = sum_i l_i(+-1) U_i along the line through every face point, into
// Tr[E][6][5][nf].  gauss_stage_kernel then forms, per node,
//   J dU_i/dt = -[ sum_d sum_m Dw_im F~^d_m + sum_d (l_i(+1) F*(+d) - l_i(-1) F*(-d)) / w_i ],
// Dw_im = -D_mi w_m / w_i (the quadrature of the weak derivative), F~^d = Ja^d . F(U) at the
// nodes, and F* the numerical flux between the element's own trace and its neighbour's, both
// read from Tr, oriented along +xi_d with the owner's metric (the element on the -xi_d side)
// interpolated to the face point as the scaled normal (Sf, formed with the geometry), so both
// elements evaluate the same flux from the same values.  Every node of a line receives the lift of both of the
// line's face fluxes (l_i(+-1) != 0 for all i), unlike the Lobatto form.
#include <hip/hip_runtime.h>

#include "dg_device.h"

namespace dg {

// the Lobatto Dhat slot of the order's table holds l_j(-1) (n values), then l_j(+1)
__host__ __device__ constexpr int gauss_tab_ends(int n) { return 2 * n + n * n; }

// Static face factors of the element's six faces, formed once after the geometry: the trace of J,
// Jt[E][6][nf] (the interior penalty's element sizes), or the traced metric factor of the face's
// BR2 lift, Mt[E][6][3][nf] = sum_i l_i(side) (+-l_i(side) / w_i) Ja^d_i / J_i
template <int N>
__global__ void __launch_bounds__(nthreads_for(N)) gauss_jtrace_kernel(View v) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n, NT = nthreads_for(N);
  const int e = block_element(v.E);
  const int t = threadIdx.x;
  const long base = (long)e * nn;
  __shared__ double sl[2][n], sw[n];
  if (t < 2 * n) sl[t / n][t % n] = v.tab[gauss_tab_ends(n) + t];
  if (t < n) sw[t] = v.tab[n + t];
  __syncthreads();
  for (int x = t; x < 6 * nf; x += NT) {
    const int f = x / nf, q = x - f * nf;
    const int d = f >> 1, side = f & 1;
    const int p = q % n, r = q / n;
    double acc = 0.0, M[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < n; i++) {
      const int node = face_node<n>(d, i, p, r);
      const double l = sl[side][i];
      if (v.Jt) acc += l * v.J[base + node];
      if (v.Mt) {
        const double wl = (side ? l : -l) * l / sw[i] * v.invJ[base + node];
#pragma unroll
        for (int y = 0; y < 3; y++) M[y] += wl * v.Ja[base * 9 + (3 * d + y) * nn + node];
      }
    }
    if (v.Jt) v.Jt[((long)e * 6 + f) * nf + q] = acc;
    if (v.Mt) {
#pragma unroll
      for (int y = 0; y < 3; y++) v.Mt[(((long)e * 6 + f) * 3 + y) * nf + q] = M[y];
    }
  }
}

template <int N>
__global__ void __launch_bounds__(nthreads_for(N)) gauss_trace_kernel(View v, int cur) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n, NT = nthreads_for(N);
  const int e = block_element(v.E);
  const int t = threadIdx.x;
  __shared__ double sU[5][nn];
  __shared__ double sl[2][n];
  const double* __restrict__ U = v.U[cur] + (long)e * 5 * nn;
  for (int x = t; x < 5 * nn; x += NT) sU[x / nn][x % nn] = U[x];
  if (t < 2 * n) sl[t / n][t % n] = v.tab[gauss_tab_ends(n) + t];
  __syncthreads();
  double* __restrict__ Tr = v.Tr + (long)e * 6 * 5 * nf;
  for (int x = t; x < 6 * nf; x += NT) {
    const int f = x / nf, q = x - f * nf;
    const int d = f >> 1, side = f & 1;
    const int p = q % n, r = q / n;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < n; i++) {
      const int node = face_node<n>(d, i, p, r);
      const double l = sl[side][i];
#pragma unroll
      for (int c = 0; c < 5; c++) acc[c] += l * sU[c][node];
    }
#pragma unroll
    for (int c = 0; c < 5; c++) Tr[(f * 5 + c) * nf + q] = acc[c];
  }
}

// Viscous face fluxes on Gauss points (Navier-Stokes), XV = 0 BR1, 1 BR2, 2 interior penalty.
// BR1's gradient of g = (v, T) is the weak form with the face values g* = (g(U_L) + g(U_R)) / 2
// of both sides' traces,
//   J grad g = sum_d Ja^d [ sum_m Dw_im g_m + (l_i(+1) g*(+d) - l_i(-1) g*(-d)) / w_i ]
// (the node's metric outside the weak derivative, as in the Lobatto BR1 gradient).  Gauss
// quadrature integrates that weak derivative exactly, so it equals the broken (strong) derivative
// sum_m D_im g_m plus, per face, the lift of g* - g(+-1), g(+-1) = sum_j l_j(+-1) g_j.  On each
// of the six faces the kernel writes this side's contravariant viscous flux F_v(U trace, face
// gradient) . S with the owner's face metric S (Sf) into Fvf[E][6][4][nf]; the stage kernel
// averages the two sides and forms the BR1 gradient again for its volume term.  The face gradient
// is the trace of the BR1 gradient (BR1), the trace of the broken gradient plus eta times the
// trace of this face's lift (BR2), or the trace of the broken gradient (interior penalty, whose
// penalty sigma F_v(v_mean, [g] n^) . S, sigma = eta (N+1)^2 |S| / (2 min(J_L, J_R)), with g of
// both traces of U and J_L, J_R the two traces of J, each side adds to its flux, so the average
// holds it once; both sides evaluate it from the same values in the same order).
template <int N, int XV>
__global__ void __launch_bounds__(nthreads_for(N)) gauss_grad_kernel(View v, int cur) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n, NT = nthreads_for(N);
  const int e = block_element(v.E);
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int ti = t % n, tj = (t / n) % n, tk = t / nf;
  __shared__ double sDw[n * n], sw[n], sl[2][n];
  __shared__ double sG[4][nn];
  __shared__ double sGs[6][4][nf];  // face values g*
  __shared__ double sQ[12][nn];     // BR1: the gradient; BR2, IP: the broken gradient
  // interior penalty: [g] = g(plus side) - g(minus side) of the two traces of U
  __shared__ double sGd[XV == 2 ? 6 : 1][4][XV == 2 ? nf : 1];
  for (int x = t; x < n * n; x += NT) {
    const int i = x / n, m = x - i * n;
    // BR1: the weak derivative matrix Dw; BR2, IP: the derivative matrix D itself
    sDw[x] = XV == 0 ? -v.tab[2 * n + m * n + i] * v.tab[n + m] / v.tab[n + i] : v.tab[2 * n + x];
  }
  if (t < n) sw[t] = v.tab[n + t];
  if (t < 2 * n) sl[t / n][t % n] = v.tab[gauss_tab_ends(n) + t];
  const long base = (long)e * nn;
  const double* __restrict__ Uin = v.U[cur];
  if (act) {
    double u[5], g[4];
#pragma unroll
    for (int c = 0; c < 5; c++) u[c] = Uin[base * 5 + c * nn + t];
    gvars(u, v.gamma, 0.0, g);
#pragma unroll
    for (int c = 0; c < 4; c++) sG[c][t] = g[c];
  }
  for (int x = t; x < 6 * nf; x += NT) {
    const int f = x / nf, q = x - f * nf;
    const int ne = v.nbr[e * 6 + f];
    const double* To = v.Tr + ((long)e * 6 + f) * 5 * nf;
    const double* Tn = v.Tr + ((long)ne * 6 + (f ^ 1)) * 5 * nf;
    double uo[5], un[5], go[4], gn[4];
#pragma unroll
    for (int c = 0; c < 5; c++) {
      uo[c] = To[c * nf + q];
      un[c] = Tn[c * nf + q];
    }
    gvars(uo, v.gamma, 0.0, go);
    gvars(un, v.gamma, 0.0, gn);
#pragma unroll
    for (int c = 0; c < 4; c++) sGs[f][c][q] = 0.5 * (go[c] + gn[c]);
    if (XV == 2) {
      const bool plus = f & 1;  // this element is the face's minus side: the neighbour is plus
#pragma unroll
      for (int c = 0; c < 4; c++) sGd[XV == 2 ? f : 0][c][XV == 2 ? q : 0] = plus ? gn[c] - go[c] : go[c] - gn[c];
    }
  }
  __syncthreads();
  if (act) {
    const int ii[3] = {ti, tj, tk};
    double a[3][4];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const int id = ii[d];
      const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
      const int b0 = t - id * stride;
      const int qd = d == 0 ? tj + n * tk : (d == 1 ? ti + n * tk : ti + n * tj);
      const double lp = sl[1][id] / sw[id], lm = sl[0][id] / sw[id];
#pragma unroll
      for (int c = 0; c < 4; c++) {
        double acc = XV == 0 ? lp * sGs[2 * d + 1][c][qd] - lm * sGs[2 * d][c][qd] : 0.0;
#pragma unroll
        for (int m = 0; m < n; m++) acc += sDw[id * n + m] * sG[c][b0 + m * stride];
        a[d][c] = acc;
      }
    }
    double ja[9];
#pragma unroll
    for (int c = 0; c < 9; c++) ja[c] = v.Ja[base * 9 + c * nn + t];
    const double ij = v.invJ[base + t];
#pragma unroll
    for (int c = 0; c < 4; c++)
#pragma unroll
      for (int x = 0; x < 3; x++) {
        sQ[3 * c + x][t] = ij * (ja[x] * a[0][c] + ja[3 + x] * a[1][c] + ja[6 + x] * a[2][c]);
      }
  }
  __syncthreads();
  double* __restrict__ Fvf = v.Fvf + (long)e * 6 * 4 * nf;
  for (int x = t; x < 6 * nf; x += NT) {
    const int f = x / nf, q = x - f * nf;
    const int d = f >> 1, side = f & 1;
    const int p = q % n, r = q / n;
    const long ne = v.nbr[e * 6 + f];
    const long owner = side ? e : ne;
    const double* So = v.Sf + (owner * 9 + 3 * d) * nf;
    const double s1 = So[q], s2 = So[nf + q], s3 = So[2 * nf + q];
    // the scheme's own face terms first, so that their operands are retired before the twelve
    // gradient traces are formed
    double Fo[4] = {0.0, 0.0, 0.0, 0.0}, jump[4], M[3] = {0.0, 0.0, 0.0};
    if (XV == 1) {  // BR2: the jump g* - g(side) and the traced metric factor of its lift (Mt)
#pragma unroll
      for (int c = 0; c < 4; c++) jump[c] = sGs[f][c][q];
#pragma unroll 1
      for (int i = 0; i < n; i++) {
        const int node = face_node<n>(d, i, p, r);
        const double l = sl[side][i];
#pragma unroll
        for (int c = 0; c < 4; c++) jump[c] -= l * sG[c][node];
      }
    }
    if (XV == 2) {  // interior penalty, from the face's minus (L) and plus (R) sides
      const long eL = side ? e : ne, eR = side ? ne : e;
      const double JL = v.Jt[(eL * 6 + 2 * d + 1) * nf + q], JR = v.Jt[(eR * 6 + 2 * d) * nf + q];
      const double area = sqrt(s1 * s1 + s2 * s2 + s3 * s3);
      const double sigma = v.visc_eta * (double)(n * n) * area / (2.0 * (JL < JR ? JL : JR));
      const double nh[3] = {s1 / area, s2 / area, s3 / area};
      double gp[4][3], Fp[3][4];
#pragma unroll
      for (int c = 0; c < 4; c++)
#pragma unroll
        for (int y = 0; y < 3; y++) gp[c][y] = sigma * sGd[XV == 2 ? f : 0][c][XV == 2 ? q : 0] * nh[y];
      // the mean velocity: g* (the same sum of the same two values on both sides)
      viscous_flux_g(sGs[f][0][q], sGs[f][1][q], sGs[f][2][q], gp, v.mu, v.kappa, Fp);
#pragma unroll
      for (int c = 0; c < 4; c++) Fo[c] = s1 * Fp[0][c] + s2 * Fp[1][c] + s3 * Fp[2][c];
    }
    double gr[4][3];
#pragma unroll
    for (int k = 0; k < 12; k++) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < n; i++) acc += sl[side][i] * sQ[k][face_node<n>(d, i, p, r)];
      gr[k / 3][k % 3] = acc;
    }
    if (XV == 1) {  // + eta times the trace of this face's lift
#pragma unroll
      for (int y = 0; y < 3; y++) M[y] = v.Mt[(((long)e * 6 + f) * 3 + y) * nf + q];
#pragma unroll
      for (int c = 0; c < 4; c++)
#pragma unroll
        for (int y = 0; y < 3; y++) gr[c][y] += v.visc_eta * M[y] * jump[c];
    }
    const double* To = v.Tr + ((long)e * 6 + f) * 5 * nf;
    double uo[5], go[4];
#pragma unroll
    for (int c = 0; c < 5; c++) uo[c] = To[c * nf + q];
    gvars(uo, v.gamma, 0.0, go);
    double Fv[3][4];
    viscous_flux_g(go[0], go[1], go[2], gr, v.mu, v.kappa, Fv);
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const double own = s1 * Fv[0][c] + s2 * Fv[1][c] + s3 * Fv[2][c];
      Fvf[(f * 4 + c) * nf + q] = XV == 2 ? own + Fo[c] : own;
    }
  }
}

// Euler flux of the conservative state u along the (not normalised) vector s
__device__ __forceinline__ void euler_flux_along(const double u[5], double gamma, double s1, double s2, double s3,
                                                 double F[5]) {
  const double i = 1.0 / u[0];
  const double v1 = u[1] * i, v2 = u[2] * i, v3 = u[3] * i;
  const double p = (gamma - 1.0) * (u[4] - 0.5 * u[0] * (v1 * v1 + v2 * v2 + v3 * v3));
  const double vn = v1 * s1 + v2 * s2 + v3 * s3;
  F[0] = u[0] * vn;
  F[1] = u[1] * vn + p * s1;
  F[2] = u[2] * vn + p * s2;
  F[3] = u[3] * vn + p * s3;
  F[4] = (u[4] + p) * vn;
}

// XS: the extended surface fluxes (codes >= 4), compiled apart; VISC: the BR1 viscous terms
// (gradients and face viscous fluxes from gauss_grad_kernel), entering with the opposite sign
template <int N, bool XS, bool VISC>
__global__ void __launch_bounds__(nthreads_for(N))
    gauss_stage_kernel(View v, int cur, double dt, double rkA, double rkB, int mode) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n, NT = nthreads_for(N);
  const int e = block_element(v.E);
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int ti = t % n, tj = (t / n) % n, tk = t / nf;
  __shared__ double sDw[n * n], sw[n], sl[2][n];
  __shared__ double sF[5][nn];      // contravariant flux of one direction
  __shared__ double sFs[6][5][nf];  // numerical flux on the six faces
  // Navier-Stokes: g = (v, T) at the nodes and the face values g* = average of the two sides'
  // traces, for the BR1 gradient (formed here as in gauss_grad_kernel, not stored)
  constexpr int nnV = VISC ? nn : 1, nfV = VISC ? nf : 1;
  __shared__ double sG[4][nnV];
  __shared__ double sGs[6][4][nfV];
  for (int x = t; x < n * n; x += NT) {
    const int i = x / n, m = x - i * n;
    sDw[x] = -v.tab[2 * n + m * n + i] * v.tab[n + m] / v.tab[n + i];
  }
  if (t < n) sw[t] = v.tab[n + t];
  if (t < 2 * n) sl[t / n][t % n] = v.tab[gauss_tab_ends(n) + t];
  const long base = (long)e * nn;
  const double* __restrict__ Uin = v.U[cur];
  // numerical fluxes on the faces, from the traces of both sides (the node's own data is loaded
  // after this phase, so that the two phases' registers do not add up)
  for (int x = t; x < 6 * nf; x += NT) {
    const int f = x / nf, q = x - f * nf;
    const int d = f >> 1, side = f & 1;
    const int ne = v.nbr[e * 6 + f];
    const double* To = v.Tr + ((long)e * 6 + f) * 5 * nf;
    const double* Tn = v.Tr + ((long)ne * 6 + (f ^ 1)) * 5 * nf;
    double uL[5], uR[5], S[3];
#pragma unroll
    for (int c = 0; c < 5; c++) {
      const double a = To[c * nf + q], b = Tn[c * nf + q];
      uL[c] = side ? a : b;
      uR[c] = side ? b : a;
    }
    const long owner = side ? e : ne;
#pragma unroll
    for (int c = 0; c < 3; c++) S[c] = v.Sf[(owner * 9 + 3 * d + c) * nf + q];
    if (VISC) {
      double go[4], gn[4];
      gvars(side ? uL : uR, v.gamma, 0.0, go);
      gvars(side ? uR : uL, v.gamma, 0.0, gn);
#pragma unroll
      for (int c = 0; c < 4; c++) sGs[f][c][q] = 0.5 * (go[c] + gn[c]);
    }
    double F[5];
    face_flux<double, XS>(v.surf, uL, uR, S, v.gamma, F, XS && v.surf == 8 ? v.adapt[3] : 0.0);
    if (VISC) {
      const double* fo = v.Fvf + ((long)e * 6 + f) * 4 * nf;
      const double* fn = v.Fvf + ((long)ne * 6 + (f ^ 1)) * 4 * nf;
#pragma unroll
      for (int c = 0; c < 4; c++) F[1 + c] -= 0.5 * (fo[c * nf + q] + fn[c * nf + q]);
    }
#pragma unroll
    for (int c = 0; c < 5; c++) sFs[f][c][q] = F[c];
  }
  double u[5], ja[9], ij = 0.0, Fv[3][4];  // Fv: physical viscous flux along x (momentum, energy)
  double gv[4] = {0.0, 0.0, 0.0, 0.0};
  if (act) {
#pragma unroll
    for (int c = 0; c < 5; c++) u[c] = Uin[base * 5 + c * nn + t];
#pragma unroll
    for (int c = 0; c < 9; c++) ja[c] = v.Ja[base * 9 + c * nn + t];
    ij = v.invJ[base + t];
    if (VISC) {
      gvars(u, v.gamma, 0.0, gv);
#pragma unroll
      for (int c = 0; c < 4; c++) sG[c][t] = gv[c];
    }
  }
  if (VISC) {
    __syncthreads();  // g and g* of the element staged
    if (act) {  // BR1 gradient (weak form) and the viscous flux of this node
      const int ii[3] = {ti, tj, tk};
      double a[3][4];
#pragma unroll
      for (int d = 0; d < 3; d++) {
        const int id = ii[d];
        const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
        const int b0 = t - id * stride;
        const int qd = d == 0 ? tj + n * tk : (d == 1 ? ti + n * tk : ti + n * tj);
        const double lp = sl[1][id] / sw[id], lm = sl[0][id] / sw[id];
#pragma unroll
        for (int c = 0; c < 4; c++) {
          double acc = lp * sGs[2 * d + 1][c][qd] - lm * sGs[2 * d][c][qd];
#pragma unroll
          for (int m = 0; m < n; m++) acc += sDw[id * n + m] * sG[c][b0 + m * stride];
          a[d][c] = acc;
        }
      }
      double gr[4][3];
#pragma unroll
      for (int c = 0; c < 4; c++)
#pragma unroll
        for (int x = 0; x < 3; x++) gr[c][x] = ij * (ja[x] * a[0][c] + ja[3 + x] * a[1][c] + ja[6 + x] * a[2][c]);
      viscous_flux_g(gv[0], gv[1], gv[2], gr, v.mu, v.kappa, Fv);
    }
  }
  // volume: sum_m Dw_im F~^d_m along each direction's line
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int ii[3] = {ti, tj, tk};
#pragma unroll
  for (int d = 0; d < 3; d++) {
    __syncthreads();  // sF free again (and, at d = 0, the tables staged)
    if (act) {
      double F[5];
      euler_flux_along(u, v.gamma, ja[3 * d], ja[3 * d + 1], ja[3 * d + 2], F);
      if (VISC) {
#pragma unroll
        for (int c = 0; c < 4; c++) F[1 + c] -= ja[3 * d] * Fv[0][c] + ja[3 * d + 1] * Fv[1][c] + ja[3 * d + 2] * Fv[2][c];
      }
#pragma unroll
      for (int c = 0; c < 5; c++) sF[c][t] = F[c];
    }
    __syncthreads();
    if (act) {
      const int id = ii[d];
      const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
      const int b0 = t - id * stride;
#pragma unroll
      for (int m = 0; m < n; m++) {
        const double Dm = sDw[id * n + m];
#pragma unroll
        for (int c = 0; c < 5; c++) acc[c] += Dm * sF[c][b0 + m * stride];
      }
    }
  }
  if (!act) return;
  // lift of the two face fluxes of each of the node's lines
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const int id = ii[d];
    const int qd = d == 0 ? tj + n * tk : (d == 1 ? ti + n * tk : ti + n * tj);
    const double lp = sl[1][id] / sw[id], lm = sl[0][id] / sw[id];
#pragma unroll
    for (int c = 0; c < 5; c++) acc[c] += lp * sFs[2 * d + 1][c][qd] - lm * sFs[2 * d][c][qd];
  }
  const long o = base * 5 + t;
  if (mode == kModeResidual) {
#pragma unroll
    for (int c = 0; c < 5; c++) v.R[o + c * nn] = -acc[c] * ij;
    return;
  }
  const double h = v.dtp ? *v.dtp : dt;
  double* __restrict__ Uout = v.U[cur ^ 1];
#pragma unroll
  for (int c = 0; c < 5; c++) {
    const double du = (rkA == 0.0 ? 0.0 : rkA * v.dU[o + c * nn]) + h * (-acc[c] * ij);
    v.dU[o + c * nn] = du;
    Uout[o + c * nn] = Uin[o + c * nn] + rkB * du;
  }
}

template <int N>
static hipError_t gauss_stage_n(const View& v, int cur, double dt, double a, double b, int mode, hipStream_t st) {
  const dim3 grid(v.E), block(nthreads_for(N));
  hipLaunchKernelGGL(gauss_trace_kernel<N>, grid, block, 0, st, v, cur);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if (v.viscous) {
    if (v.visc_flux == 1)
      hipLaunchKernelGGL((gauss_grad_kernel<N, 1>), grid, block, 0, st, v, cur);
    else if (v.visc_flux == 2)
      hipLaunchKernelGGL((gauss_grad_kernel<N, 2>), grid, block, 0, st, v, cur);
    else
      hipLaunchKernelGGL((gauss_grad_kernel<N, 0>), grid, block, 0, st, v, cur);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (v.surf >= 4)
      hipLaunchKernelGGL((gauss_stage_kernel<N, true, true>), grid, block, 0, st, v, cur, dt, a, b, mode);
    else
      hipLaunchKernelGGL((gauss_stage_kernel<N, false, true>), grid, block, 0, st, v, cur, dt, a, b, mode);
  } else if (v.surf >= 4) {
    hipLaunchKernelGGL((gauss_stage_kernel<N, true, false>), grid, block, 0, st, v, cur, dt, a, b, mode);
  } else {
    hipLaunchKernelGGL((gauss_stage_kernel<N, false, false>), grid, block, 0, st, v, cur, dt, a, b, mode);
  }
  return hipGetLastError();
}

template <int N>
static hipError_t gauss_jtrace_n(const View& v, hipStream_t st) {
  hipLaunchKernelGGL(gauss_jtrace_kernel<N>, dim3(v.E), dim3(nthreads_for(N)), 0, st, v);
  return hipGetLastError();
}

hipError_t launch_jtrace_gauss(const View& v, hipStream_t st) {
  if (!v.gauss || (!v.Jt && !v.Mt) || v.E <= 0) return hipErrorInvalidValue;
  switch (v.N) {
    case 1: return gauss_jtrace_n<1>(v, st);
    case 2: return gauss_jtrace_n<2>(v, st);
    case 3: return gauss_jtrace_n<3>(v, st);
    case 4: return gauss_jtrace_n<4>(v, st);
    case 5: return gauss_jtrace_n<5>(v, st);
    case 6: return gauss_jtrace_n<6>(v, st);
    case 7: return gauss_jtrace_n<7>(v, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stage_gauss(const View& v, int cur, double dt, double rkA, double rkB, int mode, hipStream_t st) {
  if (!v.gauss || !v.Tr) return hipErrorInvalidValue;
  if (v.viscous && v.visc_flux == 2 && !v.Jt) return hipErrorInvalidValue;  // the penalty's traces of J
  if (v.viscous && v.visc_flux == 1 && !v.Mt) return hipErrorInvalidValue;  // BR2's lift factors
  switch (v.N) {
    case 1: return gauss_stage_n<1>(v, cur, dt, rkA, rkB, mode, st);
    case 2: return gauss_stage_n<2>(v, cur, dt, rkA, rkB, mode, st);
    case 3: return gauss_stage_n<3>(v, cur, dt, rkA, rkB, mode, st);
    case 4: return gauss_stage_n<4>(v, cur, dt, rkA, rkB, mode, st);
    case 5: return gauss_stage_n<5>(v, cur, dt, rkA, rkB, mode, st);
    case 6: return gauss_stage_n<6>(v, cur, dt, rkA, rkB, mode, st);
    case 7: return gauss_stage_n<7>(v, cur, dt, rkA, rkB, mode, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dg
