// kernels.hip -- gfx950 kernels of the DGSEM residual and low-storage RK3.
//
// One workgroup per hexahedral element, one lane per Gauss-Lobatto node (64-wide waves; the
// (N+1)^3 nodes are padded to a multiple of 64).  The element's state, primitive variables
// and metric terms are staged in LDS; the split-form two-point fluxes run on the VALU.  The
// numerical flux on each face is evaluated by both adjacent elements, with identical
// arguments in identical order (owner's +xi_d side first, the owner's metric as normal), so
// the flux is single-valued without a face array or a grid-wide barrier; the state
// ping-pongs between two buffers so that the neighbour traces read in a stage are never
// overwritten during it.  Workgroups are mapped to elements so that each of the 8 XCDs works
// on a contiguous range of elements (neighbour traces then mostly hit that XCD's L2).
//
// Discretisation (HORSES3D paper, arXiv 2206.09733): eqs. compressibleNScompact,
// viscousfluxes, compressibleNScompact_transformed and NS2-NS5; split forms of section
// "Energy/Entropy stable versions"; Riemann and BR1 fluxes listed in section "Spatial
// discretisation"; Williamson RK3 of section "Time advancement".  With the Lobatto SBP
// property the diagonal of the two-point sum cancels the element's own flux in the surface
// lift (2 D_NN = 1/w_N, 2 D_00 = -1/w_0), so per node
//   J dU/dt = - sum_d sum_{m != i} D_im F#(U_i, U_m; Ja^d_i + Ja^d_m)
//             - (1/w_N) Fs(+d face) + (1/w_0) Fs(-d face)
//             + sum_d sum_m Dhat_im F~v^d_m                                  (Navier-Stokes)
// with Fs = F~* - F~v* the inviscid minus the BR1 viscous face flux and
// Dhat = D - e_N e_N^T/w_N + e_0 e_0^T/w_0 (the own-flux lift of the viscous term folded in).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "dg_device.h"
#include "grad_body.h"
#include "stage_kernel.h"
namespace dg {

// ------------------------------------------------------------------ geometry (FP64 always)
template <int N>
__global__ void __launch_bounds__(nthreads_for(N)) geometry_kernel(View v) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n, NT = nthreads_for(N);
  const int e = blockIdx.x;
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int ti = t % n, tj = (t / n) % n, tk = t / nf;
  __shared__ double sD[n * n], sxi[n];
  __shared__ double sXl[3][nn], sdX[9][nn], sA[3][nn];
  for (int x = t; x < n * n; x += NT) sD[x] = v.tab[2 * n + x];
  if (t < n) sxi[t] = v.tab[t];
  __syncthreads();
  const int cell[3] = {e % v.ex, (e / v.ex) % v.ey, e / (v.ex * v.ey)};
  const long base = (long)e * nn;
  if (act) {
    const int ii[3] = {ti, tj, tk};
    double loc[3], xu[3], dx[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; d++) {
      loc[d] = (1.0 + sxi[ii[d]]) * 0.5 * v.h[d];
      xu[d] = v.lo[d] + cell[d] * v.h[d] + loc[d];
    }
    if (v.deform) {
      dx[0] = v.amp * sin(xu[1]) * sin(xu[2]);
      dx[1] = v.amp * sin(xu[2]) * sin(xu[0]);
      dx[2] = v.amp * sin(xu[0]) * sin(xu[1]);
    }
#pragma unroll
    for (int d = 0; d < 3; d++) {
      v.X[base * 3 + d * nn + t] = xu[d] + dx[d];
      sXl[d][t] = loc[d] + dx[d];  // coordinates relative to the element's corner
    }
  }
  __syncthreads();
  auto dref = [&](const double* f, int d) {
    const int id = d == 0 ? ti : (d == 1 ? tj : tk);
    const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
    const int b0 = t - id * stride;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < n; m++) s += sD[id * n + m] * f[b0 + m * stride];
    return s;
  };
  if (act) {
#pragma unroll
    for (int m = 0; m < 3; m++)
#pragma unroll
      for (int d = 0; d < 3; d++) sdX[3 * m + d][t] = dref(sXl[m], d);
  }
  __syncthreads();
  // curl form: Ja^d_c = -[curl_xi (X_l grad_xi X_m)]_d, (c, m, l) cyclic.  A constant added to
  // X_l does not change it (the tensor-product derivatives commute), hence the corner-relative
  // coordinates.
  for (int c = 0; c < 3; c++) {
    const int m = (c + 1) % 3, l = (c + 2) % 3;
    if (act) {
#pragma unroll
      for (int d = 0; d < 3; d++) sA[d][t] = sXl[l][t] * sdX[3 * m + d][t];
    }
    __syncthreads();
    if (act) {
      const double c0 = dref(sA[2], 1) - dref(sA[1], 2);
      const double c1 = dref(sA[0], 2) - dref(sA[2], 0);
      const double c2 = dref(sA[1], 0) - dref(sA[0], 1);
      v.Ja[base * 9 + (3 * 0 + c) * nn + t] = -c0;
      v.Ja[base * 9 + (3 * 1 + c) * nn + t] = -c1;
      v.Ja[base * 9 + (3 * 2 + c) * nn + t] = -c2;
    }
    __syncthreads();
  }
  if (act) {
    const double* a = &sdX[0][0];
    auto X = [&](int m, int d) { return a[(3 * m + d) * nn + t]; };
    const double J = X(0, 0) * (X(1, 1) * X(2, 2) - X(2, 1) * X(1, 2)) +
                     X(1, 0) * (X(2, 1) * X(0, 2) - X(0, 1) * X(2, 2)) +
                     X(2, 0) * (X(0, 1) * X(1, 2) - X(1, 1) * X(0, 2));
    v.J[base + t] = J;
    v.invJ[base + t] = 1.0 / J;
  }
}

// Gauss-Legendre meshes: the map and its metric terms are those of the Lobatto grid of the same
// order (isoparametric there, curl form there), evaluated at the Gauss points.  The curl form
// makes sum_d d(Ja^d)/dxi_d vanish at the Lobatto nodes, hence identically for these
// polynomials, and the normal component on a face depends only on that face's Lobatto nodes,
// which both elements share: a uniform state stays steady.  One lane per node: coordinates,
// map derivatives and metric terms on the Lobatto nodes (21 fields in LDS), then three passes of
// the Lobatto-to-Gauss interpolation along the element's lines; J from the interpolated
// derivatives; each +xi_d face's metric Ja^d interpolated to its face points (into Sf), which
// both elements of the face take as its scaled normal.
template <int N>
__global__ void __launch_bounds__(nthreads_for(N)) geometry_gauss_kernel(View v) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n, NT = nthreads_for(N);
  constexpr int kGeo = 2 * n + 2 * n * n;  // the geometry tables after the Gauss tables
  const int e = blockIdx.x;
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int ti = t % n, tj = (t / n) % n, tk = t / nf;
  const int ii[3] = {ti, tj, tk};
  __shared__ double sD[n * n], sI[n * n], sxi[n], slb[n];
  __shared__ double sF[21][nn];  // X 0-2, Ja 3-11, dX 12-20 (dX[3m+d] = d x_m / d xi_d)
  __shared__ double sXl[3][nn], sA[3][nn];
  for (int x = t; x < n * n; x += NT) {
    sD[x] = v.tab[kGeo + n + x];
    sI[x] = v.tab[kGeo + n + n * n + x];
  }
  if (t < n) {
    sxi[t] = v.tab[kGeo + t];
    slb[t] = v.tab[2 * n + n * n + n + t];  // Gauss basis at xi = +1
  }
  __syncthreads();
  const int cell[3] = {e % v.ex, (e / v.ex) % v.ey, e / (v.ex * v.ey)};
  const long base = (long)e * nn;
  if (act) {  // the map at the Lobatto nodes
    double loc[3], xu[3], dx[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; d++) {
      loc[d] = (1.0 + sxi[ii[d]]) * 0.5 * v.h[d];
      xu[d] = v.lo[d] + cell[d] * v.h[d] + loc[d];
    }
    if (v.deform) {
      dx[0] = v.amp * sin(xu[1]) * sin(xu[2]);
      dx[1] = v.amp * sin(xu[2]) * sin(xu[0]);
      dx[2] = v.amp * sin(xu[0]) * sin(xu[1]);
    }
#pragma unroll
    for (int d = 0; d < 3; d++) {
      sF[d][t] = xu[d] + dx[d];
      sXl[d][t] = loc[d] + dx[d];  // coordinates relative to the element's corner
    }
  }
  __syncthreads();
  auto dref = [&](const double* f, int d) {
    const int id = d == 0 ? ti : (d == 1 ? tj : tk);
    const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
    const int b0 = t - id * stride;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < n; m++) s += sD[id * n + m] * f[b0 + m * stride];
    return s;
  };
  if (act) {
#pragma unroll
    for (int m = 0; m < 3; m++)
#pragma unroll
      for (int d = 0; d < 3; d++) sF[12 + 3 * m + d][t] = dref(sXl[m], d);
  }
  __syncthreads();
  for (int c = 0; c < 3; c++) {  // curl form, as in geometry_kernel
    const int m = (c + 1) % 3, l = (c + 2) % 3;
    if (act) {
#pragma unroll
      for (int d = 0; d < 3; d++) sA[d][t] = sXl[l][t] * sF[12 + 3 * m + d][t];
    }
    __syncthreads();
    if (act) {
      sF[3 + 3 * 0 + c][t] = -(dref(sA[2], 1) - dref(sA[1], 2));
      sF[3 + 3 * 1 + c][t] = -(dref(sA[0], 2) - dref(sA[2], 0));
      sF[3 + 3 * 2 + c][t] = -(dref(sA[1], 0) - dref(sA[0], 1));
    }
    __syncthreads();
  }
  // to the Gauss points: along xi_0, xi_1, xi_2 in turn
  for (int d = 0; d < 3; d++) {
    double r[21];
    if (act) {
      const int id = d == 0 ? ti : (d == 1 ? tj : tk);
      const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
      const int b0 = t - id * stride;
#pragma unroll
      for (int f = 0; f < 21; f++) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < n; l++) s += sI[id * n + l] * sF[f][b0 + l * stride];
        r[f] = s;
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int f = 0; f < 21; f++) sF[f][t] = r[f];
    }
    __syncthreads();
  }
  if (act) {
#pragma unroll
    for (int d = 0; d < 3; d++) v.X[base * 3 + d * nn + t] = sF[d][t];
#pragma unroll
    for (int c = 0; c < 9; c++) v.Ja[base * 9 + c * nn + t] = sF[3 + c][t];
    auto X = [&](int m, int d) { return sF[12 + 3 * m + d][t]; };
    const double J = X(0, 0) * (X(1, 1) * X(2, 2) - X(2, 1) * X(1, 2)) +
                     X(1, 0) * (X(2, 1) * X(0, 2) - X(0, 1) * X(2, 2)) +
                     X(2, 0) * (X(0, 1) * X(1, 2) - X(1, 1) * X(0, 2));
    v.J[base + t] = J;
    v.invJ[base + t] = 1.0 / J;
  }
  // the +xi_d faces' metric at their face points: sum_i l_i(+1) Ja^d(node i of the line)
  for (int x = t; x < 9 * nf; x += NT) {
    const int dc = x / nf, q = x - dc * nf;
    const int d = dc / 3;
    const int p = q % n, r = q / n;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < n; i++) s += slb[i] * sF[3 + dc][face_node<n>(d, i, p, r)];
    v.Sf[((long)e * 9 + dc) * nf + q] = s;
  }
}

// The face normal Ja^d on the -d side of each element is replaced by the owner's (the
// element across that face, whose +d side it is): both sides then evaluate bitwise the same
// face flux.  The two values differ only by rounding.
template <int N>
__global__ void facefix_kernel(View v) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)v.E * 3 * nf) return;
  const int e = (int)(gid / (3 * nf));
  const int rem = (int)(gid - (long)e * 3 * nf);
  const int d = rem / nf, q = rem - d * nf;
  const int p = q % n, r = q / n;
  const int ne = v.nbr[e * 6 + 2 * d + 1];
  const int io = face_node<n>(d, N, p, r), in = face_node<n>(d, 0, p, r);
#pragma unroll
  for (int c = 0; c < 3; c++)
    v.Ja[(long)ne * nn * 9 + (3 * d + c) * nn + in] = v.Ja[(long)e * nn * 9 + (3 * d + c) * nn + io];
}

// ------------------------------------------------------------------ initial conditions
__global__ void ic_kernel(View v, int cur, int ic, IcParams P) {
  const int nn = (v.N + 1) * (v.N + 1) * (v.N + 1);
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)v.E * nn) return;
  const long e = gid / nn;
  const int q = (int)(gid - e * nn);
  const double x = v.X[e * nn * 3 + q], y = v.X[e * nn * 3 + nn + q], z = v.X[e * nn * 3 + 2 * nn + q];
  double u[5];
  ic_point(v, ic, P, x, y, z, u);
  double* U = v.U[cur] + e * nn * 5;
#pragma unroll
  for (int c = 0; c < 5; c++) {
    U[c * nn + q] = u[c];
    v.dU[e * nn * 5 + c * nn + q] = 0.0;
  }
}

// ------------------------------------------------------------------ pass A (Navier-Stokes)
// grad_body (grad_body.h): BR1 gradient and face viscous fluxes of one element
template <int N, typename T, bool XV>
__global__ void __launch_bounds__(nthreads_for(N)) grad_kernel(View v, int cur) {
  grad_body<N, T, XV>(v, block_element(v.E), cur);
}

template <int N, typename T, bool XV>
__global__ void __launch_bounds__(nthreads_for(N)) grad_batch_kernel(BatchArgs B) {
  int m, e;
  batch_member(B, m, e);
  grad_body<N, T, XV>(*B.view[m], e, B.cur[m]);
}

// ------------------------------------------------------------------ diagnostics (FP64)
// slots: 0-4 integral of U, 5 integral of -rho s, 6 integral of -rho s/(gamma-1), 7 integral of
// rho|v|^2/2, 8 integral of rho|curl v|^2/2, 9 max(|v|+c), 10 min rho, 11 min p,
// 12 number of non-finite values, 13 volume, 14 integral of p
template <int N>
__global__ void __launch_bounds__(nthreads_for(N)) diag_kernel(View v, int cur) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n, NT = nthreads_for(N);
  const int e = blockIdx.x;
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int ti = t % n, tj = (t / n) % n, tk = t / nf;
  __shared__ double sD[n * n], sw[n];
  constexpr int NP = pow2_at_least(NT);  // tree size (NT need not be a power of two)
  __shared__ double sV[3][nn];
  __shared__ double red[NP];
  for (int x = t; x < n * n; x += NT) sD[x] = v.tab[2 * n + x];
  if (t < n) sw[t] = v.tab[n + t];
  const long base = (long)e * nn;
  double u[5] = {0, 0, 0, 0, 0};
  if (act) {
#pragma unroll
    for (int c = 0; c < 5; c++) u[c] = v.U[cur][base * 5 + c * nn + t];
#pragma unroll
    for (int c = 0; c < 3; c++) sV[c][t] = u[1 + c] / u[0];
  }
  __syncthreads();
  double s[kDiagSlots];
#pragma unroll
  for (int k = 0; k < kDiagSlots; k++) s[k] = 0.0;
  s[9] = -INFINITY;
  s[10] = INFINITY;
  s[11] = INFINITY;
  if (act) {
    const double g = v.gamma;
    const double wq = sw[ti] * sw[tj] * sw[tk] * v.J[base + t];
    const double ij = v.invJ[base + t];
    const double rho = u[0];
    const double v1 = sV[0][t], v2 = sV[1][t], v3 = sV[2][t];
    const double q2 = v1 * v1 + v2 * v2 + v3 * v3;
    const double p = (g - 1) * (u[4] - 0.5 * rho * q2);
    int bad = 0;
#pragma unroll
    for (int c = 0; c < 5; c++) {
      s[c] = wq * u[c];
      bad += isfinite(u[c]) ? 0 : 1;
    }
    const double sp = log(p) - g * log(rho);
    s[5] = wq * (-rho * sp);
    s[6] = s[5] / (g - 1);
    s[7] = wq * 0.5 * rho * q2;
    double gv[3][3];
    const int ii[3] = {ti, tj, tk};
    double dv[3][3];  // dv[d][c] = D_d v_c
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const int id = ii[d];
      const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
      const int b0 = t - id * stride;
#pragma unroll
      for (int c = 0; c < 3; c++) {
        double a = 0.0;
#pragma unroll
        for (int m = 0; m < n; m++) a += sD[id * n + m] * sV[c][b0 + m * stride];
        dv[d][c] = a;
      }
    }
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
      for (int x = 0; x < 3; x++) {
        double a = 0.0;
#pragma unroll
        for (int d = 0; d < 3; d++) a += v.Ja[base * 9 + (3 * d + x) * nn + t] * dv[d][c];
        gv[c][x] = a * ij;
      }
    const double o1 = gv[2][1] - gv[1][2], o2 = gv[0][2] - gv[2][0], o3 = gv[1][0] - gv[0][1];
    s[8] = wq * 0.5 * rho * (o1 * o1 + o2 * o2 + o3 * o3);
    double pw;
    s[9] = wave_speed(u, g, pw);
    s[10] = rho;
    s[11] = p;
    s[12] = (double)bad;
    s[13] = wq;
    s[14] = wq * p;
  }
  // fixed-order tree reduction, one slot at a time; slots beyond NT hold the identity
  for (int k = 0; k < 15; k++) {
    red[t] = s[k];
    if (t + NT < NP) red[t + NT] = k == 9 ? -INFINITY : ((k == 10 || k == 11) ? INFINITY : 0.0);
    __syncthreads();
    for (int w = NP / 2; w > 0; w >>= 1) {
      if (t < w) {
        const double a = red[t], b = red[t + w];
        red[t] = k == 9 ? fmax(a, b) : ((k == 10 || k == 11) ? fmin(a, b) : a + b);
      }
      __syncthreads();
    }
    if (t == 0) v.part[(long)e * kDiagSlots + k] = red[0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) diag_final_kernel(View v) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  for (int k = 0; k < 15; k++) {
    double a = k == 9 ? -INFINITY : ((k == 10 || k == 11) ? INFINITY : 0.0);
    for (int e = t; e < v.E; e += 256) {
      const double b = v.part[(long)e * kDiagSlots + k];
      a = k == 9 ? fmax(a, b) : ((k == 10 || k == 11) ? fmin(a, b) : a + b);
    }
    red[t] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) {
        const double x = red[t], y = red[t + w];
        red[t] = k == 9 ? fmax(x, y) : ((k == 10 || k == 11) ? fmin(x, y) : x + y);
      }
      __syncthreads();
    }
    if (t == 0) v.diag[k] = red[0];
    __syncthreads();
  }
}

// ------------------------------------------------------------------ adaptive step size
// Per block: the largest |v| + c over the nodes of its elements, the smallest density, and the
// count of nodes that are not finite or not physical (rho <= 0, p <= 0).  One 64-lane wave per
// element, grid-stride over the elements; uniform and mixed orders.
__global__ void __launch_bounds__(256) lambda_kernel(View v, int cur) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nu = (v.N + 1) * (v.N + 1) * (v.N + 1);
  double lam = -INFINITY, rmin = INFINITY, bad = 0.0;
  for (int e = blockIdx.x * 4 + wv; e < v.E; e += gridDim.x * 4) {
    long off = (long)e * nu;
    int nn = nu;
    if (v.mixed) {
      const int4 q = v.elem[e];
      nn = q.x * q.y * q.z;
      off = q.w;
    }
    const double* __restrict__ U = v.U[cur] + off * 5;
    for (int i = lane; i < nn; i += 64) {
      double u[5];
#pragma unroll
      for (int c = 0; c < 5; c++) u[c] = U[(long)c * nn + i];
      double p;
      const double l = wave_speed(u, v.gamma, p);
      bool ok = u[0] > 0.0 && p > 0.0 && isfinite(l);
#pragma unroll
      for (int c = 0; c < 5; c++) ok = ok && isfinite(u[c]);
      if (ok) {
        lam = fmax(lam, l);
        rmin = fmin(rmin, u[0]);
      } else {
        bad += 1.0;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lam = fmax(lam, __shfl_xor(lam, o, 64));
    rmin = fmin(rmin, __shfl_xor(rmin, o, 64));
    bad += __shfl_xor(bad, o, 64);
  }
  __shared__ double red[3][4];
  if (lane == 0) {
    red[0][wv] = lam;
    red[1][wv] = rmin;
    red[2][wv] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = red[0][0], r = red[1][0], c = red[2][0];
    for (int w = 1; w < 4; w++) {
      a = fmax(a, red[0][w]);
      r = fmin(r, red[1][w]);
      c += red[2][w];
    }
    v.part[3 * blockIdx.x + 0] = a;
    v.part[3 * blockIdx.x + 1] = r;
    v.part[3 * blockIdx.x + 2] = c;
  }
}

// Step size from the partials: the CFL limit cfl h_min/((N+1)^2 lambda_max) and, when the
// viscosity mu_eff (physical plus artificial) is positive, the cap
// 0.25 h_min^2/((N+1)^4 gamma mu_eff/(Pr rho_min)) -- the host's formula, operation for operation.  A state with a non-finite or non-physical node gets step size 0 and raises the count
// in adapt[2], which the host reports.
__global__ void __launch_bounds__(256) dt_kernel(View v, int nparts, double cfl, double hmin, double n1,
                                                 double gamma, double Pr, double mu_eff) {
  __shared__ double red[3][256];
  const int t = threadIdx.x;
  double a = -INFINITY, r = INFINITY, c = 0.0;
  for (int k = t; k < nparts; k += 256) {
    a = fmax(a, v.part[3 * k]);
    r = fmin(r, v.part[3 * k + 1]);
    c += v.part[3 * k + 2];
  }
  red[0][t] = a;
  red[1][t] = r;
  red[2][t] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      red[0][t] = fmax(red[0][t], red[0][t + w]);
      red[1][t] = fmin(red[1][t], red[1][t + w]);
      red[2][t] += red[2][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double lam = red[0][0], rmin = red[1][0];
    double bad = red[2][0];
    double dt = cfl * hmin / (n1 * n1 * lam);
    if (mu_eff > 0.0) dt = fmin(dt, 0.25 * hmin * hmin / (n1 * n1 * n1 * n1 * gamma * mu_eff / (Pr * rmin)));
    if (bad > 0.0 || !(lam > 0.0) || !(dt > 0.0) || !isfinite(dt)) {
      dt = 0.0;
      bad = bad > 0.0 ? bad : 1.0;
    }
    v.adapt[0] = dt;
    v.adapt[1] += dt;
    v.adapt[2] += bad;
  }
}

// the largest wave speed of the partials into adapt[3] (global Lax-Friedrichs)
__global__ void __launch_bounds__(256) lambda_final_kernel(View v, int nparts) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double a = 0.0;
  for (int k = t; k < nparts; k += 256) a = fmax(a, v.part[3 * k]);
  red[t] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = fmax(red[t], red[t + w]);
    __syncthreads();
  }
  if (t == 0) v.adapt[3] = red[0];
}

__global__ void adapt_reset_kernel(View v) {
  if (threadIdx.x < 4) v.adapt[threadIdx.x] = 0.0;
}

// ------------------------------------------------------------------ launchers
template <int N>
static hipError_t geometry_n(const View& v, hipStream_t st) {
  constexpr int n = N + 1, nf = n * n;
  if (v.gauss) {  // no boundary nodes: each face takes its owner's interpolated metric
    hipLaunchKernelGGL(geometry_gauss_kernel<N>, dim3(v.E), dim3(nthreads_for(N)), 0, st, v);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(geometry_kernel<N>, dim3(v.E), dim3(nthreads_for(N)), 0, st, v);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const long total = (long)v.E * 3 * nf;
  hipLaunchKernelGGL(facefix_kernel<N>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, v);
  return hipGetLastError();
}

template <int N, typename T>
static hipError_t gradient_nt(const View& v, int cur, hipStream_t st) {
  if (v.visc_flux != 0)
    hipLaunchKernelGGL((grad_kernel<N, T, true>), dim3(v.E), dim3(nthreads_for(N)), 0, st, v, cur);
  else
    hipLaunchKernelGGL((grad_kernel<N, T, false>), dim3(v.E), dim3(nthreads_for(N)), 0, st, v, cur);
  return hipGetLastError();
}

template <int N>
static hipError_t gradient_n(const View& v, int cur, hipStream_t st) {
  return v.fp32 ? gradient_nt<N, float>(v, cur, st) : gradient_nt<N, double>(v, cur, st);
}

template <int N, typename T>
static hipError_t stage_nt(const View& v, int cur, double dt, double a, double b, int mode,
                           hipStream_t st) {
  if constexpr (sizeof(T) == 8) {  // the extended fluxes run in FP64 only
    const int fx = flux_family(v.vol, v.surf);
    if (fx != 0) return launch_stage_ext(v, fx, cur, dt, a, b, mode, st);
  }
  return stage_ntx<N, T, 0>(v, cur, dt, a, b, mode, st);
}

template <int N>
static hipError_t stage_n(const View& v, int cur, double dt, double a, double b, int mode,
                          hipStream_t st) {
  return v.fp32 ? stage_nt<N, float>(v, cur, dt, a, b, mode, st)
                : stage_nt<N, double>(v, cur, dt, a, b, mode, st);
}

template <int N>
static hipError_t diag_n(const View& v, int cur, hipStream_t st) {
  hipLaunchKernelGGL(diag_kernel<N>, dim3(v.E), dim3(nthreads_for(N)), 0, st, v, cur);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, st, v);
  return hipGetLastError();
}

#define DG_DISPATCH(FN, ...)                          \
  switch (v.N) {                                      \
    case 1: return FN<1>(__VA_ARGS__);                \
    case 2: return FN<2>(__VA_ARGS__);                \
    case 3: return FN<3>(__VA_ARGS__);                \
    case 4: return FN<4>(__VA_ARGS__);                \
    case 5: return FN<5>(__VA_ARGS__);                \
    case 6: return FN<6>(__VA_ARGS__);                \
    case 7: return FN<7>(__VA_ARGS__);                \
    default: return hipErrorInvalidValue;             \
  }

hipError_t launch_geometry(const View& v, hipStream_t st) { DG_DISPATCH(geometry_n, v, st) }

hipError_t launch_gradient(const View& v, int cur, hipStream_t st) { DG_DISPATCH(gradient_n, v, cur, st) }

hipError_t launch_stage(const View& v, int cur, double dt, double rkA, double rkB, int mode,
                        hipStream_t st) {
  DG_DISPATCH(stage_n, v, cur, dt, rkA, rkB, mode, st)
}

hipError_t launch_diagnostics(const View& v, int cur, hipStream_t st) { DG_DISPATCH(diag_n, v, cur, st) }

template <int N, typename T>
static hipError_t gradient_batch_nt(const BatchArgs& B, bool xv, hipStream_t st) {
  if (xv)
    hipLaunchKernelGGL((grad_batch_kernel<N, T, true>), dim3(B.start[B.n]), dim3(nthreads_for(N)), 0, st, B);
  else
    hipLaunchKernelGGL((grad_batch_kernel<N, T, false>), dim3(B.start[B.n]), dim3(nthreads_for(N)), 0, st, B);
  return hipGetLastError();
}

template <int N>
static hipError_t gradient_batch_n(const BatchArgs& B, bool fp32, bool xv, hipStream_t st) {
  return fp32 ? gradient_batch_nt<N, float>(B, xv, st) : gradient_batch_nt<N, double>(B, xv, st);
}

template <int N>
static hipError_t stage_batch_n(const BatchArgs& B, bool fp32, bool visc, int fx, double a, double b,
                                int mode, hipStream_t st) {
  if (fp32) return stage_batch_nt<N, float, 0>(B, visc, a, b, mode, st);
  if (fx != 0) return launch_stage_batch_ext(B, N, visc, fx, a, b, mode, st);
  return stage_batch_nt<N, double, 0>(B, visc, a, b, mode, st);
}

#define DG_DISPATCH_N(NV, FN, ...)                    \
  switch (NV) {                                       \
    case 1: return FN<1>(__VA_ARGS__);                \
    case 2: return FN<2>(__VA_ARGS__);                \
    case 3: return FN<3>(__VA_ARGS__);                \
    case 4: return FN<4>(__VA_ARGS__);                \
    case 5: return FN<5>(__VA_ARGS__);                \
    case 6: return FN<6>(__VA_ARGS__);                \
    case 7: return FN<7>(__VA_ARGS__);                \
    default: return hipErrorInvalidValue;             \
  }

hipError_t launch_gradient_batch(const BatchArgs& B, int N, bool fp32, bool xv, hipStream_t st) {
  if (B.n < 1 || B.n > kMaxBatch) return hipErrorInvalidValue;
  DG_DISPATCH_N(N, gradient_batch_n, B, fp32, xv, st)
}

hipError_t launch_stage_batch(const BatchArgs& B, int N, bool fp32, bool visc, int fx, double rkA, double rkB,
                              int mode, hipStream_t st) {
  if (B.n < 1 || B.n > kMaxBatch) return hipErrorInvalidValue;
  if (fx < 0 || fx > 3 || (fp32 && fx != 0)) return hipErrorInvalidValue;
  DG_DISPATCH_N(N, stage_batch_n, B, fp32, visc, fx, rkA, rkB, mode, st)
}

hipError_t launch_adapt_reset(const View& v, hipStream_t st) {
  hipLaunchKernelGGL(adapt_reset_kernel, dim3(1), dim3(64), 0, st, v);
  return hipGetLastError();
}

hipError_t launch_lambda_max(const View& v, int cur, hipStream_t st) {
  const int blocks = std::min(1024, (v.E + 3) / 4);
  hipLaunchKernelGGL(lambda_kernel, dim3(blocks), dim3(256), 0, st, v, cur);
  hipLaunchKernelGGL(lambda_final_kernel, dim3(1), dim3(256), 0, st, v, blocks);
  return hipGetLastError();
}

hipError_t launch_step_size(const View& v, int cur, double cfl, double hmin, double n1, double gamma, double Pr,
                            double mu_eff, hipStream_t st) {
  // at most 3 partials per block in v.part, which holds kDiagSlots doubles per element
  const int blocks = std::min(1024, (v.E + 3) / 4);
  hipLaunchKernelGGL(lambda_kernel, dim3(blocks), dim3(256), 0, st, v, cur);
  hipLaunchKernelGGL(dt_kernel, dim3(1), dim3(256), 0, st, v, blocks, cfl, hmin, n1, gamma, Pr, mu_eff);
  return hipGetLastError();
}

hipError_t launch_diag_final(const View& v, hipStream_t st) {
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, st, v);
  return hipGetLastError();
}

hipError_t launch_ic(const View& v, int cur, int ic, const double* params, hipStream_t st) {
  IcParams P;
  for (int k = 0; k < 9; k++) P.p[k] = params ? params[k] : 0.0;
  const int nn = (v.N + 1) * (v.N + 1) * (v.N + 1);
  const long total = (long)v.E * nn;
  hipLaunchKernelGGL(ic_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, v, cur, ic, P);
  return hipGetLastError();
}

}  // namespace dg
