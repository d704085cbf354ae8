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

#include <cmath>

#include "dg_device.h"
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
// Lifted gradient of (v, T) and, on the six faces, the contravariant viscous flux along the
// face normal direction: Fvf[e][2d+side][c][face node].
template <int N, typename T>
__device__ __forceinline__ void grad_body(const View& v, const int e, const int cur) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n, NT = nthreads_for(N);
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int ti = t % n, tj = (t / n) % n, tk = t / nf;
  const double* __restrict__ Uin = v.U[cur];
  __shared__ double sD[n * n], sw[n];
  __shared__ T sG[4][nn];
  __shared__ T sJ[6][4][nf];
  const double Tref = sizeof(T) == 4 ? v.p_r / v.rho_r : 0.0;
  for (int x = t; x < n * n; x += NT) sD[x] = v.tab[2 * n + x];
  if (t < n) sw[t] = v.tab[n + t];
  const long base = (long)e * nn;
  if (act) {
    double u[5];
#pragma unroll
    for (int c = 0; c < 5; c++) u[c] = Uin[base * 5 + c * nn + t];
    T g[4];
    gvars(u, v.gamma, Tref, g);
#pragma unroll
    for (int c = 0; c < 4; c++) sG[c][t] = g[c];
  }
  __syncthreads();
  for (int x = t; x < 6 * nf; x += NT) {
    const int f = x / nf, q = x - f * nf;
    const int d = f >> 1, side = f & 1;
    const int p = q % n, r = q / n;
    const int io = face_node<n>(d, side ? N : 0, p, r);
    const int ne = v.nbr[e * 6 + f];
    const int inb = face_node<n>(d, side ? 0 : N, p, r);
    double un[5];
#pragma unroll
    for (int c = 0; c < 5; c++) un[c] = Uin[(long)ne * nn * 5 + c * nn + inb];
    T gn[4];
    gvars(un, v.gamma, Tref, gn);
#pragma unroll
    for (int c = 0; c < 4; c++) sJ[f][c][q] = (T)0.5 * (gn[c] - sG[c][io]);
  }
  __syncthreads();
  if (act) {
    double ja[9];
#pragma unroll
    for (int c = 0; c < 9; c++) ja[c] = v.Ja[base * 9 + c * nn + t];
    const double ij = v.invJ[base + t];
    const T iwN = (T)(1.0 / sw[N]), iw0 = (T)(1.0 / sw[0]);
    T Fvd[3][4];
    const T* const gp[4] = {sG[0], sG[1], sG[2], sG[3]};
    gradient_and_viscous_flux<n, T>(t, ti, tj, tk, sD, iwN, iw0, gp, sJ, ja, ij, (T)v.mu, (T)v.kappa,
                                    Fvd);
    T* Fvf = reinterpret_cast<T*>(v.Fvf) + (long)e * 6 * 4 * nf;
    const int ii[3] = {ti, tj, tk};
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const int qd = d == 0 ? tj + n * tk : (d == 1 ? ti + n * tk : ti + n * tj);
      if (ii[d] == N) {
#pragma unroll
        for (int c = 0; c < 4; c++) Fvf[((2 * d + 1) * 4 + c) * nf + qd] = Fvd[d][c];
      }
      if (ii[d] == 0) {
#pragma unroll
        for (int c = 0; c < 4; c++) Fvf[((2 * d) * 4 + c) * nf + qd] = Fvd[d][c];
      }
    }
  }
}

template <int N, typename T>
__global__ void __launch_bounds__(nthreads_for(N)) grad_kernel(View v, int cur) {
  grad_body<N, T>(v, block_element(v.E), cur);
}

template <int N, typename T>
__global__ void __launch_bounds__(nthreads_for(N)) grad_batch_kernel(BatchArgs B) {
  int m, e;
  batch_member(B, m, e);
  grad_body<N, T>(*B.view[m], e, B.cur[m]);
}

// ------------------------------------------------------------------ stage kernel
// Residual of one element and, in RK mode, the low-storage update
//   dU <- A dU + dt R;  U_out <- U_in + B dU   (dU not read when A = 0).
// LDS holds the primitive variables of the element, the metric components of the reference
// direction being processed, the six face-flux grids, and one phase-dependent region (BR1
// temperature and half jumps; one direction of the contravariant viscous flux; the two-point
// fluxes of one direction).
// occupancy target of the stage kernel: waves per SIMD the register allocation must allow
__host__ __device__ constexpr int stage_waves_per_eu(int N) { return N <= 5 ? 3 : 2; }

template <int N, typename T, bool VISC, int FX>
__device__ __forceinline__ void stage_body(const View& v, const int e, const int cur, const double dt,
                                           const double rkA, const double rkB, const int mode) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n, NT = nthreads_for(N);
  constexpr int np = n * (n - 1) / 2;  // pairs (a < b) on one line of n nodes
  constexpr int P = nf * np;           // pairs per direction
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int ti = t % n, tj = (t / n) % n, tk = t / nf;
  const int ii[3] = {ti, tj, tk};
  const double* __restrict__ Uin = v.U[cur];
  constexpr bool DEV = sizeof(T) == 4;  // FP32-bulk: deviation form
  const Ref Rf = make_ref(v.rho_r, v.p_r, v.gamma);
  const double Tref = DEV ? Rf.por : 0.0;

  __shared__ double sD[n * n], sDh[n * n], sw[n];
  __shared__ T sP[7][nn];      // rho, v1, v2, v3, beta, ln rho, ln beta (FP32-bulk: deviations)
  __shared__ double sJa3[3][nn];  // Ja^d of the direction d being processed
  __shared__ T sF[6][5][nf];      // face fluxes F~* - F~v*
  __shared__ unsigned char sPa[np], sPb[np];
  // FP32-bulk keeps the mass flux in FP64: velocities, face and pair mass fluxes
  constexpr int nnD = DEV ? nn : 1, nfD = DEV ? nf : 1;
  __shared__ double sVd[3][nnD];
  __shared__ double sF0d[6][nfD];
  constexpr int bytesA = VISC ? (nn + 24 * nf) * (int)sizeof(T) : 0;
  constexpr int bytesB = VISC ? 4 * nn * (int)sizeof(T) : 0;
  constexpr int bytesC = 5 * P * (int)sizeof(T) + (DEV ? 8 * P : 0);
  constexpr int bytesAB = bytesA > bytesB ? bytesA : bytesB;
  __shared__ __align__(16) char sRaw[bytesAB > bytesC ? bytesAB : bytesC];
  T* sT = reinterpret_cast<T*>(sRaw);                                   // temperature
  T(*sJ)[4][nf] = reinterpret_cast<T(*)[4][nf]>(sRaw + nn * sizeof(T));  // half jumps of g
  T(*sFv)[nn] = reinterpret_cast<T(*)[nn]>(sRaw);                      // F~v^d, 4 components
  T(*sPair)[P] = reinterpret_cast<T(*)[P]>(sRaw);
  double* sM = reinterpret_cast<double*>(sRaw + 5 * P * sizeof(T));  // FP32-bulk pair mass flux

  for (int x = t; x < n * n; x += NT) {
    sD[x] = v.tab[2 * n + x];
    sDh[x] = v.tab[2 * n + n * n + x];
  }
  if (t < n) sw[t] = v.tab[n + t];
  if (t < np) {  // pair k -> (a, b), ordered by a then b
    int a = 0, k = t;
    while (k >= n - 1 - a) {
      k -= n - 1 - a;
      a++;
    }
    sPa[t] = (unsigned char)a;
    sPb[t] = (unsigned char)(a + 1 + k);
  }
  const long base = (long)e * nn;
  double ja[9], ij = 0.0;
  if (act) {
    double u[5];
#pragma unroll
    for (int c = 0; c < 5; c++) u[c] = Uin[base * 5 + c * nn + t];
    const Prim<T> Pr = DEV ? make_prim_dev<T>(u, v.gamma, Rf) : make_prim<T>(u, v.gamma);
    sP[0][t] = Pr.rho; sP[1][t] = Pr.v1; sP[2][t] = Pr.v2; sP[3][t] = Pr.v3;
    sP[4][t] = Pr.beta; sP[5][t] = Pr.lrho; sP[6][t] = Pr.lbeta;
    if (DEV) {
      const double ir = rcp(u[0]);
      sVd[0][t] = u[1] * ir;
      sVd[1][t] = u[2] * ir;
      sVd[2][t] = u[3] * ir;
    }
    // the extended surface fluxes need the registers during the face phase: their families load
    // the metric terms after it
    if constexpr ((FX & 2) == 0) {
#pragma unroll
      for (int c = 0; c < 9; c++) ja[c] = v.Ja[base * 9 + c * nn + t];
      ij = v.invJ[base + t];
    }
    if (VISC) {
      T g[4];
      gvars(u, v.gamma, Tref, g);
      sT[t] = g[3];
    }
  }
  __syncthreads();

  // ---- faces: numerical flux (minus the BR1 viscous flux) on the 6 (N+1)^2 face grids.  Both
  // elements of a face evaluate it from the same global values in the same argument order, so
  // it is single-valued.
  const T* FvfAll = VISC ? reinterpret_cast<const T*>(v.Fvf) : nullptr;
  for (int x = t; x < 6 * nf; x += NT) {
    const int f = x / nf, q = x - f * nf;
    const int d = f >> 1, side = f & 1;
    const int p = q % n, r = q / n;
    const int io = face_node<n>(d, side ? N : 0, p, r);
    const int ne = v.nbr[e * 6 + f];
    const int inb = face_node<n>(d, side ? 0 : N, p, r);
    double un[5], uL[5], uR[5], S[3];
#pragma unroll
    for (int c = 0; c < 5; c++) {
      un[c] = Uin[(long)ne * nn * 5 + c * nn + inb];
      const double uo = Uin[base * 5 + c * nn + io];
      uL[c] = side ? uo : un[c];
      uR[c] = side ? un[c] : uo;
    }
#pragma unroll
    for (int c = 0; c < 3; c++) S[c] = v.Ja[base * 9 + (3 * d + c) * nn + io];
    T F[5];
    if (DEV) {
      double F0d;
      face_flux_dev<T>(v.surf, uL, uR, S, v.gamma, Rf, F, F0d);
      sF0d[f][q] = F0d;
    } else {
      face_flux<T, (FX & 2) != 0>(v.surf, uL, uR, S, v.gamma, F);
    }
    if (VISC) {
      const T* fo = FvfAll + ((long)e * 6 + f) * 4 * nf;
      const T* fn = FvfAll + ((long)ne * 6 + (f ^ 1)) * 4 * nf;
#pragma unroll
      for (int c = 0; c < 4; c++) F[1 + c] -= (T)0.5 * (fo[c * nf + q] + fn[c * nf + q]);
      T gn[4];
      gvars(un, v.gamma, Tref, gn);
      const T go[4] = {sP[1][io], sP[2][io], sP[3][io], sT[io]};
#pragma unroll
      for (int c = 0; c < 4; c++) sJ[f][c][q] = (T)0.5 * (gn[c] - go[c]);
    }
#pragma unroll
    for (int c = 0; c < 5; c++) sF[f][c][q] = F[c];
  }
  if constexpr ((FX & 2) != 0) {
    if (act) {
#pragma unroll
      for (int c = 0; c < 9; c++) ja[c] = v.Ja[base * 9 + c * nn + t];
      ij = v.invJ[base + t];
    }
  }
  __syncthreads();

  const T iwN = (T)(1.0 / sw[N]), iw0 = (T)(1.0 / sw[0]);
  T acc[5] = {0, 0, 0, 0, 0};
  double acc0d = 0.0;  // FP32-bulk mass accumulator
  if (VISC) {
    // BR1 gradient and contravariant viscous flux of this node, then sum_m Dhat_im F~v^d_m
    T Fvd[3][4];
    if (act) {
      const T* const gp[4] = {sP[1], sP[2], sP[3], sT};
      gradient_and_viscous_flux<n, T>(t, ti, tj, tk, sD, iwN, iw0, gp, sJ, ja, ij, (T)v.mu,
                                      (T)v.kappa, Fvd);
    }
#pragma unroll
    for (int d = 0; d < 3; d++) {
      __syncthreads();  // previous users of the phase region are done
      if (act) {
#pragma unroll
        for (int c = 0; c < 4; c++) sFv[c][t] = Fvd[d][c];
      }
      __syncthreads();
      if (act) {
        const int id = ii[d];
        const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
        const int b0 = t - id * stride;
#pragma unroll
        for (int m = 0; m < n; m++) {
          const T Dh = (T)sDh[id * n + m];
#pragma unroll
          for (int c = 0; c < 4; c++) acc[1 + c] -= Dh * sFv[c][b0 + m * stride];
        }
      }
    }
  }

  // ---- volume: split-form sums; each pair of a line is evaluated once and used by both nodes
  const T ce = (T)(0.5 / (v.gamma - 1.0)), gm1 = (T)(v.gamma - 1.0);
  for (int d = 0; d < 3; d++) {
    const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
    __syncthreads();  // previous users of sJa3 / the phase region are done
    if (act) {
#pragma unroll
      for (int c = 0; c < 3; c++) sJa3[c][t] = ja[3 * d + c];
    }
    __syncthreads();
    for (int s = t; s < P; s += NT) {
      const int line = s / np, k = s - line * np;
      const int b0 = d == 0 ? n * line : (d == 1 ? line % n + nf * (line / n) : line);
      const int na = b0 + sPa[k] * stride, nb = b0 + sPb[k] * stride;
      Prim<T> A, B;
      A.rho = sP[0][na]; A.v1 = sP[1][na]; A.v2 = sP[2][na]; A.v3 = sP[3][na];
      A.beta = sP[4][na]; A.lrho = sP[5][na]; A.lbeta = sP[6][na];
      A.h = (T)0.5 * (A.v1 * A.v1 + A.v2 * A.v2 + A.v3 * A.v3);
      B.rho = sP[0][nb]; B.v1 = sP[1][nb]; B.v2 = sP[2][nb]; B.v3 = sP[3][nb];
      B.beta = sP[4][nb]; B.lrho = sP[5][nb]; B.lbeta = sP[6][nb];
      B.h = (T)0.5 * (B.v1 * B.v1 + B.v2 * B.v2 + B.v3 * B.v3);
      T F[5];
      const double md[3] = {sJa3[0][na] + sJa3[0][nb], sJa3[1][na] + sJa3[1][nb],
                            sJa3[2][na] + sJa3[2][nb]};
      const T m1 = (T)md[0], m2 = (T)md[1], m3 = (T)md[2];
      if (DEV) {
        const double va[3] = {sVd[0][na], sVd[1][na], sVd[2][na]};
        const double vb[3] = {sVd[0][nb], sVd[1][nb], sVd[2][nb]};
        double F0d;
        if (v.vol == 0) {
          const double vn64 = 0.5 * ((va[0] + vb[0]) * md[0] + (va[1] + vb[1]) * md[1] + (va[2] + vb[2]) * md[2]);
          flux_ec_dev(A, B, m1, m2, m3, vn64, Rf, F, F0d);
        } else {
          flux_central_dev(A, B, m1, m2, m3, va, vb, md, Rf, F, F0d);
        }
        sM[s] = F0d;
      } else {
        vol_flux<T, (FX & 1) != 0>(v.vol, A, B, m1, m2, m3, ce, gm1, F);
      }
#pragma unroll
      for (int c = 0; c < 5; c++) sPair[c][s] = F[c];
    }
    __syncthreads();
    if (act) {
      const int id = ii[d];
      const int line = d == 0 ? tj + n * tk : (d == 1 ? ti + n * tk : ti + n * tj);
#pragma unroll
      for (int m = 0; m < n; m++) {
        if (m == id) continue;
        const int a = m < id ? m : id, b = m < id ? id : m;
        const int k = line * np + a * (2 * n - a - 1) / 2 + (b - a - 1);
        const T Dm = (T)sD[id * n + m];
#pragma unroll
        for (int c = 0; c < 5; c++) acc[c] += Dm * sPair[c][k];
        if (DEV) acc0d += sD[id * n + m] * sM[k];
      }
      if (id == N) {
#pragma unroll
        for (int c = 0; c < 5; c++) acc[c] += iwN * sF[2 * d + 1][c][line];
        if (DEV) acc0d += sF0d[2 * d + 1][line] / sw[N];
      }
      if (id == 0) {
#pragma unroll
        for (int c = 0; c < 5; c++) acc[c] -= iw0 * sF[2 * d][c][line];
        if (DEV) acc0d -= sF0d[2 * d][line] / sw[0];
      }
    }
  }
  if (!act) return;
  double R[5];
#pragma unroll
  for (int c = 0; c < 5; c++) R[c] = -(double)acc[c] * ij;
  if (DEV) {  // FP64 mass; energy = H_r (mass) + deviation
    R[0] = -acc0d * ij;
    R[4] -= Rf.H * acc0d * ij;
  }
  const long o = base * 5 + t;
  if (mode == kModeResidual) {
#pragma unroll
    for (int c = 0; c < 5; c++) v.R[o + c * nn] = R[c];
    return;
  }
  double* __restrict__ Uout = v.U[cur ^ 1];
#pragma unroll
  for (int c = 0; c < 5; c++) {
    const double du = (rkA == 0.0 ? 0.0 : rkA * v.dU[o + c * nn]) + dt * R[c];
    v.dU[o + c * nn] = du;
    Uout[o + c * nn] = Uin[o + c * nn] + rkB * du;
  }
}

// FX: the flux family (see flux_family); each family is compiled as separate kernels
template <int N, typename T, bool VISC, int FX>
__global__ void __launch_bounds__(nthreads_for(N))
    __attribute__((amdgpu_waves_per_eu(stage_waves_per_eu(N))))
    stage_kernel(View v, int cur, double dt, double rkA, double rkB, int mode) {
  stage_body<N, T, VISC, FX>(v, block_element(v.E), cur, dt, rkA, rkB, mode);
}

template <int N, typename T, bool VISC, int FX>
__global__ void __launch_bounds__(nthreads_for(N))
    __attribute__((amdgpu_waves_per_eu(stage_waves_per_eu(N))))
    stage_batch_kernel(BatchArgs B, double rkA, double rkB, int mode) {
  int m, e;
  batch_member(B, m, e);
  stage_body<N, T, VISC, FX>(*B.view[m], e, B.cur[m], B.dt[m], rkA, rkB, mode);
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
    s[9] = sqrt(q2) + sqrt(g * p / rho);
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

// ------------------------------------------------------------------ launchers
template <int N>
static hipError_t geometry_n(const View& v, hipStream_t st) {
  constexpr int n = N + 1, nf = n * n;
  hipLaunchKernelGGL(geometry_kernel<N>, dim3(v.E), dim3(nthreads_for(N)), 0, st, v);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const long total = (long)v.E * 3 * nf;
  hipLaunchKernelGGL(facefix_kernel<N>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, v);
  return hipGetLastError();
}

template <int N, typename T>
static hipError_t gradient_nt(const View& v, int cur, hipStream_t st) {
  hipLaunchKernelGGL((grad_kernel<N, T>), dim3(v.E), dim3(nthreads_for(N)), 0, st, v, cur);
  return hipGetLastError();
}

template <int N>
static hipError_t gradient_n(const View& v, int cur, hipStream_t st) {
  return v.fp32 ? gradient_nt<N, float>(v, cur, st) : gradient_nt<N, double>(v, cur, st);
}

template <int N, typename T, int FX>
static hipError_t stage_ntx(const View& v, int cur, double dt, double a, double b, int mode,
                            hipStream_t st) {
  const dim3 grid(v.E), block(nthreads_for(N));
  if (v.viscous)
    hipLaunchKernelGGL((stage_kernel<N, T, true, FX>), grid, block, 0, st, v, cur, dt, a, b, mode);
  else
    hipLaunchKernelGGL((stage_kernel<N, T, false, FX>), grid, block, 0, st, v, cur, dt, a, b, mode);
  return hipGetLastError();
}

template <int N, typename T>
static hipError_t stage_nt(const View& v, int cur, double dt, double a, double b, int mode,
                           hipStream_t st) {
  if constexpr (sizeof(T) == 8) {  // the extended fluxes run in FP64 only
    switch (flux_family(v.vol, v.surf)) {
      case 1: return stage_ntx<N, T, 1>(v, cur, dt, a, b, mode, st);
      case 2: return stage_ntx<N, T, 2>(v, cur, dt, a, b, mode, st);
      case 3: return stage_ntx<N, T, 3>(v, cur, dt, a, b, mode, st);
      default: break;
    }
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
static hipError_t gradient_batch_nt(const BatchArgs& B, hipStream_t st) {
  hipLaunchKernelGGL((grad_batch_kernel<N, T>), dim3(B.start[B.n]), dim3(nthreads_for(N)), 0, st, B);
  return hipGetLastError();
}

template <int N>
static hipError_t gradient_batch_n(const BatchArgs& B, bool fp32, hipStream_t st) {
  return fp32 ? gradient_batch_nt<N, float>(B, st) : gradient_batch_nt<N, double>(B, st);
}

template <int N, typename T, int FX>
static hipError_t stage_batch_nt(const BatchArgs& B, bool visc, double a, double b, int mode,
                                 hipStream_t st) {
  const dim3 grid(B.start[B.n]), block(nthreads_for(N));
  if (visc)
    hipLaunchKernelGGL((stage_batch_kernel<N, T, true, FX>), grid, block, 0, st, B, a, b, mode);
  else
    hipLaunchKernelGGL((stage_batch_kernel<N, T, false, FX>), grid, block, 0, st, B, a, b, mode);
  return hipGetLastError();
}

template <int N>
static hipError_t stage_batch_n(const BatchArgs& B, bool fp32, bool visc, int fx, double a, double b,
                                int mode, hipStream_t st) {
  if (fp32) return stage_batch_nt<N, float, 0>(B, visc, a, b, mode, st);
  switch (fx) {
    case 1: return stage_batch_nt<N, double, 1>(B, visc, a, b, mode, st);
    case 2: return stage_batch_nt<N, double, 2>(B, visc, a, b, mode, st);
    case 3: return stage_batch_nt<N, double, 3>(B, visc, a, b, mode, st);
    default: return stage_batch_nt<N, double, 0>(B, visc, a, b, mode, st);
  }
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

hipError_t launch_gradient_batch(const BatchArgs& B, int N, bool fp32, hipStream_t st) {
  if (B.n < 1 || B.n > kMaxBatch) return hipErrorInvalidValue;
  DG_DISPATCH_N(N, gradient_batch_n, B, fp32, st)
}

hipError_t launch_stage_batch(const BatchArgs& B, int N, bool fp32, bool visc, int fx, double rkA, double rkB,
                              int mode, hipStream_t st) {
  if (B.n < 1 || B.n > kMaxBatch) return hipErrorInvalidValue;
  if (fx < 0 || fx > 3 || (fp32 && fx != 0)) return hipErrorInvalidValue;
  DG_DISPATCH_N(N, stage_batch_n, B, fp32, visc, fx, rkA, rkB, mode, st)
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
