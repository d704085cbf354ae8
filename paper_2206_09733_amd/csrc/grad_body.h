// grad_body.h -- Navier-Stokes pass A for one element (the body of grad_kernel, shared with the
// kernel that also forms the spectral-vanishing-viscosity flux of the same element).
#pragma once

#include <hip/hip_runtime.h>

#include "dg_device.h"

namespace dg {

// On the six faces, the contravariant viscous flux along the face normal direction of the face
// viscous flux scheme: Fvf[e][2d+side][c][face node] (BR1: from the lifted gradient of (v, T);
// BR2 and interior penalty: see face_viscous_br2_ip).  The stage kernel averages the two sides.
// XV: the BR2 / interior-penalty face fluxes (compiled apart, the BR1 kernels keep their registers)
template <int N, typename T, bool XV>
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
  const T iwN = (T)(1.0 / sw[N]), iw0 = (T)(1.0 / sw[0]);
  const T* const gp[4] = {sG[0], sG[1], sG[2], sG[3]};
  T* Fvf = reinterpret_cast<T*>(v.Fvf) + (long)e * 6 * 4 * nf;
  if constexpr (XV) {
    // BR2 / interior penalty: broken-gradient fluxes of the face nodes, then one lane per face point
    __shared__ T sFb[6][4][nf];
    if (act) {
      double ja[9];
#pragma unroll
      for (int c = 0; c < 9; c++) ja[c] = v.Ja[base * 9 + c * nn + t];
      broken_face_fluxes<n, T>(t, ti, tj, tk, sD, gp, ja, v.invJ[base + t], (T)v.mu, (T)v.kappa, sFb);
    }
    __syncthreads();
    for (int x = t; x < 6 * nf; x += NT) {
      const int f = x / nf, q = x - f * nf;
      const int io = face_node<n>(f >> 1, (f & 1) ? N : 0, q % n, q / n);
      T Ff[4];
      face_viscous_br2_ip<n, T>(v, e, cur, Tref, f, q, io, iwN, iw0, gp, sJ, sFb, Ff);
#pragma unroll
      for (int c = 0; c < 4; c++) Fvf[(f * 4 + c) * nf + q] = Ff[c];
    }
  } else if (act) {  // BR1: the lifted gradient's flux
    double ja[9];
#pragma unroll
    for (int c = 0; c < 9; c++) ja[c] = v.Ja[base * 9 + c * nn + t];
    const double ij = v.invJ[base + t];
    T Fvd[3][4];
    gradient_and_viscous_flux<n, T>(t, ti, tj, tk, sD, iwN, iw0, gp, sJ, ja, ij, (T)v.mu, (T)v.kappa, Fvd);
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


}  // namespace dg
