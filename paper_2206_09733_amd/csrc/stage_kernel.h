// stage_kernel.h -- the stage kernel (residual of one element and the fused low-storage RK
// update) and its batched entry, as templates over the order N, the arithmetic type T, the
// viscous terms and the flux family FX.  kernels.hip instantiates family 0 (and FP32-bulk),
// kernels_ext.hip the extended families 1..3, so the two compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "dg_device.h"

namespace dg {

// ------------------------------------------------------------------ stage kernel
// Residual of one element and, in RK mode, the low-storage update
//   dU <- A dU + dt R;  U_out <- U_in + B dU   (dU not read when A = 0).
// LDS holds the primitive variables of the element, the metric components of the reference
// direction being processed, the six face-flux grids, and one phase-dependent region (BR1
// temperature and half jumps; one direction of the contravariant viscous flux; the two-point
// fluxes of one direction).
// occupancy target of the stage kernel: waves per SIMD the register allocation must allow (the
// FP32-bulk kernels fit 4 at orders 1, 2, 4, 5 with at most 2 spilled registers, measured faster
// than 3 for Euler and NS alike; at order 3 they would spill 8-10 and keep 3)
__host__ __device__ constexpr int stage_waves_per_eu(int N, bool fp32) {
  return N <= 5 ? (fp32 && N != 3 ? 4 : 3) : 2;
}

// global operands of one face point of the stage kernel's face phase: the neighbour's and the
// element's traces, the face's scaled normal, and the sum of the two sides' face viscous fluxes
template <typename T>
struct FaceIn {
  double un[5], uo[5], S[3];
  T fv[4];
};

// SVA (Navier-Stokes): the filtered spectral-vanishing-viscosity flux v.Fa (FP64; rounded to T
// as it is read) of the same state joins the viscous flux at the nodes, and on the faces the average of both sides'
// stored values (as the viscous face fluxes; a face node's lane lifts it, the sum taken in the same
// order from both sides), so the residual holds its term too
template <int N, typename T, bool VISC, int FX, bool SVA = false>
__device__ __forceinline__ void stage_body(const View& v, const int e, const int cur, const double dt,
                                           const double rkA, const double rkB, const int mode) {
  static_assert(!SVA || VISC, "the folded SVV term needs the viscous kernel");
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
  // One region holds each phase's arrays in turn:
  //   A (face phase, until the gradient and the mass-flux lift are taken): temperature, half
  //     jumps of g and (FP32-bulk) the FP64 face mass fluxes;
  //   B (viscous volume phase): one direction of the contravariant viscous flux;
  //   C (volume phase): the two-point fluxes of one direction (and their FP64 mass fluxes).
  constexpr int a16 = 16;
  constexpr int offJ = VISC ? ((nn * (int)sizeof(T) + a16 - 1) / a16) * a16 : 0;
  constexpr int offF0 = VISC ? ((offJ + 24 * nf * (int)sizeof(T) + a16 - 1) / a16) * a16 : 0;
  constexpr int bytesA = offF0 + (DEV ? 6 * nf * 8 : 0);
  constexpr int bytesB = VISC ? 4 * nn * (int)sizeof(T) : 0;
  constexpr int bytesC = ((5 * P * (int)sizeof(T) + a16 - 1) / a16) * a16 + (DEV ? 8 * P : 0);
  constexpr int bytesAB = bytesA > bytesB ? bytesA : bytesB;
  __shared__ __align__(16) char sRaw[bytesAB > bytesC ? bytesAB : bytesC];
  T* sT = reinterpret_cast<T*>(sRaw);                                // temperature
  T(*sJ)[4][nf] = reinterpret_cast<T(*)[4][nf]>(sRaw + offJ);        // half jumps of g
  double(*sF0d)[nfD] = reinterpret_cast<double(*)[nfD]>(sRaw + offF0);  // FP32-bulk face mass flux
  T(*sFv)[nn] = reinterpret_cast<T(*)[nn]>(sRaw);                    // F~v^d, 4 components
  T(*sPair)[P] = reinterpret_cast<T(*)[P]>(sRaw);
  double* sM = reinterpret_cast<double*>(sRaw + ((5 * P * (int)sizeof(T) + a16 - 1) / a16) * a16);  // pair mass flux

  // tables (every lane loads, the first n^2 store: no wait of their own before the other loads)
  static_assert(n * n <= NT, "one table entry per lane");
  const int tt = t < n * n ? t : 0;
  const double tD = v.tab[2 * n + tt], tDh = v.tab[2 * n + n * n + tt], tw = v.tab[n + (t < n ? t : 0)];
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
  // The six neighbours (uniform over the workgroup: scalar loads), and the global operands of
  // this lane's first face point, issued before the node's own state so that the two memory
  // round trips overlap.
  const int nb0 = v.nbr[e * 6], nb1 = v.nbr[e * 6 + 1], nb2 = v.nbr[e * 6 + 2], nb3 = v.nbr[e * 6 + 3],
            nb4 = v.nbr[e * 6 + 4], nb5 = v.nbr[e * 6 + 5];
  const T* FvfAll = VISC ? reinterpret_cast<const T*>(v.Fvf) : nullptr;
  auto face_load = [&](int x, FaceIn<T>& I) {
    const int f = x / nf, q = x - f * nf;
    const int d = f >> 1, side = f & 1;
    const int p = q % n, r = q / n;
    const int io = face_node<n>(d, side ? N : 0, p, r);
    const int inb = face_node<n>(d, side ? 0 : N, p, r);
    const int ne = f < 3 ? (f == 0 ? nb0 : (f == 1 ? nb1 : nb2)) : (f == 3 ? nb3 : (f == 4 ? nb4 : nb5));
#pragma unroll
    for (int c = 0; c < 5; c++) {
      I.un[c] = Uin[(long)ne * nn * 5 + c * nn + inb];
      I.uo[c] = Uin[base * 5 + c * nn + io];
    }
#pragma unroll
    for (int c = 0; c < 3; c++) I.S[c] = v.Ja[base * 9 + (3 * d + c) * nn + io];
    if (VISC) {
      const T* fo = FvfAll + ((long)e * 6 + f) * 4 * nf;
      const T* fn = FvfAll + ((long)ne * 6 + (f ^ 1)) * 4 * nf;
#pragma unroll
      for (int c = 0; c < 4; c++) I.fv[c] = fo[c * nf + q] + fn[c * nf + q];
    }
  };
  FaceIn<T> face0;
  if (t < 6 * nf) face_load(t, face0);
  if (t < n * n) {
    sD[t] = tD;
    sDh[t] = tDh;
  }
  if (t < n) sw[t] = tw;
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
    // the extended surface fluxes, and the viscous terms, need the registers during the face
    // phase: those kernels load the metric terms after it (measured: NS 499 -> 488 us at
    // 32^3, N = 4; the Euler kernel is faster with the early load)
    if constexpr ((FX & 2) == 0 && !VISC) {
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
  const double lam_g = (FX & 2) != 0 && v.surf == 8 ? v.adapt[3] : 0.0;  // global Lax-Friedrichs
  auto face_eval = [&](int x, const FaceIn<T>& I) {
    const int f = x / nf, q = x - f * nf;
    const int d = f >> 1, side = f & 1;
    const int p = q % n, r = q / n;
    const int io = face_node<n>(d, side ? N : 0, p, r);
    double uL[5], uR[5];
#pragma unroll
    for (int c = 0; c < 5; c++) {
      uL[c] = side ? I.uo[c] : I.un[c];
      uR[c] = side ? I.un[c] : I.uo[c];
    }
    T F[5];
    if (DEV) {
      double F0d;
      face_flux_dev<T>(v.surf, uL, uR, I.S, v.gamma, Rf, F, F0d);
      sF0d[f][q] = F0d;
    } else {
      face_flux<T, (FX & 2) != 0>(v.surf, uL, uR, I.S, v.gamma, F, lam_g);
    }
    if (VISC) {
#pragma unroll
      for (int c = 0; c < 4; c++) F[1 + c] -= (T)0.5 * I.fv[c];
      T gn[4];
      gvars(I.un, v.gamma, Tref, gn);
      const T go[4] = {sP[1][io], sP[2][io], sP[3][io], sT[io]};
#pragma unroll
      for (int c = 0; c < 4; c++) sJ[f][c][q] = (T)0.5 * (gn[c] - go[c]);
    }
#pragma unroll
    for (int c = 0; c < 5; c++) sF[f][c][q] = F[c];
  };
  // the metric terms of the kernels that load them late: in FP64 with the standard surface fluxes
  // issued before the remaining face points, so that their latency overlaps that work; the others
  // issue them after the face points (issued early they would spill: FP32-bulk at 4 waves per
  // SIMD, the extended surface fluxes, and FP64 Navier-Stokes at order 3)
  auto load_metric = [&]() {
    if (act) {
#pragma unroll
      for (int c = 0; c < 9; c++) ja[c] = v.Ja[base * 9 + c * nn + t];
      ij = v.invJ[base + t];
    }
  };
  constexpr bool late_metric = (FX & 2) != 0 || VISC;
  constexpr bool early = late_metric && !DEV && (FX & 2) == 0 && N != 3;
  if (t < 6 * nf) face_eval(t, face0);
  if constexpr (early) load_metric();
  for (int x = t + NT; x < 6 * nf; x += NT) {
    FaceIn<T> I;
    face_load(x, I);
    face_eval(x, I);
  }
  if constexpr (late_metric && !early) load_metric();
  __syncthreads();

  const T iwN = (T)(1.0 / sw[N]), iw0 = (T)(1.0 / sw[0]);
  T acc[5] = {0, 0, 0, 0, 0};
  double acc0d = 0.0;  // FP32-bulk mass accumulator
  // FP32-bulk: lift of the FP64 face mass fluxes, taken before their region is reused (in FP64
  // the order of the sum does not matter; the FP32 lifts stay beside each direction's volume
  // sum, which they largely cancel)
  if (DEV && act) {
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const int id = ii[d];
      const int line = d == 0 ? tj + n * tk : (d == 1 ? ti + n * tk : ti + n * tj);
      if (id == N) acc0d += sF0d[2 * d + 1][line] / sw[N];
      if (id == 0) acc0d -= sF0d[2 * d][line] / sw[0];
    }
  }
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
      T fa[4] = {0, 0, 0, 0}, fb[4] = {0, 0, 0, 0};  // SVA: this node's Fa^d, the neighbour's across a face
      const int idd = ii[d];
      const bool onf = SVA && act && (idd == 0 || idd == N);
      if (SVA && act) {
#pragma unroll
        for (int c = 0; c < 4; c++) fa[c] = (T)v.Fa[(base * 12) + (4 * d + c) * nn + t];
      }
      if (onf) {
        const int side = idd == N ? 1 : 0;
        const int ne = side ? (d == 0 ? nb1 : (d == 1 ? nb3 : nb5)) : (d == 0 ? nb0 : (d == 1 ? nb2 : nb4));
        const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
        const int inb = t + (side ? -N : N) * stride;  // the matching node across the face
#pragma unroll
        for (int c = 0; c < 4; c++) fb[c] = (T)v.Fa[((long)ne * 12 + 4 * d + c) * nn + inb];
      }
      __syncthreads();  // previous users of the phase region are done
      if (act) {
#pragma unroll
        for (int c = 0; c < 4; c++) sFv[c][t] = SVA ? Fvd[d][c] + fa[c] : Fvd[d][c];
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
        if (onf) {  // lift of the face average of Fa (the own value's lift is in Dhat)
          const T wl = id == N ? -(T)0.5 * iwN : (T)0.5 * iw0;
#pragma unroll
          for (int c = 0; c < 4; c++) acc[1 + c] += wl * (fa[c] + fb[c]);  // (commutes: the same on both sides)
        }
      }
    }
  }

  // The RK update's operands, loaded before the pair phase so that their latency hides behind it
  const long o = base * 5 + t;
  double u_in[5], du_in[5];
  if (act && mode != kModeResidual) {
#pragma unroll
    for (int c = 0; c < 5; c++) {
      u_in[c] = Uin[o + c * nn];
      du_in[c] = rkA == 0.0 ? 0.0 : v.dU[o + c * nn];
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
      }
      if (id == 0) {
#pragma unroll
        for (int c = 0; c < 5; c++) acc[c] -= iw0 * sF[2 * d][c][line];
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
  if (mode == kModeResidual) {
#pragma unroll
    for (int c = 0; c < 5; c++) v.R[o + c * nn] = R[c];
    return;
  }
  double* __restrict__ Uout = v.U[cur ^ 1];
  const double h = v.dtp ? *v.dtp : dt;
#pragma unroll
  for (int c = 0; c < 5; c++) {
    const double du = (rkA == 0.0 ? 0.0 : rkA * du_in[c]) + h * R[c];
    v.dU[o + c * nn] = du;
    Uout[o + c * nn] = u_in[c] + rkB * du;
  }
}

// FX: the flux family (see flux_family); each family is compiled as separate kernels
template <int N, typename T, bool VISC, int FX, bool SVA = false>
__global__ void __launch_bounds__(nthreads_for(N))
    __attribute__((amdgpu_waves_per_eu(stage_waves_per_eu(N, sizeof(T) == 4))))
    stage_kernel(View v, int cur, double dt, double rkA, double rkB, int mode) {
  stage_body<N, T, VISC, FX, SVA>(v, block_element(v.E), cur, dt, rkA, rkB, mode);
}

template <int N, typename T, bool VISC, int FX>
__global__ void __launch_bounds__(nthreads_for(N))
    __attribute__((amdgpu_waves_per_eu(stage_waves_per_eu(N, sizeof(T) == 4))))
    stage_batch_kernel(BatchArgs B, double rkA, double rkB, int mode) {
  int m, e;
  batch_member(B, m, e);
  stage_body<N, T, VISC, FX>(*B.view[m], e, B.cur[m], B.dt[m], rkA, rkB, mode);
}

// ------------------------------------------------------------------ launch helpers
template <int N, typename T, int FX>
inline hipError_t stage_ntx(const View& v, int cur, double dt, double a, double b, int mode,
                            hipStream_t st) {
  const dim3 grid(v.E), block(nthreads_for(N));
  if constexpr (FX == 0) {
    if (v.viscous && v.Fa) {
      hipLaunchKernelGGL((stage_kernel<N, T, true, 0, true>), grid, block, 0, st, v, cur, dt, a, b, mode);
      return hipGetLastError();
    }
  }
  if (v.Fa) return hipErrorInvalidValue;  // the folded SVV term: Navier-Stokes, standard fluxes
  if (v.viscous)
    hipLaunchKernelGGL((stage_kernel<N, T, true, FX>), grid, block, 0, st, v, cur, dt, a, b, mode);
  else
    hipLaunchKernelGGL((stage_kernel<N, T, false, FX>), grid, block, 0, st, v, cur, dt, a, b, mode);
  return hipGetLastError();
}

template <int N, typename T, int FX>
inline hipError_t stage_batch_nt(const BatchArgs& B, bool visc, double a, double b, int mode,
                                 hipStream_t st) {
  const dim3 grid(B.start[B.n]), block(nthreads_for(N));
  if (visc)
    hipLaunchKernelGGL((stage_batch_kernel<N, T, true, FX>), grid, block, 0, st, B, a, b, mode);
  else
    hipLaunchKernelGGL((stage_batch_kernel<N, T, false, FX>), grid, block, 0, st, B, a, b, mode);
  return hipGetLastError();
}

}  // namespace dg
