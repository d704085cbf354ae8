// kernels_mixed.hip -- kernels for meshes whose elements carry their own anisotropic orders
// (N1, N2, N3) (section "Spatial p-adaptation": per-element and per-direction orders; mortar
// coupling of p-nonconforming faces).  Euler equations, FP64.
//
// One workgroup per element, taken from a work list sorted by node count (largest first) so
// that the long elements start early; lanes loop over the element's nodes.  Faces whose two
// sides have equal tangential orders are evaluated pointwise; on the others both traces and
// the owner's normal are interpolated to the Lobatto grid of the larger tangential orders
// (the mortar), the numerical flux is evaluated there, and the result is L2-projected back onto
// the element's own face grid.  Both elements of a face evaluate the mortar flux with the same
// code on the same data; the projections preserve its integral, so the totals are conserved.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dg_device.h"

namespace dg {

constexpr int kMixN = kMixMaxOrder + 1;  // nodes per direction at most
constexpr int kMixNN = kMixN * kMixN * kMixN;
constexpr int kMixNF = kMixN * kMixN;

struct ElemInfo {
  int n[3];
  int nn;
  long off;
};

__device__ __forceinline__ ElemInfo elem_info(const View& v, int e) {
  const int4 q = v.elem[e];
  ElemInfo I;
  I.n[0] = q.x;
  I.n[1] = q.y;
  I.n[2] = q.z;
  I.nn = q.x * q.y * q.z;
  I.off = q.w;
  return I;
}

// tangential directions of a face normal to d (ta < tb)
__device__ __forceinline__ void tangential(int d, int& ta, int& tb) {
  ta = d == 0 ? 1 : 0;
  tb = d == 2 ? 1 : 2;
}

// node of an element with node counts n[] at reference indices ii[]
__device__ __forceinline__ int node_index(const int n[3], int i0, int i1, int i2) {
  return i0 + n[0] * (i1 + n[1] * i2);
}

// node on the face normal to d with index id along d and (p, r) along (ta, tb)
__device__ __forceinline__ int face_node_rt(const int n[3], int d, int id, int p, int r) {
  return d == 0 ? node_index(n, id, p, r) : (d == 1 ? node_index(n, p, id, r) : node_index(n, p, r, id));
}

// Lobatto table pointers of order N (node count n = N + 1)
__device__ __forceinline__ const double* tab_w(const View& v, int n) { return v.tab + v.tab_off[n - 1] + n; }
__device__ __forceinline__ const double* tab_D(const View& v, int n) { return v.tab + v.tab_off[n - 1] + 2 * n; }

// ------------------------------------------------------------------ geometry (FP64)
__global__ void __launch_bounds__(512) geometry_mixed_kernel(View v) {
  const int e = blockIdx.x;
  const ElemInfo I = elem_info(v, e);
  const int t = threadIdx.x;
  const bool act = t < I.nn;
  const int ti = t % I.n[0], tj = (t / I.n[0]) % I.n[1], tk = t / (I.n[0] * I.n[1]);
  const int ii[3] = {ti, tj, tk};
  __shared__ double sD[3][kMixNF + 15], sxi[3][8];
  __shared__ double sXl[3][512], sdX[9][512], sA[3][512];
  for (int d = 0; d < 3; d++) {
    const int n = I.n[d];
    const double* tab = v.tab + v.tab_off[n - 1];
    for (int x = t; x < n * n; x += blockDim.x) sD[d][x] = tab[2 * n + x];
    if (t < n) sxi[d][t] = tab[t];
  }
  __syncthreads();
  const int cell[3] = {e % v.ex, (e / v.ex) % v.ey, e / (v.ex * v.ey)};
  const long off = I.off, nn = I.nn;
  if (act) {
    double loc[3], xu[3], dx[3] = {0, 0, 0};
    for (int d = 0; d < 3; d++) {
      loc[d] = (1.0 + sxi[d][ii[d]]) * 0.5 * v.h[d];
      xu[d] = v.lo[d] + cell[d] * v.h[d] + loc[d];
    }
    if (v.deform) {
      dx[0] = v.amp * sin(xu[1]) * sin(xu[2]);
      dx[1] = v.amp * sin(xu[2]) * sin(xu[0]);
      dx[2] = v.amp * sin(xu[0]) * sin(xu[1]);
    }
    for (int d = 0; d < 3; d++) {
      v.X[off * 3 + d * nn + t] = xu[d] + dx[d];
      sXl[d][t] = loc[d] + dx[d];
    }
  }
  __syncthreads();
  auto dref = [&](const double* f, int d) {
    const int n = I.n[d];
    const int stride = d == 0 ? 1 : (d == 1 ? I.n[0] : I.n[0] * I.n[1]);
    const int b0 = t - ii[d] * stride;
    double s = 0.0;
    for (int m = 0; m < n; m++) s += sD[d][ii[d] * n + m] * f[b0 + m * stride];
    return s;
  };
  if (act)
    for (int m = 0; m < 3; m++)
      for (int d = 0; d < 3; d++) sdX[3 * m + d][t] = dref(sXl[m], d);
  __syncthreads();
  for (int c = 0; c < 3; c++) {
    const int m = (c + 1) % 3, l = (c + 2) % 3;
    if (act)
      for (int d = 0; d < 3; d++) sA[d][t] = sXl[l][t] * sdX[3 * m + d][t];
    __syncthreads();
    if (act) {
      const double c0 = dref(sA[2], 1) - dref(sA[1], 2);
      const double c1 = dref(sA[0], 2) - dref(sA[2], 0);
      const double c2 = dref(sA[1], 0) - dref(sA[0], 1);
      v.Ja[off * 9 + (3 * 0 + c) * nn + t] = -c0;
      v.Ja[off * 9 + (3 * 1 + c) * nn + t] = -c1;
      v.Ja[off * 9 + (3 * 2 + c) * nn + t] = -c2;
    }
    __syncthreads();
  }
  if (act) {
    auto X = [&](int m, int d) { return sdX[3 * m + d][t]; };
    const double J = X(0, 0) * (X(1, 1) * X(2, 2) - X(2, 1) * X(1, 2)) +
                     X(1, 0) * (X(2, 1) * X(0, 2) - X(0, 1) * X(2, 2)) +
                     X(2, 0) * (X(0, 1) * X(1, 2) - X(1, 1) * X(0, 2));
    v.J[off + t] = J;
    v.invJ[off + t] = 1.0 / J;
  }
}

// ------------------------------------------------------------------ initial conditions
__global__ void __launch_bounds__(512) ic_mixed_kernel(View v, int cur, int ic, IcParams P) {
  const int e = blockIdx.x;
  const ElemInfo I = elem_info(v, e);
  const long off = I.off, nn = I.nn;
  for (int q = threadIdx.x; q < I.nn; q += blockDim.x) {
    const double x = v.X[off * 3 + q], y = v.X[off * 3 + nn + q], z = v.X[off * 3 + 2 * nn + q];
    double u[5];
    ic_point(v, ic, P, x, y, z, u);
    for (int c = 0; c < 5; c++) {
      v.U[cur][off * 5 + c * nn + q] = u[c];
      v.dU[off * 5 + c * nn + q] = 0.0;
    }
  }
}

// ------------------------------------------------------------------ stage kernel
// 1D interpolation / projection along the first tangential index of a face array:
// out[c][po + no * r] = sum_p A[po][p] in[c][p + ni * r], for r < nr (A = identity if no == ni)
__device__ __forceinline__ void apply_a(const double* A, int no, int ni, int nr, int ncomp,
                                        const double* in, int in_stride, double* out, int out_stride) {
  for (int x = threadIdx.x; x < ncomp * no * nr; x += blockDim.x) {
    const int c = x / (no * nr), y = x - c * no * nr;
    const int po = y % no, r = y / no;
    double s;
    if (no == ni) {
      s = in[c * in_stride + po + ni * r];
    } else {
      s = 0.0;
      for (int p = 0; p < ni; p++) s += A[po * ni + p] * in[c * in_stride + p + ni * r];
    }
    out[c * out_stride + po + no * r] = s;
  }
}

// ... and along the second: out[c][p + np * ro] = sum_r B[ro][r] in[c][p + np * r]
__device__ __forceinline__ void apply_b(const double* B, int no, int ni, int np, int ncomp,
                                        const double* in, int in_stride, double* out, int out_stride) {
  for (int x = threadIdx.x; x < ncomp * np * no; x += blockDim.x) {
    const int c = x / (np * no), y = x - c * np * no;
    const int p = y % np, ro = y / np;
    double s;
    if (no == ni) {
      s = in[c * in_stride + p + np * ro];
    } else {
      s = 0.0;
      for (int r = 0; r < ni; r++) s += B[ro * ni + r] * in[c * in_stride + p + np * r];
    }
    out[c * out_stride + p + np * ro] = s;
  }
}

template <int BS>
__global__ void __launch_bounds__(BS) mixed_stage_kernel(View v, int cur, double dt, double rkA,
                                                         double rkB, int mode) {
  constexpr int SLOTS = (kMixNN + BS - 1) / BS;
  const int e = v.work[blockIdx.x];
  const ElemInfo I = elem_info(v, e);
  const int t = threadIdx.x;
  const long off = I.off, nn = I.nn;
  const double* __restrict__ Uin = v.U[cur];

  __shared__ double sD[3][kMixNF], sw[3][kMixN];
  __shared__ double sP[7][kMixNN];     // rho, v1, v2, v3, beta, ln rho, ln beta
  __shared__ double sJ3[3][kMixNN];    // Ja^d of the direction being processed
  __shared__ double sF[6][5][kMixNF];  // numerical flux on the element's own face grids
  __shared__ double sL[8][kMixNF];     // mortar work: left trace (5) and owner normal (3)
  __shared__ double sR[5][kMixNF];     //              right trace
  __shared__ double sT[8][kMixNF];     //              tensor-product intermediate

  for (int d = 0; d < 3; d++) {
    const int n = I.n[d];
    for (int x = t; x < n * n; x += BS) sD[d][x] = tab_D(v, n)[x];
    if (t < n) sw[d][t] = tab_w(v, n)[t];
  }
  for (int q = t; q < I.nn; q += BS) {
    double u[5];
    for (int c = 0; c < 5; c++) u[c] = Uin[off * 5 + c * nn + q];
    const Prim<double> P = make_prim<double>(u, v.gamma);
    sP[0][q] = P.rho; sP[1][q] = P.v1; sP[2][q] = P.v2; sP[3][q] = P.v3;
    sP[4][q] = P.beta; sP[5][q] = P.lrho; sP[6][q] = P.lbeta;
  }

  // ---- faces
  for (int f = 0; f < 6; f++) {
    const int d = f >> 1, side = f & 1;
    int ta, tb;
    tangential(d, ta, tb);
    const int ne = v.nbr[e * 6 + f];
    const ElemInfo In = elem_info(v, ne);
    const ElemInfo& IL = side ? I : In;   // owner: the element whose +d face this is
    const ElemInfo& IR = side ? In : I;
    const int naL = IL.n[ta], nbL = IL.n[tb], naR = IR.n[ta], nbR = IR.n[tb];
    const int na = I.n[ta], nb = I.n[tb];
    const long offL = IL.off, offR = IR.off, nnL = IL.nn, nnR = IR.nn;
    const int idL = IL.n[d] - 1;
    if (naL == naR && nbL == nbR) {
      for (int q = t; q < na * nb; q += BS) {
        const int p = q % na, r = q / na;
        const int iL = face_node_rt(IL.n, d, idL, p, r), iR = face_node_rt(IR.n, d, 0, p, r);
        double uL[5], uR[5], S[3];
        for (int c = 0; c < 5; c++) {
          uL[c] = Uin[offL * 5 + c * nnL + iL];
          uR[c] = Uin[offR * 5 + c * nnR + iR];
        }
        for (int c = 0; c < 3; c++) S[c] = v.Ja[offL * 9 + (3 * d + c) * nnL + iL];
        double F[5];
        face_flux<double>(v.surf, uL, uR, S, v.gamma, F);
        for (int c = 0; c < 5; c++) sF[f][c][q] = F[c];
      }
      continue;
    }
    const int ma = naL > naR ? naL : naR, mb = nbL > nbR ? nbL : nbR;
    __syncthreads();  // mortar work arrays free
    for (int q = t; q < naL * nbL; q += BS) {
      const int p = q % naL, r = q / naL;
      const int iL = face_node_rt(IL.n, d, idL, p, r);
      for (int c = 0; c < 5; c++) sL[c][q] = Uin[offL * 5 + c * nnL + iL];
      for (int c = 0; c < 3; c++) sL[5 + c][q] = v.Ja[offL * 9 + (3 * d + c) * nnL + iL];
    }
    for (int q = t; q < naR * nbR; q += BS) {
      const int p = q % naR, r = q / naR;
      const int iR = face_node_rt(IR.n, d, 0, p, r);
      for (int c = 0; c < 5; c++) sR[c][q] = Uin[offR * 5 + c * nnR + iR];
    }
    __syncthreads();
    // interpolate to the mortar grid (ma x mb): along the first tangential index, then the second
    const double* mt = v.mtab;
    const double* IaL = naL < ma ? mt + v.mort_off[naL - 1][ma - 1] : nullptr;
    const double* IbL = nbL < mb ? mt + v.mort_off[nbL - 1][mb - 1] : nullptr;
    const double* IaR = naR < ma ? mt + v.mort_off[naR - 1][ma - 1] : nullptr;
    const double* IbR = nbR < mb ? mt + v.mort_off[nbR - 1][mb - 1] : nullptr;
    apply_a(IaL, ma, naL, nbL, 8, &sL[0][0], kMixNF, &sT[0][0], kMixNF);
    __syncthreads();
    apply_b(IbL, mb, nbL, ma, 8, &sT[0][0], kMixNF, &sL[0][0], kMixNF);
    __syncthreads();
    apply_a(IaR, ma, naR, nbR, 5, &sR[0][0], kMixNF, &sT[0][0], kMixNF);
    __syncthreads();
    apply_b(IbR, mb, nbR, ma, 5, &sT[0][0], kMixNF, &sR[0][0], kMixNF);
    __syncthreads();
    for (int q = t; q < ma * mb; q += BS) {
      double uL[5], uR[5], S[3], F[5];
      for (int c = 0; c < 5; c++) {
        uL[c] = sL[c][q];
        uR[c] = sR[c][q];
      }
      for (int c = 0; c < 3; c++) S[c] = sL[5 + c][q];
      face_flux<double>(v.surf, uL, uR, S, v.gamma, F);
      for (int c = 0; c < 5; c++) sL[c][q] = F[c];  // mortar flux replaces the left trace
    }
    __syncthreads();
    // project onto the element's own face grid (na x nb)
    const double* Pa = na < ma ? mt + v.mort_off[na - 1][ma - 1] + ma * na : nullptr;
    const double* Pb = nb < mb ? mt + v.mort_off[nb - 1][mb - 1] + mb * nb : nullptr;
    apply_a(Pa, na, ma, mb, 5, &sL[0][0], kMixNF, &sT[0][0], kMixNF);
    __syncthreads();
    apply_b(Pb, nb, mb, na, 5, &sT[0][0], kMixNF, &sF[f][0][0], kMixNF);
  }
  __syncthreads();

  // ---- volume (every pair evaluated from both nodes), surface lift, update
  double acc[SLOTS][5];
  for (int s = 0; s < SLOTS; s++)
    for (int c = 0; c < 5; c++) acc[s][c] = 0.0;
  const double ce = 0.5 / (v.gamma - 1.0), gm1 = v.gamma - 1.0;
  for (int d = 0; d < 3; d++) {
    __syncthreads();
    for (int q = t; q < I.nn; q += BS)
      for (int c = 0; c < 3; c++) sJ3[c][q] = v.Ja[off * 9 + (3 * d + c) * nn + q];
    __syncthreads();
    const int n = I.n[d];
    const int stride = d == 0 ? 1 : (d == 1 ? I.n[0] : I.n[0] * I.n[1]);
#pragma unroll
    for (int s = 0; s < SLOTS; s++) {
      const int q = t + s * BS;
      if (q >= I.nn) continue;
      const int ii[3] = {q % I.n[0], (q / I.n[0]) % I.n[1], q / (I.n[0] * I.n[1])};
      const int id = ii[d];
      const int b0 = q - id * stride;
      Prim<double> A;
      A.rho = sP[0][q]; A.v1 = sP[1][q]; A.v2 = sP[2][q]; A.v3 = sP[3][q];
      A.beta = sP[4][q]; A.lrho = sP[5][q]; A.lbeta = sP[6][q];
      A.h = 0.5 * (A.v1 * A.v1 + A.v2 * A.v2 + A.v3 * A.v3);
      for (int m = 0; m < n; m++) {
        if (m == id) continue;
        const int qm = b0 + m * stride;
        Prim<double> B;
        B.rho = sP[0][qm]; B.v1 = sP[1][qm]; B.v2 = sP[2][qm]; B.v3 = sP[3][qm];
        B.beta = sP[4][qm]; B.lrho = sP[5][qm]; B.lbeta = sP[6][qm];
        B.h = 0.5 * (B.v1 * B.v1 + B.v2 * B.v2 + B.v3 * B.v3);
        double F[5];
        vol_flux<double>(v.vol, A, B, sJ3[0][q] + sJ3[0][qm], sJ3[1][q] + sJ3[1][qm],
                         sJ3[2][q] + sJ3[2][qm], ce, gm1, F);
        const double Dm = sD[d][id * n + m];
        for (int c = 0; c < 5; c++) acc[s][c] += Dm * F[c];
      }
      int ta, tb;
      tangential(d, ta, tb);
      const int qf = ii[ta] + I.n[ta] * ii[tb];
      if (id == n - 1)
        for (int c = 0; c < 5; c++) acc[s][c] += sF[2 * d + 1][c][qf] / sw[d][n - 1];
      if (id == 0)
        for (int c = 0; c < 5; c++) acc[s][c] -= sF[2 * d][c][qf] / sw[d][0];
    }
  }
#pragma unroll
  for (int s = 0; s < SLOTS; s++) {
    const int q = t + s * BS;
    if (q >= I.nn) continue;
    const double ij = v.invJ[off + q];
    const long o = off * 5 + q;
    for (int c = 0; c < 5; c++) {
      const double R = -acc[s][c] * ij;
      if (mode == kModeResidual) {
        v.R[o + c * nn] = R;
      } else {
        const double du = (rkA == 0.0 ? 0.0 : rkA * v.dU[o + c * nn]) + dt * R;
        v.dU[o + c * nn] = du;
        v.U[cur ^ 1][o + c * nn] = Uin[o + c * nn] + rkB * du;
      }
    }
  }
}

// ------------------------------------------------------------------ diagnostics (FP64)
// same slots as the uniform-order diagnostics
__global__ void __launch_bounds__(512) diag_mixed_kernel(View v, int cur) {
  const int e = blockIdx.x;
  const ElemInfo I = elem_info(v, e);
  const int t = threadIdx.x;
  const bool act = t < I.nn;
  const long off = I.off, nn = I.nn;
  const int ii[3] = {t % I.n[0], (t / I.n[0]) % I.n[1], t / (I.n[0] * I.n[1])};
  __shared__ double sD[3][kMixNF], sw[3][kMixN];
  __shared__ double sV[3][512];
  __shared__ double red[512];
  for (int d = 0; d < 3; d++) {
    const int n = I.n[d];
    for (int x = t; x < n * n; x += blockDim.x) sD[d][x] = tab_D(v, n)[x];
    if (t < n) sw[d][t] = tab_w(v, n)[t];
  }
  double u[5] = {0, 0, 0, 0, 0};
  if (act) {
    for (int c = 0; c < 5; c++) u[c] = v.U[cur][off * 5 + c * nn + t];
    for (int c = 0; c < 3; c++) sV[c][t] = u[1 + c] / u[0];
  }
  __syncthreads();
  double s[kDiagSlots];
  for (int k = 0; k < kDiagSlots; k++) s[k] = 0.0;
  s[9] = -INFINITY;
  s[10] = INFINITY;
  s[11] = INFINITY;
  if (act) {
    const double g = v.gamma;
    const double wq = sw[0][ii[0]] * sw[1][ii[1]] * sw[2][ii[2]] * v.J[off + t];
    const double ij = v.invJ[off + t];
    const double rho = u[0];
    const double v1 = sV[0][t], v2 = sV[1][t], v3 = sV[2][t];
    const double q2 = v1 * v1 + v2 * v2 + v3 * v3;
    const double p = (g - 1) * (u[4] - 0.5 * rho * q2);
    int bad = 0;
    for (int c = 0; c < 5; c++) {
      s[c] = wq * u[c];
      bad += isfinite(u[c]) ? 0 : 1;
    }
    const double sp = log(p) - g * log(rho);
    s[5] = wq * (-rho * sp);
    s[6] = s[5] / (g - 1);
    s[7] = wq * 0.5 * rho * q2;
    double dv[3][3];
    for (int d = 0; d < 3; d++) {
      const int n = I.n[d];
      const int stride = d == 0 ? 1 : (d == 1 ? I.n[0] : I.n[0] * I.n[1]);
      const int b0 = t - ii[d] * stride;
      for (int c = 0; c < 3; c++) {
        double a = 0.0;
        for (int m = 0; m < n; m++) a += sD[d][ii[d] * n + m] * sV[c][b0 + m * stride];
        dv[d][c] = a;
      }
    }
    double gv[3][3];
    for (int c = 0; c < 3; c++)
      for (int x = 0; x < 3; x++) {
        double a = 0.0;
        for (int d = 0; d < 3; d++) a += v.Ja[off * 9 + (3 * d + x) * nn + t] * dv[d][c];
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
  for (int k = 0; k < 15; k++) {
    red[t] = s[k];
    __syncthreads();
    for (int w = 256; w > 0; w >>= 1) {
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

// ------------------------------------------------------------------ launchers
hipError_t launch_geometry_mixed(const View& v, hipStream_t st) {
  hipLaunchKernelGGL(geometry_mixed_kernel, dim3(v.E), dim3(512), 0, st, v);
  return hipGetLastError();
}

hipError_t launch_ic_mixed(const View& v, int cur, int ic, const double* params, hipStream_t st) {
  IcParams P;
  for (int k = 0; k < 9; k++) P.p[k] = params ? params[k] : 0.0;
  hipLaunchKernelGGL(ic_mixed_kernel, dim3(v.E), dim3(512), 0, st, v, cur, ic, P);
  return hipGetLastError();
}

hipError_t launch_stage_mixed(const View& v, int cur, double dt, double rkA, double rkB, int mode,
                              int block, hipStream_t st) {
  switch (block) {
    case 128:
      hipLaunchKernelGGL(mixed_stage_kernel<128>, dim3(v.E), dim3(128), 0, st, v, cur, dt, rkA, rkB, mode);
      break;
    case 512:
      hipLaunchKernelGGL(mixed_stage_kernel<512>, dim3(v.E), dim3(512), 0, st, v, cur, dt, rkA, rkB, mode);
      break;
    default:
      hipLaunchKernelGGL(mixed_stage_kernel<256>, dim3(v.E), dim3(256), 0, st, v, cur, dt, rkA, rkB, mode);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_diagnostics_mixed(const View& v, int cur, hipStream_t st) {
  hipLaunchKernelGGL(diag_mixed_kernel, dim3(v.E), dim3(512), 0, st, v, cur);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return launch_diag_final(v, st);
}

}  // namespace dg
