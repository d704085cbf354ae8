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

// Lobatto table pointers of order N (node count n = N + 1)
// (the member arrays of the kernel argument are read with constant indices and a select: a
// runtime index makes the compiler copy the whole argument to private memory)
__device__ __forceinline__ int tab_offset(const View& v, int n) {
  int o = v.tab_off[0];
#pragma unroll
  for (int k = 1; k < kMixN; k++) o = n - 1 == k ? v.tab_off[k] : o;
  return o;
}
__device__ __forceinline__ const double* tab_w(const View& v, int n) { return v.tab + tab_offset(v, n) + n; }
__device__ __forceinline__ const double* tab_D(const View& v, int n) { return v.tab + tab_offset(v, n) + 2 * n; }
__device__ __forceinline__ double* state(const View& v, int k) { return k ? v.U[1] : v.U[0]; }

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

// lanes of a workgroup for elements of up to nnmax nodes, npl nodes per lane (whole waves)
__host__ __device__ constexpr int mix_lanes(int nnmax, int npl) { return ((nnmax + npl - 1) / npl + 63) / 64 * 64; }

// q / n for 0 <= q < 4096 and 1 <= n <= 64, from inv_n = 1.0f / n: (q + 1/2)/n lies at least
// 1/(2n) away from an integer, far more than the rounding error of the FP32 product (checked
// for every q and n in that range).
__device__ __forceinline__ int sdiv(int q, float inv_n) { return (int)(((float)q + 0.5f) * inv_n); }

// ------------------------------------------------------------------ stage: faces
// One 64-lane workgroup (a single wave) per face: the face normal to d between the owner L (its
// +xi_d side) and R = nbr(L, +d), with L's metric Ja^d as the scaled normal.  Traces are staged
// in LDS, interpolated to the mortar of the larger tangential orders (the identity where the
// orders agree), the numerical flux is evaluated at the mortar points, and it is L2-projected
// onto the face grids of both elements: Fs[e][f][c][p + n_a r], f = 2 d + side of element e,
// c = 0..4 the flux and c = 5 its FP64 mass component (FP32-bulk).  Each face is evaluated once.
// In each tangential direction at most one side has fewer nodes than the mortar: only that side
// is interpolated and projected along it (the other side's data already lies on the mortar
// grid and is used in place), so every loop has a trip count and branches that are uniform over
// the wave.
constexpr int kFsFace = 6 * kMixNF;  // doubles per element face in Fs

// XS: the extended surface fluxes (codes >= 4), compiled apart so that the others keep their
// registers
template <typename T, bool XS>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(XS ? 3 : 4)))
    mixed_face_kernel(View v, int cur) {
  constexpr bool DEV = sizeof(T) == 4;
  constexpr int NC = DEV ? 6 : 5;
  static_assert(kMixNF <= 64, "a face grid, or a mortar matrix, fits one wave");
  const int fid = block_element(3 * v.E);
  const int e = fid / 3, d = fid - 3 * e;
  const int t = threadIdx.x;
  const double* __restrict__ Uin = v.U[cur];
  const Ref Rf = make_ref(v.rho_r, v.p_r, v.gamma);
  // the face's table entry: R, both elements' node counts and first nodes (one load, where the
  // neighbour and then its element entry would be two in sequence)
  const int4 fd = v.fdesc[fid];
  const int eR = fd.x;
  const int nL0 = fd.y & 7, nL1 = (fd.y >> 3) & 7, nL2 = (fd.y >> 6) & 7;
  const int nR0 = (fd.y >> 9) & 7, nR1 = (fd.y >> 12) & 7, nR2 = (fd.y >> 15) & 7;
  // node counts along a and b, and node strides (selected by d: an array indexed by a runtime
  // value would be kept in private memory)
  const int naL = d == 0 ? nL1 : nL0, nbL = d == 2 ? nL1 : nL2;
  const int naR = d == 0 ? nR1 : nR0, nbR = d == 2 ? nR1 : nR2;
  const int ma = naL > naR ? naL : naR, mb = nbL > nbR ? nbL : nbR;
  const float ima = 1.0f / (float)ma;
  // the side (0 = L, 1 = R, -1 = none) with fewer nodes than the mortar along a and along b
  const int sa = naL < ma ? 0 : (naR < ma ? 1 : -1);
  const int sb = nbL < mb ? 0 : (nbR < mb ? 1 : -1);
  // na_s, nb_a: the a-side's node counts along a and b; nb_s: the b-side's node count along b
  const int na_s = sa == 0 ? naL : naR, nb_a = sa == 0 ? nbL : nbR, nb_s = sb == 0 ? nbL : nbR;
  // sA: rows 0-4 L's state, 5-7 L's Ja^d (L's grid), rows 8-12 R's state (R's grid); later
  // rows 0-5 the flux on the mortar.  sB: the side interpolated along a (up to 8 rows), later
  // the flux projected along a onto that side's grid (up to 6 rows).
  __shared__ double sA[13][kMixNF], sB[8][kMixNF];
  // interpolation to the mortar and projection back, along a and along b (only the sides
  // that need them)
  __shared__ double sIa[kMixNF], sPa[kMixNF], sIb[kMixNF], sPb[kMixNF];
  // Every operand is requested before any is stored (one lane per point or matrix entry, the
  // indices clamped so that no load waits on a branch): the traces on their own grids (index
  // p + n_a r) and the mortar matrices.
  const int sLa = d == 0 ? nL0 : 1, sLb = d == 2 ? nL0 : nL0 * nL1;
  const int sRa = d == 0 ? nR0 : 1, sRb = d == 2 ? nR0 : nR0 * nR1;
  const int baseL = d == 0 ? nL0 - 1 : (d == 1 ? (nL1 - 1) * nL0 : (nL2 - 1) * nL0 * nL1);
  const long offL = fd.z, offR = fd.w, nnL = nL0 * nL1 * nL2, nnR = nR0 * nR1 * nR2;
  double tL[8], tR[5];
  {
    const int x = t < naL * nbL ? t : 0;
    const int r = sdiv(x, 1.0f / (float)naL), p = x - r * naL;
    const int q = baseL + p * sLa + r * sLb;
#pragma unroll
    for (int c = 0; c < 5; c++) tL[c] = Uin[offL * 5 + c * nnL + q];
#pragma unroll
    for (int c = 0; c < 3; c++) tL[5 + c] = v.Ja[offL * 9 + (3 * d + c) * nnL + q];
  }
  {
    const int y = t < naR * nbR ? t : 0;
    const int r = sdiv(y, 1.0f / (float)naR), p = y - r * naR;
    const int q = p * sRa + r * sRb;
#pragma unroll
    for (int c = 0; c < 5; c++) tR[c] = Uin[offR * 5 + c * nnR + q];
  }
  const double* mt = v.mtab;
  double tIa = 0.0, tPa = 0.0, tIb = 0.0, tPb = 0.0;
  if (sa >= 0) {
    const double* src = mt + v.mort_off[na_s - 1][ma - 1];
    const int x = t < ma * na_s ? t : 0;
    tIa = src[x];
    tPa = src[ma * na_s + x];
  }
  if (sb >= 0) {
    const double* src = mt + v.mort_off[nb_s - 1][mb - 1];
    const int x = t < mb * nb_s ? t : 0;
    tIb = src[x];
    tPb = src[mb * nb_s + x];
  }
  if (t < naL * nbL) {
#pragma unroll
    for (int c = 0; c < 8; c++) sA[c][t] = tL[c];
  }
  if (t < naR * nbR) {
#pragma unroll
    for (int c = 0; c < 5; c++) sA[8 + c][t] = tR[c];
  }
  if (sa >= 0 && t < ma * na_s) {
    sIa[t] = tIa;
    sPa[t] = tPa;
  }
  if (sb >= 0 && t < mb * nb_s) {
    sIb[t] = tIb;
    sPb[t] = tPb;
  }
  __syncthreads();
  // along a: the smaller side to the mortar (index pm + ma r); its fields are L's 8 or R's 5.
  // Each weight is read once and applied to every field (the sum over p of each field keeps its
  // order).
  if (sa >= 0) {
    const int c0 = sa == 0 ? 0 : 8, nc = sa == 0 ? 8 : 5;
    for (int y = t; y < ma * nb_a; y += 64) {
      const int r = sdiv(y, ima), pm = y - r * ma;
      double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int p = 0; p < na_s; p++) {
        const double w = sIa[pm * na_s + p];
        const int x = p + na_s * r;
#pragma unroll
        for (int c = 0; c < 8; c++)
          if (c < nc) s[c] += w * sA[c0 + c][x];
      }
#pragma unroll
      for (int c = 0; c < 8; c++)
        if (c < nc) sB[c][y] = s[c];
    }
  }
  __syncthreads();
  // along b, and the numerical flux at the mortar point (ma mb <= 49 points: one pass)
  {
    const int x = t;
    const bool on = x < ma * mb;
    const int rm = sdiv(x, ima), pm = x - rm * ma;
    double a[13];
    // L's 8 fields (rows of sB if L was interpolated along a), then R's 5
    const double(*rowsL)[kMixNF] = sa == 0 ? sB : sA;
    const double(*rowsR)[kMixNF] = sa == 1 ? sB : sA + 8;
    if (nbL == mb) {
#pragma unroll
      for (int c = 0; c < 8; c++) a[c] = on ? rowsL[c][pm + ma * rm] : 0.0;
    } else {
#pragma unroll
      for (int c = 0; c < 8; c++) a[c] = 0.0;
      if (on)
        for (int r = 0; r < nbL; r++) {
          const double w = sIb[rm * nbL + r];
#pragma unroll
          for (int c = 0; c < 8; c++) a[c] += w * rowsL[c][pm + ma * r];
        }
    }
    if (nbR == mb) {
#pragma unroll
      for (int c = 0; c < 5; c++) a[8 + c] = on ? rowsR[c][pm + ma * rm] : 0.0;
    } else {
#pragma unroll
      for (int c = 0; c < 5; c++) a[8 + c] = 0.0;
      if (on)
        for (int r = 0; r < nbR; r++) {
          const double w = sIb[rm * nbR + r];
#pragma unroll
          for (int c = 0; c < 5; c++) a[8 + c] += w * rowsR[c][pm + ma * r];
        }
    }
    __syncthreads();  // every mortar point has read its data before the flux rows overwrite sA
    if (on) {
      const double uL[5] = {a[0], a[1], a[2], a[3], a[4]};
      const double S[3] = {a[5], a[6], a[7]};
      const double uR[5] = {a[8], a[9], a[10], a[11], a[12]};
      T F[5];
      if (DEV) {
        double F0d;
        face_flux_dev<T>(v.surf, uL, uR, S, v.gamma, Rf, F, F0d);
        sA[5][x] = F0d;
      } else {
        face_flux<T, XS>(v.surf, uL, uR, S, v.gamma, F, XS && v.surf == 8 ? v.adapt[3] : 0.0);
      }
#pragma unroll
      for (int c = 0; c < 5; c++) sA[c][x] = (double)F[c];
    }
  }
  __syncthreads();
  // L2 projection along a onto the smaller side's grid (index po + na rm), into sB
  if (sa >= 0) {
    const float ina_s = 1.0f / (float)na_s;
    for (int y = t; y < na_s * mb; y += 64) {
      const int rm = sdiv(y, ina_s), po = y - rm * na_s;
      double s[NC];
#pragma unroll
      for (int c = 0; c < NC; c++) s[c] = 0.0;
      for (int pm = 0; pm < ma; pm++) {
        const double w = sPa[po * ma + pm];
#pragma unroll
        for (int c = 0; c < NC; c++) s[c] += w * sA[c][pm + ma * rm];
      }
#pragma unroll
      for (int c = 0; c < NC; c++) sB[c][y] = s[c];
    }
  }
  __syncthreads();
  // along b onto each side's face grid, into Fs
#pragma unroll
  for (int side = 0; side < 2; side++) {
    const int na = side ? naR : naL, nb = side ? nbR : nbL;
    const double(*src)[kMixNF] = sa == side ? sB : sA;  // the flux along a on this side's grid
    double* out = v.Fs + ((long)(side ? eR : e) * 6 + (side ? 2 * d : 2 * d + 1)) * kFsFace;
    const float ina = 1.0f / (float)na;
    for (int y = t; y < na * nb; y += 64) {
      const int ro = sdiv(y, ina), po = y - ro * na;
      double s[NC];
      if (nb == mb) {
#pragma unroll
        for (int c = 0; c < NC; c++) s[c] = src[c][po + na * ro];
      } else {
#pragma unroll
        for (int c = 0; c < NC; c++) s[c] = 0.0;
        for (int rm = 0; rm < mb; rm++) {
          const double w = sPb[ro * mb + rm];
#pragma unroll
          for (int c = 0; c < NC; c++) s[c] += w * src[c][po + na * rm];
        }
      }
#pragma unroll
      for (int c = 0; c < NC; c++) out[c * kMixNF + y] = s[c];
    }
  }
}

// ------------------------------------------------------------------ stage: volume and update
// Elements are launched by bucket: bucket b holds the elements of 64 b < nn <= 64 (b + 1) nodes,
// a contiguous range of the work list (sorted by node count).  A lane holds NPL nodes (1 or 2,
// the autotuner's choice per bucket), so the workgroup has mix_lanes(NNMAX, NPL) lanes.  KEP
// selects the kinetic-energy-preserving volume fluxes (compiled apart, FP64 only).
// Bound on the face points of an element of at most nnmax nodes (sum over its six faces of the
// tangential node counts' products), for 1 <= n_d <= kMixN.
__host__ __device__ constexpr int mix_face_points(int nnmax) {
  int best = 0;
  for (int a = 1; a <= kMixN; a++)
    for (int b = 1; b <= kMixN; b++)
      for (int c = 1; c <= kMixN; c++)
        if (a * b * c <= nnmax) {
          const int f = 2 * (a * b + b * c + a * c);
          if (f > best) best = f;
        }
  return best;
}

template <int NNMAX, int NPL, typename T, bool KEP>
__global__ void __launch_bounds__(mix_lanes(NNMAX, NPL))
    mixed_stage_kernel(View v, int wbeg, int cur, double dt, double rkA, double rkB, int mode) {
  constexpr int BS = mix_lanes(NNMAX, NPL);
  constexpr bool DEV = sizeof(T) == 4;  // FP32-bulk: deviation form, FP64 mass flux
  constexpr int NC = DEV ? 6 : 5;       // face flux components read (FP32-bulk: + FP64 mass)
  constexpr int NFS = NC * mix_face_points(NNMAX);
  constexpr int KF = (NFS + BS - 1) / BS;  // face flux values per lane
  const int4 wi = v.work[wbeg + blockIdx.x];
  const int e = wi.x;
  ElemInfo I;
  I.n[0] = wi.y & 7;
  I.n[1] = (wi.y >> 3) & 7;
  I.n[2] = (wi.y >> 6) & 7;
  I.off = wi.z;
  I.nn = wi.w;
  const int t = threadIdx.x;
  const long off = I.off, nn = I.nn;
  const double* __restrict__ Uin = state(v, cur);
  const double* __restrict__ Fs = v.Fs + (long)e * 6 * kFsFace;
  const Ref Rf = make_ref(v.rho_r, v.p_r, v.gamma);
  const int str[3] = {1, I.n[0], I.n[0] * I.n[1]};
  const float inv0 = 1.0f / (float)I.n[0], inv01 = 1.0f / (float)str[2];
  // face points of the faces normal to each direction, and where face f's fluxes start in sFs
  // (the element's faces packed: f = 2 d + side, component-major within a face)
  const int n0 = I.n[0], n1 = I.n[1], n2 = I.n[2];
  const int pt0 = n1 * n2, pt1 = n0 * n2, pt2 = n0 * n1;
  const float ip0 = 1.0f / (float)pt0, ip1 = 1.0f / (float)pt1, ip2 = 1.0f / (float)pt2;
  const int fo1 = NC * pt0, fo2 = 2 * NC * pt0, fo3 = fo2 + NC * pt1, fo4 = fo2 + 2 * NC * pt1,
            fo5 = fo4 + NC * pt2, fend = fo4 + 2 * NC * pt2;

  __shared__ double sD[3][kMixNF], sw[3][kMixN];
  __shared__ T sP[7][NNMAX];             // rho, v1, v2, v3, beta, ln rho, ln beta (FP32-bulk: deviations)
  constexpr int NV = DEV ? NNMAX : 1;
  __shared__ double sVd[3][NV];          // FP32-bulk: FP64 velocities for the mass flux
  __shared__ double sJ3[3][NNMAX];       // Ja^d of the direction in work
  __shared__ double sFs[NFS];            // the element's face fluxes

  // Every operand of the element is requested before any is used: state, the first direction's
  // metric terms, the face fluxes and the tables (the tables with clamped indices, so that no
  // load waits on a branch).
  double u[NPL][5], jn[NPL][3];
#pragma unroll
  for (int s = 0; s < NPL; s++) {
    const int q = t + s * BS;
    const int qc = q < I.nn ? q : 0;
#pragma unroll
    for (int c = 0; c < 5; c++) u[s][c] = Uin[off * 5 + c * nn + qc];
#pragma unroll
    for (int c = 0; c < 3; c++) jn[s][c] = v.Ja[off * 9 + c * nn + qc];
  }
  double fv[KF];
#pragma unroll
  for (int k = 0; k < KF; k++) {
    const int x = t + k * BS;
    // face f of packed entry x, its component c and point q
    const int f = x < fo1 ? 0 : (x < fo2 ? 1 : (x < fo3 ? 2 : (x < fo4 ? 3 : (x < fo5 ? 4 : 5))));
    const int fb = f == 0 ? 0 : (f == 1 ? fo1 : (f == 2 ? fo2 : (f == 3 ? fo3 : (f == 4 ? fo4 : fo5))));
    const int pf = f < 2 ? pt0 : (f < 4 ? pt1 : pt2);
    const int c = sdiv(x - fb, f < 2 ? ip0 : (f < 4 ? ip1 : ip2)), q = x - fb - c * pf;
    fv[k] = x < fend ? Fs[f * kFsFace + c * kMixNF + q] : 0.0;
  }
  double tD[3], tw[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const int n = I.n[d];
    tD[d] = tab_D(v, n)[t < n * n ? t : 0];
    tw[d] = tab_w(v, n)[t < n ? t : 0];
  }
  static_assert(BS >= kMixNF, "one table entry per lane");
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const int n = I.n[d];
    if (t < n * n) sD[d][t] = tD[d];
    if (t < n) sw[d][t] = tw[d];
  }
#pragma unroll
  for (int k = 0; k < KF; k++)
    if (t + k * BS < fend) sFs[t + k * BS] = fv[k];

  int ii[NPL][3];
#pragma unroll
  for (int s = 0; s < NPL; s++) {
    const int q = t + s * BS;
    const int k = sdiv(q, inv01), rem = q - k * str[2];
    const int j = sdiv(rem, inv0);
    ii[s][0] = rem - j * I.n[0];
    ii[s][1] = j;
    ii[s][2] = k;
    if (q < I.nn) {
      const Prim<T> P = DEV ? make_prim_dev<T>(u[s], v.gamma, Rf) : make_prim<T>(u[s], v.gamma);
      sP[0][q] = P.rho; sP[1][q] = P.v1; sP[2][q] = P.v2; sP[3][q] = P.v3;
      sP[4][q] = P.beta; sP[5][q] = P.lrho; sP[6][q] = P.lbeta;
      if (DEV) {
        const double ir = rcp(u[s][0]);
        sVd[0][q] = u[s][1] * ir;
        sVd[1][q] = u[s][2] * ir;
        sVd[2][q] = u[s][3] * ir;
      }
    }
  }

  // For each node and direction: sum over the line of D_im F#(U_i, U_m; Ja_i + Ja_m), then the
  // surface lift of the face fluxes.  Slot s of the lane holds node t + s BS.
  T acc[NPL][5];
  double accm[NPL];  // FP32-bulk: FP64 mass accumulators
#pragma unroll
  for (int s = 0; s < NPL; s++) {
#pragma unroll
    for (int c = 0; c < 5; c++) acc[s][c] = 0;
    accm[s] = 0.0;
  }
  const T ce = (T)(0.5 / (v.gamma - 1.0)), gm1 = (T)(v.gamma - 1.0);
  // Direction d's parameters are passed in, and every per-direction choice is a select of
  // values: an array indexed by the runtime d, or a select between captured variables, would keep
  // the lambda's captures (the kernel argument among them) in private memory.
  //   n, sd: node count and node stride along d; pf: points of a face normal to d; flo, fhi:
  //   where the fluxes of the faces at index 0 and n - 1 along d start in sFs
  auto node_volume = [&](const int d, const int n, const int sd, const int pf, const int flo, const int fhi,
                         const int q, const int* iq, T* acc, double& accm) {
    const int id = d == 0 ? iq[0] : (d == 1 ? iq[1] : iq[2]);
    const int b0 = q - id * sd;
    Prim<T> A;
    A.rho = sP[0][q]; A.v1 = sP[1][q]; A.v2 = sP[2][q]; A.v3 = sP[3][q];
    A.beta = sP[4][q]; A.lrho = sP[5][q]; A.lbeta = sP[6][q];
    A.h = (T)0.5 * (A.v1 * A.v1 + A.v2 * A.v2 + A.v3 * A.v3);
    const double ja0 = sJ3[0][q], ja1 = sJ3[1][q], ja2 = sJ3[2][q];
    for (int m = 0; m < n; m++) {
      if (m == id) continue;
      const int qm = b0 + m * sd;
      Prim<T> B;
      B.rho = sP[0][qm]; B.v1 = sP[1][qm]; B.v2 = sP[2][qm]; B.v3 = sP[3][qm];
      B.beta = sP[4][qm]; B.lrho = sP[5][qm]; B.lbeta = sP[6][qm];
      B.h = (T)0.5 * (B.v1 * B.v1 + B.v2 * B.v2 + B.v3 * B.v3);
      const double md[3] = {ja0 + sJ3[0][qm], ja1 + sJ3[1][qm], ja2 + sJ3[2][qm]};
      T F[5];
      double F0d = 0.0;
      if (DEV) {
        const double va[3] = {sVd[0][q], sVd[1][q], sVd[2][q]};
        const double vb[3] = {sVd[0][qm], sVd[1][qm], sVd[2][qm]};
        if (v.vol == 0) {
          const double vn64 = 0.5 * ((va[0] + vb[0]) * md[0] + (va[1] + vb[1]) * md[1] + (va[2] + vb[2]) * md[2]);
          flux_ec_dev(A, B, (T)md[0], (T)md[1], (T)md[2], vn64, Rf, F, F0d);
        } else {
          flux_central_dev(A, B, (T)md[0], (T)md[1], (T)md[2], va, vb, md, Rf, F, F0d);
        }
      } else {
        vol_flux<T, KEP>(v.vol, A, B, (T)md[0], (T)md[1], (T)md[2], ce, gm1, F);
      }
      const double Dm = sD[d][id * n + m];
#pragma unroll
      for (int c = 0; c < 5; c++) acc[c] += (T)Dm * F[c];
      if (DEV) accm += Dm * F0d;
    }
    // the node's point on the faces normal to d (tangential indices in increasing direction)
    const int qf = d == 0 ? iq[1] + n1 * iq[2] : (d == 1 ? iq[0] + n0 * iq[2] : iq[0] + n0 * iq[1]);
    if (id == n - 1) {
      const double iw = 1.0 / sw[d][n - 1];
      const double* F = sFs + fhi;
#pragma unroll
      for (int c = 0; c < 5; c++) acc[c] += (T)(iw * F[c * pf + qf]);
      if (DEV) accm += iw * F[5 * pf + qf];
    }
    if (id == 0) {
      const double iw = 1.0 / sw[d][0];
      const double* F = sFs + flo;
#pragma unroll
      for (int c = 0; c < 5; c++) acc[c] -= (T)(iw * F[c * pf + qf]);
      if (DEV) accm -= iw * F[5 * pf + qf];
    }
  };
  for (int d = 0; d < 3; d++) {
    __syncthreads();  // the previous direction's metric is no longer read
#pragma unroll
    for (int s = 0; s < NPL; s++)
      if (t + s * BS < I.nn)
#pragma unroll
        for (int c = 0; c < 3; c++) sJ3[c][t + s * BS] = jn[s][c];
    __syncthreads();
    if (d < 2) {  // the next direction's metric terms, in flight during this direction's sums
#pragma unroll
      for (int s = 0; s < NPL; s++) {
        const int q = t + s * BS;
        const int qc = q < I.nn ? q : 0;
#pragma unroll
        for (int c = 0; c < 3; c++) jn[s][c] = v.Ja[off * 9 + (3 * (d + 1) + c) * nn + qc];
      }
    }
    const int n = d == 0 ? n0 : (d == 1 ? n1 : n2), sd = d == 0 ? 1 : (d == 1 ? n0 : n0 * n1);
    const int pf = d == 0 ? pt0 : (d == 1 ? pt1 : pt2);
    const int flo = d == 0 ? 0 : (d == 1 ? fo2 : fo4), fhi = d == 0 ? fo1 : (d == 1 ? fo3 : fo5);
    // one call site (unrolled after inlining)
#pragma unroll
    for (int s = 0; s < NPL; s++)
      if (t + s * BS < I.nn) node_volume(d, n, sd, pf, flo, fhi, t + s * BS, ii[s], acc[s], accm[s]);
  }
  auto node_update = [&](const int q, const T* acc, const double accm) {
    const long o = off * 5 + q;
    const double ij = v.invJ[off + q];
    double R[5];
#pragma unroll
    for (int c = 0; c < 5; c++) R[c] = -(double)acc[c] * ij;
    if (DEV) {  // FP64 mass; energy = H_r (mass) + deviation
      R[0] = -accm * ij;
      R[4] -= Rf.H * accm * ij;
    }
#pragma unroll
    for (int c = 0; c < 5; c++) {
      if (mode == kModeResidual) {
        v.R[o + c * nn] = R[c];
      } else {
        const double du = (rkA == 0.0 ? 0.0 : rkA * v.dU[o + c * nn]) + (v.dtp ? *v.dtp : dt) * R[c];
        v.dU[o + c * nn] = du;
        state(v, cur ^ 1)[o + c * nn] = Uin[o + c * nn] + rkB * du;
      }
    }
  };
#pragma unroll
  for (int s = 0; s < NPL; s++)
    if (t + s * BS < I.nn) node_update(t + s * BS, acc[s], accm[s]);
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
    double pw;
    s[9] = wave_speed(u, g, pw);
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

template <int NNMAX, int NPL>
static hipError_t stage_bucket(const View& v, int b, int cur, double dt, double rkA, double rkB, int mode,
                               hipStream_t st) {
  const dim3 grid(v.mix_cnt[b]), block(mix_lanes(NNMAX, NPL));
  if (v.fp32)
    hipLaunchKernelGGL((mixed_stage_kernel<NNMAX, NPL, float, false>), grid, block, 0, st, v, v.mix_beg[b], cur,
                       dt, rkA, rkB, mode);
  else if (flux_family(v.vol, v.surf) & 1)
    hipLaunchKernelGGL((mixed_stage_kernel<NNMAX, NPL, double, true>), grid, block, 0, st, v, v.mix_beg[b], cur,
                       dt, rkA, rkB, mode);
  else
    hipLaunchKernelGGL((mixed_stage_kernel<NNMAX, NPL, double, false>), grid, block, 0, st, v, v.mix_beg[b], cur,
                       dt, rkA, rkB, mode);
  return hipGetLastError();
}

template <int NNMAX>
static hipError_t stage_bucket_npl(const View& v, int b, int npl, int cur, double dt, double rkA, double rkB,
                                   int mode, hipStream_t st) {
  return npl == 2 ? stage_bucket<NNMAX, 2>(v, b, cur, dt, rkA, rkB, mode, st)
                  : stage_bucket<NNMAX, 1>(v, b, cur, dt, rkA, rkB, mode, st);
}

hipError_t launch_faces_mixed(const View& v, int cur, hipStream_t st) {
  if (v.fp32)
    hipLaunchKernelGGL((mixed_face_kernel<float, false>), dim3(3 * v.E), dim3(64), 0, st, v, cur);
  else if (v.surf >= 4)
    hipLaunchKernelGGL((mixed_face_kernel<double, true>), dim3(3 * v.E), dim3(64), 0, st, v, cur);
  else
    hipLaunchKernelGGL((mixed_face_kernel<double, false>), dim3(3 * v.E), dim3(64), 0, st, v, cur);
  return hipGetLastError();
}

hipError_t launch_stage_mixed_bucket(const View& v, int b, int npl, int cur, double dt, double rkA, double rkB,
                                     int mode, hipStream_t st) {
  if (v.mix_cnt[b] <= 0) return hipSuccess;
  switch (b) {
    case 0: return stage_bucket_npl<64>(v, b, npl, cur, dt, rkA, rkB, mode, st);
    case 1: return stage_bucket_npl<128>(v, b, npl, cur, dt, rkA, rkB, mode, st);
    case 2: return stage_bucket_npl<192>(v, b, npl, cur, dt, rkA, rkB, mode, st);
    case 3: return stage_bucket_npl<256>(v, b, npl, cur, dt, rkA, rkB, mode, st);
    case 4: return stage_bucket_npl<320>(v, b, npl, cur, dt, rkA, rkB, mode, st);
    case 5: return stage_bucket_npl<384>(v, b, npl, cur, dt, rkA, rkB, mode, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stage_mixed(const View& v, int cur, double dt, double rkA, double rkB, int mode, int tiles,
                              hipStream_t st, const MixStreams* ms) {
  hipError_t e = launch_faces_mixed(v, cur, st);
  if (e != hipSuccess) return e;
  int bk[kMixBuckets], nb = 0;
  for (int b = kMixBuckets - 1; b >= 0; b--)  // the work list starts with the largest elements
    if (v.mix_cnt[b] > 0) bk[nb++] = b;
  // the largest elements on st, up to kMixSide further buckets each on a side stream, the rest
  // after the largest on st
  const int ns = ms ? (nb - 1 < kMixSide ? nb - 1 : kMixSide) : 0;
  if (ns > 0) {
    e = hipEventRecord(ms->fork, st);
    if (e != hipSuccess) return e;
  }
  for (int i = 0; i < ns && e == hipSuccess; i++) {
    const int b = bk[1 + i];
    e = hipStreamWaitEvent(ms->side[i], ms->fork, 0);
    if (e == hipSuccess)
      e = launch_stage_mixed_bucket(v, b, (tiles >> b) & 1 ? 2 : 1, cur, dt, rkA, rkB, mode, ms->side[i]);
    if (e == hipSuccess) e = hipEventRecord(ms->join[i], ms->side[i]);
  }
  for (int i = 0; i < nb && e == hipSuccess; i++) {
    if (i >= 1 && i <= ns) continue;
    const int b = bk[i];
    e = launch_stage_mixed_bucket(v, b, (tiles >> b) & 1 ? 2 : 1, cur, dt, rkA, rkB, mode, st);
  }
  // the join, also after a failed launch: no side stream is left forked from st
  for (int i = 0; i < ns; i++) {
    const hipError_t ej = hipStreamWaitEvent(st, ms->join[i], 0);
    if (e == hipSuccess) e = ej;
  }
  return e;
}

hipError_t launch_diagnostics_mixed(const View& v, int cur, hipStream_t st) {
  hipLaunchKernelGGL(diag_mixed_kernel, dim3(v.E), dim3(512), 0, st, v, cur);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return launch_diag_final(v, st);
}

}  // namespace dg
