// dg_device.h -- device-side building blocks shared by the uniform-order kernels
// (kernels.hip) and the mixed-order kernels (kernels_mixed.hip): launch shape helpers, fast
// reciprocals, primitive variables, the two-point and face numerical fluxes (FP64 and the
// FP32-bulk deviation form), and the BR1 gradient / viscous flux of one node.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "dg_internal.h"

namespace dg {

__host__ __device__ constexpr int nthreads_for(int N) {
  return (((N + 1) * (N + 1) * (N + 1) + 63) / 64) * 64;
}

__host__ __device__ constexpr int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Workgroup -> element.  Consecutive workgroups go round-robin over the 8 XCDs; give each XCD
// a contiguous slice of elements instead.
__device__ __forceinline__ int block_element(int E) {
  const int b = blockIdx.x;
  if ((E & 7) == 0) {
    const int per = E >> 3;
    return (b & 7) * per + (b >> 3);
  }
  return b;
}

// Workgroup -> (member, element) of a batched launch, XCD-aware over the whole grid.
__device__ __forceinline__ void batch_member(const BatchArgs& B, int& m, int& e) {
  const int b = block_element(B.start[B.n]);
  m = 0;
  while (m + 1 < B.n && b >= B.start[m + 1]) m++;
  e = b - B.start[m];
}

// node index of reference indices (i_d = id, tangential p, r) on a face normal to d
template <int n>
__device__ __forceinline__ int face_node(int d, int id, int p, int r) {
  return d == 0 ? id + n * (p + n * r) : (d == 1 ? p + n * (id + n * r) : p + n * (r + n * id));
}

// Reciprocal of a positive, finite, normal operand: hardware estimate refined by two Newton
// steps (error within an ulp or two).  The IEEE division sequence also rescales operands near
// the exponent limits, which the physical quantities here never approach.
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// 1/sqrt(x) of a positive, finite, normal operand: hardware estimate refined by two Newton steps
__device__ __forceinline__ double rsq(double x) {
  double r = __builtin_amdgcn_rsq(x);
  double e = fma(-x * r, r, 1.0);
  r = fma(0.5 * r, e, r);
  e = fma(-x * r, r, 1.0);
  return fma(0.5 * r, e, r);
}
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// ------------------------------------------------------------------ physics helpers
// largest characteristic speed |v| + c of a node and its pressure (the diagnostics and the
// adaptive step size share this, so both see the same lambda_max)
__device__ __forceinline__ double wave_speed(const double u[5], double g, double& p) {
  const double v1 = u[1] / u[0], v2 = u[2] / u[0], v3 = u[3] / u[0];
  const double q2 = v1 * v1 + v2 * v2 + v3 * v3;
  p = (g - 1) * (u[4] - 0.5 * u[0] * q2);
  return sqrt(q2) + sqrt(g * p / u[0]);
}

template <typename T>
struct Prim {
  T rho, v1, v2, v3, beta, lrho, lbeta, h;  // beta = rho/(2p), h = |v|^2/2
};

// primitive variables computed in FP64 from the conservative state, then rounded to T
template <typename T>
__device__ __forceinline__ Prim<T> make_prim(const double u[5], double gamma) {
  const double inv = rcp(u[0]);
  const double v1 = u[1] * inv, v2 = u[2] * inv, v3 = u[3] * inv;
  const double h = 0.5 * (v1 * v1 + v2 * v2 + v3 * v3);
  const double p = (gamma - 1.0) * (u[4] - u[0] * h);
  const double beta = 0.5 * u[0] * rcp(p);
  Prim<T> o;
  o.rho = (T)u[0];
  o.v1 = (T)v1;
  o.v2 = (T)v2;
  o.v3 = (T)v3;
  o.beta = (T)beta;
  o.lrho = (T)log(u[0]);
  o.lbeta = (T)log(beta);
  o.h = (T)h;
  return o;
}

// Chandrashekar's entropy-conserving, kinetic-energy-preserving two-point flux along the
// (not normalised) vector n: F#(a, b; n), linear in n and symmetric in (a, b).  ce =
// 1/(2(gamma-1)).  Logarithmic means (x_a - x_b)/(ln x_a - ln x_b) of rho and beta: near
// x_a = x_b the cancelling logarithms are replaced by the series in
// u = ((x_a - x_b)/(x_a + x_b))^2, (x_a + x_b)/(2(1 + u/3 + u^2/5 + u^3/7)).  The five
// quotients of the flux share two reciprocals.
template <typename T>
__device__ __forceinline__ void flux_ec(const Prim<T>& a, const Prim<T>& b, T n1, T n2, T n3, T ce,
                                        T F[5]) {
  const T thr = sizeof(T) == 8 ? (T)1e-4 : (T)1e-2;
  const T dr = a.rho - b.rho, sr = a.rho + b.rho;
  const T db = a.beta - b.beta, sb = a.beta + b.beta;
  const T r1 = rcp(sr * sb);
  const T isb = r1 * sr;                    // 1/(beta_a + beta_b)
  const T fr = dr * (r1 * sb), fb = db * isb;
  const T ur = fr * fr, ub = fb * fb;
  const bool smr = ur < thr, smb = ub < thr;
  const T numr = smr ? sr : dr;
  const T denr = smr ? (T)2 * ((T)1 + ur * ((T)(1.0 / 3.0) + ur * ((T)0.2 + ur * (T)(1.0 / 7.0))))
                     : (a.lrho - b.lrho);
  const T numb = smb ? sb : db;
  const T denb = smb ? (T)2 * ((T)1 + ub * ((T)(1.0 / 3.0) + ub * ((T)0.2 + ub * (T)(1.0 / 7.0))))
                     : (a.lbeta - b.lbeta);
  const T r2 = rcp(denr * numb);
  const T rho_ln = numr * numb * r2;        // logmean(rho)
  const T inv_bln = denb * denr * r2;       // 1 / logmean(beta)
  const T phat = (T)0.5 * sr * isb;         // {rho} / (2 {beta})
  const T u = (T)0.5 * (a.v1 + b.v1), v = (T)0.5 * (a.v2 + b.v2), w = (T)0.5 * (a.v3 + b.v3);
  const T hb = (T)0.5 * (a.h + b.h);
  const T vn = u * n1 + v * n2 + w * n3;
  F[0] = rho_ln * vn;
  F[1] = F[0] * u + phat * n1;
  F[2] = F[0] * v + phat * n2;
  F[3] = F[0] * w + phat * n3;
  F[4] = F[0] * (ce * inv_bln - hb) + u * F[1] + v * F[2] + w * F[3];
}

// central two-point flux (F(a) + F(b)) / 2 . n from the primitive variables
template <typename T>
__device__ __forceinline__ void flux_central(const Prim<T>& a, const Prim<T>& b, T n1, T n2, T n3,
                                             T gm1, T F[5]) {
  T Fa[5], Fb[5];
  const Prim<T>* s[2] = {&a, &b};
  T* o[2] = {Fa, Fb};
#pragma unroll
  for (int q = 0; q < 2; q++) {
    const Prim<T>& P = *s[q];
    const T p = (T)0.5 * P.rho / P.beta;
    const T vn = P.v1 * n1 + P.v2 * n2 + P.v3 * n3;
    const T En = p / gm1 + P.rho * P.h;
    o[q][0] = P.rho * vn;
    o[q][1] = P.rho * P.v1 * vn + p * n1;
    o[q][2] = P.rho * P.v2 * vn + p * n2;
    o[q][3] = P.rho * P.v3 * vn + p * n3;
    o[q][4] = (En + p) * vn;
  }
#pragma unroll
  for (int c = 0; c < 5; c++) F[c] = (T)0.5 * (Fa[c] + Fb[c]);
}

// logarithmic mean of x_a, x_b from their logarithms la, lb (series near x_a = x_b, as above)
template <typename T>
__device__ __forceinline__ T logmean_logs(T xa, T xb, T la, T lb) {
  const T s = xa + xb, d = xa - xb;
  const T f = d * rcp(s), u = f * f;
  const T thr = sizeof(T) == 8 ? (T)1e-4 : (T)1e-2;
  if (u < thr) return s * rcp((T)2 * ((T)1 + u * ((T)(1.0 / 3.0) + u * ((T)0.2 + u * (T)(1.0 / 7.0)))));
  return d * rcp(la - lb);
}

// Ismail and Roe's entropy-conserving two-point flux along n, from the parameter vector
// z = sqrt(rho/p) (1, v, p): z1 = sqrt(2 beta), z5 = rho / z1, so ln z1 = (ln 2 + ln beta)/2 and
// ln z5 = ln rho - ln z1 come from the stored logarithms.
//   rho^ = {z1} (z5)^ln, v^ = {z1 v}/{z1}, p1^ = {z5}/{z1},
//   p2^ = (gamma+1)/(2 gamma) (z5)^ln/(z1)^ln + (gamma-1)/(2 gamma) p1^,
//   H^ = gamma p2^/((gamma-1) rho^) + |v^|^2/2,  F = (rho^ v^.n, rho^ v^ v^.n + p1^ n, rho^ H^ v^.n)
template <typename T>
__device__ __forceinline__ void flux_ir(const Prim<T>& a, const Prim<T>& b, T n1, T n2, T n3, T gm1, T F[5]) {
  const T g = gm1 + (T)1;
  const T z1a = sqrt((T)2 * a.beta), z1b = sqrt((T)2 * b.beta);
  const T iz1a = rcp(z1a), iz1b = rcp(z1b);
  const T z5a = a.rho * iz1a, z5b = b.rho * iz1b;
  const T hl2 = (T)0.34657359027997264;  // ln(2) / 2
  const T l1a = hl2 + (T)0.5 * a.lbeta, l1b = hl2 + (T)0.5 * b.lbeta;
  const T z1ln = logmean_logs(z1a, z1b, l1a, l1b);
  const T z5ln = logmean_logs(z5a, z5b, a.lrho - l1a, b.lrho - l1b);
  const T is1 = rcp(z1a + z1b);
  const T rho = (T)0.5 * (z1a + z1b) * z5ln;
  const T u = (z1a * a.v1 + z1b * b.v1) * is1, v = (z1a * a.v2 + z1b * b.v2) * is1,
          w = (z1a * a.v3 + z1b * b.v3) * is1;
  const T p1 = (z5a + z5b) * is1;
  const T p2 = (g + (T)1) / ((T)2 * g) * z5ln * rcp(z1ln) + gm1 / ((T)2 * g) * p1;
  const T H = g * p2 * rcp(gm1 * rho) + (T)0.5 * (u * u + v * v + w * w);
  const T vn = u * n1 + v * n2 + w * n3;
  F[0] = rho * vn;
  F[1] = F[0] * u + p1 * n1;
  F[2] = F[0] * v + p1 * n2;
  F[3] = F[0] * w + p1 * n3;
  F[4] = F[0] * H;
}

// Kinetic-energy-preserving split forms as two-point fluxes along n, from products of
// arithmetic means {.}: vn = v.n, e = p/((gamma-1) rho) + |v|^2/2 = ce/beta + h, H = e + 1/(2 beta).
//   3 Kennedy-Gruber  {rho}{vn},  {rho}{vn}{v} + {p}n,  {rho}{vn}{e} + {p}{vn}
//   4 Pirozzoli       {rho}{vn},  {rho}{vn}{v} + {p}n,  {rho}{vn}{H}
//   5 Ducros          {rho}{vn},  {rho v}{vn} + {p}n,   {rho H}{vn}
//   6 Morinishi       m = {rho vn},  m{v} + {p}n,  gamma/(gamma-1){p vn} + m |{v}|^2 - {rho vn h}
template <typename T>
__device__ __forceinline__ void flux_kep(int kind, const Prim<T>& a, const Prim<T>& b, T n1, T n2,
                                         T n3, T ce, T F[5]) {
  const T iba = rcp(a.beta), ibb = rcp(b.beta);
  const T pa = (T)0.5 * a.rho * iba, pb = (T)0.5 * b.rho * ibb;
  const T vna = a.v1 * n1 + a.v2 * n2 + a.v3 * n3, vnb = b.v1 * n1 + b.v2 * n2 + b.v3 * n3;
  const T u = (T)0.5 * (a.v1 + b.v1), v = (T)0.5 * (a.v2 + b.v2), w = (T)0.5 * (a.v3 + b.v3);
  const T pm = (T)0.5 * (pa + pb), vn = (T)0.5 * (vna + vnb), rm = (T)0.5 * (a.rho + b.rho);
  const T ea = ce * iba + a.h, eb = ce * ibb + b.h;
  if (kind == 6) {
    const T m = (T)0.5 * (a.rho * vna + b.rho * vnb);
    F[0] = m;
    F[1] = m * u + pm * n1;
    F[2] = m * v + pm * n2;
    F[3] = m * w + pm * n3;
    F[4] = ((T)1 + (T)2 * ce) * (T)0.5 * (pa * vna + pb * vnb) + m * (u * u + v * v + w * w) -
           (T)0.5 * (a.rho * vna * a.h + b.rho * vnb * b.h);
    return;
  }
  F[0] = rm * vn;
  if (kind == 5) {
    F[1] = (T)0.5 * (a.rho * a.v1 + b.rho * b.v1) * vn + pm * n1;
    F[2] = (T)0.5 * (a.rho * a.v2 + b.rho * b.v2) * vn + pm * n2;
    F[3] = (T)0.5 * (a.rho * a.v3 + b.rho * b.v3) * vn + pm * n3;
    F[4] = (T)0.5 * (a.rho * (ea + (T)0.5 * iba) + b.rho * (eb + (T)0.5 * ibb)) * vn;
    return;
  }
  F[1] = F[0] * u + pm * n1;
  F[2] = F[0] * v + pm * n2;
  F[3] = F[0] * w + pm * n3;
  if (kind == 3) F[4] = F[0] * (T)0.5 * (ea + eb) + pm * vn;
  else F[4] = F[0] * (T)0.5 * (ea + eb + (T)0.5 * (iba + ibb));
}

// volume two-point flux: 0 Chandrashekar, 1 central, 2 Ismail-Roe; with KEP the
// kinetic-energy-preserving forms 3..6 above instead
template <typename T, bool KEP = false>
__device__ __forceinline__ void vol_flux(int kind, const Prim<T>& a, const Prim<T>& b, T n1, T n2,
                                         T n3, T ce, T gm1, T F[5]) {
  if constexpr (KEP) flux_kep(kind, a, b, n1, n2, n3, ce, F);
  else if (kind == 0) flux_ec(a, b, n1, n2, n3, ce, F);
  else if (kind == 2) flux_ir(a, b, n1, n2, n3, gm1, F);
  else flux_central(a, b, n1, n2, n3, gm1, F);
}

// Numerical flux through a face with scaled normal S (|S| times the unit normal), between
// the conservative states uL (the side S points away from) and uR: Roe (0), local
// Lax-Friedrichs (1), Chandrashekar's EC flux (2), central (3).  LD turns Roe's flux into its
// low-dissipation variant: the velocity jump in the wave strengths is scaled by
// z = min(1, max(M_L, M_R)), the larger local Mach number.
template <typename T, bool LD = false>
__device__ __forceinline__ void face_flux_std(int kind, const double uL[5], const double uR[5],
                                          const double S[3], double gamma, T F[5]) {
  const T gm1 = (T)(gamma - 1.0);
  if (kind == 2) {  // entropy-conserving flux, linear in S
    const Prim<T> a = make_prim<T>(uL, gamma), b = make_prim<T>(uR, gamma);
    flux_ec(a, b, (T)S[0], (T)S[1], (T)S[2], (T)(0.5 / (gamma - 1.0)), F);
    return;
  }
  const T s1 = (T)S[0], s2 = (T)S[1], s3 = (T)S[2];
  const T a2s = s1 * s1 + s2 * s2 + s3 * s3;
  const T ia = rsq(a2s);
  const T area = a2s * ia;
  const T n1 = s1 * ia, n2 = s2 * ia, n3 = s3 * ia;
  T rL, vL[3], pL, EL, rR, vR[3], pR, ER, irL, irR;
  {
    const double i = rcp(uL[0]);
    const double a1 = uL[1] * i, a2 = uL[2] * i, a3 = uL[3] * i;
    const double p = (gamma - 1.0) * (uL[4] - 0.5 * uL[0] * (a1 * a1 + a2 * a2 + a3 * a3));
    rL = (T)uL[0]; vL[0] = (T)a1; vL[1] = (T)a2; vL[2] = (T)a3; pL = (T)p; EL = (T)uL[4];
    irL = (T)i;
  }
  {
    const double i = rcp(uR[0]);
    const double a1 = uR[1] * i, a2 = uR[2] * i, a3 = uR[3] * i;
    const double p = (gamma - 1.0) * (uR[4] - 0.5 * uR[0] * (a1 * a1 + a2 * a2 + a3 * a3));
    rR = (T)uR[0]; vR[0] = (T)a1; vR[1] = (T)a2; vR[2] = (T)a3; pR = (T)p; ER = (T)uR[4];
    irR = (T)i;
  }
  const T vnL = vL[0] * n1 + vL[1] * n2 + vL[2] * n3;
  const T vnR = vR[0] * n1 + vR[1] * n2 + vR[2] * n3;
  const T HL = (EL + pL) * irL, HR = (ER + pR) * irR;
  T Fs[5];  // F(uL).n + F(uR).n
  Fs[0] = rL * vnL + rR * vnR;
  Fs[1] = rL * vnL * vL[0] + rR * vnR * vR[0] + (pL + pR) * n1;
  Fs[2] = rL * vnL * vL[1] + rR * vnR * vR[1] + (pL + pR) * n2;
  Fs[3] = rL * vnL * vL[2] + rR * vnR * vR[2] + (pL + pR) * n3;
  Fs[4] = rL * HL * vnL + rR * HR * vnR;
  if (kind == 3) {  // central
#pragma unroll
    for (int c = 0; c < 5; c++) F[c] = (T)0.5 * area * Fs[c];
    return;
  }
  if (kind == 1) {  // local Lax-Friedrichs (Rusanov)
    const T g = (T)gamma;
    const T cL2 = g * pL * irL, cR2 = g * pR * irR;
    const T lamL = fabs(vnL) + cL2 * rsq(cL2);
    const T lamR = fabs(vnR) + cR2 * rsq(cR2);
    const T lam = lamL > lamR ? lamL : lamR;
    const T du[5] = {(T)(uR[0] - uL[0]), (T)(uR[1] - uL[1]), (T)(uR[2] - uL[2]), (T)(uR[3] - uL[3]),
                     (T)(uR[4] - uL[4])};
#pragma unroll
    for (int c = 0; c < 5; c++) F[c] = (T)0.5 * area * (Fs[c] - lam * du[c]);
    return;
  }
  // Roe: averages weighted by sqrt(rho), in the form (qL + Q qR)/(1 + Q), Q = sqrt(rhoR/rhoL);
  // waves u_n - c, u_n (entropy and shear), u_n + c
  const T x = rR * irL;
  const T Q = x * rsq(x);
  const T iw = rcp((T)1 + Q);
  const T u1 = (vL[0] + Q * vR[0]) * iw;
  const T u2 = (vL[1] + Q * vR[1]) * iw;
  const T u3 = (vL[2] + Q * vR[2]) * iw;
  const T H = (HL + Q * HR) * iw;
  const T rho = rL * Q;
  const T q2 = u1 * u1 + u2 * u2 + u3 * u3;
  const T c2 = gm1 * (H - (T)0.5 * q2);
  const T rc = rsq(c2);
  const T c = c2 * rc;
  const T ic2 = rc * rc;
  const T vn = u1 * n1 + u2 * n2 + u3 * n3;
  const T dr = rR - rL, dp = pR - pL;
  T dv1 = vR[0] - vL[0], dv2 = vR[1] - vL[1], dv3 = vR[2] - vL[2];
  if constexpr (LD) {
    const T g = (T)gamma;
    const T mL = (vL[0] * vL[0] + vL[1] * vL[1] + vL[2] * vL[2]) * rL / (g * pL);
    const T mR = (vR[0] * vR[0] + vR[1] * vR[1] + vR[2] * vR[2]) * rR / (g * pR);
    const T m2 = mL > mR ? mL : mR;
    const T z = m2 < (T)1 ? sqrt(m2) : (T)1;
    dv1 *= z;
    dv2 *= z;
    dv3 *= z;
  }
  const T dvn = dv1 * n1 + dv2 * n2 + dv3 * n3;
  const T a1 = (T)0.5 * (dp - rho * c * dvn) * ic2;
  const T a2 = dr - dp * ic2;
  const T a3 = (T)0.5 * (dp + rho * c * dvn) * ic2;
  const T l1 = fabs(vn - c), l2 = fabs(vn), l3 = fabs(vn + c);
  const T t1 = dv1 - dvn * n1, t2 = dv2 - dvn * n2, t3 = dv3 - dvn * n3;
  const T udt = u1 * t1 + u2 * t2 + u3 * t3;
  const T w1 = l1 * a1, w3 = l3 * a3;
  T W[5];
  W[0] = w1 + l2 * a2 + w3;
  W[1] = w1 * (u1 - c * n1) + l2 * (a2 * u1 + rho * t1) + w3 * (u1 + c * n1);
  W[2] = w1 * (u2 - c * n2) + l2 * (a2 * u2 + rho * t2) + w3 * (u2 + c * n2);
  W[3] = w1 * (u3 - c * n3) + l2 * (a2 * u3 + rho * t3) + w3 * (u3 + c * n3);
  W[4] = w1 * (H - vn * c) + l2 * (a2 * (T)0.5 * q2 + rho * udt) + w3 * (H + vn * c);
#pragma unroll
  for (int k = 0; k < 5; k++) F[k] = (T)0.5 * area * (Fs[k] - W[k]);
}

// Matrix dissipation R |Lambda| T R^T (w_b - w_a) along the unit normal n: eigenvectors R of the
// flux Jacobian, Barth's scaling T = diag(rho/(2 gamma), rho (gamma-1)/gamma, p, p, rho/(2 gamma))
// (so that R T R^T = du/dw), all at the averaged state rho^ = (rho)^ln, v^ = {v},
// p^ = {rho}/(2{beta}), c^2 = gamma p^/rho^, H^ = c^2/(gamma-1) + |v^|^2/2.  The jump of the
// entropy variables w = ((gamma - s)/(gamma-1) - 2 beta h, 2 beta v, -2 beta) comes from the
// stored logarithms: s = -(gamma-1) ln rho - ln 2 - ln beta.  The two shear waves are summed
// with the tangential projector I - n n^T.
template <typename T>
__device__ __forceinline__ void matrix_dissipation(const Prim<T>& a, const Prim<T>& b, T n1, T n2, T n3,
                                                   T gm1, T D[5]) {
  const T g = gm1 + (T)1;
  const T rho = logmean_logs(a.rho, b.rho, a.lrho, b.lrho);
  const T p = (a.rho + b.rho) * rcp((T)2 * (a.beta + b.beta));
  const T u = (T)0.5 * (a.v1 + b.v1), v = (T)0.5 * (a.v2 + b.v2), w = (T)0.5 * (a.v3 + b.v3);
  const T q2 = u * u + v * v + w * w;
  const T igm1 = rcp(gm1);
  const T c2 = g * p * rcp(rho);
  const T c = c2 * rsq(c2);
  const T H = c2 * igm1 + (T)0.5 * q2;
  const T vn = u * n1 + v * n2 + w * n3;
  const T dw0 = (b.lrho - a.lrho) + (b.lbeta - a.lbeta) * igm1 - (T)2 * (b.beta * b.h - a.beta * a.h);
  const T dw1 = (T)2 * (b.beta * b.v1 - a.beta * a.v1);
  const T dw2 = (T)2 * (b.beta * b.v2 - a.beta * a.v2);
  const T dw3 = (T)2 * (b.beta * b.v3 - a.beta * a.v3);
  const T dw4 = (T)-2 * (b.beta - a.beta);
  const T base = dw0 + u * dw1 + v * dw2 + w * dw3;  // r . dw without the c and energy parts
  const T cn = c * (n1 * dw1 + n2 * dw2 + n3 * dw3);
  const T s1 = (base - cn + (H - c * vn) * dw4) * fabs(vn - c) * rho * rcp((T)2 * g);
  const T s2 = (base + (T)0.5 * q2 * dw4) * fabs(vn) * rho * gm1 * rcp(g);
  const T s5 = (base + cn + (H + c * vn) * dw4) * fabs(vn + c) * rho * rcp((T)2 * g);
  const T q1 = dw1 + u * dw4, qq2 = dw2 + v * dw4, q3 = dw3 + w * dw4;
  const T qn = q1 * n1 + qq2 * n2 + q3 * n3;
  const T t1 = q1 - qn * n1, t2 = qq2 - qn * n2, t3 = q3 - qn * n3;
  const T sh = p * fabs(vn);
  const T s15 = s1 + s5;
  D[0] = s15 + s2;
  D[1] = s15 * u + c * n1 * (s5 - s1) + s2 * u + sh * t1;
  D[2] = s15 * v + c * n2 * (s5 - s1) + s2 * v + sh * t2;
  D[3] = s15 * w + c * n3 * (s5 - s1) + s2 * w + sh * t3;
  D[4] = s15 * H + c * vn * (s5 - s1) + s2 * (T)0.5 * q2 + sh * (u * t1 + v * t2 + w * t3);
}

// The extended surface fluxes: entropy stable (4: Chandrashekar's flux minus local
// Lax-Friedrichs dissipation), Ismail-Roe (5), entropy stable with matrix dissipation (6:
// Chandrashekar's flux minus the dissipation above), low-dissipation Roe (7), Lax-Friedrichs with
// the global wave speed lam_g (8: the central flux minus lam_g |S| (U_R - U_L) / 2).
template <typename T>
__device__ __forceinline__ void face_flux_xs(int kind, const double uL[5], const double uR[5],
                                             const double S[3], double gamma, T F[5], double lam_g) {
  if (kind == 8) {
    face_flux_std<T>(3, uL, uR, S, gamma, F);
    const T s1 = (T)S[0], s2 = (T)S[1], s3 = (T)S[2];
    const T a2s = s1 * s1 + s2 * s2 + s3 * s3;
    const T area = a2s * rsq(a2s);
#pragma unroll
    for (int c = 0; c < 5; c++) F[c] -= (T)0.5 * area * (T)lam_g * (T)(uR[c] - uL[c]);
    return;
  }
  if (kind == 7) {
    face_flux_std<T, true>(0, uL, uR, S, gamma, F);
    return;
  }
  const T gm1 = (T)(gamma - 1.0);
  const Prim<T> a = make_prim<T>(uL, gamma), b = make_prim<T>(uR, gamma);
  if (kind == 5) {
    flux_ir(a, b, (T)S[0], (T)S[1], (T)S[2], gm1, F);
    return;
  }
  const T s1 = (T)S[0], s2 = (T)S[1], s3 = (T)S[2];
  const T a2s = s1 * s1 + s2 * s2 + s3 * s3;
  const T ia = rsq(a2s);
  const T area = a2s * ia;
  flux_ec(a, b, s1, s2, s3, (T)(0.5 / (gamma - 1.0)), F);
  if (kind == 6) {
    T D[5];
    matrix_dissipation(a, b, s1 * ia, s2 * ia, s3 * ia, gm1, D);
#pragma unroll
    for (int c = 0; c < 5; c++) F[c] -= (T)0.5 * area * D[c];
    return;
  }
  const T g = (T)gamma;
  T lam = (T)0;
  const double* u2[2] = {uL, uR};
#pragma unroll
  for (int q = 0; q < 2; q++) {
    const double* u = u2[q];
    const double i = rcp(u[0]);
    const double a1 = u[1] * i, a2 = u[2] * i, a3 = u[3] * i;
    const T p = (T)((gamma - 1.0) * (u[4] - 0.5 * u[0] * (a1 * a1 + a2 * a2 + a3 * a3)));
    const T vn = ((T)a1 * s1 + (T)a2 * s2 + (T)a3 * s3) * ia;
    const T c2 = g * p * (T)i;
    const T l = fabs(vn) + c2 * rsq(c2);
    lam = l > lam ? l : lam;
  }
#pragma unroll
  for (int c = 0; c < 5; c++) F[c] -= (T)0.5 * area * lam * (T)(uR[c] - uL[c]);
}

// XS selects the family: the two are compiled apart so that the common one keeps its registers
template <typename T, bool XS = false>
__device__ __forceinline__ void face_flux(int kind, const double uL[5], const double uR[5],
                                          const double S[3], double gamma, T F[5], double lam_g = 0.0) {
  if constexpr (XS) face_flux_xs<T>(kind, uL, uR, S, gamma, F, lam_g);
  else face_flux_std<T>(kind, uL, uR, S, gamma, F);
}

// ------------------------------------------------------------------ FP32-bulk: deviation form
// With FP32 arithmetic the fluxes are formed as deviations from a constant reference state
// (rho_r, p_r), because at low Mach number p and rho e are large constants plus small
// variations.  Both changes below are exact in exact arithmetic:
//  - the momentum flux loses its constant part p_r n: a constant flux proportional to the metric
//    terms has zero residual (discrete metric identities, SBP lift);
//  - the energy flux is split as H_r F_rho + F'_E with H_r = gamma p_r/((gamma-1) rho_r); the
//    residual is linear in the fluxes, so R_E = H_r R_rho + R'_E, recombined in FP64.
// Per-node inputs are formed in FP64 and rounded: x = rho/rho_r - 1, y = beta/beta_r - 1,
// lx = ln(rho/rho_r), ly = ln(beta/beta_r) (beta = rho/(2p)), so that every quantity entering
// the FP32 arithmetic is either O(1) or a small deviation carried at full relative precision.
struct Ref {
  double rho, p;  // reference density and pressure
  double c;       // p/((gamma-1) rho)  = 1/(2 (gamma-1) beta_r)
  double por;     // p/rho
  double H;       // c + por, reference total enthalpy at rest
};

__device__ __forceinline__ Ref make_ref(double rho_r, double p_r, double gamma) {
  Ref r;
  r.rho = rho_r;
  r.p = p_r;
  r.por = p_r / rho_r;
  r.c = r.por / (gamma - 1.0);
  r.H = r.c + r.por;
  return r;
}

// primitive deviations stored in the Prim fields: rho <- x, beta <- y, lrho <- lx, lbeta <- ly
template <typename T>
__device__ __forceinline__ Prim<T> make_prim_dev(const double u[5], double gamma, const Ref& R) {
  const double inv = rcp(u[0]);
  const double v1 = u[1] * inv, v2 = u[2] * inv, v3 = u[3] * inv;
  const double h = 0.5 * (v1 * v1 + v2 * v2 + v3 * v3);
  const double p = (gamma - 1.0) * (u[4] - u[0] * h);
  const double rr = u[0] / R.rho;          // rho / rho_r
  const double bb = rr * R.p * rcp(p);     // beta / beta_r = (rho / rho_r)(p_r / p)
  Prim<T> o;
  o.rho = (T)(rr - 1.0);
  o.beta = (T)(bb - 1.0);
  o.lrho = (T)log(rr);
  o.lbeta = (T)log(bb);
  o.v1 = (T)v1;
  o.v2 = (T)v2;
  o.v3 = (T)v3;
  o.h = (T)h;
  return o;
}

// logarithmic mean of (1 + xa, 1 + xb) as 1 + lam, lam formed without cancellation
// (la, lb = ln(1 + xa), ln(1 + xb))
template <typename T>
__device__ __forceinline__ T logmean_dev(T xa, T xb, T la, T lb) {
  const T d = xa - xb, w = (T)2 + xa + xb;
  const T u = d * d * rcp(w * w);
  const T thr = sizeof(T) == 8 ? (T)1e-4 : (T)1e-2;
  if (u < thr) {
    const T pm1 = u * ((T)(1.0 / 3.0) + u * ((T)0.2 + u * (T)(1.0 / 7.0)));
    return ((T)0.5 * (xa + xb) - pm1) * rcp((T)1 + pm1);
  }
  const T dl = la - lb;
  return (d - dl) * rcp(dl);
}

// Chandrashekar's flux in deviation form: F[0] = F_rho, F[1..3] = F_m - p_r n,
// F[4] = F_E - H_r F_rho
// vn64 = {v}.n formed in FP64 (the mass flux is carried in FP64, see the stage kernel)
template <typename T>
__device__ __forceinline__ void flux_ec_dev(const Prim<T>& a, const Prim<T>& b, T n1, T n2, T n3,
                                            double vn64, const Ref& R, T F[5], double& F0d) {
  const T lr = logmean_dev(a.rho, b.rho, a.lrho, b.lrho);   // rho_ln = rho_r (1 + lr)
  const T lb = logmean_dev(a.beta, b.beta, a.lbeta, b.lbeta);  // beta_ln = beta_r (1 + lb)
  const T xb = (T)0.5 * (a.rho + b.rho), yb = (T)0.5 * (a.beta + b.beta);
  const T dphat = (T)R.p * (xb - yb) * rcp((T)1 + yb);       // {rho}/(2{beta}) - p_r
  const T u = (T)0.5 * (a.v1 + b.v1), v = (T)0.5 * (a.v2 + b.v2), w = (T)0.5 * (a.v3 + b.v3);
  const T hb = (T)0.5 * (a.h + b.h);
  const T vn = u * n1 + v * n2 + w * n3;
  F0d = R.rho * (1.0 + (double)lr) * vn64;
  F[0] = (T)F0d;
  F[1] = F[0] * u + dphat * n1;
  F[2] = F[0] * v + dphat * n2;
  F[3] = F[0] * w + dphat * n3;
  const T kin = u * u + v * v + w * w - hb;
  F[4] = F[0] * (kin - (T)R.c * lb * rcp((T)1 + lb) - (T)R.por * lr * rcp((T)1 + lr)) + dphat * vn;
}

// central two-point flux in deviation form
template <typename T>
__device__ __forceinline__ void flux_central_dev(const Prim<T>& a, const Prim<T>& b, T n1, T n2, T n3,
                                                 const double va[3], const double vb[3], const double m[3],
                                                 const Ref& R, T F[5], double& F0d) {
  T Fa[5], Fb[5];
  const Prim<T>* s[2] = {&a, &b};
  T* o[2] = {Fa, Fb};
#pragma unroll
  for (int q = 0; q < 2; q++) {
    const Prim<T>& P = *s[q];
    const T iy = rcp((T)1 + P.beta);
    const T rho = (T)R.rho * ((T)1 + P.rho);
    const T dp = (T)R.p * (P.rho - P.beta) * iy;        // p - p_r
    const T dH = -(T)R.H * P.beta * iy + P.h;           // H - H_r
    const T vn = P.v1 * n1 + P.v2 * n2 + P.v3 * n3;
    o[q][0] = rho * vn;
    o[q][1] = o[q][0] * P.v1 + dp * n1;
    o[q][2] = o[q][0] * P.v2 + dp * n2;
    o[q][3] = o[q][0] * P.v3 + dp * n3;
    o[q][4] = o[q][0] * dH;
  }
#pragma unroll
  for (int c = 0; c < 5; c++) F[c] = (T)0.5 * (Fa[c] + Fb[c]);
  const double ra = R.rho * (1.0 + (double)a.rho), rb = R.rho * (1.0 + (double)b.rho);
  F0d = 0.5 * (ra * (va[0] * m[0] + va[1] * m[1] + va[2] * m[2]) +
               rb * (vb[0] * m[0] + vb[1] * m[1] + vb[2] * m[2]));
  F[0] = (T)F0d;
}

// face numerical flux in deviation form (same fluxes as face_flux, same component meaning as
// flux_ec_dev)
template <typename T>
__device__ __forceinline__ void face_flux_dev(int kind, const double uL[5], const double uR[5],
                                              const double S[3], double gamma, const Ref& R, T F[5],
                                              double& F0d) {
  // FP64 parts: the central mass flux (F(uL) + F(uR))_rho . S / 2
  const double mS = 0.5 * ((uL[1] * rcp(uL[0]) + uR[1] * rcp(uR[0])) * S[0] +
                           (uL[2] * rcp(uL[0]) + uR[2] * rcp(uR[0])) * S[1] +
                           (uL[3] * rcp(uL[0]) + uR[3] * rcp(uR[0])) * S[2]);
  if (kind == 2) {
    const Prim<T> a = make_prim_dev<T>(uL, gamma, R), b = make_prim_dev<T>(uR, gamma, R);
    flux_ec_dev(a, b, (T)S[0], (T)S[1], (T)S[2], mS, R, F, F0d);
    return;
  }
  const double cm = 0.5 * ((uL[1] + uR[1]) * S[0] + (uL[2] + uR[2]) * S[1] + (uL[3] + uR[3]) * S[2]);
  const T gm1 = (T)(gamma - 1.0);
  const T s1 = (T)S[0], s2 = (T)S[1], s3 = (T)S[2];
  const T a2s = s1 * s1 + s2 * s2 + s3 * s3;
  const T ia = rsq(a2s);
  const T area = a2s * ia;
  const T n1 = s1 * ia, n2 = s2 * ia, n3 = s3 * ia;
  T rL, vL[3], dpL, dHL, irL, rR, vR[3], dpR, dHR, irR;
  {
    const double i = rcp(uL[0]);
    const double a1 = uL[1] * i, a2 = uL[2] * i, a3 = uL[3] * i;
    const double p = (gamma - 1.0) * (uL[4] - 0.5 * uL[0] * (a1 * a1 + a2 * a2 + a3 * a3));
    rL = (T)uL[0]; vL[0] = (T)a1; vL[1] = (T)a2; vL[2] = (T)a3; irL = (T)i;
    dpL = (T)(p - R.p);
    dHL = (T)((uL[4] + p) * i - R.H);
  }
  {
    const double i = rcp(uR[0]);
    const double a1 = uR[1] * i, a2 = uR[2] * i, a3 = uR[3] * i;
    const double p = (gamma - 1.0) * (uR[4] - 0.5 * uR[0] * (a1 * a1 + a2 * a2 + a3 * a3));
    rR = (T)uR[0]; vR[0] = (T)a1; vR[1] = (T)a2; vR[2] = (T)a3; irR = (T)i;
    dpR = (T)(p - R.p);
    dHR = (T)((uR[4] + p) * i - R.H);
  }
  const T vnL = vL[0] * n1 + vL[1] * n2 + vL[2] * n3;
  const T vnR = vR[0] * n1 + vR[1] * n2 + vR[2] * n3;
  T Fs[5];
  Fs[0] = rL * vnL + rR * vnR;
  Fs[1] = rL * vnL * vL[0] + rR * vnR * vR[0] + (dpL + dpR) * n1;
  Fs[2] = rL * vnL * vL[1] + rR * vnR * vR[1] + (dpL + dpR) * n2;
  Fs[3] = rL * vnL * vL[2] + rR * vnR * vR[2] + (dpL + dpR) * n3;
  Fs[4] = rL * vnL * dHL + rR * vnR * dHR;
  if (kind == 3) {
#pragma unroll
    for (int c = 0; c < 5; c++) F[c] = (T)0.5 * area * Fs[c];
    F0d = cm;
    F[0] = (T)F0d;
    return;
  }
  if (kind == 1) {
    const T g = (T)gamma;
    const T pL = (T)R.p + dpL, pR = (T)R.p + dpR;
    const T cL2 = g * pL * irL, cR2 = g * pR * irR;
    const T lamL = fabs(vnL) + cL2 * rsq(cL2);
    const T lamR = fabs(vnR) + cR2 * rsq(cR2);
    const T lam = lamL > lamR ? lamL : lamR;
    const T du[5] = {(T)(uR[0] - uL[0]), (T)(uR[1] - uL[1]), (T)(uR[2] - uL[2]), (T)(uR[3] - uL[3]),
                     (T)((uR[4] - uL[4]) - R.H * (uR[0] - uL[0]))};
#pragma unroll
    for (int c = 0; c < 5; c++) F[c] = (T)0.5 * area * (Fs[c] - lam * du[c]);
    F0d = cm - 0.5 * (double)(area * lam) * (uR[0] - uL[0]);
    F[0] = (T)F0d;
    return;
  }
  const T x = rR * irL;
  const T Q = x * rsq(x);
  const T iw = rcp((T)1 + Q);
  const T u1 = (vL[0] + Q * vR[0]) * iw;
  const T u2 = (vL[1] + Q * vR[1]) * iw;
  const T u3 = (vL[2] + Q * vR[2]) * iw;
  const T dH = (dHL + Q * dHR) * iw;  // Roe-averaged H - H_r
  const T rho = rL * Q;
  const T q2 = u1 * u1 + u2 * u2 + u3 * u3;
  const T c2 = gm1 * ((T)R.H + dH - (T)0.5 * q2);
  const T rc = rsq(c2);
  const T c = c2 * rc;
  const T ic2 = rc * rc;
  const T vn = u1 * n1 + u2 * n2 + u3 * n3;
  const T dr = rR - rL, dp = dpR - dpL;
  const T dv1 = vR[0] - vL[0], dv2 = vR[1] - vL[1], dv3 = vR[2] - vL[2];
  const T dvn = dv1 * n1 + dv2 * n2 + dv3 * n3;
  const T a1 = (T)0.5 * (dp - rho * c * dvn) * ic2;
  const T a2 = dr - dp * ic2;
  const T a3 = (T)0.5 * (dp + rho * c * dvn) * ic2;
  const T l1 = fabs(vn - c), l2 = fabs(vn), l3 = fabs(vn + c);
  const T t1 = dv1 - dvn * n1, t2 = dv2 - dvn * n2, t3 = dv3 - dvn * n3;
  const T udt = u1 * t1 + u2 * t2 + u3 * t3;
  const T w1 = l1 * a1, w3 = l3 * a3;
  T W[5];
  W[0] = w1 + l2 * a2 + w3;
  W[1] = w1 * (u1 - c * n1) + l2 * (a2 * u1 + rho * t1) + w3 * (u1 + c * n1);
  W[2] = w1 * (u2 - c * n2) + l2 * (a2 * u2 + rho * t2) + w3 * (u2 + c * n2);
  W[3] = w1 * (u3 - c * n3) + l2 * (a2 * u3 + rho * t3) + w3 * (u3 + c * n3);
  W[4] = w1 * (dH - vn * c) + l2 * (a2 * ((T)0.5 * q2 - (T)R.H) + rho * udt) + w3 * (dH + vn * c);
#pragma unroll
  for (int k = 0; k < 5; k++) F[k] = (T)0.5 * area * (Fs[k] - W[k]);
  F0d = cm - 0.5 * (double)(area * W[0]);
  F[0] = (T)F0d;
}

// ------------------------------------------------------------------ BR1 gradient + viscous flux
// Lifted gradient of g = (v1, v2, v3, T) at this lane's node and the contravariant viscous
// flux F~v^d = sum_x Ja^d_x Fv_x (momentum 1..3, energy) in each reference direction d.
//   J grad g = sum_d Ja^d [ D_d g + (1/w_N)(g* - g) at xi_d=+1 - (1/w_0)(g* - g) at xi_d=-1 ]
template <int n, typename T>
__device__ __forceinline__ void gradient_and_viscous_flux(int t, int ti, int tj, int tk,
                                                          const double* sD, T iwN, T iw0,
                                                          const T* const sG[4],
                                                          const T (*sJ)[4][n * n], const double ja[9],
                                                          double ij, T mu, T kappa, T Fvd[3][4]) {
  constexpr int N = n - 1, nf = n * n;
  T a[3][4];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const int id = d == 0 ? ti : (d == 1 ? tj : tk);
    const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
    const int b0 = t - id * stride;
#pragma unroll
    for (int c = 0; c < 4; c++) a[d][c] = (T)0;
#pragma unroll
    for (int m = 0; m < n; m++) {
      const T Dm = (T)sD[id * n + m];
#pragma unroll
      for (int c = 0; c < 4; c++) a[d][c] += Dm * sG[c][b0 + m * stride];
    }
    const int qd = d == 0 ? tj + n * tk : (d == 1 ? ti + n * tk : ti + n * tj);
    if (id == N) {
#pragma unroll
      for (int c = 0; c < 4; c++) a[d][c] += iwN * sJ[2 * d + 1][c][qd];
    }
    if (id == 0) {
#pragma unroll
      for (int c = 0; c < 4; c++) a[d][c] -= iw0 * sJ[2 * d][c][qd];
    }
  }
  T gr[4][3];  // gr[c][x] = d g_c / d x_x
#pragma unroll
  for (int c = 0; c < 4; c++)
#pragma unroll
    for (int x = 0; x < 3; x++)
      gr[c][x] = (T)ij * ((T)ja[x] * a[0][c] + (T)ja[3 + x] * a[1][c] + (T)ja[6 + x] * a[2][c]);
  const T v1 = sG[0][t], v2 = sG[1][t], v3 = sG[2][t];
  const T divv = gr[0][0] + gr[1][1] + gr[2][2];
  T tau[3][3];
#pragma unroll
  for (int p = 0; p < 3; p++)
#pragma unroll
    for (int q = 0; q < 3; q++)
      tau[p][q] = mu * (gr[p][q] + gr[q][p]) - (p == q ? (T)(2.0 / 3.0) * mu * divv : (T)0);
  T Fv[3][4];
#pragma unroll
  for (int x = 0; x < 3; x++) {
    Fv[x][0] = tau[0][x];
    Fv[x][1] = tau[1][x];
    Fv[x][2] = tau[2][x];
    Fv[x][3] = v1 * tau[0][x] + v2 * tau[1][x] + v3 * tau[2][x] + kappa * gr[3][x];
  }
#pragma unroll
  for (int d = 0; d < 3; d++)
#pragma unroll
    for (int c = 0; c < 4; c++)
      Fvd[d][c] = (T)ja[3 * d] * Fv[0][c] + (T)ja[3 * d + 1] * Fv[1][c] + (T)ja[3 * d + 2] * Fv[2][c];
}

// g = (v1, v2, v3, T - T_ref): only differences and gradients of g enter BR1, so the constant
// T_ref (0 in FP64, p_r/rho_r in FP32-bulk) changes nothing but the rounding of T
template <typename T>
__device__ __forceinline__ void gvars(const double u[5], double gamma, double T_ref, T g[4]) {
  const double i = rcp(u[0]);
  const double a1 = u[1] * i, a2 = u[2] * i, a3 = u[3] * i;
  const double p = (gamma - 1.0) * (u[4] - 0.5 * u[0] * (a1 * a1 + a2 * a2 + a3 * a3));
  g[0] = (T)a1;
  g[1] = (T)a2;
  g[2] = (T)a3;
  g[3] = (T)(p * i - T_ref);
}

// viscous flux (eq. viscousfluxes) in physical direction x from the velocity and the gradient
// gr[c][x] of g = (v, T): momentum 1..3 and energy components
template <typename T>
__device__ __forceinline__ void viscous_flux_g(T v1, T v2, T v3, const T gr[4][3], T mu, T kappa, T Fv[3][4]) {
  const T divv = gr[0][0] + gr[1][1] + gr[2][2];
  T tau[3][3];
#pragma unroll
  for (int p = 0; p < 3; p++)
#pragma unroll
    for (int q = 0; q < 3; q++)
      tau[p][q] = mu * (gr[p][q] + gr[q][p]) - (p == q ? (T)(2.0 / 3.0) * mu * divv : (T)0);
#pragma unroll
  for (int x = 0; x < 3; x++) {
    Fv[x][0] = tau[0][x];
    Fv[x][1] = tau[1][x];
    Fv[x][2] = tau[2][x];
    Fv[x][3] = v1 * tau[0][x] + v2 * tau[1][x] + v3 * tau[2][x] + kappa * gr[3][x];
  }
}

// Face viscous fluxes of BR2 (mode 1) and the symmetric interior penalty (mode 2), in two phases.
// The viscous flux is linear in the gradient at a fixed velocity, so each face flux is the
// broken-gradient flux plus a face term:
//   BR2: + F_v(v, eta (1/J) Ja^d (x) lift_d), the lift of face d's half jump alone;
//   interior penalty: + sigma F_v(v_mean, [g] n^) . S with [g] = g(+ side) - g(- side),
//        sigma = eta (N+1)^2 |S| / (2 min(J_-, J_+)).
// Phase 1 (per node): the broken gradient (1/J) sum_d' Ja^d' D_d' g, its viscous flux, and the
// contravariant component along Ja^d for every face (d, side) the node lies on, into sFb.
template <int n, typename T>
__device__ __forceinline__ void broken_face_fluxes(int t, int ti, int tj, int tk, const double* sD,
                                                   const T* const sG[4], const double ja[9], double ij,
                                                   T mu, T kappa, T (*sFb)[4][n * n]) {
  constexpr int N = n - 1, nf = n * n;
  const int ii[3] = {ti, tj, tk};
  T a[3][4];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const int id = ii[d];
    const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
    const int b0 = t - id * stride;
#pragma unroll
    for (int c = 0; c < 4; c++) a[d][c] = (T)0;
#pragma unroll
    for (int m = 0; m < n; m++) {
      const T Dm = (T)sD[id * n + m];
#pragma unroll
      for (int c = 0; c < 4; c++) a[d][c] += Dm * sG[c][b0 + m * stride];
    }
  }
  T grb[4][3];
#pragma unroll
  for (int c = 0; c < 4; c++)
#pragma unroll
    for (int x = 0; x < 3; x++)
      grb[c][x] = (T)ij * ((T)ja[x] * a[0][c] + (T)ja[3 + x] * a[1][c] + (T)ja[6 + x] * a[2][c]);
  T Fb[3][4];
  viscous_flux_g(sG[0][t], sG[1][t], sG[2][t], grb, mu, kappa, Fb);
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const int id = ii[d];
    if (id != 0 && id != N) continue;
    const int f = 2 * d + (id == N ? 1 : 0);
    const int qd = d == 0 ? tj + n * tk : (d == 1 ? ti + n * tk : ti + n * tj);
#pragma unroll
    for (int c = 0; c < 4; c++)
      sFb[f][c][qd] = (T)ja[3 * d] * Fb[0][c] + (T)ja[3 * d + 1] * Fb[1][c] + (T)ja[3 * d + 2] * Fb[2][c];
  }
}

// Phase 2 (per face point q of face f = 2 d + side, own node io): the face flux of the scheme,
// contravariant along this element's Ja^d at io (the owner's after the face normals were made
// single-valued).  For the interior penalty the neighbour's g and J are read from global memory;
// both elements evaluate the same expression on the same values, so the penalty is single-valued.
template <int n, typename T>
__device__ __forceinline__ void face_viscous_br2_ip(const View& v, int e, int cur, double Tref, int f, int q,
                                                    int io, T iwN, T iw0, const T* const sG[4],
                                                    const T (*sJ)[4][n * n], const T (*sFb)[4][n * n],
                                                    T Ff[4]) {
  constexpr int N = n - 1, nn = n * n * n;
  const T mu = (T)v.mu, kappa = (T)v.kappa, eta = (T)v.visc_eta;
  const int d = f >> 1, side = f & 1;
  const long base = (long)e * nn;
  const T s1 = (T)v.Ja[base * 9 + (3 * d) * nn + io], s2 = (T)v.Ja[base * 9 + (3 * d + 1) * nn + io],
          s3 = (T)v.Ja[base * 9 + (3 * d + 2) * nn + io];
  const T v1 = sG[0][io], v2 = sG[1][io], v3 = sG[2][io];
  T gr[4][3], m1 = v1, m2 = v2, m3 = v3;
  if (v.visc_flux == 1) {  // BR2
    const T k = eta * (T)v.invJ[base + io];
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const T lift = side ? iwN * sJ[f][c][q] : -iw0 * sJ[f][c][q];
      gr[c][0] = k * s1 * lift;
      gr[c][1] = k * s2 * lift;
      gr[c][2] = k * s3 * lift;
    }
  } else {  // interior penalty
    const int p = q % n, r = q / n;
    const int ne = v.nbr[e * 6 + f];
    const int inb = face_node<n>(d, side ? 0 : N, p, r);
    double un[5];
#pragma unroll
    for (int c = 0; c < 5; c++) un[c] = v.U[cur][(long)ne * nn * 5 + c * nn + inb];
    T gn[4];
    gvars(un, v.gamma, Tref, gn);
    const T go[4] = {v1, v2, v3, sG[3][io]};
    const double Jo = v.J[base + io], Jn = v.J[(long)ne * nn + inb];
    const T a2 = s1 * s1 + s2 * s2 + s3 * s3;
    const T ia = rsq(a2);
    const T sigma = eta * (T)(n * n) * (a2 * ia) / ((T)2 * (T)(Jo < Jn ? Jo : Jn));
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const T jump = side ? gn[c] - go[c] : go[c] - gn[c];
      gr[c][0] = sigma * jump * s1 * ia;
      gr[c][1] = sigma * jump * s2 * ia;
      gr[c][2] = sigma * jump * s3 * ia;
    }
    m1 = (T)0.5 * (go[0] + gn[0]);
    m2 = (T)0.5 * (go[1] + gn[1]);
    m3 = (T)0.5 * (go[2] + gn[2]);
  }
  T Fp[3][4];
  viscous_flux_g(m1, m2, m3, gr, mu, kappa, Fp);
#pragma unroll
  for (int c = 0; c < 4; c++) Ff[c] = sFb[f][c][q] + (s1 * Fp[0][c] + s2 * Fp[1][c] + s3 * Fp[2][c]);
}

// ------------------------------------------------------------------ initial conditions
struct IcParams {
  double p[9];
};

// conservative state of initial condition `ic` at the point (x, y, z); parameters as listed
// with DG_IC_* in dgsem.h
__device__ __forceinline__ void ic_point(const View& v, int ic, const IcParams& P, double x, double y,
                                         double z, double U[5]) {
  const double g = v.gamma;
  double rho = 1, u = 0, w = 0, s = 0, p = 1;
  if (ic == 0) {
    rho = P.p[0]; u = P.p[1]; w = P.p[2]; s = P.p[3]; p = P.p[4];
  } else if (ic == 1) {
    const double p0 = 1.0 / (g * v.Ma * v.Ma);
    u = sin(x) * cos(y) * cos(z);
    w = -cos(x) * sin(y) * cos(z);
    s = 0;
    p = p0 + (cos(2 * x) + cos(2 * y)) * (cos(2 * z) + 2) / 16;
    rho = p / p0;
  } else if (ic == 2) {
    const double beta = P.p[0], dx = x - P.p[1], dy = y - P.p[2];
    const double r2 = dx * dx + dy * dy;
    const double pi = 3.14159265358979323846;
    const double f = beta / (2 * pi) * exp(0.5 * (1 - r2));
    u = P.p[3] - f * dy;
    w = P.p[4] + f * dx;
    s = 0;
    const double T = 1 - (g - 1) * beta * beta / (8 * g * pi * pi) * exp(1 - r2);
    rho = pow(T, 1 / (g - 1));
    p = rho * T;
  } else {
    rho = 1 + P.p[0] * sin(P.p[5] * x + P.p[6] * y + P.p[7] * z + P.p[8]);
    u = P.p[1]; w = P.p[2]; s = P.p[3]; p = P.p[4];
  }
  U[0] = rho;
  U[1] = rho * u;
  U[2] = rho * w;
  U[3] = rho * s;
  U[4] = p / (g - 1) + 0.5 * rho * (u * u + w * w + s * s);
}

}  // namespace dg
