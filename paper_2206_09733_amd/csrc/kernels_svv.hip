// kernels_svv.hip -- spectral vanishing viscosity (section "Shock capturing"), FP64 for solvers
// of either precision, uniform order N on Gauss-Lobatto nodes, one workgroup per element, one
// lane per node.
//
// The artificial flux is the Navier-Stokes viscous flux with viscosity mu_a and conductivity
// kappa_a = mu_a gamma / ((gamma-1) Pr), written in the entropy variables w (eq.
// shock:fluxmatrix) as B G with G the BR1 gradient of w.  B = L^T D L with L G the symmetric
// traceless part of Z_kj = d_j w_{k+1} + v_k d_j w_5 (weights 2 mu theta, theta = p/rho) and
// grad w_5 (weights kappa theta^2).  Because the filter is linear and the same for every field,
// the half-filtered flux of eq. shock:filteredflux reduces to
//   stress tau = 2 sqrt(mu theta / J) F*( sqrt(J mu theta) sym-dev(Z) ),
//   heat   q   = theta sqrt(kappa / J) F*( theta sqrt(J kappa) grad w_5 ),
//   flux along x: momentum tau_kx, energy v . tau_x + q_x,
// so nine nodal fields are filtered.  In three directions a Legendre mode (a, b, c) is multiplied
// by 1 - (1 - s_a)(1 - s_b)(1 - s_c), i.e. F* y = y - Q_x Q_y Q_z y with the one-direction
// low-pass Q = I - Phi: three passes of an (N+1) x (N+1) matrix along the element's lines.
// Elements whose density sensor s = sum w_i w_j w_k J |grad_xi rho|^2 exceeds the threshold
// take the unfiltered flux.  The residual of the term is the divergence of the contravariant
// flux with BR1 face terms (the average of the two sides' fluxes along the owner's Ja^d): on
// Navier-Stokes with the standard fluxes the stage kernel forms it with the viscous flux (the
// flux kernel runs before it, with BR1 in one launch with the gradient pass, in FP64 or FP32-bulk);
// otherwise (Euler, the extended flux families) svv_div_kernel adds it after the stage kernel.
// Explicit LES closure (turbulence models: Smagorinsky, WALE, Vreman, SVV-Smagorinsky): the
// viscosity gains the model's rho nu_t node by node, from g = grad v = theta Z and
// Delta = 2 (J/(N+1)^3)^(1/3) (the formulas are in the C header); mu and kappa enter only through
// sqrt(mu) and sqrt(kappa) at the node itself, so the factorisation holds with the local values.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "dg_device.h"
#include "grad_body.h"
#include "svv.h"

namespace dg {

template <int N>
__device__ __forceinline__ void svv_flux_body(const View& v, const int e, const int cur, const SvvArgs& a) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n, NT = nthreads_for(N), NW = NT / 64;
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int ti = t % n, tj = (t / n) % n, tk = t / nf;
  const int ii[3] = {ti, tj, tk};
  const double* __restrict__ Uin = v.U[cur];
  __shared__ double sD[n * n], sQ[n * n], sw[n];
  __shared__ double sRed[NW];
  // phase 1: rho and the entropy variables w2..w5, the half jumps of w2..w5 on the six faces;
  // phase 2 (after the barrier of the sensor sum): the fields being filtered
  constexpr int kRaw = 5 * nn + 24 * nf > 9 * nn ? 5 * nn + 24 * nf : 9 * nn;
  __shared__ double sRaw[kRaw];
  double(*sW)[nn] = reinterpret_cast<double(*)[nn]>(sRaw);
  double(*sL)[4][nf] = reinterpret_cast<double(*)[4][nf]>(sRaw + 5 * nn);
  double(*sY)[nn] = reinterpret_cast<double(*)[nn]>(sRaw);
  for (int x = t; x < n * n; x += NT) {
    sD[x] = v.tab[2 * n + x];
    sQ[x] = a.filt[x];
  }
  if (t < n) sw[t] = v.tab[n + t];
  const long base = (long)e * nn;
  const double g1 = v.gamma - 1.0;
  double vel[3] = {0, 0, 0}, th = 1.0, rho = 1.0;
  double mu = a.mu, kappa = a.kappa;  // the node's viscosity and conductivity
  // the neighbour's state at this lane's first face point, requested with the node's own state
  // so that the two memory round trips overlap (face point clamped: every lane loads)
  auto face_nb = [&](int x, double un[5]) {
    const int f = x / nf, q = x - f * nf;
    const int d = f >> 1, side = f & 1;
    const int p = q % n, r = q / n;
    const int ne = v.nbr[e * 6 + f];
    const int inb = face_node<n>(d, side ? 0 : N, p, r);
#pragma unroll
    for (int c = 0; c < 5; c++) un[c] = Uin[(long)ne * nn * 5 + c * nn + inb];
  };
  double un0[5];
  face_nb(t < 6 * nf ? t : 0, un0);
  if (act) {
    double u[5];
#pragma unroll
    for (int c = 0; c < 5; c++) u[c] = Uin[base * 5 + c * nn + t];
    const double ir = 1.0 / u[0];
#pragma unroll
    for (int c = 0; c < 3; c++) vel[c] = u[1 + c] * ir;
    const double p = g1 * (u[4] - 0.5 * u[0] * (vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2]));
    const double b = u[0] / p;  // 1 / theta
    th = p * ir;
    rho = u[0];
    sW[0][t] = u[0];
#pragma unroll
    for (int c = 0; c < 3; c++) sW[1 + c][t] = b * vel[c];
    sW[4][t] = -b;
  }
  __syncthreads();
  // the metric terms, requested before the face work so that their latency overlaps it
  double ja[9], J = 1.0, ij = 1.0;
  if (act) {
#pragma unroll
    for (int c = 0; c < 9; c++) ja[c] = v.Ja[base * 9 + c * nn + t];
    J = v.J[base + t];
    ij = v.invJ[base + t];
  }
  for (int x = t; x < 6 * nf; x += NT) {
    const int f = x / nf, q = x - f * nf;
    const int d = f >> 1, side = f & 1;
    const int p = q % n, r = q / n;
    const int io = face_node<n>(d, side ? N : 0, p, r);
    double un[5];
    if (x == t) {
#pragma unroll
      for (int c = 0; c < 5; c++) un[c] = un0[c];
    } else {
      face_nb(x, un);
    }
    const double ir = 1.0 / un[0];
    const double w1 = un[1] * ir, w2 = un[2] * ir, w3 = un[3] * ir;
    const double pn = g1 * (un[4] - 0.5 * un[0] * (w1 * w1 + w2 * w2 + w3 * w3));
    const double b = un[0] / pn;
    sL[f][0][q] = 0.5 * (b * w1 - sW[1][io]);
    sL[f][1][q] = 0.5 * (b * w2 - sW[2][io]);
    sL[f][2][q] = 0.5 * (b * w3 - sW[3][io]);
    sL[f][3][q] = 0.5 * (-b - sW[4][io]);
  }
  __syncthreads();
  // gradients of w2..w5 (lifted), the sensor's share of this node
  double G[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double sens = 0.0;
  if (act) {
    const double iwN = 1.0 / sw[N], iw0 = 1.0 / sw[0];
    double g2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const int id = ii[d];
      const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
      const int b0 = t - id * stride;
      const int qd = d == 0 ? tj + n * tk : (d == 1 ? ti + n * tk : ti + n * tj);
      double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
      for (int m = 0; m < n; m++) {
        const double Dm = sD[id * n + m];
#pragma unroll
        for (int c = 0; c < 5; c++) acc[c] += Dm * sW[c][b0 + m * stride];
      }
      g2 += acc[0] * acc[0];
      if (id == N) {
#pragma unroll
        for (int c = 0; c < 4; c++) acc[1 + c] += iwN * sL[2 * d + 1][c][qd];
      }
      if (id == 0) {
#pragma unroll
        for (int c = 0; c < 4; c++) acc[1 + c] -= iw0 * sL[2 * d][c][qd];
      }
#pragma unroll
      for (int x = 0; x < 3; x++) {
#pragma unroll
        for (int c = 0; c < 4; c++) G[c][x] += ja[3 * d + x] * acc[1 + c];
      }
    }
#pragma unroll
    for (int c = 0; c < 4; c++)
#pragma unroll
      for (int x = 0; x < 3; x++) G[c][x] *= ij;
    sens = sw[ti] * sw[tj] * sw[tk] * J * g2;
  }
  // element sum of the sensor (fixed order: lanes of a wave, then the waves)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sens += __shfl_xor(sens, o);
  if ((t & 63) == 0) sRed[t >> 6] = sens;
  __syncthreads();
  double s_el = 0.0;
#pragma unroll
  for (int k = 0; k < NW; k++) s_el += sRed[k];
  const bool filter = !(a.sensor >= 0.0 && s_el > a.sensor);
  // the nine fields: sqrt(J mu theta) sym-dev(Z), theta sqrt(J kappa) grad w5
  double y[9], sv = 0.0, sq = 0.0;
  {
    double Z[3][3];
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
      for (int j = 0; j < 3; j++) Z[k][j] = G[k][j] + vel[k] * G[3][j];
    const double tr3 = (Z[0][0] + Z[1][1] + Z[2][2]) * (1.0 / 3.0);
    if (a.les_c > 0.0) {  // explicit LES: the model's eddy viscosity at this node
      double g[3][3], ss = 0.0;  // g = grad v, ss = S:S
#pragma unroll
      for (int k = 0; k < 3; k++)
#pragma unroll
        for (int j = 0; j < 3; j++) g[k][j] = th * Z[k][j];
#pragma unroll
      for (int k = 0; k < 3; k++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
          const double sk = 0.5 * (g[k][j] + g[j][k]);
          ss += sk * sk;
        }
      const double delta = 2.0 * cbrt(J * (1.0 / nn)), cd2 = a.les_c * a.les_c * delta * delta;
      double nu;
      if (a.les_model == DG_LES_SMAGORINSKY) {
        nu = cd2 * sqrt(2.0 * ss);
      } else if (a.les_model == DG_LES_WALE) {
        double g2[3][3], sd = 0.0;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
          for (int j = 0; j < 3; j++) g2[i][j] = g[i][0] * g[0][j] + g[i][1] * g[1][j] + g[i][2] * g[2][j];
        const double tr3 = (g2[0][0] + g2[1][1] + g2[2][2]) * (1.0 / 3.0);
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
          for (int j = 0; j < 3; j++) {
            const double x = 0.5 * (g2[i][j] + g2[j][i]) - (i == j ? tr3 : 0.0);
            sd += x * x;
          }
        const double rs = sqrt(sd), den = ss * ss * sqrt(ss) + sd * sqrt(rs);  // (S:S)^5/2 + (Sd:Sd)^5/4
        nu = den > 0.0 ? cd2 * sd * rs / den : 0.0;
      } else {  // Vreman
        double b[3][3], gg = 0.0;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
          for (int j = 0; j < 3; j++) {
            b[i][j] = delta * delta * (g[i][0] * g[j][0] + g[i][1] * g[j][1] + g[i][2] * g[j][2]);
            gg += g[i][j] * g[i][j];
          }
        const double B = b[0][0] * b[1][1] - b[0][1] * b[0][1] + b[0][0] * b[2][2] - b[0][2] * b[0][2] +
                         b[1][1] * b[2][2] - b[1][2] * b[1][2];
        nu = gg > 0.0 && B > 0.0 ? a.les_c * sqrt(B / gg) : 0.0;
      }
      mu = a.mu + rho * nu;
      kappa = mu * a.kfac;
    }
    sv = sqrt(J * mu * th);
    sq = th * sqrt(J * kappa);
    y[0] = sv * (Z[0][0] - tr3);
    y[1] = sv * (Z[1][1] - tr3);
    y[2] = sv * (Z[2][2] - tr3);
    y[3] = sv * 0.5 * (Z[0][1] + Z[1][0]);
    y[4] = sv * 0.5 * (Z[0][2] + Z[2][0]);
    y[5] = sv * 0.5 * (Z[1][2] + Z[2][1]);
#pragma unroll
    for (int x = 0; x < 3; x++) y[6 + x] = sq * G[3][x];
  }
  if (filter) {  // uniform over the workgroup
    double r[9];
#pragma unroll
    for (int c = 0; c < 9; c++) r[c] = y[c];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      if (act) {
#pragma unroll
        for (int c = 0; c < 9; c++) sY[c][t] = r[c];
      }
      __syncthreads();
      if (act) {
        const int id = ii[d];
        const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
        const int b0 = t - id * stride;
#pragma unroll
        for (int c = 0; c < 9; c++) r[c] = 0.0;
#pragma unroll
        for (int m = 0; m < n; m++) {
          const double Qm = sQ[id * n + m];
#pragma unroll
          for (int c = 0; c < 9; c++) r[c] += Qm * sY[c][b0 + m * stride];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < 9; c++) y[c] -= r[c];
  }
  if (!act) return;
  // 2 sqrt(mu theta / J) and theta sqrt(kappa / J), from the factors of the filtered fields
  const double ks = 2.0 * sv * ij, kq = sq * ij;
  const double tau[3][3] = {{ks * y[0], ks * y[3], ks * y[4]},
                            {ks * y[3], ks * y[1], ks * y[5]},
                            {ks * y[4], ks * y[5], ks * y[2]}};
  double F[3][4];  // physical flux along x: momentum, energy
#pragma unroll
  for (int x = 0; x < 3; x++) {
#pragma unroll
    for (int k = 0; k < 3; k++) F[x][k] = tau[k][x];
    F[x][3] = vel[0] * tau[0][x] + vel[1] * tau[1][x] + vel[2] * tau[2][x] + kq * y[6 + x];
  }
  double* Fa = a.Fa + base * 12;
#pragma unroll
  for (int d = 0; d < 3; d++) {  // Ja read again (this workgroup read it above: an L2 hit)
    const double j0 = v.Ja[base * 9 + (3 * d) * nn + t], j1 = v.Ja[base * 9 + (3 * d + 1) * nn + t],
                 j2 = v.Ja[base * 9 + (3 * d + 2) * nn + t];
#pragma unroll
    for (int c = 0; c < 4; c++) Fa[(4 * d + c) * nn + t] = j0 * F[0][c] + j1 * F[1][c] + j2 * F[2][c];
  }
}

template <int N>
__global__ void __launch_bounds__(nthreads_for(N))
    svv_div_kernel(View v, int cur, SvvArgs a, double dt, double rkB, int mode) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n, NT = nthreads_for(N);
  const int e = block_element(v.E);
  const int t = threadIdx.x;
  const bool act = t < nn;
  const int ti = t % n, tj = (t / n) % n, tk = t / nf;
  const int ii[3] = {ti, tj, tk};
  __shared__ double sD[n * n], sw[n];
  __shared__ double sF[4][nn];  // contravariant flux of the direction being processed
  for (int x = t; x < n * n; x += NT) sD[x] = v.tab[2 * n + x];
  if (t < n) sw[t] = v.tab[n + t];
  const long base = (long)e * nn;
  double acc[4] = {0, 0, 0, 0};
#pragma unroll
  for (int d = 0; d < 3; d++) {
    double Fd[4] = {0, 0, 0, 0};
    if (act) {
#pragma unroll
      for (int c = 0; c < 4; c++) Fd[c] = a.Fa[base * 12 + (4 * d + c) * nn + t];
    }
    __syncthreads();  // previous direction's readers are done
    if (act) {
#pragma unroll
      for (int c = 0; c < 4; c++) sF[c][t] = Fd[c];
    }
    __syncthreads();
    if (!act) continue;
    const int id = ii[d];
    const int stride = d == 0 ? 1 : (d == 1 ? n : nf);
    const int b0 = t - id * stride;
#pragma unroll
    for (int m = 0; m < n; m++) {
      const double Dm = sD[id * n + m];
#pragma unroll
      for (int c = 0; c < 4; c++) acc[c] += Dm * sF[c][b0 + m * stride];
    }
    // faces: (F~* - F~) = S . (F_other - F_own) / 2, S the owner's Ja^d.  The face normals are
    // single-valued (the -d side holds the owner's Ja^d), so the other side's stored
    // contravariant flux at the matching node is S . F_other.
#pragma unroll
    for (int side = 0; side < 2; side++) {
      if (id != (side ? N : 0)) continue;
      const int ne = v.nbr[e * 6 + 2 * d + side];
      const int p = d == 0 ? tj : ti, r = d == 2 ? tj : tk;
      const int inb = face_node<n>(d, side ? 0 : N, p, r);
      const double* Fo = a.Fa + (long)ne * nn * 12;
      const double wgt = side ? 0.5 / sw[N] : -0.5 / sw[0];
#pragma unroll
      for (int c = 0; c < 4; c++) acc[c] += wgt * (Fo[(4 * d + c) * nn + inb] - Fd[c]);
    }
  }
  if (!act) return;
  const double ij = v.invJ[base + t];
  const long o = base * 5 + t;
  if (mode == kModeResidual) {
#pragma unroll
    for (int c = 0; c < 4; c++) v.R[o + (1 + c) * nn] += acc[c] * ij;
    return;
  }
  const double h = v.dtp ? *v.dtp : dt;
  double* __restrict__ Uout = v.U[cur ^ 1];
#pragma unroll
  for (int c = 0; c < 4; c++) {
    const double du = h * (acc[c] * ij);
    v.dU[o + (1 + c) * nn] += du;
    Uout[o + (1 + c) * nn] += rkB * du;
  }
}

// occupancy target: 4 waves per SIMD up to order 6 (no spills), 3 at order 7
template <int N>
__global__ void __launch_bounds__(nthreads_for(N)) __attribute__((amdgpu_waves_per_eu(N <= 6 ? 4 : 3)))
    svv_flux_kernel(View v, int cur, SvvArgs a) {
  svv_flux_body<N>(v, block_element(v.E), cur, a);
}

// Navier-Stokes pass A (BR1, in the solver's precision T) and the SVV flux (FP64) of the same
// element in one workgroup: the second body reads the element's state, metric terms and
// neighbour traces that the first has just read, from the L2 cache instead of HBM.  The two
// bodies share no LDS and no results.
template <int N, typename T>
__global__ void __launch_bounds__(nthreads_for(N)) __attribute__((amdgpu_waves_per_eu(N <= 6 ? 4 : 3)))
    grad_svv_kernel(View v, int cur, SvvArgs a) {
  const int e = block_element(v.E);
  grad_body<N, T, false>(v, e, cur);
  svv_flux_body<N>(v, e, cur, a);
}

template <int N>
static hipError_t launch_svv_n(const View& v, int cur, const SvvArgs& a, double dt, double b, int mode,
                               hipStream_t st) {
  hipLaunchKernelGGL(svv_flux_kernel<N>, dim3(v.E), dim3(nthreads_for(N)), 0, st, v, cur, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(svv_div_kernel<N>, dim3(v.E), dim3(nthreads_for(N)), 0, st, v, cur, a, dt, b, mode);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_svv_div_n(const View& v, int cur, const SvvArgs& a, double dt, double b, int mode,
                                   hipStream_t st) {
  hipLaunchKernelGGL(svv_div_kernel<N>, dim3(v.E), dim3(nthreads_for(N)), 0, st, v, cur, a, dt, b, mode);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_svv_flux_n(const View& v, int cur, const SvvArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(svv_flux_kernel<N>, dim3(v.E), dim3(nthreads_for(N)), 0, st, v, cur, a);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_grad_svv_n(const View& v, int cur, const SvvArgs& a, hipStream_t st) {
  if (v.fp32)
    hipLaunchKernelGGL((grad_svv_kernel<N, float>), dim3(v.E), dim3(nthreads_for(N)), 0, st, v, cur, a);
  else
    hipLaunchKernelGGL((grad_svv_kernel<N, double>), dim3(v.E), dim3(nthreads_for(N)), 0, st, v, cur, a);
  return hipGetLastError();
}

hipError_t launch_grad_svv(const View& v, int cur, const SvvArgs& a, hipStream_t st) {
  if (v.mixed || v.gauss || !v.viscous || v.visc_flux != 0 || v.E <= 0 || !a.filt || !a.Fa)
    return hipErrorInvalidValue;
  switch (v.N) {
    case 1: return launch_grad_svv_n<1>(v, cur, a, st);
    case 2: return launch_grad_svv_n<2>(v, cur, a, st);
    case 3: return launch_grad_svv_n<3>(v, cur, a, st);
    case 4: return launch_grad_svv_n<4>(v, cur, a, st);
    case 5: return launch_grad_svv_n<5>(v, cur, a, st);
    case 6: return launch_grad_svv_n<6>(v, cur, a, st);
    case 7: return launch_grad_svv_n<7>(v, cur, a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_svv_div(const View& v, int cur, const SvvArgs& a, double dt, double b, int mode, hipStream_t st) {
  if (v.mixed || v.gauss || v.E <= 0 || !a.filt || !a.Fa) return hipErrorInvalidValue;
  switch (v.N) {
    case 1: return launch_svv_div_n<1>(v, cur, a, dt, b, mode, st);
    case 2: return launch_svv_div_n<2>(v, cur, a, dt, b, mode, st);
    case 3: return launch_svv_div_n<3>(v, cur, a, dt, b, mode, st);
    case 4: return launch_svv_div_n<4>(v, cur, a, dt, b, mode, st);
    case 5: return launch_svv_div_n<5>(v, cur, a, dt, b, mode, st);
    case 6: return launch_svv_div_n<6>(v, cur, a, dt, b, mode, st);
    case 7: return launch_svv_div_n<7>(v, cur, a, dt, b, mode, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_svv_flux(const View& v, int cur, const SvvArgs& a, hipStream_t st) {
  if (v.mixed || v.gauss || v.E <= 0 || !a.filt || !a.Fa) return hipErrorInvalidValue;
  switch (v.N) {
    case 1: return launch_svv_flux_n<1>(v, cur, a, st);
    case 2: return launch_svv_flux_n<2>(v, cur, a, st);
    case 3: return launch_svv_flux_n<3>(v, cur, a, st);
    case 4: return launch_svv_flux_n<4>(v, cur, a, st);
    case 5: return launch_svv_flux_n<5>(v, cur, a, st);
    case 6: return launch_svv_flux_n<6>(v, cur, a, st);
    case 7: return launch_svv_flux_n<7>(v, cur, a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_svv(const View& v, int cur, const SvvArgs& a, double dt, double b, int mode, hipStream_t st) {
  if (v.mixed || v.gauss || v.E <= 0 || !a.filt || !a.Fa) return hipErrorInvalidValue;
  switch (v.N) {
    case 1: return launch_svv_n<1>(v, cur, a, dt, b, mode, st);
    case 2: return launch_svv_n<2>(v, cur, a, dt, b, mode, st);
    case 3: return launch_svv_n<3>(v, cur, a, dt, b, mode, st);
    case 4: return launch_svv_n<4>(v, cur, a, dt, b, mode, st);
    case 5: return launch_svv_n<5>(v, cur, a, dt, b, mode, st);
    case 6: return launch_svv_n<6>(v, cur, a, dt, b, mode, st);
    case 7: return launch_svv_n<7>(v, cur, a, dt, b, mode, st);
    default: return hipErrorInvalidValue;
  }
}

// (I - Phi)_ij = delta_ij - sum_k P_k(x_i) s_k w_j P_k(x_j) / g_k, g_k = sum_i w_i P_k(x_i)^2: the
// Legendre transform by the nodal quadrature (exact: the Lobatto rule keeps the P_k orthogonal),
// the kernel s_k, and back.
void svv_filter_table(int N, int kernel, int M, const double* xi, const double* w, double* out) {
  const int n = N + 1;
  std::vector<long double> P((size_t)n * n);  // P[k * n + i] = P_k(x_i)
  for (int i = 0; i < n; i++) {
    long double pm = 1.0L, pc = xi[i];
    P[i] = 1.0L;
    if (N >= 1) P[n + i] = pc;
    for (int k = 1; k < N; k++) {
      const long double pn = ((2.0L * k + 1.0L) * xi[i] * pc - k * pm) / (k + 1.0L);
      pm = pc;
      pc = pn;
      P[(size_t)(k + 1) * n + i] = pn;
    }
  }
  std::vector<long double> s(n), g(n);
  for (int k = 0; k < n; k++) {
    if (k <= M) s[k] = 0.0L;
    else if (kernel == 0) s[k] = 1.0L;
    else {
      const long double r = (long double)(k - N) / (long double)(k - M);
      s[k] = expl(-r * r);
    }
    long double acc = 0.0L;
    for (int i = 0; i < n; i++) acc += (long double)w[i] * P[(size_t)k * n + i] * P[(size_t)k * n + i];
    g[k] = acc;
  }
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) {
      long double phi = 0.0L;
      for (int k = 0; k < n; k++) phi += P[(size_t)k * n + i] * s[k] * (long double)w[j] * P[(size_t)k * n + j] / g[k];
      out[i * n + j] = (double)((i == j ? 1.0L : 0.0L) - phi);
    }
}

}  // namespace dg
