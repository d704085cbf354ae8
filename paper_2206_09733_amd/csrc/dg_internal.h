// dg_internal.h -- layout of a bound solver as seen by the kernels, and the launch entry
// points implemented in kernels.hip.  Internal to libdgsem.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace dg {

constexpr int kMaxOrder = 7;            // largest polynomial order with a compiled kernel
constexpr int kDiagSlots = 16;          // doubles per diagnostics partial
constexpr int kTabStride = (kMaxOrder + 1) * (kMaxOrder + 1);

// Flux family of the stage kernels, compiled apart so that each kernel holds only the flux code
// its solver uses and the common family (0) keeps its registers: bit 0 = a kinetic-energy-
// preserving volume flux (codes >= 3), bit 1 = an extended surface flux (codes >= 4: entropy
// stable, Ismail-Roe, matrix dissipation, low-dissipation Roe).  Families 1..3 run in FP64 only.
__host__ __device__ constexpr int flux_family(int vol, int surf) { return (vol >= 3 ? 1 : 0) | (surf >= 4 ? 2 : 0); }

// Device tables of one order N, packed in one array (all doubles):
//   [0, n)            Lobatto nodes xi
//   [n, 2n)           quadrature weights w
//   [2n, 2n+n^2)      derivative matrix D (row-major, D[i*n+m])
//   [2n+n^2, 2n+2n^2) Dhat = D - e_N e_N^T / w_N + e_0 e_0^T / w_0
inline int tab_xi(int) { return 0; }
inline int tab_w(int n) { return n; }
inline int tab_D(int n) { return 2 * n; }
inline int tab_Dh(int n) { return 2 * n + n * n; }
inline int tab_size(int n) { return 2 * n + 2 * n * n; }
// Gauss-Legendre meshes (whose geometry is the Lobatto grid's, evaluated at the Gauss points)
// append the Lobatto nodes [g, g+n), the Lobatto derivative matrix [g+n, g+n+n^2) and the
// interpolation matrix from the Lobatto to the Gauss points [g+n+n^2, g+n+2n^2), I[q*n+l] the
// Lobatto basis function l at Gauss point q, g = tab_size(n)
inline int tab_gauss_geo_size(int n) { return n + 2 * n * n; }

// Everything a kernel needs to know about one bound uniform-order solver.
struct View {
  int E;          // elements
  int N;          // polynomial order
  int ex, ey, ez; // box cells
  int deform;
  double amp;
  double lo[3], h[3];
  double gamma, mu, kappa, Ma;
  int vol, surf, viscous, fp32;
  int visc_flux;    // 0 BR1, 1 BR2, 2 symmetric interior penalty (face viscous flux)
  int gauss;        // Gauss-Legendre nodes: tab's Dhat slot holds l_j(-1), l_j(+1) instead
  double* Tr;       // Gauss-Legendre: face traces [E][6][5][nf] of the state
  double* Sf;       // Gauss-Legendre: each element's +xi_d face metric Ja^d interpolated to its
                    // face points, [E][3 d][3 components][nf]
  double* Jt;       // Gauss-Legendre with the interior penalty: each element's trace of J on its
                    // six faces, [E][6][nf] (formed once after the geometry)
  double* Mt;       // Gauss-Legendre with BR2: the metric factor of each face's lift, traced,
                    // sum_i l_i(side) (+-l_i(side) / w_i) Ja^d_i / J_i, [E][6][3][nf]
  double visc_eta;  // BR2 lifting factor or interior-penalty factor
  double rho_r, p_r;  // FP32-bulk reference state (mean density and pressure of the state set)
  const int* nbr; // [E][6] neighbour across face f = 2 d + side (side 1: xi_d = +1)
  const double* tab;
  double* X;      // [E][3][nn]   node coordinates
  double* Ja;     // [E][9][nn]   Ja^d_c at index 3 d + c
  double* J;      // [E][nn]
  double* invJ;   // [E][nn]
  double* U[2];   // ping-pong state buffers [E][5][nn]
  double* dU;     // RK register [E][5][nn]
  double* R;      // residual [E][5][nn]
  double* Fvf;    // [E][6][4][nf] contravariant viscous flux on the element's faces
  double* part;   // diagnostics partials [E][kDiagSlots]
  double* diag;   // final diagnostics [kDiagSlots]
  // adaptive step size: while dtp is set the stage kernels take the step size from *dtp (written
  // on the device by dt_kernel) instead of their dt argument; adapt[0] the step size,
  // adapt[1] the time advanced, adapt[2] the count of non-finite or non-physical nodes seen;
  // adapt[3] the largest wave speed of the current stage's state (global Lax-Friedrichs)
  const double* dtp;
  double* adapt;
  // per-element anisotropic orders (mixed != 0): node counts per direction and first node of
  // each element, elements in launch order (largest first), Lobatto tables of every order
  // (offset tab_off[N] in tab) and mortar matrices (I_{N->M} then P_{M->N} at mort_off[N][M])
  int mixed;
  int nmax;
  const int4* elem;
  // face 3 e + d of the face pass (the face on e's +d side): {R = nbr(e, +d), node counts of e
  // then R along directions 0, 1, 2 (3 bits each, from bit 0), first node of e, first node of R}
  const int4* fdesc;
  // the launch order (largest elements first): {element, node counts along 0, 1, 2 (3 bits
  // each, from bit 0), first node, node count}
  const int4* work;
  const double* mtab;
  int tab_off[kMaxOrder + 1];
  int mort_off[kMaxOrder + 1][kMaxOrder + 1];
  // work-list range [mix_beg[b], mix_beg[b] + mix_cnt[b]) of the elements with
  // 64 b < nodes <= 64 (b + 1)
  int mix_beg[6], mix_cnt[6];
  // face fluxes of mixed-order meshes: [E][6 faces][6][49], rows 0-4 the numerical flux on the
  // element's face grid, row 5 its FP64 mass component (FP32-bulk)
  double* Fs;
  // spectral vanishing viscosity folded into the Navier-Stokes stage kernel (set only in the View
  // of that launch): the filtered contravariant flux [E][12][nn] of the stage's input state,
  // index 4 d + c (c = momentum 1..3, energy), added to the viscous flux
  const double* Fa;
};

// Several solvers of one order and precision advanced by one launch: workgroup b of the grid
// works on element b - start[m] of member m (start[m] <= b < start[m+1]); each member's View
// lives in device memory (a copy inside the member's own buffer).
constexpr int kMaxBatch = 32;
struct BatchArgs {
  const View* view[kMaxBatch];
  int start[kMaxBatch + 1];
  int cur[kMaxBatch];
  double dt[kMaxBatch];
  int n;
};

// Launchers (kernels.hip).  All enqueue on `st` and return the hipError_t of the launch.
hipError_t launch_geometry(const View& v, hipStream_t st);
hipError_t launch_ic(const View& v, int cur, int ic, const double* params, hipStream_t st);
// Navier-Stokes pass A: BR1 gradient and face viscous fluxes of U[cur]
hipError_t launch_gradient(const View& v, int cur, hipStream_t st);
// residual (+ RK update) of U[cur]; for Navier-Stokes launch_gradient must precede it
hipError_t launch_stage(const View& v, int cur, double dt, double rkA, double rkB, int mode,
                        hipStream_t st);
hipError_t launch_diagnostics(const View& v, int cur, hipStream_t st);
hipError_t launch_diag_final(const View& v, hipStream_t st);  // partials -> diag, fixed order
// batched Navier-Stokes gradient pass and stage of members of order N (all viscous, or all
// inviscid for the stage), FP32-bulk or FP64
hipError_t launch_gradient_batch(const BatchArgs& B, int N, bool fp32, bool xv, hipStream_t st);  // xv: BR2/IP
hipError_t launch_stage_batch(const BatchArgs& B, int N, bool fp32, bool visc, int fx, double rkA, double rkB,
                              int mode, hipStream_t st);  // fx: the members' flux family
// Gauss-Legendre nodes: face traces of U[cur], then the weak-form residual / RK stage
hipError_t launch_stage_gauss(const View& v, int cur, double dt, double rkA, double rkB, int mode, hipStream_t st);
// Gauss-Legendre with the interior penalty or BR2: the face factors Jt or Mt (after launch_geometry)
hipError_t launch_jtrace_gauss(const View& v, hipStream_t st);
// adaptive step size (uniform and mixed orders): clear adapt[], then per step reduce the wave
// speeds of U[cur] and write the step size to adapt[0]
hipError_t launch_adapt_reset(const View& v, hipStream_t st);
// global Lax-Friedrichs: the largest |v| + c of U[cur] into adapt[3], before each stage
hipError_t launch_lambda_max(const View& v, int cur, hipStream_t st);
hipError_t launch_step_size(const View& v, int cur, double cfl, double hmin, double n1, double gamma, double Pr,
                            double mu_eff, hipStream_t st);
// the extended flux families 1..3 (FP64), in kernels_ext.hip; called by the two launchers above
hipError_t launch_stage_ext(const View& v, int fx, int cur, double dt, double rkA, double rkB, int mode,
                            hipStream_t st);
hipError_t launch_stage_batch_ext(const BatchArgs& B, int N, bool visc, int fx, double rkA, double rkB, int mode,
                                  hipStream_t st);

// mixed-order meshes (kernels_mixed.hip).  The stage runs one launch per bucket of elements
// (bucket b: 64 b < nodes <= 64 (b + 1)); bit b of `tiles` gives bucket b two nodes per lane
// instead of one.
constexpr int kMixMaxOrder = 6;
constexpr int kMixBuckets = 6;
hipError_t launch_geometry_mixed(const View& v, hipStream_t st);
hipError_t launch_ic_mixed(const View& v, int cur, int ic, const double* params, hipStream_t st);
// Side streams (default priority) and events over which the bucket launches of a stage run
// concurrently: each bucket alone leaves the device partly idle at its end.  The fork and join
// are events recorded on st, so the launches also form one graph under stream capture.
constexpr int kMixSide = 3;
struct MixStreams {
  hipStream_t side[kMixSide];
  hipEvent_t fork, join[kMixSide];
};
// ms == nullptr: the buckets one after the other on st
hipError_t launch_stage_mixed(const View& v, int cur, double dt, double rkA, double rkB, int mode,
                              int tiles, hipStream_t st, const MixStreams* ms);
hipError_t launch_stage_mixed_bucket(const View& v, int b, int npl, int cur, double dt, double rkA,
                                     double rkB, int mode, hipStream_t st);
// the face pass alone (launch_stage_mixed runs it before the buckets)
hipError_t launch_faces_mixed(const View& v, int cur, hipStream_t st);
constexpr int kMixFaceDoubles = 6 * 6 * 49;  // Fs doubles per element
hipError_t launch_diagnostics_mixed(const View& v, int cur, hipStream_t st);

// stage modes
constexpr int kModeRK = 0;        // dU <- A dU + dt R; U[cur^1] <- U[cur] + B dU
constexpr int kModeResidual = 1;  // R <- dU/dt of U[cur]

}  // namespace dg
