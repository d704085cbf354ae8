// svv.h -- spectral vanishing viscosity (section "Shock capturing"): launch interface of the
// kernels in kernels_svv.hip, for Gauss-Lobatto, uniform-order solvers (the filtered flux in FP64
// in both precisions).  The filtered flux either enters the Navier-Stokes stage kernel's viscous
// flux (launch_svv_flux or launch_grad_svv before it), or its divergence is added to what the
// stage kernel produced (launch_svv after it).
#pragma once

#include <hip/hip_runtime.h>

#include "dg_internal.h"
#include "dgsem.h"  // DG_LES_* model codes

namespace dg {

struct SvvArgs {
  double mu, kappa;     // artificial viscosity and conductivity mu gamma / ((gamma-1) Pr)
  double les_c;         // explicit LES: the model's constant (0: constant viscosity)
  int les_model;        // DG_LES_SMAGORINSKY, DG_LES_WALE or DG_LES_VREMAN
  double kfac;          // gamma / ((gamma-1) Pr): conductivity per unit viscosity
  double sensor;        // density-sensor threshold; < 0: every element filtered
  const double* filt;   // (I - Phi) of one direction, (N+1) x (N+1) row-major: Phi = V diag(s) V^-1
  double* Fa;           // filtered contravariant flux Ja^d . F [E][12][nn]: index 4 d + c, d the
                        // reference direction, c = momentum 1..3, energy
};

// The term for stage input U[cur]: kernel 1 forms the filtered flux of every element; kernel 2
// its divergence with the averaged face flux, R_a.  mode kModeResidual: R += R_a.  mode kModeRK
// (after the stage kernel wrote dU and U[cur^1] for the same stage): dU += h R_a and
// U[cur^1] += b h R_a, h = *v.dtp if set, else dt.
hipError_t launch_svv(const View& v, int cur, const SvvArgs& a, double dt, double b, int mode, hipStream_t st);
// kernel 2 alone (after kernel 1 and, on a halo box, the exchange of the filtered flux), modes
// as launch_svv
hipError_t launch_svv_div(const View& v, int cur, const SvvArgs& a, double dt, double b, int mode, hipStream_t st);
// kernel 1 alone, for a stage kernel that takes the filtered flux itself (View::Fa = a.Fa): it
// enters that kernel's viscous volume and face terms, which then hold R_a, and kernel 2 is not run
hipError_t launch_svv_flux(const View& v, int cur, const SvvArgs& a, hipStream_t st);
// Navier-Stokes with BR1: the gradient pass (launch_gradient) and kernel 1 in one launch
hipError_t launch_grad_svv(const View& v, int cur, const SvvArgs& a, hipStream_t st);

// Host: (I - Phi) for order N, kernel (0 Tadmor, 1 Maday) and cutoff M, from the Legendre
// polynomials at the Lobatto nodes xi with weights w (long double, rounded once).
void svv_filter_table(int N, int kernel, int M, const double* xi, const double* w, double* out);

}  // namespace dg
