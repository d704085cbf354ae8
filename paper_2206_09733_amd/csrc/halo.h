// halo.h -- the halo exchange of a box run as one block of a split domain (dg_box_desc.halo):
// launch interface of the kernels in kernels_halo.hip.  Ghost element k (index E + k) stands for
// the element across box-boundary face k; entry k of the map is {source element, its face,
// ghost element, the ghost's face}, the source being the block's periodic image of the
// neighbour, and the two faces the same face number.
#pragma once

#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dg {

struct HaloArgs {
  const int4* map;  // [K] {src element, src face, ghost element, ghost face}
  int K;            // box-boundary faces (= ghost elements)
  double* send;     // state face values [K][5][nf] (also the SVV flux's [K][4][nf] and J's [K][nf])
  double* recv;
  double* sendv;    // face viscous fluxes [K][4][nf] (FP32-bulk: floats), Navier-Stokes only
  double* recvv;
};

// the state U[cur]: pack its boundary face values, move them to the receive buffer, unpack them
// into the ghosts' faces (every launch on st)
hipError_t halo_exchange_state(const View& v, int cur, const HaloArgs& h, hipStream_t st);
// the face viscous fluxes Fvf (after the gradient pass), the same way
hipError_t halo_exchange_viscous(const View& v, const HaloArgs& h, hipStream_t st);
// the filtered SVV flux Fa [E + K][12][nn] (after the flux kernel): each face's four components
// of its direction; uses the state's send / receive buffers
hipError_t halo_exchange_svv(const View& v, double* Fa, const HaloArgs& h, hipStream_t st);
// the Jacobian J [E + K][nn] on the faces (once, after the geometry); the state's buffers
hipError_t halo_exchange_jacobian(const View& v, const HaloArgs& h, hipStream_t st);

}  // namespace dg
