// kernels_ext.hip -- the stage kernels of the extended flux families (FP64): 1 the
// kinetic-energy-preserving volume fluxes, 2 the extended surface fluxes (entropy stable,
// Ismail-Roe, matrix dissipation, low-dissipation Roe), 3 both.  Same kernel bodies as the common
// family (stage_kernel.h); compiled in a translation unit of their own.
#include <hip/hip_runtime.h>

#include "dg_device.h"
#include "stage_kernel.h"

namespace dg {

template <int N>
static hipError_t stage_ext_n(const View& v, int fx, int cur, double dt, double a, double b, int mode,
                              hipStream_t st) {
  switch (fx) {
    case 1: return stage_ntx<N, double, 1>(v, cur, dt, a, b, mode, st);
    case 2: return stage_ntx<N, double, 2>(v, cur, dt, a, b, mode, st);
    case 3: return stage_ntx<N, double, 3>(v, cur, dt, a, b, mode, st);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
static hipError_t stage_batch_ext_n(const BatchArgs& B, bool visc, int fx, double a, double b, int mode,
                                    hipStream_t st) {
  switch (fx) {
    case 1: return stage_batch_nt<N, double, 1>(B, visc, a, b, mode, st);
    case 2: return stage_batch_nt<N, double, 2>(B, visc, a, b, mode, st);
    case 3: return stage_batch_nt<N, double, 3>(B, visc, a, b, mode, st);
    default: return hipErrorInvalidValue;
  }
}

#define DG_EXT_DISPATCH(NV, FN, ...)                  \
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

hipError_t launch_stage_ext(const View& v, int fx, int cur, double dt, double rkA, double rkB, int mode,
                            hipStream_t st) {
  DG_EXT_DISPATCH(v.N, stage_ext_n, v, fx, cur, dt, rkA, rkB, mode, st)
}

hipError_t launch_stage_batch_ext(const BatchArgs& B, int N, bool visc, int fx, double rkA, double rkB, int mode,
                                  hipStream_t st) {
  DG_EXT_DISPATCH(N, stage_batch_ext_n, B, visc, fx, rkA, rkB, mode, st)
}

}  // namespace dg
