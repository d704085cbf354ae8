// kernels_halo.hip -- the halo exchange of a box run as one block of a split domain: pack the
// block's boundary face values into a contiguous send buffer, move them to the receive buffer
// (here a device copy, between GPUs the inter-GPU transfer), unpack them into the ghost
// elements' faces.  One thread per (face, component, face point); the state is FP64 and the face
// viscous fluxes are stored in the stage kernel's type (FP64, or float in FP32-bulk).  With
// spectral vanishing viscosity the filtered flux's face components move too, and the Jacobian's
// face values once after the geometry (the interior penalty reads the neighbour's).
#include <hip/hip_runtime.h>

#include "dg_device.h"
#include "halo.h"

namespace dg {

// the node of face f = 2 d + side at face point q = p + n r
template <int n>
__device__ __forceinline__ int halo_face_node(int f, int q) {
  const int d = f >> 1, side = f & 1;
  return face_node<n>(d, side ? n - 1 : 0, q % n, q / n);
}

template <int N>
__global__ void __launch_bounds__(256) halo_pack_state_kernel(const double* __restrict__ U, const int4* map, int K,
                                                              double* __restrict__ send) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)K * 5 * nf) return;
  const int k = (int)(gid / (5 * nf)), rem = (int)(gid - (long)k * 5 * nf);
  const int c = rem / nf, q = rem - c * nf;
  const int4 m = map[k];
  send[gid] = U[((long)m.x * 5 + c) * nn + halo_face_node<n>(m.y, q)];
}

template <int N>
__global__ void __launch_bounds__(256) halo_unpack_state_kernel(double* __restrict__ U, const int4* map, int K,
                                                                const double* __restrict__ recv) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)K * 5 * nf) return;
  const int k = (int)(gid / (5 * nf)), rem = (int)(gid - (long)k * 5 * nf);
  const int c = rem / nf, q = rem - c * nf;
  const int4 m = map[k];
  U[((long)m.z * 5 + c) * nn + halo_face_node<n>(m.w, q)] = recv[gid];
}

// face viscous fluxes Fvf[element][6][4][nf] of type T: whole face rows move
template <int N, typename T>
__global__ void __launch_bounds__(256) halo_pack_viscous_kernel(const T* __restrict__ Fvf, const int4* map, int K,
                                                                T* __restrict__ send) {
  constexpr int nf = (N + 1) * (N + 1);
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)K * 4 * nf) return;
  const int k = (int)(gid / (4 * nf)), rem = (int)(gid - (long)k * 4 * nf);
  const int4 m = map[k];
  send[gid] = Fvf[((long)m.x * 6 + m.y) * 4 * nf + rem];
}

template <int N, typename T>
__global__ void __launch_bounds__(256) halo_unpack_viscous_kernel(T* __restrict__ Fvf, const int4* map, int K,
                                                                  const T* __restrict__ recv) {
  constexpr int nf = (N + 1) * (N + 1);
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)K * 4 * nf) return;
  const int k = (int)(gid / (4 * nf)), rem = (int)(gid - (long)k * 4 * nf);
  const int4 m = map[k];
  Fvf[((long)m.z * 6 + m.w) * 4 * nf + rem] = recv[gid];
}

// the filtered SVV flux Fa[element][12][nn] (index 4 d + c): on a face of direction d the
// neighbour's four components of that direction at the face nodes
template <int N>
__global__ void __launch_bounds__(256) halo_pack_svv_kernel(const double* __restrict__ Fa, const int4* map, int K,
                                                            double* __restrict__ send) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)K * 4 * nf) return;
  const int k = (int)(gid / (4 * nf)), rem = (int)(gid - (long)k * 4 * nf);
  const int c = rem / nf, q = rem - c * nf;
  const int4 m = map[k];
  send[gid] = Fa[((long)m.x * 12 + 4 * (m.y >> 1) + c) * nn + halo_face_node<n>(m.y, q)];
}

template <int N>
__global__ void __launch_bounds__(256) halo_unpack_svv_kernel(double* __restrict__ Fa, const int4* map, int K,
                                                              const double* __restrict__ recv) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)K * 4 * nf) return;
  const int k = (int)(gid / (4 * nf)), rem = (int)(gid - (long)k * 4 * nf);
  const int c = rem / nf, q = rem - c * nf;
  const int4 m = map[k];
  Fa[((long)m.z * 12 + 4 * (m.w >> 1) + c) * nn + halo_face_node<n>(m.w, q)] = recv[gid];
}

// the Jacobian J[element][nn] on a face (the interior penalty reads the neighbour's)
template <int N>
__global__ void __launch_bounds__(256) halo_pack_jacobian_kernel(const double* __restrict__ J, const int4* map,
                                                                 int K, double* __restrict__ send) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)K * nf) return;
  const int k = (int)(gid / nf), q = (int)(gid - (long)k * nf);
  const int4 m = map[k];
  send[gid] = J[(long)m.x * nn + halo_face_node<n>(m.y, q)];
}

template <int N>
__global__ void __launch_bounds__(256) halo_unpack_jacobian_kernel(double* __restrict__ J, const int4* map, int K,
                                                                   const double* __restrict__ recv) {
  constexpr int n = N + 1, nn = n * n * n, nf = n * n;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)K * nf) return;
  const int k = (int)(gid / nf), q = (int)(gid - (long)k * nf);
  const int4 m = map[k];
  J[(long)m.z * nn + halo_face_node<n>(m.w, q)] = recv[gid];
}

static unsigned blocks_for(long total) { return (unsigned)((total + 255) / 256); }

template <int N>
static hipError_t exchange_state_n(const View& v, int cur, const HaloArgs& h, hipStream_t st) {
  constexpr int nf = (N + 1) * (N + 1);
  const long total = (long)h.K * 5 * nf;
  hipLaunchKernelGGL(halo_pack_state_kernel<N>, dim3(blocks_for(total)), dim3(256), 0, st, v.U[cur], h.map, h.K,
                     h.send);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(h.recv, h.send, sizeof(double) * total, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(halo_unpack_state_kernel<N>, dim3(blocks_for(total)), dim3(256), 0, st, v.U[cur], h.map,
                     h.K, h.recv);
  return hipGetLastError();
}

template <int N, typename T>
static hipError_t exchange_viscous_nt(const View& v, const HaloArgs& h, hipStream_t st) {
  constexpr int nf = (N + 1) * (N + 1);
  const long total = (long)h.K * 4 * nf;
  T* F = reinterpret_cast<T*>(v.Fvf);
  T* send = reinterpret_cast<T*>(h.sendv);
  T* recv = reinterpret_cast<T*>(h.recvv);
  hipLaunchKernelGGL((halo_pack_viscous_kernel<N, T>), dim3(blocks_for(total)), dim3(256), 0, st, F, h.map, h.K,
                     send);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(recv, send, sizeof(T) * total, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((halo_unpack_viscous_kernel<N, T>), dim3(blocks_for(total)), dim3(256), 0, st, F, h.map,
                     h.K, recv);
  return hipGetLastError();
}

template <int N>
static hipError_t exchange_viscous_n(const View& v, const HaloArgs& h, hipStream_t st) {
  return v.fp32 ? exchange_viscous_nt<N, float>(v, h, st) : exchange_viscous_nt<N, double>(v, h, st);
}

template <int N>
static hipError_t exchange_svv_n(double* Fa, const HaloArgs& h, hipStream_t st) {
  constexpr int nf = (N + 1) * (N + 1);
  const long total = (long)h.K * 4 * nf;
  hipLaunchKernelGGL(halo_pack_svv_kernel<N>, dim3(blocks_for(total)), dim3(256), 0, st, Fa, h.map, h.K, h.send);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(h.recv, h.send, sizeof(double) * total, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(halo_unpack_svv_kernel<N>, dim3(blocks_for(total)), dim3(256), 0, st, Fa, h.map, h.K, h.recv);
  return hipGetLastError();
}

template <int N>
static hipError_t exchange_jacobian_n(const View& v, const HaloArgs& h, hipStream_t st) {
  constexpr int nf = (N + 1) * (N + 1);
  const long total = (long)h.K * nf;
  hipLaunchKernelGGL(halo_pack_jacobian_kernel<N>, dim3(blocks_for(total)), dim3(256), 0, st, v.J, h.map, h.K,
                     h.send);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(h.recv, h.send, sizeof(double) * total, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(halo_unpack_jacobian_kernel<N>, dim3(blocks_for(total)), dim3(256), 0, st, v.J, h.map, h.K,
                     h.recv);
  return hipGetLastError();
}

#define DG_HALO_DISPATCH(FN, ...)          \
  switch (v.N) {                           \
    case 1: return FN<1>(__VA_ARGS__);     \
    case 2: return FN<2>(__VA_ARGS__);     \
    case 3: return FN<3>(__VA_ARGS__);     \
    case 4: return FN<4>(__VA_ARGS__);     \
    case 5: return FN<5>(__VA_ARGS__);     \
    case 6: return FN<6>(__VA_ARGS__);     \
    case 7: return FN<7>(__VA_ARGS__);     \
    default: return hipErrorInvalidValue;  \
  }

hipError_t halo_exchange_state(const View& v, int cur, const HaloArgs& h, hipStream_t st) {
  if (v.mixed || v.gauss || !h.map || h.K <= 0 || !h.send || !h.recv) return hipErrorInvalidValue;
  DG_HALO_DISPATCH(exchange_state_n, v, cur, h, st)
}

hipError_t halo_exchange_svv(const View& v, double* Fa, const HaloArgs& h, hipStream_t st) {
  if (v.mixed || v.gauss || !Fa || !h.map || h.K <= 0 || !h.send || !h.recv) return hipErrorInvalidValue;
  DG_HALO_DISPATCH(exchange_svv_n, Fa, h, st)
}

hipError_t halo_exchange_jacobian(const View& v, const HaloArgs& h, hipStream_t st) {
  if (v.mixed || v.gauss || !v.J || !h.map || h.K <= 0 || !h.send || !h.recv) return hipErrorInvalidValue;
  DG_HALO_DISPATCH(exchange_jacobian_n, v, h, st)
}

hipError_t halo_exchange_viscous(const View& v, const HaloArgs& h, hipStream_t st) {
  if (v.mixed || v.gauss || !v.viscous || !v.Fvf || !h.map || h.K <= 0 || !h.sendv || !h.recvv)
    return hipErrorInvalidValue;
  DG_HALO_DISPATCH(exchange_viscous_n, v, h, st)
}

}  // namespace dg
