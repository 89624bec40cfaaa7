// __global__ wrappers of the element-wise / reduction passes (adjoint step, diagnostics).
#include "evx_launch.hpp"

namespace evx {

__global__ __launch_bounds__(AUX_THREADS) void spec_kernel(SpecArgs a) {
  __shared__ double red[2 * AUX_THREADS];
  spec_body(a, threadIdx.x, blockIdx.x, gridDim.x, red);
}

__global__ __launch_bounds__(AUX_THREADS) void realsum_kernel(RealSumArgs a) {
  __shared__ double red[2 * AUX_THREADS];
  realsum_body(a, threadIdx.x, blockIdx.x, gridDim.x, red);
}

__global__ __launch_bounds__(AUX_THREADS) void final_kernel(FinalArgs a) {
  __shared__ double red[2 * AUX_THREADS];
  final_body(a, threadIdx.x, red);
}

__global__ __launch_bounds__(AUX_THREADS) void combine_kernel(CombineArgs a) {
  combine_body(a, threadIdx.x, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(AUX_THREADS) void finite_kernel(FiniteArgs a) {
  __shared__ int red[AUX_THREADS];
  finite_body<AUX_THREADS>(a, threadIdx.x, blockIdx.x, gridDim.x, red);
}

hipError_t evx_launch_finite(const FiniteArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(finite_kernel, dim3(AUX_BLOCKS), dim3(AUX_THREADS), 0, s, a);
  return hipGetLastError();
}

__global__ __launch_bounds__(AUX_THREADS) void gs_react_kernel(GsReactArgs a) {
  gs_react_body(a, threadIdx.x, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(AUX_THREADS) void gs_update_kernel(GsUpdateArgs a) {
  gs_update_body(a, threadIdx.x, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(VF_THREADS) void vm_fused_kernel(VmStencilArgs a, int lz) {
  __shared__ float lds[VF_LDS];
  vm_fused_body(a, lz, threadIdx.x, blockIdx.x, lds);
}

hipError_t evx_launch_vm_fused(const VmStencilArgs& a, hipStream_t s) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
  }
  const int lz = vm_fused_lz(a, cus);
  const long long ncols = (long long)((a.nx + VF_X - 1) / VF_X) * ((a.ny + VF_Y - 1) / VF_Y);
  const long long grid = ncols * ((a.nz + lz - 1) / lz);
  if (grid >= (1LL << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(vm_fused_kernel, dim3(unsigned(grid)), dim3(VF_THREADS), 0, s, a, lz);
  return hipGetLastError();
}

hipError_t evx_launch_gs_react(const GsReactArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(gs_react_kernel, dim3(AUX_BLOCKS), dim3(AUX_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t evx_launch_gs_update(const GsUpdateArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(gs_update_kernel, dim3(AUX_BLOCKS), dim3(AUX_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t evx_launch_spec(const SpecArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(spec_kernel, dim3(AUX_BLOCKS), dim3(AUX_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t evx_launch_realsum(const RealSumArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(realsum_kernel, dim3(AUX_BLOCKS), dim3(AUX_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t evx_launch_final(const FinalArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(final_kernel, dim3(1), dim3(AUX_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t evx_launch_combine(const CombineArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(combine_kernel, dim3(AUX_BLOCKS), dim3(AUX_THREADS), 0, s, a);
  return hipGetLastError();
}

}  // namespace evx
