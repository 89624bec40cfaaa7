// __global__ wrappers of the pass bodies for one transform length.  This file is compiled once
// per supported length (EVX_INST_N) so the instantiations build in parallel; each object exports
// evx_launch_col_<N> and evx_launch_row_<N> (and their batched forms evx_launch_colb_<N>,
// evx_launch_rowb_<N>).
#include "evx_launch.hpp"

#ifndef EVX_INST_N
#error "compile with -DEVX_INST_N=<transform length>"
#endif

namespace evx {

template <int N, int BC, int MODE>
__global__ __launch_bounds__(ColCfg<N>::THREADS) void col_kernel(ColArgs a) {
  __shared__ float2 lds[ColCfg<N>::LDS];
  colpass_body<N, BC, MODE>(a, threadIdx.x, blockIdx.x, gridDim.x, lds);
}

// the same passes over a batch of buffer pairs (grid.y = pair)
template <int N, int BC, int MODE>
__global__ __launch_bounds__(ColCfg<N>::THREADS) void col_kernel_batch(ColArgs a, PassBatch p) {
  __shared__ float2 lds[ColCfg<N>::LDS];
  bind_batch(a, p, blockIdx.y);
  colpass_body<N, BC, MODE>(a, threadIdx.x, blockIdx.x, gridDim.x, lds);
}

template <int NH, int BC>
constexpr int row_threads() {
  return RowCfg<NH, BC>::THREADS;
}

template <int NH, int BC, int MODE>
__global__ __launch_bounds__((row_threads<NH, BC>())) void row_kernel(RowArgs a) {
  __shared__ float2 lds[RowCfg<NH, BC>::LDS];
  rowpass_body<NH, BC, MODE>(a, threadIdx.x, blockIdx.x, gridDim.x, lds);
}

template <int NH, int BC, int MODE>
__global__ __launch_bounds__((row_threads<NH, BC>())) void row_kernel_batch(RowArgs a, PassBatch p) {
  __shared__ float2 lds[RowCfg<NH, BC>::LDS];
  bind_batch(a, MODE == ROW_INV, p, blockIdx.y);
  rowpass_body<NH, BC, MODE>(a, threadIdx.x, blockIdx.x, gridDim.x, lds);
}

// One workgroup per z plane (small periodic grids; see planepass_body).
template <int NY, int NH>
constexpr int plane_threads() {
  return PlaneCfg<NY, NH>::THREADS;
}

template <int NY, int NH>
__global__ __launch_bounds__((plane_threads<NY, NH>())) void plane_kernel(PlaneArgs a) {
  __shared__ float2 lds[PlaneCfg<NY, NH>::LDS];
  planepass_body<NY, NH>(a, threadIdx.x, blockIdx.x, lds);
}

template <int NY>
static hipError_t plane_go(const PlaneArgs& a, hipStream_t s) {
  using C = PlaneCfg<NY, NY / 2>;
  if (a.nz <= 0) return hipSuccess;
  if (a.sg.ny != NY || a.ngx != (NY / 2 + 1 + 7) / 8) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((plane_kernel<NY, NY / 2>), dim3(unsigned(a.nz)), dim3(C::THREADS), 0, s, a);
  return hipGetLastError();
}

template <int N, int BC, int MODE>
static hipError_t col_go(const ColArgs& a, hipStream_t s) {
  using C = ColCfg<N>;
  const long long nblk = (a.nseq + C::B - 1) / C::B;
  if (nblk <= 0) return hipSuccess;
  // 32-bit sequence numbers and lane byte offsets (ColTile)
  const long long lane_bytes = col_lane_bytes<N>(a);
  if (nblk > 0x7fffffffLL || a.nseq > 0x7fffffffLL || lane_bytes >= (long long)kDeadLane)
    return hipErrorInvalidConfiguration;
  ColArgs b = a;
  b.lane_bytes = unsigned(lane_bytes);
  hipLaunchKernelGGL((col_kernel<N, BC, MODE>), dim3(unsigned(nblk)), dim3(C::THREADS), 0, s, b);
  return hipGetLastError();
}

template <int NH, int BC, int MODE>
static hipError_t row_go(const RowArgs& a, hipStream_t s) {
  using C = RowCfg<NH, BC>;
  const long long nblk = (a.nrows + C::ROWS - 1) / C::ROWS;
  if (nblk <= 0) return hipSuccess;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((row_kernel<NH, BC, MODE>), dim3(unsigned(nblk)), dim3(C::THREADS), 0, s, a);
  return hipGetLastError();
}

// Batched launches check every pair's buffers like the single ones (the geometry is shared).
template <int N, int BC, int MODE>
static hipError_t col_go_batch(const ColArgs& a, const PassBatch& p, hipStream_t s) {
  using C = ColCfg<N>;
  const long long nblk = (a.nseq + C::B - 1) / C::B;
  if (nblk <= 0) return hipSuccess;
  if (p.n < 1 || p.n > kMaxBatch) return hipErrorInvalidValue;
  const long long lane_bytes = col_lane_bytes<N>(a);
  if (nblk > 0x7fffffffLL || a.nseq > 0x7fffffffLL || lane_bytes >= (long long)kDeadLane)
    return hipErrorInvalidConfiguration;
  ColArgs b = a;
  b.lane_bytes = unsigned(lane_bytes);
  hipLaunchKernelGGL((col_kernel_batch<N, BC, MODE>), dim3(unsigned(nblk), unsigned(p.n)),
                     dim3(C::THREADS), 0, s, b, p);
  return hipGetLastError();
}

template <int NH, int BC, int MODE>
static hipError_t row_go_batch(const RowArgs& a, const PassBatch& p, hipStream_t s) {
  using C = RowCfg<NH, BC>;
  const long long nblk = (a.nrows + C::ROWS - 1) / C::ROWS;
  if (nblk <= 0) return hipSuccess;
  if (p.n < 1 || p.n > kMaxBatch) return hipErrorInvalidValue;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((row_kernel_batch<NH, BC, MODE>), dim3(unsigned(nblk), unsigned(p.n)),
                     dim3(C::THREADS), 0, s, a, p);
  return hipGetLastError();
}

template <int N, int BC>
static hipError_t col_mode(int mode, const ColArgs& a, hipStream_t s) {
  switch (mode) {
    case COL_FWD: return col_go<N, BC, COL_FWD>(a, s);
    case COL_INV: return col_go<N, BC, COL_INV>(a, s);
    case COL_Z_INIT: return col_go<N, BC, COL_Z_INIT>(a, s);
    case COL_Z_UPDATE: return col_go<N, BC, COL_Z_UPDATE>(a, s);
    case COL_Z_INV_STATE: return col_go<N, BC, COL_Z_INV_STATE>(a, s);
    case COL_Z_ETD: return col_go<N, BC, COL_Z_ETD>(a, s);
    case COL_Z_AC: return col_go<N, BC, COL_Z_AC>(a, s);
    case COL_Z_AC_ETD: return col_go<N, BC, COL_Z_AC_ETD>(a, s);
    case COL_Z_VM: return col_go<N, BC, COL_Z_VM>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NH, int BC>
static hipError_t row_mode(int mode, const RowArgs& a, hipStream_t s) {
  switch (mode) {
    case ROW_FUSED: return row_go<NH, BC, ROW_FUSED>(a, s);
    case ROW_FWD: return row_go<NH, BC, ROW_FWD>(a, s);
    case ROW_INV: return row_go<NH, BC, ROW_INV>(a, s);
    case ROW_INV_ADD: return row_go<NH, BC, ROW_INV_ADD>(a, s);
    case ROW_FWD_FP: return row_go<NH, BC, ROW_FWD_FP>(a, s);
    case ROW_FUSED_REC: return row_go<NH, BC, ROW_FUSED_REC>(a, s);
    case ROW_FUSED_POLY: return row_go<NH, BC, ROW_FUSED_POLY>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int BC>
static hipError_t col_mode_batch(int mode, const ColArgs& a, const PassBatch& p, hipStream_t s) {
  switch (mode) {
    case COL_FWD: return col_go_batch<N, BC, COL_FWD>(a, p, s);
    case COL_INV: return col_go_batch<N, BC, COL_INV>(a, p, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NH, int BC>
static hipError_t row_mode_batch(int mode, const RowArgs& a, const PassBatch& p, hipStream_t s) {
  switch (mode) {
    case ROW_FWD: return row_go_batch<NH, BC, ROW_FWD>(a, p, s);
    case ROW_INV: return row_go_batch<NH, BC, ROW_INV>(a, p, s);
    case ROW_FWD_FP: return row_go_batch<NH, BC, ROW_FWD_FP>(a, p, s);
    default: return hipErrorInvalidValue;
  }
}

#define EVX_PASTE2(a, b) a##b
#define EVX_PASTE(a, b) EVX_PASTE2(a, b)

hipError_t EVX_PASTE(evx_launch_col_, EVX_INST_N)(int bc, int mode, const ColArgs& a,
                                                  hipStream_t s) {
  return bc == BC_PERIODIC ? col_mode<EVX_INST_N, BC_PERIODIC>(mode, a, s)
                           : col_mode<EVX_INST_N, BC_ZERO_FLUX>(mode, a, s);
}

hipError_t EVX_PASTE(evx_launch_row_, EVX_INST_N)(int bc, int mode, const RowArgs& a,
                                                  hipStream_t s) {
  return bc == BC_PERIODIC ? row_mode<EVX_INST_N, BC_PERIODIC>(mode, a, s)
                           : row_mode<EVX_INST_N, BC_ZERO_FLUX>(mode, a, s);
}

hipError_t EVX_PASTE(evx_launch_colb_, EVX_INST_N)(int bc, int mode, const ColArgs& a,
                                                   const PassBatch& p, hipStream_t s) {
  return bc == BC_PERIODIC ? col_mode_batch<EVX_INST_N, BC_PERIODIC>(mode, a, p, s)
                           : col_mode_batch<EVX_INST_N, BC_ZERO_FLUX>(mode, a, p, s);
}

hipError_t EVX_PASTE(evx_launch_rowb_, EVX_INST_N)(int bc, int mode, const RowArgs& a,
                                                   const PassBatch& p, hipStream_t s) {
  return bc == BC_PERIODIC ? row_mode_batch<EVX_INST_N, BC_PERIODIC>(mode, a, p, s)
                           : row_mode_batch<EVX_INST_N, BC_ZERO_FLUX>(mode, a, p, s);
}

#if EVX_INST_N == 32 || EVX_INST_N == 64
hipError_t EVX_PASTE(evx_launch_plane_, EVX_INST_N)(const PlaneArgs& a, hipStream_t s) {
  return plane_go<EVX_INST_N>(a, s);
}
#endif

}  // namespace evx
