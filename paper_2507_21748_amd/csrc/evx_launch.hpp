// Declarations of the per-length launchers and the HIP launcher object used by the schedule.
#pragma once

#include <hip/hip_runtime.h>

#include "evx_adjoint.hpp"
#include "evx_schedule.hpp"

namespace evx {

#define EVX_DECL(N)                                                                     \
  hipError_t evx_launch_col_##N(int bc, int mode, const ColArgs& a, hipStream_t s);      \
  hipError_t evx_launch_row_##N(int bc, int mode, const RowArgs& a, hipStream_t s);      \
  hipError_t evx_launch_colb_##N(int bc, int mode, const ColArgs& a, const PassBatch& p, \
                                 hipStream_t s);                                         \
  hipError_t evx_launch_rowb_##N(int bc, int mode, const RowArgs& a, const PassBatch& p, \
                                 hipStream_t s);
EVX_FOR_EACH_N(EVX_DECL)
#undef EVX_DECL

hipError_t evx_launch_plane_32(const PlaneArgs& a, hipStream_t s);
hipError_t evx_launch_plane_64(const PlaneArgs& a, hipStream_t s);
hipError_t evx_launch_spec(const SpecArgs& a, hipStream_t s);
hipError_t evx_launch_realsum(const RealSumArgs& a, hipStream_t s);
hipError_t evx_launch_final(const FinalArgs& a, hipStream_t s);
hipError_t evx_launch_combine(const CombineArgs& a, hipStream_t s);
hipError_t evx_launch_gs_react(const GsReactArgs& a, hipStream_t s);
hipError_t evx_launch_finite(const FiniteArgs& a, hipStream_t s);
hipError_t evx_launch_gs_update(const GsUpdateArgs& a, hipStream_t s);
hipError_t evx_launch_vm_fused(const VmStencilArgs& a, hipStream_t s);

// Records the first launch error; the schedule keeps enqueuing nothing after one.
struct HipLauncher {
  hipStream_t stream = nullptr;
  hipError_t err = hipSuccess;
  bool bad_len = false;

  void col(int n, int bc, int mode, const ColArgs& a) {
    if (err != hipSuccess || bad_len) return;
    switch (n) {
#define EVX_CASE(N) \
  case N: err = evx_launch_col_##N(bc, mode, a, stream); return;
      EVX_FOR_EACH_N(EVX_CASE)
#undef EVX_CASE
      default: bad_len = true;
    }
  }
  void col_batch(int n, int bc, int mode, const ColArgs& a, const PassBatch& p) {
    if (err != hipSuccess || bad_len) return;
    switch (n) {
#define EVX_CASE(N) \
  case N: err = evx_launch_colb_##N(bc, mode, a, p, stream); return;
      EVX_FOR_EACH_N(EVX_CASE)
#undef EVX_CASE
      default: bad_len = true;
    }
  }
  void row_batch(int n, int bc, int mode, const RowArgs& a, const PassBatch& p) {
    if (err != hipSuccess || bad_len) return;
    switch (n) {
#define EVX_CASE(N) \
  case N: err = evx_launch_rowb_##N(bc, mode, a, p, stream); return;
      EVX_FOR_EACH_N(EVX_CASE)
#undef EVX_CASE
      default: bad_len = true;
    }
  }
  void plane(int ny, const PlaneArgs& a) {
    if (err != hipSuccess || bad_len) return;
    if (ny == 32) err = evx_launch_plane_32(a, stream);
    else if (ny == 64) err = evx_launch_plane_64(a, stream);
    else bad_len = true;
  }
  void spec(const SpecArgs& a) {
    if (err == hipSuccess && !bad_len) err = evx_launch_spec(a, stream);
  }
  void realsum(const RealSumArgs& a) {
    if (err == hipSuccess && !bad_len) err = evx_launch_realsum(a, stream);
  }
  void final(const FinalArgs& a) {
    if (err == hipSuccess && !bad_len) err = evx_launch_final(a, stream);
  }
  void combine(const CombineArgs& a) {
    if (err == hipSuccess && !bad_len) err = evx_launch_combine(a, stream);
  }
  void gs_react(const GsReactArgs& a) {
    if (err == hipSuccess && !bad_len) err = evx_launch_gs_react(a, stream);
  }
  void gs_update(const GsUpdateArgs& a) {
    if (err == hipSuccess && !bad_len) err = evx_launch_gs_update(a, stream);
  }
  void vm_fused(const VmStencilArgs& a) {
    if (err == hipSuccess && !bad_len) err = evx_launch_vm_fused(a, stream);
  }
  void row(int n, int bc, int mode, const RowArgs& a) {
    if (err != hipSuccess || bad_len) return;
    switch (n) {
#define EVX_CASE(N) \
  case N: err = evx_launch_row_##N(bc, mode, a, stream); return;
      EVX_FOR_EACH_N(EVX_CASE)
#undef EVX_CASE
      default: bad_len = true;
    }
  }
};

}  // namespace evx
