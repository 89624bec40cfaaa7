// Thin device layer shared by the gfx950 build and the host emulation build used by the CPU
// tests.  The kernels below are written as bodies that take (thread, block, LDS) explicitly and
// call evx_sync() at workgroup barriers; on the GPU those map to threadIdx/blockIdx/__shared__
// and __syncthreads(), in the emulator to one std::thread per lane and a std::barrier.
#pragma once

#include <cstdint>

#ifdef EVX_HOST_EMULATION
#include <barrier>
#include <cmath>

#define EVX_DEV inline
#define EVX_HD inline
#define EVX_RESTRICT

struct float2 {
  float x, y;
};
inline float2 make_float2(float a, float b) { return float2{a, b}; }

namespace evx_emu {
extern thread_local std::barrier<>* block_barrier;
}
inline void evx_sync() { evx_emu::block_barrier->arrive_and_wait(); }
// A value the caller knows to be the same in every lane of a wave (kept in scalar registers).
inline int evx_wave_uniform(int v) { return v; }
inline float evx_rcp(float x) { return 1.0f / x; }

// Buffer resource: a byte range [base, base + nbytes); accesses at or past nbytes read zero and
// drop stores, as the hardware's range check does.
struct evx_buf {
  unsigned char* base;
  unsigned nbytes;
};
inline evx_buf evx_make_buf(const void* base, unsigned nbytes) {
  return evx_buf{static_cast<unsigned char*>(const_cast<void*>(base)), nbytes};
}
inline float2 evx_buf_load2(evx_buf r, unsigned off) {
  if (off >= r.nbytes || r.nbytes - off < 8) return float2{0.f, 0.f};
  float2 v;
  __builtin_memcpy(&v, r.base + off, 8);
  return v;
}
inline void evx_buf_store2(evx_buf r, unsigned off, float2 v) {
  if (off >= r.nbytes || r.nbytes - off < 8) return;
  __builtin_memcpy(r.base + off, &v, 8);
}
inline void evx_buf_store1(evx_buf r, unsigned off, float v) {
  if (off >= r.nbytes || r.nbytes - off < 4) return;
  __builtin_memcpy(r.base + off, &v, 4);
}

#else
#include <hip/hip_runtime.h>

#define EVX_DEV __device__ __forceinline__
#define EVX_HD __host__ __device__ __forceinline__
#define EVX_RESTRICT __restrict__

__device__ __forceinline__ void evx_sync() { __syncthreads(); }
// A value the caller knows to be the same in every lane of a wave (kept in scalar registers).
__device__ __forceinline__ int evx_wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float evx_rcp(float x) { return 1.0f / x; }

// Buffer resource over [base, base + nbytes) (raw, stride 0; word 3 = 0x00020000, the gfx9
// untyped-buffer format).  A uniform base lives in scalar registers and every access adds one
// 32-bit vector offset; offsets at or past nbytes read zero and drop stores (hardware range check).
typedef __amdgpu_buffer_rsrc_t evx_buf;
typedef unsigned evx_u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ evx_buf evx_make_buf(const void* base, unsigned nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(nbytes), 0x00020000);
}
__device__ __forceinline__ float2 evx_buf_load2(evx_buf r, unsigned off) {
  const evx_u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}
__device__ __forceinline__ void evx_buf_store2(evx_buf r, unsigned off, float2 v) {
  evx_u32x2 u;
  u.x = __float_as_uint(v.x);
  u.y = __float_as_uint(v.y);
  __builtin_amdgcn_raw_buffer_store_b64(u, r, off, 0, 0);
}
__device__ __forceinline__ void evx_buf_store1(evx_buf r, unsigned off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, 0);
}
#endif

namespace evx {

EVX_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }

// phi1(s) = (exp(s) - 1) / s for s <= 0 (the exponential stepper's multiplier), branch-free:
// below |s| = 0.5 the Taylor series sum_k s^k / (k + 1)! to k = 7 (truncation below 1.1e-8, and
// phi1(0) = 1 exactly); from there (exp(s) - 1) / s, whose cancellation costs at most 3e-7
// relative since 1 - exp(s) >= 0.39.
EVX_HD float evx_phi1(float s) {
  float p = 1.0f / 40320.0f;
  p = __builtin_fmaf(p, s, 1.0f / 5040.0f);
  p = __builtin_fmaf(p, s, 1.0f / 720.0f);
  p = __builtin_fmaf(p, s, 1.0f / 120.0f);
  p = __builtin_fmaf(p, s, 1.0f / 24.0f);
  p = __builtin_fmaf(p, s, 1.0f / 6.0f);
  p = __builtin_fmaf(p, s, 0.5f);
  p = __builtin_fmaf(p, s, 1.0f);
  const float big = (exp2f(s * 1.44269504088896341f) - 1.0f) / (s < -0.5f ? s : -1.0f);
  return s < -0.5f ? big : p;
}
EVX_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// Explicit fused multiply-adds (the library is built without automatic contraction, so every
// kernel evaluates a complex product with the same roundings).
EVX_HD float2 cmul(float2 a, float2 b) {
  return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
EVX_HD float2 cmulc(float2 a, float2 b) {
  return make_float2(__builtin_fmaf(a.x, b.x, a.y * b.y), __builtin_fmaf(a.y, b.x, -(a.x * b.y)));
}
EVX_HD float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
EVX_HD float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by +i (dir=+1) or -i (dir=-1)
template <int SGN>
EVX_HD float2 cmul_i(float2 a) {
  return SGN > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

}  // namespace evx
