// Learned coarse stepper: periodic residual 3D CNN c_out = c + net(c), 3x3x3 kernels, channels
// 1 -> 32 -> 32 -> 32 -> 1, GELU between layers; BF16 weights and activations with FP32
// accumulation; trained with Adam on FP32 master weights.
//
// Layout: activations are channels-last BF16 [V][C] (x fastest over the grid), weights W[27][Cout]
// [Cin] with offset index d = 9 (dz+1) + 3 (dy+1) + (dx+1); conv(x)[v,o] = b[o] +
// sum_{d,i} W[d,o,i] x[(v+d) mod grid, i] (cross-correlation, circular padding).
//
// Kernels:
//   conv32_mfma   32 -> 32 layers as an implicit GEMM on v_mfma_f32_16x16x32_bf16: one MFMA per
//                 (16 voxels, 16 output channels, one offset d, all 32 input channels).  A block
//                 stages a 6x10x18-voxel halo tile (69 KB) and the layer's weights (55 KB) in LDS
//                 and computes a 4x8x16 output tile with 8 waves (4 rows of 16 voxels each).
//   conv_in_mfma  1 -> 32 layer (and the last layer's backward data) as a GEMM over the 27
//                 offsets: D[o][v] = sum_d W[d][o] x[v + d]; GELU by a BF16 table.
//   conv_out_mfma 32 -> 1 layer: P[u][d] = sum_i W[d][i] a[u][i] on MFMA, then
//                 out[v] = c[v] + sum_d P[v + d][d] + b; blocks own 16x16 columns and march up z,
//                 computing each halo plane's P once.
//   wgrad32_mfma  dW[d,o,i] = sum_v gz[v,o] x[v+d,i] and db of the 32 -> 32 layers as MFMA GEMMs
//   wgrad1_mfma   over voxels; wgrad1_mfma the same for the 1 -> 32 and 32 -> 1 layers; per-block
//                 partial sums with a fixed-order reduction (bit-reproducible).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <type_traits>

#include "../../include/evx.h"

namespace {

typedef unsigned short bf16_t;
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int CH = 32;
constexpr int NLAYER = 4;

__host__ __device__ constexpr int cin_of(int l) { return l == 0 ? 1 : CH; }
__host__ __device__ constexpr int cout_of(int l) { return l == NLAYER - 1 ? 1 : CH; }
__host__ __device__ constexpr long long layer_w(int l) { return 27LL * cin_of(l) * cout_of(l); }
// offset of layer l's weights in the flat parameter vector (each layer: W then b)
__host__ __device__ constexpr long long layer_off(int l) {
  long long o = 0;
  for (int i = 0; i < l; ++i) o += layer_w(i) + cout_of(i);
  return o;
}
// offset of layer l's weights in the packed bf16 weight arrays (no biases)
__host__ __device__ constexpr long long w_off(int l) {
  long long o = 0;
  for (int i = 0; i < l; ++i) o += layer_w(i);
  return o;
}
constexpr long long NPARAM = layer_off(NLAYER);  // 57121
static_assert(NPARAM == 57121, "parameter count");

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// FP32 -> BF16, round to nearest even: gfx950's conversion instruction (two values at once)
__device__ __forceinline__ unsigned f2bf2(float lo, float hi) {
  const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(unsigned, v);
}
__device__ __forceinline__ bf16_t f2bf(float f) { return bf16_t(f2bf2(f, 0.f)); }
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(unsigned(h) << 16); }

// GELU(z) = z Phi(z) with Phi(z) = erfc(-z / sqrt 2) / 2, evaluated through erfc so that the
// negative tail keeps its relative accuracy (1 + erf would cancel).  erfc(u), u >= 0, uses the
// Chebyshev-fitted form published in Numerical Recipes (routine erfcc):
//   erfc(u) ~= t exp(-u^2 + P(t)),  t = 1 / (1 + u / 2),
// with relative error below 1.2e-7 for every u >= 0 -- far below the BF16 resolution (2^-8) of
// the stored activations -- at a fraction of the cost of a library erfc.
__device__ __forceinline__ float exp_fast(float x) {
  return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
}
__device__ __forceinline__ float erfc_poly(float t) {
  float p = 0.17087277f;
  p = __builtin_fmaf(p, t, -0.82215223f);
  p = __builtin_fmaf(p, t, 1.48851587f);
  p = __builtin_fmaf(p, t, -1.13520398f);
  p = __builtin_fmaf(p, t, 0.27886807f);
  p = __builtin_fmaf(p, t, -0.18628806f);
  p = __builtin_fmaf(p, t, 0.09678418f);
  p = __builtin_fmaf(p, t, 0.37409196f);
  p = __builtin_fmaf(p, t, 1.00002368f);
  return __builtin_fmaf(p, t, -1.26551223f);
}
// Phi(z) and, through *g, exp(-z^2 / 2) for the derivative
__device__ __forceinline__ float phi_cdf(float z, float* g = nullptr) {
  const float u = __builtin_fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.5f, u, 1.0f));
  const float u2 = u * u;
  float e;  // erfc(u)
  if (g) {
    *g = exp_fast(-u2);
    e = t * *g * exp_fast(erfc_poly(t));
  } else {
    e = t * exp_fast(erfc_poly(t) - u2);
  }
  return z > 0.f ? 1.0f - 0.5f * e : 0.5f * e;
}
__device__ __forceinline__ float gelu(float z) { return z * phi_cdf(z); }
__device__ __forceinline__ float gelu_prime(float z) {
  float g;
  const float p = phi_cdf(z, &g);
  return p + z * 0.39894228040143268f * g;
}

// GELU of a BF16 pre-activation, rounded to BF16, by table.  For |z| in [2^-16, 8) (19 binades x
// 128 mantissas) the table holds bf16(gelu(z)) computed once by gelu() above, so those results
// are identical to evaluating it.  It has one row per sign of GT_ROW entries: entry r < GT_HALF is
// the binade-major position of |z| above 2^-16 (|z|'s bits minus those of 2^-16), and entry GT_HALF
// is a sentinel (0xFFFF, which no finite result has) that lookups of out-of-range values land on.
// Below 2^-16, gelu(z) = z (1/2 + z / sqrt(2 pi)) to a relative 1e-5, far below half a BF16 ulp;
// from 8 up, gelu(z) rounds to z; from -8 down the full evaluation runs.
constexpr int GT_EMIN = 127 - 16, GT_NEXP = 19, GT_HALF = GT_NEXP * 128, GT_ROW = GT_HALF + 1;
constexpr int GT_N = (2 * GT_ROW + 7) / 8 * 8;  // staged in 16-byte chunks
constexpr unsigned GT_SENTINEL = 0xFFFFu;
__device__ __forceinline__ unsigned gelu_table_entry(int idx) {
  const int sign = idx / GT_ROW, rel = idx % GT_ROW;
  if (sign > 1) return 0u;  // padding
  if (rel == GT_HALF) return GT_SENTINEL;
  return bf16_t((sign << 15) | ((GT_EMIN << 7) + rel));
}
// The slow path of an out-of-table pre-activation.
__device__ __forceinline__ bf16_t gelu_bf16_outside(bf16_t zb) {
  const unsigned mag = zb & 0x7FFFu;
  const float z = bf2f(zb);
  if (mag < unsigned(GT_EMIN << 7)) return f2bf(z * __builtin_fmaf(0.39894228040143268f, z, 0.5f));
  return (zb >> 15) ? f2bf(gelu(z)) : zb;  // |z| >= 8, inf, NaN
}
__device__ __forceinline__ bf16_t gelu_bf16(bf16_t zb, const bf16_t* tab) {
  const unsigned rel = (zb & 0x7FFFu) - unsigned(GT_EMIN << 7);  // wraps below 2^-16
  if (rel < unsigned(GT_HALF)) return tab[(zb >> 15) * GT_ROW + rel];
  return gelu_bf16_outside(zb);
}

// Two pre-activations packed in a dword (low half first) at once, on packed 16-bit integer
// operations: both table positions are formed together, out-of-range ones clamped to the
// sentinel, and no branch separates the reads, so an epilogue issues all of them before waiting
// for any.  *worst collects the largest clamped position seen; if it reached GT_HALF in either
// half, gelu2_fix redoes the sentinel results (rare: |z| < 2^-16 or |z| >= 8).
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned gelu2_lookup(unsigned zz, const bf16_t* tab, u16x2* worst) {
  const u16x2 z = __builtin_bit_cast(u16x2, zz);
  const u16x2 rel = __builtin_elementwise_min(
      (u16x2)(z & (u16x2)0x7FFF) - (u16x2)(GT_EMIN << 7), (u16x2)GT_HALF);
  *worst = __builtin_elementwise_max(*worst, rel);
  const u16x2 idx = (u16x2)(z >> (u16x2)15) * (u16x2)GT_ROW + rel;
  return unsigned(tab[idx.x]) | (unsigned(tab[idx.y]) << 16);
}
__device__ __forceinline__ bool gelu2_any_outside(u16x2 worst) {
  return worst.x == GT_HALF || worst.y == GT_HALF;
}
__device__ __forceinline__ unsigned gelu2_fix(unsigned zz, unsigned r) {
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    if (((r >> (16 * e)) & 0xFFFFu) == GT_SENTINEL) {
      const unsigned v = gelu_bf16_outside(bf16_t(zz >> (16 * e)));
      r = (r & ~(0xFFFFu << (16 * e))) | (v << (16 * e));
    }
  }
  return r;
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
// true modulo: tiles past a grid edge can reach more than one period away on small grids
__device__ __forceinline__ int pmod(int v, int n) {
  const int r = v % n;
  return r < 0 ? r + n : r;
}
__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }


// epilogues
enum : int {
  EPI_GELU_Z = 0,   // store zb = bf16(acc + b) and a = bf16(gelu(zb))
  EPI_GELU = 1,     // store a only (inference)
  EPI_DGELU = 2,    // store bf16(acc * gelu'(zprev))   (backward data, no bias)
  EPI_RESID = 3     // out = c + (acc + b)  (last layer, FP32)
};

struct ConvArgs {
  const void* in;        // bf16 [V][Cin] or float [V] (Cin == 1, FP32 input)
  const bf16_t* w;       // bf16 [27][Cout][Cin]
  const float* bias;     // [Cout] (fp32 master), null for EPI_DGELU
  bf16_t* z_out;         // EPI_GELU_Z
  bf16_t* a_out;         // EPI_GELU_Z, EPI_GELU, EPI_DGELU
  const bf16_t* zprev;   // EPI_DGELU: pre-activation of the layer below [V][Cout]
  const float* c;        // EPI_RESID: network input (fp32)
  float* out;            // EPI_RESID
  const bf16_t* gtab;    // GELU table (GT_N entries), for the GELU epilogues
  int nx, ny, nz;
};

// ----------------------------------------------------------------------------- MFMA 32 -> 32
// Output channels to MFMA rows: the two 16-row MFMAs of a layer (h = 0, 1) take channel
// 8 (R / 4) + 4 h + R % 4 as row R, so the D fragments of a lane of lane group lg hold the 8
// consecutive channels 8 lg .. 8 lg + 7 of its voxel (4 from each MFMA) and leave as one 16-byte
// store, full 64-byte voxel rows per 16 lanes.
__device__ __forceinline__ int out_channel(int h, int row) {
  return 8 * (row >> 2) + 4 * h + (row & 3);
}
// Backward-data epilogue of one voxel v: channels 8 lg .. 8 lg + 7 (acc[h][r] is channel
// 8 lg + 4 h + r) become bf16(acc * gelu'(zprev)), zprev read and the result written 16 bytes at
// a time.
__device__ __forceinline__ void store_dgelu(const ConvArgs& a, long long v, int lg,
                                            const f32x4 (&acc)[2]) {
  const uint4 zp = *reinterpret_cast<const uint4*>(a.zprev + v * CH + 8 * lg);
  const unsigned zz[2][2] = {{zp.x, zp.y}, {zp.z, zp.w}};
  unsigned ow[2][2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const bf16_t lo = f2bf(acc[h][2 * k] * gelu_prime(__uint_as_float(zz[h][k] << 16)));
      const bf16_t hi = f2bf(acc[h][2 * k + 1] * gelu_prime(__uint_as_float(zz[h][k] & 0xFFFF0000u)));
      ow[h][k] = unsigned(lo) | (unsigned(hi) << 16);
    }
  *reinterpret_cast<uint4*>(a.a_out + v * CH + 8 * lg) = make_uint4(ow[0][0], ow[0][1], ow[1][0], ow[1][1]);
}
constexpr int TX = 16, TY = 8, TZ = 4;
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
constexpr int HALO_VOX = HX * HY * HZ;           // 1080
constexpr int MFMA_THREADS = 512;                // 8 waves
// output rows (y within one z plane) per wave.  4 waves of 8 rows (each weight fragment read
// from LDS feeds 8 MFMAs instead of 4) measured 30% slower: one wave per SIMD, and its
// accumulators and prefetch no longer fit the architected registers.
constexpr int WROWS = TY * TZ / (MFMA_THREADS / 64);
static_assert(TY % WROWS == 0, "a wave's rows lie in one z plane");
constexpr int HALO_CHUNKS = HALO_VOX * 4;        // 16-byte chunks (64 B per voxel)
constexpr int W_CHUNKS = 27 * CH * CH * 2 / 16;  // 3456

// Halo staging by rows: lane t < ROWS_PER_IT * ROW_CHUNKS moves chunk t % ROW_CHUNKS (voxel hx =
// its index / 4, 16-byte part its index % 4) of halo rows t / ROW_CHUNKS + ROWS_PER_IT k (row =
// hz HY + hy), so the x coordinate is wrapped once per tile and each chunk costs one row's
// arithmetic.
constexpr int ROW_CHUNKS = HX * 4;                        // 72
constexpr int ROWS_PER_IT = MFMA_THREADS / ROW_CHUNKS;
constexpr int HALO_ROWS = HY * HZ;                        // 60
constexpr int HALO_IT = (HALO_ROWS + ROWS_PER_IT - 1) / ROWS_PER_IT;
// LDS layouts are chunk-major (a chunk = 8 channels, 16 bytes): halo chunk c of voxel v at
// c * HALO_CS + v, weight chunk c of output row o (= 16 h + li) for offset d at
// ((2 d + h) * 4 + c) * 16 + li.  The 8 lanes a 16-byte LDS read serves together (consecutive
// voxels or rows, one chunk) then read 128 contiguous bytes; with voxels 64 bytes apart they fell
// in two bank groups (a 4-way conflict on every fragment read).  The 2-voxel pad spreads the four
// chunks of one voxel over distinct banks when the halo is stored.
constexpr int HALO_CS = HALO_VOX + 2;

// Persistent: each block stages the weights once and walks tiles blockIdx.x, +gridDim.x, ...;
// the next tile's halo is loaded into registers while the current one is computed.
template <int EPI>
__global__ __launch_bounds__(MFMA_THREADS) void conv32_mfma(ConvArgs a, int ntiles) {
  static_assert(EPI == EPI_GELU || EPI == EPI_GELU_Z || EPI == EPI_DGELU, "epilogue kind");
  __shared__ __attribute__((aligned(16))) bf16_t s_in[HALO_CS * CH];
  __shared__ __attribute__((aligned(16))) bf16_t s_w[27 * CH * CH];
  __shared__ __attribute__((aligned(16))) bf16_t s_gt[GT_N];
  const int tid = threadIdx.x;
  if (EPI != EPI_DGELU)
    for (int i = tid; i < GT_N / 8; i += MFMA_THREADS)
      reinterpret_cast<u32x4*>(s_gt)[i] = reinterpret_cast<const u32x4*>(a.gtab)[i];
  const int ntx = (a.nx + TX - 1) / TX, nty = (a.ny + TY - 1) / TY;
  const u32x4* gin = static_cast<const u32x4*>(a.in);
  u32x4* sin4 = reinterpret_cast<u32x4*>(s_in);
  {
    const u32x4* gw = reinterpret_cast<const u32x4*>(a.w);
    u32x4* sw4 = reinterpret_cast<u32x4*>(s_w);
    for (int i0 = tid; i0 < W_CHUNKS; i0 += 4 * MFMA_THREADS) {
      u32x4 r[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = i0 + k * MFMA_THREADS;
        if (i < W_CHUNKS) r[k] = gw[i];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = i0 + k * MFMA_THREADS;
        // output channel o is row ((o / 8) * 4 + o % 4) of MFMA (o / 4) % 2
        const int row = i >> 2, d = row >> 5, o = row & 31;
        const int h = (o >> 2) & 1, mr = ((o >> 3) << 2) | (o & 3);
        if (i < W_CHUNKS) sw4[((2 * d + h) * 4 + (i & 3)) * 16 + mr] = r[k];
      }
    }
  }
  u32x4 pre[HALO_IT];
  const bool narrow = a.nx < HX || a.ny < HY || a.nz < HZ;  // uniform
  const int f_col = tid % ROW_CHUNKS, f_row0 = tid / ROW_CHUNKS;
  const int f_hx = f_col >> 2, f_part = f_col & 3;
  auto row_ok = [&](int k) {
    return f_row0 < ROWS_PER_IT && f_row0 + ROWS_PER_IT * k < HALO_ROWS;
  };
  auto fetch = [&](int tl) {
    const int fx0 = (tl % ntx) * TX;
    const int rest = tl / ntx;
    const int fy0 = (rest % nty) * TY, fz0 = (rest / nty) * TZ;
    // a partial tile reaches up to TX (TY, TZ) points past the grid edge: on grids at least a
    // tile plus its halo wide one conditional add or subtract wraps it, else a true modulo
    const int gx0 = fx0 + f_hx - 1;
    const int gx = narrow ? pmod(gx0, a.nx) : wrap(gx0, a.nx);
#pragma unroll
    for (int k = 0; k < HALO_IT; ++k) {
      // lanes without a row of their own load row 0 (always valid) and store nothing
      const int r = row_ok(k) ? f_row0 + ROWS_PER_IT * k : 0;
      const int hy = r % HY, hz = r / HY;
      int gy = fy0 + hy - 1, gz = fz0 + hz - 1;
      if (narrow) {
        gy = pmod(gy, a.ny);
        gz = pmod(gz, a.nz);
      } else {
        gy = wrap(gy, a.ny);
        gz = wrap(gz, a.nz);
      }
      pre[k] = gin[(((long long)gz * a.ny + gy) * a.nx + gx) * 4 + f_part];
    }
  };
  int tile = blockIdx.x;
  if (tile < ntiles) fetch(tile);

  const int wave = tid >> 6, lane = tid & 63;
  const int zl = wave * WROWS / TY;  // output z within the tile
  const int yb = wave * WROWS % TY;  // first of the wave's WROWS output rows
  const int li = lane & 15, lg = lane >> 4;
  float bias[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      bias[h][r] = EPI != EPI_DGELU ? a.bias[out_channel(h, 4 * lg + r)] : 0.f;

  for (; tile < ntiles; tile += gridDim.x) {
    const int x0 = (tile % ntx) * TX;
    const int rest = tile / ntx;
    const int y0 = (rest % nty) * TY, z0 = (rest / nty) * TZ;
    __syncthreads();  // the previous tile's epilogue is done with the LDS tile
#pragma unroll
    for (int k = 0; k < HALO_IT; ++k)
      if (row_ok(k)) sin4[f_part * HALO_CS + (f_row0 + ROWS_PER_IT * k) * HX + f_hx] = pre[k];
    __syncthreads();
    if (tile + int(gridDim.x) < ntiles) fetch(tile + gridDim.x);

    f32x4 acc[WROWS][2];
#pragma unroll
    for (int m = 0; m < WROWS; ++m)
#pragma unroll
      for (int h = 0; h < 2; ++h) acc[m][h] = f32x4{0.f, 0.f, 0.f, 0.f};
    // For fixed (dz, dx) an input row yr of the halo feeds output rows m = yr - 1 - dy of the
    // wave (dy in {-1, 0, 1}): load its B fragment once and apply it to each of them.  The nine
    // (dz, dx) steps are software-pipelined: step i + 1's fragments (6 weight, WROWS + 2 input)
    // are read from LDS before step i's MFMAs issue, so their latency hides behind them.
    bf16x8 fw[2][3][2], fa[2][WROWS + 2];
    auto load_step = [&](int it, int buf) {
      const int dz = it / 3 - 1, dxi = it % 3;
#pragma unroll
      for (int dyi = 0; dyi < 3; ++dyi)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int d = (dz + 1) * 9 + dyi * 3 + dxi;
          fw[buf][dyi][h] = *reinterpret_cast<const bf16x8*>(
              &reinterpret_cast<const u32x4*>(s_w)[((2 * d + h) * 4 + lg) * 16 + li]);
        }
#pragma unroll
      for (int yr = 0; yr < WROWS + 2; ++yr) {
        const int hidx = ((zl + 1 + dz) * HY + (yb + yr)) * HX + (li + dxi);
        fa[buf][yr] = *reinterpret_cast<const bf16x8*>(
            &reinterpret_cast<const u32x4*>(s_in)[lg * HALO_CS + hidx]);
      }
    };
    load_step(0, 0);
#pragma unroll
    for (int it = 0; it < 9; ++it) {
      const int buf = it & 1;
      if (it + 1 < 9) load_step(it + 1, buf ^ 1);
      // keep the scheduler from sinking those reads back down to their uses
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int yr = 0; yr < WROWS + 2; ++yr)
#pragma unroll
        for (int m = 0; m < WROWS; ++m) {
          const int dyi = yr - m;  // dy + 1
          if (dyi < 0 || dyi > 2) continue;
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc[m][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[buf][dyi][h], fa[buf][yr],
                                                                 acc[m][h], 0, 0, 0);
        }
      __builtin_amdgcn_sched_barrier(0);
    }
    // D[R][v] of lane (li, lg), element r (R = 4 lg + r): channel 8 lg + 4 h + r of voxel x0 + li
    // in output row m, so each lane leaves channels 8 lg .. 8 lg + 7 of one voxel in 16 bytes
    const int y = y0 + yb, z = z0 + zl, x = x0 + li;
    if constexpr (EPI == EPI_GELU || EPI == EPI_GELU_Z) {
      // z = bf16(acc + b) for all 32 outputs, then every GELU table read, then the rare fix-ups:
      // no branch separates the reads, so they are all in flight together
      unsigned zw[WROWS][2][2], aw[WROWS][2][2];
#pragma unroll
      for (int m = 0; m < WROWS; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int k = 0; k < 2; ++k)
            zw[m][h][k] = f2bf2(acc[m][h][2 * k] + bias[h][2 * k],
                                acc[m][h][2 * k + 1] + bias[h][2 * k + 1]);
      u16x2 worst = (u16x2)0;
#pragma unroll
      for (int m = 0; m < WROWS; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int k = 0; k < 2; ++k) aw[m][h][k] = gelu2_lookup(zw[m][h][k], s_gt, &worst);
      if (gelu2_any_outside(worst)) {
#pragma unroll
        for (int m = 0; m < WROWS; ++m)
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int k = 0; k < 2; ++k) aw[m][h][k] = gelu2_fix(zw[m][h][k], aw[m][h][k]);
      }
#pragma unroll
      for (int m = 0; m < WROWS; ++m) {
        if (x >= a.nx || y + m >= a.ny || z >= a.nz) continue;
        const long long v = ((long long)z * a.ny + y + m) * a.nx + x;
        if constexpr (EPI == EPI_GELU_Z)
          *reinterpret_cast<uint4*>(a.z_out + v * CH + 8 * lg) =
              make_uint4(zw[m][0][0], zw[m][0][1], zw[m][1][0], zw[m][1][1]);
        *reinterpret_cast<uint4*>(a.a_out + v * CH + 8 * lg) =
            make_uint4(aw[m][0][0], aw[m][0][1], aw[m][1][0], aw[m][1][1]);
      }
      continue;
    }
    if constexpr (EPI == EPI_DGELU) {
#pragma unroll
      for (int m = 0; m < WROWS; ++m) {
        if (x >= a.nx || y + m >= a.ny || z >= a.nz) continue;
        store_dgelu(a, ((long long)z * a.ny + y + m) * a.nx + x, lg, acc[m]);
      }
    }
  }
}

// The one-channel layers own the same 4x8x16 output tile as the 32 -> 32 kernel, one block each.
constexpr int SMALL_THREADS = TX * TY * TZ;  // 512

// ----------------------------------------------------------------------------- MFMA 1 -> 32
// The 1 -> 32 layer, and the backward data of the 32 -> 1 layer (with flipped weights a 1 -> 32
// convolution of FP32 dY), as one GEMM per 16 voxels with the 27 offsets as the reduction index
// (padded to 32): D[o][v] = sum_d W[d][o] x[v + d] on v_mfma_f32_16x16x32_bf16, with the weights
// as A (held in registers, rows permuted by out_channel) and B the halo values gathered for 16
// voxels of a row.  A lane's two D fragments hold 8 consecutive channels of one voxel, so results
// leave as 16-byte stores without staging.  FP32 input enters as three BF16 terms (hi + mid + lo, exact barring underflow), so
// every product is exact and only the FP32 accumulation rounds.
template <bool IN_F32, int EPI>
__global__ __launch_bounds__(SMALL_THREADS) void conv_in_mfma(ConvArgs a, int ntiles) {
  static_assert(EPI == EPI_GELU || EPI == EPI_GELU_Z || EPI == EPI_DGELU, "epilogue kind");
  typedef typename std::conditional<IN_F32, float, bf16_t>::type elem_t;
  constexpr int NT = IN_F32 ? 3 : 1;
  __shared__ elem_t s_h[HALO_VOX];
  __shared__ __attribute__((aligned(16))) bf16_t s_gt[GT_N];
  const int tid = threadIdx.x;
  if (EPI != EPI_DGELU)
    for (int i = tid; i < GT_N / 8; i += SMALL_THREADS)
      reinterpret_cast<u32x4*>(s_gt)[i] = reinterpret_cast<const u32x4*>(a.gtab)[i];
  const int ntx = (a.nx + TX - 1) / TX, nty = (a.ny + TY - 1) / TY;
  constexpr int IT = (HALO_VOX + SMALL_THREADS - 1) / SMALL_THREADS;
  const bool narrow = a.nx < HX || a.ny < HY || a.nz < HZ;  // uniform
  const elem_t* gin = static_cast<const elem_t*>(a.in);
  const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int zl = wave >> 1, yb = (wave & 1) * 4;
  // A[R][d] = W[d][o] for row R = li of MFMA h, channel o = out_channel(h, li), and this lane's
  // reduction slots d = 8 lg + j
  bf16x8 aw[2];
  float bias[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int o = out_channel(h, li);
    u32x4 q;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int d = 8 * lg + 2 * k;
      const unsigned lo = d < 27 ? a.w[d * CH + o] : 0u;
      const unsigned hi = d + 1 < 27 ? a.w[(d + 1) * CH + o] : 0u;
      q[k] = lo | (hi << 16);
    }
    aw[h] = as_bf16x8(q);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      bias[h][r] = EPI != EPI_DGELU ? a.bias[out_channel(h, 4 * lg + r)] : 0.f;
  }
  int rel[8];
  bool ok[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int d = 8 * lg + j;
    ok[j] = d < 27;
    rel[j] = ok[j] ? ((d / 9 - 1) * HY + (d / 3) % 3 - 1) * HX + d % 3 - 1 : 0;
  }
  // persistent: the table and the weights are staged once, then the block walks tiles; the next
  // tile's halo is loaded into registers while the current one is computed
  elem_t pre[IT];
  auto fetch = [&](int tl) {
    const int fx0 = (tl % ntx) * TX;
    const int fy0 = (tl / ntx % nty) * TY;
    const int fz0 = (tl / ntx / nty) * TZ;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      // lanes past the halo load voxel 0 (always valid) and store nothing
      const int i = tid + k * SMALL_THREADS < HALO_VOX ? tid + k * SMALL_THREADS : 0;
      const int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
      int gx = fx0 + hx - 1, gy = fy0 + hy - 1, gz = fz0 + hz - 1;
      if (narrow) {  // grids narrower than a tile plus halo: true modulo
        gx = pmod(gx, a.nx);
        gy = pmod(gy, a.ny);
        gz = pmod(gz, a.nz);
      } else {
        gx = wrap(gx, a.nx);
        gy = wrap(gy, a.ny);
        gz = wrap(gz, a.nz);
      }
      pre[k] = gin[((long long)gz * a.ny + gy) * a.nx + gx];
    }
  };
  if (int(blockIdx.x) < ntiles) fetch(blockIdx.x);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int x0 = (tile % ntx) * TX;
    const int y0 = (tile / ntx % nty) * TY;
    const int z0 = (tile / ntx / nty) * TZ;
    __syncthreads();  // the previous tile is done with s_h
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int i = tid + k * SMALL_THREADS;
      if (i < HALO_VOX) s_h[i] = pre[k];
    }
    __syncthreads();
    if (tile + int(gridDim.x) < ntiles) fetch(tile + gridDim.x);
    f32x4 accs[4][2];
  #pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int yl = yb + m;
      const int base = ((zl + 1) * HY + yl + 1) * HX + li + 1;
      u32x4 part[NT];
  #pragma unroll
      for (int k = 0; k < 4; ++k) {
        unsigned lo[NT], hi[NT];
  #pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int j = 2 * k + e;
          if constexpr (IN_F32) {
            float v = ok[j] ? s_h[base + rel[j]] : 0.f;
  #pragma unroll
            for (int n = 0; n < NT; ++n) {
              const bf16_t hb = f2bf(v);
              v -= bf2f(hb);
              (e ? hi : lo)[n] = hb;
            }
          } else {
            // BF16 input is its own single term: its bits, zero in the padded slots
            (e ? hi : lo)[0] = unsigned(s_h[base + rel[j]]) & (ok[j] ? 0xFFFFu : 0u);
          }
        }
  #pragma unroll
        for (int n = 0; n < NT; ++n) part[n][k] = lo[n] | (hi[n] << 16);
      }
  #pragma unroll
      for (int h = 0; h < 2; ++h) {
        accs[m][h] = f32x4{0.f, 0.f, 0.f, 0.f};
  #pragma unroll
        for (int n = 0; n < NT; ++n)
          accs[m][h] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[h], as_bf16x8(part[n]), accs[m][h], 0, 0, 0);
      }
    }
    if constexpr (EPI == EPI_GELU || EPI == EPI_GELU_Z) {
      // as in conv32_mfma, in two halves of two rows: every GELU table read of a half before any
      // is used, rare fix-ups after
  #pragma unroll
      for (int m0 = 0; m0 < 4; m0 += 2) {
        unsigned zw[2][2][2], gw[2][2][2];
        u16x2 worst = (u16x2)0;
  #pragma unroll
        for (int m = 0; m < 2; ++m)
  #pragma unroll
          for (int h = 0; h < 2; ++h)
  #pragma unroll
            for (int k = 0; k < 2; ++k) {
              zw[m][h][k] = f2bf2(accs[m0 + m][h][2 * k] + bias[h][2 * k],
                                  accs[m0 + m][h][2 * k + 1] + bias[h][2 * k + 1]);
              gw[m][h][k] = gelu2_lookup(zw[m][h][k], s_gt, &worst);
            }
        if (gelu2_any_outside(worst)) {
  #pragma unroll
          for (int m = 0; m < 2; ++m)
  #pragma unroll
            for (int h = 0; h < 2; ++h)
  #pragma unroll
              for (int k = 0; k < 2; ++k) gw[m][h][k] = gelu2_fix(zw[m][h][k], gw[m][h][k]);
        }
  #pragma unroll
        for (int m = 0; m < 2; ++m) {
          const int x = x0 + li, y = y0 + yb + m0 + m, z = z0 + zl;
          if (x >= a.nx || y >= a.ny || z >= a.nz) continue;
          const long long v = ((long long)z * a.ny + y) * a.nx + x;
          if constexpr (EPI == EPI_GELU_Z)
            *reinterpret_cast<uint4*>(a.z_out + v * CH + 8 * lg) =
                make_uint4(zw[m][0][0], zw[m][0][1], zw[m][1][0], zw[m][1][1]);
          *reinterpret_cast<uint4*>(a.a_out + v * CH + 8 * lg) =
              make_uint4(gw[m][0][0], gw[m][0][1], gw[m][1][0], gw[m][1][1]);
        }
      }
      continue;
    }
    if constexpr (EPI == EPI_DGELU) {
  #pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int x = x0 + li, y = y0 + yb + m, z = z0 + zl;
        if (x >= a.nx || y >= a.ny || z >= a.nz) continue;
        store_dgelu(a, ((long long)z * a.ny + y) * a.nx + x, lg, accs[m]);
      }
    }
  }
}

// ----------------------------------------------------------------------------- MFMA 32 -> 1
// The 32 -> 1 layer (with the residual) with its 27 offsets moved into the GEMM's output: for each
// voxel u of a halo plane, P[u][d] = sum_i W[d][i] a[u][i] on v_mfma_f32_16x16x32_bf16 (A = the
// weights, offsets d as rows of two MFMAs; B = 16 voxels' channels, read straight from memory: 64
// contiguous bytes per voxel), then out[v] = c[v] + (sum_d P[v + d][d] + b).  A block owns a
// 16 x 16 column of the grid and marches up a range of its z planes: each input plane's P (over
// the plane's 18 x 18 halo) is computed once, into LDS, and added to the three output planes that
// plane reaches, whose sums each thread carries in registers; an output plane is complete, and
// stored, once the plane above it has been added.  The next plane's loads are in flight while a
// plane is summed.  Every voxel adds its 27 terms in the order (dz, dy, dx).
constexpr int OX = 16, OY = 16;                                  // output column of a block
constexpr int OHX = OX + 2, OHY = OY + 2;
constexpr int O_HALO = OHX * OHY;                                // 324 voxels of a halo plane
constexpr int O_GROUPS = (O_HALO + 15) / 16;                     // 21 MFMA column groups
constexpr int O_THREADS = OX * OY;                               // one output column per thread
constexpr int O_WAVES = O_THREADS / 64;
constexpr int O_PER_WAVE = (O_GROUPS + O_WAVES - 1) / O_WAVES;   // 6
constexpr int O_PP = 27;  // P row pitch: odd, so the gathers of a wave's 64 voxels spread over banks

__global__ __launch_bounds__(O_THREADS) void conv_out_mfma(ConvArgs a, int ncols, int lz) {
  __shared__ float s_p[O_HALO * O_PP];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int ntx = (a.nx + OX - 1) / OX;
  const int col = int(blockIdx.x) % ncols, chunk = int(blockIdx.x) / ncols;
  const int x0 = (col % ntx) * OX, y0 = (col / ntx) * OY;
  const int z0 = chunk * lz, z1 = z0 + lz < a.nz ? z0 + lz : a.nz;
  const u32x4* gin = static_cast<const u32x4*>(a.in);
  // A[R][i] = W[16 q + R][i] for MFMA q, rows past the 27 offsets zero
  bf16x8 aw[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int d = 16 * q + li;
    u32x4 w = u32x4{0u, 0u, 0u, 0u};
    if (d < 27) w = *reinterpret_cast<const u32x4*>(a.w + d * CH + 8 * lg);
    aw[q] = as_bf16x8(w);
  }
  // in-plane offsets (16-byte chunks) of this lane's halo voxels: group g = wave + O_WAVES k,
  // voxel g * 16 + li; slots past the halo load voxel 0 and store nothing
  long long src[O_PER_WAVE];
#pragma unroll
  for (int k = 0; k < O_PER_WAVE; ++k) {
    const int u0 = (wave + O_WAVES * k) * 16 + li;
    const int u = u0 < O_HALO ? u0 : 0;
    const int hx = u % OHX, hy = u / OHX;
    const long long gx = pmod(x0 + hx - 1, a.nx), gy = pmod(y0 + hy - 1, a.ny);
    src[k] = (gy * a.nx + gx) * 4 + lg;
  }
  const long long plane4 = (long long)a.ny * a.nx * 4;
  u32x4 pre[O_PER_WAVE];
  auto fetch = [&](int zi) {
    const long long base = pmod(zi, a.nz) * plane4;
#pragma unroll
    for (int k = 0; k < O_PER_WAVE; ++k) pre[k] = gin[base + src[k]];
  };
  const float bias = a.bias[0];
  const int tx = tid % OX, ty = tid / OX;
  const int x = x0 + tx, y = y0 + ty;
  const bool own = x < a.nx && y < a.ny;
  float r_prev = 0.f, r_cur = 0.f, r_next = 0.f;  // sums of out[zi - 1], out[zi], out[zi + 1]
  fetch(z0 - 1);
  for (int zi = z0 - 1; zi <= z1; ++zi) {
#pragma unroll
    for (int k = 0; k < O_PER_WAVE; ++k) {
      const int g = wave + O_WAVES * k;
      if (g >= O_GROUPS) continue;  // wave-uniform
      const f32x4 d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[0], as_bf16x8(pre[k]),
                                                                f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      const f32x4 d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[1], as_bf16x8(pre[k]),
                                                                f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      const int u = g * 16 + li;
      if (u < O_HALO) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {  // D[4 lg + r][li] = P[u][16 q + 4 lg + r]
          s_p[u * O_PP + 4 * lg + r] = d0[r];
          if (16 + 4 * lg + r < 27) s_p[u * O_PP + 16 + 4 * lg + r] = d1[r];
        }
      }
    }
    if (zi < z1) fetch(zi + 1);
    __syncthreads();
    // plane zi reaches out[zi - dz] through the offsets of layer dz
#pragma unroll
    for (int dzi = 0; dzi < 3; ++dzi) {
      float& r = dzi == 0 ? r_next : (dzi == 1 ? r_cur : r_prev);
#pragma unroll
      for (int dyi = 0; dyi < 3; ++dyi)
#pragma unroll
        for (int dxi = 0; dxi < 3; ++dxi)
          r += s_p[((ty + dyi) * OHX + tx + dxi) * O_PP + 9 * dzi + 3 * dyi + dxi];
    }
    __syncthreads();  // the next plane rewrites P
    const int zo = zi - 1;
    if (zo >= z0 && own) {
      const long long v = ((long long)zo * a.ny + y) * a.nx + x;
      a.out[v] = a.c[v] + (r_prev + bias);
    }
    r_prev = r_cur;
    r_cur = r_next;
    r_next = 0.f;
  }
}

// ----------------------------------------------------------------------------- weight gradient
// All three kinds are GEMMs whose reduction index is the voxel, run on v_mfma_f32_16x16x32_bf16:
// one MFMA contracts 32 voxels (4 rows of 8 along x).  Blocks walk tiles of 8 x 16 x 1 voxels
// (x, y, z), keep their sums in registers across tiles and leave one partial set each, which
// wgrad_reduce adds in a fixed order (bit-reproducible).  Voxels past the grid edge of a ragged
// tile are zero in the staged operand that is not shifted, so they contribute nothing.
constexpr int WT_X = 8, WT_Y = 16, WT_KS = WT_Y / 4;
constexpr int WG_MAXBLK = 512;   // partial sets of the 32 -> 32 kernel
constexpr int WG1_MAXBLK = 512;  // partial sets of the one-channel kernel

// channel j of two voxels' 8-channel chunks as one dword (voxel a in the low half)
__device__ __forceinline__ unsigned pack_pair(const u32x4& qa, const u32x4& qb, int j) {
  const unsigned a = qa[j >> 1], b = qb[j >> 1];
  return (j & 1) ? ((a >> 16) | (b & 0xFFFF0000u)) : ((a & 0xFFFFu) | (b << 16));
}
// BF16 ones at the k-slots of lane group lg whose voxel is inside the grid
__device__ __forceinline__ bf16x8 ones_mask(int x0, int nx, bool row_ok) {
  u32x4 m;
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const unsigned lo = (row_ok && x0 + 2 * h < nx) ? 0x3F80u : 0u;
    const unsigned hi = (row_ok && x0 + 2 * h + 1 < nx) ? 0x3F80u : 0u;
    m[h] = lo | (hi << 16);
  }
  return as_bf16x8(m);
}

// 32 -> 32 layers.  With the x part of the offset moved onto gz,
//   dW[d,o,i] = sum_u gz[u - dx e_x, o] x[u + dy e_y + dz e_z, i],
// the x operand is read unshifted and one gz fragment, with its three x shifts, feeds the three
// dx offsets of a wave; wave w of the 9-wave block takes (dz, dy) = (w / 3 - 1, w % 3 - 1), 48
// accumulators per lane.  LDS holds both fields channel-major: x with a y/z halo of one (54 rows of 8 voxels), gz
// with an x halo of one (16 rows of 10).  Channel strides are 8 mod 16 bf16 so that the 16-byte
// fragment reads of 8 consecutive channels fall in distinct banks.
constexpr int WG_THREADS = 576;
constexpr int SX_ROWS = 3 * (WT_Y + 2);     // 54
constexpr int SX_CS = SX_ROWS * WT_X + 8;   // 440
constexpr int SG_P = 16;                    // row pitch; x' in [0, 10) is x0 - 1 .. x0 + 8
constexpr int SG_CS = WT_Y * SG_P + 8;      // 264
constexpr int SX_UNITS = SX_ROWS * 4 * 4;   // (row, voxel pair, 8-channel group)
constexpr int SG_UNITS = WT_Y * 5 * 4;
static_assert(SX_CS % 16 == 8 && SG_CS % 16 == 8, "conflict-free fragment reads");

struct WgradArgs {
  const void* s;      // 32->32: gz bf16 [V][32]; one channel: the scalar field (see wgrad1)
  const bf16_t* t;    // 32->32: x bf16 [V][32]; one channel: the 32-channel field
  float* partial;     // [gridDim.x][28][Cout][Cin]; row 27 holds db at [27][o][0]
  int nx, ny, nz, ntiles;
};

__global__ __launch_bounds__(WG_THREADS, 5) void wgrad32_mfma(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) bf16_t s_x[CH * SX_CS];
  __shared__ __attribute__((aligned(16))) bf16_t s_g[CH * SG_CS];
  unsigned* sx32 = reinterpret_cast<unsigned*>(s_x);
  unsigned* sg32 = reinterpret_cast<unsigned*>(s_g);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int ntx = (a.nx + WT_X - 1) / WT_X, nty = (a.ny + WT_Y - 1) / WT_Y;
  const u32x4* g4 = static_cast<const u32x4*>(a.s);
  const u32x4* x4 = reinterpret_cast<const u32x4*>(a.t);
  const int dzi = w / 3, dyi = w % 3;
  f32x4 acc[3][2][2];  // [dx + 1][o half][i half]
  f32x4 accb[2];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < 2; ++k) acc[j][h][k] = f32x4{0.f, 0.f, 0.f, 0.f};
  accb[0] = accb[1] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const int x0 = (t % ntx) * WT_X, rest = t / ntx;
    const int y0 = (rest % nty) * WT_Y, z0 = rest / nty;
    __syncthreads();  // the previous tile's fragment reads are done
    for (int q = tid; q < SX_UNITS; q += WG_THREADS) {
      const int cg = q & 3, p = (q >> 2) & 3, row = q >> 4;
      const int hz = row / (WT_Y + 2), hy = row % (WT_Y + 2);
      const long long rowv =
          ((long long)pmod(z0 + hz - 1, a.nz) * a.ny + pmod(y0 + hy - 1, a.ny)) * a.nx;
      const int xa = x0 + 2 * p;
      u32x4 qa = u32x4{0u, 0u, 0u, 0u}, qb = qa;
      if (xa < a.nx) qa = x4[(rowv + xa) * 4 + cg];
      if (xa + 1 < a.nx) qb = x4[(rowv + xa + 1) * 4 + cg];
      unsigned* dst = sx32 + (8 * cg * SX_CS + row * WT_X + 2 * p) / 2;
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[j * (SX_CS / 2)] = pack_pair(qa, qb, j);
    }
    for (int q = tid; q < SG_UNITS; q += WG_THREADS) {
      const int cg = q & 3, p = (q >> 2) % 5, r = (q >> 2) / 5;
      u32x4 qa = u32x4{0u, 0u, 0u, 0u}, qb = qa;
      if (y0 + r < a.ny) {  // rows past the grid edge stay zero: they mask out their voxels
        const long long rowv = ((long long)z0 * a.ny + y0 + r) * a.nx;
        qa = g4[(rowv + pmod(x0 - 1 + 2 * p, a.nx)) * 4 + cg];
        qb = g4[(rowv + pmod(x0 + 2 * p, a.nx)) * 4 + cg];
      }
      unsigned* dst = sg32 + (8 * cg * SG_CS + r * SG_P + 2 * p) / 2;
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[j * (SG_CS / 2)] = pack_pair(qa, qb, j);
    }
    __syncthreads();
    const bf16x8 ones = ones_mask(x0, a.nx, true);
    for (int ks = 0; ks < WT_KS; ++ks) {
      if (y0 + 4 * ks >= a.ny) break;
      const int r = 4 * ks + lg;
      u32x4 q[2];
      unsigned q4[2];
#pragma unroll
      for (int hm = 0; hm < 2; ++hm) {
        const unsigned* src = sg32 + ((16 * hm + li) * SG_CS + r * SG_P) / 2;
        q[hm] = *reinterpret_cast<const u32x4*>(src);
        q4[hm] = src[4];
      }
      bf16x8 B[2];
#pragma unroll
      for (int hn = 0; hn < 2; ++hn)
        B[hn] = *reinterpret_cast<const bf16x8*>(
            &s_x[(16 * hn + li) * SX_CS + (dzi * (WT_Y + 2) + r + dyi) * WT_X]);
      // gz fragment for shift dx: elements x' = j + 1 - dx of the staged row
      auto frag = [&](int hm, int dxi) {
        const u32x4 v = q[hm];
        if (dxi == 0) return as_bf16x8(u32x4{v[1], v[2], v[3], q4[hm]});
        if (dxi == 2) return as_bf16x8(v);
        return as_bf16x8(u32x4{__builtin_amdgcn_alignbyte(v[1], v[0], 2),
                               __builtin_amdgcn_alignbyte(v[2], v[1], 2),
                               __builtin_amdgcn_alignbyte(v[3], v[2], 2),
                               __builtin_amdgcn_alignbyte(q4[hm], v[3], 2)});
      };
#pragma unroll
      for (int dxi = 0; dxi < 3; ++dxi)
#pragma unroll
        for (int hm = 0; hm < 2; ++hm) {
          const bf16x8 A = frag(hm, dxi);
#pragma unroll
          for (int hn = 0; hn < 2; ++hn)
            acc[dxi][hm][hn] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B[hn], acc[dxi][hm][hn], 0, 0, 0);
        }
      if (w == 4) {  // db[o] = sum_u gz[u, o]
#pragma unroll
        for (int hm = 0; hm < 2; ++hm)
          accb[hm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag(hm, 1), ones, accb[hm], 0, 0, 0);
      }
    }
  }
  // D[m][n] of lane (li, lg), element r: o = 16 hm + 4 lg + r, i = 16 hn + li
  float* P = a.partial + (long long)blockIdx.x * 28 * CH * CH;
#pragma unroll
  for (int dxi = 0; dxi < 3; ++dxi) {
    const int d = 3 * w + dxi;  // 9 (dz + 1) + 3 (dy + 1) + dx + 1
#pragma unroll
    for (int hm = 0; hm < 2; ++hm)
#pragma unroll
      for (int hn = 0; hn < 2; ++hn)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          P[(d * CH + 16 * hm + 4 * lg + r) * CH + 16 * hn + li] = acc[dxi][hm][hn][r];
  }
  if (w == 4) {
#pragma unroll
    for (int hm = 0; hm < 2; ++hm)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int hn = 0; hn < 2; ++hn)
          P[(27 * CH + 16 * hm + 4 * lg + r) * CH + 16 * hn + li] = accb[hm][r];
  }
}

// 1 -> 32 and 32 -> 1 layers.  With one scalar field s and one 32-channel field T,
//   dW[d, c] = sum_u s[u + SIGMA d] T[u, c],
// SIGMA = +1: s = X0 (BF16), T = dZ1, c = o;  SIGMA = -1: s = dY (FP32), T = A3, c = i (after
// substituting u = v + d).  That is a 32 x 32 GEMM per K-step with rows m = d (27 used): the A
// fragment gathers s at u + SIGMA d from an FP32 halo tile, B is T channel-major.  FP32 dY enters
// as three BF16 terms (hi + mid + lo equals it exactly barring underflow), so every MFMA product
// is exact.  Wave w of the 4-wave block takes K-step w of each tile; the block sums its waves in
// LDS in a fixed order before leaving its partial set.
constexpr int WG1_THREADS = 256;
constexpr int ST_CS = WT_Y * WT_X + 8;          // 136 bf16 per channel (8 mod 16)
constexpr int SS_P = 12, SS_H = WT_Y + 2;       // scalar halo tile [3][18][12], x' in [0, 10)
constexpr int SS_N = 3 * SS_H * 10;
static_assert(ST_CS % 16 == 8, "conflict-free fragment reads");

template <int SIGMA>
__global__ __launch_bounds__(WG1_THREADS) void wgrad1_mfma(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) bf16_t s_t[CH * ST_CS];
  __shared__ float s_s[3 * SS_H * SS_P];
  __shared__ float s_red[4 * 28 * CH];
  unsigned* st32 = reinterpret_cast<unsigned*>(s_t);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  const int ntx = (a.nx + WT_X - 1) / WT_X, nty = (a.ny + WT_Y - 1) / WT_Y;
  const u32x4* t4 = reinterpret_cast<const u32x4*>(a.t);
  constexpr int NT = SIGMA > 0 ? 1 : 3;  // BF16 terms of the scalar
  f32x4 acc[2][2];
  f32x4 accb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    accb[h] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 2; ++k) acc[h][k] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  // this lane's two A rows: offset d = 16 hm + li (rows 27..31 are zero)
  int soff[2];
  bool dok[2];
#pragma unroll
  for (int hm = 0; hm < 2; ++hm) {
    const int d = 16 * hm + li;
    dok[hm] = d < 27;
    const int dz = d / 9 - 1, dy = (d / 3) % 3 - 1, dx = d % 3 - 1;
    soff[hm] = dok[hm] ? ((1 + SIGMA * dz) * SS_H + 1 + SIGMA * dy) * SS_P + 1 + SIGMA * dx : 0;
  }

  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const int x0 = (t % ntx) * WT_X, rest = t / ntx;
    const int y0 = (rest % nty) * WT_Y, z0 = rest / nty;
    __syncthreads();
    {  // T tile: 16 rows x 4 voxel pairs x 4 channel groups, one unit per thread
      const int cg = tid & 3, p = (tid >> 2) & 3, r = tid >> 4;
      const int xa = x0 + 2 * p;
      u32x4 qa = u32x4{0u, 0u, 0u, 0u}, qb = qa;
      if (y0 + r < a.ny) {
        const long long rowv = ((long long)z0 * a.ny + y0 + r) * a.nx;
        if (xa < a.nx) qa = t4[(rowv + xa) * 4 + cg];
        if (xa + 1 < a.nx) qb = t4[(rowv + xa + 1) * 4 + cg];
      }
      unsigned* dst = st32 + (8 * cg * ST_CS + r * WT_X + 2 * p) / 2;
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[j * (ST_CS / 2)] = pack_pair(qa, qb, j);
    }
    for (int q = tid; q < SS_N; q += WG1_THREADS) {
      const int xq = q % 10, hy = (q / 10) % SS_H, hz = q / (10 * SS_H);
      const long long v =
          ((long long)pmod(z0 + hz - 1, a.nz) * a.ny + pmod(y0 + hy - 1, a.ny)) * a.nx +
          pmod(x0 + xq - 1, a.nx);
      float sv;
      if constexpr (SIGMA > 0) sv = bf2f(static_cast<const bf16_t*>(a.s)[v]);
      else sv = static_cast<const float*>(a.s)[v];
      s_s[(hz * SS_H + hy) * SS_P + xq] = sv;
    }
    __syncthreads();
    if (y0 + 4 * w < a.ny) {
      const int r = 4 * w + lg;
      bf16x8 B[2];
#pragma unroll
      for (int hn = 0; hn < 2; ++hn)
        B[hn] = *reinterpret_cast<const bf16x8*>(&s_t[(16 * hn + li) * ST_CS + r * WT_X]);
      bf16x8 A[2][NT];
#pragma unroll
      for (int hm = 0; hm < 2; ++hm) {
        u32x4 part[NT];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          unsigned lo[NT], hi[NT];
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            float v = dok[hm] ? s_s[soff[hm] + r * SS_P + 2 * k + e] : 0.f;
#pragma unroll
            for (int n = 0; n < NT; ++n) {
              const bf16_t h = f2bf(v);
              v -= bf2f(h);  // exact: the remainder of a round-to-nearest fits in FP32
              (e ? hi : lo)[n] = h;
            }
          }
#pragma unroll
          for (int n = 0; n < NT; ++n) part[n][k] = lo[n] | (hi[n] << 16);
        }
#pragma unroll
        for (int n = 0; n < NT; ++n) A[hm][n] = as_bf16x8(part[n]);
      }
#pragma unroll
      for (int hm = 0; hm < 2; ++hm)
#pragma unroll
        for (int hn = 0; hn < 2; ++hn)
#pragma unroll
          for (int n = 0; n < NT; ++n)
            acc[hm][hn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[hm][n], B[hn], acc[hm][hn],
                                                                  0, 0, 0);
      if constexpr (SIGMA > 0) {  // db[o] = sum_u dZ1[u, o]: all-ones A
        const bf16x8 one = as_bf16x8(u32x4{0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u});
#pragma unroll
        for (int hn = 0; hn < 2; ++hn)
          accb[hn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(one, B[hn], accb[hn], 0, 0, 0);
      } else {  // db = sum_u dY[u]: row d = 13 (no offset) against the in-grid mask
        const bf16x8 msk = ones_mask(x0, a.nx, y0 + r < a.ny);
#pragma unroll
        for (int n = 0; n < NT; ++n)
          accb[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0][n], msk, accb[0], 0, 0, 0);
      }
    }
  }
  // D[m][n] of lane (li, lg), element r: d = 16 hm + 4 lg + r, c = 16 hn + li
  float* red = s_red + w * 28 * CH;
#pragma unroll
  for (int hm = 0; hm < 2; ++hm)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int d = 16 * hm + 4 * lg + r;
      if (d < 27) {
#pragma unroll
        for (int hn = 0; hn < 2; ++hn) red[d * CH + 16 * hn + li] = acc[hm][hn][r];
      }
    }
  if (lg == 0) {  // SIGMA > 0: every row of D holds db[c]; SIGMA < 0: zeros, db set below
#pragma unroll
    for (int hn = 0; hn < 2; ++hn) red[27 * CH + 16 * hn + li] = SIGMA > 0 ? accb[hn][0] : 0.f;
  }
  if constexpr (SIGMA < 0) {
    __syncthreads();  // the zero fill of row 27 lands before lane (0, 3) writes db
    if (lg == 3 && li == 0) red[27 * CH] = accb[0][1];  // D[13][0]: 4 * 3 + 1 = 13
  }
  __syncthreads();
  float* P = a.partial + (long long)blockIdx.x * 28 * CH;
  for (int k = tid; k < 28 * CH; k += WG1_THREADS)
    P[k] = ((s_red[k] + s_red[28 * CH + k]) + s_red[2 * 28 * CH + k]) + s_red[3 * 28 * CH + k];
}

// grad[param] (+)= sum over the partial sets; maps (d, o, i) -> W offset, d == 27 -> bias (only
// i == 0 of the bias rows is used).  A block takes 64 consecutive outputs; its 16 thread groups
// sum interleaved subsets of the sets (group g: sets g, g + 16, ...), and the groups are added in
// a fixed order: bit-reproducible.
constexpr int RED_K = 64, RED_G = 16;

__global__ __launch_bounds__(RED_K * RED_G) void wgrad_reduce(const float* partial, int nsets,
                                                              float* grad_w, float* grad_b,
                                                              int ci, int co) {
  __shared__ float s_sum[RED_G * RED_K];
  const int n = 28 * co * ci;
  const int kk = threadIdx.x % RED_K, g = threadIdx.x / RED_K;
  const int k = blockIdx.x * RED_K + kk;
  float acc = 0.f;
  if (k < n)
    for (int c = g; c < nsets; c += RED_G) acc += partial[(long long)c * n + k];
  s_sum[g * RED_K + kk] = acc;
  __syncthreads();
  if (g != 0 || k >= n) return;
  float t = 0.f;
#pragma unroll
  for (int j = 0; j < RED_G; ++j) t += s_sum[j * RED_K + kk];
  const int d = k / (co * ci), rem = k % (co * ci);
  if (d < 27) {
    grad_w[k] += t;
  } else if (rem % ci == 0) {
    grad_b[rem / ci] += t;
  }
}

// ----------------------------------------------------------------------------- misc element-wise
__global__ void fill_gelu_table(bf16_t* tab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= GT_N) return;
  const unsigned e = gelu_table_entry(i);
  const bool arg = i < 2 * GT_ROW && i % GT_ROW != GT_HALF;
  tab[i] = arg ? f2bf(gelu(bf2f(bf16_t(e)))) : bf16_t(e);
}


__global__ void cast_bf16(const float* c, bf16_t* out, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = f2bf(c[i]);
}

// master fp32 params -> bf16 weights in [d][o][i] and the flipped/transposed copy
// wt[26 - d][i][o] used by the backward-data convolutions (grid.y = layer).
__global__ void refresh_weights(const float* params, bf16_t* w, bf16_t* wt) {
  const int l = blockIdx.y;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= layer_w(l)) return;
  const bf16_t h = f2bf(params[layer_off(l) + k]);
  w[w_off(l) + k] = h;
  const int ci = cin_of(l), co = cout_of(l);
  const int d = int(k / (ci * co)), o = int((k / ci) % co), i = int(k % ci);
  const long long kt = w_off(l) + ((long long)(26 - d) * ci + i) * co + o;
  wt[kt] = h;
}

struct LossArgs {
  const float* out;     // c + net(c)
  const float* target;
  float* dy;            // (2 / n_total) (out - target) on the interior, 0 outside
  double* partial;      // per block sum of squares
  int n, halo;          // window edge (cubic) and halo
  double inv_total;     // 1 / (batch * interior voxels)
};

constexpr int LOSS_BLOCKS = 256;

__global__ __launch_bounds__(256) void loss_kernel(LossArgs a) {
  __shared__ double red[256];
  const long long V = (long long)a.n * a.n * a.n;
  double s = 0.0;
  for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < V;
       v += (long long)gridDim.x * 256) {
    const int x = int(v % a.n), y = int((v / a.n) % a.n), z = int(v / ((long long)a.n * a.n));
    const bool in = x >= a.halo && x < a.n - a.halo && y >= a.halo && y < a.n - a.halo &&
                    z >= a.halo && z < a.n - a.halo;
    const float d = in ? a.out[v] - a.target[v] : 0.f;
    s += double(d) * d;
    a.dy[v] = float(2.0 * a.inv_total) * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[blockIdx.x] = red[0];
}

// one block of LOSS_BLOCKS threads: fixed-order tree over the per-block sums
__global__ __launch_bounds__(LOSS_BLOCKS) void loss_final(const double* partial, double scale,
                                                          double* loss, int add) {
  __shared__ double red[LOSS_BLOCKS];
  red[threadIdx.x] = partial[threadIdx.x];
  __syncthreads();
  for (int h = LOSS_BLOCKS / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (add ? *loss : 0.0) + scale * red[0];
}

// Adam (Kingma & Ba).  omb1 = 1 - b1 and omb2 = 1 - b2 come from the host in FP64 and are rounded
// once: 1 - 0.999f in FP32 would be 1.3e-5 off 0.001 (0.999 is not representable).
__global__ void adam_kernel(float* p, float* m, float* v, const float* g, long long n, float lr,
                            float b1, float b2, float omb1, float omb2, float eps, float c1,
                            float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Mass projection of a prediction: partial[b] = sum over the block's voxels of (out - c).
constexpr int MP_BLOCKS = 1024;

__global__ __launch_bounds__(256) void increment_sum(const float* out, const float* c, long long n,
                                                     double* partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256)
    s += double(out[i]) - double(c[i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out -= (sum of partials) / n, the partial sums added in a fixed order by every block.
__global__ __launch_bounds__(256) void remove_mean(float* out, long long n, const double* partial,
                                                   int nparts) {
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 256) s += partial[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const float shift = float(red[0] / double(n));
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256)
    out[i] -= shift;
}

__global__ void zero_f32(float* p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

}  // namespace

extern "C" void evx_internal_set_error(const char* msg);

namespace {

evx_status nfail(evx_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  evx_internal_set_error(buf);
  return s;
}

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

struct evx_net {
  int device = 0;
  bf16_t* w = nullptr;   // [sum layer_w] bf16
  bf16_t* wt = nullptr;  // flipped/transposed copies
  float* params = nullptr;  // device copy of the master weights last set (biases are read here)
  bf16_t* gtab = nullptr;   // GELU table
  bool have_params = false;
};

namespace {

enum : int { K_MFMA = 0, K_IN1 = 1, K_OUT1 = 2, K_BWD_F32 = 3 };

long long g_num_cus = 256;  // set from the device at evx_surrogate_create

hipError_t launch_conv(int kind, int epi, const ConvArgs& a, hipStream_t s) {
  const long long nt = (long long)((a.nx + TX - 1) / TX) * ((a.ny + TY - 1) / TY) *
                       ((a.nz + TZ - 1) / TZ);
  const int ntiles = int(nt);
  // the 1 -> 32 kernel is persistent too: four blocks per CU (its table and halo take 12 KB)
  const unsigned in_grid = unsigned(nt < 4 * g_num_cus ? nt : 4 * g_num_cus);
  if (kind == K_MFMA) {
    // one persistent block per CU (the LDS tile and weights take 124 KB)
    const unsigned grid = unsigned(nt < g_num_cus ? nt : g_num_cus);
    if (epi == EPI_GELU_Z)
      hipLaunchKernelGGL(conv32_mfma<EPI_GELU_Z>, dim3(grid), dim3(MFMA_THREADS), 0, s, a, ntiles);
    else if (epi == EPI_GELU)
      hipLaunchKernelGGL(conv32_mfma<EPI_GELU>, dim3(grid), dim3(MFMA_THREADS), 0, s, a, ntiles);
    else
      hipLaunchKernelGGL(conv32_mfma<EPI_DGELU>, dim3(grid), dim3(MFMA_THREADS), 0, s, a, ntiles);
  } else if (kind == K_IN1) {
    if (epi == EPI_GELU_Z)
      hipLaunchKernelGGL((conv_in_mfma<false, EPI_GELU_Z>), dim3(in_grid), dim3(SMALL_THREADS), 0,
                         s, a, ntiles);
    else
      hipLaunchKernelGGL((conv_in_mfma<false, EPI_GELU>), dim3(in_grid), dim3(SMALL_THREADS), 0,
                         s, a, ntiles);
  } else if (kind == K_OUT1) {
    // columns of 16 x 16, each marching up lz planes: long runs (few halo planes re-read), but
    // at least about four blocks per CU
    const long long ncols = (long long)((a.nx + OX - 1) / OX) * ((a.ny + OY - 1) / OY);
    long long lz = (a.nz * ncols + 4 * g_num_cus - 1) / (4 * g_num_cus);
    lz = lz < 2 ? 2 : (lz > a.nz ? a.nz : lz);
    const long long grid = ncols * ((a.nz + lz - 1) / lz);
    if (grid >= (1LL << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(conv_out_mfma, dim3(unsigned(grid)), dim3(O_THREADS), 0, s, a, int(ncols),
                       int(lz));
  } else {  // backward data of the last layer: FP32 dY -> bf16 dZ
    hipLaunchKernelGGL((conv_in_mfma<true, EPI_DGELU>), dim3(in_grid), dim3(SMALL_THREADS), 0, s,
                       a, ntiles);
  }
  return hipGetLastError();
}

hipError_t launch_wgrad(int layer, const void* gz, const void* x, float* partial, float* grads,
                        int nx, int ny, int nz, hipStream_t s) {
  const long long nt =
      (long long)((nx + WT_X - 1) / WT_X) * ((ny + WT_Y - 1) / WT_Y) * (long long)nz;
  if (nt >= (1LL << 31)) return hipErrorInvalidValue;
  const bool wide = layer == 1 || layer == 2;
  const long long maxblk = wide ? WG_MAXBLK : WG1_MAXBLK;
  const long long per = (nt + maxblk - 1) / maxblk;  // tiles per block, balanced
  const int grid = int((nt + per - 1) / per);
  WgradArgs w{};
  w.partial = partial;
  w.nx = nx;
  w.ny = ny;
  w.nz = nz;
  w.ntiles = int(nt);
  if (wide) {
    w.s = gz;
    w.t = static_cast<const bf16_t*>(x);
    hipLaunchKernelGGL(wgrad32_mfma, dim3(grid), dim3(WG_THREADS), 0, s, w);
  } else if (layer == 0) {  // s = X0 (shifted), T = dZ1
    w.s = x;
    w.t = static_cast<const bf16_t*>(gz);
    hipLaunchKernelGGL(wgrad1_mfma<1>, dim3(grid), dim3(WG1_THREADS), 0, s, w);
  } else {                  // s = dY, T = A3 (shifted, moved onto dY)
    w.s = gz;
    w.t = static_cast<const bf16_t*>(x);
    hipLaunchKernelGGL(wgrad1_mfma<-1>, dim3(grid), dim3(WG1_THREADS), 0, s, w);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int ci = cin_of(layer), co = cout_of(layer), n = 28 * ci * co;
  hipLaunchKernelGGL(wgrad_reduce, dim3((n + RED_K - 1) / RED_K), dim3(RED_K * RED_G), 0, s,
                     partial, grid,
                     grads + layer_off(layer), grads + layer_off(layer) + layer_w(layer), ci, co);
  return hipGetLastError();
}

bool grid_ok(int nx, int ny, int nz) {
  return nx >= 1 && ny >= 1 && nz >= 1 && (long long)nx * ny * nz * CH < (1LL << 40);
}

// Inference workspace: X0 (bf16 [V]) | A (bf16 [V][32]) | B (bf16 [V][32]) | mass partials.
size_t infer_bytes(long long V) {
  return a256(V * 2) + 2 * a256(V * CH * 2) + a256(MP_BLOCKS * sizeof(double));
}

// Training workspace for one n^3 window: X0 | Z1 A1 Z2 A2 Z3 A3 | dZ3 dZ2 dZ1 (bf16 [V][32]) | out dY
// (f32 [V]) | target (f32 [V]) | wgrad partials | grads (f32 NPARAM) | loss partials.
struct TrainBufs {
  bf16_t *x0, *z[3], *act[3], *g[3];  // g[0] = dz3, g[1] = dz2, g[2] = dz1
  float *out, *dy, *partial, *grads;
  double* lpart;
};

size_t train_bytes(long long V) {
  return a256(V * 2) + 9 * a256(V * CH * 2) + 2 * a256(V * 4) +
         a256(size_t(WG_MAXBLK) * 28 * CH * CH * 4) + a256(NPARAM * 4) +
         a256(LOSS_BLOCKS * sizeof(double));
}

TrainBufs carve_train(void* ws, long long V) {
  char* p = static_cast<char*>(ws);
  TrainBufs b{};
  auto take = [&](size_t n) { char* q = p; p += a256(n); return q; };
  b.x0 = reinterpret_cast<bf16_t*>(take(V * 2));
  for (int i = 0; i < 3; ++i) {
    b.z[i] = reinterpret_cast<bf16_t*>(take(V * CH * 2));
    b.act[i] = reinterpret_cast<bf16_t*>(take(V * CH * 2));
  }
  for (int i = 0; i < 3; ++i) b.g[i] = reinterpret_cast<bf16_t*>(take(V * CH * 2));
  b.out = reinterpret_cast<float*>(take(V * 4));
  b.dy = reinterpret_cast<float*>(take(V * 4));
  b.partial = reinterpret_cast<float*>(take(size_t(WG_MAXBLK) * 28 * CH * CH * 4));
  b.grads = reinterpret_cast<float*>(take(NPARAM * 4));
  b.lpart = reinterpret_cast<double*>(take(LOSS_BLOCKS * sizeof(double)));
  return b;
}

ConvArgs conv_args(const evx_net* n, int layer, bool transposed, const void* in, int nx, int ny,
                   int nz) {
  ConvArgs a{};
  a.in = in;
  a.w = (transposed ? n->wt : n->w) + w_off(layer);
  a.bias = n->params + layer_off(layer) + layer_w(layer);
  a.gtab = n->gtab;
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  return a;
}

#define NET_TRY(expr)                                                        \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) return nfail(EVX_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

}  // namespace

extern "C" {

evx_status evx_surrogate_param_count(size_t* n) {
  if (!n) return nfail(EVX_ERR_ARG, "n is NULL");
  *n = size_t(NPARAM);
  return EVX_OK;
}

evx_status evx_surrogate_create(evx_net** out) {
  if (!out) return nfail(EVX_ERR_ARG, "out is NULL");
  evx_net* n = new evx_net();
  hipError_t e = hipGetDevice(&n->device);
  int cus = 0;
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, n->device);
  if (e == hipSuccess && cus > 0) g_num_cus = cus;
  const size_t wb = a256(size_t(w_off(NLAYER)) * sizeof(bf16_t));
  const size_t pb = a256(NPARAM * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&n->w, 2 * wb + pb + a256(GT_N * sizeof(bf16_t)));
  if (e != hipSuccess) {
    delete n;
    return nfail(EVX_ERR_HIP, "evx_surrogate_create: %s", hipGetErrorString(e));
  }
  char* base = reinterpret_cast<char*>(n->w);
  n->wt = reinterpret_cast<bf16_t*>(base + wb);
  n->params = reinterpret_cast<float*>(base + 2 * wb);
  n->gtab = reinterpret_cast<bf16_t*>(base + 2 * wb + pb);
  hipLaunchKernelGGL(fill_gelu_table, dim3((GT_N + 255) / 256), dim3(256), 0, nullptr, n->gtab);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(n->w);
    delete n;
    return nfail(EVX_ERR_HIP, "evx_surrogate_create: %s", hipGetErrorString(e));
  }
  *out = n;
  return EVX_OK;
}

evx_status evx_surrogate_destroy(evx_net* n) {
  if (!n) return nfail(EVX_ERR_ARG, "net is NULL");
  if (n->w) (void)hipFree(n->w);
  delete n;
  return EVX_OK;
}

evx_status evx_surrogate_set_params(evx_net* n, const float* params, void* stream) {
  if (!n || !params) return nfail(EVX_ERR_ARG, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(n->params, params, NPARAM * sizeof(float),
                                hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return nfail(EVX_ERR_HIP, "set_params copy: %s", hipGetErrorString(e));
  const long long nw = layer_w(1);  // the largest layer bounds the per-layer index range
  hipLaunchKernelGGL(refresh_weights, dim3(unsigned((nw + 255) / 256), NLAYER), dim3(256), 0, s,
                     n->params, n->w, n->wt);
  e = hipGetLastError();
  if (e != hipSuccess) return nfail(EVX_ERR_HIP, "set_params: %s", hipGetErrorString(e));
  n->have_params = true;
  return EVX_OK;
}

evx_status evx_surrogate_workspace_bytes(int nx, int ny, int nz, int train, size_t* bytes) {
  if (!bytes) return nfail(EVX_ERR_ARG, "bytes is NULL");
  if (!grid_ok(nx, ny, nz)) return nfail(EVX_ERR_SIZE, "grid %d x %d x %d", nx, ny, nz);
  const long long V = (long long)nx * ny * nz;
  *bytes = train ? train_bytes(V) : infer_bytes(V);
  return EVX_OK;
}

evx_status evx_surrogate_infer(evx_net* n, const float* c_in, float* c_out, int nx, int ny,
                               int nz, int flags, void* ws, size_t ws_bytes, void* stream) {
  if (!n || !c_in || !c_out || !ws) return nfail(EVX_ERR_ARG, "NULL argument");
  if (!n->have_params) return nfail(EVX_ERR_STATE, "parameters not set");
  if (!grid_ok(nx, ny, nz)) return nfail(EVX_ERR_SIZE, "grid %d x %d x %d", nx, ny, nz);
  const long long V = (long long)nx * ny * nz;
  if (ws_bytes < infer_bytes(V)) return nfail(EVX_ERR_NOMEM, "workspace too small");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return nfail(EVX_ERR_ARG, "workspace alignment");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* p = static_cast<char*>(ws);
  bf16_t* x0 = reinterpret_cast<bf16_t*>(p);
  bf16_t* A = reinterpret_cast<bf16_t*>(p + a256(V * 2));
  bf16_t* B = reinterpret_cast<bf16_t*>(p + a256(V * 2) + a256(V * CH * 2));
  hipLaunchKernelGGL(cast_bf16, dim3(unsigned((V + 255) / 256)), dim3(256), 0, s, c_in, x0, V);
  NET_TRY(hipGetLastError());
  ConvArgs a = conv_args(n, 0, false, x0, nx, ny, nz);
  a.a_out = A;
  NET_TRY(launch_conv(K_IN1, EPI_GELU, a, s));
  a = conv_args(n, 1, false, A, nx, ny, nz);
  a.a_out = B;
  NET_TRY(launch_conv(K_MFMA, EPI_GELU, a, s));
  a = conv_args(n, 2, false, B, nx, ny, nz);
  a.a_out = A;
  NET_TRY(launch_conv(K_MFMA, EPI_GELU, a, s));
  a = conv_args(n, 3, false, A, nx, ny, nz);
  a.c = c_in;
  a.out = c_out;
  NET_TRY(launch_conv(K_OUT1, EPI_RESID, a, s));
  if (flags & EVX_SURROGATE_CONSERVE_MASS) {
    double* partial = reinterpret_cast<double*>(p + a256(V * 2) + 2 * a256(V * CH * 2));
    hipLaunchKernelGGL(increment_sum, dim3(MP_BLOCKS), dim3(256), 0, s, c_out, c_in, V, partial);
    NET_TRY(hipGetLastError());
    hipLaunchKernelGGL(remove_mean, dim3(MP_BLOCKS), dim3(256), 0, s, c_out, V, partial,
                       MP_BLOCKS);
    NET_TRY(hipGetLastError());
  }
  return EVX_OK;
}

evx_status evx_surrogate_train_step(evx_net* n, const float* x, const float* y, int batch,
                                    int edge, int halo, float* params, float* adam_m,
                                    float* adam_v, int step, float lr, double* loss,
                                    void* ws, size_t ws_bytes, void* stream) {
  if (!n || !x || !y || !params || !adam_m || !adam_v || !loss || !ws)
    return nfail(EVX_ERR_ARG, "NULL argument");
  if (batch < 1 || edge < 1 || halo < 0 || 2 * halo >= edge || step < 1 || !(lr > 0))
    return nfail(EVX_ERR_ARG, "batch %d edge %d halo %d step %d lr %g", batch, edge, halo, step,
                 double(lr));
  if (!grid_ok(edge, edge, edge)) return nfail(EVX_ERR_SIZE, "window %d", edge);
  const long long V = (long long)edge * edge * edge;
  if (ws_bytes < train_bytes(V)) return nfail(EVX_ERR_NOMEM, "workspace too small");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return nfail(EVX_ERR_ARG, "workspace alignment");
  hipStream_t s = static_cast<hipStream_t>(stream);
  evx_status st = evx_surrogate_set_params(n, params, stream);
  if (st != EVX_OK) return st;
  TrainBufs b = carve_train(ws, V);
  hipLaunchKernelGGL(zero_f32, dim3(unsigned((NPARAM + 255) / 256)), dim3(256), 0, s, b.grads,
                     NPARAM);
  NET_TRY(hipGetLastError());
  const long long inner = (long long)(edge - 2 * halo) * (edge - 2 * halo) * (edge - 2 * halo);
  const double inv_total = 1.0 / (double(batch) * double(inner));
  const unsigned vgrid = unsigned((V + 255) / 256);
  for (int w = 0; w < batch; ++w) {
    const float* xw = x + w * V;
    const float* yw = y + w * V;
    hipLaunchKernelGGL(cast_bf16, dim3(vgrid), dim3(256), 0, s, xw, b.x0, V);
    NET_TRY(hipGetLastError());
    // forward, keeping pre-activations
    ConvArgs a = conv_args(n, 0, false, b.x0, edge, edge, edge);
    a.z_out = b.z[0];
    a.a_out = b.act[0];
    NET_TRY(launch_conv(K_IN1, EPI_GELU_Z, a, s));
    for (int l = 1; l <= 2; ++l) {
      a = conv_args(n, l, false, b.act[l - 1], edge, edge, edge);
      a.z_out = b.z[l];
      a.a_out = b.act[l];
      NET_TRY(launch_conv(K_MFMA, EPI_GELU_Z, a, s));
    }
    a = conv_args(n, 3, false, b.act[2], edge, edge, edge);
    a.c = xw;
    a.out = b.out;
    NET_TRY(launch_conv(K_OUT1, EPI_RESID, a, s));
    // loss and dL/dy
    LossArgs la{b.out, yw, b.dy, b.lpart, edge, halo, inv_total};
    hipLaunchKernelGGL(loss_kernel, dim3(LOSS_BLOCKS), dim3(256), 0, s, la);
    NET_TRY(hipGetLastError());
    hipLaunchKernelGGL(loss_final, dim3(1), dim3(LOSS_BLOCKS), 0, s, b.lpart, inv_total, loss,
                       w > 0 ? 1 : 0);
    NET_TRY(hipGetLastError());
    // backward
    NET_TRY(launch_wgrad(3, b.dy, b.act[2], b.partial, b.grads, edge, edge, edge, s));
    a = conv_args(n, 3, true, b.dy, edge, edge, edge);
    a.zprev = b.z[2];
    a.a_out = b.g[0];
    NET_TRY(launch_conv(K_BWD_F32, EPI_DGELU, a, s));                        // g0 = dZ3
    NET_TRY(launch_wgrad(2, b.g[0], b.act[1], b.partial, b.grads, edge, edge, edge, s));
    a = conv_args(n, 2, true, b.g[0], edge, edge, edge);
    a.zprev = b.z[1];
    a.a_out = b.g[1];
    NET_TRY(launch_conv(K_MFMA, EPI_DGELU, a, s));                           // g1 = dZ2
    NET_TRY(launch_wgrad(1, b.g[1], b.act[0], b.partial, b.grads, edge, edge, edge, s));
    a = conv_args(n, 1, true, b.g[1], edge, edge, edge);
    a.zprev = b.z[0];
    a.a_out = b.g[2];
    NET_TRY(launch_conv(K_MFMA, EPI_DGELU, a, s));                           // g2 = dZ1
    NET_TRY(launch_wgrad(0, b.g[2], b.x0, b.partial, b.grads, edge, edge, edge, s));
  }
  const double c1 = 1.0 - std::pow(0.9, double(step)), c2 = 1.0 - std::pow(0.999, double(step));
  hipLaunchKernelGGL(adam_kernel, dim3(unsigned((NPARAM + 255) / 256)), dim3(256), 0, s, params,
                     adam_m, adam_v, b.grads, NPARAM, lr, 0.9f, 0.999f, float(1.0 - 0.9),
                     float(1.0 - 0.999), 1e-8f, float(c1), float(c2));
  NET_TRY(hipGetLastError());
  return evx_surrogate_set_params(n, params, stream);
}

evx_status evx_surrogate_train_buffers(void* ws, size_t ws_bytes, int edge, void** ptrs) {
  if (!ws || !ptrs) return nfail(EVX_ERR_ARG, "NULL argument");
  if (!grid_ok(edge, edge, edge)) return nfail(EVX_ERR_SIZE, "window %d", edge);
  const long long V = (long long)edge * edge * edge;
  if (ws_bytes < train_bytes(V)) return nfail(EVX_ERR_NOMEM, "workspace too small");
  TrainBufs b = carve_train(ws, V);
  void* list[13] = {b.x0, b.z[0], b.act[0], b.z[1], b.act[1], b.z[2], b.act[2],
                    b.g[2], b.g[1], b.g[0], b.out, b.dy, b.grads};
  for (int i = 0; i < 13; ++i) ptrs[i] = list[i];
  return EVX_OK;
}

}  // extern "C"
