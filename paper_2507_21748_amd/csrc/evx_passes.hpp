// Pass bodies of the Cahn-Hilliard spectral step.  Each body is the work of one workgroup; it
// is wrapped by a __global__ kernel for gfx950 and by a threaded host emulator in the CPU tests.
//
// Spectral layout ("grouped").  The x columns of a spectral buffer -- periodic: the nx/2+1
// complex bins of the half spectrum; zero flux: the DCT-II spectrum is real, and its nx bins are
// handled as nx/2 float2 "column pairs" -- form groups of 8 (64 bytes), and a buffer is ordered
// [group][z][y'][8] with y' over ny + kSpecYPad rows: float2 index
//   (((x / 8) nz + z) ypitch + y) 8 + x % 8,   ypitch = ny + kSpecYPad.
// A y column pass then reads one contiguous ny x 64-byte run per (group, z); a z column pass
// reads 64-byte pieces (ny + 2) x 64 bytes apart, a stride that does not alias the memory
// channels the way a power of two does; the x pass reads 8 rows x 64 bytes per group.  Measured
// on 1024^3 with plain data-movement kernels, these patterns move a step's bytes 0.5 ms faster
// than the row-major half spectrum (rows of nx/2 + 1 values padded to 8), whose y passes read
// 64-byte pieces 4 KB apart and whose z pass 64-byte pieces 4.3 MB apart.  Ordering z outside
// the groups instead helps the x pass (its groups then lie 66 KB apart) but costs the z pass
// more.  Columns
// of the last group past the live count and the two pad rows per (group, z) hold no data: the
// column passes never address them and the x pass writes the dead columns as zeros.  Real fields
// stay in natural C order (z, y, x).  Two spectral buffers exist: S (spectral state, tile-major,
// see ColTile) and W (work).
//
// One time step is four passes over W (and one over S):
//   inverse y  ->  x: inverse x, f'(c) = c^3 - c, forward x  ->  forward y  ->
//   z: forward z, k-space update of S, inverse z.
// The real-space field is never stored between steps.
#pragma once

#include <type_traits>

#include "evx_fft.hpp"

namespace evx {

enum : int { BC_PERIODIC = 0, BC_ZERO_FLUX = 1, BC_DIRICHLET = 2, BC_VERTEX = 3 };

// Pad rows per (group, z) slab of a spectral buffer.
constexpr int kSpecYPad = 2;

// Float2 strides of the grouped spectral layout.
struct SpecGeom {
  long long xstride;  // between x groups: nz * ypitch * 8
  long long zstride;  // between z planes of a group: ypitch * 8
  int ny;
};

// Element i of a grouped spectral buffer: its x column, y and z, and whether it holds data (not a
// pad row, not a dead column of the last group).
struct SpecPos {
  int x, y, z;
  bool live;
};
EVX_HD SpecPos spec_pos(long long i, int ny, int ypitch, int nz, int ncols) {
  const long long q = i >> 3;
  const long long zq = q / ypitch;  // group nz + z
  const long long g = zq / nz;
  SpecPos p;
  p.y = int(q - zq * ypitch);
  p.z = int(zq - g * nz);
  p.x = int(g) * 8 + int(i & 7);
  p.live = p.y < ny && p.x < ncols;
  return p;
}

// Float2 offset of row r = z ny + y (x group 0, column 0).
EVX_HD long long spec_row_offset(const SpecGeom& s, long long r) {
  const long long z = r / s.ny;
  return z * s.zstride + (r - z * s.ny) * 8;
}

// The same for row (z0, y0) + j (0 <= y0 < ny, j >= 0, y0 + j < 2^31), without a branch: an
// unsigned division.  (A carry loop would be a divergent region, into which the compiler sinks the
// loads that use the offset, each then waited for before the region ends.)
EVX_HD long long spec_row_offset_from(const SpecGeom& s, long long z0, int y0, int j) {
  const unsigned y = unsigned(y0 + j), ny = unsigned(s.ny);
  const unsigned dz = y / ny;
  return (z0 + dz) * s.zstride + (long long)(y - dz * ny) * 8;
}

// column (y or z) pass modes
enum : int {
  COL_FWD = 0,         // in -> forward transform -> out
  COL_INV = 1,         // in -> inverse transform -> out
  COL_Z_INIT = 2,      // in -> forward -> state; -> inverse -> out
  COL_Z_UPDATE = 3,    // in -> forward -> k-space update of state -> inverse -> out
  COL_Z_INV_STATE = 4, // state -> inverse -> out
  COL_Z_ETD = 5,       // as COL_Z_UPDATE with the exponential (ETD1) update
  COL_Z_AC = 6,        // as COL_Z_UPDATE for the Allen-Cahn model (semi-implicit)
  COL_Z_AC_ETD = 7,    // Allen-Cahn, exponential (ETD1) update
  COL_Z_VM = 8         // in -> forward -> x dt / (1 + c4 K2^2) -> inverse -> out (no state)
};

// row (x) pass modes
enum : int {
  ROW_FUSED = 0,  // complex row -> inverse x -> f' -> forward x -> complex row
  ROW_FWD = 1,    // real row -> forward x -> complex row
  ROW_INV = 2,    // complex row -> inverse x -> real row
  ROW_FWD_FP = 3, // real row -> f'(c) -> forward x -> complex row (adjoint: T[f'(c)])
  ROW_FUSED_REC = 4, // ROW_FUSED that also stores the real row it passes through (out_r)
  ROW_INV_ADD = 5,   // ROW_INV that adds the real row to out_r instead of storing it
  ROW_FUSED_POLY = 6 // ROW_FUSED with the cubic poly(c) of RowArgs in place of f'(c)
};

// A column pass transforms nseq = 8 nouter sequences: sequence s is column s % 8 of outer index
// o = s / 8 = o_hi n_lo + o_lo, o_hi the x group (x = 8 o_hi + s % 8) and o_lo the other axis
// (z for the y pass, y for the z pass); x_lo = 1 would make o_lo the x group instead.
struct ColArgs {
  const float2* in;
  float2* out;
  float2* state;
  long long nseq;          // sequences = 8 * nouter
  int n_lo;                // outer indices per x group
  int nlive;               // x columns holding data (8 o_hi + column < nlive)
  long long stride_lo;     // float2 stride of o_lo
  long long stride_hi;     // float2 stride of o_hi (>= (n_lo - 1) stride_lo: offsets increase)
  int x_lo;                // 1: o_lo is the x group, 0: o_hi is
  int vlen;                // vertex-centred axis: its data length n (the transform length is
                           // 2(n - 1)): loads mirror point k > n - 1 to row 2(n - 1) - k, stores
                           // keep points below n; 0 otherwise
  long long row_stride;    // float2 stride between consecutive points of the transform axis
  const float2* tw;        // exp(-2 pi i j / N), j < N
  const float2* mk;        // zero flux: exp(-i pi k / (2N)), k < N
  const float* k2c;        // K2 along x: nx/2+1 entries, or nx for zero flux
  const float* k2o;        // K2 along the o_lo axis
  const float* k2r;        // K2 along the transform axis
  float a_dt;              // A dt
  float dt_m_kappa;        // dt M kappa
  float dt_m;              // dt M
  int remap;               // XCD-aware block order
  int xcomplex;            // z pass: a column is one complex x bin (else two real x bins)
  unsigned lane_bytes;     // bytes addressable from a point's block base (col_lane_bytes)
};

struct RowArgs {
  const float2* in_c;  // spectral rows (grouped layout, SpecGeom sg)
  const float* in_r;   // real rows (natural order)
  float2* out_c;
  float* out_r;
  SpecGeom sg;
  long long nrows;     // rows of nx real points (ny * nz)
  const float2* tw;    // row FFT twiddles
  const float2* post;  // periodic: exp(-2 pi i k / nx), k <= nx/2; zero flux: exp(-i pi k/(2 nx))
  float scale;         // 1/V (periodic) or 1/(8V) (zero flux), applied after the inverse
  int flip;            // Dirichlet axes (bit 0 x, 1 y, 2 z): real rows carry (-1)^(their index)
  int ny;              // rows r = j + ny l (for the sign)
  int remap;           // XCD-aware block order (consecutive row blocks on one XCD)
  int xcplx;           // cosine x: spectral columns are complex, one per bin (real data)
  int vx;              // vertex-centred x: real rows of vx = NH + 1 points, extended evenly
  float poly[4];       // ROW_FUSED_POLY: poly(c) = poly[0] + poly[1] c + poly[2] c^2 + poly[3] c^3
};

// (-1)^(i [x Dirichlet] + j [y Dirichlet] + l [z Dirichlet]) of point i of row r = j + ny l
EVX_HD float dirichlet_sign(long long r, int i, int ny, int mask) {
  const long long l = r / ny;
  const int j = int(r - l * ny);
  const int par = ((mask & 1) ? i : 0) + ((mask & 2) ? j : 0) + ((mask & 4) ? int(l & 1) : 0);
  return (par & 1) ? -1.0f : 1.0f;
}

// One launch of the same transform pass over up to four independent (in, out) buffer pairs: the
// grid's y index selects the pair (the small-grid adjoint and the two-species model run their
// transforms this way, which halves their launches).
constexpr int kMaxBatch = 4;
struct PassBatch {
  const void* in[kMaxBatch];
  void* out[kMaxBatch];
  int n;
};
EVX_HD void bind_batch(ColArgs& a, const PassBatch& b, int k) {
  a.in = static_cast<const float2*>(b.in[k]);
  a.out = static_cast<float2*>(b.out[k]);
}
// forward modes read real rows and write complex ones; the inverse does the opposite
EVX_HD void bind_batch(RowArgs& a, bool inverse, const PassBatch& b, int k) {
  if (inverse) {
    a.in_c = static_cast<const float2*>(b.in[k]);
    a.out_r = static_cast<float*>(b.out[k]);
  } else {
    a.in_r = static_cast<const float*>(b.in[k]);
    a.out_c = static_cast<float2*>(b.out[k]);
  }
}

// Block order: consecutive logical blocks (neighbouring columns, sharing 128-byte lines) are
// placed on the same XCD.  Hardware dispatches block i to XCD i % 8.
EVX_DEV int remap_block(int bid, int nblk, int on) {
  if (!on) return bid;
  const int per = nblk / 8;
  if (bid >= per * 8) return bid;
  return (bid % 8) * per + bid / 8;
}

EVX_DEV float fprime(float c) { return c * c * c - c; }

// The fused x pass's pointwise nonlinearity: f'(c) = c^3 - c, or a cubic polynomial (Horner form
// with explicit fused multiply-adds) for the reaction-diffusion step.
template <int MODE>
EVX_DEV float2 row_nonlin(const RowArgs& a, float2 v) {
  if constexpr (MODE == ROW_FUSED_POLY) {
    auto p = [&](float c) {
      return __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(a.poly[3], c, a.poly[2]), c, a.poly[1]),
                            c, a.poly[0]);
    };
    return make_float2(p(v.x), p(v.y));
  } else {
    return make_float2(fprime(v.x), fprime(v.y));
  }
}

// Index of the cell-centred input point that becomes point n of Makhoul's reordered sequence
// (v_n = x_{2n} for 2n < N, else x_{2N-2n-1}).
template <int N>
constexpr int makhoul_src(int n) {
  return (2 * n < N) ? 2 * n : 2 * N - 2 * n - 1;
}

// ------------------------------------------------------------------ column pass
template <int N>
struct ColCfg {
  static constexpr int E = FftPlan<N>::E;
  static constexpr int TPS = FftPlan<N>::TPS;
  static constexpr int B = seqs_per_block<N>();
  static constexpr int THREADS = B * TPS;
  static constexpr int TW = B * N;             // twiddle table offset (after the exchange area)
  static constexpr int K2 = TW + N;             // z update: K2 along the transform axis (floats)
  static constexpr int LDS = K2 + (N + 1) / 2;  // float2 slots
};

// src[i] if ok, else zero, with the load outside any branch: a load inside a divergent branch is
// waited for before the branch joins, which would make a lane's loads one round trip each.  The
// address is clamped to element 0 (which every caller guarantees valid) when ok is false, and the
// value is cleared with a bit mask rather than a select (the compiler turns a select of a loaded
// value into a branch around the load).
EVX_DEV float evx_keep(float v, unsigned mask) {
  return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, v) & mask);
}
EVX_DEV float2 load_or_zero(const float2* EVX_RESTRICT src, long long i, bool ok) {
  const float2 v = src[ok ? i : 0];
  const unsigned m = ok ? ~0u : 0u;
  return make_float2(evx_keep(v.x, m), evx_keep(v.y, m));
}
EVX_DEV float load_or_zero(const float* EVX_RESTRICT src, long long i, bool ok) {
  return evx_keep(src[ok ? i : 0], ok ? ~0u : 0u);
}

// A block's copy of a small constant table (COUNT entries) staged in LDS: every lane issues its
// table loads before the data loads (load) and writes them to LDS after (store), so the table
// latency overlaps the data latency.  Readers come after a barrier.
template <int COUNT, int T, class V>
struct TableStage {
  static constexpr int IT = (COUNT + T - 1) / T;
  V r[IT > 0 ? IT : 1];
  EVX_DEV void load(const V* EVX_RESTRICT src, int tid) {
    static_for<IT>([&](auto I) {
      const int i = tid + T * decltype(I)::value;
      r[I] = src[i < COUNT ? i : 0];
    });
  }
  EVX_DEV void store(V* dst, int tid) const {
    static_for<IT>([&](auto I) {
      const int i = tid + T * decltype(I)::value;
      if (i < COUNT) dst[i] = r[I];
    });
  }
};

// The N-entry FFT twiddle table; a single-stage transform reads none (its first read is in the
// second stage, which follows a barrier).
template <int N, int T>
using TwStage = TableStage<(FftPlan<N>::S > 1 ? N : 0), T, float2>;

// Zero flux, after a forward FFT of packed columns (a + i b): x holds Z[k], k = t + TPS e.
// Produces (Da[k], Db[k]) with D[k] = 2 sum_n x_n cos(pi k (2n+1) / 2N) (Makhoul).
template <int N, int B>
EVX_DEV void makhoul_post(float2 (&x)[FftPlan<N>::E], float2* lds, int b, int t,
                          const float2* EVX_RESTRICT mk) {
  constexpr int E = FftPlan<N>::E, TPS = FftPlan<N>::TPS;
  static_for<E>([&](auto e) { lds[lidx<B>(t + TPS * decltype(e)::value, b)] = x[e]; });
  evx_sync();
  static_for<E>([&](auto e) {
    const int k = t + TPS * decltype(e)::value;
    const int kr = (k == 0) ? 0 : N - k;
    const float2 P = x[e];
    const float2 Q = cconj(lds[lidx<B>(kr, b)]);
    const float2 w = mk[k];
    const float2 sp = cmul(w, cadd(P, Q));
    const float2 sm = cmul(w, csub(P, Q));
    x[e] = make_float2(sp.x, sm.y);
  });
  evx_sync();
}

// Zero flux, before an inverse FFT: x holds (Da[k], Db[k]); produces
// Z[k] = Va[k] + i Vb[k],  V[k] = exp(i pi k / 2N) (D[k] - i D[N-k]),  D[N] = 0.
template <int N, int B>
EVX_DEV void makhoul_pre(float2 (&x)[FftPlan<N>::E], float2* lds, int b, int t,
                         const float2* EVX_RESTRICT mk) {
  constexpr int E = FftPlan<N>::E, TPS = FftPlan<N>::TPS;
  static_for<E>([&](auto e) { lds[lidx<B>(t + TPS * decltype(e)::value, b)] = x[e]; });
  evx_sync();
  static_for<E>([&](auto e) {
    const int k = t + TPS * decltype(e)::value;
    const float2 D = x[e];
    const float2 Dr = (k == 0) ? make_float2(0.f, 0.f) : lds[lidx<B>(N - k, b)];
    const float2 w = cconj(mk[k]);
    const float2 va = cmul(w, make_float2(D.x, -Dr.x));
    const float2 vb = cmul(w, make_float2(D.y, -Dr.y));
    x[e] = make_float2(va.x - vb.y, va.y + vb.x);
  });
  evx_sync();
}

// Addressing of one block's B sequences.  For each point index e the block has a uniform base
// (scalar registers: a buffer resource) and every lane adds one 32-bit byte offset, the same for
// all its points.  A lane without data gets an offset past the resource's range, so its loads
// read zero and its stores are dropped without touching memory: no branches and no shared
// addresses.  Zero-flux reordered accesses (row makhoul_src(n) for point n) use the lowest row of
// the point group as base and a non-negative lane-dependent row shift.
constexpr unsigned kDeadLane = 0xfffffff0u;

// Bound on the bytes any lane addresses from a point base; the launchers check that it is below
// kDeadLane and that sequence numbers fit in 31 bits.
template <int N>
inline long long col_lane_bytes(const ColArgs& a) {
  constexpr int B = ColCfg<N>::B, TPS = ColCfg<N>::TPS;
  static_assert(B % 8 == 0, "a block covers whole outer indices");
  // outer indices o0 .. o0 + qmax of one block: at most qmax / n_lo + 1 group steps and qmax
  // steps of o_lo (offsets increase with o, see ColArgs)
  const long long qmax = B / 8 - 1;
  const long long cmax = qmax == 0 ? 7 : (qmax / a.n_lo + 1) * a.stride_hi + qmax * a.stride_lo + 7;
  // a point base plus t rows, a Makhoul row shift (< 2 TPS rows), or a vertex axis's data row
  // (< N / 2 + 1 rows) from the point-0 base: N rows cover all of them (N >= 2 TPS)
  return (cmax + (long long)N * a.row_stride + 2) * 8;
}

template <int N>
constexpr int makhoul_group_min(int e) {
  int m = N;
  for (int t = 0; t < FftPlan<N>::TPS; ++t) {
    const int r = makhoul_src<N>(t + FftPlan<N>::TPS * e);
    m = r < m ? r : m;
  }
  return m;
}

template <int N, int B>
struct ColTile {
  static constexpr int TPS = FftPlan<N>::TPS;
  long long tb = 0;  // float2 offset of the block's first sequence (uniform)
  unsigned lo = 0;   // lane byte offset of point 0 relative to tb, or kDeadLane
  unsigned lc = 0;   // lane byte offset of its column (row 0) relative to tb
  int olo = 0, x = 0, t = 0;  // the lane's o_lo index and x column
  long long tile = 0;
  unsigned so = 0;   // lane byte offset in the tile-major state (or kDeadLane)
  bool live = false;
  EVX_DEV void locate(const ColArgs& a, long long tile_, int b, int t_) {
    static_assert(B % 8 == 0, "a block covers whole outer indices");
    t = t_;
    tile = tile_;
    const unsigned n_lo = unsigned(a.n_lo);
    const unsigned s0 = unsigned(tile) * unsigned(B);
    const unsigned o0 = s0 >> 3;                 // first outer index of the block (column 0)
    const unsigned h0 = o0 / n_lo, l0 = o0 - h0 * n_lo;
    tb = (long long)h0 * a.stride_hi + (long long)l0 * a.stride_lo;
    const unsigned o = o0 + (unsigned(b) >> 3);  // the lane's outer index and column
    const unsigned c = unsigned(b) & 7u;
    const unsigned h = o / n_lo, l = o - h * n_lo;
    olo = int(l);
    x = int((a.x_lo ? l : h) * 8 + c);
    live = (long long)s0 + b < a.nseq && x < a.nlive;
    const long long cofs = (long long)(h - h0) * a.stride_hi +
                           ((long long)l - (long long)l0) * a.stride_lo + c;
    lc = unsigned(cofs * 8);
    lo = live ? unsigned((cofs + (long long)t * a.row_stride) * 8) : kDeadLane;
    so = live ? unsigned((t * B + b) * 8) : kDeadLane;
  }
  // The spectral state is stored tile-major: tile, then transform point k, then column b, at
  // (tile N + k) B + b, so that a block's state is one contiguous N B run (read and written only
  // by the z pass).  Point t + TPS e of lane (t, b): uniform base plus the lane offset `so`.
  EVX_DEV evx_buf sres(const float2* state, int e) const {
    return evx_make_buf(state + tile * ((long long)N * B) + (long long)(TPS * e) * B,
                        unsigned(TPS * B * 8));
  }
  // vertex-centred axis: lane offset of data row `row` from the point-0 base
  EVX_DEV unsigned voff(long long row_stride, int row) const {
    return live ? lc + unsigned((long long)row * row_stride * 8) : kDeadLane;
  }
  // point t + TPS e (natural order)
  EVX_DEV evx_buf res(const float2* base, long long row_stride, int e, unsigned nbytes) const {
    return evx_make_buf(base + tb + (long long)(TPS * e) * row_stride, nbytes);
  }
  // point t + TPS e stored at row makhoul_src(t + TPS e): base row of the group and lane shift
  template <int E_>
  EVX_DEV evx_buf res_m(const float2* base, long long row_stride, unsigned nbytes) const {
    constexpr int gmin = makhoul_group_min<N>(E_);
    return evx_make_buf(base + tb + (long long)gmin * row_stride, nbytes);
  }
  template <int E_>
  EVX_DEV unsigned off_m(long long row_stride) const {
    constexpr int gmin = makhoul_group_min<N>(E_);
    const int sh = makhoul_src<N>(t + TPS * E_) - gmin;
    return live ? lc + unsigned((long long)sh * row_stride * 8) : kDeadLane;
  }
};

template <int N, int BC, int MODE>
EVX_DEV void colpass_body(const ColArgs& a, int tid, int bid, int nblk, float2* lds) {
  using C = ColCfg<N>;
  constexpr int E = C::E, TPS = C::TPS, B = C::B;
  constexpr bool upd =
      MODE == COL_Z_UPDATE || MODE == COL_Z_ETD || MODE == COL_Z_AC || MODE == COL_Z_AC_ETD;
  constexpr bool vm = MODE == COL_Z_VM;
  constexpr bool kt = upd || vm;  // needs the K2 tables
  constexpr bool has_fwd = MODE == COL_FWD || MODE == COL_Z_INIT || kt;
  constexpr bool has_inv = MODE != COL_FWD;
  constexpr bool zf = BC == BC_ZERO_FLUX;
  const int b = tid % B;
  const int t = tid / B;
  const unsigned nb = a.lane_bytes;
  ColTile<N, B> ct;
  ct.locate(a, remap_block(bid, nblk, a.remap), b, t);

  // Tables first (they go to LDS after the data loads), then the data and for the update the
  // column K2, all in flight together.
  float2* const twl = lds + C::TW;
  TwStage<N, C::THREADS> tws;
  tws.load(a.tw, tid);
  float* const k2l = reinterpret_cast<float*>(lds + C::K2);
  TableStage<(kt ? N : 0), C::THREADS, float> k2s;
  if constexpr (kt) k2s.load(a.k2r, tid);

  float2 x[E];
  if constexpr (MODE == COL_Z_INV_STATE) {
    static_for<E>([&](auto e) { x[e] = evx_buf_load2(ct.sres(a.state, e), ct.so); });
  } else if constexpr (zf && has_fwd) {
    static_for<E>([&](auto e) {
      constexpr int ev = decltype(e)::value;
      x[e] = evx_buf_load2(ct.template res_m<ev>(a.in, a.row_stride, nb),
                           ct.template off_m<ev>(a.row_stride));
    });
  } else if (!zf && a.vlen) {
    // vertex-centred axis: the even extension about both end points, point n > vlen - 1 read
    // from data row N - n (N = 2 (vlen - 1))
    const evx_buf r0 = ct.res(a.in, a.row_stride, 0, nb);
    static_for<E>([&](auto e) {
      const int n = t + TPS * decltype(e)::value;
      x[e] = evx_buf_load2(r0, ct.voff(a.row_stride, n < a.vlen ? n : N - n));
    });
  } else {
    static_for<E>([&](auto e) { x[e] = evx_buf_load2(ct.res(a.in, a.row_stride, e, nb), ct.lo); });
  }
  // vertex-centred axis: keep points k < vlen (the rest of the extension mirrors them)
  auto store_points = [&](float2* out) {
    if (a.vlen) {
      const evx_buf r0 = ct.res(out, a.row_stride, 0, nb);
      static_for<E>([&](auto e) {
        const int k = t + TPS * decltype(e)::value;
        evx_buf_store2(r0, k < a.vlen ? ct.voff(a.row_stride, k) : kDeadLane, x[e]);
      });
    } else {
      static_for<E>([&](auto e) {
        evx_buf_store2(ct.res(out, a.row_stride, e, nb), ct.lo, x[e]);
      });
    }
  };
  float kca = 0.f, kcb = 0.f;
  if constexpr (kt) {
    const int o = ct.live ? ct.olo : 0, cc = ct.live ? ct.x : 0;
    const float ko = a.k2o[o];
    // Pair columns (two real x bins) occur under a cosine x whose y and z spectra stay real: a
    // cosine z, or a vertex-centred z (periodic transform of an even extension).
    if (a.xcomplex) {  // both components belong to x bin cc
      kca = a.k2c[cc] + ko;
      kcb = kca;
    } else {           // two real x bins per column
      kca = a.k2c[2 * cc] + ko;
      kcb = a.k2c[2 * cc + 1] + ko;
    }
  }
  tws.store(twl, tid);
  k2s.store(k2l, tid);

  if constexpr (has_fwd) {
    fft_regs<N, -1, B>(x, lds, b, t, twl);
    if constexpr (zf) makhoul_post<N, B>(x, lds, b, t, a.mk);
  }

  if constexpr (MODE == COL_FWD) {
    if constexpr (zf) {
      static_for<E>([&](auto e) {
        evx_buf_store2(ct.res(a.out, a.row_stride, e, nb), ct.lo, x[e]);
      });
    } else {
      store_points(a.out);
    }
    return;
  }

  if constexpr (MODE == COL_Z_INIT) {
    static_for<E>([&](auto e) {
      evx_buf_store2(ct.sres(a.state, e), ct.so, x[e]);
    });
  }

  if constexpr (vm) {
    // Increment multiplier of the variable-mobility step, x <- dt x / (1 + c4 K2^2): dt travels
    // in dt_m and c4 = 2 dt gamma0 eps M0 in dt_m_kappa.  No state.
    evx_sync();  // K2 table visible
    static_for<E>([&](auto e) {
      const int k = t + TPS * decltype(e)::value;
      const float kr = k2l[k];
      const float K2a = kca + kr, K2b = kcb + kr;
      x[e] = make_float2(a.dt_m * x[e].x / (1.0f + a.dt_m_kappa * K2a * K2a),
                         a.dt_m * x[e].y / (1.0f + a.dt_m_kappa * K2b * K2b));
    });
  }

  if constexpr (upd) {
    // C' = G (P C - dt M K2 F), P = 1 + A dt K2, G = 1 / (1 + dt M kappa K2^2 + A dt K2).
    // The library is built without FP contraction, so the rounded C' stored in the state is
    // exactly the value the inverse transform consumes, and every kernel that transforms the
    // same data rounds identically (resume from a stored state is bit-exact).
    evx_sync();  // K2 table visible (a single-stage periodic transform has no barrier of its own)
    // The state is read only now: loading it with the data would hold 32 more registers
    // through the forward transform and cost a block per compute unit.
    float2 cs[E];
    static_for<E>([&](auto e) {
      cs[e] = evx_buf_load2(ct.sres(a.state, e), ct.so);
    });
    static_for<E>([&](auto e) {
      const int k = t + TPS * decltype(e)::value;
      const float kr = k2l[k];
      const float2 Cs = cs[e];
      const float2 F = x[e];
      const float K2a = kca + kr, K2b = kcb + kr;
      if constexpr (MODE == COL_Z_ETD) {
        // C' = C + phi1(dt S) dt R, dt S = -(dt M kappa K2^2 + A dt K2),
        // dt R = -(dt M K2 F + dt M kappa K2^2 C); phi1(0) = 1 keeps the DC bin exact
        const float sa = -(a.dt_m_kappa * K2a * K2a + a.a_dt * K2a);
        const float sb = -(a.dt_m_kappa * K2b * K2b + a.a_dt * K2b);
        const float pa = evx_phi1(sa), pb = evx_phi1(sb);
        const float ra = -(a.dt_m * K2a * F.x + a.dt_m_kappa * K2a * K2a * Cs.x);
        const float rb = -(a.dt_m * K2b * F.y + a.dt_m_kappa * K2b * K2b * Cs.y);
        x[e] = make_float2(Cs.x + pa * ra, Cs.y + pb * rb);
      } else if constexpr (MODE == COL_Z_AC) {
        // Allen-Cahn: C' = G (P C - dt M F), P = 1 + A dt, G = 1 / (1 + A dt + dt M kappa K2)
        const float P = 1.0f + a.a_dt;
        const float Ga = evx_rcp(P + a.dt_m_kappa * K2a), Gb = evx_rcp(P + a.dt_m_kappa * K2b);
        x[e] = make_float2(Ga * (P * Cs.x - a.dt_m * F.x), Gb * (P * Cs.y - a.dt_m * F.y));
      } else if constexpr (MODE == COL_Z_AC_ETD) {
        // Allen-Cahn ETD1: C' = C + phi1(dt S) dt R, dt S = -(dt M kappa K2 + A dt),
        // dt R = -(dt M F + dt M kappa K2 C)
        const float sa = -(a.dt_m_kappa * K2a + a.a_dt), sb = -(a.dt_m_kappa * K2b + a.a_dt);
        const float ra = -(a.dt_m * F.x + a.dt_m_kappa * K2a * Cs.x);
        const float rb = -(a.dt_m * F.y + a.dt_m_kappa * K2b * Cs.y);
        x[e] = make_float2(Cs.x + evx_phi1(sa) * ra, Cs.y + evx_phi1(sb) * rb);
      } else {
        const float Pa = 1.0f + a.a_dt * K2a, Pb = 1.0f + a.a_dt * K2b;
        const float Ga = evx_rcp(1.0f + a.dt_m_kappa * K2a * K2a + a.a_dt * K2a);
        const float Gb = evx_rcp(1.0f + a.dt_m_kappa * K2b * K2b + a.a_dt * K2b);
        x[e] = make_float2(Ga * (Pa * Cs.x - a.dt_m * K2a * F.x),
                           Gb * (Pb * Cs.y - a.dt_m * K2b * F.y));
      }
      evx_buf_store2(ct.sres(a.state, e), ct.so, x[e]);
    });
  }

  if constexpr (has_inv) {
    if constexpr (zf) makhoul_pre<N, B>(x, lds, b, t, a.mk);
    fft_regs<N, +1, B>(x, lds, b, t, twl);
    if constexpr (zf) {
      static_for<E>([&](auto e) {
        constexpr int ev = decltype(e)::value;
        evx_buf_store2(ct.template res_m<ev>(a.out, a.row_stride, nb),
                       ct.template off_m<ev>(a.row_stride), x[e]);
      });
    } else {
      store_points(a.out);
    }
  }
}

// ------------------------------------------------------------------ row pass
// Cooperative copies between the block's contiguous slice of global memory and LDS.  Every load
// of a thread is issued before its first LDS write, so a wave waits on memory once per copy
// rather than once per element.  `valid` is the number of in-range float2 (ragged last block).
template <int COUNT, int T>
EVX_DEV void copy_in(const float2* EVX_RESTRICT src, long long valid, float2* lds, int tid) {
  constexpr int IT = (COUNT + T - 1) / T;
  float2 r[IT];
  static_for<IT>([&](auto I) {
    const int i = tid + T * decltype(I)::value;
    r[I] = load_or_zero(src, i, i < COUNT && i < valid);
  });
  static_for<IT>([&](auto I) {
    const int i = tid + T * decltype(I)::value;
    if (i < COUNT) lds[i] = r[I];
  });
}

template <int COUNT, int T, bool ADD = false>
EVX_DEV void copy_out(float2* EVX_RESTRICT dst, long long valid, const float2* lds, int tid) {
  constexpr int IT = (COUNT + T - 1) / T;
  static_for<IT>([&](auto I) {
    const int i = tid + T * decltype(I)::value;
    if (i < COUNT && i < valid) {
      if constexpr (ADD) {
        const float2 o = dst[i], v = lds[i];
        dst[i] = make_float2(o.x + v.x, o.y + v.y);
      } else {
        dst[i] = lds[i];
      }
    }
  });
}

// Vertex-centred x: ROWS real rows of NR = NH + 1 floats, contiguous in the field (the block's
// slice starts at src), copied into LDS as floats; `valid` floats are in range.
template <int COUNT, int T>
EVX_DEV void copy_in_floats(const float* EVX_RESTRICT src, long long valid, float* lds, int tid) {
  constexpr int IT = (COUNT + T - 1) / T;
  float r[IT];
  static_for<IT>([&](auto I) {
    const int i = tid + T * decltype(I)::value;
    r[I] = load_or_zero(src, i, i < COUNT && i < valid);
  });
  static_for<IT>([&](auto I) {
    const int i = tid + T * decltype(I)::value;
    if (i < COUNT) lds[i] = r[I];
  });
}

// ... and back: row b of the block holds the 2 NH points of the extension at lds[b 2 NH + j]; the
// first NR = NH + 1 of them are the field's row (stored, or added with ADD).
template <int ROWS, int NH, int T, bool ADD>
EVX_DEV void copy_out_vertex(float* EVX_RESTRICT dst, long long valid_rows, const float* lds,
                             int tid) {
  constexpr int NR = NH + 1, COUNT = ROWS * NR, IT = (COUNT + T - 1) / T;
  static_for<IT>([&](auto I) {
    const int i = tid + T * decltype(I)::value;
    const int row = i / NR, j = i - row * NR;
    if (i < COUNT && row < valid_rows) {
      const float v = lds[row * 2 * NH + j];
      if constexpr (ADD) {
        dst[i] = dst[i] + v;
      } else {
        dst[i] = v;
      }
    }
  });
}

// Periodic complex rows: ROWS rows of NLIVE values at global pitch P are staged at LDS row
// stride S.  T / ROWS consecutive lanes copy one row, so every global access is a contiguous run
// within a row; the row padding is skipped on the way in and written as zeros on the way out.
template <int ROWS, int P, int S, int NLIVE, int T>
EVX_DEV void rows_in(const float2* EVX_RESTRICT src, long long valid_rows, float2* lds, int tid) {
  static_assert(T % ROWS == 0, "rows must split the block evenly");
  constexpr int TR = T / ROWS, IT = (NLIVE + TR - 1) / TR;
  const int row = tid / TR, c0 = tid - row * TR;
  const bool ok = row < valid_rows;
  float2 r[IT];
  static_for<IT>([&](auto I) {
    const int c = c0 + TR * decltype(I)::value;
    r[I] = load_or_zero(src, (long long)row * P + c, ok && c < NLIVE);
  });
  static_for<IT>([&](auto I) {
    const int c = c0 + TR * decltype(I)::value;
    if (c < NLIVE) lds[row * S + c] = r[I];
  });
}

template <int ROWS, int P, int S, int NLIVE, int T, bool ADD = false>
EVX_DEV void rows_out(float2* EVX_RESTRICT dst, long long valid_rows, const float2* lds, int tid) {
  static_assert(T % ROWS == 0, "rows must split the block evenly");
  constexpr int TR = T / ROWS, IT = (P + TR - 1) / TR;
  const int row = tid / TR, c0 = tid - row * TR;
  if (row >= valid_rows) return;
  static_for<IT>([&](auto I) {
    const int c = c0 + TR * decltype(I)::value;
    if constexpr (ADD) {  // real rows only: NLIVE == P, no padding
      static_assert(NLIVE == P, "adding rows have no padding");
      if (c < P) {
        const float2 o = dst[row * P + c], v = lds[row * S + c];
        dst[row * P + c] = make_float2(o.x + v.x, o.y + v.y);
      }
    } else {
      if (c < P) dst[row * P + c] = (c < NLIVE) ? lds[row * S + c] : make_float2(0.f, 0.f);
    }
  });
}

// Spectral rows (grouped layout) <-> LDS: rows r0 .. r0 + ROWS - 1 (those below valid_rows) of
// NL live float2 each, staged at LDS row stride S.  Eight consecutive lanes move one row's 64-byte
// piece of one x group and 8 ROWS consecutive lanes that group for all the block's rows, so rows
// that share a z plane move one contiguous ROWS x 64-byte run per group.  Every load is issued
// before the first LDS write.  Dead columns of the last group are written as zeros.
template <int ROWS, int NL>
struct SpecRowsCfg {
  static constexpr int NG = (NL + 7) / 8;  // x groups
  static constexpr int PER = 8 * ROWS;     // float2 of one group for all rows
  static constexpr int TOT = NG * PER;
};

// With T a multiple of 8 ROWS (>= 64) a lane keeps its row and column across iterations and the
// x group is the same for a whole wave: each group's slab is then a buffer resource with a
// wave-uniform base and the lane adds one 32-bit offset (no per-element 64-bit addresses).
// Within a wave the 64 lanes move rows 8 w .. 8 w + 7 (w = wave index mod ROWS / 8) of one group,
// lane l taking column l % 8 of row 2 ((l / 8) % 4) + l / 32: the same 512 contiguous bytes per
// wave as the plain order, but the two halves of the wave write (and read) the LDS rows
// {0, 2, 4, 6} and {1, 3, 5, 7}, whose 64-byte segments fall in disjoint banks at the staging
// strides used here.
template <int ROWS, int NL, int T>
struct SpecRowsLane {
  using RC = SpecRowsCfg<ROWS, NL>;
  static constexpr bool FIXED = (T % RC::PER) == 0 && RC::PER % 64 == 0;
  int c, row;
  long long zbase;  // float2 offset of the z plane of the block's first row (uniform)
  unsigned off;     // byte offset of the lane's element from zbase + group, or kDeadLane
  unsigned range;   // bytes addressable from zbase + group: the planes the block's rows reach
  EVX_DEV SpecRowsLane(const SpecGeom& sg, long long r0, long long valid_rows, int tid) {
    const int l = tid & 63;
    c = l & 7;
    row = 8 * ((tid >> 6) % (ROWS / 8)) + 2 * ((l >> 3) & 3) + (l >> 5);
    const long long z0 = r0 / sg.ny;
    const int y0 = int(r0 - z0 * sg.ny);
    zbase = z0 * sg.zstride;
    range = unsigned((ROWS / sg.ny + 2) * sg.zstride * 8);
    off = row < valid_rows ? unsigned((spec_row_offset_from(sg, 0, y0, row) + c) * 8)
                           : kDeadLane;
  }
  // x group of iteration I (wave-uniform)
  template <int I>
  EVX_DEV int group(int tid) const {
    return evx_wave_uniform(tid / RC::PER) + (T / RC::PER) * I;
  }
};

// RE: the columns are complex values whose real part is the data (a cosine x transform under a
// periodic y or z): only the real parts are staged, as floats at row stride S.
template <int ROWS, int S, int NL, int T, bool RE = false>
EVX_DEV void spec_rows_in(const float2* EVX_RESTRICT src, const SpecGeom& sg, long long r0,
                          long long valid_rows, float2* lds, int tid) {
  auto put = [&](int row, int x, float2 v) {
    if constexpr (RE) {
      reinterpret_cast<float*>(lds)[row * S + x] = v.x;
    } else {
      lds[row * S + x] = v;
    }
  };
  using RC = SpecRowsCfg<ROWS, NL>;
  using LN = SpecRowsLane<ROWS, NL, T>;
  static_assert(T % 8 == 0, "lanes move whole 8-column pieces");
  constexpr int IT = (RC::TOT + T - 1) / T;
  float2 r[IT];
  if constexpr (LN::FIXED) {
    const LN ln(sg, r0, valid_rows, tid);
    static_for<IT>([&](auto I) {
      const int g = ln.template group<decltype(I)::value>(tid);
      const bool ok = g < RC::NG && g * 8 + ln.c < NL;
      r[I] = evx_buf_load2(evx_make_buf(src + ln.zbase + g * sg.xstride, ln.range),
                           ok ? ln.off : kDeadLane);
    });
    static_for<IT>([&](auto I) {
      const int g = ln.template group<decltype(I)::value>(tid);
      if (g < RC::NG && g * 8 + ln.c < NL) put(ln.row, g * 8 + ln.c, r[I]);
    });
    return;
  }
  const int c = tid & 7;
  const long long z0 = r0 / sg.ny;
  const int y0 = int(r0 - z0 * sg.ny);
  static_for<IT>([&](auto I) {
    const int f = tid + T * decltype(I)::value;
    const int g = f / RC::PER;
    const int row = (f >> 3) % ROWS;
    const bool ok = f < RC::TOT && row < valid_rows && g * 8 + c < NL;
    r[I] = load_or_zero(src, g * sg.xstride + spec_row_offset_from(sg, z0, y0, row) + c, ok);
  });
  static_for<IT>([&](auto I) {
    const int f = tid + T * decltype(I)::value;
    const int g = f / RC::PER;
    const int row = (f >> 3) % ROWS;
    if (f < RC::TOT && g * 8 + c < NL) put(row, g * 8 + c, r[I]);
  });
}

template <int ROWS, int S, int NL, int T, bool RE = false>
EVX_DEV void spec_rows_out(float2* EVX_RESTRICT dst, const SpecGeom& sg, long long r0,
                           long long valid_rows, const float2* lds, int tid) {
  auto get = [&](int row, int x) {
    if constexpr (RE) {
      return make_float2(reinterpret_cast<const float*>(lds)[row * S + x], 0.f);
    } else {
      return lds[row * S + x];
    }
  };
  using RC = SpecRowsCfg<ROWS, NL>;
  using LN = SpecRowsLane<ROWS, NL, T>;
  static_assert(T % 8 == 0, "lanes move whole 8-column pieces");
  constexpr int IT = (RC::TOT + T - 1) / T;
  if constexpr (LN::FIXED) {
    const LN ln(sg, r0, valid_rows, tid);
    static_for<IT>([&](auto I) {
      const int g = ln.template group<decltype(I)::value>(tid);
      const int x = g * 8 + ln.c;
      const float2 v = x < NL ? get(ln.row, x) : make_float2(0.f, 0.f);
      evx_buf_store2(evx_make_buf(dst + ln.zbase + g * sg.xstride, ln.range),
                     g < RC::NG ? ln.off : kDeadLane, v);
    });
    return;
  }
  const int c = tid & 7;
  const long long z0 = r0 / sg.ny;
  const int y0 = int(r0 - z0 * sg.ny);
  static_for<IT>([&](auto I) {
    const int f = tid + T * decltype(I)::value;
    const int g = f / RC::PER;
    const int row = (f >> 3) % ROWS;
    if (f < RC::TOT && row < valid_rows) {
      const int x = g * 8 + c;
      dst[g * sg.xstride + spec_row_offset_from(sg, z0, y0, row) + c] =
          x < NL ? get(row, x) : make_float2(0.f, 0.f);
    }
  });
}

// LDS row stride for B rows read by lanes (t, b) at row b, column t + const: the smallest
// S >= need with S = q (mod 2q), q = 32 / min(B, 32), so that the 32 lanes of a half wave touch
// distinct 64-bit bank pairs.
constexpr int row_lds_stride(int need, int b) {
  const int q = 32 / (b < 32 ? b : 32);
  int s = need;
  while (s % (2 * q) != q % (2 * q)) ++s;
  return s;
}

// Periodic: template length NH = nx/2, the complex FFT length of the packed real row; the row
// has NH+1 complex points.  Zero flux: NH = nx, one sequence carries two rows packed as a + i b.
template <int NH, int BC>
struct RowCfg {
  static constexpr int E = FftPlan<NH>::E;
  static constexpr int TPS = FftPlan<NH>::TPS;
  static constexpr int B = seqs_per_block<NH>();       // sequences per block
  static constexpr int THREADS = B * TPS;
  static constexpr int ROWS = (BC == BC_PERIODIC) ? B : 2 * B;  // rows per block
  static constexpr int SROW = row_lds_stride(NH + 1, B);  // periodic LDS row stride
  // zero flux: 2B rows of NH floats staged at a float stride ZS with ZS/2 odd (rows 2b of the
  // lanes b then fall in distinct banks), when the rows split the block's lanes evenly
  static constexpr bool ZPAD = (THREADS % (2 * B)) == 0;
  static constexpr int ZS = (!ZPAD || NH % 4 == 2) ? NH : NH + 2;
  static constexpr int STAGE = (BC == BC_PERIODIC) ? B * SROW : B * ZS;  // float2 slots
  static constexpr int TW = STAGE > B * NH ? STAGE : B * NH;  // twiddle table offset
  static constexpr int PO = TW + NH;                            // post table offset
  // post table entries: periodic keeps k <= NH/2 (the rest follows from
  // exp(-2 pi i (NH - k) / nx) = -conj(exp(-2 pi i k / nx))); zero flux keeps all NH
  static constexpr int NPOST = (BC == BC_PERIODIC) ? NH / 2 + 1 : NH;
  static constexpr int LDS = PO + NPOST;
};

// Periodic post-processing twiddle exp(-2 pi i k / nx), nx = 2 NH, 0 <= k < NH, from the half
// table held in LDS.
template <int NH>
EVX_DEV float2 post_tw(const float2* po, int k) {
  if (k <= NH / 2) return po[k];
  const float2 w = po[NH - k];
  return make_float2(-w.x, w.y);
}

template <int NH, int BC, int MODE>
EVX_DEV void rowpass_body(const RowArgs& a, int tid, int bid, int nblk, float2* lds) {
  using C = RowCfg<NH, BC>;
  constexpr int E = C::E, TPS = C::TPS, B = C::B, T = C::THREADS;
  const int b = tid % B;
  const int t = tid / B;
  // consecutive row blocks (their 8-row pieces of each x group are neighbours) on one XCD
  const long long r0 = (long long)remap_block(bid, nblk, a.remap) * C::ROWS;
  float2 x[E];
  float2* const twl = lds + C::TW;
  float2* const pol = lds + C::PO;
  TwStage<NH, T> tws;
  tws.load(a.tw, tid);
  TableStage<C::NPOST, T, float2> pos;
  pos.load(a.post, tid);

  if constexpr (BC == BC_PERIODIC) {
    constexpr int NX = 2 * NH, W = C::SROW;
    // ---------------------------------------------------------------- input
    if constexpr (MODE == ROW_FWD || MODE == ROW_FWD_FP) {
      if (a.vx) {
        // vertex-centred x: rows of NH + 1 points, extended evenly about both end points to the
        // 2 NH points the real transform takes: point j > NH is point 2 NH - j
        float* st = reinterpret_cast<float*>(lds);
        copy_in_floats<B * (NH + 1), T>(a.in_r + r0 * (NH + 1), (a.nrows - r0) * (NH + 1), st,
                                        tid);
        tws.store(twl, tid);
        pos.store(pol, tid);
        evx_sync();
        const float* row = st + b * (NH + 1);
        static_for<E>([&](auto e) {
          const int j = 2 * (t + TPS * decltype(e)::value);
          x[e] = make_float2(row[j <= NH ? j : 2 * NH - j], row[j + 1 <= NH ? j + 1 : 2 * NH - j - 1]);
        });
      } else {
        // real rows, read as pairs (c[2n], c[2n+1]) into stage[b*NH + n]
        copy_in<B * NH, T>(reinterpret_cast<const float2*>(a.in_r) + r0 * NH,
                           (a.nrows - r0) * NH, lds, tid);
        tws.store(twl, tid);
        pos.store(pol, tid);
        evx_sync();
        static_for<E>([&](auto e) { x[e] = lds[b * NH + t + TPS * decltype(e)::value]; });
      }
      if (a.flip) {  // Dirichlet y / z: one sign per row
        const float sg = dirichlet_sign(r0 + b, 0, a.ny, a.flip);
        static_for<E>([&](auto e) { x[e] = cscale(x[e], sg); });
      }
      if constexpr (MODE == ROW_FWD_FP)
        static_for<E>([&](auto e) { x[e] = make_float2(fprime(x[e].x), fprime(x[e].y)); });
      evx_sync();
    } else {
      spec_rows_in<B, W, NH + 1, T>(a.in_c, a.sg, r0, a.nrows - r0, lds, tid);
      tws.store(twl, tid);
      pos.store(pol, tid);
      evx_sync();
      // C2R pre-processing: Z[k] = (X[k] + conj X[NH-k]) + i (X[k] - conj X[NH-k]) e^{+2pi i k/NX}
      static_for<E>([&](auto e) {
        const int k = t + TPS * decltype(e)::value;
        const float2 X = lds[b * W + k];
        const float2 Xr = cconj(lds[b * W + NH - k]);
        const float2 Ev = cadd(X, Xr);
        const float2 Od = cmulc(csub(X, Xr), post_tw<NH>(pol, k));
        x[e] = make_float2(Ev.x - Od.y, Ev.y + Od.x);
      });
      evx_sync();
      fft_regs<NH, +1, B>(x, lds, b, t, twl);
      static_for<E>([&](auto e) { x[e] = cscale(x[e], a.scale); });
      if constexpr (MODE == ROW_INV || MODE == ROW_INV_ADD || MODE == ROW_FUSED_REC) {
        const float sg = a.flip ? dirichlet_sign(r0 + b, 0, a.ny, a.flip) : 1.0f;
        static_for<E>([&](auto e) {
          lds[b * NH + t + TPS * decltype(e)::value] = a.flip ? cscale(x[e], sg) : x[e];
        });
        evx_sync();
        if (a.vx)
          copy_out_vertex<B, NH, T, MODE == ROW_INV_ADD>(a.out_r + r0 * (NH + 1), a.nrows - r0,
                                                         reinterpret_cast<const float*>(lds), tid);
        else
          copy_out<B * NH, T, MODE == ROW_INV_ADD>(reinterpret_cast<float2*>(a.out_r) + r0 * NH,
                                                   (a.nrows - r0) * NH, lds, tid);
        if constexpr (MODE == ROW_INV || MODE == ROW_INV_ADD) return;
        evx_sync();  // the forward transform reuses the staging area
      }
      static_for<E>([&](auto e) { x[e] = row_nonlin<MODE>(a, x[e]); });
    }
    // ---------------------------------------------------------------- forward x (R2C)
    fft_regs<NH, -1, B>(x, lds, b, t, twl);
    static_for<E>([&](auto e) { lds[lidx<B>(t + TPS * decltype(e)::value, b)] = x[e]; });
    evx_sync();
    float2 y[E];
    float2 ynyq = make_float2(0.f, 0.f);
    static_for<E>([&](auto e) {
      const int k = t + TPS * decltype(e)::value;
      const float2 P = x[e];
      const float2 Q = cconj(lds[lidx<B>(k == 0 ? 0 : NH - k, b)]);
      const float2 Ev = cscale(cadd(P, Q), 0.5f);
      const float2 dq = cscale(csub(P, Q), 0.5f);
      const float2 Od = make_float2(dq.y, -dq.x);  // -i (P - Q) / 2
      y[e] = cadd(Ev, cmul(post_tw<NH>(pol, k), Od));
      if (k == 0) ynyq = make_float2(Ev.x - Od.x, 0.f);
    });
    evx_sync();
    static_for<E>([&](auto e) { lds[b * W + t + TPS * decltype(e)::value] = y[e]; });
    if (t == 0) lds[b * W + NH] = ynyq;
    evx_sync();
    spec_rows_out<B, W, NH + 1, T>(a.out_c, a.sg, r0, a.nrows - r0, lds, tid);
    (void)NX;
  } else {
    // zero flux: rows ra = r0 + 2b, rb = ra + 1, staged as floats [2B][ZS]
    constexpr int NX = NH, ZS = C::ZS;
    float* st = reinterpret_cast<float*>(lds);
    constexpr bool real_in = MODE == ROW_FWD || MODE == ROW_FWD_FP;
    constexpr int SS = C::ZPAD ? ZS / 2 : NX / 2;  // LDS row stride in float2
    // rows are NX floats (NX even) = NX/2 float2; r0 is even
    if constexpr (!real_in) {
      if (a.xcplx)  // complex columns, one per bin (a periodic y or z follows)
        spec_rows_in<2 * B, ZS, NX, T, true>(a.in_c, a.sg, r0, a.nrows - r0, lds, tid);
      else
        spec_rows_in<2 * B, SS, NX / 2, T>(a.in_c, a.sg, r0, a.nrows - r0, lds, tid);
    } else if constexpr (C::ZPAD) {
      rows_in<2 * B, NX / 2, ZS / 2, NX / 2, T>(
          reinterpret_cast<const float2*>(a.in_r) + r0 * (NX / 2), a.nrows - r0, lds, tid);
    } else {
      copy_in<B * NX, T>(reinterpret_cast<const float2*>(a.in_r) + r0 * (NX / 2),
                         (a.nrows - r0) * (NX / 2), lds, tid);
    }
    tws.store(twl, tid);
    pos.store(pol, tid);
    evx_sync();
    if constexpr (real_in) {
      static_for<E>([&](auto e) {
        const int n = t + TPS * decltype(e)::value;
        const int s = makhoul_src<NX>(n);
        x[e] = make_float2(st[(2 * b) * ZS + s], st[(2 * b + 1) * ZS + s]);
        if (a.flip) {
          const long long ra = r0 + 2 * b;
          x[e] = make_float2(x[e].x * dirichlet_sign(ra, s, a.ny, a.flip),
                             x[e].y * dirichlet_sign(ra + 1, s, a.ny, a.flip));
        }
      });
      if constexpr (MODE == ROW_FWD_FP)
        static_for<E>([&](auto e) { x[e] = make_float2(fprime(x[e].x), fprime(x[e].y)); });
      evx_sync();
    } else {
      static_for<E>([&](auto e) {
        const int k = t + TPS * decltype(e)::value;
        const float Da = st[(2 * b) * ZS + k], Db = st[(2 * b + 1) * ZS + k];
        const float Dar = (k == 0) ? 0.f : st[(2 * b) * ZS + NX - k];
        const float Dbr = (k == 0) ? 0.f : st[(2 * b + 1) * ZS + NX - k];
        const float2 w = cconj(pol[k]);
        const float2 va = cmul(w, make_float2(Da, -Dar));
        const float2 vb = cmul(w, make_float2(Db, -Dbr));
        x[e] = make_float2(va.x - vb.y, va.y + vb.x);
      });
      evx_sync();
      fft_regs<NX, +1, B>(x, lds, b, t, twl);
      static_for<E>([&](auto e) { x[e] = cscale(x[e], a.scale); });
      if constexpr (MODE == ROW_INV || MODE == ROW_INV_ADD || MODE == ROW_FUSED_REC) {
        static_for<E>([&](auto e) {
          const int n = t + TPS * decltype(e)::value;
          const int s = makhoul_src<NX>(n);
          float va = x[e].x, vb = x[e].y;
          if (a.flip) {
            const long long ra = r0 + 2 * b;
            va *= dirichlet_sign(ra, s, a.ny, a.flip);
            vb *= dirichlet_sign(ra + 1, s, a.ny, a.flip);
          }
          st[(2 * b) * ZS + s] = va;
          st[(2 * b + 1) * ZS + s] = vb;
        });
        evx_sync();
        if constexpr (C::ZPAD) {
          rows_out<2 * B, NX / 2, ZS / 2, NX / 2, T, MODE == ROW_INV_ADD>(
              reinterpret_cast<float2*>(a.out_r) +
                                                         r0 * (NX / 2),
                                                     a.nrows - r0, lds, tid);
        } else {
          copy_out<B * NX, T, MODE == ROW_INV_ADD>(reinterpret_cast<float2*>(a.out_r) +
                                                       r0 * (NX / 2),
                                                   (a.nrows - r0) * (NX / 2), lds, tid);
        }
        if constexpr (MODE == ROW_INV || MODE == ROW_INV_ADD) return;
        evx_sync();  // the forward transform reuses the staging area
      }
      static_for<E>([&](auto e) { x[e] = row_nonlin<MODE>(a, x[e]); });
    }
    fft_regs<NX, -1, B>(x, lds, b, t, twl);
    static_for<E>([&](auto e) { lds[lidx<B>(t + TPS * decltype(e)::value, b)] = x[e]; });
    evx_sync();
    float2 y[E];
    static_for<E>([&](auto e) {
      const int k = t + TPS * decltype(e)::value;
      const float2 P = x[e];
      const float2 Q = cconj(lds[lidx<B>(k == 0 ? 0 : NX - k, b)]);
      const float2 w = pol[k];
      const float2 sp = cmul(w, cadd(P, Q));
      const float2 sm = cmul(w, csub(P, Q));
      y[e] = make_float2(sp.x, sm.y);
    });
    evx_sync();
    static_for<E>([&](auto e) {
      const int k = t + TPS * decltype(e)::value;
      st[(2 * b) * ZS + k] = y[e].x;
      st[(2 * b + 1) * ZS + k] = y[e].y;
    });
    evx_sync();
    if (a.xcplx)
      spec_rows_out<2 * B, ZS, NX, T, true>(a.out_c, a.sg, r0, a.nrows - r0, lds, tid);
    else
      spec_rows_out<2 * B, SS, NX / 2, T>(a.out_c, a.sg, r0, a.nrows - r0, lds, tid);
  }
}

// ------------------------------------------------------------------ plane pass (small grids)
// On a grid whose xy spectral plane fits in LDS, one workgroup per z plane runs the step's first
// three passes on that plane in place: it reads the plane's NH + 1 complex x bins of NY rows once,
// runs the inverse y transforms, the fused x pass (inverse x, f', forward x) and the forward y
// transforms, and writes the plane back once.  Three launches and three trips through memory
// become one, which is what bounds a step on such grids (every launch carries a few microseconds
// of load-transform-store latency).  The transforms use the same twiddle tables and operation
// order as the column and row passes they replace (and their FFT plans where PlanePlans says so).
// Periodic x and y (and z) only.
struct PlaneArgs {
  float2* W;            // work buffer (grouped layout), read and written in place
  SpecGeom sg;
  int nz, ngx;
  const float2* tw_y;   // exp(-2 pi i j / NY)
  const float2* tw_x;   // exp(-2 pi i j / NH)
  const float2* post;   // exp(-2 pi i k / (2 NH)), k <= NH / 2
  float scale;          // 1 / (nx ny nz), applied after the inverse x transform
};

// Per plane size: the FFT plans of the y and x transforms (those of the column and row passes, so
// the results are bitwise theirs) and the lanes of the workgroup, chosen so that one batch covers
// all NH + 1 columns and all NY rows (every lane is a (sequence, part) pair in both) and the
// exchange area fits beside the plane.  Measured on 128 x 128 planes the pass lost to the three
// separate ones (27 us against about 22 us for the three: 128 workgroups fill half the chip), so
// it stops at 64 x 64.
template <int NY, int NH>
struct PlanePlans;
template <>
struct PlanePlans<32, 16> {  // 17 columns x 4 lanes, 32 rows x 1 lane
  using PY = FftPlan<32>;
  using PX = FftPlan<16>;
  static constexpr int THREADS = 68;
};
template <>
struct PlanePlans<64, 32> {  // 64 columns x 16 lanes, 256 rows x 4 lanes
  using PY = FftPlan<64>;
  using PX = FftPlan<32>;
  static constexpr int THREADS = 1024;
};

template <int NY, int NH>
struct PlaneCfg {
  using PY = typename PlanePlans<NY, NH>::PY;
  using PX = typename PlanePlans<NY, NH>::PX;
  static constexpr int THREADS = PlanePlans<NY, NH>::THREADS;
  static constexpr int EY = PY::E, TY = PY::TPS;
  static constexpr int EX = PX::E, TX = PX::TPS;
  static_assert(THREADS % TY == 0 && THREADS % TX == 0, "lanes split into whole sequences");
  static constexpr int NC = NH + 1;                       // live x bins
  // sequences per batch: every lane takes part in every transform (they hold barriers), and
  // lanes past the live columns or rows work on zeros and store nothing
  static constexpr int BY = THREADS / TY;                 // y columns per batch
  static constexpr int BX = THREADS / TX;                 // x rows per batch
  static constexpr int PW = NC % 2 ? NC : NC + 1;        // plane row pitch (odd: rows in distinct banks)
  static constexpr int PLANE = NY * PW;
  static constexpr int XCH = BY * NY > BX * NH ? BY * NY : BX * NH;  // FFT exchange area
  static constexpr int TWY = PLANE + XCH, TWX = TWY + NY, PO = TWX + NH;
  static constexpr int NPOST = NH / 2 + 1;
  static constexpr int LDS = PO + NPOST;  // float2 slots
  static constexpr int LOADS = (((NC + 7) / 8) * NY * 8 + THREADS - 1) / THREADS;
};

template <int NY, int NH>
EVX_DEV void planepass_body(const PlaneArgs& a, int tid, int bid, float2* lds) {
  using C = PlaneCfg<NY, NH>;
  constexpr int T = C::THREADS, PW = C::PW, NC = C::NC;
  float2* const P = lds;
  float2* const xch = lds + C::PLANE;
  float2* const twy = lds + C::TWY;
  float2* const twx = lds + C::TWX;
  float2* const pol = lds + C::PO;
  const long long zoff = (long long)bid * a.sg.zstride;  // plane z = bid, group 0
  // tables and the plane, all loads in flight together; group g's rows are one contiguous run
  TableStage<NY, T, float2> sty;
  sty.load(a.tw_y, tid);
  TableStage<NH, T, float2> stx;
  stx.load(a.tw_x, tid);
  TableStage<C::NPOST, T, float2> spo;
  spo.load(a.post, tid);
  constexpr int GRUN = NY * 8;  // float2 of one group's rows of the plane
  float2 r[C::LOADS];
  static_for<C::LOADS>([&](auto I) {
    const int f = tid + T * decltype(I)::value;
    const int g = f / GRUN, rem = f - g * GRUN;
    const bool ok = g < a.ngx;
    r[I] = load_or_zero(a.W, g * a.sg.xstride + zoff + rem, ok);
  });
  sty.store(twy, tid);
  stx.store(twx, tid);
  spo.store(pol, tid);
  static_for<C::LOADS>([&](auto I) {
    const int f = tid + T * decltype(I)::value;
    const int g = f / GRUN, rem = f - g * GRUN;
    const int col = g * 8 + (rem & 7), y = rem >> 3;
    if (g < a.ngx && col < NC) P[y * PW + col] = r[I];
  });
  evx_sync();

  // y transforms of the live columns, C::BY at a time (dir +1 inverse, -1 forward)
  auto y_pass = [&](auto dir_) {
    constexpr int DIR = decltype(dir_)::value;
    constexpr int B = C::BY, E = C::EY, TPS = C::TY;
    const int b = tid % B, t = tid / B;
    for (int c0 = 0; c0 < NC; c0 += B) {  // uniform
      const int col = c0 + b;
      const bool live = col < NC;
      float2 x[E];
      static_for<E>([&](auto e) {
        const int yy = t + TPS * decltype(e)::value;
        x[e] = live ? P[yy * PW + (live ? col : 0)] : make_float2(0.f, 0.f);
      });
      fft_regs<NY, DIR, B, typename C::PY>(x, xch, b, t, twy);
      if (live)
        static_for<E>([&](auto e) { P[(t + TPS * decltype(e)::value) * PW + col] = x[e]; });
      evx_sync();  // the next batch reuses the exchange area
    }
  };
  y_pass(std::integral_constant<int, +1>{});

  // fused x pass on rows of NH + 1 complex bins (the periodic row pass's arithmetic)
  {
    constexpr int B = C::BX, E = C::EX, TPS = C::TX;
    const int b = tid % B, t = tid / B;
    for (int y0 = 0; y0 < NY; y0 += B) {  // uniform
      const bool act = y0 + b < NY;
      float2* const row = P + (act ? y0 + b : 0) * PW;
      float2 x[E];
      // C2R pre-processing: Z[k] = (X[k] + conj X[NH-k]) + i (X[k] - conj X[NH-k]) e^{+2pi i k/NX}
      static_for<E>([&](auto e) {
        const int k = t + TPS * decltype(e)::value;
        if (act) {
          const float2 X = row[k];
          const float2 Xr = cconj(row[NH - k]);
          const float2 Ev = cadd(X, Xr);
          const float2 Od = cmulc(csub(X, Xr), post_tw<NH>(pol, k));
          x[e] = make_float2(Ev.x - Od.y, Ev.y + Od.x);
        } else {
          x[e] = make_float2(0.f, 0.f);
        }
      });
      fft_regs<NH, +1, B, typename C::PX>(x, xch, b, t, twx);
      static_for<E>([&](auto e) { x[e] = cscale(x[e], a.scale); });
      static_for<E>([&](auto e) { x[e] = make_float2(fprime(x[e].x), fprime(x[e].y)); });
      fft_regs<NH, -1, B, typename C::PX>(x, xch, b, t, twx);
      static_for<E>([&](auto e) { xch[lidx<B>(t + TPS * decltype(e)::value, b)] = x[e]; });
      evx_sync();
      float2 yv[E];
      float2 ynyq = make_float2(0.f, 0.f);
      static_for<E>([&](auto e) {
        const int k = t + TPS * decltype(e)::value;
        const float2 Pk = x[e];
        const float2 Q = cconj(xch[lidx<B>(k == 0 ? 0 : NH - k, b)]);
        const float2 Ev = cscale(cadd(Pk, Q), 0.5f);
        const float2 dq = cscale(csub(Pk, Q), 0.5f);
        const float2 Od = make_float2(dq.y, -dq.x);  // -i (P - Q) / 2
        yv[e] = cadd(Ev, cmul(post_tw<NH>(pol, k), Od));
        if (k == 0) ynyq = make_float2(Ev.x - Od.x, 0.f);
      });
      evx_sync();  // the exchange area is read; the next batch (or y pass) may write it
      if (act) {
        static_for<E>([&](auto e) { row[t + TPS * decltype(e)::value] = yv[e]; });
        if (t == 0) row[NH] = ynyq;
      }
    }
    evx_sync();
  }
  y_pass(std::integral_constant<int, -1>{});

  // write the plane back; the dead columns of the last group are written as zeros
  static_for<C::LOADS>([&](auto I) {
    const int f = tid + T * decltype(I)::value;
    const int g = f / GRUN, rem = f - g * GRUN;
    const int col = g * 8 + (rem & 7), y = rem >> 3;
    if (g < a.ngx)
      a.W[g * a.sg.xstride + zoff + rem] = col < NC ? P[y * PW + col] : make_float2(0.f, 0.f);
  });
}

}  // namespace evx
