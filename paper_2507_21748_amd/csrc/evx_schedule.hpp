// Host-side geometry, tables and pass schedule of the spectral CH step.  Shared by the HIP
// launcher and by the host emulator used in the CPU tests, so both run the same sequence of
// passes with the same arguments.
#pragma once

#include <cmath>
#include <cstddef>
#include <vector>

#include "evx_passes.hpp"

namespace evx {

// Supported transform lengths (every FftPlan specialisation).  A test build may predefine a
// shorter list.
#ifndef EVX_FOR_EACH_N
#define EVX_FOR_EACH_N(X) \
  X(4) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(50) X(64) X(80) X(96) \
  X(100) X(128) X(160) X(192) X(200) X(256) X(320) X(384) X(400) X(512) X(1024)
#endif

inline bool fft_len_supported(int n) {
  switch (n) {
#define EVX_CASE(N) case N:
    EVX_FOR_EACH_N(EVX_CASE)
#undef EVX_CASE
    return true;
    default:
      return false;
  }
}

// Sequences per column-pass block for a transform length (0 if unsupported).
inline int col_block_seqs(int n) {
  switch (n) {
#define EVX_CASE(N) \
  case N:           \
    return ColCfg<N>::B;
    EVX_FOR_EACH_N(EVX_CASE)
#undef EVX_CASE
    default:
      return 0;
  }
}

struct Geom {
  int nx = 0, ny = 0, nz = 0;   // points per axis (the data)
  int vert = 0;          // vertex-centred zero-flux axes (bit 0 x, 1 y, 2 z): the transform is the
                         // periodic one of the even extension about the end points, length 2(n-1)
  int nxe = 0;           // x length of the periodic transform family: nx, or 2(nx - 1) (vertex x)
  int fy = 0, fz = 0;    // y and z transform lengths: ny, nz, or 2(n - 1) for a vertex axis
  int bc = BC_PERIODIC;  // x transform family: Dirichlet axes run the zero-flux kernels
  int bcy = BC_PERIODIC, bcz = BC_PERIODIC;  // y and z transform families
  int flip = 0;          // Dirichlet (DST-II) axes, bit 0 x, 1 y, 2 z: sign and reversed K2
  int scheme = 0;        // 0 spectral, 1 stencil7
  double dx = 1.0;       // grid spacing baked into the K2 tables
  long long V = 0;       // voxels
  int xcplx = 0;         // cosine x under a periodic y or z: one complex column per x bin
  int ncols = 0;         // float2 x columns of a spectral buffer holding data
  int ngx = 0;           // x groups of 8 columns (grouped spectral layout, evx_passes.hpp)
  int ypitch = 0;        // rows per (group, z) slab: ny + kSpecYPad
  int row_len = 0;       // x-pass FFT length: nx/2 (periodic) or nx (zero flux)
  long long spec = 0;    // float2 per spectral buffer (work W): ngx nz ypitch 8
  long long state = 0;   // float2 of the state S (tile-major; whole z-pass tiles)
  long long nrows = 0;   // ny * nz
  int plane_ny = 0;      // > 0: the step's y, x, y passes run as one plane pass (planepass_body)
};

// Plane pass sizes: square periodic xy planes of 32 or 64 points (planepass_body).
inline bool plane_pass_supported(int nx, int ny) { return nx == ny && (ny == 32 || ny == 64); }

// Per-axis boundaries: any mix of periodic, zero flux (cell- or vertex-centred) and Dirichlet.
// A vertex-centred axis runs the periodic transform of the field's even extension about its end
// points (length 2(n - 1): the DCT-I), so it joins the periodic transform family; its spectrum is
// real, and the extension is formed and cut in the passes that touch real data.
inline Geom make_geom3(int nx, int ny, int nz, int bcx, int bcy, int bcz, int scheme, double dx) {
  Geom g;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.flip = (bcx == BC_DIRICHLET ? 1 : 0) | (bcy == BC_DIRICHLET ? 2 : 0) |
           (bcz == BC_DIRICHLET ? 4 : 0);
  g.vert = (bcx == BC_VERTEX ? 1 : 0) | (bcy == BC_VERTEX ? 2 : 0) | (bcz == BC_VERTEX ? 4 : 0);
  auto family = [](int b) { return (b == BC_PERIODIC || b == BC_VERTEX) ? BC_PERIODIC : BC_ZERO_FLUX; };
  const int bc = family(bcx);
  g.bc = bc;
  g.bcy = family(bcy);
  g.bcz = family(bcz);
  g.nxe = (g.vert & 1) ? 2 * (nx - 1) : nx;
  g.fy = (g.vert & 2) ? 2 * (ny - 1) : ny;
  g.fz = (g.vert & 4) ? 2 * (nz - 1) : nz;
  g.scheme = scheme;
  g.dx = dx;
  g.V = (long long)nx * ny * nz;
  // a cosine x keeps two real bins per float2 column, unless a (truly) periodic y or z transform
  // follows, whose complex output needs one complex column per bin; a vertex y or z keeps the
  // spectrum real, like a cosine one
  g.xcplx = (bc != BC_PERIODIC && (bcy == BC_PERIODIC || bcz == BC_PERIODIC)) ? 1 : 0;
  g.ncols = (bc == BC_PERIODIC) ? g.nxe / 2 + 1 : (g.xcplx ? nx : nx / 2);
  g.row_len = (bc == BC_PERIODIC) ? g.nxe / 2 : nx;
  g.ngx = (g.ncols + 7) / 8;
  g.ypitch = ny + kSpecYPad;
  g.spec = (long long)g.ngx * nz * g.ypitch * 8;
  const long long bz = col_block_seqs(g.fz), nseq_z = (long long)g.ngx * ny * 8;
  g.state = bz > 0 ? (nseq_z + bz - 1) / bz * bz * g.fz : g.spec;
  g.nrows = (long long)ny * nz;
  g.plane_ny = (bcx == BC_PERIODIC && bcy == BC_PERIODIC && bcz == BC_PERIODIC &&
                plane_pass_supported(nx, ny)) ? ny : 0;
  return g;
}

// Host copies of every table, FP64-computed and rounded once.
struct HostTables {
  std::vector<float2> tw_x, tw_y, tw_z;  // exp(-2 pi i j / N) for the x-row, y and z FFT lengths
  std::vector<float2> post_x;            // periodic exp(-2 pi i k / nx), k <= nx/2; zf below
  std::vector<float2> mk_x, mk_y, mk_z;  // zero flux exp(-i pi k / (2N)), k < N
  std::vector<float> k2_x, k2_y, k2_z;   // per-axis K2
};

inline std::vector<float2> twiddles(int n) {
  std::vector<float2> t(n);
  for (int j = 0; j < n; ++j) {
    const double a = -2.0 * M_PI * double(j) / double(n);
    t[j] = make_float2(float(std::cos(a)), float(std::sin(a)));
  }
  return t;
}

inline std::vector<float2> makhoul_twiddles(int n) {
  std::vector<float2> t(n);
  for (int k = 0; k < n; ++k) {
    const double a = -M_PI * double(k) / (2.0 * double(n));
    t[k] = make_float2(float(std::cos(a)), float(std::sin(a)));
  }
  return t;
}

// Eigenvalue of -d2/dx2 for mode m on an axis of n cells (periodic: k = 2 pi m'/(n dx), zero
// flux: k = pi m / (n dx)); spectral k^2 or 3-point stencil (4/dx^2) sin^2(k dx / 2).
inline double axis_k2(int m, int n, int bc, int scheme, double dx) {
  double k;
  if (bc == BC_PERIODIC) {
    const int mp = (m <= n / 2) ? m : m - n;
    k = 2.0 * M_PI * double(mp) / (double(n) * dx);
  } else {
    k = M_PI * double(m) / (double(n) * dx);
  }
  if (scheme == 0) return k * k;
  const double s = std::sin(0.5 * k * dx);
  return 4.0 / (dx * dx) * s * s;
}

inline Geom make_geom(int nx, int ny, int nz, int bc, int scheme, double dx) {
  return make_geom3(nx, ny, nz, bc, bc, bc, scheme, dx);
}

// Dirichlet: bin j of the zero-flux transform of the sign-alternated field holds sine mode n - j
inline std::vector<float> k2_table(int count, int n, int bc, int scheme, double dx,
                                   bool dirichlet = false) {
  std::vector<float> t(count);
  for (int m = 0; m < count; ++m)
    t[m] = float(axis_k2(dirichlet ? n - m : m, n, bc, scheme, dx));
  return t;
}

inline HostTables make_tables(const Geom& g) {
  HostTables h;
  h.tw_x = twiddles(g.row_len);
  h.tw_y = twiddles(g.fy);
  h.tw_z = twiddles(g.fz);
  if (g.bc == BC_PERIODIC) {
    // a vertex x: the periodic tables of its extension (length nxe), whose wavenumbers
    // 2 pi m / (nxe dx) are the cosine modes pi m / ((nx - 1) dx)
    h.post_x.resize(g.nxe / 2 + 1);
    for (int k = 0; k <= g.nxe / 2; ++k) {
      const double a = -2.0 * M_PI * double(k) / double(g.nxe);
      h.post_x[k] = make_float2(float(std::cos(a)), float(std::sin(a)));
    }
    h.k2_x = k2_table(g.nxe / 2 + 1, g.nxe, g.bc, g.scheme, g.dx);
  } else {
    h.post_x = makhoul_twiddles(g.nx);
    h.k2_x = k2_table(g.nx, g.nx, g.bc, g.scheme, g.dx, (g.flip & 1) != 0);
  }
  if (g.bcy != BC_PERIODIC) h.mk_y = makhoul_twiddles(g.ny);
  if (g.bcz != BC_PERIODIC) h.mk_z = makhoul_twiddles(g.nz);
  h.k2_y = k2_table(g.fy, g.fy, g.bcy, g.scheme, g.dx, (g.flip & 2) != 0);
  h.k2_z = k2_table(g.fz, g.fz, g.bcz, g.scheme, g.dx, (g.flip & 4) != 0);
  return h;
}

// Pointers to the tables as the kernels see them (device or host copies).
struct TablePtrs {
  const float2 *tw_x, *tw_y, *tw_z, *post_x, *mk_y, *mk_z;
  const float *k2_x, *k2_y, *k2_z;
};

struct StepCoef {
  float a_dt, dt_m_kappa, dt_m;
};

inline SpecGeom spec_geom(const Geom& g) {
  return SpecGeom{(long long)g.nz * g.ypitch * 8, (long long)g.ypitch * 8, g.ny};
}

// y pass: outer index (x group, z); the points of a column are 8 float2 apart, so a block's
// columns are one contiguous run of ny x 64 bytes.
inline ColArgs y_args(const Geom& g, const TablePtrs& t, const float2* in, float2* out,
                      int remap) {
  ColArgs a{};
  a.in = in;
  a.out = out;
  a.nseq = (long long)g.ngx * g.nz * 8;
  a.n_lo = g.nz;
  a.nlive = g.ncols;
  a.stride_lo = (long long)g.ypitch * 8;
  a.stride_hi = (long long)g.nz * g.ypitch * 8;
  a.x_lo = 0;
  a.row_stride = 8;
  a.vlen = (g.vert & 2) ? g.ny : 0;
  a.tw = t.tw_y;
  a.mk = t.mk_y;
  a.remap = remap;
  return a;
}

// z pass: outer index (x group, y); points ypitch x 64 bytes apart.
inline ColArgs z_args(const Geom& g, const TablePtrs& t, const float2* in, float2* out,
                      float2* state, StepCoef c, int remap) {
  ColArgs a{};
  a.in = in;
  a.out = out;
  a.state = state;
  a.nseq = (long long)g.ngx * g.ny * 8;
  a.n_lo = g.ny;
  a.nlive = g.ncols;
  a.stride_lo = 8;
  a.stride_hi = (long long)g.nz * g.ypitch * 8;
  a.x_lo = 0;
  a.row_stride = (long long)g.ypitch * 8;
  a.vlen = (g.vert & 4) ? g.nz : 0;
  a.tw = t.tw_z;
  a.mk = t.mk_z;
  a.k2c = t.k2_x;
  a.k2o = t.k2_y;
  a.k2r = t.k2_z;
  a.a_dt = c.a_dt;
  a.dt_m_kappa = c.dt_m_kappa;
  a.dt_m = c.dt_m;
  a.remap = remap;
  a.xcomplex = (g.bc == BC_PERIODIC || g.xcplx) ? 1 : 0;
  return a;
}

inline RowArgs x_args(const Geom& g, const TablePtrs& t, const float2* in_c, const float* in_r,
                      float2* out_c, float* out_r) {
  RowArgs a{};
  a.in_c = in_c;
  a.in_r = in_r;
  a.out_c = out_c;
  a.out_r = out_r;
  a.sg = spec_geom(g);
  a.xcplx = g.xcplx;
  a.nrows = g.nrows;
  a.tw = t.tw_x;
  a.post = t.post_x;
  // inverse normalisation: 1/n per periodic axis, 1/(2n) per cosine (DCT-III of DCT-II) axis,
  // 1/(2(n - 1)) per vertex axis (the periodic length of its extension)
  auto len = [](int n, int family, bool vertex) {
    return vertex ? 2.0 * (n - 1) : (family == BC_PERIODIC ? double(n) : 2.0 * n);
  };
  a.scale = float(1.0 / (len(g.nx, g.bc, g.vert & 1) * len(g.ny, g.bcy, g.vert & 2) *
                         len(g.nz, g.bcz, g.vert & 4)));
  a.flip = g.flip;
  a.ny = g.ny;
  a.remap = 1;
  a.vx = (g.vert & 1) ? g.nx : 0;
  return a;
}

inline PlaneArgs plane_args(const Geom& g, const TablePtrs& t, float2* W) {
  PlaneArgs a{};
  a.W = W;
  a.sg = spec_geom(g);
  a.nz = g.nz;
  a.ngx = g.ngx;
  a.tw_y = t.tw_y;
  a.tw_x = t.tw_x;
  a.post = t.post_x;
  a.scale = x_args(g, t, W, nullptr, W, nullptr).scale;  // the row pass's normalisation
  return a;
}

// Launcher L provides col(N, bc, mode, ColArgs), row(NH, bc, mode, RowArgs) and
// plane(NY, PlaneArgs).

// Initial forward transform of the real field c: S <- T[c], W <- F_z^{-1} S.
template <class L>
void sched_begin(L& l, const Geom& g, const TablePtrs& t, const float* c, float2* S, float2* W,
                 int remap) {
  l.row(g.row_len, g.bc, ROW_FWD, x_args(g, t, nullptr, c, W, nullptr));
  l.col(g.fy, g.bcy, COL_FWD, y_args(g, t, W, W, remap));
  l.col(g.fz, g.bcz, COL_Z_INIT, z_args(g, t, W, W, S, StepCoef{0, 0, 0}, remap));
}

// nsteps steps; W must hold F_z^{-1} S on entry and holds it again on exit.
template <class L>
void sched_advance(L& l, const Geom& g, const TablePtrs& t, float2* S, float2* W, StepCoef c,
                   int nsteps, int remap, int zmode = COL_Z_UPDATE) {
  for (int n = 0; n < nsteps; ++n) {
    if (g.plane_ny) {
      l.plane(g.plane_ny, plane_args(g, t, W));
    } else {
      l.col(g.fy, g.bcy, COL_INV, y_args(g, t, W, W, remap));
      l.row(g.row_len, g.bc, ROW_FUSED, x_args(g, t, W, nullptr, W, nullptr));
      l.col(g.fy, g.bcy, COL_FWD, y_args(g, t, W, W, remap));
    }
    l.col(g.fz, g.bcz, zmode, z_args(g, t, W, W, S, c, remap));
  }
}

// Reaction-diffusion (dc/dt = D lap c + f(c), f cubic): the same four passes, the fused x pass
// evaluating poly = -f (ROW_FUSED_POLY) and the z pass the Allen-Cahn form of the update with
// M = 1, kappa = D: C' = ((1 + A dt) C + dt T[f]) / (1 + A dt + dt D K2).
template <class L>
void sched_advance_rd(L& l, const Geom& g, const TablePtrs& t, float2* S, float2* W, StepCoef c,
                      const float poly[4], int nsteps, int remap) {
  RowArgs xa = x_args(g, t, W, nullptr, W, nullptr);
  for (int k = 0; k < 4; ++k) xa.poly[k] = poly[k];
  for (int n = 0; n < nsteps; ++n) {
    l.col(g.fy, g.bcy, COL_INV, y_args(g, t, W, W, remap));
    l.row(g.row_len, g.bc, ROW_FUSED_POLY, xa);
    l.col(g.fy, g.bcy, COL_FWD, y_args(g, t, W, W, remap));
    l.col(g.fz, g.bcz, COL_Z_AC, z_args(g, t, W, W, S, c, remap));
  }
}

// As sched_advance, also recording the real field c^n at the start of each step into
// traj + n V (the fused x pass stores the row it passes through).
template <class L>
void sched_advance_record(L& l, const Geom& g, const TablePtrs& t, float2* S, float2* W,
                          StepCoef c, int nsteps, int remap, int zmode, float* traj) {
  for (int n = 0; n < nsteps; ++n) {
    l.col(g.fy, g.bcy, COL_INV, y_args(g, t, W, W, remap));
    l.row(g.row_len, g.bc, ROW_FUSED_REC, x_args(g, t, W, nullptr, W, traj + (long long)n * g.V));
    l.col(g.fy, g.bcy, COL_FWD, y_args(g, t, W, W, remap));
    l.col(g.fz, g.bcz, zmode, z_args(g, t, W, W, S, c, remap));
  }
}

// Real field from W = F_z^{-1} S (consumes W).
template <class L>
void sched_end(L& l, const Geom& g, const TablePtrs& t, float* c, float2* W, int remap) {
  l.col(g.fy, g.bcy, COL_INV, y_args(g, t, W, W, remap));
  l.row(g.row_len, g.bc, ROW_INV, x_args(g, t, W, nullptr, nullptr, c));
}

// W <- F_z^{-1} S (restores the loop-entry buffer from the state).
template <class L>
void sched_restore(L& l, const Geom& g, const TablePtrs& t, float2* S, float2* W, int remap) {
  l.col(g.fz, g.bcz, COL_Z_INV_STATE, z_args(g, t, nullptr, W, S, StepCoef{0, 0, 0}, remap));
}

}  // namespace evx
