// Element-wise and reduction passes used by the adjoint step and by the diagnostics.  Like the
// transform passes, each body is the work of one workgroup (gfx950 kernel or host emulator).
//
// Inner products of real fields are evaluated in the spectral domain (Parseval):
//   periodic, half spectrum:  sum_x a b = (1/V) sum_k w(kx) Re(A_k conj B_k),
//                             w = 1 for kx = 0 and kx = nx/2, else 2;
//   zero flux, DCT-II D_k = 2 sum_n x_n cos(pi k (2n+1) / 2N) per axis:
//                             sum_x a b = sum_k prod_axes w(k) A_k B_k,
//                             w(0) = 1/(4N), w(k > 0) = 1/(2N).
// Partial sums are FP64 and reduced in a fixed order, so results are bit-reproducible.
#pragma once

#include "evx_passes.hpp"

namespace evx {

constexpr int AUX_THREADS = 256;
// Fixed grid (fixed summation order).  The loops are grid-stride, so a test build may shrink it.
#ifndef EVX_AUX_BLOCKS
#define EVX_AUX_BLOCKS 1024
#endif
constexpr int AUX_BLOCKS = EVX_AUX_BLOCKS;

struct SpecArgs {
  const float2* C;  // T[c^n]
  float2* F;        // in: T[f'(c^n)];  out: dt M K2 G Lam   (the B operator's multiplier)
  float2* L;        // in: T[lam^{n+1}]; out: G P Lam        (the A operator's multiplier)
  long long n;      // float2 elements of a spectral buffer
  int nx, ny, nz, ypitch, ncols, bc;  // grouped spectral layout; ncols x columns hold data
  int xcplx;                          // cosine x with one complex column per bin
  int bcy, bcz;                      // y and z transform families (x periodic may mix them)
  const float *k2x, *k2y, *k2z;
  float a_dt, dt_m_kappa, dt_m, dt, dt_kappa;
  double* partial;  // 2 per block: sum for dL/dkappa, sum for dL/dM (before the 1/V factor)
  int mode;         // 0 adjoint, 1 energy (sum w K2 |C|^2 into partial[2b])
};

// Per-axis Parseval weight of the zero-flux (DCT-II) coefficient k on an axis of n cells.
EVX_DEV double dct_weight(int k, int n) { return (k == 0 ? 0.25 : 0.5) / double(n); }

template <int T>
EVX_DEV void block_sum2(double& s0, double& s1, int tid, double* red) {
  red[2 * tid] = s0;
  red[2 * tid + 1] = s1;
  evx_sync();
  for (int h = T / 2; h > 0; h >>= 1) {
    if (tid < h) {
      red[2 * tid] += red[2 * (tid + h)];
      red[2 * tid + 1] += red[2 * (tid + h) + 1];
    }
    evx_sync();
  }
  s0 = red[0];
  s1 = red[1];
}

// adjoint (mode 0): with C1 = G (P C - dt M K2 F),
//   dkappa += w Re(conj Lam (-dt M K2^2 G C1)),  dM += w Re(conj Lam (-dt kappa K2^2 G C1
//   - dt K2 G F)),  L <- G P Lam,  F <- dt M K2 G Lam.
// energy (mode 1): partial[2b] += w K2 |C|^2.
EVX_DEV void spec_body(const SpecArgs& a, int tid, int bid, int nblk, double* red) {
  double s0 = 0.0, s1 = 0.0;
  const long long stride = (long long)nblk * AUX_THREADS;
  for (long long i = (long long)bid * AUX_THREADS + tid; i < a.n; i += stride) {
    const SpecPos sp = spec_pos(i, a.ny, a.ypitch, a.nz, a.ncols);
    if (!sp.live) continue;  // pad row or dead column
    const int xc = sp.x, y = sp.y, z = sp.z;
    const float kyz = a.k2y[y] + a.k2z[z];
    const float2 Cv = a.C[i];
    float2 Fv = make_float2(0.f, 0.f), Lv = make_float2(0.f, 0.f);
    if (a.mode == 0) {
      Fv = a.F[i];
      Lv = a.L[i];
    }
    float K2[2];
    double w[2];
    if (a.bc == BC_PERIODIC || a.xcplx) {
      K2[0] = K2[1] = a.k2x[xc] + kyz;
      // half spectrum along x (or a cosine x bin as a complex column); a cosine axis weighs its
      // bins n w_k relative to a periodic one (the 1/V normalisation is applied to the sums)
      const double wx = a.xcplx ? (xc == 0 ? 0.25 : 0.5)
                                : ((xc == 0 || 2 * xc == a.nx) ? 1.0 : 2.0);
      const double fy = a.bcy == BC_PERIODIC ? 1.0 : (y == 0 ? 0.25 : 0.5);
      const double fz = a.bcz == BC_PERIODIC ? 1.0 : (z == 0 ? 0.25 : 0.5);
      w[0] = w[1] = wx * fy * fz;
    } else {
      K2[0] = a.k2x[2 * xc] + kyz;
      K2[1] = a.k2x[2 * xc + 1] + kyz;
      const double wyz = dct_weight(y, a.ny) * dct_weight(z, a.nz);
      w[0] = dct_weight(2 * xc, a.nx) * wyz;
      w[1] = dct_weight(2 * xc + 1, a.nx) * wyz;
    }
    if (a.mode == 1) {
      if (a.bc == BC_PERIODIC || a.xcplx) {
        s0 += w[0] * double(K2[0]) * (double(Cv.x) * Cv.x + double(Cv.y) * Cv.y);
      } else {
        s0 += w[0] * double(K2[0]) * double(Cv.x) * Cv.x + w[1] * double(K2[1]) * double(Cv.y) * Cv.y;
      }
      continue;
    }
    const float cv[2] = {Cv.x, Cv.y}, fv[2] = {Fv.x, Fv.y}, lv[2] = {Lv.x, Lv.y};
    float uo[2], vo[2];
    for (int j = 0; j < 2; ++j) {
      const float k2 = K2[j], k4 = k2 * k2;
      const float P = 1.0f + a.a_dt * k2;
      const float G = evx_rcp(1.0f + a.dt_m_kappa * k4 + a.a_dt * k2);
      const float c1 = G * (P * cv[j] - a.dt_m * k2 * fv[j]);
      // periodic: Re(conj(L) X) = L.x X.x + L.y X.y, summed over both components with the
      // same weight; zero flux: two independent real coefficients
      s0 += w[j] * double(-a.dt_m * k4 * G) * double(lv[j]) * double(c1);
      s1 += w[j] * (double(-a.dt_kappa * k4 * G) * double(lv[j]) * double(c1)
                    + double(-a.dt * k2 * G) * double(lv[j]) * double(fv[j]));
      uo[j] = G * P * lv[j];
      vo[j] = a.dt_m * k2 * G * lv[j];
    }
    a.L[i] = make_float2(uo[0], uo[1]);
    a.F[i] = make_float2(vo[0], vo[1]);
  }
  block_sum2<AUX_THREADS>(s0, s1, tid, red);
  if (tid == 0) {
    a.partial[2 * bid] = s0;
    a.partial[2 * bid + 1] = s1;
  }
}

// Real-space sums.  Diagnostics (b == null): partial[2b] = sum f(c), partial[2b+1] = sum c.
// Distance (b != null): partial[2b] = sum (c - b)^2, partial[2b+1] = sum b^2.
struct RealSumArgs {
  const float* c;
  long long n;
  double* partial;
  const float* b;
};

EVX_DEV void realsum_body(const RealSumArgs& a, int tid, int bid, int nblk, double* red) {
  double s0 = 0.0, s1 = 0.0;
  const long long stride = (long long)nblk * AUX_THREADS;
  for (long long i = (long long)bid * AUX_THREADS + tid; i < a.n; i += stride) {
    const double c = a.c[i];
    if (a.b) {
      const double r = a.b[i];
      s0 += (c - r) * (c - r);
      s1 += r * r;
    } else {
      const double q = c * c - 1.0;
      s0 += 0.25 * q * q;
      s1 += c;
    }
  }
  block_sum2<AUX_THREADS>(s0, s1, tid, red);
  if (tid == 0) {
    a.partial[2 * bid] = s0;
    a.partial[2 * bid + 1] = s1;
  }
}

// Single block: out_j <- (add_j ? out_j : 0) + scale_j * sum_b partial[2b + j] (j = 0, 1),
// summed in a fixed order.  add_j = 1 accumulates (gradients), 0 overwrites.  Null outputs are
// skipped.
struct FinalArgs {
  const double* partial;
  int nparts;
  double* out0;
  double* out1;
  double scale0, scale1;
  int add0, add1;
};

EVX_DEV void final_body(const FinalArgs& a, int tid, double* red) {
  double s0 = 0.0, s1 = 0.0;
  for (int b = tid; b < a.nparts; b += AUX_THREADS) {
    s0 += a.partial[2 * b];
    s1 += a.partial[2 * b + 1];
  }
  block_sum2<AUX_THREADS>(s0, s1, tid, red);
  if (tid == 0) {
    if (a.out0) *a.out0 = (a.add0 ? *a.out0 : 0.0) + a.scale0 * s0;
    if (a.out1) *a.out1 = (a.add1 ? *a.out1 : 0.0) + a.scale1 * s1;
  }
}

// Non-finite check of a spectral buffer (the stepper's optional failure check): block b writes
// flag[b] = 1 if one of its grid-stride elements (live columns only: row padding is skipped) has
// an all-ones exponent (Inf or NaN), else 0.  Every block writes its own slot, so no clearing and
// no atomics are needed, and the host ORs the AUX_BLOCKS slots.
struct FiniteArgs {
  const float2* w;
  long long n;     // float2 elements (grouped spectral layout)
  int ny, ypitch, nz, ncols;
  int* flag;       // AUX_BLOCKS slots
};

EVX_DEV bool evx_nonfinite(float v) {
  unsigned u;
  __builtin_memcpy(&u, &v, 4);
  return (u & 0x7f800000u) == 0x7f800000u;
}

template <int T>
EVX_DEV void finite_body(const FiniteArgs& a, int tid, int bid, int nblk, int* red) {
  int bad = 0;
  const long long stride = (long long)nblk * T;
  for (long long i = (long long)bid * T + tid; i < a.n; i += stride) {
    if (!spec_pos(i, a.ny, a.ypitch, a.nz, a.ncols).live) continue;
    const float2 v = a.w[i];
    bad |= int(evx_nonfinite(v.x) || evx_nonfinite(v.y));
  }
  red[tid] = bad;
  evx_sync();
  for (int h = T / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] |= red[tid + h];
    evx_sync();
  }
  if (tid == 0) a.flag[bid] = red[0];
}

// Gray-Scott reaction terms in real space (feed F, kill k): ru = -u v^2 + F (1 - u),
// rv = u v^2 - k v.
struct GsReactArgs {
  const float* u;
  const float* v;
  float* ru;
  float* rv;
  long long n;
  float F, k;
};

EVX_DEV void gs_react_body(const GsReactArgs& a, int tid, int bid, int nblk) {
  const long long stride = (long long)nblk * AUX_THREADS;
  for (long long i = (long long)bid * AUX_THREADS + tid; i < a.n; i += stride) {
    const float u = a.u[i], v = a.v[i];
    const float uv2 = u * v * v;
    a.ru[i] = -uv2 + a.F * (1.0f - u);
    a.rv[i] = uv2 - a.k * v;
  }
}

// Gray-Scott spectral update of both species (diffusion implicit, reaction explicit):
// U <- (U + dt RU) / (1 + dt Du K2), V <- (V + dt RV) / (1 + dt Dv K2), in the layout of the
// spectral buffers (periodic x: complex half-spectrum rows; cosine x: two real bins per float2).
struct GsUpdateArgs {
  float2* U;
  float2* V;
  const float2* RU;
  const float2* RV;
  long long n;
  int ny, ypitch, nz, ncols, bc;
  int xcplx;  // cosine x with one complex column per bin
  const float *k2x, *k2y, *k2z;
  float dt, dt_du, dt_dv;
};

EVX_DEV void gs_update_body(const GsUpdateArgs& a, int tid, int bid, int nblk) {
  const long long stride = (long long)nblk * AUX_THREADS;
  for (long long i = (long long)bid * AUX_THREADS + tid; i < a.n; i += stride) {
    const SpecPos sp = spec_pos(i, a.ny, a.ypitch, a.nz, a.ncols);
    if (!sp.live) continue;  // pad row or dead column
    const int xc = sp.x;
    const float kyz = a.k2y[sp.y] + a.k2z[sp.z];
    float ka, kb;
    if (a.bc == BC_PERIODIC || a.xcplx) {
      ka = kb = a.k2x[xc] + kyz;
    } else {
      ka = a.k2x[2 * xc] + kyz;
      kb = a.k2x[2 * xc + 1] + kyz;
    }
    const float2 U = a.U[i], V = a.V[i], RU = a.RU[i], RV = a.RV[i];
    a.U[i] = make_float2((U.x + a.dt * RU.x) / (1.0f + a.dt_du * ka),
                         (U.y + a.dt * RU.y) / (1.0f + a.dt_du * kb));
    a.V[i] = make_float2((V.x + a.dt * RV.x) / (1.0f + a.dt_dv * ka),
                         (V.y + a.dt * RV.y) / (1.0f + a.dt_dv * kb));
  }
}

// Variable-mobility Cahn-Hilliard (paper, appendix "Phase transformations of first and second
// order", eq. cahn-hilliard, stepped as in "Semi-implicit timestepping"): the finite-difference
// right-hand side div(M grad mu), mu = gamma0 g(phi) - 2 gamma0 eps lap phi, M = D0 phi (1 - phi),
// g = (18 / eps) phi (1 - phi) (1 - 2 phi), in one real-space pass over the natural (z, y, x)
// layout.  Periodic axes wrap; zero-flux axes mirror the edge cell into its ghost, so mu's ghost
// equals the edge value and a boundary face carries no flux.
struct VmStencilArgs {
  const float* phi;
  float* out;       // div(M grad mu)
  int nx, ny, nz;
  int per;          // periodic axes: bit 0 x, bit 1 y, bit 2 z
  float c_g;        // gamma0 * 18 / eps
  float c_lap;      // 2 gamma0 eps / dx^2
  float c_flux;     // D0 / (2 dx^2): the face mobility is the mean of the two cells'
};

// mu and div(M grad mu) in one pass: a block owns a VF_X x VF_Y column and marches up lz of its
// z planes, with phi (2-point xy halo) and mu (1-point halo) held
// in LDS rings of 4 and 3 planes.  Per plane z it loads phi of plane z + 2, evaluates mu on plane
// z + 1 and the fluxes on plane z:
//   mu = c_g p (1 - p)(1 - 2 p) - c_lap (sum of the 6 neighbours' phi - 6 p),
//   div(M grad mu) = c_flux sum_faces (p (1 - p) + q (1 - q)) (mu_q - mu_p),
// the neighbours taken in the order +x, -x, +y, -y, +z, -z; mu never leaves LDS (8 bytes per
// voxel).  On a zero-flux axis phi is loaded clamped (the ghost is the edge cell) and mu at a
// point past the grid is evaluated at the clamped point, i.e. it is the edge cell's mu, so the
// boundary face carries no flux.
constexpr int VF_X = 32, VF_Y = 16, VF_THREADS = VF_X * VF_Y;
constexpr int VF_PX = VF_X + 4, VF_PY = VF_Y + 4, VF_PP = VF_PX * VF_PY;  // phi plane: 36 x 20
constexpr int VF_MX = VF_X + 2, VF_MY = VF_Y + 2, VF_MP = VF_MX * VF_MY;  // mu plane: 34 x 18
constexpr int VF_LDS = 4 * VF_PP + 3 * VF_MP;                              // floats

EVX_DEV int vf_mod(int v, int n) {
  const int r = v % n;
  return r < 0 ? r + n : r;
}
// grid index of point v on an axis of n points: periodic wrap, or the zero-flux clamp
EVX_DEV int vf_map(int v, int n, bool per) {
  return per ? vf_mod(v, n) : (v < 0 ? 0 : (v >= n ? n - 1 : v));
}

// z planes per block of the fused pass: long runs (few re-read halo planes), but about four
// blocks per CU
inline int vm_fused_lz(const VmStencilArgs& a, int cus) {
  const long long ncols = (long long)((a.nx + VF_X - 1) / VF_X) * ((a.ny + VF_Y - 1) / VF_Y);
  long long lz = (a.nz * ncols + 4LL * cus - 1) / (4LL * cus);
  if (lz < 4) lz = 4;
  if (lz > a.nz) lz = a.nz;
  return int(lz);
}

// Launch: ceil(nx / VF_X) ceil(ny / VF_Y) columns times ceil(nz / lz) z ranges, VF_THREADS each.
EVX_DEV void vm_fused_body(const VmStencilArgs& a, int lz, int tid, int bid, float* lds) {
  const int ntx = (a.nx + VF_X - 1) / VF_X, nty = (a.ny + VF_Y - 1) / VF_Y;
  const int ncols = ntx * nty;
  const int col = bid % ncols, chunk = bid / ncols;
  const int x0 = (col % ntx) * VF_X, y0 = (col / ntx) * VF_Y;
  const int z0 = chunk * lz, z1 = z0 + lz < a.nz ? z0 + lz : a.nz;
  float* const P = lds;               // [4][VF_PP]
  float* const M = lds + 4 * VF_PP;   // [3][VF_MP]
  auto pl = [&](int z) { return P + vf_mod(z, 4) * VF_PP; };
  auto ml = [&](int z) { return M + vf_mod(z, 3) * VF_MP; };
  // a phi plane travels through registers: its loads are issued a plane ahead of the LDS
  // writes, every lane always loads (clamped index), and the flux stores below are buffer
  // stores issued by every lane, so the compiler waits for the loads alone
  constexpr int PIT = (VF_PP + VF_THREADS - 1) / VF_THREADS;
  int src_xy[PIT];
  const bool px = a.per & 1, py = a.per & 2, pz = a.per & 4;
  for (int k = 0; k < PIT; ++k) {
    const int i0 = tid + k * VF_THREADS, i = i0 < VF_PP ? i0 : 0;
    src_xy[k] = vf_map(y0 + i / VF_PX - 2, a.ny, py) * a.nx + vf_map(x0 + i % VF_PX - 2, a.nx, px);
  }
  const int plane = a.nx * a.ny;
  float nxt[PIT];
  auto fetch_phi = [&](int z) {
    const float* src = a.phi + vf_map(z, a.nz, pz) * plane;
    for (int k = 0; k < PIT; ++k) nxt[k] = src[src_xy[k]];
  };
  auto put_phi = [&](int z) {
    float* dst = pl(z);
    for (int k = 0; k < PIT; ++k)
      if (tid + k * VF_THREADS < VF_PP) dst[tid + k * VF_THREADS] = nxt[k];
  };
  auto calc_mu = [&](int z) {
    const int zc = pz ? z : vf_map(z, a.nz, false);
    const float *pc = pl(zc), *pu = pl(zc + 1), *pd = pl(zc - 1);
    float* dst = ml(z);
    for (int i = tid; i < VF_MP; i += VF_THREADS) {
      // the point in the phi plane (clamped into the grid along zero-flux axes)
      const int gx = x0 + i % VF_MX - 1, gy = y0 + i / VF_MX - 1;
      const int mx = i % VF_MX + (px ? 0 : vf_map(gx, a.nx, false) - gx);
      const int my = i / VF_MX + (py ? 0 : vf_map(gy, a.ny, false) - gy);
      const int c = (my + 1) * VF_PX + mx + 1;
      const float p = pc[c];
      float s = 0.0f;
      s += pc[c + 1];
      s += pc[c - 1];
      s += pc[c + VF_PX];
      s += pc[c - VF_PX];
      s += pu[c];
      s += pd[c];
      dst[i] = a.c_g * p * (1.0f - p) * (1.0f - 2.0f * p) - a.c_lap * (s - 6.0f * p);
    }
  };
  const int tx = tid % VF_X, ty = tid / VF_X;
  const int pc0 = (ty + 2) * VF_PX + tx + 2, mc0 = (ty + 1) * VF_MX + tx + 1;
  const bool own = x0 + tx < a.nx && y0 + ty < a.ny;
  const unsigned out_off = own ? unsigned(((y0 + ty) * a.nx + x0 + tx) * 4) : 0xfffffff0u;
  for (int z = z0 - 2; z <= z0 + 1; ++z) {
    fetch_phi(z);
    put_phi(z);
  }
  fetch_phi(z0 + 2);
  evx_sync();
  calc_mu(z0 - 1);
  calc_mu(z0);
  for (int z = z0; z < z1; ++z) {
    evx_sync();  // the previous plane's fluxes are done with phi plane z - 2 and mu plane z - 2
    put_phi(z + 2);
    fetch_phi(z + 3);  // past the range on the last planes: a wrapped plane, loaded and unused
    evx_sync();
    calc_mu(z + 1);
    evx_sync();
    const float *pc = pl(z), *pu = pl(z + 1), *pd = pl(z - 1);
    const float *mc = ml(z), *mu_ = ml(z + 1), *md = ml(z - 1);
    const float p = pc[pc0], m = p * (1.0f - p), u = mc[mc0];
    const float qs[6] = {pc[pc0 + 1], pc[pc0 - 1], pc[pc0 + VF_PX], pc[pc0 - VF_PX], pu[pc0], pd[pc0]};
    const float us[6] = {mc[mc0 + 1], mc[mc0 - 1], mc[mc0 + VF_MX], mc[mc0 - VF_MX], mu_[mc0], md[mc0]};
    float acc = 0.0f;
    for (int d = 0; d < 6; ++d) acc += (m + qs[d] * (1.0f - qs[d])) * (us[d] - u);
    evx_buf_store1(evx_make_buf(a.out + z * plane, unsigned(plane) * 4u), out_off, a.c_flux * acc);
  }
}

// lam <- lam - f''(c) v  (f'' = 3c^2 - 1)
struct CombineArgs {
  float* lam;
  const float* c;
  const float* v;
  long long n;
};

EVX_DEV void combine_body(const CombineArgs& a, int tid, int bid, int nblk) {
  const long long stride = (long long)nblk * AUX_THREADS;
  for (long long i = (long long)bid * AUX_THREADS + tid; i < a.n; i += stride) {
    const float c = a.c[i];
    a.lam[i] = a.lam[i] - (3.0f * c * c - 1.0f) * a.v[i];
  }
}

}  // namespace evx
