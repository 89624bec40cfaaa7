// Pass schedules of the adjoint step and of the diagnostics (shared by the HIP launcher and the
// host emulator).  A launcher L additionally provides col_batch / row_batch (one pass over a
// PassBatch of buffer pairs), spec(SpecArgs), realsum(RealSumArgs), final(FinalArgs) and
// combine(CombineArgs).
//
// Adjoint of one step c^{n+1} = A c^n - B f'(c^n), A = T^{-1} diag(G P) T,
// B = T^{-1} diag(dt M K2 G) T (both symmetric):
//   lam^n = A lam^{n+1} - f''(c^n) (B lam^{n+1}),
//   dL/dkappa += <lam^{n+1}, T^{-1}[-dt M K2^2 G C^{n+1}]>,
//   dL/dM     += <lam^{n+1}, T^{-1}[-dt kappa K2^2 G C^{n+1} - dt K2 G F^n]>,
// with C^{n+1} = G (P T[c^n] - dt M K2 T[f'(c^n)]) recomputed from c^n.
#pragma once

#include "evx_aux.hpp"
#include "evx_schedule.hpp"

namespace evx {

// Full forward transform of a real field into a spectral buffer (optionally of f'(field)).
template <class L>
void sched_forward(L& l, const Geom& g, const TablePtrs& t, const float* c, float2* out,
                   bool fprime_first, int remap) {
  l.row(g.row_len, g.bc, fprime_first ? ROW_FWD_FP : ROW_FWD,
        x_args(g, t, nullptr, c, out, nullptr));
  l.col(g.fy, g.bcy, COL_FWD, y_args(g, t, out, out, remap));
  l.col(g.fz, g.bcz, COL_FWD, z_args(g, t, out, out, nullptr, StepCoef{0, 0, 0}, remap));
}

// Full inverse transform of a spectral buffer (consumed) into a real field.
template <class L>
void sched_inverse(L& l, const Geom& g, const TablePtrs& t, float2* in, float* c, int remap) {
  l.col(g.fz, g.bcz, COL_INV, z_args(g, t, in, in, nullptr, StepCoef{0, 0, 0}, remap));
  l.col(g.fy, g.bcy, COL_INV, y_args(g, t, in, in, remap));
  l.row(g.row_len, g.bc, ROW_INV, x_args(g, t, in, nullptr, nullptr, c));
}

struct AdjointBufs {
  float2 *A, *B, *Lm;  // spectral scratch
  float* v;            // real scratch
  double* partial;     // 2 * AUX_BLOCKS
  float* v2;           // second real scratch (two-species model)
};

struct AdjointCoef {
  StepCoef step;
  float dt, dt_kappa;
};

inline SpecArgs spec_args(const Geom& g, const TablePtrs& t, const AdjointBufs& b,
                          const AdjointCoef& c, int mode) {
  SpecArgs a{};
  a.C = b.A;
  a.F = b.B;
  a.L = b.Lm;
  a.n = g.spec;
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  a.ypitch = g.ypitch;
  a.ncols = g.ncols;
  a.bc = g.bc;
  a.xcplx = g.xcplx;
  a.bcy = g.bcy;
  a.bcz = g.bcz;
  a.k2x = t.k2_x;
  a.k2y = t.k2_y;
  a.k2z = t.k2_z;
  a.a_dt = c.step.a_dt;
  a.dt_m_kappa = c.step.dt_m_kappa;
  a.dt_m = c.step.dt_m;
  a.dt = c.dt;
  a.dt_kappa = c.dt_kappa;
  a.partial = b.partial;
  a.mode = mode;
  return a;
}

// lam (in: dL/dc^{n+1}, out: dL/dc^n); dk, dM accumulate (device doubles).
template <class L>
void sched_adjoint(L& l, const Geom& g, const TablePtrs& t, const float* c, float* lam,
                   const AdjointBufs& b, const AdjointCoef& co, double* dk, double* dM,
                   int remap) {
  // forward transforms of c, f'(c) and lam (A, B, Lm), each pass batched over the buffers
  const PassBatch rows_fwd{{c, lam, nullptr}, {b.A, b.Lm, nullptr}, 2};
  l.row_batch(g.row_len, g.bc, ROW_FWD, x_args(g, t, nullptr, c, b.A, nullptr), rows_fwd);
  l.row(g.row_len, g.bc, ROW_FWD_FP, x_args(g, t, nullptr, c, b.B, nullptr));
  const PassBatch spec3{{b.A, b.B, b.Lm}, {b.A, b.B, b.Lm}, 3};
  l.col_batch(g.fy, g.bcy, COL_FWD, y_args(g, t, b.A, b.A, remap), spec3);
  l.col_batch(g.fz, g.bcz, COL_FWD, z_args(g, t, b.A, b.A, nullptr, StepCoef{0, 0, 0}, remap),
              spec3);
  l.spec(spec_args(g, t, b, co, 0));
  const double norm = (g.bc == BC_PERIODIC || g.xcplx) ? 1.0 / double(g.V) : 1.0;
  l.final(FinalArgs{b.partial, AUX_BLOCKS, dk, dM, norm, norm, 1, 1});
  // inverse transforms: Lm -> lam, B -> v
  const PassBatch spec2{{b.Lm, b.B, nullptr}, {b.Lm, b.B, nullptr}, 2};
  l.col_batch(g.fz, g.bcz, COL_INV, z_args(g, t, b.Lm, b.Lm, nullptr, StepCoef{0, 0, 0}, remap),
              spec2);
  l.col_batch(g.fy, g.bcy, COL_INV, y_args(g, t, b.Lm, b.Lm, remap), spec2);
  const PassBatch rows_inv{{b.Lm, b.B, nullptr}, {lam, b.v, nullptr}, 2};
  l.row_batch(g.row_len, g.bc, ROW_INV, x_args(g, t, b.Lm, nullptr, nullptr, lam), rows_inv);
  l.combine(CombineArgs{lam, c, b.v, g.V});
}

// out[0] = mass dx^3 sum c, out[1] = energy dx^3 [sum f(c) + (kappa/2) sum c (-L c)].
template <class L>
void sched_diagnostics(L& l, const Geom& g, const TablePtrs& t, const float* c, double kappa,
                       const AdjointBufs& b, double* out, int remap) {
  sched_forward(l, g, t, c, b.A, false, remap);
  AdjointCoef co{};
  l.spec(spec_args(g, t, b, co, 1));
  const double norm = (g.bc == BC_PERIODIC || g.xcplx) ? 1.0 / double(g.V) : 1.0;
  const double dx3 = g.dx * g.dx * g.dx;
  // out[1] <- dx^3 (kappa/2) sum w K2 |C|^2, then the real-space sums add f(c) and set the mass
  l.final(FinalArgs{b.partial, AUX_BLOCKS, out + 1, nullptr, dx3 * 0.5 * kappa * norm, 0.0, 0, 0});
  l.realsum(RealSumArgs{c, g.V, b.partial, nullptr});
  l.final(FinalArgs{b.partial, AUX_BLOCKS, out + 1, out, dx3, dx3, 1, 0});
}

// out[0] = sum (a - b)^2, out[1] = sum b^2 (relative L2 distance = sqrt(out[0] / out[1])).
template <class L>
void sched_distance(L& l, const Geom& g, const float* a, const float* b, const AdjointBufs& bufs,
                    double* out) {
  l.realsum(RealSumArgs{a, g.V, bufs.partial, b});
  l.final(FinalArgs{bufs.partial, AUX_BLOCKS, out, out + 1, 1.0, 1.0, 0, 0});
}

// Gray-Scott: nsteps of both species in place in the real fields u, v.  Spectral scratch: A, B
// (U, V), Lm and W (the reactions); real scratch: v, v2.
struct GsCoef {
  float dt, dt_du, dt_dv, F, k;
};

template <class L>
void sched_gray_scott(L& l, const Geom& g, const TablePtrs& t, float* u, float* v,
                      const AdjointBufs& b, float2* W, const GsCoef& co, int nsteps, int remap) {
  float2 *U = b.A, *V = b.B, *RU = b.Lm, *RV = W;
  for (int n = 0; n < nsteps; ++n) {
    l.gs_react(GsReactArgs{u, v, b.v, b.v2, g.V, co.F, co.k});
    const PassBatch rows{{u, v, b.v, b.v2}, {U, V, RU, RV}, 4};
    l.row_batch(g.row_len, g.bc, ROW_FWD, x_args(g, t, nullptr, u, U, nullptr), rows);
    const PassBatch all{{U, V, RU, RV}, {U, V, RU, RV}, 4};
    l.col_batch(g.fy, g.bcy, COL_FWD, y_args(g, t, U, U, remap), all);
    l.col_batch(g.fz, g.bcz, COL_FWD, z_args(g, t, U, U, nullptr, StepCoef{0, 0, 0}, remap), all);
    GsUpdateArgs ua{};
    ua.U = U;
    ua.V = V;
    ua.RU = RU;
    ua.RV = RV;
    ua.n = g.spec;
    ua.ny = g.ny;
    ua.ypitch = g.ypitch;
    ua.nz = g.nz;
    ua.ncols = g.ncols;
    ua.bc = g.bc;
    ua.xcplx = g.xcplx;
    ua.k2x = t.k2_x;
    ua.k2y = t.k2_y;
    ua.k2z = t.k2_z;
    ua.dt = co.dt;
    ua.dt_du = co.dt_du;
    ua.dt_dv = co.dt_dv;
    l.gs_update(ua);
    const PassBatch two{{U, V}, {U, V}, 2};
    l.col_batch(g.fz, g.bcz, COL_INV, z_args(g, t, U, U, nullptr, StepCoef{0, 0, 0}, remap), two);
    l.col_batch(g.fy, g.bcy, COL_INV, y_args(g, t, U, U, remap), two);
    const PassBatch back{{U, V}, {u, v}, 2};
    l.row_batch(g.row_len, g.bc, ROW_INV, x_args(g, t, U, nullptr, nullptr, u), back);
  }
}

// Variable-mobility Cahn-Hilliard in the paper's increment form (appendix "Semi-implicit
// timestepping"): phi <- phi + T^{-1}[dt / (1 + c4 K2^2) T[div(M grad mu)]], the right-hand side
// from the two stencil passes; the multiplier sits between the forward and inverse z transforms
// of one column pass, and the inverse x pass adds the increment to phi.  Scratch: v (mu), v2 (the
// right-hand side), A.
struct VmCoef {
  float dt, c4, c_g, c_lap, c_flux;
};

template <class L>
void sched_varmob(L& l, const Geom& g, const TablePtrs& t, float* phi, const AdjointBufs& b,
                  const VmCoef& co, int nsteps, int remap) {
  const int per = (g.bc == BC_PERIODIC ? 1 : 0) | (g.bcy == BC_PERIODIC ? 2 : 0) |
                  (g.bcz == BC_PERIODIC ? 4 : 0);
  const StepCoef zc{0.0f, co.c4, co.dt};  // the z pass reads dt from dt_m, c4 from dt_m_kappa
  // mu and the fluxes in one z-marching pass (mu stays in LDS)
  const VmStencilArgs fused{phi, b.v2, g.nx, g.ny, g.nz, per, co.c_g, co.c_lap, co.c_flux};
  for (int n = 0; n < nsteps; ++n) {
    l.vm_fused(fused);
    l.row(g.row_len, g.bc, ROW_FWD, x_args(g, t, nullptr, b.v2, b.A, nullptr));
    l.col(g.fy, g.bcy, COL_FWD, y_args(g, t, b.A, b.A, remap));
    l.col(g.fz, g.bcz, COL_Z_VM, z_args(g, t, b.A, b.A, nullptr, zc, remap));
    l.col(g.fy, g.bcy, COL_INV, y_args(g, t, b.A, b.A, remap));
    l.row(g.row_len, g.bc, ROW_INV_ADD, x_args(g, t, b.A, nullptr, nullptr, phi));
  }
}

}  // namespace evx
