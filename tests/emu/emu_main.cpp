// Host emulator of the HIP pass kernels (test infrastructure).  It compiles the very same pass
// bodies and pass schedule as the GPU library, runs each workgroup as one std::thread per lane
// with a std::barrier at every workgroup barrier, and is built with AddressSanitizer (every
// global and LDS buffer is an exactly sized heap allocation) or ThreadSanitizer (a missing
// barrier shows up as a data race on the LDS buffer).  LDS is filled with NaN before every
// workgroup, so a read of a slot nobody wrote poisons the result.
//
// usage: evx_emu nx ny nz bc scheme dx dt M kappa A nsteps remap in.f32 out.f32 [integrator [model]]
//   integrator 0 semi-implicit / 1 ETD1; model 0 Cahn-Hilliard / 1 Allen-Cahn.
//   bc 0 periodic / 1 zero flux / 2 Dirichlet, or 1000 + 100 bc_x + 10 bc_y + bc_z per axis;
//   scheme 0 spectral / 1 stencil7.  nsteps < 0 runs |nsteps| steps
//   in two halves with an end + restore between them (the resume path).
//        evx_emu adj nx ny nz bc scheme dx dt M kappa A c.f32 lam.f32 out_lam.f32 out_grad.f64
//   one adjoint step (lam <- dL/dc^n, out_grad = [dL/dkappa, dL/dM] of the step).
//        evx_emu diag nx ny nz bc scheme dx kappa c.f32 out.f64   (mass, energy)
//        evx_emu gs nx ny nz bc scheme dx dt Du Dv F k nsteps u v out_u out_v   (Gray-Scott)
#include <barrier>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <thread>
#include <type_traits>
#include <vector>

#include <cstring>

#include "evx_adjoint.hpp"

namespace evx_emu {
thread_local std::barrier<>* block_barrier = nullptr;
}

using namespace evx;

// bc 0 / 1 / 2 for all axes, or 1000 + 100 bc_x + 10 bc_y + bc_z with periodic (0), zero flux
// (1) and Dirichlet (2) per axis
static Geom geom_of(int nx, int ny, int nz, int bc, int scheme, double dx) {
  if (bc >= 1000)
    return make_geom3(nx, ny, nz, (bc / 100) % 10, (bc / 10) % 10, bc % 10, scheme, dx);
  return make_geom(nx, ny, nz, bc, scheme, dx);
}

template <class Body>
static void run_grid(int nblk, int threads, int lds_slots, Body body) {
  std::vector<float2> lds(lds_slots);
  for (int bid = 0; bid < nblk; ++bid) {
    const float nan = std::numeric_limits<float>::quiet_NaN();
    for (auto& v : lds) v = make_float2(nan, nan);
    std::barrier<> bar(threads);
    std::vector<std::thread> th;
    th.reserve(threads);
    for (int tid = 0; tid < threads; ++tid) {
      th.emplace_back([&, tid] {
        evx_emu::block_barrier = &bar;
        body(tid, bid, nblk, lds.data());
      });
    }
    for (auto& x : th) x.join();
  }
}

struct EmuLauncher {
  template <int N, int BC, int MODE>
  void col_t(const ColArgs& a) {
    using C = ColCfg<N>;
    const int nblk = int((a.nseq + C::B - 1) / C::B);
    const long long lane_bytes = col_lane_bytes<N>(a);
    if (lane_bytes >= (long long)kDeadLane) {
      std::fprintf(stderr, "column pass offsets exceed 32 bits\n");
      std::exit(3);
    }
    ColArgs b = a;
    b.lane_bytes = unsigned(lane_bytes);
    run_grid(nblk, C::THREADS, C::LDS, [&](int tid, int bid, int nb, float2* lds) {
      colpass_body<N, BC, MODE>(b, tid, bid, nb, lds);
    });
  }
  template <int NH, int BC, int MODE>
  void row_t(const RowArgs& a) {
    using C = RowCfg<NH, BC>;
    const int nblk = int((a.nrows + C::ROWS - 1) / C::ROWS);
    run_grid(nblk, C::THREADS, C::LDS, [&](int tid, int bid, int nb, float2* lds) {
      rowpass_body<NH, BC, MODE>(a, tid, bid, nb, lds);
    });
  }
  template <int N, int BC>
  void col_m(int mode, const ColArgs& a) {
    switch (mode) {
      case COL_FWD: col_t<N, BC, COL_FWD>(a); break;
      case COL_INV: col_t<N, BC, COL_INV>(a); break;
      case COL_Z_INIT: col_t<N, BC, COL_Z_INIT>(a); break;
      case COL_Z_UPDATE: col_t<N, BC, COL_Z_UPDATE>(a); break;
      case COL_Z_ETD: col_t<N, BC, COL_Z_ETD>(a); break;
      case COL_Z_AC: col_t<N, BC, COL_Z_AC>(a); break;
      case COL_Z_AC_ETD: col_t<N, BC, COL_Z_AC_ETD>(a); break;
      case COL_Z_VM: col_t<N, BC, COL_Z_VM>(a); break;
      default: col_t<N, BC, COL_Z_INV_STATE>(a); break;
    }
  }
  template <int NH, int BC>
  void row_m(int mode, const RowArgs& a) {
    switch (mode) {
      case ROW_FUSED: row_t<NH, BC, ROW_FUSED>(a); break;
      case ROW_FWD: row_t<NH, BC, ROW_FWD>(a); break;
      case ROW_FWD_FP: row_t<NH, BC, ROW_FWD_FP>(a); break;
      case ROW_INV_ADD: row_t<NH, BC, ROW_INV_ADD>(a); break;
      case ROW_FUSED_REC: row_t<NH, BC, ROW_FUSED_REC>(a); break;
      case ROW_FUSED_POLY: row_t<NH, BC, ROW_FUSED_POLY>(a); break;
      default: row_t<NH, BC, ROW_INV>(a); break;
    }
  }
  void col(int n, int bc, int mode, const ColArgs& a) {
    switch (n) {
#define EVX_CASE(N)                                   \
  case N:                                             \
    if (bc == BC_PERIODIC) col_m<N, BC_PERIODIC>(mode, a); \
    else col_m<N, BC_ZERO_FLUX>(mode, a);             \
    return;
      EVX_FOR_EACH_N(EVX_CASE)
#undef EVX_CASE
      default: std::fprintf(stderr, "unsupported column length %d\n", n); std::exit(3);
    }
  }
  // a batched pass runs its pairs one after another (they are independent)
  void col_batch(int n, int bc, int mode, const ColArgs& a, const PassBatch& p) {
    for (int k = 0; k < p.n; ++k) {
      ColArgs b = a;
      bind_batch(b, p, k);
      col(n, bc, mode, b);
    }
  }
  void row_batch(int n, int bc, int mode, const RowArgs& a, const PassBatch& p) {
    for (int k = 0; k < p.n; ++k) {
      RowArgs b = a;
      bind_batch(b, mode == ROW_INV, p, k);
      row(n, bc, mode, b);
    }
  }
  void spec(const SpecArgs& a) {
    run_grid(AUX_BLOCKS, AUX_THREADS, 2 * AUX_THREADS, [&](int tid, int bid, int nb, float2* lds) {
      spec_body(a, tid, bid, nb, reinterpret_cast<double*>(lds));
    });
  }
  void realsum(const RealSumArgs& a) {
    run_grid(AUX_BLOCKS, AUX_THREADS, 2 * AUX_THREADS, [&](int tid, int bid, int nb, float2* lds) {
      realsum_body(a, tid, bid, nb, reinterpret_cast<double*>(lds));
    });
  }
  void final(const FinalArgs& a) {
    run_grid(1, AUX_THREADS, 2 * AUX_THREADS, [&](int tid, int, int, float2* lds) {
      final_body(a, tid, reinterpret_cast<double*>(lds));
    });
  }
  void combine(const CombineArgs& a) {
    run_grid(AUX_BLOCKS, AUX_THREADS, 1, [&](int tid, int bid, int nb, float2*) {
      combine_body(a, tid, bid, nb);
    });
  }
  void gs_react(const GsReactArgs& a) {
    run_grid(AUX_BLOCKS, AUX_THREADS, 1, [&](int tid, int bid, int nb, float2*) {
      gs_react_body(a, tid, bid, nb);
    });
  }
  void gs_update(const GsUpdateArgs& a) {
    run_grid(AUX_BLOCKS, AUX_THREADS, 1, [&](int tid, int bid, int nb, float2*) {
      gs_update_body(a, tid, bid, nb);
    });
  }
  void vm_fused(const VmStencilArgs& a) {
    const int lz = vm_fused_lz(a, 4);  // a small device: several z ranges per column
    const int ncols = ((a.nx + VF_X - 1) / VF_X) * ((a.ny + VF_Y - 1) / VF_Y);
    const int nblk = ncols * ((a.nz + lz - 1) / lz);
    run_grid(nblk, VF_THREADS, (VF_LDS + 1) / 2, [&](int tid, int bid, int, float2* lds) {
      vm_fused_body(a, lz, tid, bid, reinterpret_cast<float*>(lds));
    });
  }
  void plane(int ny, const PlaneArgs& a) {
    auto go = [&](auto ny_) {
      constexpr int NY = decltype(ny_)::value;
      using C = PlaneCfg<NY, NY / 2>;
      run_grid(a.nz, C::THREADS, C::LDS, [&](int tid, int bid, int, float2* lds) {
        planepass_body<NY, NY / 2>(a, tid, bid, lds);
      });
    };
    if (ny == 32) go(std::integral_constant<int, 32>{});
    else if (ny == 64) go(std::integral_constant<int, 64>{});
    else { std::fprintf(stderr, "unsupported plane %d\n", ny); std::exit(3); }
  }
  void row(int n, int bc, int mode, const RowArgs& a) {
    switch (n) {
#define EVX_CASE(N)                                   \
  case N:                                             \
    if (bc == BC_PERIODIC) row_m<N, BC_PERIODIC>(mode, a); \
    else row_m<N, BC_ZERO_FLUX>(mode, a);             \
    return;
      EVX_FOR_EACH_N(EVX_CASE)
#undef EVX_CASE
      default: std::fprintf(stderr, "unsupported row length %d\n", n); std::exit(3);
    }
  }
};

static bool read_f32(const char* path, std::vector<float>& v) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return false;
  const bool ok = std::fread(v.data(), sizeof(float), v.size(), f) == v.size();
  std::fclose(f);
  return ok;
}

template <class T>
static bool write_all(const char* path, const T* p, size_t n) {
  FILE* f = std::fopen(path, "wb");
  if (!f) return false;
  const bool ok = std::fwrite(p, sizeof(T), n, f) == n;
  std::fclose(f);
  return ok;
}

struct Tabs {
  HostTables h;
  TablePtrs t;
  explicit Tabs(const Geom& g) : h(make_tables(g)) {
    t = TablePtrs{h.tw_x.data(), h.tw_y.data(), h.tw_z.data(), h.post_x.data(),
                  h.mk_y.empty() ? nullptr : h.mk_y.data(),
                  h.mk_z.empty() ? nullptr : h.mk_z.data(), h.k2_x.data(), h.k2_y.data(),
                  h.k2_z.data()};
  }
};

static int run_aux(int argc, char** argv) {
  const bool adj = std::strcmp(argv[1], "adj") == 0;
  if ((adj && argc != 16) || (!adj && argc != 11)) return 2;
  const int nx = std::atoi(argv[2]), ny = std::atoi(argv[3]), nz = std::atoi(argv[4]);
  const int bc = std::atoi(argv[5]), scheme = std::atoi(argv[6]);
  const double dx = std::atof(argv[7]);
  const Geom g = geom_of(nx, ny, nz, bc, scheme, dx);
  Tabs tb(g);
  std::vector<float2> A(g.spec), B(g.spec), Lm(g.spec);
  std::vector<float> v(g.V), c(g.V);
  std::vector<double> partial(2 * AUX_BLOCKS);
  AdjointBufs bufs{A.data(), B.data(), Lm.data(), v.data(), partial.data()};
  EmuLauncher l;
  if (adj) {
    const double dt = std::atof(argv[8]), M = std::atof(argv[9]), kappa = std::atof(argv[10]);
    const double Ast = std::atof(argv[11]);
    std::vector<float> lam(g.V);
    if (!read_f32(argv[12], c) || !read_f32(argv[13], lam)) return 4;
    AdjointCoef co{StepCoef{float(Ast * dt), float(dt * M * kappa), float(dt * M)}, float(dt),
                   float(dt * kappa)};
    double grads[2] = {0.0, 0.0};
    sched_adjoint(l, g, tb.t, c.data(), lam.data(), bufs, co, &grads[0], &grads[1], 1);
    if (!write_all(argv[14], lam.data(), lam.size()) || !write_all(argv[15], grads, 2)) return 5;
  } else {
    const double kappa = std::atof(argv[8]);
    if (!read_f32(argv[9], c)) return 4;
    double out[2] = {0.0, 0.0};
    sched_diagnostics(l, g, tb.t, c.data(), kappa, bufs, out, 1);
    if (!write_all(argv[10], out, 2)) return 5;
  }
  return 0;
}

// evx_emu gs nx ny nz bc scheme dx dt Du Dv F k nsteps u.f32 v.f32 out_u.f32 out_v.f32
static int run_gs(int argc, char** argv) {
  if (argc != 18) return 2;
  const int nx = std::atoi(argv[2]), ny = std::atoi(argv[3]), nz = std::atoi(argv[4]);
  const int bc = std::atoi(argv[5]), scheme = std::atoi(argv[6]);
  const double dx = std::atof(argv[7]), dt = std::atof(argv[8]), Du = std::atof(argv[9]);
  const double Dv = std::atof(argv[10]), F = std::atof(argv[11]), k = std::atof(argv[12]);
  const int nsteps = std::atoi(argv[13]);
  const Geom g = geom_of(nx, ny, nz, bc, scheme, dx);
  const HostTables h = make_tables(g);
  TablePtrs t{h.tw_x.data(), h.tw_y.data(), h.tw_z.data(), h.post_x.data(),
              h.mk_y.empty() ? nullptr : h.mk_y.data(), h.mk_z.empty() ? nullptr : h.mk_z.data(),
              h.k2_x.data(), h.k2_y.data(), h.k2_z.data()};
  std::vector<float> u(g.V), v(g.V), ru(g.V), rv(g.V);
  if (!read_f32(argv[14], u) || !read_f32(argv[15], v)) return 4;
  std::vector<float2> A(g.spec), B(g.spec), Lm(g.spec), W(g.spec);
  AdjointBufs b{};
  b.A = A.data();
  b.B = B.data();
  b.Lm = Lm.data();
  b.v = ru.data();
  b.v2 = rv.data();
  const GsCoef co{float(dt), float(dt * Du), float(dt * Dv), float(F), float(k)};
  EmuLauncher l;
  sched_gray_scott(l, g, t, u.data(), v.data(), b, W.data(), co, nsteps, 1);
  if (!write_all(argv[16], u.data(), u.size()) || !write_all(argv[17], v.data(), v.size()))
    return 5;
  return 0;
}

// evx_emu vm nx ny nz bc scheme dx dt D0 gamma0 eps M0 nsteps phi.f32 out.f32
static int run_vm(int argc, char** argv) {
  if (argc != 16) return 2;
  const int nx = std::atoi(argv[2]), ny = std::atoi(argv[3]), nz = std::atoi(argv[4]);
  const int bc = std::atoi(argv[5]), scheme = std::atoi(argv[6]);
  const double dx = std::atof(argv[7]), dt = std::atof(argv[8]), D0 = std::atof(argv[9]);
  const double gamma0 = std::atof(argv[10]), eps = std::atof(argv[11]), M0 = std::atof(argv[12]);
  const int nsteps = std::atoi(argv[13]);
  const Geom g = geom_of(nx, ny, nz, bc, scheme, dx);
  const HostTables h = make_tables(g);
  TablePtrs t{h.tw_x.data(), h.tw_y.data(), h.tw_z.data(), h.post_x.data(),
              h.mk_y.empty() ? nullptr : h.mk_y.data(), h.mk_z.empty() ? nullptr : h.mk_z.data(),
              h.k2_x.data(), h.k2_y.data(), h.k2_z.data()};
  std::vector<float> phi(g.V), v(g.V), v2(g.V);
  if (!read_f32(argv[14], phi)) return 4;
  std::vector<float2> A(g.spec);
  AdjointBufs b{};
  b.A = A.data();
  b.v = v.data();
  b.v2 = v2.data();
  const double h2 = dx * dx;
  const VmCoef co{float(dt), float(2.0 * dt * gamma0 * eps * M0), float(gamma0 * 18.0 / eps),
                  float(2.0 * gamma0 * eps / h2), float(D0 / (2.0 * h2))};
  EmuLauncher l;
  sched_varmob(l, g, t, phi.data(), b, co, nsteps, 1);
  if (!write_all(argv[15], phi.data(), phi.size())) return 5;
  return 0;
}

// rd nx ny nz bc scheme dx dt D A a0 a1 a2 a3 nsteps in out: reaction-diffusion steps
int run_rd(int argc, char** argv) {
  if (argc != 18) {
    std::fprintf(stderr, "usage: rd nx ny nz bc scheme dx dt D A a0 a1 a2 a3 nsteps in out\n");
    return 2;
  }
  const int nx = std::atoi(argv[2]), ny = std::atoi(argv[3]), nz = std::atoi(argv[4]);
  const int bc = std::atoi(argv[5]), scheme = std::atoi(argv[6]);
  const double dx = std::atof(argv[7]), dt = std::atof(argv[8]), D = std::atof(argv[9]);
  const double A = std::atof(argv[10]);
  const float poly[4] = {float(-std::atof(argv[11])), float(-std::atof(argv[12])),
                         float(-std::atof(argv[13])), float(-std::atof(argv[14]))};
  const int nsteps = std::atoi(argv[15]);
  const Geom g = geom_of(nx, ny, nz, bc, scheme, dx);
  const HostTables h = make_tables(g);
  TablePtrs t{h.tw_x.data(), h.tw_y.data(), h.tw_z.data(), h.post_x.data(),
              h.mk_y.empty() ? nullptr : h.mk_y.data(), h.mk_z.empty() ? nullptr : h.mk_z.data(),
              h.k2_x.data(), h.k2_y.data(), h.k2_z.data()};
  std::vector<float> c(g.V);
  if (!read_f32(argv[16], c)) return 4;
  std::vector<float2> S(g.state), W(g.spec);
  const StepCoef co{float(A * dt), float(dt * D), float(dt)};
  EmuLauncher l;
  sched_begin(l, g, t, c.data(), S.data(), W.data(), 1);
  sched_advance_rd(l, g, t, S.data(), W.data(), co, poly, nsteps, 1);
  sched_end(l, g, t, c.data(), W.data(), 1);
  if (!write_all(argv[17], c.data(), c.size())) return 5;
  return 0;
}

int main(int argc, char** argv) {
  if (argc > 1 && std::strcmp(argv[1], "rd") == 0) return run_rd(argc, argv);
  if (argc > 1 && std::strcmp(argv[1], "gs") == 0) return run_gs(argc, argv);
  if (argc > 1 && std::strcmp(argv[1], "vm") == 0) return run_vm(argc, argv);
  if (argc > 1 && (std::strcmp(argv[1], "adj") == 0 || std::strcmp(argv[1], "diag") == 0))
    return run_aux(argc, argv);
  if (argc < 15 || argc > 17) {
    std::fprintf(stderr,
                 "usage: %s nx ny nz bc scheme dx dt M kappa A nsteps remap in out [integrator "
                 "[model]]\n",
                 argv[0]);
    return 2;
  }
  const bool etd = argc >= 16 && std::atoi(argv[15]) == 1;
  const bool ac = argc >= 17 && std::atoi(argv[16]) == 1;
  const int zmode = ac ? (etd ? COL_Z_AC_ETD : COL_Z_AC) : (etd ? COL_Z_ETD : COL_Z_UPDATE);
  const int nx = std::atoi(argv[1]), ny = std::atoi(argv[2]), nz = std::atoi(argv[3]);
  const int bc = std::atoi(argv[4]), scheme = std::atoi(argv[5]);
  const double dx = std::atof(argv[6]), dt = std::atof(argv[7]), M = std::atof(argv[8]);
  const double kappa = std::atof(argv[9]), A = std::atof(argv[10]);
  const int nsteps = std::atoi(argv[11]), remap = std::atoi(argv[12]);
  const Geom g = geom_of(nx, ny, nz, bc, scheme, dx);
  const HostTables h = make_tables(g);
  TablePtrs t{h.tw_x.data(), h.tw_y.data(), h.tw_z.data(), h.post_x.data(),
              h.mk_y.empty() ? nullptr : h.mk_y.data(), h.mk_z.empty() ? nullptr : h.mk_z.data(),
              h.k2_x.data(), h.k2_y.data(), h.k2_z.data()};
  std::vector<float> c(g.V);
  FILE* f = std::fopen(argv[13], "rb");
  if (!f || std::fread(c.data(), sizeof(float), g.V, f) != size_t(g.V)) return 4;
  std::fclose(f);
  std::vector<float2> S(g.state), W(g.spec);
  const StepCoef co{float(A * dt), float(dt * M * kappa), float(dt * M)};
  EmuLauncher l;
  sched_begin(l, g, t, c.data(), S.data(), W.data(), remap);
  if (nsteps >= 0) {
    sched_advance(l, g, t, S.data(), W.data(), co, nsteps, remap, zmode);
  } else {
    const int n1 = (-nsteps) / 2, n2 = -nsteps - n1;
    std::vector<float> tmp(g.V);
    sched_advance(l, g, t, S.data(), W.data(), co, n1, remap, zmode);
    sched_end(l, g, t, tmp.data(), W.data(), remap);
    sched_restore(l, g, t, S.data(), W.data(), remap);
    sched_advance(l, g, t, S.data(), W.data(), co, n2, remap, zmode);
  }
  sched_end(l, g, t, c.data(), W.data(), remap);
  f = std::fopen(argv[14], "wb");
  if (!f || std::fwrite(c.data(), sizeof(float), g.V, f) != size_t(g.V)) return 5;
  std::fclose(f);
  return 0;
}
