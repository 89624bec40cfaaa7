// C ABI of the spectral Cahn-Hilliard stepper: plan, workspace, step scheduling, timing.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/evx.h"
#include "evx_launch.hpp"

using namespace evx;

namespace {

thread_local std::string g_last_error;

evx_status fail(evx_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

evx_status hip_fail(hipError_t e, const char* what) {
  return fail(EVX_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

// Device scratch of the allocation-free step (evx_ch_step_noalloc): the state and work buffers of
// one grid.  Each device holds its own copy for the life of the process.  Host code never uses
// this name as an address: the per-device address comes from hipGetSymbolAddress at plan
// creation (resolve_scratch) and only that pointer reaches kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kMaxDevices] = {};  // per device: its copy of `scratch`

// Once per device, with that device current: look up its copy of the scratch array.
evx_status resolve_scratch(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices)
    return fail(EVX_ERR_UNSUPPORTED, "device %d beyond the %d the library tracks", dev,
                kMaxDevices);
  if (g_scratch_dev[dev]) return EVX_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  g_scratch_dev[dev] = static_cast<unsigned char*>(ptr);
  return EVX_OK;
}

unsigned char* scratch_of(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (dev >= 0 && dev < kMaxDevices) ? g_scratch_dev[dev] : nullptr;
}

}  // namespace

struct evx_plan {
  Geom g;
  int device = 0;
  void* tables = nullptr;
  TablePtrs t{};
  float2* ws = nullptr;
  size_t ws_bytes = 0;
  float2* S = nullptr;
  float2* W = nullptr;
  AdjointBufs aux{};      // diagnostics / adjoint scratch (inside the workspace)
  int* finite_flags = nullptr;  // AUX_BLOCKS slots of the non-finite check (in the table block)
  bool has_diag = false;
  bool has_adj = false;
  bool has_gs = false;
  bool begun = false;     // S holds a state
  bool w_valid = false;   // W holds F_z^{-1} S
  int remap = 1;
  // Step loop as captured chunks (evx_plan_set_step_graph): -1 automatic, 0 off, k > 0 chunks of
  // k steps.  gexec replays sched_advance over k steps for the key (coefficients, z mode, remap)
  // it was captured with, on this plan's S and W.
  int plane_ny = 0;  // the grid's plane-pass size (0: none), restored when re-enabled
  int graph_mode = -1;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  int gexec_chunk = 0, gexec_zmode = -1, gexec_remap = -1;
  StepCoef gexec_coef{};
  // pass timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_used;  // (pass kind, index of start event in pool)
  size_t ev_next = 0;
};

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t spec_bytes(const Geom& g) { return align256(size_t(g.spec) * sizeof(float2)); }
size_t state_bytes(const Geom& g) { return align256(size_t(g.state) * sizeof(float2)); }
size_t partial_bytes() { return align256(2 * AUX_BLOCKS * sizeof(double)); }
size_t real_bytes(const Geom& g) { return align256(size_t(g.V) * sizeof(float)); }

// Workspace layout: S, W | A, partial (diagnostics) | B, L, v (adjoint).
size_t ws_step(const Geom& g) { return state_bytes(g) + spec_bytes(g); }
size_t ws_diag(const Geom& g) { return ws_step(g) + spec_bytes(g) + partial_bytes(); }
size_t ws_adj(const Geom& g) { return ws_diag(g) + 2 * spec_bytes(g) + real_bytes(g); }
size_t ws_gs(const Geom& g) { return ws_adj(g) + real_bytes(g); }

evx_status check_plan(const evx_plan* p) {
  if (!p) return fail(EVX_ERR_ARG, "plan is NULL");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != p->device)
    return fail(EVX_ERR_ARG, "plan was created on device %d but device %d is current", p->device,
                dev);
  return EVX_OK;
}

evx_status check_params(const evx_ch_params* q) {
  if (!q) return fail(EVX_ERR_ARG, "params is NULL");
  if (!(q->dt > 0) || !(q->M >= 0) || !(q->kappa >= 0) || !(q->A >= 0))
    return fail(EVX_ERR_ARG, "params need dt > 0, M >= 0, kappa >= 0, A >= 0");
  if (q->integrator != EVX_INTEGRATOR_SEMI_IMPLICIT && q->integrator != EVX_INTEGRATOR_ETD1)
    return fail(EVX_ERR_ARG, "unknown integrator %d", q->integrator);
  if (q->model != EVX_MODEL_CAHN_HILLIARD && q->model != EVX_MODEL_ALLEN_CAHN)
    return fail(EVX_ERR_ARG, "unknown model %d", q->model);
  return EVX_OK;
}

// z-pass mode of a (model, integrator) pair
int zmode_of(const evx_ch_params* q) {
  const bool etd = q->integrator == EVX_INTEGRATOR_ETD1;
  if (q->model == EVX_MODEL_ALLEN_CAHN) return etd ? COL_Z_AC_ETD : COL_Z_AC;
  return etd ? COL_Z_ETD : COL_Z_UPDATE;
}

StepCoef coef_of(const evx_ch_params* q) {
  return StepCoef{float(q->A * q->dt), float(q->dt * q->M * q->kappa), float(q->dt * q->M)};
}

// Launcher that optionally brackets each launch with an event pair.
struct TimedLauncher : HipLauncher {
  evx_plan* p = nullptr;
  int kind = -1;
  hipError_t ev_err = hipSuccess;
  void mark_begin() {
    if (!p->timing || kind < 0) return;
    if (p->ev_next + 2 > p->ev_pool.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t ev;
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) { ev_err = e; return; }
        p->ev_pool.push_back(ev);
      }
    }
    const size_t i0 = p->ev_next;
    p->ev_next += 2;
    p->ev_used.emplace_back(kind, int(i0));
    hipError_t e = hipEventRecord(p->ev_pool[i0], stream);
    if (e != hipSuccess) ev_err = e;
  }
  void mark_end() {
    if (!p->timing || kind < 0 || p->ev_used.empty()) return;
    hipError_t e = hipEventRecord(p->ev_pool[p->ev_used.back().second + 1], stream);
    if (e != hipSuccess) ev_err = e;
  }
  void col(int n, int bc, int mode, const ColArgs& a) {
    kind = (mode == COL_INV)                             ? 0
           : (mode == COL_FWD)                           ? 2
           : (mode == COL_Z_UPDATE || mode == COL_Z_ETD || mode == COL_Z_AC ||
              mode == COL_Z_AC_ETD)                      ? 3
                                                         : -1;
    mark_begin();
    HipLauncher::col(n, bc, mode, a);
    mark_end();
  }
  void row(int n, int bc, int mode, const RowArgs& a) {
    kind = (mode == ROW_FUSED) ? 1 : -1;
    mark_begin();
    HipLauncher::row(n, bc, mode, a);
    mark_end();
  }
  // the plane pass (inverse y, fused x, forward y in one launch) is timed as the x pass
  void plane(int ny, const PlaneArgs& a) {
    kind = 1;
    mark_begin();
    HipLauncher::plane(ny, a);
    mark_end();
  }
};

evx_status finish(const TimedLauncher& l, const char* what) {
  if (l.bad_len) return fail(EVX_ERR_SIZE, "%s: transform length has no kernel", what);
  if (l.err != hipSuccess) return hip_fail(l.err, what);
  if (l.ev_err != hipSuccess) return hip_fail(l.ev_err, "pass timing event");
  return EVX_OK;
}

TimedLauncher launcher(evx_plan* p, void* s) {
  TimedLauncher l;
  l.stream = static_cast<hipStream_t>(s);
  l.p = p;
  return l;
}

bool axis_ok(int n) { return fft_len_supported(n); }

// Automatic step-loop capture: grids of at most this many voxels (where the four launches of a
// step cost a sizeable part of its time), in chunks of kAutoGraphSteps steps.
constexpr long long kAutoGraphVoxels = 1LL << 22;
constexpr int kAutoGraphSteps = 8;

int graph_chunk(const evx_plan* p) {
  if (p->graph_mode >= 0) return p->graph_mode;
  return p->g.V <= kAutoGraphVoxels ? kAutoGraphSteps : 0;
}

void drop_graph(evx_plan* p) {
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  p->gexec = nullptr;
  p->gexec_chunk = 0;
}

// The captured chunk of k steps for these coefficients and z mode (captured now if the cached one
// has another key).  The capture runs on the plan's own stream; nothing executes during it.
evx_status step_graph(evx_plan* p, const StepCoef& c, int zmode, int k) {
  if (p->gexec && p->gexec_chunk == k && p->gexec_zmode == zmode && p->gexec_remap == p->remap &&
      std::memcmp(&p->gexec_coef, &c, sizeof(StepCoef)) == 0)
    return EVX_OK;
  drop_graph(p);
  hipError_t e;
  if (!p->cap_stream) {
    e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      p->cap_stream = nullptr;
      return hip_fail(e, "capture stream");
    }
  }
  e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  HipLauncher l;
  l.stream = p->cap_stream;
  sched_advance(l, p->g, p->t, p->S, p->W, c, k, p->remap, zmode);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(p->cap_stream, &graph);  // ends the capture whatever happened inside
  if (l.bad_len || l.err != hipSuccess || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    if (l.bad_len) return fail(EVX_ERR_SIZE, "step graph: transform length has no kernel");
    return hip_fail(l.err != hipSuccess ? l.err : e, "step graph capture");
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  p->gexec = exec;
  p->gexec_chunk = k;
  p->gexec_zmode = zmode;
  p->gexec_remap = p->remap;
  p->gexec_coef = c;
  return EVX_OK;
}

// nsteps steps of the stepper on the plan's S and W: whole chunks as graph replays where the
// plan's mode asks for them, the rest (and everything under pass timing or inside a caller's own
// capture) as individual launches.  Either way the same kernels run with the same arguments.
evx_status run_steps(evx_plan* p, int nsteps, const StepCoef& c, int zmode, void* s,
                     const char* what) {
  hipStream_t st = static_cast<hipStream_t>(s);
  int k = p->timing ? 0 : graph_chunk(p);
  if (k > 0 && nsteps >= k) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) k = 0;
  }
  int rest = nsteps;
  if (k > 0 && nsteps >= k) {
    const evx_status r = step_graph(p, c, zmode, k);
    if (r != EVX_OK) return r;
    for (; rest >= k; rest -= k) {
      const hipError_t e = hipGraphLaunch(p->gexec, st);
      if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
  }
  TimedLauncher l = launcher(p, s);
  sched_advance(l, p->g, p->t, p->S, p->W, c, rest, p->remap, zmode);
  return finish(l, what);
}

// The optional failure check after a batch of steps: scan the work buffer W (live columns) for
// NaN / Inf, then synchronise and OR the per-block flags on the host.
evx_status check_state_finite(evx_plan* p, const float2* W, void* s) {
  hipStream_t st = static_cast<hipStream_t>(s);
  const FiniteArgs a{W, p->g.spec, p->g.ny, p->g.ypitch, p->g.nz, p->g.ncols, p->finite_flags};
  hipError_t e = evx_launch_finite(a, st);
  if (e != hipSuccess) return hip_fail(e, "non-finite check");
  int host[AUX_BLOCKS];
  e = hipMemcpyAsync(host, p->finite_flags, sizeof(host), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "non-finite flags copy");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "non-finite check sync");
  for (int b = 0; b < AUX_BLOCKS; ++b)
    if (host[b]) return fail(EVX_ERR_NONFINITE, "the state holds a NaN or an Inf");
  return EVX_OK;
}

}  // namespace

extern "C" {

const char* evx_status_string(evx_status s) {
  switch (s) {
    case EVX_OK: return "ok";
    case EVX_ERR_ARG: return "invalid argument";
    case EVX_ERR_SIZE: return "unsupported grid size";
    case EVX_ERR_UNSUPPORTED: return "unsupported request";
    case EVX_ERR_NOMEM: return "workspace missing or too small / out of memory";
    case EVX_ERR_HIP: return "HIP runtime error";
    case EVX_ERR_STATE: return "call out of order";
    case EVX_ERR_NONFINITE: return "non-finite value (NaN or Inf) in the state";
  }
  return "unknown status";
}

const char* evx_last_error(void) { return g_last_error.c_str(); }

// error channel shared with the surrogate translation unit
void evx_internal_set_error(const char* msg) { g_last_error = msg; }

evx_status evx_plan_create(evx_plan** out, int nx, int ny, int nz, evx_bc bc, evx_scheme scheme,
                           double dx) {
  return evx_plan_create_axes(out, nx, ny, nz, bc, bc, bc, scheme, dx);
}

evx_status evx_plan_create_axes(evx_plan** out, int nx, int ny, int nz, evx_bc bc_x, evx_bc bc_y,
                                evx_bc bc_z, evx_scheme scheme, double dx) {
  if (!out) return fail(EVX_ERR_ARG, "out is NULL");
  for (evx_bc b : {bc_x, bc_y, bc_z})
    if (b != EVX_BC_PERIODIC && b != EVX_BC_ZERO_FLUX && b != EVX_BC_DIRICHLET &&
        b != EVX_BC_ZERO_FLUX_VERTEX)
      return fail(EVX_ERR_ARG, "bad bc %d", b);
  const evx_bc bc = bc_x;
  if (scheme != EVX_SCHEME_SPECTRAL && scheme != EVX_SCHEME_STENCIL7)
    return fail(EVX_ERR_ARG, "bad scheme %d", scheme);
  if (!(dx > 0)) return fail(EVX_ERR_ARG, "dx must be > 0");
  if (nx <= 0 || ny <= 0 || nz <= 0) return fail(EVX_ERR_ARG, "sizes must be positive");
  // a vertex-centred axis of n points transforms its even extension of 2 (n - 1) points
  auto col_ok = [](int n, evx_bc b) {
    return b == EVX_BC_ZERO_FLUX_VERTEX ? (n >= 3 && axis_ok(2 * (n - 1))) : axis_ok(n);
  };
  if (!col_ok(ny, bc_y) || !col_ok(nz, bc_z))
    return fail(EVX_ERR_SIZE, "ny=%d / nz=%d not supported", ny, nz);
  if (bc == EVX_BC_PERIODIC) {
    if (nx % 2 != 0 || !axis_ok(nx / 2))
      return fail(EVX_ERR_SIZE, "periodic nx=%d needs nx/2 in the supported list", nx);
  } else if (bc == EVX_BC_ZERO_FLUX_VERTEX) {
    if (nx < 3 || !axis_ok(nx - 1))
      return fail(EVX_ERR_SIZE, "vertex-centred nx=%d needs nx - 1 in the supported list", nx);
  } else if (!axis_ok(nx)) {
    return fail(EVX_ERR_SIZE, "nx=%d not supported", nx);
  }
  evx_plan* p = new evx_plan();
  p->g = make_geom3(nx, ny, nz, int(bc_x), int(bc_y), int(bc_z), int(scheme), dx);
  p->plane_ny = p->g.plane_ny;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  {
    const evx_status se = resolve_scratch(p->device);
    if (se != EVX_OK) {
      delete p;
      return se;
    }
  }
  const HostTables h = make_tables(p->g);
  // one allocation: every table at a 256-byte aligned offset
  struct Part { const void* src; size_t bytes; size_t off; };
  std::vector<Part> parts = {
      {h.tw_x.data(), h.tw_x.size() * sizeof(float2), 0},
      {h.tw_y.data(), h.tw_y.size() * sizeof(float2), 0},
      {h.tw_z.data(), h.tw_z.size() * sizeof(float2), 0},
      {h.post_x.data(), h.post_x.size() * sizeof(float2), 0},
      {h.mk_y.data(), h.mk_y.size() * sizeof(float2), 0},
      {h.mk_z.data(), h.mk_z.size() * sizeof(float2), 0},
      {h.k2_x.data(), h.k2_x.size() * sizeof(float), 0},
      {h.k2_y.data(), h.k2_y.size() * sizeof(float), 0},
      {h.k2_z.data(), h.k2_z.size() * sizeof(float), 0},
      {nullptr, AUX_BLOCKS * sizeof(int), 0}};  // non-finite flags (device-written)
  size_t total = 0;
  for (auto& q : parts) {
    q.off = total;
    total += align256(q.bytes > 0 ? q.bytes : 1);
  }
  std::vector<unsigned char> host(total, 0);
  for (auto& q : parts)
    if (q.bytes && q.src) std::memcpy(host.data() + q.off, q.src, q.bytes);
  e = hipMalloc(&p->tables, total);
  if (e != hipSuccess) {
    delete p;
    return fail(EVX_ERR_NOMEM, "table allocation (%zu bytes): %s", total, hipGetErrorString(e));
  }
  e = hipMemcpy(p->tables, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(p->tables);
    delete p;
    return hip_fail(e, "table upload");
  }
  auto at = [&](int i) { return static_cast<unsigned char*>(p->tables) + parts[i].off; };
  p->t.tw_x = reinterpret_cast<const float2*>(at(0));
  p->t.tw_y = reinterpret_cast<const float2*>(at(1));
  p->t.tw_z = reinterpret_cast<const float2*>(at(2));
  p->t.post_x = reinterpret_cast<const float2*>(at(3));
  p->t.mk_y = reinterpret_cast<const float2*>(at(4));
  p->t.mk_z = reinterpret_cast<const float2*>(at(5));
  p->t.k2_x = reinterpret_cast<const float*>(at(6));
  p->t.k2_y = reinterpret_cast<const float*>(at(7));
  p->t.k2_z = reinterpret_cast<const float*>(at(8));
  p->finite_flags = reinterpret_cast<int*>(at(9));
  *out = p;
  return EVX_OK;
}

evx_status evx_plan_destroy(evx_plan* p) {
  if (!p) return fail(EVX_ERR_ARG, "plan is NULL");
  for (hipEvent_t ev : p->ev_pool) (void)hipEventDestroy(ev);
  drop_graph(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->tables) (void)hipFree(p->tables);
  delete p;
  return EVX_OK;
}

evx_status evx_plan_workspace_bytes(const evx_plan* p, int ops, size_t* bytes) {
  if (!p || !bytes) return fail(EVX_ERR_ARG, "NULL argument");
  if (ops & ~(EVX_OP_STEP | EVX_OP_DIAG | EVX_OP_ADJOINT | EVX_OP_GRAY_SCOTT |
              EVX_OP_VAR_MOBILITY))
    return fail(EVX_ERR_ARG, "unknown workspace ops 0x%x", ops);
  *bytes = (ops & (EVX_OP_GRAY_SCOTT | EVX_OP_VAR_MOBILITY)) ? ws_gs(p->g)
           : (ops & EVX_OP_ADJOINT)  ? ws_adj(p->g)
           : (ops & EVX_OP_DIAG)     ? ws_diag(p->g)
                                     : ws_step(p->g);
  return EVX_OK;
}

evx_status evx_plan_set_workspace(evx_plan* p, void* dev, size_t bytes) {
  if (!p || !dev) return fail(EVX_ERR_ARG, "NULL argument");
  if (reinterpret_cast<uintptr_t>(dev) % 256 != 0)
    return fail(EVX_ERR_ARG, "workspace must be 256-byte aligned");
  if (bytes < ws_step(p->g))
    return fail(EVX_ERR_NOMEM, "workspace of %zu bytes, need %zu", bytes, ws_step(p->g));
  drop_graph(p);  // captured on the previous workspace's buffers
  p->ws = static_cast<float2*>(dev);
  p->ws_bytes = bytes;
  unsigned char* base = static_cast<unsigned char*>(dev);
  const size_t sb = spec_bytes(p->g), stb = state_bytes(p->g);
  p->S = reinterpret_cast<float2*>(base);
  p->W = reinterpret_cast<float2*>(base + stb);
  p->has_diag = bytes >= ws_diag(p->g);
  p->has_adj = bytes >= ws_adj(p->g);
  p->aux = AdjointBufs{};
  if (p->has_diag) {
    p->aux.A = reinterpret_cast<float2*>(base + stb + sb);
    p->aux.partial = reinterpret_cast<double*>(base + stb + 2 * sb);
  }
  if (p->has_adj) {
    unsigned char* q = base + stb + 2 * sb + partial_bytes();
    p->aux.B = reinterpret_cast<float2*>(q);
    p->aux.Lm = reinterpret_cast<float2*>(q + sb);
    p->aux.v = reinterpret_cast<float*>(q + 2 * sb);
  }
  p->has_gs = bytes >= ws_gs(p->g);
  if (p->has_gs) p->aux.v2 = reinterpret_cast<float*>(base + ws_adj(p->g));
  p->begun = false;
  p->w_valid = false;
  return EVX_OK;
}

evx_status evx_plan_state(const evx_plan* p, void** dev, size_t* bytes) {
  if (!p || !dev || !bytes) return fail(EVX_ERR_ARG, "NULL argument");
  if (!p->S) return fail(EVX_ERR_NOMEM, "no workspace set");
  *dev = p->S;
  *bytes = size_t(p->g.state) * sizeof(float2);
  return EVX_OK;
}

evx_status evx_ch_begin(evx_plan* p, const float* c, void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if (!c) return fail(EVX_ERR_ARG, "c is NULL");
  if (!p->S) return fail(EVX_ERR_NOMEM, "no workspace set");
  TimedLauncher l = launcher(p, s);
  sched_begin(l, p->g, p->t, c, p->S, p->W, p->remap);
  st = finish(l, "begin");
  p->begun = (st == EVX_OK);
  p->w_valid = p->begun;
  return st;
}

evx_status evx_ch_restore(evx_plan* p, void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if (!p->S) return fail(EVX_ERR_NOMEM, "no workspace set");
  TimedLauncher l = launcher(p, s);
  sched_restore(l, p->g, p->t, p->S, p->W, p->remap);
  st = finish(l, "restore");
  p->begun = (st == EVX_OK);
  p->w_valid = p->begun;
  return st;
}

evx_status evx_ch_advance(evx_plan* p, int nsteps, const evx_ch_params* q, void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if ((st = check_params(q)) != EVX_OK) return st;
  if (nsteps < 0) return fail(EVX_ERR_ARG, "nsteps < 0");
  if (!p->begun) return fail(EVX_ERR_STATE, "advance before begin/restore");
  if (!p->w_valid) {
    if ((st = evx_ch_restore(p, s)) != EVX_OK) return st;
  }
  st = run_steps(p, nsteps, coef_of(q), zmode_of(q), s, "advance");
  if (st == EVX_OK && q->check_finite) st = check_state_finite(p, p->W, s);
  return st;
}

evx_status evx_ch_advance_record(evx_plan* p, int nsteps, const evx_ch_params* q, float* traj,
                                 void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if ((st = check_params(q)) != EVX_OK) return st;
  if (nsteps < 0) return fail(EVX_ERR_ARG, "nsteps < 0");
  if (nsteps > 0 && !traj) return fail(EVX_ERR_ARG, "traj is NULL");
  if (!p->begun) return fail(EVX_ERR_STATE, "advance before begin/restore");
  if (!p->w_valid) {
    if ((st = evx_ch_restore(p, s)) != EVX_OK) return st;
  }
  TimedLauncher l = launcher(p, s);
  sched_advance_record(l, p->g, p->t, p->S, p->W, coef_of(q), nsteps, p->remap, zmode_of(q),
                       traj);
  st = finish(l, "advance_record");
  if (st == EVX_OK && q->check_finite) st = check_state_finite(p, p->W, s);
  return st;
}

evx_status evx_ch_end(evx_plan* p, float* c, void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if (!c) return fail(EVX_ERR_ARG, "c is NULL");
  if (!p->begun) return fail(EVX_ERR_STATE, "end before begin/restore");
  if (!p->w_valid) {
    if ((st = evx_ch_restore(p, s)) != EVX_OK) return st;
  }
  TimedLauncher l = launcher(p, s);
  sched_end(l, p->g, p->t, c, p->W, p->remap);
  p->w_valid = false;
  return finish(l, "end");
}

evx_status evx_ch_step(evx_plan* p, float* c, int nsteps, const evx_ch_params* q, void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if ((st = check_params(q)) != EVX_OK) return st;
  if (nsteps < 0) return fail(EVX_ERR_ARG, "nsteps < 0");
  if ((st = evx_ch_begin(p, c, s)) != EVX_OK) return st;
  if ((st = evx_ch_advance(p, nsteps, q, s)) != EVX_OK) return st;
  return evx_ch_end(p, c, s);
}

evx_status evx_ch_step_noalloc(evx_plan* p, float* c, int nsteps, const evx_ch_params* q,
                               void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if ((st = check_params(q)) != EVX_OK) return st;
  if (!c) return fail(EVX_ERR_ARG, "c is NULL");
  if (nsteps < 0) return fail(EVX_ERR_ARG, "nsteps < 0");
  const size_t need = ws_step(p->g);
  if (need > kScratchBytes)
    return fail(EVX_ERR_NOMEM,
                "allocation-free step: the grid's state and work buffers need %zu bytes, the "
                "static scratch holds %zu",
                need, kScratchBytes);
  unsigned char* base = scratch_of(p->device);
  if (!base) return fail(EVX_ERR_STATE, "scratch address of device %d not resolved", p->device);
  float2* S = reinterpret_cast<float2*>(base);
  float2* W = reinterpret_cast<float2*>(base + state_bytes(p->g));
  HipLauncher l;  // no pass timing: its events would be created on demand
  l.stream = static_cast<hipStream_t>(s);
  sched_begin(l, p->g, p->t, c, S, W, p->remap);
  sched_advance(l, p->g, p->t, S, W, coef_of(q), nsteps, p->remap, zmode_of(q));
  if (l.bad_len) return fail(EVX_ERR_SIZE, "step_noalloc: transform length has no kernel");
  if (l.err != hipSuccess) return hip_fail(l.err, "step_noalloc");
  if (q->check_finite && (st = check_state_finite(p, W, s)) != EVX_OK) return st;
  sched_end(l, p->g, p->t, c, W, p->remap);
  if (l.err != hipSuccess) return hip_fail(l.err, "step_noalloc end");
  return EVX_OK;
}

evx_status evx_ch_adjoint_step(evx_plan* p, const float* c_n, float* lam,
                               const evx_ch_params* q, double* dkappa, double* dM, void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if ((st = check_params(q)) != EVX_OK) return st;
  if (!c_n || !lam || !dkappa || !dM) return fail(EVX_ERR_ARG, "NULL argument");
  if (q->integrator != EVX_INTEGRATOR_SEMI_IMPLICIT || q->model != EVX_MODEL_CAHN_HILLIARD)
    return fail(EVX_ERR_UNSUPPORTED, "the adjoint step is the semi-implicit Cahn-Hilliard step's");
  if (p->g.vert)
    return fail(EVX_ERR_UNSUPPORTED, "adjoint step: no vertex-centred axes");
  if (!p->has_adj)
    return fail(EVX_ERR_NOMEM, "workspace too small for the adjoint (EVX_OP_ADJOINT)");
  AdjointCoef co{coef_of(q), float(q->dt), float(q->dt * q->kappa)};
  TimedLauncher l = launcher(p, s);
  sched_adjoint(l, p->g, p->t, c_n, lam, p->aux, co, dkappa, dM, p->remap);
  return finish(l, "adjoint step");
}

evx_status evx_ch_adjoint_sweep(evx_plan* p, const float* states, int nsteps, float* lam,
                                const evx_ch_params* q, double* dkappa, double* dM, void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if ((st = check_params(q)) != EVX_OK) return st;
  if (nsteps < 0) return fail(EVX_ERR_ARG, "nsteps < 0");
  if (!states || !lam || !dkappa || !dM) return fail(EVX_ERR_ARG, "NULL argument");
  if (q->integrator != EVX_INTEGRATOR_SEMI_IMPLICIT || q->model != EVX_MODEL_CAHN_HILLIARD)
    return fail(EVX_ERR_UNSUPPORTED, "the adjoint step is the semi-implicit Cahn-Hilliard step's");
  if (p->g.vert)
    return fail(EVX_ERR_UNSUPPORTED, "adjoint sweep: no vertex-centred axes");
  if (!p->has_adj)
    return fail(EVX_ERR_NOMEM, "workspace too small for the adjoint (EVX_OP_ADJOINT)");
  const AdjointCoef co{coef_of(q), float(q->dt), float(q->dt * q->kappa)};
  TimedLauncher l = launcher(p, s);
  for (int n = nsteps - 1; n >= 0; --n)
    sched_adjoint(l, p->g, p->t, states + size_t(n) * size_t(p->g.V), lam, p->aux, co, dkappa,
                  dM, p->remap);
  return finish(l, "adjoint sweep");
}

evx_status evx_gs_step(evx_plan* p, float* u, float* v, int nsteps, const evx_gs_params* q,
                       void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if (!u || !v || !q) return fail(EVX_ERR_ARG, "NULL argument");
  if (nsteps < 0) return fail(EVX_ERR_ARG, "nsteps < 0");
  if (!(q->dt > 0) || !(q->Du >= 0) || !(q->Dv >= 0))
    return fail(EVX_ERR_ARG, "params need dt > 0, Du >= 0, Dv >= 0");
  if (!p->has_gs)
    return fail(EVX_ERR_NOMEM, "workspace too small for Gray-Scott (EVX_OP_GRAY_SCOTT)");
  const GsCoef co{float(q->dt), float(q->dt * q->Du), float(q->dt * q->Dv), float(q->F),
                  float(q->k)};
  TimedLauncher l = launcher(p, s);
  sched_gray_scott(l, p->g, p->t, u, v, p->aux, p->W, co, nsteps, p->remap);
  p->w_valid = false;  // W served as scratch
  return finish(l, "gray-scott step");
}

evx_status evx_rd_step(evx_plan* p, float* c, int nsteps, const evx_rd_params* q, void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if (!c || !q) return fail(EVX_ERR_ARG, "NULL argument");
  if (nsteps < 0) return fail(EVX_ERR_ARG, "nsteps < 0");
  if (!(q->dt > 0) || !(q->D >= 0) || !(q->A >= 0))
    return fail(EVX_ERR_ARG, "params need dt > 0, D >= 0, A >= 0");
  if (p->g.flip != 0 && (q->a0 != 0.0 || q->a2 != 0.0))
    return fail(EVX_ERR_UNSUPPORTED,
                "reaction-diffusion on Dirichlet axes needs an odd reaction (a0 = a2 = 0)");
  if (!p->S) return fail(EVX_ERR_NOMEM, "no workspace set");
  // the z pass's Allen-Cahn update with M = 1, kappa = D; the x pass evaluates -f
  const StepCoef co{float(q->A * q->dt), float(q->dt * q->D), float(q->dt)};
  const float poly[4] = {float(-q->a0), float(-q->a1), float(-q->a2), float(-q->a3)};
  TimedLauncher l = launcher(p, s);
  sched_begin(l, p->g, p->t, c, p->S, p->W, p->remap);
  sched_advance_rd(l, p->g, p->t, p->S, p->W, co, poly, nsteps, p->remap);
  sched_end(l, p->g, p->t, c, p->W, p->remap);
  p->begun = false;  // the state is the reaction-diffusion field's, not a Cahn-Hilliard one
  p->w_valid = false;
  return finish(l, "reaction-diffusion step");
}

evx_status evx_vm_step(evx_plan* p, float* phi, int nsteps, const evx_vm_params* q, void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if (!phi || !q) return fail(EVX_ERR_ARG, "NULL argument");
  if (nsteps < 0) return fail(EVX_ERR_ARG, "nsteps < 0");
  if (!(q->dt > 0) || !(q->D0 >= 0) || !(q->gamma0 >= 0) || !(q->eps > 0) || !(q->M0 >= 0))
    return fail(EVX_ERR_ARG, "params need dt > 0, eps > 0 and D0, gamma0, M0 >= 0");
  if (p->g.flip != 0 || p->g.vert != 0)
    return fail(EVX_ERR_UNSUPPORTED,
                "variable-mobility step: periodic or cell-centred zero-flux axes only");
  if (!p->has_gs)
    return fail(EVX_ERR_NOMEM,
                "workspace too small for the variable-mobility step (EVX_OP_VAR_MOBILITY)");
  const double h2 = p->g.dx * p->g.dx;
  const VmCoef co{float(q->dt), float(2.0 * q->dt * q->gamma0 * q->eps * q->M0),
                  float(q->gamma0 * 18.0 / q->eps), float(2.0 * q->gamma0 * q->eps / h2),
                  float(q->D0 / (2.0 * h2))};
  TimedLauncher l = launcher(p, s);
  sched_varmob(l, p->g, p->t, phi, p->aux, co, nsteps, p->remap);
  return finish(l, "variable-mobility step");
}

evx_status evx_ch_diagnostics(evx_plan* p, const float* c, const evx_ch_params* q, double* out,
                              void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if (!q) return fail(EVX_ERR_ARG, "params is NULL");
  if (!c || !out) return fail(EVX_ERR_ARG, "NULL argument");
  if (!p->has_diag)
    return fail(EVX_ERR_NOMEM, "workspace too small for diagnostics (EVX_OP_DIAG)");
  if (p->g.vert)
    return fail(EVX_ERR_UNSUPPORTED, "diagnostics: no vertex-centred axes");
  TimedLauncher l = launcher(p, s);
  sched_diagnostics(l, p->g, p->t, c, q->kappa, p->aux, out, p->remap);
  return finish(l, "diagnostics");
}

evx_status evx_ch_distance(evx_plan* p, const float* a, const float* b, double* out, void* s) {
  evx_status st = check_plan(p);
  if (st != EVX_OK) return st;
  if (!a || !b || !out) return fail(EVX_ERR_ARG, "NULL argument");
  if (!p->has_diag)
    return fail(EVX_ERR_NOMEM, "workspace too small for diagnostics (EVX_OP_DIAG)");
  TimedLauncher l = launcher(p, s);
  sched_distance(l, p->g, a, b, p->aux, out);
  return finish(l, "distance");
}

evx_status evx_plan_enable_pass_timing(evx_plan* p, int on) {
  if (!p) return fail(EVX_ERR_ARG, "plan is NULL");
  p->timing = on != 0;
  return EVX_OK;
}

evx_status evx_plan_read_pass_times(evx_plan* p, double ms[4], long long counts[4]) {
  if (!p || !ms || !counts) return fail(EVX_ERR_ARG, "NULL argument");
  for (int k = 0; k < 4; ++k) {
    ms[k] = 0;
    counts[k] = 0;
  }
  for (auto& u : p->ev_used) {
    hipError_t e = hipEventSynchronize(p->ev_pool[u.second + 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float t = 0;
    e = hipEventElapsedTime(&t, p->ev_pool[u.second], p->ev_pool[u.second + 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    ms[u.first] += t;
    counts[u.first] += 1;
  }
  p->ev_used.clear();
  p->ev_next = 0;
  return EVX_OK;
}

evx_status evx_plan_set_step_graph(evx_plan* p, int steps) {
  if (!p) return fail(EVX_ERR_ARG, "plan is NULL");
  if (steps < -1) return fail(EVX_ERR_ARG, "step graph chunk %d (need -1, 0 or > 0)", steps);
  p->graph_mode = steps;
  return EVX_OK;
}

evx_status evx_plan_set_plane_pass(evx_plan* p, int on) {
  if (!p) return fail(EVX_ERR_ARG, "plan is NULL");
  drop_graph(p);  // a captured step holds the launches of the previous choice
  p->g.plane_ny = on ? p->plane_ny : 0;
  return EVX_OK;
}

evx_status evx_plan_set_xcd_remap(evx_plan* p, int on) {
  if (!p) return fail(EVX_ERR_ARG, "plan is NULL");
  p->remap = on ? 1 : 0;
  return EVX_OK;
}

}  // extern "C"
