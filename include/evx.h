/*
 * evx: MI355X (gfx950) Fourier-spectral semi-implicit Cahn-Hilliard stepper, C ABI.
 *
 * The operation (paper: Appendix, "Phase transformations of first and second order" for the
 * Cahn-Hilliard equation and its free energy functional; "Semi-implicit timestepping" for the
 * scheme, its increment form and the rule that the implicit prefactor is dt / (1 - dt S) with S
 * the symbol of the implicitly treated operator):
 *
 *   dc/dt = div(M grad mu),  mu = f'(c) - kappa lap c,  f(c) = (c^2 - 1)^2 / 4,
 *   C^{n+1} = G (P C^n - dt M K2 T[f'(c^n)]),   P = 1 + A dt K2,
 *   G = 1 / (1 + dt M kappa K2^2 + A dt K2),
 *
 * i.e. the increment form c^{n+1} = c^n + T^{-1}[dt / (1 - dt S) T[rhs]] with symbol
 * S = -(M kappa K2^2 + A K2): the fourth-order operator plus a linear stabilisation A K2 (the
 * constant-coefficient splitting of the same appendix).  T is the 3D DFT (periodic boundaries)
 * or the 3D DCT-II (zero flux on a cell-centred grid; the update then carries homogeneous
 * Neumann data, so a cosine transform diagonalises it).  K2 is the eigenvalue of -lap: k^2
 * (spectral) or sum over axes of (4/dx^2) sin^2(k dx / 2) (7-point stencil).
 *
 * The same passes also run Dirichlet boundaries (DST-II) and per-axis boundary mixes (evx_bc,
 * evx_plan_create_axes), an exponential (ETD1) integrator and the Allen-Cahn model (the
 * integrator and model fields of evx_ch_params), the Gray-Scott two-species model
 * (evx_gs_step) and the paper's variable-mobility Cahn-Hilliard form (evx_vm_step).
 *
 * Conventions for every entry point:
 *   - Arrays are C order (nz, ny, nx), x fastest, FP32, in device memory of the device that was
 *     current when the plan was created; that device must be current for every call.
 *   - Large device memory belongs to the caller: fields, and the plan workspace
 *     (evx_plan_workspace_bytes / evx_plan_set_workspace).  The plan itself owns host metadata
 *     and a few KB of device tables (twiddles, per-axis K2).
 *   - Calls validate synchronously and return a status; work is enqueued asynchronously on the
 *     given HIP stream (NULL = default stream) and no call synchronises the stream except
 *     evx_plan_read_pass_times.  On error nothing further is enqueued by that call; the message
 *     is available from evx_last_error() (thread-local).
 *   - A plan is not thread-safe; calls on one plan must be serialised by the caller.
 */
#ifndef EVX_H_
#define EVX_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum evx_status {
  EVX_OK = 0,
  EVX_ERR_ARG = 1,         /* null pointer, bad enum, non-positive count, wrong device */
  EVX_ERR_SIZE = 2,        /* grid size not supported (see evx_plan_create) */
  EVX_ERR_UNSUPPORTED = 3, /* valid request this build does not implement */
  EVX_ERR_NOMEM = 4,       /* workspace missing or too small, or table allocation failed */
  EVX_ERR_HIP = 5,         /* a HIP runtime call or kernel launch failed */
  EVX_ERR_STATE = 6,       /* call out of order (e.g. advance before begin) */
  EVX_ERR_NONFINITE = 7    /* check_finite was set and the state holds a NaN or an Inf */
} evx_status;

/* Boundary conditions (the paper's "boundary conditions x grid conventions" per axis).  On the
 * cell-centred grid (points (j + 1/2) dx): EVX_BC_ZERO_FLUX mirrors the field about the outer
 * faces (DCT-II); EVX_BC_DIRICHLET: c (and its even derivatives) vanish at the outer cell faces,
 * i.e. the DST-II basis -- the homogeneous data the update inherits, which the paper notes is
 * what makes a fast transform applicable.  It runs the zero-flux kernels on (-1)^(i+j+l) c
 * (DST-II(x)[k] = DCT-II((-1)^n x)[N-1-k]) with the wavenumbers in reversed order; f' is odd, so
 * the sign cancels inside the step.  EVX_BC_ZERO_FLUX_VERTEX: zero flux on a vertex-centred grid
 * (n points j dx including both boundary vertices, the field mirrored about them; wavenumbers
 * pi m / ((n - 1) dx)): the DCT-I, run as the periodic transform of the even extension of length
 * 2 (n - 1), which must be a supported length (n - 1 itself for x); evx_ch_diagnostics,
 * evx_ch_adjoint_step and evx_vm_step refuse such plans (EVX_ERR_UNSUPPORTED). */
typedef enum evx_bc {
  EVX_BC_PERIODIC = 0,
  EVX_BC_ZERO_FLUX = 1,
  EVX_BC_DIRICHLET = 2,
  EVX_BC_ZERO_FLUX_VERTEX = 3
} evx_bc;
typedef enum evx_scheme { EVX_SCHEME_SPECTRAL = 0, EVX_SCHEME_STENCIL7 = 1 } evx_scheme;

/* Time integrator of evx_ch_advance / evx_ch_step.  Both split the k-space right-hand side as
 * dC/dt = S C + N, S = -(M kappa K2^2 + A K2), N = -M K2 F + A K2 C (F = T[f'(c)]):
 *   EVX_INTEGRATOR_SEMI_IMPLICIT: C' = (C + dt N) / (1 - dt S)  (Appendix, semi-implicit step);
 *   EVX_INTEGRATOR_ETD1: first-order exponential time differencing, one of the exponential
 *     integrators the paper lists among the supported steppers:
 *     C' = exp(dt S) C + dt phi1(dt S) N, phi1(z) = (exp(z) - 1) / z. */
typedef enum evx_integrator {
  EVX_INTEGRATOR_SEMI_IMPLICIT = 0,
  EVX_INTEGRATOR_ETD1 = 1
} evx_integrator;

/* Model stepped by evx_ch_advance / evx_ch_step (same plan, transforms and free energy):
 *   EVX_MODEL_CAHN_HILLIARD: dc/dt = M lap(f'(c) - kappa lap c) (conserved; the split above);
 *   EVX_MODEL_ALLEN_CAHN: dc/dt = -M (f'(c) - kappa lap c), the linear relaxation of the same
 *     free energy (the paper's Allen-Cahn equation for a non-conserved order parameter, M the
 *     kinetic coefficient).  Its split is S = -(M kappa K2 + A), N = -M F + A C: the
 *     stabilisation multiplies dt alone, so the semi-implicit step is
 *     C' = (P C - dt M F) / (1 + A dt + dt M kappa K2), P = 1 + A dt. */
typedef enum evx_model { EVX_MODEL_CAHN_HILLIARD = 0, EVX_MODEL_ALLEN_CAHN = 1 } evx_model;

/* Per-call physics: time step, mobility, gradient-energy coefficient, stabilisation.  They are
 * per call (not plan fields) so gradient loops over kappa and M never re-plan.  For Cahn-Hilliard
 * A multiplies dt K2 alone (not M): P = 1 + A dt K2.  integrator is an evx_integrator and model an
 * evx_model (both 0 -- semi-implicit Cahn-Hilliard -- when the struct is zero-initialised past
 * A); the adjoint supports that combination only (EVX_ERR_UNSUPPORTED otherwise).
 * check_finite != 0 asks evx_ch_advance / evx_ch_advance_record / evx_ch_step to check the new
 * state for NaN and Inf once their nsteps have been enqueued (one extra read of the work buffer,
 * which holds the state's values transformed along z, so a non-finite state value shows up there
 * too): the call then synchronises the stream and returns EVX_ERR_NONFINITE if one is found (the
 * state is left as computed; evx_ch_step skips its final inverse transform).  With 0 (the
 * default) no call synchronises. */
typedef struct evx_ch_params {
  double dt;
  double M;
  double kappa;
  double A;
  int integrator;
  int model;
  int check_finite;
} evx_ch_params;

/* Workspace users (bit mask for evx_plan_workspace_bytes). */
enum {
  EVX_OP_STEP = 1,
  EVX_OP_DIAG = 2,
  EVX_OP_ADJOINT = 4,
  EVX_OP_GRAY_SCOTT = 8,
  EVX_OP_VAR_MOBILITY = 16
};

typedef struct evx_plan evx_plan;

/* Create a plan for an nx x ny x nz grid with spacing dx.
 * Sizes: every axis length must be one of 4 6 8 10 12 16 20 24 32 40 48 50 64 80 96 100 128 160
 * 192 200 256 320 384 400 512 1024, and nx must be even with nx/2 also in that list for periodic
 * boundaries (the x transform is a real-to-complex FFT of length nx/2) -> EVX_ERR_SIZE otherwise.
 * Allocates the device tables on the current device (EVX_ERR_HIP / EVX_ERR_NOMEM on failure).
 * *out is set only on success and is released with evx_plan_destroy. */
/* As evx_plan_create with a boundary condition per axis (the paper's "BCs x grid conventions x
 * stencils" per direction): any mix of EVX_BC_PERIODIC, EVX_BC_ZERO_FLUX and EVX_BC_DIRICHLET
 * (each Dirichlet axis carries its own sign and reversed wavenumbers).  A cosine x transform keeps
 * two real bins per complex column of the spectral buffers, except under a periodic y or z, whose
 * complex transform needs one complex column per x bin (twice the spectral bytes). */
evx_status evx_plan_create_axes(evx_plan** out, int nx, int ny, int nz, evx_bc bc_x, evx_bc bc_y,
                                evx_bc bc_z, evx_scheme scheme, double dx);
evx_status evx_plan_create(evx_plan** out, int nx, int ny, int nz, evx_bc bc, evx_scheme scheme,
                           double dx);
evx_status evx_plan_destroy(evx_plan* plan);

/* Device bytes the caller must provide for the given EVX_OP_* mask.  EVX_OP_STEP needs two
 * spectral buffers (state S and work W) of nz*ny rows of complex64 (periodic: nx/2+1 values per
 * row, rows padded to a multiple of 8 values) or nz*ny*nx float (zero flux) each, S rounded up to
 * whole column blocks of the z transform, i.e. about 8 bytes per voxel; EVX_OP_DIAG adds one
 * spectral buffer and 16 KB
 * of partial sums; EVX_OP_ADJOINT adds three spectral buffers, one real field and the partial
 * sums (about 24 bytes per voxel in total); EVX_OP_GRAY_SCOTT and EVX_OP_VAR_MOBILITY add one
 * more real field to that (about 28 bytes per voxel). */
evx_status evx_plan_workspace_bytes(const evx_plan* plan, int ops, size_t* bytes);

/* Hand the plan a device buffer of at least evx_plan_workspace_bytes(plan, ops) bytes,
 * 256-byte aligned.  The plan keeps the pointer (not ownership) until it is destroyed or given
 * another buffer; contents are overwritten by the calls below. */
evx_status evx_plan_set_workspace(evx_plan* plan, void* dev, size_t bytes);

/* Spectral state S (device pointer and size in bytes), for checkpoint/resume: copying S out and
 * later back in, followed by evx_ch_restore, resumes the trajectory bit-for-bit.  The layout is
 * the library's own (tile-major over the z transform's column blocks; its first element is the
 * DC coefficient) and should be treated as opaque bytes. */
evx_status evx_plan_state(const evx_plan* plan, void** dev, size_t* bytes);

/* S <- T[c] and primes the work buffer (W <- F_z^{-1} S).  c: device, nx*ny*nz floats, read. */
evx_status evx_ch_begin(evx_plan* plan, const float* c, void* hip_stream);

/* nsteps (>= 0) semi-implicit steps on the spectral state.  Requires a prior begin (or restore);
 * runs the restore pass first if an end consumed the work buffer. */
/* As evx_ch_advance, also writing the real field c^n at the start of each of the nsteps steps to
 * traj + n V (caller-owned device memory, nsteps x V floats, C order per field).  It is the
 * recomputation a checkpointed adjoint sweep needs (the gradient of a rollout with respect to
 * c0, kappa and M, extension 3 of the paper's outlook): one fused x pass per step both stores the
 * row it passes through and continues the step, so a recorded step costs the four passes of a
 * plain one.  The recorded fields are bitwise equal to what evx_ch_end returns at the same step.
 * Errors as evx_ch_advance; EVX_ERR_ARG if traj is NULL while nsteps > 0. */
evx_status evx_ch_advance_record(evx_plan* plan, int nsteps, const evx_ch_params* params,
                                 float* traj, void* hip_stream);
evx_status evx_ch_advance(evx_plan* plan, int nsteps, const evx_ch_params* params,
                          void* hip_stream);

/* c <- T^{-1}[S].  c: device, nx*ny*nz floats, written.  Consumes the work buffer; the next
 * advance rebuilds it from S. */
evx_status evx_ch_end(evx_plan* plan, float* c, void* hip_stream);

/* W <- F_z^{-1} S after the caller has written S (resume from a checkpoint). */
evx_status evx_ch_restore(evx_plan* plan, void* hip_stream);

/* In place: c <- nsteps steps of c (begin + advance + end). */
evx_status evx_ch_step(evx_plan* plan, float* c, int nsteps, const evx_ch_params* params,
                       void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): evx_ch_step without a caller workspace.  The state and
 * work buffers live in a static device array of 64 MiB held by every device the library runs on
 * until the process ends, so grids whose two spectral buffers (evx_plan_workspace_bytes with
 * EVX_OP_STEP: about 8 bytes per voxel) exceed 64 MiB -- about 8 M voxels, e.g. 192^3 zero flux
 * or 128 x 256 x 256 periodic -- return EVX_ERR_NOMEM.  The call allocates nothing: it enqueues the
 * same kernels as evx_ch_step (results are bitwise equal) on the given stream.  The plan's own
 * workspace, state and begin/advance/end state are neither needed nor touched.  Every call on a
 * device shares that device's array and overwrites it, so calls that overlap on one device (two
 * streams, two threads) race; serialise them.  check_finite synchronises as in evx_ch_step.
 * Errors as evx_ch_step. */
evx_status evx_ch_step_noalloc(evx_plan* plan, float* c, int nsteps, const evx_ch_params* params,
                               void* hip_stream);

/* Adjoint of one step (gradients for inverse problems; the paper's Statement of Need names
 * backpropagation through the solver for parameter estimation).  With
 * c^{n+1} = A c^n - B f'(c^n), A = T^{-1} diag(G P) T, B = T^{-1} diag(dt M K2 G) T:
 *   lam^n = A lam^{n+1} - f''(c^n) (B lam^{n+1}),
 *   *dkappa += <lam^{n+1}, dc^{n+1}/dkappa>,  *dM += <lam^{n+1}, dc^{n+1}/dM>.
 * c_n: device, V floats, the state the step started from (read).  lam: device, V floats,
 * dL/dc^{n+1} on entry and dL/dc^n on return.  dkappa, dM: device doubles, accumulated (the
 * caller zeroes them once per backward sweep).  Needs a workspace sized with EVX_OP_ADJOINT
 * (EVX_ERR_NOMEM otherwise).  Results are bit-reproducible (fixed-order FP64 reductions). */
evx_status evx_ch_adjoint_step(evx_plan* plan, const float* c_n, float* lam,
                               const evx_ch_params* params, double* dkappa, double* dM,
                               void* hip_stream);

/* nsteps adjoint steps in one call, backwards through a stored trajectory: for n = nsteps - 1
 * down to 0, evx_ch_adjoint_step with c_n = states + n V.  states: device, nsteps x V floats
 * (c^0 .. c^{nsteps-1} of the forward steps, e.g. from evx_ch_advance_record plus evx_ch_end),
 * read.  lam, dkappa, dM as in evx_ch_adjoint_step: lam goes from dL/dc^{nsteps} to dL/dc^0.
 * The launches are those of nsteps single calls, so the results are bitwise equal to them.
 * nsteps = 0 does nothing; EVX_ERR_ARG for nsteps < 0 or a NULL pointer; otherwise errors as
 * evx_ch_adjoint_step. */
evx_status evx_ch_adjoint_sweep(evx_plan* plan, const float* states, int nsteps, float* lam,
                                const evx_ch_params* params, double* dkappa, double* dM,
                                void* hip_stream);

/* Mass and discrete free energy of a real field (paper: the interfacial free energy functional
 * of the Appendix, here with the double well f):  out[0] = dx^3 sum c,
 * out[1] = dx^3 [sum f(c) + (kappa/2) sum c (-L c)], L the plan's discrete Laplacian.
 * c: device, V floats (read).  out: two device doubles (written).  Only params->kappa is used.
 * Needs a workspace sized with EVX_OP_DIAG or EVX_OP_ADJOINT. */
evx_status evx_ch_diagnostics(evx_plan* plan, const float* c, const evx_ch_params* params,
                              double* out, void* hip_stream);

/* Gray-Scott two-species model (the paper's reaction-diffusion example, appendix
 * "Reaction-diffusion systems", eq. gray-scott, u = c_A, v = c_B, feed rate F, kill rate k as
 * printed there):
 *   du/dt = Du lap u - u v^2 + F (1 - u),   dv/dt = Dv lap v + u v^2 - k v,
 * stepped with the same symbol rule: diffusion implicit, reaction explicit,
 *   U' = (U + dt T[R_u]) / (1 + dt Du K2),  V' = (V + dt T[R_v]) / (1 + dt Dv K2).
 * u, v: caller-owned real fields (C order, V floats each), advanced nsteps in place on the plan's
 * grid, boundaries and scheme.  Needs a workspace sized for EVX_OP_GRAY_SCOTT (EVX_ERR_NOMEM
 * otherwise); it uses the stepper's work buffer, so a later evx_ch_advance restores it from the
 * state first.  Per step: one reaction kernel, the four forward transforms batched per pass, one
 * spectral update, the two inverse transforms batched per pass. */
typedef struct evx_gs_params {
  double dt;
  double Du;
  double Dv;
  double F;
  double k;
} evx_gs_params;
evx_status evx_gs_step(evx_plan* plan, float* u, float* v, int nsteps, const evx_gs_params* params,
                       void* hip_stream);

/* Single-species reaction-diffusion (the paper's eq. reaction-diffusion, appendix
 * "Reaction-diffusion systems") with a constant diffusivity and a cubic reaction:
 *   dc/dt = D lap c + f(c),   f(c) = a0 + a1 c + a2 c^2 + a3 c^3,
 * stepped with the symbol rule of appendix "Semi-implicit timestepping": the diffusion symbol
 * -D K2 implicit, the reaction explicit, with an optional linear stabilisation A >= 0 (A = 0 is
 * the appendix's increment form):
 *   C' = ((1 + A dt) C + dt T[f(c)]) / (1 + A dt + dt D K2).
 * c: caller-owned real field (C order, V floats), advanced nsteps in place on the plan's grid,
 * boundaries and scheme.  It runs the stepper's four passes (the fused x pass evaluates -f, the z
 * pass the update) on the plan's state and work buffers (workspace EVX_OP_STEP), so it replaces
 * any state a previous evx_ch_begin left there.  Dirichlet axes need an odd reaction
 * (a0 = a2 = 0: the transform runs on the sign-alternated field) -> EVX_ERR_UNSUPPORTED
 * otherwise.  EVX_ERR_ARG unless dt > 0, D >= 0, A >= 0. */
typedef struct evx_rd_params {
  double dt;
  double D;
  double A;
  double a0, a1, a2, a3;
} evx_rd_params;
evx_status evx_rd_step(evx_plan* plan, float* c, int nsteps, const evx_rd_params* params,
                       void* hip_stream);

/* Variable-mobility Cahn-Hilliard (the paper's second-order phase transformation, appendix
 * "Phase transformations of first and second order", eq. cahn-hilliard):
 *   dphi/dt = div(M grad mu),  mu = gamma0 g(phi) - 2 gamma0 eps lap phi,
 *   M = D0 phi (1 - phi),      g = (18 / eps) phi (1 - phi) (1 - 2 phi),
 * stepped in the increment form of appendix "Semi-implicit timestepping":
 *   phi' = phi + T^{-1}[ dt / (1 + 2 dt gamma0 eps M0 K2^2) T[ div(M grad mu) ] ],
 * M0 the constant reference mobility of the implicit part.  The right-hand side is evaluated by
 * finite differences in real space (7-point Laplacian; conservative face fluxes with the face
 * mobility the mean of the two cells'); periodic axes wrap, zero-flux axes mirror the edge cell.
 * K2 follows the plan's scheme.  phi: caller-owned real field (C order, V floats), advanced
 * nsteps in place.  Dirichlet axes return EVX_ERR_UNSUPPORTED.  Needs a workspace sized for
 * EVX_OP_VAR_MOBILITY (the Gray-Scott size; EVX_ERR_NOMEM otherwise); the stepper's own buffers
 * are untouched.  Per step: one stencil pass (mu and the fluxes), the forward x and y passes, one z pass holding
 * the multiplier between its forward and inverse transforms, the inverse y pass and an inverse x
 * pass that adds the increment to phi. */
typedef struct evx_vm_params {
  double dt;
  double D0;
  double gamma0;
  double eps;
  double M0;
} evx_vm_params;
evx_status evx_vm_step(evx_plan* plan, float* phi, int nsteps, const evx_vm_params* params,
                       void* hip_stream);

/* Distance of two fields on the plan's grid (used to judge surrogate predictions against the
 * solver): out[0] = sum (a - b)^2, out[1] = sum b^2, FP64, fixed-order reduction.  a, b: device,
 * V floats (read).  out: two device doubles (written).  Needs EVX_OP_DIAG or EVX_OP_ADJOINT. */
evx_status evx_ch_distance(evx_plan* plan, const float* a, const float* b, double* out,
                           void* hip_stream);

/* Kernel timing for measurement: when enabled, advance records a HIP event pair around every
 * pass launch on the launch stream.  read synchronises those events and returns, per pass kind
 * (0 inverse y, 1 fused x, 2 forward y, 3 fused z + update), the summed milliseconds and the
 * number of launches since the last read. */
evx_status evx_plan_enable_pass_timing(evx_plan* plan, int on);
evx_status evx_plan_read_pass_times(evx_plan* plan, double ms[4], long long counts[4]);

/* Launch mode of the time loop of evx_ch_advance (and evx_ch_step, which calls it): the
 * semi-implicit step of the Appendix, "Semi-implicit timestepping", repeated.  It changes how the
 * kernels are issued, not what they compute.
 *   steps > 0: whole chunks of `steps` time steps run as one HIP graph, captured once per plan,
 *     parameter set and workspace and replayed on the caller's stream; leftover steps are
 *     launched kernel by kernel.
 *   steps = 0: every kernel is launched individually.
 *   steps = -1 (default): chunks of 8 steps on grids of at most 2^22 voxels, where the four
 *     launches of a step are a sizeable part of its time; individual launches above.
 * The kernels and their arguments are the same in every mode, so results are bitwise identical.
 * Pass timing, and a caller's stream that is itself being captured, use individual launches.
 * The graph holds the plan's workspace addresses: evx_plan_set_workspace discards it.  The first
 * call with new parameters captures and instantiates a graph (host time, no device work).
 * EVX_ERR_ARG for steps < -1. */
evx_status evx_plan_set_step_graph(evx_plan* plan, int steps);

/* Plane pass (the step of the Appendix, "Semi-implicit timestepping", on small grids): on
 * periodic grids with nx = ny = 32 or 64, evx_ch_advance runs each step's inverse y, fused x and
 * forward y transforms as one launch per z plane that keeps the plane's spectrum in LDS (the
 * z pass is unchanged).  Same transforms, tables and operation order as the separate passes, so
 * the results are bitwise equal.  on = 1 (the default) uses it where the grid allows, on = 0
 * never; on other grids the call has no effect.  Discards a captured step graph. */
evx_status evx_plan_set_plane_pass(evx_plan* plan, int on);

/* Block-order option: 1 (default) places consecutive column tiles on the same XCD. */
evx_status evx_plan_set_xcd_remap(evx_plan* plan, int on);

/* ---------------------------------------------------------------------------------------------
 * Learned coarse stepper (the paper's Statement of Need: neural-surrogate training on solver
 * data).  A periodic residual 3D CNN predicts c after 10 solver steps:
 *   c_out = c + conv4(gelu(conv3(gelu(conv2(gelu(conv1(c))))))),
 * 3x3x3 cross-correlations with circular padding, channels 1 -> 32 -> 32 -> 32 -> 1, exact-erf
 * GELU.  BF16 weights and activations (round to nearest even), FP32 accumulation (the 32 -> 32
 * layers on MFMA), FP32 residual add.  Parameters: one FP32 vector of 57121 values, layer by
 * layer W[27][Cout][Cin] (offset d = 9 (dz+1) + 3 (dy+1) + (dx+1)) followed by b[Cout].
 * Activations and grids are C order (nz, ny, nx); fields are FP32 device arrays. */
typedef struct evx_net evx_net;

evx_status evx_surrogate_param_count(size_t* n);
/* Allocates the network's BF16 weight copies (about 230 KB) on the current device. */
evx_status evx_surrogate_create(evx_net** out);
evx_status evx_surrogate_destroy(evx_net* net);
/* params: device, 57121 FP32 master values (read; copied).  Enqueued on the stream. */
evx_status evx_surrogate_set_params(evx_net* net, const float* params, void* hip_stream);
/* Device bytes of the caller-owned workspace for inference on an nx x ny x nz grid (train = 0,
 * about 130 bytes per voxel) or for training on edge^3 windows (train = 1, nx = ny = nz = edge,
 * about 600 bytes per voxel plus 8 MB). */
evx_status evx_surrogate_workspace_bytes(int nx, int ny, int nz, int train, size_t* bytes);
/* c_out <- c_in + net(c_in) on a periodic grid.  With EVX_SURROGATE_CONSERVE_MASS in flags the
 * predicted increment's spatial mean is removed (FP64 fixed-order sum), so the prediction
 * conserves mass like the solver does.  c_in, c_out: device, V floats (may not alias).
 * ws: 256-byte aligned device workspace of at least the inference size.  EVX_ERR_STATE if no
 * parameters were set. */
enum { EVX_SURROGATE_CONSERVE_MASS = 1 };
evx_status evx_surrogate_infer(evx_net* net, const float* c_in, float* c_out, int nx, int ny,
                               int nz, int flags, void* ws, size_t ws_bytes, void* hip_stream);
/* One Adam step (b1 0.9, b2 0.999, eps 1e-8, step >= 1 counts from 1) on the mean squared error
 * over the interiors of `batch` windows of edge^3 voxels (halo cut from every face):
 * x, y: device, batch * edge^3 floats (inputs and targets); params, adam_m, adam_v: device FP32
 * vectors of 57121 values, updated in place (the network's BF16 copies are refreshed);
 * loss: device double, written with the loss at the parameters before the update. */
evx_status evx_surrogate_train_step(evx_net* net, const float* x, const float* y, int batch,
                                    int edge, int halo, float* params, float* adam_m,
                                    float* adam_v, int step, float lr, double* loss, void* ws,
                                    size_t ws_bytes, void* hip_stream);
/* Verification hook: 13 device pointers into a training workspace, holding the last window of
 * the last train step: [0] bf16(x), [1..6] z1 a1 z2 a2 z3 a3 (BF16 [V][32]), [7..9] dz1 dz2 dz3
 * (BF16 [V][32]), [10] x + net(x) (FP32), [11] dL/dy (FP32), [12] the summed parameter gradient
 * (FP32, 57121). */
evx_status evx_surrogate_train_buffers(void* ws, size_t ws_bytes, int edge, void** ptrs);

const char* evx_status_string(evx_status s);
const char* evx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EVX_H_ */
