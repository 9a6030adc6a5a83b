/*
 * npb.h - C ABI of the MI355X pseudo-transient nonlinear Poisson-Boltzmann
 * solver (LOD / AOS time splitting, Wilson & Zhao).
 *
 * Problem statement (Sec. 2.1, Eqs. (NPB), (RhoEq), (DebyeHuckel),
 * (BoundaryCond); Sec. 2.2, Eq. (TimeDepNPB)): point charges q_j at r_j
 * with radii R_j define the solute (union of balls, eps_in inside, eps_out
 * and the modified Debye-Hueckel parameter kbar^2 outside).  The solver
 * integrates  alpha du/dt = div(eps grad u) - kbar^2 sinh(u) + rho  on a
 * uniform grid with Dirichlet data on the outer shell, for a fixed number of
 * pseudo-time steps of size dt, and returns the dimensionless potential u
 * (as phi = kT u in kcal/mol/e) and the electrostatic solvation energy.
 *
 * Conventions used by every entry point
 *   - Grid arrays are [nz][ny][nx], x fastest; node (i,j,k) sits at
 *     origin + h (i, j, k).  The outer layer of nodes is the Dirichlet set.
 *   - Host pointers are borrowed for the duration of the call only.
 *   - Device pointers are caller-owned; the library never frees them.
 *   - "stream" is a hipStream_t passed as void* (0 = the null stream).
 *   - Functions return npb_status; on failure npb_last_error() gives a
 *     thread-local message.  No C++ exception crosses this boundary.
 *   - A context is bound to one device; calls on one context must not run
 *     concurrently from several host threads.
 */
#ifndef NPB_H
#define NPB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NPB_ABI_VERSION 7

typedef enum npb_status {
  NPB_OK = 0,
  NPB_EINVAL = 1,     /* bad argument: n < 5, h <= 0, eps <= 0, kbar^2 < 0,
                         alpha <= 0, dt <= 0, n_steps < 1, unknown scheme or
                         precision, null pointer, workspace too small      */
  NPB_ERANGE = 2,     /* an atom's trilinear 8-node stencil touches the
                         Dirichlet shell (or leaves the grid)              */
  NPB_ENOMEM = 3,     /* host-side allocation failed                       */
  NPB_EDEVICE = 4,    /* a HIP runtime call failed                         */
  NPB_EDIVERGED = 5,  /* a result is not finite: an energy, or a field value
                         after any step                                    */
  NPB_EBUSY = 6       /* admission refused (serving)                       */
} npb_status;

typedef enum npb_scheme {
  NPB_LODIE2 = 0,  /* source, x, y, z sweeps, nonlinear (Sec. 3.1, last paragraph) */
  NPB_LODIE1 = 1,  /* nonlinear, x, y, z sweeps, source (Eqs. (LODIE1_1)-(LODIE1_5)) */
  NPB_AOSIE2 = 2,  /* additive, source split 1/3 per direction (Eqs. (AOSIE2_2)-(AOSIE2_4)) */
  NPB_AOSIE1 = 3,  /* additive, source on x only (Eqs. (AOSIE1_1)-(AOSIE1_5)) */
  NPB_LODCN1 = 4,  /* LODIE1 order with Crank-Nicolson sweeps (Eqs. (LODCN1_2)-(LODCN1_4)) */
  NPB_LODCN2 = 5,  /* LODIE2 order with Crank-Nicolson sweeps (Sec. 3.1, last paragraph) */
  NPB_AOSCN1 = 6,  /* additive, Crank-Nicolson, source on x (Eqs. (AOSCN1_2)-(AOSCN1_4)) */
  NPB_AOSCN2 = 7,  /* additive, Crank-Nicolson, source split (Eqs. (AOSCN2_2)-(AOSCN2_4)) */
  NPB_MAOSIE = 8,  /* nonlinear sub-step, then the mean of three implicit-Euler
                      directional solves (Sec. 3.3, Eqs. (MAOS1_1)-(MAOS1_5)) */
  NPB_MAOSCN = 9,  /* the same with Crank-Nicolson directional solves (Sec. 3.3) */
  NPB_EULER = 10   /* explicit Euler step of Eq. (TimeDepNPB) with the operator of
                      Eq. (SpatialOperators): u += tau (div eps grad u - kbar^2
                      sinh u + rho), tau = dt / alpha.  The paper's reference
                      solver (Sec. 2.3; Sec. 5.2 and 5.4: dt = 1e-5, T = 10).
                      Stable only for tau below 2 / (largest eigenvalue of the
                      linearised operator), about h^2 / (6 eps_out); FP64 only */
} npb_scheme;

typedef enum npb_precision {
  NPB_FP64 = 0,    /* sweeps, sub-steps and field storage in double */
  NPB_FP32 = 1,    /* sweeps, sub-steps and field storage in float; setup,
                      energies, differences and Richardson stay double */
  NPB_FP32X = 2    /* field stored in float (FP32 traffic), line solves and
                      sub-steps computed in double */
} npb_precision;

/* Molecule: n_atoms atoms; xyz[3*i+d] in Angstrom, q[i] in e, radius[i]
 * in Angstrom.  Host pointers, read during the call only. */
typedef struct npb_molecule {
  int32_t n_atoms;
  const double* xyz;
  const double* q;
  const double* radius;
} npb_molecule;

/* Uniform grid: nx*ny*nz nodes, spacing h (Angstrom), origin = position of
 * node (0,0,0).  Each n must be at least 5. */
typedef struct npb_grid {
  int32_t nx, ny, nz;
  int32_t pad_;
  double h;
  double origin[3];
} npb_grid;

/* Run parameters.
 *   eps_in, eps_out : dielectric inside / outside the solute (Sec. 2.1)
 *   kappa_bar_sq    : kbar^2 in the solvent, Angstrom^-2 (Eq. (DebyeHuckel));
 *                     npb_kappa_bar_sq() converts an ionic strength
 *   temperature_K   : sets kT = 0.592183 T/298 kcal/mol and the Bjerrum
 *                     length 332.06371/kT Angstrom
 *   alpha, dt       : scaling parameter and step of Eq. (TimeDepNPB)
 *   n_steps         : steps at dt (the dt/2 level of Richardson runs 2 n_steps)
 *   scheme          : npb_scheme
 *   precision       : npb_precision
 *   richardson      : 1 = run dt and dt/2 and combine (Sec. 5.3, Eq. (rich))
 *   vacuum          : 1 = also solve the uniform-eps_in, kbar = 0 problem by
 *                     the same scheme and report the solvation energy
 *                     (Sec. 5.3, Eq. (deltaG3)); 0 = solvated potential only
 *   vacuum_direct   : 1 = also solve the vacuum Poisson problem directly
 *                     (no pseudo-time: the constant-eps_in 7-point problem
 *                     with the vacuum Dirichlet data, by type-I sine
 *                     transforms in FP64; the paper's "FFT" phi_0, Sec. 5.1)
 *                     and report dG_direct (Eq. (deltaG2)); with vacuum = 0
 *                     the direct solve is the only vacuum problem
 *   field_select    : which potential d_field_out receives:
 *                     0 = solvated, 1 = vacuum by the scheme (needs vacuum),
 *                     2 = vacuum by the direct solve (needs vacuum_direct),
 *                     3 = recovered potential phi_m - phi_0 + phi_0^direct
 *                         (Sec. 5.4; needs vacuum and vacuum_direct); phi_m and phi_0
 *                         Richardson-combined when richardson = 1
 *   field_units     : npb_field_units of d_field_out
 *   face_rule       : npb_face_rule: eps at the half points of the solvated
 *                     problem (the vacuum problem is uniform)               */
typedef struct npb_params {
  double eps_in, eps_out, kappa_bar_sq, temperature_K, alpha, dt;
  int32_t n_steps;
  int32_t scheme;
  int32_t precision;
  int32_t richardson;
  int32_t vacuum;
  int32_t field_select;
  int32_t vacuum_direct;
  int32_t field_units;
  int32_t face_rule;
} npb_params;

enum npb_face_rule {
  NPB_FACE_HARMONIC = 0,  /* harmonic mean of the two nodal values */
  NPB_FACE_LOCATION = 1   /* the half point's own location (Sec. 3.1, text after Eq.
                             (SpatialOperators)): eps_in on or inside a sphere, else
                             eps_out; applied to the union of balls */
};

enum npb_field_units {
  NPB_UNITS_KCAL = 0,          /* phi = kT u, kcal/mol/e */
  NPB_UNITS_DIMENSIONLESS = 1  /* u */
};

/* Results, all energies in kcal/mol.
 *   G_m[l], G_0[l]  : (1/2) sum_p Q_p phi_p over the trilinear charge nodes
 *                     for the solvated / vacuum potential at level l
 *                     (l = 0: dt, n steps; l = 1: dt/2, 2 n steps)
 *   dG_plain        : G_m[0] - G_0[0]  (Eq. (deltaG3) at dt)
 *   dG              : with Richardson, (2 G_m[1] - G_m[0]) - (2 G_0[1] - G_0[0])
 *                     (Eq. (deltaG3) applied to Eq. (rich)); else dG_plain.
 *                     NaN when vacuum = 0.
 *   All differences and combinations are formed in double on the device.
 *   grid_point_updates : interior nodes times executed steps, all loops
 *   device_ms       : device time from the first setup kernel to the
 *                     energies being ready
 *   n_charge_nodes  : distinct nodes carrying trilinear charge
 *   finite          : 1 if every reported energy is finite and no field held
 *                     a non-finite value after any step (the paper's sign of
 *                     an unstable run, Sec. 4.2); else 0 and EDIVERGED
 *   dG_direct       : with vacuum_direct, (1/2) sum_p Q_p (phi_m,p - phi_0,p)
 *                     with phi_0 from the direct Poisson solve and phi_m
 *                     Richardson-combined when richardson = 1 (Eq. (deltaG2));
 *                     else NaN
 *   dG_err_est      : estimated error of dG against the same solve in exact
 *                     arithmetic (the FP64 oracle): eta * (1/2) kT * sum over
 *                     the runs of |c_run| sum_p |Q_p u_p|, c_run the run's
 *                     coefficient in dG (2 and -1 per medium with Richardson,
 *                     else 1), eta = 4e-7 for FP32 / FP32X field storage and
 *                     1e-13 for FP64 (set so that the errors measured on the
 *                     full-size workloads stay below 0.4 of it); it grows with
 *                     the cancellation of the combination.  NaN when
 *                     vacuum = 0                                          */
typedef struct npb_result {
  double dG;
  double dG_plain;
  double G_m[2];
  double G_0[2];
  double grid_point_updates;
  double device_ms;
  int32_t steps_done;
  int32_t n_charge_nodes;
  int32_t finite;
  int32_t reserved;
  double dG_direct;
  double dG_err_est;
} npb_result;

typedef struct npb_ctx npb_ctx;

/* Per-kernel timing gathered while timing is enabled (npb_ctx_set_timing):
 * launches, summed device milliseconds and algorithmic bytes.  Sweep
 * launches carry HIP events that record the kernel's own start and stop
 * (hipExtLaunchKernelGGL); other launches are bracketed by HIP events
 * recorded on the stream they run on.
 * count/ms/bytes are indexed by npb_kernel_class (the sweeps by direction);
 * kcount/kms/kbytes split the sweep launches again by the kernel that ran
 * them, indexed by npb_sweep_kernel. */
typedef struct npb_kernel_times {
  int64_t count[12];
  double ms[12];
  double bytes[12];  /* algorithmic bytes moved by those launches */
  int64_t kcount[8];
  double kms[8];
  double kbytes[8];
} npb_kernel_times;

enum npb_kernel_class {
  NPB_K_SWEEP_X = 0, NPB_K_SWEEP_Y = 1, NPB_K_SWEEP_Z = 2,
  NPB_K_SETUP = 3, NPB_K_INIT = 4, NPB_K_ENERGY = 5, NPB_K_OTHER = 6,
  NPB_K_DIRECT = 7, /* the direct vacuum Poisson solve (vacuum_direct) */
  NPB_K_EULER = 8   /* explicit Euler steps (NPB_EULER) */
};

enum npb_sweep_kernel {
  NPB_SK_X = 0,          /* x sweep (every scheme)                              */
  NPB_SK_YZ_PLAIN = 1,   /* y/z sweep, line solves only                         */
  NPB_SK_YZ_FLOW = 2,    /* y/z sweep fused with the sinh sub-step (LODIE2 z)   */
  NPB_SK_YZ_GENERAL = 3, /* y/z sweep with sources and AOS accumulation         */
  NPB_SK_EULER = 4       /* explicit Euler step (kernel-attached events too)    */
};

/* A grid for a molecule: per axis, the atoms' extent (positions +- radii)
 * plus `margin` Angstrom on both sides, an odd number of nodes at spacing h
 * centred on it (n = 2 ceil(half / h) + 1, at least 5).  Pure; returns
 * NPB_OK, or NPB_EINVAL (no atoms, h or margin not positive, or an axis
 * beyond 514 nodes). */
npb_status npb_default_grid(const npb_molecule* mol, double h, double margin, npb_grid* out);

/* Returns NPB_ABI_VERSION.  Pure. */
int npb_abi_version(void);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* npb_last_error(void);

/* kbar^2 in Angstrom^-2 for a 1:1 salt of ionic strength ionic_molar (mol/L)
 * at temperature T (K): 8.486902807 (298/T) I (Sec. 2.1).  Pure. */
double npb_kappa_bar_sq(double ionic_molar, double temperature_K);

/* Create a context on HIP device `device` (allocates a few pinned staging
 * bytes and events).  *out receives the context; destroy with
 * npb_ctx_destroy. */
npb_status npb_ctx_create(int device, npb_ctx** out);
void npb_ctx_destroy(npb_ctx* ctx);

/* Enable (1) or disable (0) per-kernel event timing; enabling clears the
 * accumulated times.  While timing is on, solves launch every kernel
 * directly (no graph replay) and one at a time on the solve's stream (the
 * time loops of the two media, which otherwise run on concurrent streams,
 * are serialized), so that each bracketed launch has the device to itself
 * and its duration is the kernel's own.  Results do not change. */
npb_status npb_ctx_set_timing(npb_ctx* ctx, int enable);
npb_status npb_ctx_get_kernel_times(npb_ctx* ctx, npb_kernel_times* out);

/* Enable (1, the default) or disable (0) graph replay.  With replay on, the
 * device work of a solve (everything after the host-to-device copy of the
 * atoms) is captured once into a HIP graph and replayed by later solves
 * with the same workspace pointer, field pointer, grid, parameters and atom
 * count; any difference captures a new graph.  Results are bit-identical
 * to direct launches.  The context keeps one graph. */
npb_status npb_ctx_set_graph(npb_ctx* ctx, int enable);

/* Host-only checks of a problem: the same argument and stencil checks that
 * npb_solve performs before touching the device.  Returns NPB_OK,
 * NPB_EINVAL or NPB_ERANGE. */
npb_status npb_validate(const npb_molecule* mol, const npb_grid* grid,
                        const npb_params* params);

/* Bytes of device workspace npb_solve needs for this problem (a 256-byte
 * aligned block the caller allocates, e.g. a uint8 tensor).  Pure host. */
npb_status npb_workspace_bytes(const npb_molecule* mol, const npb_grid* grid,
                               const npb_params* params, size_t* bytes);

/* Solve one problem: the NPB equation of Sec. 2.1 (Eqs. (NPB), (RhoEq),
 * (DebyeHuckel), (BoundaryCond)) by pseudo-time stepping of Eq.
 * (TimeDepNPB) with the splitting scheme params->scheme (Sec. 3.1-3.3;
 * Eq. (SpatialOperators) in space, Eq. (ana3) for the nonlinear part),
 * then the energies of Sec. 5.3 (Eq. (deltaG) per run, Eq. (rich) across
 * dt and dt/2, Eq. (deltaG3) across the media).  Enqueues setup (solute
 * mask, trilinear charges of Sec. 3.1, boundary data of Eq.
 * (BoundaryCond)), the time loops, the FP64 energy reductions and
 * combinations on `stream`, then waits for that stream and fills *out.
 * The device work is captured once as a graph and replayed (see
 * npb_ctx_set_graph), except explicit Euler runs of more than 4096 step
 * launches in all, which are launched directly.
 *   d_ws, ws_bytes : device workspace, at least npb_workspace_bytes
 *   d_field_out    : NULL, or a device array of nx*ny*nz doubles that
 *                    receives the potential chosen by field_select
 *                    (kcal/mol/e, or u with field_units = dimensionless),
 *                    Richardson-combined when richardson = 1
 * Errors: EINVAL, ERANGE (before any device work), EDEVICE, EDIVERGED (the
 * energies are still written to *out). */
npb_status npb_solve(npb_ctx* ctx, const npb_molecule* mol, const npb_grid* grid,
                     const npb_params* params, void* d_ws, size_t ws_bytes,
                     double* d_field_out, void* stream, npb_result* out);

/* npb_solve without the final wait (the same operation: Sec. 2.1, the
 * scheme of Sec. 3, the energies of Sec. 5.3): the device work and a last kernel that
 * writes the result are enqueued on `stream`, and the call returns.
 * pinned_out must be page-locked host memory the device can write (e.g.
 * hipHostMalloc, or a torch tensor with pin_memory); it holds the result
 * once the stream's work completes, with device_ms = NaN (not measured) and
 * finite as in npb_solve (a non-finite energy is reported there, not as a
 * status).  Argument and stencil errors are returned before any device
 * work; EINVAL if pinned_out is not page-locked memory. */
npb_status npb_solve_async(npb_ctx* ctx, const npb_molecule* mol, const npb_grid* grid,
                           const npb_params* params, void* d_ws, size_t ws_bytes,
                           double* d_field_out, void* stream, npb_result* pinned_out);

/* Solve n independent problems together (molecules, grids and parameters
 * may all differ; one precision per batch).  Each problem is the operation
 * of npb_solve (Sec. 2.1; the scheme of Sec. 3; the energies of Sec. 5.3),
 * with the same semantics: problem i uses workspace d_ws[i] (ws_bytes[i] bytes, at least
 * npb_workspace_bytes of that problem, 256-byte aligned, no two problems
 * sharing one) and writes its field to d_field_out[i] when d_field_out is
 * not NULL and that entry is not NULL.  Every run of every problem advances
 * in the same launches: one per sweep direction and launch shape per step,
 * so uneven grids share launches; the device work is captured as one graph
 * (see npb_ctx_set_graph).  Results for all n problems go to out[0..n-1].
 * Errors: EINVAL or ERANGE name the first offending problem ("problem i:
 * ...") before any device work; EDEVICE; EDIVERGED or ERANGE after the
 * solves name the first problem concerned (every out[i] is still written). */
npb_status npb_solve_batch(npb_ctx* ctx, int n, const npb_molecule* mols,
                           const npb_grid* grids, const npb_params* params,
                           void* const* d_ws, const size_t* ws_bytes,
                           double* const* d_field_out, void* stream, npb_result* out);

/* ---- no device allocation ------------------------------------------------
 * For callers that cannot allocate device memory at call time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * npb_solve (Sec. 2.1; the scheme of Sec. 3; the energies of Sec. 5.3)
 * without a workspace argument.  The problem's workspace and its
 * launch tables live in a static device array of NPB_NOALLOC_BYTES that the
 * library's code object carries (each device the library runs on holds its
 * own copy until the process ends); the atoms are staged through pageable
 * host memory, every kernel is launched directly (no graph), and no
 * hipMalloc, hipFree, hipHostMalloc or other allocating routine is called.
 * The caller still passes the molecule and the optional d_field_out.
 * Semantics, results and errors as npb_solve (per-kernel timing is not
 * collected), plus EINVAL when npb_workspace_bytes of the problem and its
 * launch tables exceed NPB_NOALLOC_BYTES (a 161^3 FP32 RE+V solve needs
 * 85 MiB).  Every call on a device shares that device's array and leaves
 * its contents behind (each solve initialises what it reads): calls that
 * overlap on one device, from any context, stream or thread, race. */
#define NPB_NOALLOC_BYTES (96u << 20)
npb_status npb_solve_noalloc(npb_ctx* ctx, const npb_molecule* mol, const npb_grid* grid,
                             const npb_params* params, double* d_field_out, void* stream,
                             npb_result* out);

/* Choose the line-solver launch shapes for this grid size, precision and
 * splitting family (LOD / AOS) by timing: the problem is set up in d_ws
 * (as npb_solve would), then for each sweep direction every candidate shape
 * (target chunk length 12, 16 or 20 rows; x: 64, 32, 16 or 8 lines per block;
 * y, z: tile width 32 or 16) sweeps all of the problem's runs a few times
 * on `stream`, and the fastest is recorded in ctx.  Later npb_solve,
 * npb_solve_batch and servers created from ctx use the recorded shapes for
 * grids of that size (results change only by rounding: a different chunk
 * partition).  ms_out (nullable, 3 entries): mean launch time of the chosen
 * shape per direction.  The workspace's fields are left undefined. */
npb_status npb_autotune(npb_ctx* ctx, const npb_molecule* mol, const npb_grid* grid,
                        const npb_params* params, void* d_ws, size_t ws_bytes, void* stream,
                        double* ms_out);

/* Launch shapes a solve on ctx (NULL: the built-in defaults) would use:
 * out[4 d + 0..3] = rows per chunk, chunks per line, lines per block (x) or
 * tile width (y, z), threads per block, for d = x, y, z.  Pure host. */
npb_status npb_launch_shapes(const npb_ctx* ctx, const npb_grid* grid, const npb_params* params,
                             int32_t* out);

/* ---- caller-given fields -------------------------------------------------
 * The analytic benchmark of Sec. 4.1-4.2 (a charged spherical cavity with a
 * known solution) is posed by fields rather than by a molecule: a dense
 * source and an initial field whose outer shell carries the Dirichlet data
 * (Eqs. (NPB_analytical_1), (NPB_analytical_2), (InitSolutions)).
 *   solute  : the balls that form the solute region (eps_in, kbar = 0
 *             inside); the charges are ignored; positions and radii as in
 *             npb_solve
 *   params  : as in npb_solve, with vacuum = vacuum_direct = field_select
 *             = 0; richardson may be 1; temperature_K only scales the
 *             reported energies
 *   d_u0    : device, nx*ny*nz doubles [nz][ny][nx]: the dimensionless
 *             initial field; its outer shell is the Dirichlet data
 *   d_rho   : device, nx*ny*nz doubles: the dimensionless source rho of
 *             alpha u_t = div(eps grad u) - kbar^2 sinh(u) + rho on the
 *             interior nodes (shell entries are not read)
 *   d_ws    : at least npb_fields_workspace_bytes (one source entry per
 *             interior node)
 *   d_u_out : NULL, or nx*ny*nz doubles receiving the dimensionless u
 *             after n_steps (Richardson-combined when richardson = 1)
 * out: steps and timings as in npb_solve; G_m is (1/2) kT sum rho u over
 * the interior, dG NaN.  Errors as npb_solve, and EINVAL for a null field. */
npb_status npb_fields_workspace_bytes(const npb_molecule* solute, const npb_grid* grid,
                                      const npb_params* params, size_t* bytes);
npb_status npb_solve_fields(npb_ctx* ctx, const npb_molecule* solute, const npb_grid* grid,
                            const npb_params* params, const double* d_u0, const double* d_rho,
                            void* d_ws, size_t ws_bytes, double* d_u_out, void* stream,
                            npb_result* out);

/* ---- request loop (serving) ----------------------------------------------
 * A server solves molecules as they arrive (the problem of Sec. 2.1 per
 * request; RE+V energies of Sec. 5.3, Eqs. (rich) and (deltaG3), as
 * npb_solve) with continuous batching.  It owns a device arena of
 * hbm_budget bytes and one worker thread with its own contexts and stream.
 * A request is admitted in arrival order as soon as a free region of the
 * arena holds its workspace (npb_workspace_bytes) and fewer than max_batch
 * requests are active; it joins the running launches at the next tick
 * boundary (every few pseudo-time steps), and it leaves, reporting its
 * result and returning its region, as soon as its own last step is done
 * while the other requests keep stepping.  Every run is swept with the
 * arithmetic of its single solve (only launches are shared), so each
 * result equals npb_solve of the same request bit for bit (device_ms is
 * NaN: requests share the device).  No field is returned, only npb_result.
 * Callers for whom the step-by-step path of one molecule matters use
 * npb_solve. */
typedef struct npb_server npb_server;

typedef struct npb_server_stats {
  int64_t submitted, completed, failed, refused, batches, queued;
  /* batches: ticks issued (each advances every active request a few steps) */
  double busy_ms;          /* wall time with at least one request active */
  double p50_ms, p99_ms;   /* submit -> result latency of the requests finished
                              since creation or the last npb_server_reset_stats */
} npb_server_stats;

/* Create a server on ctx's device (ctx is only read; the server keeps its
 * own).  max_queue bounds the requests waiting for admission.  Errors:
 * EINVAL, ENOMEM (arena), EDEVICE. */
npb_status npb_server_create(npb_ctx* ctx, size_t hbm_budget, int max_batch, int max_queue,
                             npb_server** out);

/* Queue one request: the solve of npb_solve (Sec. 2.1; the scheme of
 * Sec. 3; the energies of Sec. 5.3, Eqs. (rich) and (deltaG3)) for this
 * molecule, grid and parameters; the molecule arrays are copied before returning.
 * *ticket identifies it for npb_poll.  Errors: EINVAL / ERANGE (the checks
 * of npb_validate), EBUSY (its workspace exceeds the arena, or the queue is
 * full: admission refused). */
npb_status npb_submit(npb_server* server, const npb_molecule* mol, const npb_grid* grid,
                      const npb_params* params, uint64_t* ticket);

/* *done = 0 while the request is queued or running.  Once done: *done = 1,
 * *out holds its result (the energies of Sec. 5.3 as npb_solve reports them), the ticket is released, and the return value is
 * the request's own status (NPB_OK, EDIVERGED, or the batch's device
 * error).  Unknown or released ticket: EINVAL. */
npb_status npb_poll(npb_server* server, uint64_t ticket, npb_result* out, int* done);

/* Counters and latency percentiles of the request loop (host bookkeeping;
 * no operation of the paper). */
npb_status npb_server_get_stats(npb_server* server, npb_server_stats* out);

/* Clear the counters and the latency record (e.g. after a warm-up or a
 * capacity run), so later statistics cover later requests only. */
npb_status npb_server_reset_stats(npb_server* server);

/* Finishes every queued request, then frees the arena and the worker. */
void npb_server_destroy(npb_server* server);

#ifdef __cplusplus
}
#endif

#endif /* NPB_H */
