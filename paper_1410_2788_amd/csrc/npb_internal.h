// Internal declarations of the NPB HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "npb.h"

namespace npb {

// ---------------------------------------------------------------------------
// FP64 elementary functions of the hot kernels, written from their series
// (no library calls): accurate to a few units in the last place over the
// ranges the kernels use.

// e^x for x <= 0: Cody and Waite's range reduction x = k ln2 + r (ln2 split
// into a head with 31 fraction bits, so that k * head is exact, and the
// rest), |r| <= ln2 / 2, e^r by its Taylor series to degree 13 (truncation
// below 5e-18 relative), then the exponent k added back.
__device__ __forceinline__ double exp_neg(double x) {
  constexpr double kLog2e = 1.4426950408889634;
  constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
  constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
  const double k = __builtin_rint(x * kLog2e);
  double r = fma(-k, kLn2Hi, x);
  r = fma(-k, kLn2Lo, r);
  // 1/n!, n = 13 .. 0
  double p = 1.0 / 6227020800.0;
  p = fma(p, r, 1.0 / 479001600.0);
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return __builtin_ldexp(p, (int)k);
}

// 1/x for x > 0 (normal): the hardware estimate refined by two Newton steps
__device__ __forceinline__ double rcp_newton(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// ln(1 + x) for x >= 0: 2 atanh(s) with s = x / (2 + x) while 1 + x < sqrt 2
// (no cancellation for small x); beyond, 1 + x = 2^e f with f in
// [sqrt(1/2), sqrt 2) and s = (f - 1) / (f + 1).  |s| <= 0.1716, so the
// odd series s + s^3/3 + ... + s^19/19 leaves a truncation below 1e-17.
__device__ __forceinline__ double log1p_nonneg(double x) {
  constexpr double kLn2 = 0.6931471805599453;
  double s, e = 0.0;
  if (x < 0.41421356237309503) {
    s = x * rcp_newton(2.0 + x);
  } else {
    const double y = 1.0 + x;
    int ex = 0;
    double f = __builtin_frexp(y, &ex);  // y = f 2^ex, f in [1/2, 1)
    if (f < 0.70710678118654752) {
      f *= 2.0;
      ex -= 1;
    }
    e = (double)ex;
    s = (f - 1.0) * rcp_newton(f + 1.0);
  }
  const double s2 = s * s;
  double p = 1.0 / 19.0;
  p = fma(p, s2, 1.0 / 17.0);
  p = fma(p, s2, 1.0 / 15.0);
  p = fma(p, s2, 1.0 / 13.0);
  p = fma(p, s2, 1.0 / 11.0);
  p = fma(p, s2, 1.0 / 9.0);
  p = fma(p, s2, 1.0 / 7.0);
  p = fma(p, s2, 1.0 / 5.0);
  p = fma(p, s2, 1.0 / 3.0);
  p = fma(p, s2, 1.0);
  return fma(e, kLn2, 2.0 * s * p);
}

// device of a context (the server's worker uses the same device), and the
// tuned line-solver shapes it hands to a server's own context
int ctx_device(const npb_ctx* ctx);
void copy_tuning(const npb_ctx* from, npb_ctx* to);

// Continuous stepping for the request loop (one precision): problems join
// at tick boundaries and leave as soon as their last step is done.
struct RollingDone {
  uint64_t id;
  npb_status status;
  npb_result res;
};
struct RollingEngine {
  virtual ~RollingEngine() {}
  // a problem checked by npb_workspace_bytes, with its own workspace (>= its
  // npb_workspace_bytes, 256-byte aligned); mol, grid and params stay valid
  // until the problem is reported by poll; its setup is enqueued by the
  // next tick
  virtual npb_status add(uint64_t id, const npb_molecule* mol, const npb_grid* grid,
                         const npb_params* params, void* ws, size_t ws_bytes) = 0;
  // enqueue the setup of added problems, up to `steps` steps of every
  // active run, and the energies and result copy of each problem whose last
  // step that was; waits while two earlier ticks are still on the device
  virtual npb_status tick(int steps) = 0;
  // problems whose results are on the host: appended to out, then forgotten
  virtual void poll(std::vector<RollingDone>& out) = 0;
  // problems added and not yet reported; of these, those with steps left
  virtual int active() const = 0;
  virtual int stepping() const = 0;
  // wait for everything enqueued
  virtual npb_status drain() = 0;
  // after a failed tick: wait for the device, then report every problem
  // with status s and forget it
  virtual void abort_all(npb_status s, std::vector<RollingDone>& out) = 0;
};
// tuned: a context whose tuned launch shapes the engine's contexts copy
npb_status rolling_create(const npb_ctx* tuned, int precision, void* stream, int max_items,
                          RollingEngine** out);

// ---------------------------------------------------------------------------
// Arguments of one implicit line sweep (one of the 1-D sub-steps of the
// LOD / AOS splitting).  The face coefficient of the row for node i is
// r * eps(i +- 1/2), r = tau / h^2, with eps at a half point chosen from the
// two nodal solute flags (both solvent, mixed = harmonic mean, both solute).
template <typename T>
struct SweepArgs {
  T* u;                   // field, [nz][ny][nxp]; read, and written in place
  T* acc;                 // additive-splitting accumulator (AOS modes)
  const uint8_t* mask;    // bit 0: solute node, [nz][ny][nxp]; nullptr = uniform medium;
                          // face rule by location: bit 1 = the half point to the next
                          // node along this sweep's direction is solute
  int nx, ny, nz;
  int nxp;                // row pitch in elements: nx rounded up to a multiple of 4
  double re[3];           // r*eps_face for (sum of the two flags) = 0, 1, 2
  double re_uniform;      // r*eps_in for the uniform (vacuum) medium
  // exact sinh flow over theta: ka = 1 + exp(-2 theta), kb = 1 - exp(-2 theta)
  int pre_nl;  double pre_ka, pre_kb;    // applied to the input before the solve
  int post_nl; double post_ka, post_kb;  // applied to the solution
  int aos_w;   double aos_ka, aos_kb;    // AOS: W = flow(u) folded into acc
  // trilinear source: value coef * rho added at charge nodes of each line
  int src_stage;          // 0 none, 1 before the solve, 2 after the solve
  double src_coef;
  const int* src_ptr;     // per-line offsets into src_lin / src_rho
  const int* src_lin;     // linear node index of each entry
  const double* src_rho;  // source density at that node
  int mode;               // 0 in place, 1 acc = (W+V)/4, 2 acc += P/4, 3 u = acc + Q/4
  int cn;                 // Crank-Nicolson: the right-hand side is (1 + r delta^2) s with
                          // the implicit side's face coefficients; 1: of the input with
                          // its sources (LOD), 2: before the sources are added (additive)
  double aos_ww, aos_wv;  // additive modes: weights of W and of this direction's
                          // solution in the mean (AOS 1/4 and 1/4, MAOS 0 and 1/3)
  int face_loc;           // 1: face class from bit 1 of the lower node's flag (0 or 2)
  // per (chunk, line) face class of this direction's launch shape: 0 = every
  // face of the chunk solvent-solvent, 2 = every face solute-solute, 1 =
  // mixed; nullptr for the uniform medium (all chunks uniform)
  const uint8_t* ccls;
  // ChunkTab<A> of this field and direction (device memory)
  const void* tab;
  // set to 1 when a stored value is not finite; the z sweep's arguments only
  // (the last sub-step of every split scheme), nullptr elsewhere
  int* nonfinite;
  // x sweep: the run's Dirichlet data in shell order (FP64), from which the
  // right end of each x-line is read when node nx-1 would be the only node
  // of its row's last cache line (the row loads then stop before it)
  const double* bcx;
  // geometry of the launch
  int M;                  // rows per chunk (compile-time in the kernel)
  int P;                  // chunks per line
  int LW;                 // lines per block (x: rows, y/z: consecutive x)
  int S;                  // x: LDS elements per row; y/z: LDS tile rows
};

enum SweepMode { MODE_INPLACE = 0, MODE_AOS_FIRST = 1, MODE_AOS_ADD = 2, MODE_AOS_FINISH = 3 };

// Runs (fields) of one problem: solvated and vacuum at dt and dt/2.
constexpr int kMaxFields = 4;

// y/z sweep variants (fused pointwise work compiled in):
//   kYzPlain   : solve only, in place
//   kYzFlow    : solve, then the exact sinh flow on solvent nodes
//   kYzGeneral : sources before/after, flow, AOS accumulation (run-time flags)
enum { kYzPlain = 0, kYzFlow = 1, kYzGeneral = 2 };

// Chunk lengths compiled into the sweep kernels (the planners keep the
// chunk within 20 rows, where a lane's chunk still fits its registers).
constexpr int kChunkChoices[] = {4, 8, 12, 16, 20};

struct LaunchShape {
  int M, P, LW, threads, blocks;
  size_t lds;
  int S;  // x: LDS elements per tile row; y/z: LDS tile rows
};

// Row pitch of every field-shaped array (the mask shares it): rows start
// on 128-byte boundaries of the field (one cache line), so the pieces of
// consecutive x that a y/z tile moves per node row cover whole lines.  The
// sweeps move the first row4(nx) elements of a row in 16-byte pieces;
// padding columns nx..nxp-1 hold zeros (field) or 0 (mask) and are never
// solved.  es = bytes per field element.
__host__ __device__ inline int row4(int nx) { return (nx + 3) & ~3; }
// LDS elements per row of an x-sweep tile.  FP32: one more than a multiple
// of 32, so that the four rows x eight 16-byte pieces a half-wave moves,
// and the 32 lines' chunk rows it reads, fall in distinct banks.  FP64
// (two banks per element): one more than row4(nx).
inline int x_tile_stride(int nx, bool fp64) {
  const int nx4 = row4(nx);
  return fp64 ? nx4 + 1 : ((nx4 + 31) & ~31) + 1;
}
inline int pitch_of(int nx, int es) {
  const int q = 128 / es;
  return (nx + q - 1) / q * q;
}

constexpr int kMaxChunk = 20;  // longest chunk compiled into the sweeps
// Elimination constants of a chunk whose M+1 faces all carry the same
// coefficient re (rows with alpha = gamma = re and leak 1), index t = 0:
// solvent chunks (or the uniform medium), t = 1: solute chunks.  inv, ga,
// al: pivot reciprocals and the negated couplings of the eliminated rows
// (ga = -gam_k, al = -lam_k); rf_c, rf_l: gamma and leak of the reduced row
// of x_0 (its alpha is re, or 0 with re added to the leak on a line's
// first chunk); rl_a, rl_c, rl_l: alpha, gamma and leak of the reduced row
// of x_{M-1}.  rf_lt: leak of the reduced row of x_0 in a line's last chunk
// when that chunk ends inside (its last real row kt = (nint - 1) mod M,
// 1 <= kt <= M - 2, couples to the right Dirichlet node; its gamma is then
// zero).  Computed in double by the leak recurrences of the sweeps.
template <typename A>
struct ChunkTab {
  A inv[2][kMaxChunk];
  A ga[2][kMaxChunk];
  A al[2][kMaxChunk];
  A re[2];
  A rf_c[2], rf_l[2], rl_a[2], rl_c[2], rl_l[2];
  A rf_lt[2];
};

// Pick chunk length / chunk count and the block shape for a line length.
// plan_x: fp64 = arithmetic type is double.  plan_yz: lines along an axis of
// n_along nodes, n_other nodes on the other transverse axis.
// mt: target chunk length (0 = default), lw / tw: preferred lines per block
// (x: 32, 16, 8) or tile width (y/z: 16, 32); 0 = default heuristic.  An
// unsupported combination returns a shape with M == 0.
LaunchShape plan_x(int nx, int ny, int nz, bool fp64, bool aos, bool uniform, int mt = 0,
                   int lw = 0);
LaunchShape plan_yz(int nx, int n_along, int n_other, bool fp64, int mt = 0, int tw = 0);

// Largest chunk count per line any planner choice can produce (chunk-class
// tables are sized for it, so the workspace does not depend on the choice).
inline int max_chunks(int n_along, bool x_dir) {
  const int nint = n_along - 2;
  int P = (nint + 11) / 12;  // shortest target chunk a tuner tries: 12 rows
  if (x_dir) {               // x chunk counts are powers of two
    int q = 1;
    while (q < P) q <<= 1;
    P = q;
  }
  return P;
}

// number of interior lines of a direction (entries per chunk of its class
// table): x lines (y, z) -> (z-1)(ny-2) + y-1; y lines (z, x) -> (z-1)(nx-2)
// + x-1; z lines (y, x) -> (y-1)(nx-2) + x-1
inline long long class_lines(int nx, int ny, int nz, int dir) {
  if (dir == 0) return (long long)(ny - 2) * (nz - 2);
  return (long long)(nx - 2) * ((dir == 1 ? nz : ny) - 2);
}

// Elimination constants for chunks of M rows whose faces all carry re_t
// (t = 0: solvent or uniform medium, t = 1: solute), computed in double.
template <typename A>
void fill_chunk_tab(ChunkTab<A>& tb, double re_solvent, double re_solute, int M, int nint);

// A sweep launch covers any set of fields (of any grids) that share a
// launch shape: args is a device array of per-field arguments, already
// shaped (shape_args), and work[b] = (field, block of that field) for each
// of the nblocks blocks.  T = storage type of the field, A = arithmetic
// type of the line solves.
template <typename T>
void shape_args(SweepArgs<T>& a, int dir, const LaunchShape& s);
template <typename T>
int sweep_variant(const SweepArgs<T>* a, int n);  // kYz* covering every field
template <typename T>
int sweep_cn(const SweepArgs<T>* a, int n);       // 1 if any field is Crank-Nicolson
// nbu > 0: every field has nbu blocks and block b is (b / nbu, b % nbu);
// work may then be null.
// cn: compile the Crank-Nicolson right-hand side in (some field has cn set)
template <typename T, typename A>
hipError_t launch_sweep_x(const SweepArgs<T>* args, const int2* work, int nbu, int nblocks,
                          int cn, const LaunchShape& s, hipStream_t st);
// Per-kernel timing of the sweeps: while (start, stop) are set (non-null),
// sweep launches from this host thread record their kernel's own start and
// stop in them.  Cleared by passing nullptrs.
void set_sweep_launch_events(hipEvent_t start, hipEvent_t stop);
template <typename T, typename A>
hipError_t launch_sweep_yz(const SweepArgs<T>* args, const int2* work, int nbu, int nblocks,
                           int dir, int var, const LaunchShape& s, hipStream_t st);

// ---------------------------------------------------------------------------
// setup

struct SetupArgs {
  int nx, ny, nz, nxp;
  double h, ox, oy, oz;
  int n_atoms;
  const double* atoms;    // [5][n_atoms]: x, y, z, q, radius
};

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st);
hipError_t launch_copy_u32(const uint32_t* src, uint32_t* dst, size_t n, hipStream_t st);
hipError_t launch_mask_raster(const SetupArgs& a, uint8_t* mask, hipStream_t st);
// face rule by location: bit 1 of fmask (a copy of the mask) on every node
// whose half point to the next node along dir (0 x, 1 y, 2 z) is solute
hipError_t launch_face_raster(const SetupArgs& a, int dir, const uint8_t* mask, uint8_t* fmask,
                              hipStream_t st);
hipError_t launch_stencil(const SetupArgs& a, int* key, int* id, double* val, int* err,
                          hipStream_t st);
// Stable LSD radix sort of (key, id) pairs by key; n items, keys < key_limit.
// Result in (key_a, id_a); (key_b, id_b) are scratch.  hist holds at least
// 256 * ceil(n/256) ints.
hipError_t radix_sort_pairs(int* key_a, int* id_a, int* key_b, int* id_b, int* hist,
                            int n, long long key_limit, hipStream_t st);
// aux: scan_aux_ints(n) ints of scratch (multi-block scan), or nullptr
hipError_t launch_exclusive_scan(int* data, int n, int* total, int* aux, hipStream_t st);
int scan_aux_ints(int n);
hipError_t launch_merge_charges(const int* key, const int* id, const double* val, int* heads,
                                int n, int* nq_dev, int* q_idx, double* q_val,
                                double* q_rho, double rho_pref, int* scan_aux, hipStream_t st);
hipError_t launch_line_ptr(const int* sorted_keys, const int* n_dev, int cap, int n_lines,
                           int keys_per_line, int* ptr, hipStream_t st);
// linear node indices are pitched (row pitch nxp); the keys order by line
// (dense line numbering z * nx + x for y lines, y * nx + x for z lines)
hipError_t launch_axis_keys(const int* q_idx, const int* nq_dev, int cap, int nx, int nxp, int ny,
                            int nz, int axis, int* key, int* id, hipStream_t st);
hipError_t launch_gather_entries(const int* id, const int* nq_dev, int cap, const int* q_idx,
                                 const double* q_rho, int* lin_out, double* rho_out,
                                 hipStream_t st);
// Dirichlet values of the solvated (eps_s, kappa; into bc_s) and the vacuum
// (eps_v, no screening; into bc_v) medium on the outer shell, in shell
// order; a null pointer skips that medium (either medium's values do not
// depend on whether the other is computed in the same launch).
// fp32_terms: per-pair terms in FP32 (sums stay FP64).
hipError_t launch_boundary(const SetupArgs& a, double eps_s, double kappa, double eps_v,
                           double lB, double* bc_s, double* bc_v, bool fp32_terms,
                           hipStream_t st);
// caller-given fields (npb_solve_fields): one source-list entry per
// interior node (key = pitched index, value = rho of the dense array), and
// the shell values of a dense field in shell order
hipError_t launch_dense_source(const double* rho, int nx, int nxp, int ny, int nz, int* key,
                               int* id, double* val, hipStream_t st);
hipError_t launch_shell_from_dense(const double* u0, int nx, int ny, int nz, double* bc,
                                   hipStream_t st);
// chunk classes of direction dir (0 = x, 1 = y, 2 = z) for chunks of M rows,
// P per line; out[p * class_lines + line]
hipError_t launch_chunk_classes(const uint8_t* mask, int nx, int nxp, int ny, int nz, int dir,
                                int M, int P, int face_loc, uint8_t* out, hipStream_t st);

// ---------------------------------------------------------------------------
// field / energy helpers

template <typename T>
hipError_t launch_field_init(T* u, const double* bc, int nx, int nxp, int ny, int nz,
                             hipStream_t st);
// pitched u = dense [nz][ny][nx] array (padding columns zero)
template <typename T>
hipError_t launch_field_from_dense(T* u, const double* src, int nx, int nxp, int ny, int nz,
                                   hipStream_t st);
// dense out[nz][ny][nx] = beta * out + gamma * u (pitched u)
template <typename T>
hipError_t launch_field_out(double* out, const T* u, int nx, int nxp, int ny, int nz, double beta,
                            double gamma, hipStream_t st);
// res = [dG, dG_plain, G_m0, G_m1, G_00, G_01, finite, dG_direct]; S[4] is the
// charge-weighted sum of the direct vacuum solve when direct != 0
hipError_t launch_combine(const double* S, double kT, int richardson, int vacuum, int direct,
                          double* res, hipStream_t st);

// the result of problem into page-locked host memory (npb_solve_async)
hipError_t launch_result(const double* res, const int* ints, npb_result* out, double points,
                         int steps, hipStream_t st);

// number of nodes on the outer shell of an nx*ny*nz grid
inline long long shell_count(int nx, int ny, int nz) {
  return (long long)nx * ny * nz - (long long)(nx - 2) * (ny - 2) * (nz - 2);
}

// Position of shell node (i, j, k) in the shell order of the boundary data:
// face z = 0 (ny*nx, x fastest), face z = nz-1, then per interior z the row
// y = 0 (nx), the row y = ny-1 (nx), and x = 0, nx-1 of each interior y.
__host__ __device__ inline long long shell_slot(int i, int j, int k, int nx, int ny, int nz) {
  const long long nxy = (long long)nx * ny;
  if (k == 0) return (long long)j * nx + i;
  if (k == nz - 1) return nxy + (long long)j * nx + i;
  const long long base = 2 * nxy + (long long)(k - 1) * (2LL * nx + 2LL * (ny - 2));
  if (j == 0) return base + i;
  if (j == ny - 1) return base + nx + i;
  return base + 2LL * nx + 2LL * (j - 1) + (i == 0 ? 0 : 1);
}

// ---------------------------------------------------------------------------
// vacuum potential by a direct Poisson solve (poisson_kernels.hip)

struct DirectPoissonArgs {
  int nx, ny, nz, nxp;     // grid (nxp: row pitch of the pitched charge indices)
  double h, eps;
  const double* bc;        // vacuum Dirichlet data, shell order
  const int* q_idx;        // charge nodes (pitched linear index)
  const double* q_rho;     // source density at them
  const double* q_val;     // trilinear charge at them (e)
  const int* nq_dev;       // number of charge nodes (device)
  int cap;                 // capacity of the charge list
  double* work;            // direct_poisson_bytes(nx, ny, nz) bytes
  double* slot;            // receives sum over charge nodes of q u
};

// Workspace of the solve: the interior field and the transform tables.
size_t direct_poisson_bytes(int nx, int ny, int nz);
// Solves into work (interior nodes, dense [nz-2][ny-2][nx-2]) and writes
// the charge-weighted sum to slot.
hipError_t launch_direct_poisson(const DirectPoissonArgs& a, hipStream_t st);
// dense out[nz][ny][nx] = beta * out + gamma * (interior u, shell bc)
hipError_t launch_direct_field_out(double* out, const double* u, const double* bc, int nx, int ny,
                                   int nz, double beta, double gamma, hipStream_t st);

// ---------------------------------------------------------------------------
// explicit Euler steps (euler_kernels.hip), FP64

struct EulerArgs {
  const double* u;        // field at step n, [nz][ny][nxp]
  double* v;              // field at step n + 1 (interior written; shell kept)
  const uint8_t* flags;   // bit 0 solute node, bits 1-6 its neighbours' solute bits,
                          // bit 7 node with a source entry (launch_euler_flags)
  const int* src_ptr;     // per-x-line offsets into q_idx / q_rho (line k*ny + j)
  const int* q_idx;       // pitched linear index of each charge node, sorted
  const double* q_rho;    // source density at it
  int nx, ny, nz, nxp;
  int zc;                 // z planes per block (euler_z_chunk)
  int uniform;            // 1: uniform medium (vacuum), re_uniform on every face
  int nl;                 // 1: kbar^2 sinh(u) term on solvent nodes
  double re[3];           // tau eps_face / h^2 for (sum of the two solute bits) = 0, 1, 2
  double re_uniform;
  double tau;             // dt / alpha (source coefficient)
  double tk;              // tau kbar^2
  int face_loc;           // 1: flag bits 1-6 are the faces' own solute bits (face rule
                          // by location): face = re[0] or re[2]
  int* nonfinite;         // set to 1 when a stored value is not finite
  int tiles_x, tiles_y, ntiles, per;  // filled by launch_euler_step
};

int euler_z_chunk(int nx, int ny, int nz);
// flags from the solute mask (nullptr: none) and the charge list; with
// the face rule by location, fmask[3] (x, y, z half-point bits in bit 1)
// give the six face bits instead of the neighbours' solute bits
hipError_t launch_euler_flags(const uint8_t* mask, const uint8_t* const* fmask, const int* q_idx,
                              const int* nq, int cap, uint8_t* flags, int nx, int nxp, int ny,
                              int nz, hipStream_t st);
// one step; start / stop (both or neither) are recorded by the kernel itself
hipError_t launch_euler_step(const EulerArgs& a, hipEvent_t start, hipEvent_t stop,
                             hipStream_t st);

}  // namespace npb
