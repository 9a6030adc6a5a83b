// Host runtime of the NPB library: C ABI, validation, workspace layout and
// the sequence of device launches of one solve.  Also the small field and
// energy kernels (field initialisation, FP64 energy gathers, the
// solvated-minus-vacuum and Richardson combinations).
#include <algorithm>
#include <array>
#include <cmath>
#include <list>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "npb.h"
#include "npb_internal.h"

using namespace npb;

// ---------------------------------------------------------------------------
// constants of the dimensionless model (Sec. 2.1)
namespace {

constexpr double kKT298 = 0.592183;          // kcal/mol at 298 K
constexpr double kKbar2PerMolar298 = 8.486902807;  // Angstrom^-2 per mol/L at 298 K
constexpr double kCoulomb = 332.06371;       // kcal Angstrom / (mol e^2)

double thermal_energy(double T) { return kKT298 * T / 298.0; }
double bjerrum(double T) { return kCoulomb / thermal_energy(T); }

thread_local std::string g_err;

npb_status fail(npb_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

}  // namespace

#define NPB_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(NPB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));      \
  } while (0)

// ---------------------------------------------------------------------------
// field / energy kernels

namespace npb {

// Dirichlet values (shell order of the boundary kernel) on the outer shell,
// zero inside and in the padding columns
template <typename T>
__global__ void field_init_kernel(T* u, const double* bc, int nx, int nxp, int ny, int nz) {
  const long long n = (long long)nxp * ny * nz;
  const long long nxy = (long long)nx * ny;
  const long long ring = 2LL * nx + 2LL * (ny - 2);
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    int i = (int)(p % nxp);
    long long t = p / nxp;
    int j = (int)(t % ny);
    int k = (int)(t / ny);
    T v = T(0);
    if (i >= nx) {
      v = T(0);
    } else if (k == 0) {
      v = (T)bc[(long long)j * nx + i];
    } else if (k == nz - 1) {
      v = (T)bc[nxy + (long long)j * nx + i];
    } else {
      long long base = 2 * nxy + (long long)(k - 1) * ring;
      if (j == 0)
        v = (T)bc[base + i];
      else if (j == ny - 1)
        v = (T)bc[base + nx + i];
      else if (i == 0)
        v = (T)bc[base + 2LL * nx + 2LL * (j - 1)];
      else if (i == nx - 1)
        v = (T)bc[base + 2LL * nx + 2LL * (j - 1) + 1];
    }
    u[p] = v;
  }
}

// the runs of one problem at once: block row blockIdx.y = run
template <typename T>
struct InitSet {
  T* u[kMaxFields];
  const double* bc[kMaxFields];
};
// One node row (j, k) per wave, 16-byte stores along it; the row's indices
// are wave-uniform, so only the boundary columns of interior rows branch.
template <typename T>
__global__ __launch_bounds__(256) void field_init_multi_kernel(InitSet<T> set, int nx, int nxp,
                                                               int ny, int nz) {
  constexpr int VX = 16 / (int)sizeof(T);
  const int r = blockIdx.y;
  const int row = blockIdx.x * 4 + (int)(threadIdx.x >> 6);  // row = k * ny + j
  if (row >= ny * nz) return;
  const int k = row / ny, j = row - k * ny;
  T* u = set.u[r] + (size_t)row * nxp;
  const double* bc = set.bc[r];
  const long long nxy = (long long)nx * ny;
  const long long ring = 2LL * nx + 2LL * (ny - 2);
  const bool face = (k == 0 || k == nz - 1 || j == 0 || j == ny - 1);
  const long long base = (k == 0)        ? (long long)j * nx
                         : (k == nz - 1) ? nxy + (long long)j * nx
                         : (j == 0)      ? 2 * nxy + (long long)(k - 1) * ring
                         : (j == ny - 1) ? 2 * nxy + (long long)(k - 1) * ring + nx
                                         : 2 * nxy + (long long)(k - 1) * ring + 2LL * nx +
                                               2LL * (j - 1);
  for (int c = (int)(threadIdx.x & 63) * VX; c < nxp; c += 64 * VX) {
    T v[VX];
#pragma unroll
    for (int q = 0; q < VX; ++q) {
      const int x = c + q;
      T val = T(0);
      if (x < nx) {
        if (face)
          val = (T)bc[base + x];
        else if (x == 0)
          val = (T)bc[base];
        else if (x == nx - 1)
          val = (T)bc[base + 1];
      }
      v[q] = val;
    }
    if constexpr (VX == 4)
      *reinterpret_cast<float4*>(u + c) = make_float4(v[0], v[1], v[2], v[3]);
    else
      *reinterpret_cast<double2*>(u + c) = make_double2(v[0], v[1]);
  }
}

template <typename T>
hipError_t launch_field_init_multi(const InitSet<T>& set, int nruns, int nx, int nxp, int ny,
                                   int nz, hipStream_t st) {
  const int rows = ny * nz;
  hipLaunchKernelGGL((field_init_multi_kernel<T>), dim3((unsigned)((rows + 3) / 4), nruns),
                     dim3(256), 0, st, set, nx, nxp, ny, nz);
  return hipGetLastError();
}

// Energy sums of the runs of one problem: sum q u and, beside it, sum |q u|
// (the scale of the rounding error of the sum's terms).  Block (b, r) sums
// entries b*1024 + t, b*1024 + t + nb*1024, ... of run r into partial (b, r)
// by a fixed tree; a second kernel adds each run's nb partials in a fixed
// order, so the result does not depend on scheduling.
template <typename T>
struct EnergySet {
  const T* u[kMaxFields];
  double* slot[kMaxFields];
  double* aslot[kMaxFields];
};
constexpr int kEnergyMaxBlocks = 64;
template <typename T>
__global__ __launch_bounds__(1024) void energy_part_kernel(EnergySet<T> set, const int* q_idx,
                                                           const double* q_val,
                                                           const int* nq_dev, double* part) {
  __shared__ double ps[1024], pa[1024];
  const int r = blockIdx.y, nb = gridDim.x;
  const T* u = set.u[r];
  const int nq = *nq_dev;
  double s = 0.0, sa = 0.0;
  for (int k = blockIdx.x * 1024 + threadIdx.x; k < nq; k += nb * 1024) {
    const double t = q_val[k] * (double)u[q_idx[k]];
    s += t;
    sa += fabs(t);
  }
  ps[threadIdx.x] = s;
  pa[threadIdx.x] = sa;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      ps[threadIdx.x] += ps[threadIdx.x + w];
      pa[threadIdx.x] += pa[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * (r * nb + blockIdx.x)] = ps[0];
    part[2 * (r * nb + blockIdx.x) + 1] = pa[0];
  }
}
template <typename T>
__global__ void energy_finish_kernel(EnergySet<T> set, const double* part, int nb) {
  const int r = threadIdx.x;
  if (r >= (int)blockDim.x) return;
  double s = 0.0, sa = 0.0;
  for (int b = 0; b < nb; ++b) {
    s += part[2 * (r * nb + b)];
    sa += part[2 * (r * nb + b) + 1];
  }
  *set.slot[r] = s;
  *set.aslot[r] = sa;
}

template <typename T>
hipError_t launch_energy_multi(const EnergySet<T>& set, int nruns, const int* q_idx,
                               const double* q_val, const int* nq_dev, int cap, double* part,
                               hipStream_t st) {
  const int nb = std::max(1, std::min(kEnergyMaxBlocks, (cap + 4095) / 4096));
  hipLaunchKernelGGL((energy_part_kernel<T>), dim3(nb, nruns), dim3(1024), 0, st, set, q_idx,
                     q_val, nq_dev, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((energy_finish_kernel<T>), dim3(1), dim3(nruns), 0, st, set, part, nb);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_field_init(T* u, const double* bc, int nx, int nxp, int ny, int nz,
                             hipStream_t st) {
  long long n = (long long)nxp * ny * nz;
  long long blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL((field_init_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, st, u, bc, nx,
                     nxp, ny, nz);
  return hipGetLastError();
}

// pitched u = dense [nz][ny][nx] array, padding columns zero
template <typename T>
__global__ void field_from_dense_kernel(T* u, const double* src, int nx, int nxp, int ny, int nz) {
  const long long n = (long long)nxp * ny * nz;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(p % nxp);
    const long long row = p / nxp;
    u[p] = i < nx ? (T)src[row * nx + i] : T(0);
  }
}

template <typename T>
hipError_t launch_field_from_dense(T* u, const double* src, int nx, int nxp, int ny, int nz,
                                   hipStream_t st) {
  long long blocks = ((long long)nxp * ny * nz + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL((field_from_dense_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, st, u,
                     src, nx, nxp, ny, nz);
  return hipGetLastError();
}

template <typename T>
__global__ void field_out_kernel(double* out, const T* u, int nx, int nxp, long long n,
                                 double beta, double gamma) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long row = i / nx;
    double v = gamma * (double)u[row * nxp + (i - row * nx)];
    out[i] = (beta != 0.0) ? beta * out[i] + v : v;
  }
}

template <typename T>
hipError_t launch_field_out(double* out, const T* u, int nx, int nxp, int ny, int nz, double beta,
                            double gamma, hipStream_t st) {
  const long long n = (long long)nx * ny * nz;
  long long blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL((field_out_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, st, out, u, nx,
                     nxp, n, beta, gamma);
  return hipGetLastError();
}

// S = [solvated dt, solvated dt/2, vacuum dt, vacuum dt/2, direct vacuum]
// sums of q u, Sa the same runs' sums of |q u|, nf the runs' non-finite
// flags (by run index), eta the relative rounding error of one run's sum
// for the storage precision.  res = [dG, dG_plain, G_m0, G_m1, G_00, G_01,
// finite, dG_direct, dG_err_est]
__global__ void combine_kernel(const double* S, const double* Sa, const int* nf, int nruns,
                               double eta, double kT, int richardson, int vacuum, int direct,
                               double* res) {
  const double h = 0.5 * kT;
  double Gm0 = h * S[0], Gm1 = richardson ? h * S[1] : 0.0;
  double G00 = vacuum ? h * S[2] : 0.0, G01 = (vacuum && richardson) ? h * S[3] : 0.0;
  double nan = __longlong_as_double(0x7ff8000000000000LL);
  double dplain = vacuum ? h * (S[0] - S[2]) : nan;
  double dG = dplain;
  if (vacuum && richardson) dG = h * ((2.0 * S[1] - S[0]) - (2.0 * S[3] - S[2]));
  res[0] = dG;
  res[1] = dplain;
  res[2] = Gm0;
  res[3] = Gm1;
  res[4] = G00;
  res[5] = G01;
  bool fin = isfinite(Gm0) && isfinite(Gm1) && isfinite(G00) && isfinite(G01) &&
             (!vacuum || (isfinite(dG) && isfinite(dplain)));
  // a field that held a non-finite value after a step
  for (int r = 0; r < nruns; ++r) fin = fin && nf[r] == 0;
  // Eq. (deltaG2): the solvated potential (Richardson-combined when on)
  // against the vacuum potential of the direct Poisson solve
  const double dd = direct ? h * ((richardson ? 2.0 * S[1] - S[0] : S[0]) - S[4]) : nan;
  res[7] = dd;
  if (direct) fin = fin && isfinite(dd);
  res[6] = fin ? 1.0 : 0.0;
  // error estimate of dG: each run's sum carries a relative error eta of
  // its scale sum |q u|, weighted by the run's coefficient in dG (2 and -1
  // per medium with Richardson, 1 without)
  double est = nan;
  if (vacuum) {
    const double w1 = richardson ? 2.0 : 0.0, w0 = 1.0;
    est = eta * h * ((w0 * Sa[0] + w1 * Sa[1]) + (w0 * Sa[2] + w1 * Sa[3]));
  }
  res[8] = est;
}

hipError_t launch_combine(const double* S, const double* Sa, const int* nf, int nruns,
                          double eta, double kT, int richardson, int vacuum, int direct,
                          double* res, hipStream_t st) {
  hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(1), 0, st, S, Sa, nf, nruns, eta, kT,
                     richardson, vacuum, direct, res);
  return hipGetLastError();
}

// npb_solve_async: the result straight into page-locked host memory
__global__ void result_kernel(const double* res, const int* ints, npb_result* out,
                              double points, int steps) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  npb_result r{};
  r.dG = res[0];
  r.dG_plain = res[1];
  r.G_m[0] = res[2];
  r.G_m[1] = res[3];
  r.G_0[0] = res[4];
  r.G_0[1] = res[5];
  r.finite = res[6] != 0.0 ? 1 : 0;
  r.dG_direct = res[7];
  r.dG_err_est = res[8];
  r.grid_point_updates = points;
  r.device_ms = __longlong_as_double(0x7ff8000000000000LL);
  r.steps_done = steps;
  r.n_charge_nodes = ints[0];
  *out = r;
}

hipError_t launch_result(const double* res, const int* ints, npb_result* out, double points,
                         int steps, hipStream_t st) {
  hipLaunchKernelGGL(result_kernel, dim3(1), dim3(64), 0, st, res, ints, out, points, steps);
  return hipGetLastError();
}

template hipError_t launch_field_init<float>(float*, const double*, int, int, int, int,
                                             hipStream_t);
template hipError_t launch_field_init<double>(double*, const double*, int, int, int, int,
                                              hipStream_t);

}  // namespace npb

// ---------------------------------------------------------------------------
// Static scratch of npb_solve_noalloc: the workspace of one problem and its
// launch tables live in this array, which the code object brings with it,
// so that call allocates no device memory.  Every device the library runs
// on holds its own copy until the process ends.  Host code never uses the
// array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device (scratch_address below).
static __device__ __align__(256) unsigned char scratch[NPB_NOALLOC_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_addr;  // device -> address of `scratch`

// With `device` current: this device's address of the static scratch.
hipError_t scratch_address(int device, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  *out = static_cast<unsigned char*>(ptr);
  g_scratch_addr[device] = *out;
  return hipSuccess;
}

}  // namespace

// ---------------------------------------------------------------------------
// context

// Everything a captured solve graph depends on besides the staged bytes,
// per problem of the batch.
struct GraphKey {
  void* ws;
  double* field_out;
  const double* fu0;   // caller-given fields (npb_solve_fields), else null
  const double* frho;
  npb_grid grid;
  npb_params params;
  int n_atoms;
};

struct npb_ctx {
  int device = 0;
  bool timing = false;
  bool graphs = true;
  hipStream_t capture = nullptr;  // stream the solve graph is captured on
  // further lanes of the time loops (runs of other media / levels) and
  // their fork / lag / join events
  static constexpr int kLanes = 4;
  hipStream_t side[kLanes - 1] = {};
  hipEvent_t fork = nullptr, lag[kLanes - 1] = {}, join[kLanes - 1] = {};
  // lanes used: 2 (by medium) measured fastest; 4 (by medium and level)
  // runs the short coarse-step runs beside the long ones and was slower
  int lanes = 2;
  hipGraphExec_t exec = nullptr;
  std::vector<unsigned char> key;  // GraphKey per problem + the launch-table buffer
  // line-solver shapes chosen by npb_autotune, per (nx, ny, nz, precision,
  // aos): for x (target chunk, lines per block), y and z (target chunk,
  // tile width); tune_gen changes whenever the table does
  std::map<std::array<int, 5>, std::array<int, 6>> tune;
  int tune_gen = 0;
  // device buffer of the launch tables (per-field sweep arguments, work
  // lists), owned by the context and grown on demand
  void* meta = nullptr;
  size_t meta_bytes = 0;
  npb_kernel_times times{};
  struct Pending {
    int cls;
    int sk;  // npb_sweep_kernel of a sweep launch, else -1
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  // Host staging: two page-locked buffers used in turn.  Each carries the
  // event recorded after the last enqueue whose copies read it, so a call
  // never rewrites bytes that an earlier call's copies (on any stream)
  // still read, and back-to-back asynchronous calls do not wait for each
  // other's solves.
  void* pin[2] = {nullptr, nullptr};
  size_t pin_bytes[2] = {0, 0};
  hipEvent_t pin_ev[2] = {nullptr, nullptr};
  bool pin_used[2] = {false, false};
  int pin_next = 0;
  // event after the last enqueue that read the launch tables (ctx->meta)
  hipEvent_t meta_ev = nullptr;
  bool meta_used = false;
  // this device's static scratch (npb_solve_noalloc)
  unsigned char* scratch = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
};

int npb::ctx_device(const npb_ctx* ctx) { return ctx->device; }
namespace npb {
npb_status rolling_create(const npb_ctx* tuned, int precision, void* stream, int max_items,
                          RollingEngine** out);
}
void npb::copy_tuning(const npb_ctx* from, npb_ctx* to) {
  to->tune = from->tune;
  to->tune_gen += 1;
}

namespace {

hipEvent_t ev_get(npb_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// collect timed launches after the stream has finished
void harvest(npb_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->times.count[p.cls] += 1;
      c->times.ms[p.cls] += ms;
      c->times.bytes[p.cls] += p.bytes;
      if (p.sk >= 0) {
        c->times.kcount[p.sk] += 1;
        c->times.kms[p.sk] += ms;
        c->times.kbytes[p.sk] += p.bytes;
      }
    }
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
}

// Runs of one solve: (medium, level) pairs, the longer (dt/2) level first so
// that the runs still stepping at any step form a prefix of the list.
struct Run {
  int medium;  // 0 solvated, 1 vacuum
  int level;   // 0: dt, n steps; 1: dt/2, 2n steps
};

int make_runs(const npb_params* p, Run* runs) {
  int nr = 0;
  const int media = p->vacuum ? 2 : 1;
  if (p->richardson)
    for (int m = 0; m < media; ++m) runs[nr++] = Run{m, 1};
  for (int m = 0; m < media; ++m) runs[nr++] = Run{m, 0};
  return nr;
}

struct Layout {
  size_t field[kMaxFields], acc[kMaxFields];
  size_t mask, bc_s, bc_v, atoms, tabs, key_a, id_a, key_b, id_b, sval, hist, heads;
  size_t q_idx, q_val, q_rho, xptr, yptr, ylin, yrho, zptr, zlin, zrho, ccls[3], slots, ints, total;
  size_t direct;  // work of the direct vacuum Poisson solve (vacuum_direct)
  size_t flags;   // explicit Euler node flags (solute bits, source bit)
  size_t epart;   // per-block partial energy sums
  size_t fmask[3];  // face rule by location: mask | half-point bit per direction
  LaunchShape shape[3];
  Run runs[kMaxFields];
  int n_runs, cap, nblocks;
};

// host staging (pinned): chunk tables first, then the atom planes
constexpr size_t kTabBytes = sizeof(ChunkTab<double>);

// Per-problem scalars in the workspace.  ints: [0] charge nodes, [1]
// stencil error, [kNonfiniteInts + r] run r stored a non-finite value.
// slots (doubles): [2 medium + level] sum q u of a run, [4] the direct
// vacuum solve's, [kResSlots ..] the combined results (kResCount of them),
// [kAbsSlots + 2 medium + level] sum |q u| of a run.
constexpr int kNonfiniteInts = 4;
constexpr int kResSlots = 8, kResCount = 9, kAbsSlots = 24;

// Relative error of one run's energy sum, in units of its scale sum |q u|,
// for the precision the fields are stored in (the dominant rounding): the
// dG error estimate of npb_result.  Set from the errors against the FP64
// oracle of the full-size workloads (321^3 complex, 64-grid batch members,
// serving requests up to 257^3), which stay below 0.4 of the estimate in
// FP32 storage and below 0.03 of it in FP64.
double energy_rel_error(int precision) {
  return precision == NPB_FP64 ? 1e-13 : 4e-7;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Per-line source lists each scheme's y and z sweeps use: AOSIE2 adds
// sources in both, LODIE1 after the z solve (LODIE2 and AOSIE1 add theirs
// in the x sweep).
bool is_maos(int scheme) { return scheme == NPB_MAOSIE || scheme == NPB_MAOSCN; }
// schemes with an accumulator: AOS (W and three directions) and MAOS (three)
bool is_aos(int scheme) {
  return scheme == NPB_AOSIE1 || scheme == NPB_AOSIE2 || scheme == NPB_AOSCN1 ||
         scheme == NPB_AOSCN2 || is_maos(scheme);
}
bool needs_y_sources(int scheme) {
  return scheme == NPB_AOSIE2 || scheme == NPB_AOSCN2 || is_maos(scheme);
}
bool needs_z_sources(int scheme) {
  return needs_y_sources(scheme) || scheme == NPB_LODIE1 || scheme == NPB_LODCN1;
}
// Crank-Nicolson forms: 1 = LOD (explicit half of the input with its
// source), 2 = additive (explicit half of u^n or W, source added after)
int cn_kind(int scheme) {
  if (scheme == NPB_LODCN1 || scheme == NPB_LODCN2) return 1;
  if (scheme == NPB_AOSCN1 || scheme == NPB_AOSCN2 || scheme == NPB_MAOSCN) return 2;
  return 0;
}
// implicit coefficient of the directional solves in units of tau:
// 1 (LODIE), 1/2 (LODCN), 4 (AOSIE), 2 (AOSCN), 3 (MAOSIE), 3/2 (MAOSCN)
double sweep_tau_factor(int scheme) {
  switch (scheme) {
    case NPB_LODCN1: case NPB_LODCN2: return 0.5;
    case NPB_AOSIE1: case NPB_AOSIE2: return 4.0;
    case NPB_AOSCN1: case NPB_AOSCN2: return 2.0;
    case NPB_MAOSIE: return 3.0;
    case NPB_MAOSCN: return 1.5;
    default: return 1.0;
  }
}

// fields: the source list holds every interior node (npb_solve_fields)
Layout make_layout(const npb_molecule* mol, const npb_grid* g, const npb_params* p,
                   bool fields = false) {
  Layout L{};
  const size_t es = p->precision == NPB_FP64 ? 8 : 4;
  const size_t n = (size_t)pitch_of(g->nx, (int)es) * g->ny * g->nz;  // pitched node count
  const int na = mol->n_atoms;
  const int cap = fields ? (g->nx - 2) * (g->ny - 2) * (g->nz - 2) : 8 * na;
  const int nb = (cap + 255) / 256;
  const size_t ns = (size_t)shell_count(g->nx, g->ny, g->nz);
  const bool aos = is_aos(p->scheme);
  const bool euler = p->scheme == NPB_EULER;
  const bool ys = needs_y_sources(p->scheme), zs = needs_z_sources(p->scheme);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  L.n_runs = make_runs(p, L.runs);
  for (int r = 0; r < kMaxFields; ++r) {
    L.field[r] = take(r < L.n_runs ? n * es : 0);
    // AOS accumulator, or the second buffer of the explicit Euler steps
    L.acc[r] = take(r < L.n_runs && (aos || euler) ? n * es : 0);
  }
  L.mask = take(n);
  L.bc_s = take(ns * 8);
  L.bc_v = take(p->vacuum || p->vacuum_direct ? ns * 8 : 0);
  L.atoms = take((size_t)5 * na * 8);
  L.tabs = take(kTabBytes * 3 * kMaxFields);
  L.key_a = take((size_t)cap * 4);
  L.id_a = take((size_t)cap * 4);
  L.key_b = take((size_t)cap * 4);
  L.id_b = take((size_t)cap * 4);
  L.sval = take((size_t)cap * 8);
  // radix histograms and, after them, the multi-block scan's tile totals
  L.hist = take(((size_t)256 * (nb > 0 ? nb : 1) + (size_t)scan_aux_ints(256 * (nb > 0 ? nb : 1))) * 4);
  L.heads = take((size_t)cap * 4);
  L.q_idx = take((size_t)cap * 4);
  L.q_val = take((size_t)cap * 8);
  L.q_rho = take((size_t)cap * 8);
  L.xptr = take(((size_t)g->ny * g->nz + 1) * 4);
  L.yptr = take(ys ? ((size_t)g->nz * g->nx + 1) * 4 : 0);
  L.ylin = take(ys ? (size_t)cap * 4 : 0);
  L.yrho = take(ys ? (size_t)cap * 8 : 0);
  L.zptr = take(zs ? ((size_t)g->ny * g->nx + 1) * 4 : 0);
  L.zlin = take(zs ? (size_t)cap * 4 : 0);
  L.zrho = take(zs ? (size_t)cap * 8 : 0);
  {
    const bool f64a = p->precision != NPB_FP32;
    L.shape[0] = plan_x(g->nx, g->ny, g->nz, f64a, aos, false);
    L.shape[1] = plan_yz(g->nx, g->ny, g->nz, f64a);
    L.shape[2] = plan_yz(g->nx, g->nz, g->ny, f64a);
    const int na_d[3] = {g->nx, g->ny, g->nz};
    for (int d = 0; d < 3; ++d) {
      const long long nl = class_lines(g->nx, g->ny, g->nz, d);
      L.ccls[d] = take((size_t)nl * (size_t)max_chunks(na_d[d], d == 0));
    }
  }
  L.slots = take(32 * 8);
  L.epart = take((size_t)2 * kMaxFields * 64 * 8);  // energy partial sums
  L.ints = take(16 * 4);
  L.direct = take(p->vacuum_direct ? direct_poisson_bytes(g->nx, g->ny, g->nz) : 0);
  L.flags = take(euler ? n : 0);
  for (int d = 0; d < 3; ++d) L.fmask[d] = take(p->face_rule == NPB_FACE_LOCATION ? n : 0);
  L.total = off;
  L.cap = cap;
  L.nblocks = nb;
  return L;
}

std::array<int, 5> tune_key(const npb_grid* g, const npb_params* p) {
  const int aos = is_aos(p->scheme) ? 1 : 0;
  return {g->nx, g->ny, g->nz, p->precision, aos};
}

// shapes of a tuned choice c = {x: mt, lw; y: mt, tw; z: mt, tw}
void tuned_shapes(const npb_grid* g, const npb_params* p, const std::array<int, 6>& c,
                  LaunchShape out[3]) {
  const bool f64a = p->precision != NPB_FP32;
  const bool aos = is_aos(p->scheme);
  out[0] = plan_x(g->nx, g->ny, g->nz, f64a, aos, false, c[0], c[1]);
  out[1] = plan_yz(g->nx, g->ny, g->nz, f64a, c[2], c[3]);
  out[2] = plan_yz(g->nx, g->nz, g->ny, f64a, c[4], c[5]);
}

// the context's tuned shapes, where it has them, replace the defaults
void apply_tuning(const npb_ctx* ctx, const npb_grid* g, const npb_params* p, Layout& L) {
  auto it = ctx->tune.find(tune_key(g, p));
  if (it == ctx->tune.end()) return;
  LaunchShape sh[3];
  tuned_shapes(g, p, it->second, sh);
  for (int d = 0; d < 3; ++d)
    if (sh[d].M != 0) L.shape[d] = sh[d];
}

constexpr int kMaxN = 514;

npb_status validate(const npb_molecule* mol, const npb_grid* g, const npb_params* p) {
  if (!mol || !g || !p) return fail(NPB_EINVAL, "null argument");
  if (g->nx < 5 || g->ny < 5 || g->nz < 5)
    return fail(NPB_EINVAL, "grid needs at least 5 nodes per axis");
  if (g->nx > kMaxN || g->ny > kMaxN || g->nz > kMaxN)
    return fail(NPB_EINVAL, "grid axis longer than 514 nodes is not supported");
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(NPB_EINVAL, "h must be positive");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(g->origin[d])) return fail(NPB_EINVAL, "origin must be finite");
  if (!(p->eps_in > 0.0) || !(p->eps_out > 0.0) || !std::isfinite(p->eps_in) ||
      !std::isfinite(p->eps_out))
    return fail(NPB_EINVAL, "dielectric constants must be positive");
  if (!(p->kappa_bar_sq >= 0.0) || !std::isfinite(p->kappa_bar_sq))
    return fail(NPB_EINVAL, "kappa_bar_sq must be >= 0");
  if (!(p->temperature_K > 0.0)) return fail(NPB_EINVAL, "temperature must be positive");
  if (!(p->alpha > 0.0) || !(p->dt > 0.0) || !std::isfinite(p->alpha) || !std::isfinite(p->dt))
    return fail(NPB_EINVAL, "alpha and dt must be positive");
  if (p->n_steps < 1) return fail(NPB_EINVAL, "n_steps must be >= 1");
  if (p->scheme < 0 || p->scheme > 10) return fail(NPB_EINVAL, "unknown scheme");
  if (p->precision < 0 || p->precision > 2) return fail(NPB_EINVAL, "unknown precision");
  if (p->scheme == NPB_EULER && p->precision != NPB_FP64)
    return fail(NPB_EINVAL, "explicit Euler runs in FP64 only (precision 0)");
  if (p->vacuum_direct != 0 && p->vacuum_direct != 1)
    return fail(NPB_EINVAL, "vacuum_direct must be 0 or 1");
  if (p->face_rule != NPB_FACE_HARMONIC && p->face_rule != NPB_FACE_LOCATION)
    return fail(NPB_EINVAL, "unknown face_rule");
  if (p->field_units != NPB_UNITS_KCAL && p->field_units != NPB_UNITS_DIMENSIONLESS)
    return fail(NPB_EINVAL, "unknown field_units");
  if (p->field_select < 0 || p->field_select > 3)
    return fail(NPB_EINVAL, "field_select must be 0, 1, 2 or 3");
  if (p->field_select == 1 && !p->vacuum) return fail(NPB_EINVAL, "field_select 1 needs vacuum = 1");
  if (p->field_select >= 2 && !p->vacuum_direct)
    return fail(NPB_EINVAL, "field_select 2 and 3 need vacuum_direct = 1");
  if (p->field_select == 3 && !p->vacuum) return fail(NPB_EINVAL, "field_select 3 needs vacuum = 1");
  if (mol->n_atoms < 0) return fail(NPB_EINVAL, "negative atom count");
  if (mol->n_atoms > 0 && (!mol->xyz || !mol->q || !mol->radius))
    return fail(NPB_EINVAL, "null atom arrays");
  if ((long long)mol->n_atoms * 8 > (1LL << 30)) return fail(NPB_EINVAL, "too many atoms");
  const int n[3] = {g->nx, g->ny, g->nz};
  for (int a = 0; a < mol->n_atoms; ++a) {
    if (!std::isfinite(mol->q[a]) || !std::isfinite(mol->radius[a]) || mol->radius[a] < 0.0)
      return fail(NPB_EINVAL, "atom " + std::to_string(a) + ": bad charge or radius");
    for (int d = 0; d < 3; ++d) {
      double c = mol->xyz[3 * a + d];
      if (!std::isfinite(c)) return fail(NPB_EINVAL, "atom " + std::to_string(a) + ": bad position");
      double gg = (c - g->origin[d]) / g->h;
      double fl = std::floor(gg);
      if (fl < 1.0 || fl + 1.0 > (double)(n[d] - 2))
        return fail(NPB_ERANGE, "atom " + std::to_string(a) +
                                    ": trilinear stencil touches the Dirichlet boundary");
    }
  }
  return NPB_OK;
}

// flow parameters of theta: ka = 1 + exp(-2 theta), kb = 1 - exp(-2 theta)
void flow_params(double theta, double& ka, double& kb) {
  ka = 1.0 + std::exp(-2.0 * theta);
  kb = -std::expm1(-2.0 * theta);
}

// One problem of a batch: its arguments, workspace and layout.
struct Problem {
  const npb_molecule* mol;
  const npb_grid* g;
  const npb_params* p;
  unsigned char* ws;
  double* fout;
  // caller-given fields (npb_solve_fields): initial field with its shell as
  // Dirichlet data, and a dense source; null for a molecule's problem
  const double* fu0 = nullptr;
  const double* frho = nullptr;
  Layout L;
  SetupArgs sa;
  double kT, lB;
  // steps a launch sequence takes each run through: -1 = all of the run's
  // steps (a solve); the request loop's engine sets the steps of one tick
  int steps_now[kMaxFields] = {-1, -1, -1, -1};
  size_t tabs_pinned, atoms_pinned;  // offsets of its staged bytes in the pinned buffer

  template <typename Ptr>
  Ptr* at(size_t off) const {
    return reinterpret_cast<Ptr*>(ws + off);
  }
  bool aos() const { return is_aos(p->scheme); }
  bool location() const { return p->face_rule == NPB_FACE_LOCATION; }
  // the solvated sweeps' flags in direction d: the mask, or under the face
  // rule by location the mask with that direction's half-point bits
  uint8_t* sweep_mask(int d) const {
    return location() ? ws + L.fmask[d] : ws + L.mask;
  }
  bool fields() const { return fu0 != nullptr; }
  double field_scale() const {
    return (fields() || p->field_units == NPB_UNITS_DIMENSIONLESS) ? 1.0 : kT;
  }
};

// coefficients of one run (Sec. 3: tau = dt / alpha; AOS sub-steps take
// 4 tau; faces carry harmonic means of the nodal permittivities)
struct Coefs {
  double tau, re[3], re_uniform, t, omt, t4, omt4;
  bool nl, vacuum;
};

Coefs run_coefs(const Problem& P, const Run& r) {
  const npb_params* p = P.p;
  Coefs c{};
  const double dt = p->dt / double(1 << r.level);
  c.vacuum = r.medium == 1;
  c.tau = dt / p->alpha;
  const double rc = sweep_tau_factor(p->scheme) * c.tau / (P.g->h * P.g->h);
  const double ein = p->eps_in, eout = p->eps_out;
  const double emix = 2.0 * ein * eout / (ein + eout);
  const double eout_f = 2.0 * eout * eout / (eout + eout);
  const double ein_f = 2.0 * ein * ein / (ein + ein);
  c.re[0] = rc * eout_f;
  c.re[1] = rc * emix;
  c.re[2] = rc * ein_f;
  c.re_uniform = rc * ein_f;
  const double kb2 = c.vacuum ? 0.0 : p->kappa_bar_sq;
  flow_params(kb2 * dt / (2.0 * p->alpha), c.t, c.omt);
  flow_params(4.0 * kb2 * dt / (2.0 * p->alpha), c.t4, c.omt4);
  c.nl = kb2 > 0.0 && !c.vacuum;
  return c;
}

// All problems of a batch advance together.  Every run (field) of every
// problem is swept by one launch per direction and launch shape per step;
// fields are ordered by step count (longest first) so that the fields
// still stepping at any step form a prefix of every launch group.
template <typename T, typename A>
struct Engine {
  npb_ctx* ctx;
  hipStream_t st;
  std::vector<Problem>& pr;

  struct Field {
    int prob, run, steps;
    int lane;         // stream of the run: by medium and level, see plan()
    double bytes[3];  // algorithmic bytes of one sweep per direction
  };
  std::vector<Field> fields;
  struct Group {
    LaunchShape s;                 // shared shape, lds = max over members
    int var = kYzPlain;
    std::vector<int> members;      // field indices, in field order
    size_t args_off = 0;           // SweepArgs<T>[members] in the launch-table buffer
    std::vector<int> nblk;         // blocks of the first k members, k = 1..size
    std::vector<size_t> work_off;  // int2[nblk[k-1]] per k
    int nbu = 0;                   // blocks per member when all members have the same count
    int lane = 0;
  };
  std::vector<Group> groups[3];
  std::vector<unsigned char> meta;  // host image of the launch tables
  // npb_solve_noalloc: the problem's workspace is the device's static
  // scratch, the launch tables follow it there, the host staging is
  // pageable memory of this call, and nothing is captured into a graph
  bool noalloc = false;
  unsigned char* hb = nullptr;     // host staging of this call
  unsigned char* dmeta = nullptr;  // device launch tables of this call
  int pin_slot = -1;               // ctx->pin buffer staged into (-1: none)
  std::vector<unsigned char> hvec;

  template <typename F>
  npb_status timed(int cls, double bytes, F&& f) {
    return timed_on(st, cls, -1, bytes, f);
  }
  // Timing: a sweep launch (sk >= 0) records its kernel's own start and
  // stop in the events (the launcher's hipExtLaunchKernelGGL path); other
  // launches are bracketed by events recorded on the stream.
  template <typename F>
  npb_status timed_on(hipStream_t s, int cls, int sk, double bytes, F&& f) {
    hipEvent_t a = nullptr, b = nullptr;
    if (ctx->timing) {
      a = ev_get(ctx);
      b = ev_get(ctx);
      if (!a || !b) return fail(NPB_EDEVICE, "event creation failed");
      if (sk >= 0)
        set_sweep_launch_events(a, b);
      else
        NPB_HIP(hipEventRecord(a, s));
    }
    hipError_t e = f();
    if (ctx->timing && sk >= 0) set_sweep_launch_events(nullptr, nullptr);
    if (e != hipSuccess) return fail(NPB_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
    if (ctx->timing) {
      if (sk < 0) NPB_HIP(hipEventRecord(b, s));
      ctx->pending.push_back({cls, sk, a, b, bytes});
    }
    return NPB_OK;
  }

  // sweep arguments of run r of problem P in direction d (scheme-specific
  // fused work: Sec. 3.1 LODIE2 / LODIE1 orders, Sec. 3.2 AOS accumulation)
  SweepArgs<T> sweep_args(const Problem& P, int r, int d) const {
    const Coefs c = run_coefs(P, P.L.runs[r]);
    const npb_params* p = P.p;
    const Layout& L = P.L;
    SweepArgs<T> a{};
    a.u = P.at<T>(L.field[r]);
    a.acc = P.aos() ? P.at<T>(L.acc[r]) : nullptr;
    a.mask = c.vacuum ? nullptr : P.sweep_mask(d);
    a.face_loc = (!c.vacuum && P.location()) ? 1 : 0;
    a.nx = P.g->nx;
    a.ny = P.g->ny;
    a.nz = P.g->nz;
    a.nxp = pitch_of(P.g->nx, (int)sizeof(T));
    for (int k = 0; k < 3; ++k) a.re[k] = c.re[k];
    a.re_uniform = c.re_uniform;
    a.ccls = c.vacuum ? nullptr : P.at<uint8_t>(L.ccls[d]);
    a.tab = P.ws + L.tabs + kTabBytes * (3 * r + d);
    // the z sweep stores each step's result: it notes non-finite values
    a.nonfinite = d == 2 ? P.at<int>(L.ints) + kNonfiniteInts + r : nullptr;
    a.bcx = d == 0 ? P.at<double>(c.vacuum ? L.bc_v : L.bc_s) : nullptr;
    if (d == 0) {
      a.src_ptr = P.at<int>(L.xptr);
      a.src_lin = P.at<int>(L.q_idx);
      a.src_rho = P.at<double>(L.q_rho);
    } else {
      a.src_ptr = P.at<int>(d == 1 ? L.yptr : L.zptr);
      a.src_lin = P.at<int>(d == 1 ? L.ylin : L.zlin);
      a.src_rho = P.at<double>(d == 1 ? L.yrho : L.zrho);
    }
    a.cn = cn_kind(p->scheme);
    if (p->scheme == NPB_LODIE2 || p->scheme == NPB_LODCN2) {
      if (d == 0) {
        a.src_stage = 1;
        a.src_coef = c.tau;
      }
      if (d == 2 && c.nl) {
        a.post_nl = 1;
        a.post_ka = c.t;
        a.post_kb = c.omt;
      }
    } else if (p->scheme == NPB_LODIE1 || p->scheme == NPB_LODCN1) {
      if (d == 0 && c.nl) {
        a.pre_nl = 1;
        a.pre_ka = c.t;
        a.pre_kb = c.omt;
      }
      if (d == 2) {
        a.src_stage = 2;
        a.src_coef = c.tau;
      }
    } else if (is_maos(p->scheme)) {
      // Sec. 3.3: every direction starts from W = flow(u^n) with the source
      // tau rho; U = (V + P + Q) / 3
      a.mode = d == 0 ? MODE_AOS_FIRST : (d == 1 ? MODE_AOS_ADD : MODE_AOS_FINISH);
      a.aos_ww = 0.0;
      a.aos_wv = 1.0 / 3.0;
      if (c.nl) {
        a.pre_nl = 1;
        a.pre_ka = c.t;
        a.pre_kb = c.omt;
      }
      a.src_stage = 1;
      a.src_coef = c.tau;
    } else {
      const bool split = p->scheme == NPB_AOSIE2 || p->scheme == NPB_AOSCN2;
      const double cx = split ? 4.0 / 3.0 : 4.0;
      const double cyz = split ? 4.0 / 3.0 : 0.0;
      a.aos_ww = 0.25;
      a.aos_wv = 0.25;
      if (d == 0) {
        a.mode = MODE_AOS_FIRST;
        a.aos_w = c.nl ? 1 : 0;
        a.aos_ka = c.t4;
        a.aos_kb = c.omt4;
        a.src_stage = 1;
        a.src_coef = cx * c.tau;
      } else {
        a.mode = d == 1 ? MODE_AOS_ADD : MODE_AOS_FINISH;
        if (cyz != 0.0) {
          a.src_stage = 1;
          a.src_coef = cyz * c.tau;
        }
      }
    }
    shape_args(a, d, L.shape[d]);
    return a;
  }

  // fields, launch groups and the host image of the launch tables
  npb_status plan() {
    for (int i = 0; i < (int)pr.size(); ++i) {
      const Problem& P = pr[i];
      if (P.p->scheme == NPB_EULER) continue;  // stepped by euler_loop
      const double pts = (double)(P.g->nx - 2) * (P.g->ny - 2) * (P.g->nz - 2);
      for (int r = 0; r < P.L.n_runs; ++r) {
        Field f{};
        f.prob = i;
        f.run = r;
        f.steps = P.steps_now[r] >= 0 ? P.steps_now[r] : P.p->n_steps << P.L.runs[r].level;
        if (f.steps == 0) continue;  // a run of the request loop that is already done
        // field read + write (+ mask) (+ accumulator)
        const double mb = P.L.runs[r].medium == 1 ? 0.0 : 1.0;
        const double ab = P.aos() ? sizeof(T) : 0.0;
        f.bytes[0] = pts * (2.0 * sizeof(T) + mb + ab);
        f.bytes[1] = pts * (2.0 * sizeof(T) + mb + 2.0 * ab);
        f.bytes[2] = pts * (2.0 * sizeof(T) + mb + ab);
        // lanes: 2 -> by medium; 4 -> by medium and level
        f.lane = ctx->lanes >= 4 ? 2 * P.L.runs[r].medium + P.L.runs[r].level
                 : ctx->lanes >= 2 ? P.L.runs[r].medium
                                   : 0;
        fields.push_back(f);
      }
      for (int d = 0; d < 3; ++d)
        if (P.L.shape[d].M == 0) return fail(NPB_EINVAL, "unsupported grid shape");
    }
    std::stable_sort(fields.begin(), fields.end(),
                     [](const Field& a, const Field& b) { return a.steps > b.steps; });
    auto align = [](size_t v) { return (v + 255) & ~size_t(255); };
    size_t off = 0;
    std::vector<std::vector<SweepArgs<T>>> gargs[3];
    for (int d = 0; d < 3; ++d) {
      for (int fi = 0; fi < (int)fields.size(); ++fi) {
        const LaunchShape& sh = pr[fields[fi].prob].L.shape[d];
        int g = 0;
        const int lane = fields[fi].lane;
        while (g < (int)groups[d].size() &&
               !(groups[d][g].s.M == sh.M && groups[d][g].s.P == sh.P &&
                 groups[d][g].s.LW == sh.LW && groups[d][g].s.threads == sh.threads &&
                 groups[d][g].lane == lane))
          ++g;
        if (g == (int)groups[d].size()) {
          groups[d].push_back(Group{});
          groups[d].back().s = sh;
          groups[d].back().lane = lane;
          gargs[d].emplace_back();
        }
        Group& G = groups[d][g];
        G.s.lds = std::max(G.s.lds, sh.lds);
        G.members.push_back(fi);
        gargs[d][g].push_back(sweep_args(pr[fields[fi].prob], fields[fi].run, d));
      }
      for (int g = 0; g < (int)groups[d].size(); ++g) {
        Group& G = groups[d][g];
        // y / z: the kernel variant; x: whether the Crank-Nicolson code is needed
        G.var = d == 0 ? sweep_cn(gargs[d][g].data(), (int)gargs[d][g].size())
                       : sweep_variant(gargs[d][g].data(), (int)gargs[d][g].size());
        G.nbu = pr[fields[G.members[0]].prob].L.shape[d].blocks;
        for (int m : G.members)
          if (pr[fields[m].prob].L.shape[d].blocks != G.nbu) G.nbu = 0;
        G.args_off = off;
        off = align(off + sizeof(SweepArgs<T>) * G.members.size());
        int nb = 0;
        for (int k = 0; k < (int)G.members.size(); ++k) {
          nb += pr[fields[G.members[k]].prob].L.shape[d].blocks;
          G.nblk.push_back(nb);
          G.work_off.push_back(off);
          off = align(off + sizeof(int2) * (size_t)nb);
        }
      }
    }
    meta.assign(off, 0);
    for (int d = 0; d < 3; ++d)
      for (int g = 0; g < (int)groups[d].size(); ++g) {
        const Group& G = groups[d][g];
        std::memcpy(meta.data() + G.args_off, gargs[d][g].data(),
                    sizeof(SweepArgs<T>) * G.members.size());
        for (int k = 0; k < (int)G.members.size(); ++k) {
          int2* w = reinterpret_cast<int2*>(meta.data() + G.work_off[k]);
          int n = 0;
          for (int m = 0; m <= k; ++m) {
            const int nbm = pr[fields[G.members[m]].prob].L.shape[d].blocks;
            for (int b = 0; b < nbm; ++b) w[n++] = make_int2(m, b);
          }
        }
      }
    return NPB_OK;
  }

  // Host staging: [results: 128 B per problem][launch tables][per problem:
  // chunk tables, atom planes].  The host fills it, then one copy per
  // region moves it to the device.  with_meta = false keeps the launch
  // tables already in the context's device buffer (a graph replay of the
  // same batch).  The staging buffer is one of the context's two
  // page-locked buffers, taken once the last enqueue that read it is done;
  // the no-allocation path stages in pageable memory of its own and puts
  // the launch tables into the static scratch after the workspace.
  bool stage_problems = true;  // false: launch tables only (the request loop's ticks)
  npb_status stage(bool with_meta) {
    const size_t res_bytes = 128 * pr.size();
    size_t need = res_bytes + (with_meta ? meta.size() : 0);
    for (Problem& P : pr) {
      P.tabs_pinned = need;
      need += kTabBytes * 3 * kMaxFields;
      P.atoms_pinned = need;
      need += (size_t)5 * P.mol->n_atoms * 8;
    }
    if (noalloc) {
      hvec.assign(need, 0);
      hb = hvec.data();
      const size_t moff = align256(pr[0].L.total);
      if (moff + meta.size() > (size_t)NPB_NOALLOC_BYTES)
        return fail(NPB_EINVAL, "workspace (" + std::to_string(pr[0].L.total) +
                                    " bytes) and launch tables (" + std::to_string(meta.size()) +
                                    " bytes) exceed the static scratch of " +
                                    std::to_string((size_t)NPB_NOALLOC_BYTES) + " bytes");
      dmeta = ctx->scratch + moff;
    } else {
      const int b = ctx->pin_next;
      ctx->pin_next ^= 1;
      if (ctx->pin_used[b]) NPB_HIP(hipEventSynchronize(ctx->pin_ev[b]));
      ctx->pin_used[b] = false;
      if (ctx->pin_bytes[b] < need) {
        if (ctx->pin[b]) (void)hipHostFree(ctx->pin[b]);
        ctx->pin[b] = nullptr;
        ctx->pin_bytes[b] = 0;
        NPB_HIP(hipHostMalloc(&ctx->pin[b], need, hipHostMallocDefault));
        ctx->pin_bytes[b] = need;
      }
      hb = reinterpret_cast<unsigned char*>(ctx->pin[b]);
      pin_slot = b;
      if (with_meta) {
        // the captured graph and earlier enqueues read the launch tables
        // being replaced: wait for them, then drop the graph
        if (ctx->meta_used) NPB_HIP(hipEventSynchronize(ctx->meta_ev));
        ctx->meta_used = false;
        if (ctx->exec) (void)hipGraphExecDestroy(ctx->exec);
        ctx->exec = nullptr;
        ctx->key.clear();
        if (ctx->meta_bytes < meta.size()) {
          if (ctx->meta) (void)hipFree(ctx->meta);
          ctx->meta = nullptr;
          ctx->meta_bytes = 0;
          NPB_HIP(hipMalloc(&ctx->meta, meta.size()));
          ctx->meta_bytes = meta.size();
        }
      }
      dmeta = reinterpret_cast<unsigned char*>(ctx->meta);
    }
    if (with_meta) {
      std::memcpy(hb + res_bytes, meta.data(), meta.size());
      NPB_HIP(hipMemcpyAsync(dmeta, hb + res_bytes, meta.size(), hipMemcpyHostToDevice, st));
    }
    for (Problem& P : pr) {
      if (!stage_problems) break;
      for (int r = 0; r < P.L.n_runs; ++r) {
        const Coefs c = run_coefs(P, P.L.runs[r]);
        for (int d = 0; d < 3; ++d) {
          ChunkTab<A>& tb =
              *reinterpret_cast<ChunkTab<A>*>(hb + P.tabs_pinned + kTabBytes * (3 * r + d));
          const int nint = (d == 0 ? P.g->nx : d == 1 ? P.g->ny : P.g->nz) - 2;
          if (c.vacuum)
            fill_chunk_tab(tb, c.re_uniform, c.re_uniform, P.L.shape[d].M, nint);
          else
            fill_chunk_tab(tb, c.re[0], c.re[2], P.L.shape[d].M, nint);
        }
      }
      NPB_HIP(hipMemcpyAsync(P.ws + P.L.tabs, hb + P.tabs_pinned, kTabBytes * 3 * P.L.n_runs,
                             hipMemcpyHostToDevice, st));
      const int na = P.mol->n_atoms;
      if (na > 0) {
        double* h = reinterpret_cast<double*>(hb + P.atoms_pinned);
        for (int a = 0; a < na; ++a) {
          h[a] = P.mol->xyz[3 * a];
          h[na + a] = P.mol->xyz[3 * a + 1];
          h[2 * na + a] = P.mol->xyz[3 * a + 2];
          h[3 * na + a] = P.mol->q[a];
          h[4 * na + a] = P.mol->radius[a];
        }
        NPB_HIP(hipMemcpyAsync(P.ws + P.L.atoms, h, (size_t)5 * na * 8, hipMemcpyHostToDevice,
                               st));
      }
    }
    return NPB_OK;
  }

  npb_status setup(Problem& P) {
    const Layout& L = P.L;
    const npb_params* p = P.p;
    const int na = P.mol->n_atoms;
    const int nx = P.g->nx, ny = P.g->ny, nz = P.g->nz;
    const int nxp = pitch_of(nx, (int)sizeof(T));
    const size_t n = (size_t)nxp * ny * nz;
    P.sa = SetupArgs{nx, ny, nz, nxp, P.g->h, P.g->origin[0], P.g->origin[1], P.g->origin[2], na,
                     P.at<double>(L.atoms)};
    const SetupArgs& sa = P.sa;
    unsigned char* ws = P.ws;
    int* ints = P.at<int>(L.ints);  // [0] nq, [1] stencil error, run flags
    return timed(NPB_K_SETUP, 0, [&] {
      hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ints), 16, 0u, st);
      if (e != hipSuccess) return e;
      e = launch_fill_u32(reinterpret_cast<uint32_t*>(ws + L.mask), (n + 3) / 4, 0u, st);
      if (e != hipSuccess) return e;
      e = launch_mask_raster(sa, P.at<uint8_t>(L.mask), st);
      if (e != hipSuccess) return e;
      if (P.location()) {
        // per direction: the mask with bit 1 on nodes whose half point to
        // the next node is solute
        for (int d = 0; d < 3 && e == hipSuccess; ++d) {
          e = launch_copy_u32(reinterpret_cast<const uint32_t*>(ws + L.mask),
                              reinterpret_cast<uint32_t*>(ws + L.fmask[d]), (n + 3) / 4, st);
          if (e == hipSuccess)
            e = launch_face_raster(sa, d, P.at<uint8_t>(L.mask), P.at<uint8_t>(L.fmask[d]), st);
        }
        if (e != hipSuccess) return e;
      }
      if (P.fields())
        e = launch_dense_source(P.frho, nx, nxp, ny, nz, P.at<int>(L.key_a), P.at<int>(L.id_a),
                                P.at<double>(L.sval), st);
      else
        e = launch_stencil(sa, P.at<int>(L.key_a), P.at<int>(L.id_a), P.at<double>(L.sval),
                           ints + 1, st);
      if (e != hipSuccess) return e;
      e = radix_sort_pairs(P.at<int>(L.key_a), P.at<int>(L.id_a), P.at<int>(L.key_b),
                           P.at<int>(L.id_b), P.at<int>(L.hist), L.cap, (long long)n, st);
      if (e != hipSuccess) return e;
      // Eq. (RhoEq): rho = 4 pi l_B Q / h^3 of the trilinear charges; a
      // caller-given source is rho itself
      const double pref = P.fields() ? 1.0 : 4.0 * M_PI * P.lB / (P.g->h * P.g->h * P.g->h);
      e = launch_merge_charges(P.at<int>(L.key_a), P.at<int>(L.id_a), P.at<double>(L.sval),
                               P.at<int>(L.heads), L.cap, ints, P.at<int>(L.q_idx),
                               P.at<double>(L.q_val), P.at<double>(L.q_rho), pref,
                               P.at<int>(L.hist), st);
      if (e != hipSuccess) return e;
      e = launch_line_ptr(P.at<int>(L.q_idx), ints, L.cap, ny * nz, nxp, P.at<int>(L.xptr), st);
      if (e != hipSuccess) return e;
      if (needs_z_sources(p->scheme) && L.cap > 0) {
        for (int axis = needs_y_sources(p->scheme) ? 1 : 2; axis <= 2; ++axis) {
          e = launch_axis_keys(P.at<int>(L.q_idx), ints, L.cap, nx, nxp, ny, nz, axis,
                               P.at<int>(L.key_a), P.at<int>(L.id_a), st);
          if (e != hipSuccess) return e;
          e = radix_sort_pairs(P.at<int>(L.key_a), P.at<int>(L.id_a), P.at<int>(L.key_b),
                               P.at<int>(L.id_b), P.at<int>(L.hist), L.cap,
                               (long long)nx * ny * nz + 1, st);
          if (e != hipSuccess) return e;
          int* lin = P.at<int>(axis == 1 ? L.ylin : L.zlin);
          double* rho = P.at<double>(axis == 1 ? L.yrho : L.zrho);
          e = launch_gather_entries(P.at<int>(L.id_a), ints, L.cap, P.at<int>(L.q_idx),
                                    P.at<double>(L.q_rho), lin, rho, st);
          if (e != hipSuccess) return e;
          if (axis == 1)
            e = launch_line_ptr(P.at<int>(L.key_a), ints, L.cap, nz * nx, ny, P.at<int>(L.yptr),
                                st);
          else
            e = launch_line_ptr(P.at<int>(L.key_a), ints, L.cap, ny * nx, nz, P.at<int>(L.zptr),
                                st);
          if (e != hipSuccess) return e;
        }
      } else if (needs_z_sources(p->scheme)) {
        if (needs_y_sources(p->scheme))
          e = launch_fill_u32(reinterpret_cast<uint32_t*>(ws + L.yptr), (size_t)nz * nx + 1, 0u,
                              st);
        if (e != hipSuccess) return e;
        e = launch_fill_u32(reinterpret_cast<uint32_t*>(ws + L.zptr), (size_t)ny * nx + 1, 0u, st);
        if (e != hipSuccess) return e;
      }
      if (P.fields()) {
        e = launch_shell_from_dense(P.fu0, nx, ny, nz, P.at<double>(L.bc_s), st);
      } else {
        const double kappa = std::sqrt(p->kappa_bar_sq / p->eps_out);
        e = launch_boundary(sa, p->eps_out, kappa, p->eps_in, P.lB, P.at<double>(L.bc_s),
                            p->vacuum || p->vacuum_direct ? P.at<double>(L.bc_v) : nullptr,
                            sizeof(A) == 4, st);
      }
      if (e != hipSuccess) return e;
      for (int d = 0; d < 3 && e == hipSuccess; ++d)
        e = launch_chunk_classes(P.sweep_mask(d), nx, nxp, ny, nz, d, L.shape[d].M,
                                 L.shape[d].P, P.location() ? 1 : 0, P.at<uint8_t>(L.ccls[d]),
                                 st);
      if (e == hipSuccess && p->scheme == NPB_EULER) {
        const uint8_t* fm[3] = {P.sweep_mask(0), P.sweep_mask(1), P.sweep_mask(2)};
        e = launch_euler_flags(P.at<uint8_t>(L.mask), P.location() ? fm : nullptr,
                               P.at<int>(L.q_idx), ints, L.cap, P.at<uint8_t>(L.flags), nx, nxp,
                               ny, nz, st);
      }
      return e;
    });
  }

  npb_status time_loop(bool init = true) {
    if (init) {
      npb_status s = init_fields();
      if (s != NPB_OK) return s;
    }
    return step_loop();
  }

  // field initialisation of every run of the problems (Dirichlet shell,
  // zero interior; or the caller-given initial field)
  npb_status init_fields() {
    for (const Problem& P : pr) {
      if (P.p->scheme == NPB_EULER) continue;
      const int nx = P.g->nx, ny = P.g->ny, nz = P.g->nz;
      const int nxp = pitch_of(nx, (int)sizeof(T));
      InitSet<T> set{};
      for (int r = 0; r < P.L.n_runs; ++r) {
        set.u[r] = P.at<T>(P.L.field[r]);
        set.bc[r] = P.at<double>(P.L.runs[r].medium == 1 ? P.L.bc_v : P.L.bc_s);
      }
      npb_status s = timed(NPB_K_INIT, (double)nxp * ny * nz * sizeof(T) * P.L.n_runs, [&] {
        if (!P.fields()) return launch_field_init_multi<T>(set, P.L.n_runs, nx, nxp, ny, nz, st);
        hipError_t e = hipSuccess;
        for (int r = 0; r < P.L.n_runs && e == hipSuccess; ++r)
          e = launch_field_from_dense<T>(set.u[r], P.fu0, nx, nxp, ny, nz, st);
        return e;
      });
      if (s != NPB_OK) return s;
    }
    return NPB_OK;
  }

  npb_status step_loop() {
    // Lanes: the runs of each medium (and, with four lanes, each level) are
    // independent problems; lane 0 sweeps on `st`, lane k > 0 on a side
    // stream of the context, started one sweep after lane k-1.  Sweeps of
    // different lanes then run at the same time in different phases (one
    // launch's loads while another's blocks solve), which one launch alone
    // cannot do: its blocks move between memory and arithmetic phases in
    // step.  The side streams join `st` before and after the loops (in a
    // captured graph these are graph dependencies).
    int nl = 1;
    for (const Field& f : fields) nl = std::max(nl, f.lane + 1);
    // While timing, the lanes keep their launches but all issue on `st`, one
    // after another, so that each bracketed launch has the device alone.
    const bool serial = ctx->timing;
    hipStream_t ls[npb_ctx::kLanes];
    ls[0] = st;
    for (int l = 1; l < nl; ++l) ls[l] = serial ? st : ctx->side[l - 1];
    if (nl > 1 && !serial) {
      NPB_HIP(hipEventRecord(ctx->fork, st));
      for (int l = 1; l < nl; ++l) NPB_HIP(hipStreamWaitEvent(ls[l], ctx->fork, 0));
    }
    // the launches of every lane in order, then issued with lane l offset
    // by l * lag launches of lane 0 (so that at any time the lanes run
    // different sweeps)
    struct Launch {
      const Group* G;
      int d, k;
      double bytes;
    };
    std::vector<Launch> seq[npb_ctx::kLanes];
    const int max_steps = fields.empty() ? 0 : fields[0].steps;
    for (int step = 0; step < max_steps; ++step)
      for (int d = 0; d < 3; ++d)
        for (const Group& G : groups[d]) {
          int k = 0;
          double bytes = 0.0;
          while (k < (int)G.members.size() && fields[G.members[k]].steps > step)
            bytes += fields[G.members[k++]].bytes[d];
          if (k > 0) seq[G.lane].push_back(Launch{&G, d, k, bytes});
        }
    // stagger of one sweep measured best (0, 2 and 3 sweeps: 2-3 % slower)
    const int lag = 1;
    unsigned char* dm = dmeta;
    size_t total = 0;
    for (int l = 0; l < nl; ++l) total = std::max(total, seq[l].size() + (size_t)l * lag);
    for (size_t i = 0; i < total; ++i) {
      for (int lane = 0; lane < nl; ++lane) {
        const long long j = (long long)i - (long long)lane * lag;
        if (j < 0 || j >= (long long)seq[lane].size()) continue;
        const Launch& L = seq[lane][j];
        // a lane starts once the previous lane has done `lag` sweeps
        if (j == 0 && lane > 0 && lag > 0 && !serial)
          NPB_HIP(hipStreamWaitEvent(ls[lane], ctx->lag[lane - 1], 0));
        const hipStream_t s = ls[lane];
        const Group& G = *L.G;
        const int d = L.d;
        const auto* args = reinterpret_cast<const SweepArgs<T>*>(dm + G.args_off);
        const auto* work = reinterpret_cast<const int2*>(dm + G.work_off[L.k - 1]);
        const int nb = G.nblk[L.k - 1];
        const int sk = d == 0 ? NPB_SK_X
                       : G.var == kYzPlain ? NPB_SK_YZ_PLAIN
                       : G.var == kYzFlow ? NPB_SK_YZ_FLOW
                                          : NPB_SK_YZ_GENERAL;
        npb_status r = timed_on(s, NPB_K_SWEEP_X + d, sk, L.bytes, [&] {
          return d == 0 ? launch_sweep_x<T, A>(args, work, G.nbu, nb, G.var, G.s, s)
                        : launch_sweep_yz<T, A>(args, work, G.nbu, nb, d, G.var, G.s, s);
        });
        if (r != NPB_OK) return r;
        if (lane + 1 < nl && lag > 0 && j + 1 == lag && !serial)
          NPB_HIP(hipEventRecord(ctx->lag[lane], s));
      }
    }
    for (int l = 1; l < nl && !serial; ++l) {
      NPB_HIP(hipEventRecord(ctx->join[l - 1], ls[l]));
      NPB_HIP(hipStreamWaitEvent(st, ctx->join[l - 1], 0));
    }
    return NPB_OK;
  }

  // Explicit Euler (NPB_EULER): both buffers of every run start from the
  // initial field; a run of s steps starts in its field buffer when s is
  // even and in the second buffer when s is odd, so that it ends in the
  // field buffer.  One launch per step and run, steps outermost.
  npb_status euler_loop() {
    if constexpr (!std::is_same<T, double>::value) {
      for (const Problem& P : pr)
        if (P.p->scheme == NPB_EULER) return fail(NPB_EINVAL, "explicit Euler runs in FP64 only");
      return NPB_OK;
    } else {
      struct ERun {
        const Problem* P;
        int r, steps;
        EulerArgs a;
        double bytes;
      };
      std::vector<ERun> runs;
      int max_steps = 0;
      for (const Problem& P : pr) {
        if (P.p->scheme != NPB_EULER) continue;
        const int nx = P.g->nx, ny = P.g->ny, nz = P.g->nz;
        const int nxp = pitch_of(nx, (int)sizeof(T));
        for (int r = 0; r < P.L.n_runs; ++r) {
          const bool vac = P.L.runs[r].medium == 1;
          for (int b = 0; b < 2; ++b) {
            T* buf = P.at<T>(b == 0 ? P.L.field[r] : P.L.acc[r]);
            npb_status s = timed(NPB_K_INIT, (double)nxp * ny * nz * sizeof(T), [&] {
              return P.fields() ? launch_field_from_dense<T>(buf, P.fu0, nx, nxp, ny, nz, st)
                                : launch_field_init<T>(buf, P.at<double>(vac ? P.L.bc_v : P.L.bc_s),
                                                       nx, nxp, ny, nz, st);
            });
            if (s != NPB_OK) return s;
          }
          const Coefs c = run_coefs(P, P.L.runs[r]);
          ERun e{};
          e.P = &P;
          e.r = r;
          e.steps = P.p->n_steps << P.L.runs[r].level;
          EulerArgs& a = e.a;
          a.flags = P.at<uint8_t>(P.L.flags);
          a.src_ptr = P.at<int>(P.L.xptr);
          a.q_idx = P.at<int>(P.L.q_idx);
          a.q_rho = P.at<double>(P.L.q_rho);
          a.nx = nx;
          a.ny = ny;
          a.nz = nz;
          a.nxp = nxp;
          a.zc = euler_z_chunk(nx, ny, nz);
          a.uniform = vac ? 1 : 0;
          a.face_loc = (!vac && P.location()) ? 1 : 0;
          a.nl = c.nl ? 1 : 0;
          for (int k = 0; k < 3; ++k) a.re[k] = c.re[k];
          a.re_uniform = c.re_uniform;
          a.tau = c.tau;
          a.tk = c.nl ? c.tau * P.p->kappa_bar_sq : 0.0;
          a.nonfinite = P.at<int>(P.L.ints) + kNonfiniteInts + r;
          // field read + write and the flag byte per interior node
          e.bytes = (double)(nx - 2) * (ny - 2) * (nz - 2) * (2.0 * sizeof(T) + 1.0);
          runs.push_back(e);
          max_steps = std::max(max_steps, e.steps);
        }
      }
      for (int step = 0; step < max_steps; ++step)
        for (ERun& e : runs) {
          if (step >= e.steps) continue;
          const bool from_field = ((step % 2) == 0) == ((e.steps % 2) == 0);
          T* fld = e.P->template at<T>(e.P->L.field[e.r]);
          T* alt = e.P->template at<T>(e.P->L.acc[e.r]);
          e.a.u = from_field ? fld : alt;
          e.a.v = from_field ? alt : fld;
          hipEvent_t a0 = nullptr, a1 = nullptr;
          if (ctx->timing) {
            a0 = ev_get(ctx);
            a1 = ev_get(ctx);
            if (!a0 || !a1) return fail(NPB_EDEVICE, "event creation failed");
          }
          const hipError_t err = launch_euler_step(e.a, a0, a1, st);
          if (err != hipSuccess)
            return fail(NPB_EDEVICE, std::string("launch: ") + hipGetErrorString(err));
          if (ctx->timing) ctx->pending.push_back({NPB_K_EULER, NPB_SK_EULER, a0, a1, e.bytes});
        }
      return NPB_OK;
    }
  }

  // The device work after staging, all on `st` (captured into a graph when
  // replay is on): setup, time loops, energies, optional fields,
  // combinations.  Launches only: no allocation, copy or synchronisation.
  npb_status device_work() {
    npb_status s = setup_all();
    if (s != NPB_OK) return s;
    s = time_loop();
    if (s != NPB_OK) return s;
    s = euler_loop();
    if (s != NPB_OK) return s;
    for (Problem& P : pr) {
      s = finish(P);
      if (s != NPB_OK) return s;
    }
    return NPB_OK;
  }

  // setup of every problem and its cleared energy slots
  npb_status setup_all() {
    for (Problem& P : pr) {
      npb_status s = setup(P);
      if (s != NPB_OK) return s;
      s = timed(NPB_K_OTHER, 0, [&] {
        return launch_fill_u32(reinterpret_cast<uint32_t*>(P.ws + P.L.slots), 64, 0u, st);
      });
      if (s != NPB_OK) return s;
    }
    return NPB_OK;
  }

  // after a problem's time loops: energies, the direct vacuum solve, the
  // requested field and the FP64 combinations
  npb_status finish(Problem& P) {
    npb_status s = NPB_OK;
    {
      const Layout& L = P.L;
      EnergySet<T> set{};
      for (int r = 0; r < L.n_runs; ++r) {
        set.u[r] = P.at<T>(L.field[r]);
        set.slot[r] = P.at<double>(L.slots) + 2 * L.runs[r].medium + L.runs[r].level;
        set.aslot[r] = P.at<double>(L.slots) + kAbsSlots + 2 * L.runs[r].medium + L.runs[r].level;
      }
      s = timed(NPB_K_ENERGY, 0, [&] {
        return launch_energy_multi<T>(set, L.n_runs, P.at<int>(L.q_idx), P.at<double>(L.q_val),
                                      P.at<int>(L.ints), L.cap, P.at<double>(L.epart), st);
      });
      if (s != NPB_OK) return s;
      const npb_params* p = P.p;
      if (p->vacuum_direct) {
        // Sec. 5.1: phi_0 from the Poisson equation solved directly
        DirectPoissonArgs da{};
        da.nx = P.g->nx;
        da.ny = P.g->ny;
        da.nz = P.g->nz;
        da.nxp = pitch_of(P.g->nx, (int)sizeof(T));
        da.h = P.g->h;
        da.eps = p->eps_in;
        da.bc = P.at<double>(L.bc_v);
        da.q_idx = P.at<int>(L.q_idx);
        da.q_rho = P.at<double>(L.q_rho);
        da.q_val = P.at<double>(L.q_val);
        da.nq_dev = P.at<int>(L.ints);
        da.cap = L.cap;
        da.work = P.at<double>(L.direct);
        da.slot = P.at<double>(L.slots) + 4;
        s = timed(NPB_K_DIRECT, 0, [&] { return launch_direct_poisson(da, st); });
        if (s != NPB_OK) return s;
      }
      if (P.fout) {
        // field_select 0 / 1: kT u of that medium (plain) or
        // kT (2 u(dt/2) - u(dt)) (Richardson); 2: kT u of the direct vacuum
        // solve; 3: solvated - vacuum (as 0 and 1) + direct vacuum (Sec. 5.4)
        const int fs = p->field_select;
        bool first = true;
        for (int medium = 0; medium < 2; ++medium) {
          const double sign = (fs == 3 && medium == 1) ? -1.0 : 1.0;
          if (!(fs == medium || fs == 3)) continue;
          for (int l = 0; l < (p->richardson ? 2 : 1); ++l) {
            int r = 0;
            while (!(L.runs[r].medium == medium && L.runs[r].level == l)) ++r;
            const double beta = first ? 0.0 : 1.0;
            // dimensionless u (caller-given fields, or asked for), else kT u
            const double scale = P.field_scale();
            const double gamma = sign * (p->richardson ? (l == 0 ? -scale : 2.0 * scale) : scale);
            s = timed(NPB_K_OTHER, 0, [&] {
              return launch_field_out<T>(P.fout, P.at<T>(L.field[r]), P.g->nx,
                                         pitch_of(P.g->nx, (int)sizeof(T)), P.g->ny, P.g->nz,
                                         beta, gamma, st);
            });
            if (s != NPB_OK) return s;
            first = false;
          }
        }
        if (fs >= 2) {
          s = timed(NPB_K_OTHER, 0, [&] {
            return launch_direct_field_out(P.fout, P.at<double>(L.direct), P.at<double>(L.bc_v),
                                           P.g->nx, P.g->ny, P.g->nz, first ? 0.0 : 1.0,
                                           P.field_scale(), st);
          });
          if (s != NPB_OK) return s;
        }
      }
      s = timed(NPB_K_OTHER, 0, [&] {
        return launch_combine(P.at<double>(L.slots), P.at<double>(L.slots) + kAbsSlots,
                              P.at<int>(L.ints) + kNonfiniteInts, L.n_runs,
                              energy_rel_error(p->precision), P.kT, p->richardson, p->vacuum,
                              p->vacuum_direct, P.at<double>(L.slots) + kResSlots, st);
      });
      if (s != NPB_OK) return s;
    }
    return NPB_OK;
  }

  std::vector<unsigned char> graph_key() const {
    std::vector<unsigned char> k(2 * sizeof(int) + sizeof(GraphKey) * pr.size(), 0);
    const int prec = (int)sizeof(T) * 16 + (int)sizeof(A);
    std::memcpy(k.data(), &prec, sizeof(int));
    std::memcpy(k.data() + sizeof(int), &ctx->tune_gen, sizeof(int));
    for (size_t i = 0; i < pr.size(); ++i) {
      GraphKey g;
      std::memset(&g, 0, sizeof(g));
      g.ws = pr[i].ws;
      g.field_out = pr[i].fout;
      g.fu0 = pr[i].fu0;
      g.frho = pr[i].frho;
      g.grid = *pr[i].g;
      g.params = *pr[i].p;
      g.n_atoms = pr[i].mol->n_atoms;
      std::memcpy(k.data() + 2 * sizeof(int) + i * sizeof(GraphKey), &g, sizeof(g));
    }
    return k;
  }

  // After the last launch or copy of a call: the events that let later
  // calls reuse this call's staging buffer and launch tables.
  npb_status mark_enqueued() {
    if (noalloc) return NPB_OK;
    if (pin_slot >= 0) {
      NPB_HIP(hipEventRecord(ctx->pin_ev[pin_slot], st));
      ctx->pin_used[pin_slot] = true;
    }
    NPB_HIP(hipEventRecord(ctx->meta_ev, st));
    ctx->meta_used = true;
    return NPB_OK;
  }

  static constexpr long long kMaxGraphEulerLaunches = 4096;

  // async: out is page-locked host memory written by a last kernel; the
  // call returns once everything is enqueued
  npb_status run(npb_result* out, bool async = false) {
    // A replay of the graph of the same batch needs only the atoms and the
    // chunk tables staged again; the launch tables in the context's buffer
    // are the ones the graph was captured with.
    // long explicit Euler runs launch once per step: no graph of that size
    long long euler_launches = 0;
    for (const Problem& P : pr)
      if (P.p->scheme == NPB_EULER)
        for (int r = 0; r < P.L.n_runs; ++r)
          euler_launches += (long long)P.p->n_steps << P.L.runs[r].level;
    const bool graph =
        ctx->graphs && !ctx->timing && !noalloc && euler_launches <= kMaxGraphEulerLaunches;
    std::vector<unsigned char> key = graph_key();
    const bool replay = graph && ctx->exec && key == ctx->key;
    npb_status s = NPB_OK;
    if (!replay) {
      s = plan();
      if (s != NPB_OK) return s;
    }
    s = stage(!replay);
    if (s != NPB_OK) return s;
    NPB_HIP(hipEventRecord(ctx->t0, st));
    if (graph) {
      if (!replay) {
        if (ctx->exec) (void)hipGraphExecDestroy(ctx->exec);
        ctx->exec = nullptr;
        ctx->key.clear();
        const hipStream_t user = st;
        st = ctx->capture;
        NPB_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        s = device_work();
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(st, &graph);
        st = user;
        if (s != NPB_OK) {
          if (graph) (void)hipGraphDestroy(graph);
          return s;
        }
        if (e != hipSuccess)
          return fail(NPB_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&ctx->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
          ctx->exec = nullptr;
          return fail(NPB_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        ctx->key = key;
      }
      NPB_HIP(hipGraphLaunch(ctx->exec, st));
    } else {
      s = device_work();
      if (s != NPB_OK) return s;
    }
    if (async) {
      for (size_t i = 0; i < pr.size(); ++i) {
        const Problem& P = pr[i];
        const double pts = (double)(P.g->nx - 2) * (P.g->ny - 2) * (P.g->nz - 2);
        int steps = 0;
        for (int r = 0; r < P.L.n_runs; ++r) steps += P.p->n_steps << P.L.runs[r].level;
        NPB_HIP(launch_result(P.at<double>(P.L.slots) + kResSlots, P.at<int>(P.L.ints), &out[i],
                              pts * steps, steps, st));
      }
      return mark_enqueued();
    }
    NPB_HIP(hipEventRecord(ctx->t1, st));
    // results to the host (first 128 bytes per problem of the staging buffer)
    for (size_t i = 0; i < pr.size(); ++i) {
      NPB_HIP(hipMemcpyAsync(hb + 128 * i, pr[i].ws + pr[i].L.slots + 8 * kResSlots,
                             8 * kResCount, hipMemcpyDeviceToHost, st));
      NPB_HIP(hipMemcpyAsync(hb + 128 * i + 96, pr[i].ws + pr[i].L.ints, 8,
                             hipMemcpyDeviceToHost, st));
    }
    npb_status sm = mark_enqueued();
    if (sm != NPB_OK) return sm;
    NPB_HIP(hipStreamSynchronize(st));
    float ms = 0.f;
    NPB_HIP(hipEventElapsedTime(&ms, ctx->t0, ctx->t1));
    if (ctx->timing) harvest(ctx);
    npb_status worst = NPB_OK;
    for (size_t i = 0; i < pr.size(); ++i) {
      const Problem& P = pr[i];
      const double* hres = reinterpret_cast<const double*>(hb + 128 * i);
      const int* hints = reinterpret_cast<const int*>(hb + 128 * i + 96);
      npb_result& o = out[i];
      std::memset(&o, 0, sizeof(o));
      o.dG = hres[0];
      o.dG_plain = hres[1];
      o.G_m[0] = hres[2];
      o.G_m[1] = hres[3];
      o.G_0[0] = hres[4];
      o.G_0[1] = hres[5];
      o.finite = hres[6] != 0.0 ? 1 : 0;
      o.dG_direct = hres[7];
      o.dG_err_est = hres[8];
      const double pts = (double)(P.g->nx - 2) * (P.g->ny - 2) * (P.g->nz - 2);
      for (int r = 0; r < P.L.n_runs; ++r) {
        const int ns = P.p->n_steps << P.L.runs[r].level;
        o.steps_done += ns;
        o.grid_point_updates += pts * ns;
      }
      o.device_ms = ms;
      o.n_charge_nodes = hints[0];
      if (hints[1] != 0 && worst == NPB_OK)
        worst = fail(NPB_ERANGE, "problem " + std::to_string(i) +
                                     ": a trilinear stencil touches the boundary");
      if (!o.finite && worst == NPB_OK)
        worst = fail(NPB_EDIVERGED, "problem " + std::to_string(i) + ": non-finite energy");
    }
    return worst;
  }
};

// Line-solver shape tuning on one problem: its setup, then for each sweep
// direction every candidate (target chunk length x lines per block or tile
// width) is timed over all of the problem's runs, as the solve sweeps them;
// the fastest is kept.  The fields end in an arbitrary state (the next solve
// initialises them again).
template <typename T, typename A>
npb_status autotune_t(npb_ctx* ctx, std::vector<Problem>& pr, hipStream_t st,
                      std::array<int, 6>& choice, double ms[3]) {
  Engine<T, A> E{ctx, st, pr, {}, {}, {}};
  Problem& P = pr[0];
  const bool timing = ctx->timing;
  ctx->timing = false;
  struct Restore {
    npb_ctx* c;
    bool t;
    ~Restore() { c->timing = t; }
  } restore{ctx, timing};
  npb_status s = E.plan();
  if (s != NPB_OK) return s;
  s = E.stage(true);
  if (s != NPB_OK) return s;
  s = E.setup(P);
  if (s != NPB_OK) return s;
  const int nx = P.g->nx, ny = P.g->ny, nz = P.g->nz;
  const int nxp = pitch_of(nx, (int)sizeof(T));
  for (int r = 0; r < P.L.n_runs; ++r) {
    const bool vac = P.L.runs[r].medium == 1;
    NPB_HIP(launch_field_init<T>(P.at<T>(P.L.field[r]), P.at<double>(vac ? P.L.bc_v : P.L.bc_s),
                                 nx, nxp, ny, nz, st));
  }
  const bool f64a = P.p->precision != NPB_FP32;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  NPB_HIP(hipEventCreate(&e0));
  NPB_HIP(hipEventCreate(&e1));
  void* dbuf = nullptr;
  size_t dbytes = 0;
  struct Free {
    hipEvent_t a, b;
    void** buf;
    ~Free() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      if (*buf) (void)hipFree(*buf);
    }
  } cleanup{e0, e1, &dbuf};
  const int nr = P.L.n_runs;
  for (int d = 0; d < 3; ++d) {
    double best = 1e300;
    LaunchShape best_shape = P.L.shape[d];
    int bc0 = 0, bc1 = 0;
    // The built-in shape (timed like the others) is kept unless a candidate
    // is faster by more than kMargin: the candidates are timed one direction
    // at a time with every run in one launch, while the solve runs the two
    // media concurrently, so near ties do not predict the solve.
    constexpr double kMargin = 0.03;
    const LaunchShape builtin = P.L.shape[d];
    double builtin_ms = -1.0;
    std::vector<std::array<int, 3>> tried;
    for (int mt : {12, 16, 20}) {
      for (int pref : {64, 32, 16, 8}) {
        if (d > 0 && (pref == 8 || pref == 64)) continue;
        const LaunchShape sh = d == 0 ? plan_x(nx, ny, nz, f64a, P.aos(), false, mt, pref)
                                      : plan_yz(nx, d == 1 ? ny : nz, d == 1 ? nz : ny, f64a, mt,
                                                pref);
        if (sh.M == 0) continue;
        const std::array<int, 3> id{sh.M, sh.P, sh.LW};
        if (std::find(tried.begin(), tried.end(), id) != tried.end()) continue;
        tried.push_back(id);
        P.L.shape[d] = sh;
        NPB_HIP(launch_chunk_classes(P.sweep_mask(d), nx, nxp, ny, nz, d, sh.M, sh.P,
                                     P.location() ? 1 : 0, P.at<uint8_t>(P.L.ccls[d]), st));
        // chunk tables of this chunk length for every run
        NPB_HIP(hipStreamSynchronize(st));
        unsigned char* hb = E.hb;
        for (int r = 0; r < nr; ++r) {
          const Coefs c = run_coefs(P, P.L.runs[r]);
          ChunkTab<A>& tb =
              *reinterpret_cast<ChunkTab<A>*>(hb + P.tabs_pinned + kTabBytes * (3 * r + d));
          const int nint = (d == 0 ? P.g->nx : d == 1 ? P.g->ny : P.g->nz) - 2;
          if (c.vacuum)
            fill_chunk_tab(tb, c.re_uniform, c.re_uniform, sh.M, nint);
          else
            fill_chunk_tab(tb, c.re[0], c.re[2], sh.M, nint);
          NPB_HIP(hipMemcpyAsync(P.ws + P.L.tabs + kTabBytes * (3 * r + d),
                                 hb + P.tabs_pinned + kTabBytes * (3 * r + d), kTabBytes,
                                 hipMemcpyHostToDevice, st));
        }
        // launch tables: every run, all blocks
        std::vector<SweepArgs<T>> args(nr);
        for (int r = 0; r < nr; ++r) args[r] = E.sweep_args(P, r, d);
        const int nb = sh.blocks * nr;
        std::vector<int2> work(nb);
        for (int r = 0, k = 0; r < nr; ++r)
          for (int b = 0; b < sh.blocks; ++b) work[k++] = make_int2(r, b);
        const size_t ab = (sizeof(SweepArgs<T>) * nr + 255) & ~size_t(255);
        const size_t need = ab + sizeof(int2) * nb;
        if (need > dbytes) {
          NPB_HIP(hipStreamSynchronize(st));
          if (dbuf) (void)hipFree(dbuf);
          dbuf = nullptr;
          NPB_HIP(hipMalloc(&dbuf, need));
          dbytes = need;
        }
        NPB_HIP(hipStreamSynchronize(st));
        NPB_HIP(hipMemcpy(dbuf, args.data(), sizeof(SweepArgs<T>) * nr, hipMemcpyHostToDevice));
        NPB_HIP(hipMemcpy(static_cast<unsigned char*>(dbuf) + ab, work.data(),
                          sizeof(int2) * nb, hipMemcpyHostToDevice));
        const auto* dargs = static_cast<const SweepArgs<T>*>(dbuf);
        const auto* dwork = reinterpret_cast<const int2*>(static_cast<unsigned char*>(dbuf) + ab);
        const int var = d == 0 ? sweep_cn(args.data(), nr) : sweep_variant(args.data(), nr);
        auto launch = [&] {
          return d == 0 ? launch_sweep_x<T, A>(dargs, dwork, sh.blocks, nb, var, sh, st)
                        : launch_sweep_yz<T, A>(dargs, dwork, sh.blocks, nb, d, var, sh, st);
        };
        constexpr int kWarm = 2, kReps = 5;
        for (int i = 0; i < kWarm; ++i) NPB_HIP(launch());
        NPB_HIP(hipEventRecord(e0, st));
        for (int i = 0; i < kReps; ++i) NPB_HIP(launch());
        NPB_HIP(hipEventRecord(e1, st));
        NPB_HIP(hipEventSynchronize(e1));
        float t = 0.f;
        NPB_HIP(hipEventElapsedTime(&t, e0, e1));
        if (sh.M == builtin.M && sh.P == builtin.P && sh.LW == builtin.LW) builtin_ms = t / kReps;
        if (t / kReps < best) {
          best = t / kReps;
          best_shape = sh;
          bc0 = mt;
          bc1 = pref;
        }
      }
    }
    if (builtin_ms > 0.0 && best > (1.0 - kMargin) * builtin_ms) {
      best_shape = builtin;
      best = builtin_ms;
      bc0 = 0;  // the built-in choice (planner defaults)
      bc1 = 0;
    }
    P.L.shape[d] = best_shape;
    choice[2 * d] = bc0;
    choice[2 * d + 1] = bc1;
    ms[d] = best;
  }
  NPB_HIP(hipStreamSynchronize(st));
  return NPB_OK;
}

template <typename T, typename A>
npb_status solve_batch_t(npb_ctx* ctx, std::vector<Problem>& pr, hipStream_t st, npb_result* out,
                         bool async, bool noalloc) {
  Engine<T, A> E{ctx, st, pr, {}, {}, {}};
  E.noalloc = noalloc;
  return E.run(out, async);
}


// ---------------------------------------------------------------------------
// Continuous stepping for the request loop.  A tick enqueues, on one stream:
// the setup and field initialisation of the problems added since the last
// tick; up to K steps of every active run in the shared launches of the
// batch path (one per sweep direction and launch shape per step, over the
// runs that still have steps, so that each run's arithmetic is that of its
// single solve); and, for each problem whose last step that was, its
// energies and combinations and a copy of its result into page-locked host
// memory behind an event.  Problems therefore join between two ticks and
// leave as soon as their last step is done.  Two contexts alternate between
// ticks: one tick's launch tables and staging are written while the
// previous tick's launches run, and a tick waits only for the tick two
// before it.  Explicit Euler problems take all their steps in the tick that
// sets them up.
template <typename T, typename A>
struct RollingT final : RollingEngine {
  npb_ctx* cx[2] = {nullptr, nullptr};
  hipStream_t st = nullptr;
  int tick_no = 0;
  hipEvent_t tick_ev[2] = {nullptr, nullptr};
  bool tick_used[2] = {false, false};
  // page-locked results: kSlot bytes per item slot (results, then the ints)
  static constexpr size_t kSlot = 128;
  unsigned char* hres = nullptr;
  std::vector<int> free_slots;
  struct Item {
    uint64_t id = 0;
    Problem P;
    int left[kMaxFields] = {0, 0, 0, 0};
    int slot = -1;
    bool started = false, finishing = false, enqueued = false;
    hipEvent_t ev = nullptr;
  };
  std::list<Item> items;

  ~RollingT() override {
    (void)drain();
    for (Item& it : items)
      if (it.ev) (void)hipEventDestroy(it.ev);
    for (int c = 0; c < 2; ++c) {
      if (tick_ev[c]) (void)hipEventDestroy(tick_ev[c]);
      if (cx[c]) npb_ctx_destroy(cx[c]);
    }
    if (hres) (void)hipHostFree(hres);
  }

  npb_status init(const npb_ctx* tuned, hipStream_t stream, int max_items) {
    st = stream;
    for (int c = 0; c < 2; ++c) {
      npb_status s = npb_ctx_create(tuned->device, &cx[c]);
      if (s != NPB_OK) return s;
      cx[c]->tune = tuned->tune;
      cx[c]->graphs = false;
      NPB_HIP(hipEventCreateWithFlags(&tick_ev[c], hipEventDisableTiming));
    }
    NPB_HIP(hipHostMalloc(reinterpret_cast<void**>(&hres), kSlot * (size_t)max_items,
                          hipHostMallocDefault));
    for (int k = max_items - 1; k >= 0; --k) free_slots.push_back(k);
    return NPB_OK;
  }

  npb_status add(uint64_t id, const npb_molecule* mol, const npb_grid* grid,
                 const npb_params* params, void* ws, size_t ws_bytes) override {
    if (free_slots.empty()) return fail(NPB_EBUSY, "request loop: no free result slot");
    Item it;
    it.id = id;
    Problem& P = it.P;
    P.mol = mol;
    P.g = grid;
    P.p = params;
    P.ws = reinterpret_cast<unsigned char*>(ws);
    P.fout = nullptr;
    P.L = make_layout(mol, grid, params);
    P.kT = thermal_energy(params->temperature_K);
    P.lB = bjerrum(params->temperature_K);
    if (!P.ws || ws_bytes < P.L.total || reinterpret_cast<uintptr_t>(P.ws) % 256 != 0)
      return fail(NPB_EINVAL, "request loop: workspace too small or misaligned");
    apply_tuning(cx[0], grid, params, P.L);
    for (int r = 0; r < P.L.n_runs; ++r) it.left[r] = params->n_steps << P.L.runs[r].level;
    NPB_HIP(hipEventCreateWithFlags(&it.ev, hipEventDisableTiming));
    it.slot = free_slots.back();
    free_slots.pop_back();
    items.push_back(it);
    return NPB_OK;
  }

  static bool has_steps(const Item& it) {
    for (int r = 0; r < it.P.L.n_runs; ++r)
      if (it.left[r] > 0) return true;
    return false;
  }

  npb_status tick(int K) override {
    const int c = tick_no & 1;
    npb_ctx* ctx = cx[c];
    NPB_HIP(hipSetDevice(ctx->device));
    // at most two ticks on the device
    if (tick_used[c]) NPB_HIP(hipEventSynchronize(tick_ev[c]));
    bool any = false;
    // 1. setup of the problems added since the last tick (explicit Euler
    // problems also take all their steps here)
    {
      std::vector<Problem> np;
      std::vector<Item*> ni;
      for (Item& it : items)
        if (!it.started) {
          np.push_back(it.P);
          ni.push_back(&it);
        }
      if (!np.empty()) {
        Engine<T, A> E{ctx, st, np, {}, {}, {}};
        npb_status s = E.stage(false);
        if (s == NPB_OK) s = E.setup_all();
        if (s == NPB_OK) s = E.init_fields();
        if (s == NPB_OK) s = E.euler_loop();
        if (s == NPB_OK) s = E.mark_enqueued();
        if (s != NPB_OK) return s;
        for (Item* it : ni) {
          it->started = true;
          if (it->P.p->scheme == NPB_EULER)
            for (int r = 0; r < it->P.L.n_runs; ++r) it->left[r] = 0;
        }
        any = true;
      }
    }
    // 2. up to K steps of every run with steps left
    {
      std::vector<Problem> ap;
      std::vector<Item*> ai;
      for (Item& it : items)
        if (it.started && has_steps(it)) {
          Problem P = it.P;
          for (int r = 0; r < kMaxFields; ++r)
            P.steps_now[r] = r < P.L.n_runs ? std::min(it.left[r], K) : 0;
          ap.push_back(P);
          ai.push_back(&it);
        }
      if (!ap.empty()) {
        Engine<T, A> E{ctx, st, ap, {}, {}, {}};
        E.stage_problems = false;
        npb_status s = E.plan();
        if (s == NPB_OK) s = E.stage(true);
        if (s == NPB_OK) s = E.step_loop();
        if (s == NPB_OK) s = E.mark_enqueued();
        if (s != NPB_OK) return s;
        for (size_t k = 0; k < ai.size(); ++k)
          for (int r = 0; r < ai[k]->P.L.n_runs; ++r) ai[k]->left[r] -= ap[k].steps_now[r];
        any = true;
      }
    }
    // 3. problems whose last step is enqueued: energies, combinations, result
    {
      std::vector<Problem> fp;
      std::vector<Item*> fi;
      for (Item& it : items)
        if (it.started && !it.enqueued && !has_steps(it)) {
          fp.push_back(it.P);
          fi.push_back(&it);
        }
      if (!fp.empty()) {
        Engine<T, A> E{ctx, st, fp, {}, {}, {}};
        for (size_t k = 0; k < fp.size(); ++k) {
          npb_status s = E.finish(fp[k]);
          if (s != NPB_OK) return s;
          const Problem& P = fp[k];
          unsigned char* h = hres + kSlot * (size_t)fi[k]->slot;
          NPB_HIP(hipMemcpyAsync(h, P.ws + P.L.slots + 8 * kResSlots, 8 * kResCount,
                                 hipMemcpyDeviceToHost, st));
          NPB_HIP(hipMemcpyAsync(h + 96, P.ws + P.L.ints, 8, hipMemcpyDeviceToHost, st));
          NPB_HIP(hipEventRecord(fi[k]->ev, st));
          fi[k]->enqueued = true;
        }
        any = true;
      }
    }
    if (any) {
      NPB_HIP(hipEventRecord(tick_ev[c], st));
      tick_used[c] = true;
      tick_no += 1;
    }
    return NPB_OK;
  }

  void poll(std::vector<RollingDone>& out) override {
    for (auto it = items.begin(); it != items.end();) {
      if (!it->enqueued || hipEventQuery(it->ev) != hipSuccess) {
        ++it;
        continue;
      }
      const Problem& P = it->P;
      const unsigned char* h = hres + kSlot * (size_t)it->slot;
      const double* r = reinterpret_cast<const double*>(h);
      const int* ints = reinterpret_cast<const int*>(h + 96);
      RollingDone d{};
      d.id = it->id;
      npb_result& o = d.res;
      o.dG = r[0];
      o.dG_plain = r[1];
      o.G_m[0] = r[2];
      o.G_m[1] = r[3];
      o.G_0[0] = r[4];
      o.G_0[1] = r[5];
      o.finite = r[6] != 0.0 ? 1 : 0;
      o.dG_direct = r[7];
      o.dG_err_est = r[8];
      const double pts = (double)(P.g->nx - 2) * (P.g->ny - 2) * (P.g->nz - 2);
      for (int k = 0; k < P.L.n_runs; ++k) {
        const int ns = P.p->n_steps << P.L.runs[k].level;
        o.steps_done += ns;
        o.grid_point_updates += pts * ns;
      }
      o.device_ms = std::nan("");
      o.n_charge_nodes = ints[0];
      d.status = ints[1] != 0 ? NPB_ERANGE : (o.finite ? NPB_OK : NPB_EDIVERGED);
      out.push_back(d);
      (void)hipEventDestroy(it->ev);
      free_slots.push_back(it->slot);
      it = items.erase(it);
    }
  }

  int active() const override { return (int)items.size(); }
  int stepping() const override {
    int n = 0;
    for (const Item& it : items)
      if (!it.started || has_steps(it)) ++n;
    return n;
  }
  npb_status drain() override {
    NPB_HIP(hipStreamSynchronize(st));
    return NPB_OK;
  }
  void abort_all(npb_status s, std::vector<RollingDone>& out) override {
    (void)hipStreamSynchronize(st);
    for (Item& it : items) {
      RollingDone d{};
      d.id = it.id;
      d.status = s;
      d.res.dG = d.res.dG_plain = d.res.dG_direct = d.res.dG_err_est = std::nan("");
      out.push_back(d);
      (void)hipEventDestroy(it.ev);
      free_slots.push_back(it.slot);
    }
    items.clear();
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

int npb_abi_version(void) { return NPB_ABI_VERSION; }

const char* npb_last_error(void) { return g_err.c_str(); }

double npb_kappa_bar_sq(double ionic_molar, double temperature_K) {
  return kKbar2PerMolar298 * (298.0 / temperature_K) * ionic_molar;
}

// streams and events of a context, then the context itself
static void ctx_release(npb_ctx* c) {
  for (hipEvent_t e : {c->t0, c->t1, c->fork, c->meta_ev, c->pin_ev[0], c->pin_ev[1]})
    if (e) (void)hipEventDestroy(e);
  for (int i = 0; i < npb_ctx::kLanes - 1; ++i) {
    if (c->lag[i]) (void)hipEventDestroy(c->lag[i]);
    if (c->join[i]) (void)hipEventDestroy(c->join[i]);
    if (c->side[i]) (void)hipStreamDestroy(c->side[i]);
  }
  if (c->capture) (void)hipStreamDestroy(c->capture);
  delete c;
}

npb_status npb_ctx_create(int device, npb_ctx** out) {
  if (!out) return fail(NPB_EINVAL, "null output pointer");
  *out = nullptr;
  int ndev = 0;
  NPB_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(NPB_EINVAL, "no such device");
  NPB_HIP(hipSetDevice(device));
  npb_ctx* c = new (std::nothrow) npb_ctx();
  if (!c) return fail(NPB_ENOMEM, "context allocation failed");
  c->device = device;
  bool ok = hipEventCreate(&c->t0) == hipSuccess && hipEventCreate(&c->t1) == hipSuccess &&
            hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&c->meta_ev, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&c->pin_ev[0], hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&c->pin_ev[1], hipEventDisableTiming) == hipSuccess &&
            hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; ok && i < npb_ctx::kLanes - 1; ++i)
    ok = hipEventCreateWithFlags(&c->lag[i], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming) == hipSuccess &&
         hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    ctx_release(c);
    return fail(NPB_EDEVICE, "event or stream creation failed");
  }
  const hipError_t se = scratch_address(device, &c->scratch);
  if (se != hipSuccess) {
    ctx_release(c);
    return fail(NPB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                 hipGetErrorString(se));
  }
  *out = c;
  return NPB_OK;
}

void npb_ctx_destroy(npb_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  // enqueued copies may still read the staging buffers and launch tables
  for (int b = 0; b < 2; ++b)
    if (c->pin_used[b]) (void)hipEventSynchronize(c->pin_ev[b]);
  if (c->meta_used) (void)hipEventSynchronize(c->meta_ev);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->meta) (void)hipFree(c->meta);
  for (int b = 0; b < 2; ++b)
    if (c->pin[b]) (void)hipHostFree(c->pin[b]);
  ctx_release(c);
}

npb_status npb_ctx_set_timing(npb_ctx* c, int enable) {
  if (!c) return fail(NPB_EINVAL, "null context");
  c->timing = enable != 0;
  if (c->timing) std::memset(&c->times, 0, sizeof(c->times));
  return NPB_OK;
}

npb_status npb_ctx_set_graph(npb_ctx* c, int enable) {
  if (!c) return fail(NPB_EINVAL, "null context");
  c->graphs = enable != 0;
  return NPB_OK;
}

npb_status npb_ctx_get_kernel_times(npb_ctx* c, npb_kernel_times* out) {
  if (!c || !out) return fail(NPB_EINVAL, "null argument");
  *out = c->times;
  return NPB_OK;
}

npb_status npb_validate(const npb_molecule* mol, const npb_grid* grid, const npb_params* params) {
  return validate(mol, grid, params);
}

npb_status npb_workspace_bytes(const npb_molecule* mol, const npb_grid* grid,
                               const npb_params* params, size_t* bytes) {
  if (!bytes) return fail(NPB_EINVAL, "null output pointer");
  npb_status s = validate(mol, grid, params);
  if (s != NPB_OK) return s;
  *bytes = make_layout(mol, grid, params).total;
  return NPB_OK;
}

}  // extern "C"

namespace {

// the device work of checked problems (one precision)
npb_status run_problems(npb_ctx* ctx, std::vector<Problem>& pr, void* stream, npb_result* out,
                        bool async = false, bool noalloc = false) {
  // every argument checked: only now is the context read
  for (Problem& P : pr) apply_tuning(ctx, P.g, P.p, P.L);
  NPB_HIP(hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int precision = pr[0].p->precision;
  // the no-allocation path takes no timing events either
  struct TimingOff {
    npb_ctx* c;
    bool was;
    ~TimingOff() { c->timing = was; }
  } keep{ctx, ctx->timing};
  if (noalloc) ctx->timing = false;
  try {
    if (precision == NPB_FP64)
      return solve_batch_t<double, double>(ctx, pr, st, out, async, noalloc);
    if (precision == NPB_FP32X)
      return solve_batch_t<float, double>(ctx, pr, st, out, async, noalloc);
    return solve_batch_t<float, float>(ctx, pr, st, out, async, noalloc);
  } catch (const std::exception& e) {
    return fail(NPB_ENOMEM, e.what());
  } catch (...) {
    return fail(NPB_EDEVICE, "unexpected failure");
  }
}

// npb_solve_fields runs one field: no vacuum problem, no direct solve, the
// solvated field out
npb_status validate_fields(const npb_params* p) {
  if (p->vacuum || p->vacuum_direct || p->field_select != 0)
    return fail(NPB_EINVAL, "caller-given fields need vacuum = vacuum_direct = field_select = 0");
  return NPB_OK;
}

}  // namespace

extern "C" {

npb_status npb_solve_batch(npb_ctx* ctx, int n, const npb_molecule* mols, const npb_grid* grids,
                           const npb_params* params, void* const* d_ws, const size_t* ws_bytes,
                           double* const* d_field_out, void* stream, npb_result* out) {
  if (!ctx || !out) return fail(NPB_EINVAL, "null context or result");
  if (n < 1 || !mols || !grids || !params || !d_ws || !ws_bytes)
    return fail(NPB_EINVAL, "empty batch or null array");
  std::vector<Problem> pr(n);
  for (int i = 0; i < n; ++i) {
    npb_status s = validate(&mols[i], &grids[i], &params[i]);
    if (s != NPB_OK) return fail(s, "problem " + std::to_string(i) + ": " + g_err);
    if (params[i].precision != params[0].precision)
      return fail(NPB_EINVAL, "problem " + std::to_string(i) + ": a batch runs one precision");
    Problem& P = pr[i];
    P.mol = &mols[i];
    P.g = &grids[i];
    P.p = &params[i];
    P.ws = reinterpret_cast<unsigned char*>(d_ws[i]);
    P.fout = d_field_out ? d_field_out[i] : nullptr;
    P.L = make_layout(P.mol, P.g, P.p);
    P.kT = thermal_energy(P.p->temperature_K);
    P.lB = bjerrum(P.p->temperature_K);
    if (!P.ws || ws_bytes[i] < P.L.total)
      return fail(NPB_EINVAL, "problem " + std::to_string(i) +
                                  ": workspace missing or smaller than npb_workspace_bytes");
    if (reinterpret_cast<uintptr_t>(P.ws) % 256 != 0)
      return fail(NPB_EINVAL, "problem " + std::to_string(i) +
                                  ": workspace must be 256-byte aligned");
    for (int j = 0; j < i; ++j)
      if (pr[j].ws == P.ws)
        return fail(NPB_EINVAL, "problem " + std::to_string(i) + ": workspace shared with problem " +
                                    std::to_string(j));
  }
  return run_problems(ctx, pr, stream, out);
}

npb_status npb_solve_async(npb_ctx* ctx, const npb_molecule* mol, const npb_grid* grid,
                           const npb_params* params, void* d_ws, size_t ws_bytes,
                           double* d_field_out, void* stream, npb_result* pinned_out) {
  if (!ctx || !pinned_out) return fail(NPB_EINVAL, "null context or result");
  if (!mol || !grid || !params) return fail(NPB_EINVAL, "null argument");
  npb_status s = validate(mol, grid, params);
  if (s != NPB_OK) return s;
  hipPointerAttribute_t attr{};
  if (hipPointerGetAttributes(&attr, pinned_out) != hipSuccess || attr.type != hipMemoryTypeHost) {
    (void)hipGetLastError();
    return fail(NPB_EINVAL, "pinned_out must be page-locked host memory");
  }
  std::vector<Problem> pr(1);
  Problem& P = pr[0];
  P.mol = mol;
  P.g = grid;
  P.p = params;
  P.ws = reinterpret_cast<unsigned char*>(d_ws);
  P.fout = d_field_out;
  P.L = make_layout(mol, grid, params);
  P.kT = thermal_energy(params->temperature_K);
  P.lB = bjerrum(params->temperature_K);
  if (!P.ws || ws_bytes < P.L.total)
    return fail(NPB_EINVAL, "workspace missing or smaller than npb_workspace_bytes");
  if (reinterpret_cast<uintptr_t>(P.ws) % 256 != 0)
    return fail(NPB_EINVAL, "workspace must be 256-byte aligned");
  return run_problems(ctx, pr, stream, pinned_out, true);
}

npb_status npb_default_grid(const npb_molecule* mol, double h, double margin, npb_grid* out) {
  if (!mol || !out) return fail(NPB_EINVAL, "null argument");
  if (mol->n_atoms < 1 || !mol->xyz || !mol->radius) return fail(NPB_EINVAL, "no atoms");
  if (!(h > 0.0) || !(margin > 0.0) || !std::isfinite(h) || !std::isfinite(margin))
    return fail(NPB_EINVAL, "h and margin must be positive");
  npb_grid g{};
  g.h = h;
  int* n[3] = {&g.nx, &g.ny, &g.nz};
  for (int d = 0; d < 3; ++d) {
    double lo = 1e300, hi = -1e300;
    for (int a = 0; a < mol->n_atoms; ++a) {
      const double c = mol->xyz[3 * a + d], r = mol->radius[a];
      if (!std::isfinite(c) || !std::isfinite(r)) return fail(NPB_EINVAL, "bad atom");
      lo = std::min(lo, c - r);
      hi = std::max(hi, c + r);
    }
    const double half = 0.5 * (hi - lo) + margin;
    const double cells = std::ceil(half / h - 1e-9);
    if (cells > 256.0) return fail(NPB_EINVAL, "grid axis longer than 514 nodes");
    const int nn = std::max(5, 2 * (int)cells + 1);
    *n[d] = nn;
    g.origin[d] = 0.5 * (lo + hi) - 0.5 * (nn - 1) * h;
  }
  *out = g;
  return NPB_OK;
}

npb_status npb_fields_workspace_bytes(const npb_molecule* mol, const npb_grid* grid,
                                      const npb_params* params, size_t* bytes) {
  if (!bytes) return fail(NPB_EINVAL, "null output pointer");
  npb_status s = validate(mol, grid, params);
  if (s != NPB_OK) return s;
  s = validate_fields(params);
  if (s != NPB_OK) return s;
  *bytes = make_layout(mol, grid, params, true).total;
  return NPB_OK;
}

npb_status npb_solve_fields(npb_ctx* ctx, const npb_molecule* solute, const npb_grid* grid,
                            const npb_params* params, const double* d_u0, const double* d_rho,
                            void* d_ws, size_t ws_bytes, double* d_u_out, void* stream,
                            npb_result* out) {
  if (!ctx || !out) return fail(NPB_EINVAL, "null context or result");
  if (!solute || !grid || !params || !d_u0 || !d_rho) return fail(NPB_EINVAL, "null argument");
  npb_status s = validate(solute, grid, params);
  if (s != NPB_OK) return s;
  s = validate_fields(params);
  if (s != NPB_OK) return s;
  std::vector<Problem> pr(1);
  Problem& P = pr[0];
  P.mol = solute;
  P.g = grid;
  P.p = params;
  P.ws = reinterpret_cast<unsigned char*>(d_ws);
  P.fout = d_u_out;
  P.fu0 = d_u0;
  P.frho = d_rho;
  P.L = make_layout(solute, grid, params, true);
  P.kT = thermal_energy(params->temperature_K);
  P.lB = bjerrum(params->temperature_K);
  if (!P.ws || ws_bytes < P.L.total)
    return fail(NPB_EINVAL, "workspace missing or smaller than npb_fields_workspace_bytes");
  if (reinterpret_cast<uintptr_t>(P.ws) % 256 != 0)
    return fail(NPB_EINVAL, "workspace must be 256-byte aligned");
  return run_problems(ctx, pr, stream, out);
}

npb_status npb_autotune(npb_ctx* ctx, const npb_molecule* mol, const npb_grid* grid,
                        const npb_params* params, void* d_ws, size_t ws_bytes, void* stream,
                        double* ms_out) {
  if (!ctx || !mol || !grid || !params) return fail(NPB_EINVAL, "null argument");
  npb_status s = validate(mol, grid, params);
  if (s != NPB_OK) return s;
  if (params->scheme == NPB_EULER)
    return fail(NPB_EINVAL, "explicit Euler has no line-solver shapes to tune");
  std::vector<Problem> pr(1);
  Problem& P = pr[0];
  P.mol = mol;
  P.g = grid;
  P.p = params;
  P.ws = reinterpret_cast<unsigned char*>(d_ws);
  P.fout = nullptr;
  P.L = make_layout(mol, grid, params);
  P.kT = thermal_energy(params->temperature_K);
  P.lB = bjerrum(params->temperature_K);
  if (!P.ws || ws_bytes < P.L.total)
    return fail(NPB_EINVAL, "workspace missing or smaller than npb_workspace_bytes");
  if (reinterpret_cast<uintptr_t>(P.ws) % 256 != 0)
    return fail(NPB_EINVAL, "workspace must be 256-byte aligned");
  NPB_HIP(hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::array<int, 6> choice{};
  double ms[3] = {0, 0, 0};
  try {
    if (params->precision == NPB_FP64)
      s = autotune_t<double, double>(ctx, pr, st, choice, ms);
    else if (params->precision == NPB_FP32X)
      s = autotune_t<float, double>(ctx, pr, st, choice, ms);
    else
      s = autotune_t<float, float>(ctx, pr, st, choice, ms);
  } catch (const std::exception& e) {
    return fail(NPB_ENOMEM, e.what());
  }
  if (s != NPB_OK) return s;
  ctx->tune[tune_key(grid, params)] = choice;
  ctx->tune_gen += 1;
  if (ms_out)
    for (int d = 0; d < 3; ++d) ms_out[d] = ms[d];
  return NPB_OK;
}

npb_status npb_launch_shapes(const npb_ctx* ctx, const npb_grid* grid, const npb_params* params,
                             int32_t* out) {
  if (!grid || !params || !out) return fail(NPB_EINVAL, "null argument");
  npb_molecule none{0, nullptr, nullptr, nullptr};
  npb_status s = validate(&none, grid, params);
  if (s != NPB_OK) return s;
  Layout L = make_layout(&none, grid, params);
  if (ctx) apply_tuning(ctx, grid, params, L);
  for (int d = 0; d < 3; ++d) {
    out[4 * d] = L.shape[d].M;
    out[4 * d + 1] = L.shape[d].P;
    out[4 * d + 2] = L.shape[d].LW;
    out[4 * d + 3] = L.shape[d].threads;
  }
  return NPB_OK;
}

npb_status npb_solve(npb_ctx* ctx, const npb_molecule* mol, const npb_grid* grid,
                     const npb_params* params, void* d_ws, size_t ws_bytes, double* d_field_out,
                     void* stream, npb_result* out) {
  if (!ctx || !out) return fail(NPB_EINVAL, "null context or result");
  if (!mol || !grid || !params) return fail(NPB_EINVAL, "null argument");
  void* ws[1] = {d_ws};
  const size_t wb[1] = {ws_bytes};
  double* fo[1] = {d_field_out};
  const npb_status s = npb_solve_batch(ctx, 1, mol, grid, params, ws, wb, fo, stream, out);
  if (s != NPB_OK && g_err.rfind("problem 0: ", 0) == 0) g_err = g_err.substr(11);
  return s;
}

npb_status npb_solve_noalloc(npb_ctx* ctx, const npb_molecule* mol, const npb_grid* grid,
                             const npb_params* params, double* d_field_out, void* stream,
                             npb_result* out) {
  if (!ctx || !out) return fail(NPB_EINVAL, "null context or result");
  if (!mol || !grid || !params) return fail(NPB_EINVAL, "null argument");
  npb_status s = validate(mol, grid, params);
  if (s != NPB_OK) return s;
  if (!ctx->scratch) return fail(NPB_EDEVICE, "no static scratch on this device");
  std::vector<Problem> pr(1);
  Problem& P = pr[0];
  P.mol = mol;
  P.g = grid;
  P.p = params;
  P.ws = ctx->scratch;
  P.fout = d_field_out;
  P.L = make_layout(mol, grid, params);
  P.kT = thermal_energy(params->temperature_K);
  P.lB = bjerrum(params->temperature_K);
  if (P.L.total > (size_t)NPB_NOALLOC_BYTES)
    return fail(NPB_EINVAL, "workspace of " + std::to_string(P.L.total) +
                                " bytes exceeds the static scratch of " +
                                std::to_string((size_t)NPB_NOALLOC_BYTES) + " bytes");
  return run_problems(ctx, pr, stream, out, false, true);
}

}  // extern "C"

npb_status npb::rolling_create(const npb_ctx* tuned, int precision, void* stream, int max_items,
                               RollingEngine** out) {
  *out = nullptr;
  if (!tuned || max_items < 1) return fail(NPB_EINVAL, "request loop: bad engine arguments");
  try {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (precision == NPB_FP64) {
      auto* e = new RollingT<double, double>();
      npb_status s = e->init(tuned, st, max_items);
      if (s != NPB_OK) {
        delete e;
        return s;
      }
      *out = e;
    } else if (precision == NPB_FP32X) {
      auto* e = new RollingT<float, double>();
      npb_status s = e->init(tuned, st, max_items);
      if (s != NPB_OK) {
        delete e;
        return s;
      }
      *out = e;
    } else {
      auto* e = new RollingT<float, float>();
      npb_status s = e->init(tuned, st, max_items);
      if (s != NPB_OK) {
        delete e;
        return s;
      }
      *out = e;
    }
  } catch (const std::exception& e) {
    return fail(NPB_ENOMEM, e.what());
  }
  return NPB_OK;
}
