// Host runtime of the NPB library: C ABI, validation, workspace layout and
// the sequence of device launches of one solve.  Also the small field and
// energy kernels (field initialisation, FP64 energy gathers, the
// solvated-minus-vacuum and Richardson combinations).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
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

// S = sum_k q_k u[idx_k] in double, fixed order (one block, tree reduction)
template <typename T>
__global__ __launch_bounds__(1024) void energy_kernel(const T* u, const int* q_idx,
                                                      const double* q_val, const int* nq_dev,
                                                      double* slot) {
  __shared__ double part[1024];
  const int nq = *nq_dev;
  double s = 0.0;
  for (int k = threadIdx.x; k < nq; k += 1024) s += q_val[k] * (double)u[q_idx[k]];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *slot = part[0];
}

template <typename T>
hipError_t launch_energy(const T* u, const int* q_idx, const double* q_val, const int* nq_dev,
                         int /*cap*/, double* slot, hipStream_t st) {
  hipLaunchKernelGGL((energy_kernel<T>), dim3(1), dim3(1024), 0, st, u, q_idx, q_val, nq_dev,
                     slot);
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

// S = [solvated dt, solvated dt/2, vacuum dt, vacuum dt/2] sums of q u.
// res = [dG, dG_plain, G_m0, G_m1, G_00, G_01, finite]
__global__ void combine_kernel(const double* S, double kT, int richardson, int vacuum,
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
  res[6] = fin ? 1.0 : 0.0;
}

hipError_t launch_combine(const double* S, double kT, int richardson, int vacuum, double* res,
                          hipStream_t st) {
  hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(1), 0, st, S, kT, richardson, vacuum, res);
  return hipGetLastError();
}

template hipError_t launch_field_init<float>(float*, const double*, int, int, int, int,
                                             hipStream_t);
template hipError_t launch_field_init<double>(double*, const double*, int, int, int, int,
                                              hipStream_t);

}  // namespace npb

// ---------------------------------------------------------------------------
// context

// Everything a captured solve graph depends on besides the staged bytes.
struct GraphKey {
  void* ws;
  double* field_out;
  void* pinned;
  npb_grid grid;
  npb_params params;
  int n_atoms;
};

struct npb_ctx {
  int device = 0;
  bool timing = false;
  bool graphs = true;
  hipStream_t capture = nullptr;  // stream the solve graph is captured on
  hipGraphExec_t exec = nullptr;
  GraphKey key{};
  npb_kernel_times times{};
  struct Pending {
    int cls;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t t0 = nullptr, t1 = nullptr;
};

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
  LaunchShape shape[3];
  Run runs[kMaxFields];
  int n_runs, cap, nblocks;
};

// host staging (pinned): chunk tables first, then the atom planes
constexpr size_t kTabBytes = sizeof(ChunkTab<double>);

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Per-line source lists each scheme's y and z sweeps use: AOSIE2 adds
// sources in both, LODIE1 after the z solve (LODIE2 and AOSIE1 add theirs
// in the x sweep).
bool needs_y_sources(int scheme) { return scheme == NPB_AOSIE2; }
bool needs_z_sources(int scheme) { return scheme == NPB_AOSIE2 || scheme == NPB_LODIE1; }

Layout make_layout(const npb_molecule* mol, const npb_grid* g, const npb_params* p) {
  Layout L{};
  const size_t es = p->precision == NPB_FP64 ? 8 : 4;
  const size_t n = (size_t)pitch_of(g->nx, (int)es) * g->ny * g->nz;  // pitched node count
  const int na = mol->n_atoms;
  const int cap = 8 * na;
  const int nb = (cap + 255) / 256;
  const size_t ns = (size_t)shell_count(g->nx, g->ny, g->nz);
  const bool aos = p->scheme == NPB_AOSIE1 || p->scheme == NPB_AOSIE2;
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
    L.acc[r] = take(r < L.n_runs && aos ? n * es : 0);
  }
  L.mask = take(n);
  L.bc_s = take(ns * 8);
  L.bc_v = take(p->vacuum ? ns * 8 : 0);
  L.atoms = take((size_t)5 * na * 8);
  L.tabs = take(kTabBytes * 3 * kMaxFields);
  L.key_a = take((size_t)cap * 4);
  L.id_a = take((size_t)cap * 4);
  L.key_b = take((size_t)cap * 4);
  L.id_b = take((size_t)cap * 4);
  L.sval = take((size_t)cap * 8);
  L.hist = take((size_t)256 * (nb > 0 ? nb : 1) * 4);
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
    for (int d = 0; d < 3; ++d) {
      const long long nl = class_lines(g->nx, g->ny, g->nz, d);
      L.ccls[d] = take((size_t)nl * (size_t)(L.shape[d].P > 0 ? L.shape[d].P : 1));
    }
  }
  L.slots = take(32 * 8);
  L.ints = take(16 * 4);
  L.total = off;
  L.cap = cap;
  L.nblocks = nb;
  return L;
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
  if (p->scheme < 0 || p->scheme > 3) return fail(NPB_EINVAL, "unknown scheme");
  if (p->precision < 0 || p->precision > 2) return fail(NPB_EINVAL, "unknown precision");
  if (p->field_select < 0 || p->field_select > 1 || (p->field_select == 1 && !p->vacuum))
    return fail(NPB_EINVAL, "field_select 1 needs vacuum = 1");
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

template <typename T, typename A>
struct Solver {
  npb_ctx* ctx;
  const npb_grid* g;
  const npb_params* p;
  hipStream_t st;
  unsigned char* ws;
  Layout L;
  SetupArgs sa;
  double kT, lB;

  template <typename Ptr>
  Ptr* at(size_t off) {
    return reinterpret_cast<Ptr*>(ws + off);
  }

  template <typename F>
  npb_status timed(int cls, double bytes, F&& f) {
    hipEvent_t a = nullptr, b = nullptr;
    if (ctx->timing) {
      a = ev_get(ctx);
      b = ev_get(ctx);
      if (!a || !b) return fail(NPB_EDEVICE, "event creation failed");
      NPB_HIP(hipEventRecord(a, st));
    }
    hipError_t e = f();
    if (e != hipSuccess) return fail(NPB_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
    if (ctx->timing) {
      NPB_HIP(hipEventRecord(b, st));
      ctx->pending.push_back({cls, a, b, bytes});
    }
    return NPB_OK;
  }

  bool aos() const { return p->scheme == NPB_AOSIE1 || p->scheme == NPB_AOSIE2; }

  // coefficients of one run (Sec. 3: tau = dt / alpha; AOS sub-steps take
  // 4 tau; faces carry harmonic means of the nodal permittivities)
  struct Coefs {
    double tau, re[3], re_uniform, t, omt, t4, omt4;
    bool nl, vacuum;
  };
  Coefs coefs(const Run& r) const {
    Coefs c{};
    const double dt = p->dt / double(1 << r.level);
    c.vacuum = r.medium == 1;
    c.tau = dt / p->alpha;
    const double rc = (aos() ? 4.0 * c.tau : c.tau) / (g->h * g->h);
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

  static size_t pinned_need(int na) { return 256 + kTabBytes * 3 * kMaxFields + (size_t)5 * na * 8; }

  // atoms and chunk tables to the device through the context's pinned
  // staging buffer
  npb_status stage(const npb_molecule* mol) {
    const int na = mol->n_atoms;
    const size_t need = pinned_need(na);
    // the staging buffer is reused: wait for earlier copies out of it
    NPB_HIP(hipStreamSynchronize(st));
    if (ctx->pinned_bytes < need) {
      if (ctx->pinned) (void)hipHostFree(ctx->pinned);
      ctx->pinned = nullptr;
      ctx->pinned_bytes = 0;
      NPB_HIP(hipHostMalloc(&ctx->pinned, need, hipHostMallocDefault));
      ctx->pinned_bytes = need;
    }
    unsigned char* hb = reinterpret_cast<unsigned char*>(ctx->pinned);
    for (int r = 0; r < L.n_runs; ++r) {
      const Coefs c = coefs(L.runs[r]);
      for (int d = 0; d < 3; ++d) {
        ChunkTab<A>& tb = *reinterpret_cast<ChunkTab<A>*>(hb + 256 + kTabBytes * (3 * r + d));
        if (c.vacuum)
          fill_chunk_tab(tb, c.re_uniform, c.re_uniform, L.shape[d].M);
        else
          fill_chunk_tab(tb, c.re[0], c.re[2], L.shape[d].M);
      }
    }
    NPB_HIP(hipMemcpyAsync(ws + L.tabs, hb + 256, kTabBytes * 3 * L.n_runs, hipMemcpyHostToDevice,
                           st));
    if (na > 0) {
      double* h = reinterpret_cast<double*>(hb + 256 + kTabBytes * 3 * kMaxFields);
      for (int a = 0; a < na; ++a) {
        h[a] = mol->xyz[3 * a];
        h[na + a] = mol->xyz[3 * a + 1];
        h[2 * na + a] = mol->xyz[3 * a + 2];
        h[3 * na + a] = mol->q[a];
        h[4 * na + a] = mol->radius[a];
      }
      NPB_HIP(hipMemcpyAsync(ws + L.atoms, h, (size_t)5 * na * 8, hipMemcpyHostToDevice, st));
    }
    return NPB_OK;
  }

  npb_status setup(const npb_molecule* mol) {
    const int na = mol->n_atoms;
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const int nxp = pitch_of(nx, (int)sizeof(T));
    const size_t n = (size_t)nxp * ny * nz;
    sa = SetupArgs{nx, ny, nz, nxp, g->h, g->origin[0], g->origin[1], g->origin[2], na,
                   at<double>(L.atoms)};
    int* ints = at<int>(L.ints);  // [0] nq, [1] stencil error
    return timed(NPB_K_SETUP, 0, [&] {
      hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ints), 16, 0u, st);
      if (e != hipSuccess) return e;
      e = launch_fill_u32(reinterpret_cast<uint32_t*>(ws + L.mask), (n + 3) / 4, 0u, st);
      if (e != hipSuccess) return e;
      e = launch_mask_raster(sa, at<uint8_t>(L.mask), st);
      if (e != hipSuccess) return e;
      e = launch_stencil(sa, at<int>(L.key_a), at<int>(L.id_a), at<double>(L.sval), ints + 1, st);
      if (e != hipSuccess) return e;
      e = radix_sort_pairs(at<int>(L.key_a), at<int>(L.id_a), at<int>(L.key_b), at<int>(L.id_b),
                           at<int>(L.hist), L.cap, (long long)n, st);
      if (e != hipSuccess) return e;
      const double pref = 4.0 * M_PI * lB / (g->h * g->h * g->h);
      e = launch_merge_charges(at<int>(L.key_a), at<int>(L.id_a), at<double>(L.sval),
                               at<int>(L.heads), L.cap, ints, at<int>(L.q_idx),
                               at<double>(L.q_val), at<double>(L.q_rho), pref, st);
      if (e != hipSuccess) return e;
      e = launch_line_ptr(at<int>(L.q_idx), ints, L.cap, ny * nz, nxp, at<int>(L.xptr), st);
      if (e != hipSuccess) return e;
      if (needs_z_sources(p->scheme) && L.cap > 0) {
        for (int axis = needs_y_sources(p->scheme) ? 1 : 2; axis <= 2; ++axis) {
          e = launch_axis_keys(at<int>(L.q_idx), ints, L.cap, nx, nxp, ny, nz, axis,
                               at<int>(L.key_a), at<int>(L.id_a), st);
          if (e != hipSuccess) return e;
          e = radix_sort_pairs(at<int>(L.key_a), at<int>(L.id_a), at<int>(L.key_b),
                               at<int>(L.id_b), at<int>(L.hist), L.cap,
                               (long long)nx * ny * nz + 1, st);
          if (e != hipSuccess) return e;
          int* lin = at<int>(axis == 1 ? L.ylin : L.zlin);
          double* rho = at<double>(axis == 1 ? L.yrho : L.zrho);
          e = launch_gather_entries(at<int>(L.id_a), ints, L.cap, at<int>(L.q_idx),
                                    at<double>(L.q_rho), lin, rho, st);
          if (e != hipSuccess) return e;
          if (axis == 1)
            e = launch_line_ptr(at<int>(L.key_a), ints, L.cap, nz * nx, ny, at<int>(L.yptr), st);
          else
            e = launch_line_ptr(at<int>(L.key_a), ints, L.cap, ny * nx, nz, at<int>(L.zptr), st);
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
      const double kappa = std::sqrt(p->kappa_bar_sq / p->eps_out);
      e = launch_boundary(sa, p->eps_out, kappa, p->eps_in, lB, at<double>(L.bc_s),
                          p->vacuum ? at<double>(L.bc_v) : nullptr, sizeof(A) == 4, st);
      if (e != hipSuccess) return e;
      for (int d = 0; d < 3 && e == hipSuccess; ++d)
        e = launch_chunk_classes(at<uint8_t>(L.mask), nx, nxp, ny, nz, d, L.shape[d].M,
                                 L.shape[d].P, at<uint8_t>(L.ccls[d]), st);
      return e;
    });
  }

  // sweep arguments of run r in direction d (scheme-specific fused work:
  // Sec. 3.1 LODIE2 / LODIE1 orders, Sec. 3.2 AOS accumulation)
  SweepArgs<T> sweep_args(int r, int d) {
    const Coefs c = coefs(L.runs[r]);
    SweepArgs<T> a{};
    a.u = at<T>(L.field[r]);
    a.acc = aos() ? at<T>(L.acc[r]) : nullptr;
    a.mask = c.vacuum ? nullptr : at<uint8_t>(L.mask);
    a.nx = g->nx;
    a.ny = g->ny;
    a.nz = g->nz;
    a.nxp = pitch_of(g->nx, (int)sizeof(T));
    for (int k = 0; k < 3; ++k) a.re[k] = c.re[k];
    a.re_uniform = c.re_uniform;
    a.ccls = c.vacuum ? nullptr : at<uint8_t>(L.ccls[d]);
    a.tab = ws + L.tabs + kTabBytes * (3 * r + d);
    if (d == 0) {
      a.src_ptr = at<int>(L.xptr);
      a.src_lin = at<int>(L.q_idx);
      a.src_rho = at<double>(L.q_rho);
    } else {
      a.src_ptr = at<int>(d == 1 ? L.yptr : L.zptr);
      a.src_lin = at<int>(d == 1 ? L.ylin : L.zlin);
      a.src_rho = at<double>(d == 1 ? L.yrho : L.zrho);
    }
    if (p->scheme == NPB_LODIE2) {
      if (d == 0) {
        a.src_stage = 1;
        a.src_coef = c.tau;
      }
      if (d == 2 && c.nl) {
        a.post_nl = 1;
        a.post_ka = c.t;
        a.post_kb = c.omt;
      }
    } else if (p->scheme == NPB_LODIE1) {
      if (d == 0 && c.nl) {
        a.pre_nl = 1;
        a.pre_ka = c.t;
        a.pre_kb = c.omt;
      }
      if (d == 2) {
        a.src_stage = 2;
        a.src_coef = c.tau;
      }
    } else {
      const double cx = p->scheme == NPB_AOSIE2 ? 4.0 / 3.0 : 4.0;
      const double cyz = p->scheme == NPB_AOSIE2 ? 4.0 / 3.0 : 0.0;
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
    return a;
  }

  // All runs advance together: at step s the runs with more than s steps
  // (a prefix of the run list) are swept by one launch per direction.
  npb_status time_loop() {
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const int nxp = pitch_of(nx, (int)sizeof(T));
    const size_t n = (size_t)nxp * ny * nz;
    for (int r = 0; r < L.n_runs; ++r) {
      const bool vac = L.runs[r].medium == 1;
      npb_status s = timed(NPB_K_INIT, (double)n * sizeof(T), [&] {
        return launch_field_init<T>(at<T>(L.field[r]), at<double>(vac ? L.bc_v : L.bc_s), nx, nxp,
                                    ny, nz, st);
      });
      if (s != NPB_OK) return s;
    }
    if (L.shape[0].M == 0 || L.shape[1].M == 0 || L.shape[2].M == 0)
      return fail(NPB_EINVAL, "unsupported grid shape");
    SweepBatch<T> bx{}, by{}, bz{};
    int steps[kMaxFields];
    int max_steps = 0;
    double pbytes[3][kMaxFields];
    const double pts = (double)(nx - 2) * (ny - 2) * (nz - 2);
    for (int r = 0; r < L.n_runs; ++r) {
      bx.f[r] = sweep_args(r, 0);
      by.f[r] = sweep_args(r, 1);
      bz.f[r] = sweep_args(r, 2);
      steps[r] = p->n_steps << L.runs[r].level;
      if (steps[r] > max_steps) max_steps = steps[r];
      // algorithmic bytes per sweep: field read + write (+ mask) (+ accumulator)
      const double mb = L.runs[r].medium == 1 ? 0.0 : 1.0;
      const double ab = aos() ? sizeof(T) : 0.0;
      pbytes[0][r] = pts * (2.0 * sizeof(T) + mb + ab);
      pbytes[1][r] = pts * (2.0 * sizeof(T) + mb + 2.0 * ab);
      pbytes[2][r] = pts * (2.0 * sizeof(T) + mb + ab);
    }
    for (int step = 0; step < max_steps; ++step) {
      int nf = 0;
      double b3[3] = {0, 0, 0};
      while (nf < L.n_runs && steps[nf] > step) {
        for (int d = 0; d < 3; ++d) b3[d] += pbytes[d][nf];
        ++nf;
      }
      npb_status s;
      s = timed(NPB_K_SWEEP_X, b3[0], [&] { return launch_sweep_x<T, A>(bx, nf, L.shape[0], st); });
      if (s != NPB_OK) return s;
      s = timed(NPB_K_SWEEP_Y, b3[1],
                [&] { return launch_sweep_yz<T, A>(by, nf, 1, L.shape[1], st); });
      if (s != NPB_OK) return s;
      s = timed(NPB_K_SWEEP_Z, b3[2],
                [&] { return launch_sweep_yz<T, A>(bz, nf, 2, L.shape[2], st); });
      if (s != NPB_OK) return s;
    }
    return NPB_OK;
  }

  npb_status energy(int r) {
    const int slot = 2 * L.runs[r].medium + L.runs[r].level;
    return timed(NPB_K_ENERGY, 0, [&] {
      return launch_energy<T>(at<T>(L.field[r]), at<int>(L.q_idx), at<double>(L.q_val),
                              at<int>(L.ints), L.cap, at<double>(L.slots) + slot, st);
    });
  }

  // The device work of a solve after staging, all on `st` (captured into a
  // graph when replay is on): setup, time loops, energies, optional field,
  // combinations.  Launches only: no allocation, copy or synchronisation.
  npb_status device_work(const npb_molecule* mol, double* d_field_out) {
    npb_status s = setup(mol);
    if (s != NPB_OK) return s;
    // zero the energy slots
    s = timed(NPB_K_OTHER, 0, [&] {
      return launch_fill_u32(reinterpret_cast<uint32_t*>(ws + L.slots), 64, 0u, st);
    });
    if (s != NPB_OK) return s;
    s = time_loop();
    if (s != NPB_OK) return s;
    for (int r = 0; r < L.n_runs; ++r) {
      s = energy(r);
      if (s != NPB_OK) return s;
    }
    if (d_field_out) {
      // selected medium: kT u (plain) or kT (2 u(dt/2) - u(dt)) (Richardson)
      for (int l = 0; l < (p->richardson ? 2 : 1); ++l) {
        int r = 0;
        while (!(L.runs[r].medium == p->field_select && L.runs[r].level == l)) ++r;
        const double beta = (l == 0) ? 0.0 : 1.0;
        const double gamma = p->richardson ? (l == 0 ? -kT : 2.0 * kT) : kT;
        s = timed(NPB_K_OTHER, 0, [&] {
          return launch_field_out<T>(d_field_out, at<T>(L.field[r]), g->nx,
                                     pitch_of(g->nx, (int)sizeof(T)), g->ny, g->nz, beta, gamma,
                                     st);
        });
        if (s != NPB_OK) return s;
      }
    }
    return timed(NPB_K_OTHER, 0, [&] {
      return launch_combine(at<double>(L.slots), kT, p->richardson, p->vacuum,
                            at<double>(L.slots) + 8, st);
    });
  }
};

template <typename T, typename A>
npb_status solve_t(npb_ctx* ctx, const npb_molecule* mol, const npb_grid* g,
                   const npb_params* p, void* d_ws, double* d_field_out, hipStream_t st,
                   npb_result* out, const Layout& L) {
  Solver<T, A> S{ctx, g, p, st, reinterpret_cast<unsigned char*>(d_ws), L, {}, 0.0, 0.0};
  S.kT = thermal_energy(p->temperature_K);
  S.lB = bjerrum(p->temperature_K);
  npb_status s = S.stage(mol);
  if (s != NPB_OK) return s;
  NPB_HIP(hipEventRecord(ctx->t0, st));
  if (ctx->graphs && !ctx->timing) {
    GraphKey k;
    std::memset(&k, 0, sizeof(k));
    k.ws = d_ws;
    k.field_out = d_field_out;
    k.pinned = ctx->pinned;
    k.grid = *g;
    k.params = *p;
    k.n_atoms = mol->n_atoms;
    if (!ctx->exec || std::memcmp(&k, &ctx->key, sizeof(k)) != 0) {
      if (ctx->exec) (void)hipGraphExecDestroy(ctx->exec);
      ctx->exec = nullptr;
      S.st = ctx->capture;
      NPB_HIP(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
      s = S.device_work(mol, d_field_out);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(ctx->capture, &graph);
      S.st = st;
      if (s != NPB_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
      }
      if (e != hipSuccess) return fail(NPB_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&ctx->exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        ctx->exec = nullptr;
        return fail(NPB_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
      }
      ctx->key = k;
    }
    NPB_HIP(hipGraphLaunch(ctx->exec, st));
  } else {
    s = S.device_work(mol, d_field_out);
    if (s != NPB_OK) return s;
  }
  int steps_done = 0;
  double gpu_updates = 0.0;
  const double pts = (double)(g->nx - 2) * (g->ny - 2) * (g->nz - 2);
  for (int r = 0; r < L.n_runs; ++r) {
    const int ns = p->n_steps << L.runs[r].level;
    steps_done += ns;
    gpu_updates += pts * ns;
  }
  NPB_HIP(hipEventRecord(ctx->t1, st));
  // results to the host (first 256 bytes of the staging buffer)
  double* hres = reinterpret_cast<double*>(ctx->pinned);
  NPB_HIP(hipMemcpyAsync(hres, S.ws + L.slots + 8 * 8, 8 * 8, hipMemcpyDeviceToHost, st));
  NPB_HIP(hipMemcpyAsync(reinterpret_cast<unsigned char*>(hres) + 64, S.ws + L.ints, 8,
                         hipMemcpyDeviceToHost, st));
  NPB_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  NPB_HIP(hipEventElapsedTime(&ms, ctx->t0, ctx->t1));
  if (ctx->timing) harvest(ctx);
  const int* hints = reinterpret_cast<const int*>(reinterpret_cast<unsigned char*>(hres) + 64);
  std::memset(out, 0, sizeof(*out));
  out->dG = hres[0];
  out->dG_plain = hres[1];
  out->G_m[0] = hres[2];
  out->G_m[1] = hres[3];
  out->G_0[0] = hres[4];
  out->G_0[1] = hres[5];
  out->finite = hres[6] != 0.0 ? 1 : 0;
  out->grid_point_updates = gpu_updates;
  out->device_ms = ms;
  out->steps_done = steps_done;
  out->n_charge_nodes = hints[0];
  if (hints[1] != 0) return fail(NPB_ERANGE, "a trilinear stencil touches the boundary");
  if (!out->finite) return fail(NPB_EDIVERGED, "non-finite energy");
  return NPB_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

int npb_abi_version(void) { return NPB_ABI_VERSION; }

const char* npb_last_error(void) { return g_err.c_str(); }

double npb_kappa_bar_sq(double ionic_molar, double temperature_K) {
  return kKbar2PerMolar298 * (298.0 / temperature_K) * ionic_molar;
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
  if (hipEventCreate(&c->t0) != hipSuccess || hipEventCreate(&c->t1) != hipSuccess ||
      hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking) != hipSuccess) {
    if (c->t0) (void)hipEventDestroy(c->t0);
    if (c->t1) (void)hipEventDestroy(c->t1);
    delete c;
    return fail(NPB_EDEVICE, "event or stream creation failed");
  }
  *out = c;
  return NPB_OK;
}

void npb_ctx_destroy(npb_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->t0) (void)hipEventDestroy(c->t0);
  if (c->t1) (void)hipEventDestroy(c->t1);
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->capture) (void)hipStreamDestroy(c->capture);
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
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

npb_status npb_solve(npb_ctx* ctx, const npb_molecule* mol, const npb_grid* grid,
                     const npb_params* params, void* d_ws, size_t ws_bytes, double* d_field_out,
                     void* stream, npb_result* out) {
  if (!ctx || !out) return fail(NPB_EINVAL, "null context or result");
  npb_status s = validate(mol, grid, params);
  if (s != NPB_OK) return s;
  const Layout L = make_layout(mol, grid, params);
  if (!d_ws || ws_bytes < L.total)
    return fail(NPB_EINVAL, "workspace missing or smaller than npb_workspace_bytes");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0)
    return fail(NPB_EINVAL, "workspace must be 256-byte aligned");
  NPB_HIP(hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  try {
    if (params->precision == NPB_FP64)
      return solve_t<double, double>(ctx, mol, grid, params, d_ws, d_field_out, st, out, L);
    if (params->precision == NPB_FP32X)
      return solve_t<float, double>(ctx, mol, grid, params, d_ws, d_field_out, st, out, L);
    return solve_t<float, float>(ctx, mol, grid, params, d_ws, d_field_out, st, out, L);
  } catch (const std::exception& e) {
    return fail(NPB_ENOMEM, e.what());
  } catch (...) {
    return fail(NPB_EDEVICE, "unexpected failure");
  }
}

}  // extern "C"
