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

template <typename T>
__global__ void field_init_kernel(T* u, const double* bc, int nx, int ny, int nz) {
  const long long n = (long long)nx * ny * nz;
  const long long nxy = (long long)nx * ny;
  const long long ring = 2LL * nx + 2LL * (ny - 2);
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    int i = (int)(p % nx);
    long long t = p / nx;
    int j = (int)(t % ny);
    int k = (int)(t / ny);
    T v = T(0);
    if (k == 0) {
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
hipError_t launch_field_init(T* u, const double* bc, int nx, int ny, int nz, hipStream_t st) {
  long long n = (long long)nx * ny * nz;
  long long blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL((field_init_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, st, u, bc, nx,
                     ny, nz);
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
__global__ void field_out_kernel(double* out, const T* u, long long n, double beta, double gamma) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double v = gamma * (double)u[i];
    out[i] = (beta != 0.0) ? beta * out[i] + v : v;
  }
}

template <typename T>
hipError_t launch_field_out(double* out, const T* u, size_t n, double beta, double gamma,
                            hipStream_t st) {
  long long blocks = ((long long)n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL((field_out_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, st, out, u,
                     (long long)n, beta, gamma);
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

template hipError_t launch_field_init<float>(float*, const double*, int, int, int, hipStream_t);
template hipError_t launch_field_init<double>(double*, const double*, int, int, int, hipStream_t);

}  // namespace npb

// ---------------------------------------------------------------------------
// context

struct npb_ctx {
  int device = 0;
  bool timing = false;
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

struct Layout {
  size_t field, acc, mask, bc_s, bc_v, atoms, key_a, id_a, key_b, id_b, sval, hist, heads;
  size_t q_idx, q_val, q_rho, xptr, yptr, ylin, yrho, zptr, zlin, zrho, ccls[3], slots, ints, total;
  LaunchShape shape[3];
  int cap, nblocks;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

bool needs_yz_sources(int scheme) { return scheme == NPB_LODIE1 || scheme == NPB_AOSIE2; }

Layout make_layout(const npb_molecule* mol, const npb_grid* g, const npb_params* p) {
  Layout L{};
  const size_t n = (size_t)g->nx * g->ny * g->nz;
  const size_t es = p->precision == NPB_FP64 ? 8 : 4;
  const int na = mol->n_atoms;
  const int cap = 8 * na;
  const int nb = (cap + 255) / 256;
  const size_t ns = (size_t)shell_count(g->nx, g->ny, g->nz);
  const bool aos = p->scheme == NPB_AOSIE1 || p->scheme == NPB_AOSIE2;
  const bool yz = needs_yz_sources(p->scheme);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  L.field = take(n * es);
  L.acc = take(aos ? n * es : 0);
  L.mask = take(n);
  L.bc_s = take(ns * 8);
  L.bc_v = take(p->vacuum ? ns * 8 : 0);
  L.atoms = take((size_t)5 * na * 8);
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
  L.yptr = take(yz ? ((size_t)g->nz * g->nx + 1) * 4 : 0);
  L.ylin = take(yz ? (size_t)cap * 4 : 0);
  L.yrho = take(yz ? (size_t)cap * 8 : 0);
  L.zptr = take(yz ? ((size_t)g->ny * g->nx + 1) * 4 : 0);
  L.zlin = take(yz ? (size_t)cap * 4 : 0);
  L.zrho = take(yz ? (size_t)cap * 8 : 0);
  {
    const bool f64a = p->precision != NPB_FP32;
    L.shape[0] = plan_x(g->nx, g->ny, g->nz, f64a, aos, false);
    L.shape[1] = plan_yz(g->ny, (g->nx - 2) * (g->nz - 2), f64a);
    L.shape[2] = plan_yz(g->nz, (g->nx - 2) * (g->ny - 2), f64a);
    const size_t nl[3] = {(size_t)(g->ny - 2) * (g->nz - 2), (size_t)(g->nx - 2) * (g->nz - 2),
                          (size_t)(g->nx - 2) * (g->ny - 2)};
    for (int d = 0; d < 3; ++d) L.ccls[d] = take(nl[d] * (size_t)(L.shape[d].P > 0 ? L.shape[d].P : 1));
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

  npb_status setup(const npb_molecule* mol) {
    const int na = mol->n_atoms;
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t n = (size_t)nx * ny * nz;
    // atoms as [x][y][z][q][R] planes, through pinned staging
    const size_t abytes = (size_t)5 * na * 8;
    if (na > 0) {
      if (ctx->pinned_bytes < abytes + 256) {
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        ctx->pinned = nullptr;
        ctx->pinned_bytes = 0;
        NPB_HIP(hipHostMalloc(&ctx->pinned, abytes + 256, hipHostMallocDefault));
        ctx->pinned_bytes = abytes + 256;
      }
      // the staging buffer is reused: wait for earlier copies out of it
      NPB_HIP(hipStreamSynchronize(st));
      double* h = reinterpret_cast<double*>(ctx->pinned);
      for (int a = 0; a < na; ++a) {
        h[a] = mol->xyz[3 * a];
        h[na + a] = mol->xyz[3 * a + 1];
        h[2 * na + a] = mol->xyz[3 * a + 2];
        h[3 * na + a] = mol->q[a];
        h[4 * na + a] = mol->radius[a];
      }
      NPB_HIP(hipMemcpyAsync(ws + L.atoms, h, abytes, hipMemcpyHostToDevice, st));
    }
    sa = SetupArgs{nx, ny, nz, g->h, g->origin[0], g->origin[1], g->origin[2], na,
                   at<double>(L.atoms)};
    int* ints = at<int>(L.ints);  // [0] nq, [1] stencil error
    npb_status s;
    s = timed(NPB_K_SETUP, 0, [&] {
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
      e = launch_line_ptr(at<int>(L.q_idx), ints, L.cap, ny * nz, nx, at<int>(L.xptr), st);
      if (e != hipSuccess) return e;
      if (needs_yz_sources(p->scheme) && L.cap > 0) {
        for (int axis = 1; axis <= 2; ++axis) {
          e = launch_axis_keys(at<int>(L.q_idx), ints, L.cap, nx, ny, nz, axis, at<int>(L.key_a),
                               at<int>(L.id_a), st);
          if (e != hipSuccess) return e;
          e = radix_sort_pairs(at<int>(L.key_a), at<int>(L.id_a), at<int>(L.key_b),
                               at<int>(L.id_b), at<int>(L.hist), L.cap, (long long)n + 1, st);
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
      } else if (needs_yz_sources(p->scheme)) {
        e = launch_fill_u32(reinterpret_cast<uint32_t*>(ws + L.yptr), (size_t)nz * nx + 1, 0u, st);
        if (e != hipSuccess) return e;
        e = launch_fill_u32(reinterpret_cast<uint32_t*>(ws + L.zptr), (size_t)ny * nx + 1, 0u, st);
        if (e != hipSuccess) return e;
      }
      const double kappa = std::sqrt(p->kappa_bar_sq / p->eps_out);
      e = launch_boundary(sa, p->eps_out, kappa, lB, at<double>(L.bc_s), st);
      if (e != hipSuccess) return e;
      if (p->vacuum) e = launch_boundary(sa, p->eps_in, 0.0, lB, at<double>(L.bc_v), st);
      if (e != hipSuccess) return e;
      for (int d = 0; d < 3 && e == hipSuccess; ++d)
        e = launch_chunk_classes(at<uint8_t>(L.mask), nx, ny, nz, d, L.shape[d].M, L.shape[d].P,
                                 at<uint8_t>(L.ccls[d]), st);
      return e;
    });
    return s;
  }

  // one time loop of one medium at one step size
  npb_status loop(bool vacuum, double dt, int n_steps) {
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t n = (size_t)nx * ny * nz;
    const double tau = dt / p->alpha;
    const bool aos = p->scheme == NPB_AOSIE1 || p->scheme == NPB_AOSIE2;
    const double r = (aos ? 4.0 * tau : tau) / (g->h * g->h);
    const double ein = p->eps_in, eout = p->eps_out;
    const double emix = 2.0 * ein * eout / (ein + eout);
    const double eout_f = 2.0 * eout * eout / (eout + eout);
    const double ein_f = 2.0 * ein * ein / (ein + ein);
    T* u = at<T>(L.field);
    const double kb2 = vacuum ? 0.0 : p->kappa_bar_sq;

    SweepArgs<T> a{};
    a.u = u;
    a.acc = aos ? at<T>(L.acc) : nullptr;
    a.mask = vacuum ? nullptr : at<uint8_t>(L.mask);
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.re[0] = r * eout_f;
    a.re[1] = r * emix;
    a.re[2] = r * ein_f;
    a.re_uniform = r * ein_f;
    double t, omt;
    flow_params(kb2 * dt / (2.0 * p->alpha), t, omt);
    double t4, omt4;
    flow_params(4.0 * kb2 * dt / (2.0 * p->alpha), t4, omt4);
    const bool nl = kb2 > 0.0 && !vacuum;

    npb_status s = timed(NPB_K_INIT, (double)n * sizeof(T), [&] {
      return launch_field_init<T>(u, at<double>(vacuum ? L.bc_v : L.bc_s), nx, ny, nz, st);
    });
    if (s != NPB_OK) return s;

    // the solvated launch shapes are the ones the chunk classes were built for
    const LaunchShape sx = vacuum ? plan_x(nx, ny, nz, sizeof(A) == 8, aos, true) : L.shape[0];
    const LaunchShape sy = L.shape[1];
    const LaunchShape sz = L.shape[2];
    if (sx.M == 0 || sy.M == 0 || sz.M == 0) return fail(NPB_EINVAL, "unsupported grid shape");
    const double pts = (double)(nx - 2) * (ny - 2) * (nz - 2);
    const double mb = vacuum ? 0.0 : 1.0;
    // algorithmic bytes per sweep: field read + write (+ mask) (+ accumulator)
    const double bx = pts * (2.0 * sizeof(T) + mb + (aos ? sizeof(T) : 0.0));
    const double by = pts * (2.0 * sizeof(T) + mb + (aos ? 2.0 * sizeof(T) : 0.0));
    const double bz = pts * (2.0 * sizeof(T) + mb + (aos ? sizeof(T) : 0.0));

    const int* ints = at<int>(L.ints);
    (void)ints;
    for (int step = 0; step < n_steps; ++step) {
      SweepArgs<T> ax = a, ay = a, az = a;
      ax.ccls = vacuum ? nullptr : at<uint8_t>(L.ccls[0]);
      ay.ccls = vacuum ? nullptr : at<uint8_t>(L.ccls[1]);
      az.ccls = vacuum ? nullptr : at<uint8_t>(L.ccls[2]);
      ax.src_ptr = at<int>(L.xptr);
      ax.src_lin = at<int>(L.q_idx);
      ax.src_rho = at<double>(L.q_rho);
      ay.src_ptr = at<int>(L.yptr);
      ay.src_lin = at<int>(L.ylin);
      ay.src_rho = at<double>(L.yrho);
      az.src_ptr = at<int>(L.zptr);
      az.src_lin = at<int>(L.zlin);
      az.src_rho = at<double>(L.zrho);
      if (p->scheme == NPB_LODIE2) {
        ax.src_stage = 1;
        ax.src_coef = tau;
        if (nl) {
          az.post_nl = 1;
          az.post_ka = t;
          az.post_kb = omt;
        }
      } else if (p->scheme == NPB_LODIE1) {
        if (nl) {
          ax.pre_nl = 1;
          ax.pre_ka = t;
          ax.pre_kb = omt;
        }
        az.src_stage = 2;
        az.src_coef = tau;
      } else {
        const double cx = p->scheme == NPB_AOSIE2 ? 4.0 / 3.0 : 4.0;
        const double cyz = p->scheme == NPB_AOSIE2 ? 4.0 / 3.0 : 0.0;
        ax.mode = MODE_AOS_FIRST;
        ax.aos_w = nl ? 1 : 0;
        ax.aos_ka = t4;
        ax.aos_kb = omt4;
        ax.src_stage = 1;
        ax.src_coef = cx * tau;
        ay.mode = MODE_AOS_ADD;
        az.mode = MODE_AOS_FINISH;
        if (cyz != 0.0) {
          ay.src_stage = 1;
          ay.src_coef = cyz * tau;
          az.src_stage = 1;
          az.src_coef = cyz * tau;
        }
      }
      s = timed(NPB_K_SWEEP_X, bx, [&] { return launch_sweep_x<T, A>(ax, sx, st); });
      if (s != NPB_OK) return s;
      s = timed(NPB_K_SWEEP_Y, by, [&] { return launch_sweep_yz<T, A>(ay, 1, sy, st); });
      if (s != NPB_OK) return s;
      s = timed(NPB_K_SWEEP_Z, bz, [&] { return launch_sweep_yz<T, A>(az, 2, sz, st); });
      if (s != NPB_OK) return s;
    }
    return NPB_OK;
  }

  npb_status energy(int slot_index) {
    return timed(NPB_K_ENERGY, 0, [&] {
      return launch_energy<T>(at<T>(L.field), at<int>(L.q_idx), at<double>(L.q_val),
                              at<int>(L.ints), L.cap, at<double>(L.slots) + slot_index, st);
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
  const size_t n = (size_t)g->nx * g->ny * g->nz;
  NPB_HIP(hipEventRecord(ctx->t0, st));
  npb_status s = S.setup(mol);
  if (s != NPB_OK) return s;
  // zero the energy slots
  s = S.timed(NPB_K_OTHER, 0, [&] {
    return launch_fill_u32(reinterpret_cast<uint32_t*>(S.ws + L.slots), 64, 0u, st);
  });
  if (s != NPB_OK) return s;
  const int levels = p->richardson ? 2 : 1;
  const int media = p->vacuum ? 2 : 1;
  int steps_done = 0;
  double gpu_updates = 0.0;
  const double pts = (double)(g->nx - 2) * (g->ny - 2) * (g->nz - 2);
  for (int m = 0; m < media; ++m) {
    const bool vac = (m == 1);
    for (int l = 0; l < levels; ++l) {
      const double dt = (l == 0) ? p->dt : p->dt / 2.0;
      const int ns = p->n_steps << l;
      s = S.loop(vac, dt, ns);
      if (s != NPB_OK) return s;
      steps_done += ns;
      gpu_updates += pts * ns;
      s = S.energy(2 * m + l);
      if (s != NPB_OK) return s;
      if (d_field_out && p->field_select == m) {
        double beta = (l == 0) ? 0.0 : 1.0;
        double gamma = p->richardson ? (l == 0 ? -S.kT : 2.0 * S.kT) : S.kT;
        s = S.timed(NPB_K_OTHER, 0, [&] {
          return launch_field_out<T>(d_field_out, S.template at<T>(L.field), n, beta, gamma, st);
        });
        if (s != NPB_OK) return s;
      }
    }
  }
  s = S.timed(NPB_K_OTHER, 0, [&] {
    return launch_combine(S.template at<double>(L.slots), S.kT, p->richardson, p->vacuum,
                          S.template at<double>(L.slots) + 8, st);
  });
  if (s != NPB_OK) return s;
  NPB_HIP(hipEventRecord(ctx->t1, st));
  // results to the host
  double* hres = reinterpret_cast<double*>(ctx->pinned);
  if (!hres || ctx->pinned_bytes < 256) {
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    NPB_HIP(hipStreamSynchronize(st));
    NPB_HIP(hipHostMalloc(&ctx->pinned, 256, hipHostMallocDefault));
    ctx->pinned_bytes = 256;
    hres = reinterpret_cast<double*>(ctx->pinned);
  }
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
  if (hipEventCreate(&c->t0) != hipSuccess || hipEventCreate(&c->t1) != hipSuccess) {
    delete c;
    return fail(NPB_EDEVICE, "event creation failed");
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
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
}

npb_status npb_ctx_set_timing(npb_ctx* c, int enable) {
  if (!c) return fail(NPB_EINVAL, "null context");
  c->timing = enable != 0;
  if (c->timing) std::memset(&c->times, 0, sizeof(c->times));
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
