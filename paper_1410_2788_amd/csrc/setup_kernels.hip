// Per-solve setup on the device: solute mask, trilinear charges, source
// density, per-line source lists and Dirichlet boundary data.
//
// All of it is deterministic: the charge at a node is summed in atom order
// (a stable sort of the 8 N_a stencil entries by node), so repeated solves
// give bit-identical inputs to the time loop.  FP64 throughout; expression
// order follows the definitions so that contraction into fused
// multiply-adds is switched off where a predicate or a weight is formed.
#include "npb_internal.h"

namespace npb {

__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t step = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += step) p[i] = v;
}

__global__ void copy_u32_kernel(const uint32_t* src, uint32_t* dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

hipError_t launch_copy_u32(const uint32_t* src, uint32_t* dst, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(copy_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// Solute region = union of atomic balls, a node on a sphere counts as
// solute (Sec. 2.1: eps_m on/inside the surface).  One block per atom walks
// the atom's bounding box of nodes.
__global__ __launch_bounds__(256) void mask_raster_kernel(SetupArgs a, uint8_t* mask) {
#pragma clang fp contract(off)
  const int at = blockIdx.x;
  const int na = a.n_atoms;
  const double c[3] = {a.atoms[at], a.atoms[na + at], a.atoms[2 * na + at]};
  const double R = a.atoms[4 * na + at];
  const double o[3] = {a.ox, a.oy, a.oz};
  const int n[3] = {a.nx, a.ny, a.nz};
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = (int)floor((c[d] - R - o[d]) / a.h) - 1;
    hi[d] = (int)ceil((c[d] + R - o[d]) / a.h) + 1;
    if (lo[d] < 0) lo[d] = 0;
    if (hi[d] > n[d] - 1) hi[d] = n[d] - 1;
    if (lo[d] > hi[d]) return;
  }
  const int bx = hi[0] - lo[0] + 1, by = hi[1] - lo[1] + 1, bz = hi[2] - lo[2] + 1;
  const long long tot = (long long)bx * by * bz;
  const double R2 = R * R;
  for (long long e = threadIdx.x; e < tot; e += blockDim.x) {
    int i = lo[0] + (int)(e % bx);
    int j = lo[1] + (int)((e / bx) % by);
    int k = lo[2] + (int)(e / ((long long)bx * by));
    double X = (double)i * a.h;
    X = a.ox + X;
    double Y = (double)j * a.h;
    Y = a.oy + Y;
    double Z = (double)k * a.h;
    Z = a.oz + Z;
    double dx = X - c[0], dy = Y - c[1], dz = Z - c[2];
    double d2 = dx * dx + dy * dy;
    d2 = d2 + dz * dz;
    if (d2 <= R2) mask[((long long)k * a.ny + j) * a.nxp + i] = 1;
  }
}

// Face rule by location (Sec. 3.1, text after Eq. (SpatialOperators)):
// the half point between node g and its successor along `dir` takes
// eps_in when it lies on or inside a sphere.  fmask already holds the
// solute mask; every such half point sets bit 1 of node g's byte there
// (each writer stores the same value, mask | 2).  Coordinates and distance
// are evaluated as in the node raster, with the half point at
// origin + (i + 1/2) h along `dir`.
__global__ __launch_bounds__(256) void face_raster_kernel(SetupArgs a, int dir, const uint8_t* mask,
                                                          uint8_t* fmask) {
#pragma clang fp contract(off)
  const int at = blockIdx.x;
  const int na = a.n_atoms;
  const double c[3] = {a.atoms[at], a.atoms[na + at], a.atoms[2 * na + at]};
  const double R = a.atoms[4 * na + at];
  const double o[3] = {a.ox, a.oy, a.oz};
  int n[3] = {a.nx, a.ny, a.nz};
  n[dir] -= 1;  // half points along dir: 0 .. n_dir - 2
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = (int)floor((c[d] - R - o[d]) / a.h) - 1;
    hi[d] = (int)ceil((c[d] + R - o[d]) / a.h) + 1;
    if (lo[d] < 0) lo[d] = 0;
    if (hi[d] > n[d] - 1) hi[d] = n[d] - 1;
    if (lo[d] > hi[d]) return;
  }
  const int bx = hi[0] - lo[0] + 1, by = hi[1] - lo[1] + 1, bz = hi[2] - lo[2] + 1;
  const long long tot = (long long)bx * by * bz;
  const double R2 = R * R;
  for (long long e = threadIdx.x; e < tot; e += blockDim.x) {
    const int idx[3] = {lo[0] + (int)(e % bx), lo[1] + (int)((e / bx) % by),
                        lo[2] + (int)(e / ((long long)bx * by))};
    double p[3];
    for (int d = 0; d < 3; ++d) {
      double t = d == dir ? ((double)idx[d] + 0.5) * a.h : (double)idx[d] * a.h;
      p[d] = o[d] + t;
    }
    double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
    double d2 = dx * dx + dy * dy;
    d2 = d2 + dz * dz;
    if (d2 <= R2) {
      const long long g = ((long long)idx[2] * a.ny + idx[1]) * a.nxp + idx[0];
      fmask[g] = (uint8_t)(mask[g] | 2u);
    }
  }
}

hipError_t launch_face_raster(const SetupArgs& a, int dir, const uint8_t* mask, uint8_t* fmask,
                              hipStream_t st) {
  if (a.n_atoms <= 0) return hipSuccess;
  hipLaunchKernelGGL(face_raster_kernel, dim3(a.n_atoms), dim3(256), 0, st, a, dir, mask, fmask);
  return hipGetLastError();
}

hipError_t launch_mask_raster(const SetupArgs& a, uint8_t* mask, hipStream_t st) {
  if (a.n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(mask_raster_kernel, dim3(a.n_atoms), dim3(256), 0, st, a, mask);
  return hipGetLastError();
}

// Trilinear stencil of each atom (Sec. 3.1: Q by trilinear interpolation):
// g = (r - origin)/h, i0 = floor(g), f = g - i0; corner weights w = f or
// 1 - f per axis, product in x, y, z order; entry value q * w.
__global__ void stencil_kernel(SetupArgs a, int* key, int* id, double* val, int* err) {
#pragma clang fp contract(off)
  const int at = blockIdx.x * blockDim.x + threadIdx.x;
  const int na = a.n_atoms;
  if (at >= na) return;
  const double o[3] = {a.ox, a.oy, a.oz};
  const int n[3] = {a.nx, a.ny, a.nz};
  int i0[3];
  double f[3];
  bool bad = false;
  for (int d = 0; d < 3; ++d) {
    double g = (a.atoms[d * na + at] - o[d]) / a.h;
    double fl = floor(g);
    i0[d] = (int)fl;
    f[d] = g - fl;
    if (i0[d] < 1 || i0[d] + 1 > n[d] - 2) bad = true;
  }
  if (bad) {
    atomicOr(err, 1);
    for (int c = 0; c < 8; ++c) {
      key[8 * at + c] = 0;
      id[8 * at + c] = 8 * at + c;
      val[8 * at + c] = 0.0;
    }
    return;
  }
  const double q = a.atoms[3 * na + at];
  for (int cz = 0; cz < 2; ++cz) {
    double wz = cz ? f[2] : 1.0 - f[2];
    for (int cy = 0; cy < 2; ++cy) {
      double wy = cy ? f[1] : 1.0 - f[1];
      for (int cx = 0; cx < 2; ++cx) {
        double wx = cx ? f[0] : 1.0 - f[0];
        double w = wx * wy;
        w = w * wz;
        int c = cz * 4 + cy * 2 + cx;
        key[8 * at + c] = ((i0[2] + cz) * a.ny + (i0[1] + cy)) * a.nxp + (i0[0] + cx);
        id[8 * at + c] = 8 * at + c;
        val[8 * at + c] = q * w;
      }
    }
  }
}

hipError_t launch_stencil(const SetupArgs& a, int* key, int* id, double* val, int* err,
                          hipStream_t st) {
  if (a.n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(stencil_kernel, dim3((a.n_atoms + 127) / 128), dim3(128), 0, st, a, key,
                     id, val, err);
  return hipGetLastError();
}

// Caller-given dense source (npb_solve_fields): one list entry per interior
// node, in node order, key = pitched linear index, value = rho.
__global__ void dense_source_kernel(const double* rho, int nx, int nxp, int ny, int nz, int* key,
                                    int* id, double* val) {
  const int X = nx - 2, Y = ny - 2;
  const long long n = (long long)X * Y * (nz - 2);
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const int i = 1 + (int)(c % X);
    const long long t = c / X;
    const int j = 1 + (int)(t % Y);
    const int k = 1 + (int)(t / Y);
    key[c] = (k * ny + j) * nxp + i;
    id[c] = (int)c;
    val[c] = rho[((long long)k * ny + j) * nx + i];
  }
}

hipError_t launch_dense_source(const double* rho, int nx, int nxp, int ny, int nz, int* key,
                               int* id, double* val, hipStream_t st) {
  const long long n = (long long)(nx - 2) * (ny - 2) * (nz - 2);
  long long blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(dense_source_kernel, dim3((unsigned)blocks), dim3(256), 0, st, rho, nx, nxp,
                     ny, nz, key, id, val);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits, 256 items per block

__global__ __launch_bounds__(256) void radix_count_kernel(const int* key, int n, int shift,
                                                          int nblocks, int* hist) {
  __shared__ int h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  int i = blockIdx.x * 256 + tid;
  if (i < n) atomicAdd(&h[(key[i] >> shift) & 255], 1);
  __syncthreads();
  hist[tid * nblocks + blockIdx.x] = h[tid];
}

__global__ __launch_bounds__(256) void radix_scatter_kernel(const int* kin, const int* iin,
                                                            int* kout, int* iout, int n,
                                                            int shift, int nblocks,
                                                            const int* hist) {
  __shared__ int dg[256];
  const int tid = threadIdx.x;
  const int i = blockIdx.x * 256 + tid;
  int k = 0, id = 0, d = 256;
  if (i < n) {
    k = kin[i];
    id = iin[i];
    d = (k >> shift) & 255;
  }
  dg[tid] = d;
  __syncthreads();
  if (i < n) {
    int r = 0;
    for (int j = 0; j < tid; ++j) r += (dg[j] == d);
    int pos = hist[d * nblocks + blockIdx.x] + r;
    kout[pos] = k;
    iout[pos] = id;
  }
}

// Exclusive prefix sum of n ints by one block of 1024 threads, tile by
// tile (kScanTile entries staged in LDS by coalesced loads and stores, with
// one padding word per 32 entries so that the per-thread walks over
// consecutive entries fall in distinct banks), carrying the running total
// from tile to tile.  The total goes to *total if given.
constexpr int kScanTile = 32768;
__host__ __device__ inline int scan_pad(int i) { return i + (i >> 5); }

__global__ __launch_bounds__(1024) void scan_lds_kernel(int* data, int n, int tile, int* total) {
  extern __shared__ int buf[];
  __shared__ int wtot[16];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  int carry = 0;
  for (int base = 0; base < n; base += tile) {
    const int m = min(tile, n - base);
    for (int i = tid; i < m; i += 1024) buf[scan_pad(i)] = data[base + i];
    __syncthreads();
    const int per = (m + 1023) / 1024;
    const int b = tid * per;
    const int e = min(b + per, m);
    int s = 0;
    for (int i = b; i < e; ++i) s += buf[scan_pad(i)];
    // inclusive scan of the per-thread sums: within each wave by shuffles,
    // then over the 16 wave totals
    int inc = s;
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(inc, off, 64);
      if (lane >= off) inc += v;
    }
    if (lane == 63) wtot[w] = inc;
    __syncthreads();
    if (w == 0) {
      int t = lane < 16 ? wtot[lane] : 0;
      for (int off = 1; off < 16; off <<= 1) {
        const int v = __shfl_up(t, off, 64);
        if (lane >= off) t += v;
      }
      if (lane < 16) wtot[lane] = t;
    }
    __syncthreads();
    int run = carry + (w > 0 ? wtot[w - 1] : 0) + inc - s;
    for (int i = b; i < e; ++i) {
      const int v = buf[scan_pad(i)];
      buf[scan_pad(i)] = run;
      run += v;
    }
    __syncthreads();
    for (int i = tid; i < m; i += 1024) data[base + i] = buf[scan_pad(i)];
    carry += wtot[15];
    __syncthreads();  // buf and wtot are reused by the next tile
  }
  if (tid == 0 && total) *total = carry;
}

hipError_t launch_exclusive_scan(int* data, int n, int* total, hipStream_t st) {
  const int tile = n < kScanTile ? (n > 0 ? n : 1) : kScanTile;
  const size_t lds = (size_t)scan_pad(tile) * sizeof(int);
  if (lds > 64 * 1024) {
    // allowed once for the largest tile
    static const hipError_t allowed = hipFuncSetAttribute(
        reinterpret_cast<const void*>(scan_lds_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)(scan_pad(kScanTile) * sizeof(int)));
    if (allowed != hipSuccess) return allowed;
  }
  hipLaunchKernelGGL(scan_lds_kernel, dim3(1), dim3(1024), lds, st, data, n, tile, total);
  return hipGetLastError();
}

hipError_t radix_sort_pairs(int* key_a, int* id_a, int* key_b, int* id_b, int* hist, int n,
                            long long key_limit, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int nblocks = (n + 255) / 256;
  int passes = 0;
  while (passes < 4 && (key_limit >> (8 * passes)) > 0) ++passes;
  if (passes & 1) ++passes;  // an even count leaves the result in (key_a, id_a)
  int *ka = key_a, *ia = id_a, *kb = key_b, *ib = id_b;
  for (int p = 0; p < passes; ++p) {
    int shift = 8 * p;
    hipLaunchKernelGGL(radix_count_kernel, dim3(nblocks), dim3(256), 0, st, ka, n, shift,
                       nblocks, hist);
    hipError_t e = launch_exclusive_scan(hist, 256 * nblocks, nullptr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblocks), dim3(256), 0, st, ka, ia, kb, ib, n,
                       shift, nblocks, hist);
    int* t = ka;
    ka = kb;
    kb = t;
    t = ia;
    ia = ib;
    ib = t;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// merge equal nodes: charge = sum of entry values in atom order, from 0

__global__ void heads_kernel(const int* key, int n, int* heads) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) heads[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

__global__ void merge_kernel(const int* key, const int* id, const double* val, const int* uid,
                             int n, int* q_idx, double* q_val, double* q_rho, double pref) {
#pragma clang fp contract(off)
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (i != 0 && key[i] == key[i - 1]) return;
  double s = 0.0;
  int j = i;
  do {
    s += val[id[j]];
    ++j;
  } while (j < n && key[j] == key[i]);
  int u = uid[i];
  q_idx[u] = key[i];
  q_val[u] = s;
  q_rho[u] = pref * s;
}

hipError_t launch_merge_charges(const int* key, const int* id, const double* val, int* heads,
                                int n, int* nq_dev, int* q_idx, double* q_val, double* q_rho,
                                double rho_pref, hipStream_t st) {
  if (n <= 0) return launch_fill_u32(reinterpret_cast<uint32_t*>(nq_dev), 1, 0u, st);
  int nb = (n + 255) / 256;
  hipLaunchKernelGGL(heads_kernel, dim3(nb), dim3(256), 0, st, key, n, heads);
  hipError_t e = launch_exclusive_scan(heads, n, nq_dev, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(merge_kernel, dim3(nb), dim3(256), 0, st, key, id, val, heads, n, q_idx,
                     q_val, q_rho, rho_pref);
  return hipGetLastError();
}

// ptr[l] = first entry whose key >= l * keys_per_line (binary search), l = 0..n_lines
__global__ void line_ptr_kernel(const int* keys, const int* n_dev, int n_lines,
                                int keys_per_line, int* ptr) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l > n_lines) return;
  const int n = *n_dev;
  const long long target = (long long)l * keys_per_line;
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if ((long long)keys[mid] < target)
      lo = mid + 1;
    else
      hi = mid;
  }
  ptr[l] = lo;
}

hipError_t launch_line_ptr(const int* sorted_keys, const int* n_dev, int /*cap*/, int n_lines,
                           int keys_per_line, int* ptr, hipStream_t st) {
  hipLaunchKernelGGL(line_ptr_kernel, dim3((n_lines + 1 + 255) / 256), dim3(256), 0, st,
                     sorted_keys, n_dev, n_lines, keys_per_line, ptr);
  return hipGetLastError();
}

// keys ordering the charge list by y-lines ((z, x, y)) or z-lines ((y, x, z));
// entries past the list end get the sentinel nx*ny*nz
__global__ void axis_keys_kernel(const int* q_idx, const int* nq_dev, int cap, int nx, int nxp,
                                 int ny, int nz, int axis, int* key, int* id) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cap) return;
  const int nq = *nq_dev;
  int kk = nx * ny * nz;
  if (k < nq) {
    int lin = q_idx[k];
    int x = lin % nxp;
    int t = lin / nxp;
    int y = t % ny;
    int z = t / ny;
    kk = (axis == 1) ? (z * nx + x) * ny + y : (y * nx + x) * nz + z;
  }
  key[k] = kk;
  id[k] = k;
}

hipError_t launch_axis_keys(const int* q_idx, const int* nq_dev, int cap, int nx, int nxp, int ny,
                            int nz, int axis, int* key, int* id, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(axis_keys_kernel, dim3((cap + 255) / 256), dim3(256), 0, st, q_idx, nq_dev,
                     cap, nx, nxp, ny, nz, axis, key, id);
  return hipGetLastError();
}

__global__ void gather_entries_kernel(const int* id, const int* nq_dev, int cap, const int* q_idx,
                                      const double* q_rho, int* lin_out, double* rho_out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap || i >= *nq_dev) return;
  lin_out[i] = q_idx[id[i]];
  rho_out[i] = q_rho[id[i]];
}

hipError_t launch_gather_entries(const int* id, const int* nq_dev, int cap, const int* q_idx,
                                 const double* q_rho, int* lin_out, double* rho_out,
                                 hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_entries_kernel, dim3((cap + 255) / 256), dim3(256), 0, st, id, nq_dev,
                     cap, q_idx, q_rho, lin_out, rho_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dirichlet data on the outer shell (Eq. (BoundaryCond)):
//   u = l_B sum_i q_i exp(-kappa d) / (eps d),  kappa = kbar / sqrt(eps)
// and its vacuum counterpart (eps_in, kappa = 0).
// Shell enumeration: face z = 0 (ny*nx), face z = nz-1 (ny*nx), then per
// interior z the ring y = 0 (nx), y = ny-1 (nx), and x = 0, nx-1 for each
// interior y.

__device__ __forceinline__ void shell_node(long long s, int nx, int ny, int nz, int& i, int& j,
                                           int& k) {
  const long long nxy = (long long)nx * ny;
  const long long ring = 2LL * nx + 2LL * (ny - 2);
  if (s < nxy) {
    k = 0;
    j = (int)(s / nx);
    i = (int)(s % nx);
  } else if (s < 2 * nxy) {
    long long t = s - nxy;
    k = nz - 1;
    j = (int)(t / nx);
    i = (int)(t % nx);
  } else {
    long long t = s - 2 * nxy;
    k = 1 + (int)(t / ring);
    int r = (int)(t % ring);
    if (r < nx) {
      j = 0;
      i = r;
    } else if (r < 2 * nx) {
      j = ny - 1;
      i = r - nx;
    } else {
      int r2 = r - 2 * nx;
      j = 1 + r2 / 2;
      i = (r2 & 1) ? nx - 1 : 0;
    }
  }
}

// Both media in one pass: the solvated value with eps_s and kappa, the
// vacuum value (kappa = 0) with eps_v, sharing the distance of every
// (shell node, atom) pair.  R is the arithmetic type of one pair's term
// (FP64 here; FP32 terms use boundary_f32_kernel below); the sums over
// atoms are FP64, and the constant factor l_B / eps is applied once at the
// end.
template <typename R>
__device__ __forceinline__ void pair_terms(R dx, R dy, R dz, R q, R kappa, R& ts, R& tv);
template <>
__device__ __forceinline__ void pair_terms<double>(double dx, double dy, double dz, double q,
                                                   double kappa, double& ts, double& tv) {
  const double d = sqrt(dx * dx + dy * dy + dz * dz);
  tv = q / d;
  ts = tv * exp(-kappa * d);
}

template <typename R>
__global__ __launch_bounds__(256) void boundary_kernel(SetupArgs a, double scale_s, double kappa,
                                                       double scale_v, double* bc_s, double* bc_v,
                                                       long long nshell) {
#pragma clang fp contract(off)
  __shared__ R sx[256], sy[256], sz[256], sq[256];
  const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
  const bool valid = s < nshell;
  R X = 0, Y = 0, Z = 0;
  if (valid) {
    int i, j, k;
    shell_node(s, a.nx, a.ny, a.nz, i, j, k);
    X = (R)(a.ox + (double)i * a.h);
    Y = (R)(a.oy + (double)j * a.h);
    Z = (R)(a.oz + (double)k * a.h);
  }
  const int na = a.n_atoms;
  const R kap = (R)kappa;
  double acc_s = 0.0, acc_v = 0.0;
  for (int t0 = 0; t0 < na; t0 += 256) {
    int t = t0 + threadIdx.x;
    if (t < na) {
      sx[threadIdx.x] = (R)a.atoms[t];
      sy[threadIdx.x] = (R)a.atoms[na + t];
      sz[threadIdx.x] = (R)a.atoms[2 * na + t];
      sq[threadIdx.x] = (R)a.atoms[3 * na + t];
    }
    __syncthreads();
    const int cnt = min(256, na - t0);
    if (valid) {
      for (int jj = 0; jj < cnt; ++jj) {
        R ts, tv;
        pair_terms<R>(X - sx[jj], Y - sy[jj], Z - sz[jj], sq[jj], kap, ts, tv);
        acc_s += (double)ts;
        acc_v += (double)tv;
      }
    }
    __syncthreads();
  }
  if (valid) {
    bc_s[s] = scale_s * acc_s;
    if (bc_v) bc_v[s] = scale_v * acc_v;
  }
}

// FP32 terms.  Block: 256 threads = 64 node groups x 4 atom slices (one
// wave per slice).  A thread takes kBcK shell nodes (group g: nodes
// g, g + 64, ... of the block's range) and the atoms sl, sl + 4, ... of
// every 256-atom tile staged in LDS as (x, y, z, q): each staged atom is
// read once (a broadcast LDS read) and used for kBcK nodes, which also
// gives every thread kBcK independent chains.  Per pair: d^2 by FMAs,
// 1/d by the hardware reciprocal square root (d^2 >= h^2 on the shell:
// no denormal inputs), e^{-kappa d} = 2^{-kappa log2(e) d} by the hardware
// base-2 exponential.  The terms of up to 32 atoms are summed in FP32
// before they join the FP64 sums (the per-term rounding of FP32 terms is of
// the same order), and the four slices' FP64 sums are added in a fixed
// order at the end.
constexpr int kBcGroups = 64, kBcSlices = 4, kBcK = 4;
constexpr int kBcNodes = kBcGroups * kBcK;  // shell nodes per block
__global__ __launch_bounds__(256) void boundary_f32_kernel(SetupArgs a, double scale_s,
                                                           double kappa, double scale_v,
                                                           double* bc_s, double* bc_v,
                                                           long long nshell) {
  __shared__ float4 sa[256];
  __shared__ double rs[kBcSlices][kBcNodes], rv[kBcSlices][kBcNodes];
  const int g = threadIdx.x % kBcGroups;
  const int sl = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kBcGroups);
  const long long s0 = (long long)blockIdx.x * kBcNodes + g;
  float X[kBcK], Y[kBcK], Z[kBcK];
#pragma unroll
  for (int k = 0; k < kBcK; ++k) {
    const long long s = s0 + (long long)k * kBcGroups;
    // past the shell: a far point, so that every term stays finite
    X[k] = Y[k] = Z[k] = 1.0e4f;
    if (s < nshell) {
      int i, j, kk;
      shell_node(s, a.nx, a.ny, a.nz, i, j, kk);
      X[k] = (float)(a.ox + (double)i * a.h);
      Y[k] = (float)(a.oy + (double)j * a.h);
      Z[k] = (float)(a.oz + (double)kk * a.h);
    }
  }
  const int na = a.n_atoms;
  const float c = (float)(-kappa * 1.4426950408889634);  // -kappa log2(e)
  double acc_s[kBcK], acc_v[kBcK];
#pragma unroll
  for (int k = 0; k < kBcK; ++k) acc_s[k] = acc_v[k] = 0.0;
  for (int t0 = 0; t0 < na; t0 += 256) {
    const int t = t0 + (int)threadIdx.x;
    if (t < na)
      sa[threadIdx.x] = make_float4((float)a.atoms[t], (float)a.atoms[na + t],
                                    (float)a.atoms[2 * na + t], (float)a.atoms[3 * na + t]);
    __syncthreads();
    const int cnt = min(256, na - t0);
    for (int j0 = sl; j0 < cnt; j0 += 32 * kBcSlices) {
      float ps[kBcK], pv[kBcK];
#pragma unroll
      for (int k = 0; k < kBcK; ++k) ps[k] = pv[k] = 0.0f;
      const int je = min(j0 + 32 * kBcSlices, cnt);
#pragma unroll 4
      for (int jj = j0; jj < je; jj += kBcSlices) {
        const float4 at = sa[jj];
#pragma unroll
        for (int k = 0; k < kBcK; ++k) {
          const float dx = X[k] - at.x, dy = Y[k] - at.y, dz = Z[k] - at.z;
          const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
          const float ri = __builtin_amdgcn_rsqf(d2);
          const float tv = at.w * ri;
          pv[k] += tv;
          ps[k] = fmaf(tv, __builtin_amdgcn_exp2f(c * (d2 * ri)), ps[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < kBcK; ++k) {
        acc_s[k] += (double)ps[k];
        acc_v[k] += (double)pv[k];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kBcK; ++k) {
    rs[sl][g + k * kBcGroups] = acc_s[k];
    rv[sl][g + k * kBcGroups] = acc_v[k];
  }
  __syncthreads();
  if (sl == 0) {
#pragma unroll
    for (int k = 0; k < kBcK; ++k) {
      const long long s = s0 + (long long)k * kBcGroups;
      if (s >= nshell) continue;
      double ts = 0.0, tv = 0.0;
#pragma unroll
      for (int q = 0; q < kBcSlices; ++q) {
        ts += rs[q][g + k * kBcGroups];
        tv += rv[q][g + k * kBcGroups];
      }
      bc_s[s] = scale_s * ts;
      if (bc_v) bc_v[s] = scale_v * tv;
    }
  }
}

hipError_t launch_boundary(const SetupArgs& a, double eps_s, double kappa, double eps_v,
                           double lB, double* bc_s, double* bc_v, bool fp32_terms,
                           hipStream_t st) {
  const long long ns = shell_count(a.nx, a.ny, a.nz);
  const dim3 g((unsigned)((ns + 255) / 256)), b(256);
  const double ss = lB / eps_s, sv = lB / eps_v;
  if (fp32_terms)
    hipLaunchKernelGGL(boundary_f32_kernel, dim3((unsigned)((ns + kBcNodes - 1) / kBcNodes)),
                       dim3(kBcGroups * kBcSlices), 0, st, a, ss, kappa, sv, bc_s, bc_v, ns);
  else
    hipLaunchKernelGGL(boundary_kernel<double>, g, b, 0, st, a, ss, kappa, sv, bc_s, bc_v, ns);
  return hipGetLastError();
}

// Dirichlet data of a caller-given field (npb_solve_fields): the shell
// values of the dense [nz][ny][nx] array, in shell order
__global__ void shell_from_dense_kernel(const double* u0, int nx, int ny, int nz, long long ns,
                                        double* bc) {
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < ns;
       s += (long long)gridDim.x * blockDim.x) {
    int i, j, k;
    shell_node(s, nx, ny, nz, i, j, k);
    bc[s] = u0[((long long)k * ny + j) * nx + i];
  }
}

hipError_t launch_shell_from_dense(const double* u0, int nx, int ny, int nz, double* bc,
                                   hipStream_t st) {
  const long long ns = shell_count(nx, ny, nz);
  long long blocks = (ns + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(shell_from_dense_kernel, dim3((unsigned)blocks), dim3(256), 0, st, u0, nx, ny,
                     nz, ns, bc);
  return hipGetLastError();
}

// Face class of every (chunk, line) of one sweep direction: 0 if all nodes
// from the chunk's left neighbour to its right neighbour are solvent, 2 if
// all are solute, 1 otherwise (and for chunks that reach the line end).
// Face rule by location (face_loc): 0 / 2 if the chunk's M + 1 half points
// (bit 1 of the flags of the left neighbour .. the last row) are all
// solvent / all solute.  Lines are numbered as class_lines describes.
__global__ void chunk_class_kernel(const uint8_t* mask, int nx, int nxp, int ny, int nz, int dir,
                                   int M, int P, long long nlines, int face_loc, uint8_t* out) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nlines * P) return;
  const int p = (int)(idx / nlines);
  const long long l = idx - (long long)p * nlines;
  long long base, stride;
  int n;
  if (dir == 0) {
    const int nyi = ny - 2;
    int y = 1 + (int)(l % nyi), z = 1 + (int)(l / nyi);
    base = ((long long)z * ny + y) * nxp;
    stride = 1;
    n = nx;
  } else {
    const int nxi = nx - 2;
    int x = 1 + (int)(l % nxi), o = 1 + (int)(l / nxi);
    base = (dir == 1) ? ((long long)o * ny * nxp + x) : ((long long)o * nxp + x);
    stride = (dir == 1) ? nxp : (long long)nxp * ny;
    n = (dir == 1) ? ny : nz;
  }
  const int j0 = p * M, j1 = p * M + M + 1;
  uint8_t c = 1;
  if (j1 <= n - 1 && face_loc) {
    const int v0 = mask[base + (long long)j0 * stride] & 2;
    bool same = true;
    for (int j = j0 + 1; j < j1; ++j) same = same && ((mask[base + (long long)j * stride] & 2) == v0);
    if (same) c = v0 ? 2 : 0;
  } else if (j1 <= n - 1) {
    const uint8_t v0 = mask[base + (long long)j0 * stride];
    bool same = true;
    for (int j = j0 + 1; j <= j1; ++j) same = same && (mask[base + (long long)j * stride] == v0);
    if (same) c = v0 ? 2 : 0;
  }
  out[idx] = c;
}

hipError_t launch_chunk_classes(const uint8_t* mask, int nx, int nxp, int ny, int nz, int dir,
                                int M, int P, int face_loc, uint8_t* out, hipStream_t st) {
  const long long nlines = class_lines(nx, ny, nz, dir);
  const long long tot = nlines * P;
  hipLaunchKernelGGL(chunk_class_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     mask, nx, nxp, ny, nz, dir, M, P, nlines, face_loc, out);
  return hipGetLastError();
}

}  // namespace npb
