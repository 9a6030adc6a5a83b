// Per-solve setup on the device: solute mask, trilinear charges, source
// density, per-line source lists and Dirichlet boundary data.
//
// All of it is deterministic: the charge at a node is summed in atom order
// (a stable sort of the 8 N_a stencil entries by node), so repeated solves
// give bit-identical inputs to the time loop.  FP64 throughout; expression
// order follows the definitions so that contraction into fused
// multiply-adds is switched off where a predicate or a weight is formed.
#include <type_traits>

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

// Visit the nodes (lo[0] + i, lo[1] + j, lo[2] + k) of a bx x by x bz box
// with one block: lane t & 31 walks x in passes of 32, t >> 5 the (j, k)
// rows in steps of blockDim / 32, carried by subtraction (no integer
// division per node).
template <typename F>
__device__ __forceinline__ void box_walk(const int (&lo)[3], int bx, int by, int bz, F&& f) {
  const int lane = (int)threadIdx.x & 31, r0 = (int)threadIdx.x >> 5;
  const int rstep = (int)blockDim.x >> 5;
  for (int i = lane; i < bx; i += 32) {
    int j = r0, k = 0;
    while (j >= by) {
      j -= by;
      ++k;
    }
    while (k < bz) {
      f(lo[0] + i, lo[1] + j, lo[2] + k);
      j += rstep;
      while (j >= by) {
        j -= by;
        ++k;
      }
    }
  }
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
  const double R2 = R * R;
  box_walk(lo, bx, by, bz, [&](int i, int j, int k) {
#pragma clang fp contract(off)
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
  });
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
  const double R2 = R * R;
  box_walk(lo, bx, by, bz, [&](int i, int j, int k) {
#pragma clang fp contract(off)
    const int idx[3] = {i, j, k};
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
  });
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

// Multi-block exclusive scan for long arrays: every block scans one tile of
// kScanTileN = 4096 entries (4 per thread) and leaves the tile's total in
// aux; the tile totals are scanned by scan_lds_kernel (which also gives the
// grand total); a last pass adds each tile's offset.  Integer sums, so the
// result does not depend on scheduling.
constexpr int kScanTileN = 4096;
__global__ __launch_bounds__(1024) void scan_tiles_kernel(int* data, int n, int* aux) {
  __shared__ int wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const long long base = (long long)blockIdx.x * kScanTileN + 4LL * tid;
  int v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = (base + q < n) ? data[base + q] : 0;
  const int s = (v[0] + v[1]) + (v[2] + v[3]);
  int inc = s;
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(inc, off, 64);
    if (lane >= off) inc += u;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  if (w == 0) {
    int t = lane < 16 ? wsum[lane] : 0;
    for (int off = 1; off < 16; off <<= 1) {
      const int u = __shfl_up(t, off, 64);
      if (lane >= off) t += u;
    }
    if (lane < 16) wsum[lane] = t;
  }
  __syncthreads();
  int run = (w > 0 ? wsum[w - 1] : 0) + inc - s;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (base + q < n) data[base + q] = run;
    run += v[q];
  }
  if (tid == 0) aux[blockIdx.x] = wsum[15];
}
__global__ __launch_bounds__(1024) void scan_add_kernel(int* data, int n, const int* aux) {
  const long long base = (long long)blockIdx.x * kScanTileN + 4LL * threadIdx.x;
  const int off = aux[blockIdx.x];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (base + q < n) data[base + q] += off;
}

int scan_aux_ints(int n) { return (n + kScanTileN - 1) / kScanTileN + 1; }

hipError_t launch_exclusive_scan(int* data, int n, int* total, int* aux, hipStream_t st) {
  if (aux != nullptr && n > 2 * kScanTileN) {
    const int nt = (n + kScanTileN - 1) / kScanTileN;
    hipLaunchKernelGGL(scan_tiles_kernel, dim3(nt), dim3(1024), 0, st, data, n, aux);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan(aux, nt, total, nullptr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_add_kernel, dim3(nt), dim3(1024), 0, st, data, n, aux);
    return hipGetLastError();
  }
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
    hipError_t e = launch_exclusive_scan(hist, 256 * nblocks, nullptr, hist + 256 * nblocks, st);
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
                                double rho_pref, int* scan_aux, hipStream_t st) {
  if (n <= 0) return launch_fill_u32(reinterpret_cast<uint32_t*>(nq_dev), 1, 0u, st);
  int nb = (n + 255) / 256;
  hipLaunchKernelGGL(heads_kernel, dim3(nb), dim3(256), 0, st, key, n, heads);
  hipError_t e = launch_exclusive_scan(heads, n, nq_dev, scan_aux, st);
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

// ---------------------------------------------------------------------------
// Dirichlet data of both media in one pass (Eq. (BoundaryCond)): the
// solvated value l_B/eps_s sum q e^{-kappa d}/d and the vacuum value
// l_B/eps_v sum q/d, sharing the distance of every (shell node, atom) pair.
//
// The shell is walked as rows of nodes along one axis: x on the two z faces
// (every row j) and on the two y faces (every interior z), y on the two x
// faces (interior y of every interior z).  A thread takes kBcK consecutive
// nodes of a row: for each atom the part of the squared distance across the
// row, (f1 - a_f1)^2 + (z - a_z)^2, is formed once and shared by the
// thread's nodes, which then need one subtraction and one FMA each.  Block:
// 256 threads = 64 row segments x 4 atom slices (one wave per slice); atoms
// are staged 256 at a time in LDS as (x, y, z, q) and read by broadcast; the
// slices' sums are added in a fixed order at the end.
//
// Per pair, 1/d comes from the hardware reciprocal square root (FP32 as is;
// FP64 refined by two Newton steps) and e^{-kappa d} from a base-2
// exponential (FP32: the hardware one; FP64: written below).  FP32 terms are
// summed in FP32 over up to 32 atoms before they join FP64 sums (the
// per-term rounding of FP32 terms is of the same order); FP64 terms go
// straight into FP64 sums.
constexpr int kBcGroups = 64, kBcSlices = 4, kBcK = 8;

template <typename R>
struct BcPair;
// One atom-node pair: ts += q e^{-kappa d} / d (solvated, kMedia bit 0),
// tv += q / d (vacuum, bit 1).  Either medium alone does the same arithmetic
// as both together, so its sums are bit-identical.
template <>
struct BcPair<float> {
  // c = -kappa log2(e).  kUnit: the coordinates come scaled by kappa log2(e)
  // (the sums then carry a factor 1 / (kappa log2(e)), taken out at the end),
  // so the exponent is the scaled distance itself
  template <int kMedia, bool kUnit>
  static __device__ __forceinline__ void add(float d2, float q, float c, float& ts, float& tv) {
    const float ri = __builtin_amdgcn_rsqf(d2);
    const float t = q * ri;
    if constexpr ((kMedia & 2) != 0) tv += t;
    if constexpr ((kMedia & 1) != 0)
      ts = fmaf(t, __builtin_amdgcn_exp2f(kUnit ? -(d2 * ri) : c * (d2 * ri)), ts);
  }
};
template <>
struct BcPair<double> {
  // c = -kappa
  template <int kMedia, bool kUnit>
  static __device__ __forceinline__ void add(double d2, double q, double c, double& ts,
                                             double& tv) {
    double ri = __builtin_amdgcn_rsq(d2);
    ri = fma(0.5 * ri, fma(-d2 * ri, ri, 1.0), ri);
    ri = fma(0.5 * ri, fma(-d2 * ri, ri, 1.0), ri);
    const double t = q * ri;
    if constexpr ((kMedia & 2) != 0) tv += t;
    if constexpr ((kMedia & 1) != 0) ts = fma(t, exp_neg(c * (d2 * ri)), ts);
  }
};

// shell row segments of kBcK nodes: faces z0, z1 (rows j, along x), y0, y1
// (rows k, along x), x0, x1 (rows k, along interior y)
struct BcSeg {
  long long nz2, ny2, nx2;  // segments of the z, y and x face pairs
};
__device__ __forceinline__ BcSeg bc_segments(int nx, int ny, int nz) {
  const long long sx = (nx + kBcK - 1) / kBcK, sy = (ny - 2 + kBcK - 1) / kBcK;
  return BcSeg{2LL * ny * sx, 2LL * (nz - 2) * sx, 2LL * (nz - 2) * sy};
}

// e^y for |y| <= 0.1 by its Taylor polynomial to degree 9 (remainder below
// 3e-17 relative)
__device__ __forceinline__ double exp_small(double y) {
  double p = 1.0 / 362880.0;
  p = fma(p, y, 1.0 / 40320.0);
  p = fma(p, y, 1.0 / 5040.0);
  p = fma(p, y, 1.0 / 720.0);
  p = fma(p, y, 1.0 / 120.0);
  p = fma(p, y, 1.0 / 24.0);
  p = fma(p, y, 1.0 / 6.0);
  p = fma(p, y, 0.5);
  p = fma(p, y, 1.0);
  return fma(p, y, 1.0);
}

// kMedia: 1 solvated values only, 2 vacuum only, 3 both.  kChain (FP64
// terms, kappa h <= 0.1): along a row the screening factor of node q + 1
// is that of node q times e^{-kappa (d_{q+1} - d_q)}, |kappa (d_{q+1} - d_q)|
// <= kappa h, from exp_small (relative error of the chain below 1e-14 over
// the row's eight nodes, from the rounding of the distance differences).
// xs: factor of every coordinate (1, or kappa log2(e) with kUnit; the sums
// then carry a factor 1 / xs, which scale_s and scale_v take out).
template <typename R, int kMedia, bool kChain = false, bool kUnit = false>
__global__ __launch_bounds__(256) void boundary_rows_kernel(SetupArgs a, double scale_s,
                                                            double c_exp, double scale_v,
                                                            double xs, double* bc_s,
                                                            double* bc_v) {
  using R4 = typename std::conditional<std::is_same<R, float>::value, float4, double4>::type;
  __shared__ R4 sa[256];
  __shared__ double rs[kBcSlices][kBcGroups * kBcK], rv[kBcSlices][kBcGroups * kBcK];
  const int g = threadIdx.x % kBcGroups;
  const int sl = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kBcGroups);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long long nxy = (long long)nx * ny, ring = 2LL * nx + 2LL * (ny - 2);
  const BcSeg sg = bc_segments(nx, ny, nz);
  const long long sxr = (nx + kBcK - 1) / kBcK, syr = (ny - 2 + kBcK - 1) / kBcK;
  // this thread's segment: face, row, first node along the row
  long long sid = (long long)blockIdx.x * kBcGroups + g;
  int face = -1, row = 0, u0 = 0;
  if (sid < sg.nz2) {
    face = (int)(sid / (ny * sxr));
    const long long t = sid - face * ny * sxr;
    row = (int)(t / sxr);
    u0 = (int)(t % sxr) * kBcK;
  } else if ((sid -= sg.nz2) < sg.ny2) {
    face = 2 + (int)(sid / ((nz - 2) * sxr));
    const long long t = sid - (face - 2) * (nz - 2) * sxr;
    row = (int)(t / sxr);
    u0 = (int)(t % sxr) * kBcK;
  } else if ((sid -= sg.ny2) < sg.nx2) {
    face = 4 + (int)(sid / ((nz - 2) * syr));
    const long long t = sid - (face - 4) * (nz - 2) * syr;
    row = (int)(t / syr);
    u0 = (int)(t % syr) * kBcK;
  }
  const bool vy = face >= 4;  // the row runs along y
  const int len = face < 0 ? 0 : (vy ? ny - 2 : nx);
  // fixed coordinates across the row, varying one per node
  R F1 = R(1e4), F2 = R(1e4), V[kBcK];
  int cnt = 0;
  if (face >= 0) {
    const int kz = face < 2 ? (face == 1 ? nz - 1 : 0) : row + 1;
    F2 = (R)((a.oz + (double)kz * a.h) * xs);
    if (face < 2)
      F1 = (R)((a.oy + (double)row * a.h) * xs);
    else if (face < 4)
      F1 = (R)((a.oy + (double)(face == 3 ? ny - 1 : 0) * a.h) * xs);
    else
      F1 = (R)((a.ox + (double)(face == 5 ? nx - 1 : 0) * a.h) * xs);
    cnt = min(kBcK, len - u0);
  }
#pragma unroll
  for (int t = 0; t < kBcK; ++t) {
    const int u = u0 + t;
    V[t] = R(1e4);
    if (t < cnt)
      V[t] = vy ? (R)((a.oy + (double)(1 + u) * a.h) * xs) : (R)((a.ox + (double)u * a.h) * xs);
  }
  const int na = a.n_atoms;
  const R c = (R)c_exp;
  double acc_s[kBcK], acc_v[kBcK];
#pragma unroll
  for (int t = 0; t < kBcK; ++t) acc_s[t] = acc_v[t] = 0.0;
  // Segments run z faces, y faces, then x faces (rows along y): the block's
  // rows are all along x or all along y except in the block that holds the
  // last y-face and first x-face segments.
  const long long sb0 = (long long)blockIdx.x * kBcGroups, yb = sg.nz2 + sg.ny2;
  const long long sall = sg.nz2 + sg.ny2 + sg.nx2;
  const long long sb1 = (sb0 + kBcGroups < sall ? sb0 + kBcGroups : sall) - 1;
  auto sum_atoms = [&](auto mode) {
    constexpr int kMode = decltype(mode)::value;
    for (int t0 = 0; t0 < na; t0 += 256) {
      const int t = t0 + (int)threadIdx.x;
      if (t < na) {
        R4 at;
        at.x = (R)(a.atoms[t] * xs);
        at.y = (R)(a.atoms[na + t] * xs);
        at.z = (R)(a.atoms[2 * na + t] * xs);
        at.w = (R)a.atoms[3 * na + t];
        sa[threadIdx.x] = at;
      }
      __syncthreads();
      const int n = min(256, na - t0);
      // FP32: partial sums over 32 atoms of the slice; FP64: one run
      constexpr int kRun = std::is_same<R, float>::value ? 32 * kBcSlices : 256;
      for (int j0 = sl; j0 < n; j0 += kRun) {
        R ps[kBcK], pv[kBcK];
#pragma unroll
        for (int q = 0; q < kBcK; ++q) ps[q] = pv[q] = R(0);
        const int je = min(j0 + kRun, n);
#pragma unroll 2
        for (int jj = j0; jj < je; jj += kBcSlices) {
          const R4 at = sa[jj];
          // the row's direction: block-uniform (kMode 0: x, 1: y) but for the
          // one block that holds rows of both kinds (kMode 2)
          const bool rv_y = kMode == 2 ? vy : kMode == 1;
          const R d1 = F1 - (rv_y ? at.x : at.y), d3 = F2 - at.z;
          const R b2 = d1 * d1 + d3 * d3;
          const R av = rv_y ? at.y : at.x;
          if constexpr (kChain) {
            double dprev = 0.0, eprev = 0.0;
#pragma unroll
            for (int q = 0; q < kBcK; ++q) {
              const double dv = V[q] - av;
              const double d2 = dv * dv + b2;
              double ri = __builtin_amdgcn_rsq(d2);
              ri = fma(0.5 * ri, fma(-d2 * ri, ri, 1.0), ri);
              ri = fma(0.5 * ri, fma(-d2 * ri, ri, 1.0), ri);
              const double t = at.w * ri;
              if constexpr ((kMedia & 2) != 0) pv[q] += t;
              if constexpr ((kMedia & 1) != 0) {
                const double dist = d2 * ri;
                const double e =
                    q == 0 ? exp_neg(c * dist) : eprev * exp_small(c * (dist - dprev));
                ps[q] = fma(t, e, ps[q]);
                dprev = dist;
                eprev = e;
              }
            }
          } else {
#pragma unroll
            for (int q = 0; q < kBcK; ++q) {
              const R dv = V[q] - av;
              BcPair<R>::template add<kMedia, kUnit>(dv * dv + b2, at.w, c, ps[q], pv[q]);
            }
          }
        }
#pragma unroll
        for (int q = 0; q < kBcK; ++q) {
          acc_s[q] += (double)ps[q];
          acc_v[q] += (double)pv[q];
        }
      }
      __syncthreads();
    }
  };
  if (sb0 >= yb)
    sum_atoms(std::integral_constant<int, 1>{});
  else if (sb1 < yb)
    sum_atoms(std::integral_constant<int, 0>{});
  else
    sum_atoms(std::integral_constant<int, 2>{});
#pragma unroll
  for (int t = 0; t < kBcK; ++t) {
    if constexpr ((kMedia & 1) != 0) rs[sl][g * kBcK + t] = acc_s[t];
    if constexpr ((kMedia & 2) != 0) rv[sl][g * kBcK + t] = acc_v[t];
  }
  __syncthreads();
  if (sl == 0) {
    for (int t = 0; t < cnt; ++t) {
      // shell index of node u (the order shell_node enumerates)
      const int u = u0 + t;
      const long long si =
          vy ? 2 * nxy + (long long)row * ring + 2LL * nx + 2LL * u + (face == 5 ? 1 : 0)
          : face < 2 ? (face == 1 ? nxy : 0) + (long long)row * nx + u
                     : 2 * nxy + (long long)row * ring + (face == 3 ? nx : 0) + u;
      double ts = 0.0, tv = 0.0;
#pragma unroll
      for (int q = 0; q < kBcSlices; ++q) {
        if constexpr ((kMedia & 1) != 0) ts += rs[q][g * kBcK + t];
        if constexpr ((kMedia & 2) != 0) tv += rv[q][g * kBcK + t];
      }
      if constexpr ((kMedia & 1) != 0) bc_s[si] = scale_s * ts;
      if constexpr ((kMedia & 2) != 0) bc_v[si] = scale_v * tv;
    }
  }
}

hipError_t launch_boundary(const SetupArgs& a, double eps_s, double kappa, double eps_v,
                           double lB, double* bc_s, double* bc_v, bool fp32_terms,
                           hipStream_t st) {
  const long long sx = (a.nx + kBcK - 1) / kBcK, sy = (a.ny - 2 + kBcK - 1) / kBcK;
  const long long nseg = 2LL * a.ny * sx + 2LL * (a.nz - 2) * sx + 2LL * (a.nz - 2) * sy;
  const dim3 g((unsigned)((nseg + kBcGroups - 1) / kBcGroups)), b(kBcGroups * kBcSlices);
  const double ss = lB / eps_s, sv = lB / eps_v;
  const int media = (bc_s ? 1 : 0) | (bc_v ? 2 : 0);
  const double cf = fp32_terms ? -kappa * 1.4426950408889634 : -kappa;
  if (media == 0) return hipSuccess;
  // FP32 terms with screening: coordinates scaled by kappa log2(e), so that
  // the exponent needs no multiply (the same for either medium alone)
  const bool unit = fp32_terms && kappa > 0.0;
  const double xs = unit ? kappa * 1.4426950408889634 : 1.0;
#define NPB_BC_LAUNCH(R, M)                                                               \
  hipLaunchKernelGGL((boundary_rows_kernel<R, M>), g, b, 0, st, a, ss, cf, sv, 1.0, bc_s, \
                     bc_v)
#define NPB_BC_LAUNCH_UNIT(M)                                                            \
  hipLaunchKernelGGL((boundary_rows_kernel<float, M, false, true>), g, b, 0, st, a, ss * xs, \
                     cf, sv * xs, xs, bc_s, bc_v)
#define NPB_BC_LAUNCH_CHAIN(M)                                                             \
  hipLaunchKernelGGL((boundary_rows_kernel<double, M, true>), g, b, 0, st, a, ss, cf, sv, 1.0, \
                     bc_s, bc_v)
  // FP64 terms: the row-chained screening factor when kappa h <= 0.1
  const bool chain = !fp32_terms && kappa * a.h <= 0.1;
  if (unit) {
    if (media == 3)
      NPB_BC_LAUNCH_UNIT(3);
    else if (media == 1)
      NPB_BC_LAUNCH_UNIT(1);
    else
      NPB_BC_LAUNCH_UNIT(2);
  } else if (fp32_terms) {
    if (media == 3)
      NPB_BC_LAUNCH(float, 3);
    else if (media == 1)
      NPB_BC_LAUNCH(float, 1);
    else
      NPB_BC_LAUNCH(float, 2);
  } else if (chain && (media & 1) != 0) {
    if (media == 3)
      NPB_BC_LAUNCH_CHAIN(3);
    else
      NPB_BC_LAUNCH_CHAIN(1);
  } else {
    if (media == 3)
      NPB_BC_LAUNCH(double, 3);
    else if (media == 1)
      NPB_BC_LAUNCH(double, 1);
    else
      NPB_BC_LAUNCH(double, 2);
  }
#undef NPB_BC_LAUNCH_CHAIN
#undef NPB_BC_LAUNCH_UNIT
#undef NPB_BC_LAUNCH
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
// all are solute, 1 otherwise.  A line's last chunk, which ends at the last
// interior node or before the chunk's end, is classed by the nodes up to
// the right Dirichlet node (a chunk with no interior row past its first
// stays 1).
// Face rule by location (face_loc): 0 / 2 if the chunk's M + 1 half points
// (bit 1 of the flags of the left neighbour .. the last row) are all
// solvent / all solute.  Lines are numbered as class_lines describes.
__global__ void chunk_class_kernel(const uint8_t* mask, int nx, int nxp, int ny, int nz, int dir,
                                   int M, int P, long long nlines, int face_loc, uint8_t* out) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nlines * P) return;
  // x lines: the P chunks of a line on consecutive lanes, so that a wave's
  // word loads fall in a few cache lines of four rows (the output keeps its
  // (chunk, line) order); y / z lines: consecutive lines on consecutive
  // lanes, whose loads are contiguous along x
  const int p = dir == 0 ? (int)(idx % P) : (int)(idx / nlines);
  const long long l = dir == 0 ? idx / P : idx - (long long)p * nlines;
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
  const int j0 = p * M;
  int j1 = p * M + M + 1;
  if (j1 > n - 1 && j0 + 2 <= n - 2) j1 = n - 1;  // the last chunk: up to the Dirichlet node
  uint8_t c = 1;
  if (dir == 0 && j1 <= n - 1) {
    // x-lines: the chunk's bytes j0 .. j1 of one row, read as the 32-bit
    // words that hold them (rows and j0 = p M are 4-byte aligned; the word
    // of byte j1 ends inside the row's row4(nx) bytes)
    const uint32_t* w = reinterpret_cast<const uint32_t*>(mask + base);
    const int w0 = j0 >> 2, w1 = j1 >> 2;
    const uint32_t first = w[w0] & 0xffu;
    const uint32_t ref = face_loc ? ((first >> 1) & 1u) : first;
    bool same = true;
    for (int q = w0; q <= w1; ++q) {
      const uint32_t v = w[q];
      for (int b = 0; b < 4; ++b) {
        const int j = 4 * q + b;
        const uint32_t byte = (v >> (8 * b)) & 0xffu;
        const uint32_t x = face_loc ? ((byte >> 1) & 1u) : byte;
        // face rule by location: half points j0 .. j1 - 1; else nodes j0 .. j1
        const bool in = face_loc ? (j >= j0 && j < j1) : (j >= j0 && j <= j1);
        same = same && (!in || x == ref);
      }
    }
    if (same) c = ref ? 2 : 0;
  } else if (j1 <= n - 1 && face_loc) {
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
  out[(long long)p * nlines + l] = c;
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
