// Explicit Euler steps of the pseudo-time NPB equation (Eq. (TimeDepNPB)
// with the 7-point operator of Eq. (SpatialOperators)): the reference
// solver the paper's energy tables are measured against (Sec. 2.3; Sec.
// 5.2 and 5.4 use dt = 1e-5 and T = 10).  FP64 throughout.
//
// One launch is one step of one field: v = u + tau (div eps grad u -
// kbar^2 sinh u + rho) on the interior nodes, reading u and writing v
// (ping-pong buffers; the Dirichlet shell of both holds the boundary data).
// The step is bound by HBM traffic: per interior node one field value is
// read, one written and one flag byte read (17 bytes); neighbours come from
// the caches (the tiles an XCD works on are contiguous, so their halos meet
// in that XCD's L2).
#include <hip/hip_ext.h>

#include "npb_internal.h"

namespace npb {

namespace {

constexpr int kTX = 32, kTY = 2, kZC = 4;

// flags of an interior node: bit 0 its solute bit, bits 1..6 the solute
// bits of its neighbours at x-1, x+1, y-1, y+1, z-1, z+1 (face rule by
// location: the solute bits of the six half points themselves), bit 7 set
// when the node has a charge-list entry.  One byte carries everything the
// step needs about the dielectric and the source.
constexpr int kSourceBit = 0x80;

// tau-free source density at pitched node c of x line `line` (0 when the
// line's sorted charge entries do not hold c)
__device__ __forceinline__ double node_source(const EulerArgs& a, long long c, int line) {
  const int end = a.src_ptr[line + 1];
  int lo = a.src_ptr[line], hi = end;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((long long)a.q_idx[mid] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < end && (long long)a.q_idx[lo] == c) ? a.q_rho[lo] : 0.0;
}

// sinh(u) = (e^u - e^-u) / 2 from one exponential: e^-u is the hardware
// reciprocal estimate of e^u refined by two Newton-Raphson steps
// (x <- x + x (1 - t x)).  Near u = 0 the difference loses relative
// accuracy but keeps an absolute error of a few 1e-16, which is what the
// additive update sees.  Non-finite for |u| beyond the exponential's range.
__device__ __forceinline__ double sinh_by_exp(double u) {
  const double t = exp(u);
  double r = __builtin_amdgcn_rcp(t);
  r = fma(fma(-t, r, 1.0), r, r);
  r = fma(fma(-t, r, 1.0), r, r);
  return 0.5 * (t - r);
}

// Block b of the launch takes tile xcd * per + b / 8 with xcd = b % 8: the
// hardware hands consecutive blocks to the eight XCDs in turn, so each XCD
// then works through one contiguous range of tiles (x fastest, then y,
// then z), whose y and z neighbours it shares in its own L2.  A tile is
// kTX x kTY (x, y) columns of kZC planes; all of a thread's loads are
// issued before any arithmetic (planes past the last interior plane are
// clamped to the boundary plane and not stored).
__global__ __launch_bounds__(kTX * kTY) void euler_step_kernel(EulerArgs a) {
  const int b0 = (int)blockIdx.x;
  const int b = (b0 % 8) * a.per + b0 / 8;
  if (b >= a.ntiles) return;  // no barriers below: whole blocks or lanes leave
  const int tx = b % a.tiles_x, ty = (b / a.tiles_x) % a.tiles_y, tz = b / (a.tiles_x * a.tiles_y);
  const int i = 1 + tx * kTX + (int)threadIdx.x % kTX;
  const int j = 1 + ty * kTY + (int)threadIdx.x / kTX;
  if (i > a.nx - 2 || j > a.ny - 2) return;
  const int k0 = 1 + tz * kZC;
  const int klast = a.nz - 2;  // last interior plane
  const long long row = a.nxp;
  const long long plane = (long long)a.nxp * a.ny;
  const double* __restrict__ u = a.u;
  double* __restrict__ v = a.v;
  const uint8_t* __restrict__ fl = a.flags;
  const long long c0 = (long long)j * row + i;
  // planes k0 - 1 .. k0 + kZC of the column, x/y neighbours and flags of
  // planes k0 .. k0 + kZC - 1
  double col[kZC + 2], uw[kZC], ue[kZC], us[kZC], un[kZC];
  int f[kZC];
#pragma unroll
  for (int z = 0; z < kZC + 2; ++z) col[z] = u[(long long)min(k0 - 1 + z, klast + 1) * plane + c0];
#pragma unroll
  for (int z = 0; z < kZC; ++z) {
    const long long c = (long long)min(k0 + z, klast) * plane + c0;
    uw[z] = u[c - 1];
    ue[z] = u[c + 1];
    us[z] = u[c - row];
    un[z] = u[c + row];
    f[z] = fl[c];
  }
  bool bad = false;
#pragma unroll
  for (int z = 0; z < kZC; ++z) {
    const int k = k0 + z;
    if (k > klast) break;
    const double uc = col[z + 1];
    const double dw = uw[z] - uc, de = ue[z] - uc, ds = us[z] - uc, dn = un[z] - uc;
    const double db = col[z] - uc, da = col[z + 2] - uc;
    const int fc = f[z];
    double r;
    if (a.uniform) {
      r = a.re_uniform * (((dw + de) + (ds + dn)) + (db + da));
    } else {
      // a solvent node's faces carry re[0] (solvent neighbour) or re[1]
      // (solute neighbour), a solute node's re[1] or re[2]: base plus
      // delta times the neighbour's solute bit
      // (by location: re[0] or re[2] by the face's own bit)
      const int s = fc & 1;
      const double base = a.face_loc ? a.re[0] : (s ? a.re[1] : a.re[0]);
      const double delta = a.face_loc ? a.re[2] - a.re[0]
                                      : (s ? a.re[2] - a.re[1] : a.re[1] - a.re[0]);
      double m = (double)((fc >> 1) & 1) * dw;
      m = fma((double)((fc >> 2) & 1), de, m);
      m = fma((double)((fc >> 3) & 1), ds, m);
      m = fma((double)((fc >> 4) & 1), dn, m);
      m = fma((double)((fc >> 5) & 1), db, m);
      m = fma((double)((fc >> 6) & 1), da, m);
      r = fma(base, ((dw + de) + (ds + dn)) + (db + da), delta * m);
      // kbar^2 sinh(u) on solvent nodes (kbar = 0 in the solute)
      if (s == 0 && a.nl) r = fma(-a.tk, sinh_by_exp(uc), r);
    }
    const long long c = (long long)k * plane + c0;
    if (fc & kSourceBit) r = fma(a.tau, node_source(a, c, k * a.ny + j), r);
    v[c] = uc + r;
    bad |= !isfinite(uc + r);
  }
  // a stored value that is not finite: the run diverged (Sec. 4.2)
  if (bad && a.nonfinite != nullptr) atomicOr(a.nonfinite, 1);
}

// flags of every node from the solute mask (nullptr: no solute) and, for
// the face rule by location, the half-point bits fx, fy, fz (bit 1 of the
// lower node's byte); shell and padding nodes get 0
__global__ __launch_bounds__(256) void euler_flags_kernel(const uint8_t* mask, const uint8_t* fx,
                                                          const uint8_t* fy, const uint8_t* fz,
                                                          uint8_t* flags, int nx, int nxp, int ny,
                                                          int nz) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long plane = (long long)nxp * ny;
  if (e >= plane * nz) return;
  const int i = (int)(e % nxp);
  const int j = (int)((e / nxp) % ny);
  const int k = (int)(e / plane);
  int f = 0;
  if (mask && i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && k >= 1 && k <= nz - 2) {
    if (fx)
      f = (mask[e] & 1) | (fx[e - 1] & 2) | ((fx[e] & 2) << 1) | ((fy[e - nxp] & 2) << 2) |
          ((fy[e] & 2) << 3) | ((fz[e - plane] & 2) << 4) | ((fz[e] & 2) << 5);
    else
      f = (mask[e] & 1) | ((mask[e - 1] & 1) << 1) | ((mask[e + 1] & 1) << 2) |
          ((mask[e - nxp] & 1) << 3) | ((mask[e + nxp] & 1) << 4) |
          ((mask[e - plane] & 1) << 5) | ((mask[e + plane] & 1) << 6);
  }
  flags[e] = (uint8_t)f;
}

// the source bit on every node with a trilinear source entry (entries are
// distinct nodes, so each byte has one writer)
__global__ __launch_bounds__(256) void euler_source_flags_kernel(const int* q_idx, const int* nq,
                                                                 int cap, uint8_t* flags) {
  const int e = (int)(blockIdx.x * 256 + threadIdx.x);
  const int n = min(*nq, cap);
  if (e < n) flags[q_idx[e]] = (uint8_t)(flags[q_idx[e]] | kSourceBit);
}

}  // namespace

int euler_z_chunk(int, int, int) { return kZC; }

hipError_t launch_euler_flags(const uint8_t* mask, const uint8_t* const* fmask, const int* q_idx,
                              const int* nq, int cap, uint8_t* flags, int nx, int nxp, int ny,
                              int nz, hipStream_t st) {
  const long long n = (long long)nxp * ny * nz;
  const uint8_t* f3[3] = {nullptr, nullptr, nullptr};
  if (fmask)
    for (int d = 0; d < 3; ++d) f3[d] = fmask[d];
  hipLaunchKernelGGL(euler_flags_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, mask,
                     f3[0], f3[1], f3[2], flags, nx, nxp, ny, nz);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || cap <= 0) return e;
  hipLaunchKernelGGL(euler_source_flags_kernel, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0,
                     st, q_idx, nq, cap, flags);
  return hipGetLastError();
}

hipError_t launch_euler_step(const EulerArgs& in, hipEvent_t start, hipEvent_t stop,
                             hipStream_t st) {
  if (in.nx < 3 || in.ny < 3 || in.nz < 3 || in.zc != kZC) return hipErrorInvalidValue;
  EulerArgs a = in;
  a.tiles_x = (a.nx - 2 + kTX - 1) / kTX;
  a.tiles_y = (a.ny - 2 + kTY - 1) / kTY;
  const int tiles_z = (a.nz - 2 + kZC - 1) / kZC;
  a.ntiles = a.tiles_x * a.tiles_y * tiles_z;
  a.per = (a.ntiles + 7) / 8;
  const dim3 grid((unsigned)(8 * a.per));
  if (start)
    hipExtLaunchKernelGGL(euler_step_kernel, grid, dim3(kTX * kTY), 0, st, start, stop, 0u, a);
  else
    hipLaunchKernelGGL(euler_step_kernel, grid, dim3(kTX * kTY), 0, st, a);
  return hipGetLastError();
}

}  // namespace npb
