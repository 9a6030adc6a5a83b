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
// the caches.  A block owns a TX x TY column of (x, y) nodes and walks a
// range of z planes, keeping the planes below, at and above the node in
// registers, so that each field value is fetched from memory once per
// block.
#include <hip/hip_ext.h>

#include "npb_internal.h"

namespace npb {

namespace {

__device__ __forceinline__ double pick_face(int s, double r0, double r1, double r2) {
  return s == 0 ? r0 : (s == 1 ? r1 : r2);
}

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

template <int TX, int TY>
__global__ __launch_bounds__(TX * TY) void euler_step_kernel(EulerArgs a) {
  const int i = 1 + (int)blockIdx.x * TX + (int)threadIdx.x % TX;
  const int j = 1 + (int)blockIdx.y * TY + (int)threadIdx.x / TX;
  // no barriers below: lanes outside the grid simply leave
  if (i > a.nx - 2 || j > a.ny - 2) return;
  const int k0 = 1 + (int)blockIdx.z * a.zc;
  const int k1 = min(k0 + a.zc, a.nz - 1);
  const long long row = a.nxp;
  const long long plane = (long long)a.nxp * a.ny;
  const double* __restrict__ u = a.u;
  double* __restrict__ v = a.v;
  const uint8_t* __restrict__ fl = a.flags;
  long long c = (long long)k0 * plane + (long long)j * row + i;
  double ub = u[c - plane], uc = u[c];
  int fb = fl[c - plane], fc = fl[c];
  const double r0 = a.re[0], r1 = a.re[1], r2 = a.re[2];
  for (int k = k0; k < k1; ++k, c += plane) {
    const double ua = u[c + plane];
    const int fa = fl[c + plane];
    const double uw = u[c - 1], ue = u[c + 1], us = u[c - row], un = u[c + row];
    double r;
    if (a.uniform) {
      r = a.re_uniform * (((uw - uc) + (ue - uc)) + ((us - uc) + (un - uc)) + ((ub - uc) + (ua - uc)));
    } else {
      const int s = fc & 1;
      const int fw = fl[c - 1], fe = fl[c + 1], fs = fl[c - row], fn = fl[c + row];
      r = pick_face(s + (fw & 1), r0, r1, r2) * (uw - uc);
      r = fma(pick_face(s + (fe & 1), r0, r1, r2), ue - uc, r);
      r = fma(pick_face(s + (fs & 1), r0, r1, r2), us - uc, r);
      r = fma(pick_face(s + (fn & 1), r0, r1, r2), un - uc, r);
      r = fma(pick_face(s + (fb & 1), r0, r1, r2), ub - uc, r);
      r = fma(pick_face(s + (fa & 1), r0, r1, r2), ua - uc, r);
      // kbar^2 sinh(u) on solvent nodes (kbar = 0 in the solute)
      if (s == 0 && a.nl) r -= a.tk * sinh(uc);
    }
    if (fc & 2) r = fma(a.tau, node_source(a, c, k * a.ny + j), r);
    v[c] = uc + r;
    ub = uc;
    uc = ua;
    fb = fc;
    fc = fa;
  }
}

constexpr int kTX = 32, kTY = 8;

// flags = solute bit of the mask (or 0 for none)
__global__ __launch_bounds__(256) void euler_flags_kernel(const uint32_t* mask, uint32_t* flags,
                                                          size_t n4) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n4) flags[e] = mask ? (mask[e] & 0x01010101u) : 0u;
}

// bit 1 on every node with a trilinear source entry (entries are distinct
// nodes, so each byte has one writer)
__global__ __launch_bounds__(256) void euler_source_flags_kernel(const int* q_idx, const int* nq,
                                                                 int cap, uint8_t* flags) {
  const int e = (int)(blockIdx.x * 256 + threadIdx.x);
  const int n = min(*nq, cap);
  if (e < n) flags[q_idx[e]] = (uint8_t)(flags[q_idx[e]] | 2u);
}

}  // namespace

int euler_z_chunk(int nx, int ny, int nz) {
  const long long bxy = (long long)((nx - 2 + kTX - 1) / kTX) * ((ny - 2 + kTY - 1) / kTY);
  // about 2048 blocks (8 per CU) when the grid allows, 4..32 planes each
  long long zc = (long long)(nz - 2) * bxy / 2048;
  if (zc < 4) zc = 4;
  if (zc > 32) zc = 32;
  return (int)zc;
}

hipError_t launch_euler_flags(const uint8_t* mask, const int* q_idx, const int* nq, int cap,
                              uint8_t* flags, size_t n, hipStream_t st) {
  const size_t n4 = (n + 3) / 4;
  hipLaunchKernelGGL(euler_flags_kernel, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st,
                     reinterpret_cast<const uint32_t*>(mask), reinterpret_cast<uint32_t*>(flags),
                     n4);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || cap <= 0) return e;
  hipLaunchKernelGGL(euler_source_flags_kernel, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0,
                     st, q_idx, nq, cap, flags);
  return hipGetLastError();
}

hipError_t launch_euler_step(const EulerArgs& a, hipEvent_t start, hipEvent_t stop,
                             hipStream_t st) {
  if (a.nx < 3 || a.ny < 3 || a.nz < 3 || a.zc < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((a.nx - 2 + kTX - 1) / kTX), (unsigned)((a.ny - 2 + kTY - 1) / kTY),
                  (unsigned)((a.nz - 2 + a.zc - 1) / a.zc));
  if (start)
    hipExtLaunchKernelGGL((euler_step_kernel<kTX, kTY>), grid, dim3(kTX * kTY), 0, st, start,
                          stop, 0u, a);
  else
    hipLaunchKernelGGL((euler_step_kernel<kTX, kTY>), grid, dim3(kTX * kTY), 0, st, a);
  return hipGetLastError();
}

}  // namespace npb
