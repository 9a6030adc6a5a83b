// Vacuum potential without pseudo-time (Sec. 5.1, text after Eq. (deltaG)):
// the Poisson problem with the constant dielectric eps_in,
//     -eps_in delta^2 u = rho   on the interior nodes,   u = g on the shell,
// delta^2 the 7-point operator of Eq. (SpatialOperators) and g the vacuum
// Dirichlet data.  The paper obtains this phi_0 with an FFT fast Poisson
// solver; it enters the energy of Eq. (deltaG2) and the recovered potential
// of Sec. 5.4.  Everything here is FP64.
//
// Method: the Dirichlet couplings move to the right-hand side, and the
// type-I discrete sine transform along each axis diagonalises what remains:
// with S_N[j][k] = sin(pi (j+1)(k+1) / (N+1)) (symmetric, S_N S_N =
// (N+1)/2 I) and the mode eigenvalues e_N[m] = 4 sin^2(pi (m+1) / (2(N+1))),
//     u = (8 / ((X+1)(Y+1)(Z+1))) S S S [ (S S S f) / ((eps/h^2)(e_X + e_Y + e_Z)) ].
// Each 1-D transform is applied as a dense N x N matrix to all lines of an
// axis at once (a batched small GEMM, N = 3..512): an O(N) flop overhead over
// an FFT, but one regular kernel for any N, with the lines staged in LDS and
// the matrix rows streamed from L2.
//
// Array: the interior nodes only, dense, [Z][Y][X] = [nz-2][ny-2][nx-2].

#include <hip/hip_runtime.h>

#include "npb_internal.h"

namespace npb {

namespace {

// lines per transform tile; LDS rows padded to keep 16-byte alignment
constexpr int kTL = 16;
constexpr int kTS = kTL + 2;

// S_N and e_N (the argument (j+1)(k+1) is reduced mod 2(N+1) in integers)
__global__ void dst_matrix_kernel(double* S, double* eig, int N) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (long long)N * N) {
    const int j = (int)(t / N), k = (int)(t - (long long)j * N);
    const long long m = ((long long)(j + 1) * (k + 1)) % (2LL * (N + 1));
    S[t] = sinpi((double)m / (double)(N + 1));
  }
  if (t < N) {
    const double s = sinpi((double)(t + 1) / (2.0 * (N + 1)));
    eig[t] = 4.0 * s * s;
  }
}

// right-hand side f = c * (Dirichlet values of the shell neighbours),
// c = eps / h^2; the charges are added by dir_charges_kernel
__global__ void dir_rhs_kernel(double* f, const double* bc, int nx, int ny, int nz, double c) {
  const int X = nx - 2, Y = ny - 2, Z = nz - 2;
  const long long n = (long long)X * Y * Z;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(p % X);
    const long long t = p / X;
    const int y = (int)(t % Y);
    const int z = (int)(t / Y);
    const int i = x + 1, j = y + 1, k = z + 1;
    double s = 0.0;
    if (i == 1) s += bc[shell_slot(0, j, k, nx, ny, nz)];
    if (i == nx - 2) s += bc[shell_slot(nx - 1, j, k, nx, ny, nz)];
    if (j == 1) s += bc[shell_slot(i, 0, k, nx, ny, nz)];
    if (j == ny - 2) s += bc[shell_slot(i, ny - 1, k, nx, ny, nz)];
    if (k == 1) s += bc[shell_slot(i, j, 0, nx, ny, nz)];
    if (k == nz - 2) s += bc[shell_slot(i, j, nz - 1, nx, ny, nz)];
    f[p] = c * s;
  }
}

// dense interior index of a pitched node index (every charge node is interior)
__device__ __forceinline__ long long dense_of(int lin, int nx, int nxp, int ny) {
  const int i = lin % nxp;
  const int t = lin / nxp;
  const int j = t % ny, k = t / ny;
  return ((long long)(k - 1) * (ny - 2) + (j - 1)) * (nx - 2) + (i - 1);
}

// f += rho at the trilinear charge nodes (distinct nodes: no collisions)
__global__ void dir_charges_kernel(double* f, const int* q_idx, const double* q_rho,
                                   const int* nq_dev, int nx, int nxp, int ny) {
  const int nq = *nq_dev;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nq; e += gridDim.x * blockDim.x)
    f[dense_of(q_idx[e], nx, nxp, ny)] += q_rho[e];
}

// In-place transform of every line along one axis: v <- S_N v.  A block
// takes kTL lines: for the x axis kTL consecutive lines (rows), else kTL
// consecutive x of one plane.  Element (line l, index k) of the tile sits
// at base + l * sl + k * sk.  The lines are staged in LDS as T[k][l]; thread
// j accumulates output j of all kTL lines, reading row k of S_N (coalesced
// over j) and broadcasting T[k][0..kTL-1].
__global__ __launch_bounds__(512) void dst_lines_kernel(double* u, const double* S, int N,
                                                        int axis, int X, int Y, int Z) {
  extern __shared__ __align__(16) double tile[];  // [N][kTS]
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  long long base;
  int valid;
  long long sl, sk;
  if (axis == 0) {
    const long long l0 = (long long)blockIdx.x * kTL;
    valid = (int)min((long long)kTL, (long long)Y * Z - l0);
    base = l0 * X;
    sl = X;
    sk = 1;
  } else {
    const int ntx = (X + kTL - 1) / kTL;
    const int o = blockIdx.x / ntx;  // z for the y axis, y for the z axis
    const int x0 = (blockIdx.x - o * ntx) * kTL;
    valid = min(kTL, X - x0);
    sl = 1;
    if (axis == 1) {
      base = (long long)o * Y * X + x0;
      sk = X;
    } else {
      base = (long long)o * X + x0;
      sk = (long long)X * Y;
    }
  }
  const int ne = N * kTL;
  // stage: consecutive threads take consecutive addresses
  for (int e = tid; e < ne; e += nthr) {
    int l, k;
    if (sk == 1) {
      l = e / N;
      k = e - l * N;
    } else {
      k = e / kTL;
      l = e - k * kTL;
    }
    tile[k * kTS + l] = (l < valid) ? u[base + l * sl + k * sk] : 0.0;
  }
  __syncthreads();
  const int j = tid;
  double acc[kTL];
#pragma unroll
  for (int l = 0; l < kTL; ++l) acc[l] = 0.0;
  if (j < N) {
    for (int k = 0; k < N; ++k) {
      const double s = S[(long long)k * N + j];
      const double2* row = reinterpret_cast<const double2*>(tile + k * kTS);
#pragma unroll
      for (int q = 0; q < kTL / 2; ++q) {
        const double2 v = row[q];
        acc[2 * q] = fma(s, v.x, acc[2 * q]);
        acc[2 * q + 1] = fma(s, v.y, acc[2 * q + 1]);
      }
    }
  }
  __syncthreads();
  if (j < N) {
#pragma unroll
    for (int l = 0; l < kTL; ++l) tile[j * kTS + l] = acc[l];
  }
  __syncthreads();
  for (int e = tid; e < ne; e += nthr) {
    int l, k;
    if (sk == 1) {
      l = e / N;
      k = e - l * N;
    } else {
      k = e / kTL;
      l = e - k * kTL;
    }
    if (l < valid) u[base + l * sl + k * sk] = tile[k * kTS + l];
  }
}

// transformed right-hand side -> transformed solution, with the inverse
// transforms' normalisation folded in
__global__ void dir_scale_kernel(double* u, const double* ex, const double* ey, const double* ez,
                                 int X, int Y, int Z, double c, double norm) {
  const long long n = (long long)X * Y * Z;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(p % X);
    const long long t = p / X;
    const int y = (int)(t % Y);
    const int z = (int)(t / Y);
    u[p] = u[p] * (norm / (c * (ex[x] + ey[y] + ez[z])));
  }
}

// S = sum over charge nodes of q u (fixed-order tree in one block)
__global__ __launch_bounds__(1024) void dir_energy_kernel(const double* u, const int* q_idx,
                                                          const double* q_val, const int* nq_dev,
                                                          int nx, int nxp, int ny, double* slot) {
  __shared__ double part[1024];
  const int nq = *nq_dev;
  double s = 0.0;
  for (int e = threadIdx.x; e < nq; e += 1024) s += q_val[e] * u[dense_of(q_idx[e], nx, nxp, ny)];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *slot = part[0];
}

// out[nz][ny][nx] = beta * out + gamma * (u inside, Dirichlet data on the shell)
__global__ void dir_field_out_kernel(double* out, const double* u, const double* bc, int nx,
                                     int ny, int nz, double beta, double gamma) {
  const long long n = (long long)nx * ny * nz;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(p % nx);
    const long long t = p / nx;
    const int j = (int)(t % ny);
    const int k = (int)(t / ny);
    const bool shell = i == 0 || j == 0 || k == 0 || i == nx - 1 || j == ny - 1 || k == nz - 1;
    const double v =
        shell ? bc[shell_slot(i, j, k, nx, ny, nz)]
              : u[((long long)(k - 1) * (ny - 2) + (j - 1)) * (nx - 2) + (i - 1)];
    out[p] = (beta != 0.0) ? beta * out[p] + gamma * v : gamma * v;
  }
}

unsigned grid_for(long long n) {
  long long b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

}  // namespace

size_t direct_poisson_bytes(int nx, int ny, int nz) {
  const size_t X = nx - 2, Y = ny - 2, Z = nz - 2;
  return 8 * (X * Y * Z + X * X + Y * Y + Z * Z + X + Y + Z);
}

hipError_t launch_direct_poisson(const DirectPoissonArgs& a, hipStream_t st) {
  const int X = a.nx - 2, Y = a.ny - 2, Z = a.nz - 2;
  if (X < 1 || Y < 1 || Z < 1 || X > 512 || Y > 512 || Z > 512) return hipErrorInvalidValue;
  double* u = a.work;
  double* Sx = u + (size_t)X * Y * Z;
  double* Sy = Sx + (size_t)X * X;
  double* Sz = Sy + (size_t)Y * Y;
  double* ex = Sz + (size_t)Z * Z;
  double* ey = ex + X;
  double* ez = ey + Y;
  const int Ns[3] = {X, Y, Z};
  double* Ss[3] = {Sx, Sy, Sz};
  double* es[3] = {ex, ey, ez};
  for (int d = 0; d < 3; ++d) {
    const long long nn = (long long)Ns[d] * Ns[d];
    hipLaunchKernelGGL(dst_matrix_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st,
                       Ss[d], es[d], Ns[d]);
  }
  const long long n = (long long)X * Y * Z;
  const double c = a.eps / (a.h * a.h);
  hipLaunchKernelGGL(dir_rhs_kernel, dim3(grid_for(n)), dim3(256), 0, st, u, a.bc, a.nx, a.ny,
                     a.nz, c);
  hipLaunchKernelGGL(dir_charges_kernel, dim3((unsigned)((a.cap + 255) / 256 > 0 ? (a.cap + 255) / 256 : 1)),
                     dim3(256), 0, st, u, a.q_idx, a.q_rho, a.nq_dev, a.nx, a.nxp, a.ny);
  auto transform = [&](int axis) -> hipError_t {
    const int N = Ns[axis];
    const unsigned blocks = axis == 0 ? (unsigned)(((long long)Y * Z + kTL - 1) / kTL)
                                      : (unsigned)((axis == 1 ? Z : Y) * ((X + kTL - 1) / kTL));
    const int threads = ((N + 63) / 64) * 64;
    const size_t lds = sizeof(double) * (size_t)N * kTS;
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(dst_lines_kernel),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(dst_lines_kernel, dim3(blocks), dim3(threads), lds, st, u, Ss[axis], N,
                       axis, X, Y, Z);
    return hipGetLastError();
  };
  for (int axis = 0; axis < 3; ++axis) {
    hipError_t e = transform(axis);
    if (e != hipSuccess) return e;
  }
  const double norm = 8.0 / ((double)(X + 1) * (double)(Y + 1) * (double)(Z + 1));
  hipLaunchKernelGGL(dir_scale_kernel, dim3(grid_for(n)), dim3(256), 0, st, u, ex, ey, ez, X, Y,
                     Z, c, norm);
  for (int axis = 2; axis >= 0; --axis) {
    hipError_t e = transform(axis);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(dir_energy_kernel, dim3(1), dim3(1024), 0, st, u, a.q_idx, a.q_val, a.nq_dev,
                     a.nx, a.nxp, a.ny, a.slot);
  return hipGetLastError();
}

hipError_t launch_direct_field_out(double* out, const double* u, const double* bc, int nx, int ny,
                                   int nz, double beta, double gamma, hipStream_t st) {
  const long long n = (long long)nx * ny * nz;
  hipLaunchKernelGGL(dir_field_out_kernel, dim3(grid_for(n)), dim3(256), 0, st, out, u, bc, nx,
                     ny, nz, beta, gamma);
  return hipGetLastError();
}

}  // namespace npb
