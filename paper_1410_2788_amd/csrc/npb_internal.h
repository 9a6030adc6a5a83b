// Internal declarations of the NPB HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace npb {

// ---------------------------------------------------------------------------
// Arguments of one implicit line sweep (one of the 1-D sub-steps of the
// LOD / AOS splitting).  The face coefficient of the row for node i is
// r * eps(i +- 1/2), r = tau / h^2, with eps at a half point chosen from the
// two nodal solute flags (both solvent, mixed = harmonic mean, both solute).
template <typename T>
struct SweepArgs {
  T* u;                   // field, [nz][ny][nx]; read, and written in place
  T* acc;                 // additive-splitting accumulator (AOS modes)
  const uint8_t* mask;    // 1 = solute node; nullptr = uniform medium
  int nx, ny, nz;
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
  // per (chunk, line) face class of this direction's launch shape: 0 = every
  // face of the chunk solvent-solvent, 2 = every face solute-solute, 1 =
  // mixed; nullptr for the uniform medium (all chunks uniform)
  const uint8_t* ccls;
  // geometry of the launch
  int M;                  // rows per chunk (compile-time in the kernel)
  int P;                  // chunks per line
  int LW;                 // y/z: lines per block; x: lines per block
  int S;                  // x: LDS row stride (elements)
};

enum SweepMode { MODE_INPLACE = 0, MODE_AOS_FIRST = 1, MODE_AOS_ADD = 2, MODE_AOS_FINISH = 3 };

// Chunk lengths compiled into the sweep kernels.
constexpr int kChunkChoices[] = {4, 8, 12, 16, 20, 24, 32};

struct LaunchShape {
  int M, P, LW, threads, blocks;
  size_t lds;
};

// Elimination constants of a chunk whose M+1 faces all carry the same
// coefficient re (rows a = c = -re, b = 1 + 2 re): pivot reciprocals,
// normalised couplings and the coefficients of the chunk's reduced rows.
// Index t = 0: solvent chunks (or the uniform medium), t = 1: solute chunks.
constexpr int kMaxChunk = 32;
template <typename A>
struct ChunkTab {
  A inv[2][kMaxChunk];
  A ga[2][kMaxChunk];
  A al[2][kMaxChunk];
  A ap[2], gp[2], re[2];
};

// number of chunks of a line per direction for a launch shape (x uses the
// padded power-of-two count)
inline int chunk_count(const LaunchShape& s) { return s.P; }

// Pick chunk length / chunk count and the block shape for a line length.
LaunchShape plan_x(int nx, int ny, int nz, bool fp64, bool aos, bool uniform);
LaunchShape plan_yz(int n_along, int n_lines, bool fp64);

// T = storage type of the field, A = arithmetic type of the line solves
template <typename T, typename A>
hipError_t launch_sweep_x(const SweepArgs<T>& a, const LaunchShape& s, hipStream_t st);
template <typename T, typename A>
hipError_t launch_sweep_yz(const SweepArgs<T>& a, int dir, const LaunchShape& s, hipStream_t st);

// ---------------------------------------------------------------------------
// setup

struct SetupArgs {
  int nx, ny, nz;
  double h, ox, oy, oz;
  int n_atoms;
  const double* atoms;    // [5][n_atoms]: x, y, z, q, radius
};

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st);
hipError_t launch_mask_raster(const SetupArgs& a, uint8_t* mask, hipStream_t st);
hipError_t launch_stencil(const SetupArgs& a, int* key, int* id, double* val, int* err,
                          hipStream_t st);
// Stable LSD radix sort of (key, id) pairs by key; n items, keys < key_limit.
// Result in (key_a, id_a); (key_b, id_b) are scratch.  hist holds at least
// 256 * ceil(n/256) ints.
hipError_t radix_sort_pairs(int* key_a, int* id_a, int* key_b, int* id_b, int* hist,
                            int n, long long key_limit, hipStream_t st);
hipError_t launch_exclusive_scan(int* data, int n, int* total, hipStream_t st);
hipError_t launch_merge_charges(const int* key, const int* id, const double* val, int* heads,
                                int n, int* nq_dev, int* q_idx, double* q_val,
                                double* q_rho, double rho_pref, hipStream_t st);
hipError_t launch_line_ptr(const int* sorted_keys, const int* n_dev, int cap, int n_lines,
                           int keys_per_line, int* ptr, hipStream_t st);
hipError_t launch_axis_keys(const int* q_idx, const int* nq_dev, int cap, int nx, int ny,
                            int nz, int axis, int* key, int* id, hipStream_t st);
hipError_t launch_gather_entries(const int* id, const int* nq_dev, int cap, const int* q_idx,
                                 const double* q_rho, int* lin_out, double* rho_out,
                                 hipStream_t st);
hipError_t launch_boundary(const SetupArgs& a, double eps, double kappa, double lB, double* bc,
                           hipStream_t st);
// chunk classes of direction dir (0 = x, 1 = y, 2 = z) for chunks of M rows,
// P per line; out[p * n_lines + line]
hipError_t launch_chunk_classes(const uint8_t* mask, int nx, int ny, int nz, int dir, int M, int P,
                                uint8_t* out, hipStream_t st);

// ---------------------------------------------------------------------------
// field / energy helpers

template <typename T>
hipError_t launch_field_init(T* u, const double* bc, int nx, int ny, int nz, hipStream_t st);
template <typename T>
hipError_t launch_energy(const T* u, const int* q_idx, const double* q_val, const int* nq_dev,
                         int cap, double* slot, hipStream_t st);
template <typename T>
hipError_t launch_field_out(double* out, const T* u, size_t n, double beta, double gamma,
                            hipStream_t st);
hipError_t launch_combine(const double* S, double kT, int richardson, int vacuum,
                          double* res, hipStream_t st);

// number of nodes on the outer shell of an nx*ny*nz grid
inline long long shell_count(int nx, int ny, int nz) {
  return (long long)nx * ny * nz - (long long)(nx - 2) * (ny - 2) * (nz - 2);
}

}  // namespace npb
