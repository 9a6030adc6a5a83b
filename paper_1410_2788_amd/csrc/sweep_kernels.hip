// Implicit line sweeps of the LOD / AOS splitting on CDNA4 (gfx950).
//
// Each sweep solves, on every interior grid line along one axis,
//     -re(i-1/2) v[i-1] + (1 + re(i-1/2) + re(i+1/2)) v[i] - re(i+1/2) v[i+1] = s[i]
// with re = (tau/h^2) eps at the half points and Dirichlet values at both
// ends: the implicit-Euler 1-D sub-steps of the paper (Sec. 3.1, Eqs.
// (LODIE1_2)-(LODIE1_4) with the central differences of Eq.
// (SpatialOperators); Sec. 3.2, Eqs. (AOSIE1_2)-(AOSIE1_4) and
// (AOSIE2_2)-(AOSIE2_4) with 4 tau).  The matrices are strictly diagonally
// dominant, so elimination needs no pivoting.
//
// Line solver: a partition method with register-resident chunks.  A line of
// n_int unknowns is cut into P chunks of M rows; each chunk lives in the
// registers of one lane.  A lane eliminates its chunk down to two rows that
// couple only to the neighbouring chunks' end unknowns; the 2P-row reduced
// tridiagonal system (a Schur complement, hence still diagonally dominant)
// is solved through LDS, and each lane back-substitutes its interior.  HBM
// sees one read and one write of the field per sweep (plus the 1-byte
// solute mask), which is what bounds these kernels.
//
//   x sweep : lines are contiguous in memory.  A block stages L whole rows
//             in LDS with 16-byte loads, lanes take (line, chunk) pairs.
//   y/z sweep: each lane holds the chunk of V adjacent x lines and moves
//             them with one 16-byte (FP32: V = 4, FP64: V = 2) access per
//             node row; LW lanes cover LW*V consecutive x.
//
// Fused pointwise work: the exact sinh flow (Eq. (ana3)), the trilinear
// source add, and the AOS accumulation happen on values already in
// registers or LDS, so they add no HBM traffic beyond the accumulator.
//
// T is the storage type of the field, A the arithmetic type of the solve.
#include <hip/hip_ext.h>

#include <algorithm>
#include <type_traits>

#include "npb_internal.h"

namespace npb {

// ---------------------------------------------------------------------------
// Exact flow of alpha w' = -kbar^2 sinh(w) over one step (Eq. (ana3)).  With
// k = exp(-2 theta), kA = 1 + k, kB = 1 - k, E = exp(-|u|), m = 1 - E, the
// printed ratio divided by cosh(theta) becomes
//   (kA + kB E) / (kB + kA E) = 1 + 2k m / (kB + kA E),
// so  w = sign(u) * log1p(2k m / (kB + kA E)): odd in u, no overflow.
// FP32 uses the hardware exp2/log2 (1 + x >= 1 is a normal number, so
// the log needs none of a library log's range handling; the rounding of
// 1 + x dominates its error either way); FP64 the series-based exp_neg and
// log1p_nonneg (m = 1 - E then loses relative accuracy as |u| -> 0 but keeps
// an absolute error of ~1e-16, which is what the field sees).
__device__ __forceinline__ float sinh_flow(float u, float kA, float kB) {
  const float E = __expf(-fabsf(u));
  const float m = 1.0f - E;
  const float x = (kA - kB) * m * __builtin_amdgcn_rcpf(fmaf(kA, E, kB));
  return copysignf(__builtin_amdgcn_logf(1.0f + x) * 0.693147180559945f, u);
}
__device__ __forceinline__ double sinh_flow(double u, double kA, double kB) {
  const double E = exp_neg(-fabs(u));
  const double m = 1.0 - E;
  return copysign(log1p_nonneg((kA - kB) * m * rcp_newton(fma(kA, E, kB))), u);
}

template <typename T>
__device__ __forceinline__ T pick3(int s, T r0, T r1, T r2) {
  return s == 0 ? r0 : (s == 1 ? r1 : r2);
}

// Reciprocal of a pivot (pivots are positive and of order one or larger:
// diagonally dominant rows with a unit identity part).  FP32: the hardware
// reciprocal (1 ulp).  FP64: the hardware estimate refined by two Newton
// steps.
__device__ __forceinline__ float rcp_pivot(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_pivot(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// ---------------------------------------------------------------------------
// Line systems and their precision.
//
// Every row of a line system (I - tau delta^2) v = s reads
//   -alpha v_{k-1} + (ell + alpha + gamma) v_k - gamma v_{k+1} = d_k,
// alpha, gamma = r * eps at the row's two faces and ell >= 1 the row-sum
// defect ("leak"): 1 from the identity, plus the coupling to a Dirichlet
// neighbour moved to the right-hand side.  The diagonal is up to a few
// thousand while the solution depends on its unit part: formed as one FP32
// number, every pivot of a line carries the same rounding at every step, a
// fixed bias of the discrete operator (~1e-5 of the energy at production
// sizes) rather than noise.  So the eliminations below never form a
// diagonal: they carry the leak of each (partially eliminated) row as its
// own non-negative quantity, the complement technique of the GTH algorithm
// for M-matrices, and every pivot is a sum of non-negative terms.  Rounding
// then stays relative to each quantity, and FP32 arithmetic gives the
// accuracy of FP64 pivots.
//
// Chunk elimination.  Rows k = 0..M-1 of one chunk are global interior rows
// g = g0 + k; reF[k] is r * eps at the face between rows k-1 and k.  The
// first interior row (g = 0) has taken its left Dirichlet value into d; the
// last one (local index kR = nint-1-g0) takes gR here.  Rows past it are
// identity rows with zero right-hand side (d is 0 there on entry).  Rows
// 1..M-1 are eliminated forward into
//   x_k = d[k] + lam_k x_0 + gam_k x_{k+1},   al[k] = -lam_k, ga[k] = -gam_k,
// with leak tau_k = 1 - lam_k - gam_k >= 0:
//   den_k = ell_k + gamma_k + alpha_k (tau_{k-1} + lam_{k-1}),
//   lam_k = alpha_k lam_{k-1} / den_k,  gam_k = gamma_k / den_k,
//   tau_k = (ell_k + alpha_k tau_{k-1}) / den_k   (lam_0 = 1, tau_0 = 0).
// Back substitution gives x_1 = D + P x_0 + G x_{M-1} with G = prod gam_k
// and leak s = 1 - P - G = sum_j tau_j prod_{i<j} gam_i (j, i = 1..M-2),
// accumulated forward.  Reduced rows (alpha, gamma, ell, d):
//   rf, row of x_0:     (alpha_0, gamma_0 G, ell_0 + gamma_0 s, d_0 + gamma_0 D)
//   rl, row of x_{M-1}: (lam_{M-1}, gam_{M-1}, tau_{M-1}, d[M-1])
template <typename A>
struct RRow {
  A a, c, l, d;  // alpha, gamma, leak, right-hand side
};

template <typename A, int M>
__device__ __forceinline__ void chunk_eliminate(A (&d)[M], A (&al)[M], A (&ga)[M], RRow<A>& rf,
                                                RRow<A>& rl, const A (&reF)[M + 1], bool first,
                                                int kR, A gR) {
  static_assert(M >= 4, "chunks of at least four rows");
  // the coefficients of row k
  auto row = [&](int k, A& ak, A& ck, A& lk) {
    const bool real = k <= kR;
    ak = (real && !(k == 0 && first)) ? reF[k] : A(0);
    ck = (k < kR) ? reF[k + 1] : A(0);
    lk = A(1);
    if (real && k == 0 && first) lk += reF[0];
    if (k == kR) {
      lk += reF[k + 1];
      d[k] = fma(reF[k + 1], gR, d[k]);
    }
  };
  A a0, c0, l0;
  row(0, a0, c0, l0);
  if constexpr (sizeof(A) == 8) {
    // FP64 arithmetic resolves the unit part of a diagonal directly: the
    // textbook recurrences (fewer live registers), with the reduced rows'
    // leaks taken as B + A + C at the end
#pragma unroll
    for (int k = 1; k < M; ++k) {
      A ak, ck, lk;
      row(k, ak, ck, lk);
      const A bk = lk + (ak + ck);
      const A inv = rcp_pivot(k == 1 ? bk : fma(ak, ga[k - 1], bk));
      al[k] = k == 1 ? -ak * inv : ak * al[k - 1] * inv;
      ga[k] = -ck * inv;
      d[k] = (k == 1 ? d[k] : fma(ak, d[k - 1], d[k])) * inv;
    }
    rl = RRow<A>{-al[M - 1], -ga[M - 1], A(1) + al[M - 1] + ga[M - 1], d[M - 1]};
    // x_1 = dp - ap x_0 - gp x_{M-1}
    A ap = al[M - 2], gp = ga[M - 2], dp = d[M - 2];
#pragma unroll
    for (int k = M - 3; k >= 1; --k) {
      ap = fma(-ga[k], ap, al[k]);
      gp = -ga[k] * gp;
      dp = fma(-ga[k], dp, d[k]);
    }
    // row 0: -a0 x_prev + (l0 + a0 + c0) x_0 - c0 x_1 = d_0
    const A bf = fma(c0, ap, l0 + (a0 + c0));
    const A cf = c0 * gp;  // = -C of the reduced row
    rf = RRow<A>{a0, -cf, bf - a0 + cf, fma(c0, dp, d[0])};
    return;
  }
  A lam = A(1), tau = A(0);
  A s = A(0), G = A(1);  // leak and far coupling of x_1
#pragma unroll
  for (int k = 1; k < M; ++k) {
    A ak, ck, lk;
    row(k, ak, ck, lk);
    const A inv = rcp_pivot(fma(ak, tau + lam, lk + ck));
    lam = ak * lam * inv;
    const A gam = ck * inv;
    tau = fma(ak, tau, lk) * inv;
    d[k] = (k == 1 ? d[k] : fma(ak, d[k - 1], d[k])) * inv;
    al[k] = -lam;
    ga[k] = -gam;
    if (k <= M - 2) {
      s = fma(tau, G, s);
      G *= gam;
    }
    if (k == M - 1) rl = RRow<A>{lam, gam, tau, d[M - 1]};
  }
  A dp = d[M - 2];
#pragma unroll
  for (int k = M - 3; k >= 1; --k) dp = fma(-ga[k], dp, d[k]);
  rf = RRow<A>{a0, c0 * G, fma(c0, s, l0), fma(c0, dp, d[0])};
}

// back substitution once x_0 (xf) and x_{M-1} (xl) are known; d becomes x
template <typename A, int M>
__device__ __forceinline__ void chunk_finish(A (&d)[M], const A (&al)[M], const A (&ga)[M],
                                             A xf, A xl) {
  d[M - 1] = xl;
#pragma unroll
  for (int k = M - 2; k >= 1; --k) d[k] = fma(-ga[k], d[k + 1], fma(-al[k], xf, d[k]));
  d[0] = xf;
}

// Chunk tables are read through the constant address space with a
// wave-uniform row index, so that they come in by scalar loads rather than
// per-lane flat loads (which wait on both memory counters).
template <typename A>
using ConstTab = const __attribute__((address_space(4))) ChunkTab<A>;

// Crank-Nicolson right-hand side (Eqs. (LODCN1_2)-(LODCN1_4)): the chunk's
// rows d[0..M-1] become (1 + r delta^2) s with the implicit side's face
// coefficients reF (face k between local rows k-1 and k), left / right the
// values next to the chunk and gR the Dirichlet value after local row kR
// (the line's last interior row when it lies in the chunk).  Rows past kR
// stay zero.  The differences are formed first, so a large coefficient
// multiplies only the variation of s.
template <typename A, int M>
__device__ __forceinline__ void cn_rhs(A (&d)[M], const A (&reF)[M + 1], A left, A right, int kR,
                                       A gR) {
  A prev = left;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const A cur = d[k];
    const A nxt = (k == kR) ? gR : (k + 1 < M ? d[k + 1] : right);
    d[k] = (k <= kR) ? fma(reF[k], prev - cur, fma(reF[k + 1], nxt - cur, cur)) : A(0);
    prev = cur;
  }
}

// the same for a chunk of uniform faces re with every row interior
template <typename A, int M>
__device__ __forceinline__ void cn_rhs_uniform(A (&d)[M], A re, A left, A right) {
  A prev = left;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const A cur = d[k];
    const A nxt = k + 1 < M ? d[k + 1] : right;
    d[k] = fma(re, (prev - cur) + (nxt - cur), cur);
    prev = cur;
  }
}

// Crank-Nicolson explicit half applied to a line held in LDS, before the
// sources are added (additive schemes, whose source stays outside the
// explicit half: Eqs. (AOSCN1_2)-(AOSCN2_4); Sec. 3.3).  Node r of the line
// sits at v[r * vs] with solute flag f[r * fs]; the lane's rows 1+g0 ..
// g0+M that are interior become (1 + r delta^2) v, the face coefficient
// chosen from the two flags as in the implicit rows (uniform medium: reu;
// face rule by location, fm: bit 1 of the lower node's flag).
// The new values are formed in registers and written after a block
// barrier, so every lane reads the unchanged line; every thread of the
// block must call this.
template <typename A, int M>
__device__ __forceinline__ void cn_tile_rows(A* v, int vs, const uint8_t* f, int fs, int g0,
                                             int nint, bool valid, bool uniform, bool fm, A re0,
                                             A re1, A re2, A reu) {
  A e[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const int r = 1 + g0 + k;
    e[k] = A(0);
    if (valid && r <= nint) {
      const A c = v[r * vs], l = v[(r - 1) * vs], rt = v[(r + 1) * vs];
      const int fa = f[(r - 1) * fs], fb = f[r * fs];
      const A fl = uniform ? reu : pick3(fm ? (fa & 2) : fa + fb, re0, re1, re2);
      const A fr = uniform ? reu : pick3(fm ? (fb & 2) : fb + (int)f[(r + 1) * fs], re0, re1, re2);
      e[k] = fma(fl, l - c, fma(fr, rt - c, c));
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const int r = 1 + g0 + k;
    if (valid && r <= nint) v[r * vs] = e[k];
  }
  __syncthreads();
}

// Uniform chunks (every face coefficient equal to re, leak 1): the pivots,
// couplings and reduced-row coefficients are the tabulated constants of
// ChunkTab (computed by the same recurrences in FP64), so only the
// right-hand side is eliminated.  tb: the table, t: its row (solvent /
// solute).  The first chunk of a line has its left Dirichlet coupling in
// the leak of row 0.
//
// A line's last chunk (tail: its last real row kt = (nint - 1) mod M, the
// same for every line of the block, 1 <= kt <= M - 1, not also the first
// chunk) takes the same path.  Row kt's right face goes to the Dirichlet
// node gR: the caller has added re gR to that row's value, and row kt's
// gamma drops to zero while its pivot stays (leak 1 + re and gamma 0 sum to
// the same diagonal).  For kt = M - 1 that changes only the reduced row of
// x_{M-1}: gamma 0, leak rl_l + rl_c.  For kt < M - 1 the rows past kt are
// identity rows: the reduced row of x_{M-1} is the identity (decoupled; its
// value and the rows past kt are never stored), the reduced row of x_0 has
// gamma 0 and the tabulated leak rf_lt, and the recurrences that run down
// through row kt drop its coupling to row kt + 1.  kt is block-uniform, so
// the row test is a scalar branch.
template <typename A, int M, typename TB>
__device__ __forceinline__ void fast_eliminate(A (&d)[M], const TB& tb, int t, bool first,
                                               bool tail, int kt, RRow<A>& rf, RRow<A>& rl) {
  const A re = tb.re[t];
  d[1] = d[1] * tb.inv[t][1];
#pragma unroll
  for (int k = 2; k < M; ++k) d[k] = fma(re, d[k - 1], d[k]) * tb.inv[t][k];
  const bool tail_in = tail && kt < M - 1;
  rl = RRow<A>{tail_in ? A(0) : tb.rl_a[t], tail ? A(0) : tb.rl_c[t],
               tail_in ? A(1) : (tail ? tb.rl_l[t] + tb.rl_c[t] : tb.rl_l[t]), d[M - 1]};
  A dp = d[M - 2];
#pragma unroll
  for (int k = M - 3; k >= 1; --k) {
    // row kt of a tail chunk takes nothing from row kt + 1 (a select of the
    // value, not of the table coefficient: one VALU op)
    dp = fma(-tb.ga[t][k], (tail && k == kt) ? A(0) : dp, d[k]);
  }
  const A lf = tail_in ? tb.rf_lt[t] : tb.rf_l[t];
  rf = RRow<A>{first ? A(0) : re, tail_in ? A(0) : tb.rf_c[t], first ? lf + re : lf,
               fma(re, dp, d[0])};
}

// back substitution of a uniform chunk (a tail chunk as in fast_eliminate:
// row kt takes nothing from row kt + 1)
template <typename A, int M, typename Ptr>
__device__ __forceinline__ void fast_finish(A (&d)[M], Ptr ga, Ptr al, A xf, A xl, bool tail,
                                            int kt) {
  d[M - 1] = xl;
#pragma unroll
  for (int k = M - 2; k >= 1; --k) {
    d[k] = fma(-ga[k], (tail && k == kt) ? A(0) : d[k + 1], fma(-al[k], xf, d[k]));
  }
  d[0] = xf;
}

// Reduced systems in LDS: entry (line l, row r, coefficient c) at
// R[r (4 rs + 1) + c rs + l] (red_at), c = alpha, gamma, leak, d;
// rs = lines + 1.  The lanes of one wave that write them (different lines,
// same row) touch distinct banks, and so do the lanes that read them for the
// cyclic reduction (one line's rows 2p, p = 0..15, 2p (4 rs + 1) apart: an
// odd row stride spreads them over the banks).  Row 2p is the first row of
// chunk p, row 2p+1 its last;
// the 2P rows of a line form a tridiagonal system in the form above, whose
// first alpha and last gamma are zero.  Both solvers keep it in that form.
//
// x sweeps (and FP32 y/z sweeps with P a power of two): parallel cyclic
// reduction with the P lanes of a line side by side in one wave (lane t:
// line t / P, rows 2p and 2p+1 of p = t % P).  Each step eliminates a row's
// couplings to the rows at distance d using those rows (from the neighbour
// lanes): with
// B = leak + alpha + gamma of each row, k1 = alpha_r / B_up, k2 = gamma_r / B_dn,
//   alpha' = alpha_up k1,  gamma' = gamma_dn k2,
//   leak'  = leak_r + leak_up k1 + leak_dn k2,  d' = d_r + d_up k1 + d_dn k2,
// after which the row couples to the rows at distance 2d; after steps
// d = 1, 2, ..., P every row stands alone and x_r = d_r / B_r.  Rows outside
// the system act as identity rows (their coupling is already zero).
__host__ __device__ constexpr int red_at(int r, int c, int rs) { return r * (4 * rs + 1) + c * rs; }
// elements of the reduced systems of a block
__host__ __device__ constexpr int red_size(int P, int rs) { return 2 * P * (4 * rs + 1); }
template <typename A>
__device__ __forceinline__ RRow<A> rrow_identity() {
  return RRow<A>{A(0), A(0), A(1), A(0)};
}

template <typename A>
__device__ __forceinline__ A rrow_b(const RRow<A>& r) {
  return r.l + (r.a + r.c);
}

template <typename A>
__device__ __forceinline__ RRow<A> pcr_combine(const RRow<A>& r, const RRow<A>& up,
                                               const RRow<A>& dn) {
  const A k1 = r.a * rcp_pivot(rrow_b(up));
  const A k2 = r.c * rcp_pivot(rrow_b(dn));
  return RRow<A>{up.a * k1, dn.c * k2, fma(up.l, k1, fma(dn.l, k2, r.l)),
                 fma(up.d, k1, fma(dn.d, k2, r.d))};
}

template <typename A>
__device__ __forceinline__ RRow<A> shfl_row_up(const RRow<A>& r, int delta, int width) {
  return RRow<A>{__shfl_up(r.a, delta, width), __shfl_up(r.c, delta, width),
                 __shfl_up(r.l, delta, width), __shfl_up(r.d, delta, width)};
}
template <typename A>
__device__ __forceinline__ RRow<A> shfl_row_down(const RRow<A>& r, int delta, int width) {
  return RRow<A>{__shfl_down(r.a, delta, width), __shfl_down(r.c, delta, width),
                 __shfl_down(r.l, delta, width), __shfl_down(r.d, delta, width)};
}

// Neighbour exchange inside 16-lane rows by DPP row shifts (one VALU move a
// 32-bit word): kUp takes lane i - D's value, else lane i + D's; a lane whose
// source lies outside its row reads zero.  A zero row in place of the
// identity is exact wherever it can reach a result: a row whose neighbour
// at the current distance lies before the start (after the end) of its
// line has alpha (gamma) exactly zero, so k1 (k2) = 0 * 0 and the zero row
// drops out; by induction over the steps this holds from the first alpha and
// last gamma of the system, which are zero.  A line that fills a whole row
// (P = 16) therefore needs no selects; smaller P select the identity for the
// lanes whose source belongs to the neighbouring line.
template <int D, bool kUp>
__device__ __forceinline__ float dpp_shift(float v) {
  constexpr int ctl = (kUp ? 0x110 : 0x100) | D;  // row_shr:D / row_shl:D
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctl, 0xf, 0xf, true));
}
template <int D, bool kUp>
__device__ __forceinline__ double dpp_shift(double v) {
  constexpr int ctl = (kUp ? 0x110 : 0x100) | D;
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), ctl, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctl, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int D, bool kUp, typename A>
__device__ __forceinline__ RRow<A> dpp_row(const RRow<A>& r) {
  return RRow<A>{dpp_shift<D, kUp>(r.a), dpp_shift<D, kUp>(r.c), dpp_shift<D, kUp>(r.l),
                 dpp_shift<D, kUp>(r.d)};
}
// pcr_combine with the neighbours' diagonal reciprocals given (iu, id)
template <typename A>
__device__ __forceinline__ RRow<A> pcr_combine_r(const RRow<A>& r, const RRow<A>& up, A iu,
                                                 const RRow<A>& dn, A id) {
  const A k1 = r.a * iu;
  const A k2 = r.c * id;
  return RRow<A>{up.a * k1, dn.c * k2, fma(up.l, k1, fma(dn.l, k2, r.l)),
                 fma(up.d, k1, fma(dn.d, k2, r.d))};
}
// One reduction step at lane distance E, E a constant, over one row per
// lane: each lane forms the reciprocal of its row's diagonal and passes it
// on with the row.  kFull: the line fills the whole 16-lane row (zero rows
// from outside it); else lanes whose source lies outside the line take the
// identity row.
template <int E, bool kFull, typename A>
__device__ __forceinline__ void pcr_step_dpp(RRow<A>& r, int p, int P) {
  if (!kFull && E >= P) return;
  const A b = rcp_pivot(rrow_b(r));
  RRow<A> u = dpp_row<E, true>(r), d = dpp_row<E, false>(r);
  A iu = dpp_shift<E, true>(b), id = dpp_shift<E, false>(b);
  if constexpr (!kFull) {
    if (p < E) {
      u = rrow_identity<A>();
      iu = A(1);
    }
    if (p + E >= P) {
      d = rrow_identity<A>();
      id = A(1);
    }
  }
  r = pcr_combine_r(r, u, iu, d, id);
}

// Reduced system of a line with its P <= 16 lanes in one 16-lane row (lane
// p: rows 2p and 2p+1).  One step of cyclic reduction first: the odd row
// 2p+1 takes in the even rows 2p (its own lane) and 2p+2 (lane p+1), after
// which the odd rows alone form a tridiagonal system, one row per lane,
// solved by the DPP steps above.  Each even row then follows from its
// original equation and the odd neighbours:
//   x_{2p} = (d_{2p} + alpha_{2p} x_{2p-1} + gamma_{2p} x_{2p+1}) / B_{2p}.
template <bool kFull, typename A>
__device__ __forceinline__ void pcr_dpp(A* R, int rs, int p, int P) {
  auto get = [&](int r) {
    return RRow<A>{R[red_at(r, 0, rs)], R[red_at(r, 1, rs)], R[red_at(r, 2, rs)],
                   R[red_at(r, 3, rs)]};
  };
  const RRow<A> r0 = get(2 * p);
  RRow<A> o = get(2 * p + 1);
  const A b0 = rcp_pivot(rrow_b(r0));
  {
    RRow<A> dn = dpp_row<1, false>(r0);
    A id = dpp_shift<1, false>(b0);
    if (!kFull && p == P - 1) {
      dn = rrow_identity<A>();
      id = A(1);
    }
    o = pcr_combine_r(o, r0, b0, dn, id);
  }
  pcr_step_dpp<1, kFull>(o, p, P);
  pcr_step_dpp<2, kFull>(o, p, P);
  pcr_step_dpp<4, kFull>(o, p, P);
  pcr_step_dpp<8, kFull>(o, p, P);
  const A xo = o.d * rcp_pivot(rrow_b(o));
  A xm = dpp_shift<1, true>(xo);  // x_{2p-1}; alpha_0 = 0 for p = 0
  if (!kFull && p == 0) xm = A(0);
  R[red_at(2 * p, 3, rs)] = fma(r0.a, xm, fma(r0.c, xo, r0.d)) * b0;
  R[red_at(2 * p + 1, 3, rs)] = xo;
}

// Solve the reduced systems of all lines of the block (every thread takes
// part); the solution overwrites the d coefficients.
template <typename A>
__device__ __forceinline__ void pcr_reduced(A* red, int rs, int P, int tid) {
  if (P <= 16) {
    const int p = tid & (P - 1);
    A* R = red + tid / P;
    if (P == 16)
      pcr_dpp<true>(R, rs, p, P);
    else
      pcr_dpp<false>(R, rs, p, P);
    return;
  }
  const int p = tid & (P - 1);
  A* R = red + tid / P;
  auto get = [&](int r) {
    return RRow<A>{R[red_at(r, 0, rs)], R[red_at(r, 1, rs)], R[red_at(r, 2, rs)],
                   R[red_at(r, 3, rs)]};
  };
  RRow<A> r0 = get(2 * p), r1 = get(2 * p + 1);
  {
    // d = 1: row 2p pairs with row 2p-1 (lane p-1) and 2p+1 (this lane)
    RRow<A> up = shfl_row_up(r1, 1, P);
    RRow<A> dn = shfl_row_down(r0, 1, P);
    if (p == 0) up = rrow_identity<A>();
    if (p == P - 1) dn = rrow_identity<A>();
    const RRow<A> n0 = pcr_combine(r0, up, r1);
    const RRow<A> n1 = pcr_combine(r1, r0, dn);
    r0 = n0;
    r1 = n1;
  }
  // d = 2e: the rows at distance d sit e lanes away, in the same slot
  for (int e = 1; e < P; e <<= 1) {
    RRow<A> u0 = shfl_row_up(r0, e, P), u1 = shfl_row_up(r1, e, P);
    RRow<A> d0 = shfl_row_down(r0, e, P), d1 = shfl_row_down(r1, e, P);
    if (p < e) u0 = u1 = rrow_identity<A>();
    if (p + e >= P) d0 = d1 = rrow_identity<A>();
    const RRow<A> n0 = pcr_combine(r0, u0, d0);
    const RRow<A> n1 = pcr_combine(r1, u1, d1);
    r0 = n0;
    r1 = n1;
  }
  R[red_at(2 * p, 3, rs)] = r0.d * rcp_pivot(rrow_b(r0));
  R[red_at(2 * p + 1, 3, rs)] = r1.d * rcp_pivot(rrow_b(r1));
}

// y/z sweeps (chunk counts need not be powers of two): Thomas on the 2P
// reduced rows of one line by one lane, with u = 1 - (upper coupling of the
// eliminated previous row) carried as a non-negative quantity:
//   den = leak + gamma + alpha u,  cp = gamma / den,
//   dp = (d + alpha dp_prev) / den,  u' = (leak + alpha u) / den;
// back substitution x_r = dp_r + cp_r x_{r+1}.  cp and dp overwrite gamma
// and d; the next row's coefficients are read before the current row's
// results are stored, so that LDS latency overlaps the arithmetic.
template <typename A>
__device__ __forceinline__ void reduced_solve(A* R, int n2, int nl) {
  A u = A(0), dp = A(0);
  A an = R[0], cn = R[1 * nl], ln = R[2 * nl], dn = R[3 * nl];
  for (int r = 0; r < n2; ++r) {
    const A ar = an, cr = cn, lr = ln, dr = dn;
    if (r + 1 < n2) {
      an = R[red_at(r + 1, 0, nl)];
      cn = R[red_at(r + 1, 1, nl)];
      ln = R[red_at(r + 1, 2, nl)];
      dn = R[red_at(r + 1, 3, nl)];
    }
    const A inv = rcp_pivot(fma(ar, u, lr + cr));
    dp = fma(ar, dp, dr) * inv;
    u = fma(ar, u, lr) * inv;
    R[red_at(r, 1, nl)] = cr * inv;
    R[red_at(r, 3, nl)] = dp;
  }
  A xn = dp;
  A cq = R[red_at(n2 - 2, 1, nl)], dq = R[red_at(n2 - 2, 3, nl)];
  for (int r = n2 - 2; r >= 0; --r) {
    const A cr = cq, dr = dq;
    if (r > 0) {
      cq = R[red_at(r - 1, 1, nl)];
      dq = R[red_at(r - 1, 3, nl)];
    }
    xn = fma(cr, xn, dr);
    R[red_at(r, 3, nl)] = xn;
  }
}

template <typename A>
__device__ __forceinline__ void put_reduced(A* R, int nl, int p, const RRow<A>& rf,
                                            const RRow<A>& rl) {
  R[red_at(2 * p, 0, nl)] = rf.a;
  R[red_at(2 * p, 1, nl)] = rf.c;
  R[red_at(2 * p, 2, nl)] = rf.l;
  R[red_at(2 * p, 3, nl)] = rf.d;
  R[red_at(2 * p + 1, 0, nl)] = rl.a;
  R[red_at(2 * p + 1, 1, nl)] = rl.c;
  R[red_at(2 * p + 1, 2, nl)] = rl.l;
  R[red_at(2 * p + 1, 3, nl)] = rl.d;
}

// 16-byte vector access of V consecutive elements (V * sizeof(T) == 16);
// the address must be 16-byte aligned.
template <typename T, int V>
struct VecIO;
// Fields and flags live in device global memory.  Accesses through
// address-space-1 pointers compile to global_* instructions, which count
// only against vmcnt; through generic pointers they become flat_* ones,
// which count against lgkmcnt as well, so that every wait for a scalar load
// or an LDS access would also wait for the field loads in flight.
#define NPB_GLOBAL __attribute__((address_space(1)))
template <typename U>
__device__ __forceinline__ U ldg(const U* p) {
  return *(const NPB_GLOBAL U*)p;
}
// (native vector types: HIP's float4 is a class, whose member functions
// would take the address back to the generic space)
typedef float npb_f4 __attribute__((ext_vector_type(4)));
typedef double npb_d2 __attribute__((ext_vector_type(2)));
template <>
struct VecIO<float, 4> {
  static __device__ __forceinline__ void ld(const float* p, float (&o)[4]) {
    const npb_f4 v = *(const NPB_GLOBAL npb_f4*)p;
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
  static __device__ __forceinline__ void st(float* p, const float (&o)[4]) {
    *(NPB_GLOBAL npb_f4*)p = npb_f4{o[0], o[1], o[2], o[3]};
  }
};
template <>
struct VecIO<double, 2> {
  static __device__ __forceinline__ void ld(const double* p, double (&o)[2]) {
    const npb_d2 v = *(const NPB_GLOBAL npb_d2*)p;
    o[0] = v.x; o[1] = v.y;
  }
  static __device__ __forceinline__ void st(double* p, const double (&o)[2]) {
    *(NPB_GLOBAL npb_d2*)p = npb_d2{o[0], o[1]};
  }
};

// solute flags of V consecutive nodes, one byte each
template <int V>
__device__ __forceinline__ uint32_t ld_mask(const uint8_t* p) {
  if constexpr (V == 4) return *(const NPB_GLOBAL uint32_t*)p;
  if constexpr (V == 2) return *(const NPB_GLOBAL uint16_t*)p;
  return *(const NPB_GLOBAL uint8_t*)p;
}

// ---------------------------------------------------------------------------
// x sweep.  Block: L lines x P chunk slots (P a power of two), L*P threads;
// lane t takes line t % L and chunk t / L.  The first row4(nx) elements of
// each row move between HBM and an odd-stride LDS tile with 16-byte vector
// accesses; the row's boundary columns are written back unchanged.
template <typename T, typename A, int M, int L, bool CN>
__global__ __launch_bounds__(L * 8 > 512 ? 512 : (L * 8 < 256 ? 256 : L * 8)) void sweep_x_kernel(
    const SweepArgs<T>* __restrict__ args, const int2* __restrict__ work, int nbu) {
  constexpr int VX = 16 / (int)sizeof(T);  // elements per vector access
  extern __shared__ __align__(16) unsigned char smem[];
  // (field, block of that field): arithmetic when every field of the
  // launch has nbu blocks, else from the work list
  const int2 w = nbu > 0 ? make_int2((int)blockIdx.x / nbu, (int)blockIdx.x % nbu)
                         : work[blockIdx.x];
  const SweepArgs<T>& a = args[w.x];
  ConstTab<A>& tb = *(ConstTab<A>*)(a.tab);
  const int nx = a.nx, ny = a.ny, nz = a.nz, nxp = a.nxp;
  const int nint = nx - 2;
  const int P = a.P, S = a.S;
  const int nthreads = L * P;
  const int nyi = ny - 2;
  const int nlines = nyi * (nz - 2);
  const int l0 = w.y * L;
  const bool uniform = (a.mask == nullptr);
  const bool aos = (a.mode == MODE_AOS_FIRST);
  const int tid = threadIdx.x;
  // Line l is interior row y = l % nyi of interior plane zi = l / nyi.  The
  // block's first line is split once (block-uniform); line l0 + q then has
  // t = yb + q < nyi + L, whose quotient by nyi comes from a float
  // reciprocal estimate (off by at most one below, for t a multiple of nyi)
  // and one correction, branch-free, so no lane runs an integer division.
  const int zb = l0 / nyi, yb = l0 - zb * nyi;
  const float rnyi = 1.0f / (float)nyi;
  auto line_yz = [&](int q, int& yi, int& zi) {
    const int t = yb + q;
    int w = (int)((float)t * rnyi);
    int r = t - w * nyi;
    if (r < 0) {
      r += nyi;
      --w;
    }
    if (r >= nyi) {
      r -= nyi;
      ++w;
    }
    yi = r;
    zi = zb + w;
  };
  // element offset of node 0 of block row q (line l0 + q), -1 past the last
  // line; offsets fit in 32 bits (n <= 514)
  auto row_base = [&](int q) -> int {
    if (q >= L || l0 + q >= nlines) return -1;
    int yi, zi;
    line_yz(q, yi, zi);
    return ((1 + zi) * ny + 1 + yi) * nxp;
  };

  size_t off = 16;
  A* red = reinterpret_cast<A*>(smem + off);  // reduced systems
  off += sizeof(A) * (size_t)red_size(P, L + 1);
  // the tile and the mask rows carry P*M+2 spare elements at their end:
  // a chunk's reads may run past the last row (values selected away)
  A* tile = reinterpret_cast<A*>(smem + off);
  off += sizeof(A) * ((size_t)L * S + P * M + 2);
  A* wtile = nullptr;
  if (aos) {
    wtile = reinterpret_cast<A*>(smem + off);
    off += sizeof(A) * (size_t)L * S;
  }
  off = (off + 15) & ~size_t(15);
  uint8_t* mt = smem + off;  // L rows of nx4 bytes
  const int nx4 = row4(nx);

  // Field elements moved per row: the first row4(nx), or the first nx - 1
  // when node nx - 1 would be the only node of the row's last 128-byte line
  // (nx - 1 a multiple of 128 / sizeof(T)); that right Dirichlet value then
  // comes from the run's shell data, and the line is neither fetched nor
  // written.  The mask rows always move row4(nx) bytes (their last face).
  const int nxl = (a.bcx != nullptr && (nx - 1) % (128 / (int)sizeof(T)) == 0) ? nx - 1 : nx4;
  // Row loads.  The block's row traffic is L rows x ncg column groups of
  // eight 16-byte vectors; item w = (row w % L, group w / L).  Lane t takes
  // vector column cv = t % 8 of items t / 8, t / 8 + RQ, ... (RQ = lanes / 8):
  // a half-wave moves four rows x eight vectors (128 contiguous bytes of
  // each row), and with the LDS row stride S (x_tile_stride) its element
  // writes fall in distinct banks; every lane takes a share even when the
  // block has more lanes than rows x 8.  All vector loads of a batch are in
  // flight before its LDS stores.
  const int vpr = nx4 / VX;         // vectors per row
  const int ncg = (vpr + 7) >> 3;   // 8-vector column groups per row
  const int cv = tid & 7;
  const int RQ = nthreads >> 3;     // item slots per pass
  const int rq = tid >> 3;
  const int nitems = L * ncg;
  // The block's lines are consecutive rows of the per-row source lists:
  // one contiguous entry range [eb, ee), whose bounds are block-uniform.
  // Each lane fetches its entry (usually at most one) with the first batch
  // of row loads and adds it once the rows are in LDS.
  const bool src = a.src_stage == 1;
  int eb = 0, ee = 0, e_lin = -1;
  double e_rho = 0.0;
  // Lane t < L fetches the right Dirichlet value of line t when the rows
  // stop before node nx - 1: node (nx-1, j, k) of the shell (shell order:
  // the two z faces, then per interior z the y = 0 and y = ny-1 rows and
  // the x = 0, nx-1 pairs of each interior y).
  const bool gr_line = nxl < nx && tid < L && l0 + tid < nlines;
  // the chunk class of lane (line tid % L, chunk tid / L), fetched ahead of
  // the rows so that its latency overlaps theirs
  int cls = 1;
  if (l0 + tid % L < nlines)
    cls = uniform ? 0 : (a.ccls ? (int)ldg(a.ccls + (size_t)(tid / L) * nlines + (l0 + tid % L)) : 1);
  A gRv = A(0);
  bool first_batch = true;
  // with the first batch of row loads in flight: the source entries and
  // the right ends, so that their latency overlaps the rows'
  auto fetch_first = [&]() {
    first_batch = false;
    if (src) {
      eb = ldg(a.src_ptr + row_base(0) / nxp);
      ee = ldg(a.src_ptr + row_base(min(L, nlines - l0) - 1) / nxp + 1);
      if (eb + tid < ee) {
        e_lin = ldg(a.src_lin + eb + tid);
        e_rho = ldg(a.src_rho + eb + tid);
      }
    }
    if (gr_line) {
      int yi, zi;
      line_yz(tid, yi, zi);
      const int s = 2 * nx * ny + zi * (2 * nx + 2 * nyi) + 2 * nx + 2 * yi + 1;
      gRv = (A)(T)ldg(a.bcx + s);
    }
  };
  // When RQ is a multiple of L (P a multiple of 8), every item of a lane
  // lies in the same block row q = rq mod L: its row base is then found once
  // (a block-uniform choice between two compiled forms of the loops).
  const bool qfix = (RQ % L) == 0;
  auto load_rows = [&](auto fixq) {
    constexpr bool kFix = decltype(fixq)::value;
    const int rb0 = kFix ? row_base(rq % L) : 0;
    const T* const ug = a.u;
    const uint8_t* const mg = a.mask;
    constexpr int kU = 8;
    for (int w0 = rq; w0 < nitems; w0 += kU * RQ) {
      T v[kU][VX];
      uint32_t m[kU];
      int lo[kU], mo[kU];
#pragma unroll
      for (int j = 0; j < kU; ++j) {
        lo[j] = -1;
        const int w = w0 + j * RQ;
        if (w < nitems) {
          const int q = kFix ? rq % L : w % L, g = w / L;
          const int c = (cv + 8 * g) * VX;
          const int rb = kFix ? rb0 : row_base(q);
          if (c < nx4 && rb >= 0) {
            lo[j] = c < nxl ? q * S + c : -1;
            mo[j] = q * nx4 + c;
            if (c < nxl) VecIO<T, VX>::ld(ug + rb + c, v[j]);
            if (!uniform) m[j] = ld_mask<VX>(mg + rb + c);
          } else {
            mo[j] = -1;
          }
        } else {
          mo[j] = -1;
        }
      }
      if (first_batch) fetch_first();
#pragma unroll
      for (int j = 0; j < kU; ++j) {
        if (lo[j] >= 0) {
#pragma unroll
          for (int i = 0; i < VX; ++i) tile[lo[j] + i] = (A)v[j][i];
        }
        if (!uniform && mo[j] >= 0) {
          if constexpr (VX == 4)
            *reinterpret_cast<uint32_t*>(mt + mo[j]) = m[j];
          else
            *reinterpret_cast<uint16_t*>(mt + mo[j]) = (uint16_t)m[j];
        }
      }
    }
  };
  if (qfix)
    load_rows(std::true_type{});
  else
    load_rows(std::false_type{});
  // lanes without row items
  if (first_batch) fetch_first();
  if (gr_line) tile[tid * S + nx - 1] = gRv;
  // A line's last chunk reads past the right Dirichlet node: into the row's
  // padding columns [z0, S), then (when P M + 1 > S) into the next row's
  // loaded values or, after the last row, the P M + 2 spare elements.  The
  // padding and the spare elements hold zeros, so every such read is finite.
  {
    // nzc = S - z0 <= 35 (S exceeds row4(nx) by at most 32), so 64 slots a
    // row cover it without a division
    const int z0 = nxl < nx ? nx : nx4;
    const int nzc = S - z0;
    if (nzc > 0)
      for (int e = tid; e < L * 64; e += nthreads)
        if ((e & 63) < nzc) tile[(e >> 6) * S + z0 + (e & 63)] = A(0);
    for (int e = tid; e < P * M + 2; e += nthreads) tile[L * S + e] = A(0);
  }
  __syncthreads();

  // pointwise pre-operations on interior nodes: AOS W = flow(u) and the
  // LODIE1 leading nonlinear sub-step
  const int total = L * nx;
  if (aos || a.pre_nl) {
    const A pka = (A)a.pre_ka, pkb = (A)a.pre_kb, wka = (A)a.aos_ka, wkb = (A)a.aos_kb;
    const int dq2 = nthreads / nx, dx2 = nthreads - dq2 * nx;
    int q = tid / nx, x = tid - (tid / nx) * nx;
    for (int e = tid; e < total; e += nthreads) {
      if (l0 + q < nlines && x >= 1 && x <= nx - 2) {
        A v = tile[q * S + x];
        // the face rule by location runs in the CN-capable variant, whose
        // flags carry half-point bits above bit 0
        bool solvent = !uniform && (CN ? (mt[q * nx4 + x] & 1) == 0 : mt[q * nx4 + x] == 0);
        if (aos) wtile[q * S + x] = (solvent && a.aos_w) ? sinh_flow(v, wka, wkb) : v;
        if (a.pre_nl && solvent) tile[q * S + x] = sinh_flow(v, pka, pkb);
      }
      q += dq2;
      x += dx2;
      if (x >= nx) {
        x -= nx;
        ++q;
      }
    }
    __syncthreads();
  }
  if (CN && a.cn == 2) {
    const int ql = tid % L;
    cn_tile_rows<A, M>(tile + ql * S, 1, mt + ql * nx4, 1, (tid / L) * M, nx - 2,
                       l0 + ql < nlines, uniform, a.face_loc != 0, (A)a.re[0], (A)a.re[1],
                       (A)a.re[2], (A)a.re_uniform);
  }
  if (src) {
    // entries are distinct nodes: the adds do not collide.  Quotients by the
    // pitch (a multiple of 16, entries below 514 * 514 * 544) and by ny
    // (rows below 514 * ny) from float reciprocal estimates with one
    // correction each way, exact over those ranges
    const float rnxp = 1.0f / (float)nxp, rny = 1.0f / (float)ny;
    auto divmod = [](int n, int dv, float rdv, int& qo, int& ro) {
      int w = (int)((float)n * rdv);
      int r = n - w * dv;
      if (r < 0) {
        r += dv;
        --w;
      }
      if (r >= dv) {
        r -= dv;
        ++w;
      }
      qo = w;
      ro = r;
    };
    auto add_entry = [&](int lin, double rho) {
      int row, x, zr, yr;
      divmod(lin, nxp, rnxp, row, x);
      divmod(row, ny, rny, zr, yr);
      const int q = (zr - 1) * nyi + (yr - 1) - l0;
      tile[q * S + x] += (A)(a.src_coef * rho);
    };
    if (e_lin >= 0) add_entry(e_lin, e_rho);
    for (int e = eb + tid + nthreads; e < ee; e += nthreads) add_entry(ldg(a.src_lin + e), ldg(a.src_rho + e));
    __syncthreads();
  }

  // chunk elimination
  const int ql = tid % L;
  const int p = tid / L;
  const bool lvalid = l0 + ql < nlines;
  const int g0 = p * M;
  A* trow = tile + ql * S;
  A* col = trow + 1 + g0;  // row element of interior node g0 + k at col[k]
  const uint8_t* mrow = mt + ql * nx4;
  const A gL = trow[0];
  const A gR = trow[nx - 1];
  const bool first = (g0 == 0);
  const int kR = lvalid ? nint - 1 - g0 : -1;
  // a line's last chunk (1 <= kR <= M - 1) takes the uniform path too,
  // unless the explicit Crank-Nicolson half is formed in registers here
  const int kt = (nint - 1) % M;
  const bool tail = kR >= 1 && kR < M && !first && !(CN && a.cn == 1);
  // lanes without a line follow whatever path their wave takes
  const bool inner = cls != 1 && (kR >= M || tail);
  const unsigned long long bv = __ballot(lvalid);
  const unsigned long long bf = __ballot(lvalid && inner);
  const unsigned long long bs = __ballot(lvalid && inner && cls == 2);
  const bool fast = bv != 0 && bf == bv && (bs == 0 || bs == bf);
  const int t = __builtin_amdgcn_readfirstlane((fast && bs != 0) ? 1 : 0);
  // uniform tail chunk: the right Dirichlet term into the last real row
  // (an LDS update of the lane's own node; the row is overwritten below)
  if (fast && tail && lvalid) col[kR] = fma(tb.re[t], gR, col[kR]);
  // rows past a line's end read zeros or the Dirichlet value (finite; their
  // results are never stored), lanes without a line whatever their rows
  // hold (their results stay in their own lanes and lines)
  A d[M];
#pragma unroll
  for (int k = 0; k < M; ++k) d[k] = col[k];
  A al[M], ga[M];
  RRow<A> rf, rl;
  if (fast) {
    if (CN && a.cn == 1) cn_rhs_uniform<A, M>(d, tb.re[t], col[-1], col[M]);
    if (first) d[0] = fma(tb.re[t], gL, d[0]);
    fast_eliminate<A, M>(d, tb, t, first, tail, kt, rf, rl);
  } else {
    const A re0 = (A)(uniform ? a.re_uniform : a.re[0]);
    const A re1 = (A)(uniform ? a.re_uniform : a.re[1]);
    const A re2 = (A)(uniform ? a.re_uniform : a.re[2]);
    A reF[M + 1];
    int prev = uniform ? 1 : (int)mrow[g0];
    if (CN && a.face_loc != 0) {
#pragma unroll
      for (int k = 0; k <= M; ++k) {
        // face between nodes g0 + k and g0 + k + 1 by location: bit 1 of
        // the lower node's flag
        const int cur = uniform ? 1 : (int)mrow[g0 + k + 1];
        reF[k] = pick3((g0 + k + 1 > nx - 1) ? 2 : (prev & 2), re0, re1, re2);
        prev = cur;
      }
    } else {
#pragma unroll
      for (int k = 0; k <= M; ++k) {
        // face between nodes g0 + k and g0 + k + 1
        const int cur = uniform ? 1 : (int)mrow[g0 + k + 1];
        reF[k] = pick3((g0 + k + 1 > nx - 1) ? 2 : prev + cur, re0, re1, re2);
        prev = cur;
      }
    }
    if (CN && a.cn == 1) cn_rhs<A, M>(d, reF, col[-1], col[M], kR, gR);
    if (first && lvalid) d[0] = fma(reF[0], gL, d[0]);
    chunk_eliminate<A, M>(d, al, ga, rf, rl, reF, first, kR, gR);
  }
  A* R = red + ql;
  put_reduced(R, L + 1, p, rf, rl);
  __syncthreads();
  pcr_reduced(red, L + 1, P, tid);
  __syncthreads();
  const A xf = R[red_at(2 * p, 3, L + 1)];
  const A xl = R[red_at(2 * p + 1, 3, L + 1)];
  if (fast)
    fast_finish<A, M>(d, &tb.ga[t][0], &tb.al[t][0], xf, xl, tail, kt);
  else
    chunk_finish<A, M>(d, al, ga, xf, xl);
  // results back into the row; a full chunk stores without per-row checks.
  // Additive modes: acc = ww W + wv V (the weights of the mean)
  const A ww = (A)a.aos_ww, wv = (A)a.aos_wv;
  if (lvalid) {
    if (!aos) {
      if (g0 + M <= nint) {
#pragma unroll
        for (int k = 0; k < M; ++k) col[k] = d[k];
      } else {
#pragma unroll
        for (int k = 0; k < M; ++k)
          if (g0 + k < nint) col[k] = d[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < M; ++k)
        if (g0 + k < nint) col[k] = fma(ww, wtile[ql * S + 1 + g0 + k], wv * d[k]);
    }
  }
  __syncthreads();

  // row stores (boundary columns carry their loaded values), same lane map
  T* out = aos ? a.acc : a.u;
  auto store_rows = [&](auto fixq) {
    constexpr bool kFix = decltype(fixq)::value;
    const int rb0 = kFix ? row_base(rq % L) : 0;
    for (int w = rq; w < nitems; w += RQ) {
      const int q = kFix ? rq % L : w % L, g = w / L;
      const int c = (cv + 8 * g) * VX;
      const int rb = kFix ? rb0 : row_base(q);
      if (c < nxl && rb >= 0) {
        T v[VX];
#pragma unroll
        for (int i = 0; i < VX; ++i) v[i] = (T)tile[q * S + c + i];
        VecIO<T, VX>::st(out + rb + c, v);
      }
    }
  };
  if (qfix)
    store_rows(std::true_type{});
  else
    store_rows(std::false_type{});
}

// Face class of lane tid's chunk (line x = xb + tid % TW, chunk tid / TW)
// in a y (dir 1) or z (dir 2) sweep of the lines at transverse index o: 0
// uniform solvent, 2 uniform solute, 1 mixed (the uniform medium: 0).
template <typename T, int TW>
__device__ __forceinline__ int yz_chunk_class(const SweepArgs<T>& a, int dir, int o, int xb,
                                              int tid) {
  const int nx = a.nx;
  const int x = xb + tid % TW;
  if (x < 1 || x > nx - 2) return 1;
  if (a.mask == nullptr) return 0;
  if (!a.ccls) return 1;
  const long long nl = (long long)(nx - 2) * ((dir == 1 ? a.nz : a.ny) - 2);
  return (int)ldg(a.ccls + (size_t)(tid / TW) * nl + (size_t)(o - 1) * (nx - 2) + (x - 1));
}

// Line solves of one y/z tile held in LDS: tile[row * ts + q] is node row
// `row` (0..n-1 along the line) of x = xb + q, mt[row * TW + q] its solute
// flag; red holds the reduced systems ((TW + 1)-strided).  Lane tid takes
// line q = tid % TW and chunk p = tid / TW; cls is the chunk's face class
// (yz_chunk_class).  On return the tile holds the solution (with the fused
// flow of kYzFlow / post_nl) on the interior rows of the lane's line; other
// columns are untouched.  Contains the block barriers of the reduced solve.
template <typename T, typename A, int M, int VAR, int TW>
__device__ __forceinline__ void yz_solve_lines(const SweepArgs<T>& a, A* tile, int ts,
                                               const uint8_t* mt, A* red, int n, int xb, int cls,
                                               int tid) {
  ConstTab<A>& tb = *(ConstTab<A>*)(a.tab);
  const int nx = a.nx, P = a.P;
  const int nint = n - 2;
  const bool uniform = (a.mask == nullptr);
  const int ql = tid % TW;
  const int p = tid / TW;
  const int x = xb + ql;
  const bool lvalid = x >= 1 && x <= nx - 2;
  // chunk elimination: the lane's column of the tile from row 1 + g0
  const int g0 = p * M;
  A* col = tile + (1 + g0) * ts + ql;
  const uint8_t* mcol = mt + g0 * TW + ql;  // flag of along node g0 + k at mcol[k * TW]
  const A gL = tile[ql];
  const A gR = tile[(n - 1) * ts + ql];
  const bool first = (g0 == 0);
  const int kR = lvalid ? nint - 1 - g0 : -1;
  // a line's last chunk (1 <= kR <= M - 1) takes the uniform path too,
  // unless the explicit Crank-Nicolson half is formed in registers here
  const int kt = (nint - 1) % M;
  const bool tail = kR >= 1 && kR < M && !first && !(VAR == kYzGeneral && a.cn == 1);
  // lanes without a line follow whatever path their wave takes
  const bool inner = cls != 1 && (kR >= M || tail);
  const unsigned long long bv = __ballot(lvalid);
  const unsigned long long bf = __ballot(lvalid && inner);
  const unsigned long long bs = __ballot(lvalid && inner && cls == 2);
  const bool fast = bv != 0 && bf == bv && (bs == 0 || bs == bf);
  const int t = __builtin_amdgcn_readfirstlane((fast && bs != 0) ? 1 : 0);
  // uniform tail chunk: the right Dirichlet term into the last real row
  // (an LDS update of the lane's own node; the row is overwritten below)
  if (fast && tail && lvalid) col[kR * ts] = fma(tb.re[t], gR, col[kR * ts]);
  // rows past the line's end read zeros or the Dirichlet value (finite;
  // their results are never stored)
  A d[M];
#pragma unroll
  for (int k = 0; k < M; ++k) d[k] = col[k * ts];
  A al[M], ga[M];
  RRow<A> rf, rl;
  if (fast) {
    if (VAR == kYzGeneral && a.cn == 1)
      cn_rhs_uniform<A, M>(d, tb.re[t], col[-ts], col[M * ts]);
    if (first) d[0] = fma(tb.re[t], gL, d[0]);
    fast_eliminate<A, M>(d, tb, t, first, tail, kt, rf, rl);
  } else {
    const A re0 = (A)(uniform ? a.re_uniform : a.re[0]);
    const A re1 = (A)(uniform ? a.re_uniform : a.re[1]);
    const A re2 = (A)(uniform ? a.re_uniform : a.re[2]);
    A reF[M + 1];
    int prev = uniform ? 1 : (int)mcol[0];
    if (VAR == kYzGeneral && a.face_loc != 0) {
#pragma unroll
      for (int k = 0; k <= M; ++k) {
        // face between along nodes g0 + k and g0 + k + 1 by location: bit 1
        // of the lower node's flag
        const int cur = uniform ? 1 : (int)mcol[(k + 1) * TW];
        reF[k] = pick3((g0 + k + 1 > n - 1) ? 2 : (prev & 2), re0, re1, re2);
        prev = cur;
      }
    } else {
#pragma unroll
      for (int k = 0; k <= M; ++k) {
        // face between along nodes g0 + k and g0 + k + 1
        const int cur = uniform ? 1 : (int)mcol[(k + 1) * TW];
        reF[k] = pick3((g0 + k + 1 > n - 1) ? 2 : prev + cur, re0, re1, re2);
        prev = cur;
      }
    }
    if (VAR == kYzGeneral && a.cn == 1) cn_rhs<A, M>(d, reF, col[-ts], col[M * ts], kR, gR);
    if (first && lvalid) d[0] = fma(reF[0], gL, d[0]);
    chunk_eliminate<A, M>(d, al, ga, rf, rl, reF, first, kR, gR);
  }
  A* R = red + ql;
  put_reduced(R, TW + 1, p, rf, rl);
  __syncthreads();
  // reduced systems: in FP32 arithmetic with a power-of-two chunk count the
  // block's lanes solve them together by cyclic reduction (the P lanes of a
  // line in one wave, as in the x sweep); otherwise one lane per line runs
  // Thomas (FP64 keeps only Thomas: the cyclic reduction's registers would
  // cost its kernels a wave per SIMD)
  bool pcr = false;
  if constexpr (sizeof(A) == 4) pcr = (P & (P - 1)) == 0 && P <= 64;
  if (pcr)
    pcr_reduced(red, TW + 1, P, tid);
  else if (p == 0 && lvalid)
    reduced_solve(R, 2 * P, TW + 1);
  __syncthreads();
  const A xf = R[red_at(2 * p, 3, TW + 1)];
  const A xl = R[red_at(2 * p + 1, 3, TW + 1)];
  if (fast)
    fast_finish<A, M>(d, &tb.ga[t][0], &tb.al[t][0], xf, xl, tail, kt);
  else
    chunk_finish<A, M>(d, al, ga, xf, xl);

  if ((VAR == kYzFlow || (VAR == kYzGeneral && a.post_nl)) && !uniform) {
    const A ka = (A)a.post_ka, kb = (A)a.post_kb;
    // a uniform chunk's face class tells its nodes' medium only under the
    // harmonic rule (the face rule by location runs in the general variant)
    if (fast && (VAR != kYzGeneral || a.face_loc == 0)) {
      if (t == 0) {
#pragma unroll
        for (int k = 0; k < M; ++k) d[k] = sinh_flow(d[k], ka, kb);
      }
    } else {
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const bool solv =
            VAR == kYzGeneral ? (mcol[(k + 1) * TW] & 1) == 0 : mcol[(k + 1) * TW] == 0;
        if constexpr (sizeof(A) == 4) {
          // FP32: every node's flow (ten instructions), kept on the solvent
          // ones by a select: no branch per node, and the flag reads need
          // not wait one by one
          const A w = sinh_flow(d[k], ka, kb);
          d[k] = solv ? w : d[k];
        } else {
          if (solv) d[k] = sinh_flow(d[k], ka, kb);
        }
      }
    }
  }
  // rows past the line end land in rows n-1.. of the tile, which are
  // neither stored nor read again
  if (lvalid) {
#pragma unroll
    for (int k = 0; k < M; ++k) col[k * ts] = d[k];
  }
}

// ---------------------------------------------------------------------------
// y / z sweep.  Block: one tile of TW consecutive x (x = xb .. xb+TW-1) of
// one plane of the other transverse index o, across the whole line length
// n; TW*P threads.  The n node rows of the tile (TW*sizeof(T) contiguous
// bytes each, one or two cache lines) move between HBM and an LDS tile
// [rows][TW+1] with 16-byte vector accesses; lane t then takes line
// xb + t % TW and chunk t / TW, as in the x sweep.  The LDS tile has
// a.S >= max(n, P*M+2) rows so that every chunk row and face a lane touches
// lies inside it (rows past the line hold don't-care values that are
// selected away).  Columns outside 1..nx-2 are loaded but never solved;
// they are stored back with the values they came with (the AOS accumulator
// keeps its own).  VAR selects the fused work at compile time:
//   kYzPlain   : solve only, in place
//   kYzFlow    : solve, then the exact sinh flow on solvent nodes, in place
//   kYzGeneral : sources before/after, flow, AOS accumulation (run-time flags)

template <typename T, typename A, int M, int VAR, int TW>
__global__ __launch_bounds__(512) void sweep_yz_kernel(const SweepArgs<T>* __restrict__ args,
                                                       const int2* __restrict__ work, int nbu,
                                                       int dir, int nblocks) {
  constexpr int VX = 16 / (int)sizeof(T);  // elements per vector access
  constexpr int TS = TW + 1;                // LDS elements per tile row
  constexpr int VPR = TW / VX;              // vectors per full tile row
  extern __shared__ __align__(16) unsigned char smem[];
  // Work item bi of the launch: the hardware hands consecutive blocks to
  // the eight XCDs in turn, so block b takes item (b % 8) * per + b / 8 and
  // each XCD works through one contiguous range of items; neighbouring
  // tiles of a plane then share their mask lines in that XCD's L2.  Blocks
  // past the last item leave before any barrier.
  const int per = (nblocks + 7) >> 3;
  const int bi = ((int)blockIdx.x & 7) * per + ((int)blockIdx.x >> 3);
  if (bi >= nblocks) return;
  // (field, block of that field): arithmetic when every field of the
  // launch has nbu blocks, else from the work list
  const int2 w = nbu > 0 ? make_int2(bi / nbu, bi % nbu) : work[bi];
  const SweepArgs<T>& a = args[w.x];
  const int nx = a.nx, ny = a.ny, nxp = a.nxp;
  const int P = a.P, nrow = a.S;
  const int nthreads = TW * P;
  const int tid = threadIdx.x;
  const int n = (dir == 1) ? ny : a.nz;
  const int nint = n - 2;
  const int ntx = (nx - 2) / TW + 1;  // tiles holding interior x
  const int xt = w.y % ntx;
  const int o = 1 + w.y / ntx;
  const int xb = xt * TW;
  // element offsets fit in 32 bits (n <= 514)
  const uint32_t stride = (dir == 1) ? (uint32_t)nxp : (uint32_t)nxp * (uint32_t)ny;
  const uint32_t plane = (dir == 1) ? (uint32_t)o * (uint32_t)ny * (uint32_t)nxp
                                    : (uint32_t)o * (uint32_t)nxp;  // node (0, o, along 0)
  const uint32_t base = plane + (uint32_t)xb;
  const bool uniform = (a.mask == nullptr);

  A* red = reinterpret_cast<A*>(smem);  // reduced systems
  A* tile = red + (size_t)red_size(P, TW + 1);
  uint8_t* mt = reinterpret_cast<uint8_t*>(tile + (size_t)nrow * TS);  // [nrow][TW]

  // Trilinear sources of the tile's lines form one contiguous range
  // [sb, se) of the per-line lists (tile-uniform bounds); each lane fetches
  // its entry (usually at most one) with the first batch of node rows and
  // adds it when needed (before the solve for stage 1, after it for stage
  // 2); entries are distinct nodes, so the adds do not collide.
  const bool src = VAR == kYzGeneral && a.src_stage != 0;
  int sb = 0, se = 0, e_lin = -1;
  double e_rho = 0.0;
  bool fetch = src;
  auto fetch_entries = [&]() {
    const int xlo = max(xb, 1), xhi = min(xb + TW - 1, nx - 2);
    sb = ldg(a.src_ptr + o * nx + xlo);
    se = ldg(a.src_ptr + o * nx + xhi + 1);
    if (sb + tid < se) {
      e_lin = ldg(a.src_lin + sb + tid);
      e_rho = ldg(a.src_rho + sb + tid);
    }
    fetch = false;
  };

  // the lane's chunk class, fetched ahead of the rows so that its latency
  // overlaps theirs
  const int cls = yz_chunk_class<T, TW>(a, dir, o, xb, tid);

  // Node-row traffic: thread = (vector column cv, first row jr); rows step
  // by RS = nthreads / VPR.  Columns past row4(nx) stay untouched.
  const int cv = tid % VPR;
  const int jr = tid / VPR;
  const int RS = nthreads / VPR;
  const bool cok = cv * VX < row4(nx) - xb;
  const uint32_t rstep = (uint32_t)RS * stride;
  if (cok) {
    constexpr int kU = 8;
    uint32_t pt = base + (uint32_t)jr * stride + (uint32_t)(cv * VX);
    for (int j0 = jr; j0 < n; j0 += kU * RS) {
      T v[kU][VX];
      uint32_t m[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (j0 + u * RS < n) {
          VecIO<T, VX>::ld(a.u + pt + (uint32_t)u * rstep, v[u]);
          if (!uniform) m[u] = ld_mask<VX>(a.mask + pt + (uint32_t)u * rstep);
        }
      }
      if (fetch) fetch_entries();
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = j0 + u * RS;
        if (j < n) {
#pragma unroll
          for (int i = 0; i < VX; ++i) tile[j * TS + cv * VX + i] = (A)v[u][i];
          if (!uniform) {
            if constexpr (VX == 4)
              *reinterpret_cast<uint32_t*>(mt + j * TW + cv * VX) = m[u];
            else
              *reinterpret_cast<uint16_t*>(mt + j * TW + cv * VX) = (uint16_t)m[u];
          }
        }
      }
      pt += (uint32_t)kU * rstep;
    }
  }
  // lanes without node rows to move
  if (fetch) fetch_entries();
  // tile rows past the line's end up to the last chunk row hold zeros, so
  // that a line's last chunk reads finite values past its end
  for (int e = tid; e < (P * M + 1 - n) * TS; e += nthreads) tile[n * TS + e] = A(0);
  __syncthreads();

  auto add_entry = [&](int lin, double rho) {
    const uint32_t off = (uint32_t)lin - plane;
    const uint32_t jj = off / stride;
    const int q = (int)(off - jj * stride) - xb;
    tile[jj * TS + q] += (A)(a.src_coef * rho);
  };
  auto add_sources = [&]() {
    if (e_lin >= 0) add_entry(e_lin, e_rho);
    for (int e = sb + tid + nthreads; e < se; e += nthreads) add_entry(ldg(a.src_lin + e), ldg(a.src_rho + e));
  };
  // general variant: the leading nonlinear sub-step on the input (Sec. 3.3)
  // and the Crank-Nicolson explicit half before the sources (additive schemes)
  if (VAR == kYzGeneral && (a.pre_nl || a.cn == 2)) {
    const int ql = tid % TW;
    const int g0 = (tid / TW) * M;
    const int x = xb + ql;
    const bool lv = x >= 1 && x <= nx - 2;
    if (a.pre_nl && !uniform && lv) {
      const A ka = (A)a.pre_ka, kb = (A)a.pre_kb;
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const int r = 1 + g0 + k;
        if (r <= nint && (mt[r * TW + ql] & 1) == 0)
          tile[r * TS + ql] = sinh_flow(tile[r * TS + ql], ka, kb);
      }
    }
    __syncthreads();
    if (a.cn == 2)
      cn_tile_rows<A, M>(tile + ql, TS, mt + ql, TW, g0, nint, lv, uniform, a.face_loc != 0,
                         (A)a.re[0], (A)a.re[1], (A)a.re[2], (A)a.re_uniform);
  }
  if (VAR == kYzGeneral && a.src_stage == 1) {
    add_sources();
    __syncthreads();
  }

  yz_solve_lines<T, A, M, VAR, TW>(a, tile, TS, mt, red, n, xb, cls, tid);
  __syncthreads();
  if (VAR == kYzGeneral && a.src_stage == 2) {
    add_sources();
    __syncthreads();
  }

  // interior node rows back to HBM; the z sweep (the last sub-step of a
  // step) notes a stored value that is not finite (Sec. 4.2: a diverged run)
  const int mode = (VAR == kYzGeneral) ? a.mode : MODE_INPLACE;
  T* out = (mode == MODE_AOS_ADD) ? a.acc : a.u;
  T nz = T(0);  // stays zero while every stored value is finite (0 * inf, 0 * nan: nan)
  auto store_rows = [&](auto check) {
    uint32_t pt = base + (uint32_t)(1 + jr) * stride + (uint32_t)(cv * VX);
    for (int j = 1 + jr; j <= nint; j += RS, pt += rstep) {
      T w[VX];
      if (mode == MODE_AOS_ADD || mode == MODE_AOS_FINISH) {
        T acc[VX];
        VecIO<T, VX>::ld(a.acc + pt, acc);
#pragma unroll
        for (int i = 0; i < VX; ++i) {
          const int xi = xb + cv * VX + i;
          const A tv = tile[j * TS + cv * VX + i];
          const bool live = xi >= 1 && xi <= nx - 2;
          if (live)
            w[i] = (T)((A)acc[i] + (A)a.aos_wv * tv);
          else
            w[i] = (mode == MODE_AOS_ADD) ? acc[i] : (T)tv;
        }
      } else {
#pragma unroll
        for (int i = 0; i < VX; ++i) w[i] = (T)tile[j * TS + cv * VX + i];
      }
      if constexpr (decltype(check)::value) {
#pragma unroll
        for (int i = 0; i < VX; ++i) nz = fma(w[i], T(0), nz);
      }
      VecIO<T, VX>::st(out + pt, w);
    }
  };
  const bool chk = a.nonfinite != nullptr;
  if (cok) {
    if (chk)
      store_rows(std::true_type{});
    else
      store_rows(std::false_type{});
  }
  if (chk && nz != nz) atomicOr(a.nonfinite, 1);
}

// ---------------------------------------------------------------------------
// planning and dispatch

static int pick_chunk(int need) {
  for (int c : kChunkChoices)
    if (c >= need) return c;
  return -1;
}

static int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

LaunchShape plan_x(int nx, int ny, int nz, bool fp64, bool aos, bool uniform, int mt, int lw) {
  LaunchShape s{};
  const int nint = nx - 2;
  const int es = fp64 ? 8 : 4;
  const int nx4 = row4(nx);
  if (mt <= 0) mt = 20;
  // default lines per block: 16 for FP32 arithmetic (measured best for the
  // 161^3 solve, whose two media sweep concurrently), 32 for FP64
  if (lw <= 0) lw = fp64 ? 32 : 16;
  int P = next_pow2((nint + mt - 1) / mt);
  int M = pick_chunk((nint + P - 1) / P);
  if (M < 0 || P > 32) return s;  // unsupported length
  const int S = x_tile_stride(nx, fp64);
  // compiled: 64, 32, 16, 8 lines; 64 only as an explicit (tuned) choice
  // (64 lines: up to 512 threads; otherwise at most 256)
  int L = (lw == 64 && 64 * P <= 512) ? 64 : std::min(lw == 64 ? 32 : lw, 256 / P);
  if (L < 8) return s;
  auto lds = [&](int Lc) {
    size_t off = 16;
    off += (size_t)es * red_size(P, Lc + 1);
    off += (size_t)es * ((size_t)Lc * S + P * M + 2);
    if (aos) off += (size_t)es * Lc * S;
    off = (off + 15) & ~size_t(15);
    if (!uniform) off += (size_t)Lc * nx4 + P * M + 2;
    return off;
  };
  const size_t cap = L == 64 ? 100 * 1024 : 60 * 1024;  // 64 lines: one block per CU half
  while (L > 8 && lds(L) > cap && L * P > 64) L >>= 1;
  // the row traffic maps lanes as 16 vector columns x rows: whole groups of 16
  if (lds(L) > 160 * 1024 || (L * P) % 16 != 0) return LaunchShape{};
  s.M = M;
  s.P = P;
  s.LW = L;
  s.threads = L * P;
  long long nlines = (long long)(ny - 2) * (nz - 2);
  s.blocks = (int)((nlines + L - 1) / L);
  s.lds = lds(L);
  s.S = S;
  return s;
}

LaunchShape plan_yz(int nx, int n_along, int n_other, bool fp64, int mt, int tw) {
  LaunchShape s{};
  const int es = fp64 ? 8 : 4;
  const int nint = n_along - 2;
  // FP64 chunks stop at 16 rows (lane state in registers); by default 12,
  // which keeps three waves per SIMD resident, unless a line would need
  // more than 32 of them
  if (mt <= 0) mt = fp64 ? ((nint + 11) / 12 <= 32 ? 12 : 16) : 20;
  if (fp64) mt = std::min(mt, 16);
  int P = (nint + mt - 1) / mt;
  if (P > 32) return s;  // unsupported length
  const int M = pick_chunk((nint + P - 1) / P);
  if (M < 0) return s;
  P = (nint + M - 1) / M;
  const int nrow = std::max(n_along, P * M + 2);  // LDS tile rows
  auto lds = [&](int tw) {
    return (size_t)es * red_size(P, tw + 1) + (size_t)es * nrow * (tw + 1) + (size_t)nrow * tw + 16;
  };
  // Tile width (measured on 161^3 batches): FP32 arithmetic runs best with
  // 32 x per tile (one 128-byte line per node row) when that fits 512
  // threads and 80 KB of LDS; FP64 arithmetic is bound by its arithmetic
  // and runs best on 16-wide tiles (more, smaller blocks).
  int TW = 16;
  if (tw == 32 || tw <= 0) {
    if (!fp64 && 32 * P <= 512 && lds(32) <= 80 * 1024) TW = 32;
  }
  if (tw == 32 && TW != 32) return s;  // asked for a width that does not fit
  if (TW * P > 512 || lds(TW) > 160 * 1024) return s;
  const int ntx = (nx - 2) / TW + 1;
  s.M = M;
  s.P = P;
  s.LW = TW;
  s.threads = TW * P;
  s.blocks = ntx * (n_other - 2);
  s.lds = lds(TW);
  s.S = nrow;
  return s;
}

// Elimination constants of uniform chunks of M rows with face coefficient
// re: the leak recurrences of chunk_eliminate in double, stored in A.
template <typename A>
static void fill_tab_row(ChunkTab<A>& tb, int t, double re, int M, int nint) {
  double inv[kMaxChunk] = {0}, ga[kMaxChunk] = {0}, al[kMaxChunk] = {0};
  double lam = 1.0, tau = 0.0, s = 0.0, G = 1.0;
  for (int k = 1; k < M; ++k) {
    const double den = 1.0 + re + re * (tau + lam);
    inv[k] = 1.0 / den;
    lam = re * lam * inv[k];
    const double gam = re * inv[k];
    tau = (1.0 + re * tau) * inv[k];
    al[k] = -lam;
    ga[k] = -gam;
    if (k <= M - 2) {
      s += tau * G;
      G *= gam;
    }
    if (k == M - 1) {
      tb.rl_a[t] = (A)lam;
      tb.rl_c[t] = (A)gam;
      tb.rl_l[t] = (A)tau;
    }
  }
  for (int k = 0; k < kMaxChunk; ++k) {
    tb.inv[t][k] = (A)inv[k];
    tb.ga[t][k] = (A)ga[k];
    tb.al[t][k] = (A)al[k];
  }
  tb.re[t] = (A)re;
  tb.rf_c[t] = (A)(re * G);
  tb.rf_l[t] = (A)(1.0 + re * s);
  // a line's last chunk ending at row kt < M - 1: the same rows up to kt,
  // whose right face goes to the Dirichlet node (gamma 0, leak 1 + re);
  // the rows past kt are identity rows and add nothing
  const int kt = nint >= 1 ? (nint - 1) % M : 0;
  tb.rf_lt[t] = tb.rf_l[t];
  if (kt >= 1 && kt <= M - 2) {
    double lm = 1.0, ta = 0.0, st = 0.0, Gt = 1.0;
    for (int k = 1; k <= kt; ++k) {
      const double iv = 1.0 / (1.0 + re + re * (ta + lm));
      lm = re * lm * iv;
      const double gm = k == kt ? 0.0 : re * iv;
      ta = (1.0 + (k == kt ? re : 0.0) + re * ta) * iv;
      st += ta * Gt;
      Gt *= gm;
    }
    tb.rf_lt[t] = (A)(1.0 + re * st);
  }
}

template <typename A>
void fill_chunk_tab(ChunkTab<A>& tb, double re_solvent, double re_solute, int M, int nint) {
  tb = ChunkTab<A>{};
  fill_tab_row(tb, 0, re_solvent, M, nint);
  fill_tab_row(tb, 1, re_solute, M, nint);
}
template void fill_chunk_tab<float>(ChunkTab<float>&, double, double, int, int);
template void fill_chunk_tab<double>(ChunkTab<double>&, double, double, int, int);

template <typename T>
void shape_args(SweepArgs<T>& a, int dir, const LaunchShape& s) {
  a.M = s.M;
  a.P = s.P;
  a.LW = s.LW;
  a.S = s.S;
}
template void shape_args<float>(SweepArgs<float>&, int, const LaunchShape&);
template void shape_args<double>(SweepArgs<double>&, int, const LaunchShape&);

// y/z: the Crank-Nicolson right-hand side is a run-time flag of the general
// variant only, so the plain and flow kernels carry none of its code
template <typename T>
int sweep_variant(const SweepArgs<T>* a, int n) {
  bool general = false, flow = false;
  for (int f = 0; f < n; ++f) {
    // the face rule by location is decoded only in the general variant
    general = general || a[f].src_stage != 0 || a[f].mode != MODE_INPLACE || a[f].cn ||
              a[f].face_loc;
    flow = flow || (a[f].post_nl && a[f].mask);
  }
  return general ? kYzGeneral : (flow ? kYzFlow : kYzPlain);
}
template int sweep_variant<float>(const SweepArgs<float>*, int);
template int sweep_variant<double>(const SweepArgs<double>*, int);

template <typename T>
int sweep_cn(const SweepArgs<T>* a, int n) {
  // the CN-capable x kernel also decodes the face rule by location
  for (int f = 0; f < n; ++f)
    if (a[f].cn || a[f].face_loc) return 1;
  return 0;
}
template int sweep_cn<float>(const SweepArgs<float>*, int);
template int sweep_cn<double>(const SweepArgs<double>*, int);

// Per-kernel timing: when set, the next sweep launches record the kernel's
// own start and stop in these events (hipExtLaunchKernelGGL), so the
// elapsed time excludes the dispatch of the launch.  Per host thread.
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;

void set_sweep_launch_events(hipEvent_t start, hipEvent_t stop) {
  t_ev_start = start;
  t_ev_stop = stop;
}

// Dynamic LDS above 64 KB (up to the 160 KB of a CU) must be allowed per
// kernel before the launch.
template <typename K>
static hipError_t allow_lds(K kernel, size_t lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename T, typename A, int L, bool CN>
static hipError_t launch_x_l(const SweepArgs<T>* args, const int2* work, int nbu, int nblocks,
                             const LaunchShape& s, hipStream_t st) {
  // the block size must stay within the instantiation's launch bound
  if (s.threads > (L == 64 ? 512 : 256) || s.threads != L * s.P) return hipErrorInvalidValue;
  dim3 g(nblocks), blk(s.threads);
  switch (s.M) {
#define NPB_X_CASE(MM)                                                                 \
  case MM: {                                                                           \
    hipError_t e = allow_lds(sweep_x_kernel<T, A, MM, L, CN>, s.lds);                  \
    if (e != hipSuccess) return e;                                                     \
    if (t_ev_start)                                                                    \
      hipExtLaunchKernelGGL((sweep_x_kernel<T, A, MM, L, CN>), g, blk, (uint32_t)s.lds, st, \
                            t_ev_start, t_ev_stop, 0u, args, work, nbu);               \
    else                                                                               \
      hipLaunchKernelGGL((sweep_x_kernel<T, A, MM, L, CN>), g, blk, s.lds, st, args, work, \
                         nbu);                                                         \
  } break;
    NPB_X_CASE(4)
    NPB_X_CASE(8)
    NPB_X_CASE(12)
    NPB_X_CASE(16)
    NPB_X_CASE(20)
#undef NPB_X_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, typename A, bool CN>
static hipError_t launch_x_cn(const SweepArgs<T>* args, const int2* work, int nbu, int nblocks,
                              const LaunchShape& s, hipStream_t st) {
  if (s.LW == 64) return launch_x_l<T, A, 64, CN>(args, work, nbu, nblocks, s, st);
  if (s.LW == 32) return launch_x_l<T, A, 32, CN>(args, work, nbu, nblocks, s, st);
  if (s.LW == 16) return launch_x_l<T, A, 16, CN>(args, work, nbu, nblocks, s, st);
  if (s.LW == 8) return launch_x_l<T, A, 8, CN>(args, work, nbu, nblocks, s, st);
  return hipErrorInvalidValue;
}

template <typename T, typename A>
hipError_t launch_sweep_x(const SweepArgs<T>* args, const int2* work, int nbu, int nblocks,
                          int cn, const LaunchShape& s, hipStream_t st) {
  if (nblocks < 1 || (nbu <= 0 && !work)) return hipErrorInvalidValue;
  return cn ? launch_x_cn<T, A, true>(args, work, nbu, nblocks, s, st)
            : launch_x_cn<T, A, false>(args, work, nbu, nblocks, s, st);
}

template <typename T, typename A, int VAR, int TW>
static hipError_t launch_yz_tw(const SweepArgs<T>* args, const int2* work, int nbu, int nblocks,
                               int dir, const LaunchShape& s, hipStream_t st) {
  if (s.threads > 512 || s.threads != TW * s.P) return hipErrorInvalidValue;
  dim3 g(8 * ((nblocks + 7) / 8)), blk(s.threads);
  switch (s.M) {
#define NPB_YZ_CASE(MM)                                                                      \
  case MM: {                                                                                \
    hipError_t e = allow_lds(sweep_yz_kernel<T, A, MM, VAR, TW>, s.lds);                    \
    if (e != hipSuccess) return e;                                                          \
    if (t_ev_start)                                                                         \
      hipExtLaunchKernelGGL((sweep_yz_kernel<T, A, MM, VAR, TW>), g, blk, (uint32_t)s.lds,  \
                            st, t_ev_start, t_ev_stop, 0u, args, work, nbu, dir, nblocks);  \
    else                                                                                    \
      hipLaunchKernelGGL((sweep_yz_kernel<T, A, MM, VAR, TW>), g, blk, s.lds, st, args,     \
                         work, nbu, dir, nblocks);                                          \
  } break;
    NPB_YZ_CASE(4)
    NPB_YZ_CASE(8)
    NPB_YZ_CASE(12)
    NPB_YZ_CASE(16)
#undef NPB_YZ_CASE
    case 20:
      // planned only for FP32 arithmetic (FP64 chunks stop at 16 rows)
      if constexpr (sizeof(A) == 4) {
        hipError_t e = allow_lds(sweep_yz_kernel<T, A, 20, VAR, TW>, s.lds);
        if (e != hipSuccess) return e;
        if (t_ev_start)
          hipExtLaunchKernelGGL((sweep_yz_kernel<T, A, 20, VAR, TW>), g, blk, (uint32_t)s.lds,
                                st, t_ev_start, t_ev_stop, 0u, args, work, nbu, dir, nblocks);
        else
          hipLaunchKernelGGL((sweep_yz_kernel<T, A, 20, VAR, TW>), g, blk, s.lds, st, args,
                             work, nbu, dir, nblocks);
        break;
      }
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// tile widths compiled: 16 and 32 for FP32 arithmetic, 16 for FP64
template <typename T, typename A, int VAR>
static hipError_t launch_yz_var(const SweepArgs<T>* args, const int2* work, int nbu, int nblocks,
                                int dir, const LaunchShape& s, hipStream_t st) {
  if (s.LW == 16) return launch_yz_tw<T, A, VAR, 16>(args, work, nbu, nblocks, dir, s, st);
  if constexpr (sizeof(A) == 4) {
    if (s.LW == 32) return launch_yz_tw<T, A, VAR, 32>(args, work, nbu, nblocks, dir, s, st);
  }
  return hipErrorInvalidValue;
}

template <typename T, typename A>
hipError_t launch_sweep_yz(const SweepArgs<T>* args, const int2* work, int nbu, int nblocks,
                           int dir, int var, const LaunchShape& s, hipStream_t st) {
  if (nblocks < 1 || (nbu <= 0 && !work)) return hipErrorInvalidValue;
  if (var == kYzGeneral)
    return launch_yz_var<T, A, kYzGeneral>(args, work, nbu, nblocks, dir, s, st);
  if (var == kYzFlow) return launch_yz_var<T, A, kYzFlow>(args, work, nbu, nblocks, dir, s, st);
  return launch_yz_var<T, A, kYzPlain>(args, work, nbu, nblocks, dir, s, st);
}

#define NPB_INST(T, A)                                                                          \
  template hipError_t launch_sweep_x<T, A>(const SweepArgs<T>*, const int2*, int, int, int,    \
                                           const LaunchShape&, hipStream_t);                    \
  template hipError_t launch_sweep_yz<T, A>(const SweepArgs<T>*, const int2*, int, int, int,   \
                                            int, const LaunchShape&, hipStream_t);
NPB_INST(float, float)
NPB_INST(float, double)
NPB_INST(double, double)
#undef NPB_INST

}  // namespace npb
