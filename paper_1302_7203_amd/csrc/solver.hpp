// Per-eigenvalue steps of the shift-and-invert method for real symmetric
// arrowhead matrices (Jakovcevic Stor, Slapnicar, Barlow, "Accurate eigenvalue
// decomposition of arrowhead matrices and applications"), written for a group
// of G lanes of one wavefront that cooperate on one eigenvalue: lane `ln`
// takes the pole terms j = ln, ln+G, ... and the partial sums are combined by
// an XOR butterfly, so every lane of the group ends with the same bits.
//
// Three problem kinds share these routines:
//   ARROW  A = [diag(d) z; z^T alpha]                              (Sec. 1)
//   DPR1   D + rho u u^T, reduced to the arrowhead with poles d_1..d_{n-1},
//          zeta_j^2 = rho u_j^2 (d_j - d_n), alpha = d_n + rho u^T u  (Sec. 6.3)
//   SVD    B = [diag(d) z; 0 alpha] through B^T B, the arrowhead with poles
//          d_j^2, shaft d_j zeta_j, corner alpha^2 + z^T z              (Sec. 6.2)
// They differ only in how a pole difference is formed: d_j - d_i, or
// (d_j - d_i)(d_j + d_i) for SVD, which keeps it accurate (Sec. 6.2).
//
// A shift is held as (pv, s): the pole value pv (an unsquared d_i, or 0) plus
// an offset s; the shifted pole differences are e_j = pdiff(d_j, pv) - s.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd.hpp"

namespace ahd {

// KIND_HERM: a Hermitian arrowhead, solved as the real arrowhead with shaft
// |z| (Sec. 6.1); the root and check stages treat it as KIND_ARROW.
enum Kind { KIND_ARROW = 0, KIND_DPR1 = 1, KIND_SVD = 2, KIND_HERM = 3 };

// per-eigenvalue info bits (the public header repeats them)
constexpr uint32_t INFO_DD_B = 1u;        // b evaluated in double-double (Theorem 6)
constexpr uint32_t INFO_REMEDY_A = 2u;    // shifted to the other neighbouring pole (Remark 2(a))
constexpr uint32_t INFO_REMEDY_B = 4u;    // DPR1 inverse at a shift near lambda (Remark 2(b))
constexpr uint32_t INFO_NEAR_ZERO = 8u;   // eigenvalue from the inverse of A (Remark 1)
constexpr uint32_t INFO_REDUCIBLE = 16u;  // zero shaft entry or repeated pole: not solved
constexpr uint32_t INFO_NONFINITE = 32u;  // non-finite input: not solved
constexpr uint32_t INFO_KB_LARGE = 64u;   // K_b beyond what double-double resolves (Sec. 4 footnote)
constexpr uint32_t INFO_KNU_LARGE = 128u; // K_nu above threshold after the remedies
constexpr uint32_t INFO_BAD_INPUT = 256u; // kind-specific domain error (SVD: d_j = 0)
constexpr uint32_t INFO_POLE_SHIFT = 512u;// DPR1 eigenvalue re-measured from the pole d_n
constexpr uint32_t INFO_DEFLATED = 1024u; // eigenpair deflated from a reducible arrowhead (Sec. 1)
constexpr uint32_t INFO_F0_UNRESOLVED = 2048u; // Remark 1: f(0) is 0 to the reach of the exact sum
constexpr uint32_t INFO_NOT_SOLVED = INFO_REDUCIBLE | INFO_NONFINITE | INFO_BAD_INPUT;

constexpr double EPS = 2.220446049250313080847e-16;  // 2^-52, eps of Algorithm 3
constexpr int MAX_BISECT = 4000;
constexpr int MAX_RATIONAL = 60;     // rational steps before falling back to bisection steps
constexpr int RATIONAL_TO_BISECT = 14;
#ifndef AHD_START_MODEL
#define AHD_START_MODEL 1
#endif
#ifndef AHD_EARLY2
#define AHD_EARLY2 24
#define AHD_EARLY1 36
#endif

enum RootMethod { ROOT_BISECT = 0, ROOT_RATIONAL = 1 };

struct Options {
  double tau_nu;     // K_nu threshold for the Remark 2 remedies
  double tau_zero;   // threshold on (|d_i| + |mu|) / |lambda| for Remark 1
  int fp64_b;        // 1: b by Algorithm 2 in FP64 only (negative control)
  int remedies;      // 0: skip the K_nu and near-zero remedies
  int root;          // RootMethod for the extreme eigenvalue of the inverse
  double tau_b;      // > 0: b from an FP64 pass alone where its K_b <= tau_b
                     // (Algorithm 5's test), else the double-double pass; 0: always
  int check_lanes;   // batched plans: lanes per eigenvalue in the check stage (0: the first pass's)
};

// Read-only view of one problem after normalisation (sorted order).
struct Prob {
  int n;              // matrix order
  int m;              // number of arrowhead poles (n - 1)
  int nsorted;        // entries of ds/zs (DPR1: n, else n - 1)
  const double* ds;   // sorted d (descending d, or descending |d| for SVD)
  const double* zs;   // z (or u for DPR1) in the same order
  const double* ch;   // arrowhead shaft squared, hi part (m)
  const double* cl;   // lo part
  const double* dz;   // |shaft_j| (m)
  dd corner;          // arrowhead corner
  double rho;         // DPR1 weight
};

template <int KIND>
__host__ __device__ inline double pval(double d) {
  if constexpr (KIND == KIND_SVD) return d * d;
  else return d;
}

template <int KIND>
__host__ __device__ inline double pdiff(double dj, double di) {
  if constexpr (KIND == KIND_SVD) return (dj - di) * (dj + di);
  else return dj - di;
}

template <int KIND>
__host__ __device__ inline dd pdiff_dd(double dj, double di) {
  if constexpr (KIND == KIND_SVD) return dd_mul(two_sum(dj, -di), two_sum(dj, di));
  else return two_sum(dj, -di);
}

template <int KIND>
__host__ __device__ inline dd pval_dd(double d) {
  if constexpr (KIND == KIND_SVD) return two_prod(d, d);
  else return dd_from(d);
}

// Reciprocals (x finite, nonzero and in the normal range, as every
// denominator here is).  On the device the hardware estimate is good to about
// 2^-24 relative; one Newton step brings it within 11 ulps and two to the
// correctly rounded value (measured over 4M operands spanning 2^+-300).  On
// the host each is an ordinary division.
//   recip_est: the bare estimate, where only a sign is used;
//   recip1:    one step, where a following correction absorbs the error;
//   recip:     two steps, everywhere else.
__host__ __device__ inline double recip_est(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcp(x);
#else
  return 1.0 / x;
#endif
}

__host__ __device__ inline double recip1(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
#else
  return 1.0 / x;
#endif
}

__host__ __device__ inline double recip(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / x;
#endif
}

// ---------------------------------------------------------------------------
// group reductions.  Every step adds a value and its partner's, so every lane
// of the group ends with the same bits.  Partners within 16 lanes come from
// DPP lane permutes (quad xor 1, quad xor 2, half-row mirror, row mirror);
// the 16- and 32-lane steps use the LDS crossbar (ds_bpermute).

#if defined(__HIP_DEVICE_COMPILE__)
template <int CTRL>
__device__ inline double dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
#endif

constexpr int DPP_QUAD_XOR1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;   // lane i <-> 7 - i within 8
constexpr int DPP_MIRROR = 0x140;        // lane i <-> 15 - i within 16

#if defined(__HIP_DEVICE_COMPILE__)
// Groups wider than a wavefront are whole blocks (blockDim.x == G): after the
// wavefront butterfly, lane 0 of each wavefront posts its value to LDS and
// every lane combines the NW posted values in wavefront order, so all lanes
// again hold identical bits.  Every lane of the block must reach the call.
template <int NW, class Op>
__device__ inline double block_combine(double v, Op op) {
  __shared__ double slot[NW];
  if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = slot[0];
#pragma unroll
  for (int q = 1; q < NW; ++q) r = op(r, slot[q]);
  __syncthreads();
  return r;
}
#endif

template <int G, class Op>
__host__ __device__ inline double greduce(double v, Op op) {
  static_assert(G <= 64 || G % 64 == 0, "a group is part of a wavefront or whole wavefronts");
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (G >= 2) v = op(v, dpp<DPP_QUAD_XOR1>(v));
  if constexpr (G >= 4) v = op(v, dpp<DPP_QUAD_XOR2>(v));
  if constexpr (G >= 8) v = op(v, dpp<DPP_HALF_MIRROR>(v));
  if constexpr (G >= 16) v = op(v, dpp<DPP_MIRROR>(v));
  if constexpr (G >= 32) v = op(v, __shfl_xor(v, 16, G > 64 ? 64 : G));
  if constexpr (G >= 64) v = op(v, __shfl_xor(v, 32, 64));
  if constexpr (G > 64) v = block_combine<G / 64>(v, op);
#endif
  return v;
}

struct OpAdd {
  __host__ __device__ double operator()(double a, double b) const { return a + b; }
};
struct OpMax {
  __host__ __device__ double operator()(double a, double b) const { return fmax(a, b); }
};
struct OpMin {
  __host__ __device__ double operator()(double a, double b) const { return fmin(a, b); }
};

template <int G>
__host__ __device__ inline double gsum(double v) { return greduce<G>(v, OpAdd()); }

template <int G>
__host__ __device__ inline double gmax(double v) { return greduce<G>(v, OpMax()); }

template <int G>
__host__ __device__ inline double gmin(double v) { return greduce<G>(v, OpMin()); }

template <int G>
__host__ __device__ inline dd gsum_dd(dd v) {
#if defined(__HIP_DEVICE_COMPILE__)
  constexpr int W = G > 64 ? 64 : G;
  if constexpr (G >= 2) v = dd_add(v, dd{dpp<DPP_QUAD_XOR1>(v.hi), dpp<DPP_QUAD_XOR1>(v.lo)});
  if constexpr (G >= 4) v = dd_add(v, dd{dpp<DPP_QUAD_XOR2>(v.hi), dpp<DPP_QUAD_XOR2>(v.lo)});
  if constexpr (G >= 8) v = dd_add(v, dd{dpp<DPP_HALF_MIRROR>(v.hi), dpp<DPP_HALF_MIRROR>(v.lo)});
  if constexpr (G >= 16) v = dd_add(v, dd{dpp<DPP_MIRROR>(v.hi), dpp<DPP_MIRROR>(v.lo)});
  if constexpr (G >= 32) v = dd_add(v, dd{__shfl_xor(v.hi, 16, W), __shfl_xor(v.lo, 16, W)});
  if constexpr (G >= 64) v = dd_add(v, dd{__shfl_xor(v.hi, 32, W), __shfl_xor(v.lo, 32, W)});
  if constexpr (G > 64) {
    constexpr int NW = G / 64;
    __shared__ double slot_hi[NW], slot_lo[NW];
    if ((threadIdx.x & 63) == 0) {
      slot_hi[threadIdx.x >> 6] = v.hi;
      slot_lo[threadIdx.x >> 6] = v.lo;
    }
    __syncthreads();
    dd r = {slot_hi[0], slot_lo[0]};
#pragma unroll
    for (int q = 1; q < NW; ++q) r = dd_add(r, dd{slot_hi[q], slot_lo[q]});
    __syncthreads();
    v = r;
  }
#endif
  return v;
}

// ---------------------------------------------------------------------------
// Lane ln's pole indices j = ln, ln + G, ... below m, visited as two runs: the
// indices below `excl` (f(j, false)) and those above it (f(j, true)); excl
// itself is skipped.  With excl outside [0, m) there is one run.  Splitting
// the loop at the excluded pole keeps every iteration free of a per-term test.
#ifndef AHD_TERM_UNROLL
#define AHD_TERM_UNROLL 4
#endif
constexpr int TERM_UNROLL = AHD_TERM_UNROLL;   // terms per unrolled loop trip

template <int G, class F>
__host__ __device__ inline void for_terms(int ln, int m, int excl, F&& f) {
  const int cut = (excl >= 0 && excl < m) ? excl : m;
  int j = ln;
#pragma unroll TERM_UNROLL
  for (; j < cut; j += G) f(j, false);
  if (j == excl) j += G;
#pragma unroll TERM_UNROLL
  for (; j < m; j += G) f(j, true);
}

// As for_terms, in the same order, with the loads of TERM_UNROLL terms issued
// together ahead of their arithmetic: load(j) returns term j's data and
// f(j, above, data) uses it.  Where a term's arithmetic is long (the
// double-double b pass) the compiler otherwise issues each term's loads just
// before its arithmetic and waits on them one term at a time.
struct v2 {   // two doubles of one term
  double a, b;
};

template <int G, class L, class F>
__host__ __device__ inline void for_terms_ld(int ln, int m, int excl, L&& load, F&& f) {
  using T = decltype(load(0));
  const int cut = (excl >= 0 && excl < m) ? excl : m;
  int j = ln;
  auto run = [&](int end, bool above) {
    for (; j + (TERM_UNROLL - 1) * G < end; j += TERM_UNROLL * G) {
      T t[TERM_UNROLL];
#pragma unroll
      for (int u = 0; u < TERM_UNROLL; ++u) t[u] = load(j + u * G);
#pragma unroll
      for (int u = 0; u < TERM_UNROLL; ++u) f(j + u * G, above, t[u]);
    }
    for (; j < end; j += G) f(j, above, load(j));
  };
  run(cut, false);
  if (j == excl) j += G;
  run(m, true);
}

// The positive zero of t^2 - beta t - s^2 (s >= 0), in the form that avoids
// cancellation.  beta and s are first brought below 2 by a power of two, so
// neither square leaves the exponent range: x-space quantities are of the
// order of 1/(lambda - d_i), whose square overflows once lambda lies within
// about 2^-512 of its pole, long before the quantities themselves do.
__host__ __device__ inline double pos_root(double beta, double s) {
  const double mx = fmax(fabs(beta), s);
  if (mx == 0.0) return 0.0;
  if (mx == INFINITY) return (beta == -INFINITY && s < INFINITY) ? 0.0 : INFINITY;
  const int k = ilogb(mx);
  const double b = ldexp(beta, -k), q = ldexp(s, -k);
  const double r = sqrt(fma(b, b, 4.0 * q * q));
  return (b >= 0.0) ? ldexp(0.5 * (b + r), k) : (2.0 * s) * (q / (r - b));
}

// ---------------------------------------------------------------------------
// Shift selection (Algorithm 1, first part): eigenvalue k (0-based, descending)
// lies in (d_k, d_{k-1}); the sign of the Pick function (eq. Pick) at the
// midpoint of that interval, evaluated in the frame shifted to d_k, tells
// which end-pole is nearer.  side = +1: lambda right of pole i ('R'),
// side = -1: left of it ('L').

template <int KIND, int G>
__host__ __device__ inline void select_shift(const Prob& P, int k, int ln, int& i, int& side) {
  const int m = P.m;
  if (k == 0) { i = 0; side = +1; return; }
  if (k == m) { i = m - 1; side = -1; return; }
  const double dk = P.ds[k];
  const double mid = 0.5 * pdiff<KIND>(P.ds[k - 1], dk);
  // only the sign of the Pick function at mid is used, and where the terms'
  // 2^-24 errors could flip it the eigenvalue is that near the midpoint, so
  // either end-pole is a valid shift: the bare reciprocal estimate suffices
  double s = 0.0;
  for_terms_ld<G>(ln, m, -1, [&](int j) { return v2{P.ds[j], P.ch[j]}; },
                  [&](int, bool, const v2& t) { s = fma(t.b, recip_est(pdiff<KIND>(t.a, dk) - mid), s); });
  s = gsum<G>(s);
  const double a = dd_to_d(dd_sub(P.corner, pval_dd<KIND>(dk)));
  const double fmid = (a - mid) - s;
  if (fmid < 0) { i = k; side = +1; }
  else { i = k - 1; side = -1; }
}

// ---------------------------------------------------------------------------
// One O(n) pass for pole i: the element b = [A_i^{-1}]_ii (eq. b_ob) and the
// Gershgorin interval of A_i^{-1} (eq. invAi) on the requested side.
// b in double-double follows Theorem 6: P and Q >= 0 are summed separately,
// with d_j - d_i, alpha - d_i and zeta_j^2 formed exactly.  K_b is eq. (K2).

struct BPass {
  double b, Kb, lo, hi;
  double x0;   // a start for the root in x = side*nu from a two-pole model (NaN: none)
};

// RUNS: split the term loop where FastTwoSum applies (a shorter loop body, a
// larger kernel); the results are the same bits either way.
template <int KIND, int G, bool FP64_B, bool RUNS = true>
__host__ __device__ inline BPass b_pass_t(const Prob& P, int i, int side, int ln) {
  const int m = P.m;
  const double di = P.ds[i];
  const double sg = (double)side;
  dd p1 = {0.0, 0.0}, p2 = {0.0, 0.0};  // sum over j < i (>= 0), j > i (<= 0)
  double f1 = 0.0, f2 = 0.0;            // the same sums in FP64 (Algorithm 2 only)
  // sum_{j != i} zeta_j^2 (gs / e_j)^2 with gs the power of two at or below
  // the distance to the nearest pole, so that every gs / e_j is at most 1
  double r2 = 0.0, r3 = 0.0;   // and sum zeta_j^2 (gs / e_j)^3, for the start model
  double dn = INFINITY;
  if (i > 0) dn = fabs(pdiff<KIND>(P.ds[i - 1], di));
  if (i + 1 < m) dn = fmin(dn, fabs(pdiff<KIND>(P.ds[i + 1], di)));
  const double gs = (dn > 0.0 && dn < INFINITY) ? ldexp(1.0, ilogb(dn)) : 1.0;
  struct Term {
    double d, ch, cl;
  };
  auto load = [&](int j) { return Term{P.ds[j], P.ch[j], FP64_B ? 0.0 : P.cl[j]}; };
  // ORD: how the exact difference d_j - d_i = e.hi + e.lo is formed -- 0 by
  // TwoSum (and, for SVD, the product of two), 1 by FastTwoSum(d_j, -d_i), valid
  // where |d_j| >= |d_i|, 2 by FastTwoSum(-d_i, d_j), valid where |d_j| <= |d_i|:
  // the same exact pair in 3 operations instead of 6
  auto term = [&](auto above_c, auto ord_c, const Term& t) {
    constexpr bool above = decltype(above_c)::value;
    constexpr int ord = decltype(ord_c)::value;
    const double ej = pdiff<KIND>(t.d, di);
    // delta_j, the diagonal of A_i^{-1}, within 11 ulps: the two-digit
    // quotient's remainder corrects its first digit, so c/e stays good to
    // about 2^-98, and the upper end below is widened for it
    const double rj = recip1(ej);
    if constexpr (FP64_B) {
      const double q = t.ch * rj;
      if (above) f2 += q; else f1 += q;
    } else {
      dd e;
      if constexpr (ord == 1) e = dd{ej, (-di) - (ej - t.d)};
      else if constexpr (ord == 2) e = dd{ej, t.d - (ej + di)};
      else e = pdiff_dd<KIND>(t.d, di);
      if (above) dd_acc_div2(p2, dd{t.ch, t.cl}, e, rj); else dd_acc_div2(p1, dd{t.ch, t.cl}, e, rj);
    }
    // zeta_j^2 (gs / e_j)^2 = w gs and zeta_j^2 (gs / e_j)^3 = w (gs / e_j) gs with
    // w = (zeta_j^2 / e_j)(gs / e_j) <= |zeta_j^2 / e_j|: the factor gs is applied
    // after the sums
    const double rs = rj * gs;
    const double w = (t.ch * rj) * rs;
    r2 += w;
#if AHD_START_MODEL
    r3 = fma(w, rs, r3);
#endif
  };
  // lane ln's poles j = ln, ln + G, ... of [j, end), loads of TERM_UNROLL terms ahead
  int j = ln;
  auto run = [&](int end, auto above_c, auto ord_c) {
    for (; j + (TERM_UNROLL - 1) * G < end; j += TERM_UNROLL * G) {
      Term t[TERM_UNROLL];
#pragma unroll
      for (int u = 0; u < TERM_UNROLL; ++u) t[u] = load(j + u * G);
#pragma unroll
      for (int u = 0; u < TERM_UNROLL; ++u) term(above_c, ord_c, t[u]);
    }
    for (; j < end; j += G) term(above_c, ord_c, load(j));
  };
  using below_t = std::integral_constant<bool, false>;
  using above_t = std::integral_constant<bool, true>;
  using two_sum_t = std::integral_constant<int, 0>;
  using fast_t = std::integral_constant<int, 1>;
  using fast_swap_t = std::integral_constant<int, 2>;
  if constexpr (FP64_B || KIND == KIND_SVD || !RUNS) {
    run(i, below_t(), two_sum_t());
    if (j == i) j += G;
    run(m, above_t(), two_sum_t());
  } else if (di >= 0.0) {
    // j < i: d_j > d_i >= 0; j > i: |d_j| < d_i until d_j <= -d_i (from j2 on)
    int lo = i + 1, hi = m;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (P.ds[mid] <= -di) hi = mid; else lo = mid + 1;
    }
    run(i, below_t(), fast_t());
    if (j == i) j += G;
    run(lo, above_t(), fast_swap_t());
    run(m, above_t(), fast_t());
  } else {
    // j > i: d_j < d_i < 0; j < i: d_j >= -d_i up to j1, then |d_j| < -d_i
    int lo = 0, hi = i;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (P.ds[mid] < -di) hi = mid; else lo = mid + 1;
    }
    run(lo, below_t(), fast_t());
    run(i, below_t(), fast_swap_t());
    if (j == i) j += G;
    run(m, above_t(), fast_t());
  }
  r2 = gsum<G>(r2) * gs;
#if AHD_START_MODEL
  r3 = gsum<G>(r3) * gs;
#endif
  const dd a = dd_sub(P.corner, pval_dd<KIND>(di));  // a = alpha - d_i
  const double ci = P.ch[i];
  BPass r;
  double num_abs;
  if constexpr (FP64_B) {
    // Algorithm 2: b = (-a + sum_{j<i} + sum_{j>i}) / zeta_i^2, all in FP64
    f1 = gsum<G>(f1);
    f2 = gsum<G>(f2);
    r.b = ((-a.hi + f1) + f2) / ci;
    num_abs = fabs(r.b) * ci;
  } else {
    p1 = gsum_dd<G>(dd_norm(p1));
    p2 = gsum_dd<G>(dd_norm(p2));
    f1 = p1.hi;
    f2 = p2.hi;
    dd pp, qq;
    if (-a.hi > 0) { pp = dd_add(dd_neg(a), p1); qq = dd_neg(p2); }
    else { pp = p1; qq = dd_sub(a, p2); }
    const dd num = dd_sub(pp, qq);
    r.b = dd_to_d(dd_div(num, dd{P.ch[i], P.cl[i]}));
    num_abs = fabs(num.hi);
  }
  r.Kb = (fabs(a.hi) + fabs(f1) + fabs(f2)) / num_abs;
  // The bracket of the extreme eigenvalue on the requested side, in the
  // variable x = side*nu.  Lower end: the rightmost pole of A_i^{-1}'s Pick
  // function, y = side*delta_j of the pole next to d_i on that side (the
  // smallest |e_j| of that sign), or 0 with none (Gershgorin's rightmost
  // centre, as in Algorithm 3).  Upper end: right of y the Pick function is
  // h(x) = c0 - x + sum_j R_j/(x - p_j) with every pole p_j <= y and R_j > 0,
  // R_j = zeta_j^2/(zeta_i^2 e_j^2) and R = 1/zeta_i^2 at p = 0, so
  // h(x) <= c0 - x + R_tot/(x - y); the zero of that bound, y + u with
  // u^2 - (c0 - y) u - R_tot = 0, lies right of the wanted zero.  It takes
  // one sum of zeta_j^2/e_j^2 instead of the Gershgorin discs' sum and maximum
  // and is mostly much the tighter, which saves rational steps too.
  const int jn = i - side;
  const double xl = (jn >= 0 && jn < m) ? fmax(sg * recip(pdiff<KIND>(P.ds[jn], di)), 0.0) : 0.0;
  // the square root of the total residue (sum_j c_j / e_j^2 + 1) / zeta_i^2
  const double srt = (sqrt(fma(gs, gs, r2)) / gs) / sqrt(ci);
  const double u = pos_root(sg * r.b - xl, srt);
  const double xh = (xl + u) * (1.0 + 64.0 * EPS);
  if (side > 0) { r.lo = xl; r.hi = xh; }
  else { r.lo = -xh; r.hi = -xl; }
  r.x0 = NAN;
#if AHD_START_MODEL
  // A start nearer the zero than xh: keep the nearest pole y = xl and the next
  // one on the same side exact with their residues and put the rest of the
  // residue mass at its mean position p (first moment over mass), so
  // h(x) ~ c0 - x + ry/(x - y) + r2/(x - y2) + Rr/(x - p).
  // In units of 1/gs (x' = gs x) every quantity is of moderate size.  The model
  // lies below the bound whose zero is xh (p <= y), so it is negative there;
  // it is decreasing and convex right of y, and Newton's steps from a point left
  // of its zero approach the zero from the left: a first step from xh, then steps
  // from wherever it lands, kept inside (y, xh).
  if (jn >= 0 && jn < m && xl > 0.0) {
    const double rci = 1.0 / ci;
    const double rg = gs * recip(pdiff<KIND>(P.ds[jn], di));
    const double ry = P.ch[jn] * rci * (rg * rg);
    const double rt = (r2 + gs * gs) * rci;
    const double rr = rt - ry;
    const double yy = xl * gs, c0 = sg * r.b * gs, xhh = xh * gs;
    double m1 = sg * r3 * rci - ry * yy;   // first moment of the rest (the pole at 0 adds none)
    // the next pole on the same side is kept exact too
    const int j2 = jn - side;
    double y2 = 0.0, rx2 = 0.0;
    if (j2 >= 0 && j2 < m) {
      const double g2 = gs * recip(pdiff<KIND>(P.ds[j2], di));
      y2 = sg * g2;
      rx2 = P.ch[j2] * rci * (g2 * g2);
    }
    const double rrest = rr - rx2;
    m1 -= rx2 * y2;
    if (rr > 0.0 && yy < xhh) {
      const double pp = rrest > 0.0 ? fmin(m1 / rrest, yy) : 0.0;
      const double rq = fmax(rrest, 0.0);
      // the model is only a start, good to about 1e-3 of the zero: four steps
      // with the fast reciprocal solve it well past that
      double x = xhh;
      for (int k = 0; k < 4; ++k) {
        const double a1 = recip(x - yy), a2 = recip(x - pp), a3 = recip(x - y2);
        const double h = c0 - x + ry * a1 + rq * a2 + rx2 * a3;
        const double dh = -1.0 - ry * a1 * a1 - rq * a2 * a2 - rx2 * a3 * a3;
        double xn = x - h * recip(dh);
        if (!(xn > yy)) xn = 0.5 * (x + yy);
        if (!(xn < xhh)) xn = xhh;
        x = xn;
      }
      r.x0 = sg * (x / gs);   // back to nu
    }
  }
#endif
  return r;
}

// the FP64-only variant is the negative control of Algorithm 2; the choice is
// made once per call so that the term loop carries no branch.  For the
// remedies, rare enough that code size matters more than the loop body.
template <int KIND, int G>
__host__ __device__ inline BPass b_pass(const Prob& P, int i, int side, int ln, int fp64_b) {
  return fp64_b ? b_pass_t<KIND, G, true>(P, i, side, ln) : b_pass_t<KIND, G, false, false>(P, i, side, ln);
}

// ---------------------------------------------------------------------------
// Bisection (Algorithm 3) for the extreme eigenvalue nu of A_i^{-1} in
// (lo, hi].  Its Pick function is
//   g(nu) = b - nu - sum_{j != i} w_j^2 / (delta_j - nu) - w_zeta^2 / (0 - nu)
// and with delta_j = 1/e_j, w_j = -zeta_j/(e_j zeta_i), w_zeta = 1/zeta_i
// each term is  w_j^2/(delta_j - nu) = c_j / (zeta_i^2 e_j (1 - nu e_j)),
// so  g(nu) = b - nu - (S(nu) - 1/nu) / zeta_i^2,
//   S(nu) = sum_{j != i} c_j / (e_j (1 - nu e_j)).
// On either exterior side all terms of S - 1/nu share one sign, so the sum
// has no cancellation and may be accumulated in any order.

template <int KIND, int G>
__host__ __device__ inline double bisect_inverse(const Prob& P, int i, double b, double lo, double hi,
                                                 int ln, int* iters) {
  const int m = P.m;
  const double di = P.ds[i];
  const double ci = P.ch[i];
  double mid = 0.5 * (lo + hi);
  int it = 0;
  while ((hi - lo) / fabs(mid) > 2.0 * EPS && it < MAX_BISECT) {
    double S = 0.0;
    for_terms<G>(ln, m, i, [&](int j, bool) {
      const double e = pdiff<KIND>(P.ds[j], di);
      S = fma(P.ch[j], recip(e * fma(-mid, e, 1.0)), S);
    });
    S = gsum<G>(S);
    const double g = (b - mid) - (S - 1.0 / mid) / ci;
    if (g > 0) lo = mid; else hi = mid;
    mid = 0.5 * (lo + hi);
    ++it;
  }
  if (iters) *iters = it;
  return hi;
}

// ---------------------------------------------------------------------------
// Secular (rational) iteration for the same exterior eigenvalue.  With the
// poles of the inverse, delta_j = 1/e_j, and weights W_j = w_j^2 the Pick
// function reads g(nu) = b - nu + psi(nu), psi(nu) = sum_k W_k / (nu - delta_k),
// and on the exterior side all terms of psi share one sign.  In the variable
// x = side * nu the problem takes the one form
//     h(x) = c0 - kappa x + psi_x(x) = 0,  x > y = max_k side*delta_k,
// with psi_x positive, decreasing and convex.  Each step fits psi_x by
// A/(x - y) + B through its value and slope at the current point (the
// nearest pole carries the singularity) and solves the fitted equation in
// closed form; a step that leaves the bracket kept from the signs of h is
// replaced by the bracket midpoint, and after RATIONAL_TO_BISECT steps only
// midpoints are taken.  One O(n) pass per step gives psi and psi'.

// sums over j != excl of  c_j / (e_j (nu e_j - 1)),  c_j / (nu e_j - 1)^2  and
// nu c_j e_j / (nu e_j - 1)^3, with e_j = pdiff(d_j, pv) - s (the pole terms of
// psi and of its first two derivatives, up to constant factors); OFF = false
// when the offset s is known to be zero.  The third sum is taken times nu: it
// is then of the size of the second, whereas the plain sum of c_j e_j v_j^3
// underflows when the poles are as small as 1e-220 and nu as large as 1e220.
template <int KIND, int G, bool OFF>
__host__ __device__ inline void psi_pass(const Prob& P, double pv, double s, int excl, double nu, int ln,
                                         double& sum, double& dsum, double& d2sum) {
  double a = 0.0, b = 0.0, c = 0.0;
  for_terms_ld<G>(ln, P.m, excl, [&](int j) { return v2{P.ds[j], P.ch[j]}; }, [&](int, bool, const v2& t) {
    const double e = OFF ? pdiff<KIND>(t.a, pv) - s : pdiff<KIND>(t.a, pv);
    const double q = recip(e * fma(nu, e, -1.0));
    const double v = e * q;                // 1 / (nu e - 1)
    a = fma(t.b, q, a);
    const double d1 = (t.b * v) * v;
    b += d1;
    c = fma(d1, v, c);
  });
  sum = gsum<G>(a);
  dsum = gsum<G>(b);
  // the third sum's terms d1 (nu e) v are d1 (1 + v), since nu e v = 1 + v: it is
  // the second sum plus sum d1 v.  Where the shift is the nearest pole, |nu e| >= 2
  // near the root for every pole, so 1 + v lies in [2/3, 2] and nothing cancels
  d2sum = dsum + gsum<G>(c);
}

// The same pass on groups of gc lanes, gc one of G, 2G, ..., 64 chosen at run
// time (the same in every lane of the wavefront): each width is its own
// compiled loop, so the stride and the butterfly stay compile-time.
template <int KIND, bool OFF, int G>
__host__ __device__ inline void psi_pass_wide(const Prob& P, double pv, double s, int excl, double nu, int ln, int gc,
                                              double& sum, double& dsum, double& d2sum) {
  if constexpr (G < 64) {
    if (gc > G) {
      psi_pass_wide<KIND, OFF, 2 * G>(P, pv, s, excl, nu, ln, gc, sum, dsum, d2sum);
      return;
    }
  }
  psi_pass<KIND, G, OFF>(P, pv, s, excl, nu, ln, sum, dsum, d2sum);
}

// The rational step in x-space: the zero of c0 - kappa x + A/(x - p) + B with
// A, B fitted to psi_x and its slope at x and the pole p either the nearest
// pole y of psi_x or p = x + 2 psi'/psi'' (the pole that also matches psi'';
// it never lies right of y since every pole is left of x).  NaN when the
// fitted equation has no zero right of p.
__host__ __device__ inline double rational_candidate(double x, double psi_x, double dpsi_x, double pole, double c0,
                                                     int kappa) {
  // A = -psi' u^2, B = psi_x - A / u (psi' <= 0).  The zero un = u t is taken
  // in units of u, t^2 - (beta / u) t + psi' = 0: A itself, of the order of
  // x^2, would overflow when x passes about 2^512, while beta / u and psi'
  // are ratios of x-sized quantities
  const double u = x - pole;
  const double B = fma(dpsi_x, u, psi_x);
  double un = NAN;
  if (kappa) {
    const double bb = (c0 + B - pole) / u;
    const double r = sqrt(fma(bb, bb, -4.0 * dpsi_x));
    un = u * ((bb >= 0) ? 0.5 * (bb + r) : -2.0 * dpsi_x / (r - bb));
  } else {
    const double beta = c0 + B;
    if (beta < 0) un = (dpsi_x * u) * (u / beta);
  }
  return (un > 0) ? pole + un : NAN;
}

// Midpoint of a bracket 0 <= lo < hi in the ordering of the FP64 bit patterns
// (monotone for non-negative numbers): the arithmetic midpoint when lo and hi
// are within a binade or two, the geometric one when they are decades apart.
__host__ __device__ inline double bits_mid(double lo, double hi) {
  uint64_t a, b;
  lo += 0.0;   // -0 -> +0
  hi += 0.0;
  __builtin_memcpy(&a, &lo, sizeof a);
  __builtin_memcpy(&b, &hi, sizeof b);
  const uint64_t c = a + (b - a) / 2;
  double r;
  __builtin_memcpy(&r, &c, sizeof r);
  return r;
}

// Next point of the safeguarded iteration and whether to stop.  During the
// rational phase the second-order candidate is taken when it lies inside the
// bracket, else the nearest-pole candidate, else the midpoint.  Candidates
// that make slow progress across a bracket spanning decades are replaced by
// the midpoint (see below).  Stop when a
// candidate no longer moves x, when |h| is down to its rounding level hnoise,
// or when the bracket is within 4 ulps.
__host__ __device__ inline double rational_next(double x, double h, double hnoise, double psi_x, double dpsi_x,
                                                double d2psi_x, double y, double c0, int kappa, double lo, double hi,
                                                int it, double prev_step, int hi_open, int* done) {
  *done = 0;
  if ((hi - lo) <= 4.0 * EPS * fabs(x)) { *done = 1; return x; }
  if (it < RATIONAL_TO_BISECT) {
    double cand = NAN;
    if (d2psi_x > 0) {
      const double pe = x + 2.0 * dpsi_x / d2psi_x;
      if (pe <= y && pe < x) cand = rational_candidate(x, psi_x, dpsi_x, pe, c0, kappa);
    }
    if (!(cand > lo && cand < hi)) cand = rational_candidate(x, psi_x, dpsi_x, y, c0, kappa);
    if (cand == cand && (fabs(cand - x) <= 2.0 * EPS * fabs(cand) || fabs(h) <= hnoise)) {
      *done = 1;
      return (cand > lo && cand < hi) ? cand : x;
    }
    // the zero may sit at an upper bound that was never evaluated (to within
    // rounding): go there rather than bisect towards it
    if (hi_open && cand >= hi) return hi;
    // a bracket spanning decades above a positive end: slow steps -- no less
    // than 0.3 times the previous one, or, right of the zero, a move left by
    // less than a factor 4 -- are replaced by its (near-geometric) bit-pattern
    // midpoint; far from the zero a sum of poles spread over many decades
    // makes the one-pole model advance by a nearly constant factor per step
    const bool decades = lo > 0.0 && hi > 16.0 * lo;
    const double step = fabs(cand - x);
    const bool slow = decades && step > 1e-3 * fabs(x) &&
                      ((it >= 2 && step > 0.3 * prev_step) || (it >= 1 && h < 0 && cand > 0.25 * x));
    if (cand > lo && cand < hi && !slow) return cand;
  }
  return (lo > 0.0 && hi > 16.0 * lo) ? bits_mid(lo, hi) : 0.5 * (lo + hi);
}

// Lower bound on the zero from the model that keeps the nearest pole exact
// and replaces the rest of psi_x by its tangent at x:
//   c0 - t + ry/(t - y) + rest(x) + rest'(x) (t - x),  rest = psi_x - ry/(x - y).
// Every other pole lies left of y with a positive residue, so the rest is
// convex right of y, its tangent lies below it and the model's zero lies left
// of the true one.  In u = t - y the model is beta - gamma u + ry/u with
//   beta = h + u_x (1 - psi_x') - 2 ry/u_x,  gamma = 1 - psi_x' - ry/u_x^2 >= 1,
// whose positive zero u = u_x tau is taken in units of u_x,
//   gamma tau^2 - (beta / u_x) tau - ry / u_x^2 = 0,
// in the form that avoids cancellation.  The residue comes as sry = sqrt(ry):
// ry, of the order of x^2, overflows when x passes about 2^512, while sry and
// the coefficients in units of u_x stay in range.  NaN or a value outside the
// bracket (rounding) is ignored by the caller.
__host__ __device__ inline double tangent_rest_bound(double x, double h, double dpsi_x, double y, double sry) {
  const double ux = x - y;
  const double t = sry / ux;   // sqrt(ry) / u_x
  const double beta = h + ux * (1.0 - dpsi_x) - 2.0 * (sry * t);
  const double gamma = fmax(1.0 - dpsi_x - t * t, 1.0);
  const double bb = beta / ux;
  const double r = sqrt(fma(bb, bb, 4.0 * gamma * (t * t)));
  return y + ux * ((bb >= 0.0) ? (bb + r) / (2.0 * gamma) : 2.0 * (t * t) / (r - bb));
}

// The step of rational_inverse, which also knows the residue ry of psi_x at
// its nearest pole y, as sry = sqrt(ry).  Two closed-form models bound the zero before rounding:
// the nearest-pole fit A/(t - y) + B lies above psi_x everywhere right of y
// (for each pole p < y the difference times (t - y)(t - p) is a quadratic
// with a double zero at x and a positive leading coefficient), so its zero is
// an upper bound; tangent_rest_bound gives a lower one.  The tightest bounds
// met so far, [slo, shi] inside the bracket kept from the signs of h, confine
// the step: the second-order candidate clipped into them, or else a split of
// them -- the bit-pattern midpoint across decades, the geometric mean across
// more than a factor 2, the arithmetic mean otherwise.  Far from the zero the
// nearest-pole candidate alone advances by a nearly constant factor when the
// mass of psi_x sits on poles far left of y; the lower bound is what lets the
// split close in from both sides.  The stopping rules are rational_next's.
__host__ __device__ inline double bounded_next(double x, double h, double hnoise, double psi_x, double dpsi_x,
                                               double d2psi_x, double y, double sry, double c0, double lo,
                                               double hi, int it, int hi_open, double& slo, double& shi,
                                               int* done) {
  *done = 0;
  if ((hi - lo) <= 4.0 * EPS * fabs(x)) { *done = 1; return x; }
  if (it < RATIONAL_TO_BISECT) {
    double cand = NAN;
    if (d2psi_x > 0) {
      const double pe = x + 2.0 * dpsi_x / d2psi_x;
      if (pe <= y && pe < x) cand = rational_candidate(x, psi_x, dpsi_x, pe, c0, 1);
    }
    const double up = rational_candidate(x, psi_x, dpsi_x, y, c0, 1);
    const bool second = cand > lo && cand < hi;
    if (!second) cand = up;
    if (cand == cand && (fabs(cand - x) <= 2.0 * EPS * fabs(cand) || fabs(h) <= hnoise)) {
      *done = 1;
      return (cand > lo && cand < hi) ? cand : x;
    }
#if AHD_EARLY2 > 0
    if (cand > lo && cand < hi &&
        fabs(cand - x) <= (second ? ldexp(1.0, -AHD_EARLY2) : ldexp(1.0, -AHD_EARLY1)) * (x - fmax(y, 0.0))) {
      *done = 1;
      return cand;
    }
#endif
    if (hi_open && cand >= hi) return hi;
    slo = fmax(slo, lo);
    shi = fmin(shi, hi);
    if (!(slo < shi)) { slo = lo; shi = hi; }
    const double down = tangent_rest_bound(x, h, dpsi_x, y, sry);
    // the models agree when the lower bound meets the upper one to within the
    // zero's uncertainty from the rounding of h; then slo == shi
    const double tol = hnoise / (1.0 - dpsi_x);
    if (up > slo && up < shi) shi = up;
    if (down > slo && down < shi + tol) slo = fmin(down, shi);
    double xn;
    if (cand > slo && cand < shi) xn = cand;
    else if (slo > 0.0 && shi > 16.0 * slo) xn = bits_mid(slo, shi);
    else if (second) xn = fmin(fmax(cand, slo), shi);
    else xn = (slo > 0.0 && shi > 2.0 * slo) ? sqrt(slo * shi) : 0.5 * (slo + shi);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (slo + shi);
    if (xn > lo && xn < hi) return xn;
  }
  return (lo > 0.0 && hi > 16.0 * lo) ? bits_mid(lo, hi) : 0.5 * (lo + hi);
}

// Extreme eigenvalue of A_i^{-1} on the given side, by the rational iteration.
// The iteration is split into its set-up and its steps so that a caller can
// stop after a few passes and resume later, possibly on other lanes: RatState
// is everything a step reads and updates, RatConsts what follows from (i, side)
// and the lower end y alone.
struct RatState {
  double x, xlo, xhi;   // next point and the bracket kept from the signs of h, in x = side*nu
  double slo, shi;      // the tightest model bounds met so far (bounded_next)
  double c0, y;         // side*b and the nearest pole of psi_x (x-space)
  int it, hi_open;      // steps taken; xhi is a bound that has not been evaluated
};

struct RatConsts {
  double sg, rci, src, sry;
};

// rci = 1/zeta_i^2, src = its square root and sry the square root of the
// residue of psi_x at y: c_jn / (zeta_i^2 e_jn^2) for the neighbouring pole jn,
// or 1/zeta_i^2 for the pole at 0 when no pole lies right of it
template <int KIND>
__host__ __device__ inline RatConsts rat_consts(const Prob& P, int i, int side, double y) {
  RatConsts c;
  c.sg = (double)side;
  c.rci = 1.0 / P.ch[i];
  c.src = 1.0 / sqrt(P.ch[i]);
  c.sry = c.src;
  if (y > 0.0) {
    const double e = pdiff<KIND>(P.ds[i - side], P.ds[i]);
    c.sry = sqrt(P.ch[i - side]) * c.src / fabs(e);
  }
  return c;
}

__host__ __device__ inline RatState rat_init(const RatConsts& c, double b, double lo, double hi, double ymax_nu,
                                             double nu_est) {
  RatState s;
  // x-space bracket
  s.xlo = (c.sg > 0) ? lo : -hi;
  s.xhi = (c.sg > 0) ? hi : -lo;
  s.y = c.sg * ymax_nu;
  s.c0 = c.sg * b;
  s.x = s.xhi;
  s.hi_open = 0;
  if (s.y <= 0.0) {
    // exterior eigenvalue: every other pole of psi_x lies left of 0 and its
    // term is positive for x > 0, so h(x) >= c0 - x + rci / x and the zero of
    // that two-by-two model (the corner block of A_i^{-1}) bounds the wanted
    // zero from below.  Across the decades between it and the Gershgorin bound
    // the iteration starts from the bit-pattern midpoint.
    const double x2 = pos_root(s.c0, c.src);
    s.xlo = fmax(s.xlo, x2 * (1.0 - 4.0 * EPS));
    if (s.xlo > 0.0 && s.xhi > 16.0 * s.xlo) {
      s.x = bits_mid(s.xlo, s.xhi);
      s.hi_open = 1;
    }
  }
  // an estimate (a repair re-solving a known eigenvalue from another shift)
  // inside the bracket is the better start
  const double x_est = c.sg * nu_est;
  if (x_est > s.xlo && x_est < s.xhi) s.x = x_est;
  s.slo = s.xlo;
  s.shi = s.xhi;
  s.it = 0;
  return s;
}

// One pass at s.x and the next point; true when the iteration has finished
// (s.x is then the root).  last[] receives the pass's point and sums.  WIDE:
// the group has gc lanes, gc one of G, 2G, ..., 64 (psi_pass_wide).
template <int KIND, int G, bool WIDE = false>
__host__ __device__ inline bool rat_step(const Prob& P, int i, const RatConsts& c, RatState& s, int ln,
                                         double* last, int gc = G) {
  if (s.x >= s.xhi) s.hi_open = 0;
  const double nu = c.sg * s.x;
  double s1, s2, s3;
  if constexpr (WIDE) psi_pass_wide<KIND, false, G>(P, P.ds[i], 0.0, i, nu, ln, gc, s1, s2, s3);
  else psi_pass<KIND, G, false>(P, P.ds[i], 0.0, i, nu, ln, s1, s2, s3);
  if (last) { last[0] = nu; last[1] = s2; last[2] = s3; }   // the sums at the latest point
  const double rnu = 1.0 / nu;
  const double psi = (s1 + rnu) * c.rci;                       // psi(nu)
  const double dpsi = -(s2 + rnu * rnu) * c.rci;               // psi'(nu)
  const double d2psi = 2.0 * (s3 * rnu + rnu * rnu * rnu) * c.rci;   // psi''(nu)
  const double psi_x = c.sg * psi, dpsi_x = dpsi, d2psi_x = c.sg * d2psi;
  const double h = s.c0 - s.x + psi_x;
  if (h > 0) s.xlo = s.x; else s.xhi = s.x;
  if (h == 0) return true;
  const double hnoise = 8.0 * EPS * (fabs(s.c0) + fabs(s.x) + fabs(psi_x));
  int done = 0;
  s.x = bounded_next(s.x, h, hnoise, psi_x, dpsi_x, d2psi_x, s.y, c.sry, s.c0, s.xlo, s.xhi, s.it, s.hi_open, s.slo,
                     s.shi, &done);
  ++s.it;
  return done || s.it >= MAX_RATIONAL + MAX_BISECT;
}

template <int KIND, int G>
__host__ __device__ inline double rational_inverse(const Prob& P, int i, int side, double b, double lo,
                                                   double hi, double ymax_nu, int ln, int* iters,
                                                   double nu_est = NAN, double* last = nullptr) {
  const RatConsts c = rat_consts<KIND>(P, i, side, (double)side * ymax_nu);
  RatState s = rat_init(c, b, lo, hi, ymax_nu, nu_est);
  while (!rat_step<KIND, G>(P, i, c, s, ln, last)) {
  }
  if (iters) *iters = s.it;
  return c.sg * s.x;
}

// ---------------------------------------------------------------------------
// Remark 1 / Remark 2(b): the extreme eigenvalue of (A - sigma I)^{-1}, a DPR1
// matrix diag((D - sigma)^{-1}, 0) + rho u u^T with u = [(D - sigma)^{-1} z; -1]
// and rho = 1 / f(sigma), f the Pick function; f(sigma) is evaluated in
// double-double.  sigma = pval(pv) + s.  Its eigenvalues are the zeros of
//   phi(nu) = 1 + rho sum_j u_j^2 / (Delta_j - nu),  Delta_j = 1/e_j, Delta_n = 0,
// i.e. phi(nu) = 1 + rho (S(nu) - 1/nu) with S as in bisect_inverse.  The
// wanted zero is exterior on the side of sign(rho).  Returns mu = 1/nu, or
// sets *zero when f(sigma) evaluates to 0 (then lambda = sigma).

template <int KIND, int G>
__host__ __device__ inline double dpr1_inverse(const Prob& P, double pv, double s, int ln, int* zero,
                                               int* iters, int method, double nu_est = NAN,
                                               double* last = nullptr) {
  const int m = P.m;
  dd fs = {0.0, 0.0};
  double usum = 0.0, dmx = -INFINITY, dmn = INFINITY;
  for_terms<G>(ln, m, -1, [&](int j, bool) {
    const dd e = dd_add_d(pdiff_dd<KIND>(P.ds[j], pv), -s);
    const double Dj = recip(e.hi);
    fs = dd_add(fs, dd_div2(dd{P.ch[j], P.cl[j]}, e, Dj));
    usum += P.ch[j] * Dj * Dj;
    dmx = fmax(dmx, Dj);
    dmn = fmin(dmn, Dj);
  });
  fs = gsum_dd<G>(fs);
  usum = gsum<G>(usum);
  dmx = gmax<G>(dmx);
  dmn = gmin<G>(dmn);
  const dd asig = dd_add_d(dd_sub(P.corner, pval_dd<KIND>(pv)), -s);
  const dd f = dd_sub(asig, fs);
  *zero = 0;
  *iters = 0;
  if (f.hi == 0.0) { *zero = 1; return 0.0; }
  const double rho = dd_to_d(dd_div(dd_from(1.0), f));
  const double u2 = usum + 1.0;
  double lo, hi;
  if (rho > 0) { lo = fmax(dmx, 0.0); hi = lo + rho * u2; }
  else { hi = fmin(dmn, 0.0); lo = hi + rho * u2; }
  int it = 0;
  if (method == ROOT_RATIONAL) {
    // phi(nu) = 1 - rho psi(nu), psi(nu) = sum_j c_j/(e_j (nu e_j - 1)) + 1/nu;
    // in x = sign(rho) nu:  h(x) = psi_x(x) - 1/|rho|, psi_x = sign(rho) psi
    const double sg = rho > 0 ? 1.0 : -1.0;
    double xlo = (rho > 0) ? lo : -hi;
    double xhi = (rho > 0) ? hi : -lo;
    const double y = (rho > 0) ? lo : -hi;
    const double c0 = -1.0 / fabs(rho);
    double x = xhi;
    const double x_est = sg * nu_est;   // a known estimate inside the bracket is the better start
    if (x_est > xlo && x_est < xhi) x = x_est;
    double prev_step = INFINITY;
    for (; it < MAX_RATIONAL + MAX_BISECT; ++it) {
      const double nu = sg * x;
      double s1, s2, s3;
      psi_pass<KIND, G, true>(P, pv, s, -1, nu, ln, s1, s2, s3);
      if (last) { last[0] = nu; last[1] = s2; last[2] = s3; }   // the sums at the latest point
      const double rnu = 1.0 / nu;
      const double psi_x = sg * (s1 + rnu);
      const double dpsi_x = -(s2 + rnu * rnu);
      const double d2psi_x = sg * 2.0 * (s3 * rnu + rnu * rnu * rnu);
      const double h = c0 + psi_x;
      if (h > 0) xlo = x; else xhi = x;
      if (h == 0) break;
      const double hnoise = 8.0 * EPS * (fabs(c0) + fabs(psi_x));
      int done = 0;
      const double xn =
          rational_next(x, h, hnoise, psi_x, dpsi_x, d2psi_x, y, c0, 0, xlo, xhi, it, prev_step, 0, &done);
      prev_step = fabs(xn - x);
      x = xn;
      if (done) { ++it; break; }
    }
    *iters = it;
    return 1.0 / (sg * x);
  }
  double mid = 0.5 * (lo + hi);
  while ((hi - lo) / fabs(mid) > 2.0 * EPS && it < MAX_BISECT) {
    double S = 0.0;
#pragma unroll 4
    for (int j = ln; j < m; j += G) {
      const double e = pdiff<KIND>(P.ds[j], pv) - s;
      S = fma(P.ch[j], recip(e * fma(-mid, e, 1.0)), S);
    }
    S = gsum<G>(S);
    const double phi = 1.0 + rho * (S - 1.0 / mid);
    const bool above = (rho > 0) ? (phi < 0) : (phi > 0);
    if (above) lo = mid; else hi = mid;
    mid = 0.5 * (lo + hi);
    ++it;
  }
  *iters = it;
  return 1.0 / hi;
}

// ---------------------------------------------------------------------------
// Remark 1: the eigenvalue nearest the origin from the extreme eigenvalue nu of
// A^{-1}, the DPR1 matrix diag(1/d_j, 0) + rho u u^T, u = [D^{-1} z; -1],
// rho = 1/f(0).  Its secular equation 1 + rho sum_j u_j^2 / (Delta_j - nu) = 0
// (Delta_j = 1/d_j, Delta_n = 0), multiplied by f(0), reads
//   h = f(0) - 1/nu - sum_j T_j,   T_j = c_j / (d_j (nu d_j - 1)),
// since u_j^2/(Delta_j - nu) = -c_j/(d_j (nu d_j - 1)) and the last term is -1/nu.
// It is solved for lambda = 1/nu with nu d_j formed as d_j/lambda: between the
// two poles around the origin every T_j has the sign of lambda (no
// cancellation in lambda + sum T_j), d_j/lambda - 1 is of order one at the
// poles that matter, and neither nu nor a square of 1/d_j is ever formed, so
// nothing leaves the exponent range when lambda or the poles are tiny.  Where
// |d_j/lambda| passes 2^900, T_j = (c_j/d_j) lambda / d_j, its limit to far
// below rounding.  h decreases; with W_j = T_j / (1 - lambda/d_j),
// -dh/dlambda = (lambda + sum_j W_j) / lambda, so a Newton step moves lambda
// by lambda h / (lambda + sum_j W_j).  The zero lies on the side of sign f(0),
// within |f(0)| (every term of h/lambda beyond -1 is negative) and the nearer
// pole; a step that leaves that bracket is replaced by its midpoint.
// f(0) = corner - sum_j c_j / d_j is summed in double-double; where that does
// not resolve it, exact_f(&ok) (every lane of the group calls it) returns the
// exact sum (ok = 0: unresolved), or NaN.  Sets *zero when f(0) is 0 (lambda
// = 0) and *unres when f(0) stays unresolved.
template <int KIND, int G, class Exact>
__host__ __device__ inline double origin_root(const Prob& P, int ln, double lam_est, int* zero, int* unres,
                                              int* iters, Exact&& exact_f) {
  const int m = P.m;
  dd fs = {0.0, 0.0};
  double fmag = 0.0, ppos = INFINITY, pneg = INFINITY;
  for_terms<G>(ln, m, -1, [&](int j, bool) {
    const dd e = pval_dd<KIND>(P.ds[j]);
    const dd t = dd_div(dd{P.ch[j], P.cl[j]}, e);
    fs = dd_add(fs, t);
    fmag += fabs(t.hi);
    if (e.hi > 0.0) ppos = fmin(ppos, e.hi);
    else pneg = fmin(pneg, -e.hi);
  });
  fs = gsum_dd<G>(fs);
  fmag = gsum<G>(fmag);
  ppos = gmin<G>(ppos);
  pneg = gmin<G>(pneg);
  dd f = dd_sub(P.corner, fs);
  *zero = 0;
  *unres = 0;
  // double-double (and, for DPR1 and SVD, the reduction to the arrowhead) is
  // good to about (m + 8) 2^-100 of the terms' size
  const double err = (double)(m + 8) * 0x1p-100 * (fmag + fabs(P.corner.hi));
  if (!(fabs(f.hi) > err * 0x1p56)) {
    int ok = 1;
    const double fx = exact_f(&ok);
    if (fx == fx) f = dd_from(fx);
    *unres = !ok;
  }
  const double f0 = dd_to_d(f);
  int it = 0;
  if (f0 == 0.0) { *zero = 1; *iters = 0; return 0.0; }
  const double sg = f0 > 0.0 ? 1.0 : -1.0;
  // t = sg * lambda in (0, thi]
  double tlo = 0.0, thi = fmin(fabs(f0), sg > 0.0 ? ppos : pneg);
  double t = sg * lam_est;
  if (!(t > tlo && t < thi)) t = fmin(fabs(f0), 0.5 * thi);
  for (; it < 80; ++it) {
    const double lam = sg * t;
    double a = 0.0, w = 0.0;
#pragma unroll 4
    for (int j = ln; j < m; j += G) {
      const double dj = pval<KIND>(P.ds[j]);
      const double q = dj / lam;
      const double T = (fabs(q) < 0x1p900) ? P.ch[j] / (dj * (q - 1.0)) : ((P.ch[j] / dj) * lam) / dj;
      a += T;
      w += T / (1.0 - lam / dj);
    }
    a = gsum<G>(a);
    w = gsum<G>(w);
    const double h = (f0 - lam) - a;
    const double ht = sg * h;        // decreasing in t
    if (ht > 0.0) tlo = t; else thi = t;
    if (h == 0.0) break;
    double tn = t + sg * (lam * h / (lam + w));
    if (!(tn > tlo && tn < thi)) tn = (tlo > 0.0 && thi > 16.0 * tlo) ? bits_mid(tlo, thi) : 0.5 * (tlo + thi);
    const bool stop = fabs(tn - t) <= 2.0 * EPS * t || !(thi - tlo > 2.0 * EPS * thi);
    t = tn;
    if (stop) { ++it; break; }
  }
  *iters = it;
  return sg * t;
}

// ---------------------------------------------------------------------------
// DPR1 only: the smallest eigenvalue lies in (d_n, d_{n-1}) and may sit much
// closer to d_n, which is not a pole of the reduced arrowhead.  Re-measure it
// from d_n: tau = lambda - d_n is the zero in (0, d_{n-1} - d_n) of
//   phi(d_n + tau) = 1 + rho (sum_{j<n} u_j^2 / (e_j - tau) - u_n^2 / tau),
// e_j = d_j - d_n.  In x = 1 / tau, with u_j^2/(e_j - 1/x) = u_j^2/e_j +
// u_j^2/(e_j (x e_j - 1)), dividing by rho u_n^2 gives the form the rational
// iteration solves,
//   h(x) = c0 - x + psi(x),  c0 = (1/rho + sum_j u_j^2/e_j) / u_n^2,
//   psi(x) = sum_j u_j^2 / (e_j (x e_j - 1)) / u_n^2,
// with every term positive right of the nearest pole y = 1/(d_{n-1} - d_n).
// For x >= 2/e_j each term is at most 2 u_j^2 / (e_j^2 x), so x <= c0 + Q/x
// with Q = 2 sum_j u_j^2/e_j^2 / u_n^2 bounds the zero from above (or it is
// below 2y).  tau_est, the first pass's estimate, is the starting point.

template <int G>
__host__ __device__ inline double dpr1_from_last_pole(const Prob& P, double tau_est, int ln, int* iters) {
  const int m = P.nsorted - 1;          // the poles d_1 .. d_{n-1}
  const double dn = P.ds[m];
  const double un = P.zs[m];
  const double ru = 1.0 / (un * un);
  const double y = 1.0 / (P.ds[m - 1] - dn);
  double K = 0.0, Q = 0.0;
  for_terms<G>(ln, m, -1, [&](int j, bool) {
    const double r = recip(P.ds[j] - dn);
    const double cr = (P.zs[j] * P.zs[j]) * r;
    K += cr;
    Q = fma(cr, r, Q);
  });
  K = gsum<G>(K);
  Q = gsum<G>(Q);
  const double c0 = (1.0 / P.rho + K) * ru;
  const double q2 = 2.0 * Q * ru;
  double xlo = y;
  double xhi = fmax(2.0 * y, 0.5 * (c0 + sqrt(c0 * c0 + 4.0 * q2))) * (1.0 + 8.0 * EPS);
  double x = 1.0 / tau_est;
  if (!(x > xlo && x < xhi)) x = xhi;
  int it = 0;
  double prev_step = INFINITY;
  for (; it < MAX_RATIONAL + MAX_BISECT; ++it) {
    double a = 0.0, b = 0.0, c = 0.0;
    for_terms<G>(ln, m, -1, [&](int j, bool) {
      const double e = P.ds[j] - dn;
      const double q = recip(e * fma(x, e, -1.0));
      const double v = e * q;                 // 1 / (x e - 1)
      const double u2 = P.zs[j] * P.zs[j];
      a = fma(u2, q, a);
      const double d1 = (u2 * v) * v;
      b += d1;
      c = fma(d1, e * v, c);
    });
    a = gsum<G>(a);
    b = gsum<G>(b);
    c = gsum<G>(c);
    const double psi = a * ru, dpsi = -b * ru, d2psi = 2.0 * c * ru;
    const double h = c0 - x + psi;
    if (h > 0) xlo = x; else xhi = x;
    if (h == 0) break;
    const double hnoise = 8.0 * EPS * (fabs(c0) + fabs(x) + fabs(psi));
    int done = 0;
    const double xn = rational_next(x, h, hnoise, psi, dpsi, d2psi, y, c0, 1, xlo, xhi, it, prev_step, 0, &done);
    prev_step = fabs(xn - x);
    x = xn;
    if (done) { ++it; break; }
  }
  *iters = it;
  return 1.0 / x;
}

// ---------------------------------------------------------------------------
// 1 / ||x|| for the eigenvector of eq. (eigenvecAi) at the shift (pv, s, mu):
//   ARROW/SVD: x_j = shaft_j / (e_j - mu), x_n = -1
//   DPR1:      q_j = u_j / ((d_j - pv) - s - mu) over all n DPR1 poles
// The terms are all positive.

// The squares are taken on g x, g the power of two at or below the distance
// s + mu from the shift pole to lambda (kept within [2^-1000, 2^500]): the
// entries are of the order of 1/(s + mu), whose square overflows when lambda
// lies within about 2^-512 of that pole.  Scaling by a power of two is exact,
// so where nothing overflows the result is that of the unscaled sum.

// off, when given, replaces the distance |s + mu| as the scale: the shift of
// Remark 1 is the origin, not a pole, and the entries are of the order of the
// reciprocal distance to the nearest pole instead.
template <int KIND, int G>
__host__ __device__ inline double inv_norm(const Prob& P, double pv, double s, double mu, int ln,
                                           double off_hint = -1.0) {
  const double off = off_hint >= 0.0 ? off_hint : fabs(s + mu);
  const double g = (off > 0.0) ? ldexp(1.0, ilogb(fmin(fmax(off, 0x1p-1000), 0x1p500))) : 1.0;
  double acc = 0.0;
  if constexpr (KIND == KIND_DPR1) {
    for_terms_ld<G>(ln, P.nsorted, -1, [&](int j) { return v2{P.ds[j], P.zs[j]}; }, [&](int, bool, const v2& t) {
      const double x = t.b * (recip(((t.a - pv) - s) - mu) * g);
      acc = fma(x, x, acc);
    });
    acc = gsum<G>(acc);
  } else {
    for_terms_ld<G>(ln, P.m, -1, [&](int j) { return v2{P.ds[j], P.ch[j]}; }, [&](int, bool, const v2& t) {
      const double r = recip((pdiff<KIND>(t.a, pv) - s) - mu) * g;
      acc = fma(t.b * r, r, acc);
    });
    acc = gsum<G>(acc) + g * g;
  }
  return g / sqrt(acc);
}

}  // namespace ahd
