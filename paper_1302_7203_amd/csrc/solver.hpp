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

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd.hpp"

namespace ahd {

enum Kind { KIND_ARROW = 0, KIND_DPR1 = 1, KIND_SVD = 2 };

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
constexpr uint32_t INFO_NOT_SOLVED = INFO_REDUCIBLE | INFO_NONFINITE | INFO_BAD_INPUT;

constexpr double EPS = 2.220446049250313080847e-16;  // 2^-52, eps of Algorithm 3
constexpr int MAX_BISECT = 4000;

struct Options {
  double tau_nu;     // K_nu threshold for the Remark 2 remedies
  double tau_zero;   // threshold on (|d_i| + |mu|) / |lambda| for Remark 1
  int fp64_b;        // 1: b by Algorithm 2 in FP64 only (negative control)
  int remedies;      // 0: skip the K_nu and near-zero remedies
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

// ---------------------------------------------------------------------------
// group reductions (XOR butterfly: every lane of the group gets the same bits)

template <int G>
__host__ __device__ inline double gsum(double v) {
  if constexpr (G > 1) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  }
  return v;
}

template <int G>
__host__ __device__ inline double gmax(double v) {
  if constexpr (G > 1) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, G));
  }
  return v;
}

template <int G>
__host__ __device__ inline double gmin(double v) {
  if constexpr (G > 1) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, G));
  }
  return v;
}

template <int G>
__host__ __device__ inline dd gsum_dd(dd v) {
  if constexpr (G > 1) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
      dd w = {__shfl_xor(v.hi, o, G), __shfl_xor(v.lo, o, G)};
      v = dd_add(v, w);
    }
  }
  return v;
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
  double s = 0.0;
  for (int j = ln; j < m; j += G) s += P.ch[j] / (pdiff<KIND>(P.ds[j], dk) - mid);
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
};

template <int KIND, int G>
__host__ __device__ inline BPass b_pass(const Prob& P, int i, int side, int ln, int fp64_b) {
  const int m = P.m;
  const double di = P.ds[i];
  dd p1 = {0.0, 0.0}, p2 = {0.0, 0.0};  // sum over j < i (>= 0), j > i (<= 0)
  double f1 = 0.0, f2 = 0.0;            // the same sums in FP64
  double wsum = 0.0;                    // sum_{j != i} |shaft_j| / |e_j|
  double dmx = -INFINITY, dmn = INFINITY, gmx = -INFINITY, gmn = INFINITY;
  const double rzi = 1.0 / P.dz[i];
  for (int j = ln; j < m; j += G) {
    if (j == i) continue;
    const double ej = pdiff<KIND>(P.ds[j], di);
    const double t = P.ch[j] / ej;
    if (j < i) f1 += t; else f2 += t;
    if (!fp64_b) {
      const dd q = dd_div(dd{P.ch[j], P.cl[j]}, pdiff_dd<KIND>(P.ds[j], di));
      if (j < i) p1 = dd_add(p1, q); else p2 = dd_add(p2, q);
    }
    const double delta = 1.0 / ej;                  // diagonal of A_i^{-1}
    const double wj = P.dz[j] / fabs(ej);           // |w_j| |zeta_i|
    wsum += wj;
    dmx = fmax(dmx, delta);
    dmn = fmin(dmn, delta);
    gmx = fmax(gmx, delta + wj * rzi);
    gmn = fmin(gmn, delta - wj * rzi);
  }
  f1 = gsum<G>(f1);
  f2 = gsum<G>(f2);
  wsum = gsum<G>(wsum);
  dmx = gmax<G>(dmx);
  dmn = gmin<G>(dmn);
  gmx = gmax<G>(gmx);
  gmn = gmin<G>(gmn);
  const dd a = dd_sub(P.corner, pval_dd<KIND>(di));  // a = alpha - d_i
  const double ci = P.ch[i];
  BPass r;
  double num_abs;
  if (fp64_b) {
    // Algorithm 2: b = (-a + sum_{j<i} + sum_{j>i}) / zeta_i^2, all in FP64
    r.b = ((-a.hi + f1) + f2) / ci;
    num_abs = fabs(r.b) * ci;
  } else {
    p1 = gsum_dd<G>(p1);
    p2 = gsum_dd<G>(p2);
    dd pp, qq;
    if (-a.hi > 0) { pp = dd_add(dd_neg(a), p1); qq = dd_neg(p2); }
    else { pp = p1; qq = dd_sub(a, p2); }
    const dd num = dd_sub(pp, qq);
    r.b = dd_to_d(dd_div(num, dd{P.ch[i], P.cl[i]}));
    num_abs = fabs(num.hi);
  }
  r.Kb = (fabs(a.hi) + fabs(f1) + fabs(f2)) / num_abs;
  // Gershgorin discs of A_i^{-1}: rows j != i (centre delta_j, radius |w_j|),
  // row i (centre 0, radius 1/|zeta_i|), last row (centre b, radius ||w||_1).
  const double w1 = (wsum + 1.0) * rzi;
  if (side > 0) {
    r.lo = fmax(dmx, 0.0);
    r.hi = fmax(fmax(gmx, rzi), r.b + w1);
  } else {
    r.hi = fmin(dmn, 0.0);
    r.lo = fmin(fmin(gmn, -rzi), r.b - w1);
  }
  return r;
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
    for (int j = ln; j < m; j += G) {
      const double e = pdiff<KIND>(P.ds[j], di);
      const double t = P.ch[j] / (e * fma(-mid, e, 1.0));
      S += (j == i) ? 0.0 : t;
    }
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
// Remark 1 / Remark 2(b): the extreme eigenvalue of (A - sigma I)^{-1}, a DPR1
// matrix diag((D - sigma)^{-1}, 0) + rho u u^T with u = [(D - sigma)^{-1} z; -1]
// and rho = 1 / f(sigma), f the Pick function; f(sigma) is evaluated in
// double-double.  sigma = pval(pv) + s.  Its eigenvalues are the zeros of
//   phi(nu) = 1 + rho sum_j u_j^2 / (Delta_j - nu),  Delta_j = 1/e_j, Delta_n = 0,
// i.e. phi(nu) = 1 + rho (S(nu) - 1/nu) with S as in bisect_inverse.  The
// wanted zero is exterior on the side of sign(rho).  Returns mu = 1/nu, or
// sets *zero when f(sigma) evaluates to 0 (then lambda = sigma, Remark 1).

template <int KIND, int G>
__host__ __device__ inline double dpr1_inverse(const Prob& P, double pv, double s, int ln, int* zero,
                                               int* iters) {
  const int m = P.m;
  dd fs = {0.0, 0.0};
  double usum = 0.0, dmx = -INFINITY, dmn = INFINITY;
  for (int j = ln; j < m; j += G) {
    const dd e = dd_add_d(pdiff_dd<KIND>(P.ds[j], pv), -s);
    fs = dd_add(fs, dd_div(dd{P.ch[j], P.cl[j]}, e));
    const double eh = e.hi;
    const double Dj = 1.0 / eh;
    usum += P.ch[j] / (eh * eh);
    dmx = fmax(dmx, Dj);
    dmn = fmin(dmn, Dj);
  }
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
  double mid = 0.5 * (lo + hi);
  int it = 0;
  while ((hi - lo) / fabs(mid) > 2.0 * EPS && it < MAX_BISECT) {
    double S = 0.0;
    for (int j = ln; j < m; j += G) {
      const double e = pdiff<KIND>(P.ds[j], pv) - s;
      S += P.ch[j] / (e * fma(-mid, e, 1.0));
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
// DPR1 only: the smallest eigenvalue lies in (d_n, d_{n-1}) and may sit much
// closer to d_n, which is not a pole of the reduced arrowhead.  Re-measure it
// from d_n: tau = lambda - d_n in (0, d_{n-1} - d_n) is the zero of
//   phi(d_n + tau) = 1 + rho (sum_{j<n} u_j^2 / ((d_j - d_n) - tau) - u_n^2 / tau),
// whose terms inside the bracket are all positive except the last.

template <int G>
__host__ __device__ inline double dpr1_from_last_pole(const Prob& P, double hi, int ln, int* iters) {
  const int n = P.nsorted;
  const double dn = P.ds[n - 1];
  const double un = P.zs[n - 1];
  const double un2 = un * un;
  double lo = 0.0;
  double mid = 0.5 * (lo + hi);
  int it = 0;
  while ((hi - lo) / fabs(mid) > 2.0 * EPS && it < MAX_BISECT) {
    double S = 0.0;
    for (int j = ln; j < n - 1; j += G) {
      const double u = P.zs[j];
      S += (u * u) / ((P.ds[j] - dn) - mid);
    }
    S = gsum<G>(S);
    const double phi = 1.0 + P.rho * (S - un2 / mid);
    if (phi < 0) lo = mid; else hi = mid;
    mid = 0.5 * (lo + hi);
    ++it;
  }
  *iters = it;
  return hi;
}

// ---------------------------------------------------------------------------
// 1 / ||x|| for the eigenvector of eq. (eigenvecAi) at the shift (pv, s, mu):
//   ARROW/SVD: x_j = shaft_j / (e_j - mu), x_n = -1
//   DPR1:      q_j = u_j / ((d_j - pv) - s - mu) over all n DPR1 poles
// The terms are all positive.

template <int KIND, int G>
__host__ __device__ inline double inv_norm(const Prob& P, double pv, double s, double mu, int ln) {
  double acc = 0.0;
  if constexpr (KIND == KIND_DPR1) {
    for (int j = ln; j < P.nsorted; j += G) {
      const double x = P.zs[j] / (((P.ds[j] - pv) - s) - mu);
      acc = fma(x, x, acc);
    }
    acc = gsum<G>(acc);
  } else {
    for (int j = ln; j < P.m; j += G) {
      const double den = (pdiff<KIND>(P.ds[j], pv) - s) - mu;
      acc += P.ch[j] / (den * den);
    }
    acc = gsum<G>(acc) + 1.0;
  }
  return 1.0 / sqrt(acc);
}

}  // namespace ahd
