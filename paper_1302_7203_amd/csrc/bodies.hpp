// Problem descriptor, workspace layout and the per-element / per-eigenvalue
// bodies of the kernels in arrow.hip.  Each body is a __host__ __device__
// function of (problem, index, lane) so that a kernel is a thin wrapper that
// maps its grid onto these indices.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "exact.hpp"
#include "solver.hpp"

namespace ahd {

// One problem as the caller hands it over (all pointers are device memory).
struct ProbDesc {
  int32_t kind;        // KIND_ARROW / KIND_DPR1 / KIND_SVD
  int32_t n;           // matrix order
  int32_t neg;         // DPR1 with rho < 0: solve (-D) + |rho| u u^T (scalar holds |rho|) and negate
  const double* d;     // ARROW, SVD: n-1 poles; DPR1: n diagonal entries (any order)
  const double* z;     // ARROW, SVD: n-1 shaft entries; DPR1: u (n); HERM: n-1 complex (re, im) pairs
  double scalar;       // ARROW, SVD: alpha; DPR1: |rho|
  double* lam;         // n: eigenvalues (SVD: singular values), descending
  double* V;           // n x n column-major (ARROW: V, DPR1: Q, SVD: right vectors, HERM: complex U
                       // as (re, im) pairs) or null
  int64_t ldv;         // leading dimension (HERM: in complex entries)
  double* U;           // SVD left vectors or null
  int64_t ldu;
  double* shift;       // n or null: lambda_k = shift_k + mu_k (Remark 3 pairs)
  double* mu;          // n or null
  uint32_t* info;      // n or null: INFO_* bits
  double* ws;          // workspace of ws_doubles(n) doubles
};

__host__ __device__ inline size_t ws_doubles(int64_t n) { return 16 + (size_t)n * 26; }

// Workspace of one problem.
struct Ws {
  double* hdr;      // [0],[1] corner (dd); [2] 1 if some pole is exactly 0; [4] problem flags (uint32)
  uint32_t* st;     // per-input status written by the sort
  double* ds;       // sorted d
  double* zs;       // z (u) in sorted order
  double* ch;       // arrowhead shaft^2, hi part
  double* cl;       // arrowhead shaft^2, lo part
  double* dz;       // |arrowhead shaft|
  double* pv1;      // first pass: shift pole value
  double* mu1;      // first pass: mu
  double* kb1;      // first pass: K_b
  int32_t* ip1;     // first pass: shift pole index
  uint32_t* fl1;    // first pass: info bits
  double* pv;       // final shift pole value (0 for an absolute shift)
  double* sf;       // final shift offset
  double* mu;       // final mu
  double* inrm;     // final 1 / ||x||
  int32_t* cnt;     // per eigenvalue, 6 counters: (bisection steps, double-double passes, plain O(n)
                    // passes) of k_root, then the same three of k_check
  // deflation of a reducible arrowhead (Sec. 1): hdr[8] = poles m' of the
  // irreducible problem that the root and check stages solve, hdr[9] = number
  // of deflated eigenpairs, hdr[10] = completion count of the repair launch
  double* lr;       // the irreducible problem's eigenvalues, by its index
  double* dv;       // deflated eigenvalues, descending
  double* da;       // per deflated eigenpair: factor of the earlier rows of its run ...
  double* db;       // ... and its own entry (see deflate_run)
  int32_t* dm;      // per deflated eigenpair: its row (sorted index)
  int32_t* df;      // ... and the first nonzero row of its run (-1: a unit vector)
  int32_t* cm;      // per output column: deflated eigenpair index, or -1
  int32_t* iperm;   // caller row -> sorted index
  double* nr1;      // first pass: 1 / ||x|| at the first-pass mu, from the root's last pass (NaN: none)
  double* kbc;      // per output column: K_b (eq. K2) of the first pass's shift (NaN: none)
  double* knu;      // per output column: K_nu (eq. K0) of the first pass (NaN: not evaluated)
};

__host__ __device__ inline Ws ws_view(double* base, int64_t n) {
  const size_t N = (size_t)n;
  Ws w;
  w.hdr = base;
  w.st = (uint32_t*)(base + 16);
  double* p = base + 16 + N;
  w.ds = p; p += N;
  w.zs = p; p += N;
  w.ch = p; p += N;
  w.cl = p; p += N;
  w.dz = p; p += N;
  w.pv1 = p; p += N;
  w.mu1 = p; p += N;
  w.kb1 = p; p += N;
  w.ip1 = (int32_t*)p;
  w.fl1 = (uint32_t*)p + N; p += N;
  w.pv = p; p += N;
  w.sf = p; p += N;
  w.mu = p; p += N;
  w.inrm = p; p += N;
  w.cnt = (int32_t*)p; p += 3 * N;
  w.lr = p; p += N;
  w.dv = p; p += N;
  w.da = p; p += N;
  w.db = p; p += N;
  w.dm = (int32_t*)p;
  w.df = w.dm + N; p += N;
  w.cm = (int32_t*)p;
  w.iperm = w.cm + N; p += N;
  w.nr1 = p; p += N;
  w.kbc = p; p += N;
  w.knu = p; p += N;
  return w;
}

__host__ __device__ inline uint32_t* prob_flags(const Ws& w) { return (uint32_t*)(w.hdr + 4); }

__host__ __device__ inline int sorted_count(const ProbDesc& D) {
  return D.kind == KIND_DPR1 ? D.n : D.n - 1;
}

// poles of the problem the root and check stages solve: the arrowhead itself,
// or, once a reducible one is deflated, the irreducible remainder
__host__ __device__ inline int reduced_m(const Ws& w) { return (int)w.hdr[8]; }
__host__ __device__ inline int deflated_count(const Ws& w) { return (int)w.hdr[9]; }
__host__ __device__ inline uint32_t* place_done(const Ws& w) { return (uint32_t*)(w.hdr + 10); }

// number of entries of the descending a[0..len) that are > x (strict) or >= x
__host__ __device__ inline int count_above(const double* a, int len, double x, bool or_equal) {
  int lo = 0, hi = len;   // a[0..lo) qualify, a[hi..len) do not
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (or_equal ? (a[mid] >= x) : (a[mid] > x)) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// HOT = 1: hot_d / hot_c are copies of the sorted poles and shaft weights (in
// LDS) used by the O(n) passes in place of the workspace arrays; HOT = 2: the
// poles alone (hot_c unused).  A compile-time choice, so that the compiler
// knows which memory the passes read.
template <int HOT = 0>
__host__ __device__ inline Prob make_prob(const ProbDesc& D, const Ws& w, const double* hot_d = nullptr,
                                          const double* hot_c = nullptr) {
  Prob P;
  P.m = reduced_m(w);
  P.n = P.m + 1;
  P.nsorted = (D.kind == KIND_DPR1) ? P.n : P.m;
  P.ds = w.ds;
  P.zs = w.zs;
  P.ch = w.ch;
  P.cl = w.cl;
  P.dz = w.dz;
  P.corner = {w.hdr[0], w.hdr[1]};
  P.rho = D.scalar;
  if constexpr (HOT >= 1) P.ds = hot_d;
  if constexpr (HOT == 1) P.ch = hot_c;
  return P;
}

__host__ __device__ inline bool finite_d(double x) { return x - x == 0.0; }

// sqrt of a double-double, to about one ulp
__host__ __device__ inline double dd_sqrt_d(dd x) {
  const double s = sqrt(x.hi);
  return s == 0.0 ? 0.0 : s + (fma(-s, s, x.hi) + x.lo) * (0.5 / s);
}

// pole j of the problem the kernels solve, read from the caller's array: for
// a DPR1 matrix with rho < 0 the spectrum of D + rho u u^T is the negated
// spectrum of (-D) + |rho| u u^T (same eigenvectors), so its poles are -d_j
template <int KIND>
__host__ __device__ inline double in_pole(const ProbDesc& D, int j) {
  if constexpr (KIND == KIND_DPR1) return D.neg ? -D.d[j] : D.d[j];
  else return D.d[j];
}

// ---------------------------------------------------------------------------
// normalisation (symmetric permutation to decreasing poles, Sec. 1 eq. (order)):
// the rank of input j among all keys; ties broken by input index.

template <int KIND>
__host__ __device__ inline double sort_key(double d) {
  if constexpr (KIND == KIND_SVD) return fabs(d);
  else return d;
}

// status of input j: reducibility (Sec. 1) and domain checks
template <int KIND>
__host__ __device__ inline uint32_t input_status(const ProbDesc& D, int j, bool dup) {
  uint32_t st = 0;
  const double dj = D.d[j];
  if constexpr (KIND == KIND_HERM) {
    const double re = D.z[2 * j], im = D.z[2 * j + 1];
    if (!finite_d(dj) || !finite_d(re) || !finite_d(im)) st |= INFO_NONFINITE;
    if ((re == 0.0 && im == 0.0) || dup) st |= INFO_REDUCIBLE;
  } else {
    const double zj = D.z[j];
    if (!finite_d(dj) || !finite_d(zj)) st |= INFO_NONFINITE;
    if (zj == 0.0 || dup) st |= INFO_REDUCIBLE;
  }
  if (KIND == KIND_SVD && dj == 0.0) st |= INFO_BAD_INPUT;
  return st;
}

// sorted entry r from the caller's entry q: the pole, the shaft entry (HERM:
// the weight |z_q|^2 = re^2 + im^2 as an exact-product double-double, which
// Sec. 6.1 asks for in doubled precision), and for ARROW the row's sorted index
struct SortedEntry {
  double d, z;   // the sorted pole and shaft entry as stored
  dd c;          // HERM: the weight |z_q|^2 as stored; else unused
};

template <int KIND>
__host__ __device__ inline SortedEntry put_sorted_v(const ProbDesc& D, const Ws& w, int r, int q) {
  SortedEntry e;
  e.d = in_pole<KIND>(D, q);
  e.c = dd_from(0.0);
  w.ds[r] = e.d;
  if constexpr (KIND == KIND_HERM) {
    const double re = D.z[2 * q], im = D.z[2 * q + 1];
    e.c = dd_add(two_prod(re, re), two_prod(im, im));
    w.ch[r] = e.c.hi;
    w.cl[r] = e.c.lo;
    e.z = hypot(re, im);   // |z_q| rounded (only the bounds use it); exact when im = 0
  } else {
    e.z = D.z[q];
  }
  w.zs[r] = e.z;
  if constexpr (KIND == KIND_ARROW) w.iperm[q] = r;
  return e;
}

template <int KIND>
__host__ __device__ inline void put_sorted(const ProbDesc& D, const Ws& w, int r, int q) {
  (void)put_sorted_v<KIND>(D, w, r, q);
}

// ---------------------------------------------------------------------------
// prologue: the reduced arrowhead's shaft weights, exactly in double-double.

// sorted entry j from its values: pole dj, shaft entry zj, HERM weight cj, and
// for DPR1 the last pole dn
template <int KIND>
__host__ __device__ inline void prologue_vals(const ProbDesc& D, const Ws& w, int j, double dj, double zj, dd cj,
                                              double dn) {
  dd c;
  if constexpr (KIND == KIND_HERM) {
    c = cj;                                               // |zeta_j|^2, formed by the sort
  } else if constexpr (KIND == KIND_ARROW) {
    c = two_prod(zj, zj);                                 // zeta_j^2
  } else if constexpr (KIND == KIND_SVD) {
    const dd p = two_prod(dj, zj);                        // d_j zeta_j (Sec. 6.2)
    c = dd_mul(p, p);
  } else {
    const dd diff = two_sum(dj, -dn);                     // Sec. 6.3: zeta_j^2 = rho u_j^2 (d_j - d_n)
    c = dd_mul_d(dd_mul(two_prod(zj, zj), diff), D.scalar);
  }
  w.ch[j] = c.hi;
  w.cl[j] = c.lo;
  w.dz[j] = (KIND == KIND_ARROW || KIND == KIND_HERM) ? fabs(zj) : sqrt(c.hi);
}

template <int KIND>
__host__ __device__ inline void prologue_elem(const ProbDesc& D, const Ws& w, int j) {
  const dd cj = (KIND == KIND_HERM) ? dd{w.ch[j], w.cl[j]} : dd_from(0.0);
  const double dn = (KIND == KIND_DPR1) ? w.ds[D.n - 1] : 0.0;
  prologue_vals<KIND>(D, w, j, w.ds[j], w.zs[j], cj, dn);
}

// contribution of a sorted shaft entry zj to the corner
template <int KIND>
__host__ __device__ inline dd corner_term_v(const ProbDesc& D, double zj) {
  if constexpr (KIND == KIND_ARROW || KIND == KIND_HERM) return dd_from(0.0);
  else if constexpr (KIND == KIND_SVD) return two_prod(zj, zj);                   // z^T z
  else return dd_mul_d(two_prod(zj, zj), D.scalar);                                // rho u^T u
}

template <int KIND>
__host__ __device__ inline dd corner_term(const ProbDesc& D, const Ws& w, int j) {
  return corner_term_v<KIND>(D, w.zs[j]);
}

template <int KIND>
__host__ __device__ inline dd corner_base(const ProbDesc& D, const Ws& w) {
  if constexpr (KIND == KIND_ARROW || KIND == KIND_HERM) return dd_from(D.scalar);   // alpha
  else if constexpr (KIND == KIND_SVD) return two_prod(D.scalar, D.scalar);            // alpha^2
  else return dd_from(w.ds[D.n - 1]);                                                  // d_n
}

// ---------------------------------------------------------------------------
// Deflation of a reducible arrowhead (Sec. 1).  A zero shaft entry z_j makes
// d_j an eigenvalue with the unit vector e_j as eigenvector.  Poles equal to
// d_j that carry nonzero shaft entries are merged, by rotations in their
// planes, into one pole whose shaft entry is the root of their sum of squares;
// each direction a rotation removes is an eigenvector for d_j.  What is left
// is an irreducible arrowhead, which the root and check stages solve.
//
// Equal poles are adjacent in the sorted order; a run of them is handled by
// the thread that owns its first element.  Within a run, the members are
// taken in sorted order: the first nonzero member carries the merged pole,
// each zero member is a unit-vector item, and each later nonzero member t is
// a rotation item whose eigenvector has the entries
//     z_i z_t / (R_{t-1} R_t)   at the run's earlier rows i,
//     -R_{t-1} / R_t            at row t,
// where R_t^2 sums z_i^2 over the run's rows up to t (the direction that the
// rotation folding z_t into the merged pole leaves behind; its own entry is
// negative).  Items are numbered in the order of the runs, then of the rows.
// The reduced eigenvectors keep eq. (Aeigenvec) over the caller's rows: the
// rotation carries x of the merged pole back to z_i / (d_i - lambda) on each
// member, and to 0 on the zero members.

struct DeflCount {
  int keep, items;   // 1 if the run keeps a pole; its deflated eigenpairs
};

__host__ __device__ inline bool run_start(const double* ds, int j) { return j == 0 || ds[j] != ds[j - 1]; }

__host__ __device__ inline DeflCount deflate_count(const Ws& w, int m, int j) {
  const double dj = w.ds[j];
  bool nz = false;
  int e = j;
  for (; e < m && w.ds[e] == dj; ++e) nz |= w.zs[e] != 0.0;
  const int keep = nz ? 1 : 0;
  return DeflCount{keep, (e - j) - keep};
}

// the run starting at sorted index j: its pole goes to reduced index r (poles
// into pole_out, weights into ch/cl/dz, which no other run reads), its items
// to q, q+1, ...; r and q are advanced past them.  Returns whether the kept
// pole is exactly zero.
__host__ __device__ inline bool deflate_run(const Ws& w, int m, int j, int& r, int& q, double* pole_out) {
  const double dj = w.ds[j];
  dd R2 = {0.0, 0.0};
  double rp = 0.0;   // R of the members so far
  int f = -1;
  for (int e = j; e < m && w.ds[e] == dj; ++e) {
    const double ze = w.zs[e];
    if (ze == 0.0) {
      w.dv[q] = dj; w.dm[q] = e; w.df[q] = -1; w.da[q] = 0.0; w.db[q] = 1.0;
      ++q;
      continue;
    }
    const dd z2 = two_prod(ze, ze);
    if (f < 0) {
      f = e;
      R2 = z2;
      rp = fabs(ze);
      continue;
    }
    R2 = dd_add(R2, z2);
    const double rt = dd_sqrt_d(R2);
    w.dv[q] = dj; w.dm[q] = e; w.df[q] = f;
    w.da[q] = ze / (rp * rt);
    w.db[q] = -(rp / rt);
    ++q;
    rp = rt;
  }
  if (f < 0) return false;
  pole_out[r] = dj;
  w.ch[r] = R2.hi;
  w.cl[r] = R2.lo;
  w.dz[r] = rp;
  ++r;
  return dj == 0.0;
}

// entry of the deflated eigenvector s at the sorted row j, z_r the caller's
// shaft entry of that row
__host__ __device__ inline double deflated_entry(const Ws& w, int s, int j, double zr) {
  const int t = w.dm[s], f = w.df[s];
  if (j == t) return w.db[s];
  return (f >= 0 && j >= f && j < t) ? zr * w.da[s] : 0.0;
}

// Output columns are the merge of the reduced eigenvalues (descending, as
// computed) with the deflated ones (descending); on a tie the reduced one
// comes first.  Reduced eigenvalue k goes to column k + #{deflated > lambda_k},
// deflated item s to column s + #{reduced >= delta_s}.
__host__ __device__ inline void place_deflated(const ProbDesc& D, const Ws& w, int s) {
  const int np = reduced_m(w) + 1;
  const double v = w.dv[s];
  const int col = s + count_above(w.lr, np, v, true);
  D.lam[col] = v;
  if (D.shift) D.shift[col] = v;
  if (D.mu) D.mu[col] = 0.0;
  if (D.info) D.info[col] = INFO_DEFLATED;
  w.pv[col] = v; w.sf[col] = 0.0; w.mu[col] = 0.0; w.inrm[col] = 0.0;
  w.kbc[col] = NAN; w.knu[col] = NAN;
  w.cm[col] = s;
}

// ---------------------------------------------------------------------------
// first pass for eigenvalue k: shift, b, bisection (Algorithm 5 without the
// final K_nu test).

// 1/||x|| of eq. (eigenvecAi) at the root nu of a rational pass over the poles
// shifted by (pv, s), from that pass's last point last[0] and its sums
// last[1] = S2 = sum zeta_j^2 v_j^2 and last[2] = l S3, S3 = sum zeta_j^2 e_j v_j^3,
// v_j = 1/(nu e_j - 1): the entries are nu zeta_j v_j, the excluded pole's (weight
// cx; 0 when none is excluded) -nu zeta_x, and -1, so ||x||^2 = nu^2 (S2 + cx) + 1,
// carried from l = last[0] to nu to first order (d(nu^2 S2)/dnu = 2 nu S2 - 2 nu^2 S3).
// The rational iteration may stop on a candidate it has not evaluated, once
// its step is below 2^-24 of the distance to the nearest pole: each v_j then
// moves by less than 2^-24 relative, and the neglected second-order term is
// below 2^-46 of ||x||^2.
// The DPR1 eigenvector q = (D - lambda I)^{-1} u of D + rho u u^T (Sec. 6.3) from
// the norm of the reduced arrowhead's x: its Pick function is
// f(lambda) = (d_n - lambda) phi(lambda), phi the DPR1 secular function
// 1 + rho sum_j u_j^2 / (d_j - lambda), so at an eigenvalue (phi = 0)
// f'(lambda) = (d_n - lambda) phi'(lambda) = (d_n - lambda) rho ||q||^2, while
// f'(lambda) = -||x||^2.  Hence 1/||q|| = sqrt(rho (lambda - d_n)) / ||x||, with
// lambda - d_n = (pole - d_n) + offset, no cancellation while lambda is not the
// eigenvalue next to d_n that the check stage re-measures.  NaN (a norm pass
// then runs) when lambda - d_n is not positive.
__host__ __device__ inline double dpr1_inorm(const Prob& P, double inrm_x, double lam_minus_pole, double pole) {
  const double ldn = (pole - P.ds[P.nsorted - 1]) + lam_minus_pole;
  return (ldn > 0.0 && inrm_x == inrm_x) ? inrm_x * sqrt(P.rho * ldn) : NAN;
}

__host__ __device__ inline double norm_from_pass(const double* last, double nu, double cx) {
  const double l = last[0], a0 = last[1] + cx;
  // the step enters as (nu - l) / l: the product of the sums with 1/l alone
  // underflows when the sums are near 1e-225 and l near 1e225
  const double rl = 1.0 / l;
  const double dl = 2.0 * (a0 - last[2]) * ((nu - l) * rl);
  const double acc = l * l * (a0 + dl) + 1.0;
  if (acc < INFINITY) return 1.0 / sqrt(acc);
  // l^2 overflowed (lambda within about 2^-512 of its pole): in units of l^2
  return fabs(rl) / sqrt(a0 + dl + rl * rl);
}

// The results of a first pass that depend on its root: mu, the step count and
// the norm.  ||x||^2 of eq. (eigenvecAi) at mu = 1/nu: with v_j = 1/(nu e_j - 1)
// the entry x_j = zeta_j/(e_j - mu) is nu zeta_j v_j (j != i) and x_i = -nu zeta_i,
// so ||x||^2 = nu^2 (S2 + zeta_i^2) + 1, S2 = sum_{j != i} zeta_j^2 v_j^2 -- the sum
// the rational pass forms for psi'.  It was formed at that pass's point; the
// step to the final nu is taken to first order, d/dnu (nu^2 S2(nu)) =
// 2 nu S2 - 2 nu^2 S3 with S3 = sum zeta_j^2 e_j v_j^3, also formed there.
// DPR1's vector is not the arrowhead's; its norm follows from the arrowhead's
// (dpr1_inorm).
template <int KIND>
__host__ __device__ inline void root_finish(const Prob& P, const Ws& w, int k, int i, int ln, double nu, int iters,
                                            const double* last) {
  double nr1 = NAN;
  if (last[0] == last[0]) {
    nr1 = norm_from_pass(last, nu, P.ch[i]);
    if constexpr (KIND == KIND_DPR1) nr1 = dpr1_inorm(P, nr1, 1.0 / nu, P.ds[i]);
  }
  if (ln == 0) {
    w.cnt[6 * k + 0] = iters;
    w.mu1[k] = 1.0 / nu;
    w.nr1[k] = nr1;
  }
}

// The first pass up to its root: the cases with nothing to solve, the shift,
// b and the outputs that follow from them.  Returns true when the rational
// iteration is left to run from (i, c, s); otherwise the pass is complete
// (the bisection of Algorithm 3 runs here).
template <int KIND, int G, int HOT = 0>
__host__ __device__ inline bool root_begin(const ProbDesc& D, const Options& opt, const Ws& w, const Prob& P, int k,
                                           int ln, int& i, RatConsts& c, RatState& s) {
  const uint32_t pf = *prob_flags(w);
  if (ln == 0) w.nr1[k] = NAN;   // the norm from the root pass, set below when there is one
  if (k >= P.n) {   // past the order of a deflated problem
    if (ln == 0) { w.cnt[6 * k + 0] = 0; w.cnt[6 * k + 1] = 0; w.cnt[6 * k + 2] = 0; }
    return false;
  }
  if (pf & INFO_NOT_SOLVED) {
    if (ln == 0) {
      w.cnt[6 * k + 0] = 0; w.cnt[6 * k + 1] = 0; w.cnt[6 * k + 2] = 0;
      w.pv1[k] = NAN; w.mu1[k] = NAN; w.kb1[k] = NAN; w.ip1[k] = -1; w.fl1[k] = pf;
    }
    return false;
  }
  if (P.m == 0) {  // n == 1: lambda = corner, x = [-1]
    if (ln == 0) {
      w.cnt[6 * k + 0] = 0; w.cnt[6 * k + 1] = 0; w.cnt[6 * k + 2] = 0;
      w.pv1[k] = 0.0; w.mu1[k] = dd_to_d(P.corner); w.kb1[k] = 0.0; w.ip1[k] = -1; w.fl1[k] = 0;
    }
    return false;
  }
  int side;
  select_shift<KIND, G>(P, k, ln, i, side);
  // b in double-double (Theorem 6) unless FP64 is asked for, or unless the
  // FP64 pass's K_b (eq. K2) is at most tau_b: Algorithm 5 keeps b from
  // Algorithm 2 where its cancellation is mild.  K_b is the same in every lane
  // of the eigenvalue, so the choice does not split them.
  BPass bp;
  bool dd_b = !opt.fp64_b;
  if (opt.fp64_b || opt.tau_b > 0.0) {
    bp = b_pass_t<KIND, G, true>(P, i, side, ln);
    if (dd_b) dd_b = !(bp.Kb <= opt.tau_b);
  }
  if (dd_b) bp = b_pass_t<KIND, G, false>(P, i, side, ln);
  const int plain_b = (opt.fp64_b || opt.tau_b > 0.0) ? 1 : 0;
  if (ln == 0) {
    w.cnt[6 * k + 1] = dd_b ? 1 : 0;
    w.cnt[6 * k + 2] = ((k > 0 && k < P.m) ? 1 : 0) + plain_b;
    w.pv1[k] = P.ds[i];
    w.kb1[k] = bp.Kb;
    w.ip1[k] = i;
    uint32_t fl = dd_b ? INFO_DD_B : 0u;
    // Theorem 6 needs K_b <= O(1/eps); flag when the double-double b cannot hold it
    if (bp.Kb * (double)(D.n + 4) * 4.930380657631324e-32 > 1e-3) fl |= INFO_KB_LARGE;
    w.fl1[k] = fl;
  }
  if (opt.root == ROOT_RATIONAL) {
    const double ymax = side > 0 ? bp.lo : bp.hi;
    c = rat_consts<KIND>(P, i, side, (double)side * ymax);
    s = rat_init(c, bp.b, bp.lo, bp.hi, ymax, bp.x0);
    return true;
  }
  int iters = 0;
  const double last[3] = {NAN, NAN, NAN};
  const double nu = bisect_inverse<KIND, G>(P, i, bp.b, bp.lo, bp.hi, ln, &iters);
  root_finish<KIND>(P, w, k, i, ln, nu, iters, last);
  return false;
}

// First pass for eigenvalue k (Algorithm 5 without the final K_nu test): shift,
// b, root of the inverse and the norm of the eigenvector from the root's passes.
template <int KIND, int G, int HOT = 0>
__host__ __device__ inline void root_body(const ProbDesc& D, const Options& opt, int k, int ln,
                                          const double* hot_d = nullptr, const double* hot_c = nullptr) {
  const Ws w = ws_view(D.ws, D.n);
  const Prob P = make_prob<HOT>(D, w, hot_d, hot_c);
  int i = 0;
  RatConsts c;
  RatState s;
  if (!root_begin<KIND, G, HOT>(D, opt, w, P, k, ln, i, c, s)) return;
  double last[3] = {NAN, NAN, NAN};   // the rational pass's last point nu and its sums S2, S3
  while (!rat_step<KIND, G>(P, i, c, s, ln, last)) {
  }
  root_finish<KIND>(P, w, k, i, ln, c.sg * s.x, s.it, last);
}

// ---------------------------------------------------------------------------
// K_nu test and remedies (Algorithm 5, last part; Remarks 1 and 2), then the
// eigenvector norm.  Writes the final shift pair and the caller's outputs.
//
// DEFER = DEFER_ALL: an eigenvalue that needs one of the O(n)-per-step repairs
// (Remark 1, Remark 2, the DPR1 re-measure from d_n) is only appended to the
// problem's repair list and left for a second launch, which runs check_body on
// the listed eigenvalues with a whole block each; everything else is finished
// here.  DEFER = DEFER_NEAR_ZERO: only Remark 1 is listed (its exact sum of f(0)
// runs on whole wavefronts); Remark 2 and the DPR1 re-measure run here on the
// caller's G lanes, as the first pass does.  DEFER = DEFER_WAVE: Remark 1 is
// listed as for DEFER_NEAR_ZERO; an eigenvalue that needs Remark 2 or the DPR1
// re-measure writes nothing and makes the call return true, and the caller runs
// check_body on it again (DEFER_NEAR_ZERO) with all lanes of its wavefront.
// Every other call returns false.
// The list reuses the sort's rank array, free once the poles are sorted; its
// length sits in hdr[6] and is cleared by the prologue.

// f(0) of the arrowhead the kernels solve, summed exactly from the caller's
// inputs (exact.hpp) for Remark 1.
//   ARROW / HERM: f(0) = alpha - sum_j |z_j|^2 / d_j, |z_j|^2 as exact products;
//   DPR1 (Sec. 6.3 reduction, poles d_1 > ... > d_n of the solved sign):
//     f(0) = alpha - sum_{j<n} zeta_j^2/d_j = d_n phi(0), phi(0) = 1 + |rho| sum_j u_j^2/d_j,
//     or |rho| u_n^2 when d_n = 0;
//   SVD: B^T B has corner alpha^2 + z^T z and terms (d_j z_j)^2 / d_j^2 = z_j^2,
//     so f(0) = alpha^2 exactly.
// *ok is 0 when the sum stays unresolved (f(0) = 0 as far as it reaches).
template <int KIND, int G>
__host__ __device__ inline double f_origin(const ProbDesc& D, const Prob& P, int ln, int* ok) {
  *ok = 1;
  if constexpr (KIND == KIND_SVD) {
    return D.scalar * D.scalar;
  } else if constexpr (KIND == KIND_DPR1) {
    const double dn = P.ds[P.nsorted - 1];
    const double rho = D.scalar;   // |rho|
    if (dn == 0.0) {
      const double un = P.zs[P.nsorted - 1];
      return rho * un * un;
    }
    return origin_exact<KIND, G>(ln, D.n, 1.0, 1.0, dn, [&](int r, double* p, double* nn) {
      *p = in_pole<KIND>(D, r);
      const dd u2 = two_prod(D.z[r], D.z[r]);
      const dd a = two_prod(rho, u2.hi), b = two_prod(rho, u2.lo);
      nn[0] = a.hi; nn[1] = a.lo; nn[2] = b.hi; nn[3] = b.lo;
      return 4;
    }, ok);
  } else {
    const bool herm = D.kind == KIND_HERM;
    return origin_exact<KIND, G>(ln, D.n - 1, D.scalar, -1.0, 1.0, [&](int r, double* p, double* nn) {
      *p = D.d[r];
      if (herm) {
        const dd a = two_prod(D.z[2 * r], D.z[2 * r]), b = two_prod(D.z[2 * r + 1], D.z[2 * r + 1]);
        nn[0] = a.hi; nn[1] = a.lo; nn[2] = b.hi; nn[3] = b.lo;
        return (a.hi == 0.0 && b.hi == 0.0) ? 0 : 4;
      }
      const dd a = two_prod(D.z[r], D.z[r]);
      nn[0] = a.hi; nn[1] = a.lo;
      return a.hi == 0.0 ? 0 : 2;
    }, ok);
  }
}

__host__ __device__ inline uint32_t* repair_count(const Ws& w) { return (uint32_t*)(w.hdr + 6); }
__host__ __device__ inline uint32_t* repair_list(const Ws& w, int64_t n) { return w.st + n; }

__host__ __device__ inline void defer_repair(const Ws& w, int64_t n, int k, int ln) {
  if (ln != 0) return;
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t at = atomicAdd(repair_count(w), 1u);
#else
  const uint32_t at = (*repair_count(w))++;
#endif
  repair_list(w, n)[at] = (uint32_t)k;
}

constexpr int DEFER_NONE = 0, DEFER_ALL = 1, DEFER_NEAR_ZERO = 2, DEFER_WAVE = 3;

template <int KIND, int G, bool HOT = false, int DEFER = DEFER_NONE>
__host__ __device__ inline bool check_body(const ProbDesc& D, const Options& opt, int k, int ln,
                                           const double* hot_d = nullptr, const double* hot_c = nullptr) {
  const Ws w = ws_view(D.ws, D.n);
  const Prob P = make_prob<HOT>(D, w, hot_d, hot_c);
  const uint32_t pf = *prob_flags(w);
  if (k >= P.n) {
    if (ln == 0) { w.cnt[6 * k + 3] = 0; w.cnt[6 * k + 4] = 0; w.cnt[6 * k + 5] = 0; }
    return false;
  }
  if (pf & INFO_NOT_SOLVED) {
    if (ln == 0) {
      w.pv[k] = NAN; w.sf[k] = NAN; w.mu[k] = NAN; w.inrm[k] = NAN;
      w.kbc[k] = NAN; w.knu[k] = NAN;
      D.lam[k] = NAN;
      if (D.shift) D.shift[k] = NAN;
      if (D.mu) D.mu[k] = NAN;
      if (D.info) D.info[k] = pf;
    }
    return false;
  }
  double pv = w.pv1[k], s = 0.0, mu = w.mu1[k];
  uint32_t fl = w.fl1[k];
  const int m = P.m;
  int c_it = 0, c_dd = 0, c_plain = 1;   // the norm pass
  double rn = NAN;   // 1/||x|| from a remedy's last rational pass, when it ran one
  double off_hint = -1.0;   // the norm pass's scale, when it is not |s + mu|
  double knu_out = NAN;     // K_nu of the first pass, for the outputs
  if (m > 0 && opt.remedies) {
    const int i = w.ip1[k];
    const int side = (k == i) ? +1 : -1;
    const double di = P.ds[i];
    const double lam1 = dd_to_d(dd_add_d(pval_dd<KIND>(di), mu));
    // Theorem 2 (C1) and its exceptions (a)-(c): lambda near zero
    const double quot = (fabs(pval<KIND>(di)) + fabs(mu)) / fabs(lam1);
    // K_nu (eq. K0): ||A_i^{-1}||_2 = 1 / distance from d_i to the nearer of
    // the two eigenvalues adjacent to d_i
    const int o = (side > 0) ? k + 1 : k - 1;
    const double dist_o = fabs(pdiff<KIND>(w.pv1[o], di) + w.mu1[o]);
    const double knu = fabs(mu) / fmin(fabs(mu), dist_o);
    knu_out = knu;
    const bool zero_pole = w.hdr[2] != 0.0;
    const bool near_zero = quot > opt.tau_zero && !zero_pole;
    if constexpr (DEFER == DEFER_ALL) {
      if (near_zero || knu > opt.tau_nu) {
        defer_repair(w, D.n, k, ln);
        return false;
      }
    }
    if constexpr (DEFER == DEFER_NEAR_ZERO || DEFER == DEFER_WAVE) {
      if (near_zero) {
        defer_repair(w, D.n, k, ln);
        return false;
      }
    }
    if constexpr (DEFER == DEFER_WAVE) {
      if (knu > opt.tau_nu) return true;
    }
    if constexpr (DEFER != DEFER_ALL) {   // the fully deferring check stage returned above
      // Remark 1 runs only where nothing was deferred: its exact sum needs whole wavefronts
      bool r1 = false;
      if constexpr (DEFER == DEFER_NONE) r1 = near_zero;
      if (r1) {
        if constexpr (DEFER == DEFER_NONE) {
          // Remark 1: lambda from the absolutely largest eigenvalue of A^{-1}, whose
          // weight rho = 1/f(0) is summed exactly where double-double cannot resolve it
          int z0 = 0, it = 0, unres = 0;
          const double l0 = origin_root<KIND, G>(P, ln, lam1, &z0, &unres, &it,
                                                 [&](int* ok) { return f_origin<KIND, G>(D, P, ln, ok); });
          pv = 0.0; s = 0.0; mu = z0 ? 0.0 : l0;
          // entries z_j / (d_j - lambda): their scale is the nearest pole's
          // distance from the origin, which the norm pass below is given
          off_hint = fabs(pval<KIND>(di));
          fl |= INFO_NEAR_ZERO;
          if (unres) fl |= INFO_F0_UNRESOLVED;
          c_it += it; c_dd += 1;
        }
      } else if (knu > opt.tau_nu) {
        bool done = false;
        const int i2 = (side > 0) ? i - 1 : i + 1;
        if (i2 >= 0 && i2 < m) {
          // Remark 2(a): the other neighbouring pole, if K_nu is small there and
          // lambda is not so close to d_i that its vector entries would suffer
          const double d2 = P.ds[i2];
          const double mu2 = fabs(pdiff<KIND>(di, d2) + mu);
          const int o2 = (side > 0) ? k - 1 : k + 1;
          const double dist2 = fabs(pdiff<KIND>(w.pv1[o2], d2) + w.mu1[o2]);
          const double knu2 = mu2 / fmin(mu2, dist2);
          // the eigenvector entry of the nearer pole d_i is then formed as
          // (d_i - d_{i2}) - mu2, which cancels by |d_i - d_{i2}| / |lambda - d_i|
          const double cancel = fabs(pdiff<KIND>(di, d2)) / fabs(mu);
          if (knu2 <= opt.tau_nu && cancel <= 8.0) {
            const BPass bp = b_pass<KIND, G>(P, i2, -side, ln, opt.fp64_b);
            int it = 0;
            const int side2 = -side;
            // first-pass lambda seen from the other pole: 1 / (lambda - d_i2)
            const double nu_est = 1.0 / (pdiff<KIND>(di, d2) + mu);
            double last[3] = {NAN, NAN, NAN};
            const double nu = (opt.root == ROOT_RATIONAL)
                ? rational_inverse<KIND, G>(P, i2, side2, bp.b, bp.lo, bp.hi, side2 > 0 ? bp.lo : bp.hi, ln, &it,
                                            nu_est, last)
                : bisect_inverse<KIND, G>(P, i2, bp.b, bp.lo, bp.hi, ln, &it);
            pv = d2; s = 0.0; mu = 1.0 / nu;
            if (last[0] == last[0]) {
              rn = norm_from_pass(last, nu, P.ch[i2]);
              if constexpr (KIND == KIND_DPR1) rn = dpr1_inorm(P, rn, mu, d2);
            }
            fl |= INFO_REMEDY_A;
            done = true;
            c_it += it; c_dd += opt.fp64_b ? 0 : 1; c_plain += opt.fp64_b ? 1 : 0;
          }
        }
        if (!done) {
          // Remark 2(b): invert A - sigma I with sigma between d_i and lambda,
          // 2^-10 |mu| away from lambda
          s = mu - mu * (1.0 / 1024.0);
          int z0 = 0, it = 0;
          double last[3] = {NAN, NAN, NAN};
          const double m2 = dpr1_inverse<KIND, G>(P, di, s, ln, &z0, &it, opt.root, 1.0 / (mu - s), last);
          pv = di; mu = z0 ? 0.0 : m2;
          if (!z0 && last[0] == last[0]) {
            rn = norm_from_pass(last, 1.0 / m2, 0.0);
            if constexpr (KIND == KIND_DPR1) rn = dpr1_inorm(P, rn, s + m2, di);
          }
          fl |= INFO_REMEDY_B;
          c_it += it; c_dd += 1;
        }
      }
    }
  }
  if constexpr (KIND == KIND_DPR1) {
    // the smallest eigenvalue, when nearer to d_n than to d_{n-1} (not after
    // Remark 1, whose eigenvalue is accurate relative to itself and far from d_n)
    if (m > 0 && k == m && !(fl & INFO_NEAR_ZERO)) {
      const double dn = P.ds[P.nsorted - 1];
      const double gap = P.ds[P.nsorted - 2] - dn;
      const double tau = (pv - dn) + s + mu;
      if (tau < 0.5 * gap) {
        if constexpr (DEFER == DEFER_ALL) {
          defer_repair(w, D.n, k, ln);
          return false;
        }
        if constexpr (DEFER == DEFER_WAVE) return true;
        int it = 0;
        const double t2 = dpr1_from_last_pole<G>(P, tau, ln, &it);
        pv = dn; s = 0.0; mu = t2;
        rn = NAN;   // a remedy's norm above was for the eigenvalue before this re-measure
        fl |= INFO_POLE_SHIFT;
        c_it += it;
      }
    }
  }
  // the first pass's norm holds while its shift and mu stand (no remedy)
  const double nr1 = w.nr1[k];
  const bool first = pv == w.pv1[k] && s == 0.0 && mu == w.mu1[k] && nr1 == nr1;
  const double inrm = first ? nr1 : (rn == rn ? rn : inv_norm<KIND, G>(P, pv, s, mu, ln, off_hint));
  if (first || rn == rn) c_plain -= 1;   // no norm pass
  if (ln == 0) {
    w.cnt[6 * k + 3] = c_it;
    w.cnt[6 * k + 4] = c_dd;
    w.cnt[6 * k + 5] = c_plain;
    const dd sh = dd_add_d(pval_dd<KIND>(pv), s);
    const double lam = dd_to_d(dd_add_d(sh, mu));
    int col = k;   // output column: k unless eigenpairs were deflated
    double sg = 1.0;   // -1: DPR1 with rho < 0, whose eigenvalue order is reversed
    if constexpr (KIND == KIND_ARROW) {
      const int nd = deflated_count(w);
      if (nd > 0) {
        col = k + count_above(w.dv, nd, lam, false);
        w.lr[k] = lam;
        w.cm[col] = -1;
      }
    }
    if constexpr (KIND == KIND_DPR1) {
      if (D.neg) {
        col = D.n - 1 - k;
        sg = -1.0;
      }
    }
    w.pv[col] = pv;
    w.kbc[col] = w.kb1[k];
    w.knu[col] = knu_out;
    w.sf[col] = s;
    w.mu[col] = mu;
    // q = (D - lambda)^{-1} u for rho < 0 is minus the vector of (-D) + |rho| u u^T
    w.inrm[col] = sg * inrm;
    if constexpr (KIND == KIND_SVD) D.lam[col] = sqrt(fmax(lam, 0.0));
    else D.lam[col] = sg * lam;
    if (D.shift) D.shift[col] = sg * dd_to_d(sh);
    if (D.mu) D.mu[col] = sg * mu;
    if (D.info) D.info[col] = fl;
  }
  return false;
}

// ---------------------------------------------------------------------------
// eigenvector entry (row r, caller order) of column k; eq. (eigenvecAi) with
// the shift pair, normalised.  SVD also returns u_r (Sec. 6.2).

template <int KIND>
__host__ __device__ inline double vec_elem(const ProbDesc& D, double pv, double s, double mu, double inrm,
                                           int r) {
  const int n = D.n;
  if constexpr (KIND == KIND_DPR1) {
    return (D.z[r] * inrm) * recip(((in_pole<KIND>(D, r) - pv) - s) - mu);
  } else {
    if (r == n - 1) return -inrm;
    if (KIND == KIND_ARROW && D.z[r] == 0.0) return 0.0;   // a deflated row
    const double num = (KIND == KIND_SVD) ? D.d[r] * D.z[r] : D.z[r];
    return (num * inrm) * recip((pdiff<KIND>(D.d[r], pv) - s) - mu);
  }
}

// the same entry from values preloaded per row: dr = d_r, num = z_r (u_r for
// DPR1, d_r z_r for SVD); last marks the corner row of ARROW / SVD
template <int KIND>
__host__ __device__ inline double vec_entry(double dr, double num, bool last, double pv, double s, double mu,
                                            double inrm) {
  if constexpr (KIND == KIND_DPR1) {
    return (num * inrm) * recip(((dr - pv) - s) - mu);
  } else {
    if (last) return -inrm;
    if (KIND == KIND_ARROW && num == 0.0) return 0.0;   // a deflated row
    return (num * inrm) * recip((pdiff<KIND>(dr, pv) - s) - mu);
  }
}

// Hermitian arrowhead (Sec. 6.1): u = Phi v with Phi = diag(z_j/|z_j|, 1), so
// u_r = z_r / ((d_r - pole) - s - mu) / ||x|| with the complex z_r = zr + i zi,
// and the corner entry is -1/||x||.  Each part is rounded as vec_entry rounds
// the real case, so zi = 0 gives vec_entry's value.
__host__ __device__ inline void vec_entry_c(double dr, double zr, double zi, bool last, double pv, double s,
                                            double mu, double inrm, double* ur, double* ui) {
  if (last) {
    *ur = -inrm;
    *ui = 0.0;
    return;
  }
  const double f = recip(((dr - pv) - s) - mu);
  *ur = (zr * inrm) * f;
  *ui = (zi * inrm) * f;
}

// SVD left vector entry from the right vector entry v_r: u_j = sigma v_j / d_j,
// u_n = alpha v_n / sigma
__host__ __device__ inline double svd_left(const ProbDesc& D, double sigma, double v, int r) {
  return (r == D.n - 1) ? D.scalar * v / sigma : sigma * v / D.d[r];
}

}  // namespace ahd
