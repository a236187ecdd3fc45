// Double-double arithmetic on FP64, written from the published error-free
// transformations: TwoSum (Knuth, TAOCP vol. 2, 4.2.2), FastTwoSum (Dekker
// 1971), TwoProd through one fused multiply-add, and the double-double
// add/mul/div built from them.  dd_add (two TwoSums, the low parts added and
// renormalised twice) and dd_div (three quotient digits) follow the
// "accurate" addition and the long division of Hida, Li and Bailey's
// double-double/quad-double library (QD; "Algorithms for quad-double precision
// floating point arithmetic", ARITH-15, 2001), written here from that paper's
// description; dd_mul is Dekker's product with its cross terms gathered by
// FMA.  A value is the unevaluated sum hi + lo with
// |lo| <= ulp(hi)/2; the unit roundoff of the format is about 2^-104, which
// realises the "double of the working precision" of Sec. 4 (Theorem 6).
//
// Everything here must be compiled without floating-point contraction
// (-ffp-contract=off): the transformations rely on each + and - being
// rounded separately.
#pragma once

#include <hip/hip_runtime.h>

namespace ahd {

struct dd {
  double hi, lo;
};

__host__ __device__ inline dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

// requires |a| >= |b| (or a == 0)
__host__ __device__ inline dd fast_two_sum(double a, double b) {
  double s = a + b;
  double e = b - (s - a);
  return {s, e};
}

__host__ __device__ inline dd two_prod(double a, double b) {
  double p = a * b;
  double e = fma(a, b, -p);
  return {p, e};
}

__host__ __device__ inline dd dd_from(double a) { return {a, 0.0}; }
__host__ __device__ inline dd dd_neg(dd a) { return {-a.hi, -a.lo}; }

__host__ __device__ inline dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

__host__ __device__ inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

__host__ __device__ inline dd dd_add_d(dd a, double b) {
  dd s = two_sum(a.hi, b);
  s.lo += a.lo;
  return fast_two_sum(s.hi, s.lo);
}

__host__ __device__ inline dd dd_mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo = fma(a.hi, b.lo, fma(a.lo, b.hi, p.lo));
  return fast_two_sum(p.hi, p.lo);
}

__host__ __device__ inline dd dd_mul_d(dd a, double b) {
  dd p = two_prod(a.hi, b);
  p.lo = fma(a.lo, b, p.lo);
  return fast_two_sum(p.hi, p.lo);
}

// three quotient digits, then renormalise
__host__ __device__ inline dd dd_div(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd r = dd_sub(a, dd_mul_d(b, q1));
  double q2 = r.hi / b.hi;
  r = dd_sub(r, dd_mul_d(b, q2));
  double q3 = r.hi / b.hi;
  dd q = fast_two_sum(q1, q2);
  return dd_add_d(q, q3);
}

__host__ __device__ inline double dd_to_d(dd a) { return a.hi + a.lo; }

// c / e with two quotient digits, given r ~ 1/e.hi to about one ulp:
// q1 = c.hi r, then the remainder c - q1 e (its leading part c.hi - q1 e.hi is
// exact through TwoProd) times r once more.  q1 need not be the rounded
// quotient: the remainder carries its error exactly, so the pair is good to a
// few units of 2^-104 -- enough where quotients of one sign are summed, which
// is the only use.  dd_div2_raw leaves the pair unnormalised (|q.lo| is a few
// ulps of q.hi); dd_div2 renormalises it.
__host__ __device__ inline dd dd_div2_raw(dd c, dd e, double r) {
  const double q1 = c.hi * r;
  const dd p = two_prod(q1, e.hi);
  const double rem = (((c.hi - p.hi) - p.lo) + c.lo) - q1 * e.lo;
  return {q1, rem * r};
}

__host__ __device__ inline dd dd_div2(dd c, dd e, double r) {
  const dd q = dd_div2_raw(c, e, r);
  return fast_two_sum(q.hi, q.lo);
}

// s += c / e for a running sum of quotients of one sign, given r ~ 1/e.hi (as
// for dd_div2_raw): the first digit q1 = c.hi r enters s.hi through TwoSum, and
// the second digit, the remainder c - q1 e times r, is folded by one FMA into
// the addition error that s.lo gathers.  The remainder's last term q1 e.lo is
// an FMA too: two operations fewer than forming the pair (dd_div2_raw) and
// adding it, for the same two digits.
__host__ __device__ inline void dd_acc_div2(dd& s, dd c, dd e, double r) {
  const double q1 = c.hi * r;
  const dd p = two_prod(q1, e.hi);
  const double rem = fma(-q1, e.lo, ((c.hi - p.hi) - p.lo) + c.lo);
  const dd t = two_sum(s.hi, q1);
  s.hi = t.hi;
  s.lo += fma(rem, r, t.lo);
}

__host__ __device__ inline dd dd_norm(dd s) { return fast_two_sum(s.hi, s.lo); }

}  // namespace ahd
