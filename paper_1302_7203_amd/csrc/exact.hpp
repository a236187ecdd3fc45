// The value f(0) of the Pick function at the origin, accurate relative to
// itself however much its terms cancel.
//
// Remark 1 of Sec. 3 takes the eigenvalue of A nearest 0 from the extreme
// eigenvalue of A^{-1}, a DPR1 matrix whose weight is rho = 1/f(0); that
// eigenvalue inherits the relative error of f(0).  The paper evaluates f(0) in
// doubled precision, which resolves it while its terms cancel by less than
// about 2^-100 of their size.  Below that (an eigenvalue at 1e-30 next to poles
// of size 1, say) this routine sums the terms exactly:
//
//   f(0) = K + sgn * sum_t n_t / p_t        with exact doubles n_t, p_t, K,
//
// each quotient written as a sum of FP64 digits q_1 + q_2 + ... (q = RN(r/p),
// r <- r - q p, the new remainder exact through one FMA: the remainder of a
// rounded quotient is a double), and all digits added into a fixed-point long
// accumulator: 72 limbs of 32 bits from 2^-1152 up to 2^1152, each limb an
// int64 that takes signed 32-bit chunks, so the sum is exact and independent
// of the order of the additions.  The idea of a long accumulator for exact
// floating-point sums is Kulisch's; the 32-bit chunks in 64-bit words with
// deferred carries follow the long accumulators of ExBLAS (Collange, Defour,
// Graillat, Iakymchuk).  Digits stop when the remaining quotient is below a
// threshold T; the dropped tail is bounded and T lowered until f(0) is resolved
// to 2^-56 of itself.
//
// The group of G lanes that calls this is a whole block on the device (the
// repair kernels run one eigenvalue per block); the accumulator sits in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dd.hpp"

namespace ahd {

constexpr int XL = 72;        // limbs
constexpr int XBASE = -1152;  // exponent of limb 0's lowest bit; a double's lowest bit is >= 2^-1126

// Add q exactly: q = M 2^(e-53) with the integer M < 2^53 placed across three
// 32-bit chunks.
__host__ __device__ inline void xacc_add(unsigned long long* acc, double q) {
  if (q == 0.0) return;
  int e = 0;
  const double m = frexp(q, &e);                                       // q = m 2^e, 1/2 <= |m| < 1
  const unsigned long long M = (unsigned long long)ldexp(fabs(m), 53);  // exact
  const int b = e - 53 - XBASE;                                        // >= 0 for every double
  const int L = b >> 5, sh = b & 31;
  const unsigned long long lo = M << sh;                               // bits 0..63 of M 2^sh
  const unsigned long long hi = sh ? (M >> (64 - sh)) : 0ull;          // bits 64..84
  unsigned long long c0 = lo & 0xffffffffull, c1 = lo >> 32, c2 = hi;
  if (q < 0.0) { c0 = 0ull - c0; c1 = 0ull - c1; c2 = 0ull - c2; }    // two's complement
#if defined(__HIP_DEVICE_COMPILE__)
  atomicAdd(&acc[L], c0);
  if (c1) atomicAdd(&acc[L + 1], c1);
  if (c2) atomicAdd(&acc[L + 2], c2);
#else
  acc[L] += c0;
  acc[L + 1] += c1;
  acc[L + 2] += c2;
#endif
}

// The accumulated value, rounded (relative error below 2^-52).
__host__ __device__ inline double xacc_value(const unsigned long long* acc) {
  uint32_t lim[XL];
  long long carry = 0;
  for (int L = 0; L < XL; ++L) {
    const long long v = (long long)acc[L] + carry;
    const long long low = v & 0xffffffffll;
    lim[L] = (uint32_t)low;
    carry = (v - low) / 4294967296ll;   // exact: v - low is a multiple of 2^32
  }
  double sgn = 1.0;
  if (carry < 0) {   // negative: take the two's complement of the limbs
    sgn = -1.0;
    unsigned long long c = 1;
    for (int L = 0; L < XL; ++L) {
      const unsigned long long t = (unsigned long long)(uint32_t)~lim[L] + c;
      lim[L] = (uint32_t)t;
      c = t >> 32;
    }
  }
  int top = XL - 1;
  while (top >= 0 && lim[top] == 0) --top;
  if (top < 0) return 0.0;
  double v = (double)lim[top];
  if (top >= 1) v = v * 4294967296.0 + (double)lim[top - 1];
  if (top >= 2) v = v * 4294967296.0 + (double)lim[top - 2];
  const int low = top >= 2 ? top - 2 : 0;
  return sgn * ldexp(v, XBASE + 32 * low);
}

// Digits of n/p with |remainder/p| > T, each added with sign sgn; returns the
// dropped tail's bound (and sets *bad for a non-finite quotient).
__host__ __device__ inline double xacc_quotient(unsigned long long* acc, double n, double p, double sgn, double T,
                                                int* bad) {
  double r = n, tail = 0.0;
  for (int t = 0; t < 48 && r != 0.0; ++t) {
    const double q = r / p;
    if (!(fabs(q) < INFINITY)) { *bad = 1; return 0.0; }
    if (fabs(q) <= T) { tail += fabs(q) * (1.0 + 0x1p-40); r = 0.0; break; }
    xacc_add(acc, sgn * q);
    r = fma(-q, p, r);
    // below 2^-960 the remainder may lose bits under 2^-1074 to underflow
    if (r != 0.0 && fabs(r) < 0x1p-960) tail += 0x1p-1074 / fabs(p);
  }
  if (r != 0.0) tail += fabs(r / p) * (1.0 + 0x1p-40);
  return tail;
}

#if defined(__HIP_DEVICE_COMPILE__)
__device__ inline double block_sum_max(double v, bool take_max) {
  __shared__ double slot[16];
  const int w = threadIdx.x >> 6;
  for (int o = 32; o >= 1; o >>= 1) {
    const double u = __shfl_xor(v, o, 64);
    v = take_max ? fmax(v, u) : v + u;
  }
  if ((threadIdx.x & 63) == 0) slot[w] = v;
  __syncthreads();
  double r = slot[0];
  for (int q = 1; q < (int)(blockDim.x >> 6); ++q) r = take_max ? fmax(r, slot[q]) : r + slot[q];
  __syncthreads();
  return r;
}
#endif

// f(0) for the problem the kernels solve (KIND_ARROW also covers Hermitian
// input, D.kind == 3, whose shaft is |z|; DPR1 is reduced as in Sec. 6.3, so
// its arrowhead has f(0) = d_n phi(0), phi(0) = 1 + |rho| sum_j u_j^2 / d_j).
// rows(r, &p, n) gives caller row r's pole p and its exact numerator parts
// n[0..3], returning how many there are; the result is scale times the sum.
// *resolved is 0 when even the full expansion leaves f(0) unresolved (f(0) is
// then 0 to within the accumulator's reach).
template <int KIND, int G, class Rows>
__host__ __device__ inline double origin_exact(int ln, int nrows, double K, double sgn, double scale, Rows&& rows,
                                               int* resolved) {
#if defined(__HIP_DEVICE_COMPILE__)
  static_assert(G % 64 == 0, "the exact sum runs on whole blocks");
  __shared__ unsigned long long acc[XL];
#else
  unsigned long long acc[XL];
#endif
  // magnitude of the terms, for the first threshold
  double mag = 0.0;
  for (int r = ln; r < nrows; r += G) {
    double p, nn[4];
    const int np = rows(r, &p, nn);
    for (int a = 0; a < np; ++a) mag = fmax(mag, fabs(nn[a] / p));
  }
#if defined(__HIP_DEVICE_COMPILE__)
  mag = block_sum_max(mag, true);
#endif
  mag = fmax(mag, fabs(K));
  double T = mag * 0x1p-180;
  double val = 0.0;
  *resolved = 0;
  for (int round = 0; round < 8; ++round) {
    const double Tt = T / (4.0 * (double)(nrows + 1));   // per part: the parts' tails add to at most T
#if defined(__HIP_DEVICE_COMPILE__)
    for (int L = threadIdx.x; L < XL; L += blockDim.x) acc[L] = 0ull;
    __syncthreads();
#else
    for (int L = 0; L < XL; ++L) acc[L] = 0ull;
#endif
    double tail = 0.0;
    int bad = 0;
    if (ln == 0) xacc_add(acc, K);
    for (int r = ln; r < nrows; r += G) {
      double p, nn[4];
      const int np = rows(r, &p, nn);
      for (int a = 0; a < np; ++a) tail += xacc_quotient(acc, nn[a], p, sgn, Tt, &bad);
    }
#if defined(__HIP_DEVICE_COMPILE__)
    tail = block_sum_max(tail, false);
    const double badsum = block_sum_max((double)bad, false);
    __shared__ double res;
    if (threadIdx.x == 0) res = xacc_value(acc);
    __syncthreads();
    val = res;
    __syncthreads();
    if (badsum > 0.0) return NAN;
#else
    val = xacc_value(acc);
    if (bad) return NAN;
#endif
    tail *= 1.0 + 0x1p-30;
    if (tail == 0.0 || fabs(val) > tail * 0x1p56) { *resolved = 1; break; }
    if (T <= 0x1p-1074) break;         // digits reached the bottom of the exponent range
    T = fmax(T * 0x1p-300, 0x1p-1074);
  }
  return val * scale;
}

}  // namespace ahd
