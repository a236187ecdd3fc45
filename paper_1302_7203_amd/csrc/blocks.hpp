// Block-level device routines shared by the single-problem and batched
// kernels: the prologue of one problem and the sort of one problem by one block.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bodies.hpp"

namespace ahd {

constexpr int BLOCK = 256;

// Shaft weights and corner of the (reduced) arrowhead in double-double, the
// problem flags, and whether some pole is exactly zero.  One block of NT threads.
template <int KIND, int NT = BLOCK>
__device__ inline void prologue_block(const ProbDesc& D) {
  __shared__ double shi[NT], slo[NT];
  __shared__ uint32_t sst[NT];
  const Ws w = ws_view(D.ws, D.n);
  const int ms = sorted_count(D);
  const int m = D.n - 1;
  const int t = threadIdx.x;
  uint32_t st = 0;
  uint32_t zp = 0;
  dd acc = {0.0, 0.0};
  for (int j = t; j < ms; j += NT) {
    st |= w.st[j];
    acc = dd_add(acc, corner_term<KIND>(D, w, j));
  }
  for (int j = t; j < m; j += NT) {
    prologue_elem<KIND>(D, w, j);
    zp |= (w.ds[j] == 0.0) ? 1u : 0u;
  }
  shi[t] = acc.hi;
  slo[t] = acc.lo;
  sst[t] = st | (zp << 31);
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (t < o) {
      const dd a = dd_add(dd{shi[t], slo[t]}, dd{shi[t + o], slo[t + o]});
      shi[t] = a.hi;
      slo[t] = a.lo;
      sst[t] |= sst[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    const dd c = dd_add(corner_base<KIND>(D, w), dd{shi[0], slo[0]});
    w.hdr[0] = c.hi;
    w.hdr[1] = c.lo;
    w.hdr[2] = (sst[0] >> 31) ? 1.0 : 0.0;
    *prob_flags(w) = sst[0] & 0x7fffffffu;
    *repair_count(w) = 0u;
  }
  __syncthreads();
}

// Sort of one problem by one block: a copy when the input already has
// strictly decreasing keys, else the rank of every key (ties by index).
template <int KIND>
__device__ inline void sort_block(const ProbDesc& D) {
  __shared__ double tile[BLOCK];
  const Ws w = ws_view(D.ws, D.n);
  const int ms = sorted_count(D);
  int bad = 0;
  for (int j = threadIdx.x; j + 1 < ms; j += BLOCK)
    if (!(sort_key<KIND>(D.d[j]) > sort_key<KIND>(D.d[j + 1]))) bad = 1;
  bad = __syncthreads_or(bad);
  if (!bad) {
    for (int j = threadIdx.x; j < ms; j += BLOCK) {
      w.ds[j] = D.d[j];
      w.zs[j] = D.z[j];
      w.st[j] = input_status<KIND>(D, j, false);
    }
    __syncthreads();
    return;
  }
  for (int j0 = 0; j0 < ms; j0 += BLOCK) {
    const int j = j0 + threadIdx.x;
    const double kj = (j < ms) ? sort_key<KIND>(D.d[j]) : NAN;
    int rank = 0;
    bool dup = false;
    for (int base = 0; base < ms; base += BLOCK) {
      const int l = base + threadIdx.x;
      tile[threadIdx.x] = (l < ms) ? sort_key<KIND>(D.d[l]) : NAN;
      __syncthreads();
      const int lim = min(BLOCK, ms - base);
      for (int t = 0; t < lim; ++t) {
        const double kl = tile[t];
        const int idx = base + t;
        rank += (kl > kj) || (kl == kj && idx < j);
        dup |= (kl == kj) && (idx != j);
      }
      __syncthreads();
    }
    if (j < ms) {
      w.ds[rank] = D.d[j];
      w.zs[rank] = D.z[j];
      w.st[j] = input_status<KIND>(D, j, dup);
    }
  }
  __syncthreads();
}

}  // namespace ahd
