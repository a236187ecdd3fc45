// Block-level device routines shared by the single-problem and batched
// kernels: the prologue of one problem and the sort of one problem by one block.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bodies.hpp"

namespace ahd {

constexpr int BLOCK = 256;

// Deflation of a reducible arrowhead (see deflate_run) by one block: thread t
// takes the runs that start in its chunk of the sorted poles; a block-wide
// scan of the per-chunk counts gives every run its reduced index and item
// numbers.  The kept poles are gathered in pv1 (free until the first pass)
// and copied back over the sorted poles, which the runs read until then.
template <int NT>
__device__ inline void deflate_block(const Ws& w, int m) {
  __shared__ int kc[NT], ic[NT];
  const int t = threadIdx.x;
  const int chunk = (m + NT - 1) / NT;
  const int j0 = min(m, t * chunk), j1 = min(m, j0 + chunk);
  int keep = 0, items = 0;
  for (int j = j0; j < j1; ++j) {
    if (!run_start(w.ds, j)) continue;
    const DeflCount c = deflate_count(w, m, j);
    keep += c.keep;
    items += c.items;
  }
  kc[t] = keep;
  ic[t] = items;
  __syncthreads();
  for (int o = 1; o < NT; o <<= 1) {   // inclusive scan
    const int a = (t >= o) ? kc[t - o] : 0, b = (t >= o) ? ic[t - o] : 0;
    __syncthreads();
    kc[t] += a;
    ic[t] += b;
    __syncthreads();
  }
  int r = kc[t] - keep, q = ic[t] - items;
  const int mr = kc[NT - 1], nd = ic[NT - 1];
  int zp = 0;
  for (int j = j0; j < j1; ++j)
    if (run_start(w.ds, j)) zp |= deflate_run(w, m, j, r, q, w.pv1) ? 1 : 0;
  zp = __syncthreads_or(zp);
  for (int j = t; j < mr; j += NT) w.ds[j] = w.pv1[j];
  if (t == 0) {
    w.hdr[8] = (double)mr;
    w.hdr[9] = (double)nd;
    w.hdr[2] = zp ? 1.0 : 0.0;
    *prob_flags(w) = 0u;
  }
}

// Shaft weights and corner of the (reduced) arrowhead in double-double, the
// problem flags, and whether some pole is exactly zero.  One block of NT
// threads.  prologue_reduce combines the threads' corner partial sums (in a
// fixed order: each wavefront's by a butterfly, then the wavefronts'),
// statuses and zero-pole bits and writes the header; a reducible arrowhead is
// then deflated.
template <int KIND, int NT>
__device__ inline void prologue_reduce(const ProbDesc& D, const Ws& w, dd acc, uint32_t st, uint32_t zp) {
  static_assert(NT % 64 == 0, "whole wavefronts");
  constexpr int NW = NT / 64;
  __shared__ double whi[NW], wlo[NW];
  __shared__ uint32_t wst[NW];
  __shared__ uint32_t sflags;
  const int m = D.n - 1;
  const int t = threadIdx.x;
  // each wavefront's partial sums by the lanes' butterfly (every lane ends
  // with the same bits), then the wavefronts' in order by one thread
  const dd a = gsum_dd<64>(acc);
  uint32_t f = st | (zp << 31);
  for (int o = 32; o > 0; o >>= 1) f |= (uint32_t)__shfl_xor((int)f, o, 64);
  if ((t & 63) == 0) {
    whi[t >> 6] = a.hi;
    wlo[t >> 6] = a.lo;
    wst[t >> 6] = f;
  }
  __syncthreads();
  if (t == 0) {
    dd c = corner_base<KIND>(D, w);
    uint32_t all = 0;
    dd sum = {whi[0], wlo[0]};
    all |= wst[0];
    for (int q = 1; q < NW; ++q) {
      sum = dd_add(sum, dd{whi[q], wlo[q]});
      all |= wst[q];
    }
    c = dd_add(c, sum);
    w.hdr[0] = c.hi;
    w.hdr[1] = c.lo;
    w.hdr[2] = (all >> 31) ? 1.0 : 0.0;
    *prob_flags(w) = all & 0x7fffffffu;
    *repair_count(w) = 0u;
    *place_done(w) = 0u;
    w.hdr[8] = (double)m;
    w.hdr[9] = 0.0;
    sflags = all & 0x7fffffffu;
  }
  __syncthreads();
  if constexpr (KIND == KIND_ARROW) {
    if (sflags == INFO_REDUCIBLE) deflate_block<NT>(w, m);
  }
  __syncthreads();
}

// The prologue over the sorted copy in the workspace: statuses (w.st), the
// corner partial sums by thread over j = t, t + NT, ..., and the weights.
template <int KIND, int NT = BLOCK>
__device__ inline void prologue_block(const ProbDesc& D) {
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
  prologue_reduce<KIND, NT>(D, w, acc, st, zp);
}

// Sort of one problem by one block: a copy when the input already has
// strictly decreasing (or strictly increasing) keys, else the rank of every
// key (ties by index).
template <int KIND>
__device__ inline void sort_block(const ProbDesc& D) {
  __shared__ double tile[BLOCK];
  const Ws w = ws_view(D.ws, D.n);
  const int ms = sorted_count(D);
  int down = 0, up = 0;
  for (int j = threadIdx.x; j + 1 < ms; j += BLOCK) {
    const double a = sort_key<KIND>(in_pole<KIND>(D, j)), b = sort_key<KIND>(in_pole<KIND>(D, j + 1));
    if (!(a > b)) down = 1;
    if (!(a < b)) up = 1;
  }
  down = __syncthreads_or(down);
  up = __syncthreads_or(up);
  if (!(down && up)) {
    const bool rev = down != 0;
    for (int j = threadIdx.x; j < ms; j += BLOCK) {
      put_sorted<KIND>(D, w, rev ? ms - 1 - j : j, j);
      w.st[j] = input_status<KIND>(D, j, false);
    }
    __syncthreads();
    return;
  }
  for (int j0 = 0; j0 < ms; j0 += BLOCK) {
    const int j = j0 + threadIdx.x;
    const double kj = (j < ms) ? sort_key<KIND>(in_pole<KIND>(D, j)) : NAN;
    int rank = 0;
    bool dup = false;
    for (int base = 0; base < ms; base += BLOCK) {
      const int l = base + threadIdx.x;
      tile[threadIdx.x] = (l < ms) ? sort_key<KIND>(in_pole<KIND>(D, l)) : NAN;
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
      put_sorted<KIND>(D, w, rank, j);
      w.st[j] = input_status<KIND>(D, j, dup);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Eigenvector entries (eq. eigenvecAi, Algorithm 4), streamed to HBM.
//
// vec_tile: the block owns rows [rt*BLOCK*RPT, ...) of columns [ct*cols,
// ...): each thread keeps its RPT rows' d_r and numerators in registers and
// writes one entry per row and column.  W = 2 lets a lane write two
// consecutive rows with one 16-byte non-temporal store (n and the leading
// dimensions even, V and U 16-byte aligned); W = 1 writes one row per store.
// The measured best tile shape depends on n (vec_shape).
//
// The block's column data (shift pole, offset, mu, 1/||x||, ...) is staged in
// LDS before the column loop: read from the workspace inside the loop, each
// column's loads would wait behind the previous column's stores, which the
// compiler cannot tell apart from them.
#ifndef AHD_VEC_RPT
#define AHD_VEC_RPT 2
#endif
constexpr int VEC_RPT = AHD_VEC_RPT;           // rows per thread (batched path)
constexpr int VEC_TILE = BLOCK * VEC_RPT;      // rows per block
#ifndef AHD_VEC_COLS
#define AHD_VEC_COLS 8
#endif
constexpr int VEC_COLS = AHD_VEC_COLS;         // columns per block (batched path)
constexpr int VEC_COLS_MAX = 32;               // most columns a row-tile block takes (vec_shape)
constexpr int VEC_FLAT_COLS = 256;             // most columns a flat tile takes
#ifndef AHD_VEC_FLAT_ROWS
#define AHD_VEC_FLAT_ROWS 512
#endif
constexpr int VEC_FLAT_ROWS = AHD_VEC_FLAT_ROWS; // flat tiles serve orders below this
typedef double v2d __attribute__((ext_vector_type(2)));

// LDS of a vector block: C columns' data and, for flat tiles, R rows' data
template <int C, int R>
struct VecStage {
  double pv[C], sf[C], mu[C], inrm[C], sig[C];
  int cm[C];
  double dr[R], num[R];
};
using VecTileStage = VecStage<VEC_COLS_MAX, 1>;
using VecFlatStage = VecStage<VEC_FLAT_COLS, VEC_FLAT_ROWS>;

struct VecShape {
  int rpt, cols;
};

// rows per thread and columns per block for a single problem of order n:
// tall tiles for large n, wide ones around n = 4096, and for smaller n narrow
// ones so that the grid keeps a few hundred blocks
__host__ __device__ inline VecShape vec_shape(int64_t n) {
  if (n > 4096) return VecShape{8, 16};
  if (n > 2048) return VecShape{4, 32};
  if (n > 1024) return VecShape{4, 8};
  if (n > 512) return VecShape{4, 4};
  return VecShape{2, n >= 512 ? 2 : 1};
}

// columns [c0, c0 + nc) of the workspace's final shift pairs into L (every
// thread of the block calls this; it ends with a barrier)
template <int KIND, class S>
__device__ inline void stage_cols(const ProbDesc& D, const Ws& w, int c0, int nc, int nd, S& L) {
  for (int c = threadIdx.x; c < nc; c += BLOCK) {
    const int col = c0 + c;
    L.pv[c] = w.pv[col];
    L.sf[c] = w.sf[col];
    L.mu[c] = w.mu[col];
    L.inrm[c] = w.inrm[col];
    if constexpr (KIND == KIND_SVD) L.sig[c] = D.lam[col];
    if constexpr (KIND == KIND_ARROW) L.cm[c] = nd > 0 ? w.cm[col] : -1;
  }
  __syncthreads();
}

template <int KIND, int W, int RPT, class S, bool STAGE = true>
__device__ inline void vec_tile(const ProbDesc& D, int rt, int ct, int cols, S& L) {
  static_assert(W == 1 || W == 2, "one or two rows per store");
  static_assert(RPT % W == 0, "rows per thread");
  constexpr int PER = RPT / W;                 // stores per column per thread
  constexpr int TILE = BLOCK * RPT;
  const int n = D.n;
  const Ws w = ws_view(D.ws, n);
  double dr[RPT], num[RPT];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
#pragma unroll
    for (int e = 0; e < W; ++e) {
      const int r = rt * TILE + q * BLOCK * W + threadIdx.x * W + e;
      const bool body = (KIND == KIND_DPR1) ? (r < n) : (r < n - 1);
      dr[q * W + e] = body ? in_pole<KIND>(D, r) : 0.0;
      num[q * W + e] = body ? ((KIND == KIND_SVD) ? dr[q * W + e] * D.z[r] : D.z[r]) : 0.0;
    }
  }
  const int c0 = ct * cols;
  const int nc = min(n - c0, cols);
  const int nd = (KIND == KIND_ARROW) ? deflated_count(w) : 0;
  if constexpr (STAGE) stage_cols<KIND>(D, w, c0, nc, nd, L);
  for (int c = 0; c < nc; ++c) {
    const int col = c0 + c;
    double* vc = D.V + (size_t)col * (size_t)D.ldv;
    if (KIND == KIND_ARROW && nd > 0) {
      const int it = STAGE ? L.cm[c] : w.cm[col];
      if (it >= 0 && it < nd) {   // a deflated eigenvector (the whole block takes this branch)
        auto entry = [&](int r, double zr) { return r < n - 1 ? deflated_entry(w, it, w.iperm[r], zr) : 0.0; };
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          const int r = rt * TILE + q * BLOCK * W + threadIdx.x * W;
          if (r < n) {
            if constexpr (W == 1) {
              __builtin_nontemporal_store(entry(r, num[q]), vc + r);
            } else {
              const v2d vv = {entry(r, num[2 * q]), entry(r + 1, num[2 * q + 1])};
              __builtin_nontemporal_store(vv, (v2d*)(vc + r));
            }
          }
        }
        continue;
      }
    }
    const double pv = STAGE ? L.pv[c] : w.pv[col], s = STAGE ? L.sf[c] : w.sf[col];
    const double mu = STAGE ? L.mu[c] : w.mu[col], inrm = STAGE ? L.inrm[c] : w.inrm[col];
    double* uc = (KIND == KIND_SVD && D.U) ? D.U + (size_t)col * (size_t)D.ldu : nullptr;
    const double sigma = (KIND == KIND_SVD) ? (STAGE ? L.sig[c] : D.lam[col]) : 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int r = rt * TILE + q * BLOCK * W + threadIdx.x * W;
      if (r < n) {   // W = 2: n is even, so r + 1 < n as well
        if constexpr (W == 1) {
          const double v = vec_entry<KIND>(dr[q], num[q], r == n - 1, pv, s, mu, inrm);
          __builtin_nontemporal_store(v, vc + r);
          if (KIND == KIND_SVD && uc) __builtin_nontemporal_store(svd_left(D, sigma, v, r), uc + r);
        } else {
          const double v0 = vec_entry<KIND>(dr[2 * q], num[2 * q], false, pv, s, mu, inrm);
          const double v1 = vec_entry<KIND>(dr[2 * q + 1], num[2 * q + 1], r + 1 == n - 1, pv, s, mu, inrm);
          const v2d vv = {v0, v1};
          __builtin_nontemporal_store(vv, (v2d*)(vc + r));
          if (KIND == KIND_SVD && uc) {
            const v2d uu = {svd_left(D, sigma, v0, r), svd_left(D, sigma, v1, r + 1)};
            __builtin_nontemporal_store(uu, (v2d*)(uc + r));
          }
        }
      }
    }
  }
}

// Complex eigenvector entries of a Hermitian arrowhead (vec_entry_c), one
// 16-byte (re, im) store each; rows and columns are tiled as in vec_tile.
template <int RPT, class S>
__device__ inline void vec_tile_c(const ProbDesc& D, int rt, int ct, int cols, S& L) {
  constexpr int TILE = BLOCK * RPT;
  const int n = D.n;
  const Ws w = ws_view(D.ws, n);
  double dr[RPT], zr[RPT], zi[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = rt * TILE + q * BLOCK + threadIdx.x;
    const bool body = r < n - 1;
    dr[q] = body ? D.d[r] : 0.0;
    zr[q] = body ? D.z[2 * r] : 0.0;
    zi[q] = body ? D.z[2 * r + 1] : 0.0;
  }
  const int c0 = ct * cols;
  const int nc = min(n - c0, cols);
  stage_cols<KIND_HERM>(D, w, c0, nc, 0, L);
  for (int c = 0; c < nc; ++c) {
    const double pv = L.pv[c], s = L.sf[c], mu = L.mu[c], inrm = L.inrm[c];
    v2d* uc = (v2d*)D.V + (size_t)(c0 + c) * (size_t)D.ldv;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = rt * TILE + q * BLOCK + threadIdx.x;
      if (r < n) {
        double ur, ui;
        vec_entry_c(dr[q], zr[q], zi[q], r == n - 1, pv, s, mu, inrm, &ur, &ui);
        const v2d u = {ur, ui};
        __builtin_nontemporal_store(u, uc + r);
      }
    }
  }
}

// vec_flat, for small n (a row tile would leave most threads idle): tile t is
// the columns [t*C, (t+1)*C) of the n x n block (ld = n), C = vec_flat_cols(n),
// whose entries are contiguous.  The problem's rows and the tile's columns are
// staged in LDS; BLOCK consecutive entries are written per step, and a thread
// finds its (row, column) once and then steps it without dividing.
#ifndef AHD_VEC_FLAT_ENTRIES
#define AHD_VEC_FLAT_ENTRIES 4096
#endif
constexpr int VEC_FLAT_ENTRIES = AHD_VEC_FLAT_ENTRIES;   // entries a flat tile aims at

__host__ __device__ inline int vec_flat_cols(int64_t n) {
  const int64_t c = VEC_FLAT_ENTRIES / n;
  return (int)(c < 1 ? 1 : (c > VEC_FLAT_COLS ? VEC_FLAT_COLS : c));
}

template <int KIND, class S>
__device__ inline void vec_flat(const ProbDesc& D, int t, S& L) {
  const int n = D.n;   // below VEC_FLAT_ROWS
  const Ws w = ws_view(D.ws, n);
  const int C = vec_flat_cols(n);
  const int c0 = t * C;
  const int nc = min(C, n - c0);
  const int nd = (KIND == KIND_ARROW) ? deflated_count(w) : 0;
  for (int r = threadIdx.x; r < n; r += BLOCK) {
    const bool body = (KIND == KIND_DPR1) ? true : (r < n - 1);
    const double d = body ? in_pole<KIND>(D, r) : 0.0;
    L.dr[r] = d;
    L.num[r] = body ? ((KIND == KIND_SVD) ? d * D.z[r] : D.z[r]) : 0.0;
  }
  stage_cols<KIND>(D, w, c0, nc, nd, L);
  const int ne = nc * n;
  double* out = D.V + (size_t)c0 * (size_t)n;
  double* uout = (KIND == KIND_SVD && D.U) ? D.U + (size_t)c0 * (size_t)n : nullptr;
  int e = threadIdx.x;
  int c = e / n;
  int row = e - c * n;
  const int q = BLOCK / n, rem = BLOCK - q * n;
  for (; e < ne; e += BLOCK) {
    const int it = (KIND == KIND_ARROW && nd > 0) ? L.cm[c] : -1;
    const double v = (it >= 0 && it < nd)
        ? (row < n - 1 ? deflated_entry(w, it, w.iperm[row], L.num[row]) : 0.0)
        : vec_entry<KIND>(L.dr[row], L.num[row], row == n - 1, L.pv[c], L.sf[c], L.mu[c], L.inrm[c]);
    __builtin_nontemporal_store(v, out + e);
    if (KIND == KIND_SVD && uout) __builtin_nontemporal_store(svd_left(D, L.sig[c], v, row), uout + e);
    row += rem;
    c += q;
    if (row >= n) {
      row -= n;
      ++c;
    }
  }
}

// The deflated eigenpairs are placed among the solved ones once every block
// of the launch that finishes the solved eigenvalues is done: each block
// counts itself in the workspace, and the last to arrive places them.  Every
// one of the `blocks` blocks must call this.
__device__ inline void place_deflated_last(const ProbDesc& D, const Ws& w, uint32_t blocks) {
  __shared__ int last;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // this thread's results, device-wide
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(place_done(w), 1u) == blocks - 1;
  __syncthreads();
  if (!last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // every block's results, in the last block
  const int nd = deflated_count(w);
  for (int s = threadIdx.x; s < nd; s += blockDim.x) place_deflated(D, w, s);
}

}  // namespace ahd
