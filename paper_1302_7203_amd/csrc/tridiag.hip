// Symmetric tridiagonal eigen-decomposition by divide and conquer, each merge
// a DPR1 eigenproblem solved by the accurate arrowhead method (Sec. 1 names
// the arrowhead / DPR1 eigenproblem as the merge step of such solvers; Sec. 6.3
// and the closing remark of Sec. 6 for DPR1 matrices of either sign of rho).
//
// T = tridiag(b, a, b) of order n is torn at every off-diagonal: with the
// split between rows m-1 and m and beta = b[m-1],
//     T = diag(T1', T2') + beta v v^T,   v = e_{m-1} + e_m,
// where T1', T2' are T's diagonal blocks with beta taken off their corner
// entries.  Recursing to 1x1 leaves, leaf i is a_i - b_{i-1} - b_i.  With
// T1' = Q1 L1 Q1^T and T2' = Q2 L2 Q2^T,
//     T = diag(Q1, Q2) (diag(L1, L2) + beta u u^T) diag(Q1, Q2)^T,
//     u = [last row of Q1; first row of Q2],
// so a merge is the DPR1 eigenproblem diag(L1, L2) + beta u u^T = Qh L Qh^T
// (dpr1_eig's kernels, every merge of a tree level in one batched plan) and
// Q = diag(Q1, Q2) Qh, two plain FP64 GEMMs per merge (rocBLAS).  beta = 0
// splits T: that merge is a merge of two sorted lists and Qh a permutation.
//
// Storage: the eigenvalues of every current block sit at its rows of one
// n-vector; its eigenvectors are its diagonal block of one of two n x n
// buffers (ld n).  A node of height h keeps its block in buffer h % 2; its
// parent (height h+1) reads buffer h % 2 and writes the other.  A node whose
// sibling is taller (height h-1 under a parent of height h+1) is copied to the
// other buffer first, so that a merge never writes the block it reads.

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/arrow.h"
#include "host.hpp"

namespace {

constexpr int TD_BLOCK = 256;

struct Node {
  int lo, mid, hi;   // rows [lo, hi); children [lo, mid) and [mid, hi) (leaf: mid = -1)
  int left, right;   // child indices, -1 for a leaf
  int height;
  double beta;       // b[mid-1]
};

struct MergeDev {
  int lo, mid, hi;
  int nk;            // entries kept for the DPR1 solve (the others are deflated)
  int64_t out;       // offset of the merge's eigenvalues in the output pool; Qh follows (ld hi-lo)
  int64_t dout;      // offset of the DPR1 solve's eigenvalues in its pool; its vectors follow (ld nk)
};

int build(std::vector<Node>& nodes, const std::vector<double>& b, int lo, int hi) {
  Node nd{};
  nd.lo = lo;
  nd.hi = hi;
  if (hi - lo == 1) {
    nd.mid = -1;
    nd.left = nd.right = -1;
    nd.height = 0;
    nd.beta = 0.0;
    nodes.push_back(nd);
    return (int)nodes.size() - 1;
  }
  const int mid = lo + (hi - lo) / 2;
  const int l = build(nodes, b, lo, mid);
  const int r = build(nodes, b, mid, hi);
  nd.mid = mid;
  nd.left = l;
  nd.right = r;
  nd.height = 1 + std::max(nodes[l].height, nodes[r].height);
  nd.beta = b[mid - 1];
  nodes.push_back(nd);
  return (int)nodes.size() - 1;
}

// leaves: lam_i = a_i - b_{i-1} - b_i, Q = [1] at (i, i) of buffer 0
__global__ __launch_bounds__(TD_BLOCK) void k_td_leaf(const double* a, const double* b, int n, double* lam,
                                                      double* Q) {
  const int i = blockIdx.x * TD_BLOCK + threadIdx.x;
  if (i >= n) return;
  lam[i] = (a[i] - (i > 0 ? b[i - 1] : 0.0)) - (i + 1 < n ? b[i] : 0.0);
  Q[(size_t)i * n + i] = 1.0;
}

// copy the diagonal block [lo, hi) of src into dst (block y = one node)
__global__ __launch_bounds__(TD_BLOCK) void k_td_copy(const int2* spans, int n, const double* src, double* dst) {
  const int2 s = spans[blockIdx.y];
  const int w = s.y - s.x;
  for (int64_t e = (int64_t)blockIdx.x * TD_BLOCK + threadIdx.x; e < (int64_t)w * w; e += (int64_t)gridDim.x * TD_BLOCK) {
    const int c = (int)(e / w), r = (int)(e - (int64_t)c * w);
    const size_t at = (size_t)(s.x + c) * n + (s.x + r);
    dst[at] = src[at];
  }
}

// u of each merge: the last row of the left block and the first row of the right one
__global__ __launch_bounds__(TD_BLOCK) void k_td_gather_u(const MergeDev* mg, int n, const double* Q, double* u) {
  const MergeDev m = mg[blockIdx.y];
  for (int j = m.lo + (int)(blockIdx.x * TD_BLOCK + threadIdx.x); j < m.hi; j += (int)gridDim.x * TD_BLOCK) {
    const int row = j < m.mid ? m.mid - 1 : m.mid;
    u[j] = Q[(size_t)j * n + row];
  }
}

// One merge's eigenvalues and Qh from the DPR1 solve of its kept entries
// (map[lo .. lo+nk): their rows, in the order given to the solve) and its
// deflated entries (map[lo+nk .. hi): their rows, by decreasing eigenvalue;
// eigenpair (d_f, e_f)).  Both lists descend; they are merged with a solved
// eigenvalue first on ties.  info: the solve's bits, or ARROW_INFO_DEFLATED.
__global__ __launch_bounds__(TD_BLOCK) void k_td_expand(const MergeDev* mg, const int* map, const double* lam,
                                                        const double* dpool, const uint32_t* dinfo, double* out,
                                                        uint32_t* info) {
  const MergeDev m = mg[blockIdx.y];
  const int s = m.hi - m.lo, nk = m.nk, nf = s - nk;
  const int* kept = map + m.lo;
  const int* defl = kept + nk;
  const double* dl = dpool + m.dout;       // solved eigenvalues, descending
  const double* dq = dl + nk;              // their vectors over the kept rows (ld nk)
  double* lo_out = out + m.out;
  double* qh = lo_out + s;
  for (int c = (int)(blockIdx.x * TD_BLOCK + threadIdx.x); c < s; c += (int)gridDim.x * TD_BLOCK) {
    int pos;
    if (c < nk) {
      const double v = dl[c];
      int lo = 0, hi = nf;                 // deflated values > v
      while (lo < hi) { const int md = (lo + hi) >> 1; if (lam[m.lo + defl[md]] > v) lo = md + 1; else hi = md; }
      pos = c + lo;
      lo_out[pos] = v;
      double* col = qh + (size_t)pos * s;
      for (int r = 0; r < s; ++r) col[r] = 0.0;
      for (int r = 0; r < nk; ++r) col[kept[r]] = dq[(size_t)c * nk + r];
      info[m.lo + pos] = dinfo[m.lo + c];
    } else {
      const int f = c - nk;
      const double v = lam[m.lo + defl[f]];
      int lo = 0, hi = nk;                 // solved values >= v
      while (lo < hi) { const int md = (lo + hi) >> 1; if (dl[md] >= v) lo = md + 1; else hi = md; }
      pos = f + lo;
      lo_out[pos] = v;
      double* col = qh + (size_t)pos * s;
      for (int r = 0; r < s; ++r) col[r] = (r == defl[f]) ? 1.0 : 0.0;
      info[m.lo + pos] = ARROW_INFO_DEFLATED;
    }
  }
}

// merged eigenvalues back to the block's rows
__global__ __launch_bounds__(TD_BLOCK) void k_td_put_lam(const MergeDev* mg, const double* out, double* lam) {
  const MergeDev m = mg[blockIdx.y];
  for (int j = m.lo + (int)(blockIdx.x * TD_BLOCK + threadIdx.x); j < m.hi; j += (int)gridDim.x * TD_BLOCK)
    lam[j] = out[m.out + (j - m.lo)];
}

unsigned grid_x(int64_t items) {
  const int64_t g = (items + TD_BLOCK - 1) / TD_BLOCK;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 64));
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  int alloc(size_t bytes) {
    return hipMalloc(&p, bytes) == hipSuccess ? ARROW_OK : ARROW_ERR_NOMEM;
  }
};

}  // namespace

void tridiag_release(arrow_handle_t h) {
  if (h->blas) {
    (void)rocblas_destroy_handle((rocblas_handle)h->blas);
    h->blas = nullptr;
  }
}

extern "C" {

int tridiag_eig(arrow_handle_t h, int64_t n, const double* a, const double* b, double* lambda, double* Q,
                int64_t ldq, uint32_t* info) {
  if (!valid(h)) return -1;
  if (n < 1 || n > 46340) return -2;
  if (!a) return -3;
  if (n > 1 && !b) return -4;
  if (!lambda) return -5;
  if (!Q) return -6;
  if (ldq < n) return -7;
  DeviceGuard g(h->device);
  hipStream_t st = h->stream;
  (void)hipGetLastError();
  std::vector<double> hb((size_t)std::max<int64_t>(1, n - 1), 0.0);
  if (n > 1) {
    if (hipMemcpyAsync(hb.data(), b, (size_t)(n - 1) * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return ARROW_ERR_HIP;
    for (int64_t i = 0; i + 1 < n; ++i)
      if (!(hb[(size_t)i] - hb[(size_t)i] == 0.0)) return -4;   // the tree needs finite off-diagonals
  }
  std::vector<Node> nodes;
  nodes.reserve((size_t)(2 * n));
  const int root = build(nodes, hb, 0, (int)n);
  const int H = nodes[(size_t)root].height;

  // device memory: eigenvalues and u, the compacted DPR1 inputs, two Q
  // buffers, the merges' output pool, the DPR1 solves' pool, info words, the
  // row maps, merge records and GEMM pointer arrays
  const size_t nn = (size_t)n * (size_t)n;
  DevBuf lamu, cpool, qbuf, outp, dpool, infop, infod, mapb, recs, ptrs;
  int rc;
  if ((rc = lamu.alloc(2 * (size_t)n * sizeof(double))) || (rc = cpool.alloc(2 * (size_t)n * sizeof(double))) ||
      (rc = qbuf.alloc(2 * nn * sizeof(double))) || (rc = outp.alloc(((size_t)n + nn) * sizeof(double))) ||
      (rc = dpool.alloc(((size_t)n + nn) * sizeof(double))) || (rc = infop.alloc((size_t)n * sizeof(uint32_t))) ||
      (rc = infod.alloc((size_t)n * sizeof(uint32_t))) || (rc = mapb.alloc((size_t)n * sizeof(int))) ||
      (rc = recs.alloc((size_t)n * sizeof(MergeDev) + 16)) || (rc = ptrs.alloc(6 * (size_t)n * sizeof(double*) + 16)))
    return rc;
  double* lam = (double*)lamu.p;
  double* u = lam + n;
  double* qb[2] = {(double*)qbuf.p, (double*)qbuf.p + nn};
  hipLaunchKernelGGL(k_td_leaf, dim3((unsigned)((n + TD_BLOCK - 1) / TD_BLOCK)), dim3(TD_BLOCK), 0, st, a, b, (int)n,
                     lam, qb[0]);
  if (!h->blas) {
    rocblas_handle bh;
    if (rocblas_create_handle(&bh) != rocblas_status_success) return ARROW_ERR_HIP;
    h->blas = bh;
  }
  rocblas_handle bh = (rocblas_handle)h->blas;
  if (rocblas_set_stream(bh, st) != rocblas_status_success) return ARROW_ERR_HIP;
  (void)rocblas_set_pointer_mode(bh, rocblas_pointer_mode_host);

  const double eps = 0x1p-53;
  std::vector<MergeDev> all;
  std::vector<int2> copies;
  std::vector<arrow_desc_t> descs;
  std::vector<double> hl((size_t)2 * n), hc((size_t)2 * n, 0.0);
  std::vector<int> hmap((size_t)n), idx;
  for (int lev = 1; lev <= H; ++lev) {
    const int in = (lev - 1) & 1, outb = lev & 1;
    // nodes of height lev-2 under a parent of height lev: to the input buffer first
    copies.clear();
    for (const Node& p : nodes) {
      if (p.height != lev || p.left < 0) continue;
      for (int c : {p.left, p.right})
        if (nodes[(size_t)c].height == lev - 2) copies.push_back(make_int2(nodes[(size_t)c].lo, nodes[(size_t)c].hi));
    }
    if (!copies.empty()) {
      int2* dsp = (int2*)recs.p;
      if (hipMemcpyAsync(dsp, copies.data(), copies.size() * sizeof(int2), hipMemcpyHostToDevice, st) != hipSuccess)
        return ARROW_ERR_HIP;
      hipLaunchKernelGGL(k_td_copy, dim3(64, (unsigned)copies.size()), dim3(TD_BLOCK), 0, st, dsp, (int)n,
                         qb[in ^ 1], qb[in]);
      if (hipStreamSynchronize(st) != hipSuccess) return ARROW_ERR_HIP;   // recs is reused below
    }
    // the merges of this level; u of every one, then eigenvalues and u to the host
    all.clear();
    for (const Node& p : nodes)
      if (p.height == lev && p.left >= 0) all.push_back(MergeDev{p.lo, p.mid, p.hi, 0, 0, 0});
    MergeDev* drec = (MergeDev*)recs.p;
    const int64_t widest = (int64_t)n;   // grid-stride loops cover any block
    if (hipMemcpyAsync(drec, all.data(), all.size() * sizeof(MergeDev), hipMemcpyHostToDevice, st) != hipSuccess)
      return ARROW_ERR_HIP;
    hipLaunchKernelGGL(k_td_gather_u, dim3(grid_x(widest), (unsigned)all.size()), dim3(TD_BLOCK), 0, st, drec, (int)n,
                       qb[in], u);
    if (hipMemcpyAsync(hl.data(), lam, 2 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return ARROW_ERR_HIP;
    // Deflation (the usual one of divide and conquer): entry j is dropped when
    // sqrt2 |beta| |u_j| <= 8 eps max(|d|_max, |u|_max / sqrt2) -- u has norm
    // sqrt2 -- a perturbation of T of that size; it leaves (d_j, e_j).  The
    // rest is solved as a DPR1 problem; beta = 0 drops every entry.
    descs.clear();
    int64_t off = 0, doff = 0;
    size_t mi = 0;
    for (const Node& p : nodes) {
      if (p.height != lev || p.left < 0) continue;
      MergeDev& m = all[mi++];
      const int s = p.hi - p.lo;
      double dmax = 0.0, umax = 0.0;
      for (int t = p.lo; t < p.hi; ++t) {
        dmax = std::max(dmax, fabs(hl[(size_t)t]));
        umax = std::max(umax, fabs(hl[(size_t)n + t]));
      }
      const double tol = 8.0 * eps * std::max(dmax, umax * 0.7071067811865476);
      int nk = 0;
      idx.clear();
      for (int t = 0; t < s; ++t) {
        const double ut = hl[(size_t)n + p.lo + t];
        if (p.beta != 0.0 && 1.4142135623730951 * fabs(p.beta) * fabs(ut) > tol) {
          hmap[(size_t)p.lo + nk] = t;
          hc[(size_t)p.lo + nk] = hl[(size_t)p.lo + t];
          hc[(size_t)n + p.lo + nk] = ut;
          ++nk;
        } else {
          idx.push_back(t);
        }
      }
      std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return hl[(size_t)p.lo + x] > hl[(size_t)p.lo + y]; });
      for (size_t f = 0; f < idx.size(); ++f) hmap[(size_t)p.lo + nk + f] = idx[f];
      m.nk = nk;
      m.out = off;
      m.dout = doff;
      off += (int64_t)s + (int64_t)s * s;
      if (nk > 0) {
        arrow_desc_t d{};
        d.kind = ARROW_KIND_DPR1;
        d.n = nk;
        d.d_off = p.lo;
        d.z_off = n + p.lo;
        d.scalar = p.beta;
        d.lam_off = doff;
        d.vec_off = doff + nk;
        d.left_off = -1;
        d.info_off = p.lo;
        descs.push_back(d);
        doff += (int64_t)nk + (int64_t)nk * nk;
      }
    }
    if (hipMemcpyAsync(drec, all.data(), all.size() * sizeof(MergeDev), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(mapb.p, hmap.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(cpool.p, hc.data(), 2 * (size_t)n * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess)
      return ARROW_ERR_HIP;
    if (!descs.empty()) {
      arrow_batch_t plan = nullptr;
      rc = arrow_batch_create(h, (int64_t)descs.size(), descs.data(), (double*)cpool.p, (double*)dpool.p,
                              (uint32_t*)infod.p, nullptr, 0, 0, &plan);
      if (rc != ARROW_OK) return rc > 0 ? rc : ARROW_ERR_STATE;
      rc = arrow_batch_run(plan);
      const int rc2 = arrow_batch_destroy(plan);   // synchronises the stream: the host arrays may be reused
      if (rc != ARROW_OK) return rc;
      if (rc2 != ARROW_OK) return rc2;
    }
    hipLaunchKernelGGL(k_td_expand, dim3(grid_x(widest), (unsigned)all.size()), dim3(TD_BLOCK), 0, st, drec,
                       (const int*)mapb.p, lam, (const double*)dpool.p, (const uint32_t*)infod.p, (double*)outp.p,
                       (uint32_t*)infop.p);
    hipLaunchKernelGGL(k_td_put_lam, dim3(grid_x(widest), (unsigned)all.size()), dim3(TD_BLOCK), 0, st, drec,
                       (const double*)outp.p, lam);
    // Q of each merge = diag(Q1, Q2) Qh: the top rows from Q1, the bottom rows
    // from Q2; merges of equal shape go to one batched call
    std::vector<const MergeDev*> order;
    for (const MergeDev& m : all) order.push_back(&m);
    std::sort(order.begin(), order.end(), [](const MergeDev* x, const MergeDev* y) {
      const int ax = x->mid - x->lo, bx = x->hi - x->mid, ay = y->mid - y->lo, by = y->hi - y->mid;
      return ax != ay ? ax < ay : bx < by;
    });
    const double one = 1.0, zero = 0.0;
    double** dptr = (double**)ptrs.p;
    std::vector<double*> hp;
    for (size_t g0 = 0; g0 < order.size();) {
      size_t g1 = g0 + 1;
      const int sl = order[g0]->mid - order[g0]->lo, sr = order[g0]->hi - order[g0]->mid;
      while (g1 < order.size() && order[g1]->mid - order[g1]->lo == sl && order[g1]->hi - order[g1]->mid == sr) ++g1;
      const int cnt = (int)(g1 - g0), s = sl + sr;
      hp.assign((size_t)6 * cnt, nullptr);
      for (int q = 0; q < cnt; ++q) {
        const MergeDev& m = *order[g0 + q];
        double* qh = (double*)outp.p + m.out + s;
        hp[(size_t)q] = qb[in] + (size_t)m.lo * n + m.lo;                    // Q1
        hp[(size_t)cnt + q] = qh;                                            // Qh rows [0, sl)
        hp[(size_t)2 * cnt + q] = qb[outb] + (size_t)m.lo * n + m.lo;        // rows [lo, mid) of the result
        hp[(size_t)3 * cnt + q] = qb[in] + (size_t)m.mid * n + m.mid;        // Q2
        hp[(size_t)4 * cnt + q] = qh + sl;                                   // Qh rows [sl, s)
        hp[(size_t)5 * cnt + q] = qb[outb] + (size_t)m.lo * n + m.mid;       // rows [mid, hi)
      }
      if (hipMemcpyAsync(dptr, hp.data(), hp.size() * sizeof(double*), hipMemcpyHostToDevice, st) != hipSuccess)
        return ARROW_ERR_HIP;
      if (rocblas_dgemm_batched(bh, rocblas_operation_none, rocblas_operation_none, sl, s, sl, &one, dptr, (int)n,
                                dptr + cnt, s, &zero, dptr + 2 * cnt, (int)n, cnt) != rocblas_status_success ||
          rocblas_dgemm_batched(bh, rocblas_operation_none, rocblas_operation_none, sr, s, sr, &one, dptr + 3 * cnt,
                                (int)n, dptr + 4 * cnt, s, &zero, dptr + 5 * cnt, (int)n, cnt) != rocblas_status_success)
        return ARROW_ERR_HIP;
      if (hipStreamSynchronize(st) != hipSuccess) return ARROW_ERR_HIP;   // the pointer array is reused
      g0 = g1;
    }
  }
  // results: eigenvalues (descending) and the root's block
  const int fin = H & 1;
  if (hipMemcpyAsync(lambda, lam, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpy2DAsync(Q, (size_t)ldq * sizeof(double), qb[fin], (size_t)n * sizeof(double), (size_t)n * sizeof(double),
                       (size_t)n, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return ARROW_ERR_HIP;
  if (info) {
    if (H == 0) {
      if (hipMemsetAsync(info, 0, sizeof(uint32_t), st) != hipSuccess) return ARROW_ERR_HIP;
    } else if (hipMemcpyAsync(info, infop.p, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st) != hipSuccess) {
      return ARROW_ERR_HIP;
    }
  }
  if (hipStreamSynchronize(st) != hipSuccess) return ARROW_ERR_HIP;   // before the buffers are freed
  return hipGetLastError() == hipSuccess ? ARROW_OK : ARROW_ERR_HIP;
}

}  // extern "C"
