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
  int big;           // its product goes to rocBLAS (else to k_td_update)
  int64_t out;       // offset of the merge's eigenvalues in the output pool; Qh follows (s x nk, ld s)
  int64_t dout;      // offset of the DPR1 solve's eigenvalues in its pool; its vectors follow (ld nk)
  int64_t cout;      // big merges: offset of diag(Q1, Q2) Qh (s x nk, ld s) in the scratch pool
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

// One merge's eigenvalues, the column each eigenpair goes to, and Qh over
// the solved ones.  The DPR1 solve had the kept entries (map[lo .. lo+nk):
// their rows, ascending); the deflated ones (map[lo+nk .. hi): their rows, by
// decreasing eigenvalue) keep (d_f, e_f).  Both lists descend and are merged
// with a solved eigenvalue first on ties; pos[lo + j] is the column of source
// j (the same numbering as map).  Qh (s x nk, ld s) holds the solved vectors
// on the kept rows and zeros elsewhere.  info: the solve's bits, or
// ARROW_INFO_DEFLATED.
__global__ __launch_bounds__(TD_BLOCK) void k_td_expand(const MergeDev* mg, const int* map, const double* lam,
                                                        const double* dpool, const uint32_t* dinfo, double* out,
                                                        uint32_t* info, int* pos) {
  const MergeDev m = mg[blockIdx.y];
  const int s = m.hi - m.lo, nk = m.nk, nf = s - nk;
  const int* kept = map + m.lo;
  const int* defl = kept + nk;
  const double* dl = dpool + m.dout;       // solved eigenvalues, descending
  const double* dq = dl + nk;              // their vectors over the kept rows (ld nk)
  double* lo_out = out + m.out;
  double* qh = lo_out + s;
  for (int c = (int)(blockIdx.x * TD_BLOCK + threadIdx.x); c < s; c += (int)gridDim.x * TD_BLOCK) {
    if (c < nk) {
      const double v = dl[c];
      int lo = 0, hi = nf;                 // deflated values > v
      while (lo < hi) { const int md = (lo + hi) >> 1; if (lam[m.lo + defl[md]] > v) lo = md + 1; else hi = md; }
      lo_out[c + lo] = v;
      pos[m.lo + c] = c + lo;
      info[m.lo + c + lo] = dinfo[m.lo + c];
      double* col = qh + (size_t)c * s;
      for (int r = 0; r < s; ++r) col[r] = 0.0;
      for (int r = 0; r < nk; ++r) col[kept[r]] = dq[(size_t)c * nk + r];
    } else {
      const int f = c - nk;
      const double v = lam[m.lo + defl[f]];
      int lo = 0, hi = nk;                 // solved values >= v
      while (lo < hi) { const int md = (lo + hi) >> 1; if (dl[md] >= v) lo = md + 1; else hi = md; }
      lo_out[f + lo] = v;
      pos[m.lo + c] = f + lo;
      info[m.lo + f + lo] = ARROW_INFO_DEFLATED;
    }
  }
}

// The merged block's columns in the output buffer: a deflated pair's vector
// is column f of diag(Q1, Q2); a solved one is diag(Q1, Q2) times its Qh
// column, summed here over the kept rows (small merges) or scattered from the
// rocBLAS product (k_td_scatter, big merges).
__global__ __launch_bounds__(TD_BLOCK) void k_td_update(const MergeDev* mg, const int* map, const int* pos,
                                                        const double* out, int n, const double* Qold, double* Qnew) {
  const MergeDev m = mg[blockIdx.y];
  const int s = m.hi - m.lo, sl = m.mid - m.lo, nk = m.nk;
  const int* kept = map + m.lo;
  const double* qh = out + m.out + s;
  for (int64_t e = (int64_t)blockIdx.x * TD_BLOCK + threadIdx.x; e < (int64_t)s * s; e += (int64_t)gridDim.x * TD_BLOCK) {
    const int j = (int)(e / s), i = (int)(e - (int64_t)j * s);   // source j, row i
    if (j < nk && m.big) continue;
    double v = 0.0;
    if (j < nk) {
      const bool top = i < sl;
      for (int r = 0; r < nk; ++r) {
        const int kr = kept[r];
        if ((kr < sl) == top) v = fma(Qold[(size_t)(m.lo + kr) * n + (m.lo + i)], qh[(size_t)j * s + kr], v);
      }
    } else {
      const int d = kept[j];                                    // deflated row (map continues past nk)
      if ((i < sl) == (d < sl)) v = Qold[(size_t)(m.lo + d) * n + (m.lo + i)];
    }
    Qnew[(size_t)(m.lo + pos[m.lo + j]) * n + (m.lo + i)] = v;
  }
}

__global__ __launch_bounds__(TD_BLOCK) void k_td_scatter(const MergeDev* mg, const int* pos, const double* C, int n,
                                                         double* Qnew) {
  const MergeDev m = mg[blockIdx.y];
  if (!m.big) return;
  const int s = m.hi - m.lo, nk = m.nk;
  for (int64_t e = (int64_t)blockIdx.x * TD_BLOCK + threadIdx.x; e < (int64_t)s * nk; e += (int64_t)gridDim.x * TD_BLOCK) {
    const int c = (int)(e / s), i = (int)(e - (int64_t)c * s);
    Qnew[(size_t)(m.lo + pos[m.lo + c]) * n + (m.lo + i)] = C[m.cout + e];
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
  if (h->td_ws) {
    (void)hipFree(h->td_ws);
    h->td_ws = nullptr;
    h->td_cap = 0;
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
  // buffers, the merges' output pool, the DPR1 solves' pool (then the GEMM
  // scratch), info words, the row and column maps and the merge records
  const size_t nn = (size_t)n * (size_t)n;
  // one buffer, kept in the handle, holds them all (256-byte aligned parts)
  struct Part {
    void** p;
    size_t bytes;
  };
  void *p_lamu, *p_cpool, *p_qbuf, *p_outp, *p_dpool, *p_infop, *p_infod, *p_map, *p_pos, *p_recs;
  const Part parts[] = {{&p_lamu, 2 * (size_t)n * sizeof(double)},  {&p_cpool, 2 * (size_t)n * sizeof(double)},
                        {&p_qbuf, 2 * nn * sizeof(double)},          {&p_outp, ((size_t)n + nn) * sizeof(double)},
                        {&p_dpool, ((size_t)n + nn) * sizeof(double)}, {&p_infop, (size_t)n * sizeof(uint32_t)},
                        {&p_infod, (size_t)n * sizeof(uint32_t)},    {&p_map, (size_t)n * sizeof(int)},
                        {&p_pos, (size_t)n * sizeof(int)},           {&p_recs, (size_t)n * sizeof(MergeDev) + 16}};
  size_t total = 0;
  for (const Part& q : parts) total += (q.bytes + 255) / 256 * 256;
  if (total > h->td_cap) {
    if (h->td_ws) (void)hipFree(h->td_ws);
    h->td_ws = nullptr;
    h->td_cap = 0;
    if (hipMalloc(&h->td_ws, total) != hipSuccess) {
      h->td_ws = nullptr;
      return ARROW_ERR_NOMEM;
    }
    h->td_cap = total;
  }
  {
    char* at = (char*)h->td_ws;
    for (const Part& q : parts) {
      *q.p = at;
      at += (q.bytes + 255) / 256 * 256;
    }
  }
  struct View {
    void* p;
  } lamu{p_lamu}, cpool{p_cpool}, qbuf{p_qbuf}, outp{p_outp}, dpool{p_dpool}, infop{p_infop}, infod{p_infod},
      mapb{p_map}, posb{p_pos}, recs{p_recs};
  DevBuf bws;
  size_t bws_bytes = 0;
  int rc;
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
      // recs is written again below, after this kernel in stream order; the host's copy
      // list is refilled only after the next synchronisation
      hipLaunchKernelGGL(k_td_copy, dim3(64, (unsigned)copies.size()), dim3(TD_BLOCK), 0, st, dsp, (int)n,
                         qb[in ^ 1], qb[in]);
    }
    // the merges of this level; u of every one, then eigenvalues and u to the host
    all.clear();
    for (const Node& p : nodes)
      if (p.height == lev && p.left >= 0) all.push_back(MergeDev{p.lo, p.mid, p.hi, 0, 0, 0, 0, 0});
    MergeDev* drec = (MergeDev*)recs.p;
    int64_t widest = 1;   // the largest merge of the level sizes the grids (they stride over the rest)
    for (const MergeDev& m : all) widest = std::max<int64_t>(widest, m.hi - m.lo);
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
    int64_t off = 0, doff = 0, coff = 0;
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
      // products of more than 2^22 multiply-adds go to rocBLAS
      m.big = (int64_t)s * nk * (s / 2) > ((int64_t)1 << 22);
      m.cout = coff;
      if (m.big) coff += (int64_t)s * nk;
      off += (int64_t)s + (int64_t)s * nk;
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
      // the plan's device block comes from one buffer, grown when a level needs more
      const size_t need = arrow_batch_workspace_size((int64_t)descs.size(), descs.data());
      if (need > bws_bytes) {
        (void)hipStreamSynchronize(st);
        if (bws.p) (void)hipFree(bws.p);
        bws.p = nullptr;
        bws_bytes = 0;
        if ((rc = bws.alloc(need))) return rc;
        bws_bytes = need;
      }
      arrow_batch_t plan = nullptr;
      rc = arrow_batch_create(h, (int64_t)descs.size(), descs.data(), (double*)cpool.p, (double*)dpool.p,
                              (uint32_t*)infod.p, bws.p, bws_bytes, 0, &plan);
      if (rc != ARROW_OK) return rc > 0 ? rc : ARROW_ERR_STATE;
      rc = arrow_batch_run(plan);
      const int rc2 = arrow_batch_destroy(plan);   // synchronises the stream: the host arrays may be reused
      if (rc != ARROW_OK) return rc;
      if (rc2 != ARROW_OK) return rc2;
    }
    hipLaunchKernelGGL(k_td_expand, dim3(grid_x(widest), (unsigned)all.size()), dim3(TD_BLOCK), 0, st, drec,
                       (const int*)mapb.p, lam, (const double*)dpool.p, (const uint32_t*)infod.p, (double*)outp.p,
                       (uint32_t*)infop.p, (int*)posb.p);
    hipLaunchKernelGGL(k_td_put_lam, dim3(grid_x(widest), (unsigned)all.size()), dim3(TD_BLOCK), 0, st, drec,
                       (const double*)outp.p, lam);
    // big merges: diag(Q1, Q2) Qh by rocBLAS into the scratch pool (the DPR1
    // pool, read by k_td_expand before), Q1 against Qh's top rows, Q2 against
    // its bottom rows
    const double one = 1.0, zero = 0.0;
    double* scratch = (double*)dpool.p;
    for (const MergeDev& m : all) {
      if (!m.big) continue;
      const int s = m.hi - m.lo, sl = m.mid - m.lo, sr = m.hi - m.mid;
      const double* qh = (const double*)outp.p + m.out + s;
      if (rocblas_dgemm(bh, rocblas_operation_none, rocblas_operation_none, sl, m.nk, sl, &one,
                        qb[in] + (size_t)m.lo * n + m.lo, (int)n, qh, s, &zero, scratch + m.cout, s) !=
              rocblas_status_success ||
          rocblas_dgemm(bh, rocblas_operation_none, rocblas_operation_none, sr, m.nk, sr, &one,
                        qb[in] + (size_t)m.mid * n + m.mid, (int)n, qh + sl, s, &zero, scratch + m.cout + sl, s) !=
              rocblas_status_success)
        return ARROW_ERR_HIP;
    }
    hipLaunchKernelGGL(k_td_update, dim3(grid_x(widest * widest), (unsigned)all.size()), dim3(TD_BLOCK), 0, st, drec,
                       (const int*)mapb.p, (const int*)posb.p, (const double*)outp.p, (int)n, (const double*)qb[in],
                       qb[outb]);
    hipLaunchKernelGGL(k_td_scatter, dim3(grid_x(widest * widest), (unsigned)all.size()), dim3(TD_BLOCK), 0, st, drec,
                       (const int*)posb.p, (const double*)scratch, (int)n, qb[outb]);
    // the host arrays copied to the device above are refilled next level: the plan's
    // destruction synchronised the stream after those copies; without a plan, wait here
    if (descs.empty() && hipStreamSynchronize(st) != hipSuccess) return ARROW_ERR_HIP;
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
  if (hipStreamSynchronize(st) != hipSuccess) return ARROW_ERR_HIP;   // results complete; the buffers are reused
  return hipGetLastError() == hipSuccess ? ARROW_OK : ARROW_ERR_HIP;
}

}  // extern "C"
