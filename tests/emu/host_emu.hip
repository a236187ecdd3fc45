// Host-only driver of the library's kernel bodies (test infrastructure).
//
// It runs the same __host__ __device__ per-eigenvalue bodies that the GPU
// kernels wrap, with one lane per eigenvalue (G = 1) and plain loops in place
// of the grid, so that the method itself can be checked against the oracle on
// a machine without a GPU.  The GPU path never uses this file.
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <vector>

#include "../../paper_1302_7203_amd/csrc/bodies.hpp"

using namespace ahd;

// 1: the batched plan's check stage -- Remark 2 and the DPR1 re-measure in the
// check itself, eigenvalues near the origin listed and repaired afterwards
static int g_batch_check = 0;

template <int KIND>
static void run(ProbDesc D, const Options& opt, double* U) {
  const int ms = sorted_count(D);
  Ws w = ws_view(D.ws, D.n);
  for (int j = 0; j < ms; ++j) {
    const double kj = sort_key<KIND>(in_pole<KIND>(D, j));
    int rank = 0;
    bool dup = false;
    for (int l = 0; l < ms; ++l) {
      const double kl = sort_key<KIND>(in_pole<KIND>(D, l));
      rank += (kl > kj) || (kl == kj && l < j);
      dup |= (kl == kj) && (l != j);
    }
    put_sorted<KIND>(D, w, rank, j);
    w.st[j] = input_status<KIND>(D, j, dup);
  }
  uint32_t st = 0;
  int zp = 0;
  dd acc = {0.0, 0.0};
  for (int j = 0; j < ms; ++j) {
    st |= w.st[j];
    acc = dd_add(acc, corner_term<KIND>(D, w, j));
  }
  for (int j = 0; j < D.n - 1; ++j) {
    prologue_elem<KIND>(D, w, j);
    zp |= w.ds[j] == 0.0;
  }
  const dd c = dd_add(corner_base<KIND>(D, w), acc);
  w.hdr[0] = c.hi;
  w.hdr[1] = c.lo;
  w.hdr[2] = zp ? 1.0 : 0.0;
  *prob_flags(w) = st;
  w.hdr[8] = (double)(D.n - 1);
  w.hdr[9] = 0.0;
  if (KIND == KIND_ARROW && st == INFO_REDUCIBLE) {
    // deflation, one run after another (the device splits the runs over a block)
    const int m = D.n - 1;
    int r = 0, q = 0;
    bool zr = false;
    for (int j = 0; j < m; ++j)
      if (run_start(w.ds, j)) zr |= deflate_run(w, m, j, r, q, w.pv1);
    for (int j = 0; j < r; ++j) w.ds[j] = w.pv1[j];
    w.hdr[8] = (double)r;
    w.hdr[9] = (double)q;
    w.hdr[2] = zr ? 1.0 : 0.0;
    *prob_flags(w) = 0u;
  }
  // a Hermitian arrowhead is solved as the real one with shaft |z|
  constexpr int SK = KIND == KIND_HERM ? KIND_ARROW : KIND;
#pragma omp parallel for schedule(dynamic, 4)
  for (int k = 0; k < D.n; ++k) root_body<SK, 1>(D, opt, k, 0);
  if (g_batch_check) {
    // as the batched check stage: Remark 2 and the DPR1 re-measure gathered and
    // re-run (DEFER_WAVE, then DEFER_NEAR_ZERO), Remark 1 listed for the repairs
    *repair_count(w) = 0u;
    std::vector<int> again;
    for (int k = 0; k < D.n; ++k)
      if (check_body<SK, 1, false, DEFER_WAVE>(D, opt, k, 0)) again.push_back(k);
    for (int k : again) check_body<SK, 1, false, DEFER_NEAR_ZERO>(D, opt, k, 0);
    const uint32_t c = *repair_count(w);
    if (c > (uint32_t)D.n) abort();
    for (uint32_t q = 0; q < c; ++q) check_body<SK, 1>(D, opt, (int)repair_list(w, D.n)[q], 0);
  } else {
#pragma omp parallel for schedule(dynamic, 4)
    for (int k = 0; k < D.n; ++k) check_body<SK, 1>(D, opt, k, 0);
  }
  const int nd = deflated_count(w);
  for (int s = 0; s < nd; ++s) place_deflated(D, w, s);
  if (KIND == KIND_HERM && D.V) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < D.n; ++k)
      for (int r = 0; r < D.n; ++r) {
        const bool body = r < D.n - 1;
        double* u = D.V + 2 * ((size_t)k * D.ldv + r);
        vec_entry_c(body ? D.d[r] : 0.0, body ? D.z[2 * r] : 0.0, body ? D.z[2 * r + 1] : 0.0, !body, w.pv[k],
                    w.sf[k], w.mu[k], w.inrm[k], u, u + 1);
      }
  } else if (D.V) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < D.n; ++k) {
      const int it = (nd > 0 && w.cm[k] < nd) ? w.cm[k] : -1;
      for (int r = 0; r < D.n; ++r) {
        const double v = it >= 0 ? (r < D.n - 1 ? deflated_entry(w, it, w.iperm[r], D.z[r]) : 0.0)
                                 : vec_elem<KIND>(D, w.pv[k], w.sf[k], w.mu[k], w.inrm[k], r);
        D.V[(size_t)k * D.ldv + r] = v;
        if (KIND == KIND_SVD && U) U[(size_t)k * D.ldv + r] = svd_left(D, D.lam[k], v, r);
      }
    }
  }
}

extern "C" void emu_set_batch_check(int on) { g_batch_check = on; }

extern "C" int emu_solve(int kind, int64_t n, const double* d, const double* z, double scalar, double* lam,
                         double* V, double* U, double* shift, double* mu, uint32_t* info, double tau_nu,
                         double tau_zero, int fp64_b, int remedies, double* kb, int root, int32_t* cnt,
                         double tau_b, double* knu) {
  std::vector<double> ws(ws_doubles(n), 0.0);
  ProbDesc D{};
  D.kind = kind;
  D.n = (int32_t)n;
  D.d = d;
  D.z = z;
  D.neg = kind == KIND_DPR1 && scalar < 0.0;
  D.scalar = D.neg ? -scalar : scalar;
  D.lam = lam;
  D.V = V;
  D.ldv = n;
  D.U = U;
  D.ldu = n;
  D.shift = shift;
  D.mu = mu;
  D.info = info;
  D.ws = ws.data();
  Options opt{tau_nu, tau_zero, fp64_b, remedies, root, tau_b, 0};
  if (kind == KIND_ARROW) run<KIND_ARROW>(D, opt, U);
  else if (kind == KIND_DPR1) run<KIND_DPR1>(D, opt, U);
  else if (kind == KIND_HERM) run<KIND_HERM>(D, opt, U);
  else run<KIND_SVD>(D, opt, U);
  if (kb) {
    const Ws w = ws_view(D.ws, D.n);
    for (int k = 0; k < D.n; ++k) kb[k] = w.kb1[k];
  }
  if (knu) {
    const Ws w = ws_view(D.ws, D.n);
    for (int k = 0; k < D.n; ++k) knu[k] = w.knu[k];
  }
  if (cnt) {
    const Ws w = ws_view(D.ws, D.n);
    for (int64_t k = 0; k < 6 * (int64_t)D.n; ++k) cnt[k] = w.cnt[k];
  }
  return 0;
}
