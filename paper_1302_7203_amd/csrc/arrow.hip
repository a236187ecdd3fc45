// libarrow: gfx950 kernels and the C ABI declared in include/arrow.h.
//
// One call runs five launches on the handle's stream:
//   k_sort      rank of every pole (symmetric permutation to decreasing order, Sec. 1)
//   k_prologue  shaft weights and corner of the (reduced) arrowhead in double-double
//   k_root      per eigenvalue: shift selection, b, bisection (Algorithms 1-3, Theorem 6)
//   k_check     per eigenvalue: K_nu test and remedies (Algorithm 5, Remarks 1-2), norm
//   k_vec       eigenvector entries, streamed to HBM (eq. eigenvecAi, Algorithm 4)
// k_root / k_check give G lanes of a wavefront to each eigenvalue (G = 64: one
// wavefront per eigenvalue); k_vec is bound by the n^2 FP64 stores.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/arrow.h"
#include "bodies.hpp"

using namespace ahd;

static_assert(ARROW_INFO_DD_B == INFO_DD_B && ARROW_INFO_REMEDY_A == INFO_REMEDY_A &&
                  ARROW_INFO_REMEDY_B == INFO_REMEDY_B && ARROW_INFO_NEAR_ZERO == INFO_NEAR_ZERO &&
                  ARROW_INFO_REDUCIBLE == INFO_REDUCIBLE && ARROW_INFO_NONFINITE == INFO_NONFINITE &&
                  ARROW_INFO_KB_LARGE == INFO_KB_LARGE && ARROW_INFO_BAD_INPUT == INFO_BAD_INPUT &&
                  ARROW_INFO_POLE_SHIFT == INFO_POLE_SHIFT,
              "info bits");

constexpr int BLOCK = 256;
constexpr int VEC_ROWS = 1024;  // rows of one column written by one k_vec block

// ---------------------------------------------------------------------------
// kernels

template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_sort(ProbDesc D) {
  __shared__ double tile[BLOCK];
  const int ms = sorted_count(D);
  const int j = blockIdx.x * BLOCK + threadIdx.x;
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
    const Ws w = ws_view(D.ws, D.n);
    w.ds[rank] = D.d[j];
    w.zs[rank] = D.z[j];
    w.st[j] = input_status<KIND>(D, j, dup);
  }
}

template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_prologue(ProbDesc D) {
  __shared__ double shi[BLOCK], slo[BLOCK];
  __shared__ uint32_t sst[BLOCK];
  const Ws w = ws_view(D.ws, D.n);
  const int ms = sorted_count(D);
  const int m = D.n - 1;
  const int t = threadIdx.x;
  uint32_t st = 0;
  uint32_t zp = 0;
  dd acc = {0.0, 0.0};
  for (int j = t; j < ms; j += BLOCK) {
    st |= w.st[j];
    acc = dd_add(acc, corner_term<KIND>(D, w, j));
  }
  for (int j = t; j < m; j += BLOCK) {
    prologue_elem<KIND>(D, w, j);
    zp |= (w.ds[j] == 0.0) ? 1u : 0u;
  }
  shi[t] = acc.hi;
  slo[t] = acc.lo;
  sst[t] = st | (zp << 31);
  __syncthreads();
  for (int o = BLOCK / 2; o > 0; o >>= 1) {
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
  }
}

template <int KIND, int G>
__global__ __launch_bounds__(BLOCK) void k_root(ProbDesc D, Options opt) {
  const int gid = blockIdx.x * BLOCK + threadIdx.x;
  const int k = gid / G;
  if (k >= D.n) return;
  root_body<KIND, G>(D, opt, k, gid % G);
}

template <int KIND, int G>
__global__ __launch_bounds__(BLOCK) void k_check(ProbDesc D, Options opt) {
  const int gid = blockIdx.x * BLOCK + threadIdx.x;
  const int k = gid / G;
  if (k >= D.n) return;
  check_body<KIND, G>(D, opt, k, gid % G);
}

template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_vec(ProbDesc D, int tiles) {
  const int col = blockIdx.x / tiles;
  const int tile = blockIdx.x - col * tiles;
  const Ws w = ws_view(D.ws, D.n);
  const double pv = w.pv[col], s = w.sf[col], mu = w.mu[col], inrm = w.inrm[col];
  double* vc = D.V + (size_t)col * (size_t)D.ldv;
  double* uc = (KIND == KIND_SVD && D.U) ? D.U + (size_t)col * (size_t)D.ldu : nullptr;
  const double sigma = (KIND == KIND_SVD) ? D.lam[col] : 0.0;
#pragma unroll
  for (int q = 0; q < VEC_ROWS / BLOCK; ++q) {
    const int r = tile * VEC_ROWS + q * BLOCK + threadIdx.x;
    if (r < D.n) {
      const double v = vec_elem<KIND>(D, pv, s, mu, inrm, r);
      __builtin_nontemporal_store(v, vc + r);
      if (KIND == KIND_SVD && uc) __builtin_nontemporal_store(svd_left(D, sigma, v, r), uc + r);
    }
  }
}

// ---------------------------------------------------------------------------
// host side

struct arrow_handle_s {
  int device;
  hipStream_t stream;
  double* ws;
  size_t ws_cap;  // doubles
  Options opt;
  int lanes;      // 0: automatic
  int timing;     // record stage events
  hipEvent_t ev[6];
  int ev_made;
  int have_last;  // a timed call has been launched
  int64_t last_n;
  uint32_t magic;
};

static constexpr uint32_t HANDLE_MAGIC = 0xA770E16u;

static bool valid(arrow_handle_t h) { return h && h->magic == HANDLE_MAGIC; }

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

static int ensure_ws(arrow_handle_t h, size_t doubles) {
  if (doubles <= h->ws_cap) return ARROW_OK;
  if (h->ws) {
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(h->ws);
    h->ws = nullptr;
    h->ws_cap = 0;
  }
  if (hipMalloc((void**)&h->ws, doubles * sizeof(double)) != hipSuccess) {
    h->ws = nullptr;
    return ARROW_ERR_NOMEM;
  }
  h->ws_cap = doubles;
  return ARROW_OK;
}

static int auto_lanes(int64_t n) {
  int64_t want = n / 8;
  int g = 1;
  while (g < 64 && g < want) g <<= 1;
  return g;
}

template <int KIND, int G>
static void launch_rc(const ProbDesc& D, const Options& opt, hipStream_t st, bool check) {
  const int64_t threads = (int64_t)D.n * G;
  const dim3 grid((unsigned)((threads + BLOCK - 1) / BLOCK));
  if (!check) hipLaunchKernelGGL((k_root<KIND, G>), grid, dim3(BLOCK), 0, st, D, opt);
  else hipLaunchKernelGGL((k_check<KIND, G>), grid, dim3(BLOCK), 0, st, D, opt);
}

template <int KIND>
static void launch_rc_any(int G, const ProbDesc& D, const Options& opt, hipStream_t st, bool check) {
  switch (G) {
    case 1: launch_rc<KIND, 1>(D, opt, st, check); break;
    case 2: launch_rc<KIND, 2>(D, opt, st, check); break;
    case 4: launch_rc<KIND, 4>(D, opt, st, check); break;
    case 8: launch_rc<KIND, 8>(D, opt, st, check); break;
    case 16: launch_rc<KIND, 16>(D, opt, st, check); break;
    case 32: launch_rc<KIND, 32>(D, opt, st, check); break;
    default: launch_rc<KIND, 64>(D, opt, st, check); break;
  }
}

template <int KIND>
static int launch_problem(arrow_handle_t h, const ProbDesc& D) {
  hipStream_t st = h->stream;
  (void)hipGetLastError();
  const bool tm = h->timing && h->ev_made;
  auto mark = [&](int e) {
    if (tm) (void)hipEventRecord(h->ev[e], st);
  };
  const int ms = sorted_count(D);
  mark(0);
  if (ms > 0) hipLaunchKernelGGL(k_sort<KIND>, dim3((ms + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, D);
  mark(1);
  hipLaunchKernelGGL(k_prologue<KIND>, dim3(1), dim3(BLOCK), 0, st, D);
  mark(2);
  const int G = h->lanes ? h->lanes : auto_lanes(D.n);
  launch_rc_any<KIND>(G, D, h->opt, st, false);
  mark(3);
  launch_rc_any<KIND>(G, D, h->opt, st, true);
  mark(4);
  if (D.V) {
    const int tiles = (D.n + VEC_ROWS - 1) / VEC_ROWS;
    hipLaunchKernelGGL(k_vec<KIND>, dim3((unsigned)((int64_t)tiles * D.n)), dim3(BLOCK), 0, st, D, tiles);
  }
  mark(5);
  h->have_last = tm ? 1 : 0;
  h->last_n = D.n;
  return hipGetLastError() == hipSuccess ? ARROW_OK : ARROW_ERR_HIP;
}

static bool finite_h(double x) { return x - x == 0.0; }

extern "C" {

int arrow_create(arrow_handle_t* h, int device) {
  if (!h) return -1;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return ARROW_ERR_HIP;
  if (device < 0 || device >= count) return -2;
  arrow_handle_t p = (arrow_handle_t)calloc(1, sizeof(*p));
  if (!p) return ARROW_ERR_NOMEM;
  p->device = device;
  p->stream = nullptr;
  p->opt.tau_nu = 10.0;
  p->opt.tau_zero = 10.0;
  p->opt.fp64_b = 0;
  p->opt.remedies = 1;
  p->lanes = 0;
  p->magic = HANDLE_MAGIC;
  *h = p;
  return ARROW_OK;
}

int arrow_destroy(arrow_handle_t h) {
  if (!valid(h)) return ARROW_ERR_STATE;
  DeviceGuard g(h->device);
  (void)hipStreamSynchronize(h->stream);
  if (h->ws) (void)hipFree(h->ws);
  if (h->ev_made)
    for (int e = 0; e < 6; ++e) (void)hipEventDestroy(h->ev[e]);
  h->magic = 0;
  free(h);
  return ARROW_OK;
}

int arrow_set_stream(arrow_handle_t h, void* hip_stream) {
  if (!valid(h)) return ARROW_ERR_STATE;
  h->stream = (hipStream_t)hip_stream;
  return ARROW_OK;
}

int arrow_set_option(arrow_handle_t h, int option, double value) {
  if (!valid(h)) return ARROW_ERR_STATE;
  switch (option) {
    case ARROW_OPT_TAU_NU:
      if (!(value >= 1.0)) return -3;
      h->opt.tau_nu = value;
      return ARROW_OK;
    case ARROW_OPT_TAU_ZERO:
      if (!(value >= 1.0)) return -3;
      h->opt.tau_zero = value;
      return ARROW_OK;
    case ARROW_OPT_FP64_B:
      h->opt.fp64_b = value != 0.0;
      return ARROW_OK;
    case ARROW_OPT_REMEDIES:
      h->opt.remedies = value != 0.0;
      return ARROW_OK;
    case ARROW_OPT_TIMING:
      if (value != 0.0 && !h->ev_made) {
        DeviceGuard g(h->device);
        for (int e = 0; e < 6; ++e)
          if (hipEventCreate(&h->ev[e]) != hipSuccess) return ARROW_ERR_HIP;
        h->ev_made = 1;
      }
      h->timing = value != 0.0;
      return ARROW_OK;
    case ARROW_OPT_LANES: {
      const int g = (int)value;
      if (g != 0 && g != 1 && g != 2 && g != 4 && g != 8 && g != 16 && g != 32 && g != 64) return -3;
      h->lanes = g;
      return ARROW_OK;
    }
    default:
      return -2;
  }
}

size_t arrow_workspace_size(int64_t n) { return n < 1 ? 0 : ws_doubles(n) * sizeof(double); }

int arrow_last_timing(arrow_handle_t h, double* ms) {
  if (!valid(h)) return -1;
  if (!ms) return -2;
  if (!h->have_last) return ARROW_ERR_STATE;
  DeviceGuard g(h->device);
  if (hipEventSynchronize(h->ev[5]) != hipSuccess) return ARROW_ERR_HIP;
  for (int e = 0; e < 5; ++e) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, h->ev[e], h->ev[e + 1]) != hipSuccess) return ARROW_ERR_HIP;
    ms[e] = t;
  }
  return ARROW_OK;
}

int arrow_last_counters(arrow_handle_t h, int64_t* out) {
  if (!valid(h)) return -1;
  if (!out) return -2;
  if (!h->ws || h->last_n < 1) return ARROW_ERR_STATE;
  DeviceGuard g(h->device);
  if (hipStreamSynchronize(h->stream) != hipSuccess) return ARROW_ERR_HIP;
  const int64_t n = h->last_n;
  const Ws w = ws_view(h->ws, n);
  int32_t* host = (int32_t*)malloc((size_t)n * 6 * sizeof(int32_t));
  if (!host) return ARROW_ERR_NOMEM;
  if (hipMemcpy(host, w.cnt, (size_t)n * 6 * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
    free(host);
    return ARROW_ERR_HIP;
  }
  for (int c = 0; c < 6; ++c) out[c] = 0;
  for (int64_t k = 0; k < n; ++k)
    for (int c = 0; c < 6; ++c) out[c] += host[6 * k + c];
  out[6] = n;
  free(host);
  return ARROW_OK;
}

int arrow_eig(arrow_handle_t h, int64_t n, const double* d, const double* z, double alpha, double* lambda,
              double* V, int64_t ldv, double* shift, double* mu, uint32_t* info) {
  if (!valid(h)) return -1;
  if (n < 1 || n > (int64_t)1 << 28) return -2;
  if (n > 1 && !d) return -3;
  if (n > 1 && !z) return -4;
  if (!finite_h(alpha)) return -5;
  if (!lambda) return -6;
  if (V && ldv < n) return -8;
  DeviceGuard g(h->device);
  const int rc = ensure_ws(h, ws_doubles(n));
  if (rc) return rc;
  ProbDesc D{};
  D.kind = KIND_ARROW;
  D.n = (int32_t)n;
  D.d = d;
  D.z = z;
  D.scalar = alpha;
  D.lam = lambda;
  D.V = V;
  D.ldv = ldv;
  D.shift = shift;
  D.mu = mu;
  D.info = info;
  D.ws = h->ws;
  return launch_problem<KIND_ARROW>(h, D);
}

int dpr1_eig(arrow_handle_t h, int64_t n, const double* d, const double* u, double rho, double* lambda,
             double* Q, int64_t ldq, uint32_t* info) {
  if (!valid(h)) return -1;
  if (n < 1 || n > (int64_t)1 << 28) return -2;
  if (!d) return -3;
  if (!u) return -4;
  if (!finite_h(rho) || !(rho > 0.0)) return -5;
  if (!lambda) return -6;
  if (Q && ldq < n) return -8;
  DeviceGuard g(h->device);
  const int rc = ensure_ws(h, ws_doubles(n));
  if (rc) return rc;
  ProbDesc D{};
  D.kind = KIND_DPR1;
  D.n = (int32_t)n;
  D.d = d;
  D.z = u;
  D.scalar = rho;
  D.lam = lambda;
  D.V = Q;
  D.ldv = ldq;
  D.info = info;
  D.ws = h->ws;
  return launch_problem<KIND_DPR1>(h, D);
}

int arrow_svd(arrow_handle_t h, int64_t n, const double* d, const double* z, double alpha, double* sigma,
              double* U, int64_t ldu, double* V, int64_t ldv, uint32_t* info) {
  if (!valid(h)) return -1;
  if (n < 1 || n > (int64_t)1 << 28) return -2;
  if (n > 1 && !d) return -3;
  if (n > 1 && !z) return -4;
  if (!finite_h(alpha)) return -5;
  if (!sigma) return -6;
  if (U && ldu < n) return -8;
  if (V && ldv < n) return -10;
  if (U && !V) return -9;  // left vectors are formed from the right ones
  DeviceGuard g(h->device);
  const int rc = ensure_ws(h, ws_doubles(n));
  if (rc) return rc;
  ProbDesc D{};
  D.kind = KIND_SVD;
  D.n = (int32_t)n;
  D.d = d;
  D.z = z;
  D.scalar = alpha;
  D.lam = sigma;
  D.V = V;
  D.ldv = ldv;
  D.U = U;
  D.ldu = ldu;
  D.info = info;
  D.ws = h->ws;
  return launch_problem<KIND_SVD>(h, D);
}

}  // extern "C"
