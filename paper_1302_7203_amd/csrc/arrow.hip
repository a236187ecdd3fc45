// libarrow: gfx950 kernels and the C ABI declared in include/arrow.h.
//
// One call runs these launches on the handle's stream:
//   k_front     sortedness check; for sorted input also the copy to the
//               workspace and the prologue: shaft weights and corner of the
//               (reduced) arrowhead in double-double, and the deflation of a
//               reducible arrowhead (Sec. 1)
//   k_sort      unsorted input only: rank of every pole (symmetric permutation
//               to decreasing order, Sec. 1), the permuted copy, the prologue
//   k_root      per eigenvalue: shift selection, b, root of the inverse (Algorithms 1-3, Theorem 6)
//   k_check     per eigenvalue: K_nu test (Algorithm 5), norm; repairs are deferred
//   k_repair    the deferred repairs (Remarks 1-2, DPR1 re-measure), a block per eigenvalue;
//               then the eigenpairs a reducible arrowhead deflated (Sec. 1) are placed
//   k_vec       eigenvector entries, streamed to HBM (eq. eigenvecAi, Algorithm 4);
//               k_vec_c the complex ones of a Hermitian arrowhead (Sec. 6.1)
// k_root / k_check give G lanes of a wavefront to each eigenvalue (G = 64: one
// wavefront per eigenvalue); k_vec is bound by the n^2 FP64 stores.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <math.h>
#include <mutex>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/arrow.h"
#include "blocks.hpp"
#include "host.hpp"

using namespace ahd;

// orders the single-problem calls accept: the root and check launches index
// n * G <= 2^31 lanes (G <= 64) in 64-bit arithmetic
static bool order_ok(int64_t n) { return n >= 1 && n <= ARROW_N_MAX; }

static_assert(ARROW_INFO_DD_B == INFO_DD_B && ARROW_INFO_REMEDY_A == INFO_REMEDY_A &&
                  ARROW_INFO_REMEDY_B == INFO_REMEDY_B && ARROW_INFO_NEAR_ZERO == INFO_NEAR_ZERO &&
                  ARROW_INFO_REDUCIBLE == INFO_REDUCIBLE && ARROW_INFO_NONFINITE == INFO_NONFINITE &&
                  ARROW_INFO_KB_LARGE == INFO_KB_LARGE && ARROW_INFO_BAD_INPUT == INFO_BAD_INPUT &&
                  ARROW_INFO_POLE_SHIFT == INFO_POLE_SHIFT && ARROW_INFO_DEFLATED == INFO_DEFLATED &&
                  ARROW_INFO_F0_UNRESOLVED == INFO_F0_UNRESOLVED,
              "info bits");


// ---------------------------------------------------------------------------
// kernels

// Sorting (symmetric permutation to decreasing poles, Sec. 1): a one-block
// check whether the input already is in that order, or in the reverse one
// (the usual cases), then, only if not, a rank count over a 2-D grid of (pole
// tile, comparison chunk) blocks, then the scatter.  rank[] holds the count
// in its low 30 bits and a duplicate marker in bit 30.
constexpr int SORT_CHUNK = 256;   // keys of one comparison chunk
constexpr int SORT_BLOCK = 1024;  // the last block also scatters and runs the prologue: a wide one

__host__ __device__ inline uint32_t* rank_array(const Ws& w, int64_t n) { return w.st + n; }

// One block of FRONT_BLOCK threads: whether the input already is in that
// order (the usual case); if it is, the copy to the workspace and the whole
// prologue are done here and k_sort returns at once, else the rank array and
// k_sort's completion counter are cleared for it.
constexpr int FRONT_BLOCK = 1024;

__host__ __device__ inline uint32_t* sort_done(const Ws& w) { return (uint32_t*)(w.hdr + 7); }

template <int KIND>
__global__ __launch_bounds__(FRONT_BLOCK) void k_front(ProbDesc D) {
  const Ws w = ws_view(D.ws, D.n);
  const int ms = sorted_count(D);
  int down = 0, up = 0;   // some pair not strictly decreasing / not strictly increasing
  for (int j = threadIdx.x; j + 1 < ms; j += FRONT_BLOCK) {
    const double a = sort_key<KIND>(in_pole<KIND>(D, j)), b = sort_key<KIND>(in_pole<KIND>(D, j + 1));
    if (!(a > b)) down = 1;
    if (!(a < b)) up = 1;
  }
  down = __syncthreads_or(down);
  up = __syncthreads_or(up);
  const bool rev = down && !up;   // strictly increasing: sorted index ms-1-j
  const int bad = down && up;
  if (bad) {
    uint32_t* rank = rank_array(w, D.n);
    for (int j = threadIdx.x; j < ms; j += FRONT_BLOCK) rank[j] = 0;
    if (threadIdx.x == 0) {
      w.hdr[5] = 1.0;
      *sort_done(w) = 0u;
    }
    return;
  }
  // the copy and the prologue of each sorted entry r by the thread that reads
  // its source q, from registers; the corner partial sums run over r = t,
  // t + FRONT_BLOCK, ... as in prologue_block, so the corner is the same bits
  // either way the input arrives
  const int m = D.n - 1;
  const double dn = (KIND == KIND_DPR1) ? in_pole<KIND>(D, rev ? 0 : ms - 1) : 0.0;   // the last sorted pole
  uint32_t st = 0, zp = 0;
  dd acc = {0.0, 0.0};
  for (int r = threadIdx.x; r < ms; r += FRONT_BLOCK) {
    const int q = rev ? ms - 1 - r : r;
    const SortedEntry e = put_sorted_v<KIND>(D, w, r, q);
    st |= input_status<KIND>(D, q, false);
    acc = dd_add(acc, corner_term_v<KIND>(D, e.z));
    if (r < m) {
      prologue_vals<KIND>(D, w, r, e.d, e.z, e.c, dn);
      zp |= (e.d == 0.0) ? 1u : 0u;
    }
  }
  prologue_reduce<KIND, FRONT_BLOCK>(D, w, acc, st, zp);
  if (threadIdx.x == 0) w.hdr[5] = 0.0;
}

// Unsorted input: the rank of every key over a 2-D grid of (key tile,
// comparison chunk) blocks, accumulated with atomics; the last block to finish
// (a completion count) then holds every rank, scatters the poles into
// decreasing order and runs the prologue.
template <int KIND>
__global__ __launch_bounds__(SORT_BLOCK) void k_sort(ProbDesc D, int chunk, int nchunks) {
  __shared__ double tile[SORT_BLOCK];
  __shared__ int last;
  const Ws w = ws_view(D.ws, D.n);
  if (w.hdr[5] == 0.0) return;  // already sorted: k_front did everything
  const int ms = sorted_count(D);
  uint32_t* rank = rank_array(w, D.n);
  const int j = blockIdx.x * SORT_BLOCK + threadIdx.x;
  const double kj = (j < ms) ? sort_key<KIND>(in_pole<KIND>(D, j)) : NAN;
  uint32_t cnt = 0;
  bool dup = false;
  for (int cy = blockIdx.y; cy < nchunks; cy += gridDim.y) {   // this block's comparison chunks
    const int l0 = cy * chunk;
    const int l1 = min(ms, l0 + chunk);
    for (int base = l0; base < l1; base += SORT_BLOCK) {
      const int l = base + threadIdx.x;
      tile[threadIdx.x] = (l < l1) ? sort_key<KIND>(in_pole<KIND>(D, l)) : NAN;
      __syncthreads();
      const int lim = min(SORT_BLOCK, l1 - base);
      for (int t = 0; t < lim; ++t) {
        const double kl = tile[t];
        const int idx = base + t;
        cnt += (kl > kj) || (kl == kj && idx < j);
        dup |= (kl == kj) && (idx != j);
      }
      __syncthreads();
    }
  }
  if (j < ms) {
    if (cnt) atomicAdd(&rank[j], cnt);
    if (dup) atomicOr(&rank[j], 1u << 30);
  }
  // Every thread releases its counts at device scope (a write-back, no
  // invalidation of the L2), then one thread counts the block in; only the
  // last block acquires before it reads the ranks.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(sort_done(w), 1u) == gridDim.x * gridDim.y - 1;
  __syncthreads();
  if (!last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  for (int q = threadIdx.x; q < ms; q += SORT_BLOCK) {
    const uint32_t raw = __hip_atomic_load(&rank[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int r = (int)(raw & 0x3fffffffu);
    if (r < ms) put_sorted<KIND>(D, w, r, q);   // a rank is < ms by construction
    w.st[q] = input_status<KIND>(D, q, (raw >> 30) & 1u);
  }
  __syncthreads();
  prologue_block<KIND, SORT_BLOCK>(D);
}

// Root and check stages: ROOT_BLOCK threads per block, G lanes per
// eigenvalue.  When the sorted poles and shaft weights fit, the block first
// copies them to LDS and every O(n) pass reads them from there.
constexpr int ROOT_BLOCK = 512;

__device__ inline void stage_hot(const ProbDesc& D, double* lds) {
  const Ws w = ws_view(D.ws, D.n);
  const int ns = sorted_count(D), m = D.n - 1;
  const int top = ns > m ? ns : m;
  // four rows of both arrays in flight per thread before the LDS stores
  for (int j0 = threadIdx.x; j0 < top; j0 += 4 * blockDim.x) {
    double a[4], c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + q * blockDim.x;
      a[q] = (j < ns) ? w.ds[j] : 0.0;
      c[q] = (j < m) ? w.ch[j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + q * blockDim.x;
      if (j < ns) lds[j] = a[q];
      if (j < m) lds[ns + j] = c[q];
    }
  }
  __syncthreads();
}

// STAGE is a template argument so that, once the bodies are inlined, the
// compiler sees the hot arrays as LDS and reads them with ds_read.
template <int KIND, int G, bool STAGE>
__global__ __launch_bounds__(ROOT_BLOCK) void k_root(ProbDesc D, Options opt) {
  extern __shared__ double lds[];
  if constexpr (STAGE) stage_hot(D, lds);
  const int64_t gid = (int64_t)blockIdx.x * ROOT_BLOCK + threadIdx.x;
  const int k = (int)(gid / G);
  if (k >= D.n) return;
  if constexpr (STAGE) root_body<KIND, G, true>(D, opt, k, (int)(gid % G), lds, lds + sorted_count(D));
  else root_body<KIND, G>(D, opt, k, (int)(gid % G));
}

template <int KIND, int G, bool STAGE>
__global__ __launch_bounds__(ROOT_BLOCK) void k_check(ProbDesc D, Options opt) {
  extern __shared__ double lds[];
  if constexpr (STAGE) stage_hot(D, lds);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // blocks of ROOT_BLOCK, or CHECK_LANE_BLOCK
  const int k = (int)(gid / G);
  if (k >= D.n) return;
  if constexpr (STAGE) check_body<KIND, G, true, DEFER_ALL>(D, opt, k, (int)(gid % G), lds, lds + sorted_count(D));
  else check_body<KIND, G, false, DEFER_ALL>(D, opt, k, (int)(gid % G));
}

// The eigenvalues k_check deferred (Remarks 1 and 2, the DPR1 re-measure),
// GR lanes each (GR = REPAIR_BLOCK: a block per eigenvalue; GR = 64: a
// wavefront per eigenvalue, REPAIR_BLOCK/64 of them sharing the block's staged
// arrays): the repairs are a handful of eigenvalues with several O(n) passes
// apiece, so they get their own launch instead of stretching k_check.
// Groups beyond the list length skip the work.  When the arrowhead was
// deflated, the last block to finish then places the deflated eigenpairs
// among the solved ones, whose values are all final at that point.
constexpr int REPAIR_BLOCK = 256;

template <int KIND, bool STAGE, int GR>
__global__ __launch_bounds__(REPAIR_BLOCK) void k_repair(ProbDesc D, Options opt) {
  extern __shared__ double lds[];
  constexpr int PER = REPAIR_BLOCK / GR;       // repairs per block
  const Ws w = ws_view(D.ws, D.n);
  const uint32_t count = min(*repair_count(w), (uint32_t)D.n);
  if (blockIdx.x * PER < count) {
    if constexpr (STAGE) stage_hot(D, lds);
    const uint32_t* list = repair_list(w, D.n);
    const int grp = threadIdx.x / GR, ln = threadIdx.x % GR;
    for (uint32_t q = blockIdx.x * PER + grp; q < count; q += gridDim.x * PER) {
      const int k = (int)list[q];
      if (k < 0 || k >= D.n) continue;
      if constexpr (STAGE) check_body<KIND, GR, true>(D, opt, k, ln, lds, lds + sorted_count(D));
      else check_body<KIND, GR>(D, opt, k, ln);
    }
  }
  if constexpr (KIND == KIND_ARROW) {
    if (deflated_count(w) > 0) place_deflated_last(D, w, gridDim.x);
  }
}

// cols <= VEC_COLS_MAX (vec_shape).  A single problem's tiles read their
// columns' shift data straight from the workspace: staged in LDS first they
// were slower at n = 4096 (27.8 against 25.7 us) and equal at n = 16384.
#ifndef AHD_SINGLE_VEC_STAGE
#define AHD_SINGLE_VEC_STAGE 0
#endif
template <int KIND, int W, int RPT>
__global__ __launch_bounds__(BLOCK) void k_vec(ProbDesc D, int row_tiles, int cols) {
  __shared__ VecTileStage L;
  const int ct = blockIdx.x / row_tiles;
  vec_tile<KIND, W, RPT, VecTileStage, AHD_SINGLE_VEC_STAGE != 0>(D, blockIdx.x - ct * row_tiles, ct, cols, L);
}

template <int RPT>
__global__ __launch_bounds__(BLOCK) void k_vec_c(ProbDesc D, int row_tiles, int cols) {
  __shared__ VecTileStage L;
  const int ct = blockIdx.x / row_tiles;
  vec_tile_c<RPT>(D, blockIdx.x - ct * row_tiles, ct, cols, L);
}

// ---------------------------------------------------------------------------
// host side

// A launch whose timing events, when given, are stamped by the dispatch itself
// at the kernel's start and end: no marker packets between the launches, which
// would add a dispatch gap of their own at every stage boundary.
template <typename F, typename... A>
static void launch_timed(F kern, dim3 grid, dim3 block, size_t lds, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                         A... args) {
  if (e0 || e1) hipExtLaunchKernelGGL(kern, grid, block, (uint32_t)lds, st, e0, e1, 0u, args...);
  else hipLaunchKernelGGL(kern, grid, block, lds, st, args...);
}

// the check with one lane per eigenvalue and nothing staged is latency-bound
// scalar work: small blocks spread it over more compute units
constexpr int CHECK_LANE_BLOCK = 64;

template <int KIND, int G>
static void launch_rc(const ProbDesc& D, const Options& opt, hipStream_t st, bool check, size_t lds,
                      hipEvent_t e0, hipEvent_t e1) {
  const int64_t threads = (int64_t)D.n * G;
  if (check && G == 1 && lds == 0) {
    const dim3 grid((unsigned)((threads + CHECK_LANE_BLOCK - 1) / CHECK_LANE_BLOCK));
    launch_timed(k_check<KIND, G, false>, grid, dim3(CHECK_LANE_BLOCK), 0, st, e0, e1, D, opt);
    return;
  }
  const dim3 grid((unsigned)((threads + ROOT_BLOCK - 1) / ROOT_BLOCK));
  if (lds > 0) {
    if (!check) launch_timed(k_root<KIND, G, true>, grid, dim3(ROOT_BLOCK), lds, st, e0, e1, D, opt);
    else launch_timed(k_check<KIND, G, true>, grid, dim3(ROOT_BLOCK), lds, st, e0, e1, D, opt);
  } else {
    if (!check) launch_timed(k_root<KIND, G, false>, grid, dim3(ROOT_BLOCK), 0, st, e0, e1, D, opt);
    else launch_timed(k_check<KIND, G, false>, grid, dim3(ROOT_BLOCK), 0, st, e0, e1, D, opt);
  }
}

template <int KIND>
static void launch_rc_any(int G, const ProbDesc& D, const Options& opt, hipStream_t st, bool check, size_t lds,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  switch (G) {
    case 1: launch_rc<KIND, 1>(D, opt, st, check, lds, e0, e1); break;
    case 2: launch_rc<KIND, 2>(D, opt, st, check, lds, e0, e1); break;
    case 4: launch_rc<KIND, 4>(D, opt, st, check, lds, e0, e1); break;
    case 8: launch_rc<KIND, 8>(D, opt, st, check, lds, e0, e1); break;
    case 16: launch_rc<KIND, 16>(D, opt, st, check, lds, e0, e1); break;
    case 32: launch_rc<KIND, 32>(D, opt, st, check, lds, e0, e1); break;
    default: launch_rc<KIND, 64>(D, opt, st, check, lds, e0, e1); break;
  }
}

template <int KIND>
static int launch_problem(arrow_handle_t h, const ProbDesc& D);

// one single-problem solve (all launches) on the handle's stream; used by the
// sequential reference path of the batched API
int launch_single(arrow_handle_t h, const ProbDesc& D) {
  switch (D.kind) {
    case KIND_ARROW: return launch_problem<KIND_ARROW>(h, D);
    case KIND_DPR1: return launch_problem<KIND_DPR1>(h, D);
    case KIND_HERM: return launch_problem<KIND_HERM>(h, D);
    default: return launch_problem<KIND_SVD>(h, D);
  }
}

// A Hermitian problem is sorted and its weights formed as KIND_HERM, then
// solved by the real arrowhead's root, check and repair kernels.
template <int KIND>
static int launch_problem(arrow_handle_t h, const ProbDesc& D) {
  constexpr int SK = (KIND == KIND_HERM) ? KIND_ARROW : KIND;
  hipStream_t st = h->stream;
  (void)hipGetLastError();
  const bool tm = h->timing && h->ev_made;
  // a timed call takes the event set the previous timed call did not use
  const int es = (tm && h->timed_calls > 0) ? 1 - h->ev_set : 0;
  hipEvent_t* ev = h->ev[es];
  auto mark = [&](int e) {
    if (tm) (void)hipEventRecord(ev[e], st);
  };
  auto at = [&](int e) -> hipEvent_t { return tm ? ev[e] : nullptr; };
  const int ms = sorted_count(D);
  // every stage boundary is the start (or end) of a kernel
  launch_timed(k_front<KIND>, dim3(1), dim3(FRONT_BLOCK), 0, st, at(0), nullptr, D);
  if (ms == 0) mark(1);
  if (ms > 0) {
    // about SORT_GRID blocks in all (they return at once when k_front found the
    // order), each comparing its key tile against one or more chunks
    constexpr int64_t SORT_GRID = 256;
    const int64_t jt = (ms + SORT_BLOCK - 1) / SORT_BLOCK;
    const int64_t nchunks = (ms + SORT_CHUNK - 1) / SORT_CHUNK;
    const int64_t lc = std::max<int64_t>(1, std::min<int64_t>({nchunks, SORT_GRID / jt, 65535}));
    launch_timed(k_sort<KIND>, dim3((unsigned)jt, (unsigned)lc), dim3(SORT_BLOCK), 0, st, at(1), nullptr, D,
                 SORT_CHUNK, (int)nchunks);
  }
  // the root and vector stages are timed by their kernels' own start and end;
  // the stages between take up the dispatch gaps
  const int G = single_lanes(h, D.n);
  const size_t hot = (size_t)(ms + D.n - 1) * sizeof(double);
  const size_t lds = (hot <= h->lds_max) ? hot : 0;
  launch_rc_any<SK>(G, D, h->opt, st, false, lds, at(2), at(3));
  // the check stage reads the poles only for DPR1 norms or after bisection;
  // otherwise the root pass left the norm and what remains per eigenvalue is
  // scalar work: one lane each, no staged copy
  const bool check_reads_poles = SK == KIND_DPR1 || h->opt.root != ROOT_RATIONAL;
  if (check_reads_poles) launch_rc_any<SK>(G, D, h->opt, st, true, lds);
  else launch_rc_any<SK>(1, D, h->opt, st, true, 0);
  {
    // deferred repairs; the block reductions add a little static LDS
    const size_t lds_r = (hot + 4096 <= h->lds_max) ? hot : 0;
    constexpr int GR = REPAIR_BLOCK;   // a block per repair (measured faster than a wavefront for n >= 4096)
    const dim3 grid((unsigned)std::min<int64_t>((D.n + REPAIR_BLOCK / GR - 1) / (REPAIR_BLOCK / GR), h->cus));
    if (lds_r > 0) hipLaunchKernelGGL((k_repair<SK, true, GR>), grid, dim3(REPAIR_BLOCK), lds_r, st, D, h->opt);
    else hipLaunchKernelGGL((k_repair<SK, false, GR>), grid, dim3(REPAIR_BLOCK), 0, st, D, h->opt);
  }
  hipEvent_t v0 = D.V ? at(4) : nullptr, v1 = D.V ? at(5) : nullptr;
  if (!v0) mark(4);
  if (KIND == KIND_HERM && D.V) {
    const VecShape sh = vec_shape(D.n);
    const int row_tiles = (int)((D.n + (int64_t)BLOCK * sh.rpt - 1) / ((int64_t)BLOCK * sh.rpt));
    const int col_chunks = (D.n + sh.cols - 1) / sh.cols;
    const dim3 grid((unsigned)((int64_t)row_tiles * col_chunks));
    if (sh.rpt == 8) launch_timed(k_vec_c<8>, grid, dim3(BLOCK), 0, st, v0, v1, D, row_tiles, sh.cols);
    else if (sh.rpt == 2) launch_timed(k_vec_c<2>, grid, dim3(BLOCK), 0, st, v0, v1, D, row_tiles, sh.cols);
    else launch_timed(k_vec_c<4>, grid, dim3(BLOCK), 0, st, v0, v1, D, row_tiles, sh.cols);
  } else if (D.V) {
    const VecShape sh = vec_shape(D.n);
    const int row_tiles = (int)((D.n + (int64_t)BLOCK * sh.rpt - 1) / ((int64_t)BLOCK * sh.rpt));
    const int col_chunks = (D.n + sh.cols - 1) / sh.cols;
    const dim3 grid((unsigned)((int64_t)row_tiles * col_chunks));
    const bool pair = (D.n % 2 == 0) && (D.ldv % 2 == 0) && (((uintptr_t)D.V & 15) == 0) &&
                      (!D.U || ((D.ldu % 2 == 0) && (((uintptr_t)D.U & 15) == 0)));
    if (sh.rpt == 8) {
      if (pair) launch_timed(k_vec<KIND, 2, 8>, grid, dim3(BLOCK), 0, st, v0, v1, D, row_tiles, sh.cols);
      else launch_timed(k_vec<KIND, 1, 8>, grid, dim3(BLOCK), 0, st, v0, v1, D, row_tiles, sh.cols);
    } else if (sh.rpt == 2) {
      if (pair) launch_timed(k_vec<KIND, 2, 2>, grid, dim3(BLOCK), 0, st, v0, v1, D, row_tiles, sh.cols);
      else launch_timed(k_vec<KIND, 1, 2>, grid, dim3(BLOCK), 0, st, v0, v1, D, row_tiles, sh.cols);
    } else {
      if (pair) launch_timed(k_vec<KIND, 2, 4>, grid, dim3(BLOCK), 0, st, v0, v1, D, row_tiles, sh.cols);
      else launch_timed(k_vec<KIND, 1, 4>, grid, dim3(BLOCK), 0, st, v0, v1, D, row_tiles, sh.cols);
    }
  }
  if (!v1) mark(5);
  if (tm) {
    h->ev_set = es;
    h->timed_calls = std::min(h->timed_calls + 1, 2);
  }
  h->last_n = D.n;
  h->last_ws = D.ws;
  return hipGetLastError() == hipSuccess ? ARROW_OK : ARROW_ERR_HIP;
}

static bool finite_h(double x) { return x - x == 0.0; }

// ---------------------------------------------------------------------------
// Scratch of arrow_eig_noalloc: one problem's workspace at the largest order
// that call takes, in static device memory (each device holds its own copy
// until the process ends).  Host code never uses the array's name as a device
// address: arrow_create looks up each device's address once, with that device
// current, and every later use goes through scratch_dev[].
constexpr size_t NOALLOC_WS_DOUBLES = 16 + (size_t)ARROW_NOALLOC_N_MAX * 26;
static __device__ __align__(256) double scratch[NOALLOC_WS_DOUBLES];
constexpr int SCRATCH_DEVICES = 64;
static double* scratch_dev[SCRATCH_DEVICES];
static int scratch_rc[SCRATCH_DEVICES];   // 0: not looked up yet, 1: found, -1: lookup failed
static std::mutex scratch_mu;

static void scratch_lookup(int device) {
  if (device < 0 || device >= SCRATCH_DEVICES) return;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_rc[device] != 0) return;
  DeviceGuard g(device);
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess && ptr) {
    scratch_dev[device] = (double*)ptr;
    scratch_rc[device] = 1;
  } else {
    (void)hipGetLastError();
    scratch_rc[device] = -1;
  }
}

static double* scratch_of(int device) {
  if (device < 0 || device >= SCRATCH_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  return scratch_rc[device] == 1 ? scratch_dev[device] : nullptr;
}

static_assert(NOALLOC_WS_DOUBLES == 16 + (size_t)ARROW_NOALLOC_N_MAX * 26, "workspace of ws_doubles()");

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
  p->opt.tau_nu = 100.0;
  p->opt.check_lanes = 4;
  p->opt.tau_zero = 10.0;
  p->opt.fp64_b = 0;
  p->opt.tau_b = 0.0;
  p->opt.remedies = 1;
  p->opt.root = ROOT_RATIONAL;
  p->lanes = 0;
  {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) v = 0;
    p->lds_max = v > 0 ? (size_t)v : 0;
    v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) v = 0;
    p->cus = v > 0 ? v : 1;
  }
  p->ntab[ARROW_SCHEDULE_SINGLE] = 0;
  default_batch_table(p);
  scratch_lookup(device);   // arrow_eig_noalloc's scratch address on this device
  p->magic = HANDLE_MAGIC;
  *h = p;
  return ARROW_OK;
}

int arrow_destroy(arrow_handle_t h) {
  if (!valid(h)) return ARROW_ERR_STATE;
  DeviceGuard g(h->device);
  (void)hipStreamSynchronize(h->stream);
  tridiag_release(h);
  if (h->ws) (void)hipFree(h->ws);
  if (h->ev_made)
    for (int k = 0; k < 2; ++k)
      for (int e = 0; e < 6; ++e) (void)hipEventDestroy(h->ev[k][e]);
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
    case ARROW_OPT_TAU_B:
      if (!(value >= 0.0 && value < INFINITY)) return -3;
      h->opt.tau_b = value;
      return ARROW_OK;
    case ARROW_OPT_FP64_B:
      h->opt.fp64_b = value != 0.0;
      return ARROW_OK;
    case ARROW_OPT_REMEDIES:
      h->opt.remedies = value != 0.0;
      return ARROW_OK;
    case ARROW_OPT_ROOT:
      if (value != 0.0 && value != 1.0) return -3;
      h->opt.root = (int)value;
      return ARROW_OK;
    case ARROW_OPT_CHECK_LANES: {
      const int g = (int)value;
      if (!((double)g == value && (g == 0 || (g >= 4 && g <= 64 && (g & (g - 1)) == 0)))) return -3;
      h->opt.check_lanes = g;
      return ARROW_OK;
    }
    case ARROW_OPT_TIMING:
      if (value != 0.0 && !h->ev_made) {
        DeviceGuard g(h->device);
        for (int k = 0; k < 2; ++k)
          for (int e = 0; e < 6; ++e)
            if (hipEventCreate(&h->ev[k][e]) != hipSuccess) return ARROW_ERR_HIP;
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

size_t arrow_workspace_size(int64_t n) { return order_ok(n) ? ws_doubles(n) * sizeof(double) : 0; }

int arrow_timing_of(arrow_handle_t h, int age, double* ms) {
  if (!valid(h)) return -1;
  if (!ms) return -2;
  if (age != 0 && age != 1) return -3;
  if (h->timed_calls <= age) return ARROW_ERR_STATE;
  DeviceGuard g(h->device);
  hipEvent_t* ev = h->ev[age == 0 ? h->ev_set : 1 - h->ev_set];
  if (hipEventSynchronize(ev[5]) != hipSuccess) return ARROW_ERR_HIP;
  for (int e = 0; e < 5; ++e) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, ev[e], ev[e + 1]) != hipSuccess) return ARROW_ERR_HIP;
    ms[e] = t;
  }
  return ARROW_OK;
}

int arrow_last_timing(arrow_handle_t h, double* ms) { return arrow_timing_of(h, 0, ms); }

int arrow_conditions(arrow_handle_t h, double* kb, double* knu) {
  if (!valid(h)) return -1;
  if (!h->last_ws || h->last_n < 1) return ARROW_ERR_STATE;
  DeviceGuard g(h->device);
  const Ws w = ws_view(h->last_ws, h->last_n);
  const size_t bytes = (size_t)h->last_n * sizeof(double);
  if (kb && hipMemcpyAsync(kb, w.kbc, bytes, hipMemcpyDeviceToDevice, h->stream) != hipSuccess) return ARROW_ERR_HIP;
  if (knu && hipMemcpyAsync(knu, w.knu, bytes, hipMemcpyDeviceToDevice, h->stream) != hipSuccess) return ARROW_ERR_HIP;
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

}  // extern "C"

// arrow_eig's body: ws = null grows and uses the handle's workspace, else ws
// (room for ws_doubles(n) doubles) is used and nothing is allocated
static int arrow_eig_in(arrow_handle_t h, int64_t n, const double* d, const double* z, double alpha,
                        double* lambda, double* V, int64_t ldv, double* shift, double* mu, uint32_t* info,
                        double* ws) {
  if (!valid(h)) return -1;
  if (!order_ok(n)) return -2;
  if (n > 1 && !d) return -3;
  if (n > 1 && !z) return -4;
  if (!finite_h(alpha)) return -5;
  if (!lambda) return -6;
  if (V && ldv < n) return -8;
  DeviceGuard g(h->device);
  if (!ws) {
    const int rc = ensure_ws(h, ws_doubles(n));
    if (rc) return rc;
    ws = h->ws;
  }
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
  D.ws = ws;
  return launch_problem<KIND_ARROW>(h, D);
}

extern "C" {

int arrow_eig(arrow_handle_t h, int64_t n, const double* d, const double* z, double alpha, double* lambda,
              double* V, int64_t ldv, double* shift, double* mu, uint32_t* info) {
  return arrow_eig_in(h, n, d, z, alpha, lambda, V, ldv, shift, mu, info, nullptr);
}

int arrow_eig_noalloc(arrow_handle_t h, int64_t n, const double* d, const double* z, double alpha,
                      double* lambda, double* V, int64_t ldv, double* shift, double* mu, uint32_t* info) {
  if (!valid(h)) return -1;
  if (n > ARROW_NOALLOC_N_MAX) return -2;   // beyond what the scratch holds
  double* ws = scratch_of(h->device);
  if (!ws) return ARROW_ERR_HIP;            // the address lookup at arrow_create failed
  return arrow_eig_in(h, n, d, z, alpha, lambda, V, ldv, shift, mu, info, ws);
}

int arrow_eig_herm(arrow_handle_t h, int64_t n, const double* d, const double* z, double alpha, double* lambda,
                   double* U, int64_t ldu, double* shift, double* mu, uint32_t* info) {
  if (!valid(h)) return -1;
  if (!order_ok(n)) return -2;
  if (n > 1 && !d) return -3;
  if (n > 1 && (!z || ((uintptr_t)z & 7))) return -4;
  if (!finite_h(alpha)) return -5;
  if (!lambda) return -6;
  if (U && ((uintptr_t)U & 15)) return -7;
  if (U && ldu < n) return -8;
  DeviceGuard g(h->device);
  const int rc = ensure_ws(h, ws_doubles(n));
  if (rc) return rc;
  ProbDesc D{};
  D.kind = KIND_HERM;
  D.n = (int32_t)n;
  D.d = d;
  D.z = z;
  D.scalar = alpha;
  D.lam = lambda;
  D.V = U;
  D.ldv = ldu;
  D.shift = shift;
  D.mu = mu;
  D.info = info;
  D.ws = h->ws;
  return launch_problem<KIND_HERM>(h, D);
}

int dpr1_eig(arrow_handle_t h, int64_t n, const double* d, const double* u, double rho, double* lambda,
             double* Q, int64_t ldq, uint32_t* info) {
  if (!valid(h)) return -1;
  if (!order_ok(n)) return -2;
  if (!d) return -3;
  if (!u) return -4;
  if (!finite_h(rho) || rho == 0.0) return -5;
  if (!lambda) return -6;
  if (Q && ldq < n) return -8;
  DeviceGuard g(h->device);
  const int rc = ensure_ws(h, ws_doubles(n));
  if (rc) return rc;
  ProbDesc D{};
  D.kind = KIND_DPR1;
  D.n = (int32_t)n;
  D.neg = rho < 0.0;
  D.d = d;
  D.z = u;
  D.scalar = fabs(rho);
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
  if (!order_ok(n)) return -2;
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
