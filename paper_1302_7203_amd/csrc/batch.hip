// Batched solves: many independent ARROW / DPR1 / SVD / Hermitian problems of
// uneven order in one plan of five launches.
//
//   k_b_prep    one block per problem: sort (Sec. 1 ordering) and prologue
//   k_b_root    persistent: every wavefront takes (problem, eigenvalue-group)
//               items from an atomic queue and runs the first pass (shift,
//               b, root of the inverse) on them, reading the problem's poles
//               (and weights) from its own LDS slice where they fit, and
//               regrouping unfinished roots onto wider lane groups; problems
//               are queued by decreasing order n so the long items start first
//   k_b_check   a second queue of the same kind for the K_nu test and the
//               norms; the eigenvalues that need a remedy of Remark 2 or the
//               DPR1 re-measure are gathered per wavefront and re-solved on
//               all its lanes; eigenvalues near the origin (Remark 1) are listed
//   k_b_repair  the listed Remark 1 repairs, a block per eigenvalue; then the
//               eigenpairs of a deflated arrowhead (Sec. 1) are placed
//   k_b_vec     every problem's vector tiles (row tiles for large n, flat
//               column-major runs for small n) mapped onto blocks
//
// A wavefront gives G lanes to each eigenvalue, so one item covers 64/G
// consecutive eigenvalues of one problem; G comes from the handle's table of
// lanes by order n (filled by the autotuner).

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "blocks.hpp"
#include "host.hpp"

using namespace ahd;

namespace {

constexpr int WAVE = 64;
constexpr int STAGE_BLOCK = 256;
#ifndef AHD_VEC_TALL_MIN
#define AHD_VEC_TALL_MIN 512
#endif
constexpr int VEC_TALL_MIN = AHD_VEC_TALL_MIN; // n from which vectors are written in row tiles
static_assert(VEC_TALL_MIN - 1 <= VEC_FLAT_ROWS, "flat tiles stage every row of their problem in LDS");

struct BatchArgs {
  const ProbDesc* descs;     // problems in queue order
  const int32_t* item_start; // count + 1 prefix sums of items
  const int32_t* lanes;      // G per problem
  const int32_t* vec_start;  // count + 1 prefix sums of vector tiles
  const int32_t* vec_mode;   // per problem: 0 flat tiles, 1 row tiles, 2 row tiles with 16-byte stores
  const int32_t* check_start;// count + 1 prefix sums of check-stage items
  const int32_t* check_lanes;// lanes per eigenvalue in the check stage, per problem
  const int32_t* vec_prob;   // per vector tile: its problem
  uint32_t* counters;        // [0] first-pass queue, [1] check queue
  int32_t count;
  int32_t total_items;
  int32_t total_check;
};

__device__ inline int find_problem(const int32_t* start, int count, int x) {
  int lo = 0, hi = count;   // start[lo] <= x < start[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(BLOCK) void k_b_prep(BatchArgs B) {
  if (blockIdx.x == 0 && threadIdx.x < 2) B.counters[threadIdx.x] = 0;
  const ProbDesc D = B.descs[blockIdx.x];
  if (sorted_count(D) > 0) {
    switch (D.kind) {
      case KIND_ARROW: sort_block<KIND_ARROW>(D); break;
      case KIND_DPR1: sort_block<KIND_DPR1>(D); break;
      case KIND_HERM: sort_block<KIND_HERM>(D); break;
      default: sort_block<KIND_SVD>(D); break;
    }
  }
  switch (D.kind) {
    case KIND_ARROW: prologue_block<KIND_ARROW>(D); break;
    case KIND_DPR1: prologue_block<KIND_DPR1>(D); break;
    case KIND_HERM: prologue_block<KIND_HERM>(D); break;
    default: prologue_block<KIND_SVD>(D); break;
  }
}

// First pass of the 64/G eigenvalues of an item, G lanes each (every lane of
// the wavefront calls this; `valid`: the lane's eigenvalue k exists).  The
// rational iteration takes from one to several passes, and on fixed groups
// every group would wait for the slowest of its wavefront.  Instead, after
// each step, once the unfinished eigenvalues fit in groups twice as wide,
// they are regrouped: the g-th unfinished one moves (its state copied lane to
// lane) to lanes [g gc, (g + 1) gc) with gc the widest power of two that fits,
// so its further passes run on more lanes (each width a compiled loop of its
// own).  All groups solve the item's problem, so they keep reading the same
// poles.  The regrouping depends only
// on the item's own eigenvalues: a problem gives the same bits alone or in any
// batch.  HOT: what the wavefront's LDS slice holds (make_prob).
template <int KIND, int G, int HOT>
__device__ __forceinline__ void root_item(const ProbDesc& D, const Options& opt, int k, int lane, bool valid,
                                 const double* lds) {
  const int ln = lane & (G - 1);
  const Ws w = ws_view(D.ws, D.n);
  const Prob P = make_prob<HOT>(D, w, lds, lds + sorted_count(D));
  int i = 0;
  RatConsts c{};
  RatState s{};
  bool mine = false;   // the lane's group holds an unfinished eigenvalue
  if (valid) mine = root_begin<KIND, G, HOT>(D, opt, w, P, k, ln, i, c, s);
  double last[3] = {NAN, NAN, NAN};
  if constexpr (G == WAVE) {
    if (mine) {
      while (!rat_step<KIND, G>(P, i, c, s, ln, last)) {
      }
      root_finish<KIND>(P, w, k, i, ln, c.sg * s.x, s.it, last);
    }
  } else {
    int gc = G, lc = ln;
    for (;;) {
      if (mine && rat_step<KIND, G, true>(P, i, c, s, lc, last, gc)) {
        root_finish<KIND>(P, w, k, i, lc, c.sg * s.x, s.it, last);
        mine = false;
      }
      const uint64_t live = __ballot(mine && lc == 0);   // first lanes of the unfinished groups
      if (live == 0) break;
      const int a = __popcll(live);
      int gn = gc;
      while (gn < WAVE && 2 * gn * a <= WAVE) gn *= 2;
      if (gn != gc) {
        const int g = lane / gn;
        uint64_t rest = live;
        for (int t = 0; t < g && rest; ++t) rest &= rest - 1;
        const int src = rest ? __builtin_ctzll(rest) : lane;
        k = __shfl(k, src);
        i = __shfl(i, src);
        c.sg = __shfl(c.sg, src);
        c.rci = __shfl(c.rci, src);
        c.sry = __shfl(c.sry, src);
        s.x = __shfl(s.x, src);
        s.xlo = __shfl(s.xlo, src);
        s.xhi = __shfl(s.xhi, src);
        s.slo = __shfl(s.slo, src);
        s.shi = __shfl(s.shi, src);
        s.c0 = __shfl(s.c0, src);
        s.y = __shfl(s.y, src);
        s.it = __shfl(s.it, src);
        s.hi_open = __shfl(s.hi_open, src);
        mine = g < a;
        gc = gn;
        lc = lane & (gn - 1);
      }
    }
  }
}

// hot: what the wavefront's LDS slice holds -- 1 the sorted poles and then
// the shaft weights, 2 the poles alone, 0 nothing (G <= 16 only).
template <int KIND>
__device__ __forceinline__ void root_kind(const ProbDesc& D, const Options& opt, int G, int k, int lane, bool valid, int hot,
                                 const double* lds) {
  if (hot == 1) {
    switch (G) {
      case 4: root_item<KIND, 4, 1>(D, opt, k, lane, valid, lds); return;
      case 8: root_item<KIND, 8, 1>(D, opt, k, lane, valid, lds); return;
      default: root_item<KIND, 16, 1>(D, opt, k, lane, valid, lds); return;
    }
  }
  if (hot == 2) {
    switch (G) {
      case 4: root_item<KIND, 4, 2>(D, opt, k, lane, valid, lds); return;
      case 8: root_item<KIND, 8, 2>(D, opt, k, lane, valid, lds); return;
      default: root_item<KIND, 16, 2>(D, opt, k, lane, valid, lds); return;
    }
  }
  switch (G) {
    case 4: root_item<KIND, 4, 0>(D, opt, k, lane, valid, lds); break;
    case 8: root_item<KIND, 8, 0>(D, opt, k, lane, valid, lds); break;
    case 16: root_item<KIND, 16, 0>(D, opt, k, lane, valid, lds); break;
    case 32: root_item<KIND, 32, 0>(D, opt, k, lane, valid, lds); break;
    default: root_item<KIND, 64, 0>(D, opt, k, lane, valid, lds); break;
  }
}

// Doubles of LDS per wavefront for a problem's sorted poles and shaft weights
// (2 (n - 1), DPR1 2n), or for the poles alone when both do not fit: every
// pass of the root stage reads them, each lane a term at a time, and from LDS
// they come without the vector memory path.
#ifndef AHD_ROOT_STAGE
#define AHD_ROOT_STAGE 1280
#endif
constexpr int ROOT_STAGE = AHD_ROOT_STAGE;

// Check stage of one item: the 64/G eigenvalues k0, k0 + 1, ... of one
// problem, G lanes each (every lane of the wavefront calls this; lanes past
// the order idle).  Remark 2 and the DPR1 re-measure -- a few percent of the
// eigenvalues, each a full re-solve -- are not run on the item's G lanes,
// which would leave the wavefront's other groups waiting: the eigenvalues that
// need one are gathered by a ballot and re-run one after the other on all 64
// lanes.  Only Remark 1 is listed for k_b_repair (its exact sum of f(0) runs on
// a whole block).
template <int KIND, int G>
__device__ inline void check_item(const ProbDesc& D, const Options& opt, int k0, int lane) {
  const int k = k0 + lane / G, ln = lane & (G - 1);
  bool need = false;
  if (k < D.n) need = check_body<KIND, G, false, DEFER_WAVE>(D, opt, k, ln);
  uint64_t mask = __ballot(need && ln == 0);
  while (mask) {
    const int g = __builtin_ctzll(mask) / G;
    mask &= mask - 1;
    check_body<KIND, WAVE, false, DEFER_NEAR_ZERO>(D, opt, k0 + g, lane);
  }
}

template <int KIND>
__device__ inline void check_kind(const ProbDesc& D, const Options& opt, int G, int k0, int lane) {
  switch (G) {
    case 4: check_item<KIND, 4>(D, opt, k0, lane); break;
    case 8: check_item<KIND, 8>(D, opt, k0, lane); break;
    case 16: check_item<KIND, 16>(D, opt, k0, lane); break;
    case 32: check_item<KIND, 32>(D, opt, k0, lane); break;
    default: check_item<KIND, 64>(D, opt, k0, lane); break;
  }
}

// Items are taken from the queue a chunk at a time (one atomic per chunk): the
// queue counter is a single L2 address, and with one atomic per item its
// serialised updates (a few ns each over ~10^6 items) set the stage's time.
// The check stage's items are short and alike, so its chunks are longer.
constexpr int ROOT_CHUNK = 2;
constexpr int CHECK_CHUNK = 8;

// at least ROOT_WAVES wavefronts per SIMD: the pole loads come from L2 and need company to hide
#ifndef AHD_ROOT_WAVES
#define AHD_ROOT_WAVES 4
#endif
constexpr int ROOT_WAVES = AHD_ROOT_WAVES;
__global__ __launch_bounds__(STAGE_BLOCK) __attribute__((amdgpu_waves_per_eu(ROOT_WAVES))) void k_b_root(
    BatchArgs B, Options opt) {
  const int lane = threadIdx.x & (WAVE - 1);
  __shared__ double lds_all[STAGE_BLOCK / WAVE][ROOT_STAGE > 0 ? ROOT_STAGE : 1];
  double* lds = lds_all[threadIdx.x / WAVE];
  int staged = -1;   // the problem whose arrays the slice holds
  for (;;) {
    int first = 0;
    if (lane == 0) first = (int)atomicAdd(&B.counters[0], (unsigned)ROOT_CHUNK);
    first = __shfl(first, 0);
    if (first >= B.total_items) break;
    const int last = min(first + ROOT_CHUNK, B.total_items);
    for (int item = first; item < last; ++item) {
      const int p = find_problem(B.item_start, B.count, item);
      const ProbDesc D = B.descs[p];
      const int G = B.lanes[p];
      const int k = (item - B.item_start[p]) * (WAVE / G) + lane / G;
      const int ns = sorted_count(D);
      const int hot = G > 16 ? 0 : (2 * ns <= ROOT_STAGE ? 1 : (ns <= ROOT_STAGE ? 2 : 0));
      if (hot && staged != p) {
        // the slice is the wavefront's own: its LDS reads and writes run in
        // order, so only the compiler must not move them across the copy
        const Ws w = ws_view(D.ws, D.n);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int j = lane; j < ns; j += WAVE) {
          lds[j] = w.ds[j];
          if (hot == 1) lds[ns + j] = w.ch[j];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        staged = p;
      }
      const bool valid = k < D.n;
      switch (D.kind) {
        case KIND_ARROW:
        case KIND_HERM: root_kind<KIND_ARROW>(D, opt, G, k, lane, valid, hot, lds); break;   // HERM: the real arrowhead on |z|
        case KIND_DPR1: root_kind<KIND_DPR1>(D, opt, G, k, lane, valid, hot, lds); break;
        default: root_kind<KIND_SVD>(D, opt, G, k, lane, valid, hot, lds); break;
      }
    }
  }
}

__global__ __launch_bounds__(STAGE_BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_b_check(BatchArgs B,
                                                                                                 Options opt) {
  const int lane = threadIdx.x & (WAVE - 1);
  // the current problem and its items [p_lo, p_hi), kept across items: items
  // are short, and those of a chunk are consecutive, so the search runs about
  // once per chunk
  int p = 0, p_lo = 0, p_hi = 0;
  for (;;) {
    int first = 0;
    if (lane == 0) first = (int)atomicAdd(&B.counters[1], (unsigned)CHECK_CHUNK);
    first = __builtin_amdgcn_readfirstlane(first);
    if (first >= B.total_check) break;
    const int last = min(first + CHECK_CHUNK, B.total_check);
    for (int item = first; item < last; ++item) {
      if (item < p_lo || item >= p_hi) {
        p = find_problem(B.check_start, B.count, item);
        p_lo = B.check_start[p];
        p_hi = B.check_start[p + 1];
      }
      const ProbDesc D = B.descs[p];
      const int G = B.check_lanes[p];
      const int k0 = (item - p_lo) * (WAVE / G);
      switch (D.kind) {
        case KIND_ARROW:
        case KIND_HERM: check_kind<KIND_ARROW>(D, opt, G, k0, lane); break;   // HERM: the real arrowhead on |z|
        case KIND_DPR1: check_kind<KIND_DPR1>(D, opt, G, k0, lane); break;
        default: check_kind<KIND_SVD>(D, opt, G, k0, lane); break;
      }
    }
  }
}

// The repairs the check stage deferred (each problem keeps its own list in its
// workspace, as in the single-problem path): `per` blocks of REPAIR_BLOCK
// lanes per problem stride over that problem's list, each listed eigenvalue
// run by a whole block.  Blocks beyond a problem's list length skip the repairs.
constexpr int REPAIR_BLOCK = 256;

__global__ __launch_bounds__(REPAIR_BLOCK) void k_b_repair(BatchArgs B, Options opt, int per) {
  const int p = (int)blockIdx.x / per;
  const int x = (int)blockIdx.x - p * per;
  const ProbDesc D = B.descs[p];
  const Ws w = ws_view(D.ws, D.n);
  const uint32_t c = min(*repair_count(w), (uint32_t)D.n);
  const uint32_t* list = repair_list(w, D.n);
  for (uint32_t q = (uint32_t)x; q < c; q += (uint32_t)per) {
    const int k = (int)list[q];
    if (k < 0 || k >= D.n) continue;
    switch (D.kind) {
      case KIND_ARROW:
      case KIND_HERM: check_body<KIND_ARROW, REPAIR_BLOCK>(D, opt, k, threadIdx.x); break;
      case KIND_DPR1: check_body<KIND_DPR1, REPAIR_BLOCK>(D, opt, k, threadIdx.x); break;
      default: check_body<KIND_SVD, REPAIR_BLOCK>(D, opt, k, threadIdx.x); break;
    }
  }
  // a deflated arrowhead: the last of its `per` blocks places the deflated eigenpairs
  if (D.kind == KIND_ARROW && deflated_count(w) > 0) place_deflated_last(D, w, (uint32_t)per);
}

template <int KIND>
__device__ inline void vec_one(const ProbDesc& D, int t, int mode, VecFlatStage& L) {
  if (mode == 0) {
    vec_flat<KIND>(D, t, L);
  } else {
    const int row_tiles = (D.n + VEC_TILE - 1) / VEC_TILE;
    const int ct = t / row_tiles;
    if (mode == 2) vec_tile<KIND, 2, VEC_RPT>(D, t - ct * row_tiles, ct, VEC_COLS, L);
    else vec_tile<KIND, 1, VEC_RPT>(D, t - ct * row_tiles, ct, VEC_COLS, L);
  }
}

// every problem's vectors: its tiles are a contiguous range of blocks
__global__ __launch_bounds__(BLOCK) void k_b_vec(BatchArgs B) {
  __shared__ VecFlatStage L;
  const int p = B.vec_prob[blockIdx.x];
  const ProbDesc D = B.descs[p];
  const int t = (int)blockIdx.x - B.vec_start[p];
  const int mode = B.vec_mode[p];
  switch (D.kind) {
    case KIND_ARROW: vec_one<KIND_ARROW>(D, t, mode, L); break;
    case KIND_DPR1: vec_one<KIND_DPR1>(D, t, mode, L); break;
    case KIND_HERM: {   // complex row tiles at every n
      const int row_tiles = (D.n + VEC_TILE - 1) / VEC_TILE;
      const int ct = t / row_tiles;
      vec_tile_c<VEC_RPT>(D, t - ct * row_tiles, ct, VEC_COLS, L);
      break;
    }
    default: vec_one<KIND_SVD>(D, t, mode, L); break;
  }
}

// diagnostics: per problem, the six pass counters of the root and check stages
// summed over its eigenvalues, and the number of poles a pass visits
__global__ __launch_bounds__(BLOCK) void k_b_counters(BatchArgs B, long long* out) {
  __shared__ unsigned long long part[6];
  const ProbDesc D = B.descs[blockIdx.x];
  const Ws w = ws_view(D.ws, D.n);
  if (threadIdx.x < 6) part[threadIdx.x] = 0ull;
  __syncthreads();
  long long s[6] = {0, 0, 0, 0, 0, 0};
  for (int k = threadIdx.x; k < D.n; k += blockDim.x)
    for (int c = 0; c < 6; ++c) s[c] += w.cnt[6 * k + c];
  for (int c = 0; c < 6; ++c)
    if (s[c]) atomicAdd(&part[c], (unsigned long long)s[c]);
  __syncthreads();
  if (threadIdx.x < 6) out[7 * (int64_t)blockIdx.x + threadIdx.x] = (long long)part[threadIdx.x];
  if (threadIdx.x == 6) out[7 * (int64_t)blockIdx.x + 6] = reduced_m(w);
}

// a launch whose start and end events, when given, are stamped by the dispatch itself
template <typename F, typename... Args>
void launch_ev(F kern, dim3 grid, dim3 block, hipStream_t st, hipEvent_t e0, hipEvent_t e1, Args... args) {
  if (e0) hipExtLaunchKernelGGL(kern, grid, block, 0u, st, e0, e1, 0u, args...);
  else hipLaunchKernelGGL(kern, grid, block, 0, st, args...);
}

}  // namespace

// ---------------------------------------------------------------------------
// host side

struct arrow_batch_s {
  arrow_handle_t h;
  int64_t count;
  int flags;
  int32_t total_items, total_vec;
  int repair_per;       // k_b_repair blocks per problem
  Options opt;          // the handle's options when the plan was created
  void* dev;            // device block: counters, descriptors, tables, workspaces
  int own_dev;          // dev allocated by the plan
  size_t dev_bytes;
  std::vector<ProbDesc> descs;
  std::vector<int32_t> tabs;   // item_start (count+1), lanes (count), vec_start (count+1), vec_mode (count),
                               // check_start (count+1), check_lanes (count), vec_prob (one per vector tile)
  BatchArgs args;
  int persistent_blocks;
  hipGraph_t graph;
  hipGraphExec_t exec;
  int captured;
  hipEvent_t ev[10];    // ARROW_BATCH_TIMING: start and end of each of the five kernels
  int ev_made;
  int timed_runs;
  uint32_t magic;
};

static constexpr uint32_t BATCH_MAGIC = 0xBA7C4EDu;

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// vector tiles of one problem: complex row tiles (Hermitian), flat tiles of
// whole columns (n < VEC_TALL_MIN), or row tiles
static int64_t vec_tiles(const arrow_desc_t& a) {
  if (a.vec_off < 0) return 0;
  const int64_t n = a.n;
  if (a.kind != ARROW_KIND_HERM && n < VEC_TALL_MIN) {
    const int64_t c = vec_flat_cols(n);
    return (n + c - 1) / c;
  }
  return ((n + VEC_TILE - 1) / VEC_TILE) * ((n + VEC_COLS - 1) / VEC_COLS);
}

struct Layout {
  size_t off_desc, off_tab, off_ws, total;
  int64_t vec_total;
};

static Layout plan_layout(int64_t count, const arrow_desc_t* descs) {
  Layout L;
  L.vec_total = 0;
  for (int64_t p = 0; p < count; ++p) L.vec_total += vec_tiles(descs[p]);
  size_t off = 256;                                   // counters
  L.off_desc = off;
  off = align_up(off + (size_t)count * sizeof(ProbDesc), 256);
  L.off_tab = off;
  off = align_up(off + (size_t)(6 * count + 3 + L.vec_total) * sizeof(int32_t), 256);
  L.off_ws = off;
  for (int64_t p = 0; p < count; ++p) off += align_up(ws_doubles(descs[p].n) * sizeof(double), 256);
  L.total = off;
  return L;
}

static int check_desc(const arrow_desc_t& a) {
  if (a.kind < ARROW_KIND_ARROW || a.kind > ARROW_KIND_HERM) return 1;
  if (a.n < 1 || a.n > 46340) return 1;
  if (!(a.scalar - a.scalar == 0.0)) return 1;
  if (a.kind == ARROW_KIND_DPR1 && a.scalar == 0.0) return 1;
  const int64_t ms = a.kind == ARROW_KIND_DPR1 ? a.n : a.n - 1;
  if (ms > 0 && (a.d_off < 0 || a.z_off < 0)) return 1;
  if (a.lam_off < 0) return 1;
  if (a.kind == ARROW_KIND_SVD && a.left_off >= 0 && a.vec_off < 0) return 1;
  return 0;
}

extern "C" {

size_t arrow_batch_workspace_size(int64_t count, const arrow_desc_t* descs) {
  if (count < 1 || !descs) return 0;
  return plan_layout(count, descs).total;
}

int arrow_set_lanes_table(arrow_handle_t h, int scope, int32_t entries, const int32_t* n_max, const int32_t* lanes) {
  if (!valid(h)) return -1;
  if (scope != ARROW_SCHEDULE_SINGLE && scope != ARROW_SCHEDULE_BATCH) return -2;
  if (entries < 0 || entries > LANE_TABLE_MAX) return -3;
  if (entries == 0) {
    if (scope == ARROW_SCHEDULE_BATCH) default_batch_table(h);
    else h->ntab[scope] = 0;
    return ARROW_OK;
  }
  if (!n_max) return -4;
  if (!lanes) return -5;
  const int gmin = scope == ARROW_SCHEDULE_BATCH ? 4 : 1;
  for (int e = 0; e < entries; ++e) {
    const int g = lanes[e];
    if (g < gmin || g > 64 || (g & (g - 1)) != 0) return -5;
    if (n_max[e] < 1 || (e > 0 && n_max[e] <= n_max[e - 1])) return -4;
  }
  h->ntab[scope] = entries;
  for (int e = 0; e < entries; ++e) {
    h->tab_n[scope][e] = n_max[e];
    h->tab_g[scope][e] = lanes[e];
  }
  return ARROW_OK;
}

int arrow_batch_create(arrow_handle_t h, int64_t count, const arrow_desc_t* descs, const double* in_pool,
                       double* out_pool, uint32_t* info_pool, void* workspace, size_t workspace_bytes, int flags,
                       arrow_batch_t* plan) {
  if (!valid(h)) return -1;
  if (count < 1 || count > (int64_t)1 << 24) return -2;
  if (!descs) return -3;
  if (!in_pool) return -4;
  if (!out_pool) return -5;
  if (!plan) return -10;
  for (int64_t p = 0; p < count; ++p) {
    if (check_desc(descs[p])) return -3;
    if (descs[p].info_off >= 0 && !info_pool) return -6;
    // Hermitian vectors are complex: 16-byte aligned
    if (descs[p].kind == ARROW_KIND_HERM && descs[p].vec_off >= 0 && ((uintptr_t)(out_pool + descs[p].vec_off) & 15))
      return -3;
  }
  DeviceGuard g(h->device);
  const Layout L = plan_layout(count, descs);
  if (L.vec_total > INT32_MAX / 2) return -2;
  if (workspace && workspace_bytes < L.total) return -8;
  arrow_batch_s* b = new (std::nothrow) arrow_batch_s();
  if (!b) return ARROW_ERR_NOMEM;
  b->h = h;
  b->opt = h->opt;
  b->count = count;
  b->flags = flags;
  b->dev_bytes = L.total;
  if (workspace) {
    b->dev = workspace;
    b->own_dev = 0;
  } else {
    if (hipMalloc(&b->dev, L.total) != hipSuccess) {
      delete b;
      return ARROW_ERR_NOMEM;
    }
    b->own_dev = 1;
  }
  // queue order: decreasing n (stable), so the longest items are taken first
  std::vector<int64_t> order((size_t)count);
  for (int64_t p = 0; p < count; ++p) order[(size_t)p] = p;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t c) { return descs[a].n > descs[c].n; });
  b->descs.resize((size_t)count);
  b->tabs.assign((size_t)(6 * count + 3 + L.vec_total), 0);
  int32_t* item_start = b->tabs.data();
  int32_t* lanes = item_start + count + 1;
  int32_t* vec_start = lanes + count;
  int32_t* vec_mode = vec_start + count + 1;
  int32_t* check_start = vec_mode + count;
  int32_t* check_lanes = check_start + count + 1;
  int32_t* vec_prob = check_lanes + count;
  char* base = (char*)b->dev;
  size_t wsoff = L.off_ws;
  int64_t items = 0, vchunks = 0, citems = 0;
  for (int64_t q = 0; q < count; ++q) {
    const arrow_desc_t& a = descs[order[(size_t)q]];
    ProbDesc D{};
    D.kind = a.kind;
    D.n = a.n;
    D.d = in_pool + a.d_off;
    D.z = in_pool + a.z_off;
    D.neg = a.kind == ARROW_KIND_DPR1 && a.scalar < 0.0;
    D.scalar = D.neg ? -a.scalar : a.scalar;
    D.lam = out_pool + a.lam_off;
    D.V = a.vec_off >= 0 ? out_pool + a.vec_off : nullptr;
    D.ldv = a.n;
    D.U = (a.kind == ARROW_KIND_SVD && a.left_off >= 0) ? out_pool + a.left_off : nullptr;
    D.ldu = a.n;
    D.info = a.info_off >= 0 ? info_pool + a.info_off : nullptr;
    D.ws = (double*)(base + wsoff);
    wsoff += align_up(ws_doubles(a.n) * sizeof(double), 256);
    b->descs[(size_t)q] = D;
    const int G = batch_lanes(h, a.n);
    lanes[q] = G;
    item_start[q] = (int32_t)items;
    items += (a.n + (WAVE / G) - 1) / (WAVE / G);
    const int Gc = b->opt.check_lanes ? b->opt.check_lanes : G;
    check_lanes[q] = Gc;
    check_start[q] = (int32_t)citems;
    citems += (a.n + (WAVE / Gc) - 1) / (WAVE / Gc);
    vec_start[q] = (int32_t)vchunks;
    if (D.V && a.kind == ARROW_KIND_HERM) {
      vec_mode[q] = 1;
    } else if (D.V) {
      const int64_t n = a.n;
      if (n < VEC_TALL_MIN) {
        vec_mode[q] = 0;
      } else {
        const bool pair = (n % 2 == 0) && (((uintptr_t)D.V & 15) == 0) && (!D.U || (((uintptr_t)D.U & 15) == 0));
        vec_mode[q] = pair ? 2 : 1;
      }
    }
    for (int64_t t = vec_tiles(a); t > 0; --t) vec_prob[vchunks++] = (int32_t)q;
  }
  item_start[count] = (int32_t)items;
  vec_start[count] = (int32_t)vchunks;
  check_start[count] = (int32_t)citems;
  if (items > INT32_MAX / 2 || vchunks > INT32_MAX / 2 || citems > INT32_MAX / 2) {
    if (b->own_dev) (void)hipFree(b->dev);
    delete b;
    return -2;
  }
  b->total_items = (int32_t)items;
  b->repair_per = (int)std::max<int64_t>(1, 1024 / count);
  b->total_vec = (int32_t)vchunks;
  hipStream_t st = h->stream;
  if (hipMemcpyAsync(base + L.off_desc, b->descs.data(), (size_t)count * sizeof(ProbDesc), hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      hipMemcpyAsync(base + L.off_tab, b->tabs.data(), b->tabs.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                     st) != hipSuccess) {
    if (b->own_dev) (void)hipFree(b->dev);
    delete b;
    return ARROW_ERR_HIP;
  }
  BatchArgs& A = b->args;
  A.descs = (const ProbDesc*)(base + L.off_desc);
  A.item_start = (const int32_t*)(base + L.off_tab);
  A.lanes = A.item_start + count + 1;
  A.vec_start = A.lanes + count;
  A.vec_mode = A.vec_start + count + 1;
  A.check_start = A.vec_mode + count;
  A.check_lanes = A.check_start + count + 1;
  A.vec_prob = A.check_lanes + count;
  A.total_check = (int32_t)citems;
  A.counters = (uint32_t*)base;
  A.count = (int32_t)count;
  A.total_items = b->total_items;
  // persistent grid: enough resident wavefronts to fill every SIMD several times
  const int64_t want = (int64_t)h->cus * 4 * ROOT_WAVES * WAVE / STAGE_BLOCK;
  const int64_t need = ((int64_t)items * WAVE + STAGE_BLOCK - 1) / STAGE_BLOCK;
  b->persistent_blocks = (int)std::max<int64_t>(1, std::min(want, need));
  if ((flags & ARROW_BATCH_TIMING) && !(flags & ARROW_BATCH_GRAPH)) {
    b->ev_made = 1;
    for (int e = 0; e < 10; ++e)
      if (hipEventCreate(&b->ev[e]) != hipSuccess) b->ev_made = 0;
  }
  b->magic = BATCH_MAGIC;
  *plan = b;
  return ARROW_OK;
}

static int batch_launch(arrow_batch_s* b, hipStream_t st) {
  const BatchArgs A = b->args;
  const Options opt = b->opt;   // fixed at creation, so eager and graph runs agree
  const bool tm = b->ev_made && !(b->flags & ARROW_BATCH_GRAPH);
  auto ev = [&](int e) -> hipEvent_t { return tm ? b->ev[e] : nullptr; };
  launch_ev(k_b_prep, dim3((unsigned)b->count), dim3(BLOCK), st, ev(0), ev(1), A);
  launch_ev(k_b_root, dim3((unsigned)b->persistent_blocks), dim3(STAGE_BLOCK), st, ev(2), ev(3), A, opt);
  launch_ev(k_b_check, dim3((unsigned)b->persistent_blocks), dim3(STAGE_BLOCK), st, ev(4), ev(5), A, opt);
  launch_ev(k_b_repair, dim3((unsigned)(b->count * b->repair_per)), dim3(REPAIR_BLOCK), st, ev(6), ev(7), A, opt,
            b->repair_per);
  if (b->total_vec > 0) launch_ev(k_b_vec, dim3((unsigned)b->total_vec), dim3(BLOCK), st, ev(8), ev(9), A);
  else if (tm) { (void)hipEventRecord(b->ev[8], st); (void)hipEventRecord(b->ev[9], st); }
  if (tm) b->timed_runs += 1;
  return hipGetLastError() == hipSuccess ? ARROW_OK : ARROW_ERR_HIP;
}

int arrow_batch_run(arrow_batch_t b) {
  if (!b || b->magic != BATCH_MAGIC || !valid(b->h)) return -1;
  DeviceGuard g(b->h->device);
  hipStream_t st = b->h->stream;
  (void)hipGetLastError();
  if (!(b->flags & ARROW_BATCH_GRAPH)) return batch_launch(b, st);
  if (!b->captured) {
    // capture on a private stream: the legacy null stream cannot be captured
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return ARROW_ERR_HIP;
    int rc = ARROW_OK;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = ARROW_ERR_HIP;
    if (rc == ARROW_OK) {
      rc = batch_launch(b, cap);
      if (hipStreamEndCapture(cap, &b->graph) != hipSuccess) rc = ARROW_ERR_HIP;
    }
    if (rc == ARROW_OK && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
      rc = ARROW_ERR_HIP;
    (void)hipStreamDestroy(cap);
    if (rc != ARROW_OK) return rc;
    b->captured = 1;
  }
  return hipGraphLaunch(b->exec, st) == hipSuccess ? ARROW_OK : ARROW_ERR_HIP;
}

int arrow_batch_timing(arrow_batch_t b, double* ms) {
  if (!b || b->magic != BATCH_MAGIC || !valid(b->h)) return -1;
  if (!ms) return -2;
  if (!b->ev_made || b->timed_runs < 1) return ARROW_ERR_STATE;
  DeviceGuard g(b->h->device);
  if (hipEventSynchronize(b->ev[9]) != hipSuccess) return ARROW_ERR_HIP;
  for (int k = 0; k < 5; ++k) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, b->ev[2 * k], b->ev[2 * k + 1]) != hipSuccess) return ARROW_ERR_HIP;
    ms[k] = (double)t;
  }
  return ARROW_OK;
}

int arrow_batch_counters(arrow_batch_t b, double* out) {
  if (!b || b->magic != BATCH_MAGIC || !valid(b->h)) return -1;
  if (!out) return -2;
  DeviceGuard g(b->h->device);
  long long* dev = nullptr;
  const size_t bytes = (size_t)b->count * 7 * sizeof(long long);
  if (hipMalloc((void**)&dev, bytes) != hipSuccess) return ARROW_ERR_NOMEM;
  std::vector<long long> host((size_t)b->count * 7);
  hipLaunchKernelGGL(k_b_counters, dim3((unsigned)b->count), dim3(BLOCK), 0, b->h->stream, b->args, dev);
  int rc = hipGetLastError() == hipSuccess ? ARROW_OK : ARROW_ERR_HIP;
  if (rc == ARROW_OK && (hipStreamSynchronize(b->h->stream) != hipSuccess ||
                         hipMemcpy(host.data(), dev, bytes, hipMemcpyDeviceToHost) != hipSuccess))
    rc = ARROW_ERR_HIP;
  (void)hipFree(dev);
  if (rc != ARROW_OK) return rc;
  for (int c = 0; c < 7; ++c) out[c] = 0.0;
  for (int64_t p = 0; p < b->count; ++p) {
    const double m = (double)host[(size_t)(7 * p + 6)];
    for (int c = 0; c < 6; ++c) out[c] += m * (double)host[(size_t)(7 * p + c)];
    out[6] += (double)b->descs[(size_t)p].n;
  }
  return ARROW_OK;
}

int arrow_batch_destroy(arrow_batch_t b) {
  if (!b || b->magic != BATCH_MAGIC) return -1;
  DeviceGuard g(b->h->device);
  (void)hipStreamSynchronize(b->h->stream);
  if (b->ev_made)
    for (int e = 0; e < 10; ++e) (void)hipEventDestroy(b->ev[e]);
  if (b->captured) {
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
  }
  if (b->own_dev) (void)hipFree(b->dev);
  b->magic = 0;
  delete b;
  return ARROW_OK;
}

int arrow_solve_sequential(arrow_handle_t h, int64_t count, const arrow_desc_t* descs, const double* in_pool,
                           double* out_pool, uint32_t* info_pool) {
  if (!valid(h)) return -1;
  if (count < 1) return -2;
  if (!descs) return -3;
  if (!in_pool) return -4;
  if (!out_pool) return -5;
  int64_t nmax = 1;
  for (int64_t p = 0; p < count; ++p) {
    if (check_desc(descs[p])) return -3;
    if (descs[p].info_off >= 0 && !info_pool) return -6;
    nmax = std::max<int64_t>(nmax, descs[p].n);
  }
  DeviceGuard g(h->device);
  const int rc = ensure_ws(h, ws_doubles(nmax));
  if (rc) return rc;
  for (int64_t p = 0; p < count; ++p) {
    const arrow_desc_t& a = descs[p];
    ProbDesc D{};
    D.kind = a.kind;
    D.n = a.n;
    D.d = in_pool + a.d_off;
    D.z = in_pool + a.z_off;
    D.neg = a.kind == ARROW_KIND_DPR1 && a.scalar < 0.0;
    D.scalar = D.neg ? -a.scalar : a.scalar;
    D.lam = out_pool + a.lam_off;
    D.V = a.vec_off >= 0 ? out_pool + a.vec_off : nullptr;
    D.ldv = a.n;
    D.U = (a.kind == ARROW_KIND_SVD && a.left_off >= 0) ? out_pool + a.left_off : nullptr;
    D.ldu = a.n;
    D.info = a.info_off >= 0 ? info_pool + a.info_off : nullptr;
    D.ws = h->ws;
    const int r = launch_single(h, D);
    if (r) return r;
  }
  return ARROW_OK;
}

int arrow_solve_batched(arrow_handle_t h, int64_t count, const arrow_desc_t* descs, const double* in_pool,
                        double* out_pool, uint32_t* info_pool) {
  arrow_batch_t b = nullptr;
  int rc = arrow_batch_create(h, count, descs, in_pool, out_pool, info_pool, nullptr, 0, 0, &b);
  if (rc != ARROW_OK) return rc;
  rc = arrow_batch_run(b);
  const int rc2 = arrow_batch_destroy(b);
  return rc != ARROW_OK ? rc : rc2;
}

}  // extern "C"
