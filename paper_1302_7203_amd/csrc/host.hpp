// Host-side state shared by the single-problem and batched entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/arrow.h"
#include "bodies.hpp"

constexpr int LANE_TABLE_MAX = 16;

struct arrow_handle_s {
  int device;
  hipStream_t stream;
  double* ws;
  size_t ws_cap;      // doubles
  ahd::Options opt;
  int lanes;          // single problems: 0 = automatic, else lanes per eigenvalue
  int timing;         // record stage events
  // stage events of the two most recent timed calls, used in turn, so that a
  // caller may read one call's stages after queuing the next
  hipEvent_t ev[2][6];
  int ev_made;
  int ev_set;         // set of the most recent timed call
  int timed_calls;    // timed calls launched so far, up to 2
  int64_t last_n;
  double* last_ws;    // workspace of the most recent single-problem call (the handle's, or the scratch)
  size_t lds_max;     // bytes of dynamic LDS one block may use
  int cus;            // compute units of the device
  // lanes per eigenvalue by order n: [ARROW_SCHEDULE_SINGLE] for single
  // problems (empty: the built-in rule), [ARROW_SCHEDULE_BATCH] inside batches
  int ntab[2];
  int32_t tab_n[2][LANE_TABLE_MAX];
  int32_t tab_g[2][LANE_TABLE_MAX];
  void* blas;         // rocBLAS handle of tridiag_eig's GEMMs, made on first use
  void* td_ws;        // tridiag_eig's device buffers (grown on demand, kept)
  size_t td_cap;      // bytes
  uint32_t magic;
};

static constexpr uint32_t HANDLE_MAGIC = 0xA770E16u;

static inline bool valid(arrow_handle_t h) { return h && h->magic == HANDLE_MAGIC; }

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

static inline int ensure_ws(arrow_handle_t h, size_t doubles) {
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

static inline int table_lookup(const arrow_handle_s* h, int scope, int64_t n, int fallback) {
  for (int e = 0; e < h->ntab[scope]; ++e)
    if (n <= h->tab_n[scope][e]) return h->tab_g[scope][e];
  return fallback;
}

// lanes per eigenvalue for a single problem: a fixed option, else the tuned
// table, else about 8 pole terms per lane
static inline int single_lanes(const arrow_handle_s* h, int64_t n) {
  if (h->lanes) return h->lanes;
  int g = 1;
  while (g < 64 && g < n / 8) g <<= 1;
  return table_lookup(h, ARROW_SCHEDULE_SINGLE, n, g);
}

// all launches of one single-problem solve (defined with the single-problem kernels)
int launch_single(arrow_handle_t h, const ahd::ProbDesc& D);

// frees what tridiag_eig keeps in the handle
void tridiag_release(arrow_handle_t h);

// lanes per eigenvalue for a problem of order n inside a batch
static inline int batch_lanes(const arrow_handle_s* h, int64_t n) {
  return table_lookup(h, ARROW_SCHEDULE_BATCH, n, 64);
}

// the built-in batched table
static inline void default_batch_table(arrow_handle_s* h) {
  static const int32_t tn[5] = {24, 48, 96, 192, 2147483647};
  static const int32_t tg[5] = {4, 8, 16, 32, 64};
  h->ntab[ARROW_SCHEDULE_BATCH] = 5;
  for (int e = 0; e < 5; ++e) {
    h->tab_n[ARROW_SCHEDULE_BATCH][e] = tn[e];
    h->tab_g[ARROW_SCHEDULE_BATCH][e] = tg[e];
  }
}
