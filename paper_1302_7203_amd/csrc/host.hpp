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
  hipEvent_t ev[6];
  int ev_made;
  int have_last;      // a timed call has been launched
  int64_t last_n;
  size_t lds_max;     // bytes of dynamic LDS one block may use
  int cus;            // compute units of the device
  int ntab;           // batched schedule: lanes per eigenvalue by order n
  int32_t tab_n[LANE_TABLE_MAX];
  int32_t tab_g[LANE_TABLE_MAX];
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

// lanes per eigenvalue for a single problem: about 8 pole terms per lane
static inline int auto_lanes(int64_t n) {
  int64_t want = n / 8;
  int g = 1;
  while (g < 64 && g < want) g <<= 1;
  return g;
}

// all launches of one single-problem solve (defined with the single-problem kernels)
int launch_single(arrow_handle_t h, const ahd::ProbDesc& D);

// lanes per eigenvalue for a problem of order n inside a batch
static inline int table_lanes(const arrow_handle_s* h, int64_t n) {
  for (int e = 0; e < h->ntab; ++e)
    if (n <= h->tab_n[e]) return h->tab_g[e];
  return 64;
}
