// Host-side helpers shared by the single-structure and batched entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "pcv_internal.h"

namespace pcv {

inline int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Owner of a set of device allocations released together.
struct DevMem {
  std::vector<void*> ptrs;
  hipError_t alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

inline int num_cus(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 256;
  return prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
}

// Lanes per landmark for a tiling, or 0 if it cannot hold n atoms.
inline int team_size(int n, EngineCfg c) {
  const int ts = std::max(16, next_pow2((n + c.apt - 1) / c.apt));
  return ts > c.wg ? 0 : ts;
}

// Per-landmark cost model (lane-instructions) used to rank tilings: lanes per
// landmark times (per-atom work + reduction + solve).
inline double landmark_cost(int n, EngineCfg c, int ts) {
  (void)n;
  const double red = 9.0 * 3.0 * std::log2((double)std::min(ts, 64)) + (ts > 64 ? 60.0 : 0.0);
  const double regs_penalty = (c.wg == 512) ? 1.15 : 1.0;
  return ts * (c.apt * 30.0 + red + 320.0) * regs_penalty;
}

// ---- split-role engine planning
// Two landmark buffers of one pipeline batch must fit in this much LDS.
constexpr size_t kE2LdsBudget = 124 * 1024;

// Landmarks per pipeline batch: enough atoms in flight per workgroup
// (about 4096 per batch), limited by LDS and by the 64 solver lanes.
inline int e2_batch(int n_pad, bool fp64) {
  const size_t per = (size_t)3 * n_pad * (fp64 ? 8 : 4);
  const int bmax = (int)(kE2LdsBudget / (2 * per));
  if (bmax < 1) return 0;
  const int want = std::max(1, (4096 + n_pad - 1) / n_pad);
  return std::min(std::min(want, bmax), 64);
}

inline bool e2_lds_ok(int n_pad, int B, bool fp64) {
  return B >= 1 && B <= 64 && (size_t)2 * B * 3 * n_pad * (fp64 ? 8 : 4) <= kE2LdsBudget;
}

// Lanes per landmark in the correlation stage: the smallest group that holds
// n_pad atoms within aptc per lane, preferring no more groups than landmarks
// per batch (64 * ncw = all correlation lanes).  0 if none fits.
inline int e2_group(int n_pad, Engine2Cfg c, int B) {
  const int full = 64 * c.ncw;
  const int gs[4] = {16, 32, 64, full};
  int first = 0;
  for (int g : gs) {
    if ((n_pad + g - 1) / g > c.aptc) continue;
    if (first == 0) first = g;
    if (full / g <= B) return g;
  }
  return first;
}

inline bool e2_group_ok(int g, Engine2Cfg c) { return g == 16 || g == 32 || g == 64 || g == 64 * c.ncw; }

inline bool e2_fits(int n_pad, Engine2Cfg c) {
  const int gl = 64 * (7 - c.ncw);
  return (n_pad + gl - 1) / gl <= c.aptg;
}

}  // namespace pcv
