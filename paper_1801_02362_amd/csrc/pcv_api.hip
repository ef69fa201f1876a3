// C ABI of the path-CV library (include/pcv.h): handle, planning, Algorithm 1
// and Algorithm 2 entry points, batched walkers.  Host code only; kernels
// live in pcv_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pcv.h"
#include "pcv_host_util.h"
#include "pcv_internal.h"

using namespace pcv;

namespace {

constexpr int kMaxAtomsF32 = 512 * 16;
constexpr int kMaxAtomsF64 = 256 * 8;
// Largest structure (padded atoms) engine 4 holds; engine 3 takes larger
// FP32 structures.
constexpr int kEngine4MaxAtoms = 2048;

struct Plan {
  int engine = 1;
  EngineCfg cfg{256, 1};    // engine 1
  int ts = 16;
  Engine2Cfg c2{0, 0};      // engine 2
  int g = 0, B = 1, lbuf = 0;
  int bpw = 0;              // engines 3 and 5: 256-atom blocks per worker wave
  int spw = 0;              // engine 4: units per worker wave (B = landmark lanes K)
  int grid = 0;
  int n_items = 0;
  size_t lds = 0;
};

}  // namespace

// ============================================================ single handle
// Serial numbers of handles: with the plan version they name the handle's
// current device buffers (a host address can be reused after destruction).
static std::atomic<unsigned long long> g_handle_serial{0};

// Fixed device scratch for pcv_eval_properties_noalloc: one array per GPU
// (the module's own copy on every device it is loaded on), held until the
// process ends.  Host code never passes `scratch` itself to a kernel (in host
// code the name stands for a host-side placeholder); it uses the device
// address from hipGetSymbolAddress, taken once per device.
constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// With `device` current: record the address of this device's scratch array.
static hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

static void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

struct pcv_handle {
  unsigned long long serial = 0;
  pcv_options opt{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  bool fp64 = false;
  int n = 0, n_pad = 0, L = 0;
  double lam = 0.0;
  int cus = 256;
  DevMem mem;      // landmark-sized buffers (reallocated on load)
  DevMem pmem;     // plan-sized buffers (partials, descriptors)
  // landmarks
  void* A = nullptr;
  double *ca = nullptr, *Ga = nullptr, *q = nullptr, *w = nullptr;
  // frame
  double* xw = nullptr;
  float* xw32 = nullptr;   // FP32 handles: [3][n_x] copy of xw for engine 3
  int n_x = 0;
  double* Gx = nullptr;
  double* Gx32 = nullptr;
  double* xres = nullptr;
  int* status = nullptr;
  double* corr = nullptr;       // [3 * n_pad / 64][2]: rounding-correction shares of the merges
  double* corr_prop = nullptr;  // [kPropsMax][3 n / 256]: the same for the property maps
  unsigned* close_ticket = nullptr;   // arrival counter of the close merge (zero between launches)
  // close structure
  double *y64 = nullptr, *Gy = nullptr, *Fxy = nullptr, *lamxy = nullptr, *qxy = nullptr,
         *Rxy = nullptr, *Dxy = nullptr, *Rsave = nullptr, *gtmp = nullptr, *scratch_sz = nullptr;
  int *flag = nullptr, *init = nullptr, *force = nullptr;
  long long* counters = nullptr;
  // plan
  Plan plan;
  bool user_plan = false;
  double* hdr = nullptr;
  void* vec = nullptr;
  double* xuv = nullptr;   // engine 4: per-item XU / XV sums of approximate steps
  Problem* d_prob = nullptr;    // [3]: EXACT, EXACT_SAVE, APPROX
  Item* d_items = nullptr;
  int* d_wgoff = nullptr;
  PrepArgs* d_prep = nullptr;   // Algorithm 1 prep arguments (one problem)
  int plan_version = 0;
  // neighbour list (Section 2): members, their compact landmark set and its
  // work items (the engine configuration is the full set's)
  // property maps: rotations and distances of their exact pass, scratch
  double *Rprop = nullptr, *Dprop = nullptr, *Wprop = nullptr, *part_prop = nullptr;
  DevMem propmem;
  // separate displacement weights (w != w'; off while wd is null): the
  // weights, per-landmark statistics and the three-pass scratch
  DevMem f2mem;
  double *wd = nullptr, *Gaw = nullptr, *mua = nullptr, *Caa = nullptr, *xc2 = nullptr, *fs2 = nullptr,
         *Rl2 = nullptr, *Gl2 = nullptr, *Rmu2 = nullptr, *cw2 = nullptr, *pw2 = nullptr, *part2 = nullptr,
         *D2 = nullptr;
  int nl_M = 0, nl_stride = 0;
  long long nl_step = 0;
  DevMem nlmem, nlpmem;
  int* nl_members = nullptr;
  void* A_nl = nullptr;
  double *ca_nl = nullptr, *Ga_nl = nullptr, *q_nl = nullptr, *Rsave_nl = nullptr, *dfull = nullptr;
  double* hdr_nl = nullptr;
  void* vec_nl = nullptr;
  Problem* d_prob_nl = nullptr;   // [3]: EXACT, EXACT_SAVE, APPROX
  Item* d_items_nl = nullptr;
  int* d_wgoff_nl = nullptr;
  PrepArgs* d_prep_nl = nullptr;
  int grid_nl = 0, items_nl = 0;
  // graphs
  struct GraphEntry {
    const void* key[7];
    int version;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  // kernel timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
  double timed_ms = 0.0;
  long long timed_launches = 0;
  std::string err;
};

static pcv_status fail(pcv_handle* h, pcv_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

static pcv_status hip_fail(pcv_handle* h, hipError_t e, const char* where) {
  return fail(h, e == hipErrorOutOfMemory ? PCV_ENOMEM : PCV_EHIP,
              std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(h, expr)                                  \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) return hip_fail((h), _e, #expr); \
  } while (0)

static void collect_timing(pcv_handle* h);

// FP32 engines 2-5 contract with w x_c rounded to FP32 (see Problem::x_rounded).
static bool x_rounded(const pcv_handle* h) { return !h->fp64 && h->plan.engine != 1; }

static void drop_graphs(pcv_handle* h) {
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
  h->graphs.clear();
}

extern "C" void pcv_default_options(pcv_options* opt) {
  if (!opt) return;
  opt->device = 0;
  opt->stream = nullptr;
  opt->precision = PCV_FP32;
  opt->eps = 0.01;
  opt->use_graph = 0;
}

extern "C" int pcv_max_atoms(int precision) {
  return precision == PCV_FP64 ? kMaxAtomsF64 : kMaxAtomsF32;
}

extern "C" pcv_status pcv_create(pcv_handle** out, const pcv_options* opt) {
  if (!out) return PCV_EINVAL;
  *out = nullptr;
  pcv_options o;
  pcv_default_options(&o);
  if (opt) o = *opt;
  if (o.precision != PCV_FP32 && o.precision != PCV_FP64) return PCV_EINVAL;
  if (std::isnan(o.eps)) return PCV_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || o.device < 0 || o.device >= ndev) return PCV_EHIP;
  if (hipSetDevice(o.device) != hipSuccess) return PCV_EHIP;
  pcv_handle* h = new pcv_handle();
  h->serial = ++g_handle_serial;
  h->opt = o;
  h->fp64 = (o.precision == PCV_FP64);
  h->stream = (hipStream_t)o.stream;
  h->cus = num_cus(o.device);
  if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete h;
    return PCV_EHIP;
  }
  if (engine_init_attributes() != hipSuccess || engine2_init_attributes() != hipSuccess ||
      scratch_init(o.device) != hipSuccess) {
    (void)hipStreamDestroy(h->cap_stream);
    delete h;
    return PCV_EHIP;
  }
  *out = h;
  return PCV_OK;
}

extern "C" pcv_status pcv_destroy(pcv_handle* h) {
  if (!h) return PCV_OK;
  (void)hipSetDevice(h->opt.device);
  (void)hipStreamSynchronize(h->stream);
  collect_timing(h);
  drop_graphs(h);
  h->f2mem.release();
  h->propmem.release();
  h->nlpmem.release();
  h->nlmem.release();
  h->pmem.release();
  h->mem.release();
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  delete h;
  return PCV_OK;
}

static pcv_status build_nl_plan(pcv_handle* h, const Problem& full);

// Build (or rebuild) work items and problem descriptors for the current plan.
static pcv_status build_plan(pcv_handle* h) {
  Plan& p = h->plan;
  // Work-item granularity: a team's landmark (engine 1) or a batch (engine 2).
  const int unit = (p.engine == 2 || p.engine == 4) ? p.B : ((p.engine == 3 || p.engine == 5) ? 1 : p.cfg.wg / p.ts);
  const int units = (h->L + unit - 1) / unit;
  if (!h->user_plan || p.n_items <= 0) {
    const int cap = (p.engine >= 2 || p.cfg.wg >= 512) ? h->cus : 2 * h->cus;
    p.n_items = std::max(1, std::min(units, cap));
  }
  if (p.engine == 5) {
    // Engine 5 addresses an item through one range-checked buffer
    // descriptor, whose offsets must stay below 2 GiB.
    const long long lm_bytes = 12LL * h->n_pad;
    const long long per_item = (1LL << 30) / lm_bytes;
    p.n_items = std::max(p.n_items, (int)((h->L + per_item - 1) / per_item));
  }
  p.n_items = std::min(p.n_items, units);
  p.n_items = std::min(p.n_items, kMaxCloseSlots);
  p.grid = p.n_items;
  if (p.engine == 2) {
    p.lbuf = p.B * 3 * h->n_pad * (h->fp64 ? 8 : 4);
    p.lds = engine2_lds_bytes((size_t)p.lbuf, p.B);
  } else if (p.engine == 3 || p.engine == 4 || p.engine == 5) {
    p.lds = 0;   // static LDS
  } else {
    p.lds = engine_lds_bytes(p.cfg, p.ts, h->fp64);
  }
  h->pmem.release();
  const size_t n_slots = (size_t)p.n_items;
  HIP_TRY(h, h->pmem.alloc((void**)&h->hdr, n_slots * 4 * sizeof(double)));
  HIP_TRY(h, h->pmem.alloc(&h->vec, n_slots * (h->fp64 ? partial_bytes<double>(h->n_pad)
                                                       : partial_bytes<float>(h->n_pad))));
  h->xuv = nullptr;
  if (p.engine == 4 && !h->fp64)
    HIP_TRY(h, h->pmem.alloc((void**)&h->xuv, n_slots * 18 * sizeof(double)));
  HIP_TRY(h, h->pmem.alloc((void**)&h->d_prob, 4 * sizeof(Problem)));
  HIP_TRY(h, h->pmem.alloc((void**)&h->d_items, (size_t)p.n_items * sizeof(Item)));
  HIP_TRY(h, h->pmem.alloc((void**)&h->d_wgoff, (size_t)(p.grid + 1) * sizeof(int)));
  HIP_TRY(h, h->pmem.alloc((void**)&h->d_prep, sizeof(PrepArgs)));
  PrepArgs pa{0, h->w, h->xw, h->Gx, h->Gx32, h->xres, h->status, h->counters, h->n, h->n_pad, h->L};
  pa.xw32 = h->xw32;
  pa.n_x = h->n_x;
  HIP_TRY(h, hipMemcpy(h->d_prep, &pa, sizeof(pa), hipMemcpyHostToDevice));
  std::vector<Item> items(p.n_items);
  std::vector<int> wgoff(p.grid + 1);
  for (int k = 0; k < p.n_items; ++k) {
    items[k].prob = 0;
    const int u0 = (int)((long long)k * units / p.n_items);
    const int u1 = (int)((long long)(k + 1) * units / p.n_items);
    items[k].i0 = std::min(h->L, u0 * unit);
    items[k].i1 = std::min(h->L, u1 * unit);
    items[k].slot = k;
    wgoff[k] = k;
  }
  wgoff[p.grid] = p.n_items;
  Problem base{};
  base.A = h->A;
  base.ca = h->ca;
  base.Ga = h->Ga;
  base.q = h->q;
  base.w = h->w;
  base.xw = h->xw;
  base.Gx = h->Gx;
  base.Rxy = h->Rxy;
  base.Rsave = h->Rsave;
  base.hdr = h->hdr;
  base.vec = h->vec;
  base.fallbacks = h->counters + CNT_FALLBACK;
  base.Gx32 = h->Gx32;
  base.xres = h->xres;
  base.bsz = p.B;
  base.cg = p.g;
  base.n = h->n;
  base.n_pad = h->n_pad;
  base.L = h->L;
  base.ts = p.ts;
  base.n_slots = p.n_items;
  base.out_off = 0;
  base.out_idx = 0;
  base.lam = h->lam;
  base.xw32 = h->xw32;
  base.n_x = h->n_x;
  base.x_rounded = x_rounded(h) ? 1 : 0;
  base.corr = h->corr;
  base.xuv = h->xuv;
  // Entry 3: the property maps' exact pass (rotations saved to their own buffer).
  Problem props_prob = base;
  props_prob.Rsave = h->Rprop;
  Problem probs[4] = {base, base, base, props_prob};
  HIP_TRY(h, hipMemcpy(h->d_prob, probs, sizeof(probs), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_items, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_wgoff, wgoff.data(), wgoff.size() * sizeof(int), hipMemcpyHostToDevice));
  h->plan_version++;
  drop_graphs(h);
  if (h->nl_M > 0) {
    pcv_status s = build_nl_plan(h, base);
    if (s != PCV_OK) return s;
  }
  return PCV_OK;
}

// Work items and descriptors of the neighbour-list set (M landmarks in the
// compact buffers), with the full set's engine configuration; `full` is the
// full set's problem descriptor (frame buffers, lambda, tiling).
static pcv_status build_nl_plan(pcv_handle* h, const Problem& full) {
  const Plan& p = h->plan;
  const int M = h->nl_M;
  // Engine 4 on the short member set: fewer landmark lanes per step, so that
  // up to 64 workgroups share the M members (the lanes per step are a
  // per-problem value; the launch's units per worker stay the plan's).
  const int K_nl = p.engine == 4 ? std::max(1, std::min(p.B, M / 64)) : p.B;
  const int unit = (p.engine == 2 || p.engine == 4) ? K_nl : ((p.engine == 3 || p.engine == 5) ? 1 : p.cfg.wg / p.ts);
  const int units = (M + unit - 1) / unit;
  const int cap = (p.engine >= 2 || p.cfg.wg >= 512) ? h->cus : 2 * h->cus;
  const int n_items = std::max(1, std::min(units, cap));
  h->nlpmem.release();
  HIP_TRY(h, h->nlpmem.alloc((void**)&h->hdr_nl, (size_t)n_items * 4 * sizeof(double)));
  HIP_TRY(h, h->nlpmem.alloc(&h->vec_nl, (size_t)n_items * (h->fp64 ? partial_bytes<double>(h->n_pad)
                                                                     : partial_bytes<float>(h->n_pad))));
  HIP_TRY(h, h->nlpmem.alloc((void**)&h->d_prob_nl, 3 * sizeof(Problem)));
  HIP_TRY(h, h->nlpmem.alloc((void**)&h->d_items_nl, (size_t)n_items * sizeof(Item)));
  HIP_TRY(h, h->nlpmem.alloc((void**)&h->d_wgoff_nl, (size_t)(n_items + 1) * sizeof(int)));
  HIP_TRY(h, h->nlpmem.alloc((void**)&h->d_prep_nl, sizeof(PrepArgs)));
  PrepArgs pa{0, h->w, h->xw, h->Gx, h->Gx32, h->xres, h->status, h->counters, h->n, h->n_pad, M};
  pa.xw32 = h->xw32;
  pa.n_x = h->n_x;
  HIP_TRY(h, hipMemcpy(h->d_prep_nl, &pa, sizeof(pa), hipMemcpyHostToDevice));
  std::vector<Item> items(n_items);
  std::vector<int> wgoff(n_items + 1);
  for (int k = 0; k < n_items; ++k) {
    const int u0 = (int)((long long)k * units / n_items);
    const int u1 = (int)((long long)(k + 1) * units / n_items);
    items[k] = Item{0, std::min(M, u0 * unit), std::min(M, u1 * unit), k};
    wgoff[k] = k;
  }
  wgoff[n_items] = n_items;
  Problem b = full;
  b.xuv = nullptr;   // the list set's close merge takes the two-stage path
  b.A = h->A_nl;
  b.ca = h->ca_nl;
  b.Ga = h->Ga_nl;
  b.q = h->q_nl;
  b.Rsave = h->Rsave_nl;
  b.hdr = h->hdr_nl;
  b.vec = h->vec_nl;
  b.L = M;
  b.bsz = K_nl;
  b.n_slots = n_items;
  Problem probs[3] = {b, b, b};
  HIP_TRY(h, hipMemcpy(h->d_prob_nl, probs, sizeof(probs), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_items_nl, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->d_wgoff_nl, wgoff.data(), wgoff.size() * sizeof(int), hipMemcpyHostToDevice));
  h->grid_nl = n_items;
  h->items_nl = n_items;
  h->plan_version++;
  drop_graphs(h);
  return PCV_OK;
}

static bool default_plan2(pcv_handle* h) {
  const int B = e2_batch(h->n_pad, h->fp64);
  if (B == 0) return false;
  int nw[16], ac[16], ag[16], cnt = 0;
  engine2_configs(h->fp64, nw, ac, ag, &cnt);
  for (int k = 0; k < cnt; ++k) {
    const Engine2Cfg c{nw[k], ac[k], ag[k]};
    if (!e2_fits(h->n_pad, c)) continue;
    const int g = e2_group(h->n_pad, c, B);
    if (g == 0) continue;
    h->plan.engine = 2;
    h->plan.c2 = c;
    h->plan.g = g;
    h->plan.B = B;
    h->plan.cfg = EngineCfg{512, c.aptc};
    h->plan.ts = g;
    return true;
  }
  return false;
}

// Engine 3 for large FP32 structures: every worker wave owns at most bpw
// blocks of 256 atoms.
static int e3_bpw_for(int n_pad) {
  const int nblk = (n_pad + 255) / 256;
  for (int bpw = 1; bpw <= 4; ++bpw)
    if (nblk <= engine3_max_blocks(bpw)) return bpw;
  return 0;
}

// Three units per worker and the most landmark lanes when the landmark set
// is long enough to give most CUs an item; otherwise two units per worker
// and fewer lanes, so that at least 64 items (workgroups) share the work
// (measured at 150-1,000 atoms x 300-500 landmarks: 8-11 % shorter steps).
static bool default_plan4(pcv_handle* h) {
  if (h->fp64 || h->n_pad > kEngine4MaxAtoms) return false;
  int spw = 3;
  int K = engine4_lanes(h->n_pad, 3);
  if (K < 1) return false;
  if ((long long)h->L < 200LL * K) {
    const int K2 = engine4_lanes(h->n_pad, 2);
    if (K2 >= 1) {
      spw = 2;
      K = std::max(1, std::min(K2, h->L / 64));
    }
  }
  h->plan.engine = 4;
  h->plan.spw = spw;
  h->plan.B = K;
  h->plan.cfg = EngineCfg{512, 4 * spw};
  h->plan.ts = 0;
  return true;
}

// Structures above engine 4's range: engine 5 (register-stream workers)
// while the structure fits three blocks per worker, engine 3 (LDS copy ring)
// at four.
static bool default_plan3(pcv_handle* h) {
  if (h->fp64 || h->n_pad <= kEngine4MaxAtoms) return false;
  const int bpw = e3_bpw_for(h->n_pad);
  if (bpw == 0) return false;
  h->plan.engine = bpw <= 3 ? 5 : 3;
  h->plan.bpw = bpw;
  h->plan.cfg = EngineCfg{512, 4 * bpw};
  h->plan.ts = 0;
  return true;
}

static void default_plan(pcv_handle* h) {
  h->plan.n_items = 0;
  h->user_plan = false;
  if (default_plan4(h)) return;
  if (default_plan3(h)) return;
  if (default_plan2(h)) return;
  h->plan.engine = 1;
  EngineCfg menu[16];
  int cnt = 0;
  engine_configs(h->fp64, menu, &cnt);
  double best = 1e300;
  for (int k = 0; k < cnt; ++k) {
    const int ts = team_size(h->n, menu[k]);
    if (ts == 0) continue;
    const double c = landmark_cost(h->n, menu[k], ts);
    if (c < best) {
      best = c;
      h->plan.cfg = menu[k];
      h->plan.ts = ts;
    }
  }
  h->plan.n_items = 0;
  h->user_plan = false;
}

extern "C" pcv_status pcv_load_landmarks(pcv_handle* h, int n_atoms, int n_landmarks, const void* coords,
                                         const double* q, const double* w, double lambda) {
  if (!h) return PCV_EINVAL;
  if (!coords || n_atoms < 1 || n_landmarks < 1) return fail(h, PCV_EINVAL, "bad sizes or null coords");
  if (n_atoms > pcv_max_atoms(h->opt.precision))
    return fail(h, PCV_ESHAPE, "n_atoms exceeds pcv_max_atoms()");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(h, PCV_EINVAL, "lambda must be positive and finite");
  std::vector<double> hw(n_atoms, 1.0);
  if (w) {
    double s = 0.0;
    for (int j = 0; j < n_atoms; ++j) {
      if (!(w[j] >= 0.0) || !std::isfinite(w[j])) return fail(h, PCV_EINVAL, "weights must be finite and >= 0");
      s += w[j];
    }
    if (!(s > 0.0)) return fail(h, PCV_EINVAL, "weights must have a positive sum");
    for (int j = 0; j < n_atoms; ++j) hw[j] = w[j] / s;
  } else {
    for (int j = 0; j < n_atoms; ++j) hw[j] = 1.0 / n_atoms;
  }
  std::vector<double> hq(n_landmarks);
  for (int i = 0; i < n_landmarks; ++i) {
    hq[i] = q ? q[i] : (double)(i + 1);
    if (!std::isfinite(hq[i])) return fail(h, PCV_EINVAL, "properties must be finite");
  }
  HIP_TRY(h, hipSetDevice(h->opt.device));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  drop_graphs(h);
  h->nlpmem.release();
  h->nlmem.release();
  h->nl_M = 0;
  h->nl_stride = 0;
  h->nl_step = 0;
  h->propmem.release();
  h->Wprop = h->part_prop = h->corr_prop = nullptr;
  h->f2mem.release();
  h->wd = nullptr;
  h->pmem.release();
  h->xuv = nullptr;
  h->mem.release();
  h->n = n_atoms;
  h->n_pad = round_up(n_atoms, 64);
  h->L = n_landmarks;
  h->lam = lambda;
  const size_t tsz = h->fp64 ? 8 : 4;
  const size_t np = h->n_pad, L = h->L;
  DevMem& m = h->mem;
  HIP_TRY(h, m.alloc(&h->A, L * 3 * np * tsz));
  HIP_TRY(h, m.alloc((void**)&h->ca, L * 3 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Ga, L * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->q, L * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->w, np * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->xw, 3 * np * sizeof(double)));
  h->n_x = round_up(h->n_pad, 256);
  h->xw32 = nullptr;
  if (!h->fp64) {
    HIP_TRY(h, m.alloc((void**)&h->xw32, 3 * (size_t)h->n_x * sizeof(float)));
    HIP_TRY(h, hipMemset(h->xw32, 0, 3 * (size_t)h->n_x * sizeof(float)));
  }
  HIP_TRY(h, m.alloc((void**)&h->Gx, sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Gx32, sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->xres, 3 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->status, sizeof(int)));
  HIP_TRY(h, m.alloc((void**)&h->corr, 6 * (np / 64) * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->close_ticket, sizeof(unsigned)));
  HIP_TRY(h, hipMemset(h->close_ticket, 0, sizeof(unsigned)));
  HIP_TRY(h, m.alloc((void**)&h->y64, 3 * np * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Gy, sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Fxy, 10 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->lamxy, sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->qxy, 4 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Rxy, 9 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Dxy, sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Rsave, L * 9 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Rprop, L * 9 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Dprop, L * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->gtmp, 12 * np * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->scratch_sz, 2 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->flag, sizeof(int)));
  HIP_TRY(h, m.alloc((void**)&h->init, sizeof(int)));
  HIP_TRY(h, m.alloc((void**)&h->force, sizeof(int)));
  HIP_TRY(h, m.alloc((void**)&h->counters, CNT_N * sizeof(long long)));
  std::vector<double> wpad(np, 0.0);
  std::copy(hw.begin(), hw.end(), wpad.begin());
  HIP_TRY(h, hipMemcpy(h->w, wpad.data(), np * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->q, hq.data(), L * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemset(h->init, 0, sizeof(int)));
  HIP_TRY(h, hipMemset(h->force, 0, sizeof(int)));
  HIP_TRY(h, hipMemset(h->flag, 0, sizeof(int)));
  HIP_TRY(h, hipMemset(h->status, 0, sizeof(int)));
  HIP_TRY(h, hipMemset(h->counters, 0, CNT_N * sizeof(long long)));
  HIP_TRY(h, hipMemset(h->y64, 0, 3 * np * sizeof(double)));
  HIP_TRY(h, hipMemset(h->Rsave, 0, L * 9 * sizeof(double)));
  hipError_t e = h->fp64 ? launch_load_landmarks<double>((const double*)coords, (double*)h->A, h->ca, h->Ga,
                                                         h->w, h->n, h->n_pad, h->L, h->stream)
                         : launch_load_landmarks<float>((const float*)coords, (float*)h->A, h->ca, h->Ga,
                                                        h->w, h->n, h->n_pad, h->L, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "load_landmarks");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  default_plan(h);
  return build_plan(h);
}

extern "C" pcv_status pcv_set_lambda(pcv_handle* h, double lambda) {
  if (!h) return PCV_EINVAL;
  if (h->L == 0) return fail(h, PCV_ESTATE, "no landmarks loaded");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(h, PCV_EINVAL, "lambda must be positive and finite");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->lam = lambda;
  HIP_TRY(h, hipMemset(h->init, 0, sizeof(int)));
  return build_plan(h);
}

extern "C" pcv_status pcv_path_lambda(pcv_handle* h, double factor, double* lambda_out) {
  if (!h || !lambda_out) return PCV_EINVAL;
  if (h->L < 2) return fail(h, PCV_ESTATE, "needs at least two landmarks");
  double* d = nullptr;
  HIP_TRY(h, hipMalloc((void**)&d, (h->L - 1) * sizeof(double)));
  hipError_t e = h->fp64 ? launch_pair_msd<double>((const double*)h->A, h->ca, h->Ga, h->w, h->n, h->n_pad,
                                                   h->L, d, h->stream)
                         : launch_pair_msd<float>((const float*)h->A, h->ca, h->Ga, h->w, h->n, h->n_pad,
                                                  h->L, d, h->stream);
  std::vector<double> hd(h->L - 1);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = hipMemcpy(hd.data(), d, hd.size() * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(h, e, "pair_msd");
  double s = 0.0;
  for (double v : hd) s += v;
  const double mean = s / hd.size();
  if (!(mean > 0.0)) return fail(h, PCV_EINVAL, "consecutive landmarks coincide; lambda undefined");
  *lambda_out = factor / mean;
  return PCV_OK;
}

// ---------------------------------------------------------------- Algorithm 1
// Engine launch bracketed by events when kernel timing is on.
template <typename T>
static hipError_t engine_launch(pcv_handle* h, hipStream_t st, int mode, const int* flag, int run_if, double* msd,
                                bool nl = false, int prob_slot = -1) {
  const Plan& p = h->plan;
  const Problem* probs = (nl ? h->d_prob_nl : h->d_prob) + (prob_slot >= 0 ? prob_slot : mode);
  const Item* items = nl ? h->d_items_nl : h->d_items;
  const int* wgoff = nl ? h->d_wgoff_nl : h->d_wgoff;
  const int grid = nl ? h->grid_nl : p.grid;
  hipError_t e;
  if (p.engine == 4)
    e = launch_engine4<T>(p.spw, grid, probs, items, wgoff, mode, flag, run_if, msd, st);
  else if (p.engine == 5)
    e = launch_engine5<T>(p.bpw, grid, probs, items, wgoff, mode, flag, run_if, msd, st);
  else if (p.engine == 3)
    e = launch_engine3<T>(p.bpw, grid, probs, items, wgoff, mode, flag, run_if, msd, st);
  else if (p.engine == 2)
    e = launch_engine2<T>(p.c2.ncw, p.c2.aptc, p.c2.aptg, grid, p.lds, p.lbuf, p.B, probs, items, wgoff, mode, flag,
                          run_if, msd, st);
  else
    e = launch_engine<T>(p.cfg, grid, p.lds, probs, items, wgoff, mode, flag, run_if, msd, st);
  return e;
}

template <typename T>
static hipError_t engine_timed(pcv_handle* h, hipStream_t st, int mode, const int* flag, int run_if, double* msd,
                               bool nl = false, int prob_slot = -1) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->timing) {
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, st);
  }
  const hipError_t e = engine_launch<T>(h, st, mode, flag, run_if, msd, nl, prob_slot);
  if (h->timing) {
    (void)hipEventRecord(e1, st);
    h->ev_pending.emplace_back(e0, e1);
  }
  return e;
}

template <typename T>
static hipError_t enqueue_exact(pcv_handle* h, hipStream_t st, const void* x, double* sz, void* ds,
                                void* dz, double* msd, PrepArgs* d_pa) {
  hipError_t e = launch_prep<T>(d_pa, x, 1, h->n, st);
  if (e != hipSuccess) return e;
  e = engine_timed<T>(h, st, MODE_EXACT, nullptr, 0, msd);
  if (e != hipSuccess) return e;
  Outs o{ds, dz, sz, nullptr};
  return launch_merge_exact<T>(h->d_prob + MODE_EXACT, o, 1, h->n_pad, nullptr, 0, st, x_rounded(h));
}

template <typename T>
static hipError_t enqueue_close(pcv_handle* h, hipStream_t st, const void* x, double* sz, void* ds,
                                void* dz, double* msd, int* rec) {
  PrepArgs pa{0, h->w, h->xw, h->Gx, h->Gx32, h->xres, h->status, nullptr, h->n, h->n_pad, h->L};
  pa.xw32 = h->xw32;
  pa.n_x = h->n_x;
  CloseArgs ca{h->y64, h->Gy, h->Fxy, h->lamxy, h->qxy, h->Rxy, h->Dxy,
               h->flag, h->init, h->force, h->counters, h->opt.eps, h->L, h->close_ticket};
  Outs o{ds, dz, sz, rec};
  hipError_t e = launch_prep_close<T>(pa, x, ca, o, st);
  if (e != hipSuccess) return e;
  // One engine launch and one merge serve both branches (the flag decides
  // on the device which problem they take).
  e = engine_timed<T>(h, st, MODE_APPROX, h->flag, kRunDual, msd, false, 0);
  if (e != hipSuccess) return e;
  return launch_merge_close<T>(h->d_prob + MODE_APPROX, h->n_pad, o, ca, h->gtmp, st, h->d_prob + MODE_EXACT_SAVE,
                               h->xuv != nullptr);
}

template <typename T>
static hipError_t nl_gather(pcv_handle* h, hipStream_t st, const int* flag, int run_if) {
  NlGather g{h->nl_members, h->nl_M, h->n_pad, h->A, h->ca, h->Ga, h->q, h->Rsave,
             h->A_nl, h->ca_nl, h->Ga_nl, h->q_nl, h->Rsave_nl};
  return launch_nl_gather<T>(g, flag, run_if, st);
}

// Algorithm 1 with a neighbour list: an update step evaluates every
// reference (its CV uses all of them) and keeps the M nearest; the steps in
// between evaluate the list only.
template <typename T>
static hipError_t enqueue_exact_nl(pcv_handle* h, hipStream_t st, const void* x, double* sz, void* ds, void* dz,
                                   bool update) {
  Outs o{ds, dz, sz, nullptr};
  if (update) {
    hipError_t e = launch_prep<T>(h->d_prep, x, 1, h->n, st);
    if (e == hipSuccess) e = engine_timed<T>(h, st, MODE_EXACT, nullptr, 0, h->dfull);
    if (e == hipSuccess)
      e = launch_merge_exact<T>(h->d_prob + MODE_EXACT, o, 1, h->n_pad, nullptr, 0, st, x_rounded(h));
    if (e == hipSuccess) e = launch_nl_select(h->dfull, h->L, h->nl_M, h->nl_members, st);
    if (e == hipSuccess) e = nl_gather<T>(h, st, nullptr, 0);
    return e;
  }
  hipError_t e = launch_prep<T>(h->d_prep_nl, x, 1, h->n, st);
  if (e == hipSuccess) e = engine_timed<T>(h, st, MODE_EXACT, nullptr, 0, nullptr, true);
  if (e == hipSuccess)
    e = launch_merge_exact<T>(h->d_prob_nl + MODE_EXACT, o, 1, h->n_pad, nullptr, 0, st, x_rounded(h));
  return e;
}

// Algorithm 2 with a neighbour list (Section 3.2): a reassignment evaluates
// every reference exactly (its CV uses all of them); an update step without
// reassignment evaluates every reference by Eq. 5; both update steps keep the
// M nearest by that step's distances.  Other steps evaluate the list by
// Eq. 5; a reassignment between updates refreshes the members' rotations.
template <typename T>
static hipError_t enqueue_close_nl(pcv_handle* h, hipStream_t st, const void* x, double* sz, void* ds, void* dz,
                                   int* rec, bool update) {
  PrepArgs pa{0, h->w, h->xw, h->Gx, h->Gx32, h->xres, h->status, nullptr, h->n, h->n_pad, h->L};
  pa.xw32 = h->xw32;
  pa.n_x = h->n_x;
  CloseArgs ca{h->y64, h->Gy, h->Fxy, h->lamxy, h->qxy, h->Rxy, h->Dxy,
               h->flag, h->init, h->force, h->counters, h->opt.eps, h->L, h->close_ticket};
  Outs o{ds, dz, sz, rec};
  hipError_t e = launch_prep_close<T>(pa, x, ca, o, st);
  if (e != hipSuccess) return e;
  if (update) {
    e = engine_timed<T>(h, st, MODE_APPROX, h->flag, kRunDual, h->dfull, false, 0);
    if (e == hipSuccess)
      e = launch_merge_close<T>(h->d_prob + MODE_APPROX, h->n_pad, o, ca, h->gtmp, st, h->d_prob + MODE_EXACT_SAVE,
                                h->xuv != nullptr);
    if (e == hipSuccess) e = launch_nl_select(h->dfull, h->L, h->nl_M, h->nl_members, st);
    if (e == hipSuccess) e = nl_gather<T>(h, st, nullptr, 0);
    return e;
  }
  e = engine_timed<T>(h, st, MODE_EXACT_SAVE, h->flag, 1, nullptr);
  if (e == hipSuccess)
    e = launch_merge_exact<T>(h->d_prob + MODE_EXACT_SAVE, o, 1, h->n_pad, h->flag, 1, st, x_rounded(h));
  if (e == hipSuccess) e = nl_gather<T>(h, st, h->flag, 1);
  if (e == hipSuccess) e = engine_timed<T>(h, st, MODE_APPROX, h->flag, 0, nullptr, true);
  if (e == hipSuccess) e = launch_merge_close<T>(h->d_prob_nl + MODE_APPROX, h->n_pad, o, ca, h->gtmp, st);
  return e;
}

// Run an enqueue function directly or through a cached hipGraph keyed on the
// call's pointers.
template <typename F>
static pcv_status run_maybe_graph(pcv_handle* h, const void* const key[7], F&& enqueue) {
  if (!h->opt.use_graph || h->timing) {
    hipError_t e = enqueue(h->stream);
    return e == hipSuccess ? PCV_OK : hip_fail(h, e, "enqueue");
  }
  for (auto& g : h->graphs) {
    if (g.version == h->plan_version && std::equal(key, key + 7, g.key)) {
      HIP_TRY(h, hipGraphLaunch(g.exec, h->stream));
      return PCV_OK;
    }
  }
  hipGraph_t graph = nullptr;
  HIP_TRY(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue(h->cap_stream);
  hipError_t e2 = hipStreamEndCapture(h->cap_stream, &graph);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(h, e, "capture");
  }
  if (e2 != hipSuccess) return hip_fail(h, e2, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(h, e, "hipGraphInstantiate");
  if (h->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(h->graphs.front().exec);
    h->graphs.erase(h->graphs.begin());
  }
  pcv_handle::GraphEntry ge;
  std::copy(key, key + 7, ge.key);
  ge.version = h->plan_version;
  ge.exec = exec;
  h->graphs.push_back(ge);
  HIP_TRY(h, hipGraphLaunch(exec, h->stream));
  return PCV_OK;
}

// ------------------------------------------- separate displacement weights
static F2Args f2_args(pcv_handle* h) {
  F2Args a{};
  a.A = h->A;
  a.ca = h->ca;
  a.Ga = h->Ga;
  a.Gaw = h->Gaw;
  a.mua = h->mua;
  a.Caa = h->Caa;
  a.wa = h->w;
  a.wd = h->wd;
  a.xc = h->xc2;
  a.fs = h->fs2;
  a.Rl = h->Rl2;
  a.Gl = h->Gl2;
  a.Rmu = h->Rmu2;
  a.cw = h->cw2;
  a.pw = h->pw2;
  a.part = h->part2;
  a.q = h->q;
  a.status = h->status;
  a.fallbacks = h->counters + CNT_FALLBACK;
  a.lam = h->lam;
  a.L = h->L;
  a.n = h->n;
  a.n_pad = h->n_pad;
  return a;
}

extern "C" pcv_status pcv_set_displacement_weights(pcv_handle* h, const double* w_disp) {
  if (!h) return PCV_EINVAL;
  if (h->L == 0) return fail(h, PCV_ESTATE, "no landmarks loaded");
  std::vector<double> hw;
  if (w_disp) {
    if (h->nl_M > 0) return fail(h, PCV_EUNSUPPORTED, "displacement weights with a neighbour list");
    double s = 0.0;
    for (int j = 0; j < h->n; ++j) {
      if (!(w_disp[j] >= 0.0) || !std::isfinite(w_disp[j]))
        return fail(h, PCV_EINVAL, "displacement weights must be finite and >= 0");
      s += w_disp[j];
    }
    if (!(s > 0.0)) return fail(h, PCV_EINVAL, "displacement weights must have a positive sum");
    hw.assign(h->n_pad, 0.0);
    for (int j = 0; j < h->n; ++j) hw[j] = w_disp[j] / s;
  }
  HIP_TRY(h, hipSetDevice(h->opt.device));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  drop_graphs(h);
  h->plan_version++;
  h->f2mem.release();
  h->wd = nullptr;
  if (!w_disp) return PCV_OK;
  const size_t np = h->n_pad, L = h->L, chunks = f2_chunks(h->n_pad, h->L);
  DevMem& m = h->f2mem;
  double* wd = nullptr;
  HIP_TRY(h, m.alloc((void**)&wd, np * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Gaw, L * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->mua, L * 3 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Caa, L * 6 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->xc2, 3 * np * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->fs2, 11 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Rl2, L * 9 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Gl2, L * 9 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Rmu2, L * 3 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->cw2, L * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->pw2, L * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->D2, L * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->part2, chunks * 12 * np * sizeof(double)));
  HIP_TRY(h, hipMemcpy(wd, hw.data(), np * sizeof(double), hipMemcpyHostToDevice));
  h->wd = wd;
  const F2Args a = f2_args(h);
  hipError_t e = h->fp64 ? launch_f2_stats<double>(a, h->stream) : launch_f2_stats<float>(a, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    h->f2mem.release();
    h->wd = nullptr;
    return hip_fail(h, e, "f2_stats");
  }
  return PCV_OK;
}

extern "C" pcv_status pcv_eval(pcv_handle* h, const void* x, double* sz, void* ds_dx, void* dz_dx, double* msd) {
  if (!h) return PCV_EINVAL;
  if (h->L == 0) return fail(h, PCV_ESTATE, "no landmarks loaded");
  if (!x || !sz) return fail(h, PCV_EINVAL, "x and sz are required");
  PrepArgs* d_pa = h->d_prep;
  if (h->wd) {
    const void* key[7] = {x, sz, ds_dx, dz_dx, msd, nullptr, (const void*)8};
    return run_maybe_graph(h, key, [&](hipStream_t st) {
      const F2Args a = f2_args(h);
      double* dout = msd ? msd : h->D2;
      return h->fp64 ? launch_f2_eval<double>(a, x, sz, ds_dx, dz_dx, dout, h->counters, st)
                     : launch_f2_eval<float>(a, x, sz, ds_dx, dz_dx, dout, h->counters, st);
    });
  }
  if (h->nl_M > 0) {
    if (msd) return fail(h, PCV_EINVAL, "msd output is not available with a neighbour list");
    const bool update = h->nl_step % h->nl_stride == 0;
    const void* key[7] = {x, sz, ds_dx, dz_dx, nullptr, nullptr, (const void*)(update ? 3 : 4)};
    pcv_status s = run_maybe_graph(h, key, [&](hipStream_t st) {
      return h->fp64 ? enqueue_exact_nl<double>(h, st, x, sz, ds_dx, dz_dx, update)
                     : enqueue_exact_nl<float>(h, st, x, sz, ds_dx, dz_dx, update);
    });
    if (s == PCV_OK) h->nl_step++;
    return s;
  }
  const void* key[7] = {x, sz, ds_dx, dz_dx, msd, nullptr, (const void*)1};
  return run_maybe_graph(h, key, [&](hipStream_t st) {
    return h->fp64 ? enqueue_exact<double>(h, st, x, sz, ds_dx, dz_dx, msd, d_pa)
                   : enqueue_exact<float>(h, st, x, sz, ds_dx, dz_dx, msd, d_pa);
  });
}

// ---------------------------------------------------------------- Algorithm 2
// advance: a simulation step (counts toward the neighbour-list stride).
static pcv_status eval_close_impl(pcv_handle* h, const void* x, double* sz, void* ds_dx, void* dz_dx, double* msd,
                                  int* recomputed, bool advance) {
  if (!h) return PCV_EINVAL;
  if (h->L == 0) return fail(h, PCV_ESTATE, "no landmarks loaded");
  if (!x || !sz) return fail(h, PCV_EINVAL, "x and sz are required");
  if (h->wd) return fail(h, PCV_EUNSUPPORTED, "the close structure with displacement weights");
  if (h->nl_M > 0) {
    if (msd) return fail(h, PCV_EINVAL, "msd output is not available with a neighbour list");
    const bool update = advance && h->nl_step % h->nl_stride == 0;
    const void* key[7] = {x, sz, ds_dx, dz_dx, nullptr, recomputed, (const void*)(update ? 5 : 6)};
    pcv_status s = run_maybe_graph(h, key, [&](hipStream_t st) {
      return h->fp64 ? enqueue_close_nl<double>(h, st, x, sz, ds_dx, dz_dx, recomputed, update)
                     : enqueue_close_nl<float>(h, st, x, sz, ds_dx, dz_dx, recomputed, update);
    });
    if (s == PCV_OK && advance) h->nl_step++;
    return s;
  }
  const void* key[7] = {x, sz, ds_dx, dz_dx, msd, recomputed, (const void*)2};
  return run_maybe_graph(h, key, [&](hipStream_t st) {
    return h->fp64 ? enqueue_close<double>(h, st, x, sz, ds_dx, dz_dx, msd, recomputed)
                   : enqueue_close<float>(h, st, x, sz, ds_dx, dz_dx, msd, recomputed);
  });
}

extern "C" pcv_status pcv_eval_close(pcv_handle* h, const void* x, double* sz, void* ds_dx, void* dz_dx,
                                     double* msd, int* recomputed) {
  return eval_close_impl(h, x, sz, ds_dx, dz_dx, msd, recomputed, true);
}

// Property maps: the exact pass with rotations and distances saved, then the
// shared weights, every component and all P gradients (pcv_props.hip).
static PropsArgs props_args(const pcv_handle* h, int P, double* corr) {
  PropsArgs a{h->A, h->ca, h->Rprop, h->Dprop, h->w, h->L, h->n, h->n_pad, P};
  a.xw = h->xw;
  a.x_rounded = x_rounded(h) ? 1 : 0;
  a.corr = corr;
  return a;
}

template <typename T>
static hipError_t enqueue_props(pcv_handle* h, hipStream_t st, const void* x, int P, const double* q, double* S,
                                void* dS) {
  hipError_t e = launch_prep<T>(h->d_prep, x, 1, h->n, st);
  if (e == hipSuccess) e = engine_timed<T>(h, st, MODE_EXACT_SAVE, nullptr, 0, h->Dprop, false, 3);
  if (e != hipSuccess) return e;
  const PropsArgs a = props_args(h, P, h->corr_prop);
  return launch_props<T>(a, q, h->lam, S, h->Wprop, h->part_prop, dS, st);
}

extern "C" pcv_status pcv_eval_properties(pcv_handle* h, const void* x, int P, const double* q, double* S,
                                          void* dS_dx) {
  if (!h) return PCV_EINVAL;
  if (h->L == 0) return fail(h, PCV_ESTATE, "no landmarks loaded");
  if (!x || !q || !S) return fail(h, PCV_EINVAL, "x, q and S are required");
  if (P < 1 || P > kPropsMax) return fail(h, PCV_EINVAL, "need 1 <= P <= " + std::to_string(kPropsMax));
  if (h->wd) return fail(h, PCV_EUNSUPPORTED, "property maps with displacement weights");
  if (!h->Wprop) {
    HIP_TRY(h, hipSetDevice(h->opt.device));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const size_t chunks = props_chunks(h->n_pad, h->L);
    HIP_TRY(h, h->propmem.alloc((void**)&h->Wprop, (size_t)h->L * kPropsMax * sizeof(double)));
    HIP_TRY(h, h->propmem.alloc((void**)&h->part_prop, chunks * kPropsMax * 3 * (size_t)h->n_pad * sizeof(double)));
    HIP_TRY(h, h->propmem.alloc((void**)&h->corr_prop, (size_t)props_corr_doubles(h->n) * kPropsMax * sizeof(double)));
  }
  const void* key[7] = {x, q, S, dS_dx, (const void*)(uintptr_t)P, nullptr, (const void*)7};
  return run_maybe_graph(h, key, [&](hipStream_t st) {
    return h->fp64 ? enqueue_props<double>(h, st, x, P, q, S, dS_dx)
                   : enqueue_props<float>(h, st, x, P, q, S, dS_dx);
  });
}

// pcv_eval_properties with its weights W [L][P] and gradient-pass partials
// [chunks][P][3][n_pad] in the GPU's fixed scratch array: no allocation, no
// graph, eager launches on the handle's stream.  Both buffers are written
// in full before they are read, so nothing needs clearing between calls.
extern "C" pcv_status pcv_eval_properties_noalloc(pcv_handle* h, const void* x, int P, const double* q, double* S,
                                                  void* dS_dx) {
  if (!h) return PCV_EINVAL;
  if (h->L == 0) return fail(h, PCV_ESTATE, "no landmarks loaded");
  if (!x || !q || !S) return fail(h, PCV_EINVAL, "x, q and S are required");
  if (P < 1 || P > kPropsMax) return fail(h, PCV_EINVAL, "need 1 <= P <= " + std::to_string(kPropsMax));
  if (h->wd) return fail(h, PCV_EUNSUPPORTED, "property maps with displacement weights");
  const size_t chunks = props_chunks(h->n_pad, h->L);
  const size_t w_bytes = ((size_t)h->L * P * sizeof(double) + 255) / 256 * 256;
  const size_t part_bytes = (chunks * P * 3 * (size_t)h->n_pad * sizeof(double) + 255) / 256 * 256;
  const size_t corr_bytes = (size_t)props_corr_doubles(h->n) * P * sizeof(double);
  if (w_bytes + part_bytes + corr_bytes > kScratchBytes)
    return fail(h, PCV_EINVAL,
                "property maps need " + std::to_string(w_bytes + part_bytes + corr_bytes) +
                    " bytes of scratch; the fixed array holds " + std::to_string(kScratchBytes));
  unsigned char* base = (unsigned char*)scratch_ptr(h->opt.device);
  if (!base) return fail(h, PCV_ESTATE, "no scratch address for this device");
  double* W = (double*)base;
  double* part = (double*)(base + w_bytes);
  double* corr = (double*)(base + w_bytes + part_bytes);
  HIP_TRY(h, hipSetDevice(h->opt.device));
  const hipStream_t st = h->stream;
  hipError_t e;
  if (h->fp64) {
    e = launch_prep<double>(h->d_prep, x, 1, h->n, st);
    if (e == hipSuccess) e = engine_launch<double>(h, st, MODE_EXACT_SAVE, nullptr, 0, h->Dprop, false, 3);
    const PropsArgs a = props_args(h, P, corr);
    if (e == hipSuccess) e = launch_props<double>(a, q, h->lam, S, W, part, dS_dx, st);
  } else {
    e = launch_prep<float>(h->d_prep, x, 1, h->n, st);
    if (e == hipSuccess) e = engine_launch<float>(h, st, MODE_EXACT_SAVE, nullptr, 0, h->Dprop, false, 3);
    const PropsArgs a = props_args(h, P, corr);
    if (e == hipSuccess) e = launch_props<float>(a, q, h->lam, S, W, part, dS_dx, st);
  }
  if (e != hipSuccess) return hip_fail(h, e, "property maps (fixed scratch)");
  return PCV_OK;
}

extern "C" pcv_status pcv_set_neighbour_list(pcv_handle* h, int M, int stride) {
  if (!h) return PCV_EINVAL;
  if (h->L == 0) return fail(h, PCV_ESTATE, "no landmarks loaded");
  if (M < 0 || (M > 0 && (M > h->L || stride < 1))) return fail(h, PCV_EINVAL, "need 1 <= M <= L and stride >= 1");
  if (M > 0 && h->L > nl_select_max())
    return fail(h, PCV_EUNSUPPORTED, "neighbour lists need L <= " + std::to_string(nl_select_max()));
  if (M > 0 && h->wd) return fail(h, PCV_EUNSUPPORTED, "a neighbour list with displacement weights");
  HIP_TRY(h, hipSetDevice(h->opt.device));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  drop_graphs(h);
  h->nlpmem.release();
  h->nlmem.release();
  h->nl_M = 0;
  h->nl_stride = 0;
  h->nl_step = 0;
  h->plan_version++;
  if (M == 0) return PCV_OK;
  const size_t tsz = h->fp64 ? 8 : 4;
  DevMem& m = h->nlmem;
  HIP_TRY(h, m.alloc((void**)&h->nl_members, (size_t)M * sizeof(int)));
  HIP_TRY(h, m.alloc(&h->A_nl, (size_t)M * 3 * h->n_pad * tsz));
  HIP_TRY(h, m.alloc((void**)&h->ca_nl, (size_t)M * 3 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Ga_nl, (size_t)M * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->q_nl, (size_t)M * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->Rsave_nl, (size_t)M * 9 * sizeof(double)));
  HIP_TRY(h, m.alloc((void**)&h->dfull, (size_t)h->L * sizeof(double)));
  std::vector<int> first(M);
  for (int k = 0; k < M; ++k) first[k] = k;
  HIP_TRY(h, hipMemcpy(h->nl_members, first.data(), M * sizeof(int), hipMemcpyHostToDevice));
  h->nl_M = M;
  h->nl_stride = stride;
  pcv_status s = build_plan(h);
  if (s != PCV_OK) return s;
  // Start from the first M references so that every buffer holds valid data.
  hipError_t e = h->fp64 ? nl_gather<double>(h, h->stream, nullptr, 0) : nl_gather<float>(h, h->stream, nullptr, 0);
  if (e != hipSuccess) return hip_fail(h, e, "neighbour-list gather");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return PCV_OK;
}

extern "C" pcv_status pcv_get_neighbour_list(pcv_handle* h, int* members, int capacity, int* count) {
  if (!h || !count) return PCV_EINVAL;
  *count = h->nl_M;
  if (h->nl_M == 0 || !members) return PCV_OK;   // NULL members: size query
  if (capacity < h->nl_M) return fail(h, PCV_EINVAL, "members buffer too small");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  HIP_TRY(h, hipMemcpy(members, h->nl_members, (size_t)h->nl_M * sizeof(int), hipMemcpyDeviceToHost));
  return PCV_OK;
}

// ------------------------------------------------------- checkpoint / resume
// The state that carries over between steps: the close structure y (centred,
// FP64), G_y, the saved rotations R_{a_i y}, the first-frame and forced
// flags, the counters, and the neighbour list (size, stride, step count,
// members and their saved rotations).  A fingerprint of the landmark set
// (sums of G_a and of the centroids' squared norms) guards against loading
// a state into a handle with other landmarks.
namespace {
constexpr unsigned long long kStateMagic = 0x3130455441545350ull;   // "PSTATE01"
constexpr int kStateVersion = 1;
struct StateHeader {
  unsigned long long magic;
  int version, precision, n, L, nl_M, nl_stride, init, force;
  long long nl_step;
  double ga_sum, ca_sum;
};
}  // namespace

static size_t state_bytes(const pcv_handle* h, int nl_M) {
  return sizeof(StateHeader) + (3 * (size_t)h->n_pad + 1 + 9 * (size_t)h->L) * sizeof(double) +
         CNT_N * sizeof(long long) + (size_t)nl_M * (sizeof(int) + 9 * sizeof(double));
}

static pcv_status landmark_fingerprint(pcv_handle* h, double& ga_sum, double& ca_sum) {
  std::vector<double> ga(h->L), ca(3 * (size_t)h->L);
  HIP_TRY(h, hipMemcpy(ga.data(), h->Ga, ga.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIP_TRY(h, hipMemcpy(ca.data(), h->ca, ca.size() * sizeof(double), hipMemcpyDeviceToHost));
  ga_sum = 0.0;
  ca_sum = 0.0;
  for (double v : ga) ga_sum += v;
  for (double v : ca) ca_sum += v * v;
  return PCV_OK;
}

extern "C" pcv_status pcv_save_state(pcv_handle* h, void* buf, size_t* bytes) {
  if (!h || !bytes) return PCV_EINVAL;
  if (h->L == 0) return fail(h, PCV_ESTATE, "no landmarks loaded");
  const size_t need = state_bytes(h, h->nl_M);
  if (!buf) {
    *bytes = need;
    return PCV_OK;
  }
  if (*bytes < need) {
    *bytes = need;
    return fail(h, PCV_EINVAL, "state buffer too small");
  }
  HIP_TRY(h, hipSetDevice(h->opt.device));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  StateHeader hd{};
  hd.magic = kStateMagic;
  hd.version = kStateVersion;
  hd.precision = h->fp64 ? PCV_FP64 : PCV_FP32;
  hd.n = h->n;
  hd.L = h->L;
  hd.nl_M = h->nl_M;
  hd.nl_stride = h->nl_stride;
  hd.nl_step = h->nl_step;
  HIP_TRY(h, hipMemcpy(&hd.init, h->init, sizeof(int), hipMemcpyDeviceToHost));
  HIP_TRY(h, hipMemcpy(&hd.force, h->force, sizeof(int), hipMemcpyDeviceToHost));
  pcv_status st = landmark_fingerprint(h, hd.ga_sum, hd.ca_sum);
  if (st != PCV_OK) return st;
  char* p = (char*)buf;
  std::memcpy(p, &hd, sizeof(hd));
  p += sizeof(hd);
  const size_t ny = 3 * (size_t)h->n_pad * sizeof(double), nr = 9 * (size_t)h->L * sizeof(double);
  HIP_TRY(h, hipMemcpy(p, h->y64, ny, hipMemcpyDeviceToHost));
  p += ny;
  HIP_TRY(h, hipMemcpy(p, h->Gy, sizeof(double), hipMemcpyDeviceToHost));
  p += sizeof(double);
  HIP_TRY(h, hipMemcpy(p, h->Rsave, nr, hipMemcpyDeviceToHost));
  p += nr;
  HIP_TRY(h, hipMemcpy(p, h->counters, CNT_N * sizeof(long long), hipMemcpyDeviceToHost));
  p += CNT_N * sizeof(long long);
  if (h->nl_M > 0) {
    HIP_TRY(h, hipMemcpy(p, h->nl_members, (size_t)h->nl_M * sizeof(int), hipMemcpyDeviceToHost));
    p += (size_t)h->nl_M * sizeof(int);
    HIP_TRY(h, hipMemcpy(p, h->Rsave_nl, (size_t)h->nl_M * 9 * sizeof(double), hipMemcpyDeviceToHost));
  }
  *bytes = need;
  return PCV_OK;
}

extern "C" pcv_status pcv_load_state(pcv_handle* h, const void* buf, size_t bytes) {
  if (!h || !buf) return PCV_EINVAL;
  if (h->L == 0) return fail(h, PCV_ESTATE, "no landmarks loaded");
  if (bytes < sizeof(StateHeader)) return fail(h, PCV_EINVAL, "state buffer too small");
  StateHeader hd;
  std::memcpy(&hd, buf, sizeof(hd));
  if (hd.magic != kStateMagic || hd.version != kStateVersion) return fail(h, PCV_EINVAL, "not a saved state");
  if (hd.precision != (h->fp64 ? PCV_FP64 : PCV_FP32) || hd.n != h->n || hd.L != h->L)
    return fail(h, PCV_ESHAPE, "state saved for another precision, atom count or landmark count");
  if (hd.nl_M < 0 || hd.nl_M > h->L || (hd.nl_M > 0 && hd.nl_stride < 1))
    return fail(h, PCV_EINVAL, "corrupt neighbour-list fields");
  if (bytes < state_bytes(h, hd.nl_M)) return fail(h, PCV_EINVAL, "state buffer too small");
  HIP_TRY(h, hipSetDevice(h->opt.device));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  double ga_sum, ca_sum;
  pcv_status st = landmark_fingerprint(h, ga_sum, ca_sum);
  if (st != PCV_OK) return st;
  auto close = [](double a, double b) { return std::fabs(a - b) <= 1e-12 * std::max(1.0, std::fabs(b)); };
  if (!close(hd.ga_sum, ga_sum) || !close(hd.ca_sum, ca_sum))
    return fail(h, PCV_EINVAL, "state saved for another landmark set");
  if (hd.nl_M != h->nl_M || (hd.nl_M > 0 && hd.nl_stride != h->nl_stride)) {
    st = pcv_set_neighbour_list(h, hd.nl_M, hd.nl_M > 0 ? hd.nl_stride : 1);
    if (st != PCV_OK) return st;
  }
  const char* p = (const char*)buf + sizeof(hd);
  const size_t ny = 3 * (size_t)h->n_pad * sizeof(double), nr = 9 * (size_t)h->L * sizeof(double);
  HIP_TRY(h, hipMemcpy(h->y64, p, ny, hipMemcpyHostToDevice));
  p += ny;
  HIP_TRY(h, hipMemcpy(h->Gy, p, sizeof(double), hipMemcpyHostToDevice));
  p += sizeof(double);
  HIP_TRY(h, hipMemcpy(h->Rsave, p, nr, hipMemcpyHostToDevice));
  p += nr;
  HIP_TRY(h, hipMemcpy(h->counters, p, CNT_N * sizeof(long long), hipMemcpyHostToDevice));
  p += CNT_N * sizeof(long long);
  HIP_TRY(h, hipMemcpy(h->init, &hd.init, sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->force, &hd.force, sizeof(int), hipMemcpyHostToDevice));
  if (hd.nl_M > 0) {
    std::vector<int> mem(hd.nl_M);
    std::memcpy(mem.data(), p, mem.size() * sizeof(int));
    p += mem.size() * sizeof(int);
    for (int v : mem)
      if (v < 0 || v >= h->L) return fail(h, PCV_EINVAL, "corrupt neighbour-list members");
    HIP_TRY(h, hipMemcpy(h->nl_members, mem.data(), mem.size() * sizeof(int), hipMemcpyHostToDevice));
    hipError_t e = h->fp64 ? nl_gather<double>(h, h->stream, nullptr, 0) : nl_gather<float>(h, h->stream, nullptr, 0);
    if (e != hipSuccess) return hip_fail(h, e, "neighbour-list gather");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpy(h->Rsave_nl, p, (size_t)hd.nl_M * 9 * sizeof(double), hipMemcpyHostToDevice));
    h->nl_step = hd.nl_step;
  }
  return PCV_OK;
}

// Token naming a handle and its current buffers (for callers that cache
// hipGraphs capturing the handle's kernels).
extern "C" __attribute__((visibility("hidden"))) unsigned long long pcv_internal_handle_token(const pcv_handle* h) {
  return (h->serial << 32) ^ (unsigned long long)(unsigned)h->plan_version;
}

// Exact half of the surrogate's fallback step: the close-structure drift test
// and, on a reassignment, the exact pass (no Eq. 5 branch).  Returns the
// device flag the surrogate's tail kernel reads.
extern "C" __attribute__((visibility("hidden"))) hipError_t pcv_internal_exact_for_surrogate(
    pcv_handle* h, int n_atoms, hipStream_t st, const void* x,
                                                       double* sz, void* ds, void* dz, const int** flag) {
  if (h->fp64 || h->L == 0 || h->n != n_atoms) return hipErrorInvalidValue;
  if (h->wd) return hipErrorNotSupported;
  PrepArgs pa{0, h->w, h->xw, h->Gx, h->Gx32, h->xres, h->status, nullptr, h->n, h->n_pad, h->L};
  pa.xw32 = h->xw32;
  pa.n_x = h->n_x;
  CloseArgs ca{h->y64, h->Gy, h->Fxy, h->lamxy, h->qxy, h->Rxy, h->Dxy,
               h->flag, h->init, h->force, h->counters, h->opt.eps, h->L, h->close_ticket};
  Outs o{ds, dz, sz, nullptr};
  hipError_t e = launch_prep_close<float>(pa, x, ca, o, st);
  if (e != hipSuccess) return e;
  e = engine_timed<float>(h, st, MODE_EXACT_SAVE, h->flag, 1, nullptr);
  if (e != hipSuccess) return e;
  e = launch_merge_exact<float>(h->d_prob + MODE_EXACT_SAVE, o, 1, h->n_pad, h->flag, 1, st, x_rounded(h));
  *flag = h->flag;
  return e;
}

extern "C" pcv_status pcv_force_reassign(pcv_handle* h) {
  if (!h) return PCV_EINVAL;
  if (h->L == 0) return fail(h, PCV_ESTATE, "no landmarks loaded");
  hipError_t e = launch_set_int(h->force, 1, h->stream);
  return e == hipSuccess ? PCV_OK : hip_fail(h, e, "force");
}

extern "C" pcv_status pcv_update_close(pcv_handle* h, const void* x) {
  if (h && h->wd) return fail(h, PCV_EUNSUPPORTED, "the close structure with displacement weights");
  pcv_status s = pcv_force_reassign(h);
  if (s != PCV_OK) return s;
  return eval_close_impl(h, x, h->scratch_sz, nullptr, nullptr, nullptr, nullptr, false);
}

extern "C" pcv_status pcv_get_stats(pcv_handle* h, pcv_stats* out) {
  if (!h || !out) return PCV_EINVAL;
  std::memset(out, 0, sizeof(*out));
  if (h->L == 0) return PCV_OK;
  long long c[CNT_N];
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  HIP_TRY(h, hipMemcpy(c, h->counters, sizeof(c), hipMemcpyDeviceToHost));
  out->frames = c[CNT_FRAMES];
  out->recomputes = c[CNT_RECOMPUTES];
  out->expensive_msd = c[CNT_EXPENSIVE];
  out->approx_frames = c[CNT_APPROX];
  out->exact_evals = c[CNT_EVALS];
  out->eigen_fallbacks = c[CNT_FALLBACK];
  return PCV_OK;
}

extern "C" pcv_status pcv_reset_stats(pcv_handle* h) {
  if (!h) return PCV_EINVAL;
  if (h->L == 0) return PCV_OK;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  HIP_TRY(h, hipMemset(h->counters, 0, CNT_N * sizeof(long long)));
  return PCV_OK;
}

extern "C" pcv_status pcv_check(pcv_handle* h) {
  if (!h) return PCV_EINVAL;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (h->L == 0) return PCV_OK;
  int st = 0;
  HIP_TRY(h, hipMemcpy(&st, h->status, sizeof(int), hipMemcpyDeviceToHost));
  if (st) {
    HIP_TRY(h, hipMemset(h->status, 0, sizeof(int)));
    return fail(h, PCV_ENONFINITE, "non-finite coordinates in an input structure");
  }
  return PCV_OK;
}

extern "C" pcv_status pcv_get_plan(pcv_handle* h, pcv_plan* out) {
  if (!h || !out) return PCV_EINVAL;
  if (h->L == 0) return fail(h, PCV_ESTATE, "no landmarks loaded");
  const Plan& p = h->plan;
  out->engine = p.engine;
  out->wg = p.engine >= 2 ? 512 : p.cfg.wg;
  out->apt = p.engine == 2 ? p.c2.aptc
             : ((p.engine == 3 || p.engine == 5) ? 4 * p.bpw : (p.engine == 4 ? 4 * p.spw : p.cfg.apt));
  out->team = p.engine == 2 ? p.g : (p.engine >= 3 ? 0 : p.ts);
  out->aptg = p.engine == 2 ? p.c2.aptg : 0;
  out->batch = (p.engine == 2 || p.engine == 4) ? p.B : 0;
  out->grid = p.grid;
  out->items = p.n_items;
  return PCV_OK;
}

extern "C" pcv_status pcv_set_plan(pcv_handle* h, const pcv_plan* q) {
  if (!h || !q) return PCV_EINVAL;
  if (h->L == 0) return fail(h, PCV_ESTATE, "no landmarks loaded");
  Plan p = h->plan;
  if (q->engine == 1) {
    const EngineCfg c{q->wg, q->apt};
    if (!engine_supported(c, h->fp64)) return fail(h, PCV_EUNSUPPORTED, "engine 1 tiling not compiled in");
    if (q->team < 16 || q->team > q->wg || (q->team & (q->team - 1)) || (long long)q->team * q->apt < h->n)
      return fail(h, PCV_EINVAL, "team must be a power of two in [16, wg] with team*apt >= n");
    p.engine = 1;
    p.cfg = c;
    p.ts = q->team;
  } else if (q->engine == 2) {
    int nw[16], ac[16], ag[16], cnt = 0;
    engine2_configs(h->fp64, nw, ac, ag, &cnt);
    int ncw = 0;
    for (int k = 0; k < cnt; ++k)
      if (ac[k] == q->apt && ag[k] == q->aptg) ncw = nw[k];
    if (!ncw) return fail(h, PCV_EUNSUPPORTED, "engine 2 tiling not compiled in");
    const Engine2Cfg c{ncw, q->apt, q->aptg};
    const int g = q->team;
    if (!e2_group_ok(g, c) || (h->n_pad + g - 1) / g > c.aptc || !e2_fits(h->n_pad, c))
      return fail(h, PCV_EINVAL, "engine 2 tiling cannot hold the structure");
    if (!e2_lds_ok(h->n_pad, q->batch, h->fp64)) return fail(h, PCV_EINVAL, "batch does not fit in LDS");
    p.engine = 2;
    p.c2 = c;
    p.g = g;
    p.B = q->batch;
    p.cfg = EngineCfg{512, c.aptc};
    p.ts = g;
  } else if (q->engine == 3) {
    if (h->fp64) return fail(h, PCV_EUNSUPPORTED, "engine 3 is FP32 only");
    const int bpw = q->apt / 4;
    if (q->apt % 4 != 0 || bpw < 1 || bpw > 4) return fail(h, PCV_EUNSUPPORTED, "engine 3 needs apt = 4, 8, 12 or 16");
    if ((h->n_pad + 255) / 256 > engine3_max_blocks(bpw))
      return fail(h, PCV_EINVAL, "engine 3 tiling cannot hold the structure");
    p.engine = 3;
    p.bpw = bpw;
    p.cfg = EngineCfg{512, 4 * bpw};
    p.ts = 0;
  } else if (q->engine == 5) {
    if (h->fp64) return fail(h, PCV_EUNSUPPORTED, "engine 5 is FP32 only");
    const int bpw = q->apt / 4;
    if (q->apt % 4 != 0 || bpw < 1 || bpw > 3) return fail(h, PCV_EUNSUPPORTED, "engine 5 needs apt = 4, 8 or 12");
    if ((h->n_pad + 255) / 256 > engine5_max_blocks(bpw))
      return fail(h, PCV_EINVAL, "engine 5 tiling cannot hold the structure");
    p.engine = 5;
    p.bpw = bpw;
    p.cfg = EngineCfg{512, 4 * bpw};
    p.ts = 0;
  } else if (q->engine == 4) {
    if (h->fp64) return fail(h, PCV_EUNSUPPORTED, "engine 4 is FP32 only");
    const int spw = q->apt / 4;
    if (q->apt % 4 != 0 || spw < 2 || spw > 3) return fail(h, PCV_EUNSUPPORTED, "engine 4 needs apt = 8 or 12");
    const int kmax = engine4_lanes(h->n_pad, spw);
    if (kmax < 1) return fail(h, PCV_EINVAL, "engine 4 cannot hold the structure");
    const int K = q->batch > 0 ? q->batch : kmax;
    if (K > kmax) return fail(h, PCV_EINVAL, "engine 4: batch exceeds the landmark lanes of the tiling");
    p.engine = 4;
    p.spw = spw;
    p.B = K;
    p.cfg = EngineCfg{512, 4 * spw};
    p.ts = 0;
  } else {
    return fail(h, PCV_EINVAL, "engine must be 1, 2, 3, 4 or 5");
  }
  p.n_items = q->items;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->plan = p;
  h->user_plan = true;
  return build_plan(h);
}

static void collect_timing(pcv_handle* h) {
  for (auto& pr : h->ev_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(pr.second) == hipSuccess && hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
      h->timed_ms += ms;
      h->timed_launches += 1;
    }
    hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  h->ev_pending.clear();
}

extern "C" pcv_status pcv_set_kernel_timing(pcv_handle* h, int enable) {
  if (!h) return PCV_EINVAL;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  collect_timing(h);
  h->timing = enable != 0;
  h->timed_ms = 0.0;
  h->timed_launches = 0;
  return PCV_OK;
}

extern "C" pcv_status pcv_get_kernel_timing(pcv_handle* h, double* engine_ms, int64_t* engine_launches) {
  if (!h || !engine_ms || !engine_launches) return PCV_EINVAL;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  collect_timing(h);
  *engine_ms = h->timed_ms;
  *engine_launches = h->timed_launches;
  return PCV_OK;
}

extern "C" const char* pcv_status_string(pcv_status s) {
  switch (s) {
    case PCV_OK: return "ok";
    case PCV_EINVAL: return "invalid argument";
    case PCV_ESTATE: return "invalid call order";
    case PCV_ESHAPE: return "unsupported size";
    case PCV_ENONFINITE: return "non-finite input";
    case PCV_EHIP: return "HIP runtime error";
    case PCV_ENOMEM: return "out of device memory";
    case PCV_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

extern "C" const char* pcv_last_error(const pcv_handle* h) { return h ? h->err.c_str() : "null handle"; }
