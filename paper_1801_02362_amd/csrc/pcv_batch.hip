// Batched walkers: many independent (structure, landmark set) problems of
// uneven size in one persistent launch of the landmark engine (Algorithm 1
// per walker), a static longest-processing-time schedule of work items over
// the workgroups, hipGraph replay, and an autotuner over tilings and
// schedules whose candidates must reproduce the heuristic plan's results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "pcv.h"
#include "pcv_host_util.h"
#include "pcv_internal.h"

using namespace pcv;

namespace {

struct BatchPlan {
  int engine = 2;
  EngineCfg cfg{256, 8};   // engine 1 tiling
  Engine2Cfg c2{3, 16, 8}; // engine 2 tiling
  int spw = 3;             // engine 4: units per worker wave
  int per_team = 4;        // engine 1: landmarks per team per item; engine 2: batches per item;
                           // engine 4: landmark steps per item
  int grid_mult = 2;       // workgroups = grid_mult * CUs
  int lpt = 1;             // 1: longest-processing-time schedule, 0: round robin
  std::string str() const {
    std::ostringstream o;
    if (engine == 4)
      o << "engine=4 spw=" << spw;
    else if (engine == 2)
      o << "engine=2 ncw=" << c2.ncw << " aptc=" << c2.aptc << " aptg=" << c2.aptg;
    else
      o << "engine=1 wg=" << cfg.wg << " apt=" << cfg.apt;
    o << " per_item=" << per_team << " grid_mult=" << grid_mult << " schedule=" << (lpt ? "lpt" : "rr");
    return o.str();
  }
};

}  // namespace

struct pcv_batch {
  pcv_options opt{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  bool fp64 = false;
  int cus = 256;
  int W = 0;
  std::vector<int> n, L, n_pad, atom_off, lm_off, pad_off;
  std::vector<double> lam;
  long long total_pairs = 0;
  DevMem mem, pmem;
  void* A = nullptr;
  double *ca = nullptr, *Ga = nullptr, *q = nullptr, *w = nullptr, *xw = nullptr, *Gx = nullptr,
         *Gx32 = nullptr, *xres = nullptr;
  float* xw32 = nullptr;      // FP32 batches: [3][n_x] per walker (engine 4)
  std::vector<size_t> x32_off;
  int* status = nullptr;
  double* corr = nullptr;       // per walker [3 * n_pad / 64][2]: rounding-correction shares of the merge
  std::vector<size_t> corr_off;
  PrepArgs* d_prep = nullptr;
  // plan
  BatchPlan plan;
  bool planned = false;
  int grid = 0, n_items = 0;
  size_t lds = 0;
  int lbuf = 0, bmax = 1;
  Problem* d_prob = nullptr;
  Item* d_items = nullptr;
  int* d_wgoff = nullptr;
  double* hdr = nullptr;
  void* vec = nullptr;
  int max_n_pad = 0;
  int plan_version = 0;
  struct GraphEntry {
    const void* key[4];
    int version;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  std::string plan_str, err;
  // kernel timing (eager launches, events around the engine launch)
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
  double timed_ms = 0.0;
  long long timed_launches = 0;
};

static void bcollect_timing(pcv_batch* b) {
  for (auto& pr : b->ev_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(pr.second) == hipSuccess && hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
      b->timed_ms += ms;
      ++b->timed_launches;
    }
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  b->ev_pending.clear();
}

static pcv_status bfail(pcv_batch* b, pcv_status s, const std::string& m) {
  if (b) b->err = m;
  return s;
}
static pcv_status bhip(pcv_batch* b, hipError_t e, const char* where) {
  return bfail(b, e == hipErrorOutOfMemory ? PCV_ENOMEM : PCV_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}
#define BHIP_TRY(b, expr)                                 \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) return bhip((b), _e, #expr);     \
  } while (0)

static void bdrop_graphs(pcv_batch* b) {
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
  b->graphs.clear();
}

extern "C" pcv_status pcv_batch_create(pcv_batch** out, const pcv_options* opt) {
  if (!out) return PCV_EINVAL;
  *out = nullptr;
  pcv_options o;
  pcv_default_options(&o);
  if (opt) o = *opt;
  if (o.precision != PCV_FP32 && o.precision != PCV_FP64) return PCV_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || o.device < 0 || o.device >= ndev) return PCV_EHIP;
  if (hipSetDevice(o.device) != hipSuccess) return PCV_EHIP;
  pcv_batch* b = new pcv_batch();
  b->opt = o;
  b->fp64 = o.precision == PCV_FP64;
  b->stream = (hipStream_t)o.stream;
  b->cus = num_cus(o.device);
  if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess ||
      engine_init_attributes() != hipSuccess) {
    delete b;
    return PCV_EHIP;
  }
  *out = b;
  return PCV_OK;
}

extern "C" pcv_status pcv_batch_destroy(pcv_batch* b) {
  if (!b) return PCV_OK;
  (void)hipSetDevice(b->opt.device);
  (void)hipStreamSynchronize(b->stream);
  bcollect_timing(b);
  bdrop_graphs(b);
  b->pmem.release();
  b->mem.release();
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
  return PCV_OK;
}

extern "C" pcv_status pcv_batch_load(pcv_batch* b, int W, const int* n_atoms, const int* n_landmarks,
                                     const void* coords, const double* lambdas) {
  if (!b) return PCV_EINVAL;
  if (W < 1 || !n_atoms || !n_landmarks || !coords || !lambdas) return bfail(b, PCV_EINVAL, "bad arguments");
  const int maxn = pcv_max_atoms(b->opt.precision);
  for (int i = 0; i < W; ++i) {
    if (n_atoms[i] < 1 || n_landmarks[i] < 1) return bfail(b, PCV_EINVAL, "walker sizes must be >= 1");
    if (n_atoms[i] > maxn) return bfail(b, PCV_ESHAPE, "walker n_atoms exceeds pcv_max_atoms()");
    if (!(lambdas[i] > 0.0) || !std::isfinite(lambdas[i])) return bfail(b, PCV_EINVAL, "lambda must be positive");
  }
  BHIP_TRY(b, hipSetDevice(b->opt.device));
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  bdrop_graphs(b);
  b->pmem.release();
  b->mem.release();
  b->planned = false;
  b->W = W;
  b->n.assign(n_atoms, n_atoms + W);
  b->L.assign(n_landmarks, n_landmarks + W);
  b->lam.assign(lambdas, lambdas + W);
  b->n_pad.resize(W);
  b->atom_off.resize(W + 1);
  b->lm_off.resize(W + 1);
  b->pad_off.resize(W + 1);
  b->atom_off[0] = b->lm_off[0] = b->pad_off[0] = 0;
  b->total_pairs = 0;
  b->max_n_pad = 0;
  size_t a_elems = 0;
  std::vector<size_t> a_off(W + 1, 0), in_off(W + 1, 0);
  for (int i = 0; i < W; ++i) {
    b->n_pad[i] = round_up(b->n[i], 64);
    b->max_n_pad = std::max(b->max_n_pad, b->n_pad[i]);
    b->atom_off[i + 1] = b->atom_off[i] + b->n[i];
    b->lm_off[i + 1] = b->lm_off[i] + b->L[i];
    b->pad_off[i + 1] = b->pad_off[i] + b->n_pad[i];
    a_off[i + 1] = a_off[i] + (size_t)b->L[i] * 3 * b->n_pad[i];
    in_off[i + 1] = in_off[i] + (size_t)b->L[i] * b->n[i] * 3;
    b->total_pairs += (long long)b->n[i] * b->L[i];
  }
  a_elems = a_off[W];
  const size_t tsz = b->fp64 ? 8 : 4;
  const size_t Ltot = b->lm_off[W], Ptot = b->pad_off[W];
  DevMem& m = b->mem;
  BHIP_TRY(b, m.alloc(&b->A, a_elems * tsz));
  BHIP_TRY(b, m.alloc((void**)&b->ca, Ltot * 3 * sizeof(double)));
  BHIP_TRY(b, m.alloc((void**)&b->Ga, Ltot * sizeof(double)));
  BHIP_TRY(b, m.alloc((void**)&b->q, Ltot * sizeof(double)));
  BHIP_TRY(b, m.alloc((void**)&b->w, Ptot * sizeof(double)));
  BHIP_TRY(b, m.alloc((void**)&b->xw, 3 * Ptot * sizeof(double)));
  BHIP_TRY(b, m.alloc((void**)&b->Gx, W * sizeof(double)));
  BHIP_TRY(b, m.alloc((void**)&b->Gx32, W * sizeof(double)));
  BHIP_TRY(b, m.alloc((void**)&b->xres, 3 * W * sizeof(double)));
  BHIP_TRY(b, m.alloc((void**)&b->status, W * sizeof(int)));
  b->corr_off.assign(W + 1, 0);
  for (int i = 0; i < W; ++i) b->corr_off[i + 1] = b->corr_off[i] + 6 * (size_t)(b->n_pad[i] / 64);
  BHIP_TRY(b, m.alloc((void**)&b->corr, b->corr_off[W] * sizeof(double)));
  BHIP_TRY(b, m.alloc((void**)&b->d_prep, W * sizeof(PrepArgs)));
  b->x32_off.assign(W + 1, 0);
  for (int i = 0; i < W; ++i) b->x32_off[i + 1] = b->x32_off[i] + 3 * (size_t)round_up(b->n_pad[i], 256);
  b->xw32 = nullptr;
  if (!b->fp64) {
    BHIP_TRY(b, m.alloc((void**)&b->xw32, b->x32_off[W] * sizeof(float)));
    BHIP_TRY(b, hipMemset(b->xw32, 0, b->x32_off[W] * sizeof(float)));
  }
  std::vector<double> hw(Ptot, 0.0), hq(Ltot);
  std::vector<PrepArgs> pa(W);
  for (int i = 0; i < W; ++i) {
    for (int j = 0; j < b->n[i]; ++j) hw[b->pad_off[i] + j] = 1.0 / b->n[i];
    for (int k = 0; k < b->L[i]; ++k) hq[b->lm_off[i] + k] = k + 1;
    const size_t po = b->pad_off[i];
    pa[i] = PrepArgs{(long long)b->atom_off[i], b->w + po, b->xw + 3 * po, b->Gx + i, b->Gx32 + i,
                     b->xres + 3 * i, b->status + i, nullptr, b->n[i], b->n_pad[i], b->L[i]};
    pa[i].xw32 = b->xw32 ? b->xw32 + b->x32_off[i] : nullptr;
    pa[i].n_x = round_up(b->n_pad[i], 256);
  }
  BHIP_TRY(b, hipMemcpy(b->w, hw.data(), hw.size() * sizeof(double), hipMemcpyHostToDevice));
  BHIP_TRY(b, hipMemcpy(b->q, hq.data(), hq.size() * sizeof(double), hipMemcpyHostToDevice));
  BHIP_TRY(b, hipMemcpy(b->d_prep, pa.data(), W * sizeof(PrepArgs), hipMemcpyHostToDevice));
  BHIP_TRY(b, hipMemset(b->status, 0, W * sizeof(int)));
  for (int i = 0; i < W; ++i) {
    const size_t lo = b->lm_off[i], po = b->pad_off[i];
    hipError_t e = b->fp64
        ? launch_load_landmarks<double>((const double*)coords + in_off[i], (double*)b->A + a_off[i], b->ca + 3 * lo,
                                        b->Ga + lo, b->w + po, b->n[i], b->n_pad[i], b->L[i], b->stream)
        : launch_load_landmarks<float>((const float*)coords + in_off[i], (float*)b->A + a_off[i], b->ca + 3 * lo,
                                       b->Ga + lo, b->w + po, b->n[i], b->n_pad[i], b->L[i], b->stream);
    if (e != hipSuccess) return bhip(b, e, "load_landmarks");
  }
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  return PCV_OK;
}

// Lay out items and partial slots for a plan and upload the descriptors.
static pcv_status batch_apply(pcv_batch* b, const BatchPlan& p) {
  const size_t tsz = b->fp64 ? 8 : 4;
  std::vector<int> ts(b->W, 0), gsz(b->W, 0), bsz(b->W, 1);
  int bmax = 1, lbuf = 0;
  for (int i = 0; i < b->W; ++i) {
    if (p.engine == 4) {
      if (b->fp64) return bfail(b, PCV_EUNSUPPORTED, "engine 4 is FP32 only");
      const int K = engine4_lanes(b->n_pad[i], p.spw);
      if (K < 1) return bfail(b, PCV_ESHAPE, "engine 4 cannot hold a walker");
      bsz[i] = K;
    } else if (p.engine == 2) {
      const int B = e2_batch(b->n_pad[i], b->fp64);
      if (B == 0 || !e2_fits(b->n_pad[i], p.c2)) return bfail(b, PCV_ESHAPE, "engine 2 cannot hold a walker");
      const int g = e2_group(b->n_pad[i], p.c2, B);
      if (g == 0) return bfail(b, PCV_ESHAPE, "engine 2 group cannot hold a walker");
      gsz[i] = g;
      bsz[i] = B;
      bmax = std::max(bmax, B);
      lbuf = std::max(lbuf, B * 3 * b->n_pad[i] * (int)tsz);
    } else {
      ts[i] = team_size(b->n[i], p.cfg);
      if (ts[i] == 0) return bfail(b, PCV_ESHAPE, "tiling cannot hold a walker");
    }
  }
  struct It {
    Item it;
    double cost;
  };
  std::vector<It> items;
  std::vector<int> slots(b->W, 0), slot_base(b->W + 1, 0);
  size_t vec_elems = 0;
  std::vector<size_t> vec_off(b->W);
  for (int i = 0; i < b->W; ++i) {
    int chunk;
    double per_lm;
    double item_cost = 3000.0;
    if (p.engine == 4) {
      // A step streams K n_pad 12 bytes (about 25 B/ns per CU) and waits for
      // at least one eigen-solve (about 1.5 us); an item also stages the
      // structure and writes its partial.
      chunk = std::max(1, bsz[i] * p.per_team);
      per_lm = std::max((double)bsz[i] * b->n_pad[i] * 12.0 / 25.0, 1500.0) / bsz[i];
      item_cost = 4000.0 + 36.0 * b->n_pad[i] / 25.0;
    } else if (p.engine == 2) {
      chunk = std::max(1, bsz[i] * p.per_team);
      per_lm = (double)b->n_pad[i] * 24.0 + 4000.0 / bsz[i];
    } else {
      const int teams = p.cfg.wg / ts[i];
      chunk = std::max(1, teams * p.per_team);
      per_lm = landmark_cost(b->n[i], p.cfg, ts[i]) / teams;
    }
    const int cnt = (b->L[i] + chunk - 1) / chunk;
    for (int k = 0; k < cnt; ++k) {
      Item it;
      it.prob = i;
      it.i0 = k * chunk;
      it.i1 = std::min(b->L[i], (k + 1) * chunk);
      it.slot = k;
      items.push_back({it, per_lm * (it.i1 - it.i0) + item_cost});
    }
    slots[i] = cnt;
    slot_base[i + 1] = slot_base[i] + slots[i];
    vec_off[i] = vec_elems;   // bytes
    vec_elems += (size_t)slots[i] * (b->fp64 ? partial_bytes<double>(b->n_pad[i]) : partial_bytes<float>(b->n_pad[i]));
  }
  const int G = std::max(1, std::min((int)items.size(), p.grid_mult * b->cus));
  std::vector<std::vector<int>> per_wg(G);
  std::vector<int> order(items.size());
  std::iota(order.begin(), order.end(), 0);
  if (p.lpt) {
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return items[a].cost > items[c].cost; });
    std::vector<double> load(G, 0.0);
    for (int k : order) {
      int best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      per_wg[best].push_back(k);
      load[best] += items[k].cost;
    }
  } else {
    for (size_t k = 0; k < items.size(); ++k) per_wg[k % G].push_back((int)k);
  }
  std::vector<Item> flat;
  std::vector<int> wgoff(G + 1, 0);
  for (int g = 0; g < G; ++g) {
    wgoff[g] = (int)flat.size();
    for (int k : per_wg[g]) flat.push_back(items[k].it);
  }
  wgoff[G] = (int)flat.size();
  size_t lds = 0;
  if (p.engine == 4) lds = 0;   // static LDS
  else if (p.engine == 2) lds = engine2_lds_bytes((size_t)lbuf, bmax);
  else
    for (int i = 0; i < b->W; ++i) lds = std::max(lds, engine_lds_bytes(p.cfg, ts[i], b->fp64));

  bdrop_graphs(b);
  b->pmem.release();
  BHIP_TRY(b, b->pmem.alloc((void**)&b->hdr, (size_t)slot_base[b->W] * 4 * sizeof(double)));
  BHIP_TRY(b, b->pmem.alloc(&b->vec, vec_elems));
  BHIP_TRY(b, b->pmem.alloc((void**)&b->d_prob, b->W * sizeof(Problem)));
  BHIP_TRY(b, b->pmem.alloc((void**)&b->d_items, flat.size() * sizeof(Item)));
  BHIP_TRY(b, b->pmem.alloc((void**)&b->d_wgoff, (G + 1) * sizeof(int)));
  std::vector<Problem> probs(b->W);
  size_t a_off = 0;
  for (int i = 0; i < b->W; ++i) {
    const size_t lo = b->lm_off[i], po = b->pad_off[i];
    Problem P{};
    P.A = (const char*)b->A + a_off * tsz;
    P.ca = b->ca + 3 * lo;
    P.Ga = b->Ga + lo;
    P.q = b->q + lo;
    P.w = b->w + po;
    P.xw = b->xw + 3 * po;
    P.Gx = b->Gx + i;
    P.Rxy = nullptr;
    P.Rsave = nullptr;
    P.hdr = b->hdr + (size_t)slot_base[i] * 4;
    P.vec = (char*)b->vec + vec_off[i];
    P.fallbacks = nullptr;
    P.Gx32 = b->Gx32 + i;
    P.xres = b->xres + 3 * i;
    P.xw32 = b->xw32 ? b->xw32 + b->x32_off[i] : nullptr;
    P.n_x = round_up(b->n_pad[i], 256);
    P.bsz = bsz[i];
    P.cg = gsz[i];
    P.n = b->n[i];
    P.n_pad = b->n_pad[i];
    P.L = b->L[i];
    P.ts = ts[i];
    P.n_slots = slots[i];
    P.out_off = b->atom_off[i];
    P.out_idx = i;
    P.lam = b->lam[i];
    P.x_rounded = (!b->fp64 && p.engine != 1) ? 1 : 0;
    P.corr = b->corr + b->corr_off[i];
    probs[i] = P;
    a_off += (size_t)b->L[i] * 3 * b->n_pad[i];
  }
  BHIP_TRY(b, hipMemcpy(b->d_prob, probs.data(), probs.size() * sizeof(Problem), hipMemcpyHostToDevice));
  BHIP_TRY(b, hipMemcpy(b->d_items, flat.data(), flat.size() * sizeof(Item), hipMemcpyHostToDevice));
  BHIP_TRY(b, hipMemcpy(b->d_wgoff, wgoff.data(), wgoff.size() * sizeof(int), hipMemcpyHostToDevice));
  b->plan = p;
  b->lbuf = lbuf;
  b->bmax = bmax;
  b->grid = G;
  b->n_items = (int)flat.size();
  b->lds = lds;
  b->planned = true;
  b->plan_version++;
  b->plan_str = p.str() + " items=" + std::to_string(b->n_items) + " grid=" + std::to_string(G);
  return PCV_OK;
}

template <typename T>
static hipError_t batch_enqueue(pcv_batch* b, hipStream_t st, const void* x, double* sz, void* ds, void* dz) {
  hipError_t e = launch_prep<T>(b->d_prep, x, b->W, *std::max_element(b->n.begin(), b->n.end()), st);
  if (e != hipSuccess) return e;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (b->timing) {
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, st);
  }
  if (b->plan.engine == 4)
    e = launch_engine4<T>(b->plan.spw, b->grid, b->d_prob, b->d_items, b->d_wgoff, MODE_EXACT, nullptr, 0, nullptr, st);
  else
  e = (b->plan.engine == 2)
          ? launch_engine2<T>(b->plan.c2.ncw, b->plan.c2.aptc, b->plan.c2.aptg, b->grid, b->lds, b->lbuf, b->bmax, b->d_prob,
                              b->d_items, b->d_wgoff, MODE_EXACT, nullptr, 0, nullptr, st)
          : launch_engine<T>(b->plan.cfg, b->grid, b->lds, b->d_prob, b->d_items, b->d_wgoff, MODE_EXACT, nullptr,
                             0, nullptr, st);
  if (b->timing) {
    (void)hipEventRecord(e1, st);
    b->ev_pending.emplace_back(e0, e1);
  }
  if (e != hipSuccess) return e;
  Outs o{ds, dz, sz, nullptr};
  return launch_merge_exact<T>(b->d_prob, o, b->W, b->max_n_pad, nullptr, 0, st, !b->fp64 && b->plan.engine != 1);
}

static pcv_status batch_run(pcv_batch* b, const void* x, double* sz, void* ds, void* dz, bool allow_graph) {
  auto enq = [&](hipStream_t st) {
    return b->fp64 ? batch_enqueue<double>(b, st, x, sz, ds, dz) : batch_enqueue<float>(b, st, x, sz, ds, dz);
  };
  if (!b->opt.use_graph || !allow_graph || b->timing) {
    hipError_t e = enq(b->stream);
    return e == hipSuccess ? PCV_OK : bhip(b, e, "batch enqueue");
  }
  const void* key[4] = {x, sz, ds, dz};
  for (auto& g : b->graphs)
    if (g.version == b->plan_version && std::equal(key, key + 4, g.key)) {
      BHIP_TRY(b, hipGraphLaunch(g.exec, b->stream));
      return PCV_OK;
    }
  hipGraph_t graph = nullptr;
  BHIP_TRY(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = enq(b->cap_stream);
  hipError_t e2 = hipStreamEndCapture(b->cap_stream, &graph);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return bhip(b, e, "capture");
  }
  if (e2 != hipSuccess) return bhip(b, e2, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return bhip(b, e, "hipGraphInstantiate");
  if (b->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(b->graphs.front().exec);
    b->graphs.erase(b->graphs.begin());
  }
  pcv_batch::GraphEntry ge;
  std::copy(key, key + 4, ge.key);
  ge.version = b->plan_version;
  ge.exec = exec;
  b->graphs.push_back(ge);
  BHIP_TRY(b, hipGraphLaunch(exec, b->stream));
  return PCV_OK;
}

static bool heuristic_plan2(const pcv_batch* b, BatchPlan* out) {
  const int maxpad = *std::max_element(b->n_pad.begin(), b->n_pad.end());
  int nw[16], ac[16], ag[16], cnt = 0;
  engine2_configs(b->fp64, nw, ac, ag, &cnt);
  for (int k = 0; k < cnt; ++k) {
    const Engine2Cfg c{nw[k], ac[k], ag[k]};
    bool ok = true;
    for (int i = 0; i < b->W && ok; ++i) {
      const int B = e2_batch(b->n_pad[i], b->fp64);
      ok = B > 0 && e2_fits(b->n_pad[i], c) && e2_group(b->n_pad[i], c, B) > 0;
    }
    (void)maxpad;
    if (!ok) continue;
    out->engine = 2;
    out->c2 = c;
    out->per_team = 4;
    out->grid_mult = 1;
    out->lpt = 1;
    return true;
  }
  return false;
}

// Engine 4 holds every FP32 walker of up to 2048 padded atoms.
static bool heuristic_plan4(const pcv_batch* b, BatchPlan* out) {
  if (b->fp64) return false;
  for (int i = 0; i < b->W; ++i)
    if (engine4_lanes(b->n_pad[i], 3) < 1) return false;
  out->engine = 4;
  out->spw = 3;
  out->per_team = 24;
  out->grid_mult = 1;
  out->lpt = 1;
  return true;
}

static BatchPlan heuristic_plan(const pcv_batch* b) {
  BatchPlan p2;
  if (heuristic_plan4(b, &p2)) return p2;
  if (heuristic_plan2(b, &p2)) return p2;
  EngineCfg menu[16];
  int cnt = 0;
  engine_configs(b->fp64, menu, &cnt);
  const int maxn = *std::max_element(b->n.begin(), b->n.end());
  BatchPlan best;
  best.engine = 1;
  double best_cost = 1e300;
  for (int k = 0; k < cnt; ++k) {
    if (team_size(maxn, menu[k]) == 0) continue;
    double c = 0.0;
    for (int i = 0; i < b->W; ++i) c += b->L[i] * landmark_cost(b->n[i], menu[k], team_size(b->n[i], menu[k]));
    if (c < best_cost) {
      best_cost = c;
      best.cfg = menu[k];
    }
  }
  best.per_team = 4;
  best.grid_mult = best.cfg.wg >= 512 ? 1 : 2;
  best.lpt = 1;
  return best;
}

static std::string shape_key(const pcv_batch* b) {
  unsigned long long hsh = 1469598103934665603ull;
  for (int i = 0; i < b->W; ++i) {
    hsh = (hsh ^ (unsigned long long)b->n[i]) * 1099511628211ull;
    hsh = (hsh ^ (unsigned long long)b->L[i]) * 1099511628211ull;
  }
  hipDeviceProp_t prop;
  std::string dev = "unknown";
  if (hipGetDeviceProperties(&prop, b->opt.device) == hipSuccess) dev = prop.gcnArchName;
  std::ostringstream o;
  o << dev << ":" << (b->fp64 ? "f64" : "f32") << ":W" << b->W << ":" << std::hex << hsh;
  return o.str();
}

// Minimal JSON cache: one line per entry,
// "key": "engine wg apt ncw aptc aptg per_team grid_mult lpt spw".
static bool cache_lookup(const char* path, const std::string& key, BatchPlan* p) {
  if (!path) return false;
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  while (std::getline(f, line)) {
    const std::string k = "\"" + key + "\": \"";
    const size_t at = line.find(k);
    if (at == std::string::npos) continue;
    std::istringstream v(line.substr(at + k.size()));
    BatchPlan q;
    if (v >> q.engine >> q.cfg.wg >> q.cfg.apt >> q.c2.ncw >> q.c2.aptc >> q.c2.aptg >> q.per_team >> q.grid_mult >>
        q.lpt >> q.spw) {
      *p = q;
      return true;
    }
  }
  return false;
}

static void cache_store(const char* path, const std::string& key, const BatchPlan& p) {
  if (!path) return;
  std::vector<std::string> lines;
  {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line))
      if (line.find("\"" + key + "\"") == std::string::npos && line.find("\": \"") != std::string::npos)
        lines.push_back(line);
  }
  std::ofstream f(path);
  f << "{\n";
  for (auto& l : lines) {
    std::string t = l;
    while (!t.empty() && (t.back() == ',' || t.back() == ' ')) t.pop_back();
    f << t << ",\n";
  }
  f << "  \"" << key << "\": \"" << p.engine << " " << p.cfg.wg << " " << p.cfg.apt << " " << p.c2.ncw << " "
    << p.c2.aptc << " " << p.c2.aptg << " " << p.per_team << " " << p.grid_mult << " " << p.lpt << " " << p.spw
    << "\"\n}\n";
}

extern "C" pcv_status pcv_batch_plan(pcv_batch* b, int tune, const char* cache_path) {
  if (!b) return PCV_EINVAL;
  if (b->W == 0) return bfail(b, PCV_ESTATE, "no walkers loaded");
  BHIP_TRY(b, hipSetDevice(b->opt.device));
  const BatchPlan base = heuristic_plan(b);
  const std::string key = shape_key(b);
  pcv_status s = batch_apply(b, base);
  if (s != PCV_OK || !tune) return s;

  // Reference outputs of the heuristic plan on probe structures; a plan is
  // eligible (a cached one included) only if its s, z and both gradients
  // match them.
  const size_t tsz = b->fp64 ? 8 : 4;
  const int natoms = b->atom_off[b->W];
  void *x = nullptr, *ds = nullptr, *dz = nullptr, *ds_ref = nullptr, *dz_ref = nullptr;
  double *sz = nullptr, *sz_ref = nullptr;
  DevMem tmp;
  BHIP_TRY(b, tmp.alloc(&x, (size_t)natoms * 3 * tsz));
  BHIP_TRY(b, tmp.alloc(&ds, (size_t)natoms * 3 * tsz));
  BHIP_TRY(b, tmp.alloc(&dz, (size_t)natoms * 3 * tsz));
  BHIP_TRY(b, tmp.alloc(&ds_ref, (size_t)natoms * 3 * tsz));
  BHIP_TRY(b, tmp.alloc(&dz_ref, (size_t)natoms * 3 * tsz));
  BHIP_TRY(b, tmp.alloc((void**)&sz, (size_t)b->W * 2 * sizeof(double)));
  BHIP_TRY(b, tmp.alloc((void**)&sz_ref, (size_t)b->W * 2 * sizeof(double)));
  {
    // Probe structures: the midpoint of every walker's first two landmarks
    // (as stored) moved by a fixed pattern of up to 2 pm per coordinate, so
    // the weights spread over several landmarks and every gradient term is
    // exercised.
    size_t a_off = 0;
    std::vector<double> host((size_t)natoms * 3);
    for (int i = 0; i < b->W; ++i) {
      const int n_pad = b->n_pad[i];
      const int two = b->L[i] >= 2 ? 2 : 1;
      std::vector<char> soa((size_t)two * 3 * n_pad * tsz);
      BHIP_TRY(b, hipMemcpy(soa.data(), (const char*)b->A + a_off * tsz, soa.size(), hipMemcpyDeviceToHost));
      auto at = [&](int l, int d, int j) {
        const size_t k = ((size_t)l * 3 + d) * n_pad + j;
        return b->fp64 ? ((const double*)soa.data())[k] : (double)((const float*)soa.data())[k];
      };
      for (int j = 0; j < b->n[i]; ++j)
        for (int d = 0; d < 3; ++d) {
          const double mid = 0.5 * (at(0, d, j) + at(two - 1, d, j));
          const double pattern = 0.002 * ((double)((j * 7 + d * 3 + i) % 11) - 5.0) / 5.0;
          host[(size_t)(b->atom_off[i] + j) * 3 + d] = mid + pattern;
        }
      a_off += (size_t)b->L[i] * 3 * n_pad;
    }
    if (b->fp64) {
      BHIP_TRY(b, hipMemcpy(x, host.data(), host.size() * 8, hipMemcpyHostToDevice));
    } else {
      std::vector<float> h32(host.begin(), host.end());
      BHIP_TRY(b, hipMemcpy(x, h32.data(), h32.size() * 4, hipMemcpyHostToDevice));
    }
  }
  s = batch_run(b, x, sz_ref, ds_ref, dz_ref, false);
  if (s != PCV_OK) return s;
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  std::vector<double> hsz_ref(2 * b->W), hsz(2 * b->W);
  BHIP_TRY(b, hipMemcpy(hsz_ref.data(), sz_ref, hsz_ref.size() * sizeof(double), hipMemcpyDeviceToHost));
  auto to_f64 = [&](const void* dev_p, std::vector<double>& out) -> bool {
    out.resize((size_t)natoms * 3);
    if (b->fp64) return hipMemcpy(out.data(), dev_p, out.size() * 8, hipMemcpyDeviceToHost) == hipSuccess;
    std::vector<float> t(out.size());
    if (hipMemcpy(t.data(), dev_p, t.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) return false;
    std::copy(t.begin(), t.end(), out.begin());
    return true;
  };
  std::vector<double> hds_ref, hdz_ref, hds, hdz;
  if (!to_f64(ds_ref, hds_ref) || !to_f64(dz_ref, hdz_ref)) return bfail(b, PCV_EHIP, "autotuner reference copy");
  // The applied plan reproduces the reference: s and z to 1e-7 (relative to
  // 1 + |value|), each walker's gradients to 1e-5 of its largest entry.
  auto matches = [&]() -> bool {
    if (batch_run(b, x, sz, ds, dz, false) != PCV_OK) return false;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return false;
    if (hipMemcpy(hsz.data(), sz, hsz.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return false;
    for (int i = 0; i < 2 * b->W; ++i)
      if (!(std::fabs(hsz[i] - hsz_ref[i]) <= 1e-7 * (1 + std::fabs(hsz_ref[i])))) return false;
    if (!to_f64(ds, hds) || !to_f64(dz, hdz)) return false;
    for (int w = 0; w < b->W; ++w) {
      const size_t a0 = (size_t)b->atom_off[w] * 3, a1 = (size_t)b->atom_off[w + 1] * 3;
      for (int g = 0; g < 2; ++g) {
        const std::vector<double>& r = g ? hdz_ref : hds_ref;
        const std::vector<double>& v = g ? hdz : hds;
        double scale = 0.0;
        for (size_t k = a0; k < a1; ++k) scale = std::max(scale, std::fabs(r[k]));
        for (size_t k = a0; k < a1; ++k)
          if (!(std::fabs(v[k] - r[k]) <= 1e-5 * scale + 1e-12)) return false;
      }
    }
    return true;
  };
  // A cached plan is applied only after it reproduces the reference here.
  BatchPlan cached;
  if (cache_lookup(cache_path, key, &cached)) {
    if (batch_apply(b, cached) == PCV_OK && matches()) return PCV_OK;
    s = batch_apply(b, base);
    if (s != PCV_OK) return s;
  }

  EngineCfg menu[16];
  int cnt = 0;
  engine_configs(b->fp64, menu, &cnt);
  int nw[16], ac[16], ag[16], cnt2 = 0;
  engine2_configs(b->fp64, nw, ac, ag, &cnt2);
  const int maxn = *std::max_element(b->n.begin(), b->n.end());
  std::vector<BatchPlan> cands{base};   // the heuristic plan competes too
  if (!b->fp64)
    for (int spw : {3, 2})
      for (int per : {8, 16, 24, 32, 64})
        for (int lpt : {1, 0}) {
          BatchPlan c;
          c.engine = 4;
          c.spw = spw;
          c.per_team = per;
          c.grid_mult = 1;
          c.lpt = lpt;
          cands.push_back(c);
        }
  for (int k = 0; k < cnt2; ++k)
    for (int per : {1, 2, 4, 8})
      for (int gm : {1, 2})
        for (int lpt : {1, 0}) {
          BatchPlan c;
          c.engine = 2;
          c.c2 = Engine2Cfg{nw[k], ac[k], ag[k]};
          c.per_team = per;
          c.grid_mult = gm;
          c.lpt = lpt;
          cands.push_back(c);
        }
  for (int k = 0; k < cnt; ++k) {
    if (team_size(maxn, menu[k]) == 0) continue;
    for (int per : {1, 4, 16})
      for (int gm : {1, 2}) {
        BatchPlan c;
        c.engine = 1;
        c.cfg = menu[k];
        c.per_team = per;
        c.grid_mult = gm;
        c.lpt = 1;
        cands.push_back(c);
      }
  }
  hipEvent_t e0, e1;
  BHIP_TRY(b, hipEventCreate(&e0));
  BHIP_TRY(b, hipEventCreate(&e1));
  // Time `reps` back-to-back runs of the applied plan (ms per run).
  auto time_runs = [&](int reps) {
    (void)hipEventRecord(e0, b->stream);
    for (int r = 0; r < reps; ++r) batch_run(b, x, sz, ds, nullptr, false);
    (void)hipEventRecord(e1, b->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms / reps;
  };
  // Screen: every candidate whose s, z and gradients match the heuristic
  // plan's, three runs each.  Then the three fastest are timed again, ten
  // runs in each of three interleaved rounds, and the best round decides.
  std::vector<std::pair<float, int>> screened;
  for (int k = 0; k < (int)cands.size(); ++k) {
    if (batch_apply(b, cands[k]) != PCV_OK) continue;
    if (!matches()) continue;
    screened.emplace_back(time_runs(3), k);
  }
  std::sort(screened.begin(), screened.end());
  if (screened.size() > 3) screened.resize(3);
  std::vector<float> best_round(screened.size(), 1e30f);
  for (int round = 0; round < 3; ++round)
    for (size_t r = 0; r < screened.size(); ++r) {
      if (batch_apply(b, cands[screened[r].second]) != PCV_OK) continue;
      batch_run(b, x, sz, ds, nullptr, false);
      best_round[r] = std::min(best_round[r], time_runs(10));
    }
  BatchPlan best = base;
  float best_ms = 1e30f;
  for (size_t r = 0; r < screened.size(); ++r)
    if (best_round[r] < best_ms) {
      best_ms = best_round[r];
      best = cands[screened[r].second];
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tmp.release();
  cache_store(cache_path, key, best);
  return batch_apply(b, best);
}

extern "C" pcv_status pcv_batch_eval(pcv_batch* b, const void* x_all, double* sz_all, void* ds_all, void* dz_all) {
  if (!b) return PCV_EINVAL;
  if (b->W == 0) return bfail(b, PCV_ESTATE, "no walkers loaded");
  if (!x_all || !sz_all) return bfail(b, PCV_EINVAL, "x_all and sz_all are required");
  if (!b->planned) {
    pcv_status s = batch_apply(b, heuristic_plan(b));
    if (s != PCV_OK) return s;
  }
  return batch_run(b, x_all, sz_all, ds_all, dz_all, true);
}

extern "C" pcv_status pcv_batch_set_kernel_timing(pcv_batch* b, int enable) {
  if (!b) return PCV_EINVAL;
  BHIP_TRY(b, hipSetDevice(b->opt.device));
  bcollect_timing(b);
  b->timing = enable != 0;
  b->timed_ms = 0.0;
  b->timed_launches = 0;
  return PCV_OK;
}

extern "C" pcv_status pcv_batch_get_kernel_timing(pcv_batch* b, double* engine_ms, int64_t* engine_launches) {
  if (!b || !engine_ms || !engine_launches) return PCV_EINVAL;
  BHIP_TRY(b, hipSetDevice(b->opt.device));
  bcollect_timing(b);
  *engine_ms = b->timed_ms;
  *engine_launches = b->timed_launches;
  return PCV_OK;
}

extern "C" const char* pcv_batch_plan_string(const pcv_batch* b) { return b ? b->plan_str.c_str() : ""; }
extern "C" const char* pcv_batch_last_error(const pcv_batch* b) { return b ? b->err.c_str() : "null batch"; }
