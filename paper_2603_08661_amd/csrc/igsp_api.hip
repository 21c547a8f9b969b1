// Host layer of libigsp: the C ABI entry points, the plan cache (device view
// tables, work lists, median workspaces, intermediate maps), the launch
// sequence of each form, and the graph-captured densification step.
#include <algorithm>
#include <cstdio>
#include <string>
#include <tuple>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "igsp_internal.h"
#include "validate.h"

namespace igsp {
namespace {

// Slots (248 pixels each) per work-group of the element-wise passes, about
// 4 Ki pixels (measured best for normalisation), per work-group of the
// median's refinement passes (coarser: each work-group clears and flushes a
// histogram) and per element-wise task of the persistent form.
constexpr int kChunkSlots = 16;
constexpr int kPersistChunkSlots = 264;
// Distance, in tasks, between a view's phases in the persistent task list, as
// a multiple of the resident work-groups: a task handed out that many
// positions later finds the earlier phase finished.
constexpr int kLagGenerations = 3;
constexpr int kMaxPlans = 8;

std::mutex g_mu;

struct DeviceInfo {
  bool checked = false;
  bool ok = false;
};
constexpr int kMaxDevices = 64;
DeviceInfo g_dev[kMaxDevices];  // a fixed table: checking a device allocates nothing

igsp_status check_device(int* dev_out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return IGSP_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return IGSP_ERR_UNSUPPORTED;
  DeviceInfo& d = g_dev[dev];
  if (!d.checked) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return IGSP_ERR_HIP;
    d.ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    d.checked = true;
  }
  *dev_out = dev;
  return d.ok ? IGSP_OK : IGSP_ERR_UNSUPPORTED;
}

template <class T>
hipError_t upload(T** dptr, const std::vector<T>& v) {
  *dptr = nullptr;
  if (v.empty()) return hipSuccess;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dptr), v.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

// ------------------------------------------------------------------ edge

struct EdgeKey {
  int device;
  int precision, seg_rows, wg_waves;
  std::vector<igsp_view> views;
  bool operator==(const EdgeKey& o) const {
    if (device != o.device || precision != o.precision || seg_rows != o.seg_rows || wg_waves != o.wg_waves ||
        views.size() != o.views.size())
      return false;
    return std::memcmp(views.data(), o.views.data(), views.size() * sizeof(igsp_view)) == 0;
  }
};

struct EdgePlan {
  EdgeKey key;
  int n_views = 0;
  ViewDesc* d_views = nullptr;
  EdgeItem* d_items = nullptr;
  EdgeItem* d_items_all = nullptr;  // the same items in the order of a launch over every view
  RowChunk* d_chunks = nullptr;
  RowChunk* d_rchunks = nullptr;  // the refinement passes' coarser chunks
  uint32_t* d_cand = nullptr;     // FP32: median candidates and their counts per view
  uint32_t* d_cand_n = nullptr;
  std::vector<int> item_begin, chunk_begin, rchunk_begin;  // per view, size n_views + 1
  void* d_map = nullptr;
  uint32_t* d_hist = nullptr;
  uint32_t* d_rhist = nullptr;
  MedState* d_state = nullptr;
  // persistent form (built on first use): its own coarser row chunks, the
  // ordered task list, per-view phase counters and the queue
  RowChunk* d_pchunks = nullptr;
  PTask* d_tasks = nullptr;
  PViewSync* d_sync = nullptr;
  PCtl* d_ctl = nullptr;
  int n_tasks = 0, grid = 0, lag = 0;
  // unfused form (built on first use): its tiles and per-step buffers
  UfLaunch uf{};
  int64_t map_elems = 0;
  ~EdgePlan() {
    (void)hipFree(d_views); (void)hipFree(d_items); (void)hipFree(d_items_all); (void)hipFree(d_chunks);
    (void)hipFree(d_rchunks); (void)hipFree(d_cand); (void)hipFree(d_cand_n); (void)hipFree(d_map);
    (void)hipFree(d_hist); (void)hipFree(d_rhist); (void)hipFree(d_state);
    (void)hipFree(d_pchunks); (void)hipFree(d_tasks); (void)hipFree(d_sync); (void)hipFree(d_ctl);
    (void)hipFree(const_cast<UfItem*>(uf.items)); (void)hipFree(uf.gray); (void)hipFree(uf.blur);
    (void)hipFree(uf.mag); (void)hipFree(uf.code);
  }
};

std::list<std::shared_ptr<EdgePlan>> g_edge_plans;  // most recently used first

int default_wg_waves() { return 4; }

// Compute units of the current device (256 where none can be queried).
int device_cus() {
  static std::mutex mu;
  static std::map<int, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
  return cache[dev] = cus;
}

// Segment height when none is given or tuned: the tallest of a few heights
// that still gives a stencil launch 16 wavefronts per CU (four per SIMD),
// else the shortest. A wavefront's march is a chain of dependent rows, so a
// launch with fewer wavefronts than the chip holds lasts about one segment:
// shorter segments then save more time than their extra halo rows cost. The
// plain form launches each view on its own, so it counts per view. (Each
// height plus the 8 halo rows is a multiple of the loop's 6-row unroll.)
int default_seg_rows(const igsp_view* views, int32_t n, int form) {
  static const int kHeights[] = {64, 40, 28, 22, 16, 10};
  const int64_t target = 16 * (int64_t)device_cus();
  for (int seg : kHeights) {
    int64_t waves = 0;
    for (int i = 0; i < n; ++i)
      waves += (int64_t)((views[i].width + kStripCols - 1) / kStripCols) * ((views[i].height + seg - 1) / seg);
    if (form == IGSP_PLAIN && n > 0) waves /= n;
    if (waves >= target) return seg;
  }
  return kHeights[sizeof(kHeights) / sizeof(kHeights[0]) - 1];
}

// ------------------------------------------------------------------ tuning

// Size class of a batch: tuned tile shapes apply to geometries in the same
// class (device architecture, precision, form, total pixels and mean width
// rounded to powers of two).
struct TuneKey {
  std::string arch;
  int precision, batched, log2_px, log2_w;
  bool operator<(const TuneKey& o) const {
    return std::tie(arch, precision, batched, log2_px, log2_w) <
           std::tie(o.arch, o.precision, o.batched, o.log2_px, o.log2_w);
  }
};
struct TuneVal {
  int seg_rows, wg_waves, form;
  double ms;
};
std::map<TuneKey, TuneVal> g_tuned;
bool g_tune_loaded = false;

int ilog2(int64_t v) {
  int r = 0;
  while (v > 1) { v >>= 1; ++r; }
  return r;
}

// Architecture name of the current device ("gfx950"), cached per device.
std::string device_arch() {
  static std::mutex mu;
  static std::map<int, std::string> cache;
  std::lock_guard<std::mutex> lk(mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  return cache[dev] = a.substr(0, a.find(':'));
}

TuneKey tune_key(const igsp_view* views, int32_t n, int precision, int batched) {
  int64_t px = 0, w = 0;
  for (int i = 0; i < n; ++i) {
    px += (int64_t)views[i].width * views[i].height;
    w += views[i].width;
  }
  return TuneKey{device_arch(), precision, batched, ilog2(std::max<int64_t>(px, 1)),
                 ilog2(std::max<int64_t>(w / std::max(n, 1), 1))};
}

// The cache file: one JSON object per line,
// {"arch":"gfx950","precision":2,"batched":1,"log2_px":29,"log2_w":10,"seg_rows":64,"wg_waves":4,
//  "form":3,"ms":1.3}
void read_tune_file(const char* path) {
  if (!path || !*path) return;
  std::FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[512], arch[64];
  while (std::fgets(line, sizeof(line), f)) {
    TuneKey k;
    TuneVal v;
    if (std::sscanf(line,
                    " {\"arch\":\"%63[^\"]\",\"precision\":%d,\"batched\":%d,\"log2_px\":%d,\"log2_w\":%d,"
                    "\"seg_rows\":%d,\"wg_waves\":%d,\"form\":%d,\"ms\":%lf",
                    arch, &k.precision, &k.batched, &k.log2_px, &k.log2_w, &v.seg_rows, &v.wg_waves, &v.form,
                    &v.ms) != 9)
      continue;
    const bool ok = k.precision >= IGSP_FP32 && k.precision <= IGSP_BF16 && k.batched >= IGSP_PLAIN &&
                    k.batched <= IGSP_BATCHED_PERSISTENT && v.seg_rows >= 8 && v.seg_rows <= 4096 &&
                    (v.wg_waves == 1 || v.wg_waves == 2 || v.wg_waves == 4 || v.wg_waves == 8) &&
                    v.form >= IGSP_PLAIN && v.form <= IGSP_BATCHED_PERSISTENT && v.form != IGSP_BATCHED;
    if (!ok) continue;  // malformed entries are ignored
    k.arch = arch;
    g_tuned[k] = v;
  }
  std::fclose(f);
}

// Tuned entries: first the shipped table (IGSP_TUNE_DEFAULTS, read only), then
// the caller's cache (IGSP_TUNE_CACHE), whose entries win.
void load_tune_cache() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  read_tune_file(std::getenv("IGSP_TUNE_DEFAULTS"));
  read_tune_file(std::getenv("IGSP_TUNE_CACHE"));
}

void save_tune_cache() {
  const char* path = std::getenv("IGSP_TUNE_CACHE");
  if (!path || !*path) return;
  std::FILE* f = std::fopen(path, "w");
  if (!f) return;
  for (const auto& kv : g_tuned)
    std::fprintf(f,
                 "{\"arch\":\"%s\",\"precision\":%d,\"batched\":%d,\"log2_px\":%d,\"log2_w\":%d,"
                 "\"seg_rows\":%d,\"wg_waves\":%d,\"form\":%d,\"ms\":%.6f}\n",
                 kv.first.arch.c_str(), kv.first.precision, kv.first.batched, kv.first.log2_px, kv.first.log2_w,
                 kv.second.seg_rows, kv.second.wg_waves, kv.second.form, kv.second.ms);
  std::fclose(f);
}

// Chunks of a view's slots (one strip's stored row each, 248 pixels) with
// `slots` slots each, the last one shorter.
void row_chunks(int v, int W, int H, int slots, std::vector<RowChunk>* out) {
  const int64_t n = (int64_t)H * ((W + kStripCols - 1) / kStripCols);
  for (int64_t u0 = 0; u0 < n; u0 += slots) out->push_back(RowChunk{v, (int32_t)u0, (int32_t)std::min(n, u0 + slots), 0});
}

igsp_status build_edge_plan(const EdgeKey& key, std::shared_ptr<EdgePlan>* out) {
  auto plan = std::make_shared<EdgePlan>();
  plan->key = key;
  const int n = (int)key.views.size();
  plan->n_views = n;
  const int band = key.seg_rows * key.wg_waves;
  const int esz = key.precision == IGSP_FP32 ? 4 : 2;
  std::vector<ViewDesc> vd(n);
  std::vector<EdgeItem> items;
  std::vector<RowChunk> chunks, rchunks;
  plan->item_begin.resize(n + 1);
  plan->chunk_begin.resize(n + 1);
  plan->rchunk_begin.resize(n + 1);
  int64_t map_elems = 0, cand_elems = 0;
  for (int v = 0; v < n; ++v) {
    const igsp_view& d = key.views[v];
    // the stored map, strip by strip (each strip's rows one after another,
    // in slots of 256 values)
    const int strips = (d.width + kStripCols - 1) / kStripCols;
    vd[v] = ViewDesc{d.width, d.height, d.in_offset, d.out_offset, map_elems, d.height, 0, cand_elems};
    if (key.precision == IGSP_FP32) {
      // room for 1/16 of the view's pixels: the first histogram's median
      // bucket (1/128 of a binade) holds far fewer survivors unless the
      // view's magnitudes are nearly all equal, and then the list is not used
      const int64_t px = (int64_t)d.width * d.height;
      vd[v].cand_cap = (int32_t)std::min<int64_t>(std::max<int64_t>(px / 16, 256), INT32_MAX);
      cand_elems += vd[v].cand_cap;
    }
    map_elems += (int64_t)strips * d.height * kSlotPitch;
    plan->item_begin[v] = (int)items.size();
    for (int x0 = 0; x0 < d.width; x0 += kStripCols)
      for (int y0 = 0; y0 < d.height; y0 += band)
        items.push_back(EdgeItem{v, x0, y0, std::min(band, d.height - y0)});
    plan->chunk_begin[v] = (int)chunks.size();
    row_chunks(v, d.width, d.height, kChunkSlots, &chunks);
    plan->rchunk_begin[v] = (int)rchunks.size();
    row_chunks(v, d.width, d.height, kRefineChunkSlots, &rchunks);
  }
  plan->item_begin[n] = (int)items.size();
  plan->chunk_begin[n] = (int)chunks.size();
  plan->rchunk_begin[n] = (int)rchunks.size();
  plan->map_elems = map_elems;
  // A launch over every view gives each XCD a contiguous eighth of the list
  // (the kernel's block remap); inside each eighth, full bands come first and
  // the shorter last bands of the strips after them, longest first, so the
  // short waves fill the XCD while its last long ones finish.
  std::vector<EdgeItem> all(items);
  {
    const int64_t ni = (int64_t)all.size(), q = ni >> 3, r = ni & 7;
    for (int64_t x = 0, b = 0; x < 8; ++x) {
      const int64_t e = b + q + (x < r ? 1 : 0);
      std::stable_sort(all.begin() + b, all.begin() + e,
                       [](const EdgeItem& u, const EdgeItem& v) { return u.rows > v.rows; });
      b = e;
    }
  }
  if (upload(&plan->d_views, vd) != hipSuccess || upload(&plan->d_items, items) != hipSuccess ||
      upload(&plan->d_items_all, all) != hipSuccess ||
      upload(&plan->d_chunks, chunks) != hipSuccess || upload(&plan->d_rchunks, rchunks) != hipSuccess)
    return IGSP_ERR_HIP;
  if (hipMalloc(&plan->d_map, (size_t)std::max<int64_t>(map_elems, 64) * esz) != hipSuccess) return IGSP_ERR_HIP;
  if (cand_elems > 0 &&
      (hipMalloc(reinterpret_cast<void**>(&plan->d_cand), (size_t)cand_elems * sizeof(uint32_t)) != hipSuccess ||
       hipMalloc(reinterpret_cast<void**>(&plan->d_cand_n), (size_t)n * sizeof(uint32_t)) != hipSuccess))
    return IGSP_ERR_HIP;
  // refinement histograms of up to two passes, selection states after 0, 1
  // and 2 refinement steps
  const size_t hb = (size_t)n * kBinsMax * sizeof(uint32_t), rb = (size_t)2 * n * kRefineBins * sizeof(uint32_t),
               sb = (size_t)3 * n * sizeof(MedState);
  if (hipMalloc(reinterpret_cast<void**>(&plan->d_hist), hb) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&plan->d_rhist), rb) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&plan->d_state), sb) != hipSuccess)
    return IGSP_ERR_HIP;
  // Histograms start at zero once; every call's selection kernels clear them
  // again after reading, so later calls need no memset (capturable).
  if (hipMemset(plan->d_hist, 0, hb) != hipSuccess || hipMemset(plan->d_rhist, 0, rb) != hipSuccess ||
      hipMemset(plan->d_state, 0, sb) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess)
    return IGSP_ERR_HIP;
  g_edge_plans.push_front(std::move(plan));
  while ((int)g_edge_plans.size() > kMaxPlans) g_edge_plans.pop_back();
  *out = g_edge_plans.front();
  return IGSP_OK;
}

// Task list of the persistent form: phase p of view v is emitted at step
// v + p * lag, so each phase follows the one before it by `lag` views of
// other work (topological order: every task comes after what it waits for).
igsp_status ensure_persistent(EdgePlan* P) {
  if (P->d_tasks) return IGSP_OK;
  const int n = P->n_views;
  const int prec = P->key.precision;
  const int levels = prec == IGSP_FP16 ? 1 : (prec == IGSP_FP32 ? 2 : 0);
  const int phases = levels + 2;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return IGSP_ERR_HIP;
  const int per_cu = persistent_blocks_per_cu(prec, P->key.wg_waves);
  if (per_cu <= 0 || cus <= 0) return IGSP_ERR_HIP;
  std::vector<RowChunk> pchunks;
  std::vector<int> pchunk_begin(n + 1);
  for (int v = 0; v < n; ++v) {
    pchunk_begin[v] = (int)pchunks.size();
    row_chunks(v, P->key.views[v].width, P->key.views[v].height, kPersistChunkSlots, &pchunks);
  }
  pchunk_begin[n] = (int)pchunks.size();
  // resident work-groups, but no more than there are tasks (a small batch
  // then starts and retires only the work-groups it can use)
  const int64_t total = (int64_t)P->item_begin[n] + (int64_t)(phases - 1) * pchunk_begin[n];
  P->grid = (int)std::min<int64_t>((int64_t)per_cu * cus, std::max<int64_t>(total, 1));
  const int64_t per_view = ((int64_t)P->item_begin[n] + (int64_t)(phases - 1) * pchunk_begin[n]) / std::max(n, 1);
  P->lag = (int)std::min<int64_t>(std::max<int64_t>(1, ((int64_t)kLagGenerations * P->grid + per_view - 1) /
                                                           std::max<int64_t>(per_view, 1)),
                                  std::max(n, 1));
  std::vector<PTask> tasks;
  for (int k = 0; k < n + (phases - 1) * P->lag; ++k)
    for (int p = 0; p < phases; ++p) {
      const int v = k - p * P->lag;
      if (v < 0 || v >= n) continue;
      if (p == 0) {
        for (int i = P->item_begin[v]; i < P->item_begin[v + 1]; ++i) tasks.push_back(PTask{kTaskStencil, v, i, 0});
      } else {
        const int type = p <= levels ? kTaskRefine : kTaskNorm;
        for (int f = pchunk_begin[v]; f < pchunk_begin[v + 1]; ++f) tasks.push_back(PTask{type, v, f, p});
      }
    }
  std::vector<PViewSync> sync(n);
  for (int v = 0; v < n; ++v) {
    const uint32_t ni = (uint32_t)(P->item_begin[v + 1] - P->item_begin[v]);
    const uint32_t nf = (uint32_t)(pchunk_begin[v + 1] - pchunk_begin[v]);
    sync[v] = PViewSync{{ni, nf, nf, nf}, 0u, ni, nf, 0u};
  }
  std::vector<PCtl> ctl(1, PCtl{0u, 0u, 0u, 0u});
  P->n_tasks = (int)tasks.size();
  if (upload(&P->d_pchunks, pchunks) != hipSuccess || upload(&P->d_sync, sync) != hipSuccess ||
      upload(&P->d_ctl, ctl) != hipSuccess || upload(&P->d_tasks, tasks) != hipSuccess) {
    (void)hipFree(P->d_pchunks); (void)hipFree(P->d_sync); (void)hipFree(P->d_ctl); (void)hipFree(P->d_tasks);
    P->d_pchunks = nullptr; P->d_sync = nullptr; P->d_ctl = nullptr; P->d_tasks = nullptr;
    return IGSP_ERR_HIP;
  }
  return IGSP_OK;
}

// Tiles and per-step buffers of the unfused form (gray, blur: int32;
// magnitude: float; orientation code: byte; all in the plan's map layout).
igsp_status ensure_unfused(EdgePlan* P) {
  if (P->uf.items) return IGSP_OK;
  std::vector<UfItem> items;
  for (int v = 0; v < P->n_views; ++v) {
    const igsp_view& d = P->key.views[v];
    for (int y0 = 0; y0 < d.height; y0 += kUfRows)
      for (int x0 = 0; x0 < d.width; x0 += kUfCols) items.push_back(UfItem{v, x0, y0, 0});
  }
  UfItem* d_items = nullptr;
  const size_t n = (size_t)std::max<int64_t>(P->map_elems, 64);
  UfLaunch u{};
  if (upload(&d_items, items) != hipSuccess || hipMalloc(reinterpret_cast<void**>(&u.gray), n * 4) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&u.blur), n * 4) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&u.mag), n * 4) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&u.code), n) != hipSuccess) {
    (void)hipFree(d_items); (void)hipFree(u.gray); (void)hipFree(u.blur); (void)hipFree(u.mag);
    (void)hipFree(u.code);
    return IGSP_ERR_HIP;
  }
  u.items = d_items;
  u.n_items = (int32_t)items.size();
  P->uf = u;
  return IGSP_OK;
}

// The concrete form of a call: plain per view, staged batched, or one
// persistent launch. IGSP_BATCHED lets the library choose (tuned, else
// staged).
int resolve_form(const igsp_view* views, int32_t n_views, const igsp_edge_opts* opts) {
  const int b = opts ? opts->batched : IGSP_BATCHED;
  if (b != IGSP_BATCHED) return b;
  load_tune_cache();
  auto it = g_tuned.find(tune_key(views, n_views, opts ? opts->precision : IGSP_FP32, IGSP_BATCHED));
  return it != g_tuned.end() ? it->second.form : IGSP_BATCHED_STAGED;
}

igsp_status get_edge_plan(const igsp_view* views, int32_t n_views, const igsp_edge_opts* opts,
                          std::shared_ptr<EdgePlan>* out) {
  int dev = 0;
  igsp_status st = check_device(&dev);
  if (st != IGSP_OK) return st;
  EdgeKey key;
  key.device = dev;
  key.precision = opts ? opts->precision : IGSP_FP32;
  const int form = resolve_form(views, n_views, opts);
  int seg = default_seg_rows(views, n_views, form), wgw = default_wg_waves();
  if (!opts || (opts->seg_rows == 0 && opts->wg_waves == 0)) {
    load_tune_cache();
    auto it = g_tuned.find(tune_key(views, n_views, key.precision, opts ? opts->batched : IGSP_BATCHED));
    if (it != g_tuned.end()) {
      seg = it->second.seg_rows;
      wgw = it->second.wg_waves;
    }
  }
  key.seg_rows = (opts && opts->seg_rows) ? opts->seg_rows : seg;
  key.wg_waves = (opts && opts->wg_waves) ? opts->wg_waves : wgw;
  key.views.assign(views, views + n_views);
  auto extras = [form](EdgePlan* P) -> igsp_status {
    if (form == IGSP_BATCHED_PERSISTENT) return ensure_persistent(P);
    if (form == IGSP_UNFUSED) return ensure_unfused(P);
    return IGSP_OK;
  };
  for (auto it = g_edge_plans.begin(); it != g_edge_plans.end(); ++it) {
    if ((*it)->key == key) {
      g_edge_plans.splice(g_edge_plans.begin(), g_edge_plans, it);
      *out = g_edge_plans.front();
      return extras(out->get());
    }
  }
  st = build_edge_plan(key, out);
  if (st == IGSP_OK) st = extras(out->get());
  return st;
}

igsp_status enqueue_edge(EdgePlan* P, const uint8_t* images, int64_t img_end, float* out_maps,
                         const igsp_edge_opts* opts, hipStream_t s) {
  EdgeLaunch L;
  L.images = images;
  L.img_end = img_end;
  L.out = out_maps;
  L.views = P->d_views;
  L.items = P->d_items;
  L.chunks = P->d_chunks;
  L.map = P->d_map;
  L.hist = P->d_hist;
  L.rhist = P->d_rhist;
  L.state = P->d_state;
  L.cand = P->d_cand;
  L.cand_n = P->d_cand_n;
  L.use_cand = 0;
  L.n_views = P->n_views;
  L.medians_dn = opts ? opts->medians : nullptr;
  L.survivors = opts ? opts->survivors : nullptr;
  L.stage_events = opts ? reinterpret_cast<hipEvent_t*>(opts->stage_events) : nullptr;
  L.status = opts ? opts->status : nullptr;
  L.precision = P->key.precision;
  L.wg_waves = P->key.wg_waves;
  L.seg_rows = P->key.seg_rows;
  const int form = resolve_form(P->key.views.data(), P->n_views, opts);
  const bool batched = form != IGSP_PLAIN;
  const int n = P->n_views;
  // refinement passes of the median's radix selection (3-bit digits for
  // FP16, 8-bit for FP32; BF16 is resolved by the first histogram)
  const int passes = L.precision == IGSP_FP16 ? 1 : (L.precision == IGSP_FP32 ? 2 : 0);
  hipEvent_t* ev = L.stage_events;
  auto mark = [&](int k, hipStream_t st) -> hipError_t { return ev ? hipEventRecord(ev[k], st) : hipSuccess; };
  // median selection (+ refinement passes) and normalisation of views [v0, v1)
  auto tail = [&](int v0, int v1, hipStream_t st) -> hipError_t {
    const int f0 = P->rchunk_begin[v0], f1 = P->rchunk_begin[v1];
    EdgeLaunch LR = L;
    LR.chunks = P->d_rchunks;
    // FP32 candidate lists where a launch covers several views (one view's
    // launches are bound by latency, and the list's extra steps cost more
    // than the second pass's bytes: +2% for the plain form, measured)
    LR.use_cand = L.cand && v1 - v0 > 1;
    hipError_t e = launch_median_select(L, v0, v1 - v0, st);
    // each refinement pass takes the previous pass's selection step itself;
    // the last one is taken by a launch of its own or by the normalisation
    for (int p = 0; p < passes && e == hipSuccess; ++p) e = launch_median_refine(LR, f0, f1 - f0, p, st);
    if (e == hipSuccess) e = launch_median_step(L, v0, v1 - v0, st);
    return e;
  };
  auto stencil = [&](int v0, int v1, hipStream_t st) -> hipError_t {
    if (v0 == 0 && v1 == n) {
      EdgeLaunch LA = L;
      LA.items = P->d_items_all;
      return launch_edge_fused(LA, 0, P->item_begin[n], st);
    }
    return launch_edge_fused(L, P->item_begin[v0], P->item_begin[v1] - P->item_begin[v0], st);
  };
  auto norm = [&](int v0, int v1, hipStream_t st) -> hipError_t {
    return launch_normalise(L, P->chunk_begin[v0], P->chunk_begin[v1] - P->chunk_begin[v0], st);
  };
  hipError_t e = mark(0, s);
  if (e == hipSuccess && form == IGSP_BATCHED_PERSISTENT) {
    if (!P->d_tasks) return IGSP_ERR_HIP;  // tables are built with the plan
    PersistLaunch PL;
    PL.tasks = P->d_tasks;
    PL.sync = P->d_sync;
    PL.ctl = P->d_ctl;
    PL.n_tasks = P->n_tasks;
    PL.levels = passes;
    PL.n_views = P->n_views;
    PL.spin_limit = kSpinLimit;
    PL.wait_bias = 0;
    // Test facility: IGSP_PERSIST_FORCE_TIMEOUT=1 makes every wait of the
    // persistent form give up after a few polls (the level it waits for is
    // never reached), so the timeout path runs and every kernel still exits.
    const char* force = std::getenv("IGSP_PERSIST_FORCE_TIMEOUT");
    if (force && force[0] == '1') {
      PL.spin_limit = 16;
      PL.wait_bias = 1u << 24;
    }
    EdgeLaunch LP = L;
    LP.chunks = P->d_pchunks;
    e = launch_edge_persistent(LP, PL, P->grid, s);
    for (int k = 1; k < 4 && e == hipSuccess; ++k) e = mark(k, s);
  } else if (e == hipSuccess && form == IGSP_UNFUSED) {
    if (!P->uf.items) return IGSP_ERR_HIP;  // buffers are built with the plan
    e = launch_edge_unfused(L, P->uf, s);
    if (e == hipSuccess) e = mark(1, s);
    if (e == hipSuccess) e = tail(0, n, s);
    if (e == hipSuccess) e = mark(2, s);
    if (e == hipSuccess) e = norm(0, n, s);
    if (e == hipSuccess) e = mark(3, s);
  } else if (e == hipSuccess && batched) {
    e = stencil(0, n, s);
    if (e == hipSuccess) e = mark(1, s);
    if (e == hipSuccess) e = tail(0, n, s);
    if (e == hipSuccess) e = mark(2, s);
    if (e == hipSuccess) e = norm(0, n, s);
    if (e == hipSuccess) e = mark(3, s);
  } else if (e == hipSuccess) {
    for (int v = 0; v < n && e == hipSuccess; ++v) {
      e = stencil(v, v + 1, s);
      if (e == hipSuccess) e = tail(v, v + 1, s);
      if (e == hipSuccess) e = norm(v, v + 1, s);
    }
    for (int k = 1; k < 4 && e == hipSuccess; ++k) e = mark(k, s);
  }
  return e == hipSuccess ? IGSP_OK : IGSP_ERR_HIP;
}

// ------------------------------------------------------------------ LAS

struct LasPlan {
  int device = 0;
  int n_blocks = 0;
  int32_t* d_counts = nullptr;
  int64_t* d_offsets = nullptr;
  LasScalars* d_scalars = nullptr;
  ~LasPlan() { (void)hipFree(d_counts); (void)hipFree(d_offsets); (void)hipFree(d_scalars); }
};
std::list<std::shared_ptr<LasPlan>> g_las_plans;

igsp_status get_las_plan(int64_t capacity, std::shared_ptr<LasPlan>* out) {
  int dev = 0;
  igsp_status st = check_device(&dev);
  if (st != IGSP_OK) return st;
  const int nb = (int)std::max<int64_t>(1, (capacity + kLasRows - 1) / kLasRows);
  for (auto& p : g_las_plans)
    if (p->device == dev && p->n_blocks == nb) {
      *out = p;
      return IGSP_OK;
    }
  auto plan = std::make_shared<LasPlan>();
  plan->device = dev;
  plan->n_blocks = nb;
  if (hipMalloc(reinterpret_cast<void**>(&plan->d_counts), nb * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&plan->d_offsets), nb * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&plan->d_scalars), sizeof(LasScalars)) != hipSuccess)
    return IGSP_ERR_HIP;
  g_las_plans.push_front(std::move(plan));
  *out = g_las_plans.front();
  return IGSP_OK;
}

// The launch description of a split; its workspace fields are left for the
// caller (a plan, or the fixed array of the allocation-free entry point).
LasLaunch las_launch(const igsp_gaussians* g, const igsp_adam_moments* adam, const uint8_t* mask,
                     const igsp_las_out* out, const igsp_las_params* p) {
  const double a = p ? p->alpha : 0.5, gm = p ? p->gamma : 0.85, b = p ? p->beta : 0.6;
  LasLaunch L;
  L.g = *g;
  L.adam = adam ? *adam : igsp_adam_moments{};
  if (g->feat_dim == 0) L.adam.features[0] = L.adam.features[1] = nullptr;
  L.mask = mask;
  L.split_idx = out->split_idx;
  L.status = out->status;
  L.n_split = out->n_split;
  L.alpha = (float)a;
  L.ln_alpha = (float)std::log(a);
  L.ln_gamma = (float)std::log(gm);
  L.ln_beta = (float)std::log(b);
  L.one_minus_beta = (float)(1.0 - b);
  L.block_counts = nullptr;
  L.block_offsets = nullptr;
  L.scalars = nullptr;
  L.n_blocks = (int)std::max<int64_t>(1, (g->capacity + kLasRows - 1) / kLasRows);
  return L;
}

igsp_status enqueue_las(LasPlan* P, const igsp_gaussians* g, const igsp_adam_moments* adam, const uint8_t* mask,
                        const igsp_las_out* out, const igsp_las_params* p, hipStream_t s) {
  LasLaunch L = las_launch(g, adam, mask, out, p);
  L.block_counts = P->d_counts;
  L.block_offsets = P->d_offsets;
  L.scalars = P->d_scalars;
  L.n_blocks = P->n_blocks;
  return launch_las(L, s) == hipSuccess ? IGSP_OK : IGSP_ERR_HIP;
}

}  // namespace

// ------------------------------------------------------------------ allocation-free LAS
//
// Workspace of long_axis_split_noalloc: the per-tile selected counts, their
// exclusive offsets and the split's scalars, in a fixed device array (one
// copy per GPU, held until the process ends). Nothing in it needs to start at
// zero: the count kernel writes every live tile's count, the scan kernel every
// live tile's offset and all the scalars, before anything reads them.
constexpr int64_t kNoAllocCapacity = int64_t(1) << 28;   // rows
constexpr int kNoAllocTiles = (int)(kNoAllocCapacity / kLasRows);
struct LasScratch {
  LasScalars scalars;
  int64_t offsets[kNoAllocTiles];
  int32_t counts[kNoAllocTiles];
};
static_assert(kNoAllocCapacity % kLasRows == 0, "whole tiles");
static_assert(sizeof(LasScratch) < (size_t(2) << 20), "under 2 MiB per GPU");

// In host code this name stands for the array but is not its device
// address: only the pointer hipGetSymbolAddress returns for the current
// device may reach a kernel or a copy.
static __device__ __align__(256) LasScratch scratch;

namespace {

struct ScratchSlot {
  bool resolved = false;
  char* ptr = nullptr;
};
ScratchSlot g_scratch[kMaxDevices];

// The device address of this device's `scratch`, looked up once per device
// with that device current (caller holds g_mu).
igsp_status scratch_of_device(char** out) {
  int dev = 0;
  igsp_status st = check_device(&dev);
  if (st != IGSP_OK) return st;
  ScratchSlot& s = g_scratch[dev];
  if (!s.resolved) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return IGSP_ERR_HIP;
    s.ptr = static_cast<char*>(p);
    s.resolved = true;
  }
  *out = s.ptr;
  return IGSP_OK;
}

// ------------------------------------------------------------------ split mask

struct SelPlan {
  int device = 0;
  int64_t capacity = 0;
  std::vector<igsp_view> views;
  SelView* d_views = nullptr;
  uint32_t* d_hist = nullptr;
  uint32_t* d_counts = nullptr;
  int64_t* d_offsets = nullptr;
  SelState* d_state = nullptr;
  SelRadix* d_ring = nullptr;
  uint64_t* d_ckeys = nullptr;
  ~SelPlan() {
    (void)hipFree(d_views); (void)hipFree(d_hist); (void)hipFree(d_counts); (void)hipFree(d_offsets);
    (void)hipFree(d_state); (void)hipFree(d_ring); (void)hipFree(d_ckeys);
  }
};
std::list<std::shared_ptr<SelPlan>> g_sel_plans;

igsp_status get_sel_plan(const igsp_view* views, int32_t n_views, int64_t capacity,
                         std::shared_ptr<SelPlan>* out) {
  int dev = 0;
  igsp_status st = check_device(&dev);
  if (st != IGSP_OK) return st;
  for (auto it = g_sel_plans.begin(); it != g_sel_plans.end(); ++it) {
    const SelPlan& p = **it;
    if (p.device == dev && p.capacity == capacity && (int32_t)p.views.size() == n_views &&
        (n_views == 0 || std::memcmp(p.views.data(), views, n_views * sizeof(igsp_view)) == 0)) {
      g_sel_plans.splice(g_sel_plans.begin(), g_sel_plans, it);
      *out = g_sel_plans.front();
      return IGSP_OK;
    }
  }
  auto plan = std::make_shared<SelPlan>();
  plan->device = dev;
  plan->capacity = capacity;
  plan->views.assign(views, views + n_views);
  std::vector<SelView> sv(n_views);
  for (int v = 0; v < n_views; ++v) sv[v] = SelView{views[v].out_offset, (int64_t)views[v].width * views[v].height};
  const int64_t tiles = std::max<int64_t>(1, (capacity + kSelTile - 1) / kSelTile);
  // (the radix histograms and the key OR are cleared by each call's first
  // kernel, so the plan needs no memset)
  if (upload(&plan->d_views, sv) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&plan->d_hist), 3 * 256 * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&plan->d_counts), tiles * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&plan->d_offsets), tiles * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&plan->d_state), sizeof(SelState)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&plan->d_ring), 2 * sizeof(SelRadix)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&plan->d_ckeys), std::max<int64_t>(capacity, 1) * sizeof(uint64_t)) !=
          hipSuccess)
    return IGSP_ERR_HIP;
  g_sel_plans.push_front(std::move(plan));
  while ((int)g_sel_plans.size() > kMaxPlans) g_sel_plans.pop_back();
  *out = g_sel_plans.front();
  return IGSP_OK;
}

}  // namespace
}  // namespace igsp

using namespace igsp;

extern "C" igsp_status split_mask(const float* maps, const igsp_view* views, int32_t n_views,
                                  const igsp_contributions* contrib, const float* grad, const int64_t* count,
                                  int64_t capacity, const igsp_select_params* params, uint8_t* mask,
                                  int64_t* scores, int64_t* n_selected, void* stream) {
  igsp_status st = validate_select(maps, views, n_views, contrib, grad, count, capacity, params, mask, scores);
  if (st != IGSP_OK) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  std::shared_ptr<SelPlan> plan;
  st = get_sel_plan(views, n_views, capacity, &plan);
  if (st != IGSP_OK) return st;
  SelLaunch S{};
  S.maps = maps;
  S.views = plan->d_views;
  S.n_views = n_views;
  S.gauss = contrib->gauss;
  S.view = contrib->view;
  S.pixel = contrib->pixel;
  S.weight = contrib->weight;
  S.n_contrib = contrib->n;
  S.grad = grad;
  S.count = count;
  S.capacity = capacity;
  S.grad_threshold = params->grad_threshold;
  S.warmup = params->warmup;
  S.budget = params->budget;
  S.mask = mask;
  S.scores = scores;
  S.n_selected = n_selected;
  S.hist = plan->d_hist;
  S.tile_counts = plan->d_counts;
  S.tile_offsets = plan->d_offsets;
  S.state = plan->d_state;
  S.ring = plan->d_ring;
  S.ckeys = plan->d_ckeys;
  const int64_t tiles = std::max<int64_t>(1, (capacity + kSelTile - 1) / kSelTile);
  S.grid = (int)std::min<int64_t>(tiles, kSelGrid);
  return launch_select(S, static_cast<hipStream_t>(stream)) == hipSuccess ? IGSP_OK : IGSP_ERR_HIP;
}

extern "C" int32_t igsp_version(void) { return 1; }

extern "C" igsp_status edge_importance(const uint8_t* images, const igsp_view* views, int32_t n_views,
                                       float* out_maps, const igsp_edge_opts* opts, void* stream) {
  EdgeExtent ext{};
  igsp_status st = validate_edge(images, views, n_views, out_maps, opts, &ext);
  if (st != IGSP_OK || n_views == 0) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  std::shared_ptr<EdgePlan> plan;
  st = get_edge_plan(views, n_views, opts, &plan);
  if (st != IGSP_OK) return st;
  return enqueue_edge(plan.get(), images, ext.img_end, out_maps, opts, static_cast<hipStream_t>(stream));
}

extern "C" igsp_status long_axis_split(const igsp_gaussians* g, const uint8_t* mask, const igsp_las_out* out,
                                       const igsp_las_params* params, void* stream) {
  igsp_status st = validate_las(g, mask, out, params);
  if (st != IGSP_OK) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  std::shared_ptr<LasPlan> plan;
  st = get_las_plan(g->capacity, &plan);
  if (st != IGSP_OK) return st;
  return enqueue_las(plan.get(), g, nullptr, mask, out, params, static_cast<hipStream_t>(stream));
}

extern "C" igsp_status long_axis_split_noalloc(const igsp_gaussians* g, const uint8_t* mask,
                                               const igsp_las_out* out, const igsp_las_params* params,
                                               void* stream) {
  igsp_status st = validate_las(g, mask, out, params);
  if (st != IGSP_OK) return st;
  if (g->capacity > kNoAllocCapacity) return IGSP_ERR_TOO_LARGE;
  char* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    st = scratch_of_device(&ws);
  }
  if (st != IGSP_OK) return st;
  LasLaunch L = las_launch(g, nullptr, mask, out, params);
  L.scalars = reinterpret_cast<LasScalars*>(ws + offsetof(LasScratch, scalars));
  L.block_offsets = reinterpret_cast<int64_t*>(ws + offsetof(LasScratch, offsets));
  L.block_counts = reinterpret_cast<int32_t*>(ws + offsetof(LasScratch, counts));
  return launch_las(L, static_cast<hipStream_t>(stream)) == hipSuccess ? IGSP_OK : IGSP_ERR_HIP;
}

extern "C" igsp_status long_axis_split_full(const igsp_gaussians* g, const igsp_adam_moments* adam,
                                            const uint8_t* mask, const igsp_las_out* out,
                                            const igsp_las_params* params, void* stream) {
  igsp_status st = validate_las(g, mask, out, params);
  if (st != IGSP_OK) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  std::shared_ptr<LasPlan> plan;
  st = get_las_plan(g->capacity, &plan);
  if (st != IGSP_OK) return st;
  return enqueue_las(plan.get(), g, adam, mask, out, params, static_cast<hipStream_t>(stream));
}

extern "C" igsp_status igsp_edge_resolve(const igsp_view* views, int32_t n_views, igsp_edge_opts* opts) {
  if (!opts || (n_views > 0 && !views)) return IGSP_ERR_NULL;
  if (n_views < 0) return IGSP_ERR_DIMS;
  if (opts->precision < IGSP_FP32 || opts->precision > IGSP_BF16) return IGSP_ERR_PARAM;
  if (opts->batched < IGSP_PLAIN || opts->batched > IGSP_UNFUSED) return IGSP_ERR_PARAM;
  std::lock_guard<std::mutex> lk(g_mu);
  const int form = resolve_form(views, n_views, opts);
  int seg = default_seg_rows(views, n_views, form), wgw = default_wg_waves();
  if (opts->seg_rows == 0 && opts->wg_waves == 0) {
    load_tune_cache();
    auto it = g_tuned.find(tune_key(views, n_views, opts->precision, opts->batched));
    if (it != g_tuned.end()) {
      seg = it->second.seg_rows;
      wgw = it->second.wg_waves;
    }
  }
  opts->batched = form;
  if (opts->seg_rows == 0) opts->seg_rows = seg;
  if (opts->wg_waves == 0) opts->wg_waves = wgw;
  return IGSP_OK;
}

extern "C" igsp_status igsp_edge_autotune(const uint8_t* images, const igsp_view* views, int32_t n_views,
                                          float* out_maps, int32_t precision, int32_t batched,
                                          igsp_edge_opts* best, void* stream) {
  igsp_edge_opts base{precision, batched, 0, 0, nullptr, nullptr, nullptr, nullptr};
  EdgeExtent ext{};
  igsp_status st = validate_edge(images, views, n_views, out_maps, &base, &ext);
  if (st != IGSP_OK) return st;
  if (n_views == 0) return IGSP_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // segment heights whose rows plus the 8 halo rows are a multiple of the
  // stencil loop's 6-row unroll (no row computed past a full segment's end)
  static const int kSeg[] = {10, 16, 22, 28, 40, 64, 88, 100, 124, 148, 196, 244};
  static const int kWaves[] = {1, 2, 4, 8};
  std::vector<int> forms;
  if (batched == IGSP_BATCHED) forms = {IGSP_BATCHED_STAGED, IGSP_BATCHED_PERSISTENT};
  else forms = {batched};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return IGSP_ERR_HIP;
  }
  // Mean time per launch of one candidate over `reps` launches after one
  // untimed launch (the plan is built or fetched from the cache first).
  auto time_candidate = [&](const TuneVal& c, int reps, float* out_ms) -> igsp_status {
    igsp_edge_opts o = base;
    o.batched = c.form;
    o.seg_rows = c.seg_rows;
    o.wg_waves = c.wg_waves;
    std::shared_ptr<EdgePlan> plan;
    igsp_status r;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      r = get_edge_plan(views, n_views, &o, &plan);
    }
    if (r != IGSP_OK) return r;
    r = enqueue_edge(plan.get(), images, ext.img_end, out_maps, &o, s);  // warm-up
    if (r == IGSP_OK && hipEventRecord(e0, s) != hipSuccess) r = IGSP_ERR_HIP;
    for (int k = 0; k < reps && r == IGSP_OK; ++k) r = enqueue_edge(plan.get(), images, ext.img_end, out_maps, &o, s);
    if (r == IGSP_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
      r = IGSP_ERR_HIP;
    float ms = 0.0f;
    if (r == IGSP_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) r = IGSP_ERR_HIP;
    *out_ms = ms / reps;
    return r;
  };
  std::vector<TuneVal> cands;
  for (int seg : kSeg)
    for (int wgw : kWaves)
      for (int form : forms) cands.push_back(TuneVal{seg, wgw, form, 1e30});
  // the clocks ramp up from idle over several launches: run the first
  // candidate untimed a while before any timing
  float ms = 0.0f;
  for (int k = 0; k < 4 && st == IGSP_OK; ++k) st = time_candidate(cands.front(), 4, &ms);
  // round 1: every candidate once; round 2: the three fastest again, five
  // times each in turn over twice the launches, each keeping its best (the
  // choice between close candidates then rests on more than one sample)
  for (auto& c : cands) {
    if (st != IGSP_OK) break;
    st = time_candidate(c, 8, &ms);
    c.ms = ms;
  }
  std::sort(cands.begin(), cands.end(), [](const TuneVal& x, const TuneVal& y) { return x.ms < y.ms; });
  const size_t top = std::min<size_t>(3, cands.size());
  for (int round = 0; round < 5 && st == IGSP_OK; ++round)
    for (size_t k = 0; k < top && st == IGSP_OK; ++k) {
      st = time_candidate(cands[k], 16, &ms);
      cands[k].ms = std::min<double>(cands[k].ms, ms);
    }
  TuneVal bestv{default_seg_rows(views, n_views, forms.back()), default_wg_waves(), forms.back(), 1e30};
  for (size_t k = 0; k < top; ++k)
    if (cands[k].ms < bestv.ms) bestv = cands[k];
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != IGSP_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    load_tune_cache();
    g_tuned[tune_key(views, n_views, precision, batched)] = bestv;
    save_tune_cache();
  }
  if (best) {
    *best = base;
    best->batched = bestv.form;
    best->seg_rows = bestv.seg_rows;
    best->wg_waves = bestv.wg_waves;
  }
  return IGSP_OK;
}

struct igsp_step {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::shared_ptr<EdgePlan> edge;  // the graph's kernels use these buffers
  std::shared_ptr<LasPlan> las;
};

extern "C" igsp_status igsp_step_create(const uint8_t* images, const igsp_view* views, int32_t n_views,
                                        float* out_maps, const igsp_edge_opts* opts, const igsp_gaussians* g,
                                        const uint8_t* mask, const igsp_las_out* out,
                                        const igsp_las_params* params, void* stream, igsp_step** step) {
  if (!step) return IGSP_ERR_NULL;
  *step = nullptr;
  EdgeExtent ext{};
  igsp_status st = validate_edge(images, views, n_views, out_maps, opts, &ext);
  if (st != IGSP_OK) return st;
  st = validate_las(g, mask, out, params);
  if (st != IGSP_OK) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  std::shared_ptr<EdgePlan> eplan;
  if (n_views > 0) {
    st = get_edge_plan(views, n_views, opts, &eplan);
    if (st != IGSP_OK) return st;
  }
  std::shared_ptr<LasPlan> lplan;
  st = get_las_plan(g->capacity, &lplan);
  if (st != IGSP_OK) return st;
  hipStream_t cs = static_cast<hipStream_t>(stream);
  hipStream_t own = nullptr;
  if (!cs) {  // the null stream cannot be captured
    if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess) return IGSP_ERR_HIP;
    cs = own;
  }
  igsp_edge_opts eo = opts ? *opts : igsp_edge_opts{IGSP_FP32, 1, 0, 0, nullptr, nullptr, nullptr, nullptr};
  eo.stage_events = nullptr;  // no event records inside a graph
  opts = &eo;
  auto s = std::make_unique<igsp_step>();
  igsp_status rs = IGSP_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rs = IGSP_ERR_HIP;
  } else {
    if (eplan) rs = enqueue_edge(eplan.get(), images, ext.img_end, out_maps, opts, cs);
    if (rs == IGSP_OK) rs = enqueue_las(lplan.get(), g, nullptr, mask, out, params, cs);
    hipError_t e = hipStreamEndCapture(cs, &s->graph);
    if (rs == IGSP_OK && e != hipSuccess) rs = IGSP_ERR_HIP;
    if (rs == IGSP_OK && hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0) != hipSuccess)
      rs = IGSP_ERR_HIP;
  }
  if (own) (void)hipStreamDestroy(own);
  if (rs != IGSP_OK) {
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    return rs;
  }
  s->edge = eplan;
  s->las = lplan;
  *step = s.release();
  return IGSP_OK;
}

extern "C" igsp_status igsp_step_launch(igsp_step* step, void* stream) {
  if (!step || !step->exec) return IGSP_ERR_NULL;
  return hipGraphLaunch(step->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? IGSP_OK : IGSP_ERR_HIP;
}

extern "C" void igsp_step_destroy(igsp_step* step) {
  if (!step) return;
  if (step->exec) (void)hipGraphExecDestroy(step->exec);
  if (step->graph) (void)hipGraphDestroy(step->graph);
  delete step;
}

extern "C" void igsp_release_plans(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_edge_plans.clear();
  g_las_plans.clear();
  g_sel_plans.clear();
}
