// C ABI of the local-expansion-move library: context, argument validation,
// kernel launches, one batch of disjoint local expansions, and the
// optimisation procedure (Alg. 2 with Alg. 1 per cell).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <sched.h>
#include <string>
#include <thread>
#include <vector>

#include "lexp.h"
#include "lexp_device.h"
#include "lexp_host.h"

using lexp::DevParams;
using lexp::Item;
using lexp::PairDev;
using lexp::Tile;

namespace {

thread_local std::string g_err;

lexp_status fail(lexp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(LEXP_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Device scratch of lexp_energy_noalloc (for callers that cannot allocate):
// k_energy's partial sums, two doubles per block of 256 pixels, then the two
// totals.  Every GPU the library runs on holds its own copy until the process
// ends.  In host code the array's name is not a device address: host code
// uses the address hipGetSymbolAddress gives for the current device, looked
// up once per device (at lexp_create) and kept in g_scratch_addr.
constexpr int kNoAllocBlocks = LEXP_NOALLOC_MAX_PIXELS / 256;
static __device__ __align__(256) double scratch[2 * kNoAllocBlocks + 2];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_addr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up the
// first time a context is created on that device (with the device current).
lexp_status scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(LEXP_EDEVICE, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LEXP_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_addr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_addr[dev];
  return LEXP_OK;
}

// grow-only device buffer
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t n) {
    if (n <= cap) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc((void**)&p, std::max<size_t>(n, 1) * sizeof(T));
    if (e == hipSuccess) cap = n;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

// grow-only pinned host buffer; `coherent` ones are read and written by
// kernels in place (fine-grained: the device caches none of it, so host
// stores made before a launch are what the kernel reads, and the kernel's
// stores are what the host reads after waiting for it)
template <class T>
struct PinBuf {
  T* p = nullptr;
  size_t cap = 0;
  bool coherent = false;
  hipError_t ensure(size_t n) {
    if (n <= cap) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    const unsigned flags = coherent ? (hipHostMallocMapped | hipHostMallocCoherent) : hipHostMallocDefault;
    hipError_t e = hipHostMalloc((void**)&p, std::max<size_t>(n, 1) * sizeof(T), flags);
    if (e == hipSuccess) cap = n;
    return e;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
  }
};

constexpr int kMaxTileRows = 128;  // bounds the length of the running sums


struct TileCaps {
  int wp = 1, tw = 1, ws = 1;
};

}  // namespace

struct lexp_ctx {
  lexp_params prm{};
  DevParams dp{};
  int W = 0, H = 0, r = 0;
  int tw_lim = 1;           // widest R tile column strip
  int n_cu = 256;           // compute units (the fused kernel runs one tile per CU)
  size_t lds_limit = 65536; // dynamic LDS per workgroup
  float4* left4 = nullptr;
  float4* left4T = nullptr;  // column-major copy (index u*H + v)
  float4* right4 = nullptr;
  float* guide = nullptr;
  double* wts = nullptr;
  // the context's own entry of a pair table (labels and costs of the call)
  DevBuf<PairDev> d_pair;
  PinBuf<PairDev> h_pair;
  // pair table of an optimisation run (one entry per pair of the run)
  DevBuf<PairDev> d_run_pairs;
  PinBuf<PairDev> h_run_pairs;
  DevBuf<Item> d_items;
  DevBuf<Tile> d_tiles;
  DevBuf<float> d_phi;
  DevBuf<int> d_terms;
  DevBuf<uint8_t> d_x;
  DevBuf<int> d_flag;
  DevBuf<double> d_partial;
  DevBuf<float4> d_labels_tmp;
  DevBuf<int> d_status;
  PinBuf<int> h_status;
  DevBuf<unsigned char> d_post;  // post-processing scratch (disparity, fill, flags, row links)
  PinBuf<Item> h_items;
  PinBuf<Tile> h_tiles;
  PinBuf<int> h_terms;
  PinBuf<uint8_t> h_x;
  PinBuf<int> h_flag;
  PinBuf<double> h_partial;
  PinBuf<float> h_labels4;
  hipEvent_t staging_done = nullptr;  // host staging buffers may be rewritten once this has completed
  int n_threads = 1;  // host threads of the min-cut pool (started on first use)
  std::unique_ptr<lexp::ThreadPool> pool;
  std::vector<std::unique_ptr<lexp::BKSolver>> solvers;
  bool timing = false;
  int time_every = 1;    // time every time_every-th fused launch
  int64_t time_seq = 0;  // fused launches since timing was turned on
  lexp_stats stats{};
  std::vector<hipEvent_t> ev_free;
  int time_level = -1;  // grid level the timed launches are counted under (lexp_optimize), -1: none
  struct Pending { hipEvent_t a, b; double bytes; int level; };
  std::vector<Pending> ev_pending;
  // two halves of a group step in flight at once (host cuts one half while
  // the device evaluates the other)
  // Buffers of one part of a group in flight in lexp_optimize.  terms[0] is
  // the overflow flag of the graph terms (cleared once per run, never reset by
  // a step), the terms of the part follow from terms[1].  On the host path
  // k_graph_terms writes the flag and the terms straight into h_terms, and
  // k_apply reads the host's cut from h_x; with the device cut the terms stay
  // in d_terms and the device writes the flag, a status per region and the
  // cut (x, one byte per pixel) straight into h_res, which k_apply reads.
  // Those three host buffers are coherent pinned memory (no copies).
  struct PartBuf {
    DevBuf<Item> d_items;
    DevBuf<float> d_phi;
    DevBuf<int> d_terms;
    PinBuf<Item> h_items;
    PinBuf<int> h_terms;
    PinBuf<uint8_t> h_x;
    PinBuf<unsigned char> h_res;
    hipEvent_t ready = nullptr;
    // host path: the terms of the first `split` regions (the larger ones) come
    // from a launch of their own, followed by `half`, so the host pool starts
    // on them while the rest are written (0: one launch)
    hipEvent_t half = nullptr;
    int split = 0;
    hipEvent_t cut0 = nullptr, cut1 = nullptr;  // around a timed device max-flow launch
    bool cut_timed = false;
    int cut_block = 0, cut_every = 0;  // shape of that launch
    // speculative costs of the next step (lexp_optimize, single-part
    // groups), double-buffered by step parity
    DevBuf<Item> d_sitems[2];
    DevBuf<Tile> d_stiles[2];
    DevBuf<float> d_sphi[2];
    PinBuf<Item> h_sitems[2];
    PinBuf<Tile> h_stiles[2];
  } part[2];
  size_t res_items = 0;  // status slots in the result buffers
  // batch cycle: one launch per group step for every region and candidate
  DevBuf<Item> d_bitems;
  DevBuf<Tile> d_btiles;
  DevBuf<float> d_bphi;
  PinBuf<Item> h_bitems;
  PinBuf<Tile> h_btiles;
  lexp_net* net = nullptr;  // learned proposals for lexp_optimize (not owned)
  hipStream_t capture_stream = nullptr;  // graph mode: work is captured here, replayed on the caller's stream
  double* noalloc_scratch = nullptr;     // this context's device's copy of `scratch`
};

// The learned proposal network (five 3x3 convolutions, channels 16 -> 32 ->
// 32 -> 32 -> 32 -> 16): FP32 master parameters with Adam moments, BF16
// weight copies, and activation buffers for images up to max_w x max_h.
struct lexp_net {
  static constexpr int kLayers = 5;
  static constexpr int kCh[kLayers + 1] = {16, 32, 32, 32, 32, 16};
  // weight-gradient partial sums (one per chunk of kWgRows rows x kWgTiles
  // tiles of 32 columns) of an image
  static int grad_chunks(int W, int H) {
    return ((H + lexp::kWgRows - 1) / lexp::kWgRows) * (((W + 31) / 32 + lexp::kWgTiles - 1) / lexp::kWgTiles);
  }
  int max_w = 0, max_h = 0;
  size_t w_off[kLayers] = {}, b_off[kLayers] = {}, n_prm = 0;  // parameter layout: per layer [w][b]
  size_t w16_off[kLayers] = {}, n_w16 = 0;
  float* prm = nullptr;     // FP32 master parameters
  float* grad = nullptr;
  float* mom1 = nullptr;
  float* mom2 = nullptr;
  uint16_t* w16 = nullptr;  // BF16 weights [tap][out][in]
  uint16_t* wt16 = nullptr; // BF16 weights [tap][in][out]
  uint16_t* act[kLayers] = {};  // layer inputs x0..x4
  uint16_t* gbuf[2] = {};       // gradients of the layer outputs (ping-pong)
  float* y = nullptr;           // last layer output, 16 FP32 per pixel
  float4* planes = nullptr;     // candidate planes per pixel
  float* part_w = nullptr;
  float* part_b = nullptr;
  double* part_loss = nullptr;
  PinBuf<double> h_loss;
  int steps = 0;  // Adam steps taken
};

namespace {

PairDev pair_entry(const lexp_ctx* c, float* labels, float* cur_cost) {
  PairDev e{};
  e.P = c->dp;
  e.left4 = c->left4;
  e.left4T = c->left4T;
  e.right4 = c->right4;
  e.guide = c->guide;
  e.wts = c->wts;
  e.labels = reinterpret_cast<float4*>(labels);
  e.cur_cost = cur_cost;
  return e;
}

bool finite_plane(const lexp_plane& p) { return std::isfinite(p.a) && std::isfinite(p.b) && std::isfinite(p.c); }

void clip_rect(const lexp_ctx* c, const lexp_rect& r, int* u0, int* v0, int* u1, int* v1) {
  *u0 = std::max(r.u0, 0);
  *v0 = std::max(r.v0, 0);
  *u1 = std::min(r.u1, c->W);
  *v1 = std::min(r.v1, c->H);
  if (*u1 < *u0) *u1 = *u0;
  if (*v1 < *v0) *v1 = *v0;
}

int64_t clipped_area(const lexp_ctx* c, int u0, int v0, int u1, int v1, int m) {
  const int a0 = std::max(u0 - m, 0), b0 = std::max(v0 - m, 0);
  const int a1 = std::min(u1 + m, c->W), b1 = std::min(v1 + m, c->H);
  return (int64_t)std::max(a1 - a0, 0) * std::max(b1 - b0, 0);
}

// Algorithmic bytes of one item: right-image band and left tile over M (16 B
// each per pixel), guide statistics over R+ (36 B), phi over R (4 B).
double item_alg_bytes(const lexp_ctx* c, const Item& it) {
  const int u1 = it.ru0 + it.rw, v1 = it.rv0 + it.rh;
  const double m = (double)clipped_area(c, it.ru0, it.rv0, u1, v1, 2 * c->r);
  const double p = (double)clipped_area(c, it.ru0, it.rv0, u1, v1, c->r);
  return 32.0 * m + 36.0 * p + 4.0 * (double)it.rw * it.rh;
}

int max_tile_width(int r, size_t budget) {
  const int ring = lexp::unary_ring_rows(r);
  int tw = std::min({lexp::kMaxTW, lexp::kMaxWP - 2 * r, lexp::kMaxWM - 4 * r});
  for (; tw >= 1; --tw)
    if (lexp::unary_lds_bytes(ring, tw + 2 * r, tw, std::max(tw + 4 * r, tw + 2 * r)) <= budget) return tw;
  return 0;
}

// Splits items into column strips (width bounded by LDS and the kernel's
// register layout) and row strips.  When a launch has fewer column strips
// than CUs, taller items are also cut into row strips (of at least
// kMinStripRows rows) so the launch fills the device; every strip recomputes
// its own vertical margin.
constexpr int kFillTiles = 256;

// A tile plan: the widest column strip (at most the kernel's LDS limit
// tw_lim) and the tiles a launch is filled to with row strips.
struct TilePlan {
  int cols = 0;  // 0: tw_lim
  int fill = kFillTiles;
};

// Column strips of a region rw wide: the fewest strips of width <= the
// plan's widest (and tw_lim), or up to two more when narrower strips need
// fewer 32-column segments per M row (the raw-cost stage's work per row grows
// with those segments).
int column_strips(const lexp_ctx* c, int rw, const TilePlan& plan) {
  const int lim = plan.cols > 0 ? std::min(plan.cols, c->tw_lim) : c->tw_lim;
  const int n0 = (rw + lim - 1) / lim;
  auto segs = [&](int n) { return ((rw + n - 1) / n + 4 * c->r + 31) / 32; };
  int best = n0;
  for (int n = n0 + 1; n <= n0 + 2 && n <= rw; ++n)
    if (segs(n) < segs(best)) best = n;
  return best;
}
constexpr int kMinStripRows = 16;

void plan_tiles(const lexp_ctx* c, const Item* items, int n, std::vector<Tile>& tiles, TileCaps& caps,
                const TilePlan& plan = TilePlan{}) {
  tiles.clear();
  caps = TileCaps{};
  int64_t col_tiles = 0;
  for (int i = 0; i < n; ++i)
    if (items[i].rw > 0 && items[i].rh > 0) col_tiles += column_strips(c, items[i].rw, plan);
  const int fill = col_tiles > 0 ? (int)std::max<int64_t>(1, plan.fill / col_tiles) : 1;
  for (int i = 0; i < n; ++i) {
    const Item& it = items[i];
    if (it.rw <= 0 || it.rh <= 0) continue;
    const int ncs = column_strips(c, it.rw, plan);
    const int nrs = std::max((it.rh + kMaxTileRows - 1) / kMaxTileRows,
                             std::min((it.rh + kMinStripRows - 1) / kMinStripRows, fill));
    for (int rs = 0; rs < nrs; ++rs) {
      const int tv0 = it.rv0 + (int)((int64_t)it.rh * rs / nrs);
      const int tv1 = it.rv0 + (int)((int64_t)it.rh * (rs + 1) / nrs);
      for (int cs = 0; cs < ncs; ++cs) {
        const int tu0 = it.ru0 + (int)((int64_t)it.rw * cs / ncs);
        const int tu1 = it.ru0 + (int)((int64_t)it.rw * (cs + 1) / ncs);
        Tile t{};
        t.item = i;
        t.tu0 = tu0; t.tv0 = tv0; t.tu1 = tu1; t.tv1 = tv1;
        t.flags = (cs == 0 ? lexp::kFirstCol : 0) | (cs == ncs - 1 ? lexp::kLastCol : 0) |
                  (rs == 0 ? lexp::kFirstRow : 0) | (rs == nrs - 1 ? lexp::kLastRow : 0);
        tiles.push_back(t);
        const int wp = std::min(tu1 + c->r, c->W) - std::max(tu0 - c->r, 0);
        const int wm = std::min(tu1 + 2 * c->r, c->W) - std::max(tu0 - 2 * c->r, 0);
        caps.wp = std::max(caps.wp, wp);
        caps.tw = std::max(caps.tw, tu1 - tu0);
        caps.ws = std::max(caps.ws, std::max(wm, wp));
      }
    }
  }
}

hipEvent_t take_event(lexp_ctx* c) {
  if (!c->ev_free.empty()) {
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Folds completed kernel timings into the counters (synchronises the events).
void collect_timing(lexp_ctx* c) {
  for (auto& p : c->ev_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->stats.unary_kernel_ms += ms;
      if (p.level >= 0 && p.level < 4) {
        c->stats.unary_level_ms[p.level] += ms;
        c->stats.unary_level_alg_bytes[p.level] += p.bytes;
        c->stats.unary_level_launches[p.level] += 1;
      }
    }
    c->ev_free.push_back(p.a);
    c->ev_free.push_back(p.b);
  }
  c->ev_pending.clear();
}

// 1 when tile i is the only tile of item i for every item (the fused kernel
// then loads a tile's item without waiting for the tile).
int tiles_direct(const Tile* tiles, size_t n_tiles, size_t n_items) {
  if (n_tiles != n_items) return 0;
  for (size_t i = 0; i < n_tiles; ++i)
    if (tiles[i].item != (int)i) return 0;
  return 1;
}

// Fused cost kernel over n_tiles tiles of the items (pairs: the table the
// items' pair indices refer to; MODE 2 covers every pixel of pairs[0]).
template <int MODE>
lexp_status launch_unary(lexp_ctx* c, const PairDev* d_pairs, const Item* d_items, const Tile* d_tiles, int n_tiles,
                         const TileCaps& caps,
                         const float4* label_field, float* out, hipStream_t s, double alg_bytes, int64_t evals,
                         int64_t n_items, int pair_hint = -1, int direct = 0, bool count_evals = true) {
  if (n_tiles <= 0) return LEXP_OK;
  const int ring = lexp::unary_ring_rows(c->r);
  const size_t lds = lexp::unary_lds_bytes(ring, caps.wp, caps.tw, caps.ws);
  if (lds > c->lds_limit || caps.wp > lexp::kMaxWP || caps.tw > lexp::kMaxTW || caps.ws > lexp::kMaxWM)
    return fail(LEXP_EINVAL, "tile exceeds kernel limits (lds %zu > %zu or width)", lds, c->lds_limit);
  const int grid = ((n_tiles + 7) / 8) * 8;
  // Region costs with r >= 20: waves 8-15 also run stage A in a tile's first
  // step (32 rows instead of 16).  The choice changes the tile's row schedule
  // and so the rounding of its vertical sums; it depends on r alone, never on
  // the launch.  Their scan rows (16 rows of M, float4 and FP32 count) go to
  // the ring-1 slots past the first 32 rows: 320 ws <= 16 (2r+1) wp, which
  // holds for every tile once r >= 20 (the M width exceeds the R+ width by at
  // most r on each side where R+ itself extends r past the tile).
  const int fill2 = MODE == 0 && c->r >= 20 ? 1 : 0;
  if (fill2 && (size_t)lexp::kChunk * caps.ws * 20 > (size_t)(ring - 2 * lexp::kChunk) * caps.wp * 16)
    return fail(LEXP_EINVAL, "internal: first-step scan rows exceed the ring (ws %d, wp %d)", caps.ws, caps.wp);
  // timing covers the region-cost launches (MODE 0), the hot loop of the method
  // (timed launches go through hipExtLaunchKernel, whose two events take the
  // kernel's own start and end on the stream)
  const bool timed = c->timing && MODE == 0;
  hipEvent_t ea = nullptr, eb = nullptr;
  if (timed && c->time_seq++ % c->time_every == 0) {
    ea = take_event(c);
    eb = take_event(c);
    if (!(ea && eb)) {  // (no events to be had: this launch goes untimed)
      if (ea) c->ev_free.push_back(ea);
      if (eb) c->ev_free.push_back(eb);
      ea = eb = nullptr;
    }
  }
  const bool tev = ea && eb;
  // instance by the 32-column segments of an M row (64-lane segments of a row
  // pair) and of an R+ row
  const int nseg = (caps.ws + 31) / 32, nc = (std::max(caps.wp, caps.tw) + 31) / 32;
#define LEXP_LAUNCH(M, S, C)                                                                                      \
  do {                                                                                                            \
    if (tev)                                                                                                      \
      hipExtLaunchKernelGGL((lexp::k_unary<M, S, C>), dim3(grid), dim3(lexp::kWaves * 64), (uint32_t)lds, s, ea, eb, \
                            0u, d_pairs, d_items, d_tiles, n_tiles, label_field, out, ring, caps.wp, caps.tw,     \
                            caps.ws, pair_hint, direct, fill2);                                                   \
    else                                                                                                          \
      hipLaunchKernelGGL((lexp::k_unary<M, S, C>), dim3(grid), dim3(lexp::kWaves * 64), lds, s, d_pairs, d_items,  \
                         d_tiles, n_tiles, label_field, out, ring, caps.wp, caps.tw, caps.ws, pair_hint, direct,  \
                         fill2);                                                                                  \
  } while (0)
#define LEXP_LAUNCH_C(M, S)  \
  if (nc <= 1) {             \
    LEXP_LAUNCH(M, S, 1);    \
  } else if (nc <= 2) {      \
    LEXP_LAUNCH(M, S, 2);    \
  } else if (nc <= 3) {      \
    LEXP_LAUNCH(M, S, 3);    \
  } else {                   \
    LEXP_LAUNCH(M, S, 4);    \
  }
  if constexpr (MODE == 1) {
    LEXP_LAUNCH(1, 4, 4);
  } else if (nseg <= 1) {
    LEXP_LAUNCH(MODE, 1, 1);
  } else if (nseg <= 2) {
    if (nc <= 1) {
      LEXP_LAUNCH(MODE, 2, 1);
    } else {
      LEXP_LAUNCH(MODE, 2, 2);
    }
  } else if (nseg <= 3) {
    if (nc <= 1) {
      LEXP_LAUNCH(MODE, 3, 1);
    } else if (nc <= 2) {
      LEXP_LAUNCH(MODE, 3, 2);
    } else {
      LEXP_LAUNCH(MODE, 3, 3);
    }
  } else {
    LEXP_LAUNCH_C(MODE, 4)
  }
#undef LEXP_LAUNCH_C
#undef LEXP_LAUNCH
  HIP_TRY(hipGetLastError());
  if (timed) {
    c->stats.unary_launches += 1;
    c->stats.unary_alg_bytes += alg_bytes;
    if (count_evals) c->stats.unary_evals += evals;
    c->stats.unary_items += n_items;
  }
  if (tev) {
    c->ev_pending.push_back({ea, eb, alg_bytes, c->time_level});
    c->stats.unary_timed_launches += 1;
    c->stats.unary_timed_alg_bytes += alg_bytes;
    c->stats.unary_timed_evals += evals;
  }
  return LEXP_OK;
}

// Rounds the device max-flow may take per region node before it leaves the
// region to the host (the kernel adds 256); converged regions need far fewer.
constexpr int kCutRoundFactor = 4;

// Push-relabel rounds between global relabels: a global relabel costs about
// one workgroup barrier per breadth-first level (up to the region's diameter),
// a round two.
int cut_relabel_every(int max_px) {
  return max_px <= 512 ? 8 : 16;
}

// Whether the device max-flow holds a region of px nodes (its arrays live in
// LDS, in the compact layout when the full one does not fit).
bool cut_fits(const lexp_ctx* c, int64_t px) {
  return px * lexp::kCutBytesCompact <= (int64_t)c->lds_limit - 64;
}

// Launch shape of the device max-flow: threads per region and push-relabel
// rounds between global relabels.  Every shape returns the same exact cut.
struct CutShape {
  int block = 0;  // 0: the default rule
  int every = 0;
};

bool cut_full_fits(const lexp_ctx* c, int64_t px) {
  return px * lexp::kCutBytesFull + 64 <= (int64_t)c->lds_limit;
}

// Shapes worth trying for a launch whose largest region has max_px nodes.
std::vector<CutShape> cut_shapes(const lexp_ctx* c, int max_px) {
  std::vector<CutShape> v;
  if (max_px <= 512) {
    for (int b : {128, 256, 512})
      for (int e : {4, 8, 16}) v.push_back({b, e});
  } else if (cut_full_fits(c, max_px)) {
    for (int b : {512, 1024})
      for (int e : {8, 16, 32}) v.push_back({b, e});
  } else {
    for (int e : {8, 16, 32}) v.push_back({1024, e});
  }
  return v;
}

// Device minimum cuts of n regions whose terms start at the items' aux_off;
// x at the same offsets, one status per item.  Every region must fit.
lexp_status launch_cut(lexp_ctx* c, const Item* d_items, int n, const int* d_terms, uint8_t* d_x, int* d_status,
                       int max_px, hipStream_t s, CutShape shape = CutShape{}) {
  if (n <= 0) return LEXP_OK;
  if (!cut_fits(c, max_px)) return fail(LEXP_ESTATE, "region of %d pixels too large for the device max-flow", max_px);
  const int nf = c->dp.nf;
  const bool full = cut_full_fits(c, max_px);
  if (shape.block == 0) shape = CutShape{max_px <= 512 ? 256 : 1024, cut_relabel_every(max_px)};
  const int every = shape.every;
  const size_t lds = (size_t)max_px * (full ? lexp::kCutBytesFull : lexp::kCutBytesCompact);
#define LEXP_CUT(L, B)                                                                                        \
  hipLaunchKernelGGL((lexp::k_cut_lds<lexp::L, B>), dim3(n), dim3(B), lds, s, d_items, d_terms, nf, d_x, d_status, \
                     max_px, kCutRoundFactor, every)
  if (!full) {
    if (shape.block != 1024) return fail(LEXP_ESTATE, "compact device max-flow runs 1024 threads per region");
    LEXP_CUT(CompactLayout, 1024);
  } else if (shape.block == 128) {
    LEXP_CUT(FullLayout, 128);
  } else if (shape.block == 256) {
    LEXP_CUT(FullLayout, 256);
  } else if (shape.block == 512) {
    LEXP_CUT(FullLayout, 512);
  } else if (shape.block == 1024) {
    LEXP_CUT(FullLayout, 1024);
  } else {
    return fail(LEXP_ESTATE, "device max-flow block %d not built", shape.block);
  }
#undef LEXP_CUT
  HIP_TRY(hipGetLastError());
  return LEXP_OK;
}

lexp_status wait_staging(lexp_ctx* c) {
  HIP_TRY(hipEventSynchronize(c->staging_done));
  return LEXP_OK;
}

// Writes the context's pair entry with the call's label field and costs
// (after wait_staging: the pinned entry is staging memory).
lexp_status stage_pair(lexp_ctx* c, float* labels, float* cur_cost, hipStream_t s) {
  c->h_pair.p[0] = pair_entry(c, labels, cur_cost);
  HIP_TRY(hipMemcpyAsync(c->d_pair.p, c->h_pair.p, sizeof(PairDev), hipMemcpyHostToDevice, s));
  return LEXP_OK;
}

// Builds the item table for (rects, labels) on the host staging buffer.
lexp_status stage_items(lexp_ctx* c, int n, const lexp_rect* rects, const lexp_plane* labels, const int64_t* offsets,
                        const int64_t* aux) {
  HIP_TRY(c->h_items.ensure((size_t)n));
  for (int i = 0; i < n; ++i) {
    int u0, v0, u1, v1;
    clip_rect(c, rects[i], &u0, &v0, &u1, &v1);
    Item& it = c->h_items.p[i];
    it.ru0 = u0; it.rv0 = v0; it.rw = u1 - u0; it.rh = v1 - v0;
    it.a = labels[i].a; it.b = labels[i].b; it.c = labels[i].c; it.pair = 0;
    it.out_off = offsets ? offsets[i] : 0;
    it.aux_off = aux ? aux[i] : 0;
  }
  return LEXP_OK;
}

lexp_status validate_items(lexp_ctx* c, int32_t n, const lexp_rect* rects, const lexp_plane* labels,
                           const int64_t* offsets) {
  if (!c) return fail(LEXP_EINVAL, "null context");
  if (n < 0) return fail(LEXP_EINVAL, "negative item count");
  if (n > 0 && (!rects || !labels || !offsets)) return fail(LEXP_EINVAL, "null item array");
  for (int i = 0; i < n; ++i) {
    if (!finite_plane(labels[i])) return fail(LEXP_EINVAL, "label %d is not finite", i);
    if (offsets[i] < 0) return fail(LEXP_EINVAL, "negative offset %d", i);
  }
  return LEXP_OK;
}

// Rejects regions that overlap or touch (8-neighbour contact).
lexp_status check_separated(lexp_ctx* c, int n, const Item* items) {
  std::vector<int32_t> owner((size_t)c->W * c->H, -1);
  for (int i = 0; i < n; ++i) {
    const Item& it = items[i];
    if (it.rw <= 0 || it.rh <= 0) continue;
    const int a0 = std::max(it.ru0 - 1, 0), a1 = std::min(it.ru0 + it.rw + 1, c->W);
    const int b0 = std::max(it.rv0 - 1, 0), b1 = std::min(it.rv0 + it.rh + 1, c->H);
    for (int v = it.rv0; v < it.rv0 + it.rh; ++v)
      for (int u = it.ru0; u < it.ru0 + it.rw; ++u) {
        int32_t& o = owner[(size_t)v * c->W + u];
        if (o >= 0) return fail(LEXP_EINVAL, "regions %d and %d overlap", o, i);
        o = i;
      }
    for (int v = b0; v < b1; ++v)
      for (int u = a0; u < a1; ++u) {
        const int32_t o = owner[(size_t)v * c->W + u];
        if (o >= 0 && o != i) return fail(LEXP_EINVAL, "regions %d and %d touch", o, i);
      }
  }
  return LEXP_OK;
}

// Binary energy of a cut in quantum units.
int64_t cut_energy(int w, int h, int nf, const int* terms, const uint8_t* x) {
  static const int DU[4] = {1, 0, 1, -1}, DV[4] = {0, 1, 1, 1};
  int64_t e = 0;
  for (int i = 0; i < w * h; ++i) {
    if (x[i]) e += terms[(size_t)i * 5];
    else {
      const int u = i % w, v = i / w;
      for (int d = 0; d < nf; ++d) {
        const int nu = u + DU[d], nv = v + DV[d];
        if (nu < 0 || nu >= w || nv < 0 || nv >= h) continue;
        if (x[nv * w + nu]) e += terms[(size_t)i * 5 + 1 + d];
      }
    }
  }
  return e;
}

lexp::ThreadPool& pool_of(lexp_ctx* c);

// Graph terms on the device, host max-flow per item, label update on the
// device.  Items are staged in c->h_items (aux_off = compact pixel offset,
// total pixels n_px).  mirror (optional): host HxWx3 labels to update.
lexp_status expand_batch(lexp_ctx* c, int n, int64_t n_px, const float* alpha_cost, float* labels, float* cur_cost,
                         int64_t* delta_Eq, int32_t* n_changed, float* mirror, int64_t* total_dE, hipStream_t s,
                         bool items_on_device) {
  if (n <= 0) return LEXP_OK;
  if (!items_on_device) {
    HIP_TRY(c->d_items.ensure((size_t)n));
    HIP_TRY(hipMemcpyAsync(c->d_items.p, c->h_items.p, sizeof(Item) * n, hipMemcpyHostToDevice, s));
  }
  HIP_TRY(c->d_terms.ensure((size_t)n_px * 5));
  HIP_TRY(c->d_x.ensure((size_t)n_px));
  HIP_TRY(c->h_terms.ensure((size_t)n_px * 5));
  HIP_TRY(c->h_x.ensure((size_t)n_px));
  HIP_TRY(c->d_flag.ensure(1));
  HIP_TRY(c->h_flag.ensure(1));
  int max_px = 1;
  for (int i = 0; i < n; ++i) max_px = std::max(max_px, c->h_items.p[i].rw * c->h_items.p[i].rh);
  HIP_TRY(hipMemsetAsync(c->d_flag.p, 0, sizeof(int), s));
  lexp_status st = stage_pair(c, labels, cur_cost, s);
  if (st) return st;
  hipLaunchKernelGGL(lexp::k_graph_terms, dim3((max_px + 255) / 256, n), dim3(256), 0, s, c->d_pair.p,
                     c->d_items.p, alpha_cost, c->d_terms.p, c->d_flag.p);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(c->h_terms.p, c->d_terms.p, sizeof(int) * 5 * n_px, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(c->h_flag.p, c->d_flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  const auto t0 = std::chrono::steady_clock::now();
  HIP_TRY(hipStreamSynchronize(s));
  const auto t1 = std::chrono::steady_clock::now();
  if (c->h_flag.p[0]) return fail(LEXP_EINVAL, "binary-problem term exceeds 2^30 quanta (parameters too large)");
  const int nf = c->dp.nf;
  std::vector<int64_t> de(n, 0);
  std::vector<int32_t> nc(n, 0);
  const Item* items = c->h_items.p;
  pool_of(c).parallel_for(n, [&](int i, int worker) {
    const Item& it = items[i];
    if (it.rw <= 0 || it.rh <= 0) return;
    const int* t = c->h_terms.p + (size_t)it.aux_off * 5;
    uint8_t* x = c->h_x.p + it.aux_off;
    lexp::BKSolver& bk = *c->solvers[worker];
    bk.load<int32_t>(it.rw, it.rh, nf, t, 5, t + 1, 5);
    bk.solve(x);
    de[i] = cut_energy(it.rw, it.rh, nf, t, x);
    int32_t cnt = 0;
    for (int q = 0; q < it.rw * it.rh; ++q) {
      if (!x[q]) continue;
      ++cnt;
      if (mirror) {
        float* m = mirror + ((size_t)(it.rv0 + q / it.rw) * c->W + (it.ru0 + q % it.rw)) * 3;
        m[0] = it.a; m[1] = it.b; m[2] = it.c;
      }
    }
    nc[i] = cnt;
  });
  const auto t2 = std::chrono::steady_clock::now();
  HIP_TRY(hipMemcpyAsync(c->d_x.p, c->h_x.p, (size_t)n_px, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(lexp::k_apply, dim3((max_px + 255) / 256, n), dim3(256), 0, s, c->d_pair.p, c->d_items.p,
                     c->d_x.p, alpha_cost);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(c->staging_done, s));
  int64_t sum = 0;
  for (int i = 0; i < n; ++i) {
    if (delta_Eq) delta_Eq[i] = de[i];
    if (n_changed) n_changed[i] = nc[i];
    sum += de[i];
  }
  if (total_dE) *total_dE += sum;
  c->stats.expand_calls += 1;
  c->stats.host_wait_ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
  c->stats.host_cut_ms += std::chrono::duration<double, std::milli>(t2 - t1).count();
  return LEXP_OK;
}

// Host threads for the min-cut pool: OMP_NUM_THREADS when set (the share of
// cores the job was given), else the CPUs this process may run on.
int default_threads() {
  if (const char* e = std::getenv("OMP_NUM_THREADS")) {
    const int v = std::atoi(e);
    if (v > 0) return v;
  }
  cpu_set_t set;
  if (sched_getaffinity(0, sizeof(set), &set) == 0) return std::max(1, CPU_COUNT(&set));
  return (int)std::max(1u, std::thread::hardware_concurrency());
}

// The context's min-cut pool and one max-flow solver per thread, started on
// first use (a context used only for costs, or as a non-first pair of a batched
// run, starts no threads).
lexp::ThreadPool& pool_of(lexp_ctx* c) {
  if (!c->pool) {
    c->pool.reset(new lexp::ThreadPool(c->n_threads));
    for (int i = 0; i < c->pool->size(); ++i) c->solvers.emplace_back(new lexp::BKSolver());
  }
  return *c->pool;
}

lexp_status energy_impl(lexp_ctx* c, const float* labels, const float* cur_cost, double* total, double* unary,
                        double* pair, hipStream_t s) {
  const int n = c->W * c->H;
  const int nb = (n + 255) / 256;
  HIP_TRY(c->d_partial.ensure((size_t)nb * 2));
  HIP_TRY(c->h_partial.ensure((size_t)nb * 2));
  hipLaunchKernelGGL(lexp::k_energy, dim3(nb), dim3(256), 0, s, c->dp, (const float4*)labels, cur_cost, c->wts,
                     c->d_partial.p);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(c->h_partial.p, c->d_partial.p, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double eu = 0.0, ep = 0.0;
  for (int b = 0; b < nb; ++b) {
    eu += c->h_partial.p[2 * b];
    ep += c->h_partial.p[2 * b + 1];
  }
  if (total) *total = eu + ep;
  if (unary) *unary = eu;
  if (pair) *pair = ep;
  return LEXP_OK;
}

lexp_status pixel_costs_impl(lexp_ctx* c, const float* labels, float* out, hipStream_t s) {
  TileCaps caps;
  caps.tw = 1;
  caps.wp = std::min(2 * c->r + 1, c->W);
  caps.ws = std::max(std::min(4 * c->r + 1, c->W), caps.wp);
  return launch_unary<2>(c, c->d_pair.p, nullptr, nullptr, c->W * c->H, caps, (const float4*)labels, out, s, 0.0,
                         (int64_t)c->W * c->H, (int64_t)c->W * c->H);
}

// Host labels (HxWx3) -> device field (HxWx4).
lexp_status upload_labels(lexp_ctx* c, const float* hw3, float* dev4, hipStream_t s) {
  const size_t n = (size_t)c->W * c->H;
  HIP_TRY(c->h_labels4.ensure(n * 4));
  for (size_t i = 0; i < n; ++i) {
    c->h_labels4.p[4 * i + 0] = hw3[3 * i + 0];
    c->h_labels4.p[4 * i + 1] = hw3[3 * i + 1];
    c->h_labels4.p[4 * i + 2] = hw3[3 * i + 2];
    c->h_labels4.p[4 * i + 3] = 0.f;
  }
  HIP_TRY(hipMemcpyAsync(dev4, c->h_labels4.p, sizeof(float) * 4 * n, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return LEXP_OK;
}

}  // namespace

// ===========================================================================
// ABI
// ===========================================================================
extern "C" {

const char* lexp_last_error(void) { return g_err.c_str(); }

lexp_status lexp_create(const lexp_params* params, const float* left_hwc, const float* right_hwc, void* hip_stream,
                        lexp_ctx** out) {
  if (!params || !left_hwc || !right_hwc || !out) return fail(LEXP_EINVAL, "null argument");
  const lexp_params& p = *params;
  // the fused kernel addresses the packed images with 32-bit byte offsets
  if (p.width <= 0 || p.height <= 0 || (int64_t)p.width * p.height >= (1ll << 27))
    return fail(LEXP_EINVAL, "bad image size %dx%d (at most 2^27 - 1 pixels)", p.width, p.height);
  if (p.gf_radius < 1 || p.gf_radius > 32) return fail(LEXP_EINVAL, "gf_radius %d outside [1, 32]", p.gf_radius);
  if (p.neighbours != 4 && p.neighbours != 8) return fail(LEXP_EINVAL, "neighbours must be 4 or 8");
  if (!(p.gf_eps > 0.0) || !(p.gamma > 0.0) || !(p.lambda >= 0.0) || !(p.tau_dis >= 0.0) || !(p.w_floor >= 0.0) ||
      !(p.tau_col >= 0.0) || !(p.tau_grad >= 0.0) || !(p.alpha >= 0.0 && p.alpha <= 1.0) ||
      !std::isfinite(p.disp_max))
    return fail(LEXP_EINVAL, "parameter out of range");
  if (p.lambda * p.tau_dis > 64.0 || p.tau_col > 1e4 || p.tau_grad > 1e4)
    return fail(LEXP_EINVAL, "lambda*tau_dis or truncations too large for 32-bit binary terms");
  if (p.host_threads < 0 || p.host_threads > 64) return fail(LEXP_EINVAL, "host_threads outside [0, 64]");
  if (p.device_cut != 0 && p.device_cut != 1) return fail(LEXP_EINVAL, "device_cut must be 0 or 1");
  if (p.view != 0 && p.view != 1) return fail(LEXP_EINVAL, "view must be 0 (left) or 1 (right)");
  if (p.graph != 0 && p.graph != 1) return fail(LEXP_EINVAL, "graph must be 0 or 1");
  hipStream_t s = (hipStream_t)hip_stream;
  std::unique_ptr<lexp_ctx> c(new lexp_ctx());
  c->prm = p;
  c->W = p.width;
  c->H = p.height;
  c->r = p.gf_radius;
  DevParams& d = c->dp;
  d.W = c->W; d.H = c->H; d.r = c->r; d.nf = p.neighbours == 8 ? 4 : 2;
  d.oma = (float)(1.0 - p.alpha);
  d.al = (float)p.alpha;
  d.tc = (float)p.tau_col;
  d.tg = (float)p.tau_grad;
  d.rho_max = (float)((1.0 - p.alpha) * p.tau_col + p.alpha * p.tau_grad);
  d.lam = p.lambda; d.tau_dis = p.tau_dis; d.w_floor = p.w_floor;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  {
    const lexp_status st = scratch_address(dev, &c->noalloc_scratch);
    if (st != LEXP_OK) return st;
  }
  int lds = 0;
  HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  c->lds_limit = (size_t)std::max(lds, 16384);
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  c->n_cu = std::max(cus, 1);
  // one 16-wave workgroup per CU: a tile may use all of the CU's LDS
  c->tw_lim = max_tile_width(c->r, c->lds_limit);
  if (c->tw_lim < 1)
    return fail(LEXP_EINVAL, "gf_radius %d exceeds the fused kernel's limits (LDS or row width)", c->r);
  const size_t n = (size_t)c->W * c->H;
  HIP_TRY(hipMalloc((void**)&c->left4, n * sizeof(float4)));
  HIP_TRY(hipMalloc((void**)&c->left4T, n * sizeof(float4)));
  // one zeroed pixel after the right image: the fused kernel's second
  // interpolation tap may read it (with weight zero)
  HIP_TRY(hipMalloc((void**)&c->right4, (n + 1) * sizeof(float4)));
  HIP_TRY(hipMemsetAsync(c->right4 + n, 0, sizeof(float4), s));
  HIP_TRY(hipMalloc((void**)&c->guide, n * 9 * sizeof(float)));
  HIP_TRY(hipMalloc((void**)&c->wts, n * 4 * sizeof(double)));
  double* tmp = nullptr;
  HIP_TRY(hipMalloc((void**)&tmp, n * 9 * sizeof(double)));
  const int nb = (int)((n + 255) / 256);
  // the right view is the left-view problem of the mirrored pair (roles swapped)
  const int mirror = p.view;
  const float* own = mirror ? right_hwc : left_hwc;
  const float* other = mirror ? left_hwc : right_hwc;
  hipLaunchKernelGGL(lexp::k_pack, dim3(nb), dim3(256), 0, s, own, c->left4, c->left4T, c->W, c->H, mirror);
  hipLaunchKernelGGL(lexp::k_pack, dim3(nb), dim3(256), 0, s, other, c->right4, (float4*)nullptr, c->W, c->H,
                     mirror);
  hipLaunchKernelGGL(lexp::k_guide_h, dim3(nb), dim3(256), 0, s, c->left4, tmp, c->W, c->H, c->r);
  hipLaunchKernelGGL(lexp::k_guide_v, dim3(nb), dim3(256), 0, s, tmp, c->guide, c->W, c->H, c->r, p.gf_eps);
  hipLaunchKernelGGL(lexp::k_weights, dim3(nb), dim3(256), 0, s, own, c->wts, c->W, c->H, p.gamma, mirror);
  hipError_t e = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(s);
  (void)hipFree(tmp);
  if (e != hipSuccess || e2 != hipSuccess)
    return fail(LEXP_EDEVICE, "set-up kernels: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  HIP_TRY(c->d_pair.ensure(1));
  HIP_TRY(c->h_pair.ensure(1));
  c->h_pair.p[0] = pair_entry(c.get(), nullptr, nullptr);
  HIP_TRY(hipMemcpy(c->d_pair.p, c->h_pair.p, sizeof(PairDev), hipMemcpyHostToDevice));
  HIP_TRY(hipEventCreateWithFlags(&c->staging_done, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(c->staging_done, s));
  int nt = p.host_threads;
  if (nt == 0) nt = std::min(default_threads(), 64);
  c->n_threads = nt;
  *out = c.release();
  return LEXP_OK;
}

lexp_status lexp_destroy(lexp_ctx* c) {
  if (!c) return LEXP_OK;
  (void)hipDeviceSynchronize();
  collect_timing(c);
  for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
  if (c->staging_done) (void)hipEventDestroy(c->staging_done);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  (void)hipFree(c->left4);
  (void)hipFree(c->left4T);
  (void)hipFree(c->right4);
  (void)hipFree(c->guide);
  (void)hipFree(c->wts);
  c->d_items.release(); c->d_tiles.release(); c->d_phi.release(); c->d_terms.release(); c->d_x.release();
  c->d_flag.release(); c->d_partial.release(); c->d_labels_tmp.release();
  c->d_status.release(); c->h_status.release();
  c->d_pair.release(); c->h_pair.release(); c->d_run_pairs.release(); c->h_run_pairs.release();
  c->d_post.release();
  c->h_items.release(); c->h_tiles.release(); c->h_terms.release(); c->h_x.release(); c->h_flag.release();
  c->h_partial.release(); c->h_labels4.release();
  c->d_bitems.release(); c->d_btiles.release(); c->d_bphi.release(); c->h_bitems.release(); c->h_btiles.release();
  for (auto& B : c->part)
    for (int i = 0; i < 2; ++i) {
      B.d_sitems[i].release(); B.d_stiles[i].release(); B.d_sphi[i].release();
      B.h_sitems[i].release(); B.h_stiles[i].release();
    }
  for (auto& b : c->part) {
    b.d_items.release(); b.d_phi.release(); b.d_terms.release();
    b.h_items.release(); b.h_terms.release(); b.h_x.release(); b.h_res.release();
    if (b.ready) (void)hipEventDestroy(b.ready);
    if (b.half) (void)hipEventDestroy(b.half);
    if (b.cut0) (void)hipEventDestroy(b.cut0);
    if (b.cut1) (void)hipEventDestroy(b.cut1);
  }
  delete c;
  return LEXP_OK;
}

lexp_status lexp_unary_cost(lexp_ctx* c, int32_t n, const lexp_rect* rects, const lexp_plane* labels,
                            const int64_t* offsets, float* out_cost, void* hip_stream) {
  lexp_status st = validate_items(c, n, rects, labels, offsets);
  if (st) return st;
  if (n > 0 && !out_cost) return fail(LEXP_EINVAL, "null output");
  if (n == 0) return LEXP_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  if ((st = wait_staging(c))) return st;
  if ((st = stage_items(c, n, rects, labels, offsets, nullptr))) return st;
  std::vector<Tile> tiles;
  TileCaps caps;
  plan_tiles(c, c->h_items.p, n, tiles, caps);
  HIP_TRY(c->h_tiles.ensure(tiles.size()));
  std::copy(tiles.begin(), tiles.end(), c->h_tiles.p);
  HIP_TRY(c->d_items.ensure((size_t)n));
  HIP_TRY(c->d_tiles.ensure(tiles.size()));
  HIP_TRY(hipMemcpyAsync(c->d_items.p, c->h_items.p, sizeof(Item) * n, hipMemcpyHostToDevice, s));
  if (!tiles.empty())
    HIP_TRY(hipMemcpyAsync(c->d_tiles.p, c->h_tiles.p, sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, s));
  double bytes = 0.0;
  int64_t evals = 0;
  for (int i = 0; i < n; ++i) {
    bytes += item_alg_bytes(c, c->h_items.p[i]);
    evals += (int64_t)c->h_items.p[i].rw * c->h_items.p[i].rh;
  }
  st = launch_unary<0>(c, c->d_pair.p, c->d_items.p, c->d_tiles.p, (int)tiles.size(), caps, nullptr, out_cost, s,
                       bytes, evals, n, 0, tiles_direct(tiles.data(), tiles.size(), (size_t)n));
  if (st) return st;
  HIP_TRY(hipEventRecord(c->staging_done, s));
  return LEXP_OK;
}

lexp_status lexp_guided_coeffs(lexp_ctx* c, int32_t n, const lexp_rect* rects, const lexp_plane* labels,
                               const int64_t* offsets, float* out_ab, void* hip_stream) {
  lexp_status st = validate_items(c, n, rects, labels, offsets);
  if (st) return st;
  if (n > 0 && !out_ab) return fail(LEXP_EINVAL, "null output");
  if (n == 0) return LEXP_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  if ((st = wait_staging(c))) return st;
  if ((st = stage_items(c, n, rects, labels, offsets, nullptr))) return st;
  std::vector<Tile> tiles;
  TileCaps caps;
  plan_tiles(c, c->h_items.p, n, tiles, caps);
  HIP_TRY(c->h_tiles.ensure(tiles.size()));
  std::copy(tiles.begin(), tiles.end(), c->h_tiles.p);
  HIP_TRY(c->d_items.ensure((size_t)n));
  HIP_TRY(c->d_tiles.ensure(tiles.size()));
  HIP_TRY(hipMemcpyAsync(c->d_items.p, c->h_items.p, sizeof(Item) * n, hipMemcpyHostToDevice, s));
  if (!tiles.empty())
    HIP_TRY(hipMemcpyAsync(c->d_tiles.p, c->h_tiles.p, sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, s));
  st = launch_unary<1>(c, c->d_pair.p, c->d_items.p, c->d_tiles.p, (int)tiles.size(), caps, nullptr, out_ab, s, 0.0,
                       0, n, 0, tiles_direct(tiles.data(), tiles.size(), (size_t)n));
  if (st) return st;
  HIP_TRY(hipEventRecord(c->staging_done, s));
  return LEXP_OK;
}

lexp_status lexp_pixel_costs(lexp_ctx* c, const float* labels, float* out_cost, void* hip_stream) {
  if (!c || !labels || !out_cost) return fail(LEXP_EINVAL, "null argument");
  return pixel_costs_impl(c, labels, out_cost, (hipStream_t)hip_stream);
}

static lexp_status prepare_expand(lexp_ctx* c, int32_t n, const lexp_rect* rects, const lexp_plane* alpha,
                                  const float* alpha_cost, const int64_t* offsets, const float* labels,
                                  const float* cur_cost, int64_t* n_px) {
  lexp_status st = validate_items(c, n, rects, alpha, offsets);
  if (st) return st;
  if (n > 0 && (!alpha_cost || !labels || !cur_cost)) return fail(LEXP_EINVAL, "null device buffer");
  if ((st = wait_staging(c))) return st;
  if ((st = stage_items(c, n, rects, alpha, offsets, nullptr))) return st;
  int64_t acc = 0;
  for (int i = 0; i < n; ++i) {
    c->h_items.p[i].aux_off = acc;
    acc += (int64_t)c->h_items.p[i].rw * c->h_items.p[i].rh;
  }
  *n_px = acc;
  return check_separated(c, n, c->h_items.p);
}

lexp_status lexp_expand_region(lexp_ctx* c, int32_t n, const lexp_rect* rects, const lexp_plane* alpha,
                               const float* alpha_cost, const int64_t* offsets, float* labels, float* cur_cost,
                               int64_t* delta_Eq, int32_t* n_changed, void* hip_stream) {
  int64_t n_px = 0;
  lexp_status st = prepare_expand(c, n, rects, alpha, alpha_cost, offsets, labels, cur_cost, &n_px);
  if (st) return st;
  if (n == 0) return LEXP_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  st = expand_batch(c, n, n_px, alpha_cost, labels, cur_cost, delta_Eq, n_changed, nullptr, nullptr, s, false);
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(s));
  return LEXP_OK;
}

lexp_status lexp_graph_terms(lexp_ctx* c, int32_t n, const lexp_rect* rects, const lexp_plane* alpha,
                             const float* alpha_cost, const int64_t* offsets, const float* labels,
                             const float* cur_cost, int32_t* out_terms, void* hip_stream) {
  int64_t n_px = 0;
  lexp_status st = prepare_expand(c, n, rects, alpha, alpha_cost, offsets, labels, cur_cost, &n_px);
  if (st) return st;
  if (n > 0 && !out_terms) return fail(LEXP_EINVAL, "null output");
  if (n == 0) return LEXP_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  for (int i = 0; i < n; ++i) c->h_items.p[i].aux_off = offsets[i];
  int max_px = 1;
  for (int i = 0; i < n; ++i) max_px = std::max(max_px, c->h_items.p[i].rw * c->h_items.p[i].rh);
  HIP_TRY(c->d_items.ensure((size_t)n));
  HIP_TRY(c->d_flag.ensure(1));
  HIP_TRY(hipMemcpyAsync(c->d_items.p, c->h_items.p, sizeof(Item) * n, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(c->d_flag.p, 0, sizeof(int), s));
  if ((st = stage_pair(c, const_cast<float*>(labels), const_cast<float*>(cur_cost), s))) return st;
  hipLaunchKernelGGL(lexp::k_graph_terms, dim3((max_px + 255) / 256, n), dim3(256), 0, s, c->d_pair.p,
                     c->d_items.p, alpha_cost, out_terms, c->d_flag.p);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(c->staging_done, s));
  return LEXP_OK;
}

lexp_status lexp_pairwise(lexp_ctx* c, int32_t pu, int32_t pv, int32_t qu, int32_t qv, lexp_plane fp, lexp_plane fq,
                          double* out) {
  if (!c || !out) return fail(LEXP_EINVAL, "null argument");
  if (pu < 0 || pv < 0 || qu < 0 || qv < 0 || pu >= c->W || qu >= c->W || pv >= c->H || qv >= c->H)
    return fail(LEXP_EINVAL, "pixel outside the image");
  if (std::abs(pu - qu) > 1 || std::abs(pv - qv) > 1 || (pu == qu && pv == qv))
    return fail(LEXP_EINVAL, "p and q are not 8-neighbours");
  if (!finite_plane(fp) || !finite_plane(fq)) return fail(LEXP_EINVAL, "label not finite");
  HIP_TRY(c->d_partial.ensure(2));
  hipLaunchKernelGGL(lexp::k_pair1, dim3(1), dim3(1), 0, 0, c->dp, c->wts, pu, pv, qu, qv,
                     make_float4(fp.a, fp.b, fp.c, 0.f), make_float4(fq.a, fq.b, fq.c, 0.f), c->d_partial.p);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpy(out, c->d_partial.p, sizeof(double), hipMemcpyDeviceToHost));
  return LEXP_OK;
}

lexp_status lexp_energy(lexp_ctx* c, const float* labels, const float* cur_cost, double* total, double* unary,
                        double* pairwise, void* hip_stream) {
  if (!c || !labels || !cur_cost) return fail(LEXP_EINVAL, "null argument");
  return energy_impl(c, labels, cur_cost, total, unary, pairwise, (hipStream_t)hip_stream);
}

lexp_status lexp_energy_noalloc(lexp_ctx* c, const float* labels, const float* cur_cost, double* total,
                                double* unary, double* pairwise, void* hip_stream) {
  if (!c || !labels || !cur_cost) return fail(LEXP_EINVAL, "null argument");
  const int64_t n = (int64_t)c->W * c->H;
  if (n > LEXP_NOALLOC_MAX_PIXELS)
    return fail(LEXP_EINVAL, "image of %lld pixels: the no-allocation energy holds at most %d", (long long)n,
                LEXP_NOALLOC_MAX_PIXELS);
  if (!c->noalloc_scratch) return fail(LEXP_ESTATE, "no scratch address for the context's device");
  const int nb = (int)((n + 255) / 256);
  hipStream_t s = (hipStream_t)hip_stream;
  double* partial = c->noalloc_scratch;
  double* totals = partial + 2 * kNoAllocBlocks;
  // every partial read is written first, and so are the totals: nothing needs clearing
  hipLaunchKernelGGL(lexp::k_energy, dim3(nb), dim3(256), 0, s, c->dp, (const float4*)labels, cur_cost, c->wts,
                     partial);
  hipLaunchKernelGGL(lexp::k_energy_total, dim3(1), dim3(256), 0, s, (const double*)partial, nb, totals);
  HIP_TRY(hipGetLastError());
  double host[2] = {0.0, 0.0};
  HIP_TRY(hipMemcpyAsync(host, totals, sizeof(host), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (total) *total = host[0] + host[1];
  if (unary) *unary = host[0];
  if (pairwise) *pairwise = host[1];
  return LEXP_OK;
}

lexp_status lexp_view_labels(lexp_ctx* c, const float* labels_in, float* labels_out, void* hip_stream) {
  if (!c || !labels_in || !labels_out) return fail(LEXP_EINVAL, "null argument");
  const size_t n = (size_t)c->W * c->H;
  const float* a = labels_in;
  const float* b = labels_out;
  if (a < b + 4 * n && b < a + 4 * n) return fail(LEXP_EINVAL, "labels_in and labels_out overlap");
  hipLaunchKernelGGL(lexp::k_view_labels, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)hip_stream,
                     (const float4*)labels_in, (float4*)labels_out, c->W, c->H, c->prm.view);
  HIP_TRY(hipGetLastError());
  return LEXP_OK;
}

lexp_status lexp_postprocess(lexp_ctx* left, const float* labels_left, lexp_ctx* right, const float* labels_right,
                             float* out_disp, uint8_t* out_invalid, void* hip_stream) {
  if (!left || !right || !labels_left || !labels_right || !out_disp) return fail(LEXP_EINVAL, "null argument");
  if (left->prm.view != 0 || right->prm.view != 1)
    return fail(LEXP_EINVAL, "left must be a left-view context and right a right-view context");
  if (left->W != right->W || left->H != right->H) return fail(LEXP_EINVAL, "the two views differ in size");
  hipStream_t s = (hipStream_t)hip_stream;
  const int W = left->W, H = left->H;
  const size_t n = (size_t)W * H;
  // scratch: disparity and fill (FP64), next-consistent links (int), flags (byte)
  HIP_TRY(left->d_post.ensure(n * (8 + 8 + 4 + 1)));
  double* disp = reinterpret_cast<double*>(left->d_post.p);
  double* fill = disp + n;
  int* next_ok = reinterpret_cast<int*>(fill + n);
  uint8_t* ok = reinterpret_cast<uint8_t*>(next_ok + n);
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(lexp::k_pp_check, dim3(nb), dim3(256), 0, s, (const float4*)labels_left,
                     (const float4*)labels_right, W, H, disp, ok);
  hipLaunchKernelGGL(lexp::k_pp_fill, dim3((unsigned)((H + 63) / 64)), dim3(64), 0, s, (const float4*)labels_left,
                     disp, ok, W, H, next_ok, fill);
  hipLaunchKernelGGL(lexp::k_pp_median, dim3((unsigned)n), dim3(256), 0, s, left->left4, disp, fill, ok, W, H,
                     left->prm.gamma, out_disp, out_invalid);
  HIP_TRY(hipGetLastError());
  return LEXP_OK;
}

lexp_status lexp_init_labels(lexp_ctx* c, uint64_t seed, float* labels, void* hip_stream) {
  if (!c || !labels) return fail(LEXP_EINVAL, "null argument");
  std::vector<float> h((size_t)c->W * c->H * 3);
  lexp_status st = lexp_init_labels_host(c->W, c->H, c->prm.disp_max, seed, h.data());
  if (st) return st;
  if ((st = wait_staging(c))) return st;
  return upload_labels(c, h.data(), labels, (hipStream_t)hip_stream);
}

}  // extern "C"

namespace {

constexpr int lexp_net_ch(int l) { return lexp_net::kCh[l]; }

// Forward pass of the network on a context's images and a label field
// (device HxWx4); the output stays in net->y, the planes in net->planes.
lexp_status net_forward(lexp_net* net, lexp_ctx* c, const float* labels, hipStream_t s) {
  const int W = c->W, H = c->H;
  if (W > net->max_w || H > net->max_h)
    return fail(LEXP_EINVAL, "image %dx%d larger than the network's %dx%d", W, H, net->max_w, net->max_h);
  const int n = W * H;
  hipLaunchKernelGGL(lexp::k_net_input, dim3((n + 255) / 256), dim3(256), 0, s, c->left4, c->right4,
                     (const float4*)labels, W, H, (double)c->prm.disp_max, net->act[0]);
  // forward: a workgroup per kConvRows rows of a run of 16 kConvSegs columns
  const int run = 16 * lexp::kConvSegs;
  const dim3 grid(((W + run - 1) / run) * ((H + lexp::kConvRows - 1) / lexp::kConvRows)), block(lexp::kConvThreads);
  for (int l = 0; l < lexp_net::kLayers; ++l) {
    const uint16_t* w16 = net->w16 + net->w16_off[l];
    const float* b = net->prm + net->b_off[l];
    if (l == 0)
      hipLaunchKernelGGL((lexp::k_conv_fwd<16, 32, false>), grid, block, 0, s, net->act[0], w16, b, W, H,
                         net->act[1], (float*)nullptr);
    else if (l < lexp_net::kLayers - 1)
      hipLaunchKernelGGL((lexp::k_conv_fwd<32, 32, false>), grid, block, 0, s, net->act[l], w16, b, W, H,
                         net->act[l + 1], (float*)nullptr);
    else
      hipLaunchKernelGGL((lexp::k_conv_fwd<32, 16, true>), grid, block, 0, s, net->act[l], w16, b, W, H,
                         (uint16_t*)nullptr, net->y);
  }
  hipLaunchKernelGGL(lexp::k_net_planes, dim3((n + 255) / 256), dim3(256), 0, s, net->y, W, H,
                     (double)c->prm.disp_max, net->planes);
  HIP_TRY(hipGetLastError());
  return LEXP_OK;
}

// Weight and bias gradients of layer l from the gradient g of its output.
template <int CI, int CO>
void net_weight_grad(lexp_net* net, int l, const uint16_t* g, int W, int H, hipStream_t s) {
  const int chunks = lexp_net::grad_chunks(W, H);
  hipLaunchKernelGGL((lexp::k_conv_bwd_w<CI, CO>), dim3(chunks), dim3(lexp::kWgThreads), 0, s, g, net->act[l], W, H,
                     net->part_w, net->part_b);
  hipLaunchKernelGGL(lexp::k_sum_chunks, dim3((9 * CO * CI + 63) / 64), dim3(256), 0, s, net->part_w, chunks,
                     9 * CO * CI, net->grad + net->w_off[l]);
  hipLaunchKernelGGL(lexp::k_sum_chunks, dim3((CO + 63) / 64), dim3(256), 0, s, net->part_b, chunks, CO,
                     net->grad + net->b_off[l]);
}

}  // namespace

namespace {

// One stereo pair of an optimisation run.
struct RunPair {
  lexp_ctx* c = nullptr;
  uint64_t seed = 0;
  float* labels = nullptr;
  float* cur_cost = nullptr;
  double* energy_trace = nullptr;
  std::vector<float> mirror;  // host copy of the labels (HxWx3) for the proposers
  std::vector<float> net_planes;  // learned proposals of the current level pass (HxWx4), if any
};

// One part of a group step: regions of one or more pairs (Item::pair), their
// cells, compact offsets and tiles.
struct Part {
  std::vector<int> ci, cj;
  std::vector<Item> items;
  int64_t n_px = 0;
  int max_px = 1;
  size_t tile_off = 0, n_tiles = 0;
  TileCaps caps;
  double bytes = 0.0;
  bool device_cut = false;  // minimum cuts by the device max-flow
  int pair_hint = -1;       // the pair of every item, if they share one
  int direct = 0;           // tile i is the only tile of item i
  hipGraphExec_t graph = nullptr;  // captured device sequence of one step of this part (graph mode)
  float* phi_ext = nullptr;  // batch cycle: the group's costs, evaluated for every step at once (items'
                             // out_off index it); speculation: the costs of the step's matched candidates;
                             // nullptr: this part's own buffer, evaluated per step
  int spec_step = -1;            // step whose two possible candidates per region were evaluated (-1: none)
  std::vector<float> spec_al;    // those candidates: region q's at 6q (label at r kept) and 6q+3 (changed)
};

// Per grid level: picks the device max-flow's launch shape by timing each
// candidate shape twice, interleaved, on the level's first device-cut steps,
// then keeps the fastest on average.  A launch whose largest region is of
// another size class than the first gets the default shape.
struct CutTuner {
  static constexpr int kRounds = 2;
  std::vector<CutShape> cand;
  std::vector<double> ms;
  int cls = -1, trials = 0;
  bool done = false;
  CutShape best{};

  static int size_class(const lexp_ctx* c, int max_px) { return max_px <= 512 ? 0 : (cut_full_fits(c, max_px) ? 1 : 2); }

  CutShape pick(const lexp_ctx* c, int max_px, bool* timed) {
    *timed = false;
    if (cls < 0) {
      cls = size_class(c, max_px);
      cand = cut_shapes(c, max_px);
      ms.assign(cand.size(), 0.0);
    }
    if (size_class(c, max_px) != cls) return CutShape{};
    if (done) return best;
    *timed = true;
    return cand[trials % cand.size()];
  }

  void report(int block, int every, double t) {
    for (size_t i = 0; i < cand.size(); ++i)
      if (cand[i].block == block && cand[i].every == every) ms[i] += t;
    if (++trials >= kRounds * (int)cand.size()) {
      size_t b = 0;
      for (size_t i = 1; i < cand.size(); ++i)
        if (ms[i] < ms[b]) b = i;
      best = cand[b];
      done = true;
    }
  }
};

void drop_graph(Part& P) {
  if (P.graph) (void)hipGraphExecDestroy(P.graph);
  P.graph = nullptr;
}

// Split of each grid level's cuts between the device max-flow and the host
// pool.  Per group step the device evaluates and cuts part 0 while the host
// cuts part 1 (whose costs the device evaluates too); part 0 takes a share
// `share` of the regions the device can hold.  A level whose groups have more
// than four regions per host thread starts at an even split and is tuned by
// hill climbing on the wall time per region pixel of its group steps: the
// share keeps moving while that time falls, and turns back with half the
// step when it rises.  A level of smaller groups is cut on the host only (one
// part, all threads).  Any split gives the same labels: every cut is exact.
struct CutBalance {
  bool tune = false;
  double share = 0.0, step = 0.125;
  int dir = 1;
  double prev = -1.0;  // previous group step's milliseconds per region pixel

  void update(double ms_per_px) {
    if (!tune) return;
    if (prev >= 0.0) {
      if (ms_per_px > prev) {
        dir = -dir;
        step *= 0.5;
      } else {
        step *= 1.25;
      }
      step = std::min(0.25, std::max(1.0 / 64, step));
    }
    prev = ms_per_px;
    share = std::min(1.0, std::max(0.0, share + dir * step));
  }
};

struct StepArgs {
  int it, level, cell, kp, kr;  // kr: RANSAC steps of the level (after its kp propagation steps)
  double scale;  // 0.5^it: the iteration's perturbation sizes relative to the first (Alg. 2)
  RunPair* pairs;
};

// Alg. 1 candidate of region q of a part for a step, from its pair's host
// label mirror as it stands.
// (label_at_r: see lexp::propose)
void propose_plane(const Part& P, const StepArgs& a, int q, int step, float al[3],
                   const float* label_at_r = nullptr) {
  const Item& item = P.items[q];
  const RunPair& rp = a.pairs[item.pair];
  const lexp_ctx* c = rp.c;
  lexp::propose(c->W, c->H, rp.mirror.data(), 3, rp.seed, a.it, a.level, a.cell, P.ci[q], P.cj[q], step, a.kp,
                a.kr, c->prm.disp_max / 2.0 * a.scale, a.scale, al,
                rp.net_planes.empty() ? nullptr : rp.net_planes.data(), label_at_r);
}

// Alg. 1 candidate of region q of a part for a step, into its item.
void propose_item(Part& P, const StepArgs& a, int q, int step) {
  float al[3];
  propose_plane(P, a, q, step, al);
  Item& item = P.items[q];
  item.a = al[0];
  item.b = al[1];
  item.c = al[2];
}

// A part's items (with their candidates already proposed), cost kernel and
// graph terms (and the device cut), all queued on the stream; the terms (or
// the device's cuts) land in the host's pinned buffers.
lexp_status part_device_work(lexp_ctx* c, Part& P, lexp_ctx::PartBuf& B, const PairDev* d_pairs, const Tile* d_tiles,
                             CutTuner* tuner, bool capture, hipStream_t s) {
  const int n = (int)P.items.size();
  HIP_TRY(hipMemcpyAsync(B.d_items.p, B.h_items.p, sizeof(Item) * n, hipMemcpyHostToDevice, s));
  lexp_status st = LEXP_OK;
  const float* phi = P.phi_ext ? P.phi_ext : B.d_phi.p;
  if (!P.phi_ext) {
    st = launch_unary<0>(c, d_pairs, B.d_items.p, d_tiles + P.tile_off, (int)P.n_tiles, P.caps, nullptr, B.d_phi.p,
                         s, P.bytes, P.n_px, n, P.pair_hint, P.direct);
    if (st) return st;
  }
  B.split = 0;
  if (P.device_cut) {
    // the flag, the regions' status and their cuts go straight to the host's
    // pinned result buffer (no copy of their own)
    int* flag = reinterpret_cast<int*>(B.h_res.p);
    hipLaunchKernelGGL(lexp::k_graph_terms, dim3((P.max_px + 255) / 256, n), dim3(256), 0, s, d_pairs, B.d_items.p,
                       phi, B.d_terms.p + 1, flag);
    HIP_TRY(hipGetLastError());
    bool timed = false;
    const CutShape shape = tuner ? tuner->pick(c, P.max_px, &timed) : CutShape{};
    if (timed) HIP_TRY(hipEventRecord(B.cut0, s));
    if ((st = launch_cut(c, B.d_items.p, n, B.d_terms.p + 1, B.h_res.p + 4 + 4 * c->res_items, flag + 1, P.max_px, s,
                         shape)))
      return st;
    if (timed) HIP_TRY(hipEventRecord(B.cut1, s));
    B.cut_timed = timed;
    B.cut_block = shape.block;
    B.cut_every = shape.every;
  } else {
    // the terms go straight to the host's pinned buffer (the kernel writes
    // through PCIe; no copy of its own), flag first; outside graph capture
    // in two launches, the first half of the regions' terms ready on their own
    // (the writes are bound by the PCIe link, so the host cuts the larger
    // regions while the rest are in flight)
    const int split = !capture && n >= 8 ? n / 2 : 0;
    const int n1 = split ? split : n;
    hipLaunchKernelGGL(lexp::k_graph_terms, dim3((P.max_px + 255) / 256, n1), dim3(256), 0, s, d_pairs, B.d_items.p,
                       phi, B.h_terms.p + 1, B.h_terms.p);
    HIP_TRY(hipGetLastError());
    if (split) {
      HIP_TRY(hipEventRecord(B.half, s));
      hipLaunchKernelGGL(lexp::k_graph_terms, dim3((P.max_px + 255) / 256, n - split), dim3(256), 0, s, d_pairs,
                         B.d_items.p + split, phi, B.h_terms.p + 1, B.h_terms.p);
      HIP_TRY(hipGetLastError());
    }
    B.split = split;
  }
  return LEXP_OK;
}

// Queues one step of a part: its items (candidates already proposed) go to
// the pinned staging buffer, then the device work.  In graph mode the device
// work of the part's current split is captured once into a HIP graph (the
// items copy from the same pinned buffer and the kernels) and replayed for
// every candidate step.
lexp_status enqueue_part(lexp_ctx* c, Part& P, lexp_ctx::PartBuf& B, const PairDev* d_pairs, const Tile* d_tiles,
                         bool use_graph, CutTuner* tuner, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  std::copy(P.items.begin(), P.items.end(), B.h_items.p);
  if (use_graph) {
    if (!P.graph) {
      // captured on a stream of the context's own (the caller's stream may be
      // the legacy default stream, which cannot be captured); nothing runs
      // during capture, and the graph is launched on the caller's stream
      if (!c->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
      const hipStream_t cs = c->capture_stream;
      HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      lexp_status st = part_device_work(c, P, B, d_pairs, d_tiles, nullptr, true, cs);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(cs, &g);
      if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(LEXP_EDEVICE, "graph capture: %s", hipGetErrorString(e));
      const hipError_t e2 = hipGraphInstantiate(&P.graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e2 != hipSuccess) {
        P.graph = nullptr;
        return fail(LEXP_EDEVICE, "graph instantiation: %s", hipGetErrorString(e2));
      }
      c->stats.graphs_captured += 1;
    }
    HIP_TRY(hipGraphLaunch(P.graph, s));
    B.split = 0;
  } else {
    lexp_status st = part_device_work(c, P, B, d_pairs, d_tiles, tuner, false, s);
    if (st) return st;
  }
  HIP_TRY(hipEventRecord(B.ready, s));
  c->stats.host_enqueue_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return LEXP_OK;
}

// Waits for a part's cut (device path) or terms (host path), completes the
// cut on the host pool (every region on the host path; on the device path
// only the regions the kernel left unfinished, whose terms are fetched then),
// updates the host label mirrors and queues the label update on the device.
// With next_step >= 0, each worker then proposes its region's candidate for
// that step: a candidate reads labels of the region's own centre cell only,
// which no other region of the group changes (Lemma 3).
lexp_status finish_part(lexp_ctx* c, Part& P, lexp_ctx::PartBuf& B, const StepArgs& a, int next_step,
                        const PairDev* d_pairs, CutTuner* tuner, hipStream_t s) {
  const int n = (int)P.items.size();
  const bool dev = P.device_cut;
  // host path in two launches: regions [0, split) are ready with B.half, the
  // rest with B.ready (the first worker to reach one of them waits for it)
  const int split = dev ? 0 : B.split;
  lexp::ThreadPool& pool = pool_of(c);
  const auto t0 = std::chrono::steady_clock::now();
  HIP_TRY(hipEventSynchronize(split ? B.half : B.ready));
  const auto t1 = std::chrono::steady_clock::now();
  if (B.cut_timed && tuner) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, B.cut0, B.cut1));
    tuner->report(B.cut_block, B.cut_every, ms);
    B.cut_timed = false;
  }
  const char* overflow = "binary-problem term exceeds 2^30 quanta (parameters too large)";
  if (dev ? reinterpret_cast<const int*>(B.h_res.p)[0] : B.h_terms.p[0]) return fail(LEXP_EINVAL, "%s", overflow);
  const int nf = c->dp.nf;
  const int* terms = B.h_terms.p + 1;
  // the cut, in the host's pinned buffer, which the label update reads in place
  uint8_t* xs = dev ? B.h_res.p + 4 + 4 * c->res_items : B.h_x.p;
  std::vector<int> host_cut;  // device path: regions the kernel left to the host
  if (dev) {
    const int* status = reinterpret_cast<const int*>(B.h_res.p) + 1;
    for (int i = 0; i < n; ++i)
      if (!status[i]) host_cut.push_back(i);
    for (int i : host_cut) {
      const Item& it = P.items[i];
      HIP_TRY(hipMemcpyAsync(B.h_terms.p + 1 + (size_t)it.aux_off * 5, B.d_terms.p + 1 + (size_t)it.aux_off * 5,
                             sizeof(int) * 5 * (size_t)it.rw * it.rh, hipMemcpyDeviceToHost, s));
    }
    if (!host_cut.empty()) HIP_TRY(hipStreamSynchronize(s));
    c->stats.device_cut_fallbacks += (int64_t)host_cut.size();
  }
  // per-worker CPU time of the solves (summed into the statistics below)
  double solve_ms[lexp::kMaxPoolThreads] = {};
  int64_t solves[lexp::kMaxPoolThreads] = {};
  // the second launch's regions: 0 not yet waited for, 1 a worker waits, 2
  // ready, 3 failed (device error or overflow: every later region is skipped)
  std::atomic<int> rest{0};
  hipError_t rest_err = hipSuccess;
  double rest_wait_ms = 0.0;
  auto wait_rest = [&]() -> bool {
    int st = rest.load(std::memory_order_acquire);
    if (st == 0 && rest.compare_exchange_strong(st, 1, std::memory_order_acq_rel)) {
      const auto w0 = std::chrono::steady_clock::now();
      rest_err = hipEventSynchronize(B.ready);
      rest_wait_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
      st = rest_err == hipSuccess && B.h_terms.p[0] == 0 ? 2 : 3;
      rest.store(st, std::memory_order_release);
      return st == 2;
    }
    while ((st = rest.load(std::memory_order_acquire)) == 1) std::this_thread::yield();
    return st == 2;
  };
  auto host_solve = [&](int i, int worker) {
    const auto s0 = std::chrono::steady_clock::now();
    const Item& it = P.items[i];
    const int* t = terms + (size_t)it.aux_off * 5;
    lexp::BKSolver& bk = *c->solvers[worker];
    bk.load<int32_t>(it.rw, it.rh, nf, t, 5, t + 1, 5);
    bk.solve(xs + it.aux_off);
    solve_ms[worker] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - s0).count();
    solves[worker] += 1;
  };
  if (dev && !host_cut.empty())
    pool.parallel_for((int)host_cut.size(), [&](int q, int worker) { host_solve(host_cut[q], worker); });
  pool.parallel_for(n, [&](int i, int worker) {
    if (split && i >= split && !wait_rest()) return;
    const Item& it = P.items[i];
    if (it.rw > 0 && it.rh > 0) {
      if (!dev) host_solve(i, worker);
      const uint8_t* x = xs + it.aux_off;
      RunPair& rp = a.pairs[it.pair];
      const int W = rp.c->W;
      for (int q = 0; q < it.rw * it.rh; ++q) {
        if (!x[q]) continue;
        float* m = rp.mirror.data() + ((size_t)(it.rv0 + q / it.rw) * W + (it.ru0 + q % it.rw)) * 3;
        m[0] = it.a; m[1] = it.b; m[2] = it.c;
      }
    }
    if (next_step >= 0) propose_item(P, a, i, next_step);
  });
  if (split) {
    if (rest.load() == 0) wait_rest();  // (no worker reached the second launch's regions)
    if (rest_err != hipSuccess) return fail(LEXP_EDEVICE, "%s", hipGetErrorString(rest_err));
    if (B.h_terms.p[0]) return fail(LEXP_EINVAL, "%s", overflow);
  }
  const auto t2 = std::chrono::steady_clock::now();
  hipLaunchKernelGGL(lexp::k_apply, dim3((P.max_px + 255) / 256, n), dim3(256), 0, s, d_pairs, B.d_items.p, xs,
                     P.phi_ext ? P.phi_ext : B.d_phi.p);
  HIP_TRY(hipGetLastError());
  const auto t3 = std::chrono::steady_clock::now();
  c->stats.expand_calls += 1;
  c->stats.host_wait_ms += std::chrono::duration<double, std::milli>(t1 - t0).count() + rest_wait_ms;
  c->stats.host_cut_ms += std::chrono::duration<double, std::milli>(t2 - t1).count();
  c->stats.host_cut_level_ms[a.level] += std::chrono::duration<double, std::milli>(t2 - t1).count();
  for (int w = 0; w < pool.size(); ++w) {
    c->stats.host_solve_level_ms[a.level] += solve_ms[w];
    c->stats.host_solves[a.level] += solves[w];
  }
  c->stats.host_update_ms += std::chrono::duration<double, std::milli>(t3 - t2).count();
  return LEXP_OK;
}

// Clipped 3x3-cell region of cell (i, j).
void cell_region(const lexp_ctx* c, int cell, int i, int j, int* u0, int* v0, int* u1, int* v1) {
  lexp_rect rr{(i - 1) * cell, (j - 1) * cell, (i + 2) * cell, (j + 2) * cell};
  clip_rect(c, rr, u0, v0, u1, v1);
}

// All regions of one group step of a run (every pair), largest first, each
// with its tiles.
struct GroupPlan {
  std::vector<Item> items;               // pair, region and size (offsets set per part)
  std::vector<int> ci, cj, pair_part;    // cell of each region; its part in the pair's own split
  std::vector<std::vector<Tile>> tiles;  // tiles of each region (Tile::item unset)
  std::vector<TileCaps> caps;            // their widths
  size_t tile_off = 0, n_tiles = 0;      // the group's range in the run's tile table
  int64_t n_px = 0;
  double share = -2.0;                   // share of its current split (-2: not split yet)
};

// Appends one pair's regions of group k at grid level `cell` to a group plan.
// The pair's cells (Eq. (15): group 4 (j mod 4) + (i mod 4)) are ordered
// largest region first; when the pair has more than four regions per host
// thread in the group they alternate between two parts, otherwise all are in
// part 0.  Tiles are planned once for all of the pair's regions of the group,
// so a region's tiles (and with them the rounding of its costs) depend on the
// pair, the level and the group only: not on the host threads, not on which
// part of the run's group step it is put in, not on other pairs batched with
// it.
void plan_pair_group(const lexp_ctx* c, int pair, int cell, int k, const TilePlan& plan, GroupPlan& g) {
  const int nci = (c->W + cell - 1) / cell, ncj = (c->H + cell - 1) / cell;
  std::vector<std::pair<int, int>> cells;
  for (int j = k / 4; j < ncj; j += 4)
    for (int i = k % 4; i < nci; i += 4) cells.emplace_back(i, j);
  auto area = [&](const std::pair<int, int>& q) {
    int u0, v0, u1, v1;
    cell_region(c, cell, q.first, q.second, &u0, &v0, &u1, &v1);
    return (int64_t)(u1 - u0) * (v1 - v0);
  };
  std::stable_sort(cells.begin(), cells.end(),
                   [&](const std::pair<int, int>& x, const std::pair<int, int>& y) { return area(x) > area(y); });
  const bool split = cells.size() > (size_t)4 * c->n_threads;
  std::vector<Item> mine;
  for (const auto& q : cells) {
    int u0, v0, u1, v1;
    cell_region(c, cell, q.first, q.second, &u0, &v0, &u1, &v1);
    Item it{};
    it.ru0 = u0; it.rv0 = v0; it.rw = u1 - u0; it.rh = v1 - v0;
    it.pair = pair;
    mine.push_back(it);
  }
  std::vector<Tile> t;
  TileCaps unused;
  plan_tiles(c, mine.data(), (int)mine.size(), t, unused, plan);
  const size_t base = g.items.size();
  for (size_t q = 0; q < mine.size(); ++q) {
    g.items.push_back(mine[q]);
    g.ci.push_back(cells[q].first);
    g.cj.push_back(cells[q].second);
    g.pair_part.push_back(split ? (int)(q & 1) : 0);
    g.tiles.emplace_back();
    g.caps.emplace_back();
    g.n_px += (int64_t)mine[q].rw * mine[q].rh;
  }
  for (Tile tl : t) {
    const size_t q = base + (size_t)tl.item;
    tl.item = 0;
    TileCaps& cp = g.caps[q];
    cp.wp = std::max(cp.wp, std::min(tl.tu1 + c->r, c->W) - std::max(tl.tu0 - c->r, 0));
    cp.tw = std::max(cp.tw, tl.tu1 - tl.tu0);
    const int wm = std::min(tl.tu1 + 2 * c->r, c->W) - std::max(tl.tu0 - 2 * c->r, 0);
    cp.ws = std::max(cp.ws, std::max(wm, cp.wp));
    g.tiles[q].push_back(tl);
    g.n_tiles += 1;
  }
}

// Orders a group plan largest region first (stable: ties keep pair order).
void sort_group(GroupPlan& g) {
  std::vector<size_t> ord(g.items.size());
  for (size_t q = 0; q < ord.size(); ++q) ord[q] = q;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
    return (int64_t)g.items[x].rw * g.items[x].rh > (int64_t)g.items[y].rw * g.items[y].rh;
  });
  GroupPlan o;
  o.n_px = g.n_px;
  o.n_tiles = g.n_tiles;
  for (size_t q : ord) {
    o.items.push_back(g.items[q]);
    o.ci.push_back(g.ci[q]);
    o.cj.push_back(g.cj[q]);
    o.pair_part.push_back(g.pair_part[q]);
    o.tiles.push_back(std::move(g.tiles[q]));
    o.caps.push_back(g.caps[q]);
  }
  g = std::move(o);
}

// Splits a group step into its two parts and writes their tiles (part 0 then
// part 1) to the group's range of the tile table.  share < 0: every cut on
// the host, the parts being the pairs' own splits.  Otherwise part 0 takes
// that share of the regions the device max-flow can hold (every region of
// part 0 is cut on the device) and part 1 the rest; when the group's tiles
// fit two rounds of one tile per CU, part 0 takes at most one round (a launch
// of a few more tiles than CUs would take two rounds).
void assign_parts(const RunPair* pairs, const GroupPlan& g, double share, Part* P, Tile* table) {
  const lexp_ctx* c = pairs[0].c;
  for (int hp = 0; hp < 2; ++hp) P[hp] = Part{};
  std::vector<int> which(g.items.size());
  const size_t budget = g.n_tiles <= (size_t)2 * c->n_cu ? (size_t)c->n_cu : g.n_tiles;
  size_t tiles0 = 0;
  double acc = 0.5;
  for (size_t q = 0; q < g.items.size(); ++q) {
    const Item& it = g.items[q];
    if (share < 0) {
      which[q] = g.pair_part[q];
    } else if (cut_fits(c, (int64_t)it.rw * it.rh)) {
      acc += share;
      which[q] = acc >= 1.0 && tiles0 + g.tiles[q].size() <= budget ? 0 : 1;
      if (acc >= 1.0) acc -= 1.0;
      if (which[q] == 0) tiles0 += g.tiles[q].size();
    } else {
      which[q] = 1;
    }
  }
  size_t t_at = g.tile_off;
  for (int hp = 0; hp < 2; ++hp) {
    Part& Q = P[hp];
    Q.tile_off = t_at;
    for (size_t q = 0; q < g.items.size(); ++q) {
      if (which[q] != hp) continue;
      Item it = g.items[q];
      it.out_off = Q.n_px;
      it.aux_off = Q.n_px;
      Q.n_px += (int64_t)it.rw * it.rh;
      Q.max_px = std::max(Q.max_px, it.rw * it.rh);
      Q.bytes += item_alg_bytes(pairs[it.pair].c, it);
      Q.caps.wp = std::max(Q.caps.wp, g.caps[q].wp);
      Q.caps.tw = std::max(Q.caps.tw, g.caps[q].tw);
      Q.caps.ws = std::max(Q.caps.ws, g.caps[q].ws);
      const int idx = (int)Q.items.size();
      for (Tile tl : g.tiles[q]) {
        tl.item = idx;
        table[t_at++] = tl;
      }
      Q.items.push_back(it);
      Q.ci.push_back(g.ci[q]);
      Q.cj.push_back(g.cj[q]);
    }
    Q.n_tiles = t_at - Q.tile_off;
    Q.direct = tiles_direct(table + Q.tile_off, Q.n_tiles, Q.items.size());
    Q.pair_hint = Q.items.empty() ? -1 : Q.items[0].pair;
    for (const Item& it : Q.items)
      if (it.pair != Q.pair_hint) Q.pair_hint = -1;
  }
  P[0].device_cut = share >= 0 && !P[0].items.empty();
}

// Batch cycle of one group step: the candidates of every step of every
// region are drawn from the labels at the group's start (cand, per part:
// region-major, 3 floats per step), and one fused-cost launch evaluates all
// of them.  Each region keeps its own tiles, so a cost has the rounding it
// has in a step-by-step run.  Costs of step t, part hp, region q go to
// d_bphi at t * G + base_hp + (the region's compact offset), G being the
// group's pixels and base_1 the pixels of part 0.
lexp_status batch_costs(lexp_ctx* c, RunPair* pairs, Part* const* P, const StepArgs& a, int K,
                        const PairDev* d_pairs, hipStream_t s) {
  if (K <= 0) return LEXP_OK;
  const int64_t G = P[0]->n_px + P[1]->n_px;
  size_t n_items = 0, n_tiles = 0;
  for (int hp = 0; hp < 2; ++hp) {
    n_items += P[hp]->items.size();
    n_tiles += P[hp]->n_tiles;
  }
  if (n_items == 0) return LEXP_OK;
  HIP_TRY(c->h_bitems.ensure(n_items * K));
  HIP_TRY(c->h_btiles.ensure(n_tiles * K));
  HIP_TRY(c->d_bitems.ensure(n_items * K));
  HIP_TRY(c->d_btiles.ensure(n_tiles * K));
  HIP_TRY(c->d_bphi.ensure((size_t)G * K));
  // the staging buffers were last read by the previous group step's launch,
  // which the host has waited for through that step's parts
  Item* bi = c->h_bitems.p;
  Tile* bt = c->h_btiles.p;
  size_t ii = 0, ti = 0;
  TileCaps caps;
  double bytes = 0.0;
  int hint = -2;
  for (int hp = 0; hp < 2; ++hp) {
    Part& Q = *P[hp];
    const int64_t base = hp == 0 ? 0 : P[0]->n_px;
    caps.wp = std::max(caps.wp, Q.caps.wp);
    caps.tw = std::max(caps.tw, Q.caps.tw);
    caps.ws = std::max(caps.ws, Q.caps.ws);
    for (const Item& it : Q.items) hint = hint == -2 ? it.pair : (hint == it.pair ? hint : -1);
    const size_t first = ii;
    pool_of(c).parallel_for((int)Q.items.size(), [&](int q, int) {
      for (int t = 0; t < K; ++t) {
        Item it = Q.items[q];
        float al[3];
        propose_plane(Q, a, q, t, al);
        it.a = al[0];
        it.b = al[1];
        it.c = al[2];
        it.out_off = (long long)t * G + base + Q.items[q].aux_off;
        bi[first + (size_t)t * Q.items.size() + q] = it;
      }
    });
    for (int t = 0; t < K; ++t)
      for (size_t j = 0; j < Q.n_tiles; ++j) {
        Tile tl = c->h_tiles.p[Q.tile_off + j];
        tl.item += (int)(first + (size_t)t * Q.items.size());
        bt[ti++] = tl;
      }
    ii += Q.items.size() * K;
    bytes += Q.bytes * K;
  }
  HIP_TRY(hipMemcpyAsync(c->d_bitems.p, bi, sizeof(Item) * ii, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(c->d_btiles.p, bt, sizeof(Tile) * ti, hipMemcpyHostToDevice, s));
  return launch_unary<0>(c, d_pairs, c->d_bitems.p, c->d_btiles.p, (int)ti, caps, nullptr, c->d_bphi.p, s, bytes,
                         G * K, (int64_t)ii, hint >= 0 ? hint : -1, 0);
}

// Speculative costs of a part's step t (t >= 1, not a RANSAC step), queued
// before the host cuts step t-1.  A region's candidate for step t reads the
// label at one drawn pixel r of its centre cell (Alg. 1 propagation and
// refinement), and the cut of step t-1 either keeps that label or sets it to
// step t-1's candidate (r lies inside the region, which no other region of
// the group touches, Lemma 3).  Both possible candidates of every region are
// evaluated in one launch over the part's own tiles, so each candidate's costs
// are those its own launch would give; after the cut, spec_match picks the
// one the updated labels propose.
lexp_status spec_launch(lexp_ctx* c, Part& Q, lexp_ctx::PartBuf& B, const StepArgs& a, int t, const PairDev* d_pairs,
                        hipStream_t s) {
  const size_t n = Q.items.size();
  const int par = t & 1;
  // the buffers of this parity were last read by step t-2's work, which the
  // host has waited for (its cut) before queueing anything of step t-1
  HIP_TRY(B.h_sitems[par].ensure(2 * n));
  HIP_TRY(B.d_sitems[par].ensure(2 * n));
  HIP_TRY(B.h_stiles[par].ensure(2 * Q.n_tiles));
  HIP_TRY(B.d_stiles[par].ensure(2 * Q.n_tiles));
  HIP_TRY(B.d_sphi[par].ensure((size_t)(2 * Q.n_px)));
  Q.spec_al.resize(6 * n);
  Item* si = B.h_sitems[par].p;
  pool_of(c).parallel_for((int)n, [&](int q, int) {
    const Item& cur = Q.items[q];  // its candidate is step t-1's
    const float alt[3] = {cur.a, cur.b, cur.c};
    float* al = &Q.spec_al[6 * (size_t)q];
    propose_plane(Q, a, q, t, al);            // r keeps its label
    propose_plane(Q, a, q, t, al + 3, alt);   // r takes step t-1's candidate
    for (int h = 0; h < 2; ++h) {
      Item it = cur;
      it.a = al[3 * h]; it.b = al[3 * h + 1]; it.c = al[3 * h + 2];
      it.out_off = (long long)h * Q.n_px + cur.aux_off;
      si[(size_t)h * n + q] = it;
    }
  });
  Tile* st = B.h_stiles[par].p;
  for (int h = 0; h < 2; ++h)
    for (size_t j = 0; j < Q.n_tiles; ++j) {
      Tile tl = c->h_tiles.p[Q.tile_off + j];
      tl.item += (int)((size_t)h * n);
      st[(size_t)h * Q.n_tiles + j] = tl;
    }
  HIP_TRY(hipMemcpyAsync(B.d_sitems[par].p, si, sizeof(Item) * 2 * n, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(B.d_stiles[par].p, st, sizeof(Tile) * 2 * Q.n_tiles, hipMemcpyHostToDevice, s));
  Q.spec_step = t;
  // evaluations count toward the run's total when used (spec_match)
  return launch_unary<0>(c, d_pairs, B.d_sitems[par].p, B.d_stiles[par].p, (int)(2 * Q.n_tiles), Q.caps, nullptr,
                         B.d_sphi[par].p, s, 2.0 * Q.bytes, 2 * Q.n_px, (int64_t)(2 * n), Q.pair_hint, 0, false);
}

// After the cut of step t-1 and the proposal of step t's candidates from the
// updated labels: when every candidate equals one of the two evaluated for
// its region (bit for bit), the step takes their costs; otherwise it
// evaluates its own.
// (t < 0: the part's own cost buffer, nothing speculated.)
void spec_match(lexp_ctx* c, Part& Q, lexp_ctx::PartBuf& B, int t) {
  Q.phi_ext = nullptr;
  for (Item& it : Q.items) it.out_off = it.aux_off;
  const bool ready = t >= 0 && Q.spec_step == t;
  Q.spec_step = -1;
  if (!ready) return;
  const size_t n = Q.items.size();
  std::vector<long long> off(n);
  for (size_t q = 0; q < n; ++q) {
    const Item& it = Q.items[q];
    const float got[3] = {it.a, it.b, it.c};
    int h = -1;
    for (int k = 0; k < 2 && h < 0; ++k)
      if (std::memcmp(got, &Q.spec_al[6 * q + 3 * k], sizeof(got)) == 0) h = k;
    if (h < 0) {
      c->stats.spec_misses += 1;
      return;
    }
    off[q] = (long long)h * Q.n_px + it.aux_off;
  }
  for (size_t q = 0; q < n; ++q) Q.items[q].out_off = off[q];
  Q.phi_ext = B.d_sphi[t & 1].p;
  c->stats.spec_steps += 1;
  if (c->timing) c->stats.unary_evals += Q.n_px;
}

// Items of a part for step t of a batch cycle (the part's items start at
// `first` in the group's batch table): the candidates drawn at the group's
// start, their costs' offsets in d_bphi.
void batch_step_items(const lexp_ctx* c, Part& Q, size_t first, int t) {
  const size_t n = Q.items.size();
  for (size_t q = 0; q < n; ++q) Q.items[q] = c->h_bitems.p[first + (size_t)t * n + q];
  Q.phi_ext = c->d_bphi.p;
}

// Alg. 2 for the pairs of a run, with one set of launches per group step for
// all pairs (the scratch, host pool and statistics of pairs[0]'s context).
lexp_status optimize_run(RunPair* pairs, int np, const lexp_schedule* sch, double* time_trace, hipStream_t s) {
  if (sch->n_levels < 1 || sch->n_levels > 4 || sch->iterations < 0) return fail(LEXP_EINVAL, "bad schedule");
  for (int h = 0; h < sch->n_levels; ++h)
    if (sch->cell[h] < 1 || sch->k_prop[h] < 0 || sch->k_rand[h] < 0 || sch->k_rans[h] < 0 ||
        sch->k_prop[h] + sch->k_rans[h] + sch->k_rand[h] > 64 || sch->tile_cols[h] < 0 ||
        sch->tile_cols[h] > lexp::kMaxTW || sch->tile_fill[h] < 0 || sch->tile_fill[h] > (1 << 20))
      return fail(LEXP_EINVAL, "bad grid level %d", h);
  if (sch->speculate != 0 && sch->speculate != 1) return fail(LEXP_EINVAL, "speculate must be 0 or 1");
  if (sch->batch_cycle != 0 && sch->batch_cycle != 1) return fail(LEXP_EINVAL, "batch_cycle must be 0 or 1");
  lexp_ctx* c = pairs[0].c;
  if (sch->learned != 0 && sch->learned != 1) return fail(LEXP_EINVAL, "learned must be 0 or 1");
  if (sch->learned)
    for (int p = 0; p < np; ++p)
      if (!pairs[p].c->net) return fail(LEXP_ESTATE, "pair %d: learned proposals need lexp_set_net", p);
  const auto t_start = std::chrono::steady_clock::now();
  auto now_s = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count(); };
  lexp_status st;
  for (int p = 0; p < np; ++p)
    if ((st = wait_staging(pairs[p].c))) return st;
  HIP_TRY(c->d_run_pairs.ensure((size_t)np));
  HIP_TRY(c->h_run_pairs.ensure((size_t)np));
  for (int p = 0; p < np; ++p) c->h_run_pairs.p[p] = pair_entry(pairs[p].c, pairs[p].labels, pairs[p].cur_cost);
  HIP_TRY(hipMemcpyAsync(c->d_run_pairs.p, c->h_run_pairs.p, sizeof(PairDev) * np, hipMemcpyHostToDevice, s));
  const PairDev* d_pairs = c->d_run_pairs.p;

  // Per (level, group): the regions of every pair and their tiles, split in
  // two parts that overlap: one is cut while the device evaluates the other's
  // next candidate.  With the device max-flow enabled, part 0 is cut on the
  // device and part 1 on the host, in a proportion balanced per level after
  // every iteration; otherwise both are cut on the host.
  const bool dev_cut = c->prm.device_cut != 0;
  // kernel timing events are not captured, so a timed run launches eagerly
  const bool use_graph = c->prm.graph != 0 && !c->timing && !sch->batch_cycle;
  // speculative costs of the next step (not with the batch cycle, whose
  // candidates are all drawn at a group's start, nor with graphs, whose
  // captured steps include their own cost launch)
  const bool speculate = sch->speculate != 0 && !sch->batch_cycle && !use_graph;
  std::vector<GroupPlan> groups((size_t)sch->n_levels * 16);
  std::vector<Part> parts((size_t)sch->n_levels * 16 * 2);
  struct GraphGuard {  // frees the captured graphs on every way out
    std::vector<Part>& p;
    ~GraphGuard() {
      for (Part& x : p) drop_graph(x);
    }
  } graph_guard{parts};
  struct LevelGuard {  // outside the run, timed launches are counted under no level
    lexp_ctx* c;
    ~LevelGuard() { c->time_level = -1; }
  } level_guard{c};
  std::vector<CutBalance> balance((size_t)sch->n_levels);
  std::vector<CutTuner> tuners((size_t)sch->n_levels);
  size_t n_tiles = 0;
  int64_t max_px = 1;
  size_t max_items = 1;
  for (int h = 0; h < sch->n_levels; ++h)
    for (int k = 0; k < 16; ++k) {
      GroupPlan& g = groups[(size_t)h * 16 + k];
      TilePlan plan;
      plan.cols = sch->tile_cols[h];
      if (sch->tile_fill[h] > 0) plan.fill = sch->tile_fill[h];
      for (int p = 0; p < np; ++p) plan_pair_group(pairs[p].c, p, sch->cell[h], k, plan, g);
      sort_group(g);
      g.tile_off = n_tiles;
      n_tiles += g.n_tiles;
      max_px = std::max(max_px, g.n_px);
      max_items = std::max(max_items, g.items.size());
    }
  for (int h = 0; h < sch->n_levels; ++h) {
    size_t regions = 0;
    for (int k = 0; k < 16; ++k) regions += groups[(size_t)h * 16 + k].items.size();
    balance[h].tune = dev_cut && regions > (size_t)16 * 4 * c->n_threads;
    balance[h].share = balance[h].tune ? 0.5 : 0.0;
  }
  HIP_TRY(c->d_tiles.ensure(n_tiles));
  HIP_TRY(c->h_tiles.ensure(n_tiles));
  // Splits group step (h, k) with its level's current share unless it is
  // split that way already, and uploads its tiles (the range was last read by
  // the group's previous step, queued earlier on the same stream, and last
  // copied before that step).
  auto split_group = [&](int h, int k) -> lexp_status {
    GroupPlan& g = groups[(size_t)h * 16 + k];
    const double share = dev_cut ? balance[h].share : -1.0;
    if (g.share == share) return LEXP_OK;
    g.share = share;
    drop_graph(parts[((size_t)h * 16 + k) * 2]);
    drop_graph(parts[((size_t)h * 16 + k) * 2 + 1]);
    assign_parts(pairs, g, share, &parts[((size_t)h * 16 + k) * 2], c->h_tiles.p);
    if (g.n_tiles > 0)
      HIP_TRY(hipMemcpyAsync(c->d_tiles.p + g.tile_off, c->h_tiles.p + g.tile_off, sizeof(Tile) * g.n_tiles,
                             hipMemcpyHostToDevice, s));
    return LEXP_OK;
  };
  c->res_items = max_items;

  for (auto& B : c->part) {
    HIP_TRY(B.d_items.ensure(max_items));
    HIP_TRY(B.d_phi.ensure((size_t)max_px));
    HIP_TRY(B.d_terms.ensure(1 + (size_t)max_px * 5));
    HIP_TRY(B.h_items.ensure(max_items));
    B.h_terms.coherent = true;  // written by k_graph_terms in place (host cuts)
    B.h_x.coherent = true;      // read by k_apply in place (host cuts)
    B.h_res.coherent = true;    // written by k_graph_terms and the device max-flow, read by k_apply, in place
    HIP_TRY(B.h_terms.ensure(1 + (size_t)max_px * 5));
    HIP_TRY(B.h_x.ensure((size_t)max_px));
    HIP_TRY(B.h_res.ensure(4 + 4 * max_items + (size_t)max_px));
    if (!B.ready) HIP_TRY(hipEventCreateWithFlags(&B.ready, hipEventDisableTiming));
    if (!B.half) HIP_TRY(hipEventCreateWithFlags(&B.half, hipEventDisableTiming));
    B.split = 0;
    if (!B.cut0) HIP_TRY(hipEventCreate(&B.cut0));
    if (!B.cut1) HIP_TRY(hipEventCreate(&B.cut1));
    B.cut_timed = false;
    B.h_terms.p[0] = 0;  // the overflow flags of both paths, written by the device in place
    reinterpret_cast<int*>(B.h_res.p)[0] = 0;
  }

  // Alg. 2, initialisation: random labels and their per-pixel costs.
  for (int p = 0; p < np; ++p) {
    RunPair& rp = pairs[p];
    lexp_ctx* pc = rp.c;
    rp.mirror.assign((size_t)pc->W * pc->H * 3, 0.f);
    if ((st = lexp_init_labels_host(pc->W, pc->H, pc->prm.disp_max, rp.seed, rp.mirror.data()))) return st;
    if ((st = upload_labels(pc, rp.mirror.data(), rp.labels, s))) return st;
    if ((st = pixel_costs_impl(pc, rp.labels, rp.cur_cost, s))) return st;
    if (rp.energy_trace)
      if ((st = energy_impl(pc, rp.labels, rp.cur_cost, &rp.energy_trace[0], nullptr, nullptr, s))) return st;
  }
  if (time_trace) time_trace[0] = now_s();

  double scale = 1.0;  // Alg. 2: perturbation sizes (r_d, r_n) = (disp_max / 2, 1) times scale
  for (int it = 0; it < sch->iterations; ++it) {
    for (int h = 0; h < sch->n_levels; ++h) {
      const int K = sch->k_prop[h] + sch->k_rans[h] + sch->k_rand[h];
      const StepArgs a{it, h, sch->cell[h], sch->k_prop[h], sch->k_rans[h], scale, pairs};
      c->time_level = h;
      if (sch->learned && it == 0) {
        for (int p = 0; p < np; ++p) pairs[p].net_planes.clear();  // random labels: nothing to learn from yet
      } else if (sch->learned) {
        // the network's planes from the labels at the start of the level pass
        for (int p = 0; p < np; ++p) {
          RunPair& rp = pairs[p];
          if ((st = net_forward(rp.c->net, rp.c, rp.labels, s))) return st;
          rp.net_planes.resize((size_t)rp.c->W * rp.c->H * 4);
          HIP_TRY(hipMemcpyAsync(rp.net_planes.data(), rp.c->net->planes, sizeof(float) * rp.net_planes.size(),
                                 hipMemcpyDeviceToHost, s));
        }
        HIP_TRY(hipStreamSynchronize(s));
      }
      for (int k = 0; k < 16; ++k) {
        const auto g0 = std::chrono::steady_clock::now();
        if ((st = split_group(h, k))) return st;
        Part* P[2] = {&parts[((size_t)h * 16 + k) * 2], &parts[((size_t)h * 16 + k) * 2 + 1]};
        if (sch->batch_cycle) {
          if ((st = batch_costs(c, pairs, P, a, K, d_pairs, s))) return st;
          for (int hp = 0; hp < 2; ++hp) batch_step_items(c, *P[hp], hp == 0 ? 0 : P[0]->items.size() * K, 0);
        }
        // Alg. 1 for every cell of the group.  The cells are independent
        // (Lemma 3), so the two parts run staggered: while the host cuts
        // one part, the device evaluates the other part's next candidate.
        // A single-part group overlaps nothing with its cuts, so each step's
        // successor is evaluated speculatively while the host cuts it
        // (spec_launch); propagation and refinement steps only.
        const bool spec = speculate && (P[0]->items.empty() || P[1]->items.empty());
        auto spec_next = [&](Part& Q, int hp, int step) -> lexp_status {
          const int t = step + 1;
          if (!spec || t >= K || (t >= a.kp && t < a.kp + a.kr)) return LEXP_OK;
          return spec_launch(c, Q, c->part[hp], a, t, d_pairs, s);
        };
        for (int hp = 0; hp < 2; ++hp)
          if (!P[hp]->items.empty() && K > 0) {
            Part& Q = *P[hp];
            if (!sch->batch_cycle) {
              spec_match(c, Q, c->part[hp], -1);  // step 0 evaluates its own costs
              pool_of(c).parallel_for((int)Q.items.size(), [&](int q, int) { propose_item(Q, a, q, 0); });
            }
            if ((st = enqueue_part(c, Q, c->part[hp], d_pairs, c->d_tiles.p, use_graph, &tuners[h], s))) return st;
            if ((st = spec_next(Q, hp, 0))) return st;
          }
        for (int step = 0; step < K; ++step)
          for (int hp = 0; hp < 2; ++hp) {
            if (P[hp]->items.empty()) continue;
            const int next = step + 1 < K ? step + 1 : -1;
            // (batch cycle: the candidates were drawn at the group's start)
            if ((st = finish_part(c, *P[hp], c->part[hp], a, sch->batch_cycle ? -1 : next, d_pairs, &tuners[h], s)))
              return st;
            if (next >= 0) {
              if (sch->batch_cycle)
                batch_step_items(c, *P[hp], hp == 0 ? 0 : P[0]->items.size() * K, next);
              else
                spec_match(c, *P[hp], c->part[hp], next);
              if ((st = enqueue_part(c, *P[hp], c->part[hp], d_pairs, c->d_tiles.p, use_graph, &tuners[h], s))) return st;
              if ((st = spec_next(*P[hp], hp, next))) return st;
            }
          }
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - g0).count();
        balance[h].update(ms / (double)std::max<int64_t>(1, groups[(size_t)h * 16 + k].n_px));
      }
    }
    // graph mode keeps the splits tuned in the first iteration, so each
    // group's captured graphs are replayed by the later iterations
    if (use_graph)
      for (CutBalance& b : balance) b.tune = false;
    scale *= 0.5;  // Alg. 2: the perturbation sizes halve after every iteration
    for (int p = 0; p < np; ++p) {
      RunPair& rp = pairs[p];
      if (rp.energy_trace)
        if ((st = energy_impl(rp.c, rp.labels, rp.cur_cost, &rp.energy_trace[it + 1], nullptr, nullptr, s)))
          return st;
    }
    if (time_trace) time_trace[it + 1] = now_s();
  }
  HIP_TRY(hipStreamSynchronize(s));
  for (Part& P : parts) drop_graph(P);
  for (int h = 0; h < 4; ++h) {
    c->stats.device_cut_share[h] = dev_cut && h < sch->n_levels ? balance[h].share : 0.0;
    const bool tuned = h < sch->n_levels && tuners[h].done;
    c->stats.device_cut_block[h] = tuned ? tuners[h].best.block : 0;
    c->stats.device_cut_relabel[h] = tuned ? tuners[h].best.every : 0;
  }
  for (int p = 0; p < np; ++p) HIP_TRY(hipEventRecord(pairs[p].c->staging_done, s));
  if (c->timing) collect_timing(c);
  return LEXP_OK;
}

}  // namespace

extern "C" lexp_status lexp_optimize(lexp_ctx* c, const lexp_schedule* sch, uint64_t seed, float* labels,
                                     float* cur_cost, double* energy_trace, double* time_trace, void* hip_stream) {
  if (!c || !sch || !labels || !cur_cost) return fail(LEXP_EINVAL, "null argument");
  RunPair rp;
  rp.c = c;
  rp.seed = seed;
  rp.labels = labels;
  rp.cur_cost = cur_cost;
  rp.energy_trace = energy_trace;
  return optimize_run(&rp, 1, sch, time_trace, (hipStream_t)hip_stream);
}

extern "C" lexp_status lexp_optimize_batch(int32_t n_pairs, lexp_ctx* const* ctxs, const lexp_schedule* sch,
                                           const uint64_t* seeds, float* const* labels, float* const* cur_cost,
                                           double* const* energy_traces, double* time_trace, void* hip_stream) {
  if (n_pairs < 1) return fail(LEXP_EINVAL, "n_pairs must be at least 1");
  if (!ctxs || !sch || !seeds || !labels || !cur_cost) return fail(LEXP_EINVAL, "null argument");
  std::vector<RunPair> pairs((size_t)n_pairs);
  for (int p = 0; p < n_pairs; ++p) {
    if (!ctxs[p] || !labels[p] || !cur_cost[p]) return fail(LEXP_EINVAL, "null entry for pair %d", p);
    const lexp_ctx* c0 = ctxs[0];
    const lexp_ctx* c = ctxs[p];
    if (c->r != c0->r || c->dp.nf != c0->dp.nf || c->lds_limit != c0->lds_limit)
      return fail(LEXP_EINVAL, "pair %d: every context of a batch needs the same gf_radius and neighbourhood", p);
    for (int q = 0; q < p; ++q)
      if (ctxs[q] == c || labels[q] == labels[p] || cur_cost[q] == cur_cost[p])
        return fail(LEXP_EINVAL, "pairs %d and %d share a context or an output buffer", q, p);
    pairs[p].c = ctxs[p];
    pairs[p].seed = seeds[p];
    pairs[p].labels = labels[p];
    pairs[p].cur_cost = cur_cost[p];
    pairs[p].energy_trace = energy_traces ? energy_traces[p] : nullptr;
  }
  return optimize_run(pairs.data(), n_pairs, sch, time_trace, (hipStream_t)hip_stream);
}

extern "C" {

lexp_status lexp_net_sizes(int32_t* n_weights, int32_t* n_biases) {
  int32_t nw = 0, nb = 0;
  for (int l = 0; l < lexp_net::kLayers; ++l) {
    nw += 9 * lexp_net_ch(l) * lexp_net_ch(l + 1);
    nb += lexp_net_ch(l + 1);
  }
  if (n_weights) *n_weights = nw;
  if (n_biases) *n_biases = nb;
  return LEXP_OK;
}

lexp_status lexp_net_destroy(lexp_net* net) {
  if (!net) return LEXP_OK;
  (void)hipDeviceSynchronize();
  for (void* p : {(void*)net->prm, (void*)net->grad, (void*)net->mom1, (void*)net->mom2, (void*)net->w16,
                  (void*)net->wt16, (void*)net->act[0], (void*)net->gbuf[0], (void*)net->y, (void*)net->planes,
                  (void*)net->part_w, (void*)net->part_b, (void*)net->part_loss})
    if (p) (void)hipFree(p);
  net->h_loss.release();
  delete net;
  return LEXP_OK;
}

lexp_status lexp_net_set_weights(lexp_net* net, const float* weights, const float* biases) {
  if (!net || !weights || !biases) return fail(LEXP_EINVAL, "null argument");
  std::vector<float> h(net->n_prm);
  size_t wi = 0, bi = 0;
  for (int l = 0; l < lexp_net::kLayers; ++l) {
    const size_t nw = (size_t)9 * lexp_net_ch(l) * lexp_net_ch(l + 1), nb = (size_t)lexp_net_ch(l + 1);
    for (size_t e = 0; e < nw; ++e) h[net->w_off[l] + e] = weights[wi + e];
    for (size_t e = 0; e < nb; ++e) h[net->b_off[l] + e] = biases[bi + e];
    wi += nw;
    bi += nb;
  }
  HIP_TRY(hipMemcpy(net->prm, h.data(), sizeof(float) * net->n_prm, hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(net->mom1, 0, sizeof(float) * net->n_prm));
  HIP_TRY(hipMemset(net->mom2, 0, sizeof(float) * net->n_prm));
  net->steps = 0;
  for (int l = 0; l < lexp_net::kLayers; ++l) {
    const int co = lexp_net_ch(l + 1), ci = lexp_net_ch(l), nw = 9 * co * ci;
    hipLaunchKernelGGL(lexp::k_net_w16, dim3((nw + 255) / 256), dim3(256), 0, 0, net->prm + net->w_off[l], nw, co,
                       ci, net->w16 + net->w16_off[l], net->wt16 + net->w16_off[l]);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipDeviceSynchronize());
  return LEXP_OK;
}

lexp_status lexp_net_get_weights(lexp_net* net, float* weights, float* biases) {
  if (!net || !weights || !biases) return fail(LEXP_EINVAL, "null argument");
  std::vector<float> h(net->n_prm);
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(h.data(), net->prm, sizeof(float) * net->n_prm, hipMemcpyDeviceToHost));
  size_t wi = 0, bi = 0;
  for (int l = 0; l < lexp_net::kLayers; ++l) {
    const size_t nw = (size_t)9 * lexp_net_ch(l) * lexp_net_ch(l + 1), nb = (size_t)lexp_net_ch(l + 1);
    for (size_t e = 0; e < nw; ++e) weights[wi + e] = h[net->w_off[l] + e];
    for (size_t e = 0; e < nb; ++e) biases[bi + e] = h[net->b_off[l] + e];
    wi += nw;
    bi += nb;
  }
  return LEXP_OK;
}

namespace {

// Allocates a network's buffers and sets its initial weights.
lexp_status net_init(lexp_net* net, int32_t max_width, int32_t max_height, uint64_t seed) {
  net->max_w = max_width;
  net->max_h = max_height;
  size_t off = 0, off16 = 0;
  for (int l = 0; l < lexp_net::kLayers; ++l) {
    const size_t nw = (size_t)9 * lexp_net_ch(l) * lexp_net_ch(l + 1);
    net->w_off[l] = off;
    net->b_off[l] = off + nw;
    off += nw + lexp_net_ch(l + 1);
    net->w16_off[l] = off16;
    off16 += nw;
  }
  net->n_prm = off;
  net->n_w16 = off16;
  const size_t n = (size_t)max_width * max_height;
  const size_t chunks = (size_t)lexp_net::grad_chunks(max_width, max_height);
  HIP_TRY(hipMalloc((void**)&net->prm, sizeof(float) * off));
  HIP_TRY(hipMalloc((void**)&net->grad, sizeof(float) * off));
  HIP_TRY(hipMalloc((void**)&net->mom1, sizeof(float) * off));
  HIP_TRY(hipMalloc((void**)&net->mom2, sizeof(float) * off));
  HIP_TRY(hipMalloc((void**)&net->w16, sizeof(uint16_t) * off16));
  HIP_TRY(hipMalloc((void**)&net->wt16, sizeof(uint16_t) * off16));
  size_t act = 0;
  for (int l = 0; l < lexp_net::kLayers; ++l) act += n * lexp_net_ch(l);
  HIP_TRY(hipMalloc((void**)&net->act[0], sizeof(uint16_t) * act));
  for (int l = 1; l < lexp_net::kLayers; ++l) net->act[l] = net->act[l - 1] + n * lexp_net_ch(l - 1);
  HIP_TRY(hipMalloc((void**)&net->gbuf[0], sizeof(uint16_t) * n * 32 * 2));
  net->gbuf[1] = net->gbuf[0] + n * 32;
  HIP_TRY(hipMalloc((void**)&net->y, sizeof(float) * n * 16));
  HIP_TRY(hipMalloc((void**)&net->planes, sizeof(float4) * n));
  HIP_TRY(hipMalloc((void**)&net->part_w, sizeof(float) * chunks * 9 * 32 * 32));
  HIP_TRY(hipMalloc((void**)&net->part_b, sizeof(float) * chunks * 32));
  HIP_TRY(hipMalloc((void**)&net->part_loss, sizeof(double) * ((n + 255) / 256)));
  HIP_TRY(net->h_loss.ensure((n + 255) / 256));
  // He-uniform weights from the counter-based generator, zero biases
  std::vector<float> w, b;
  for (int l = 0; l < lexp_net::kLayers; ++l) {
    const int ci = lexp_net_ch(l), co = lexp_net_ch(l + 1);
    const double lim = std::sqrt(6.0 / (9.0 * ci));
    for (int e = 0; e < 9 * co * ci; ++e) {
      const uint64_t key[3] = {5, (uint64_t)l, (uint64_t)e};
      w.push_back((float)((2.0 * lexp::u01_open1(lexp::key_chain(seed, key, 3)) - 1.0) * lim));
    }
    for (int e = 0; e < co; ++e) b.push_back(0.f);
  }
  return lexp_net_set_weights(net, w.data(), b.data());
}

}  // namespace

lexp_status lexp_net_create(int32_t max_width, int32_t max_height, uint64_t seed, lexp_net** out) {
  if (!out || max_width <= 0 || max_height <= 0 || (int64_t)max_width * max_height > (1ll << 26))
    return fail(LEXP_EINVAL, "bad argument");
  lexp_net* net = new lexp_net();
  const lexp_status st = net_init(net, max_width, max_height, seed);
  if (st) {
    (void)lexp_net_destroy(net);  // frees whatever was allocated (keeps the error message)
    return st;
  }
  *out = net;
  return LEXP_OK;
}

lexp_status lexp_net_forward(lexp_net* net, lexp_ctx* c, const float* labels, float* out, void* hip_stream) {
  if (!net || !c || !labels || !out) return fail(LEXP_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)hip_stream;
  lexp_status st = net_forward(net, c, labels, s);
  if (st) return st;
  HIP_TRY(hipMemcpyAsync(out, net->y, sizeof(float) * 16 * c->W * c->H, hipMemcpyDeviceToDevice, s));
  return LEXP_OK;
}

lexp_status lexp_net_train_step(lexp_net* net, lexp_ctx* c, const float* labels, const float* target, float lr,
                                double* loss, void* hip_stream) {
  if (!net || !c || !labels || !target) return fail(LEXP_EINVAL, "null argument");
  if (!(lr > 0.f)) return fail(LEXP_EINVAL, "learning rate must be positive");
  hipStream_t s = (hipStream_t)hip_stream;
  lexp_status st = net_forward(net, c, labels, s);
  if (st) return st;
  const int W = c->W, H = c->H, n = W * H;
  const int nb = (n + 255) / 256;
  uint16_t* g = net->gbuf[0];
  hipLaunchKernelGGL(lexp::k_net_loss, dim3(nb), dim3(256), 0, s, net->y, (const float4*)target, W, H,
                     (double)c->prm.disp_max, g, net->part_loss);
  // input gradients: workgroups as in the forward pass
  const int run = 16 * lexp::kConvSegs;
  const dim3 grid(((W + run - 1) / run) * ((H + lexp::kConvRows - 1) / lexp::kConvRows)), block(lexp::kConvThreads);
  // backward through the layers: weight gradients, then the gradient of the
  // layer's input (through the ReLU that produced it)
  for (int l = lexp_net::kLayers - 1; l >= 0; --l) {
    uint16_t* gp = net->gbuf[(lexp_net::kLayers - l) & 1];
    const uint16_t* wt = net->wt16 + net->w16_off[l];
    if (l == lexp_net::kLayers - 1) {
      net_weight_grad<32, 16>(net, l, g, W, H, s);
      hipLaunchKernelGGL((lexp::k_conv_bwd_x<32, 16>), grid, block, 0, s, g, wt, net->act[l], W, H, gp);
    } else if (l > 0) {
      net_weight_grad<32, 32>(net, l, g, W, H, s);
      hipLaunchKernelGGL((lexp::k_conv_bwd_x<32, 32>), grid, block, 0, s, g, wt, net->act[l], W, H, gp);
    } else {
      net_weight_grad<16, 32>(net, l, g, W, H, s);
    }
    g = gp;
  }
  net->steps += 1;
  const float c1 = (float)(1.0 - std::pow(0.9, net->steps)), c2 = (float)(1.0 - std::pow(0.999, net->steps));
  for (int l = 0; l < lexp_net::kLayers; ++l) {
    const int co = lexp_net_ch(l + 1), ci = lexp_net_ch(l), nw = 9 * co * ci;
    hipLaunchKernelGGL(lexp::k_net_adam, dim3((nw + co + 255) / 256), dim3(256), 0, s, net->prm + net->w_off[l],
                       net->grad + net->w_off[l], net->mom1 + net->w_off[l], net->mom2 + net->w_off[l], nw + co, nw,
                       co, ci, lr, c1, c2, net->w16 + net->w16_off[l], net->wt16 + net->w16_off[l]);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(net->h_loss.p, net->part_loss, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double sum = 0.0;
  for (int b = 0; b < nb; ++b) sum += net->h_loss.p[b];
  if (loss) *loss = sum / (double)n;
  return LEXP_OK;
}

lexp_status lexp_net_get_grads(lexp_net* net, float* weights, float* biases) {
  if (!net || !weights || !biases) return fail(LEXP_EINVAL, "null argument");
  std::vector<float> h(net->n_prm);
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(h.data(), net->grad, sizeof(float) * net->n_prm, hipMemcpyDeviceToHost));
  size_t wi = 0, bi = 0;
  for (int l = 0; l < lexp_net::kLayers; ++l) {
    const size_t nw = (size_t)9 * lexp_net_ch(l) * lexp_net_ch(l + 1), nb = (size_t)lexp_net_ch(l + 1);
    for (size_t e = 0; e < nw; ++e) weights[wi + e] = h[net->w_off[l] + e];
    for (size_t e = 0; e < nb; ++e) biases[bi + e] = h[net->b_off[l] + e];
    wi += nw;
    bi += nb;
  }
  return LEXP_OK;
}

lexp_status lexp_set_net(lexp_ctx* c, lexp_net* net) {
  if (!c) return fail(LEXP_EINVAL, "null context");
  c->net = net;
  return LEXP_OK;
}

lexp_status lexp_set_timing(lexp_ctx* c, int32_t enable) {
  if (!c) return fail(LEXP_EINVAL, "null context");
  if (enable < 0) return fail(LEXP_EINVAL, "timing period %d < 0", enable);
  c->timing = enable != 0;
  c->time_every = enable > 0 ? enable : 1;
  c->time_seq = 0;
  return LEXP_OK;
}

lexp_status lexp_get_stats(lexp_ctx* c, lexp_stats* out) {
  if (!c || !out) return fail(LEXP_EINVAL, "null argument");
  collect_timing(c);
  *out = c->stats;
  return LEXP_OK;
}

lexp_status lexp_reset_stats(lexp_ctx* c) {
  if (!c) return fail(LEXP_EINVAL, "null context");
  collect_timing(c);
  c->stats = lexp_stats{};
  return LEXP_OK;
}

lexp_status lexp_debug_guide(lexp_ctx* c, float* left4, float* right4, float* guide, double* weights,
                             void* hip_stream) {
  if (!c) return fail(LEXP_EINVAL, "null context");
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t n = (size_t)c->W * c->H;
  if (left4) HIP_TRY(hipMemcpyAsync(left4, c->left4, n * 16, hipMemcpyDeviceToDevice, s));
  if (right4) HIP_TRY(hipMemcpyAsync(right4, c->right4, n * 16, hipMemcpyDeviceToDevice, s));
  if (guide) {
    hipLaunchKernelGGL(lexp::k_guide_planes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c->guide, guide,
                       c->W, c->H);
    HIP_TRY(hipGetLastError());
  }
  if (weights) HIP_TRY(hipMemcpyAsync(weights, c->wts, n * 32, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return LEXP_OK;
}

// ---- host-side pieces ------------------------------------------------------
lexp_status lexp_solve_binary_device(lexp_ctx* c, int32_t n, const int32_t* dims, const int32_t* terms, uint8_t* x,
                                     int32_t* status, void* hip_stream) {
  if (!c || n < 0) return fail(LEXP_EINVAL, "bad argument");
  if (n == 0) return LEXP_OK;
  if (!dims || !terms || !x || !status) return fail(LEXP_EINVAL, "null argument");
  // problems whose arrays do not fit in LDS get status 0 and are not run
  std::vector<Item> items;
  std::vector<int> run;
  int64_t tot = 0;
  int max_px = 1;
  for (int i = 0; i < n; ++i) {
    const int w = dims[2 * i], h = dims[2 * i + 1];
    if (w < 0 || h < 0 || (int64_t)w * h > (1 << 24)) return fail(LEXP_EINVAL, "bad grid size of problem %d", i);
    status[i] = 0;
    if (cut_fits(c, (int64_t)w * h)) {
      Item it{};
      it.rw = w; it.rh = h; it.aux_off = tot;
      items.push_back(it);
      run.push_back(i);
      max_px = std::max(max_px, w * h);
    }
    tot += (int64_t)w * h;
  }
  const int64_t lim = (int64_t)1 << 30;
  for (int64_t q = 0; q < tot; ++q) {
    if (terms[q * 5] > lim || terms[q * 5] < -lim) return fail(LEXP_EINVAL, "unary term exceeds 2^30 in magnitude");
    for (int d = 0; d < 4; ++d)
      if (terms[q * 5 + 1 + d] < 0 || terms[q * 5 + 1 + d] > lim)
        return fail(LEXP_EINVAL, "pairwise weight outside [0, 2^30]");
  }
  const int m = (int)items.size();
  if (m == 0 || tot == 0) {
    for (int i : run) status[i] = 1;
    return LEXP_OK;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  lexp_status st = wait_staging(c);
  if (st) return st;
  HIP_TRY(c->d_items.ensure((size_t)m));
  HIP_TRY(c->d_terms.ensure((size_t)tot * 5));
  HIP_TRY(c->d_x.ensure((size_t)tot));
  HIP_TRY(c->d_status.ensure((size_t)m));
  HIP_TRY(c->h_status.ensure((size_t)m));
  HIP_TRY(hipMemcpyAsync(c->d_items.p, items.data(), sizeof(Item) * m, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(c->d_terms.p, terms, sizeof(int) * 5 * tot, hipMemcpyHostToDevice, s));
  if ((st = launch_cut(c, c->d_items.p, m, c->d_terms.p, c->d_x.p, c->d_status.p, max_px, s))) return st;
  HIP_TRY(hipMemcpyAsync(x, c->d_x.p, (size_t)tot, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(c->h_status.p, c->d_status.p, sizeof(int) * m, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int k = 0; k < m; ++k) status[run[k]] = c->h_status.p[k];
  HIP_TRY(hipEventRecord(c->staging_done, s));
  return LEXP_OK;
}

lexp_status lexp_solve_binary(int32_t w, int32_t h, int32_t neighbours, const int64_t* U, const int64_t* w4,
                              uint8_t* x) {
  if (w < 0 || h < 0 || (neighbours != 4 && neighbours != 8)) return fail(LEXP_EINVAL, "bad grid");
  if ((int64_t)w * h > 0 && (!U || !w4 || !x)) return fail(LEXP_EINVAL, "null argument");
  const int64_t lim = (int64_t)1 << 30;
  for (int64_t i = 0; i < (int64_t)w * h * 4; ++i) {
    if (w4[i] < 0) return fail(LEXP_EINVAL, "negative pairwise weight (not submodular)");
    if (w4[i] > lim) return fail(LEXP_EINVAL, "pairwise weight exceeds 2^30");
  }
  for (int64_t i = 0; i < (int64_t)w * h; ++i)
    if (U[i] > lim || U[i] < -lim) return fail(LEXP_EINVAL, "unary term exceeds 2^30 in magnitude");
  if ((int64_t)w * h == 0) return LEXP_OK;
  lexp::BKSolver bk;
  bk.load<int64_t>(w, h, neighbours == 8 ? 4 : 2, U, 1, w4, 4);
  bk.solve(x);
  return LEXP_OK;
}

uint64_t lexp_rng_key(uint64_t seed, const uint64_t* fields, int32_t n_fields) {
  return lexp::key_chain(seed, fields, n_fields > 0 && fields ? n_fields : 0);
}

lexp_status lexp_init_labels_host(int32_t width, int32_t height, double disp_max, uint64_t seed, float* labels) {
  if (width <= 0 || height <= 0 || !labels) return fail(LEXP_EINVAL, "bad argument");
  for (int v = 0; v < height; ++v)
    for (int u = 0; u < width; ++u) lexp::init_label(width, u, v, disp_max, seed, labels + ((size_t)v * width + u) * 3);
  return LEXP_OK;
}

lexp_status lexp_propose(int32_t width, int32_t height, const float* labels, uint64_t seed, int32_t iteration,
                         int32_t level, int32_t cell, int32_t ci, int32_t cj, int32_t step, int32_t k_prop,
                         int32_t k_rans, double r_d, double r_n, lexp_plane* out) {
  if (width <= 0 || height <= 0 || !labels || !out || cell < 1) return fail(LEXP_EINVAL, "bad argument");
  if (ci < 0 || cj < 0 || ci * cell >= width || cj * cell >= height) return fail(LEXP_EINVAL, "cell outside the image");
  float a[3];
  if (k_prop < 0 || k_rans < 0) return fail(LEXP_EINVAL, "negative proposer count");
  lexp::propose(width, height, labels, 3, seed, iteration, level, cell, ci, cj, step, k_prop, k_rans, r_d, r_n, a);
  out->a = a[0];
  out->b = a[1];
  out->c = a[2];
  return LEXP_OK;
}

}  // extern "C"
