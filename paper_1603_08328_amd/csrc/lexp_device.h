// Types shared by the device kernels and their host-side launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lexp {

constexpr int kWaves = 16;              // waves per fused-cost workgroup (1024 threads)
constexpr int kChunk = kWaves;          // rows per pipeline step of the fused cost kernel (one per wave)
constexpr double kQuantum = 1048576.0;  // 2^20: binary-problem terms are ceil(x * 2^20)

// forward neighbour offsets: each unordered pair of the 8-neighbourhood once
__device__ constexpr int kFwdDU[4] = {1, 0, 1, -1};
__device__ constexpr int kFwdDV[4] = {0, 1, 1, 1};

enum TileFlags : int { kFirstCol = 1, kLastCol = 2, kFirstRow = 4, kLastRow = 8 };

struct DevParams {
  int W, H, r, nf;
  float oma, al, tc, tg, rho_max;  // 1-alpha, alpha, tau_col, tau_grad, rho_max (FP32 data term)
  double lam, tau_dis, w_floor;    // smoothness term (FP64)
};

// What the kernels read of one stereo pair: sizes and parameters, packed
// images, guide statistics, contrast weights, and the label field and current
// costs the expansion kernels update.  Kernels index a table of these by the
// item's pair, so one launch can cover many pairs of different sizes.
struct PairDev {
  DevParams P;
  const float4* left4;
  const float4* left4T;
  const float4* right4;
  const float* guide;
  const double* wts;
  float4* labels;
  float* cur_cost;
};

// One (region, label) item: pair, clipped region, candidate label, output offset.
struct Item {
  int ru0, rv0, rw, rh;
  float a, b, c;
  int pair;           // index into the launch's pair table
  long long out_off;  // first phi value of the item (caller layout)
  long long aux_off;  // first pixel of the item in the graph-term / cut buffers
};

// One workgroup's sub-rectangle of an item's region.
struct Tile {
  int item;
  int tu0, tv0, tu1, tv1;
  int flags;
  int pad0, pad1;
};

// LDS bytes of one fused-cost workgroup for the given capacities.
// Rows held by the fused kernel's rings: the 2r+1 rows of a vertical window,
// plus the rows one stage may run ahead of the next (two pipeline steps).
inline int unary_ring_rows(int r) { return 2 * r + 1 + 2 * kChunk; }

// LDS of one fused-cost workgroup: rings (R+ and R widths, each with one more
// row that stays zero), two buffers of coefficient rows, one scan row per wave
// and the vertical-sum carries (float4 each); FP32 counts of the scan rows and
// carries; byte counts of the ring and coefficient entries.
inline size_t unary_lds_bytes(int ring, int wp_cap, int tw_cap, int ws_cap) {
  const size_t rows = (size_t)ring + 1;
  const size_t f4 = rows * wp_cap + (size_t)2 * kChunk * wp_cap + rows * tw_cap + (size_t)kWaves * ws_cap +
                    (size_t)wp_cap + (size_t)tw_cap;
  const size_t f1 = (size_t)kWaves * ws_cap + (size_t)wp_cap + (size_t)tw_cap;
  const size_t b1 = rows * wp_cap + (size_t)2 * kChunk * wp_cap + rows * tw_cap;
  return f4 * 16 + f1 * 4 + b1;
}

// Widths the fused kernel's register layout supports: a pair of M rows in up
// to four 64-lane segments, R+ and R rows in up to two.
constexpr int kMaxWM = 128;
constexpr int kMaxWP = 128;
constexpr int kMaxTW = 128;

template <int MODE, int NSEG, int NC>
__global__ void k_unary(const PairDev* pairs, const Item* items, const Tile* tiles, int n_tiles,
                        const float4* label_field, float* out, int ring, int wp_cap, int tw_cap, int ws_cap,
                        int pair_hint, int direct, int fill2);
__global__ void k_pack(const float* img, float4* out, float4* outT, int W, int H, int mirror);
__global__ void k_guide_h(const float4* left4, double* tmp, int W, int H, int r);
__global__ void k_guide_v(const double* tmp, float* guide, int W, int H, int r, double eps);
__global__ void k_guide_planes(const float* guide, float* planes, int W, int H);
__global__ void k_weights(const float* img, double* wts, int W, int H, double gamma, int mirror);
__global__ void k_view_labels(const float4* in, float4* out, int W, int H, int mirror);
__global__ void k_pp_check(const float4* labels_left, const float4* labels_right, int W, int H, double* disp,
                           uint8_t* ok);
__global__ void k_pp_fill(const float4* labels_left, const double* disp, const uint8_t* ok, int W, int H,
                          int* next_ok, double* fill);
__global__ void k_pp_median(const float4* left4, const double* disp, const double* fill, const uint8_t* ok, int W,
                            int H, double gamma, float* out, uint8_t* invalid);
__global__ void k_graph_terms(const PairDev* pairs, const Item* items, const float* phi_alpha, int* terms,
                              int* flag);
__global__ void k_apply(const PairDev* pairs, const Item* items, const uint8_t* x, const float* phi_alpha);
__global__ void k_energy(DevParams P, const float4* labels, const float* cur_cost, const double* wts,
                         double* partial);
__global__ void k_energy_total(const double* partial, int n_blocks, double* out);
struct FullLayout;
struct CompactLayout;
template <class Layout, int BLOCK>
__global__ void k_cut_lds(const Item* items, const int* terms, int nf, uint8_t* x, int* status, int max_nodes,
                          int round_factor, int relabel_every);
// device max-flow arrays per node in LDS: all eight residuals and 64-bit
// excess, or forward residuals only with 32-bit excess and 16-bit heights
constexpr int kCutBytesFull = 52;
constexpr int kCutBytesCompact = 28;
// learned proposal network (lexp_net.hip).  The forward and input-gradient
// convolutions run a workgroup of kConvRows waves per kConvRows rows of a run
// of 16 kConvSegs columns (one row per wave).
constexpr int kConvSegs = 2;
constexpr int kConvRows = 8;
constexpr int kConvThreads = 64 * kConvRows;
// The weight gradients take a layer's pixels in chunks of kWgRows rows by
// kWgTiles tiles of 32 columns (one partial sum per chunk).
constexpr int kWgRows = 4;
constexpr int kWgTiles = 8;
constexpr int kWgThreads = 1024;  // 16 waves: the staging of a tile spread over more lanes
__global__ void k_net_input(const float4* left4, const float4* right4, const float4* labels, int W, int H,
                            double disp_max, uint16_t* x0);
template <int CI, int CO, bool LAST>
__global__ void k_conv_fwd(const uint16_t* x, const uint16_t* w16, const float* bias, int W, int H, uint16_t* xo,
                           float* yo);
template <int CI, int CO>
__global__ void k_conv_bwd_x(const uint16_t* g, const uint16_t* wt16, const uint16_t* x, int W, int H,
                             uint16_t* gp);
template <int CI, int CO>
__global__ void k_conv_bwd_w(const uint16_t* g, const uint16_t* x, int W, int H, float* part_w, float* part_b);
__global__ void k_sum_chunks(const float* part, int n_chunks, int n, float* out);
__global__ void k_net_loss(const float* y, const float4* target, int W, int H, double disp_max, uint16_t* g,
                           double* part);
__global__ void k_net_adam(float* prm, const float* grad, float* m1, float* m2, int n, int n_w, int co, int ci,
                           float lr, float c1, float c2, uint16_t* w16, uint16_t* wt16);
__global__ void k_net_w16(const float* prm, int n_w, int co, int ci, uint16_t* w16, uint16_t* wt16);
__global__ void k_net_planes(const float* y, int W, int H, double disp_max, float4* planes);
__global__ void k_pair1(DevParams P, const double* wts, int pu, int pv, int qu, int qv, float4 fp, float4 fq,
                        double* out);

}  // namespace lexp
