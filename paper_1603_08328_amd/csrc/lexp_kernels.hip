// Device kernels of the local-expansion-move hot path for CDNA4 (gfx950).
//
//   k_pack / k_guide_h / k_guide_v / k_weights : label-independent set-up
//   k_unary<MODE>                              : fused raw cost (Eqs. 8, 9, 18)
//                                                + guided-filter aggregation
//                                                (Eq. 7 box form, Eq. 19)
//   k_graph_terms                              : binary problem of one local
//                                                expansion (Eq. 13, Lemma 2)
//   k_apply, k_energy, k_pair1                 : label update, Eq. (5), Eq. (10)
// (the device max-flow of the binary problems is in lexp_cut.hip)
//
// Built with -ffp-contract=off: products and sums are rounded as written and
// fused multiply-adds appear only where fmaf() is called explicitly.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lexp_device.h"

namespace lexp {

// ---------------------------------------------------------------------------
// Set-up
// ---------------------------------------------------------------------------
__device__ inline float gray_of(const float* px) {
  return 0.299f * px[0] + 0.587f * px[1] + 0.114f * px[2];
}

// (R, G, B, x-gradient of the gray value by [-0.5 0 0.5], replicated borders),
// row-major; a column-major copy too where outT is given.  mirror != 0 packs
// the horizontally mirrored image (column u from column W-1-u), its gradient
// taken on the mirrored image.
__global__ void k_pack(const float* __restrict__ img, float4* __restrict__ out, float4* __restrict__ outT, int W,
                       int H, int mirror) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W * H) return;
  const int u = i % W, v = i / W;
  const int ul = u > 0 ? u - 1 : 0, ur = u < W - 1 ? u + 1 : W - 1;
  auto src = [&](int x) { return mirror ? W - 1 - x : x; };
  const float* row = img + (size_t)v * W * 3;
  const float gx = 0.5f * (gray_of(row + src(ur) * 3) - gray_of(row + src(ul) * 3));
  const int us = src(u);
  const float4 val = make_float4(row[us * 3 + 0], row[us * 3 + 1], row[us * 3 + 2], gx);
  out[i] = val;
  if (outT) outT[(size_t)u * H + v] = val;
}

// Horizontal window sums of I = I_L/255 and I I^T (FP64).
__global__ void k_guide_h(const float4* __restrict__ left4, double* __restrict__ tmp, int W, int H, int r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W * H) return;
  const int u = i % W, v = i / W;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int x0 = u - r > 0 ? u - r : 0, x1 = u + r < W - 1 ? u + r : W - 1;
  for (int x = x0; x <= x1; ++x) {
    const float4 p = left4[(size_t)v * W + x];
    const double I0 = (double)p.x / 255.0, I1 = (double)p.y / 255.0, I2 = (double)p.z / 255.0;
    acc[0] += I0; acc[1] += I1; acc[2] += I2;
    acc[3] += I0 * I0; acc[4] += I0 * I1; acc[5] += I0 * I2;
    acc[6] += I1 * I1; acc[7] += I1 * I2; acc[8] += I2 * I2;
  }
  for (int q = 0; q < 9; ++q) tmp[(size_t)q * W * H + i] = acc[q];
}

// Vertical sums -> mean mu_k and (Sigma_k + eU)^-1 by the adjugate.  Stored
// column-major (index u*H + v) as float4 (mu0, mu1, mu2, i00), float4 (i01,
// i02, i11, i12) and float i22, for the fused kernel, whose lanes read runs of
// consecutive rows of one column.
__global__ void k_guide_v(const double* __restrict__ tmp, float* __restrict__ guide, int W, int H, int r,
                          double eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W * H) return;
  const int u = i % W, v = i / W;
  const int y0 = v - r > 0 ? v - r : 0, y1 = v + r < H - 1 ? v + r : H - 1;
  const int x0 = u - r > 0 ? u - r : 0, x1 = u + r < W - 1 ? u + r : W - 1;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int y = y0; y <= y1; ++y)
    for (int q = 0; q < 9; ++q) acc[q] += tmp[(size_t)q * W * H + (size_t)y * W + u];
  const double n = (double)(x1 - x0 + 1) * (double)(y1 - y0 + 1);
  const double m0 = acc[0] / n, m1 = acc[1] / n, m2 = acc[2] / n;
  const double a00 = acc[3] / n - m0 * m0 + eps, a01 = acc[4] / n - m0 * m1, a02 = acc[5] / n - m0 * m2;
  const double a11 = acc[6] / n - m1 * m1 + eps, a12 = acc[7] / n - m1 * m2;
  const double a22 = acc[8] / n - m2 * m2 + eps;
  const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
  const double c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
  const double det = a00 * c00 + a01 * c01 + a02 * c02;
  const double id = 1.0 / det;
  const size_t hw = (size_t)W * H, t = (size_t)u * H + v;
  float4* g0 = reinterpret_cast<float4*>(guide);
  float4* g1 = g0 + hw;
  float* g2 = reinterpret_cast<float*>(g1 + hw);
  g0[t] = make_float4((float)m0, (float)m1, (float)m2, (float)(c00 * id));
  g1[t] = make_float4((float)(c01 * id), (float)(c02 * id), (float)(c11 * id), (float)(c12 * id));
  g2[t] = (float)(c22 * id);
}

// The guide statistics as nine row-major planes (for inspection).
__global__ void k_guide_planes(const float* __restrict__ guide, float* __restrict__ planes, int W, int H) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W * H) return;
  const int u = i % W, v = i / W;
  const size_t hw = (size_t)W * H, t = (size_t)u * H + v;
  const float4* g0 = reinterpret_cast<const float4*>(guide);
  const float4 a = g0[t], b = g0[hw + t];
  const float c = reinterpret_cast<const float*>(g0 + 2 * hw)[t];
  const float vals[9] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c};
  for (int q = 0; q < 9; ++q) planes[q * hw + i] = vals[q];
}

// Contrast weights w_pq = exp(-||I(p) - I(q)||_1 / gamma), Eq. (11), of the
// view's own image I, for the forward neighbours q = p + (1,0), (0,1), (1,1),
// (-1,1); 0 outside.  mirror != 0: I is the mirrored image.
__global__ void k_weights(const float* __restrict__ img, double* __restrict__ wts, int W, int H, double gamma,
                          int mirror) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W * H) return;
  const int u = i % W, v = i / W;
  auto px = [&](int x, int y) { return img + ((size_t)y * W + (mirror ? W - 1 - x : x)) * 3; };
  const float* a = px(u, v);
  for (int d = 0; d < 4; ++d) {
    const int qu = u + kFwdDU[d], qv = v + kFwdDV[d];
    double w = 0.0;
    if (qu >= 0 && qu < W && qv < H) {
      const float* b = px(qu, qv);
      double s = fabs((double)a[0] - (double)b[0]) + fabs((double)a[1] - (double)b[1]);
      s = s + fabs((double)a[2] - (double)b[2]);
      w = exp(-s / gamma);
    }
    wts[(size_t)i * 4 + d] = w;
  }
}

// ---------------------------------------------------------------------------
// Fused unary cost.  One workgroup (16 wave64) per tile: a sub-rectangle of
// one item's region.  Rows stream top to bottom through four stages; in every
// pipeline step each stage handles up to kChunk rows and consumes what the
// previous stage produced in the previous step, so one workgroup barrier per
// step suffices:
//   A  (waves 0-7, two M rows each) raw cost rho' = rho - rho_max and rho' * I
//      over the pair's pixels, then an in-place prefix along each row (serial
//      runs per lane, DPP scan over 32 lanes), then horizontal window sums at
//      the R+ columns -> ring1
//   C  (waves 8-15, 4 columns x 16 rows per column group) vertical window
//      sums (carried sum of the previous row, plus the row that entered,
//      minus the row that left) -> means over W'_k
//      -> a_k = (Sigma_k + eU)^-1 (mean(I rho) - mu mean(rho)), b_k
//   E  (waves 0-7, two coefficient rows each) in-place prefix of the rows,
//      window sums at the R columns -> ring3
//   G  (waves 8-15, as C) vertical window sums -> phi = abar^T I_p + bbar + rho_max
// Global operands of a step (image taps, guide statistics, I_p) are loaded
// one step ahead with clamped, unconditional loads; barriers wait on LDS
// traffic only.  A fifth channel counts samples with rho' != 0 exactly (a
// byte in the rings): where a window holds none, the sums are zero exactly,
// so a fully truncated or out-of-view patch costs exactly rho_max.
// ---------------------------------------------------------------------------
__device__ inline float4 f4add(float4 a, float4 b) { return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
__device__ inline float4 f4sub(float4 a, float4 b) { return make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w); }

// Workgroup barrier that orders LDS accesses only: outstanding global loads
// are not waited for, so prefetches stay in flight across it.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <int CTRL, int ROWMASK>
__device__ inline float dpp_add(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xf, false));
}

// Inclusive prefix sums over lanes 0-31 and over lanes 32-63: shifts by 1, 2,
// 4, 8 inside each row of 16 lanes, then lane 15 of rows 0 and 2 added to rows
// 1 and 3.
__device__ inline float half_scan(float v) {
  v = dpp_add<0x111, 0xf>(v);
  v = dpp_add<0x112, 0xf>(v);
  v = dpp_add<0x114, 0xf>(v);
  v = dpp_add<0x118, 0xf>(v);
  v = dpp_add<0x142, 0xa>(v);
  return v;
}

// Inclusive prefix sum inside each row of 16 lanes.
__device__ inline float row_scan16(float v) {
  v = dpp_add<0x111, 0xf>(v);
  v = dpp_add<0x112, 0xf>(v);
  v = dpp_add<0x114, 0xf>(v);
  v = dpp_add<0x118, 0xf>(v);
  return v;
}

// Value of lane 15 of this lane's row of 16 lanes.
__device__ inline float row_last(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute((lane | 15) << 2, __float_as_int(v)));
}

// Ring slot of a row, given the slot of a base row no more than `ring` rows earlier.
__device__ inline int slot_of(int y, int base_row, int base_slot, int ring) {
  const int s = base_slot + (y - base_row);
  return s >= ring ? s - ring : s;
}

// A wave's pair of M rows, flattened: segment s, lane l holds pixel
// t = 64 s + l of the two rows laid end to end (row t / wM, column t % wM).
// What depends on the tile only is set once per lane.
template <int NSEG>
struct RowLanes {
  float uf[NSEG];  // column u of the pixel
  int h[NSEG];     // 1 on the pair's second row
  int xl16[NSEG];  // byte offset of column min(u, W-1) within an image row
  int lds[NSEG];   // index of the pixel in the wave's scan rows; -1 past the M columns
};

template <int NSEG>
__device__ inline void row_lanes(RowLanes<NSEG>& rl, int w2, int xm0, int wM, int W, int ws_cap, int lane) {
#pragma unroll
  for (int s = 0; s < NSEG; ++s) {
    const int t = s * 64 + lane;
    const int h = t >= wM ? 1 : 0;
    const int xi = t - h * wM;
    const int x = xm0 + xi;
    rl.uf[s] = (float)x;
    rl.h[s] = h;
    rl.xl16[s] = (x < W - 1 ? x : W - 1) * 16;
    rl.lds[s] = xi < wM ? (w2 + h) * ws_cap + xi : -1;
  }
}

template <int NSEG>
struct RowTaps {  // prefetched operands of the pair, per lane
  float4 L[NSEG], R0[NSEG], R1[NSEG];
  float t[NSEG];
  bool ok[NSEG];
};

// Loads of a row pair starting at row y: always issued (rows clamped into the
// image, out-of-view samples read column 0), so the number of loads in flight
// is known to the compiler.  Addresses are 32-bit byte offsets from the image
// bases (images below 2^27 pixels).  The second tap is the pixel after the
// first: where the first is a row's last pixel its weight is exactly zero and
// the read lands on the next row or on the zeroed pixel after the image.
// Segments [S0, S1) only: a step issues its loads in a few such runs between
// its LDS phases, so that waiting for the memory pipeline to take them
// overlaps other work.
template <int NSEG, int S0 = 0, int S1 = NSEG>
__device__ inline void load_rows2(RowTaps<NSEG>& tp, const RowLanes<NSEG>& rl, int y, int W, int H, float la,
                                  float lb, float lc, const char* __restrict__ left_b,
                                  const char* __restrict__ right_b) {
  const float fW1 = (float)(W - 1);
  const int W16 = W * 16;
  // row offsets as scalars (kept from being folded into a per-lane product)
  const int ro0 = __builtin_amdgcn_readfirstlane((y < H - 1 ? y : H - 1) * W16);
  const int ro1 = __builtin_amdgcn_readfirstlane((y + 1 < H - 1 ? y + 1 : H - 1) * W16);
  const float s0 = fmaf(lb, (float)y, lc), s1 = fmaf(lb, (float)(y + 1), lc);
#pragma unroll
  for (int s = S0; s < S1; ++s) {
    const bool h = rl.h[s] != 0;
    const int ro = h ? ro1 : ro0;
    const float d = fmaf(la, rl.uf[s], h ? s1 : s0);
    const float xs = rl.uf[s] - d;
    const bool ok = rl.lds[s] >= 0 && xs >= 0.f && xs <= fW1;
    const float xc = ok ? xs : 0.f;
    const float xf = floorf(xc);
    const unsigned a = (unsigned)((int)xf * 16 + ro);
    tp.R0[s] = *reinterpret_cast<const float4*>(right_b + a);
    tp.R1[s] = *reinterpret_cast<const float4*>(right_b + a + 16);
    tp.L[s] = *reinterpret_cast<const float4*>(left_b + (unsigned)(rl.xl16[s] + ro));
    tp.t[s] = xc - xf;
    tp.ok[s] = ok;
  }
}

// Stage A of the fused kernel, in three phases over a wave's pair of M rows
// (scan rows w2 and w2+1 of a scan buffer):
// raw cost rho' and rho' * I of the pair's pixels into the scan rows ...
template <int NSEG>
__device__ inline void a_raw(const DevParams& P, const RowTaps<NSEG>& taps, const RowLanes<NSEG>& rl,
                             float4* scanv, float* scanc) {
  const float inv255 = 1.0f / 255.0f;
#pragma unroll
  for (int s = 0; s < NSEG; ++s) {
    // out-of-view samples cost rho_max: rho' = 0
    const float tt = taps.t[s];
    const float4 L = taps.L[s], R0 = taps.R0[s], R1 = taps.R1[s];
    const float col = fabsf(L.x - fmaf(tt, R1.x - R0.x, R0.x)) + fabsf(L.y - fmaf(tt, R1.y - R0.y, R0.y)) +
                      fabsf(L.z - fmaf(tt, R1.z - R0.z, R0.z));
    const float gr = fabsf(L.w - fmaf(tt, R1.w - R0.w, R0.w));
    const float rp0 = P.oma * (fminf(col, P.tc) - P.tc) + P.al * (fminf(gr, P.tg) - P.tg);
    const float rp = taps.ok[s] ? rp0 : 0.f;
    const float q = rp * inv255;
    const float4 val = make_float4(rp, q * L.x, q * L.y, q * L.z);
    const float nz = rp != 0.f ? 1.f : 0.f;
    const int o = rl.lds[s];
    if (o >= 0) {
      scanv[o] = val;
      scanc[o] = nz;
    }
  }
}

// ... an in-place prefix along each scan row: lane (h, l) runs over columns
// run*l .. run*l + run-1 of row w2+h (serial prefix of the run, scan of the
// run totals over the 32 lanes of the row, offset added).  run = ceil(wM/32)
// is the tile's own (at most NSEG): the order of the sums, and so their
// rounding, depends on the tile alone, not on the instance a launch picks for
// its widest tile.  Entries past the run add +0, which changes no sum ...
template <int NSEG>
__device__ inline void a_prefix(float4* scanv, float* scanc, int w2, int ws_cap, int wM, int run, int lane) {
  const int h = lane >> 5, l = lane & 31;
  float4* rv = scanv + (size_t)(w2 + h) * ws_cap;
  float* rc = scanc + (size_t)(w2 + h) * ws_cap;
  float4 v[NSEG];
  float n[NSEG];
#pragma unroll
  for (int i = 0; i < NSEG; ++i) {
    const int c = l * run + i;
    v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    n[i] = 0.f;
    if (i < run && c < wM) { v[i] = rv[c]; n[i] = rc[c]; }
  }
#pragma unroll
  for (int i = 1; i < NSEG; ++i) { v[i] = f4add(v[i - 1], v[i]); n[i] = n[i - 1] + n[i]; }
  const float4 tot = v[NSEG - 1];
  const float nt = n[NSEG - 1];
  const float4 ex = make_float4(half_scan(tot.x) - tot.x, half_scan(tot.y) - tot.y, half_scan(tot.z) - tot.z,
                                half_scan(tot.w) - tot.w);
  const float exn = half_scan(nt) - nt;
#pragma unroll
  for (int i = 0; i < NSEG; ++i) {
    const int c = l * run + i;
    if (i < run && c < wM) { rv[c] = f4add(v[i], ex); rc[c] = n[i] + exn; }
  }
}

// ... and horizontal window sums at the R+ columns of the first `rows` rows of
// the pair (pixel t of the pair's R+ rows), into ring 1 at the slots of image
// rows row0 and row0+1.
template <int NC>
__device__ inline void a_wsum(const float4* scanv, const float* scanc, int w2, int rows, int ws_cap, int wP, int xp0,
                              int xm0, int r, int W, int row0, int lo_c, int sb1, int ring, float4* ring1v,
                              uint8_t* ring1c, int wp_cap, int lane) {
#pragma unroll
  for (int m = 0; m < NC; ++m) {
    const int t = m * 64 + lane;
    const int h = t >= wP ? 1 : 0;
    const int xi = t - h * wP;
    if (xi < wP && h < rows) {
      const float4* rv = scanv + (size_t)(w2 + h) * ws_cap;
      const float* rc = scanc + (size_t)(w2 + h) * ws_cap;
      const int x = xp0 + xi;
      const int lo = (x - r > 0 ? x - r : 0) - xm0;
      const int hi = (x + r < W - 1 ? x + r : W - 1) - xm0;
      const int lm = lo > 0 ? lo - 1 : 0;
      const float4 a = rv[hi], b = rv[lm];
      const float ac = rc[hi], bc = rc[lm];
      float4 hs = lo > 0 ? f4sub(a, b) : a;
      const float hc = lo > 0 ? ac - bc : ac;
      if (hc == 0.f) hs = make_float4(0.f, 0.f, 0.f, 0.f);
      const int slot = slot_of(row0 + h, lo_c, sb1, ring);
      ring1v[(size_t)slot * wp_cap + xi] = hs;
      ring1c[(size_t)slot * wp_cap + xi] = (uint8_t)hc;
    }
  }
}

// Entry i of a pair table, read through the constant address space: the
// compiler then takes the pointers it holds for global memory and loads
// through them with global (not flat) instructions.  The table is not written
// while a kernel runs.  (The host pass only type-checks kernel bodies.)
__device__ inline PairDev pair_of(const PairDev* pairs, int i) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const __attribute__((address_space(4))) PairDev*)pairs)[i];
#else
  return pairs[i];
#endif
}

template <int MODE, int NSEG, int NC>
__global__ __launch_bounds__(1024) void k_unary(const PairDev* __restrict__ pairs, const Item* __restrict__ items,
                                               const Tile* __restrict__ tiles, int n_tiles,
                                               const float4* __restrict__ label_field, float* __restrict__ out,
                                               int ring, int wp_cap, int tw_cap, int ws_cap, int pair_hint,
                                               int direct, int fill2) {
  extern __shared__ float4 smem4[];
  // blocks are dispatched round-robin over the 8 XCDs; give every XCD a
  // contiguous run of tiles so neighbouring tiles share its L2
  const int per = (int)(gridDim.x >> 3);
  const int t_id = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  if (t_id >= n_tiles) return;

  // MODE 2 covers every pixel of pair 0 (one 1x1 region per tile).  The
  // descriptor loads overlap where the launch allows: the pair table entry
  // with the tile when every tile is of pair pair_hint (>= 0), the item with
  // the tile when tile t is the only tile of item t (direct != 0).
  const bool hinted = MODE == 2 || pair_hint >= 0;
  PairDev pd{};
  if (hinted) pd = pair_of(pairs, MODE == 2 ? 0 : pair_hint);
  Tile tl{};
  Item it{};
  if (MODE != 2) {
    if (direct) {
      tl = tiles[t_id];
      it = items[t_id];
    } else {
      tl = tiles[t_id];
      it = items[tl.item];
    }
  }
  if (!hinted) pd = pair_of(pairs, it.pair);
  const DevParams P = pd.P;
  const float4* __restrict__ left4 = pd.left4;
  const float4* __restrict__ left4T = pd.left4T;
  const float4* __restrict__ right4 = pd.right4;
  const float* __restrict__ guide = pd.guide;
  const int W = P.W, H = P.H, r = P.r;
  int tu0, tv0, tu1, tv1, ru0 = 0, rv0 = 0, rw = 1, flags = 15;
  float la, lb, lc;
  long long out_off;
  if (MODE == 2) {
    tu0 = t_id % W; tv0 = t_id / W; tu1 = tu0 + 1; tv1 = tv0 + 1;
    const float4 f = label_field[t_id];
    la = f.x; lb = f.y; lc = f.z;
    ru0 = tu0; rv0 = tv0; rw = 1;
    out_off = t_id;
  } else {
    tu0 = tl.tu0; tv0 = tl.tv0; tu1 = tl.tu1; tv1 = tl.tv1; flags = tl.flags;
    la = it.a; lb = it.b; lc = it.c;
    ru0 = it.ru0; rv0 = it.rv0; rw = it.rw;
    out_off = it.out_off;
    if (MODE == 1) {  // output indexed over the item's R+
      const int pu0 = ru0 - r > 0 ? ru0 - r : 0, pv0 = rv0 - r > 0 ? rv0 - r : 0;
      const int pu1 = ru0 + rw + r < W ? ru0 + rw + r : W;
      rw = pu1 - pu0;
      ru0 = pu0;
      rv0 = pv0;
    }
  }
  const int xp0 = tu0 - r > 0 ? tu0 - r : 0, xp1 = tu1 + r < W ? tu1 + r : W;
  const int yp0 = tv0 - r > 0 ? tv0 - r : 0, yp1 = tv1 + r < H ? tv1 + r : H;
  const int xm0 = tu0 - 2 * r > 0 ? tu0 - 2 * r : 0, xm1 = tu1 + 2 * r < W ? tu1 + 2 * r : W;
  const int ym0 = tv0 - 2 * r > 0 ? tv0 - 2 * r : 0, ym1 = tv1 + 2 * r < H ? tv1 + 2 * r : H;
  const int wM = xm1 - xm0, wP = xp1 - xp0, tw = tu1 - tu0;
  // serial runs of the in-place row prefixes (stage A over M rows, stage E
  // over R+ rows), from the tile's own widths
  const int runA = (wM + 31) >> 5, runE = (wP + 31) >> 5;
  // R+ part this tile reports in MODE 1 (column / row strips own disjoint parts)
  const int own_u0 = (flags & kFirstCol) ? xp0 : tu0, own_u1 = (flags & kLastCol) ? xp1 : tu1;
  const int own_v0 = (flags & kFirstRow) ? yp0 : tv0, own_v1 = (flags & kLastRow) ? yp1 : tv1;

  // shared memory: float4 arrays, float arrays, then byte counts.  Slot
  // `ring` of each ring stays zero: the vertical sums read it for rows
  // outside a window.
  float4* ring1v = smem4;
  float4* coefv = ring1v + (size_t)(ring + 1) * wp_cap;
  float4* ring3v = coefv + (size_t)2 * kChunk * wp_cap;
  float4* scanv = ring3v + (size_t)(ring + 1) * tw_cap;
  float4* car1v = scanv + (size_t)kChunk * ws_cap;
  float4* car2v = car1v + (size_t)wp_cap;
  float* scanc = reinterpret_cast<float*>(car2v + (size_t)tw_cap);
  float* car1c = scanc + (size_t)kChunk * ws_cap;
  float* car2c = car1c + (size_t)wp_cap;
  uint8_t* ring1c = reinterpret_cast<uint8_t*>(car2c + (size_t)tw_cap);
  uint8_t* coefc = ring1c + (size_t)(ring + 1) * wp_cap;
  uint8_t* ring3c = coefc + (size_t)2 * kChunk * wp_cap;

  const int tid = threadIdx.x;
  // the wave index is uniform: say so, so that what derives from it stays scalar
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const float inv255 = 1.0f / 255.0f;
  const size_t hw = (size_t)W * H;

  const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int i = tid; i < wp_cap; i += kWaves * 64) {
    car1v[i] = zero4; car1c[i] = 0.f;
    ring1v[(size_t)ring * wp_cap + i] = zero4; ring1c[(size_t)ring * wp_cap + i] = 0;
  }
  for (int i = tid; i < tw_cap; i += kWaves * 64) {
    car2v[i] = zero4; car2c[i] = 0.f;
    ring3v[(size_t)ring * tw_cap + i] = zero4; ring3c[(size_t)ring * tw_cap + i] = 0;
  }

  // Pipeline schedule (wave-uniform scalars).  Both wave groups below run
  // the same recurrence, so they meet the same barriers.  Rings hold M rows
  // >= ym0 (ring1) and R+ rows >= yp0 (ring3); rows above those never enter
  // a window of the rows this tile emits.
  int produced = ym0;            // M rows handed to ring1 (visible after the step)
  int kv = yp0;                  // next R+ row to emit
  int lo_c = ym0, sb1 = 0;       // ring1 slot sb1 holds row lo_c
  int e_first = yp0, e_rows = 0; // coefficient rows emitted in the previous step
  int kv_e = yp0;                // R+ rows in ring3 (visible to G)
  int pv = tv0;                  // next R row to output
  int lo2_base = yp0, sb3 = 0;   // ring3 slot sb3 holds row lo2_base
  int pc = 0;                    // coefficient buffer parity
  int nA = 0, nC = 0, nG = 0;
  auto finished = [&]() { return MODE == 1 ? (kv >= own_v1) : (pv >= tv1); };
  // Rows each stage takes this step.  Row k's window reaches row min(k+r, H-1),
  // which grows with k, so the rows whose windows are complete form a prefix:
  // every remaining row once the image's last row is in, else rows k < in - r.
  // (Closed forms: every wave evaluates them, on the one scalar unit of the CU.)
  // (with fill2, waves 8-15 take rows 16-31 of the first step as stage A)
  auto count_rows = [&]() {
    nA = min(fill2 && produced == ym0 ? 2 * kChunk : kChunk, ym1 - produced);
    // R+ rows whose window rows are all in ring1
    nC = min(kChunk, yp1 - kv);
    if (produced <= H - 1) nC = max(0, min(nC, produced - r - kv));
    nG = 0;  // R rows whose window rows are all in ring3
    if (MODE != 1) {
      nG = tv1 - pv;
      if (kv_e <= H - 1) nG = max(0, min(nG, kv_e - r - pv));
    }
  };
  auto advance = [&]() {
    const int emitted_first = kv;
    if (nC > 0) {  // the next step's leaving rows start at row kv+nC-r-1
      const int k = kv + nC - 1;
      const int new_lo = k - r > ym0 ? k - r : ym0;
      sb1 = slot_of(new_lo, lo_c, sb1, ring);
      lo_c = new_lo;
      kv += nC;
    }
    if (nG > 0) {
      const int p = pv + nG - 1;
      const int new_lo2 = p - r > yp0 ? p - r : yp0;
      sb3 = slot_of(new_lo2, lo2_base, sb3, ring);
      lo2_base = new_lo2;
      pv += nG;
    }
    kv_e = e_first + e_rows;  // rows E wrote this step become visible next step
    e_first = emitted_first;
    e_rows = nC;
    pc ^= 1;
    produced += nA;
  };

  if (wave < kWaves / 2) {
    // ======== waves 0-7: stage A, M rows 2w and 2w+1 of each step ========
    const int w2 = 2 * wave;
    const char* left_b = reinterpret_cast<const char*>(left4);
    const char* right_b = reinterpret_cast<const char*>(right4);
    RowLanes<NSEG> rl;
    row_lanes<NSEG>(rl, w2, xm0, wM, W, ws_cap, lane);
    RowTaps<NSEG> taps;
    load_rows2<NSEG>(taps, rl, produced + w2, W, H, la, lb, lc, left_b, right_b);
    lds_barrier();
    while (!finished()) {
      count_rows();
      if (w2 < nA) {
        // raw cost of the pair's pixels -> scan rows 2w, 2w+1 (private to this wave)
        a_raw<NSEG>(P, taps, rl, scanv, scanc);
        // next step's image taps, in flight from here (issued in three runs).
        // The taps of this step are consumed: wait for them explicitly
        // (vmcnt 0, other counters untouched) so that no wait on the runs
        // issued below is needed before the next run.
        __builtin_amdgcn_s_waitcnt(0x0F70);
        constexpr int kL1 = (NSEG + 2) / 3, kL2 = (2 * NSEG + 2) / 3;
        const bool more = produced + nA < ym1;
        const int y_next = produced + nA + w2;
        if (more) load_rows2<NSEG, 0, kL1>(taps, rl, y_next, W, H, la, lb, lc, left_b, right_b);
        asm volatile("" ::: "memory");
        a_prefix<NSEG>(scanv, scanc, w2, ws_cap, wM, runA, lane);
        asm volatile("" ::: "memory");
        if (more) load_rows2<NSEG, kL1, kL2>(taps, rl, y_next, W, H, la, lb, lc, left_b, right_b);
        asm volatile("" ::: "memory");
        a_wsum<NC>(scanv, scanc, w2, nA - w2, ws_cap, wP, xp0, xm0, r, W, produced + w2, lo_c, sb1, ring, ring1v,
                   ring1c, wp_cap, lane);
        asm volatile("" ::: "memory");
        if (more) load_rows2<NSEG, kL2, NSEG>(taps, rl, y_next, W, H, la, lb, lc, left_b, right_b);
      }
      if (MODE != 1) {
        // ---- E: horizontal sums of (a, b) at the R columns ----------------
        // Rows 2e and 2e+1 of the previous step's coefficient rows: in-place
        // prefix as in A, then window sums at the R columns -> ring3.
        const int e = wave;
        if (2 * e < e_rows) {
          {
            const int h = lane >> 5, l = lane & 31;
            float4* cv = coefv + ((size_t)(pc ^ 1) * kChunk + 2 * e + h) * wp_cap;
            uint8_t* cc = coefc + ((size_t)(pc ^ 1) * kChunk + 2 * e + h) * wp_cap;
            float4 v[NC];
            float n[NC];
#pragma unroll
            for (int i = 0; i < NC; ++i) {
              const int c = l * runE + i;
              v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
              n[i] = 0.f;
              if (i < runE && c < wP) { v[i] = cv[c]; n[i] = (float)cc[c]; }
            }
#pragma unroll
            for (int i = 1; i < NC; ++i) { v[i] = f4add(v[i - 1], v[i]); n[i] = n[i - 1] + n[i]; }
            const float4 tot = v[NC - 1];
            const float nt = n[NC - 1];
            const float4 ex = make_float4(half_scan(tot.x) - tot.x, half_scan(tot.y) - tot.y,
                                          half_scan(tot.z) - tot.z, half_scan(tot.w) - tot.w);
            const float exn = half_scan(nt) - nt;
#pragma unroll
            for (int i = 0; i < NC; ++i) {
              const int c = l * runE + i;
              // prefix counts stay below 256: an R+ row is at most kMaxWP wide
              if (i < runE && c < wP) { cv[c] = f4add(v[i], ex); cc[c] = (uint8_t)(n[i] + exn); }
            }
          }
#pragma unroll
          for (int m = 0; m < NC; ++m) {
            const int t = m * 64 + lane;
            const int h = t >= tw ? 1 : 0;
            const int xi = t - h * tw;
            if (xi < tw && 2 * e + h < e_rows) {
              const float4* cv = coefv + ((size_t)(pc ^ 1) * kChunk + 2 * e + h) * wp_cap;
              const uint8_t* cc = coefc + ((size_t)(pc ^ 1) * kChunk + 2 * e + h) * wp_cap;
              const int x = tu0 + xi;
              const int lo = (x - r > 0 ? x - r : 0) - xp0;
              const int hi = (x + r < W - 1 ? x + r : W - 1) - xp0;
              const int lm = lo > 0 ? lo - 1 : 0;
              const float4 a = cv[hi], b = cv[lm];
              const float ac = (float)cc[hi], bc = (float)cc[lm];
              float4 hs = lo > 0 ? f4sub(a, b) : a;
              const float hc = lo > 0 ? ac - bc : ac;
              if (hc == 0.f) hs = make_float4(0.f, 0.f, 0.f, 0.f);
              const int slot = slot_of(e_first + 2 * e + h, lo2_base, sb3, ring);
              ring3v[(size_t)slot * tw_cap + xi] = hs;
              ring3c[(size_t)slot * tw_cap + xi] = (uint8_t)hc;
            }
          }
        }
      }
      advance();
      lds_barrier();
    }
  } else {
    // ======== waves 8-15: stages C and G ========
    // C and G lanes: column j*32 + 4*cw + lane/16, row lane%16 of the step.
    const int cw = wave - kWaves / 2;
    const int q16 = lane & 15;
    int cl[NC];
    float ncC[NC], ncG[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      cl[j] = j * 32 + cw * 4 + (lane >> 4);
      const int x1 = xp0 + cl[j], x2 = tu0 + cl[j];
      ncC[j] = (float)((x1 + r < W - 1 ? x1 + r : W - 1) - (x1 - r > 0 ? x1 - r : 0) + 1);
      ncG[j] = (float)((x2 + r < W - 1 ? x2 + r : W - 1) - (x2 - r > 0 ? x2 - r : 0) + 1);
    }
    // guide statistics, column-major: a lane group reads 16 consecutive rows
    const float4* g0 = reinterpret_cast<const float4*>(guide);
    const float4* g1 = g0 + hw;
    const float* g2 = reinterpret_cast<const float*>(g1 + hw);
    float gs[NC][9];
    auto load_guide = [&](int kbase) {
      const int k = kbase + q16;
      const int kc = k < yp1 - 1 ? k : yp1 - 1;
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const int ci = cl[j];
        const size_t gi = (size_t)(xp0 + (ci < wP - 1 ? ci : wP - 1)) * H + kc;
        const float4 a = g0[gi], b = g1[gi];
        gs[j][0] = a.x; gs[j][1] = a.y; gs[j][2] = a.z; gs[j][3] = a.w;
        gs[j][4] = b.x; gs[j][5] = b.y; gs[j][6] = b.z; gs[j][7] = b.w;
        gs[j][8] = g2[gi];
      }
    };
    float4 lp[NC];
    auto load_left = [&](int pbase) {
      const int p = pbase + q16;
      const int pc_ = p < tv1 - 1 ? p : tv1 - 1;
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const int ci = cl[j];
        lp[j] = left4T[(size_t)(tu0 + (ci < tw - 1 ? ci : tw - 1)) * H + pc_];
      }
    };
    if (fill2 && !finished()) {
      // First step: nothing for C and G yet, so these waves run stage A on
      // rows 16-31 of the step, with scan rows in ring-1 slots 32 and up
      // (rows of later steps only).  Their taps and registers die here.
      const int w2c = 2 * cw;
      float4* sv = ring1v + (size_t)2 * kChunk * wp_cap;
      float* sc = reinterpret_cast<float*>(sv + (size_t)kChunk * ws_cap);
      RowLanes<NSEG> rlc;
      row_lanes<NSEG>(rlc, w2c, xm0, wM, W, ws_cap, lane);
      RowTaps<NSEG> tc;
      load_rows2<NSEG>(tc, rlc, produced + kChunk + w2c, W, H, la, lb, lc, reinterpret_cast<const char*>(left4),
                       reinterpret_cast<const char*>(right4));
      lds_barrier();
      count_rows();
      if (kChunk + w2c < nA) {
        a_raw<NSEG>(P, tc, rlc, sv, sc);
        a_prefix<NSEG>(sv, sc, w2c, ws_cap, wM, runA, lane);
        a_wsum<NC>(sv, sc, w2c, nA - kChunk - w2c, ws_cap, wP, xp0, xm0, r, W, produced + kChunk + w2c, lo_c, sb1,
                   ring, ring1v, ring1c, wp_cap, lane);
      }
      load_guide(kv + nC);
      if (MODE != 1) load_left(pv + nG);
      advance();
      lds_barrier();
    } else {
      load_guide(kv);
      if (MODE != 1) load_left(pv);
      lds_barrier();
    }
    while (!finished()) {
      count_rows();

      // ---- C: vertical sums over W'_k, linear coefficients ---------------
      // Row k's window differs from row k-1's by at most one entering row
      // (k+r) and one leaving row (k-r-1); a prefix over the 16 lanes of a
      // column gives every row's sum from the carried sum of the previous
      // step's last row.  Before the first row the carried sum is that of the
      // (possibly virtual) row yp0-1, summed here by the 16 lanes of the column.
      // The column groups j are independent; each phase below runs over all of
      // them without per-lane branches so their latencies overlap.
      if (nC > 0) {
        const int k = kv + q16;
        const bool rowok = q16 < nC;
        const int ent = k + r, lev = k - r - 1;
        const bool has_ent = rowok && ent <= H - 1, has_lev = rowok && lev >= ym0;
        // rows outside the window read the zero slot
        const int sl_ent = has_ent ? slot_of(ent, lo_c, sb1, ring) : ring;
        const int sl_lev = has_lev ? slot_of(lev, lo_c, sb1, ring) : ring;
        const float rows = (float)((k + r < H - 1 ? k + r : H - 1) - (k - r > 0 ? k - r : 0) + 1);
        float4 V[NC], Cv[NC];
        float Vc[NC], Cc[NC];
        int cr[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          const bool colok = cl[j] < wP;
          cr[j] = colok ? cl[j] : 0;
          Cv[j] = car1v[cr[j]];  // carried sums (zero before the first rows)
          Cc[j] = car1c[cr[j]];
          const float4 ev = ring1v[(size_t)sl_ent * wp_cap + cr[j]], lv = ring1v[(size_t)sl_lev * wp_cap + cr[j]];
          const float ec = (float)ring1c[(size_t)sl_ent * wp_cap + cr[j]];
          const float lcn = (float)ring1c[(size_t)sl_lev * wp_cap + cr[j]];
          // (columns past the R+ row compute values nobody stores)
          V[j] = f4sub(ev, lv);
          Vc[j] = ec - lcn;
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          V[j].x = row_scan16(V[j].x);
          V[j].y = row_scan16(V[j].y);
          V[j].z = row_scan16(V[j].z);
          V[j].w = row_scan16(V[j].w);
          Vc[j] = row_scan16(Vc[j]);
        }
        if (kv == yp0) {  // first rows of the tile (uniform branch)
          const int i_lo = yp0 - 1 - r > ym0 ? yp0 - 1 - r : ym0;
          const int i_hi = yp0 - 1 + r < H - 1 ? yp0 - 1 + r : H - 1;
          // the column groups' reads of one row are issued together (columns
          // past the R+ row read column 0; nobody stores their sums)
          float4 I[NC];
          float Ic[NC];
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            I[j] = make_float4(0.f, 0.f, 0.f, 0.f);
            Ic[j] = 0.f;
          }
          for (int y = i_lo + q16; y <= i_hi; y += 16) {
            const int sl = slot_of(y, lo_c, sb1, ring);
#pragma unroll
            for (int j = 0; j < NC; ++j) {
              I[j] = f4add(I[j], ring1v[(size_t)sl * wp_cap + cr[j]]);
              Ic[j] += (float)ring1c[(size_t)sl * wp_cap + cr[j]];
            }
          }
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            I[j].x = row_last(row_scan16(I[j].x), lane);
            I[j].y = row_last(row_scan16(I[j].y), lane);
            I[j].z = row_last(row_scan16(I[j].z), lane);
            I[j].w = row_last(row_scan16(I[j].w), lane);
            Ic[j] = row_last(row_scan16(Ic[j]), lane);
            V[j] = f4add(I[j], V[j]);
            Vc[j] = Ic[j] + Vc[j];
          }
        } else {
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            V[j] = f4add(Cv[j], V[j]);
            Vc[j] = Cc[j] + Vc[j];
          }
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          const float inv_n = __builtin_amdgcn_rcpf(ncC[j] * rows);
          const float* g = gs[j];
          const float m0 = V[j].x * inv_n;
          const float c0 = V[j].y * inv_n - g[0] * m0;
          const float c1 = V[j].z * inv_n - g[1] * m0;
          const float c2 = V[j].w * inv_n - g[2] * m0;
          const float a0 = g[3] * c0 + g[4] * c1 + g[5] * c2;
          const float a1 = g[4] * c0 + g[6] * c1 + g[7] * c2;
          const float a2 = g[5] * c0 + g[7] * c1 + g[8] * c2;
          const float b = m0 - (a0 * g[0] + a1 * g[1] + a2 * g[2]);
          // a window without a nonzero sample has zero coefficients exactly
          const bool nz = Vc[j] != 0.f;
          const float4 coef = make_float4(nz ? a0 : 0.f, nz ? a1 : 0.f, nz ? a2 : 0.f, nz ? b : 0.f);
          if (cl[j] < wP && rowok) {
            const int ci = cl[j];
            if (MODE == 1) {
              const int x = xp0 + ci;
              if (x >= own_u0 && x < own_u1 && k >= own_v0 && k < own_v1) {
                // coefficients of rho itself: a is unchanged by the shift, b gains rho_max
                float* o = out + (out_off + (long long)(k - rv0) * rw + (x - ru0)) * 4;
                o[0] = coef.x; o[1] = coef.y; o[2] = coef.z; o[3] = coef.w + P.rho_max;
              }
            } else {
              coefv[((size_t)pc * kChunk + q16) * wp_cap + ci] = coef;
              coefc[((size_t)pc * kChunk + q16) * wp_cap + ci] = nz ? 1 : 0;
            }
            // the carried sum of a column is read and written by its own wave only
            if (q16 == nC - 1) {
              car1v[ci] = V[j];
              car1c[ci] = Vc[j];
            }
          }
        }
      }
      load_guide(kv + nC);

      if (MODE != 1) {
        // ---- G: vertical sums over W'(p), output ---------------------------
        // Same lane layout and update rule as C, over the R+ rows in ring3.
        for (int q0 = 0; q0 < nG; q0 += kChunk) {
          if (q0 > 0) load_left(pv + q0);  // (rows were prefetched for the first batch only)
          const int p = pv + q0 + q16;
          const bool rowok = q0 + q16 < nG;
          const int ent = p + r, lev = p - r - 1;
          const bool has_ent = rowok && ent <= H - 1, has_lev = rowok && lev >= yp0;
          const int sl_ent = has_ent ? slot_of(ent, lo2_base, sb3, ring) : ring;
          const int sl_lev = has_lev ? slot_of(lev, lo2_base, sb3, ring) : ring;
          const float rows = (float)((p + r < H - 1 ? p + r : H - 1) - (p - r > 0 ? p - r : 0) + 1);
          const int last = (nG - q0 < kChunk ? nG - q0 : kChunk) - 1;
          float4 V2[NC], Cv[NC];
          float V2c[NC], Cc[NC];
          int cr[NC];
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            if (j * 32 + cw * 4 >= tw) break;  // no column of this wave in group j (uniform)
            const bool colok = cl[j] < tw;
            cr[j] = colok ? cl[j] : 0;
            Cv[j] = car2v[cr[j]];  // carried sums (zero before the first rows)
            Cc[j] = car2c[cr[j]];
            const float4 ev = ring3v[(size_t)sl_ent * tw_cap + cr[j]], lv = ring3v[(size_t)sl_lev * tw_cap + cr[j]];
            const float ec = (float)ring3c[(size_t)sl_ent * tw_cap + cr[j]];
            const float lcn = (float)ring3c[(size_t)sl_lev * tw_cap + cr[j]];
            V2[j] = f4sub(ev, lv);
            V2c[j] = ec - lcn;
          }
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            if (j * 32 + cw * 4 >= tw) break;  // no column of this wave in group j (uniform)
            V2[j].x = row_scan16(V2[j].x);
            V2[j].y = row_scan16(V2[j].y);
            V2[j].z = row_scan16(V2[j].z);
            V2[j].w = row_scan16(V2[j].w);
            V2c[j] = row_scan16(V2c[j]);
          }
          if (pv + q0 == tv0) {  // first rows of the tile (uniform branch)
            const int i_lo = tv0 - 1 - r > yp0 ? tv0 - 1 - r : yp0;
            const int i_hi = tv0 - 1 + r < H - 1 ? tv0 - 1 + r : H - 1;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
              if (j * 32 + cw * 4 >= tw) break;  // no column of this wave in group j (uniform)
              float4 I = make_float4(0.f, 0.f, 0.f, 0.f);
              float Ic = 0.f;
              if (cl[j] < tw)
                for (int y = i_lo + q16; y <= i_hi; y += 16) {
                  const int sl = slot_of(y, lo2_base, sb3, ring);
                  I = f4add(I, ring3v[(size_t)sl * tw_cap + cl[j]]);
                  Ic += (float)ring3c[(size_t)sl * tw_cap + cl[j]];
                }
              I.x = row_last(row_scan16(I.x), lane);
              I.y = row_last(row_scan16(I.y), lane);
              I.z = row_last(row_scan16(I.z), lane);
              I.w = row_last(row_scan16(I.w), lane);
              Ic = row_last(row_scan16(Ic), lane);
              V2[j] = f4add(I, V2[j]);
              V2c[j] = Ic + V2c[j];
            }
          } else {
#pragma unroll
            for (int j = 0; j < NC; ++j) {
              if (j * 32 + cw * 4 >= tw) break;  // no column of this wave in group j (uniform)
              V2[j] = f4add(Cv[j], V2[j]);
              V2c[j] = Cc[j] + V2c[j];
            }
          }
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            if (j * 32 + cw * 4 >= tw) break;  // no column of this wave in group j (uniform)
            const float4 L = lp[j];
            const float phi = (V2[j].x * (L.x * inv255) + V2[j].y * (L.y * inv255) + V2[j].z * (L.z * inv255) +
                               V2[j].w) * __builtin_amdgcn_rcpf(ncG[j] * rows);
            if (cl[j] < tw && rowok) {
              const int ci = cl[j];
              const int x = tu0 + ci;
              // a window without a nonzero coefficient row costs rho_max exactly
              out[out_off + (long long)(p - rv0) * rw + (x - ru0)] = (V2c[j] != 0.f ? phi : 0.f) + P.rho_max;
              if (q16 == last) {
                car2v[ci] = V2[j];
                car2c[ci] = V2c[j];
              }
            }
          }
        }
        load_left(pv + nG);
      }
      advance();
      lds_barrier();
    }
  }
}

#define LEXP_UNARY_INST(M, S, C)                                                                                    \
  template __global__ void k_unary<M, S, C>(const PairDev*, const Item*, const Tile*, int, const float4*, float*, \
                                            int, int, int, int, int, int, int);
LEXP_UNARY_INST(0, 1, 1)
LEXP_UNARY_INST(0, 2, 1)
LEXP_UNARY_INST(0, 2, 2)
LEXP_UNARY_INST(0, 3, 1)
LEXP_UNARY_INST(0, 3, 2)
LEXP_UNARY_INST(0, 3, 3)
LEXP_UNARY_INST(0, 4, 1)
LEXP_UNARY_INST(0, 4, 2)
LEXP_UNARY_INST(0, 4, 3)
LEXP_UNARY_INST(0, 4, 4)
LEXP_UNARY_INST(2, 1, 1)
LEXP_UNARY_INST(2, 2, 1)
LEXP_UNARY_INST(2, 2, 2)
LEXP_UNARY_INST(2, 3, 1)
LEXP_UNARY_INST(2, 3, 2)
LEXP_UNARY_INST(2, 3, 3)
LEXP_UNARY_INST(2, 4, 1)
LEXP_UNARY_INST(2, 4, 2)
LEXP_UNARY_INST(2, 4, 3)
LEXP_UNARY_INST(2, 4, 4)
LEXP_UNARY_INST(1, 4, 4)
#undef LEXP_UNARY_INST

// ---------------------------------------------------------------------------
// Smoothness term (Eqs. 10-12) in FP64, rounded as written.
// ---------------------------------------------------------------------------
__device__ inline double plane_at(float a, float b, float c, int u, int v) {
  const double t1 = (double)a * (double)u;
  const double t2 = (double)b * (double)v;
  const double s = t1 + t2;
  return s + (double)c;
}

__device__ inline double psi(const DevParams& P, double w, float4 fp, float4 fq, int pu, int pv, int qu, int qv) {
  const double dpp = plane_at(fp.x, fp.y, fp.z, pu, pv), dpq = plane_at(fq.x, fq.y, fq.z, pu, pv);
  const double dqq = plane_at(fq.x, fq.y, fq.z, qu, qv), dqp = plane_at(fp.x, fp.y, fp.z, qu, qv);
  const double pb = fabs(dpp - dpq) + fabs(dqq - dqp);
  const double wt = w > P.w_floor ? w : P.w_floor;
  const double tr = pb < P.tau_dis ? pb : P.tau_dis;
  return P.lam * wt * tr;
}

__device__ inline long long qceil(double x) { return (long long)ceil(x * kQuantum); }

__device__ inline bool same_label(float4 a, float4 b) {
  return __float_as_uint(a.x) == __float_as_uint(b.x) && __float_as_uint(a.y) == __float_as_uint(b.y) &&
         __float_as_uint(a.z) == __float_as_uint(b.z);
}

// Binary problem of one local expansion per item: for every p in the region,
// U_p (cost of taking alpha) and w_d (cost of x_p = 0, x_{p+fwd_d} = 1).
__global__ void k_graph_terms(const PairDev* __restrict__ pairs, const Item* __restrict__ items,
                              const float* __restrict__ phi_alpha, int* __restrict__ terms, int* __restrict__ flag) {
  const Item it = items[blockIdx.y];
  const int li = blockIdx.x * blockDim.x + threadIdx.x;
  if (li >= it.rw * it.rh) return;
  const PairDev pd = pair_of(pairs, it.pair);
  const DevParams P = pd.P;
  const float4* __restrict__ labels = pd.labels;
  const double* __restrict__ wts = pd.wts;
  const int W = P.W, H = P.H;
  const int pu = it.ru0 + li % it.rw, pv = it.rv0 + li / it.rw;
  const float4 fp = labels[(size_t)pv * W + pu];
  const float4 al = make_float4(it.a, it.b, it.c, 0.f);
  int* o = terms + (size_t)(it.aux_off + li) * 5;
  if (same_label(fp, al)) {  // phi_p(alpha) = phi_p(f_p): every term cancels
    o[0] = 0; o[1] = 0; o[2] = 0; o[3] = 0; o[4] = 0;
    return;
  }
  long long U = qceil((double)phi_alpha[it.out_off + li]) - qceil((double)pd.cur_cost[(size_t)pv * W + pu]);
  long long wf[4] = {0, 0, 0, 0};
  const int nf = P.nf;
  for (int q = 0; q < 2 * nf; ++q) {
    const bool fwd = q < nf;
    const int d = fwd ? q : q - nf;
    const int nu = fwd ? pu + kFwdDU[d] : pu - kFwdDU[d];
    const int nv = fwd ? pv + kFwdDV[d] : pv - kFwdDV[d];
    if (nu < 0 || nu >= W || nv < 0 || nv >= H) continue;
    const float4 fn = labels[(size_t)nv * W + nu];
    const double w = fwd ? wts[((size_t)pv * W + pu) * 4 + d] : wts[((size_t)nv * W + nu) * 4 + d];
    const bool inside = nu >= it.ru0 && nu < it.ru0 + it.rw && nv >= it.rv0 && nv < it.rv0 + it.rh;
    if (!inside) {
      U += qceil(psi(P, w, al, fn, pu, pv, nu, nv)) - qceil(psi(P, w, fp, fn, pu, pv, nu, nv));
    } else if (fwd) {
      const long long A = qceil(psi(P, w, fp, fn, pu, pv, nu, nv));
      const long long B = qceil(psi(P, w, fp, al, pu, pv, nu, nv));
      const long long C = qceil(psi(P, w, al, fn, pu, pv, nu, nv));
      U += C - A;
      const long long e = B + C - A;
      wf[d] = e > 0 ? e : 0;
    } else {
      U -= qceil(psi(P, w, al, fp, nu, nv, pu, pv));
    }
  }
  const long long lim = 1ll << 30;
  if (U > lim || U < -lim || wf[0] > lim || wf[1] > lim || wf[2] > lim || wf[3] > lim) atomicOr(flag, 1);
  o[0] = (int)U;
  o[1] = (int)wf[0];
  o[2] = (int)wf[1];
  o[3] = (int)wf[2];
  o[4] = (int)wf[3];
}

// labels[p] = alpha and cur_cost[p] = phi_p(alpha) where the cut took alpha.
__global__ void k_apply(const PairDev* __restrict__ pairs, const Item* __restrict__ items,
                        const uint8_t* __restrict__ x, const float* __restrict__ phi_alpha) {
  const Item it = items[blockIdx.y];
  const int li = blockIdx.x * blockDim.x + threadIdx.x;
  if (li >= it.rw * it.rh) return;
  if (!x[it.aux_off + li]) return;
  const PairDev pd = pair_of(pairs, it.pair);
  const int W = pd.P.W;
  const int pu = it.ru0 + li % it.rw, pv = it.rv0 + li / it.rw;
  pd.labels[(size_t)pv * W + pu] = make_float4(it.a, it.b, it.c, 0.f);
  pd.cur_cost[(size_t)pv * W + pu] = phi_alpha[it.out_off + li];
}

// Eq. (5): per-block partial sums (FP64) of the unary and pairwise parts.
__global__ void k_energy(DevParams P, const float4* __restrict__ labels, const float* __restrict__ cur_cost,
                         const double* __restrict__ wts, double* __restrict__ partial) {
  __shared__ double su[256], sp[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double eu = 0.0, ep = 0.0;
  if (i < P.W * P.H) {
    const int u = i % P.W, v = i / P.W;
    eu = (double)cur_cost[i];
    const float4 fp = labels[i];
    for (int d = 0; d < P.nf; ++d) {
      const int qu = u + kFwdDU[d], qv = v + kFwdDV[d];
      if (qu < 0 || qu >= P.W || qv >= P.H) continue;
      ep += psi(P, wts[(size_t)i * 4 + d], fp, labels[(size_t)qv * P.W + qu], u, v, qu, qv);
    }
  }
  su[threadIdx.x] = eu;
  sp[threadIdx.x] = ep;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      su[threadIdx.x] += su[threadIdx.x + s];
      sp[threadIdx.x] += sp[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = su[0];
    partial[2 * blockIdx.x + 1] = sp[0];
  }
}

// Totals of k_energy's per-block partial sums, added in block order (the
// order in which the host adds them for lexp_energy, so the sums are the same
// bit for bit): out[0] the unary part, out[1] the pairwise part.  One
// workgroup of 256 threads stages runs of partials in LDS; thread 0 adds them.
__global__ void k_energy_total(const double* __restrict__ partial, int n_blocks, double* __restrict__ out) {
  __shared__ double run[2 * 1024];
  double eu = 0.0, ep = 0.0;
  for (int b0 = 0; b0 < n_blocks; b0 += 1024) {
    const int nb = n_blocks - b0 < 1024 ? n_blocks - b0 : 1024;
    for (int i = threadIdx.x; i < 2 * nb; i += blockDim.x) run[i] = partial[(size_t)2 * b0 + i];
    __syncthreads();
    if (threadIdx.x == 0)
      for (int b = 0; b < nb; ++b) {
        eu += run[2 * b];
        ep += run[2 * b + 1];
      }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = eu;
    out[1] = ep;
  }
}

// One smoothness term through the device path (inspection).
__global__ void k_pair1(DevParams P, const double* __restrict__ wts, int pu, int pv, int qu, int qv, float4 fp,
                        float4 fq, double* out) {
  // weight of the unordered pair: stored at the endpoint it is forward from
  double w = 0.0;
  for (int d = 0; d < 4; ++d) {
    if (qu - pu == kFwdDU[d] && qv - pv == kFwdDV[d]) w = wts[((size_t)pv * P.W + pu) * 4 + d];
    if (pu - qu == kFwdDU[d] && pv - qv == kFwdDV[d]) w = wts[((size_t)qv * P.W + qu) * 4 + d];
  }
  out[0] = psi(P, w, fp, fq, pu, pv, qu, qv);
}


}  // namespace lexp
