// Learned proposal network on CDNA4 (gfx950): five 3x3 convolutions as
// implicit GEMMs on the BF16 matrix cores (FP32 sums), their backward
// passes, the plane loss and Adam.  The forward and input-gradient products
// and weight-gradient products use v_mfma_f32_16x16x32_bf16 (K = 32 per
// instruction).
//
// Layout: activations and gradients pixel-major (index (v W + u) C + c), BF16;
// the last layer's output FP32; weights [tap][out][in] (tap = 3 ky + kx,
// offset (kx-1, ky-1)) with a BF16 copy in that order and one in
// [tap][in][out] for the backward-data products.
//
// One matrix instruction computes one 16 x 16 block of a product.
// Operand fragments (checked on the device): lane l holds
// A[l % 16][8 (l/16) + i] and B[8 (l/16) + i][l % 16] for i < 8 and gets
// D[4 (l/16) + i][l % 16] for i < 4.
//   forward     : M = 16 pixels of a row, N = output channels, K = 9 taps x
//                 input channels, tap-major, in chunks of 32 (one tap of 32
//                 channels, or two taps of 16, the last chunk then half
//                 zero); a wave takes four such blocks of a row;
//   backward x  : M = 16 pixels, N = input channels, K = 9 taps x output
//                 channels (gradient at p - offset; four blocks per wave);
//   backward w  : per tap, M = output channels, N = input channels, K = the
//                 pixels of a chunk, 32 columns of one row at a time; chunk
//                 partial sums are added in a fixed order by a second kernel
//                 (the result does not depend on scheduling).
// BF16 values are rounded to nearest even from FP32 (FP64 values through
// FP32 first), at the points the network's training recipe fixes.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lexp_device.h"

namespace lexp {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite values)
  return (uint16_t)(u >> 16);
}

// Eight BF16 values from 16 aligned bytes (LDS).
__device__ inline bf16x8 load8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

}  // namespace

// Network input, 16 BF16 channels per pixel: RGB/255 of the context's left
// image, RGB/255 of its right image at the pixel's match x = u - d (linear
// interpolation in FP64; zero outside the image), a, b, d/disp_max of the
// label (d = a u + b v + c in FP64), 1 where the match lies inside the right
// image, then zeros.
__global__ void k_net_input(const float4* __restrict__ left4, const float4* __restrict__ right4,
                            const float4* __restrict__ labels, int W, int H, double disp_max,
                            uint16_t* __restrict__ x0) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= W * H) return;
  const int u = p % W, v = p / W;
  const float4 L = left4[p], f = labels[p];
  const double d = ((double)f.x * (double)u + (double)f.y * (double)v) + (double)f.z;
  const double x = (double)u - d;
  double r0 = 0.0, r1 = 0.0, r2 = 0.0, inside = 0.0;
  if (x >= 0.0 && x <= (double)(W - 1)) {
    const int i0 = (int)floor(x);
    const int i1 = i0 + 1 < W ? i0 + 1 : W - 1;
    const double t = x - (double)i0;
    const float4 a = right4[(size_t)v * W + i0], b = right4[(size_t)v * W + i1];
    r0 = (1.0 - t) * (double)a.x + t * (double)b.x;
    r1 = (1.0 - t) * (double)a.y + t * (double)b.y;
    r2 = (1.0 - t) * (double)a.z + t * (double)b.z;
    inside = 1.0;
  }
  float ch[16];
  ch[0] = (float)((double)L.x / 255.0);
  ch[1] = (float)((double)L.y / 255.0);
  ch[2] = (float)((double)L.z / 255.0);
  ch[3] = (float)(r0 / 255.0);
  ch[4] = (float)(r1 / 255.0);
  ch[5] = (float)(r2 / 255.0);
  ch[6] = f.x;
  ch[7] = f.y;
  ch[8] = (float)(d / disp_max);
  ch[9] = (float)inside;
  for (int c = 10; c < 16; ++c) ch[c] = 0.f;
  for (int c = 0; c < 16; ++c) x0[(size_t)p * 16 + c] = to_bf16(ch[c]);
}

// Pixels per wave in the forward and input-gradient convolutions: kSegs
// segments of 16 consecutive pixels of one row, each weight fragment loaded
// once and used for all of them; kConvRows rows (waves) per workgroup.
constexpr int kSegs = kConvSegs;

// Patch of a pixel-major BF16 map with C channels that a workgroup's rows
// v0..v0+kConvRows-1 of one run of kSegs x 16 columns read through 3x3 taps:
// rows v0-1..v0+kConvRows, columns u0-1..u0+16 kSegs, zero outside the image,
// pixels C + kPatchPad elements apart (16-byte aligned, and the 16 pixels of
// a fragment start in distinct groups of four LDS banks).  Coalesced 16-byte
// loads, 8-byte LDS stores.
constexpr int kPatchW = 16 * kSegs + 2;
constexpr int kPatchR = kConvRows + 2;
constexpr int kPatchPad = 8;

template <int C>
struct PatchStage {
  static constexpr int kPS = C + kPatchPad;
  static constexpr int kPieces = C / 8, kTotal = kPatchR * kPatchW * kPieces, kPer = (kTotal + kConvThreads - 1) / kConvThreads;
  uint4 val[kPer];
  // global loads of this thread's pieces (all issued before any is used)
  __device__ inline void load(const uint16_t* __restrict__ src, int W, int H, int u0, int v0) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = (int)threadIdx.x + k * kConvThreads;
      const int pc = i % kPieces, px = i / kPieces;
      const int col = px % kPatchW, row = px / kPatchW;
      const int yy = v0 - 1 + row, xx = u0 - 1 + col;
      val[k] = make_uint4(0u, 0u, 0u, 0u);
      if (i < kTotal && yy >= 0 && yy < H && xx >= 0 && xx < W)
        val[k] = *reinterpret_cast<const uint4*>(src + ((size_t)yy * W + xx) * C + pc * 8);
    }
  }
  __device__ inline void store(uint16_t* patch) const {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = (int)threadIdx.x + k * kConvThreads;
      if (i < kTotal) {
        const int pc = i % kPieces, px = i / kPieces;
        uint2* dst = reinterpret_cast<uint2*>(patch + (size_t)px * kPS + pc * 8);
        dst[0] = make_uint2(val[k].x, val[k].y);
        dst[1] = make_uint2(val[k].z, val[k].w);
      }
    }
  }
};

// A layer's BF16 weights ([tap][n][k] for N rows n of K elements k) copied to
// LDS in the order the K = 32 fragments read them: element (tap, n, k), at
// position j = tap K + k of the product's K dimension, goes to
// [j / 32][n / 16][(j % 32) / 8][n % 16][j % 8], so the 64 lanes of a wave read
// one fragment as 1 KB of consecutive bytes.  Chunks past 9 K (K = 16: the
// last chunk's second half) are zero.
template <int N, int K, int THREADS = kConvThreads>
struct WeightStage {
  static constexpr int kChunks = (9 * K + 31) / 32, kTotal = kChunks * 32 * N / 8, kPer = (kTotal + THREADS - 1) / THREADS;
  uint4 val[kPer];
  __device__ inline void load(const uint16_t* __restrict__ w) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = (int)threadIdx.x + k * THREADS;
      // piece i of the fragment order: chunk c, block nb, lane group g, row m
      const int m = i % 16, g = (i / 16) % 4, nb = (i / 64) % (N / 16), c = i / (64 * (N / 16));
      const int j = c * 32 + g * 8, n = nb * 16 + m;
      val[k] = make_uint4(0u, 0u, 0u, 0u);
      if (i < kTotal && j < 9 * K) {
        const int tap = j / K, kk = j % K;
        val[k] = *reinterpret_cast<const uint4*>(w + ((size_t)tap * N + n) * K + kk);
      }
    }
  }
  __device__ inline void store(uint16_t* ws) const {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = (int)threadIdx.x + k * THREADS;
      if (i < kTotal) *reinterpret_cast<uint4*>(ws + (size_t)i * 8) = val[k];
    }
  }
};

// LDS of a forward or input-gradient workgroup: the input patch (CP
// channels) and the weights (N outputs) while the products run, then every
// wave's block of 16 kSegs pixels x N channels (rows N + 8 elements apart, so
// the four pixel rows a write instruction touches fall in distinct banks) for
// coalesced 16-byte stores.
template <int CP, int N>
struct ConvLds {
  static constexpr int kPS = CP + kPatchPad;
  static constexpr int kChunks = (9 * CP + 31) / 32;
  static constexpr int kPatch = kPatchR * kPatchW * kPS;
  static constexpr int kW = kChunks * 32 * N;
  static constexpr int kOS = N + 8;
  static constexpr int kOut = kConvRows * 16 * kSegs * kOS;
  static constexpr int kFS = N + 4;                      // FP32 output blocks: floats per pixel row
  static constexpr int kOutF = 2 * kConvRows * 16 * kSegs * kFS;  // in 16-bit elements
  static constexpr int kOutMax = kOut > kOutF ? kOut : kOutF;
  static constexpr int kElems = kPatch + kW > kOutMax ? kPatch + kW : kOutMax;
};

// Products of a forward (MIRROR false) or input-gradient (MIRROR true)
// workgroup: stages the patch and the weights, then wave w accumulates row
// v0 + w of the run: acc[s][nb] = the 16 x 16 block of pixels u0 + 16 s ..
// and outputs 16 nb .. over K = 9 taps x CP channels, one K = 32 chunk at a
// time, each weight fragment read once for the row's blocks.  Blocks past the
// image's last column are skipped.  Ends with a barrier, after which the LDS
// is free for the output blocks.
template <int CP, int N, bool MIRROR>
__device__ inline void conv_products(const uint16_t* __restrict__ src, const uint16_t* __restrict__ w, int W, int H,
                                     int u0, int v0, uint16_t* smem, f32x4 (&acc)[kSegs][N / 16]) {
  using Lds = ConvLds<CP, N>;
  constexpr int kPS = Lds::kPS;
  uint16_t* patch = smem;
  uint16_t* wsh = smem + Lds::kPatch;
  {
    PatchStage<CP> ps;
    WeightStage<N, CP> ws;
    ps.load(src, W, H, u0, v0);
    ws.load(w);
    ps.store(patch);
    ws.store(wsh);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = lane & 15, g = lane >> 4;
  const int live_segs = __builtin_amdgcn_readfirstlane(min(kSegs, (W - u0 + 15) / 16));
#pragma unroll
  for (int sg = 0; sg < kSegs; ++sg)
#pragma unroll
    for (int nb = 0; nb < N / 16; ++nb) acc[sg][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < Lds::kChunks; ++c) {
    const int j = c * 32 + g * 8;  // this lane's first K index: tap j / CP, channel j % CP
    const bool live = j < 9 * CP;
    const int tap = live ? j / CP : 0, ch = j % CP;
    bf16x8 b[N / 16];
#pragma unroll
    for (int nb = 0; nb < N / 16; ++nb) b[nb] = load8(wsh + ((size_t)((c * (N / 16) + nb) * 4 + g) * 16 + m) * 8);
    // forward: image row v + tap/3 - 1, column u + tap%3 - 1; input gradient:
    // the mirrored offset (g at p - offset)
    const int prow = MIRROR ? wv + 2 - tap / 3 : wv + tap / 3;
    const int pcol = MIRROR ? 2 - tap % 3 : tap % 3;
#pragma unroll
    for (int sg = 0; sg < kSegs; ++sg) {
      if (sg < live_segs) {
        bf16x8 a = load8(patch + ((size_t)prow * kPatchW + sg * 16 + m + pcol) * kPS + ch);
        if (!live) a = bf16x8{};
#pragma unroll
        for (int nb = 0; nb < N / 16; ++nb)
          acc[sg][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[nb], acc[sg][nb], 0, 0, 0);
      }
    }
  }
  __syncthreads();
}

// Forward convolution of one layer.  A workgroup takes kConvRows rows from v0 of
// one run of kSegs x 16 columns; each wave computes one row of the run (all
// output channels).  Bias, then ReLU and BF16 (hidden layers) or FP32 output
// (last layer), through LDS so that every store writes 16 bytes of a pixel.
template <int CI, int CO, bool LAST>
__global__ __launch_bounds__(kConvThreads) void k_conv_fwd(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w16,
                                                  const float* __restrict__ bias, int W, int H,
                                                  uint16_t* __restrict__ xo, float* __restrict__ yo) {
  using Lds = ConvLds<CI, CO>;
  __shared__ __align__(16) uint16_t smem[Lds::kElems];
  const int nrun = (W + 16 * kSegs - 1) / (16 * kSegs);
  const int u0 = (blockIdx.x % nrun) * 16 * kSegs, v0 = (blockIdx.x / nrun) * kConvRows;
  f32x4 acc[kSegs][CO / 16];
  conv_products<CI, CO, false>(x, w16, W, H, u0, v0, smem, acc);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int v = v0 + wv;
  const int m = lane & 15, kq = (lane >> 4) * 4;
  if (LAST) {
    float* of = reinterpret_cast<float*>(smem) + (size_t)wv * 16 * kSegs * Lds::kFS;
#pragma unroll
    for (int nb = 0; nb < CO / 16; ++nb) {
      const int co = nb * 16 + m;
      const float bb = bias[co];
#pragma unroll
      for (int sg = 0; sg < kSegs; ++sg)
#pragma unroll
        for (int i = 0; i < 4; ++i) of[(sg * 16 + kq + i) * Lds::kFS + co] = acc[sg][nb][i] + bb;
    }
    __syncthreads();
    if (v >= H) return;
    constexpr int kPf = CO / 4;  // 16-byte pieces per pixel
#pragma unroll
    for (int k = 0; k < 16 * kSegs * kPf / 64; ++k) {
      const int q = lane + 64 * k, px = q / kPf, pc = q % kPf;
      const int u = u0 + px;
      if (u < W)
        *reinterpret_cast<float4*>(yo + ((size_t)v * W + u) * CO + pc * 4) =
            *reinterpret_cast<const float4*>(of + px * Lds::kFS + pc * 4);
    }
    return;
  }
  uint16_t* ob = smem + (size_t)wv * 16 * kSegs * Lds::kOS;
#pragma unroll
  for (int nb = 0; nb < CO / 16; ++nb) {
    const int co = nb * 16 + m;
    const float bb = bias[co];
#pragma unroll
    for (int sg = 0; sg < kSegs; ++sg)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float z = acc[sg][nb][i] + bb;
        ob[(sg * 16 + kq + i) * Lds::kOS + co] = to_bf16(z > 0.f ? z : 0.f);
      }
  }
  __syncthreads();
  if (v >= H) return;
  constexpr int kPc = CO / 8;  // 16-byte pieces per pixel
#pragma unroll
  for (int k = 0; k < 16 * kSegs * kPc / 64; ++k) {
    const int q = lane + 64 * k, px = q / kPc, pc = q % kPc;
    const int u = u0 + px;
    if (u < W)
      *reinterpret_cast<uint4*>(xo + ((size_t)v * W + u) * CO + pc * 8) =
          *reinterpret_cast<const uint4*>(ob + px * Lds::kOS + pc * 8);
  }
}

// Gradient of a layer's input: dx(p) = sum over taps and output channels of
// W[tap][o][i] g(p - offset)[o], then gp = BF16(dx) * [x(p) > 0] (the input
// came from a ReLU).  Workgroups as in the forward convolution, with the
// patch of g (the taps mirrored) and the weights in [tap][in][out] order;
// the mask is applied on the 16-byte stores.
template <int CI, int CO>
__global__ __launch_bounds__(kConvThreads) void k_conv_bwd_x(const uint16_t* __restrict__ g, const uint16_t* __restrict__ wt16,
                                                    const uint16_t* __restrict__ x, int W, int H,
                                                    uint16_t* __restrict__ gp) {
  using Lds = ConvLds<CO, CI>;
  __shared__ __align__(16) uint16_t smem[Lds::kElems];
  const int nrun = (W + 16 * kSegs - 1) / (16 * kSegs);
  const int u0 = (blockIdx.x % nrun) * 16 * kSegs, v0 = (blockIdx.x / nrun) * kConvRows;
  f32x4 acc[kSegs][CI / 16];
  conv_products<CO, CI, true>(g, wt16, W, H, u0, v0, smem, acc);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int v = v0 + wv;
  const int m = lane & 15, kq = (lane >> 4) * 4;
  uint16_t* ob = smem + (size_t)wv * 16 * kSegs * Lds::kOS;
#pragma unroll
  for (int nb = 0; nb < CI / 16; ++nb)
#pragma unroll
    for (int sg = 0; sg < kSegs; ++sg)
#pragma unroll
      for (int i = 0; i < 4; ++i) ob[(sg * 16 + kq + i) * Lds::kOS + nb * 16 + m] = to_bf16(acc[sg][nb][i]);
  __syncthreads();
  if (v >= H) return;
  constexpr int kPc = CI / 8;
#pragma unroll
  for (int k = 0; k < 16 * kSegs * kPc / 64; ++k) {
    const int q = lane + 64 * k, px = q / kPc, pc = q % kPc;
    const int u = u0 + px;
    if (u < W) {
      const size_t o = ((size_t)v * W + u) * CI + pc * 8;
      const uint4 xv = *reinterpret_cast<const uint4*>(x + o);
      uint4 d = *reinterpret_cast<const uint4*>(ob + px * Lds::kOS + pc * 8);
      // BF16 x > 0: sign bit clear and not zero, per 16-bit half
      auto mask = [](uint32_t xw, uint32_t dw) {
        const uint32_t lo = ((xw & 0x8000u) == 0u && (xw & 0xffffu) != 0u) ? 0xffffu : 0u;
        const uint32_t hi = ((xw & 0x80000000u) == 0u && (xw >> 16) != 0u) ? 0xffff0000u : 0u;
        return dw & (lo | hi);
      };
      d.x = mask(xv.x, d.x); d.y = mask(xv.y, d.y); d.z = mask(xv.z, d.z); d.w = mask(xv.w, d.w);
      *reinterpret_cast<uint4*>(gp + o) = d;
    }
  }
}

// Weight and bias gradients of one layer, partial sums per chunk:
// part_w[chunk][tap][o][i] = sum over the chunk's pixels p of g(p)[o]
// x(p + offset(tap))[i] (x zero outside the image); part_b[chunk][o] = sum of
// g(p)[o].  A chunk is kWgRows image rows by kWgTiles tiles of 32 columns;
// one workgroup (kWgThreads / 64 waves) per chunk, all nine taps.
//
// Products: per tap, M = output channels, N = input channels, K = 32 pixels
// of one tile row (v_mfma_f32_16x16x32_bf16).  Both operands take 8
// consecutive pixels of one channel per lane, so the tile goes to LDS
// channel-major: g as gT[o][row][col], x as three copies xT[dx][i][row][col]
// (rows from one above the tile to one below it, copy dx shifted by dx
// columns), so that every fragment is one aligned 16-byte read.  Channel
// strides of 68 and 100 words put the 16 channels of a fragment read in
// distinct LDS banks.  Wave w takes input block nb = w % (CI/16) and the
// taps tg, tg + TG, ... (tg = w / (CI/16), TG = waves / (CI/16); waves with
// tg >= 9 only stage), for every output block; wave 0 also adds up g for the
// bias.  The next tile's global loads
// are in flight while the current tile's products run.
template <int CI, int CO>
__global__ __launch_bounds__(kWgThreads) void k_conv_bwd_w(const uint16_t* __restrict__ g, const uint16_t* __restrict__ x,
                                                    int W, int H, float* __restrict__ part_w,
                                                    float* __restrict__ part_b) {
  constexpr int kR = kWgRows;
  constexpr int kSG = kR * 32 + 8, kSX = (kR + 2) * 32 + 8;  // channel strides (elements)
  constexpr int kNB = CI / 16, kMB = CO / 16, kTG = kWgThreads / 64 / kNB, kTaps = (9 + kTG - 1) / kTG;
  // staging pieces: a pair of adjacent pixels x 8 channels
  constexpr int kGItems = kR * 16 * (CO / 8), kXItems = 3 * (kR + 2) * 16 * (CI / 8);
  constexpr int kGPer = (kGItems + kWgThreads - 1) / kWgThreads, kXPer = (kXItems + kWgThreads - 1) / kWgThreads;
  __shared__ __align__(16) uint16_t gT[CO * kSG];
  __shared__ __align__(16) uint16_t xT[3 * CI * kSX];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = lane & 15, grp = lane >> 4;
  const int nb = wv % kNB, tg = wv / kNB;
  const int n_tiles = (W + 31) / 32, n_groups = (n_tiles + kWgTiles - 1) / kWgTiles;
  const int chunk = blockIdx.x;
  const int v0 = (chunk / n_groups) * kR;
  const int t_begin = (chunk % n_groups) * kWgTiles, t_end = min(t_begin + kWgTiles, n_tiles);
  // two tiles' staging registers: a tile's loads are issued two tiles ahead
  struct Stage {
    uint4 gv[kGPer][2], xv[kXPer][2];
  };
  Stage st[2];
  auto fetch = [&](Stage& S, int u0) {
#pragma unroll
    for (int k = 0; k < kGPer; ++k) {
      const int it = (int)threadIdx.x + k * kWgThreads;
      const int pp = it % 16, c8 = (it / 16) % (CO / 8), r = it / (16 * (CO / 8));
      const int v = v0 + r;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int u = u0 + 2 * pp + e;
        S.gv[k][e] = make_uint4(0u, 0u, 0u, 0u);
        if (it < kGItems && u < W && v < H)
          S.gv[k][e] = *reinterpret_cast<const uint4*>(g + ((size_t)v * W + u) * CO + c8 * 8);
      }
    }
#pragma unroll
    for (int k = 0; k < kXPer; ++k) {
      const int it = (int)threadIdx.x + k * kWgThreads;
      const int pp = it % 16, c8 = (it / 16) % (CI / 8), rest = it / (16 * (CI / 8));
      const int r = rest % (kR + 2), d = rest / (kR + 2);
      const int v = v0 - 1 + r;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int u = u0 + 2 * pp + e + d - 1;
        S.xv[k][e] = make_uint4(0u, 0u, 0u, 0u);
        if (it < kXItems && u >= 0 && u < W && v >= 0 && v < H)
          S.xv[k][e] = *reinterpret_cast<const uint4*>(x + ((size_t)v * W + u) * CI + c8 * 8);
      }
    }
  };
  // a pixel pair's 8 channels as 8 words (channel j of both pixels), channel-major
  auto put = [](uint16_t* base, int stride, const uint4 (&pv)[2]) {
    const uint32_t a[4] = {pv[0].x, pv[0].y, pv[0].z, pv[0].w}, b[4] = {pv[1].x, pv[1].y, pv[1].z, pv[1].w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *reinterpret_cast<uint32_t*>(base + (2 * q) * stride) = (a[q] & 0xffffu) | (b[q] << 16);
      *reinterpret_cast<uint32_t*>(base + (2 * q + 1) * stride) = (a[q] >> 16) | (b[q] & 0xffff0000u);
    }
  };
  // the staged tile into LDS, between barriers (the previous tile's fragments are read first)
  auto stage = [&](const Stage& S) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kGPer; ++k) {
      const int it = (int)threadIdx.x + k * kWgThreads;
      if (it < kGItems) {
        const int pp = it % 16, c8 = (it / 16) % (CO / 8), r = it / (16 * (CO / 8));
        put(gT + (size_t)(c8 * 8) * kSG + r * 32 + 2 * pp, kSG, S.gv[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < kXPer; ++k) {
      const int it = (int)threadIdx.x + k * kWgThreads;
      if (it < kXItems) {
        const int pp = it % 16, c8 = (it / 16) % (CI / 8), rest = it / (16 * (CI / 8));
        const int r = rest % (kR + 2), d = rest / (kR + 2);
        put(xT + (size_t)(d * CI + c8 * 8) * kSX + r * 32 + 2 * pp, kSX, S.xv[k]);
      }
    }
    __syncthreads();
  };
  f32x4 acc[kTaps][kMB];
#pragma unroll
  for (int q = 0; q < kTaps; ++q)
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb) acc[q][mb] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum[kMB];
#pragma unroll
  for (int mb = 0; mb < kMB; ++mb) bsum[mb] = 0.f;
  auto products = [&]() {
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      bf16x8 a[kMB];
#pragma unroll
      for (int mb = 0; mb < kMB; ++mb) a[mb] = load8(gT + (size_t)(mb * 16 + m) * kSG + r * 32 + grp * 8);
      if (wv == 0) {
#pragma unroll
        for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
          for (int j = 0; j < 8; ++j) bsum[mb] += (float)a[mb][j];
      }
#pragma unroll
      for (int q = 0; q < kTaps; ++q) {
        const int tap = tg + q * kTG;
        if (tap < 9) {
          const int dy = tap / 3 - 1, d = tap % 3;
          const bf16x8 b = load8(xT + (size_t)(d * CI + nb * 16 + m) * kSX + (r + 1 + dy) * 32 + grp * 8);
#pragma unroll
          for (int mb = 0; mb < kMB; ++mb)
            acc[q][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mb], b, acc[q][mb], 0, 0, 0);
        }
      }
    }
  };
  const int nt = t_end - t_begin;
  if (nt > 0) fetch(st[0], t_begin * 32);
  if (nt > 1) fetch(st[1], (t_begin + 1) * 32);
  for (int q = 0; q < nt; q += 2) {
    stage(st[0]);
    if (q + 2 < nt) fetch(st[0], (t_begin + q + 2) * 32);
    products();
    if (q + 1 < nt) {
      stage(st[1]);
      if (q + 3 < nt) fetch(st[1], (t_begin + q + 3) * 32);
      products();
    }
  }
  // D[4 grp + i][m] of block (mb, nb): output channel mb 16 + 4 grp + i, input nb 16 + m
#pragma unroll
  for (int q = 0; q < kTaps; ++q) {
    const int tap = tg + q * kTG;
    if (tap < 9) {
#pragma unroll
      for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          part_w[(((size_t)chunk * 9 + tap) * CO + mb * 16 + grp * 4 + i) * CI + nb * 16 + m] = acc[q][mb][i];
    }
  }
  if (wv == 0) {
#pragma unroll
    for (int mb = 0; mb < kMB; ++mb) {
      float s = bsum[mb];
      s += __shfl_xor(s, 16);
      s += __shfl_xor(s, 32);
      if (lane < 16) part_b[(size_t)chunk * CO + mb * 16 + lane] = s;
    }
  }
}

// Sum of the chunk partials: out[e] = sum over chunks c of part[c n + e].
// Wave s of a workgroup adds the chunks c = s mod 4 in order (loads in
// batches of 16, one memory round trip per batch), then the four sums are
// added in wave order: a fixed order, so the result does not depend on
// scheduling.  64 elements per workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_sum_chunks(const float* __restrict__ part, int n_chunks, int n,
                                                    float* __restrict__ out) {
  constexpr int kBatch = 16;
  __shared__ float red[4][64];
  const int s = threadIdx.x >> 6, e = blockIdx.x * 64 + (threadIdx.x & 63);
  float acc = 0.f;
  if (e < n) {
    for (int c0 = s; c0 < n_chunks; c0 += 4 * kBatch) {
      float v[kBatch];
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int c = c0 + 4 * k;
        v[k] = c < n_chunks ? part[(size_t)c * n + e] : 0.f;
      }
#pragma unroll
      for (int k = 0; k < kBatch; ++k)
        if (c0 + 4 * k < n_chunks) acc += v[k];
    }
  }
  red[s][threadIdx.x & 63] = acc;
  __syncthreads();
  if (s == 0 && e < n) out[e] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

// Plane loss of the output and its gradient (FP64): for every pixel p the
// mean over its 5x5 neighbourhood q (clipped) of |d_p + a_p (u_q - u_p) +
// b_p (v_q - v_p) - d*_q|, averaged over pixels; g = dloss/dy in BF16
// (channels 0..2; the others 0).  Per-block loss partial sums in FP64.
__global__ void k_net_loss(const float* __restrict__ y, const float4* __restrict__ target, int W, int H,
                           double disp_max, uint16_t* __restrict__ g, double* __restrict__ part) {
  __shared__ double red[256];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (p < W * H) {
    const int u = p % W, v = p / W;
    const double a = y[(size_t)p * 16 + 0], b = y[(size_t)p * 16 + 1];
    const double d = (double)y[(size_t)p * 16 + 2] * disp_max;
    double ga = 0.0, gb = 0.0, gd = 0.0, tot = 0.0;
    int cnt = 0;
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        const int qu = u + dx, qv = v + dy;
        if (qu < 0 || qu >= W || qv < 0 || qv >= H) continue;
        const float4 t = target[(size_t)qv * W + qu];
        const double dt = ((double)t.x * (double)qu + (double)t.y * (double)qv) + (double)t.z;
        const double r = ((d + a * dx) + b * dy) - dt;
        const double s = r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0);
        tot += fabs(r);
        gd += s;
        ga += s * dx;
        gb += s * dy;
        ++cnt;
      }
    const double n = (double)W * H;
    l = tot / cnt;
    uint16_t* gp = g + (size_t)p * 16;
    gp[0] = to_bf16((float)(ga / cnt / n));
    gp[1] = to_bf16((float)(gb / cnt / n));
    gp[2] = to_bf16((float)(gd / cnt / n * disp_max));
    for (int c = 3; c < 16; ++c) gp[c] = 0;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam on the FP32 master parameters (n of them, the first n_w weights of
// a layer laid out [tap][out][in]); refreshes the BF16 copies of the weights
// in [tap][out][in] and [tap][in][out] order.
__global__ void k_net_adam(float* __restrict__ prm, const float* __restrict__ grad, float* __restrict__ m1,
                           float* __restrict__ m2, int n, int n_w, int co, int ci, float lr, float c1, float c2,
                           uint16_t* __restrict__ w16, uint16_t* __restrict__ wt16) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float g = grad[e];
  const float a = 0.9f * m1[e] + 0.1f * g;
  const float b = 0.999f * m2[e] + 0.001f * (g * g);
  m1[e] = a;
  m2[e] = b;
  const float mh = a / c1, vh = b / c2;
  const float w = prm[e] - lr * mh / (sqrtf(vh) + 1e-8f);
  prm[e] = w;
  if (e < n_w) {
    const int tap = e / (co * ci), r = e % (co * ci), o = r / ci, i = r % ci;
    const uint16_t h = to_bf16(w);
    w16[e] = h;
    wt16[((size_t)tap * ci + i) * co + o] = h;
  }
}

// BF16 copies of a layer's weights (after they are set).
__global__ void k_net_w16(const float* __restrict__ prm, int n_w, int co, int ci, uint16_t* __restrict__ w16,
                          uint16_t* __restrict__ wt16) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_w) return;
  const int tap = e / (co * ci), r = e % (co * ci), o = r / ci, i = r % ci;
  const uint16_t h = to_bf16(prm[e]);
  w16[e] = h;
  wt16[((size_t)tap * ci + i) * co + o] = h;
}

// Candidate planes of the output: (a, b, d disp_max - a u - b v), FP64, one float4 per pixel.
__global__ void k_net_planes(const float* __restrict__ y, int W, int H, double disp_max,
                             float4* __restrict__ planes) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= W * H) return;
  const int u = p % W, v = p / W;
  const double a = y[(size_t)p * 16], b = y[(size_t)p * 16 + 1];
  const double c = ((double)y[(size_t)p * 16 + 2] * disp_max - a * u) - b * v;
  planes[p] = make_float4((float)a, (float)b, (float)c, 0.f);
}

template __global__ void k_conv_fwd<16, 32, false>(const uint16_t*, const uint16_t*, const float*, int, int,
                                                   uint16_t*, float*);
template __global__ void k_conv_fwd<32, 32, false>(const uint16_t*, const uint16_t*, const float*, int, int,
                                                   uint16_t*, float*);
template __global__ void k_conv_fwd<32, 16, true>(const uint16_t*, const uint16_t*, const float*, int, int,
                                                  uint16_t*, float*);
template __global__ void k_conv_bwd_x<32, 32>(const uint16_t*, const uint16_t*, const uint16_t*, int, int,
                                              uint16_t*);
template __global__ void k_conv_bwd_x<32, 16>(const uint16_t*, const uint16_t*, const uint16_t*, int, int,
                                              uint16_t*);
template __global__ void k_conv_bwd_w<16, 32>(const uint16_t*, const uint16_t*, int, int, float*, float*);
template __global__ void k_conv_bwd_w<32, 32>(const uint16_t*, const uint16_t*, int, int, float*, float*);
template __global__ void k_conv_bwd_w<32, 16>(const uint16_t*, const uint16_t*, int, int, float*, float*);

}  // namespace lexp
