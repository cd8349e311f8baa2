// Learned proposal network on CDNA4 (gfx950): five 3x3 convolutions as
// implicit GEMMs on the BF16 matrix cores (v_mfma_f32_16x16x16_bf16, FP32
// sums), their backward passes, the plane loss and Adam.
//
// Layout: activations and gradients pixel-major (index (v W + u) C + c), BF16;
// the last layer's output FP32; weights [tap][out][in] (tap = 3 ky + kx,
// offset (kx-1, ky-1)) with a BF16 copy in that order and one in
// [tap][in][out] for the backward-data products.
//
// One matrix instruction computes one 16 x 16 block of a product.
// Operand fragments (checked on the device): lane l holds A[l % 16][4 (l/16)
// + i] and B[4 (l/16) + i][l % 16] for i < 4, and receives
// D[4 (l/16) + i][l % 16].
//   forward     : M = 16 pixels of a row, N = output channels, K = 9 taps x
//                 input channels (a wave takes four such blocks of a row);
//   backward x  : M = 16 pixels, N = input channels, K = 9 taps x output
//                 channels (gradient at p - offset; four blocks per wave);
//   backward w  : per tap, M = output channels, N = input channels, K = the
//                 pixels of a chunk; chunk partial sums are added in chunk
//                 order by a second kernel (the result does not depend on
//                 scheduling).
// BF16 values are rounded to nearest even from FP32 (FP64 values through
// FP32 first), at the points listed in the reference's description.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lexp_device.h"

namespace lexp {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite values)
  return (uint16_t)(u >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline bf16x4 load4(const uint16_t* p) {
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  bf16x4 r;
  r[0] = (short)(v.x & 0xffffu);
  r[1] = (short)(v.x >> 16);
  r[2] = (short)(v.y & 0xffffu);
  r[3] = (short)(v.y >> 16);
  return r;
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
// once and used for all of them.
constexpr int kSegs = 4;

// Patch of a pixel-major BF16 map with C channels that a workgroup's four
// rows v0..v0+3 of one run of kSegs x 16 columns read through 3x3 taps: rows
// v0-1..v0+4, columns u0-1..u0+16 kSegs, zero outside the image, a pixel's
// channels kPatchPad elements apart (the 16 pixels of a fragment then fall in
// distinct LDS banks).  Coalesced 16-byte loads, 8-byte LDS stores.
constexpr int kPatchW = 16 * kSegs + 2;
constexpr int kPatchR = 4 + 2;
constexpr int kPatchPad = 4;

template <int C>
__device__ inline void stage_patch(const uint16_t* __restrict__ src, int W, int H, int u0, int v0,
                                   uint16_t* patch) {
  constexpr int kPS = C + kPatchPad;
  constexpr int kPieces = C / 8;
  for (int i = threadIdx.x; i < kPatchR * kPatchW * kPieces; i += blockDim.x) {
    const int pc = i % kPieces, px = i / kPieces;
    const int col = px % kPatchW, row = px / kPatchW;
    const int yy = v0 - 1 + row, xx = u0 - 1 + col;
    uint4 val = make_uint4(0u, 0u, 0u, 0u);
    if (yy >= 0 && yy < H && xx >= 0 && xx < W)
      val = *reinterpret_cast<const uint4*>(src + ((size_t)yy * W + xx) * C + pc * 8);
    uint2* dst = reinterpret_cast<uint2*>(patch + (size_t)px * kPS + pc * 8);
    dst[0] = make_uint2(val.x, val.y);
    dst[1] = make_uint2(val.z, val.w);
  }
}

// A layer's BF16 weights, rows of K elements ([tap][row][K] for 9 x R rows),
// copied to LDS with rows K+4 elements apart (the 16 rows of a fragment then
// fall in distinct banks).
template <int R, int K>
__device__ inline void stage_weights(const uint16_t* __restrict__ w, uint16_t* ws) {
  constexpr int kPieces = K / 8;
  for (int i = threadIdx.x; i < 9 * R * kPieces; i += blockDim.x) {
    const int row = i / kPieces, pc = i % kPieces;
    const uint4 val = *reinterpret_cast<const uint4*>(w + (size_t)row * K + pc * 8);
    uint2* dst = reinterpret_cast<uint2*>(ws + (size_t)row * (K + 4) + pc * 8);
    dst[0] = make_uint2(val.x, val.y);
    dst[1] = make_uint2(val.z, val.w);
  }
}

// Forward convolution of one layer.  A workgroup takes four rows v0..v0+3 of
// one run of kSegs x 16 columns: it stages the input patch those rows read and
// the layer's weights in LDS, then each wave computes one row of the run (all
// output channels) from LDS fragments.  Bias, then ReLU and BF16 (hidden layers) or FP32 output
// (last layer).
template <int CI, int CO, bool LAST>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w16,
                                                  const float* __restrict__ bias, int W, int H,
                                                  uint16_t* __restrict__ xo, float* __restrict__ yo) {
  constexpr int kPW = kPatchW, kPS = CI + kPatchPad;
  __shared__ __align__(16) uint16_t patch[kPatchR * kPatchW * kPS];
  __shared__ __align__(16) uint16_t wsh[9 * CO * (CI + 4)];
  const int nrun = (W + 16 * kSegs - 1) / (16 * kSegs);
  const int u0 = (blockIdx.x % nrun) * 16 * kSegs, v0 = (blockIdx.x / nrun) * 4;
  stage_patch<CI>(x, W, H, u0, v0, patch);
  stage_weights<CO, CI>(w16, wsh);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int v = v0 + wv;
  if (v >= H) return;
  const int m = lane & 15, kq = (lane >> 4) * 4;
  f32x4 acc[kSegs][CO / 16];
#pragma unroll
  for (int sg = 0; sg < kSegs; ++sg)
#pragma unroll
    for (int nb = 0; nb < CO / 16; ++nb) acc[sg][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int prow = wv + tap / 3;  // patch row of image row v + tap/3 - 1
#pragma unroll
    for (int cb = 0; cb < CI / 16; ++cb) {
      bf16x4 b[CO / 16];
#pragma unroll
      for (int nb = 0; nb < CO / 16; ++nb) b[nb] = load4(wsh + (tap * CO + nb * 16 + m) * (CI + 4) + cb * 16 + kq);
#pragma unroll
      for (int sg = 0; sg < kSegs; ++sg) {
        // patch column of image column u0 + 16 sg + m + tap%3 - 1
        const bf16x4 a = load4(patch + ((size_t)prow * kPW + sg * 16 + m + tap % 3) * kPS + cb * 16 + kq);
#pragma unroll
        for (int nb = 0; nb < CO / 16; ++nb)
          acc[sg][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[nb], acc[sg][nb], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int nb = 0; nb < CO / 16; ++nb) {
    const int co = nb * 16 + m;
    const float bb = bias[co];
#pragma unroll
    for (int sg = 0; sg < kSegs; ++sg)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int u = u0 + sg * 16 + kq + i;
        if (u >= W) continue;
        const size_t p = (size_t)v * W + u;
        const float z = acc[sg][nb][i] + bb;
        if (LAST)
          yo[p * CO + co] = z;
        else
          xo[p * CO + co] = to_bf16(z > 0.f ? z : 0.f);
      }
  }
}

// Gradient of a layer's input: dx(p) = sum over taps and output channels of
// W[tap][o][i] g(p - offset)[o], then gp = BF16(dx * [x(p) > 0]) (the input
// came from a ReLU).  Workgroups as in the forward convolution, with the
// patch of g (the taps mirrored).
template <int CI, int CO>
__global__ __launch_bounds__(256) void k_conv_bwd_x(const uint16_t* __restrict__ g, const uint16_t* __restrict__ wt16,
                                                    const uint16_t* __restrict__ x, int W, int H,
                                                    uint16_t* __restrict__ gp) {
  constexpr int kPW = kPatchW, kPS = CO + kPatchPad;
  __shared__ __align__(16) uint16_t patch[kPatchR * kPatchW * kPS];
  __shared__ __align__(16) uint16_t wsh[9 * CI * (CO + 4)];
  const int nrun = (W + 16 * kSegs - 1) / (16 * kSegs);
  const int u0 = (blockIdx.x % nrun) * 16 * kSegs, v0 = (blockIdx.x / nrun) * 4;
  stage_patch<CO>(g, W, H, u0, v0, patch);
  stage_weights<CI, CO>(wt16, wsh);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int v = v0 + wv;
  if (v >= H) return;
  const int m = lane & 15, kq = (lane >> 4) * 4;
  f32x4 acc[kSegs][CI / 16];
#pragma unroll
  for (int sg = 0; sg < kSegs; ++sg)
#pragma unroll
    for (int nb = 0; nb < CI / 16; ++nb) acc[sg][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int prow = wv + 2 - tap / 3;  // patch row of image row v - (tap/3 - 1)
#pragma unroll
    for (int cb = 0; cb < CO / 16; ++cb) {
      bf16x4 b[CI / 16];
#pragma unroll
      for (int nb = 0; nb < CI / 16; ++nb) b[nb] = load4(wsh + (tap * CI + nb * 16 + m) * (CO + 4) + cb * 16 + kq);
#pragma unroll
      for (int sg = 0; sg < kSegs; ++sg) {
        // patch column of image column u0 + 16 sg + m - (tap%3 - 1)
        const bf16x4 a = load4(patch + ((size_t)prow * kPW + sg * 16 + m + 2 - tap % 3) * kPS + cb * 16 + kq);
#pragma unroll
        for (int nb = 0; nb < CI / 16; ++nb)
          acc[sg][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[nb], acc[sg][nb], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int nb = 0; nb < CI / 16; ++nb) {
    const int ci = nb * 16 + m;
#pragma unroll
    for (int sg = 0; sg < kSegs; ++sg)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int u = u0 + sg * 16 + kq + i;
        if (u >= W) continue;
        const size_t p = (size_t)v * W + u;
        const uint16_t xv = x[p * CI + ci];
        const bool pos = (xv & 0x8000u) == 0 && xv != 0;
        gp[p * CI + ci] = to_bf16(pos ? acc[sg][nb][i] : 0.f);
      }
  }
}

// Weight and bias gradients of one layer, partial sums per pixel chunk:
// part_w[chunk][tap][o][i] = sum over the chunk's pixels p of g(p)[o]
// x(p + offset(tap))[i]; part_b[chunk][o] (tap-0 workgroups) = sum of g(p)[o].
// Grid (chunks, 9 taps).  The chunk goes through LDS in tiles of kTile
// pixels (g and the shifted x, pixel-major, coalesced 16-byte loads, the next
// tile's loads in flight during this tile's products); wave w takes the
// 16-pixel blocks w, w+4, ... of the chunk, in order.
template <int CI, int CO>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const uint16_t* __restrict__ g, const uint16_t* __restrict__ x,
                                                    int W, int H, int chunk_px, float* __restrict__ part_w,
                                                    float* __restrict__ part_b) {
  constexpr int kTile = 256;
  constexpr int kGS = CO + 8, kXS = CI + 8;  // LDS elements per pixel (16-byte aligned rows)
  constexpr int kGP = kTile * CO / 8 / 256, kXP = kTile * CI / 8 / 256;  // 16-byte pieces per thread
  __shared__ __align__(16) uint16_t gs[kTile * kGS];
  __shared__ __align__(16) uint16_t xs[kTile * kXS];
  __shared__ float red[4][CO * CI];
  __shared__ float redb[4][CO];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int chunk = blockIdx.x, tap = blockIdx.y;
  const int P = W * H;
  const int p0 = chunk * chunk_px, p1 = min(p0 + chunk_px, P);
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  const int m = lane & 15, kq = (lane >> 4) * 4;
  uint4 gv[kGP], xv[kXP];
  auto fetch = [&](int t0) {
#pragma unroll
    for (int k = 0; k < kGP; ++k) {
      const int piece = threadIdx.x + k * 256;
      const int p = t0 + piece / (CO / 8), c8 = piece % (CO / 8);
      gv[k] = p < p1 ? *reinterpret_cast<const uint4*>(g + (size_t)p * CO + c8 * 8) : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int k = 0; k < kXP; ++k) {
      const int piece = threadIdx.x + k * 256;
      const int p = t0 + piece / (CI / 8), c8 = piece % (CI / 8);
      const int u = p % W, v = p / W;
      const int xx = u + dx, yy = v + dy;
      const bool in = p < p1 && xx >= 0 && xx < W && yy >= 0 && yy < H;
      xv[k] = in ? *reinterpret_cast<const uint4*>(x + ((size_t)yy * W + xx) * CI + c8 * 8)
                 : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  f32x4 acc[CO / 16][CI / 16];
#pragma unroll
  for (int mb = 0; mb < CO / 16; ++mb)
#pragma unroll
    for (int nb = 0; nb < CI / 16; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum[CO / 16];
#pragma unroll
  for (int mb = 0; mb < CO / 16; ++mb) bsum[mb] = 0.f;
  fetch(p0);
  for (int t0 = p0; t0 < p1; t0 += kTile) {
    __syncthreads();  // the previous tile's fragments are read
#pragma unroll
    for (int k = 0; k < kGP; ++k) {
      const int piece = threadIdx.x + k * 256;
      *reinterpret_cast<uint4*>(gs + (piece / (CO / 8)) * kGS + (piece % (CO / 8)) * 8) = gv[k];
    }
#pragma unroll
    for (int k = 0; k < kXP; ++k) {
      const int piece = threadIdx.x + k * 256;
      *reinterpret_cast<uint4*>(xs + (piece / (CI / 8)) * kXS + (piece % (CI / 8)) * 8) = xv[k];
    }
    __syncthreads();
    if (t0 + kTile < p1) fetch(t0 + kTile);
    for (int bl = wave; bl < kTile / 16 && t0 + bl * 16 < p1; bl += 4) {
      // this lane's four pixels of the block (zero past the chunk)
      bf16x4 a[CO / 16], b[CI / 16];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int px = bl * 16 + kq + i;
#pragma unroll
        for (int mb = 0; mb < CO / 16; ++mb) {
          const uint16_t gq = gs[px * kGS + mb * 16 + m];
          a[mb][i] = (short)gq;
          if (tap == 0) bsum[mb] += from_bf16(gq);
        }
#pragma unroll
        for (int nb = 0; nb < CI / 16; ++nb) b[nb][i] = (short)xs[px * kXS + nb * 16 + m];
      }
      // A[o][pixel] and B[pixel][i]: lane m is the row of A and the column of B
#pragma unroll
      for (int mb = 0; mb < CO / 16; ++mb)
#pragma unroll
        for (int nb = 0; nb < CI / 16; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mb], b[nb], acc[mb][nb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mb = 0; mb < CO / 16; ++mb)
#pragma unroll
    for (int nb = 0; nb < CI / 16; ++nb)
#pragma unroll
      for (int i = 0; i < 4; ++i) red[wave][(mb * 16 + kq + i) * CI + nb * 16 + m] = acc[mb][nb][i];
  if (tap == 0) {
#pragma unroll
    for (int mb = 0; mb < CO / 16; ++mb) {
      float s = bsum[mb];
      s += __shfl_xor(s, 16);
      s += __shfl_xor(s, 32);
      if (lane < 16) redb[wave][mb * 16 + lane] = s;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < CO * CI; e += 256)
    part_w[((size_t)chunk * 9 + tap) * CO * CI + e] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
  if (tap == 0)
    for (int e = threadIdx.x; e < CO; e += 256)
      part_b[(size_t)chunk * CO + e] = ((redb[0][e] + redb[1][e]) + redb[2][e]) + redb[3][e];
}

// Sum of the chunk partials in chunk order: out[e] = sum_c part[c * n + e].
__global__ void k_sum_chunks(const float* __restrict__ part, int n_chunks, int n, float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float s = 0.f;
  for (int c = 0; c < n_chunks; ++c) s += part[(size_t)c * n + e];
  out[e] = s;
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
template __global__ void k_conv_bwd_w<16, 32>(const uint16_t*, const uint16_t*, int, int, int, float*, float*);
template __global__ void k_conv_bwd_w<32, 32>(const uint16_t*, const uint16_t*, int, int, int, float*, float*);
template __global__ void k_conv_bwd_w<32, 16>(const uint16_t*, const uint16_t*, int, int, int, float*, float*);

}  // namespace lexp
