// Post-processing of the left view and label-frame conversion (CDNA4, gfx950).
//
// The paper finishes with the left-right consistency check and weighted
// median filtering of Bleyer, Rhemann and Rother (2011).  Here:
//   k_pp_check  : disparity of every left pixel; consistent when the right
//                 view's disparity at the matched pixel x = floor(u - d + 1/2)
//                 of its row is within 1 (right labels in the mirrored frame
//                 of the right image);
//   k_pp_fill   : one thread per row: an inconsistent pixel takes, of the
//                 planes of the nearest consistent pixels to its left and
//                 right, the one with the lower disparity at the pixel;
//   k_pp_median : one workgroup per pixel: an inconsistent pixel takes the
//                 weighted median of the filled disparities of its 35x35
//                 window, colour weights exp(-L1 / gamma) quantised down to
//                 multiples of 2^-24, values ordered by (disparity, index) by
//                 a bitonic sort in LDS and the median found on integer
//                 prefix sums (the same choice whatever the summation order).
// Disparities are a u + b v + c in FP64 from the FP32 labels, rounded as
// written (built with -ffp-contract=off).
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <cstdint>

#include "lexp_device.h"

namespace lexp {

namespace {

constexpr int kPpRadius = 17;                           // weighted-median window (2r+1)^2
constexpr int kPpSide = 2 * kPpRadius + 1;
constexpr int kPpSort = 2048;                           // sort size: next power of two above kPpSide^2
constexpr int kPpThreads = 256;
constexpr double kPpWeightQuantum = 16777216.0;         // 2^24
static_assert(kPpSide * kPpSide <= kPpSort, "the sort holds a whole window");

__device__ inline double disp_of(float4 f, int u, int v) {
  const double t1 = (double)f.x * (double)u;
  const double t2 = (double)f.y * (double)v;
  const double s = t1 + t2;
  return s + (double)f.z;
}

}  // namespace

// Label field between a context's frame and its view image's own frame:
// mirror == 0 copies; otherwise out(u, v) is in(W-1-u, v) as the plane of the
// other frame, (a, b, c) -> (-a, b, c + a (W-1)) (c in FP64, rounded once).
__global__ void k_view_labels(const float4* __restrict__ in, float4* __restrict__ out, int W, int H, int mirror) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W * H) return;
  const int u = i % W, v = i / W;
  if (!mirror) {
    out[i] = in[i];
    return;
  }
  const float4 f = in[(size_t)v * W + (W - 1 - u)];
  const double c = (double)f.z + (double)f.x * (double)(W - 1);
  out[i] = make_float4(-f.x, f.y, (float)c, 0.f);
}

__global__ void k_pp_check(const float4* __restrict__ labels_left, const float4* __restrict__ labels_right, int W,
                           int H, double* __restrict__ disp, uint8_t* __restrict__ ok) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W * H) return;
  const int u = i % W, v = i / W;
  const double d = disp_of(labels_left[i], u, v);
  disp[i] = d;
  const double xd = floor((double)u - d + 0.5);
  uint8_t good = 0;
  if (xd >= 0.0 && xd <= (double)(W - 1)) {
    const int um = W - 1 - (int)xd;  // the right pixel in the right view's mirrored frame
    const double dr = disp_of(labels_right[(size_t)v * W + um], um, v);
    good = fabs(d - dr) <= 1.0 ? 1 : 0;
  }
  ok[i] = good;
}

__global__ void k_pp_fill(const float4* __restrict__ labels_left, const double* __restrict__ disp,
                          const uint8_t* __restrict__ ok, int W, int H, int* __restrict__ next_ok,
                          double* __restrict__ fill) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= H) return;
  const size_t row = (size_t)v * W;
  int next = W;  // nearest consistent pixel at or right of u (W: none)
  for (int u = W - 1; u >= 0; --u) {
    if (ok[row + u]) next = u;
    next_ok[row + u] = next;
  }
  int last = -1;  // nearest consistent pixel left of u
  for (int u = 0; u < W; ++u) {
    double f = disp[row + u];
    if (!ok[row + u]) {
      const int ur = u + 1 < W ? next_ok[row + u + 1] : W;
      const bool hl = last >= 0, hr = ur < W;
      if (hl && hr) {
        const double a = disp_of(labels_left[row + last], u, v);
        const double b = disp_of(labels_left[row + ur], u, v);
        f = a <= b ? a : b;
      } else if (hl) {
        f = disp_of(labels_left[row + last], u, v);
      } else if (hr) {
        f = disp_of(labels_left[row + ur], u, v);
      }
    } else {
      last = u;
    }
    fill[row + u] = f;
  }
}

__global__ __launch_bounds__(kPpThreads) void k_pp_median(const float4* __restrict__ left4,
                                                          const double* __restrict__ disp,
                                                          const double* __restrict__ fill,
                                                          const uint8_t* __restrict__ ok, int W, int H,
                                                          double gamma, float* __restrict__ out,
                                                          uint8_t* __restrict__ invalid) {
  __shared__ double val[kPpSort];
  __shared__ int idx[kPpSort];
  __shared__ long long wq[kPpSort];
  __shared__ long long part[kPpThreads];
  __shared__ long long total_w;
  __shared__ int found;
  const int p = blockIdx.x;
  if (p >= W * H) return;
  const int tid = threadIdx.x;
  if (ok[p]) {
    if (tid == 0) {
      out[p] = (float)disp[p];
      if (invalid) invalid[p] = 0;
    }
    return;
  }
  const int u = p % W, v = p / W;
  const int x0 = u - kPpRadius > 0 ? u - kPpRadius : 0, x1 = u + kPpRadius < W - 1 ? u + kPpRadius : W - 1;
  const int y0 = v - kPpRadius > 0 ? v - kPpRadius : 0, y1 = v + kPpRadius < H - 1 ? v + kPpRadius : H - 1;
  const int ww = x1 - x0 + 1, n = ww * (y1 - y0 + 1);
  const float4 cp = left4[p];
  // window in row-major order, padded with (+max, INT_MAX, 0)
  for (int k = tid; k < kPpSort; k += kPpThreads) {
    if (k < n) {
      const int q = (y0 + k / ww) * W + (x0 + k % ww);
      const float4 cq = left4[q];
      const double s = fabs((double)cp.x - (double)cq.x) + fabs((double)cp.y - (double)cq.y) +
                       fabs((double)cp.z - (double)cq.z);
      val[k] = fill[q];
      idx[k] = q;
      wq[k] = (long long)floor(exp(-s / gamma) * kPpWeightQuantum);
    } else {
      val[k] = DBL_MAX;
      idx[k] = INT_MAX;
      wq[k] = 0;
    }
  }
  __syncthreads();
  // bitonic sort by (val, idx), ascending
  for (int k = 2; k <= kPpSort; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = tid; t < kPpSort / 2; t += kPpThreads) {
        const int l = 2 * j * (t / j) + (t % j), r = l + j;
        const bool up = (l & k) == 0;
        const bool gt = val[l] > val[r] || (val[l] == val[r] && idx[l] > idx[r]);
        if (gt == up) {
          const double tv = val[l]; val[l] = val[r]; val[r] = tv;
          const int ti = idx[l]; idx[l] = idx[r]; idx[r] = ti;
          const long long tw = wq[l]; wq[l] = wq[r]; wq[r] = tw;
        }
      }
      __syncthreads();
    }
  // integer prefix sums: each thread owns a run of 8 sorted entries
  constexpr int kRun = kPpSort / kPpThreads;
  long long s = 0;
  for (int k = 0; k < kRun; ++k) s += wq[tid * kRun + k];
  part[tid] = s;
  if (tid == 0) found = INT_MAX;
  __syncthreads();
  if (tid == 0) {
    long long acc = 0;
    for (int t = 0; t < kPpThreads; ++t) {
      const long long x = part[t];
      part[t] = acc;  // exclusive prefix of the runs
      acc += x;
    }
    total_w = acc;
  }
  __syncthreads();
  // the first entry whose cumulative weight reaches half the total (the
  // padding at the end weighs nothing, so it is a window entry)
  long long cum = part[tid];
  for (int k = 0; k < kRun; ++k) {
    cum += wq[tid * kRun + k];
    if (2 * cum >= total_w) {
      atomicMin(&found, tid * kRun + k);
      break;
    }
  }
  __syncthreads();
  if (tid == 0) {
    out[p] = (float)val[found];
    if (invalid) invalid[p] = 1;
  }
}

}  // namespace lexp
