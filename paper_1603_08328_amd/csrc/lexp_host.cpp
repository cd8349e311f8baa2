// Host-side pieces: random numbers, proposers, Boykov-Kolmogorov max-flow,
// thread pool.  Compiled by the host compiler with -ffp-contract=off so the
// double-precision proposer arithmetic is rounded exactly as written.
#include "lexp_host.h"

#include <sched.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

namespace lexp {

// ---------------------------------------------------------------------------
// SplitMix64 output function (Steele, Lea, Flood 2014) on state x, and the
// key chain h0 = sm64(seed), h_{i+1} = sm64(h_i ^ field_i).
// ---------------------------------------------------------------------------
uint64_t sm64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t key_chain(uint64_t seed, const uint64_t* fields, int n) {
  uint64_t h = sm64(seed);
  for (int i = 0; i < n; ++i) h = sm64(h ^ fields[i]);
  return h;
}

double u01_open1(uint64_t x) { return std::ldexp((double)(x >> 11), -53); }
double u01_open0(uint64_t x) { return std::ldexp((double)((x >> 11) + 1), -53); }

static constexpr uint64_t kTagInit = 1;
static constexpr uint64_t kTagPropose = 2;
static constexpr double kTwoPi = 6.283185307179586;

// Plane through (u, v, z0) whose unit normal n = (nx, ny, nz), nz > 0, is
// uniform on the upper hemisphere: nz ~ U(0,1], azimuth ~ U[0, 2pi).
void init_label(int width, int u, int v, double disp_max, uint64_t seed, float out[3]) {
  uint64_t key[3] = {kTagInit, (uint64_t)v * (uint64_t)width + (uint64_t)u, 0};
  const double z0 = u01_open1(key_chain(seed, key, 3)) * disp_max;
  key[2] = 1;
  const double nz = u01_open0(key_chain(seed, key, 3));
  key[2] = 2;
  const double az = kTwoPi * u01_open1(key_chain(seed, key, 3));
  const double s = std::sqrt(1.0 - nz * nz);
  const double nx = s * std::cos(az);
  const double ny = s * std::sin(az);
  out[0] = (float)(-nx / nz);
  out[1] = (float)(-ny / nz);
  out[2] = (float)((nx * (double)u + ny * (double)v + nz * z0) / nz);
}

static double plane_at(const float* f, int u, int v) {
  const double t1 = (double)f[0] * (double)u;
  const double t2 = (double)f[1] * (double)v;
  const double s = t1 + t2;
  return s + (double)f[2];
}

// RANSAC proposer (Alg. 1): LO-RANSAC (Chum, Matas, Kittler 2003) plane fit
// d = a u + b v + c to the current disparities of the clipped centre cell.
// kRansSamples minimal samples, pixel k of sample m from draw 1 + 3m + k of
// the step's key; a sample with a repeated pixel or collinear pixels is
// skipped.  A sample plane comes from the normal (e1 x e2) of the edge
// vectors from its first point; inliers are within kRansTau in disparity.  A
// sample that beats the best inlier count is refined up to kRansLocal times
// by the least-squares plane of its inliers (centred normal equations), kept
// while the inlier count does not fall.  Returns false when no sample is
// valid.
namespace {

constexpr int kRansSamples = 32;
constexpr double kRansTau = 1.0;
constexpr int kRansLocal = 4;

struct CellPoints {
  std::vector<double> u, v, d;
  int n = 0;

  int count(const double m[3], std::vector<unsigned char>& in) const {
    int k = 0;
    for (int i = 0; i < n; ++i) {
      const double pred = m[0] * u[i] + m[1] * v[i] + m[2];
      in[i] = std::fabs(d[i] - pred) <= kRansTau ? 1 : 0;
      k += in[i];
    }
    return k;
  }

  bool least_squares(const std::vector<unsigned char>& in, double m[3]) const {
    double su = 0.0, sv = 0.0, sd = 0.0;
    int k = 0;
    for (int i = 0; i < n; ++i) {
      if (!in[i]) continue;
      su += u[i];
      sv += v[i];
      sd += d[i];
      ++k;
    }
    if (k < 3) return false;
    const double mu = su / k, mv = sv / k, md = sd / k;
    double suu = 0.0, suv = 0.0, svv = 0.0, sud = 0.0, svd = 0.0;
    for (int i = 0; i < n; ++i) {
      if (!in[i]) continue;
      const double du = u[i] - mu, dv = v[i] - mv, dd = d[i] - md;
      suu += du * du;
      suv += du * dv;
      svv += dv * dv;
      sud += du * dd;
      svd += dv * dd;
    }
    const double det = suu * svv - suv * suv;
    if (!(det > 1e-9 * suu * svv)) return false;
    m[0] = (sud * svv - svd * suv) / det;
    m[1] = (svd * suu - sud * suv) / det;
    m[2] = md - m[0] * mu - m[1] * mv;
    return true;
  }
};

}  // namespace

static bool ransac_plane(int width, const float* labels, int stride, uint64_t seed, uint64_t key[7], int cu0,
                         int cv0, int cw, int chh, float out[3]) {
  CellPoints P;
  P.n = cw * chh;
  if (P.n < 3) return false;
  P.u.resize(P.n);
  P.v.resize(P.n);
  P.d.resize(P.n);
  for (int i = 0; i < P.n; ++i) {
    const int u = cu0 + i % cw, v = cv0 + i / cw;
    P.u[i] = u;
    P.v[i] = v;
    P.d[i] = plane_at(labels + ((size_t)v * width + u) * stride, u, v);
  }
  std::vector<unsigned char> in(P.n), trial(P.n);
  int best = -1;
  double bm[3] = {0.0, 0.0, 0.0};
  for (int m = 0; m < kRansSamples; ++m) {
    int s[3];
    for (int k = 0; k < 3; ++k) {
      key[6] = (uint64_t)(1 + 3 * m + k);
      int64_t idx = (int64_t)(u01_open1(key_chain(seed, key, 7)) * (double)P.n);
      if (idx >= P.n) idx = P.n - 1;
      s[k] = (int)idx;
    }
    if (s[0] == s[1] || s[0] == s[2] || s[1] == s[2]) continue;
    const double e1u = P.u[s[1]] - P.u[s[0]], e1v = P.v[s[1]] - P.v[s[0]], e1d = P.d[s[1]] - P.d[s[0]];
    const double e2u = P.u[s[2]] - P.u[s[0]], e2v = P.v[s[2]] - P.v[s[0]], e2d = P.d[s[2]] - P.d[s[0]];
    const double nu = e1v * e2d - e1d * e2v;
    const double nv = e1d * e2u - e1u * e2d;
    const double nd = e1u * e2v - e1v * e2u;
    if (nd == 0.0) continue;
    double mdl[3];
    mdl[0] = -nu / nd;
    mdl[1] = -nv / nd;
    mdl[2] = P.d[s[0]] - mdl[0] * P.u[s[0]] - mdl[1] * P.v[s[0]];
    int cnt = P.count(mdl, in);
    if (cnt <= best) continue;
    for (int r = 0; r < kRansLocal; ++r) {
      double ls[3];
      if (!P.least_squares(in, ls)) break;
      const int c2 = P.count(ls, trial);
      if (c2 < cnt) break;
      mdl[0] = ls[0];
      mdl[1] = ls[1];
      mdl[2] = ls[2];
      in.swap(trial);
      cnt = c2;
    }
    best = cnt;
    bm[0] = mdl[0];
    bm[1] = mdl[1];
    bm[2] = mdl[2];
  }
  if (best < 0) return false;
  out[0] = (float)bm[0];
  out[1] = (float)bm[1];
  out[2] = (float)bm[2];
  return true;
}

void propose(int width, int height, const float* labels, int stride, uint64_t seed, int iteration, int level,
             int cell, int ci, int cj, int step, int k_prop, int k_rans, double r_d, double r_n, float out[3],
             const float* net_planes, const float* label_at_r) {
  const int cu0 = ci * cell, cv0 = cj * cell;
  const int cw = std::min(cu0 + cell, width) - cu0;
  const int chh = std::min(cv0 + cell, height) - cv0;
  uint64_t key[7] = {kTagPropose, (uint64_t)iteration, (uint64_t)level, (uint64_t)ci,
                     (uint64_t)cj, (uint64_t)step, 0};
  const int64_t npx = (int64_t)cw * chh;
  int64_t idx = (int64_t)(u01_open1(key_chain(seed, key, 7)) * (double)npx);
  if (idx >= npx) idx = npx - 1;
  const int ru = cu0 + (int)(idx % cw);
  const int rv = cv0 + (int)(idx / cw);
  const float* fr = label_at_r ? label_at_r : labels + ((size_t)rv * width + ru) * stride;
  if (step < k_prop || (step < k_prop + k_rans && !ransac_plane(width, labels, stride, seed, key, cu0, cv0, cw, chh,
                                                                   out))) {
    out[0] = fr[0]; out[1] = fr[1]; out[2] = fr[2];
    return;
  }
  if (step < k_prop + k_rans) return;
  if (net_planes && ((step - k_prop - k_rans) & 1)) {  // learned refinement step
    const float* g = net_planes + ((size_t)rv * width + ru) * 4;
    out[0] = g[0]; out[1] = g[1]; out[2] = g[2];
    return;
  }
  double rd = r_d, rn = r_n;
  for (int k = 0; k < step - k_prop - k_rans; ++k) { rd *= 0.5; rn *= 0.5; }
  key[6] = 1;
  const double dd = (2.0 * u01_open1(key_chain(seed, key, 7)) - 1.0) * rd;
  key[6] = 2;
  const double z = 2.0 * u01_open1(key_chain(seed, key, 7)) - 1.0;
  key[6] = 3;
  const double az = kTwoPi * u01_open1(key_chain(seed, key, 7));
  const double s = std::sqrt(1.0 - z * z);
  const double dn[3] = {rn * (s * std::cos(az)), rn * (s * std::sin(az)), rn * z};
  const double a = fr[0], b = fr[1];
  const double d = plane_at(fr, ru, rv);
  const double len = std::sqrt(a * a + b * b + 1.0);
  const double n0[3] = {-a / len, -b / len, 1.0 / len};
  double n1[3] = {n0[0] + dn[0], n0[1] + dn[1], n0[2] + dn[2]};
  const double l1 = std::sqrt(n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
  n1[0] /= l1; n1[1] /= l1; n1[2] /= l1;
  if (!(std::fabs(n1[2]) >= 1e-3)) { n1[0] = n0[0]; n1[1] = n0[1]; n1[2] = n0[2]; }
  const double d1 = d + dd;
  out[0] = (float)(-n1[0] / n1[2]);
  out[1] = (float)(-n1[1] / n1[2]);
  out[2] = (float)((n1[0] * (double)ru + n1[1] * (double)rv + n1[2] * d1) / n1[2]);
  (void)height;
}

// ---------------------------------------------------------------------------
// Boykov-Kolmogorov max-flow (Boykov & Kolmogorov, "An experimental
// comparison of min-cut/max-flow algorithms for energy minimization in
// vision", TPAMI 2004): two search trees grown from the terminals, augmenting
// along the first path found, then adoption of orphans.  Arcs of node i are
// indexed by direction k: (1,0), (0,1), (1,1), (-1,1), (-1,0), (0,-1),
// (-1,-1), (1,-1); the reverse of direction k is k ^ 4.
// ---------------------------------------------------------------------------
static const int kDU[8] = {1, 0, 1, -1, -1, 0, -1, 1};
static const int kDV[8] = {0, 1, 1, 1, 0, -1, -1, -1};

template <class V>
static void reset(std::vector<V>& v, size_t n, V val) {
  if (v.size() < n) v.resize(n);
  std::fill(v.begin(), v.begin() + n, val);
}

template <class T>
void BKSolver::load(int w, int h, int nf, const T* U, int u_stride, const T* w4, int w_stride) {
  w_ = w; h_ = h; nf_ = nf;
  pw_ = w + 2;
  pn_ = (w + 2) * (h + 2);
  ndirs_ = 0;
  for (int k = 0; k < nf; ++k) dirs_[ndirs_++] = k;
  for (int k = 0; k < nf; ++k) dirs_[ndirs_++] = k ^ 4;
  for (int k = 0; k < 8; ++k) off_[k] = kDV[k] * pw_ + kDU[k];
  reset(tr_, (size_t)pn_, 0);
  reset(rc_, (size_t)pn_ * 8, 0);
  for (int v = 0; v < h; ++v)
    for (int u = 0; u < w; ++u) {
      const size_t q = (size_t)v * w + u;
      const int i = (v + 1) * pw_ + (u + 1);
      tr_[i] = -(int32_t)U[q * u_stride];  // U > 0: residual i->t; U < 0: residual s->i
      for (int d = 0; d < nf; ++d) {
        const int nu = u + kDU[d], nv = v + kDV[d];
        if (nu < 0 || nu >= w || nv < 0 || nv >= h) continue;
        const int32_t c = (int32_t)w4[q * w_stride + d];
        if (c > 0) rc_[(size_t)(i + off_[d]) * 8 + (d ^ 4)] = c;  // arc n -> i: paid when x_n = 1, x_i = 0
      }
    }
}

template void BKSolver::load<int64_t>(int, int, int, const int64_t*, int, const int64_t*, int);
template void BKSolver::load<int32_t>(int, int, int, const int32_t*, int, const int32_t*, int);

void BKSolver::push_active(int i) {
  if (in_active_[i]) return;
  in_active_[i] = 1;
  active_[a_tail_] = i;
  a_tail_ = a_tail_ + 1 == a_cap_ ? 0 : a_tail_ + 1;
}

void BKSolver::make_orphan(int i) {
  parent_[i] = kOrphan;
  orphans_.push_back(i);
}

void BKSolver::augment(int a, int k, int b) {
  int32_t f = rc_[(size_t)a * 8 + k];
  for (int i = a;;) {  // source side: tree arcs parent -> child
    const int p = parent_[i];
    if (p == kTerm) { f = std::min(f, tr_[i]); break; }
    const int j = i + off_[p];
    f = std::min(f, rc_[(size_t)j * 8 + (p ^ 4)]);
    i = j;
  }
  for (int i = b;;) {  // sink side: tree arcs child -> parent
    const int p = parent_[i];
    if (p == kTerm) { f = std::min(f, -tr_[i]); break; }
    f = std::min(f, rc_[(size_t)i * 8 + p]);
    i += off_[p];
  }
  rc_[(size_t)a * 8 + k] -= f;
  rc_[(size_t)b * 8 + (k ^ 4)] += f;
  for (int i = a;;) {
    const int p = parent_[i];
    if (p == kTerm) {
      tr_[i] -= f;
      if (tr_[i] == 0) make_orphan(i);
      break;
    }
    const int j = i + off_[p];
    rc_[(size_t)j * 8 + (p ^ 4)] -= f;
    rc_[(size_t)i * 8 + p] += f;
    if (rc_[(size_t)j * 8 + (p ^ 4)] == 0) make_orphan(i);
    i = j;
  }
  for (int i = b;;) {
    const int p = parent_[i];
    if (p == kTerm) {
      tr_[i] += f;
      if (tr_[i] == 0) make_orphan(i);
      break;
    }
    const int j = i + off_[p];
    rc_[(size_t)i * 8 + p] -= f;
    rc_[(size_t)j * 8 + (p ^ 4)] += f;
    if (rc_[(size_t)i * 8 + p] == 0) make_orphan(i);
    i = j;
  }
  flow_ += f;
}

void BKSolver::adopt() {
  ++time_;
  while (o_head_ < orphans_.size()) {
    const int i = orphans_[o_head_++];
    const uint8_t t = tree_[i];
    int best_k = -1;
    int best_d = INT_MAX;
    for (int q = 0; q < ndirs_; ++q) {
      const int k = dirs_[q];
      const int j = i + off_[k];
      if (tree_[j] != t) continue;
      const int32_t cap = (t == kS) ? rc_[(size_t)j * 8 + (k ^ 4)] : rc_[(size_t)i * 8 + k];
      if (cap <= 0) continue;
      // does j still lead to its terminal?
      int d = 0;
      int m = j;
      bool ok;
      for (;;) {
        if (ts_[m] == time_) { d += dist_[m]; ok = true; break; }
        ++d;
        const int pm = parent_[m];
        if (pm == kTerm) { ts_[m] = time_; dist_[m] = 1; ok = true; break; }
        if (pm == kOrphan || pm == kNone) { ok = false; break; }
        m += off_[pm];
      }
      if (!ok) continue;
      if (d < best_d) { best_d = d; best_k = k; }
      int dd = d;
      for (m = j; ts_[m] != time_; m += off_[parent_[m]]) {
        ts_[m] = time_;
        dist_[m] = dd--;
      }
    }
    if (best_k >= 0) {
      parent_[i] = (int8_t)best_k;
      ts_[i] = time_;
      dist_[i] = best_d + 1;
      continue;
    }
    // no valid parent: i becomes free; its neighbours in the tree that can
    // reach it become active, its children become orphans.
    for (int q = 0; q < ndirs_; ++q) {
      const int k = dirs_[q];
      const int j = i + off_[k];
      if (tree_[j] != t) continue;
      const int32_t cap = (t == kS) ? rc_[(size_t)j * 8 + (k ^ 4)] : rc_[(size_t)i * 8 + k];
      if (cap > 0) push_active(j);
      if (parent_[j] == (k ^ 4)) make_orphan(j);
    }
    tree_[i] = kFree;
    parent_[i] = kNone;
  }
  orphans_.clear();
  o_head_ = 0;
}

void BKSolver::solve(uint8_t* x) {
  flow_ = 0;
  // Saturate the length-one paths s -> i -> j -> t first, in one linear pass:
  // most augmentations of these small grids are of this kind, and pushing
  // them here spares the search trees their bookkeeping.  The search below
  // then completes a maximum flow from this residual graph.
  for (int v = 0; v < h_; ++v)
    for (int u = 0; u < w_; ++u) {
      const int i = (v + 1) * pw_ + (u + 1);
      for (int q = 0; q < ndirs_ && tr_[i] > 0; ++q) {
        const int k = dirs_[q];
        const int j = i + off_[k];
        const int32_t c = rc_[(size_t)i * 8 + k];
        if (c <= 0 || tr_[j] >= 0) continue;
        const int32_t f = std::min(std::min(tr_[i], c), -tr_[j]);
        tr_[i] -= f;
        tr_[j] += f;
        rc_[(size_t)i * 8 + k] -= f;
        rc_[(size_t)j * 8 + (k ^ 4)] += f;
        flow_ += f;
      }
    }
  time_ = 0;
  reset(parent_, (size_t)pn_, (int8_t)kNone);
  reset(tree_, (size_t)pn_, (uint8_t)kFree);
  reset(in_active_, (size_t)pn_, (uint8_t)0);
  reset(ts_, (size_t)pn_, 0);
  reset(dist_, (size_t)pn_, 0);
  a_cap_ = (size_t)pn_ + 1;
  if (active_.size() < a_cap_) active_.resize(a_cap_);
  a_head_ = a_tail_ = 0;
  orphans_.clear();
  o_head_ = 0;
  for (int v = 0; v < h_; ++v)
    for (int u = 0; u < w_; ++u) {
      const int i = (v + 1) * pw_ + (u + 1);
      if (tr_[i] > 0) { tree_[i] = kS; parent_[i] = kTerm; dist_[i] = 1; push_active(i); }
      else if (tr_[i] < 0) { tree_[i] = kT; parent_[i] = kTerm; dist_[i] = 1; push_active(i); }
    }
  for (;;) {
    int a = -1, b = -1, k_ab = -1;
    while (a_head_ != a_tail_) {
      const int i = active_[a_head_];
      if (tree_[i] == kFree) {
        a_head_ = a_head_ + 1 == a_cap_ ? 0 : a_head_ + 1;
        in_active_[i] = 0;
        continue;
      }
      if (tree_[i] == kS) {
        for (int q = 0; q < ndirs_; ++q) {
          const int k = dirs_[q];
          if (rc_[(size_t)i * 8 + k] <= 0) continue;
          const int j = i + off_[k];
          if (tree_[j] == kFree) {
            tree_[j] = kS; parent_[j] = (int8_t)(k ^ 4); ts_[j] = ts_[i]; dist_[j] = dist_[i] + 1;
            push_active(j);
          } else if (tree_[j] == kT) {
            a = i; b = j; k_ab = k;
            break;
          }
        }
      } else {
        for (int q = 0; q < ndirs_; ++q) {
          const int k = dirs_[q];
          const int j = i + off_[k];
          if (rc_[(size_t)j * 8 + (k ^ 4)] <= 0) continue;
          if (tree_[j] == kFree) {
            tree_[j] = kT; parent_[j] = (int8_t)(k ^ 4); ts_[j] = ts_[i]; dist_[j] = dist_[i] + 1;
            push_active(j);
          } else if (tree_[j] == kS) {
            a = j; b = i; k_ab = k ^ 4;
            break;
          }
        }
      }
      if (a >= 0) break;  // i stays at the head of the queue
      a_head_ = a_head_ + 1 == a_cap_ ? 0 : a_head_ + 1;
      in_active_[i] = 0;
    }
    if (a < 0) break;
    augment(a, k_ab, b);
    adopt();
  }
  // source side of the residual graph
  reset(seen_, (size_t)pn_, (uint8_t)0);
  bfs_.clear();
  for (int v = 0; v < h_; ++v)
    for (int u = 0; u < w_; ++u) {
      const int i = (v + 1) * pw_ + (u + 1);
      if (tr_[i] > 0) { seen_[i] = 1; bfs_.push_back(i); }
    }
  for (size_t hd = 0; hd < bfs_.size(); ++hd) {
    const int i = bfs_[hd];
    for (int q = 0; q < ndirs_; ++q) {
      const int k = dirs_[q];
      const int j = i + off_[k];
      if (!seen_[j] && rc_[(size_t)i * 8 + k] > 0) { seen_[j] = 1; bfs_.push_back(j); }
    }
  }
  for (int v = 0; v < h_; ++v)
    for (int u = 0; u < w_; ++u) x[(size_t)v * w_ + u] = seen_[(v + 1) * pw_ + (u + 1)];
}

// ---------------------------------------------------------------------------
// Thread pool
// ---------------------------------------------------------------------------
ThreadPool::ThreadPool(int n_threads) {
  for (int i = 1; i < n_threads; ++i) workers_.emplace_back([this, i] { worker_loop(i); });
}

ThreadPool::~ThreadPool() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_.store(true);
  }
  cv_start_.notify_all();
  for (auto& t : workers_) t.join();
}

// A worker waits for the next job by polling the generation for up to
// kSpinUs (the method's steps follow each other within that), then sleeps on
// the condition variable: a sleeping worker takes tens of microseconds to
// wake, a polling one a fraction of one.  At most one poller per CPU the
// process may run on, less one, across all pools; the others sleep at once.
// A poller yields its CPU between polls, so a thread with work (a woken
// worker of another pool, the caller) is not kept from running.  The caller
// waits for the workers the same way.
static constexpr double kSpinUs = 2000.0;
static std::atomic<int> g_pollers{0};

static int poller_cap() {
  static const int cap = [] {
    cpu_set_t set;
    const int n = sched_getaffinity(0, sizeof(set), &set) == 0 ? CPU_COUNT(&set)
                                                                 : (int)std::thread::hardware_concurrency();
    return std::max(0, n - 1);
  }();
  return cap;
}

static inline void cpu_pause(int k) {
  if ((k & 15) == 0) {
    sched_yield();
  } else {
#if defined(__x86_64__) || defined(__i386__)
    __builtin_ia32_pause();
#endif
  }
}

void ThreadPool::worker_loop(int id) {
  uint64_t seen = 0;
  for (;;) {
    uint64_t g = generation_.load(std::memory_order_acquire);
    if (g == seen) {
      bool sleep = true;
      if (g_pollers.fetch_add(1, std::memory_order_relaxed) < poller_cap()) {
        const auto t0 = std::chrono::steady_clock::now();
        for (int k = 1;; ++k) {
          g = generation_.load(std::memory_order_acquire);
          if (g != seen || stop_.load(std::memory_order_relaxed)) {
            sleep = false;
            break;
          }
          cpu_pause(k);
          if ((k & 127) == 0 &&
              std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count() > kSpinUs)
            break;
        }
      }
      g_pollers.fetch_sub(1, std::memory_order_relaxed);
      if (sleep) {
        std::unique_lock<std::mutex> lk(mu_);
        cv_start_.wait(lk, [&] { return stop_.load() || generation_.load() != seen; });
        g = generation_.load(std::memory_order_acquire);
      }
    }
    if (stop_.load(std::memory_order_acquire)) return;
    seen = g;
    const std::function<void(int, int)>* job = job_;
    const int n = n_items_;
    for (int it = next_.fetch_add(1); it < n; it = next_.fetch_add(1)) (*job)(it, id);
    if (pending_.fetch_sub(1, std::memory_order_acq_rel) == 1) {
      std::lock_guard<std::mutex> lk(mu_);
      cv_done_.notify_one();
    }
  }
}

void ThreadPool::parallel_for(int n, const std::function<void(int, int)>& fn) {
  if (n <= 0) return;
  if (workers_.empty() || n == 1) {
    for (int i = 0; i < n; ++i) fn(i, 0);
    return;
  }
  job_ = &fn;
  n_items_ = n;
  next_.store(0, std::memory_order_relaxed);
  pending_.store((int)workers_.size(), std::memory_order_relaxed);
  generation_.fetch_add(1, std::memory_order_release);
  {
    std::lock_guard<std::mutex> lk(mu_);  // orders the new generation before a sleeper's check
  }
  cv_start_.notify_all();
  for (int it = next_.fetch_add(1); it < n; it = next_.fetch_add(1)) fn(it, 0);
  const auto t0 = std::chrono::steady_clock::now();
  for (int k = 1; pending_.load(std::memory_order_acquire) != 0; ++k) {
    cpu_pause(k);
    if ((k & 127) == 0 &&
        std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count() > kSpinUs) {
      std::unique_lock<std::mutex> lk(mu_);
      cv_done_.wait(lk, [&] { return pending_.load(std::memory_order_acquire) == 0; });
      break;
    }
  }
}

}  // namespace lexp
