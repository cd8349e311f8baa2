// Host-side pieces: random numbers, proposers, Boykov-Kolmogorov max-flow,
// thread pool.  Compiled by the host compiler with -ffp-contract=off so the
// double-precision proposer arithmetic is rounded exactly as written.
#include "lexp_host.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

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

void propose(int width, int height, const float* labels, int stride, uint64_t seed, int iteration, int level,
             int cell, int ci, int cj, int step, int k_prop, double r_d, double r_n, float out[3]) {
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
  const float* fr = labels + ((size_t)rv * width + ru) * stride;
  if (step < k_prop) {
    out[0] = fr[0]; out[1] = fr[1]; out[2] = fr[2];
    return;
  }
  double rd = r_d, rn = r_n;
  for (int k = 0; k < step - k_prop; ++k) { rd *= 0.5; rn *= 0.5; }
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

template <class T>
void BKSolver::load(int w, int h, int nf, const T* U, int u_stride, const T* w4, int w_stride) {
  w_ = w; h_ = h; n_ = w * h; nf_ = nf;
  ndirs_ = 0;
  for (int k = 0; k < nf; ++k) dirs_[ndirs_++] = k;
  for (int k = 0; k < nf; ++k) dirs_[ndirs_++] = k ^ 4;
  tr_.assign(n_, 0);
  rc_.assign((size_t)n_ * 8, 0);
  nbr_.assign((size_t)n_ * 8, -1);
  for (int i = 0; i < n_; ++i) {
    const int u = i % w, v = i / w;
    for (int k = 0; k < 8; ++k) {
      const int nu = u + kDU[k], nv = v + kDV[k];
      if (nu >= 0 && nu < w && nv >= 0 && nv < h) nbr_[(size_t)i * 8 + k] = nv * w + nu;
    }
  }
  for (int i = 0; i < n_; ++i) {
    tr_[i] = -(int64_t)U[(size_t)i * u_stride];  // U > 0: residual i->t; U < 0: residual s->i
    for (int d = 0; d < nf; ++d) {
      const int j = nbr(i, d);
      if (j < 0) continue;
      const int64_t c = (int64_t)w4[(size_t)i * w_stride + d];
      if (c > 0) rc_[(size_t)j * 8 + (d ^ 4)] = c;  // arc j -> i: paid when x_j = 1, x_i = 0
    }
  }
}

template void BKSolver::load<int64_t>(int, int, int, const int64_t*, int, const int64_t*, int);
template void BKSolver::load<int32_t>(int, int, int, const int32_t*, int, const int32_t*, int);

void BKSolver::push_active(int i) {
  if (in_active_[i]) return;
  in_active_[i] = 1;
  active_[a_tail_] = i;
  a_tail_ = (a_tail_ + 1) % a_cap_;
}

void BKSolver::make_orphan(int i) {
  parent_[i] = kOrphan;
  orphans_.push_back(i);
}

void BKSolver::augment(int a, int k, int b) {
  int64_t f = rc_[(size_t)a * 8 + k];
  for (int i = a;;) {  // source side: tree arcs parent -> child
    const int p = parent_[i];
    if (p == kTerm) { f = std::min(f, tr_[i]); break; }
    const int j = nbr(i, p);
    f = std::min(f, rc_[(size_t)j * 8 + (p ^ 4)]);
    i = j;
  }
  for (int i = b;;) {  // sink side: tree arcs child -> parent
    const int p = parent_[i];
    if (p == kTerm) { f = std::min(f, -tr_[i]); break; }
    const int j = nbr(i, p);
    f = std::min(f, rc_[(size_t)i * 8 + p]);
    i = j;
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
    const int j = nbr(i, p);
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
    const int j = nbr(i, p);
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
      const int j = nbr(i, k);
      if (j < 0 || tree_[j] != t) continue;
      const int64_t cap = (t == kS) ? rc_[(size_t)j * 8 + (k ^ 4)] : rc_[(size_t)i * 8 + k];
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
        m = nbr(m, pm);
      }
      if (!ok) continue;
      if (d < best_d) { best_d = d; best_k = k; }
      int dd = d;
      for (m = j; ts_[m] != time_; m = nbr(m, parent_[m])) {
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
      const int j = nbr(i, k);
      if (j < 0 || tree_[j] != t) continue;
      const int64_t cap = (t == kS) ? rc_[(size_t)j * 8 + (k ^ 4)] : rc_[(size_t)i * 8 + k];
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
  time_ = 0;
  parent_.assign(n_, kNone);
  tree_.assign(n_, kFree);
  in_active_.assign(n_, 0);
  ts_.assign(n_, 0);
  dist_.assign(n_, 0);
  a_cap_ = (size_t)n_ + 1;
  active_.assign(a_cap_, 0);
  a_head_ = a_tail_ = 0;
  orphans_.clear();
  o_head_ = 0;
  for (int i = 0; i < n_; ++i) {
    if (tr_[i] > 0) { tree_[i] = kS; parent_[i] = kTerm; dist_[i] = 1; push_active(i); }
    else if (tr_[i] < 0) { tree_[i] = kT; parent_[i] = kTerm; dist_[i] = 1; push_active(i); }
  }
  for (;;) {
    int a = -1, b = -1, k_ab = -1;
    while (a_head_ != a_tail_) {
      const int i = active_[a_head_];
      if (tree_[i] == kFree) {
        a_head_ = (a_head_ + 1) % a_cap_;
        in_active_[i] = 0;
        continue;
      }
      if (tree_[i] == kS) {
        for (int q = 0; q < ndirs_ && a < 0; ++q) {
          const int k = dirs_[q];
          const int j = nbr(i, k);
          if (j < 0 || rc_[(size_t)i * 8 + k] <= 0) continue;
          if (tree_[j] == kFree) {
            tree_[j] = kS; parent_[j] = (int8_t)(k ^ 4); ts_[j] = ts_[i]; dist_[j] = dist_[i] + 1;
            push_active(j);
          } else if (tree_[j] == kT) {
            a = i; b = j; k_ab = k;
          }
        }
      } else {
        for (int q = 0; q < ndirs_ && a < 0; ++q) {
          const int k = dirs_[q];
          const int j = nbr(i, k);
          if (j < 0 || rc_[(size_t)j * 8 + (k ^ 4)] <= 0) continue;
          if (tree_[j] == kFree) {
            tree_[j] = kT; parent_[j] = (int8_t)(k ^ 4); ts_[j] = ts_[i]; dist_[j] = dist_[i] + 1;
            push_active(j);
          } else if (tree_[j] == kS) {
            a = j; b = i; k_ab = k ^ 4;
          }
        }
      }
      if (a >= 0) break;  // i stays at the head of the queue
      a_head_ = (a_head_ + 1) % a_cap_;
      in_active_[i] = 0;
    }
    if (a < 0) break;
    augment(a, k_ab, b);
    adopt();
  }
  // source side of the residual graph
  std::memset(x, 0, (size_t)n_);
  bfs_.clear();
  for (int i = 0; i < n_; ++i)
    if (tr_[i] > 0) { x[i] = 1; bfs_.push_back(i); }
  for (size_t h = 0; h < bfs_.size(); ++h) {
    const int i = bfs_[h];
    for (int q = 0; q < ndirs_; ++q) {
      const int k = dirs_[q];
      const int j = nbr(i, k);
      if (j >= 0 && !x[j] && rc_[(size_t)i * 8 + k] > 0) { x[j] = 1; bfs_.push_back(j); }
    }
  }
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
    stop_ = true;
  }
  cv_start_.notify_all();
  for (auto& t : workers_) t.join();
}

void ThreadPool::worker_loop(int id) {
  uint64_t seen = 0;
  for (;;) {
    const std::function<void(int, int)>* job;
    int n;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_start_.wait(lk, [&] { return stop_ || generation_ != seen; });
      if (stop_) return;
      seen = generation_;
      job = job_;
      n = n_items_;
    }
    for (int it = next_.fetch_add(1); it < n; it = next_.fetch_add(1)) (*job)(it, id);
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (--pending_ == 0) cv_done_.notify_one();
    }
  }
}

void ThreadPool::parallel_for(int n, const std::function<void(int, int)>& fn) {
  if (n <= 0) return;
  if (workers_.empty() || n == 1) {
    for (int i = 0; i < n; ++i) fn(i, 0);
    return;
  }
  {
    std::lock_guard<std::mutex> lk(mu_);
    job_ = &fn;
    n_items_ = n;
    next_.store(0);
    pending_ = (int)workers_.size();
    ++generation_;
  }
  cv_start_.notify_all();
  for (int it = next_.fetch_add(1); it < n; it = next_.fetch_add(1)) fn(it, 0);
  std::unique_lock<std::mutex> lk(mu_);
  cv_done_.wait(lk, [&] { return pending_ == 0; });
}

}  // namespace lexp
