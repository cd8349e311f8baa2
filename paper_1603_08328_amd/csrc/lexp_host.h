// Host-side pieces of the library that need no device: counter-based random
// numbers, the proposers of Alg. 1 / Alg. 2, the Boykov-Kolmogorov max-flow
// used to solve one local expansion exactly, and a small thread pool.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace lexp {

// ---- random numbers ------------------------------------------------------
uint64_t sm64(uint64_t x);
uint64_t key_chain(uint64_t seed, const uint64_t* fields, int n);
double u01_open1(uint64_t x);    // [0, 1)
double u01_open0(uint64_t x);    // (0, 1]

// Random initial label of pixel (u, v) (Alg. 2, initialisation).
void init_label(int width, int u, int v, double disp_max, uint64_t seed, float out[3]);

// Candidate label of one alpha_ij-expansion step (Alg. 1), in its order:
// k_prop propagation steps, k_rans RANSAC steps, then refinement steps.
// labels: HxWx3 host mirror (stride `stride` floats per pixel).
// net_planes (optional, HxWx4): planes proposed by the learned network; the
// refinement steps with an odd refinement index then take the plane of the
// chosen pixel r instead of a perturbation.
// label_at_r (optional): the label to take as the one at the drawn pixel r
// instead of labels' (propagation and refinement steps read no other label;
// not for RANSAC steps, which read the whole cell).
void propose(int width, int height, const float* labels, int stride, uint64_t seed, int iteration, int level,
             int cell, int ci, int cj, int step, int k_prop, int k_rans, double r_d, double r_n, float out[3],
             const float* net_planes = nullptr, const float* label_at_r = nullptr);

// ---- exact binary minimisation ------------------------------------------
// E(x) = sum_i U_i x_i + sum_{i, d < nf} w_{i,d} (1 - x_i) x_{i + fwd_d} on a
// w x h grid, forward directions (1,0), (0,1), (1,1), (-1,1) (nf = 4 for the
// 8-neighbourhood, 2 for the 4-neighbourhood).
class BKSolver {
 public:
  // terms: per node U at u_stride, w_0..w_3 at w_stride (w_d >= 0).
  template <class T>
  void load(int w, int h, int nf, const T* U, int u_stride, const T* w4, int w_stride);
  // Max-flow, then x_i = 1 for nodes reachable from the source in the
  // residual graph (the minimiser with the fewest ones).
  void solve(uint8_t* x);
  int64_t flow() const { return flow_; }

 private:
  // Nodes live on a grid padded by one dead node on every side, so
  // neighbours are plain index offsets; dead nodes have no capacity and
  // never join a search tree.
  enum : int8_t { kNone = -1, kTerm = 8, kOrphan = 9 };
  enum : uint8_t { kFree = 0, kS = 1, kT = 2 };
  void push_active(int i);
  void make_orphan(int i);
  void augment(int a, int k, int b);
  void adopt();

  int w_ = 0, h_ = 0, pw_ = 0, pn_ = 0, nf_ = 4;
  int off_[8];
  int dirs_[8];
  int ndirs_ = 0;
  int64_t flow_ = 0;
  int32_t time_ = 0;
  std::vector<int32_t> tr_;   // residual terminal capacity: > 0 from s, < 0 to t
  std::vector<int32_t> rc_;   // residual arc capacities, 8 per node
  std::vector<int8_t> parent_;
  std::vector<uint8_t> tree_;
  std::vector<uint8_t> in_active_;
  std::vector<int32_t> ts_, dist_;
  std::vector<int32_t> active_;   // circular FIFO
  size_t a_head_ = 0, a_tail_ = 0, a_cap_ = 0;
  std::vector<int32_t> orphans_;
  size_t o_head_ = 0;
  std::vector<int32_t> bfs_;
  std::vector<uint8_t> seen_;
};

// ---- thread pool -----------------------------------------------------------
constexpr int kMaxPoolThreads = 64;  // threads of one pool (the caller is worker 0)

class ThreadPool {
 public:
  explicit ThreadPool(int n_threads);
  ~ThreadPool();
  int size() const { return (int)workers_.size() + 1; }
  // Runs fn(item, worker) for item in [0, n); the caller takes part as worker 0.
  void parallel_for(int n, const std::function<void(int, int)>& fn);

 private:
  void worker_loop(int id);
  std::vector<std::thread> workers_;
  std::mutex mu_;
  std::condition_variable cv_start_, cv_done_;
  const std::function<void(int, int)>* job_ = nullptr;
  int n_items_ = 0;
  std::atomic<int> next_{0};
  std::atomic<int> pending_{0};
  std::atomic<uint64_t> generation_{0};
  std::atomic<bool> stop_{false};
};

}  // namespace lexp
