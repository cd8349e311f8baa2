// Device max-flow of the binary problems of local expansion moves (CDNA4,
// gfx950): exact minimum cuts, one workgroup per region, arrays in LDS.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lexp_device.h"

namespace lexp {

// ---------------------------------------------------------------------------
// Exact minimum cut of the binary problems of a batch of regions, one
// workgroup per region.  Region problem (terms as k_graph_terms writes them):
// E(x) = sum U_p x_p + sum_d w_d(p) (1 - x_p) x_{p+fwd_d}.  As a graph
// (source side = x 1): source->p with capacity -U_p when U_p < 0, p->sink with
// U_p when U_p > 0, and an arc p+fwd_d -> p of capacity w_d(p).  The kernel
// works on the reversed graph (every arc turned round, source and sink
// swapped): there p has excess max(U_p, 0) after the source arcs are
// saturated, an arc to the sink of capacity max(-U_p, 0), and arcs
// p -> p+fwd_d of capacity w_d(p).  A maximum preflow of the reversed graph
// by synchronous push-relabel (every active node pushes along its admissible
// arcs with the heights held fixed, then every active node without an
// admissible arc relabels), with a breadth-first global relabel from the
// sink every relabel_every rounds, leaves exactly those nodes able to reach
// the sink that the source reaches in the residual graph of a maximum flow of
// the original problem: x = 1 on them is the minimiser with the fewest ones,
// the cut the host max-flow returns.  A region that has not converged after
// its round limit gets status 0 and is left to the host.  Regions whose
// arrays do not fit in LDS (in the compact layout) are left to the host as
// well.
// ---------------------------------------------------------------------------
__device__ constexpr int kCutDU[8] = {1, 0, 1, -1, -1, 0, -1, 1};
__device__ constexpr int kCutDV[8] = {0, 1, 1, 1, 0, -1, -1, -1};

// Workgroup-wide "any" over three flags in turn: call i sets flag i % 3
// before its barrier and reads it after; the call clears flag (i + 2) % 3,
// which no thread sets before passing the barrier of call i + 1 and which no
// reader of call i - 1 can still be reading.  One barrier per call.
struct BlockAny {
  int* flags;  // three ints in LDS, zero at the first call
  int i = 0;
  __device__ int operator()(int pred) {
    int* f = flags + i;
    if (pred) *f = 1;
    __syncthreads();
    const int r = *f;
    if (threadIdx.x == 0) flags[i == 0 ? 2 : i - 1] = 0;
    i = i == 2 ? 0 : i + 1;
    return r;
  }
};

// Full layout, 52 B per node: all eight residuals of a node, 64-bit excess.
struct FullLayout {
  using Ex = unsigned long long;
  using Ht = int;
  static constexpr int kBytesPerNode = 52;
  uint32_t* rc;  // residual capacities, 8 per node (direction k, reverse k ^ 4)
  Ex* ex;        // excess (never negative in a preflow)
  uint32_t* ct;  // residual capacity to the sink
  Ht* h;         // heights
  Ht* h2;        // next heights (relabel phase)

  __device__ void carve(void* smem, int max_nodes, const int*, int) {
    ex = reinterpret_cast<Ex*>(smem);
    rc = reinterpret_cast<uint32_t*>(ex + max_nodes);
    ct = rc + (size_t)8 * max_nodes;
    h = reinterpret_cast<Ht*>(ct + max_nodes);
    h2 = h + max_nodes;
  }
  __device__ void init_arcs(int q, const int* t, int nf) {
    for (int k = 0; k < 8; ++k) rc[(size_t)q * 8 + k] = (k < nf) ? (uint32_t)t[(size_t)q * 5 + 1 + k] : 0u;
  }
  // residual of the arc q -> j (direction k from q) and of j -> q
  __device__ uint32_t out(int q, int k, int) const { return rc[(size_t)q * 8 + k]; }
  __device__ uint32_t in(int, int k, int j) const { return rc[(size_t)j * 8 + (k ^ 4)]; }
  // pushes d along q -> j whose residuals were o (q -> j) and i (j -> q)
  __device__ void push(int q, int k, int j, uint32_t o, uint32_t i, uint32_t d) {
    rc[(size_t)q * 8 + k] = o - d;
    rc[(size_t)j * 8 + (k ^ 4)] = i + d;
  }
  // adds d to the excess of j; false if it no longer fits the excess type
  __device__ bool add_ex(int j, Ex d) {
    atomicAdd(&ex[j], d);
    return true;
  }
};

// Compact layout, 28 B per node: one residual per forward arc (the residuals
// of an arc and of its reverse sum to the arc's capacity, which is read from
// the terms), 32-bit excess and 16-bit heights.  An excess that would pass
// 2^32 - 1 stops the region (status 0), which is then cut on the host.
struct CompactLayout {
  using Ex = uint32_t;
  using Ht = uint16_t;
  static constexpr int kBytesPerNode = 28;
  uint32_t* rf;  // residual of the forward arc q -> q + fwd_k, 4 per node
  Ex* ex;
  uint32_t* ct;
  Ht* h;
  Ht* h2;
  const int* t;  // the region's terms (read only): capacity w_k(q) at t[q*5 + 1 + k]
  int nf;

  __device__ void carve(void* smem, int max_nodes, const int* terms, int n_fwd) {
    rf = reinterpret_cast<uint32_t*>(smem);
    ex = rf + (size_t)4 * max_nodes;
    ct = ex + max_nodes;
    h = reinterpret_cast<Ht*>(ct + max_nodes);
    h2 = h + max_nodes;
    t = terms;
    nf = n_fwd;
  }
  __device__ uint32_t cap(int p, int m) const { return m < nf ? (uint32_t)t[(size_t)p * 5 + 1 + m] : 0u; }
  __device__ void init_arcs(int q, const int*, int) {
    for (int k = 0; k < 4; ++k) rf[(size_t)q * 4 + k] = cap(q, k);
  }
  __device__ uint32_t out(int q, int k, int j) const {
    return k < 4 ? rf[(size_t)q * 4 + k] : cap(j, k - 4) - rf[(size_t)j * 4 + (k - 4)];
  }
  __device__ uint32_t in(int q, int k, int j) const {
    return k < 4 ? cap(q, k) - rf[(size_t)q * 4 + k] : rf[(size_t)j * 4 + (k - 4)];
  }
  __device__ void push(int q, int k, int j, uint32_t o, uint32_t i, uint32_t d) {
    if (k < 4)
      rf[(size_t)q * 4 + k] = o - d;
    else
      rf[(size_t)j * 4 + (k - 4)] = i + d;
  }
  __device__ bool add_ex(int j, Ex d) {
    const Ex old = atomicAdd(&ex[j], d);
    return (unsigned long long)old + d <= 0xffffffffull;
  }
};

// The arrays are in LDS (the workgroup's own memory): excess changes are
// LDS atomics, every other array entry is written by one thread per phase.
// Each node's thread loads its eight neighbours' heights and the residuals of
// both directions of its eight arcs at once, decides its pushes in registers
// and writes back: in a push round only q changes the residual of q -> j and
// of j -> q when j is admissible for q (j cannot push to q then).  Heights
// are double-buffered: the relabel phase writes every node's next height.
template <class Layout, int BLOCK>
__device__ void cut_region(Layout& A, int rw, int rh, int nf, const int* __restrict__ t, uint8_t* __restrict__ x,
                           int* __restrict__ status, int max_rounds, int relabel_every, int* any_flags,
                           int* overflow) {
  using Ex = typename Layout::Ex;
  using Ht = typename Layout::Ht;
  BlockAny any{any_flags};
  const int n = rw * rh;
  const int inf = n + 1;  // height of nodes that cannot reach the sink (a distance is at most n)
  const int tid = threadIdx.x;
  for (int q = tid; q < n; q += BLOCK) {
    const int U = t[(size_t)q * 5];
    A.ex[q] = U > 0 ? (Ex)U : (Ex)0;
    A.ct[q] = U < 0 ? (uint32_t)(-(long long)U) : 0u;
    A.init_arcs(q, t, nf);
  }
  Ht* hc = A.h;   // current heights
  Ht* hn = A.h2;  // heights of the next round
  // neighbour j of q in direction k, or q itself where the grid ends (masked)
  auto nbrs = [&](int q, int (&j)[8]) -> int {
    const int u = q % rw, v = q / rw;
    int valid = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int nu = u + kCutDU[k], nv = v + kCutDV[k];
      const bool ok = nu >= 0 && nu < rw && nv >= 0 && nv < rh;
      j[k] = ok ? nv * rw + nu : q;
      valid |= ok ? 1 << k : 0;
    }
    return valid;
  };
  // breadth-first distances to the sink over residual arcs (inf = cannot reach)
  auto global_relabel = [&]() {
    __syncthreads();
    for (int q = tid; q < n; q += BLOCK) hc[q] = (Ht)(A.ct[q] > 0 ? 1 : inf);
    __syncthreads();
    for (int level = 1;; ++level) {
      int changed = 0;
      for (int q = tid; q < n; q += BLOCK) {
        if ((int)hc[q] != level) continue;
        int j[8];
        const int valid = nbrs(q, j);
        int hj[8];
        uint32_t rj[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) { hj[k] = hc[j[k]]; rj[k] = A.in(q, k, j[k]); }
#pragma unroll
        for (int k = 0; k < 8; ++k)  // arc j -> q with residual capacity
          if (((valid >> k) & 1) && hj[k] == inf && rj[k] > 0) { hc[j[k]] = (Ht)(level + 1); changed = 1; }
      }
      if (!any(changed)) break;
    }
  };
  auto any_active = [&]() {
    int active = 0;
    for (int q = tid; q < n; q += BLOCK) active |= (A.ex[q] > 0 && (int)hc[q] < inf) ? 1 : 0;
    return any(active);
  };
  global_relabel();
  int rounds = 0;
  bool done = !any_active();
  bool lost = false;  // an excess passed its type: the region is left to the host
  while (!done && rounds < max_rounds) {
    // push: heights fixed, so no arc carries flow both ways in one round
    for (int q = tid; q < n; q += BLOCK) {
      const Ex e0 = A.ex[q];
      const int hq = hc[q];
      if (e0 == 0 || hq >= inf) continue;
      int j[8];
      const int valid = nbrs(q, j);
      int hj[8];
      uint32_t rq[8], rj[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        hj[k] = hc[j[k]];
        rq[k] = A.out(q, k, j[k]);
        rj[k] = A.in(q, k, j[k]);
      }
      Ex e = e0;
      if (hq == 1) {
        const uint32_t cq = A.ct[q];
        if (cq > 0) {
          const Ex d = e < (Ex)cq ? e : (Ex)cq;
          A.ct[q] = cq - (uint32_t)d;
          e -= d;
        }
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (e == 0 || !((valid >> k) & 1) || hj[k] != hq - 1 || rq[k] == 0u) continue;
        const Ex d = e < (Ex)rq[k] ? e : (Ex)rq[k];
        A.push(q, k, j[k], rq[k], rj[k], (uint32_t)d);
        if (!A.add_ex(j[k], d)) *overflow = 1;
        e -= d;
      }
      if (e != e0) atomicSub(&A.ex[q], (Ex)(e0 - e));
    }
    __syncthreads();
    // relabel: 1 + the lowest height across a residual arc, when no arc is admissible
    int active = 0;
    for (int q = tid; q < n; q += BLOCK) {
      const int hq = hc[q];
      int nh = hq;
      const bool has_ex = A.ex[q] > 0;
      if (has_ex && hq < inf) {
        int j[8];
        const int valid = nbrs(q, j);
        int hj[8];
        uint32_t rq[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) { hj[k] = hc[j[k]]; rq[k] = A.out(q, k, j[k]); }
        int m = A.ct[q] > 0 ? 0 : inf;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (((valid >> k) & 1) && rq[k] != 0u && hj[k] < m) m = hj[k];
        if (m >= hq) nh = m + 1 < inf ? m + 1 : inf;
      }
      hn[q] = (Ht)nh;
      active |= (has_ex && nh < inf) ? 1 : 0;
    }
    Ht* tmp = hc;
    hc = hn;
    hn = tmp;
    ++rounds;
    if (rounds % relabel_every == 0) {
      global_relabel();
      done = !any_active();
    } else {
      done = !any(active);
    }
    // the overflow flag is only written in the push phase, before the barrier
    // of the call above, so every thread reads the same value here
    if (*overflow) {
      lost = true;
      break;
    }
  }
  if (lost) {
    if (tid == 0) *status = 0;
    return;
  }
  global_relabel();
  for (int q = tid; q < n; q += BLOCK) x[q] = (int)hc[q] < inf ? 1 : 0;
  if (tid == 0) *status = done ? 1 : 0;
}

// One workgroup per region; the region's arrays in LDS with the given layout.
template <class Layout, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_cut_lds(const Item* __restrict__ items, const int* __restrict__ terms,
                                                  int nf, uint8_t* __restrict__ x, int* __restrict__ status,
                                                  int max_nodes, int round_factor, int relabel_every) {
  extern __shared__ unsigned long long smem_cut[];
  __shared__ int any_flags[3];
  __shared__ int overflow;
  const Item it = items[blockIdx.x];
  const int n = it.rw * it.rh;
  if (n <= 0) {
    if (threadIdx.x == 0) status[blockIdx.x] = 1;
    return;
  }
  const int* t = terms + (size_t)it.aux_off * 5;
  Layout A;
  A.carve(smem_cut, max_nodes, t, nf);
  if (threadIdx.x < 3) any_flags[threadIdx.x] = 0;
  if (threadIdx.x == 0) overflow = 0;
  cut_region<Layout, BLOCK>(A, it.rw, it.rh, nf, t, x + it.aux_off, status + blockIdx.x, round_factor * n + 256,
                            relabel_every, any_flags, &overflow);
}

template __global__ void k_cut_lds<FullLayout, 128>(const Item*, const int*, int, uint8_t*, int*, int, int, int);
template __global__ void k_cut_lds<FullLayout, 256>(const Item*, const int*, int, uint8_t*, int*, int, int, int);
template __global__ void k_cut_lds<FullLayout, 512>(const Item*, const int*, int, uint8_t*, int*, int, int, int);
template __global__ void k_cut_lds<FullLayout, 1024>(const Item*, const int*, int, uint8_t*, int*, int, int, int);
template __global__ void k_cut_lds<CompactLayout, 1024>(const Item*, const int*, int, uint8_t*, int*, int, int,
                                                        int);

}  // namespace lexp
