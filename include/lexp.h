/*
 * lexp.h -- C ABI of the MI355X local-expansion-move stereo library.
 *
 * Method: Taniai, Matsushita, Sato, Naemura, "Continuous 3D Label Stereo
 * Matching using Local Expansion Moves" (TPAMI; arXiv 1603.08328).
 *
 * Conventions shared by every call
 *   - Images are HxWx3 float32, row-major HWC, values in [0, 255]; u is the
 *     column and v the row, both 0-based.
 *   - A label is a disparity plane d(u, v) = a*u + b*v + c (Eq. (1)).  Label
 *     fields on the device are HxWx4 float32 (a, b, c, unused).
 *   - A rectangle is half-open [u0, u1) x [v0, v1); every call clips it to the
 *     image.  A rectangle that clips to nothing is a no-op item.
 *   - "device" pointers are HIP device memory owned by the caller (PyTorch
 *     tensors in the Python binding); "host" pointers are read before return.
 *   - hip_stream is a hipStream_t (NULL = legacy default stream).  Calls are
 *     stream-ordered unless stated otherwise.  One context is used from one
 *     host thread at a time; calls on one context are not re-entrant.
 *   - Every call returns a status: LEXP_OK (0) or a negative error code.
 *     Nothing is modified when a call fails its argument validation.
 *     lexp_last_error() returns a message for the calling thread's last
 *     failure; it stays valid until the next call on that thread.
 *
 * Units of the binary problem: the terms of one expansion are rounded up to
 * integer multiples of LEXP_QUANTUM (2^-20) of the energy; energy changes
 * reported as int64 are in those units.
 */
#ifndef LEXP_H
#define LEXP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lexp_status;
#define LEXP_OK 0
#define LEXP_EINVAL (-1)  /* invalid argument: null pointer, size, range, overlap, non-finite label */
#define LEXP_ENOMEM (-2)  /* device or host allocation failed */
#define LEXP_EDEVICE (-3) /* HIP runtime error (message holds the HIP error string) */
#define LEXP_ESTATE (-4)  /* the context is unusable after an earlier device error */

#define LEXP_QUANTUM_LOG2 20

typedef struct lexp_ctx lexp_ctx;

typedef struct {
  float a, b, c;
} lexp_plane;

typedef struct {
  int32_t u0, v0, u1, v1;
} lexp_rect;

/* Parameters of the energy (Sec. 3.2) and of the guided filter.
 *   alpha, tau_col, tau_grad : raw cost weights and truncations, Eq. (9)
 *   gf_radius                : radius r of the regression window W'_k of
 *                              Eq. (7), (2r+1)^2 pixels; 1 <= r, and r <= 28 on
 *                              MI355X: a tile of the fused cost kernel holds its
 *                              rings and rows of M (1 + 4r columns and more) in
 *                              one workgroup's 160 KB of LDS; lexp_create rejects
 *                              a larger r (LEXP_EINVAL)
 *   gf_eps                   : e of Eq. (7) (0.01^2 in the paper)
 *   lambda, tau_dis, w_floor,
 *   gamma                    : smoothness weight, truncation, lower bound
 *                              epsilon and contrast gamma, Eqs. (5),(10),(11)
 *   neighbours               : 8 or 4
 *   host_threads             : threads of the host min-cut pool (0 = all cores, at most 64)
 *   device_cut               : lexp_optimize: 1 = minimum cuts of the expansion
 *                              moves by the device push-relabel kernel, any region
 *                              it leaves unfinished is cut on the host; 0 = every
 *                              cut on the host (Boykov-Kolmogorov).  Both return the
 *                              same cut (the minimiser with the fewest ones).
 *   view                     : 0 = the left view (data term on I_L, samples of I_R
 *                              at u - d); 1 = the right view: I_L and I_R swapped
 *                              in Eqs. (7) and (9), samples at u + d, contrast
 *                              weights of Eq. (11) from I_R.  A right-view context
 *                              evaluates it as the left-view term of the mirrored
 *                              pair, and all its pixels, rects and label fields are
 *                              in the mirrored frame of the right image: pixel
 *                              (u, v) is right pixel (W-1-u, v), and label (a, b, c)
 *                              is the right image's plane (-a, b, c + a (W-1))
 *                              (lexp_view_labels converts).  The images passed to
 *                              lexp_create are (left, right) for both views.
 *   graph                    : lexp_optimize: 1 = the device work of each step of a
 *                              part (items copy, cost kernel, graph terms, device
 *                              max-flow) is captured once per split of
 *                              its group into a HIP graph and replayed for every
 *                              candidate step (the device/host split of each level
 *                              is tuned in the first iteration only, then kept, so
 *                              later iterations replay); runs with timing enabled launch
 *                              eagerly (timing events are not captured).  Same
 *                              results either way.
 */
typedef struct {
  int32_t width, height;
  double disp_max;
  double alpha, tau_col, tau_grad;
  int32_t gf_radius;
  double gf_eps;
  double lambda, tau_dis, w_floor, gamma;
  int32_t neighbours;
  int32_t host_threads;
  int32_t device_cut;
  int32_t view;
  int32_t graph;
} lexp_params;

/* Grid levels of the optimisation procedure (Alg. 2): cell size in pixels and
 * the proposer counts of Alg. 1 per level, run in Alg. 1's order: k_prop
 * propagation, k_rans RANSAC (LO-RANSAC plane fit to the current disparities
 * of the centre cell), k_rand refinement steps (k_prop + k_rans + k_rand <= 64). */
typedef struct {
  int32_t n_levels; /* 1..4 */
  int32_t cell[4];
  int32_t k_prop[4];
  int32_t k_rand[4];
  int32_t iterations;
  int32_t k_rans[4];
  int32_t learned; /* 1: from the second iteration on, refinement steps with an odd
                      index take the plane of the learned network (lexp_set_net) at
                      the chosen pixel, computed from the labels at the start of each
                      level pass (the first iteration starts from random labels,
                      unlike anything the network is trained on); 0: none */
  int32_t batch_cycle; /* 1: the "batch cycle" of Alg. 1 (Sec. 3.4): every candidate of a
                          cell's Alg. 1 is drawn from the labels at the start of its group
                          step, the costs of all regions of the group for all their
                          candidates are evaluated in one launch, then the moves are
                          applied in Alg. 1's order, each an exact expansion on the
                          current labels; 0: each candidate from the latest labels (the
                          method as the paper runs it).  The graph option is not used
                          in this mode. */
  int32_t tile_cols[4]; /* fused cost kernel, per level: widest column strip of a region's
                           tiles (0: the widest the kernel's LDS allows) */
  int32_t tile_fill[4]; /* per level: tiles a group step's launch is filled to with row
                           strips (0: 256).  Both decide the tiles, and so the rounding of
                           the costs; a committed table of tuned values keeps labels
                           independent of any run's timing. */
  int32_t speculate;    /* 1: in groups whose regions form one part, the next step's two possible
                           candidates of every region (its drawn pixel's label kept, or set to
                           the current step's candidate: Alg. 1 reads no other label for
                           propagation and refinement steps) are evaluated while the host cuts
                           the current step, and the one the updated labels propose is used;
                           the same labels and costs as 0 (each step evaluates its own
                           candidate after the cut).  The discarded half counts among the
                           kernel's timed evaluations, not among unary_evals.  Not with the
                           batch cycle or graphs. */
} lexp_schedule;

/* Counters of the hot kernel, accumulated while timing is enabled. */
typedef struct {
  int64_t unary_launches;   /* launches of the fused cost kernel */
  int64_t unary_items;      /* (region, label) items evaluated */
  int64_t unary_evals;      /* phi_p evaluations (sum of clipped |R|) */
  double unary_kernel_ms;   /* sum of the timed launches' kernel durations (HIP events on the launch stream) */
  double unary_alg_bytes;   /* algorithmic bytes: sum over items of 16|M| + 16|M| + 36|R+| + 4|R| */
  int64_t expand_calls;     /* group steps (one batch of disjoint expansions) */
  double host_cut_ms;       /* host max-flow time, or with the device cut the host time after
                               the cut (label mirror, candidates), wall, summed over steps */
  double host_wait_ms;      /* time the host waited for the device's terms or cuts (terms in two
                               launches: the wait for the first, plus a worker's for the second) */
  double host_enqueue_ms;   /* lexp_optimize: host time queueing device work (copies, launches) */
  double host_update_ms;    /* lexp_optimize: host time queueing label updates after the cuts */
  double host_cut_level_ms[4]; /* lexp_optimize: host_cut_ms by grid level */
  int64_t device_cut_fallbacks; /* lexp_optimize: regions the device max-flow left to the host */
  double device_cut_share[4];   /* lexp_optimize: share of each level's device-sized regions cut on
                                   the device in the last iteration (0 with device_cut off) */
  int64_t graphs_captured;      /* lexp_optimize: HIP graphs captured (graph mode) */
  int32_t device_cut_block[4];  /* lexp_optimize: threads per region the device max-flow's launch-shape
                                   tuner chose per level (0: not tuned; every shape gives the same cut) */
  int32_t device_cut_relabel[4];/* its rounds between global relabels */
  int64_t unary_timed_launches; /* fused-kernel launches timed (every N-th, see lexp_set_timing) */
  double unary_timed_alg_bytes; /* their algorithmic bytes */
  int64_t unary_timed_evals;    /* their phi_p evaluations */
  double host_solve_level_ms[4];/* lexp_optimize: host max-flow time per level summed over regions (CPU time of
                                   the solves, all threads; against host_cut_level_ms: the pool's efficiency) */
  int64_t host_solves[4];       /* lexp_optimize: regions cut on the host, per level */
  double unary_level_ms[4];        /* lexp_optimize: timed fused-kernel milliseconds per grid level */
  double unary_level_alg_bytes[4]; /* their algorithmic bytes */
  int64_t unary_level_launches[4]; /* their launches */
  int64_t spec_steps;   /* lexp_optimize: part steps that took speculatively evaluated costs */
  int64_t spec_misses;  /* part steps whose candidates matched neither speculative one */
} lexp_stats;

/* Creates a context for one stereo pair and runs the label-independent set-up
 * on the device: packed images (R, G, B, x-gradient of the BT.601 gray value
 * by [-0.5 0 0.5], replicated borders), guide statistics of Eq. (7) (mean of
 * I = I_L/255 and (Sigma_k + eU)^-1 over W'_k, computed in FP64, stored FP32)
 * and the contrast weights w_pq of Eq. (11) for the forward neighbours (FP64).
 * left_hwc / right_hwc: device, HxWx3 float32; they may be freed after return
 * (the call synchronises hip_stream).  The context owns its device scratch.
 * Images of at most 2^27 - 1 pixels (LEXP_EINVAL otherwise). */
lexp_status lexp_create(const lexp_params* params, const float* left_hwc, const float* right_hwc,
                        void* hip_stream, lexp_ctx** out);

/* Frees the context and its device scratch.  NULL is accepted. */
lexp_status lexp_destroy(lexp_ctx* ctx);

const char* lexp_last_error(void);

/* Unary term phi_p(alpha) of Eq. (6) for n (region, label) items, computed as
 * Sec. 3.5 describes: the raw cost rho_alpha of Eqs. (8),(9),(18) over the
 * filtering region M (the region dilated by 2r, Eq. (20)), aggregated by the
 * box form of the guided filter of Eq. (7) (Eq. (19)).  Windows clipped by
 * the image border are count-normalised; a sample outside the right image
 * costs (1-alpha)*tau_col + alpha*tau_grad.
 *   rects, labels, offsets: host arrays [n].
 *   out_cost: device float32; item i writes |clip(rects[i])| values,
 *             row-major over the clipped rectangle, at out_cost[offsets[i]].
 * Asynchronous on hip_stream. */
lexp_status lexp_unary_cost(lexp_ctx* ctx, int32_t n, const lexp_rect* rects, const lexp_plane* labels,
                            const int64_t* offsets, float* out_cost, void* hip_stream);

/* Linear coefficients (a_k[0..2], b_k) of the guided filter of Eq. (7) for the
 * cost slice of each item, over R+ = clip(rect dilated by r), row-major, 4
 * float32 per pixel at out_ab[4 * offsets[i]].  Inspection and tests. */
lexp_status lexp_guided_coeffs(lexp_ctx* ctx, int32_t n, const lexp_rect* rects, const lexp_plane* labels,
                               const int64_t* offsets, float* out_ab, void* hip_stream);

/* Per-pixel unary phi_p(f_p) of Eq. (6) with every pixel's own label (each
 * pixel is a 1x1 region): the state after the random initialisation of
 * Alg. 2.  labels: device HxWx4; out_cost: device HxW float32. */
lexp_status lexp_pixel_costs(lexp_ctx* ctx, const float* labels, float* out_cost, void* hip_stream);

/* One local alpha-expansion per region (Eq. (13) restricted to the region,
 * binary problem of Lemma 2, solved exactly by a host Boykov-Kolmogorov
 * max-flow; among minimisers, the one that takes alpha at the fewest pixels).
 * Regions must be pairwise separated by at least one pixel (no 8-neighbour
 * contact), else LEXP_EINVAL and nothing is modified (Lemma 3 independence).
 *   rects, alpha, offsets: host [n]; alpha_cost: device, phi(alpha) laid out
 *   as lexp_unary_cost writes it; labels (device HxWx4) and cur_cost (device
 *   HxW, phi_p(f_p)) are updated in place; delta_Eq (host [n], may be NULL):
 *   energy change in LEXP_QUANTUM units (<= 0); n_changed (host [n], may be
 *   NULL): pixels that took alpha.  Synchronises hip_stream. */
lexp_status lexp_expand_region(lexp_ctx* ctx, int32_t n, const lexp_rect* rects, const lexp_plane* alpha,
                               const float* alpha_cost, const int64_t* offsets, float* labels, float* cur_cost,
                               int64_t* delta_Eq, int32_t* n_changed, void* hip_stream);

/* The device-built binary problem of lexp_expand_region without solving it:
 * per pixel of each region (row-major at 5 * offsets[i]) the int32 terms
 * (U_p, w_0..w_3): E(x) = sum U_p x_p + sum_d w_d (1 - x_p) x_{p + fwd_d},
 * forward directions (1,0), (0,1), (1,1), (-1,1).  out_terms: device. */
lexp_status lexp_graph_terms(lexp_ctx* ctx, int32_t n, const lexp_rect* rects, const lexp_plane* alpha,
                             const float* alpha_cost, const int64_t* offsets, const float* labels,
                             const float* cur_cost, int32_t* out_terms, void* hip_stream);

/* Smoothness term of Eq. (10) times lambda, for neighbours p and q, evaluated
 * by the device code path (FP64).  Synchronous. */
lexp_status lexp_pairwise(lexp_ctx* ctx, int32_t pu, int32_t pv, int32_t qu, int32_t qv, lexp_plane fp,
                          lexp_plane fq, double* out);

/* Energy of Eq. (5) (FP64): sum of cur_cost plus lambda * sum of Eq. (10)
 * over unordered neighbour pairs.  labels: device HxWx4, cur_cost: device HxW.
 * Any output pointer may be NULL.  Synchronises hip_stream. */
lexp_status lexp_energy(lexp_ctx* ctx, const float* labels, const float* cur_cost, double* total,
                        double* unary, double* pairwise, void* hip_stream);

/* lexp_energy for callers that cannot allocate memory (tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments, the same values bit
 * for bit (the same per-block partial sums, added in the same order), and no
 * allocation of any kind.  (It copies the totals to the host and waits for
 * them, so it is not for a stream under HIP graph capture.)  The partial sums
 * and totals live in a fixed device array of the library, one per GPU, held
 * from the first lexp_create on that GPU until the process ends (about
 * 128 KB).  Images of at most LEXP_NOALLOC_MAX_PIXELS pixels (LEXP_EINVAL
 * beyond, before any work).  Every call on one GPU uses that GPU's array and
 * leaves its contents there, so calls that overlap on one GPU (other streams
 * or host threads) race; nothing in the array needs to start at zero.
 * Synchronises hip_stream. */
#define LEXP_NOALLOC_MAX_PIXELS 2097152
lexp_status lexp_energy_noalloc(lexp_ctx* ctx, const float* labels, const float* cur_cost, double* total,
                                double* unary, double* pairwise, void* hip_stream);

/* Random initialisation of Alg. 2 (plane through (p, z0), z0 ~ U[0, disp_max],
 * normal uniform on the upper hemisphere) from a counter-based generator
 * keyed by (seed, pixel).  labels: device HxWx4. */
lexp_status lexp_init_labels(lexp_ctx* ctx, uint64_t seed, float* labels, void* hip_stream);

/* Runs the optimisation procedure of Alg. 2 with Alg. 1 per cell and the
 * grouping of Eq. (15): random init, per-pixel costs, then for every
 * iteration, grid level and group, K_prop propagation and K_rand
 * randomisation steps for all cells of the group together.
 *   labels (device HxWx4) and cur_cost (device HxW) receive the result.
 *   energy_trace (host, iterations+1 values, may be NULL): Eq. (5) after the
 *   init and after each iteration.  time_trace (same size, may be NULL):
 *   seconds since the call started at those points.  Synchronous. */
lexp_status lexp_optimize(lexp_ctx* ctx, const lexp_schedule* schedule, uint64_t seed, float* labels,
                          float* cur_cost, double* energy_trace, double* time_trace, void* hip_stream);

/* lexp_optimize for n_pairs stereo pairs at once, each with its own context
 * (sizes and disparity ranges may differ; gf_radius and neighbours must be the
 * same, and every context must live on the current device).  Every group step
 * of Alg. 2 (Eq. (15)) is evaluated for all pairs together: one fused cost
 * launch, one graph-term launch, one device max-flow launch and one host-pool
 * pass cover the regions of that step in every pair.  Pair i's labels,
 * cur_cost and energy trace equal, bit for bit, what lexp_optimize returns for
 * (ctxs[i], seeds[i]) alone.
 *   ctxs, seeds, labels, cur_cost: host arrays [n_pairs] (distinct contexts
 *   and buffers); labels[i] device HxWx4 and cur_cost[i] device HxW of pair i.
 *   energy_traces: NULL, or host array [n_pairs] of per-pair traces
 *   (iterations+1 values each, entries may be NULL).  time_trace: as in
 *   lexp_optimize, for the whole batch.  The scratch, host threads, device_cut
 *   setting and statistics of ctxs[0] serve the run.  Synchronous. */
lexp_status lexp_optimize_batch(int32_t n_pairs, lexp_ctx* const* ctxs, const lexp_schedule* schedule,
                                const uint64_t* seeds, float* const* labels, float* const* cur_cost,
                                double* const* energy_traces, double* time_trace, void* hip_stream);

/* Label field of a context (device HxWx4) in its view image's own frame:
 * a copy for the left view; for the right view, out(u, v) = the plane of
 * in(W-1-u, v) in right-image coordinates, (a, b, c) -> (-a, b, c + a (W-1)),
 * with c rounded once to FP32.  in and out must not overlap.  Stream-ordered. */
lexp_status lexp_view_labels(lexp_ctx* ctx, const float* labels_in, float* labels_out, void* hip_stream);

/* Post-processing of the left view (the final step of the paper's method,
 * after Bleyer et al. 2011): left-right consistency check, filling of the
 * inconsistent pixels from the nearest consistent ones of their row (the
 * plane with the lower disparity there) and a weighted median over a 35x35
 * window on the filled pixels (colour weights exp(-||I_L(p)-I_L(q)||_1/gamma)
 * quantised down to multiples of 2^-24).
 *   left, labels_left  : a left-view context and its labels (device HxWx4);
 *   right, labels_right: a right-view context of the same pair and its labels
 *                        (device HxWx4, in its mirrored frame, as lexp_optimize
 *                        leaves them);
 *   out_disp           : device HxW float32, the left disparity map;
 *   out_invalid        : device HxW uint8 (1 = failed the check), may be NULL.
 * Scratch belongs to the left context (calls on one left context must share a
 * stream).  Stream-ordered. */
lexp_status lexp_postprocess(lexp_ctx* left, const float* labels_left, lexp_ctx* right, const float* labels_right,
                             float* out_disp, uint8_t* out_invalid, void* hip_stream);

/* ---- learned proposal network ---------------------------------------------
 * Five 3x3 convolutions (zero padding), ReLU after the first four, channels
 * 16 -> 32 -> 32 -> 32 -> 32 -> 16, on the BF16 matrix cores with FP32 sums.
 * Input per pixel: left RGB / 255 of the context's packed images, right
 * RGB / 255 at the pixel's match u - d (linear interpolation, zero outside),
 * a, b, d / disp_max of the label (d = a u + b v + c), 1 where the match is
 * inside the right image, then zeros.
 * Output channels 0..2: (a, b, d / disp_max) of a proposed plane.  Training
 * loss: mean over pixels of the mean over the 5x5 neighbourhood q of
 * |d_p + a_p (u_q - u_p) + b_p (v_q - v_p) - d*_q| (d* from the target
 * labels); Adam (0.9, 0.999, 1e-8) on FP32 master weights.  Weights are laid
 * out per layer [tap][out][in] (tap = 3 ky + kx), layers one after the other;
 * biases likewise.  Not in the paper: the method admits any proposer. */
typedef struct lexp_net lexp_net;
lexp_status lexp_net_sizes(int32_t* n_weights, int32_t* n_biases);
/* He-uniform weights from the counter-based generator keyed by seed, zero
 * biases; buffers for images up to max_width x max_height. */
lexp_status lexp_net_create(int32_t max_width, int32_t max_height, uint64_t seed, lexp_net** out);
lexp_status lexp_net_destroy(lexp_net* net);
/* Host arrays of lexp_net_sizes' lengths; setting resets the Adam state.  Synchronous. */
lexp_status lexp_net_set_weights(lexp_net* net, const float* weights, const float* biases);
lexp_status lexp_net_get_weights(lexp_net* net, float* weights, float* biases);
/* Gradients of the last training step (same layout; inspection).  Synchronous. */
lexp_status lexp_net_get_grads(lexp_net* net, float* weights, float* biases);
/* Output of the network on ctx's images and labels (device HxWx4): out is
 * device HxWx16 FP32.  Stream-ordered. */
lexp_status lexp_net_forward(lexp_net* net, lexp_ctx* ctx, const float* labels, float* out, void* hip_stream);
/* One Adam step on the loss of the network's output for labels against
 * target labels (both device HxWx4); loss (host, may be NULL) receives the
 * loss before the step.  Synchronises hip_stream. */
lexp_status lexp_net_train_step(lexp_net* net, lexp_ctx* ctx, const float* labels, const float* target_labels,
                                float learning_rate, double* loss, void* hip_stream);
/* The network lexp_optimize uses when schedule->learned is 1 (NULL: none). */
lexp_status lexp_set_net(lexp_ctx* ctx, lexp_net* net);

/* Timing of the fused cost kernel and of the host phases.  enable = N > 0
 * turns it on: every launch is counted, and every N-th fused launch (N = 1:
 * all) is launched with two HIP events on its stream that take the kernel's
 * own start and end (their host cost is about 12 us per launch, so a sample
 * keeps the whole job's time close to an untimed run); 0 turns it off,
 * negative values are LEXP_EINVAL.  reset clears the counters. */
lexp_status lexp_set_timing(lexp_ctx* ctx, int32_t enable);
lexp_status lexp_get_stats(lexp_ctx* ctx, lexp_stats* out);
lexp_status lexp_reset_stats(lexp_ctx* ctx);

/* Copies of the set-up buffers for inspection (device destinations, any may
 * be NULL): left4/right4 HxWx4 (R, G, B, x-gradient); guide as nine HxW
 * planes, one after the other (mu_0..2 of the window W'_k, then inv00, inv01,
 * inv02, inv11, inv12, inv22 of (Sigma_k + eU)^-1, Eq. 7); weights HxWx4
 * float64 (w_pq for the forward neighbours, 0 outside the image). */
lexp_status lexp_debug_guide(lexp_ctx* ctx, float* left4, float* right4, float* guide, double* weights,
                             void* hip_stream);

/* Exact minimisation on the device (the push-relabel kernel lexp_optimize
 * uses) of n binary problems of the form lexp_solve_binary takes, on grids
 * dims[2i] x dims[2i+1] (width, height), with the context's neighbourhood.
 * terms: host, per problem w*h nodes of 5 int32 (U, then w_0..w_3 for the
 * forward neighbours (1,0), (0,1), (1,1), (-1,1); |U| <= 2^30, 0 <= w_d <= 2^30,
 * w_d = 0 where the neighbour is outside the grid), problems back to back.
 * x: host, per problem w*h bytes (x = 1: the minimiser with the fewest ones).
 * status[i] = 1 where the kernel finished problem i, 0 where it stopped at its
 * round limit (x of that problem is then undefined).  Synchronises hip_stream. */
lexp_status lexp_solve_binary_device(lexp_ctx* ctx, int32_t n, const int32_t* dims, const int32_t* terms, uint8_t* x,
                                     int32_t* status, void* hip_stream);

/* ---- host-side pieces, usable without a device ---------------------------- */

/* Exact minimisation of E(x) = sum U_p x_p + sum_d w_d (1 - x_p) x_{p+fwd_d}
 * on a w x h grid by the library's Boykov-Kolmogorov max-flow; returns in x
 * the minimiser with the fewest ones.  U: [w*h], |U_p| <= 2^30; w4: [w*h*4],
 * 0 <= w_d <= 2^30 (LEXP_EINVAL otherwise); neighbours 8 or 4; x: [w*h].
 * Host memory. */
lexp_status lexp_solve_binary(int32_t w, int32_t h, int32_t neighbours, const int64_t* U, const int64_t* w4,
                              uint8_t* x);

/* Counter-based random numbers: SplitMix64 output function applied along the
 * key chain h0 = sm64(seed), h_{i+1} = sm64(h_i ^ fields[i]). */
uint64_t lexp_rng_key(uint64_t seed, const uint64_t* fields, int32_t n_fields);

/* Random initial labels (host, HxWx3 float32); same values lexp_init_labels
 * writes to the device. */
lexp_status lexp_init_labels_host(int32_t width, int32_t height, double disp_max, uint64_t seed,
                                  float* labels_hw3);

/* Candidate label of one alpha_ij-expansion step (Alg. 1) for the clipped
 * centre cell (ci, cj) of a grid with cells of `cell` pixels, r a random
 * pixel of that cell: alpha = f_r for step < k_prop; for the next k_rans
 * steps the LO-RANSAC plane of the cell's current disparities (f_r where the
 * cell defines no plane: fewer than three pixels, or all in one row or
 * column); after that f_r perturbed (Sec. 3.4) with sizes (r_d, r_n) halved
 * once per refinement step already taken.  labels_hw3: host HxWx3 float32. */
lexp_status lexp_propose(int32_t width, int32_t height, const float* labels_hw3, uint64_t seed,
                         int32_t iteration, int32_t level, int32_t cell, int32_t ci, int32_t cj, int32_t step,
                         int32_t k_prop, int32_t k_rans, double r_d, double r_n, lexp_plane* out);

#ifdef __cplusplus
}
#endif

#endif /* LEXP_H */
