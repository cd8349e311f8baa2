/*
 * lexp_oracle.c -- plain FP64 CPU reference ("oracle") for local expansion
 * move stereo (Taniai, Matsushita, Sato, Naemura: "Continuous 3D Label Stereo
 * Matching using Local Expansion Moves").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or helper with the HIP library; the product path never calls it.
 *
 * Everything is computed in double precision by direct summation, following
 * the paper's definitions in the paper's order.  Two points are decided in a
 * fixed precision on purpose (they turn floating point into an integer
 * decision, so both implementations take them the same way):
 *   - the warped sample position x = u - (a*u + b*v + c) is formed in single
 *     precision (fmaf), because it selects the interpolation taps and whether
 *     the sample lies inside the right image;
 *   - the terms of the binary energy of one expansion are rounded up to
 *     multiples of 2^-20 before the exact minimisation (ceil keeps the
 *     expansion submodularity of Lemma 1 exact on the integers).
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 * BT.601 luma for the gray image; central difference [-0.5 0 0.5] with
 * replicated borders; a sample outside the right image costs the fully
 * truncated value (1-alpha)*tau_col + alpha*tau_grad; guided-filter windows
 * clipped to the image with count normalisation; colour differences on the
 * [0,255] scale; unordered 8-neighbour pairs counted once with equal weight;
 * the minimum cut that takes the candidate label at the fewest pixels (the
 * intersection of all minimisers); the random-init plane passes through
 * (p, z0); perturbation as described for Alg. 2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_Q 1048576.0 /* 2^20 energy quantum of the binary problem */

typedef struct {
  int32_t width, height;
  double disp_max;
  double alpha, tau_col, tau_grad;
  int32_t gf_radius;
  double gf_eps;
  double lambda, tau_dis, w_floor, gamma;
  int32_t neighbours;
} ora_params;

typedef struct {
  ora_params p;
  int W, H;
  double *L, *R;    /* H*W*3, [0,255] */
  double *gL, *gR;  /* x-gradient of the gray image, H*W */
  double *I;        /* guide image I_L/255, H*W*3 */
  double *mu;       /* mean of I over W'_k, H*W*3 */
  double *sig;      /* population covariance over W'_k, H*W*6 (00 01 02 11 12 22) */
} ora_ctx;

static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }

/* ---------------------------------------------------------------------------
 * Gray value and its x-gradient (Sec. 3.2, data term: gray-value gradient by
 * the kernel [-0.5 0 0.5]).
 * ------------------------------------------------------------------------- */
static void gray_grad(const double* img, int H, int W, double* grad) {
  double* g = (double*)malloc(sizeof(double) * (size_t)H * W);
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      const double* px = img + ((size_t)v * W + u) * 3;
      g[(size_t)v * W + u] = 0.299 * px[0] + 0.587 * px[1] + 0.114 * px[2];
    }
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      int ul = imax(u - 1, 0), ur = imin(u + 1, W - 1);
      grad[(size_t)v * W + u] = 0.5 * (g[(size_t)v * W + ur] - g[(size_t)v * W + ul]);
    }
  free(g);
}

/* Window W'_k: the (2r+1)^2 square centred at k, clipped to the image. */
static void window(const ora_ctx* c, int ku, int kv, int* u0, int* u1, int* v0, int* v1) {
  int r = c->p.gf_radius;
  *u0 = imax(ku - r, 0);
  *u1 = imin(ku + r, c->W - 1);
  *v0 = imax(kv - r, 0);
  *v1 = imin(kv + r, c->H - 1);
}

/* Guide statistics of Eq.(7): mean and covariance of I over W'_k, by direct
 * separable window sums. */
static void guide_stats(ora_ctx* c) {
  int W = c->W, H = c->H, r = c->p.gf_radius;
  size_t n = (size_t)W * H;
  double* hs = (double*)calloc(n * 9, sizeof(double)); /* horizontal sums of I (3) and I I^T (6) */
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      double acc[9] = {0};
      for (int x = imax(u - r, 0); x <= imin(u + r, W - 1); ++x) {
        const double* I = c->I + ((size_t)v * W + x) * 3;
        acc[0] += I[0]; acc[1] += I[1]; acc[2] += I[2];
        acc[3] += I[0] * I[0]; acc[4] += I[0] * I[1]; acc[5] += I[0] * I[2];
        acc[6] += I[1] * I[1]; acc[7] += I[1] * I[2]; acc[8] += I[2] * I[2];
      }
      memcpy(hs + ((size_t)v * W + u) * 9, acc, sizeof(acc));
    }
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      double acc[9] = {0};
      for (int y = imax(v - r, 0); y <= imin(v + r, H - 1); ++y)
        for (int q = 0; q < 9; ++q) acc[q] += hs[((size_t)y * W + u) * 9 + q];
      int u0, u1, v0, v1;
      window(c, u, v, &u0, &u1, &v0, &v1);
      double N = (double)(u1 - u0 + 1) * (double)(v1 - v0 + 1);
      double* mu = c->mu + ((size_t)v * W + u) * 3;
      double* sg = c->sig + ((size_t)v * W + u) * 6;
      for (int q = 0; q < 3; ++q) mu[q] = acc[q] / N;
      sg[0] = acc[3] / N - mu[0] * mu[0];
      sg[1] = acc[4] / N - mu[0] * mu[1];
      sg[2] = acc[5] / N - mu[0] * mu[2];
      sg[3] = acc[6] / N - mu[1] * mu[1];
      sg[4] = acc[7] / N - mu[1] * mu[2];
      sg[5] = acc[8] / N - mu[2] * mu[2];
    }
  free(hs);
}

ora_ctx* ora_create(const ora_params* p, const float* left, const float* right) {
  if (!p || !left || !right || p->width <= 0 || p->height <= 0 || p->gf_radius < 1) return NULL;
  ora_ctx* c = (ora_ctx*)calloc(1, sizeof(ora_ctx));
  c->p = *p;
  c->W = p->width;
  c->H = p->height;
  size_t n = (size_t)c->W * c->H;
  c->L = (double*)malloc(sizeof(double) * n * 3);
  c->R = (double*)malloc(sizeof(double) * n * 3);
  c->I = (double*)malloc(sizeof(double) * n * 3);
  c->gL = (double*)malloc(sizeof(double) * n);
  c->gR = (double*)malloc(sizeof(double) * n);
  c->mu = (double*)malloc(sizeof(double) * n * 3);
  c->sig = (double*)malloc(sizeof(double) * n * 6);
  for (size_t i = 0; i < n * 3; ++i) {
    c->L[i] = (double)left[i];
    c->R[i] = (double)right[i];
    c->I[i] = c->L[i] / 255.0;
  }
  gray_grad(c->L, c->H, c->W, c->gL);
  gray_grad(c->R, c->H, c->W, c->gR);
  guide_stats(c);
  return c;
}

void ora_destroy(ora_ctx* c) {
  if (!c) return;
  free(c->L); free(c->R); free(c->I); free(c->gL); free(c->gR); free(c->mu); free(c->sig);
  free(c);
}

void ora_gray_grad(const ora_ctx* c, double* gradL, double* gradR) {
  size_t n = (size_t)c->W * c->H;
  if (gradL) memcpy(gradL, c->gL, sizeof(double) * n);
  if (gradR) memcpy(gradR, c->gR, sizeof(double) * n);
}

void ora_guide(const ora_ctx* c, double* mu, double* sig) {
  size_t n = (size_t)c->W * c->H;
  if (mu) memcpy(mu, c->mu, sizeof(double) * n * 3);
  if (sig) memcpy(sig, c->sig, sizeof(double) * n * 6);
}

double ora_rho_max(const ora_ctx* c) {
  return (1.0 - c->p.alpha) * c->p.tau_col + c->p.alpha * c->p.tau_grad;
}

/* ---------------------------------------------------------------------------
 * Raw matching cost rho(s | f), Eqs.(8),(9): warp s to s' = s - (a s_u + b s_v
 * + c, 0), sample the right image there by linear interpolation, and take the
 * truncated colour (L1, [0,255] scale) plus gray x-gradient difference.
 * ------------------------------------------------------------------------- */
double ora_raw_cost(const ora_ctx* c, int u, int v, const float* f) {
  const ora_params* p = &c->p;
  int W = c->W;
  float uf = (float)u, vf = (float)v;
  float d = fmaf(f[0], uf, fmaf(f[1], vf, f[2]));
  float x = uf - d;
  if (!(x >= 0.0f && x <= (float)(W - 1))) return ora_rho_max(c);
  float xf = floorf(x);
  int i0 = (int)xf;
  int i1 = i0 + 1;
  double t = (double)(x - xf);
  if (i0 >= W - 1) { i0 = W - 1; i1 = W - 1; t = 0.0; }
  const double* Lp = c->L + ((size_t)v * W + u) * 3;
  const double* R0 = c->R + ((size_t)v * W + i0) * 3;
  const double* R1 = c->R + ((size_t)v * W + i1) * 3;
  double col = 0.0;
  for (int ch = 0; ch < 3; ++ch) {
    double J = (1.0 - t) * R0[ch] + t * R1[ch];
    col += fabs(Lp[ch] - J);
  }
  double K = (1.0 - t) * c->gR[(size_t)v * W + i0] + t * c->gR[(size_t)v * W + i1];
  double gr = fabs(c->gL[(size_t)v * W + u] - K);
  return (1.0 - p->alpha) * dmin(col, p->tau_col) + p->alpha * dmin(gr, p->tau_grad);
}

/* rho over the whole image for one label (test helper). */
void ora_rho_map(const ora_ctx* c, const float* f, double* out) {
  for (int v = 0; v < c->H; ++v)
    for (int u = 0; u < c->W; ++u) out[(size_t)v * c->W + u] = ora_raw_cost(c, u, v, f);
}

/* Solve (S + e U) x = y for a symmetric 3x3 S given by its 6 unique entries,
 * by Gaussian elimination with partial pivoting. */
static void solve3(const double* s6, double e, const double* y, double* x) {
  double A[3][4] = {
      {s6[0] + e, s6[1], s6[2], y[0]},
      {s6[1], s6[3] + e, s6[4], y[1]},
      {s6[2], s6[4], s6[5] + e, y[2]},
  };
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (piv != col)
      for (int k = 0; k < 4; ++k) { double t = A[col][k]; A[col][k] = A[piv][k]; A[piv][k] = t; }
    for (int r = col + 1; r < 3; ++r) {
      double m = A[r][col] / A[col][col];
      for (int k = col; k < 4; ++k) A[r][k] -= m * A[col][k];
    }
  }
  for (int r = 2; r >= 0; --r) {
    double s = A[r][3];
    for (int k = r + 1; k < 3; ++k) s -= A[r][k] * x[k];
    x[r] = s / A[r][r];
  }
}

/* ---------------------------------------------------------------------------
 * Guided-filter weights of Eq.(7), written out literally (count-normalised
 * where windows are clipped by the image border):
 *   w_ps = 1/N_p * sum_{k in W'(p), s in W'_k} 1/N_k (1 + (I_p-mu_k)^T
 *          (Sigma_k + eU)^-1 (I_s - mu_k)).
 * Output covers W_p = the (4r+1)^2 square centred at p; entries outside the
 * image are 0.  O(|W'|^2) per pixel: tiny inputs only.
 * ------------------------------------------------------------------------- */
void ora_gf_weights(const ora_ctx* c, int pu, int pv, double* w_out) {
  int r = c->p.gf_radius, W = c->W, H = c->H;
  int side = 4 * r + 1;
  memset(w_out, 0, sizeof(double) * side * side);
  int ku0, ku1, kv0, kv1;
  window(c, pu, pv, &ku0, &ku1, &kv0, &kv1);
  double Np = (double)(ku1 - ku0 + 1) * (double)(kv1 - kv0 + 1);
  const double* Ip = c->I + ((size_t)pv * W + pu) * 3;
  for (int kv = kv0; kv <= kv1; ++kv)
    for (int ku = ku0; ku <= ku1; ++ku) {
      const double* mu = c->mu + ((size_t)kv * W + ku) * 3;
      const double* sg = c->sig + ((size_t)kv * W + ku) * 6;
      double dp[3] = {Ip[0] - mu[0], Ip[1] - mu[1], Ip[2] - mu[2]};
      double y[3];
      solve3(sg, c->p.gf_eps, dp, y); /* y = (Sigma_k + eU)^-1 (I_p - mu_k), symmetric */
      int su0, su1, sv0, sv1;
      window(c, ku, kv, &su0, &su1, &sv0, &sv1);
      double Nk = (double)(su1 - su0 + 1) * (double)(sv1 - sv0 + 1);
      for (int sv = sv0; sv <= sv1; ++sv)
        for (int su = su0; su <= su1; ++su) {
          const double* Is = c->I + ((size_t)sv * W + su) * 3;
          double q = y[0] * (Is[0] - mu[0]) + y[1] * (Is[1] - mu[1]) + y[2] * (Is[2] - mu[2]);
          w_out[(size_t)(sv - pv + 2 * r) * side + (su - pu + 2 * r)] += (1.0 + q) / Nk / Np;
        }
    }
  (void)H;
}

/* phi_p(f) = sum_s w_ps rho(s|f), Eq.(6) with the weights above. */
double ora_unary_direct(const ora_ctx* c, int pu, int pv, const float* f) {
  int r = c->p.gf_radius;
  int side = 4 * r + 1;
  double* w = (double*)malloc(sizeof(double) * side * side);
  ora_gf_weights(c, pu, pv, w);
  double acc = 0.0;
  for (int dy = 0; dy < side; ++dy)
    for (int dx = 0; dx < side; ++dx) {
      int su = pu + dx - 2 * r, sv = pv + dy - 2 * r;
      if (su < 0 || sv < 0 || su >= c->W || sv >= c->H) continue;
      acc += w[(size_t)dy * side + dx] * ora_raw_cost(c, su, sv, f);
    }
  free(w);
  return acc;
}

/* ---------------------------------------------------------------------------
 * Guided filter of a cost slice rho over a rectangle, in the box form of He et
 * al. that the paper uses for Eq.(7) (Sec. 3.5): for every k,
 *   a_k = (Sigma_k + eU)^-1 (mean_k(I rho) - mu_k mean_k(rho)),
 *   b_k = mean_k(rho) - a_k^T mu_k,
 * and phi_p = mean_{k in W'(p)}(a_k)^T I_p + mean_{k in W'(p)}(b_k).
 * Means use direct (non-running) separable window sums.  rho is supplied on
 * the filtering region M (the rectangle dilated by 2r, clipped), as in
 * Eqs.(18)-(20): only its values there reach phi over the rectangle.
 *
 * rect [u0,u1) x [v0,v1) is clipped to the image.  rho_M is indexed
 * (y - m.v0) * m.w + (x - m.u0).  out_phi receives the clipped rectangle
 * row-major; out_ab (optional) receives (a0,a1,a2,b) over R+ = rect dilated
 * by r, clipped, row-major.
 * ------------------------------------------------------------------------- */
typedef struct { int u0, v0, u1, v1; } rect_t;

static rect_t clip_dilate(const ora_ctx* c, int u0, int v0, int u1, int v1, int m) {
  rect_t o;
  o.u0 = imax(u0 - m, 0);
  o.v0 = imax(v0 - m, 0);
  o.u1 = imin(u1 + m, c->W);
  o.v1 = imin(v1 + m, c->H);
  if (o.u1 < o.u0) o.u1 = o.u0;
  if (o.v1 < o.v0) o.v1 = o.v0;
  return o;
}

static void filter_rect(const ora_ctx* c, rect_t R, const double* rho_M, rect_t M,
                        double* out_phi, double* out_ab) {
  int r = c->p.gf_radius, W = c->W;
  rect_t P = clip_dilate(c, R.u0, R.v0, R.u1, R.v1, r); /* R+ */
  int mw = M.u1 - M.u0, mh = M.v1 - M.v0;
  int pw = P.u1 - P.u0, ph = P.v1 - P.v0;
  int rw = R.u1 - R.u0;
  /* Pass 1, horizontal: over rows of M, columns of R+ -> 4 channels (rho, I rho). */
  double* h1 = (double*)calloc((size_t)mh * pw * 4, sizeof(double));
  for (int y = M.v0; y < M.v1; ++y)
    for (int x = P.u0; x < P.u1; ++x) {
      double acc[4] = {0, 0, 0, 0};
      for (int xs = imax(x - r, 0); xs <= imin(x + r, W - 1); ++xs) {
        double rh_ = rho_M[(size_t)(y - M.v0) * mw + (xs - M.u0)];
        const double* Is = c->I + ((size_t)y * W + xs) * 3;
        acc[0] += rh_;
        acc[1] += Is[0] * rh_;
        acc[2] += Is[1] * rh_;
        acc[3] += Is[2] * rh_;
      }
      memcpy(h1 + ((size_t)(y - M.v0) * pw + (x - P.u0)) * 4, acc, sizeof(acc));
    }
  /* Pass 1, vertical + linear coefficients at every k in R+. */
  double* ab = (double*)malloc(sizeof(double) * (size_t)ph * pw * 4);
  for (int kv = P.v0; kv < P.v1; ++kv)
    for (int ku = P.u0; ku < P.u1; ++ku) {
      double acc[4] = {0, 0, 0, 0};
      for (int y = imax(kv - r, 0); y <= imin(kv + r, c->H - 1); ++y)
        for (int q = 0; q < 4; ++q) acc[q] += h1[((size_t)(y - M.v0) * pw + (ku - P.u0)) * 4 + q];
      int su0, su1, sv0, sv1;
      window(c, ku, kv, &su0, &su1, &sv0, &sv1);
      double Nk = (double)(su1 - su0 + 1) * (double)(sv1 - sv0 + 1);
      double mrho = acc[0] / Nk;
      const double* mu = c->mu + ((size_t)kv * W + ku) * 3;
      double cov[3] = {acc[1] / Nk - mu[0] * mrho, acc[2] / Nk - mu[1] * mrho, acc[3] / Nk - mu[2] * mrho};
      double a[3];
      solve3(c->sig + ((size_t)kv * W + ku) * 6, c->p.gf_eps, cov, a);
      double b = mrho - (a[0] * mu[0] + a[1] * mu[1] + a[2] * mu[2]);
      double* o = ab + ((size_t)(kv - P.v0) * pw + (ku - P.u0)) * 4;
      o[0] = a[0]; o[1] = a[1]; o[2] = a[2]; o[3] = b;
    }
  if (out_ab) memcpy(out_ab, ab, sizeof(double) * (size_t)ph * pw * 4);
  /* Pass 2: mean of (a, b) over W'(p) for p in R, then phi_p = abar^T I_p + bbar. */
  if (out_phi) {
    double* h2 = (double*)calloc((size_t)ph * rw * 4, sizeof(double));
    for (int y = P.v0; y < P.v1; ++y)
      for (int x = R.u0; x < R.u1; ++x) {
        double acc[4] = {0, 0, 0, 0};
        for (int xs = imax(x - r, 0); xs <= imin(x + r, W - 1); ++xs)
          for (int q = 0; q < 4; ++q) acc[q] += ab[((size_t)(y - P.v0) * pw + (xs - P.u0)) * 4 + q];
        memcpy(h2 + ((size_t)(y - P.v0) * rw + (x - R.u0)) * 4, acc, sizeof(acc));
      }
    for (int pv = R.v0; pv < R.v1; ++pv)
      for (int pu = R.u0; pu < R.u1; ++pu) {
        double acc[4] = {0, 0, 0, 0};
        for (int y = imax(pv - r, 0); y <= imin(pv + r, c->H - 1); ++y)
          for (int q = 0; q < 4; ++q) acc[q] += h2[((size_t)(y - P.v0) * rw + (pu - R.u0)) * 4 + q];
        int ku0, ku1, kv0, kv1;
        window(c, pu, pv, &ku0, &ku1, &kv0, &kv1);
        double Np = (double)(ku1 - ku0 + 1) * (double)(kv1 - kv0 + 1);
        const double* Ip = c->I + ((size_t)pv * W + pu) * 3;
        out_phi[(size_t)(pv - R.v0) * rw + (pu - R.u0)] =
            (acc[0] * Ip[0] + acc[1] * Ip[1] + acc[2] * Ip[2]) / Np + acc[3] / Np;
      }
    free(h2);
  }
  free(h1);
  free(ab);
}

/* Unary term phi_p(f) for all p in a rectangle under one label (Eqs.(18)-(20)).
 * Returns the number of outputs (clipped rectangle size). */
int64_t ora_unary_region(const ora_ctx* c, int u0, int v0, int u1, int v1, const float* f,
                         double* out_phi, double* out_ab) {
  rect_t R = clip_dilate(c, u0, v0, u1, v1, 0);
  if (R.u1 <= R.u0 || R.v1 <= R.v0) return 0;
  rect_t M = clip_dilate(c, R.u0, R.v0, R.u1, R.v1, 2 * c->p.gf_radius);
  int mw = M.u1 - M.u0, mh = M.v1 - M.v0;
  double* rho = (double*)malloc(sizeof(double) * (size_t)mw * mh);
  for (int y = M.v0; y < M.v1; ++y)
    for (int x = M.u0; x < M.u1; ++x) rho[(size_t)(y - M.v0) * mw + (x - M.u0)] = ora_raw_cost(c, x, y, f);
  filter_rect(c, R, rho, M, out_phi, out_ab);
  free(rho);
  return (int64_t)(R.u1 - R.u0) * (R.v1 - R.v0);
}

/* Guided filter of an arbitrary whole-image map (test helper). */
void ora_filter_map(const ora_ctx* c, const double* rho, double* out) {
  rect_t R = {0, 0, c->W, c->H};
  filter_rect(c, R, rho, R, out, NULL);
}

/* Per-pixel unary phi_p(f_p) with every pixel's own label (the state after the initialisation of Alg. 2):
 * each pixel is a 1x1 region. */
void ora_pixel_costs(const ora_ctx* c, const float* labels, const uint8_t* mask, double* out) {
  int n = c->W * c->H;
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < n; ++i) {
    if (mask && !mask[i]) continue;
    int u = i % c->W, v = i / c->W;
    ora_unary_region(c, u, v, u + 1, v + 1, labels + (size_t)i * 3, out + i, NULL);
  }
}

/* ---------------------------------------------------------------------------
 * Smoothness term, Eqs.(10)-(12), including lambda of Eq.(5):
 *   lambda * max(w_pq, eps) * min(|d_p(f_p)-d_p(f_q)| + |d_q(f_q)-d_q(f_p)|, tau_dis)
 * with w_pq = exp(-||I_L(p)-I_L(q)||_1 / gamma) and d_p(f) = a p_u + b p_v + c.
 * ------------------------------------------------------------------------- */
static double disp_at(const float* f, int u, int v) {
  double t1 = (double)f[0] * (double)u;
  double t2 = (double)f[1] * (double)v;
  double s = t1 + t2;
  return s + (double)f[2];
}

double ora_weight(const ora_ctx* c, int pu, int pv, int qu, int qv) {
  const double* a = c->L + ((size_t)pv * c->W + pu) * 3;
  const double* b = c->L + ((size_t)qv * c->W + qu) * 3;
  double s = fabs(a[0] - b[0]) + fabs(a[1] - b[1]);
  s = s + fabs(a[2] - b[2]);
  return exp(-s / c->p.gamma);
}

double ora_pairwise(const ora_ctx* c, int pu, int pv, int qu, int qv, const float* fp, const float* fq) {
  double w = ora_weight(c, pu, pv, qu, qv);
  double dpp = disp_at(fp, pu, pv), dpq = disp_at(fq, pu, pv);
  double dqq = disp_at(fq, qu, qv), dqp = disp_at(fp, qu, qv);
  double pb = fabs(dpp - dpq) + fabs(dqq - dqp);
  double wt = w > c->p.w_floor ? w : c->p.w_floor;
  double tr = pb < c->p.tau_dis ? pb : c->p.tau_dis;
  return c->p.lambda * wt * tr;
}

/* Forward neighbour offsets: each unordered pair of N once. */
static const int FWD_DU[4] = {1, 0, 1, -1};
static const int FWD_DV[4] = {0, 1, 1, 1};
static int n_fwd(const ora_ctx* c) { return c->p.neighbours == 4 ? 2 : 4; }

/* Energy Eq.(5).  costs: per-pixel phi_p(f_p); if NULL they are computed. */
double ora_energy(const ora_ctx* c, const float* labels, const double* costs, double* unary_out,
                  double* pair_out) {
  int W = c->W, H = c->H;
  double* own = NULL;
  if (!costs) {
    own = (double*)malloc(sizeof(double) * (size_t)W * H);
    ora_pixel_costs(c, labels, NULL, own);
    costs = own;
  }
  double eu = 0.0, ep = 0.0;
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      eu += costs[(size_t)v * W + u];
      for (int d = 0; d < n_fwd(c); ++d) {
        int qu = u + FWD_DU[d], qv = v + FWD_DV[d];
        if (qu < 0 || qu >= W || qv >= H) continue;
        ep += ora_pairwise(c, u, v, qu, qv, labels + ((size_t)v * W + u) * 3, labels + ((size_t)qv * W + qu) * 3);
      }
    }
  free(own);
  if (unary_out) *unary_out = eu;
  if (pair_out) *pair_out = ep;
  return eu + ep;
}

/* ---------------------------------------------------------------------------
 * One local alpha-expansion on a rectangle R (Eq.(13) restricted to R; the
 * construction of Lemma 2's footnote): variables x_p in {0 keep f_p, 1 take
 * alpha} for p in R.  Terms are quantised (ceil to 2^-20) and the binary
 * energy is written as
 *   E(x) = sum_p U_p x_p + sum_{(p,n) in R, n forward of p} w_pn (1 - x_p) x_n
 * (up to a constant), with, for A = psi(f_p,f_n), B = psi(f_p,alpha),
 * C = psi(alpha,f_n), D = psi(alpha,alpha) = 0:
 *   U_p += C - A, U_n += D - C, w_pn = B + C - A - D,
 * and edges leaving R folded into U_p as psi(alpha,f_n) - psi(f_p,f_n).
 * ------------------------------------------------------------------------- */
static int64_t qceil(double x) { return (int64_t)ceil(x * ORA_Q); }

static int same_label(const float* a, const float* b) {
  return memcmp(a, b, sizeof(float) * 3) == 0;
}

/* Binary problem of one expansion.  U: rw*rh, w4: rw*rh*4 (forward dirs). */
void ora_expand_problem(const ora_ctx* c, const float* labels, const double* costs, const double* phi_alpha,
                        int u0, int v0, int u1, int v1, const float* alpha, int64_t* U, int64_t* w4) {
  rect_t R = clip_dilate(c, u0, v0, u1, v1, 0);
  int rw = R.u1 - R.u0, rh = R.v1 - R.v0, W = c->W, H = c->H;
  memset(U, 0, sizeof(int64_t) * (size_t)rw * rh);
  memset(w4, 0, sizeof(int64_t) * (size_t)rw * rh * 4);
  static const int ALL_DU[8] = {1, 0, 1, -1, -1, 0, -1, 1};
  static const int ALL_DV[8] = {0, 1, 1, 1, 0, -1, -1, -1};
  int nf = n_fwd(c);
  for (int pv = R.v0; pv < R.v1; ++pv)
    for (int pu = R.u0; pu < R.u1; ++pu) {
      size_t li = (size_t)(pv - R.v0) * rw + (pu - R.u0);
      const float* fp = labels + ((size_t)pv * W + pu) * 3;
      if (same_label(fp, alpha)) continue; /* phi_p(alpha) = phi_p(f_p); every term cancels */
      U[li] += qceil(phi_alpha[li]) - qceil(costs[(size_t)pv * W + pu]);
      /* all neighbours: forward ones (p first) and backward ones (n first) */
      for (int d = 0; d < 2 * nf; ++d) {
        int dir = d < nf ? d : 4 + (d - nf);
        int nu = pu + ALL_DU[dir], nv = pv + ALL_DV[dir];
        if (nu < 0 || nu >= W || nv < 0 || nv >= H) continue;
        const float* fn = labels + ((size_t)nv * W + nu) * 3;
        int inside = nu >= R.u0 && nu < R.u1 && nv >= R.v0 && nv < R.v1;
        if (!inside) {
          U[li] += qceil(ora_pairwise(c, pu, pv, nu, nv, alpha, fn)) - qceil(ora_pairwise(c, pu, pv, nu, nv, fp, fn));
        } else if (d < nf) {
          /* p first, n second */
          int64_t A = qceil(ora_pairwise(c, pu, pv, nu, nv, fp, fn));
          int64_t B = qceil(ora_pairwise(c, pu, pv, nu, nv, fp, alpha));
          int64_t C = qceil(ora_pairwise(c, pu, pv, nu, nv, alpha, fn));
          U[li] += C - A;
          int64_t w = B + C - A;
          w4[li * 4 + d] = w > 0 ? w : 0;
        } else {
          /* n first, p second: p receives D - C with C = psi(alpha, f_p) on the pair (n,p) */
          U[li] -= qceil(ora_pairwise(c, nu, nv, pu, pv, alpha, fp));
        }
      }
    }
}

/* The same term when n is equal to alpha is handled by the cancellation rule
 * above: when f_n == alpha the forward edge has w = 0 and C - A = 0 exactly. */

/* --- Dinic max-flow on the binary problem, then the source side of the
 *     residual graph = the minimal alpha-set. ------------------------------ */
typedef struct { int to; int64_t cap; } arc_t;

typedef struct {
  int n, s, t;
  int* head;     /* first arc index per node (CSR) */
  int* deg;
  arc_t* arcs;   /* arcs[2i] forward, arcs[2i+1] reverse */
  int* adj;      /* arc ids in CSR order */
  int n_arcs;
} graph_t;

static void solve_binary(int rw, int rh, int nf, const int64_t* U, const int64_t* w4, uint8_t* x) {
  int n = rw * rh;
  int S = n, T = n + 1, N = n + 2;
  int max_arcs = 2 * (n + 4 * n);
  arc_t* arcs = (arc_t*)malloc(sizeof(arc_t) * max_arcs);
  int* from = (int*)malloc(sizeof(int) * max_arcs);
  int na = 0;
#define ADD_EDGE(a, b, cp)                                   \
  do {                                                       \
    arcs[na].to = (b); arcs[na].cap = (cp); from[na] = (a); ++na; \
    arcs[na].to = (a); arcs[na].cap = 0; from[na] = (b); ++na;     \
  } while (0)
  for (int i = 0; i < n; ++i) {
    if (U[i] > 0) ADD_EDGE(i, T, U[i]);
    else if (U[i] < 0) ADD_EDGE(S, i, -U[i]);
  }
  for (int i = 0; i < n; ++i) {
    int pu = i % rw, pv = i / rw;
    for (int d = 0; d < nf; ++d) {
      int64_t w = w4[(size_t)i * 4 + d];
      if (w <= 0) continue;
      int nu = pu + FWD_DU[d], nv = pv + FWD_DV[d];
      if (nu < 0 || nu >= rw || nv < 0 || nv >= rh) continue;
      ADD_EDGE(nv * rw + nu, i, w); /* cut when x_n = 1 and x_p = 0 */
    }
  }
#undef ADD_EDGE
  /* CSR adjacency */
  int* cnt = (int*)calloc(N + 1, sizeof(int));
  for (int a = 0; a < na; ++a) cnt[from[a] + 1]++;
  for (int i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
  int* adj = (int*)malloc(sizeof(int) * (na > 0 ? na : 1));
  int* fill = (int*)malloc(sizeof(int) * N);
  memcpy(fill, cnt, sizeof(int) * N);
  for (int a = 0; a < na; ++a) adj[fill[from[a]]++] = a;
  int* level = (int*)malloc(sizeof(int) * N);
  int* it = (int*)malloc(sizeof(int) * N);
  int* queue = (int*)malloc(sizeof(int) * N);
  int* stack_n = (int*)malloc(sizeof(int) * (N + 1));
  int* stack_a = (int*)malloc(sizeof(int) * (N + 1));
  for (;;) {
    /* BFS levels from S */
    for (int i = 0; i < N; ++i) level[i] = -1;
    int qh = 0, qt = 0;
    level[S] = 0;
    queue[qt++] = S;
    while (qh < qt) {
      int v = queue[qh++];
      for (int k = cnt[v]; k < cnt[v + 1]; ++k) {
        arc_t* e = &arcs[adj[k]];
        if (e->cap > 0 && level[e->to] < 0) { level[e->to] = level[v] + 1; queue[qt++] = e->to; }
      }
    }
    if (level[T] < 0) break;
    for (int i = 0; i < N; ++i) it[i] = cnt[i];
    /* blocking flow by iterative DFS */
    for (;;) {
      int sp = 0;
      stack_n[0] = S;
      int found = 0;
      while (sp >= 0) {
        int v = stack_n[sp];
        if (v == T) { found = 1; break; }
        int advanced = 0;
        for (; it[v] < cnt[v + 1]; ++it[v]) {
          int a = adj[it[v]];
          arc_t* e = &arcs[a];
          if (e->cap > 0 && level[e->to] == level[v] + 1) {
            stack_a[sp] = a;
            stack_n[++sp] = e->to;
            advanced = 1;
            break;
          }
        }
        if (!advanced) {
          level[v] = -1; /* dead end */
          --sp;
          if (sp >= 0) ++it[stack_n[sp]];
        }
      }
      if (!found) break;
      int64_t f = INT64_MAX;
      for (int k = 0; k < sp; ++k) if (arcs[stack_a[k]].cap < f) f = arcs[stack_a[k]].cap;
      for (int k = 0; k < sp; ++k) { arcs[stack_a[k]].cap -= f; arcs[stack_a[k] ^ 1].cap += f; }
    }
  }
  /* source side of the residual graph */
  for (int i = 0; i < N; ++i) level[i] = 0;
  int qh = 0, qt = 0;
  level[S] = 1;
  queue[qt++] = S;
  while (qh < qt) {
    int v = queue[qh++];
    for (int k = cnt[v]; k < cnt[v + 1]; ++k) {
      arc_t* e = &arcs[adj[k]];
      if (e->cap > 0 && !level[e->to]) { level[e->to] = 1; queue[qt++] = e->to; }
    }
  }
  for (int i = 0; i < n; ++i) x[i] = (uint8_t)level[i];
  free(arcs); free(from); free(cnt); free(adj); free(fill); free(level); free(it); free(queue);
  free(stack_n); free(stack_a);
}

/* Quantised binary energy of a labelling (relative to x = 0). */
int64_t ora_binary_energy(int rw, int rh, int nf, const int64_t* U, const int64_t* w4, const uint8_t* x) {
  int64_t e = 0;
  for (int i = 0; i < rw * rh; ++i) {
    if (x[i]) e += U[i];
    int pu = i % rw, pv = i / rw;
    for (int d = 0; d < nf; ++d) {
      int nu = pu + FWD_DU[d], nv = pv + FWD_DV[d];
      if (nu < 0 || nu >= rw || nv < 0 || nv >= rh) continue;
      if (!x[i] && x[nv * rw + nu]) e += w4[(size_t)i * 4 + d];
    }
  }
  return e;
}

void ora_solve_maxflow(int rw, int rh, int neighbours, const int64_t* U, const int64_t* w4, uint8_t* x) {
  solve_binary(rw, rh, neighbours == 4 ? 2 : 4, U, w4, x);
}

/* Exhaustive minimisation (<= 24 variables): returns the intersection of all
 * minimisers (the minimal alpha-set) and the minimum. */
int64_t ora_solve_bruteforce(int rw, int rh, int neighbours, const int64_t* U, const int64_t* w4, uint8_t* x) {
  int n = rw * rh, nf = neighbours == 4 ? 2 : 4;
  if (n > 24) return INT64_MIN;
  uint8_t* y = (uint8_t*)malloc(n > 0 ? n : 1);
  int64_t best = INT64_MAX;
  uint32_t inter = 0;
  for (uint32_t m = 0; m < (1u << n); ++m) {
    for (int i = 0; i < n; ++i) y[i] = (m >> i) & 1u;
    int64_t e = ora_binary_energy(rw, rh, nf, U, w4, y);
    if (e < best) { best = e; inter = m; }
    else if (e == best) inter &= m;
  }
  for (int i = 0; i < n; ++i) x[i] = (inter >> i) & 1u;
  free(y);
  return best;
}

/* One expansion: computes phi(alpha) over R, builds and solves the binary
 * problem, applies it to labels/costs.  Returns the quantised energy change
 * (<= 0) and the number of pixels that took alpha. */
static int64_t expand_one(const ora_ctx* c, float* labels, double* costs, int u0, int v0, int u1, int v1,
                          const float* alpha, int bruteforce, int32_t* n_changed, double* phi_out) {
  rect_t R = clip_dilate(c, u0, v0, u1, v1, 0);
  int rw = R.u1 - R.u0, rh = R.v1 - R.v0, W = c->W;
  if (n_changed) *n_changed = 0;
  if (rw <= 0 || rh <= 0) return 0;
  size_t n = (size_t)rw * rh;
  double* phi = (double*)malloc(sizeof(double) * n);
  int64_t* U = (int64_t*)malloc(sizeof(int64_t) * n);
  int64_t* w4 = (int64_t*)malloc(sizeof(int64_t) * n * 4);
  uint8_t* x = (uint8_t*)malloc(n);
  ora_unary_region(c, R.u0, R.v0, R.u1, R.v1, alpha, phi, NULL);
  ora_expand_problem(c, labels, costs, phi, R.u0, R.v0, R.u1, R.v1, alpha, U, w4);
  int nf = n_fwd(c);
  if (bruteforce && n <= 24) ora_solve_bruteforce(rw, rh, c->p.neighbours, U, w4, x);
  else solve_binary(rw, rh, nf, U, w4, x);
  int64_t de = ora_binary_energy(rw, rh, nf, U, w4, x);
  int32_t nc = 0;
  for (size_t i = 0; i < n; ++i) {
    if (!x[i]) continue;
    int pu = R.u0 + (int)(i % rw), pv = R.v0 + (int)(i / rw);
    memcpy(labels + ((size_t)pv * W + pu) * 3, alpha, sizeof(float) * 3);
    costs[(size_t)pv * W + pu] = phi[i];
    ++nc;
  }
  if (n_changed) *n_changed = nc;
  if (phi_out) memcpy(phi_out, phi, sizeof(double) * n);
  free(phi); free(U); free(w4); free(x);
  return de;
}

int64_t ora_expand(const ora_ctx* c, float* labels, double* costs, int u0, int v0, int u1, int v1,
                   const float* alpha, int bruteforce, int32_t* n_changed) {
  return expand_one(c, labels, costs, u0, v0, u1, v1, alpha, bruteforce, n_changed, NULL);
}

/* One step of a group (Alg. 2: the same step of Alg. 1 for every cell of a
 * group at once): ora_expand on each of n regions with its own candidate.
 * The regions must be pairwise separated by a pixel (Lemma 3: the moves are
 * then independent), so they run in parallel.  rects: n x (u0, v0, u1, v1);
 * alphas: n x 3.  phi_out (may be NULL) receives phi_p(alpha) of Eq. (6) over
 * each clipped region, row-major, regions back to back; dEq and n_changed
 * (may be NULL) one value per region. */
void ora_expand_step(const ora_ctx* c, float* labels, double* costs, int n, const int32_t* rects,
                     const float* alphas, double* phi_out, int64_t* dEq, int32_t* n_changed) {
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  off[0] = 0;
  for (int q = 0; q < n; ++q) {
    rect_t R = clip_dilate(c, rects[4 * q], rects[4 * q + 1], rects[4 * q + 2], rects[4 * q + 3], 0);
    int64_t a = (int64_t)imax(R.u1 - R.u0, 0) * imax(R.v1 - R.v0, 0);
    off[q + 1] = off[q] + a;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int q = 0; q < n; ++q) {
    const int32_t* rc = rects + 4 * q;
    int32_t nc = 0;
    int64_t de = expand_one(c, labels, costs, rc[0], rc[1], rc[2], rc[3], alphas + 3 * q, 0, &nc,
                            phi_out ? phi_out + off[q] : NULL);
    if (dEq) dEq[q] = de;
    if (n_changed) n_changed[q] = nc;
  }
  free(off);
}

/* ---------------------------------------------------------------------------
 * Random numbers: counter-based.  sm64 is the SplitMix64 output function
 * (Steele, Lea and Flood, OOPSLA 2014) applied to a state x:
 *   z = x + 0x9E3779B97F4A7C15; z = (z ^ z>>30) * 0xBF58476D1CE4E5B9;
 *   z = (z ^ z>>27) * 0x94D049BB133111EB; return z ^ z>>31.
 * A draw is keyed by a chain h0 = sm64(seed), h_{i+1} = sm64(h_i ^ field_i).
 * ------------------------------------------------------------------------- */
static uint64_t sm64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static uint64_t key_chain(uint64_t seed, const uint64_t* fields, int nfields) {
  uint64_t h = sm64(seed);
  for (int i = 0; i < nfields; ++i) h = sm64(h ^ fields[i]);
  return h;
}

static double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }         /* [0,1) */
static double u01c(uint64_t x) { return (double)((x >> 11) + 1) * 0x1.0p-53; }  /* (0,1] */

#define TAG_INIT 1u
#define TAG_PROP 2u
static const double TWO_PI = 6.283185307179586;

uint64_t ora_rng_key(uint64_t seed, const uint64_t* fields, int nfields) {
  return key_chain(seed, fields, nfields);
}

/* Random initialisation (Alg. 2): z0 ~ U[0, dispmax], n uniform on the
 * upper unit hemisphere, plane through (p_u, p_v, z0) with normal n. */
void ora_init_labels(const ora_ctx* c, uint64_t seed, float* labels) {
  int W = c->W, H = c->H;
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      uint64_t f[3] = {TAG_INIT, (uint64_t)v * (uint64_t)W + (uint64_t)u, 0};
      double z0 = u01(key_chain(seed, f, 3)) * c->p.disp_max;
      f[2] = 1;
      double nz = u01c(key_chain(seed, f, 3));
      f[2] = 2;
      double ph = TWO_PI * u01(key_chain(seed, f, 3));
      double s = sqrt(1.0 - nz * nz);
      double nx = s * cos(ph), ny = s * sin(ph);
      float* o = labels + ((size_t)v * W + u) * 3;
      o[0] = (float)(-nx / nz);
      o[1] = (float)(-ny / nz);
      o[2] = (float)((nx * (double)u + ny * (double)v + nz * z0) / nz);
    }
}

/* ---------------------------------------------------------------------------
 * RANSAC proposer of Alg. 1 (between the propagation and refinement steps): a
 * plane fitted to the current disparity map over the clipped centre cell
 * C_ij by LO-RANSAC (Chum, Matas, Kittler 2003).  The paper names the method
 * only; the readings:
 *   - points: every pixel p of C_ij with its current disparity
 *     d_p = a_p u + b_p v + c_p (FP64 from the FP32 label);
 *   - RANS_HYP minimal samples; sample m takes pixels floor(U n) of draws
 *     1 + 3m, 2 + 3m, 3 + 3m of the step's key (n pixels in the cell); a
 *     sample with a repeated pixel, or whose three pixels are collinear in
 *     the image, is skipped;
 *   - plane through three points by the normal e1 x e2 of the edge vectors
 *     from the first point: a = -n_u / n_d, b = -n_v / n_d,
 *     c = d_0 - a u_0 - b v_0;
 *   - inlier: |d_p - (a u + b v + c)| <= RANS_TAU;
 *   - a sample with more inliers than the best so far is refined by local
 *     optimisation: up to RANS_LO times, the least-squares plane of the
 *     current inliers (centred normal equations) replaces the model if it
 *     keeps at least as many inliers; the refined model becomes the best;
 *   - no valid sample (fewer than three pixels, or all collinear): the label
 *     of the pixel of draw 0, as the propagation proposer would choose it.
 * ------------------------------------------------------------------------- */
#define RANS_HYP 32
#define RANS_TAU 1.0
#define RANS_LO 4

static int rans_inliers(const double* pu, const double* pv, const double* pd, int n, const double* m,
                        unsigned char* in) {
  int cnt = 0;
  for (int i = 0; i < n; ++i) {
    double pred = m[0] * pu[i] + m[1] * pv[i] + m[2];
    in[i] = fabs(pd[i] - pred) <= RANS_TAU;
    cnt += in[i];
  }
  return cnt;
}

/* least-squares plane d = a u + b v + c over the marked points; 0 if they are
 * fewer than three or (nearly) collinear in the image */
static int rans_lsq(const double* pu, const double* pv, const double* pd, int n, const unsigned char* in,
                    double* m) {
  double su = 0.0, sv = 0.0, sd = 0.0;
  int k = 0;
  for (int i = 0; i < n; ++i)
    if (in[i]) { su += pu[i]; sv += pv[i]; sd += pd[i]; ++k; }
  if (k < 3) return 0;
  double mu = su / k, mv = sv / k, md = sd / k;
  double suu = 0.0, suv = 0.0, svv = 0.0, sud = 0.0, svd = 0.0;
  for (int i = 0; i < n; ++i) {
    if (!in[i]) continue;
    double du = pu[i] - mu, dv = pv[i] - mv, dd = pd[i] - md;
    suu += du * du; suv += du * dv; svv += dv * dv; sud += du * dd; svd += dv * dd;
  }
  double det = suu * svv - suv * suv;
  if (!(det > 1e-9 * suu * svv)) return 0;
  m[0] = (sud * svv - svd * suv) / det;
  m[1] = (svd * suu - sud * suv) / det;
  m[2] = md - m[0] * mu - m[1] * mv;
  return 1;
}

/* Returns 1 and the fitted plane in alpha, or 0 when no sample is valid. */
static int ora_ransac(const ora_ctx* c, const float* labels, uint64_t seed, const uint64_t* key6, int cu0, int cv0,
                      int cw, int ch, float* alpha) {
  int n = cw * ch;
  if (n < 3) return 0;
  double* pu = (double*)malloc(sizeof(double) * 3 * n);
  double* pv = pu + n;
  double* pd = pv + n;
  unsigned char* in = (unsigned char*)malloc((size_t)2 * n);
  unsigned char* tmp = in + n;
  for (int i = 0; i < n; ++i) {
    int u = cu0 + i % cw, v = cv0 + i / cw;
    pu[i] = u;
    pv[i] = v;
    pd[i] = disp_at(labels + ((size_t)v * c->W + u) * 3, u, v);
  }
  uint64_t f[7];
  memcpy(f, key6, sizeof(uint64_t) * 6);
  int best = -1;
  double bm[3] = {0.0, 0.0, 0.0};
  for (int m = 0; m < RANS_HYP; ++m) {
    int s[3];
    for (int k = 0; k < 3; ++k) {
      f[6] = (uint64_t)(1 + 3 * m + k);
      int64_t idx = (int64_t)(u01(key_chain(seed, f, 7)) * (double)n);
      if (idx >= n) idx = n - 1;
      s[k] = (int)idx;
    }
    if (s[0] == s[1] || s[0] == s[2] || s[1] == s[2]) continue;
    double e1u = pu[s[1]] - pu[s[0]], e1v = pv[s[1]] - pv[s[0]], e1d = pd[s[1]] - pd[s[0]];
    double e2u = pu[s[2]] - pu[s[0]], e2v = pv[s[2]] - pv[s[0]], e2d = pd[s[2]] - pd[s[0]];
    double nu = e1v * e2d - e1d * e2v;
    double nv = e1d * e2u - e1u * e2d;
    double nd = e1u * e2v - e1v * e2u;
    if (nd == 0.0) continue;
    double mdl[3];
    mdl[0] = -nu / nd;
    mdl[1] = -nv / nd;
    mdl[2] = pd[s[0]] - mdl[0] * pu[s[0]] - mdl[1] * pv[s[0]];
    int cnt = rans_inliers(pu, pv, pd, n, mdl, in);
    if (cnt <= best) continue;
    for (int it = 0; it < RANS_LO; ++it) {  /* local optimisation */
      double ls[3];
      if (!rans_lsq(pu, pv, pd, n, in, ls)) break;
      int c2 = rans_inliers(pu, pv, pd, n, ls, tmp);
      if (c2 < cnt) break;
      memcpy(mdl, ls, sizeof(ls));
      memcpy(in, tmp, (size_t)n);
      cnt = c2;
    }
    best = cnt;
    memcpy(bm, mdl, sizeof(bm));
  }
  free(pu);
  free(in);
  if (best < 0) return 0;
  alpha[0] = (float)bm[0];
  alpha[1] = (float)bm[1];
  alpha[2] = (float)bm[2];
  return 1;
}

/* Candidate label of one alpha_ij-expansion step (Alg. 1), in the order of
 * Alg. 1: k_prop propagation steps (alpha = f_r for a random pixel r of the
 * clipped centre cell), then k_rans RANSAC steps (above), then refinement
 * steps: f_r perturbed with the sizes halved once per refinement step already
 * taken.  Perturbation: disparity d at r plus U[-r_d, r_d]; unit normal plus a
 * vector of length r_n uniform on the sphere, renormalised; converted back to
 * (a, b, c). */
void ora_propose(const ora_ctx* c, const float* labels, uint64_t seed, int iteration, int level, int cell,
                 int ci, int cj, int step, int k_prop, int k_rans, double r_d, double r_n, float* alpha) {
  int W = c->W, H = c->H;
  int cu0 = ci * cell, cv0 = cj * cell;
  int cu1 = imin(cu0 + cell, W), cv1 = imin(cv0 + cell, H);
  int cw = cu1 - cu0, ch = cv1 - cv0;
  uint64_t f[7] = {TAG_PROP, (uint64_t)iteration, (uint64_t)level, (uint64_t)ci, (uint64_t)cj, (uint64_t)step, 0};
  int64_t npx = (int64_t)cw * ch;
  int64_t idx = (int64_t)(u01(key_chain(seed, f, 7)) * (double)npx);
  if (idx >= npx) idx = npx - 1;
  int ru = cu0 + (int)(idx % cw), rv = cv0 + (int)(idx / cw);
  const float* fr = labels + ((size_t)rv * W + ru) * 3;
  if (step < k_prop) { memcpy(alpha, fr, sizeof(float) * 3); return; }
  if (step < k_prop + k_rans) {
    if (!ora_ransac(c, labels, seed, f, cu0, cv0, cw, ch, alpha)) memcpy(alpha, fr, sizeof(float) * 3);
    return;
  }
  int halvings = step - k_prop - k_rans;
  double rd = r_d, rn = r_n;
  for (int k = 0; k < halvings; ++k) { rd *= 0.5; rn *= 0.5; }
  f[6] = 1;
  double dd = (2.0 * u01(key_chain(seed, f, 7)) - 1.0) * rd;
  f[6] = 2;
  double z = 2.0 * u01(key_chain(seed, f, 7)) - 1.0;
  f[6] = 3;
  double ph = TWO_PI * u01(key_chain(seed, f, 7));
  double s = sqrt(1.0 - z * z);
  double dn[3] = {rn * (s * cos(ph)), rn * (s * sin(ph)), rn * z};
  double a = fr[0], b = fr[1], cc = fr[2];
  double d = disp_at(fr, ru, rv);
  double len = sqrt(a * a + b * b + 1.0);
  double n0[3] = {-a / len, -b / len, 1.0 / len};
  double n1[3] = {n0[0] + dn[0], n0[1] + dn[1], n0[2] + dn[2]};
  double l1 = sqrt(n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
  n1[0] /= l1; n1[1] /= l1; n1[2] /= l1;
  if (!(fabs(n1[2]) >= 1e-3)) { n1[0] = n0[0]; n1[1] = n0[1]; n1[2] = n0[2]; }
  double d1 = d + dd;
  alpha[0] = (float)(-n1[0] / n1[2]);
  alpha[1] = (float)(-n1[1] / n1[2]);
  alpha[2] = (float)((n1[0] * (double)ru + n1[1] * (double)rv + n1[2] * d1) / n1[2]);
  (void)H; (void)cc;
}

/* Candidate of one step with learned proposals (a proposer of alpha_ij, which
 * Alg. 1 leaves open): a refinement step whose refinement index (step - k_prop
 * - k_rans) is odd takes planes[r], the plane a network proposes at the pixel
 * r the step draws (draw 0 of the step's key, as above); every other step is
 * ora_propose's.  planes: H*W*3 floats (a, b, c) or NULL (no learned steps). */
void ora_propose_learned(const ora_ctx* c, const float* labels, const float* planes, uint64_t seed,
                         int iteration, int level, int cell, int ci, int cj, int step, int k_prop, int k_rans,
                         double r_d, double r_n, float* alpha) {
  int first = k_prop + k_rans;
  if (planes && step >= first && ((step - first) % 2) == 1) {
    int W = c->W, H = c->H;
    int cu0 = ci * cell, cv0 = cj * cell;
    int cw = imin(cu0 + cell, W) - cu0, ch = imin(cv0 + cell, H) - cv0;
    uint64_t f[7] = {TAG_PROP, (uint64_t)iteration, (uint64_t)level, (uint64_t)ci, (uint64_t)cj, (uint64_t)step, 0};
    int64_t npx = (int64_t)cw * ch;
    int64_t idx = (int64_t)(u01(key_chain(seed, f, 7)) * (double)npx);
    if (idx >= npx) idx = npx - 1;
    int ru = cu0 + (int)(idx % cw), rv = cv0 + (int)(idx / cw);
    memcpy(alpha, planes + ((size_t)rv * W + ru) * 3, sizeof(float) * 3);
    return;
  }
  ora_propose(c, labels, seed, iteration, level, cell, ci, cj, step, k_prop, k_rans, r_d, r_n, alpha);
}

/* ---------------------------------------------------------------------------
 * Optimisation procedure (Alg. 2 with Alg. 1 per cell).  Grid level h has
 * cells of `cells[h]` pixels; cell (i, j) (i = column index, j = row index)
 * belongs to group 4 (j mod 4) + (i mod 4) (Eq.(15)); its expansion region is
 * the 3x3 block of cells around it, clipped.  Cells of one group are mutually
 * independent (Lemma 3) and run in parallel.
 * ------------------------------------------------------------------------- */

/* Runs Alg. 1 for every cell of group k of one grid level.  Returns the number
 * of cost evaluations (sum of |R| over the expansions). */
int64_t ora_run_group_ex(const ora_ctx* c, float* labels, double* costs, uint64_t seed, int iteration, int level,
                         int cell, int k_prop, int k_rans, int k_rand, double r_d, double r_n, int group,
                         int batch_cycle, int64_t* dEq);

int64_t ora_run_group(const ora_ctx* c, float* labels, double* costs, uint64_t seed, int iteration, int level,
                      int cell, int k_prop, int k_rans, int k_rand, double r_d, double r_n, int group,
                      int64_t* dEq) {
  return ora_run_group_ex(c, labels, costs, seed, iteration, level, cell, k_prop, k_rans, k_rand, r_d, r_n, group, 0,
                          dEq);
}

/* As ora_run_group; with batch_cycle != 0 every candidate of a cell's Alg. 1
 * is drawn from the labels as they stand before the cell's first move (the
 * "batch cycle" of Sec. 3.4), then the moves are made in Alg. 1's order. */
int64_t ora_run_group_ex(const ora_ctx* c, float* labels, double* costs, uint64_t seed, int iteration, int level,
                         int cell, int k_prop, int k_rans, int k_rand, double r_d, double r_n, int group,
                         int batch_cycle, int64_t* dEq) {
  int W = c->W, H = c->H;
  int nci = (W + cell - 1) / cell, ncj = (H + cell - 1) / cell;
  int gi = group % 4, gj = group / 4;
  int ni = gi < nci ? (nci - gi + 3) / 4 : 0;
  int nj = gj < ncj ? (ncj - gj + 3) / 4 : 0;
  int ncell = ni * nj;
  int64_t evals = 0, de = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : evals, de)
  for (int q = 0; q < ncell; ++q) {
    int ci = gi + 4 * (q % ni), cj = gj + 4 * (q / ni);
    int u0 = (ci - 1) * cell, v0 = (cj - 1) * cell;
    int u1 = (ci + 2) * cell, v1 = (cj + 2) * cell;
    rect_t R = clip_dilate(c, u0, v0, u1, v1, 0);
    int K = k_prop + k_rans + k_rand;
    float* batch = batch_cycle ? (float*)malloc(sizeof(float) * 3 * (size_t)(K > 0 ? K : 1)) : NULL;
    if (batch)
      for (int t = 0; t < K; ++t)
        ora_propose(c, labels, seed, iteration, level, cell, ci, cj, t, k_prop, k_rans, r_d, r_n, batch + 3 * t);
    for (int t = 0; t < K; ++t) {
      float alpha[3];
      if (batch) memcpy(alpha, batch + 3 * t, sizeof(alpha));
      else ora_propose(c, labels, seed, iteration, level, cell, ci, cj, t, k_prop, k_rans, r_d, r_n, alpha);
      de += ora_expand(c, labels, costs, R.u0, R.v0, R.u1, R.v1, alpha, 0, NULL);
      evals += (int64_t)(R.u1 - R.u0) * (R.v1 - R.v0);
    }
    free(batch);
  }
  (void)H;
  if (dEq) *dEq += de;
  return evals;
}

/* Full plain method.  labels/costs are outputs (H*W*3 / H*W).  energy (may be
 * NULL) receives iterations+1 values: after initialisation and after each
 * iteration.  Returns the number of cost evaluations including the per-pixel
 * initial costs. */
int64_t ora_optimize_ex(const ora_ctx* c, uint64_t seed, int n_levels, const int* cells, const int* k_prop,
                        const int* k_rans, const int* k_rand, int iterations, int batch_cycle, float* labels,
                        double* costs, double* energy);

int64_t ora_optimize(const ora_ctx* c, uint64_t seed, int n_levels, const int* cells, const int* k_prop,
                     const int* k_rans, const int* k_rand, int iterations, float* labels, double* costs,
                     double* energy) {
  return ora_optimize_ex(c, seed, n_levels, cells, k_prop, k_rans, k_rand, iterations, 0, labels, costs, energy);
}

/* As ora_optimize, with the batch cycle of ora_run_group_ex as an option. */
int64_t ora_optimize_ex(const ora_ctx* c, uint64_t seed, int n_levels, const int* cells, const int* k_prop,
                        const int* k_rans, const int* k_rand, int iterations, int batch_cycle, float* labels,
                        double* costs, double* energy) {
  ora_init_labels(c, seed, labels);
  ora_pixel_costs(c, labels, NULL, costs);
  int64_t evals = (int64_t)c->W * c->H;
  if (energy) energy[0] = ora_energy(c, labels, costs, NULL, NULL);
  double r_d = c->p.disp_max / 2.0, r_n = 1.0;
  for (int it = 0; it < iterations; ++it) {
    for (int h = 0; h < n_levels; ++h)
      for (int k = 0; k < 16; ++k)
        evals += ora_run_group_ex(c, labels, costs, seed, it, h, cells[h], k_prop[h], k_rans[h], k_rand[h], r_d,
                                  r_n, k, batch_cycle, NULL);
    r_d *= 0.5;
    r_n *= 0.5;
    if (energy) energy[it + 1] = ora_energy(c, labels, costs, NULL, NULL);
  }
  return evals;
}

/* ---------------------------------------------------------------------------
 * Post-processing of the left view (the paper applies that of Bleyer, Rhemann
 * and Rother 2011 without restating it).  Readings:
 *   - left-right check: pixel p = (u, v) of the left map with disparity d_L
 *     matches right pixel x = floor(u - d_L + 1/2) of its row; p is consistent
 *     when 0 <= x < W and |d_L - d_R(x)| <= PP_TOL, where d_R(x) is the right
 *     view's disparity at x (its labels are in the mirrored frame of the right
 *     image: right pixel x is mirrored pixel W-1-x);
 *   - filling: an inconsistent pixel takes, of the planes of the nearest
 *     consistent pixels to its left and right in its row, the one with the
 *     lower disparity at the pixel (either one if the other is missing; its
 *     own disparity if the row has none);
 *   - weighted median: each inconsistent pixel then takes the weighted median
 *     of the filled disparities in the (2 PP_R + 1)^2 window around it
 *     (clipped), with weights exp(-||I_L(p) - I_L(q)||_1 / gamma) quantised
 *     down to multiples of 2^-24; values ordered by (disparity, row-major
 *     index), the median being the first whose cumulative weight reaches half
 *     the total (integer sums, so the choice does not depend on summation
 *     order).  Consistent pixels keep their disparity.
 * Disparities are d = a u + b v + c in FP64 from the FP32 labels.
 * ------------------------------------------------------------------------- */
#define PP_R 17
#define PP_TOL 1.0
#define PP_WQ 16777216.0

typedef struct { double d; int idx; int64_t w; } pp_item;

static int pp_cmp(const void* x, const void* y) {
  const pp_item* a = (const pp_item*)x;
  const pp_item* b = (const pp_item*)y;
  if (a->d < b->d) return -1;
  if (a->d > b->d) return 1;
  return (a->idx > b->idx) - (a->idx < b->idx);
}

void ora_postprocess(const ora_ctx* c, const float* labL, const float* labR, double* out, uint8_t* invalid) {
  int W = c->W, H = c->H;
  size_t n = (size_t)W * H;
  double* dL = (double*)malloc(sizeof(double) * n);
  double* fill = (double*)malloc(sizeof(double) * n);
  uint8_t* ok = (uint8_t*)malloc(n);
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      size_t p = (size_t)v * W + u;
      dL[p] = disp_at(labL + p * 3, u, v);
      double xd = floor((double)u - dL[p] + 0.5);
      ok[p] = 0;
      if (xd >= 0.0 && xd <= (double)(W - 1)) {
        int x = (int)xd, um = W - 1 - x;
        double dR = disp_at(labR + ((size_t)v * W + um) * 3, um, v);
        ok[p] = fabs(dL[p] - dR) <= PP_TOL;
      }
    }
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      size_t p = (size_t)v * W + u;
      fill[p] = dL[p];
      if (ok[p]) continue;
      int ul = u - 1, ur = u + 1;
      while (ul >= 0 && !ok[(size_t)v * W + ul]) --ul;
      while (ur < W && !ok[(size_t)v * W + ur]) ++ur;
      int have_l = ul >= 0, have_r = ur < W;
      if (have_l && have_r) {
        double a = disp_at(labL + ((size_t)v * W + ul) * 3, u, v);
        double b = disp_at(labL + ((size_t)v * W + ur) * 3, u, v);
        fill[p] = a <= b ? a : b;
      } else if (have_l) {
        fill[p] = disp_at(labL + ((size_t)v * W + ul) * 3, u, v);
      } else if (have_r) {
        fill[p] = disp_at(labL + ((size_t)v * W + ur) * 3, u, v);
      }
    }
  int side = 2 * PP_R + 1;
  pp_item* items = (pp_item*)malloc(sizeof(pp_item) * side * side);
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      size_t p = (size_t)v * W + u;
      if (invalid) invalid[p] = !ok[p];
      if (ok[p]) { out[p] = dL[p]; continue; }
      const double* cp = c->L + p * 3;
      int m = 0;
      int64_t total = 0;
      for (int y = imax(v - PP_R, 0); y <= imin(v + PP_R, H - 1); ++y)
        for (int x = imax(u - PP_R, 0); x <= imin(u + PP_R, W - 1); ++x) {
          size_t q = (size_t)y * W + x;
          const double* cq = c->L + q * 3;
          double sdist = fabs(cp[0] - cq[0]) + fabs(cp[1] - cq[1]) + fabs(cp[2] - cq[2]);
          items[m].d = fill[q];
          items[m].idx = (int)q;
          items[m].w = (int64_t)floor(exp(-sdist / c->p.gamma) * PP_WQ);
          total += items[m].w;
          ++m;
        }
      qsort(items, (size_t)m, sizeof(pp_item), pp_cmp);
      int64_t cum = 0;
      double med = items[m - 1].d;
      for (int k = 0; k < m; ++k) {
        cum += items[k].w;
        if (2 * cum >= total) { med = items[k].d; break; }
      }
      out[p] = med;
    }
  free(items);
  free(dL);
  free(fill);
  free(ok);
}

/* Threads of the oracle's parallel loops (n <= 0: the default). */
void ora_set_threads(int n) {
#ifdef _OPENMP
  static int dflt = 0;
  if (!dflt) dflt = omp_get_max_threads();
  omp_set_num_threads(n > 0 ? n : dflt);
#else
  (void)n;
#endif
}

int ora_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
